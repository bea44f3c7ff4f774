// Soft steric forces plus gravity (paper, Sec. III, eq. soft_potential).
//
// U(r) = U0 + U0 (d - r)/b for r < d and U0 exp(-(r - d)/b) for r >= d, with d = 2a and r
// the centre distance for sphere pairs, d = a and r = z for the wall (absent in free space);
// the force is -grad U, magnitude U0/b or (U0/b) exp(-(r - d)/b), repulsive.  Gravity adds
// f_g along z.  Pairs farther than d + 40 b are skipped (their force is below 4.3e-18 U0/b).
// Brute-force O(N^2) distance tests over LDS tiles, float64 throughout, unclamped positions,
// minimum-image separations in a pseudo-periodic box (App. B); the sources are split over
// workgroups and the chunk sums added in a fixed order (deterministic).
#include <algorithm>
#include <cmath>

#include "rpb_internal.h"

namespace rpb {

namespace {

constexpr int kBlock = 256;
constexpr int kMinWorkgroups = 2048;   // source chunks are added until the grid reaches this

// Sources [s0, s1) against the lane's targets t0 + q kBlock + tid (q < KT) that lie below t1;
// accumulates into f[q][3].  Every lane must call (synchronises).
template <int KT>
__device__ __forceinline__ void steric_accumulate(const double *__restrict__ pos, int64_t t0,
                                                  int64_t t1, int64_t s0, int64_t s1, double a,
                                                  double u0, double b, double lx, double ly,
                                                  double (&f)[KT][3], const double (&tq)[KT][3],
                                                  double *sx, double *sy, double *sz) {
  const int tid = threadIdx.x;
  const double d = 2.0 * a;
  const double cut = d + 40.0 * b;
  const double cut2 = cut * cut;
  const double fmax_ = u0 / b;
  const double inv_b = 1.0 / b;
  for (int64_t j0 = s0; j0 < s1; j0 += kBlock) {
    const int cnt = int(min<int64_t>(kBlock, s1 - j0));
    __syncthreads();
    if (tid < cnt) {
      const int64_t j = j0 + tid;
      sx[tid] = pos[3 * j];
      sy[tid] = pos[3 * j + 1];
      sz[tid] = pos[3 * j + 2];
    }
    __syncthreads();
    for (int jj = 0; jj < cnt; ++jj) {
      const double xj = sx[jj], yj = sy[jj], zj = sz[jj];
      double dx[KT], dy[KT], dz[KT], r2[KT];
      bool hit = false;
#pragma unroll
      for (int q = 0; q < KT; ++q) {
        dx[q] = tq[q][0] - xj;
        dy[q] = tq[q][1] - yj;
        if (lx > 0.0) {   // pseudo-periodic box: minimum image
          dx[q] -= lx * rint(dx[q] / lx);
          dy[q] -= ly * rint(dy[q] / ly);
        }
        dz[q] = tq[q][2] - zj;
        r2[q] = dx[q] * dx[q] + dy[q] * dy[q] + dz[q] * dz[q];
        hit |= r2[q] < cut2;
      }
      if (hit) {   // rare: a handful of neighbours per target
#pragma unroll
        for (int q = 0; q < KT; ++q) {
          const int64_t i = t0 + q * kBlock + tid;
          if (r2[q] < cut2 && r2[q] > 0.0 && j0 + jj != i && i < t1) {
            const double r = sqrt(r2[q]);
            const double fm = r < d ? fmax_ : fmax_ * exp(-(r - d) * inv_b);
            const double sc = fm / r;
            f[q][0] += sc * dx[q];
            f[q][1] += sc * dy[q];
            f[q][2] += sc * dz[q];
          }
        }
      }
    }
  }
}

// Targets [t0, min(t0 + KT kBlock, t1)) against sources [s0, s1).  FINAL: adds the wall force
// and gravity and stores the force; otherwise stores the pair sum into `out` (a partial).
template <int KT, bool FINAL>
__device__ __forceinline__ void steric_tile(const double *__restrict__ pos, int64_t t0, int64_t t1,
                                            int64_t s0, int64_t s1, double a, double u0, double b,
                                            double lx, double ly, double f_grav_z, int wall,
                                            double *__restrict__ out) {
  __shared__ double sx[kBlock], sy[kBlock], sz[kBlock];
  const int tid = threadIdx.x;
  double f[KT][3], tq[KT][3];
#pragma unroll
  for (int q = 0; q < KT; ++q) {
    const int64_t i = t0 + q * kBlock + tid;
    const int64_t ii = i < t1 ? i : t0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      tq[q][c] = pos[3 * ii + c];
      f[q][c] = 0.0;
    }
  }
  steric_accumulate<KT>(pos, t0, t1, s0, s1, a, u0, b, lx, ly, f, tq, sx, sy, sz);
#pragma unroll
  for (int q = 0; q < KT; ++q) {
    const int64_t i = t0 + q * kBlock + tid;
    if (i < t1) {
      double fz = f[q][2];
      if (FINAL) {
        const double zi = tq[q][2];
        const double fmax_ = u0 / b;
        if (wall) fz += zi < a ? fmax_ : fmax_ * exp(-(zi - a) / b);
        fz += f_grav_z;
      }
      out[3 * i] = f[q][0];
      out[3 * i + 1] = f[q][1];
      out[3 * i + 2] = fz;
    }
  }
}

// grid (target tiles of KT kBlock, source chunks).  One chunk: final forces straight into
// `out`; several: chunk c writes its pair sums to out + 3 n c.
template <int KT, bool FINAL>
__global__ __launch_bounds__(kBlock) void steric_kernel(int64_t n, int64_t chunk,
                                                        const double *__restrict__ pos, double a,
                                                        double u0, double b, double lx, double ly,
                                                        double f_grav_z, int wall,
                                                        double *__restrict__ out) {
  const int64_t t0 = int64_t(blockIdx.x) * kBlock * KT;
  const int64_t s0 = int64_t(blockIdx.y) * chunk;
  const int64_t s1 = min(n, s0 + chunk);
  steric_tile<KT, FINAL>(pos, t0, n, s0, s1, a, u0, b, lx, ly, f_grav_z, wall,
                         out + 3 * n * blockIdx.y);
}

// Sums the chunk partials in chunk order, then adds the wall force and gravity.
__global__ __launch_bounds__(kBlock) void steric_finish(int64_t n, int nchunks,
                                                        const double *__restrict__ pos,
                                                        const double *__restrict__ part, double a,
                                                        double u0, double b, double f_grav_z,
                                                        int wall, double *__restrict__ force) {
  const int64_t e = int64_t(blockIdx.x) * kBlock + threadIdx.x;   // element of the (n, 3) array
  if (e >= 3 * n) return;
  double acc = 0.0;
  for (int c = 0; c < nchunks; ++c) acc += part[3 * n * c + e];
  if (e % 3 == 2) {
    const double z = pos[e];
    const double fmax_ = u0 / b;
    if (wall) acc += z < a ? fmax_ : fmax_ * exp(-(z - a) / b);
    acc += f_grav_z;
  }
  force[e] = acc;
}

// One workgroup per (system, tile of kBlock targets) item, against all of the system's spheres.
__global__ __launch_bounds__(kBlock) void steric_kernel_batched(const int64_t *__restrict__ offs,
                                                                const int2 *__restrict__ tiles,
                                                                const double *__restrict__ pos,
                                                                double a, double u0, double b,
                                                                double f_grav_z, int wall,
                                                                double *__restrict__ force) {
  const int2 tl = tiles[blockIdx.x];
  const int64_t s0 = offs[tl.x], s1 = offs[tl.x + 1];
  steric_tile<1, true>(pos, s0 + int64_t(tl.y) * kBlock, s1, s0, s1, a, u0, b, 0.0, 0.0, f_grav_z,
                       wall, force);
}

}  // namespace

int forces_batched_run(rpb_ctx *ctx, const rpb_params *p, const Batch &bt, const double *pos,
                       double f_grav_z, double u0, double b, double *force, hipStream_t stream) {
  if (bt.ntiles <= 0) return RPB_OK;
  steric_kernel_batched<<<unsigned(bt.ntiles), kBlock, 0, stream>>>(
      bt.offs, bt.tiles, pos, p->a, u0, b, f_grav_z, p->wall, force);
  RPB_LAUNCHED(ctx);
  return RPB_OK;
}

int forces_run(rpb_ctx *ctx, const rpb_params *p, int64_t n, const double *pos, double f_grav_z,
               double u0, double b, double *force, hipStream_t stream) {
  if (n <= 0) return RPB_OK;
  const double cut = 2.0 * p->a + 40.0 * b;
  if (p->lx > 0.0 && (p->lx <= 2.0 * cut || p->ly <= 2.0 * cut))
    return fail(ctx, RPB_EINVAL, "box %g x %g too small for the minimum image (need > %g)", p->lx,
                p->ly, 2.0 * cut);
  constexpr int kTargets = 2;
  const int64_t per = int64_t(kBlock) * kTargets;
  const int64_t tiles = (n + per - 1) / per;
  // split the sources (in whole LDS tiles) until the grid fills the chip
  const int64_t ltiles = (n + kBlock - 1) / kBlock;
  const int64_t want = std::min<int64_t>({(kMinWorkgroups + tiles - 1) / tiles, ltiles, 64});
  const int64_t chunk = (ltiles + want - 1) / want * kBlock;
  const int64_t nchunks = (n + chunk - 1) / chunk;
  if (tiles > 0x7fffffff) return fail(ctx, RPB_EINVAL, "too many spheres");
  if (nchunks == 1) {
    steric_kernel<kTargets, true><<<dim3{unsigned(tiles), 1u, 1u}, kBlock, 0, stream>>>(
        n, chunk, pos, p->a, u0, b, p->lx, p->ly, f_grav_z, p->wall, force);
    RPB_LAUNCHED(ctx);
    return RPB_OK;
  }
  int st;
  double *part = static_cast<double *>(
      workspace(ctx, WS_PART, size_t(nchunks) * 3 * size_t(n) * sizeof(double), &st));
  if (!part) return st;
  steric_kernel<kTargets, false><<<dim3{unsigned(tiles), unsigned(nchunks), 1u}, kBlock, 0,
                                   stream>>>(n, chunk, pos, p->a, u0, b, p->lx, p->ly, f_grav_z,
                                             p->wall, part);
  RPB_LAUNCHED(ctx);
  const int64_t elems = 3 * n;
  steric_finish<<<unsigned((elems + kBlock - 1) / kBlock), kBlock, 0, stream>>>(
      n, int(nchunks), pos, part, p->a, u0, b, f_grav_z, p->wall, force);
  RPB_LAUNCHED(ctx);
  return RPB_OK;
}

}  // namespace rpb

using namespace rpb;

extern "C" int rpb_forces(rpb_ctx *ctx, const rpb_params *p, int64_t n, const double *pos,
                          double f_grav_z, double u0, double b, double *force_out,
                          rpb_stream_t stream_) {
  RPB_TRY(check_params(ctx, p));
  if (n < 0) return fail(ctx, RPB_EINVAL, "n must be >= 0");
  if (!(u0 >= 0.0) || !(b > 0.0)) return fail(ctx, RPB_EINVAL, "need u0 >= 0 and b > 0");
  if (n == 0) return RPB_OK;
  if (!pos || !force_out) return fail(ctx, RPB_EINVAL, "pos and force_out must not be NULL");
  const size_t nb = size_t(n) * 3 * sizeof(double);
  if (overlaps(force_out, nb, pos, nb)) return fail(ctx, RPB_EINVAL, "force_out overlaps pos");
  hipStream_t stream = static_cast<hipStream_t>(stream_);
  RPB_HIP(ctx, hipSetDevice(ctx->device));
  RPB_TRY(check_finite(ctx, pos, n, stream));
  return forces_run(ctx, p, n, pos, f_grav_z, u0, b, force_out, stream);
}
