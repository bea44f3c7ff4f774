// Soft steric forces plus gravity (paper, Sec. III, eq. soft_potential).
//
// U(r) = U0 + U0 (d - r)/b for r < d and U0 exp(-(r - d)/b) for r >= d, with d = 2a and r
// the centre distance for sphere pairs, d = a and r = z for the wall; the force is -grad U,
// magnitude U0/b or (U0/b) exp(-(r - d)/b), repulsive.  Gravity adds f_g along z.  Pairs
// farther than d + 40 b are skipped (their force is below 4.3e-18 U0/b).  Brute-force
// O(N^2) distance tests over LDS tiles (4 targets per lane), float64 throughout; unclamped
// positions.
#include <cmath>

#include "rpb_internal.h"

namespace rpb {

namespace {

constexpr int kBlock = 256;

constexpr int kTargets = 4;   // targets per lane

// Sources [s0, s1) against the lane's targets [t0 + q kBlock + tid], q < kTargets, below t1;
// accumulates into f[q][3].  Every lane must call (synchronises).
__device__ __forceinline__ void steric_block(const double *__restrict__ pos, int64_t t0,
                                             int64_t t1, int64_t s0, int64_t s1, double a,
                                             double u0, double b, double (&f)[kTargets][3],
                                             const double (&tq)[kTargets][3], double *sx,
                                             double *sy, double *sz) {
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
#pragma unroll
      for (int q = 0; q < kTargets; ++q) {
        const double dx = tq[q][0] - xj, dy = tq[q][1] - yj, dz = tq[q][2] - zj;
        const double r2 = dx * dx + dy * dy + dz * dz;
        if (r2 < cut2) {
          const int64_t i = t0 + q * kBlock + tid;
          if (r2 > 0.0 && j0 + jj != i && i < t1) {
            const double r = sqrt(r2);
            const double fm = r < d ? fmax_ : fmax_ * exp(-(r - d) * inv_b);
            const double sc = fm / r;
            f[q][0] += sc * dx;
            f[q][1] += sc * dy;
            f[q][2] += sc * dz;
          }
        }
      }
    }
  }
}

// Targets [t0, t1) (kBlock lanes x kTargets per workgroup) against sources [s0, s1).
__device__ __forceinline__ void steric_tile(const double *__restrict__ pos, int64_t t0, int64_t t1,
                                            int64_t s0, int64_t s1, double a, double u0, double b,
                                            double f_grav_z, double *__restrict__ force) {
  __shared__ double sx[kBlock], sy[kBlock], sz[kBlock];
  const int tid = threadIdx.x;
  double f[kTargets][3], tq[kTargets][3];
#pragma unroll
  for (int q = 0; q < kTargets; ++q) {
    const int64_t i = t0 + q * kBlock + tid;
    const int64_t ii = i < t1 ? i : t0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      tq[q][c] = pos[3 * ii + c];
      f[q][c] = 0.0;
    }
  }
  steric_block(pos, t0, t1, s0, s1, a, u0, b, f, tq, sx, sy, sz);
  const double fmax_ = u0 / b;
#pragma unroll
  for (int q = 0; q < kTargets; ++q) {
    const int64_t i = t0 + q * kBlock + tid;
    if (i < t1) {
      const double zi = tq[q][2];
      const double fw = zi < a ? fmax_ : fmax_ * exp(-(zi - a) / b);
      force[3 * i] = f[q][0];
      force[3 * i + 1] = f[q][1];
      force[3 * i + 2] = f[q][2] + fw + f_grav_z;
    }
  }
}

__global__ __launch_bounds__(kBlock) void steric_kernel(int64_t n, const double *__restrict__ pos,
                                                        double a, double u0, double b,
                                                        double f_grav_z,
                                                        double *__restrict__ force) {
  const int64_t t0 = int64_t(blockIdx.x) * kBlock * kTargets;
  steric_tile(pos, t0, n, 0, n, a, u0, b, f_grav_z, force);
}

// One workgroup per (system, tile of kBlock targets) item; each workgroup covers up to
// kBlock * kTargets targets, so only the items with tile % kTargets == 0 do work.
__global__ __launch_bounds__(kBlock) void steric_kernel_batched(const int64_t *__restrict__ offs,
                                                                const int2 *__restrict__ tiles,
                                                                const double *__restrict__ pos,
                                                                double a, double u0, double b,
                                                                double f_grav_z,
                                                                double *__restrict__ force) {
  const int2 tl = tiles[blockIdx.x];
  if (tl.y % kTargets != 0) return;
  const int64_t s0 = offs[tl.x], s1 = offs[tl.x + 1];
  steric_tile(pos, s0 + int64_t(tl.y) * kBlock, s1, s0, s1, a, u0, b, f_grav_z, force);
}

}  // namespace

int forces_batched_run(rpb_ctx *ctx, const rpb_params *p, const Batch &bt, const double *pos,
                       double f_grav_z, double u0, double b, double *force, hipStream_t stream) {
  if (bt.ntiles <= 0) return RPB_OK;
  steric_kernel_batched<<<unsigned(bt.ntiles), kBlock, 0, stream>>>(bt.offs, bt.tiles, pos, p->a,
                                                                    u0, b, f_grav_z, force);
  RPB_LAUNCHED(ctx);
  return RPB_OK;
}

int forces_run(rpb_ctx *ctx, const rpb_params *p, int64_t n, const double *pos, double f_grav_z,
               double u0, double b, double *force, hipStream_t stream) {
  if (n <= 0) return RPB_OK;
  const int64_t per = int64_t(kBlock) * kTargets;
  steric_kernel<<<unsigned((n + per - 1) / per), kBlock, 0, stream>>>(n, pos, p->a, u0, b,
                                                                      f_grav_z, force);
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
