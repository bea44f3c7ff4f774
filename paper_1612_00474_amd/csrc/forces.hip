// Soft steric forces plus gravity (paper, Sec. III, eq. soft_potential).
//
// U(r) = U0 + U0 (d - r)/b for r < d and U0 exp(-(r - d)/b) for r >= d, with d = 2a and r
// the centre distance for sphere pairs, d = a and r = z for the wall; the force is -grad U,
// magnitude U0/b or (U0/b) exp(-(r - d)/b), repulsive.  Gravity adds f_g along z.  Pairs
// farther than d + 40 b are skipped (their force is below 4.3e-18 U0/b).  Brute-force
// O(N^2) distance tests over LDS tiles, float64 throughout; unclamped positions.
#include <cmath>

#include "rpb_internal.h"

namespace rpb {

namespace {

constexpr int kBlock = 256;

__global__ __launch_bounds__(kBlock) void steric_kernel(int64_t n, const double *__restrict__ pos,
                                                        double a, double u0, double b,
                                                        double f_grav_z,
                                                        double *__restrict__ force) {
  __shared__ double sx[kBlock], sy[kBlock], sz[kBlock];
  const int tid = threadIdx.x;
  const int64_t i = int64_t(blockIdx.x) * kBlock + tid;
  const bool active = i < n;
  const int64_t ii = active ? i : 0;
  const double xi = pos[3 * ii], yi = pos[3 * ii + 1], zi = pos[3 * ii + 2];
  const double d = 2.0 * a;
  const double cut = d + 40.0 * b;
  const double cut2 = cut * cut;
  const double fmax_ = u0 / b;
  const double inv_b = 1.0 / b;
  double fx = 0.0, fy = 0.0, fz = 0.0;
  for (int64_t t0 = 0; t0 < n; t0 += kBlock) {
    const int cnt = int(min<int64_t>(kBlock, n - t0));
    __syncthreads();
    if (tid < cnt) {
      const int64_t j = t0 + tid;
      sx[tid] = pos[3 * j];
      sy[tid] = pos[3 * j + 1];
      sz[tid] = pos[3 * j + 2];
    }
    __syncthreads();
    for (int jj = 0; jj < cnt; ++jj) {
      const double dx = xi - sx[jj], dy = yi - sy[jj], dz = zi - sz[jj];
      const double r2 = dx * dx + dy * dy + dz * dz;
      if (r2 < cut2 && r2 > 0.0 && t0 + jj != ii) {
        const double r = sqrt(r2);
        const double f = r < d ? fmax_ : fmax_ * exp(-(r - d) * inv_b);
        const double s = f / r;
        fx += s * dx;
        fy += s * dy;
        fz += s * dz;
      }
    }
  }
  if (active) {
    const double fw = zi < a ? fmax_ : fmax_ * exp(-(zi - a) * inv_b);
    force[3 * i] = fx;
    force[3 * i + 1] = fy;
    force[3 * i + 2] = fz + fw + f_grav_z;
  }
}

// One workgroup per (system, 256-target tile); sources are the system's own spheres.
__global__ __launch_bounds__(kBlock) void steric_kernel_batched(const int64_t *__restrict__ offs,
                                                                const int2 *__restrict__ tiles,
                                                                const double *__restrict__ pos,
                                                                double a, double u0, double b,
                                                                double f_grav_z,
                                                                double *__restrict__ force) {
  __shared__ double sx[kBlock], sy[kBlock], sz[kBlock];
  const int2 tl = tiles[blockIdx.x];
  const int64_t s0 = offs[tl.x], s1 = offs[tl.x + 1];
  const int tid = threadIdx.x;
  const int64_t i = s0 + int64_t(tl.y) * kBlock + tid;
  const bool active = i < s1;
  const int64_t ii = active ? i : s0;
  const double xi = pos[3 * ii], yi = pos[3 * ii + 1], zi = pos[3 * ii + 2];
  const double d = 2.0 * a;
  const double cut = d + 40.0 * b;
  const double cut2 = cut * cut;
  const double fmax_ = u0 / b;
  const double inv_b = 1.0 / b;
  double fx = 0.0, fy = 0.0, fz = 0.0;
  for (int64_t t0 = s0; t0 < s1; t0 += kBlock) {
    const int cnt = int(min<int64_t>(kBlock, s1 - t0));
    __syncthreads();
    if (tid < cnt) {
      const int64_t j = t0 + tid;
      sx[tid] = pos[3 * j];
      sy[tid] = pos[3 * j + 1];
      sz[tid] = pos[3 * j + 2];
    }
    __syncthreads();
    for (int jj = 0; jj < cnt; ++jj) {
      const double dx = xi - sx[jj], dy = yi - sy[jj], dz = zi - sz[jj];
      const double r2 = dx * dx + dy * dy + dz * dz;
      if (r2 < cut2 && r2 > 0.0 && t0 + jj != ii) {
        const double r = sqrt(r2);
        const double f = r < d ? fmax_ : fmax_ * exp(-(r - d) * inv_b);
        const double sc = f / r;
        fx += sc * dx;
        fy += sc * dy;
        fz += sc * dz;
      }
    }
  }
  if (active) {
    const double fw = zi < a ? fmax_ : fmax_ * exp(-(zi - a) * inv_b);
    force[3 * i] = fx;
    force[3 * i + 1] = fy;
    force[3 * i + 2] = fz + fw + f_grav_z;
  }
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
  steric_kernel<<<unsigned((n + kBlock - 1) / kBlock), kBlock, 0, stream>>>(n, pos, p->a, u0, b,
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
