// Random numbers and the random finite difference for the stochastic drift.
//
// Normals: Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11) keyed by (seed, stream id) on
// the counter (block, step, 0, 0); each block yields four uniforms
// u = ((x >> 12) + 1/2) 2^-52 in (0, 1) and Box-Muller turns (u0, u1), (u2, u3) into four
// normals.  A time step is therefore reproducible from (seed, step) alone.
//
// Drift (paper, Sec. II.A, last term of eq. EM and eq. AB): the centred random finite
// difference (kT/delta)[M(q + delta/2 W~) W~ - M(q - delta/2 W~) W~], two products at
// shifted configurations (geometry packed twice), then one elementwise difference.
#include <cmath>

#include "rpb_internal.h"

namespace rpb {

namespace {

constexpr uint64_t kPhiloxM0 = 0xD2E7470EE14C6C93ull;
constexpr uint64_t kPhiloxM1 = 0xCA5A826395121157ull;
constexpr uint64_t kWeyl0 = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kWeyl1 = 0xBB67AE8584CAA73Bull;

__device__ __forceinline__ void philox4x64_10(uint64_t x[4], uint64_t k0, uint64_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t lo0 = kPhiloxM0 * x[0], hi0 = __umul64hi(kPhiloxM0, x[0]);
    const uint64_t lo1 = kPhiloxM1 * x[2], hi1 = __umul64hi(kPhiloxM1, x[2]);
    const uint64_t y0 = hi1 ^ x[1] ^ k0, y2 = hi0 ^ x[3] ^ k1;
    x[0] = y0;
    x[1] = lo1;
    x[2] = y2;
    x[3] = lo0;
    k0 += kWeyl0;
    k1 += kWeyl1;
  }
}

__device__ __forceinline__ double to_uniform(uint64_t w) {
  return (double(w >> 12) + 0.5) * 0x1p-52;
}

__global__ void normals_kernel(int64_t count, uint64_t seed, uint64_t stream_id, uint64_t step,
                               double *__restrict__ out) {
  const int64_t b = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (4 * b >= count) return;
  uint64_t x[4] = {uint64_t(b), step, 0ull, 0ull};
  philox4x64_10(x, seed, stream_id);
  double v[4];
#pragma unroll
  for (int q = 0; q < 4; q += 2) {
    const double rad = sqrt(-2.0 * log(to_uniform(x[q])));
    double s, c;
    sincospi(2.0 * to_uniform(x[q + 1]), &s, &c);
    v[q] = rad * c;
    v[q + 1] = rad * s;
  }
#pragma unroll
  for (int q = 0; q < 4; ++q)
    if (4 * b + q < count) out[4 * b + q] = v[q];
}

__global__ void normals_kernel_devstep(int64_t count, uint64_t seed, uint64_t stream_id,
                                      const int64_t *__restrict__ step, double *__restrict__ out) {
  const int64_t b = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (4 * b >= count) return;
  uint64_t x[4] = {uint64_t(b), uint64_t(step[0]), 0ull, 0ull};
  philox4x64_10(x, seed, stream_id);
  double v[4];
#pragma unroll
  for (int q = 0; q < 4; q += 2) {
    const double rad = sqrt(-2.0 * log(to_uniform(x[q])));
    double s, c;
    sincospi(2.0 * to_uniform(x[q + 1]), &s, &c);
    v[q] = rad * c;
    v[q + 1] = rad * s;
  }
#pragma unroll
  for (int q = 0; q < 4; ++q)
    if (4 * b + q < count) out[4 * b + q] = v[q];
}

// q+ = q + sp w, q- = q - sm w: (delta/2, delta/2) for the centred difference, (delta, 0) for
// the one-sided one (q- = q exactly).
__global__ void shifted_pair(int64_t m, const double *__restrict__ q, const double *__restrict__ w,
                             double sp, double sm, double *__restrict__ qp,
                             double *__restrict__ qm) {
  // q +- s w with the product rounded before the sum (no fused multiply-add): the positions
  // then carry the rounding of the difference as it is written, which the drift divides by delta
#pragma clang fp contract(off)
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= m) return;
  qp[i] = q[i] + sp * w[i];
  qm[i] = q[i] - sm * w[i];
}

__global__ void scaled_difference(int64_t m, const double *__restrict__ a,
                                  const double *__restrict__ b, double s,
                                  double *__restrict__ out) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= m) return;
  out[i] = s * (a[i] - b[i]);
}

inline unsigned nblk(int64_t m) { return unsigned((m + 255) / 256); }

}  // namespace

int normals_run(rpb_ctx *ctx, int64_t count, uint64_t seed, uint64_t stream_id, uint64_t step,
                double *out, hipStream_t stream) {
  if (count <= 0) return RPB_OK;
  const int64_t blocks = (count + 3) / 4;
  normals_kernel<<<nblk(blocks), 256, 0, stream>>>(count, seed, stream_id, step, out);
  RPB_LAUNCHED(ctx);
  return RPB_OK;
}

int rfd_run(rpb_ctx *ctx, const rpb_params *p, int64_t n, const double *pos, const double *wt,
            double delta, int rfd_precision, bool one_sided, double *drift, hipStream_t stream,
            const double *base) {
  const int64_t m = 3 * n;
  const size_t vb = size_t(m) * sizeof(double);
  int st;
  double *qp = static_cast<double *>(workspace(ctx, WS_VEC_B, vb, &st));
  if (!qp) return st;
  double *qm = static_cast<double *>(workspace(ctx, WS_VEC_C, vb, &st));
  if (!qm) return st;
  double *up = static_cast<double *>(workspace(ctx, WS_VEC_D, vb, &st));
  if (!up) return st;
  double *um = static_cast<double *>(workspace(ctx, WS_VEC_E, vb, &st));
  if (!um) return st;
  shifted_pair<<<nblk(m), 256, 0, stream>>>(m, pos, wt, one_sided ? delta : 0.5 * delta,
                                             one_sided ? 0.0 : 0.5 * delta, qp, qm);
  RPB_LAUNCHED(ctx);
  rpb_params q = *p;
  q.precision = rfd_precision;
  Packed gp, gm;
  RPB_TRY(pack_geometry(ctx, &q, n, qp, WS_GEOM, &gp, stream));
  RPB_TRY(matvec_packed(ctx, &q, gp, wt, nullptr, 0, n, up, stream));
  if (!(one_sided && base)) {   // the product at q- (= q when one-sided)
    RPB_TRY(pack_geometry(ctx, &q, n, qm, WS_GEOM2, &gm, stream));
    RPB_TRY(matvec_packed(ctx, &q, gm, wt, nullptr, 0, n, um, stream));
    base = um;
  }
  scaled_difference<<<nblk(m), 256, 0, stream>>>(m, up, base, p->kT / delta, drift);
  RPB_LAUNCHED(ctx);
  return RPB_OK;
}

int normals_devstep_run(rpb_ctx *ctx, int64_t count, uint64_t seed, uint64_t stream_id,
                        const int64_t *step_dev, double *out, hipStream_t stream) {
  if (count <= 0) return RPB_OK;
  const int64_t blocks = (count + 3) / 4;
  normals_kernel_devstep<<<nblk(blocks), 256, 0, stream>>>(count, seed, stream_id, step_dev, out);
  RPB_LAUNCHED(ctx);
  return RPB_OK;
}

int rfd_batched_run(rpb_ctx *ctx, const rpb_params *p, const Batch &bt, const double *pos,
                    const double *wt, double delta, int rfd_precision, bool one_sided,
                    double *drift, hipStream_t stream) {
  const int64_t n = bt.n;
  const int64_t m = 3 * n;
  const size_t vb = size_t(m) * sizeof(double);
  int st;
  double *qp = static_cast<double *>(workspace(ctx, WS_VEC_B, vb, &st));
  if (!qp) return st;
  double *qm = static_cast<double *>(workspace(ctx, WS_VEC_C, vb, &st));
  if (!qm) return st;
  double *up = static_cast<double *>(workspace(ctx, WS_VEC_D, vb, &st));
  if (!up) return st;
  double *um = static_cast<double *>(workspace(ctx, WS_VEC_E, vb, &st));
  if (!um) return st;
  shifted_pair<<<nblk(m), 256, 0, stream>>>(m, pos, wt, one_sided ? delta : 0.5 * delta,
                                             one_sided ? 0.0 : 0.5 * delta, qp, qm);
  RPB_LAUNCHED(ctx);
  rpb_params q = *p;
  q.precision = rfd_precision;
  Packed gp, gm;
  RPB_TRY(pack_geometry(ctx, &q, n, qp, WS_GEOM, &gp, stream));
  RPB_TRY(pack_geometry(ctx, &q, n, qm, WS_GEOM2, &gm, stream));
  RPB_TRY(matvec_batched(ctx, &q, bt, gp, wt, nullptr, nullptr, up, stream));
  RPB_TRY(matvec_batched(ctx, &q, bt, gm, wt, nullptr, nullptr, um, stream));
  scaled_difference<<<nblk(m), 256, 0, stream>>>(m, up, um, p->kT / delta, drift);
  RPB_LAUNCHED(ctx);
  return RPB_OK;
}

}  // namespace rpb

using namespace rpb;

namespace {

int rfd_entry(rpb_ctx *ctx, const rpb_params *p, int64_t n, const double *pos,
              const double *w_tilde, double delta, int rfd_precision, bool one_sided,
              double *drift_out, rpb_stream_t stream_) {
  RPB_TRY(check_params(ctx, p));
  if (n < 0) return fail(ctx, RPB_EINVAL, "n must be >= 0");
  if (!(delta > 0.0)) return fail(ctx, RPB_EINVAL, "delta must be > 0");
  if (rfd_precision != RPB_FP64 && rfd_precision != RPB_MIXED)
    return fail(ctx, RPB_EINVAL, "unknown rfd_precision %d", rfd_precision);
  if (n == 0) return RPB_OK;
  if (!pos || !w_tilde || !drift_out)
    return fail(ctx, RPB_EINVAL, "pos, w_tilde and drift_out must not be NULL");
  const size_t nb = size_t(n) * 3 * sizeof(double);
  if (overlaps(drift_out, nb, pos, nb) || overlaps(drift_out, nb, w_tilde, nb))
    return fail(ctx, RPB_EINVAL, "drift_out overlaps an input");
  hipStream_t stream = static_cast<hipStream_t>(stream_);
  RPB_HIP(ctx, hipSetDevice(ctx->device));
  RPB_TRY(check_finite(ctx, pos, n, stream));
  RPB_TRY(rfd_run(ctx, p, n, pos, w_tilde, delta, rfd_precision, one_sided, drift_out, stream));
  return check_output(ctx, drift_out, 3 * n, stream, "the drift");
}

}  // namespace

extern "C" {

int rfd_drift(rpb_ctx *ctx, const rpb_params *p, int64_t n, const double *pos,
              const double *w_tilde, double delta, int rfd_precision, double *drift_out,
              rpb_stream_t stream) {
  return rfd_entry(ctx, p, n, pos, w_tilde, delta, rfd_precision, false, drift_out, stream);
}

int rfd_drift_one_sided(rpb_ctx *ctx, const rpb_params *p, int64_t n, const double *pos,
                        const double *w_tilde, double delta, int rfd_precision,
                        double *drift_out, rpb_stream_t stream) {
  return rfd_entry(ctx, p, n, pos, w_tilde, delta, rfd_precision, true, drift_out, stream);
}

int rpb_normals(rpb_ctx *ctx, int64_t count, uint64_t seed, uint64_t stream_id, uint64_t step,
                double *out, rpb_stream_t stream_) {
  if (!ctx) return RPB_EINVAL;
  if (count < 0) return fail(ctx, RPB_EINVAL, "count must be >= 0");
  if (count == 0) return RPB_OK;
  if (!out) return fail(ctx, RPB_EINVAL, "out must not be NULL");
  RPB_HIP(ctx, hipSetDevice(ctx->device));
  return normals_run(ctx, count, seed, stream_id, step, out, static_cast<hipStream_t>(stream_));
}

}  // extern "C"
