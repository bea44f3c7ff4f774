// One Brownian dynamics step (paper, Sec. II.A: eq. EM and the stochastic Adams-Bashforth
// scheme eq. AB; Sec. III for the constant driving torque and the soft potential).
//
//   F^n  = steric + gravity at q^n                       (forces.hip)
//   u^n  = M^n F^n + M_C^n T                             (matvec.hip, multi.hip)
//   g^n  ~ M^{n 1/2} W^n                                 (lanczos.hip)
//   D^n  = (kT/delta)[M(q^n + delta/2 W~) - M(q^n - delta/2 W~)] W~   (stochastic.hip)
//   q^{n+1} = q^n + dt (c0 u^n - c1 u^{n-1}) + sqrt(2 kT dt) g^n + dt D^n
// with (c0, c1) = (3/2, 1/2) for SAB after the first step and (1, 0) for EM or the first
// SAB step (no u^{-1} exists).  u^n is stored into the caller's u_prev for the next step.
// The products at q^n (u^n, the first Lanczos product M W^n and, for a one-sided RFD in the
// step's precision, M W~) share one multi-vector launch.
#include <cmath>

#include "rpb_internal.h"

namespace rpb {

namespace {

__global__ void fill_torque(int64_t n, double tx, double ty, double tz, double *__restrict__ t) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  t[3 * i] = tx;
  t[3 * i + 1] = ty;
  t[3 * i + 2] = tz;
}

__global__ void combine_kernel(int64_t m, double *__restrict__ pos, double *__restrict__ u_prev,
                               const double *__restrict__ u, const double *__restrict__ g,
                               const double *__restrict__ drift, double dt, double c0, double c1,
                               double noise) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const double ui = u[i];
  const double det = c1 != 0.0 ? c0 * ui - c1 * u_prev[i] : c0 * ui;
  pos[i] = pos[i] + dt * det + noise * g[i] + dt * drift[i];
  u_prev[i] = ui;
}

// Same update with the have-previous flag read from the device step record.
__global__ void combine_kernel_dev(int64_t m, double *__restrict__ pos, double *__restrict__ u_prev,
                                   const double *__restrict__ u, const double *__restrict__ g,
                                   const double *__restrict__ drift, double dt, int scheme,
                                   const StepRecord *__restrict__ rec, double noise) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const bool ab = scheme == 0 && rec->have_prev;
  const double ui = u[i];
  const double det = ab ? 1.5 * ui - 0.5 * u_prev[i] : ui;
  pos[i] = pos[i] + dt * det + noise * g[i] + dt * drift[i];
  u_prev[i] = ui;
}

__global__ void set_step_record(StepRecord *rec, int64_t step, int have_prev) {
  rec->step = step;
  rec->have_prev = have_prev;
}

__global__ void advance_step_record(StepRecord *rec) {
  rec->step += 1;
  rec->have_prev = 1;
}

inline unsigned nblk(int64_t m) { return unsigned((m + 255) / 256); }

}  // namespace

int step_batched_enqueue(rpb_ctx *ctx, const rpb_params *p, const rpb_sab_config *cfg,
                         const Batch &bt, double *pos, double *u_prev, const double *w,
                         const double *w_tilde, void *step_state, bool sync_lanczos,
                         LzStatus *status_host, hipStream_t stream) {
  const int64_t n = bt.n;
  const int64_t m3 = 3 * n;
  const size_t nb = size_t(n) * 3 * sizeof(double);
  StepRecord *rec = static_cast<StepRecord *>(step_state);
  int st;
  double *F = static_cast<double *>(workspace(ctx, WS_FORCE, nb, &st));
  if (!F) return st;
  double *T = static_cast<double *>(workspace(ctx, WS_TORQUE, nb, &st));
  if (!T) return st;
  double *u = static_cast<double *>(workspace(ctx, WS_VEC_F, nb, &st));
  if (!u) return st;
  double *g = static_cast<double *>(workspace(ctx, WS_VEC_G, nb, &st));
  if (!g) return st;
  double *drift = static_cast<double *>(workspace(ctx, WS_VEC_H, nb, &st));
  if (!drift) return st;
  const double *W = w;
  const double *Wt = w_tilde;
  if (!W) {
    double *buf = static_cast<double *>(workspace(ctx, WS_NOISE_W, nb, &st));
    if (!buf) return st;
    RPB_TRY(normals_devstep_run(ctx, m3, cfg->seed, 0, &rec->step, buf, stream));
    W = buf;
  }
  if (!Wt) {
    double *buf = static_cast<double *>(workspace(ctx, WS_NOISE_WT, nb, &st));
    if (!buf) return st;
    RPB_TRY(normals_devstep_run(ctx, m3, cfg->seed, 1, &rec->step, buf, stream));
    Wt = buf;
  }
  RPB_TRY(forces_batched_run(ctx, p, bt, pos, cfg->f_grav_z, cfg->steric_u0, cfg->steric_b, F,
                             stream));
  fill_torque<<<nblk(n), 256, 0, stream>>>(n, cfg->torque[0], cfg->torque[1], cfg->torque[2], T);
  RPB_LAUNCHED(ctx);
  Packed geo;
  RPB_TRY(pack_geometry(ctx, p, n, pos, WS_GEOM, &geo, stream));
  // M F + M_C T and the first Lanczos product M W of every system in one persistent launch
  double *mw = nullptr;
  if (cfg->lanczos_precond == 0 && matvec_first_batched_supported(p, bt)) {
    mw = static_cast<double *>(workspace(ctx, WS_VEC_B, nb, &st));
    if (!mw) return st;
    RPB_TRY(matvec_first_batched(ctx, p, bt, geo, F, T, W, u, mw, stream));
  } else {
    RPB_TRY(matvec_batched(ctx, p, bt, geo, F, T, nullptr, u, stream));
  }
  RPB_TRY(lanczos_batched_run(ctx, p, bt, geo, W, cfg->lanczos_tol, cfg->lanczos_max_iter,
                              cfg->lanczos_precond != 0, g, sync_lanczos, status_host, stream,
                              mw));
  RPB_TRY(rfd_batched_run(ctx, p, bt, pos, Wt, cfg->delta, cfg->rfd_precision,
                          cfg->rfd_scheme == 1, drift, stream));
  combine_kernel_dev<<<nblk(m3), 256, 0, stream>>>(m3, pos, u_prev, u, g, drift, cfg->dt,
                                                   cfg->scheme, rec,
                                                   std::sqrt(2.0 * p->kT * cfg->dt));
  RPB_LAUNCHED(ctx);
  advance_step_record<<<1, 1, 0, stream>>>(rec);
  RPB_LAUNCHED(ctx);
  return RPB_OK;
}

int set_step_state(rpb_ctx *ctx, void *step_state, int64_t step, int have_prev,
                   hipStream_t stream) {
  set_step_record<<<1, 1, 0, stream>>>(static_cast<StepRecord *>(step_state), step, have_prev);
  RPB_LAUNCHED(ctx);
  return RPB_OK;
}

int check_step_config(rpb_ctx *ctx, const rpb_sab_config *cfg) {
  if (!cfg) return fail(ctx, RPB_EINVAL, "cfg must not be NULL");
  if (!(cfg->dt > 0.0) || !(cfg->delta > 0.0) || !(cfg->lanczos_tol > 0.0))
    return fail(ctx, RPB_EINVAL, "dt, delta and lanczos_tol must be > 0");
  if (cfg->lanczos_max_iter < 1 || cfg->lanczos_max_iter > 64)
    return fail(ctx, RPB_EINVAL, "lanczos_max_iter must be in [1, 64]");
  if (cfg->scheme != 0 && cfg->scheme != 1) return fail(ctx, RPB_EINVAL, "unknown scheme");
  if (cfg->rfd_precision != RPB_FP64 && cfg->rfd_precision != RPB_MIXED)
    return fail(ctx, RPB_EINVAL, "unknown rfd_precision");
  if (cfg->rfd_scheme != 0 && cfg->rfd_scheme != 1)
    return fail(ctx, RPB_EINVAL, "unknown rfd_scheme");
  if (cfg->lanczos_precond != 0 && cfg->lanczos_precond != 1)
    return fail(ctx, RPB_EINVAL, "lanczos_precond must be 0 or 1");
  if (!(cfg->steric_u0 >= 0.0) || !(cfg->steric_b > 0.0))
    return fail(ctx, RPB_EINVAL, "need steric_u0 >= 0 and steric_b > 0");
  return RPB_OK;
}

}  // namespace rpb

using namespace rpb;

extern "C" int sab_step(rpb_ctx *ctx, const rpb_params *p, const rpb_sab_config *cfg,
                        rpb_sab_state *state, const double *w, const double *w_tilde,
                        int *iters_out, double *eps_out, rpb_stream_t stream_) {
  RPB_TRY(check_params(ctx, p));
  if (!cfg || !state) return fail(ctx, RPB_EINVAL, "cfg and state must not be NULL");
  RPB_TRY(check_step_config(ctx, cfg));
  const int64_t n = state->n;
  if (iters_out) *iters_out = 0;
  if (eps_out) *eps_out = 0.0;
  if (n < 0) return fail(ctx, RPB_EINVAL, "n must be >= 0");
  if (n == 0) return RPB_OK;
  if (!state->pos || !state->u_prev)
    return fail(ctx, RPB_EINVAL, "state->pos and state->u_prev must not be NULL");
  const size_t nb = size_t(n) * 3 * sizeof(double);
  if (overlaps(state->pos, nb, state->u_prev, nb) || overlaps(state->pos, nb, w, nb) ||
      overlaps(state->pos, nb, w_tilde, nb) || overlaps(state->u_prev, nb, w, nb) ||
      overlaps(state->u_prev, nb, w_tilde, nb))
    return fail(ctx, RPB_EINVAL, "state arrays overlap the noise arrays or each other");

  hipStream_t stream = static_cast<hipStream_t>(stream_);
  RPB_HIP(ctx, hipSetDevice(ctx->device));
  // The position check is read back only once the noise, the forces and the first product
  // are enqueued, so the device goes on from the previous call's work without a pause.
  // Those kernels index memory by sphere, tile and hashed (clamped) cell, never by a raw
  // position value, and write only workspace; the state changes after the check has passed.
  RPB_TRY(check_finite_begin(ctx, state->pos, n, stream));
  const int64_t m3 = 3 * n;
  int st;
  double *F = static_cast<double *>(workspace(ctx, WS_FORCE, nb, &st));
  if (!F) return st;
  double *T = static_cast<double *>(workspace(ctx, WS_TORQUE, nb, &st));
  if (!T) return st;
  double *u = static_cast<double *>(workspace(ctx, WS_VEC_F, nb, &st));
  if (!u) return st;
  double *g = static_cast<double *>(workspace(ctx, WS_VEC_G, nb, &st));
  if (!g) return st;
  double *drift = static_cast<double *>(workspace(ctx, WS_VEC_H, nb, &st));
  if (!drift) return st;

  // noise
  const double *W = w;
  const double *Wt = w_tilde;
  if (!W) {
    double *buf = static_cast<double *>(workspace(ctx, WS_NOISE_W, nb, &st));
    if (!buf) return st;
    RPB_TRY(normals_run(ctx, m3, cfg->seed, 0, uint64_t(state->step), buf, stream));
    W = buf;
  }
  if (!Wt) {
    double *buf = static_cast<double *>(workspace(ctx, WS_NOISE_WT, nb, &st));
    if (!buf) return st;
    RPB_TRY(normals_run(ctx, m3, cfg->seed, 1, uint64_t(state->step), buf, stream));
    Wt = buf;
  }

  // deterministic velocity
  RPB_TRY(forces_run(ctx, p, n, state->pos, cfg->f_grav_z, cfg->steric_u0, cfg->steric_b, F,
                     stream));
  fill_torque<<<nblk(n), 256, 0, stream>>>(n, cfg->torque[0], cfg->torque[1], cfg->torque[2], T);
  RPB_LAUNCHED(ctx);
  Packed geo;
  RPB_TRY(pack_geometry(ctx, p, n, state->pos, WS_GEOM, &geo, stream));
  // M F + M_C T, the first Lanczos product M W and, for the one-sided RFD in the step's own
  // precision, its product M W~ at q share the configuration: one launch evaluates each pair's
  // coefficients once for all of them.  That launch takes one workgroup per pair of 256-sphere
  // tiles; a system of a few tiles leaves most of the device idle, so there the products run
  // apart, each split over enough workgroups.
  constexpr int64_t kJointMinN = 4 * 256;
  double *mw = nullptr, *mwt = nullptr;
  const bool one_sided = cfg->rfd_scheme == 1;
  if (cfg->lanczos_precond == 0 && n > kJointMinN && matvec_first_supported(p, n)) {
    mw = static_cast<double *>(workspace(ctx, WS_VEC_B, nb, &st));
    if (!mw) return st;
    if (one_sided && cfg->rfd_precision == p->precision) {
      mwt = static_cast<double *>(workspace(ctx, WS_VEC_E, nb, &st));   // rfd_run's q- product
      if (!mwt) return st;
    }
    RPB_TRY(matvec_first(ctx, p, geo, F, T, W, mwt ? Wt : nullptr, u, mw, mwt, stream));
  } else {
    RPB_TRY(matvec_packed(ctx, p, geo, F, T, 0, n, u, stream));
  }

  RPB_TRY(check_finite_end(ctx));

  // Brownian increment (the last iterate is used if the tolerance is not met)
  int iters = 0;
  double eps = 0.0;
  const int lz = lanczos_run(ctx, p, geo, W, cfg->lanczos_tol, cfg->lanczos_max_iter,
                             cfg->lanczos_precond != 0, g, &iters, &eps, stream, mw);
  if (lz != RPB_OK && lz != RPB_ENOCONV) return lz;

  // stochastic drift
  RPB_TRY(rfd_run(ctx, p, n, state->pos, Wt, cfg->delta, cfg->rfd_precision, one_sided, drift,
                  stream, mwt));

  const bool ab = cfg->scheme == 0 && state->have_prev;
  combine_kernel<<<nblk(m3), 256, 0, stream>>>(m3, state->pos, state->u_prev, u, g, drift,
                                               cfg->dt, ab ? 1.5 : 1.0, ab ? 0.5 : 0.0,
                                               std::sqrt(2.0 * p->kT * cfg->dt));
  RPB_LAUNCHED(ctx);
  state->step += 1;
  state->have_prev = 1;
  if (iters_out) *iters_out = iters;
  if (eps_out) *eps_out = eps;
  RPB_TRY(check_output(ctx, state->pos, m3, stream, "the new positions"));
  return lz;
}

extern "C" int sab_step_batched(rpb_ctx *ctx, const rpb_params *p, const rpb_sab_config *cfg,
                                int32_t nsys, const int64_t *offs, double *pos, double *u_prev,
                                int64_t step, int have_prev, const double *w,
                                const double *w_tilde, int *iters_out, double *eps_out,
                                rpb_stream_t stream_) {
  RPB_TRY(check_params(ctx, p));
  RPB_TRY(check_step_config(ctx, cfg));
  RPB_TRY(check_offsets(ctx, nsys, offs));
  if (p->lx > 0.0)
    return fail(ctx, RPB_EINVAL, "pseudo-periodic boundaries are supported for single systems");
  if (nsys > kMaxBatchSystems)
    return fail(ctx, RPB_EINVAL, "at most %d systems per batch", kMaxBatchSystems);
  const int64_t n = offs[nsys];
  for (int s = 0; s < nsys; ++s) {
    if (iters_out) iters_out[s] = 0;
    if (eps_out) eps_out[s] = 0.0;
  }
  if (n == 0) return RPB_OK;
  if (!pos || !u_prev) return fail(ctx, RPB_EINVAL, "pos and u_prev must not be NULL");
  const size_t nb = size_t(n) * 3 * sizeof(double);
  if (overlaps(pos, nb, u_prev, nb) || overlaps(pos, nb, w, nb) || overlaps(pos, nb, w_tilde, nb) ||
      overlaps(u_prev, nb, w, nb) || overlaps(u_prev, nb, w_tilde, nb))
    return fail(ctx, RPB_EINVAL, "state arrays overlap the noise arrays or each other");
  hipStream_t stream = static_cast<hipStream_t>(stream_);
  RPB_HIP(ctx, hipSetDevice(ctx->device));
  RPB_TRY(check_finite(ctx, pos, n, stream));
  Batch bt;
  RPB_TRY(prepare_batch(ctx, nsys, offs, p->precision, &bt, stream));
  int st;
  char *small = static_cast<char *>(workspace(ctx, WS_SMALL, kSmallBytes, &st));
  if (!small) return st;
  void *rec = small + kSmallStepState;
  RPB_TRY(set_step_state(ctx, rec, step, have_prev, stream));
  LzStatus *stat = static_cast<LzStatus *>(host_scratch(ctx));
  RPB_TRY(step_batched_enqueue(ctx, p, cfg, bt, pos, u_prev, w, w_tilde, rec, true, stat, stream));
  RPB_HIP(ctx, hipStreamSynchronize(stream));
  for (int s = 0; s < nsys; ++s) {
    if (iters_out) iters_out[s] = stat[s].m;
    if (eps_out) eps_out[s] = stat[s].eps;
  }
  const int code = lanczos_status_code(ctx, stat, nsys);
  return code == RPB_ENOCONV ? RPB_ENOCONV : code;
}
