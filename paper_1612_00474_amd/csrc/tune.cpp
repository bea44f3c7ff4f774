// Launch-shape tuner for the pair kernels.
//
// Candidates (targets per lane, symmetric or ordered evaluation, source split / work-item size,
// workgroup count) are timed with HIP events on the caller's configuration and the fastest is
// kept in the context; single-system and batched products have fields of their own.  Results
// are cached per (precision, single or batched, log2 of the sphere count), so a later call
// with a similar problem reuses the choice without timing.
#include <cmath>
#include <vector>

#include "rpb_internal.h"

namespace rpb {

namespace {

using Key = std::tuple<int, int, int>;   // precision, batched, log2(n)

std::map<Key, Tuning> &cache(rpb_ctx *ctx) { return ctx->tune_cache; }

int time_candidate(rpb_ctx *ctx, const rpb_params *p, int32_t nsys, const int64_t *offs,
                   const double *pos, int reps, hipStream_t stream, double *ms_out) {
  const int64_t n = offs[nsys];
  int st;
  double *vel =
      static_cast<double *>(workspace(ctx, WS_VEC_A, size_t(3 * n) * sizeof(double), &st));
  if (!vel) return st;
  Packed g;
  RPB_TRY(pack_geometry(ctx, p, n, pos, WS_GEOM, &g, stream));
  Batch b;
  if (nsys > 1) RPB_TRY(prepare_batch(ctx, nsys, offs, p->precision, &b, stream));
  // the positions serve as a finite source vector: only the time matters here
  auto once = [&]() -> int {
    return nsys > 1 ? matvec_batched(ctx, p, b, g, pos, nullptr, nullptr, vel, stream)
                    : matvec_packed(ctx, p, g, pos, nullptr, 0, n, vel, stream);
  };
  RPB_TRY(once());
  hipEvent_t e0, e1;
  RPB_HIP(ctx, hipEventCreate(&e0));
  RPB_HIP(ctx, hipEventCreate(&e1));
  int rc = hipEventRecord(e0, stream) == hipSuccess ? RPB_OK : RPB_EDEVICE;
  for (int r = 0; r < reps && rc == RPB_OK; ++r) rc = once();
  float ms = 0.0f;
  if (rc == RPB_OK && (hipEventRecord(e1, stream) != hipSuccess ||
                       hipEventSynchronize(e1) != hipSuccess ||
                       hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
    rc = fail(ctx, RPB_EDEVICE, "tuning timer failed");
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *ms_out = ms / reps;
  return rc;
}

}  // namespace

}  // namespace rpb

using namespace rpb;

extern "C" {

int rpb_get_tuning(const rpb_ctx *ctx, rpb_tuning *out) {
  if (!ctx || !out) return RPB_EINVAL;
  rpb_shape *dst[2] = {&out->fp64, &out->mixed};
  for (int q = 0; q < 2; ++q) {
    const Shape &v = ctx->tune.s[q];
    *dst[q] = rpb_shape{v.tpt,       v.target_wgs, v.batch_chunk,    v.batch_wgs,
                        v.symmetric, v.batch_tpt,  v.batch_symmetric};
  }
  return RPB_OK;
}

int rpb_set_tuning(rpb_ctx *ctx, const rpb_tuning *t) {
  if (!ctx || !t) return RPB_EINVAL;
  const rpb_shape *src[2] = {&t->fp64, &t->mixed};
  for (int q = 0; q < 2; ++q) {
    const rpb_shape &v = *src[q];
    if ((v.tpt != 1 && v.tpt != 2 && v.tpt != 4) || v.target_wgs < 1 || v.target_wgs > (1 << 20) ||
        v.batch_chunk < 256 || v.batch_chunk % 256 != 0 || v.batch_chunk > (1 << 20) ||
        v.batch_wgs < 1 || v.batch_wgs > (1 << 20) || (v.symmetric != 0 && v.symmetric != 1) ||
        (v.batch_tpt != 1 && v.batch_tpt != 2) ||
        (v.batch_symmetric != 0 && v.batch_symmetric != 1))
      return fail(ctx, RPB_EINVAL, "tuning values out of range");
  }
  for (int q = 0; q < 2; ++q) {
    const rpb_shape &v = *src[q];
    ctx->tune.s[q] = Shape{v.tpt,       v.target_wgs, v.batch_chunk,    v.batch_wgs,
                           v.symmetric, v.batch_tpt,  v.batch_symmetric};
  }
  return RPB_OK;
}

int rpb_autotune(rpb_ctx *ctx, const rpb_params *p, int32_t nsys, const int64_t *offs,
                 const double *pos, int reps, rpb_tuning *out, double *best_ms_out,
                 rpb_stream_t stream_) {
  RPB_TRY(check_params(ctx, p));
  RPB_TRY(check_offsets(ctx, nsys, offs));
  if (nsys > 1 && p->lx > 0.0)
    return fail(ctx, RPB_EINVAL, "pseudo-periodic boundaries are supported for single systems");
  if (reps < 1 || reps > 100) return fail(ctx, RPB_EINVAL, "reps must be in [1, 100]");
  const int64_t n = offs[nsys];
  if (n == 0) return fail(ctx, RPB_EINVAL, "nothing to tune");
  if (!pos) return fail(ctx, RPB_EINVAL, "pos must not be NULL");
  hipStream_t stream = static_cast<hipStream_t>(stream_);
  RPB_HIP(ctx, hipSetDevice(ctx->device));
  RPB_TRY(check_finite(ctx, pos, n, stream));
  const bool batched = nsys > 1;
  const int q = p->precision == RPB_FP64 ? RPB_FP64 : RPB_MIXED;
  const Key key{q, batched ? 1 : 0, int(std::floor(std::log2(double(n))))};
  auto &tab = cache(ctx);
  double best_ms = -1.0;
  auto it = tab.find(key);
  if (it != tab.end()) {
    ctx->tune.s[q] = it->second.s[q];
  } else {
    const Shape base = ctx->tune.s[q];
    const bool timing = ctx->timing;
    ctx->timing = false;
    Shape best = base;
    std::vector<Shape> cands;
    for (int tpt : {1, 2}) {
      // a system within one tile of 256 targets (one per lane of a 256-lane workgroup): two
      // targets per lane would leave half of each lane's targets empty
      if (!batched && tpt == 2 && n <= 256) continue;
      if (batched) {
        for (int wgs : {1024, 2048, 4096}) {
          Shape c = base;
          c.batch_tpt = tpt;
          c.batch_wgs = wgs;
          c.batch_symmetric = 1;
          cands.push_back(c);
          c.batch_symmetric = 0;
          for (int chunk : {512, 1024, 2048}) {
            c.batch_chunk = chunk;
            cands.push_back(c);
          }
        }
      } else {
        Shape c = base;
        c.tpt = tpt;
        c.symmetric = 1;
        cands.push_back(c);
        c.symmetric = 0;
        for (int wgs : {2048, 4096, 8192, 16384}) {
          c.target_wgs = wgs;
          cands.push_back(c);
        }
      }
    }
    if (!batched && n >= 4 * 1024) {   // 4 targets per lane: tiles of 1,024 spheres, symmetric
      // kernel only; on smaller systems most of a tile's lanes would idle
      Shape c = base;
      c.tpt = 4;
      c.symmetric = 1;
      cands.push_back(c);
    }
    int rc = RPB_OK;
    for (const Shape &sh : cands) {
      ctx->tune.s[q] = sh;
      double ms = 0.0;
      rc = time_candidate(ctx, p, nsys, offs, pos, reps, stream, &ms);
      if (rc != RPB_OK) break;
      if (best_ms < 0.0 || ms < best_ms) {
        best_ms = ms;
        best = sh;
      }
    }
    ctx->timing = timing;
    ctx->tune.s[q] = rc == RPB_OK ? best : base;
    if (rc != RPB_OK) return rc;
    tab[key] = ctx->tune;
  }
  if (best_ms_out) *best_ms_out = best_ms;
  return rpb_get_tuning(ctx, out);
}

}  // extern "C"
