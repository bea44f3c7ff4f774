// Context, workspace, error reporting and timing for librpb.
#include <cmath>
#include <cstdarg>
#include <cstdlib>
#include <cstring>

#include "rpb_internal.h"

namespace rpb {

int fail(rpb_ctx *ctx, int code, const char *fmt, ...) {
  if (ctx) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    ctx->err = buf;
  }
  return code;
}

void *workspace(rpb_ctx *ctx, Slot slot, size_t bytes, int *status) {
  DevBuf &b = ctx->ws[slot];
  *status = RPB_OK;
  if (bytes <= b.bytes && b.ptr) return b.ptr;
  // growth: earlier work on any stream may still use the old buffer
  if (b.ptr) {
    if (hipDeviceSynchronize() != hipSuccess || hipFree(b.ptr) != hipSuccess) {
      *status = fail(ctx, RPB_EDEVICE, "workspace release failed");
      return nullptr;
    }
    b.ptr = nullptr;
    b.bytes = 0;
  }
  size_t want = bytes < 4096 ? 4096 : bytes;
  want = (want + 4095) & ~size_t(4095);
  if (hipMalloc(&b.ptr, want) != hipSuccess) {
    (void)hipGetLastError();
    b.ptr = nullptr;
    *status = fail(ctx, RPB_ENOMEM, "hipMalloc of %zu bytes failed (workspace slot %d)", want,
                   int(slot));
    return nullptr;
  }
  b.bytes = want;
  return b.ptr;
}

int check_params(rpb_ctx *ctx, const rpb_params *p) {
  if (!ctx) return RPB_EINVAL;
  if (!p) return fail(ctx, RPB_EINVAL, "params is NULL");
  if (!(p->a > 0.0) || !(p->eta > 0.0) || !(p->kT > 0.0))
    return fail(ctx, RPB_EINVAL, "a, eta and kT must be positive (got %g, %g, %g)", p->a, p->eta,
                p->kT);
  if (p->precision != RPB_FP64 && p->precision != RPB_MIXED)
    return fail(ctx, RPB_EINVAL, "unknown precision %d", p->precision);
  if (p->wall != 0 && p->wall != 1) return fail(ctx, RPB_EINVAL, "wall must be 0 or 1");
  const bool box = p->lx > 0.0 && p->ly > 0.0 && std::isfinite(p->lx) && std::isfinite(p->ly);
  if (!box && !(p->lx == 0.0 && p->ly == 0.0))
    return fail(ctx, RPB_EINVAL, "box lengths must both be positive and finite, or both 0");
  return RPB_OK;
}

bool overlaps(const void *a, size_t abytes, const void *b, size_t bbytes) {
  if (!a || !b) return false;
  const char *pa = static_cast<const char *>(a);
  const char *pb = static_cast<const char *>(b);
  return pa < pb + bbytes && pb < pa + abytes;
}

int timing_begin(rpb_ctx *ctx, hipStream_t stream, hipEvent_t *start) {
  *start = nullptr;
  if (!ctx->timing) return RPB_OK;
  hipEvent_t e;
  if (!ctx->ev_pool.empty()) {
    e = ctx->ev_pool.back();
    ctx->ev_pool.pop_back();
  } else {
    RPB_HIP(ctx, hipEventCreate(&e));
  }
  RPB_HIP(ctx, hipEventRecord(e, stream));
  *start = e;
  return RPB_OK;
}

int timing_end(rpb_ctx *ctx, hipStream_t stream, hipEvent_t start, double pairs, int kind) {
  if (!ctx->timing || !start) return RPB_OK;
  hipEvent_t e;
  if (!ctx->ev_pool.empty()) {
    e = ctx->ev_pool.back();
    ctx->ev_pool.pop_back();
  } else {
    RPB_HIP(ctx, hipEventCreate(&e));
  }
  RPB_HIP(ctx, hipEventRecord(e, stream));
  ctx->ev_start.push_back(start);
  ctx->ev_stop.push_back(e);
  ctx->ev_pairs.push_back(pairs);
  ctx->ev_kind.push_back(kind);
  return RPB_OK;
}

void timing_discard(rpb_ctx *ctx, size_t first) {
  for (size_t i = first; i < ctx->ev_start.size(); ++i) {
    ctx->ev_pool.push_back(ctx->ev_start[i]);
    ctx->ev_pool.push_back(ctx->ev_stop[i]);
  }
  if (first < ctx->ev_start.size()) {
    ctx->ev_start.resize(first);
    ctx->ev_stop.resize(first);
    ctx->ev_pairs.resize(first);
    ctx->ev_kind.resize(first);
  }
}

}  // namespace rpb

using namespace rpb;

extern "C" {

const char *rpb_version(void) { return "librpb 0.1 (gfx950)"; }

int rpb_create(int hip_device, rpb_ctx **out) {
  if (!out) return RPB_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || hip_device < 0 || hip_device >= ndev)
    return RPB_EDEVICE;
  if (hipSetDevice(hip_device) != hipSuccess) return RPB_EDEVICE;
  rpb_ctx *c = new (std::nothrow) rpb_ctx();
  if (!c) return RPB_ENOMEM;
  c->device = hip_device;
  // launch-shape overrides for experiments:
  // RPB_<FP64|MIXED>_<TPT|WGS|CHUNK|BWGS|SYM|BTPT|BSYM>
  const char *pre[2] = {"RPB_FP64_", "RPB_MIXED_"};
  for (int q = 0; q < 2; ++q) {
    auto env = [&](const char *key, int lo, int hi, int mult, int *dst) {
      const std::string name = std::string(pre[q]) + key;
      if (const char *v = getenv(name.c_str())) {
        const int w = atoi(v);
        if (w >= lo && w <= hi && w % mult == 0) *dst = w;
      }
    };
    Shape &sh = c->tune.s[q];
    env("TPT", 1, 4, 1, &sh.tpt);
    if (sh.tpt == 3) sh.tpt = 2;
    env("WGS", 1, 1 << 20, 1, &sh.target_wgs);
    env("CHUNK", 256, 1 << 20, 256, &sh.batch_chunk);
    env("BWGS", 1, 1 << 20, 1, &sh.batch_wgs);
    env("SYM", 0, 1, 1, &sh.symmetric);
    env("BTPT", 1, 2, 1, &sh.batch_tpt);
    env("BSYM", 0, 1, 1, &sh.batch_symmetric);
  }
  if (const char *v = getenv("RPB_CHUNK_KIB")) {   // partial-sum chunk limit, for experiments
    const long long kib = atoll(v);
    if (kib >= 1 && kib <= (1ll << 30)) c->chunk_bytes = size_t(kib) << 10;
  }
  if (hipHostMalloc(&c->host_pinned, kHostScratchBytes, hipHostMallocDefault) != hipSuccess) {
    delete c;
    return RPB_ENOMEM;
  }
  if (hipHostGetDevicePointer(&c->host_pinned_dev, c->host_pinned, 0) != hipSuccess) {
    (void)hipHostFree(c->host_pinned);
    delete c;
    return RPB_EDEVICE;
  }
  if (noalloc_setup(c, hip_device) != RPB_OK) {
    (void)hipHostFree(c->host_pinned);
    delete c;
    return RPB_EDEVICE;
  }
  bool ok = hipStreamCreateWithFlags(&c->lz_stream, hipStreamNonBlocking) == hipSuccess &&
            hipEventCreateWithFlags(&c->lz_join_ev, hipEventDisableTiming) == hipSuccess;
  for (auto &e : c->lz_vec_ev)
    ok = ok && hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess;
  if (!ok) {
    rpb_destroy(c);
    return RPB_EDEVICE;
  }
  *out = c;
  return RPB_OK;
}

void rpb_destroy(rpb_ctx *ctx) {
  if (!ctx) return;
  lz_helper_destroy(ctx);
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  for (auto &b : ctx->ws)
    if (b.ptr) (void)hipFree(b.ptr);
  for (auto e : ctx->ev_start) (void)hipEventDestroy(e);
  for (auto e : ctx->ev_stop) (void)hipEventDestroy(e);
  for (auto e : ctx->ev_pool) (void)hipEventDestroy(e);
  for (auto e : ctx->lz_ev)
    if (e) (void)hipEventDestroy(e);
  for (auto e : ctx->lz_vec_ev)
    if (e) (void)hipEventDestroy(e);
  if (ctx->lz_join_ev) (void)hipEventDestroy(ctx->lz_join_ev);
  if (ctx->lz_stream) (void)hipStreamDestroy(ctx->lz_stream);
  if (ctx->fin_ev) (void)hipEventDestroy(ctx->fin_ev);
  if (ctx->host_pinned) (void)hipHostFree(ctx->host_pinned);
  if (ctx->batch_host) (void)hipHostFree(ctx->batch_host);
  delete ctx;
}

const char *rpb_last_error(const rpb_ctx *ctx) { return ctx ? ctx->err.c_str() : "no context"; }

int rpb_output_check_enable(rpb_ctx *ctx, int enable) {
  if (!ctx) return RPB_EINVAL;
  ctx->check_output = enable != 0;
  return RPB_OK;
}

int rpb_timing_enable(rpb_ctx *ctx, int enable) {
  if (!ctx) return RPB_EINVAL;
  ctx->timing = enable != 0;
  return RPB_OK;
}

int rpb_timing_read(rpb_ctx *ctx, int kind, double *ms_out, int64_t *launches_out,
                    double *pairs_out) {
  if (!ctx) return RPB_EINVAL;
  double ms = 0.0, pairs = 0.0;
  int64_t k = 0;
  std::vector<hipEvent_t> keep_start, keep_stop;
  std::vector<double> keep_pairs;
  std::vector<int> keep_kind;
  for (size_t i = 0; i < ctx->ev_start.size(); ++i) {
    if (kind >= 0 && ctx->ev_kind[i] != kind) {
      keep_start.push_back(ctx->ev_start[i]);
      keep_stop.push_back(ctx->ev_stop[i]);
      keep_pairs.push_back(ctx->ev_pairs[i]);
      keep_kind.push_back(ctx->ev_kind[i]);
      continue;
    }
    RPB_HIP(ctx, hipEventSynchronize(ctx->ev_stop[i]));
    float t = 0.0f;
    RPB_HIP(ctx, hipEventElapsedTime(&t, ctx->ev_start[i], ctx->ev_stop[i]));
    ms += t;
    pairs += ctx->ev_pairs[i];
    ++k;
    ctx->ev_pool.push_back(ctx->ev_start[i]);
    ctx->ev_pool.push_back(ctx->ev_stop[i]);
  }
  ctx->ev_start.swap(keep_start);
  ctx->ev_stop.swap(keep_stop);
  ctx->ev_pairs.swap(keep_pairs);
  ctx->ev_kind.swap(keep_kind);
  if (ms_out) *ms_out = ms;
  if (launches_out) *launches_out = k;
  if (pairs_out) *pairs_out = pairs;
  return RPB_OK;
}

}  // extern "C"
