// One batched time step captured in a hipGraph and replayed step after step.
//
// The graph owns a private context (its own workspace), so its baked-in device addresses are
// never reallocated by other calls.  It is created by
//   1. preparing the batch (work lists, offsets) and the device step record,
//   2. one warm-up step on scratch copies of the state, which sizes every workspace slot,
//   3. capturing step_batched_enqueue with a fixed Lanczos budget (device-side freezing of the
//      converged systems, no host synchronisation) on a private stream.
// Each launch advances the caller's positions and stored velocities by one step and the
// device step counter by one; the noise is drawn on the device from (seed, step).
#include <cstring>

#include "rpb_internal.h"

struct rpb_graph {
  rpb_ctx *ctx = nullptr;        // private context
  hipStream_t cap = nullptr;     // capture stream
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  rpb::Batch batch;
  void *rec = nullptr;           // device StepRecord
  int nsys = 0;
};

namespace {

using namespace rpb;

void destroy_graph(rpb_graph *g) {
  if (!g) return;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  if (g->cap) (void)hipStreamDestroy(g->cap);
  if (g->ctx) rpb_destroy(g->ctx);
  delete g;
}

}  // namespace

extern "C" {

int rpb_step_graph_create(rpb_ctx *ctx, const rpb_params *p, const rpb_sab_config *cfg,
                          int32_t nsys, const int64_t *offs, double *pos, double *u_prev,
                          int64_t step, int have_prev, rpb_graph **out, rpb_stream_t stream_) {
  if (!out) return RPB_EINVAL;
  *out = nullptr;
  RPB_TRY(check_params(ctx, p));
  RPB_TRY(check_step_config(ctx, cfg));
  RPB_TRY(check_offsets(ctx, nsys, offs));
  if (p->lx > 0.0)
    return fail(ctx, RPB_EINVAL, "pseudo-periodic boundaries are supported for single systems");
  if (nsys > kMaxBatchSystems)
    return fail(ctx, RPB_EINVAL, "at most %d systems per batch", kMaxBatchSystems);
  const int64_t n = offs[nsys];
  if (n == 0) return fail(ctx, RPB_EINVAL, "empty batch");
  if (!pos || !u_prev) return fail(ctx, RPB_EINVAL, "pos and u_prev must not be NULL");
  const size_t nb = size_t(n) * 3 * sizeof(double);
  if (overlaps(pos, nb, u_prev, nb)) return fail(ctx, RPB_EINVAL, "pos overlaps u_prev");
  hipStream_t stream = static_cast<hipStream_t>(stream_);
  RPB_HIP(ctx, hipSetDevice(ctx->device));
  RPB_TRY(check_finite(ctx, pos, n, stream));
  RPB_HIP(ctx, hipStreamSynchronize(stream));

  rpb_graph *g = new (std::nothrow) rpb_graph();
  if (!g) return fail(ctx, RPB_ENOMEM, "graph allocation failed");
  int st = rpb_create(ctx->device, &g->ctx);
  if (st != RPB_OK) {
    destroy_graph(g);
    return fail(ctx, st, "private context creation failed");
  }
  g->ctx->tune = ctx->tune;
  g->nsys = nsys;
  rpb_ctx *c = g->ctx;
  auto bail = [&](int code) {
    const std::string msg = c->err;
    destroy_graph(g);
    return fail(ctx, code, "graph creation: %s", msg.c_str());
  };
  if (hipStreamCreateWithFlags(&g->cap, hipStreamNonBlocking) != hipSuccess)
    return bail(fail(c, RPB_EDEVICE, "stream creation failed"));

  st = prepare_batch(c, nsys, offs, p->precision, &g->batch, g->cap);
  if (st != RPB_OK) return bail(st);
  char *small = static_cast<char *>(workspace(c, WS_SMALL, kSmallBytes, &st));
  if (!small) return bail(st);
  g->rec = small + kSmallStepState;

  // warm-up on scratch copies of the state: sizes every workspace slot
  double *scratch = nullptr;
  if (hipMalloc(&scratch, 2 * nb) != hipSuccess) return bail(fail(c, RPB_ENOMEM, "scratch"));
  bool ok = hipMemcpyAsync(scratch, pos, nb, hipMemcpyDeviceToDevice, g->cap) == hipSuccess &&
            hipMemcpyAsync(scratch + 3 * n, u_prev, nb, hipMemcpyDeviceToDevice, g->cap) ==
                hipSuccess;
  st = ok ? set_step_state(c, g->rec, step, have_prev, g->cap) : RPB_EDEVICE;
  if (st == RPB_OK)
    st = step_batched_enqueue(c, p, cfg, g->batch, scratch, scratch + 3 * n, nullptr, nullptr,
                              g->rec, false, nullptr, g->cap);
  const bool synced = hipStreamSynchronize(g->cap) == hipSuccess;
  (void)hipFree(scratch);
  if (st != RPB_OK) return bail(st);
  if (!synced) return bail(fail(c, RPB_EDEVICE, "warm-up step failed"));

  // the step record restarts at the caller's step
  st = set_step_state(c, g->rec, step, have_prev, g->cap);
  if (st != RPB_OK) return bail(st);
  if (hipStreamSynchronize(g->cap) != hipSuccess)
    return bail(fail(c, RPB_EDEVICE, "synchronisation failed"));

  c->timing = false;
  if (hipStreamBeginCapture(g->cap, hipStreamCaptureModeThreadLocal) != hipSuccess)
    return bail(fail(c, RPB_EDEVICE, "hipStreamBeginCapture failed"));
  st = step_batched_enqueue(c, p, cfg, g->batch, pos, u_prev, nullptr, nullptr, g->rec, false,
                            nullptr, g->cap);
  hipGraph_t graph = nullptr;
  const hipError_t ec = hipStreamEndCapture(g->cap, &graph);
  g->graph = graph;
  if (st != RPB_OK) return bail(st);
  if (ec != hipSuccess || !graph) return bail(fail(c, RPB_EDEVICE, "hipStreamEndCapture failed"));
  if (hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0) != hipSuccess)
    return bail(fail(c, RPB_EDEVICE, "hipGraphInstantiate failed"));
  *out = g;
  return RPB_OK;
}

int rpb_step_graph_launch(rpb_graph *g, rpb_stream_t stream) {
  if (!g || !g->exec) return RPB_EINVAL;
  if (hipSetDevice(g->ctx->device) != hipSuccess) return RPB_EDEVICE;
  if (hipGraphLaunch(g->exec, static_cast<hipStream_t>(stream)) != hipSuccess)
    return fail(g->ctx, RPB_EDEVICE, "hipGraphLaunch failed");
  return RPB_OK;
}

int rpb_step_graph_status(rpb_graph *g, int64_t *step_out, int *iters_out, double *eps_out,
                          rpb_stream_t stream_) {
  if (!g) return RPB_EINVAL;
  rpb_ctx *c = g->ctx;
  hipStream_t stream = static_cast<hipStream_t>(stream_);
  RPB_HIP(c, hipStreamSynchronize(stream));
  LzStatus *host = static_cast<LzStatus *>(host_scratch(c));
  RPB_TRY(lanczos_batched_status_copy(c, g->nsys, host, g->cap));
  StepRecord rec;
  RPB_HIP(c, hipMemcpy(&rec, g->rec, sizeof rec, hipMemcpyDeviceToHost));
  if (step_out) *step_out = rec.step;
  for (int s = 0; s < g->nsys; ++s) {
    if (iters_out) iters_out[s] = host[s].m;
    if (eps_out) eps_out[s] = host[s].eps;
  }
  return lanczos_status_code(c, host, g->nsys);
}

void rpb_step_graph_destroy(rpb_graph *g) {
  if (!g) return;
  (void)hipSetDevice(g->ctx->device);
  (void)hipDeviceSynchronize();
  destroy_graph(g);
}

}  // extern "C"
