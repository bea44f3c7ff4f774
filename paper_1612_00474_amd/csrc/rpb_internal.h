// Internal declarations shared by the librpb translation units (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "rpb.h"

namespace rpb {

// Workspace slots owned by a context.  Each slot is one device allocation that grows
// on demand; slots never alias, so a driver can hold several at once.
enum Slot {
  WS_GEOM = 0,      // packed target/source geometry
  WS_GEOM2,         // second geometry (RFD minus configuration)
  WS_SRC,           // packed source vectors (H-weighted force / torque)
  WS_PART,          // per-source-chunk partial sums of the pair kernel
  WS_VEC_A,         // float64 3n scratch vectors ...
  WS_VEC_B,
  WS_VEC_C,
  WS_VEC_D,
  WS_VEC_E,
  WS_VEC_F,
  WS_VEC_G,
  WS_VEC_H,
  WS_FORCE,         // forces of the time step
  WS_TORQUE,        // torques of the time step
  WS_NOISE_W,       // device-drawn W
  WS_NOISE_WT,      // device-drawn W~
  WS_KRYLOV,        // Lanczos basis V (max_iter x 3n)
  WS_REDUCE,        // reduction partials
  WS_SMALL,         // small device scalars (Lanczos coefficients, status, flags)
  WS_BATCH,         // batched products: offsets, work items, sphere -> system map
  WS_LZBATCH,       // batched Lanczos: per-system scalars and status
  WS_PRECOND,       // block-diagonal preconditioner: L (3n) and a scaled vector (3n)
  WS_CELLS,         // steric cell list: cells, buckets, sorted lists, bucket counts and starts
  WS_MBATCH,        // batched multi-vector products: per-system item and partial offsets
  WS_LZEIG,         // Lanczos: eigendecomposition of T_m per Krylov process
  WS_NSLOTS
};

// Slots of the Lanczos status ring: iterations whose status may be in flight at once.
constexpr int kLzRing = 4;

// The host thread that issues the second stream's work of small-system Lanczos solves
// (lanczos.hip); created on first use, stopped by lz_helper_destroy.
struct LzHelper;
void lz_helper_destroy(rpb_ctx *ctx);

// Default limit of the partial sums of one launch of the symmetric tile-pair kernels.
constexpr size_t kMaxChunkBytes = size_t(512) << 20;

// Layout of the WS_SMALL slot.
constexpr size_t kSmallBytes = 1 << 16;
constexpr size_t kSmallWorkCounter = 8192;          // int: work counter of persistent kernels
constexpr size_t kSmallFiniteFlag = kSmallBytes - 4; // int: non-finite input flag
constexpr size_t kSmallStepState = 16384;           // int64 step, int have_prev (time step)

struct DevBuf {
  void *ptr = nullptr;
  size_t bytes = 0;
};

}  // namespace rpb

namespace rpb {
// Launch shape of a pair kernel (chosen by the tuner; defaults from measurements).
struct Shape {
  int tpt;              // targets per lane (1 or 2)
  int target_wgs;       // workgroups to aim for when splitting the sources into chunks
  int batch_chunk;      // sources per ordered work item of the batched kernel (multiple of 256)
  int batch_wgs;        // persistent workgroups of the batched kernel
  int symmetric;        // 1: whole-system products evaluate each unordered pair once
  int batch_tpt;        // targets per lane of the batched kernel
  int batch_symmetric;  // 1: batched products evaluate each unordered pair once
};
// One shape per precision, indexed by rpb_precision (RPB_FP64 = 0, RPB_MIXED = 1).
struct Tuning {
  Shape s[2] = {{2, 4096, 1024, 2048, 1, 2, 1}, {2, 4096, 1024, 2048, 1, 2, 1}};
};
}  // namespace rpb

struct rpb_ctx {
  int device = 0;
  // partials of one chunk of the symmetric tile-pair kernels (the triangle of tile pairs is
  // walked in chunks of at most this many bytes); RPB_CHUNK_KIB overrides it
  size_t chunk_bytes = rpb::kMaxChunkBytes;
  rpb::Tuning tune;
  std::map<std::tuple<int, int, int>, rpb::Tuning> tune_cache;   // (precision, batched, log2 n)
  std::string err;
  rpb::DevBuf ws[rpb::WS_NSLOTS];
  void *host_pinned = nullptr;          // small pinned host buffer for device scalars
  void *host_pinned_dev = nullptr;      // the same buffer as kernels address it
  void *batch_host = nullptr;           // pinned staging of batched offsets / work items
  size_t batch_host_bytes = 0;
  // pair-kernel timing
  bool timing = false;
  std::vector<hipEvent_t> ev_start, ev_stop;
  std::vector<double> ev_pairs;
  std::vector<int> ev_kind;             // 2 * (precision == mixed) + (torque present)
  std::vector<hipEvent_t> ev_pool;
  // Lanczos status ring (rpb::kLzRing slots in the upper half of the pinned scratch) and the
  // events that mark each slot's status as landed; `lz_live` is set while one may be in flight
  hipEvent_t lz_ev[rpb::kLzRing] = {};
  bool lz_live[rpb::kLzRing] = {};
  // the second stream on which small systems run the Lanczos eigensolve and stop test beside
  // the vector recurrence, and the events that order the two streams
  hipStream_t lz_stream = nullptr;
  hipEvent_t lz_vec_ev[rpb::kLzRing] = {};
  hipEvent_t lz_join_ev = nullptr;
  rpb::LzHelper *lz_helper = nullptr;   // issues the second stream's calls from its own thread
  // deferred position check (check_finite_begin / _end): its flag's copy and event
  hipEvent_t fin_ev = nullptr;
  bool fin_live = false;
  // opt-in scan of each entry point's output for NaN / Inf (rpb_output_check_enable)
  bool check_output = false;
};

namespace rpb {

// Record an error message and return `code`.
int fail(rpb_ctx *ctx, int code, const char *fmt, ...);

// Device buffer of at least `bytes` for `slot` (grows; synchronises the device on growth).
void *workspace(rpb_ctx *ctx, Slot slot, size_t bytes, int *status);

// Pinned host scratch (kHostScratchBytes).  The lower half holds device scalars and
// per-system records copied back by one call and read before it returns; the upper half
// holds the Lanczos status ring, whose last copy may still land after the call returns.
constexpr size_t kHostScratchBytes = 1 << 17;
constexpr size_t kHostLzRingOffset = kHostScratchBytes / 2;
constexpr size_t kHostFiniteOffset = kHostLzRingOffset + 1024;   // deferred position check
inline void *host_scratch(rpb_ctx *ctx) { return ctx->host_pinned; }
inline void *host_scratch_dev(rpb_ctx *ctx) { return ctx->host_pinned_dev; }

#define RPB_HIP(ctx, call)                                                              \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess)                                                               \
      return ::rpb::fail((ctx), RPB_EDEVICE, "%s failed: %s (%s:%d)", #call,            \
                         hipGetErrorString(e_), __FILE__, __LINE__);                     \
  } while (0)

#define RPB_LAUNCHED(ctx)                                                               \
  do {                                                                                  \
    hipError_t e_ = hipGetLastError();                                                  \
    if (e_ != hipSuccess)                                                               \
      return ::rpb::fail((ctx), RPB_EDEVICE, "kernel launch failed: %s (%s:%d)",        \
                         hipGetErrorString(e_), __FILE__, __LINE__);                     \
  } while (0)

#define RPB_TRY(expr)                                                                   \
  do {                                                                                  \
    int s_ = (expr);                                                                    \
    if (s_ != RPB_OK) return s_;                                                        \
  } while (0)

// Common argument validation for the mobility entry points.
int check_params(rpb_ctx *ctx, const rpb_params *p);
// True when [a, a + abytes) and [b, b + bbytes) overlap (NULL never overlaps).
bool overlaps(const void *a, size_t abytes, const void *b, size_t bbytes);
// Checks that every position is finite (synchronises `stream`).
int check_finite(rpb_ctx *ctx, const double *pos, int64_t n, hipStream_t stream);
// The same check in two halves: _begin enqueues it and the copy of its flag to pinned host
// memory; _end waits for that copy only (not for work enqueued after it) and returns
// RPB_ENONFINITE if a position is NaN or Inf.  Work enqueued between the two may see those
// values, so it must not index memory by position value, and must write only workspace.
int check_finite_begin(rpb_ctx *ctx, const double *pos, int64_t n, hipStream_t stream);
int check_finite_end(rpb_ctx *ctx);
// With ctx->check_output set: scan m values at v for NaN / Inf on `stream`, synchronise, and
// return RPB_ENONFINITE naming `what` if one is found; RPB_OK at once otherwise.
int check_output(rpb_ctx *ctx, const double *v, int64_t m, hipStream_t stream, const char *what);

// Timing hooks around the pair kernel.
int timing_begin(rpb_ctx *ctx, hipStream_t stream, hipEvent_t *start);
int timing_end(rpb_ctx *ctx, hipStream_t stream, hipEvent_t start, double pairs, int kind);
// Drops the timing records from index `first` on (launches that turned out to do no work).
void timing_discard(rpb_ctx *ctx, size_t first);

// ---- mobility product (matvec.hip) ------------------------------------------------------

// Geometry of one configuration, packed once and reused by several products.
struct Packed {
  int64_t n = 0;
  double a = 1.0;         // radius: the packed lengths are in units of a
  int precision = RPB_FP64;
  void *geom = nullptr;   // precision-dependent structure-of-arrays
};

// Pack positions (clamp heights, weights H) into the geometry slot `slot`.
int pack_geometry(rpb_ctx *ctx, const rpb_params *p, int64_t n, const double *pos, Slot slot,
                  Packed *out, hipStream_t stream);

// The same packing into a caller-provided buffer of packed_geometry_bytes(n, precision).
int pack_geometry_into(rpb_ctx *ctx, const rpb_params *p, int64_t n, const double *pos,
                       void *buf, Packed *out, hipStream_t stream);
size_t packed_geometry_bytes(int64_t n, int precision);

// Whole-system U = M F + M_C T with every intermediate in the caller's device buffer `buf`
// (`bytes` long): packed geometry, packed sources and the ordered kernel's partial sums, with
// as many source chunks as fit (at most the tuned count).  No workspace, no position check, no
// synchronisation and no timing record.  RPB_EINVAL when even one chunk does not fit;
// noalloc_matvec_bytes(n, precision, c) is the size needed with c chunks.
size_t noalloc_matvec_bytes(int64_t n, int precision, int64_t nchunks);
int matvec_into(rpb_ctx *ctx, const rpb_params *p, int64_t n, const double *pos,
                const double *force, const double *torque, double *vel, void *buf, size_t bytes,
                hipStream_t stream);
// Resolves the device address of the library's static scratch array on the current device
// `device` (noalloc.hip); called once per device by rpb_create.
int noalloc_setup(rpb_ctx *ctx, int device);

// vel[r] for rows [row0, row0 + nrows) of U = M F + M_C T for packed geometry `g`.
// force / torque are [n][3] float64 device arrays (nullable, not both).  `skip` (nullable)
// is a device flag read by every kernel of the product when it runs: while it is nonzero
// they return at once and `vel` keeps its contents.
int matvec_packed(rpb_ctx *ctx, const rpb_params *p, const Packed &g, const double *force,
                  const double *torque, int64_t row0, int64_t nrows, double *vel,
                  hipStream_t stream, const int *skip = nullptr);

// The H weights of packed geometry `g` (n float64 values on the device).
const double *packed_weights(const Packed &g);
// The buffer the products read their packed sources from: 6 n values of the pair precision
// (float64 for RPB_FP64, float32 for RPB_MIXED), component-major: rows c = 0..2 hold the
// H-weighted force, f[c * n + i] = H_i F_i,c (the product in float64, then rounded), rows
// 3..5 the H-weighted torque divided by the radius.
void *source_buffer(rpb_ctx *ctx, const Packed &g, int *status);
// U = M F for the whole system from force sources already written into `src` (rows 0..2 of
// source_buffer's layout; no torque), as matvec_packed would form them.
int matvec_prepacked(rpb_ctx *ctx, const rpb_params *p, const Packed &g, const void *src,
                     double *vel, hipStream_t stream, const int *skip = nullptr);

// ---- batched products (matvec.hip) -----------------------------------------------------

// Work list of a batch of independent systems (built on the host, copied to the device).
struct Batch {
  int nsys = 0;
  int64_t n = 0;                 // total spheres
  int64_t chunk = 0;             // sources per work item
  int tpt = 1;                   // targets per lane of the launch
  int wgs = 1;                   // persistent workgroups of the launch
  int nitems = 0;
  int64_t max_chunks = 0;        // source chunks of the largest system
  std::vector<int64_t> host_offs;
  int64_t *offs = nullptr;       // device
  int4 *items = nullptr;         // device
  int *sys_of = nullptr;         // device, n entries
  bool symmetric = false;        // items are (system, I, J, part) of the symmetric kernel
  int nsplit = 1;                // source parts per symmetric tile pair
  int64_t *part_base = nullptr;  // device, nsys entries: each system's first partial slot
  int64_t part_elems = 0;        // partial elements of the symmetric layout (float32 in mixed precision)
};

int check_offsets(rpb_ctx *ctx, int32_t nsys, const int64_t *offs);
// work_items = false builds the offsets and the sphere -> system map only (for segment-wise
// vector kernels), no pair work items.
int prepare_batch(rpb_ctx *ctx, int32_t nsys, const int64_t *offs, int precision, Batch *b,
                  hipStream_t stream, bool work_items = true);
// Batched product for packed geometry `g` (all systems); systems with done[s] != 0 are
// skipped (their output rows are left untouched), and the launch returns at once when
// done[nsys] != 0 (every system done).  `done` (nsys + 1 flags) may be NULL.
int matvec_batched(rpb_ctx *ctx, const rpb_params *p, const Batch &b, const Packed &g,
                   const double *force, const double *torque, const int *done, double *vel,
                   hipStream_t stream);

// ---- multi-vector products (multi.hip) --------------------------------------------------

// vel[v] = M force[v] for the nvec vectors force[v] ([n][3] float64 each, v-major) of packed
// geometry `g`; vectors with done[v] != 0 (host array, nullable) are skipped.
int matvec_multi(rpb_ctx *ctx, const rpb_params *p, const Packed &g, int nvec, const int *done,
                 const double *force, double *vel, hipStream_t stream);
// The products of a step at its own configuration in one launch (the pair coefficients shared):
// u_force = M force + M_C torque, u_w = M w and, when w3 is not NULL, u_w3 = M w3; torque
// nullable.  Available when matvec_first_supported(p, n) (no box, partials within the
// workspace limit).
bool matvec_first_supported(const rpb_params *p, int64_t n);
int matvec_first(rpb_ctx *ctx, const rpb_params *p, const Packed &g, const double *force,
                 const double *torque, const double *w, const double *w3, double *u_force,
                 double *u_w, double *u_w3, hipStream_t stream);

// Batched form of matvec_first with two vectors (u_force = M force + M_C torque, u_w = M w per
// system), one persistent launch; available when matvec_first_batched_supported(p, bt).
bool matvec_first_batched_supported(const rpb_params *p, const Batch &bt);
int matvec_first_batched(rpb_ctx *ctx, const rpb_params *p, const Batch &bt, const Packed &g,
                         const double *force, const double *torque, const double *w,
                         double *u_force, double *u_w, hipStream_t stream);

// ---- vector kernels (lanczos.hip) -------------------------------------------------------
constexpr int kMaxBatchSystems = 4096;   // per-system records must fit the pinned scratch

// Per-system outcome of a batched Lanczos solve.
struct LzStatus {
  int m;          // iterations used
  int reason;     // 0 not converged, 1 converged, 2 breakdown (exact), 3 not SPD, 4 solver failed
  double eps;     // last relative change
};

// Batched Lanczos: one Krylov process per system of `b`.  sync_each = true reads the per-system
// flags after every iteration and stops when all systems are done; false runs max_iter
// iterations with device-side freezing only (no host synchronisation: capturable).
// status_host (pinned, nsys records) is filled when not NULL (synchronises).
// mw (nullable, ignored with precond): M w computed by the caller for every system, used for
// the first iteration.
int lanczos_batched_run(rpb_ctx *ctx, const rpb_params *p, const Batch &b, const Packed &g,
                        const double *w, double tol, int max_iter, bool precond, double *out,
                        bool sync_each, LzStatus *status_host, hipStream_t stream,
                        const double *mw = nullptr);
// L (3n, float64) with L^2 = the diagonal of the self blocks M_ii of the packed geometry
// (1 where H = 0).
int block_diag_scale(rpb_ctx *ctx, const rpb_params *p, const Packed &g, double *scale,
                     hipStream_t stream);
// Map per-system outcomes to a status code (first failure wins; ENOCONV when any missed tol).
int lanczos_status_code(rpb_ctx *ctx, const LzStatus *s, int nsys);
// Copy the per-system outcomes of the last batched solve (synchronises `stream`).
int lanczos_batched_status_copy(rpb_ctx *ctx, int nsys, LzStatus *host, hipStream_t stream);

// precond: square-root preconditioning with the self-block diagonal (block_diag_scale):
// Lanczos on B = L^-1 M L^-1, result L B^{1/2} w.  mw (nullable, only without precond): the
// product M w computed by the caller, which then replaces the first iteration's product.
int lanczos_run(rpb_ctx *ctx, const rpb_params *p, const Packed &g, const double *w, double tol,
                int max_iter, bool precond, double *out, int *iters, double *eps,
                hipStream_t stream, const double *mw = nullptr);

// ---- RFD / RNG / forces / step ----------------------------------------------------------
// base (one-sided only, nullable): M(q) w~ already computed in rfd_precision by the caller.
int rfd_run(rpb_ctx *ctx, const rpb_params *p, int64_t n, const double *pos, const double *wt,
            double delta, int rfd_precision, bool one_sided, double *drift, hipStream_t stream,
            const double *base = nullptr);
int normals_run(rpb_ctx *ctx, int64_t count, uint64_t seed, uint64_t stream_id, uint64_t step,
                double *out, hipStream_t stream);
int forces_run(rpb_ctx *ctx, const rpb_params *p, int64_t n, const double *pos, double f_grav_z,
               double u0, double b, double *force, hipStream_t stream);
// Steric forces within each system of a batch (no interaction across systems).
int forces_batched_run(rpb_ctx *ctx, const rpb_params *p, const Batch &bt, const double *pos,
                       double f_grav_z, double u0, double b, double *force, hipStream_t stream);
// Normals for the step number held on the device (*step_dev).
int normals_devstep_run(rpb_ctx *ctx, int64_t count, uint64_t seed, uint64_t stream_id,
                        const int64_t *step_dev, double *out, hipStream_t stream);
// RFD over a batch of systems.
int rfd_batched_run(rpb_ctx *ctx, const rpb_params *p, const Batch &bt, const double *pos,
                    const double *wt, double delta, int rfd_precision, bool one_sided,
                    double *drift, hipStream_t stream);

// ---- time step (step.hip) ---------------------------------------------------------------
// Device record of a time-stepped batch: read by the noise and update kernels, advanced by
// the last kernel of a step.
struct StepRecord {
  int64_t step;
  int have_prev;
};
int set_step_state(rpb_ctx *ctx, void *step_state, int64_t step, int have_prev,
                   hipStream_t stream);
int check_step_config(rpb_ctx *ctx, const rpb_sab_config *cfg);
// Enqueue one batched step without host synchronisation (capturable).  The step number and
// the have-previous flag are read from the device record at `step_state` (int64 step, int
// have_prev) and advanced at the end.
int step_batched_enqueue(rpb_ctx *ctx, const rpb_params *p, const rpb_sab_config *cfg,
                         const Batch &bt, double *pos, double *u_prev, const double *w,
                         const double *w_tilde, void *step_state, bool sync_lanczos,
                         LzStatus *status_host, hipStream_t stream);

}  // namespace rpb
