// Internal declarations shared by the librpb translation units (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
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
  WS_NSLOTS
};

struct DevBuf {
  void *ptr = nullptr;
  size_t bytes = 0;
};

}  // namespace rpb

namespace rpb {
// Launch shapes of the pair kernels (chosen by the tuner; defaults from measurements).
struct Tuning {
  int tpt_f64 = 2;          // targets per lane, float64 kernel (1 or 2)
  int tpt_mixed = 1;        // targets per lane, mixed kernel (1 or 2)
  int target_wgs = 4096;    // workgroups to aim for when splitting the sources into chunks
};
}  // namespace rpb

struct rpb_ctx {
  int device = 0;
  rpb::Tuning tune;
  std::string err;
  rpb::DevBuf ws[rpb::WS_NSLOTS];
  void *host_pinned = nullptr;          // small pinned host buffer for device scalars
  // pair-kernel timing
  bool timing = false;
  std::vector<hipEvent_t> ev_start, ev_stop;
  std::vector<double> ev_pairs;
  std::vector<int> ev_kind;             // 2 * (precision == mixed) + (torque present)
  std::vector<hipEvent_t> ev_pool;
};

namespace rpb {

// Record an error message and return `code`.
int fail(rpb_ctx *ctx, int code, const char *fmt, ...);

// Device buffer of at least `bytes` for `slot` (grows; synchronises the device on growth).
void *workspace(rpb_ctx *ctx, Slot slot, size_t bytes, int *status);

// Pinned host scratch of at least 4 KiB.
inline void *host_scratch(rpb_ctx *ctx) { return ctx->host_pinned; }

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

// Timing hooks around the pair kernel.
int timing_begin(rpb_ctx *ctx, hipStream_t stream, hipEvent_t *start);
int timing_end(rpb_ctx *ctx, hipStream_t stream, hipEvent_t start, double pairs, int kind);

// ---- mobility product (matvec.hip) ------------------------------------------------------

// Geometry of one configuration, packed once and reused by several products.
struct Packed {
  int64_t n = 0;
  int precision = RPB_FP64;
  void *geom = nullptr;   // precision-dependent structure-of-arrays
};

// Pack positions (clamp heights, weights H) into the geometry slot `slot`.
int pack_geometry(rpb_ctx *ctx, const rpb_params *p, int64_t n, const double *pos, Slot slot,
                  Packed *out, hipStream_t stream);

// vel[r] for rows [row0, row0 + nrows) of U = M F + M_C T for packed geometry `g`.
// force / torque are [n][3] float64 device arrays (nullable, not both).  `scale_out`
// multiplies the result (1 for plain products).
int matvec_packed(rpb_ctx *ctx, const rpb_params *p, const Packed &g, const double *force,
                  const double *torque, int64_t row0, int64_t nrows, double *vel,
                  hipStream_t stream);

// ---- vector kernels (lanczos.hip) -------------------------------------------------------
int lanczos_run(rpb_ctx *ctx, const rpb_params *p, const Packed &g, const double *w, double tol,
                int max_iter, double *out, int *iters, double *eps, hipStream_t stream);

// ---- RFD / RNG / forces / step ----------------------------------------------------------
int rfd_run(rpb_ctx *ctx, const rpb_params *p, int64_t n, const double *pos, const double *wt,
            double delta, int rfd_precision, double *drift, hipStream_t stream);
int normals_run(rpb_ctx *ctx, int64_t count, uint64_t seed, uint64_t stream_id, uint64_t step,
                double *out, hipStream_t stream);
int forces_run(rpb_ctx *ctx, const rpb_params *p, int64_t n, const double *pos, double f_grav_z,
               double u0, double b, double *force, hipStream_t stream);

}  // namespace rpb
