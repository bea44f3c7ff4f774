// Mobility product that allocates nothing: for callers that cannot call hipMalloc (code under
// hipGraph capture, tight serving loops, harnesses that forbid allocation).
//
// Every intermediate of the product (packed geometry, packed sources, the ordered pair
// kernel's partial sums) lives in `scratch`, a file-scope device array of kScratchBytes that
// each GPU the library runs on holds until the process ends.  Host code never passes the
// array's name to a kernel: the name is only a host-side stand-in.  rpb_create resolves the
// array's device address once per device (hipGetSymbolAddress, with that device current) and
// the entry point passes that address on.
//
// All calls on one GPU share its array and it keeps the last call's contents; every value a
// call reads is written earlier by the same call, so nothing needs clearing.  Calls that
// overlap in time on one GPU (two streams, two host threads) race on the array.
#include <mutex>

#include "rpb_internal.h"

namespace rpb {

constexpr size_t kScratchBytes = size_t(32) << 20;   // 32 MiB per device
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Device address of `scratch` per device, resolved by noalloc_setup.
static std::mutex g_scratch_mutex;
static void *g_scratch_ptr[kMaxDevices] = {};

int noalloc_setup(rpb_ctx *ctx, int device) {
  if (device < 0 || device >= kMaxDevices)
    return fail(ctx, RPB_EDEVICE, "device %d beyond the %d the no-alloc scratch supports", device,
                kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (g_scratch_ptr[device]) return RPB_OK;
  void *ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) {
    (void)hipGetLastError();
    return fail(ctx, RPB_EDEVICE, "hipGetSymbolAddress of the scratch array failed: %s",
                hipGetErrorString(e));
  }
  g_scratch_ptr[device] = ptr;
  return RPB_OK;
}

}  // namespace rpb

using namespace rpb;

extern "C" {

int rpb_mobility_matvec_noalloc(rpb_ctx *ctx, const rpb_params *p, int64_t n, const double *pos,
                                const double *force, const double *torque, double *vel_out,
                                rpb_stream_t stream) {
  RPB_TRY(check_params(ctx, p));
  if (n < 0) return fail(ctx, RPB_EINVAL, "n must be >= 0");
  if (n == 0) return RPB_OK;
  if (!pos || !vel_out) return fail(ctx, RPB_EINVAL, "pos and vel_out must not be NULL");
  if (!force && !torque) return fail(ctx, RPB_EINVAL, "force and torque are both NULL");
  const size_t nb = size_t(n) * 3 * sizeof(double);
  if (overlaps(vel_out, nb, pos, nb) || overlaps(vel_out, nb, force, nb) ||
      overlaps(vel_out, nb, torque, nb))
    return fail(ctx, RPB_EINVAL, "vel_out overlaps an input");
  void *buf = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    buf = ctx->device >= 0 && ctx->device < kMaxDevices ? g_scratch_ptr[ctx->device] : nullptr;
  }
  if (!buf) return fail(ctx, RPB_EDEVICE, "no-alloc scratch not set up on device %d", ctx->device);
  RPB_HIP(ctx, hipSetDevice(ctx->device));
  return matvec_into(ctx, p, n, pos, force, torque, vel_out, buf, kScratchBytes,
                     static_cast<hipStream_t>(stream));
}

}  // extern "C"
