// Allocation-free sampling entry point: smg_sample_field with the hierarchy's workspace held in
// a device array of the library instead of caller-bound memory.
//
// The array `scratch` is a file-scope __device__ object: every device the library runs on holds
// its own copy (for the life of the process) at its own address.  In host code `scratch` names
// a host-side stand-in, not device memory, so its device address is fetched once per device
// with hipGetSymbolAddress (with that device current) and kept in g_dev[device].ptr; only that
// pointer ever reaches a kernel or a copy.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "smg_internal.hpp"

namespace smg {
namespace {

constexpr size_t kScratchBytes = (size_t)SMG_STATIC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
struct DeviceScratch {
  void* ptr = nullptr;  // device address of this device's copy of `scratch`
  uint64_t owner = 0;   // uid of the hierarchy whose tables the copy holds (0: none)
};
DeviceScratch g_dev[kMaxDevices];
std::mutex g_mu;  // guards g_dev (host-side bookkeeping only)

}  // namespace
}  // namespace smg

using namespace smg;

extern "C" int smg_sample_field_static(smg_hierarchy* hh, int64_t n, uint64_t seed,
                                       uint64_t first_cycle, void* state, void* out,
                                       int32_t out_dtype, void* stream) {
  if (!hh) {
    set_error("null hierarchy");
    return SMG_EINVAL;
  }
  Hierarchy& h = hh->h;
  if (h.ws_bytes > kScratchBytes) {
    set_error("hierarchy needs " + std::to_string(h.ws_bytes) +
              " workspace bytes; the static scratch holds " + std::to_string(kScratchBytes) +
              " (use smg_bind_workspace and smg_sample_field)");
    return SMG_ENOMEM;
  }
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    set_error(std::string("hipGetDevice: ") + hipGetErrorString(e));
    return SMG_EHIP;
  }
  hipStream_t s = (hipStream_t)stream;
  std::lock_guard<std::mutex> lock(g_mu);
  DeviceScratch& d = g_dev[dev];
  if (!d.ptr) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      set_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
      return SMG_EHIP;
    }
    d.ptr = p;
  }
  // The hierarchy may also be bound to caller memory: keep that binding and restore it after
  // the call (host pointers only; the caller's workspace is not touched).
  char* const prev_ws = h.ws;
  const int prev_dev = h.device;
  // The copy keeps the last call's contents: upload this hierarchy's tables unless they are the
  // ones already there.  Fields that must start at zero are cleared by the sampling path itself.
  int rc = bind_impl(h, (char*)d.ptr, d.owner != h.uid, s);
  if (rc != SMG_OK) {
    // the copy's tables are in an unknown state, and the hierarchy's device pointers may point
    // into it: point them back at the caller's workspace (tables there are untouched)
    d.owner = 0;
    if (prev_ws) {
      bind_impl(h, prev_ws, false, s);
      h.device = prev_dev;
    } else {
      h.ws = nullptr;
    }
    return rc;
  }
  d.owner = h.uid;
  // one stream: side streams and events are not made here
  rc = sample_field_impl(hh, n, seed, first_cycle, state, out, out_dtype, stream, 1);
  if (prev_ws) {
    const int rc2 = bind_impl(h, prev_ws, false, s);
    h.device = prev_dev;
    if (rc == SMG_OK) rc = rc2;
  } else {
    h.ws = nullptr;  // unbound again: the ordinary entry points still ask for a workspace
  }
  return rc;
}
