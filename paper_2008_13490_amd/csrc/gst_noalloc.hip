// The allocation-free evaluation: gst_loglik with its scratch in a file-scope
// device array, for callers that cannot allocate device memory (code under
// HIP graph capture, tight serving loops, harnesses that forbid allocation).
//
// The plain evaluation's kernels need scratch beyond their inputs and outputs:
// one row of partial sums per workgroup, the first-stage sums of the ordered
// reduction, and the checkpoints of the reverse sweeps.  Here they live in
// `scratch`, a static device array of kScratchBytes that every GPU running the
// library holds until the process ends.  Its device address is resolved once
// per device when a context is created on it (hipGetSymbolAddress with that
// device current) and only that address is handed to kernels: the array's
// name in host code is a host-side stand-in, not a device address.
//
// All calls on one GPU share that GPU's array and leave their contents in it;
// nothing in it has to start at zero (every entry is written before it is
// read).  Two calls that overlap on one GPU (on different streams) race on the
// array: the caller keeps them apart, e.g. on one stream.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/gst.h"
#include "gst_internal.h"

namespace {

constexpr size_t kScratchBytes = (size_t)128 << 20;
constexpr int kMaxDevices = 64;

__device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};  // device address of `scratch` on each device

}  // namespace

namespace gst {

int scratch_bind(int device) {
  if (device < 0 || device >= kMaxDevices) return GST_EINVAL;
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_scratch[device]) return GST_OK;
  int prev = 0;
  if (hipGetDevice(&prev) != hipSuccess) return GST_EDEVICE;
  if (hipSetDevice(device) != hipSuccess) return GST_EDEVICE;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  (void)hipSetDevice(prev);
  if (e != hipSuccess || !p) return GST_EDEVICE;
  g_scratch[device] = p;
  return GST_OK;
}

}  // namespace gst

extern "C" int gst_loglik_noalloc(gst_ctx* ctx, const gst_gateset* gs, const gst_seqlist* seqs,
                                  const int32_t* counts, double* probs, double* objective, double* grad) {
  const int device = ctx ? gst::ctx_device(ctx) : -1;
  void* p = nullptr;
  if (device >= 0 && device < kMaxDevices) {
    std::lock_guard<std::mutex> lock(g_mu);
    p = g_scratch[device];
  }
  return gst::loglik_into_scratch(ctx, gs, seqs, counts, probs, objective, grad, p, kScratchBytes);
}
