// Host side of the C ABI (include/gst.h): argument checks, workspaces,
// launches and the resident request.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "../../include/gst.h"
#include "gst_internal.h"

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIP_TRY(expr)                                                                        \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      return fail(e_ == hipErrorOutOfMemory ? GST_ENOMEM : GST_EDEVICE,                      \
                  std::string(#expr) + ": " + hipGetErrorString(e_));                        \
  } while (0)

int dim_of(int n_qubits) { return n_qubits == 1 ? 4 : n_qubits == 2 ? 16 : n_qubits == 3 ? 64 : 0; }

}  // namespace

// A growable device buffer owned by a context or request.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  // Ensure capacity; the stream is drained first so that no queued kernel
  // still uses the old allocation.
  int reserve(size_t need, hipStream_t stream) {
    if (need <= bytes) return GST_OK;
    const size_t cap = std::max(need, bytes + bytes / 2);
    HIP_TRY(hipStreamSynchronize(stream));
    if (p) HIP_TRY(hipFree(p));
    p = nullptr;
    bytes = 0;
    HIP_TRY(hipMalloc(&p, cap));
    bytes = cap;
    return GST_OK;
  }
};

struct gst_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  unsigned long long* status = nullptr;  // device [2]
  DevBuf ws;
};

struct gst_req {
  gst_ctx* ctx = nullptr;
  int n_qubits = 0, D = 0, M = 0, K = 0;
  int64_t S = 0;
  int32_t* counts = nullptr;
  DevBuf ws;
  size_t resident_bytes = 0;
};

namespace {

int check_gateset(const gst_gateset* gs, int* D) {
  if (!gs) return fail(GST_EINVAL, "gateset is NULL");
  const int d = dim_of(gs->n_qubits);
  if (!d) return fail(GST_EINVAL, "n_qubits must be 1, 2 or 3");
  if (gs->n_gates < 1 || gs->n_gates > gst_max_gates(gs->n_qubits))
    return fail(GST_EINVAL, "n_gates out of range for this qubit count (see gst_max_gates)");
  if (gs->n_outcomes < 1 || gs->n_outcomes > d) return fail(GST_EINVAL, "n_outcomes must be in 1..D");
  if (!gs->rho || !gs->effects || !gs->gates) return fail(GST_EINVAL, "gateset pointer is NULL");
  *D = d;
  return GST_OK;
}

int check_seqs(const gst_seqlist* sl) {
  if (!sl) return fail(GST_EINVAL, "seqlist is NULL");
  if (sl->n_seq < 0) return fail(GST_EINVAL, "n_seq < 0");
  if (sl->n_seq > 0 && (!sl->offsets || !sl->gate_idx)) return fail(GST_EINVAL, "seqlist pointer is NULL");
  return GST_OK;
}

// max_len from the caller, or read back from the device offsets.
int resolve_max_len(const gst_seqlist* sl, hipStream_t stream, int64_t* out) {
  if (sl->max_len >= 0) {
    *out = sl->max_len;
    return GST_OK;
  }
  std::vector<int64_t> off((size_t)sl->n_seq + 1);
  HIP_TRY(hipMemcpyAsync(off.data(), sl->offsets, off.size() * 8, hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  int64_t mx = 0;
  for (int64_t s = 0; s < sl->n_seq; ++s) {
    const int64_t L = off[s + 1] - off[s];
    if (L < 0) return fail(GST_EINVAL, "offsets decrease");
    mx = std::max(mx, L);
  }
  *out = mx;
  return GST_OK;
}

// Enqueue the sequence kernel over `n_items` work items and the slab reduction.
int run_leaf(gst_ctx* ctx, DevBuf& ws, const gst::LeafLaunch& base, int64_t max_len, double* objective,
             double* grad) {
  gst::LeafLaunch a = base;
  const int D = a.D;
  const bool need_slab = a.want_grad || a.mode == gst::MODE_LOGLIK;
  const int blocks = gst::leaf_blocks_for(D, a.n_items);
  const int64_t P = gst::slab_width(D, a.M, a.K);
  const int C = gst::leaf_ckpt_interval(D);
  const int64_t ck_team = a.want_grad ? ((max_len + C - 1) / C + 1) * 16 : 0;
  const size_t slab_bytes = need_slab ? (size_t)blocks * P * 8 : 0;
  const size_t ck_bytes = (size_t)blocks * gst::leaf_teams_per_block(D) * ck_team * 8;
  int rc = ws.reserve(slab_bytes + ck_bytes + 256, ctx->stream);
  if (rc) return rc;
  a.slab = need_slab ? reinterpret_cast<double*>(ws.p) : nullptr;
  a.ckpt = a.want_grad ? reinterpret_cast<double*>((char*)ws.p + slab_bytes) : nullptr;
  a.ckpt_per_team = ck_team;
  a.max_len = (int)max_len;
  a.status = ctx->status;
  if (max_len > (int64_t)1 << 30) return fail(GST_EINVAL, "sequence too long");
  HIP_TRY(gst::launch_leaf(a, blocks, ctx->stream));
  if (need_slab) HIP_TRY(gst::launch_reduce(a.slab, blocks, P, objective, grad, ctx->status, ctx->stream));
  return GST_OK;
}

int plain_eval(gst_ctx* ctx, const gst_gateset* gs, const gst_seqlist* sl, int mode, const int32_t* counts,
               const double* w, double* probs, double* objective, double* grad) {
  if (!ctx) return fail(GST_EINVAL, "ctx is NULL");
  int D = 0;
  int rc = check_gateset(gs, &D);
  if (rc) return rc;
  rc = check_seqs(sl);
  if (rc) return rc;
  if (D == 64) return fail(GST_EINVAL, "three-qubit gate sets are not supported by this build");
  HIP_TRY(hipSetDevice(ctx->device));
  int64_t max_len = 0;
  rc = resolve_max_len(sl, ctx->stream, &max_len);
  if (rc) return rc;
  gst::LeafLaunch a{};
  a.D = D;
  a.M = gs->n_outcomes;
  a.K = gs->n_gates;
  a.rho = gs->rho;
  a.E = gs->effects;
  a.G = gs->gates;
  a.n_items = sl->n_seq;
  a.off = sl->offsets;
  a.gates = sl->gate_idx;
  a.items = nullptr;
  a.anchor_states = nullptr;
  a.anchor_adj = nullptr;
  a.counts = counts;
  a.W = w;
  a.probs = probs;
  a.mode = mode;
  a.want_grad = grad != nullptr;
  return run_leaf(ctx, ctx->ws, a, max_len, objective, grad);
}

}  // namespace

extern "C" {

int gst_max_gates(int n_qubits) {
  const int d = dim_of(n_qubits);
  return d ? gst::max_gates_for(d) : 0;
}

const char* gst_last_error(void) { return g_err.c_str(); }

int gst_create(gst_ctx** out, int device_ordinal, void* hip_stream) {
  if (!out) return fail(GST_EINVAL, "out is NULL");
  int n = 0;
  HIP_TRY(hipGetDeviceCount(&n));
  if (device_ordinal < 0 || device_ordinal >= n) return fail(GST_EINVAL, "no such device");
  HIP_TRY(hipSetDevice(device_ordinal));
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, device_ordinal));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(GST_EDEVICE, std::string("this library is built for gfx950, device is ") + prop.gcnArchName);
  std::unique_ptr<gst_ctx> c(new (std::nothrow) gst_ctx());
  if (!c) return fail(GST_ENOMEM, "host allocation failed");
  c->device = device_ordinal;
  c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  HIP_TRY(hipMalloc(&c->status, 2 * sizeof(unsigned long long)));
  HIP_TRY(hipMemset(c->status, 0, 2 * sizeof(unsigned long long)));
  *out = c.release();
  return GST_OK;
}

int gst_destroy(gst_ctx* ctx) {
  if (!ctx) return GST_OK;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  if (ctx->status) (void)hipFree(ctx->status);
  delete ctx;
  return GST_OK;
}

int gst_sync(gst_ctx* ctx, gst_diag* diag) {
  if (!ctx) return fail(GST_EINVAL, "ctx is NULL");
  HIP_TRY(hipSetDevice(ctx->device));
  unsigned long long st[2] = {0, 0};
  HIP_TRY(hipMemcpyAsync(st, ctx->status, sizeof(st), hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  const unsigned long long zero[2] = {0, 0};
  HIP_TRY(hipMemcpyAsync(ctx->status, zero, sizeof(zero), hipMemcpyHostToDevice, ctx->stream));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  if (diag) {
    diag->n_bad_index = (int64_t)st[0];
    diag->n_nonpos = (int64_t)st[1];
  }
  if (st[0]) return fail(GST_EINDEX, std::to_string(st[0]) + " gate indices >= n_gates");
  if (st[1]) return fail(GST_ENONPOS, std::to_string(st[1]) + " probabilities <= 0 with positive counts");
  return GST_OK;
}

int gst_probs(gst_ctx* ctx, const gst_gateset* gs, const gst_seqlist* seqs, double* probs) {
  if (seqs && seqs->n_seq > 0 && !probs) return fail(GST_EINVAL, "probs is NULL");
  return plain_eval(ctx, gs, seqs, gst::MODE_PROBS, nullptr, nullptr, probs, nullptr, nullptr);
}

int gst_loglik(gst_ctx* ctx, const gst_gateset* gs, const gst_seqlist* seqs, const int32_t* counts,
               double* probs, double* objective, double* grad) {
  if (!objective) return fail(GST_EINVAL, "objective is NULL");
  if (seqs && seqs->n_seq > 0 && !counts) return fail(GST_EINVAL, "counts is NULL");
  return plain_eval(ctx, gs, seqs, gst::MODE_LOGLIK, counts, nullptr, probs, objective, grad);
}

int gst_vjp(gst_ctx* ctx, const gst_gateset* gs, const gst_seqlist* seqs, const double* w, double* grad) {
  if (!grad) return fail(GST_EINVAL, "grad is NULL");
  if (seqs && seqs->n_seq > 0 && !w) return fail(GST_EINVAL, "w is NULL");
  return plain_eval(ctx, gs, seqs, gst::MODE_VJP, nullptr, w, nullptr, nullptr, grad);
}

}  // extern "C"
