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
#include "gst_fit_core.h"
#include "gst_metrics.h"
#include "gst_internal.h"
#include "gst_plan.h"
#include "gst_plan64.h"

namespace gst {
LaunchTimer*& launch_timer() {
  static thread_local LaunchTimer* t = nullptr;
  return t;
}
}  // namespace gst

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
  // Ensure capacity; when an old allocation is replaced, the stream is
  // drained first so that no queued kernel still uses it (a first
  // allocation waits for nothing).
  int reserve(size_t need, hipStream_t stream) {
    if (need <= bytes) return GST_OK;
    const size_t cap = std::max(need, bytes + bytes / 2);
    if (p) {
      HIP_TRY(hipStreamSynchronize(stream));
      HIP_TRY(hipFree(p));
    }
    p = nullptr;
    bytes = 0;
    HIP_TRY(hipMalloc(&p, cap));
    bytes = cap;
    return GST_OK;
  }
};

// Pinned host staging for small per-call host arrays: the caller's arrays are
// copied into it on the host, then one asynchronous copy moves them to the
// device, so the call returns without waiting for the stream.  The next user
// waits for the previous copy out of the buffer (normally long finished).
struct HostStage {
  void* p = nullptr;
  size_t bytes = 0;
  hipEvent_t done = nullptr;
  ~HostStage() {
    if (done) (void)hipEventDestroy(done);
    if (p) (void)hipHostFree(p);
  }
  int acquire(size_t need) {
    if (done) HIP_TRY(hipEventSynchronize(done));
    if (need > bytes) {
      if (p) HIP_TRY(hipHostFree(p));
      p = nullptr;
      bytes = 0;
      const size_t cap = std::max(need, (size_t)4096);
      HIP_TRY(hipHostMalloc(&p, cap, hipHostMallocDefault));
      bytes = cap;
    }
    if (!done) HIP_TRY(hipEventCreateWithFlags(&done, hipEventDisableTiming));
    return GST_OK;
  }
  int copy_to(void* dst, size_t n, hipStream_t stream) {
    HIP_TRY(hipMemcpyAsync(dst, p, n, hipMemcpyHostToDevice, stream));
    HIP_TRY(hipEventRecord(done, stream));
    return GST_OK;
  }
};

// Per-kernel-family event timing (gst_profile_*).
struct Profiler {
  bool on = false;
  int only = -1;  // record only this family (-1 = all)
  struct Pending {
    int family;
    hipEvent_t a, b;
    bool owner;  // returns the events to the pool (a kernel counts for every enclosing family)
  };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;
  static constexpr int kMaxFamilies = 24;
  double total_ms[kMaxFamilies] = {0};
  int64_t launches[kMaxFamilies] = {0};
  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  ~Profiler() {
    for (auto& p : pending) {
      if (!p.owner) continue;
      (void)hipEventDestroy(p.a);
      (void)hipEventDestroy(p.b);
    }
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

enum Family { FAM_LEAF = 0, FAM_REDUCE = 1, FAM_TRUNK_FWD = 2, FAM_TRUNK_BWD = 3, FAM_INJECT = 4, FAM_GEMM = 5,
              FAM_BATCH = 6, FAM_TILES16 = 7, FAM_TILES4 = 8, FAM_TILES_RED = 9, FAM_CHAIN64 = 10,
              FAM_GEMM64 = 11, FAM_REDUCE64 = 12, FAM_FILL = 13, FAM_PRED_CHAIN = 14,
              FAM_PRED_FILL = 15, FAM_TV = 16, FAM_PARAM_FWD = 17, FAM_PARAM_BWD = 18, FAM_P64_FWD = 19,
              FAM_P64_BWD = 20, FAM_P64_READ = 21, FAM_N = 22 };
static_assert(FAM_N <= Profiler::kMaxFamilies, "profiler arrays too small");
static const char* kFamilyNames[FAM_N] = {"leaf",  "reduce",  "trunk_fwd", "trunk_bwd",   "inject",
                                          "grad_gemm", "batch", "tiles_2q",  "tiles_1q", "tiles_reduce",
                                          "chain_3q",  "gemm_3q", "reduce_3q", "fill", "predict_chain",
                                          "predict_fill", "tv_distance", "param_fwd", "param_bwd", "tiles_3q_fwd",
                                          "tiles_3q_bwd", "readout_3q"};

// Carve consecutive aligned regions out of one allocation.
struct Carver {
  size_t off = 0;
  template <class T>
  size_t take(size_t n) {
    off = (off + 255) / 256 * 256;
    const size_t at = off;
    off += n * sizeof(T);
    return at;
  }
};

struct gst_ctx {
  int device = 0;
  int n_cu = 0;
  int tune_tile[4] = {0, 0, 0, 0};  // sequences per tile by qubit count (0 = default)
  int tune_bpc[4] = {0, 0, 0, 0};   // workgroups per CU by qubit count (0 = as many as fit)
  int plan_jump = gst::PlanOptions().jump;  // germ-power jump repetitions of new plans (0 = none)
  hipStream_t stream = nullptr;
  unsigned long long* status = nullptr;  // device [2]
  DevBuf ws;
  HostStage stage;
  DevBuf param_tab[3];  // generator structure tables by qubit count (1, 2), uploaded on first use
  Profiler prof;
};

// Brackets one launch with events when profiling is on.
// Times the kernels launched in its lifetime as family `family`: each launch
// gets its own event pair stamped with the kernel's start and end (no marker
// between kernels), and the family's time is the sum over its kernels.
struct ProfScope : gst::LaunchTimer {
  gst_ctx* c;
  int fam;
  gst::LaunchTimer* prev = nullptr;
  ProfScope* outer = nullptr;  // the enclosing scope, if one is timing
  bool active = false;
  ProfScope(gst_ctx* ctx, int family) : c(ctx), fam(family) {
    // a family indexes the profiler's per-family arrays
    if (fam < 0 || fam >= FAM_N) return;
    if (c && c->prof.on && (c->prof.only < 0 || c->prof.only == fam)) {
      active = true;
      prev = gst::launch_timer();
      outer = dynamic_cast<ProfScope*>(prev);
      gst::launch_timer() = this;
    }
  }
  bool events(hipEvent_t* start, hipEvent_t* stop) override {
    hipEvent_t a = c->prof.get(), b = c->prof.get();
    if (!a || !b) {
      if (a) c->prof.pool.push_back(a);
      if (b) c->prof.pool.push_back(b);
      return false;
    }
    c->prof.pending.push_back({fam, a, b, true});
    for (ProfScope* o = outer; o; o = o->outer) c->prof.pending.push_back({o->fam, a, b, false});
    *start = a;
    *stop = b;
    return true;
  }
  ~ProfScope() override {
    if (active) gst::launch_timer() = prev;
  }
};

// Device copy of a sharing plan (gst_plan.h).
struct DevicePlan {
  bool used = false;
  gst::HostPlan host;                    // kept for sizes and level ranges
  std::vector<int64_t> inj_level_ptr;    // [n_levels + 1] injection slot ranges per level
  DevBuf buf;
  int64_t* items = nullptr;
  int64_t* trunk_ptr = nullptr;
  int64_t* trunk_anchor = nullptr;

  int64_t* inj_ptr = nullptr;
  int32_t* item_src = nullptr;
  uint8_t* item_kv = nullptr;
  int32_t* item_cnt = nullptr;   // counts in item order (null without counts)
  int32_t* trunk_src = nullptr;
  int64_t* op_ptr = nullptr;
  uint32_t* op_desc = nullptr;
  int32_t* op_slot = nullptr;
  int64_t* item_step_ptr = nullptr;
  int64_t* rec_b = nullptr;
  int64_t* rec_f = nullptr;
  int64_t* chunk_gate = nullptr;
  int64_t* chunk_beg = nullptr;
  int64_t* chunk_end = nullptr;
  double* FA = nullptr;         // state arena [1 + trunk_steps + item_steps][D]
  double* BA = nullptr;         // adjoint arena [trunk_steps + item_steps][D]
  double* src_adj = nullptr;    // [source rows][D]: adjoints arriving at stored states, slot by slot
  double* inj = nullptr;        // [n_inj][D]
  // germ-power jumps: each trunk's jump pattern, and the fill tasks
  uint32_t* trunk_jpat = nullptr;
  uint8_t* trunk_jg3 = nullptr;
  uint8_t* trunk_jlev = nullptr;
  double* jump_t = nullptr;      // [n_trunks][jump_levels][256]: the jump matrices, transposed
  int64_t* fill_first = nullptr;
  int64_t* fill_in = nullptr;
  int32_t* fill_n = nullptr;
  uint32_t* fill_pattern = nullptr;
  uint8_t* fill_gate3 = nullptr;
};

// Levels whose longest chain has at least this many steps run the sweeps
// with the gate operands held in registers (loaded once per tile); the others
// load each step's operands (a tile of a few steps would load all K gates for
// nothing).
constexpr int kRegGateSteps = 32;

// Device copy of a three-qubit grouped-chain plan (gst_plan64.h) with its
// arenas: the states and adjoints of every trie node, the seeds and chain
// adjoints, the rearranged gate set and the partial sums.
struct DevicePlan64 {
  bool used = false;
  gst::Plan64 host;          // sizes and level ranges (the big arrays are released after upload)
  std::vector<int64_t> level_tile_ptr;
  std::vector<char> level_long;  // per level: chains long enough to keep the gates in registers
  DevBuf buf;
  int64_t *tile_row0 = nullptr, *tile_word = nullptr, *tile_ev = nullptr, *col_anchor = nullptr,
          *col_chain = nullptr, *ev_ptr = nullptr, *ev_src = nullptr, *slot_row = nullptr, *slot_ptr = nullptr,
          *slot_seq = nullptr, *slot_pack = nullptr, *root_chains = nullptr, *ts_tile = nullptr, *chunk_beg = nullptr,
          *chunk_end = nullptr, *gate_chunk_ptr = nullptr;
  int32_t *tile_len = nullptr, *ts_step = nullptr, *slot_cnt = nullptr;
  uint8_t* ev_cend = nullptr;
  uint8_t* words = nullptr;
  int64_t* lvl_tile = nullptr;   // device copies of level_tile_ptr and level_long
  uint8_t* lvl_long = nullptr;
  double *FA = nullptr, *BA = nullptr, *INJ = nullptr, *GA = nullptr, *GAT = nullptr, *slab = nullptr,
         *part = nullptr, *chunk_slab = nullptr, *root_vec = nullptr;
  int readout_blocks = 0;
  int n_root_chains = 0;
  int64_t n_chunks = 0;
};

// Sequences per batch tile: a request's sequences, sorted by length, are cut
// into tiles of this many (16 chains x 8); fixed, so a request's tiling and
// summation order depend on the request alone.
// Sequences per tile of a request: a multiple of the 16 chains of one
// workgroup, chosen from S alone so that the cut (and with it the order of
// the partial sums) is a property of the request.
// Device words of a request's work-queue area: six queue counters 16 words
// apart (zeroed by the queue-reset kernel), then the nonpos counter (64-bit).
constexpr int kQueueWords = 96;

static int64_t tile_seqs_for(int64_t S) {
  const int64_t per = (S + 16 * 1024 - 1) / (16 * 1024);
  return 16 * std::min<int64_t>(std::max<int64_t>(per, 1), 8);
}

struct gst_req {
  gst_ctx* ctx = nullptr;
  int n_qubits = 0, D = 0, M = 0, K = 0;
  int64_t S = 0, max_len = 0;
  double total_counts = 0.0;  // sum of all counts (the fit's per-shot scale)
  DevBuf data;  // offsets | gate indices | counts | order | tile slabs
  int64_t* offsets = nullptr;
  uint8_t* gates = nullptr;
  int32_t* counts = nullptr;
  int64_t* order = nullptr;             // sequences by length, descending
  std::vector<int64_t> tile_q;          // tile boundaries in `order` (n_tiles + 1)
  std::vector<int64_t> tile_cost;       // summed lengths per tile
  double* tile_slab = nullptr;          // [n_tiles][P]
  gst::BatchTile* tiles = nullptr;      // device tile list of the request alone (longest first)
  unsigned* queue = nullptr;            // device: work-queue counter [64] + nonpos counter
  int64_t n_steps = 0;
  // three-qubit requests (D = 64)
  int64_t tile_seqs64 = 0, n_tiles64 = 0, n_chunks64 = 0;
  int64_t* pos64 = nullptr;             // step positions grouped by gate
  int64_t* chunk_beg64 = nullptr;
  int64_t* chunk_end64 = nullptr;
  int64_t* gate_chunk_ptr64 = nullptr;  // [K + 1]
  double* tile_slab64 = nullptr;        // [n_tiles64][1 + 64 + 64 M]
  double* chunk_slab64 = nullptr;       // [n_chunks64][4096]
  double* part64 = nullptr;             // scratch of the ordered tile reduction
  size_t eval_ws_bytes = 0;             // context workspace one evaluation with gradient needs
  DevicePlan plan;
  DevicePlan64 plan64;
  DevBuf ws;
  size_t resident_bytes = 0;
  int64_t n_tiles() const { return tile_q.empty() ? 0 : (int64_t)tile_q.size() - 1; }
};

struct gst_batch {
  gst_ctx* ctx = nullptr;
  std::vector<gst_req*> reqs;
  std::vector<gst_gateset> thetas;
  std::vector<double*> probs, objectives, grads;
  std::vector<int> plan_reqs;           // three qubits without the grouped-chain plan: their own launch sequences
  // three-qubit grouped-chain plans: one launch per kernel and level for all of them
  struct P64Group {
    int n = 0, K_max = 1, n_levels = 0, ro_grid = 0, gemm_grid = 0, red_x = 0, red_parts = 1, r64_x = 0;
    bool any_grad = false, any_slab = false;
    std::vector<int> grid_long, grid_short;  // per level: most tiles of a request's level of each kind
    const gst::Plan64Req* dev = nullptr;
  } p64;
  // one- and two-qubit sharing plans, batched per D (0: D = 4, 1: D = 16): one
  // launch per kernel and level for all of them
  struct PlanGroup {
    int D = 0, n = 0, K_max = 1, M_max = 1, jl_max = 0, n_levels = 0;
    bool any_grad = false, any_slab = false;
    std::vector<int> fwd_grid, bwd_grid, inj_grid;  // per level
    int item_grid = 0, fill_grid = 0, gemm_grid = 0, red_x = 0, red_parts = 1;
    gst::PlanBatch dev{};
  } pgroup[2];
  DevBuf plan_ws;                       // the batched plans' scratch, one region per request
  // one group of tiles per tile kernel (see TileKind), each with its own queue
  int n_tiles[6] = {0, 0, 0, 0, 0, 0}, grid_of[6] = {0, 0, 0, 0, 0, 0};
  gst::BatchLaunch launch[6] = {};
  int n_items = 0, kmax = 1;
  int red_chunks = 0;                   // most chunks of the tile-slab sum over the requests
  int64_t max_len = 0;
  DevBuf desc;
  gst::BatchReduce red{};
  unsigned long long* req_nonpos = nullptr;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  ~gst_batch() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
  }
};

// Checkpoint rows per chain of the tile kernel for sequences up to max_len.
static int64_t tile_ckpt_per_team(int64_t max_len) {
  const int C = gst::leaf_ckpt_interval(16);
  return ((max_len + C - 1) / C + 1) * 16;
}

// Tile kernels of the requests without a plan.  Group g of a batch: 0 = the
// 16-lane-team kernel for two qubits, 1 = the same for one qubit with more
// than four gates, 2 + K - 1 = the lane-per-chain one-qubit kernel for K
// gates (K <= 4).
static int tile_group(int D, int K) { return D == 16 ? 0 : (gst::lane1q_supported(K) ? 1 + K : 1); }
static bool group_is_lane(int g) { return g >= 2; }
// Sequences per tile: the context's tuned value (rounded up to the kernel's
// granularity: 64 for the lane kernel, 16 for the team kernels) or the
// default.  Fixed into the request when it is created.
static int64_t tile_seqs_of_group(const gst_ctx* ctx, int g, int64_t S) {
  const int t = ctx->tune_tile[g == 0 ? 2 : 1];
  const int64_t gran = group_is_lane(g) ? 64 : 16;
  if (t > 0) return (t + gran - 1) / gran * gran;
  return group_is_lane(g) ? 64 : tile_seqs_for(S);
}
static int group_family(int g) { return g == 0 ? FAM_TILES16 : FAM_TILES4; }

// Workgroups of a launch over n tiles (lane kernel: four waves, one tile each).
static int capped(int bpc, int cap) { return cap > 0 ? std::min(bpc, cap) : bpc; }

static int group_grid(gst_ctx* ctx, int g, int kmax, int64_t n) {
  if (n <= 0) return 0;
  const int cap = ctx->tune_bpc[g == 0 ? 2 : 1];
  if (group_is_lane(g)) {
    const int64_t blocks = (n + 3) / 4;
    return (int)std::min<int64_t>(blocks, (int64_t)capped(gst::lane1q_blocks_per_cu(g - 1), cap) * ctx->n_cu);
  }
  return (int)std::min<int64_t>(n, (int64_t)capped(gst::batch_blocks_per_cu(g == 0 ? 16 : 4, kmax), cap) * ctx->n_cu);
}

// Checkpoint doubles of one chain group (team or wave) and of a whole launch.
static int64_t group_ckpt_stride(int g, int64_t max_len) {
  return group_is_lane(g) ? gst::lane1q_ckpt_per_wave(max_len) : tile_ckpt_per_team(max_len);
}
static size_t group_ckpt_doubles(int g, int grid, int64_t max_len) {
  return (size_t)grid * (group_is_lane(g) ? 4 : gst::leaf_teams_per_block(16)) * group_ckpt_stride(g, max_len);
}

static hipError_t group_launch(int g, const gst::BatchLaunch& l, int grid, hipStream_t stream) {
  return group_is_lane(g) ? gst::launch_lane1q(l, g - 1, grid, stream) : gst::launch_batch(l, grid, stream);
}


namespace {

int check_gateset(const gst_gateset* gs, int* D) {
  if (!gs) return fail(GST_EINVAL, "gateset is NULL");
  const int d = dim_of(gs->n_qubits);
  if (!d) return fail(GST_EINVAL, "n_qubits must be 1, 2 or 3");
  if (gs->n_gates < 1 || gs->n_gates > gst_max_gates(gs->n_qubits))
    return fail(GST_EINVAL, "n_gates out of range for this qubit count (see gst_max_gates)");
  if (gs->n_outcomes < 1 || gs->n_outcomes > std::min(d, 16))
    return fail(GST_EINVAL, "n_outcomes must be in 1..min(D, 16)");
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

// Scratch of the sequence kernel and its slab reduction: the slab of partial
// sums, their first-stage sums and the checkpoints of the reverse sweeps.
struct LeafScratch {
  int blocks = 0;
  int64_t P = 0, ck_team = 0;
  size_t slab_bytes = 0, part_bytes = 0, ck_bytes = 0;
  size_t total() const { return slab_bytes + part_bytes + ck_bytes; }
};
LeafScratch leaf_scratch(const gst::LeafLaunch& a, int64_t max_len) {
  LeafScratch z;
  const int D = a.D;
  const bool need_slab = a.want_grad || a.mode == gst::MODE_LOGLIK;
  z.blocks = gst::leaf_blocks_for(D, a.n_items);
  z.P = gst::slab_width(D, a.M, a.K);
  const int C = gst::leaf_ckpt_interval(D);
  z.ck_team = a.want_grad ? ((max_len + C - 1) / C + 1) * 16 : 0;
  z.slab_bytes = need_slab ? (size_t)z.blocks * z.P * 8 : 0;
  z.part_bytes = need_slab ? (size_t)gst::reduce_parts(z.blocks) * z.P * 8 : 0;
  z.ck_bytes = (size_t)z.blocks * gst::leaf_teams_per_block(D) * z.ck_team * 8;
  return z;
}

// Enqueue the sequence kernel over `n_items` work items and the slab
// reduction, with their scratch at `buf` (leaf_scratch(...).total() bytes).
int enqueue_leaf(gst_ctx* ctx, const gst::LeafLaunch& base, int64_t max_len, double* objective, double* grad,
                 void* buf) {
  gst::LeafLaunch a = base;
  const int D = a.D;
  const bool need_slab = a.want_grad || a.mode == gst::MODE_LOGLIK;
  const LeafScratch z = leaf_scratch(a, max_len);
  const int blocks = z.blocks;
  const int64_t P = z.P;
  a.slab = need_slab ? reinterpret_cast<double*>(buf) : nullptr;
  double* part = reinterpret_cast<double*>((char*)buf + z.slab_bytes);
  a.ckpt = a.want_grad ? reinterpret_cast<double*>((char*)buf + z.slab_bytes + z.part_bytes) : nullptr;
  const int64_t ck_team = z.ck_team;
  a.ckpt_per_team = ck_team;
  a.max_len = (int)max_len;
  a.status = ctx->status;
  if (max_len > (int64_t)1 << 30) return fail(GST_EINVAL, "sequence too long");
  {
    ProfScope ps(ctx, FAM_LEAF);
    HIP_TRY(gst::launch_leaf(a, blocks, ctx->stream));
  }
  if (need_slab) {
    ProfScope ps(ctx, FAM_REDUCE);
    HIP_TRY(gst::launch_reduce(a.slab, blocks, P, objective, grad, nullptr, D, part, ctx->stream));
  }
  return GST_OK;
}

int run_leaf(gst_ctx* ctx, DevBuf& ws, const gst::LeafLaunch& base, int64_t max_len, double* objective,
             double* grad) {
  int rc = ws.reserve(leaf_scratch(base, max_len).total() + 256, ctx->stream);
  if (rc) return rc;
  return enqueue_leaf(ctx, base, max_len, objective, grad, ws.p);
}

int plain_eval64(gst_ctx* ctx, const gst_gateset* gs, const gst_seqlist* sl, int mode, const int32_t* counts,
                 const double* w, double* probs, double* objective, double* grad);

gst::LeafLaunch plain_launch(int D, const gst_gateset* gs, const gst_seqlist* sl, int mode, const int32_t* counts,
                             const double* w, double* probs, double* grad);

int plain_eval(gst_ctx* ctx, const gst_gateset* gs, const gst_seqlist* sl, int mode, const int32_t* counts,
               const double* w, double* probs, double* objective, double* grad) {
  if (!ctx) return fail(GST_EINVAL, "ctx is NULL");
  int D = 0;
  int rc = check_gateset(gs, &D);
  if (rc) return rc;
  rc = check_seqs(sl);
  if (rc) return rc;
  HIP_TRY(hipSetDevice(ctx->device));
  if (D == 64) return plain_eval64(ctx, gs, sl, mode, counts, w, probs, objective, grad);
  int64_t max_len = 0;
  rc = resolve_max_len(sl, ctx->stream, &max_len);
  if (rc) return rc;
  const gst::LeafLaunch a = plain_launch(D, gs, sl, mode, counts, w, probs, grad);
  return run_leaf(ctx, ctx->ws, a, max_len, objective, grad);
}

gst::LeafLaunch plain_launch(int D, const gst_gateset* gs, const gst_seqlist* sl, int mode, const int32_t* counts,
                             const double* w, double* probs, double* grad) {
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
  return a;
}

int upload_plan(gst_req* r, const gst::HostPlan& P, const int32_t* counts_host) {
  DevicePlan& d = r->plan;
  d.host = P;
  const int D = r->D;
  const int64_t nI = P.n_items(), nT = P.n_trunks(), nTS = P.trunk_steps(), nJ = (int64_t)P.inj_loc.size(),
                nIS = P.item_steps(), nR = (int64_t)P.rec_b.size(), nC = P.n_chunks();
  // injection list of each trunk, steps descending
  Carver c;
  const size_t nOp = P.op_desc.size();
  const size_t o_op = c.take<int64_t>(nT + 1), o_od = c.take<uint32_t>(nOp + 1), o_os = c.take<int32_t>(nOp + 1);
  const size_t o_items = c.take<int64_t>(4 * nI), o_tp = c.take<int64_t>(nT + 1), o_ta = c.take<int64_t>(nT + 1),
               o_ip = c.take<int64_t>(nJ + 1),
               o_isrc = c.take<int32_t>(nI + 1), o_ikv = c.take<uint8_t>((size_t)nI * 16 + 1),
               o_icnt = c.take<int32_t>((size_t)nI * r->M + 1), o_tsrc = c.take<int32_t>(nT + 1), o_isp = c.take<int64_t>(nI + 1),
               o_rb = c.take<int64_t>(nR + 1), o_rf = c.take<int64_t>(nR + 1), o_cg = c.take<int64_t>(nC + 1),
               o_cb = c.take<int64_t>(nC + 1), o_ce = c.take<int64_t>(nC + 1),
               o_fa = c.take<double>((size_t)(1 + nTS + nIS) * D), o_ba = c.take<double>((size_t)(nTS + nIS + 1) * D),
               o_src = c.take<double>((size_t)(P.n_src_rows() + 1) * D), o_inj = c.take<double>((size_t)(nJ + 1) * D);
  const size_t nF = P.fill_first.size();
  const size_t o_jp = c.take<uint32_t>(nT + 1), o_jg3 = c.take<uint8_t>(nT + 1), o_jlv = c.take<uint8_t>(nT + 1),
               o_jt = c.take<double>((size_t)nT * std::max(P.jump_levels, 1) * 256 + 1), o_ff = c.take<int64_t>(nF + 1),
               o_fi = c.take<int64_t>(nF + 1), o_fn = c.take<int32_t>(nF + 1), o_fp = c.take<uint32_t>(nF + 1),
               o_fg3 = c.take<uint8_t>(nF + 1);
  int rc = d.buf.reserve(c.off + 256, r->ctx->stream);
  if (rc) return rc;
  char* b = reinterpret_cast<char*>(d.buf.p);
  d.op_ptr = reinterpret_cast<int64_t*>(b + o_op);
  d.op_desc = reinterpret_cast<uint32_t*>(b + o_od);
  d.op_slot = reinterpret_cast<int32_t*>(b + o_os);
  d.items = reinterpret_cast<int64_t*>(b + o_items);
  d.trunk_ptr = reinterpret_cast<int64_t*>(b + o_tp);
  d.trunk_anchor = reinterpret_cast<int64_t*>(b + o_ta);
  d.inj_ptr = reinterpret_cast<int64_t*>(b + o_ip);
  d.item_src = reinterpret_cast<int32_t*>(b + o_isrc);
  d.item_kv = reinterpret_cast<uint8_t*>(b + o_ikv);
  d.item_cnt = counts_host ? reinterpret_cast<int32_t*>(b + o_icnt) : nullptr;
  d.trunk_src = reinterpret_cast<int32_t*>(b + o_tsrc);
  d.item_step_ptr = reinterpret_cast<int64_t*>(b + o_isp);
  d.rec_b = reinterpret_cast<int64_t*>(b + o_rb);
  d.rec_f = reinterpret_cast<int64_t*>(b + o_rf);
  d.chunk_gate = reinterpret_cast<int64_t*>(b + o_cg);
  d.chunk_beg = reinterpret_cast<int64_t*>(b + o_cb);
  d.chunk_end = reinterpret_cast<int64_t*>(b + o_ce);
  d.FA = reinterpret_cast<double*>(b + o_fa);
  d.BA = reinterpret_cast<double*>(b + o_ba);
  d.src_adj = reinterpret_cast<double*>(b + o_src);
  d.inj = reinterpret_cast<double*>(b + o_inj);
  d.trunk_jpat = reinterpret_cast<uint32_t*>(b + o_jp);
  d.trunk_jg3 = reinterpret_cast<uint8_t*>(b + o_jg3);
  d.trunk_jlev = reinterpret_cast<uint8_t*>(b + o_jlv);
  d.jump_t = reinterpret_cast<double*>(b + o_jt);
  d.fill_first = reinterpret_cast<int64_t*>(b + o_ff);
  d.fill_in = reinterpret_cast<int64_t*>(b + o_fi);
  d.fill_n = reinterpret_cast<int32_t*>(b + o_fn);
  d.fill_pattern = reinterpret_cast<uint32_t*>(b + o_fp);
  d.fill_gate3 = reinterpret_cast<uint8_t*>(b + o_fg3);
  auto put = [&](void* dst, const void* src, size_t bytes) -> int {
    if (bytes) HIP_TRY(hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice));
    return GST_OK;
  };
  if ((rc = put(d.op_ptr, P.op_ptr.data(), P.op_ptr.size() * 8))) return rc;
  if ((rc = put(d.op_desc, P.op_desc.data(), nOp * 4))) return rc;
  if ((rc = put(d.op_slot, P.op_slot.data(), nOp * 4))) return rc;
  if ((rc = put(d.items, P.items.data(), P.items.size() * 8))) return rc;
  if ((rc = put(d.trunk_ptr, P.trunk_ptr.data(), P.trunk_ptr.size() * 8))) return rc;
  if ((rc = put(d.trunk_anchor, P.trunk_anchor.data(), P.trunk_anchor.size() * 8))) return rc;
  if ((rc = put(d.inj_ptr, P.inj_ptr.data(), P.inj_ptr.size() * 8))) return rc;
  if ((rc = put(d.item_src, P.item_src.data(), (size_t)nI * 4))) return rc;
  if ((rc = put(d.item_kv, P.item_kv.data(), P.item_kv.size()))) return rc;
  if (counts_host) {
    std::vector<int32_t> cnt((size_t)nI * r->M);
    for (int64_t q = 0; q < nI; ++q)
      for (int m = 0; m < r->M; ++m) cnt[(size_t)q * r->M + m] = counts_host[P.items[4 * q] * r->M + m];
    if ((rc = put(d.item_cnt, cnt.data(), cnt.size() * 4))) return rc;
  }
  if ((rc = put(d.trunk_src, P.trunk_src.data(), (size_t)nT * 4))) return rc;
  if ((rc = put(d.item_step_ptr, P.item_step_ptr.data(), P.item_step_ptr.size() * 8))) return rc;
  if ((rc = put(d.rec_b, P.rec_b.data(), P.rec_b.size() * 8))) return rc;
  if ((rc = put(d.rec_f, P.rec_f.data(), P.rec_f.size() * 8))) return rc;
  if ((rc = put(d.chunk_gate, P.chunk_gate.data(), P.chunk_gate.size() * 8))) return rc;
  if ((rc = put(d.chunk_beg, P.chunk_beg.data(), P.chunk_beg.size() * 8))) return rc;
  if ((rc = put(d.chunk_end, P.chunk_end.data(), P.chunk_end.size() * 8))) return rc;
  if ((rc = put(d.trunk_jpat, P.trunk_jump_pattern.data(), P.trunk_jump_pattern.size() * 4))) return rc;
  if ((rc = put(d.trunk_jg3, P.trunk_jump_gate3.data(), P.trunk_jump_gate3.size()))) return rc;
  if ((rc = put(d.trunk_jlev, P.trunk_jump_levels.data(), P.trunk_jump_levels.size()))) return rc;
  if ((rc = put(d.fill_first, P.fill_first.data(), nF * 8))) return rc;
  if ((rc = put(d.fill_in, P.fill_in.data(), nF * 8))) return rc;
  if ((rc = put(d.fill_n, P.fill_n.data(), nF * 4))) return rc;
  if ((rc = put(d.fill_pattern, P.fill_pattern.data(), nF * 4))) return rc;
  if ((rc = put(d.fill_gate3, P.fill_gate3.data(), nF))) return rc;
  // injection slots of each level: slots of stored locations are sorted by
  // location (the root slot comes last) and a level's locations are contiguous
  d.inj_level_ptr.assign(P.n_levels + 1, 0);
  const auto loc_end = P.inj_loc.begin() + P.root_slot;
  for (int l = 0; l <= P.n_levels; ++l) {
    const int64_t loc = P.trunk_ptr[P.trunk_level_ptr[l]];
    d.inj_level_ptr[l] = std::lower_bound(P.inj_loc.begin(), loc_end, loc) - P.inj_loc.begin();
  }
  d.inj_level_ptr[P.n_levels] = P.root_slot;
  d.used = true;
  return GST_OK;
}

int upload_plan64(gst_req* r, gst::Plan64& P, const int32_t* counts_host) {
  DevicePlan64& d = r->plan64;
  const int M = r->M, K = r->K;
  const int64_t T = P.n_tiles(), TS = P.tile_steps(), NE = (int64_t)P.ev_col.size(), NR = (int64_t)P.ts_tile.size(),
                NC = (int64_t)P.chunk_beg.size(), NRC = (int64_t)P.root_chains.size();
  // the reverse kernel finds a column's events through the per-step table and
  // stages the events' INJ rows as 32-bit indices
  if ((int64_t)P.ev_cend.size() != TS * 16 || P.n_slots + P.n_chains >= INT32_MAX) return GST_EINVAL;
  // the gradient GEMM stages a chunk's rows in LDS
  for (int64_t i = 0; i < NC; ++i)
    if (P.chunk_end[i] - P.chunk_beg[i] > gst::GEMM64_TS_CHUNK_MAX) return GST_EINVAL;
  // the readout takes groups of 16 slots, a wave per group at a time
  const int64_t n_groups = (P.n_slots + 15) / 16;
  d.readout_blocks = (int)std::min<int64_t>(std::max<int64_t>((n_groups + gst::READOUT64_WAVES - 1) /
                                                                  gst::READOUT64_WAVES, 1),
                                            (int64_t)gst::readout64_blocks_per_cu() * r->ctx->n_cu);
  const int64_t n_waves = (int64_t)d.readout_blocks * gst::READOUT64_WAVES;
  const int64_t Pc = 1 + 64 + (int64_t)M * 64;
  Carver c;
  const size_t o_r0 = c.take<int64_t>(T + 1), o_len = c.take<int32_t>(T + 1), o_w = c.take<int64_t>(T + 1),
               o_tev = c.take<int64_t>(T + 1), o_anc = c.take<int64_t>(T * 16 + 1), o_ch = c.take<int64_t>(T * 16 + 1),
               o_words = c.take<uint8_t>(P.words.size() + 1), o_evp = c.take<int64_t>(TS + 2),
               o_evc = c.take<uint8_t>(TS * 16 + 16), o_evs = c.take<int64_t>(NE + 1),
               o_sr = c.take<int64_t>(P.n_slots + 1), o_sp = c.take<int64_t>(P.n_slots + 2),
               o_sq = c.take<int64_t>(P.S + 1), o_spk = c.take<int64_t>(P.n_slots * 4 + 4),
               o_scn = c.take<int32_t>(P.n_slots * M + 1), o_rc = c.take<int64_t>(NRC + 1),
               o_rb = c.take<int64_t>(NR + 1),
               o_rf = c.take<int32_t>(NR + 1), o_cb = c.take<int64_t>(NC + 1), o_ce = c.take<int64_t>(NC + 1),
               o_gcp = c.take<int64_t>(K + 1), o_fa = c.take<double>((size_t)P.n_rows * 64),
               o_ba = c.take<double>((size_t)P.n_rows * 64),
               o_inj = c.take<double>((size_t)(P.n_slots + P.n_chains + 1) * 64),
               o_ga = c.take<double>((size_t)K * 4096), o_gat = c.take<double>((size_t)K * 4096),
               o_slab = c.take<double>((size_t)n_waves * Pc),
               o_part = c.take<double>((size_t)gst::reduce_parts((int)n_waves) * Pc),
               o_cs = c.take<double>((size_t)std::max<int64_t>(NC, 1) * 4096), o_root = c.take<double>(64),
               o_lt = c.take<int64_t>(P.n_levels + 1), o_ll = c.take<uint8_t>(P.n_levels + 1);
  int rc = d.buf.reserve(c.off + 256, r->ctx->stream);
  if (rc) return rc;
  char* b = reinterpret_cast<char*>(d.buf.p);
  d.tile_row0 = reinterpret_cast<int64_t*>(b + o_r0);
  d.tile_len = reinterpret_cast<int32_t*>(b + o_len);
  d.tile_word = reinterpret_cast<int64_t*>(b + o_w);
  d.tile_ev = reinterpret_cast<int64_t*>(b + o_tev);
  d.col_anchor = reinterpret_cast<int64_t*>(b + o_anc);
  d.col_chain = reinterpret_cast<int64_t*>(b + o_ch);
  d.words = reinterpret_cast<uint8_t*>(b + o_words);
  d.ev_ptr = reinterpret_cast<int64_t*>(b + o_evp);
  d.ev_cend = reinterpret_cast<uint8_t*>(b + o_evc);
  d.ev_src = reinterpret_cast<int64_t*>(b + o_evs);
  d.slot_row = reinterpret_cast<int64_t*>(b + o_sr);
  d.slot_ptr = reinterpret_cast<int64_t*>(b + o_sp);
  d.slot_seq = reinterpret_cast<int64_t*>(b + o_sq);
  d.slot_pack = reinterpret_cast<int64_t*>(b + o_spk);
  d.slot_cnt = reinterpret_cast<int32_t*>(b + o_scn);
  d.root_chains = reinterpret_cast<int64_t*>(b + o_rc);
  d.ts_tile = reinterpret_cast<int64_t*>(b + o_rb);
  d.ts_step = reinterpret_cast<int32_t*>(b + o_rf);
  d.chunk_beg = reinterpret_cast<int64_t*>(b + o_cb);
  d.chunk_end = reinterpret_cast<int64_t*>(b + o_ce);
  d.gate_chunk_ptr = reinterpret_cast<int64_t*>(b + o_gcp);
  d.FA = reinterpret_cast<double*>(b + o_fa);
  d.BA = reinterpret_cast<double*>(b + o_ba);
  d.INJ = reinterpret_cast<double*>(b + o_inj);
  d.GA = reinterpret_cast<double*>(b + o_ga);
  d.GAT = reinterpret_cast<double*>(b + o_gat);
  d.slab = reinterpret_cast<double*>(b + o_slab);
  d.part = reinterpret_cast<double*>(b + o_part);
  d.chunk_slab = reinterpret_cast<double*>(b + o_cs);
  d.root_vec = reinterpret_cast<double*>(b + o_root);
  d.lvl_tile = reinterpret_cast<int64_t*>(b + o_lt);
  d.lvl_long = reinterpret_cast<uint8_t*>(b + o_ll);
  auto put = [&](void* dst, const void* src, size_t bytes) -> int {
    if (bytes) HIP_TRY(hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice));
    return GST_OK;
  };
  if ((rc = put(d.tile_row0, P.tile_row0.data(), T * 8))) return rc;
  if ((rc = put(d.tile_len, P.tile_len.data(), T * 4))) return rc;
  if ((rc = put(d.tile_word, P.tile_word.data(), T * 8))) return rc;
  if ((rc = put(d.tile_ev, P.tile_ev.data(), T * 8))) return rc;
  if ((rc = put(d.col_anchor, P.col_anchor.data(), T * 16 * 8))) return rc;
  if ((rc = put(d.col_chain, P.col_chain.data(), T * 16 * 8))) return rc;
  if ((rc = put(d.words, P.words.data(), P.words.size()))) return rc;
  if ((rc = put(d.ev_ptr, P.ev_ptr.data(), P.ev_ptr.size() * 8))) return rc;
  if ((rc = put(d.ev_cend, P.ev_cend.data(), TS * 16))) return rc;
  if ((rc = put(d.ev_src, P.ev_src.data(), NE * 8))) return rc;
  if ((rc = put(d.slot_row, P.slot_row.data(), P.n_slots * 8))) return rc;
  if ((rc = put(d.slot_ptr, P.slot_ptr.data(), P.slot_ptr.size() * 8))) return rc;
  if ((rc = put(d.slot_seq, P.slot_seq.data(), P.slot_seq.size() * 8))) return rc;
  {
    // per slot: its node row, its first sequence and its sequence range, and
    // the first sequence's counts (the readout loads them together, by slot)
    std::vector<int64_t> pack((size_t)P.n_slots * 4);
    std::vector<int32_t> cnt((size_t)P.n_slots * M, 0);
    for (int64_t x = 0; x < P.n_slots; ++x) {
      const int64_t q0 = P.slot_ptr[x], q1 = P.slot_ptr[x + 1];
      const int64_t seq0 = q1 > q0 ? P.slot_seq[q0] : 0;
      pack[4 * x + 0] = P.slot_row[x];
      pack[4 * x + 1] = seq0;
      pack[4 * x + 2] = q0;
      pack[4 * x + 3] = q1;
      if (counts_host && q1 > q0)
        for (int m = 0; m < M; ++m) cnt[(size_t)x * M + m] = counts_host[seq0 * M + m];
    }
    if ((rc = put(d.slot_pack, pack.data(), pack.size() * 8))) return rc;
    if ((rc = put(d.slot_cnt, cnt.data(), cnt.size() * 4))) return rc;
  }
  if ((rc = put(d.root_chains, P.root_chains.data(), NRC * 8))) return rc;
  if ((rc = put(d.ts_tile, P.ts_tile.data(), NR * 8))) return rc;
  if ((rc = put(d.ts_step, P.ts_step.data(), NR * 4))) return rc;
  if ((rc = put(d.chunk_beg, P.chunk_beg.data(), NC * 8))) return rc;
  if ((rc = put(d.chunk_end, P.chunk_end.data(), NC * 8))) return rc;
  if ((rc = put(d.gate_chunk_ptr, P.gate_chunk_ptr.data(), (K + 1) * 8))) return rc;
  d.level_tile_ptr = P.level_tile_ptr;
  d.level_long.assign((size_t)P.n_levels, 0);
  for (int l = 0; l < P.n_levels; ++l)
    for (int64_t t = P.level_tile_ptr[l]; t < P.level_tile_ptr[l + 1]; ++t)
      if (P.tile_len[t] >= kRegGateSteps) d.level_long[l] = 1;
  if ((rc = put(d.lvl_tile, d.level_tile_ptr.data(), d.level_tile_ptr.size() * 8))) return rc;
  if ((rc = put(d.lvl_long, d.level_long.data(), d.level_long.size()))) return rc;
  d.n_root_chains = (int)NRC;
  d.n_chunks = NC;
  // keep the sizes, drop the host copies of the big arrays
  d.host = gst::Plan64();
  d.host.K = P.K;
  d.host.S = P.S;
  d.host.sum_len = P.sum_len;
  d.host.n_nodes = P.n_nodes;
  d.host.n_rows = P.n_rows;
  d.host.n_chains = P.n_chains;
  d.host.n_slots = P.n_slots;
  d.host.n_levels = P.n_levels;
  d.host.root_slot = P.root_slot;
  d.host.tile_row0.resize((size_t)T);  // n_tiles()
  d.used = true;
  return GST_OK;
}

// One evaluation with the grouped-chain plan (three qubits): the gate set
// rearranged for the MFMA operands, the chains forward level by level, the
// readouts per seed slot, the chains backward deepest level first, the
// gradient GEMM over the (adjoint, parent state) records, the root adjoint,
// and the ordered sums.
// The arguments of a request's grouped-chain evaluation: the standalone launch
// sequence below and the batched one (gst_batch_run) read the same values.
static gst::Plan64Req plan64_req(gst_req* r, const gst_gateset* th, int mode, const double* w, double* probs,
                                 double* objective, double* grad, unsigned long long* np) {
  DevicePlan64& d = r->plan64;
  const bool want_grad = grad != nullptr;
  const bool need_slab = objective || grad;
  gst::Plan64Req q{};
  gst::Plan64Launch& a = q.tiles;
  a.GA = d.GA;
  a.GAT = d.GAT;
  a.tile_row0 = d.tile_row0;
  a.tile_len = d.tile_len;
  a.tile_word = d.tile_word;
  a.tile_ev = d.tile_ev;
  a.col_anchor = d.col_anchor;
  a.col_chain = d.col_chain;
  a.words = d.words;
  a.ev_ptr = d.ev_ptr;
  a.ev_cend = d.ev_cend;
  a.ev_src = d.ev_src;
  a.FA = d.FA;
  a.BA = d.BA;
  a.INJ = d.INJ;
  a.n_slots = d.host.n_slots;
  a.K = r->K;
  q.level_tile = d.lvl_tile;
  q.level_long = d.lvl_long;
  q.n_levels = d.host.n_levels;
  q.want_grad = want_grad ? 1 : 0;
  q.G = th->gates;
  q.rho = th->rho;
  gst::Readout64Launch& ro = q.ro;
  ro.M = r->M;
  ro.E = th->effects;
  ro.FA = d.FA;
  ro.n_slots = d.host.n_slots;
  ro.slot_row = d.slot_row;
  ro.slot_ptr = d.slot_ptr;
  ro.slot_seq = d.slot_seq;
  ro.slot_pack = d.slot_pack;
  ro.slot_cnt = d.slot_cnt;
  ro.counts = r->counts;
  ro.W = w;
  ro.probs = probs;
  ro.mode = mode;
  ro.want_grad = want_grad ? 1 : 0;
  ro.INJ = d.INJ;
  ro.slab = need_slab ? d.slab : nullptr;
  ro.status = r->ctx->status;
  ro.nonpos = np;
  q.ro_blocks = d.readout_blocks;
  if (want_grad && d.n_chunks > 0) {
    gst::Gemm64TsLaunch& g = q.gemm;
    g.BA = d.BA;
    g.FA = d.FA;
    g.tile_row0 = d.tile_row0;
    g.col_anchor = d.col_anchor;
    g.ts_tile = d.ts_tile;
    g.ts_step = d.ts_step;
    g.chunk_beg = d.chunk_beg;
    g.chunk_end = d.chunk_end;
    g.slab = d.chunk_slab;
    g.n_chunks = (int)d.n_chunks;
  }
  q.root.INJ = d.INJ;
  q.root.root_slot = d.host.root_slot;
  q.root.n_slots = d.host.n_slots;
  q.root.root_chains = d.root_chains;
  q.root.n_root_chains = d.n_root_chains;
  q.root.out = d.root_vec;
  if (need_slab) {
    q.slab = d.slab;
    q.n_slabs = d.readout_blocks * gst::READOUT64_WAVES;
    q.red_parts = gst::reduce_parts(q.n_slabs);
    q.red_per = (q.n_slabs + q.red_parts - 1) / q.red_parts;
    q.P = 1 + 64 + (int64_t)r->M * 64;
    q.part = d.part;
    q.objective = objective;
    q.grad = grad;
    q.extra_rho = want_grad ? d.root_vec : nullptr;
    if (want_grad) {
      q.r64.M = r->M;
      q.r64.K = r->K;
      q.r64.chunk_slab = d.chunk_slab;
      q.r64.gate_chunk_ptr = d.gate_chunk_ptr;
      q.r64.grad = grad;
      q.r64.nonpos = np;
    }
  }
  return q;
}

int run_plan64(gst_req* r, const gst_gateset* th, int mode, const double* w, double* probs, double* objective,
               double* grad, unsigned long long* nonpos) {
  gst_ctx* ctx = r->ctx;
  DevicePlan64& d = r->plan64;
  const bool want_grad = grad != nullptr;
  unsigned long long* np = nonpos ? nonpos : reinterpret_cast<unsigned long long*>(r->queue + kQueueWords);
  HIP_TRY(gst::launch_queue_reset(r->queue, np, 1, ctx->stream));
  const gst::Plan64Req q = plan64_req(r, th, mode, w, probs, objective, grad, np);
  HIP_TRY(gst::launch_gate_prep64(q.G, q.rho, r->K, d.GA, d.GAT, d.FA, ctx->stream));
  gst::Plan64Launch a = q.tiles;
  const int L = d.host.n_levels;
  {
    ProfScope ps(ctx, FAM_P64_FWD);
    for (int l = 0; l < L; ++l) {
      a.t_begin = d.level_tile_ptr[l];
      HIP_TRY(gst::launch_plan64_fwd(a, (int)(d.level_tile_ptr[l + 1] - d.level_tile_ptr[l]), d.level_long[l] != 0,
                                     ctx->stream));
    }
  }
  {
    ProfScope ps(ctx, FAM_P64_READ);
    HIP_TRY(gst::launch_readout64(q.ro, q.ro_blocks, ctx->stream));
  }
  if (want_grad) {
    {
      ProfScope ps(ctx, FAM_P64_BWD);
      for (int l = L - 1; l >= 0; --l) {
        a.t_begin = d.level_tile_ptr[l];
        HIP_TRY(gst::launch_plan64_bwd(a, (int)(d.level_tile_ptr[l + 1] - d.level_tile_ptr[l]),
                                       d.level_long[l] != 0, ctx->stream));
      }
    }
    if (q.gemm.n_chunks > 0) {
      ProfScope ps(ctx, FAM_GEMM64);
      HIP_TRY(gst::launch_gemm64_ts(q.gemm, ctx->stream));
    }
    HIP_TRY(gst::launch_root64(q.root, ctx->stream));
  }
  if (q.slab) {
    ProfScope ps(ctx, FAM_REDUCE64);
    HIP_TRY(gst::launch_reduce(q.slab, q.n_slabs, q.P, q.objective, q.grad, q.extra_rho, 64, q.part, ctx->stream));
    if (want_grad) HIP_TRY(gst::launch_reduce64(q.r64, ctx->stream));
  }
  return GST_OK;
}

// One evaluation with the sharing plan: trunks forward (per level), items,
// injections and trunks backward (deepest level first), the gradient GEMM
// over all stored steps, and the slab reduction.
// The launch arguments of one evaluation of a request's sharing plan, and the
// sizes of its scratch: head rows [objective | dL/drho | dL/dE] from the item
// and trunk-backward workgroups, one D x D tile per gradient chunk, and the
// first-stage partials of the reduction.
struct PlanSetup {
  gst::PlanArgs a{};
  gst::InjectLaunch in{};
  gst::GemmLaunch g{};
  gst::PlanReduce red{};
  std::vector<int> tb_blocks, tb_at;  // per level: reverse trunk workgroups, their first head row
  bool want_grad = false, need_slab = false;
  int64_t H = 0;
  size_t head_bytes = 0, tile_bytes = 0, part_bytes = 0;
  size_t ws_bytes() const { return head_bytes + tile_bytes + part_bytes + 256; }
  void bind(void* ws) {
    double* slab = reinterpret_cast<double*>(ws);
    double* tiles = reinterpret_cast<double*>((char*)ws + head_bytes);
    double* part = reinterpret_cast<double*>((char*)ws + head_bytes + tile_bytes);
    a.slab = slab;
    g.tiles = tiles;
    red.head = slab;
    red.tiles = tiles;
    red.part = part;
  }
};

void plan_setup(gst_req* r, const gst_gateset* th, int mode, const double* w, double* probs, double* objective,
                double* grad, unsigned long long* req_nonpos, PlanSetup* out) {
  gst_ctx* ctx = r->ctx;
  const DevicePlan& d = r->plan;
  const gst::HostPlan& P = d.host;
  const int D = r->D;
  PlanSetup& s = *out;
  s.want_grad = grad != nullptr;
  s.need_slab = s.want_grad || mode == gst::MODE_LOGLIK;
  s.H = gst::slab_width(D, r->M, 0);
  const int64_t Pw = s.want_grad ? gst::slab_width(D, r->M, r->K) : s.H;
  // the item and fill workgroups of the launch within one round of resident
  // workgroups: past that the waves take several groups of items each, where
  // a second round of workgroups would start only as the first ends
  const int64_t resident = (int64_t)ctx->n_cu * gst::item_blocks_per_cu(D, r->K, r->M);
  const int64_t fill_blocks = s.want_grad && P.n_fill() > 0 ? gst::fill_blocks_for(P.n_fill()) : 0;
  const int item_blocks = gst::item_blocks_for(P.n_items(), std::max<int64_t>(resident - fill_blocks, resident / 2));
  s.tb_blocks.assign(P.n_levels, 0);
  s.tb_at.assign(P.n_levels, 0);
  // one head row per chunk of items (whatever the item workgroups), then one
  // per reverse trunk workgroup of each level
  int n_head = s.need_slab ? (int)((P.n_items() + gst::kItemChunk - 1) / gst::kItemChunk) : 0;
  for (int l = 0; l < P.n_levels; ++l) {
    s.tb_blocks[l] = gst::trunk_blocks_for(P.trunk_level_ptr[l + 1] - P.trunk_level_ptr[l]);
    s.tb_at[l] = n_head;
    if (s.want_grad) n_head += s.tb_blocks[l];
  }
  const int64_t n_chunks = s.want_grad ? P.n_chunks() : 0;
  gst::PlanReduce& red = s.red;
  red.D = D;
  red.M = r->M;
  red.K = s.want_grad ? r->K : 0;
  red.n_head = n_head;
  red.P = s.need_slab ? Pw : 0;
  red.n_part = gst::reduce_parts(n_head);
  for (int k = 0; k <= red.K; ++k) {
    red.chunk_ptr[k] = std::lower_bound(P.chunk_gate.begin(), P.chunk_gate.end(), (int64_t)k) - P.chunk_gate.begin();
    if (k > 0) {
      const int64_t nk = red.chunk_ptr[k] - red.chunk_ptr[k - 1];
      red.n_part = std::max(red.n_part, gst::reduce_parts((int)std::min<int64_t>(nk, 1 << 20)));
    }
  }
  red.objective = objective;
  red.grad = grad;
  s.head_bytes = (size_t)n_head * s.H * 8;
  s.tile_bytes = (size_t)n_chunks * D * D * 8;
  s.part_bytes = s.need_slab ? (size_t)red.n_part * Pw * 8 : 0;

  gst::PlanArgs& a = s.a;
  a.D = D;
  a.M = r->M;
  a.K = r->K;
  a.rho = th->rho;
  a.E = th->effects;
  a.G = th->gates;
  a.nTS = P.trunk_steps();
  a.trunk_ptr = d.trunk_ptr;
  a.trunk_anchor = d.trunk_anchor;
  a.trunk_src = d.trunk_src;
  a.op_ptr = d.op_ptr;
  a.op_desc = d.op_desc;
  a.op_slot = d.op_slot;
  a.n_items = P.n_items();
  a.items = d.items;
  a.item_step_ptr = d.item_step_ptr;
  a.gates = r->gates;
  a.item_src = d.item_src;
  a.item_kv = d.item_kv;
  a.item_cnt = d.item_cnt;
  a.counts = r->counts;
  a.W = w;
  a.probs = probs;
  a.mode = mode;
  a.want_grad = s.want_grad;
  a.FA = d.FA;
  a.BA = d.BA;
  a.src_adj = d.src_adj;
  a.inj = d.inj;
  a.status = ctx->status;
  a.req_nonpos = req_nonpos;
  a.trunk_jpat = d.trunk_jpat;
  a.trunk_jg3 = d.trunk_jg3;
  a.trunk_jlev = d.trunk_jlev;
  a.jump_t = d.jump_t;
  a.jump_levels = P.jump_levels;
  a.item_blocks = item_blocks;
  a.n_fill = P.n_fill();
  a.fill_first = d.fill_first;
  a.fill_in = d.fill_in;
  a.fill_n = d.fill_n;
  a.fill_pattern = d.fill_pattern;
  a.fill_gate3 = d.fill_gate3;
  a.n_levels = P.n_levels;
  a.fill_blocks = (int)fill_blocks;

  gst::InjectLaunch& in = s.in;
  in.D = D;
  in.inj_ptr = d.inj_ptr;
  in.src_adj = d.src_adj;
  in.inj = d.inj;
  in.n_levels = s.want_grad ? P.n_levels : 0;

  gst::GemmLaunch& g = s.g;
  g.D = D;
  g.M = r->M;
  g.K = r->K;
  g.n_chunks = n_chunks;
  g.chunk_gate = d.chunk_gate;
  g.chunk_beg = d.chunk_beg;
  g.chunk_end = d.chunk_end;
  g.rec_b = d.rec_b;
  g.rec_f = d.rec_f;
  g.FA = d.FA;
  g.BA = d.BA;
}

int run_plan(gst_req* r, const gst_gateset* th, int mode, const double* w, double* probs, double* objective,
             double* grad, unsigned long long* req_nonpos = nullptr) {
  gst_ctx* ctx = r->ctx;
  const DevicePlan& d = r->plan;
  const gst::HostPlan& P = d.host;
  PlanSetup s;
  plan_setup(r, th, mode, w, probs, objective, grad, req_nonpos, &s);
  int rc = r->ws.reserve(s.ws_bytes(), ctx->stream);
  if (rc) return rc;
  s.bind(r->ws.p);
  gst::PlanArgs a = s.a;
  double* slab = a.slab;
  for (int l = 0; l < P.n_levels; ++l) {
    a.t_begin = P.trunk_level_ptr[l];
    a.t_end = P.trunk_level_ptr[l + 1];
    ProfScope ps(ctx, FAM_TRUNK_FWD);
    HIP_TRY(gst::launch_trunk_fwd(a, ctx->stream));
  }
  {  // with the gradient, extra workgroups fill the states inside the jumps
    ProfScope ps(ctx, FAM_LEAF);
    HIP_TRY(gst::launch_items(a, a.item_blocks, ctx->stream));
  }
  if (s.want_grad) {
    gst::InjectLaunch in = s.in;
    for (int l = P.n_levels - 1; l >= 0; --l) {
      in.s_begin = d.inj_level_ptr[l];
      in.s_end = d.inj_level_ptr[l + 1];
      {
        ProfScope ps(ctx, FAM_INJECT);
        HIP_TRY(gst::launch_inject(in, ctx->stream));
      }
      a.t_begin = P.trunk_level_ptr[l];
      a.t_end = P.trunk_level_ptr[l + 1];
      a.slab = slab + (size_t)s.tb_at[l] * s.H;
      ProfScope ps(ctx, FAM_TRUNK_BWD);
      HIP_TRY(gst::launch_trunk_bwd(a, ctx->stream));
    }
    if (a.n_fill > 0) {
      ProfScope ps(ctx, FAM_FILL);
      HIP_TRY(gst::launch_fill_rev(a, ctx->stream));
    }
    ProfScope ps(ctx, FAM_GEMM);
    HIP_TRY(gst::launch_grad_gemm(s.g, ctx->stream));
  }
  if (s.need_slab) {
    ProfScope ps(ctx, FAM_REDUCE);
    HIP_TRY(gst::launch_reduce_plan(s.red, ctx->stream));
  }
  return GST_OK;
}

}  // namespace

int gst::ctx_device(const gst_ctx* ctx) { return ctx->device; }

// gst_loglik on the caller's scratch (see gst_noalloc.hip): one or two qubits,
// max_len given; no allocation anywhere on the way.
int gst::loglik_into_scratch(gst_ctx* ctx, const gst_gateset* gs, const gst_seqlist* sl, const int32_t* counts,
                             double* probs, double* objective, double* grad, void* scratch, size_t scratch_bytes) {
  if (!ctx) return fail(GST_EINVAL, "ctx is NULL");
  if (!objective) return fail(GST_EINVAL, "objective is NULL");
  int D = 0;
  int rc = check_gateset(gs, &D);
  if (rc) return rc;
  rc = check_seqs(sl);
  if (rc) return rc;
  if (D == 64) return fail(GST_EINVAL, "the allocation-free call takes one or two qubits");
  if (sl->max_len < 0) return fail(GST_EINVAL, "the allocation-free call needs max_len");
  if (sl->max_len > (int64_t)1 << 30) return fail(GST_EINVAL, "sequence too long");
  if (!scratch) return fail(GST_EDEVICE, "no scratch array on this device");
  const gst::LeafLaunch a = plain_launch(D, gs, sl, gst::MODE_LOGLIK, counts, nullptr, probs, grad);
  const size_t need = leaf_scratch(a, sl->max_len).total();
  if (need > scratch_bytes)
    return fail(GST_EINVAL, "the evaluation needs " + std::to_string(need) + " bytes of scratch, the array holds " +
                                std::to_string(scratch_bytes));
  HIP_TRY(hipSetDevice(ctx->device));
  return enqueue_leaf(ctx, a, sl->max_len, objective, grad, scratch);
}

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
  c->n_cu = prop.multiProcessorCount;
  c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  HIP_TRY(hipMalloc(&c->status, 2 * sizeof(unsigned long long)));
  HIP_TRY(hipMemset(c->status, 0, 2 * sizeof(unsigned long long)));
  const int rc = gst::scratch_bind(device_ordinal);
  if (rc) return fail(rc, "binding the scratch array of the allocation-free call failed");
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

int gst_tune_set(gst_ctx* ctx, int n_qubits, int seqs_per_tile, int blocks_per_cu) {
  if (!ctx) return fail(GST_EINVAL, "ctx is NULL");
  if (n_qubits < 1 || n_qubits > 3) return fail(GST_EINVAL, "n_qubits must be 1, 2 or 3");
  if (seqs_per_tile < 0 || seqs_per_tile > 4096 || blocks_per_cu < 0 || blocks_per_cu > 64)
    return fail(GST_EINVAL, "tile policy out of range");
  ctx->tune_tile[n_qubits] = seqs_per_tile;
  ctx->tune_bpc[n_qubits] = blocks_per_cu;
  return GST_OK;
}

int gst_predict(gst_ctx* ctx, const gst_gateset* theta, int n_prep, const int64_t* prep_offsets,
                const uint8_t* prep_gates, int n_gates, const int32_t* gates, int r_max, double* probs) {
  if (!ctx) return fail(GST_EINVAL, "ctx is NULL");
  int D = 0;
  int rc = check_gateset(theta, &D);
  if (rc) return rc;
  if (D > 16) return fail(GST_EINVAL, "predictions take one or two qubits");
  if (n_prep < 1 || n_gates < 1 || r_max < 0 || r_max > (1 << 24))
    return fail(GST_EINVAL, "n_prep, n_gates >= 1 and 0 <= r_max <= 2^24 required");
  if (!prep_offsets || !gates || !probs) return fail(GST_EINVAL, "NULL argument");
  if ((int64_t)n_prep * n_gates > (1 << 24)) return fail(GST_EINVAL, "at most 2^24 (preparation, gate) pairs");
  if (prep_offsets[0] != 0) return fail(GST_EINVAL, "prep_offsets[0] != 0");
  for (int p = 0; p < n_prep; ++p) {
    const int64_t L = prep_offsets[p + 1] - prep_offsets[p];
    if (L < 0 || L > 64) return fail(GST_EINVAL, "preparation words take 0 to 64 gates");
  }
  const int64_t n_steps = prep_offsets[n_prep];
  if (n_steps > 0 && !prep_gates) return fail(GST_EINVAL, "prep_gates is NULL");
  for (int64_t x = 0; x < n_steps; ++x)
    if (prep_gates[x] >= theta->n_gates) return fail(GST_EINVAL, "preparation gate index out of range");
  for (int s = 0; s < n_gates; ++s)
    if (gates[s] < 0 || gates[s] >= theta->n_gates) return fail(GST_EINVAL, "gate index out of range");
  HIP_TRY(hipSetDevice(ctx->device));
  const int levels = 6;  // blocks of 32 repetitions
  const int B = 1 << (levels - 1);
  const int Q = (r_max + 1 + B - 1) / B;
  const int n_pairs = n_prep * n_gates;
  Carver c;
  const size_t o_po = c.take<int64_t>(n_prep + 1), o_pg = c.take<uint8_t>(n_steps + 1),
               o_go = c.take<int32_t>(n_gates), o_v = c.take<double>((size_t)n_pairs * Q * D);
  if ((rc = ctx->ws.reserve(c.off + 256, ctx->stream))) return rc;
  char* b = reinterpret_cast<char*>(ctx->ws.p);
  // the three host arrays, laid out as in the workspace, in one copy
  const size_t span = o_v - o_po;
  if ((rc = ctx->stage.acquire(span))) return rc;
  char* h = reinterpret_cast<char*>(ctx->stage.p);
  std::memcpy(h + (o_po - o_po), prep_offsets, (size_t)(n_prep + 1) * 8);
  if (n_steps > 0) std::memcpy(h + (o_pg - o_po), prep_gates, (size_t)n_steps);
  std::memcpy(h + (o_go - o_po), gates, (size_t)n_gates * 4);
  if ((rc = ctx->stage.copy_to(b + o_po, span, ctx->stream))) return rc;
  gst::PredictLaunch a{};
  a.D = D;
  a.M = theta->n_outcomes;
  a.K = theta->n_gates;
  a.rho = theta->rho;
  a.E = theta->effects;
  a.G = theta->gates;
  a.n_pairs = n_pairs;
  a.n_gates = n_gates;
  a.prep_off = reinterpret_cast<const int64_t*>(b + o_po);
  a.prep_gates = reinterpret_cast<const uint8_t*>(b + o_pg);
  a.gate_of = reinterpret_cast<const int32_t*>(b + o_go);
  a.r_max = r_max;
  a.levels = levels;
  a.Q = Q;
  a.V = reinterpret_cast<double*>(b + o_v);
  a.probs = probs;
  {
    ProfScope ps(ctx, FAM_PRED_CHAIN);
    HIP_TRY(gst::launch_predict_chain(a, ctx->stream));
  }
  {
    ProfScope ps(ctx, FAM_PRED_FILL);
    HIP_TRY(gst::launch_predict_fill(a, ctx->stream));
  }
  return GST_OK;
}

int gst_tv_distance(gst_ctx* ctx, const double* p, const double* q, int64_t n, int m, double* out) {
  if (!ctx) return fail(GST_EINVAL, "ctx is NULL");
  if (n < 0 || m < 1) return fail(GST_EINVAL, "n >= 0 and m >= 1 required");
  if (n > 0 && (!p || !q || !out)) return fail(GST_EINVAL, "NULL argument");
  HIP_TRY(hipSetDevice(ctx->device));
  ProfScope ps(ctx, FAM_TV);
  HIP_TRY(gst::launch_tv_distance(p, q, n, m, out, ctx->stream));
  return GST_OK;
}

// ---------------------------------------------------------------------------
// Parameterizations (estimation modes)
// ---------------------------------------------------------------------------
static int64_t param_count_of(int mode, int D, int M, int K) {
  if (mode == GST_PARAM_FULL) return D + (int64_t)M * D + (int64_t)K * D * D;
  return (mode == GST_PARAM_TP ? D - 1 : D) + (int64_t)(M - 1) * D + (int64_t)K * D * (D - 1);
}

static int check_param_args(int mode, int n_qubits, int n_outcomes, int n_gates, int* D) {
  if (mode != GST_PARAM_FULL && mode != GST_PARAM_TP && mode != GST_PARAM_CPTP)
    return fail(GST_EINVAL, "mode must be GST_PARAM_FULL, GST_PARAM_TP or GST_PARAM_CPTP");
  const int d = dim_of(n_qubits);
  if (!d) return fail(GST_EINVAL, "n_qubits must be 1, 2 or 3");
  if (mode == GST_PARAM_CPTP && n_qubits > 2) return fail(GST_EINVAL, "the CPTP parameterization takes one or two qubits");
  if (n_gates < 1 || n_gates > gst_max_gates(n_qubits))
    return fail(GST_EINVAL, "n_gates out of range for this qubit count (see gst_max_gates)");
  if (n_outcomes < 1 || n_outcomes > std::min(d, 16)) return fail(GST_EINVAL, "n_outcomes must be in 1..min(D, 16)");
  *D = d;
  return GST_OK;
}

int gst_param_count(int mode, int n_qubits, int n_outcomes, int n_gates, int64_t* count) {
  int D = 0;
  int rc = check_param_args(mode, n_qubits, n_outcomes, n_gates, &D);
  if (rc) return rc;
  if (!count) return fail(GST_EINVAL, "count is NULL");
  *count = param_count_of(mode, D, n_outcomes, n_gates);
  return GST_OK;
}

static int param_launch(gst_ctx* ctx, int mode, int n_qubits, int n_outcomes, int n_gates, const double* theta,
                        const double* targets, gst::ParamLaunch* a) {
  int D = 0;
  int rc = check_param_args(mode, n_qubits, n_outcomes, n_gates, &D);
  if (rc) return rc;
  if (!theta) return fail(GST_EINVAL, "theta is NULL");
  if (mode == GST_PARAM_CPTP && !targets) return fail(GST_EINVAL, "the CPTP parameterization needs the target gates");
  HIP_TRY(hipSetDevice(ctx->device));
  *a = gst::ParamLaunch{};
  a->mode = mode;
  a->n = n_qubits;
  a->D = D;
  a->d = 1 << n_qubits;
  a->M = n_outcomes;
  a->K = n_gates;
  a->sqrt_d = std::sqrt((double)a->d);
  a->inv_sqrt_d = 1.0 / std::sqrt((double)a->d);
  a->theta = theta;
  a->targets = targets;
  if (mode == GST_PARAM_CPTP) {
    DevBuf& tab = ctx->param_tab[n_qubits];
    const size_t nd = (size_t)D * D + 2 * (size_t)D * D * D;
    if (!tab.p) {
      std::vector<double> y, zr, zi;
      gst::param_tables(n_qubits, &y, &zr, &zi);
      std::vector<double> all(y);
      all.insert(all.end(), zr.begin(), zr.end());
      all.insert(all.end(), zi.begin(), zi.end());
      if ((rc = tab.reserve(nd * sizeof(double), ctx->stream))) return rc;
      HIP_TRY(hipMemcpyAsync(tab.p, all.data(), nd * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
      HIP_TRY(hipStreamSynchronize(ctx->stream));  // `all` is freed on return
    }
    const double* t = reinterpret_cast<const double*>(tab.p);
    a->ty = t;
    a->tzr = t + (size_t)D * D;
    a->tzi = a->tzr + (size_t)D * D * D;
  }
  return GST_OK;
}

int gst_param_forward(gst_ctx* ctx, int mode, int n_qubits, int n_outcomes, int n_gates, const double* theta,
                      const double* targets, double* rho, double* effects, double* gates) {
  if (!ctx) return fail(GST_EINVAL, "ctx is NULL");
  gst::ParamLaunch a;
  int rc = param_launch(ctx, mode, n_qubits, n_outcomes, n_gates, theta, targets, &a);
  if (rc) return rc;
  if (!rho || !effects || !gates) return fail(GST_EINVAL, "output pointer is NULL");
  if (mode == GST_PARAM_FULL) {
    const int D = a.D, M = a.M, K = a.K;
    HIP_TRY(hipMemcpyAsync(rho, theta, (size_t)D * 8, hipMemcpyDeviceToDevice, ctx->stream));
    HIP_TRY(hipMemcpyAsync(effects, theta + D, (size_t)M * D * 8, hipMemcpyDeviceToDevice, ctx->stream));
    HIP_TRY(hipMemcpyAsync(gates, theta + D + (size_t)M * D, (size_t)K * D * D * 8, hipMemcpyDeviceToDevice,
                           ctx->stream));
    return GST_OK;
  }
  a.rho = rho;
  a.E = effects;
  a.G = gates;
  ProfScope ps(ctx, FAM_PARAM_FWD);
  HIP_TRY(gst::launch_param_forward(a, ctx->stream));
  return GST_OK;
}

int gst_param_backward(gst_ctx* ctx, int mode, int n_qubits, int n_outcomes, int n_gates, const double* theta,
                       const double* targets, const double* grad_full, double* grad_theta) {
  if (!ctx) return fail(GST_EINVAL, "ctx is NULL");
  gst::ParamLaunch a;
  int rc = param_launch(ctx, mode, n_qubits, n_outcomes, n_gates, theta, targets, &a);
  if (rc) return rc;
  if (!grad_full || !grad_theta) return fail(GST_EINVAL, "gradient pointer is NULL");
  if (mode == GST_PARAM_FULL) {
    HIP_TRY(hipMemcpyAsync(grad_theta, grad_full, (size_t)param_count_of(mode, a.D, a.M, a.K) * 8,
                           hipMemcpyDeviceToDevice, ctx->stream));
    return GST_OK;
  }
  a.grad_full = grad_full;
  a.grad_theta = grad_theta;
  ProfScope ps(ctx, FAM_PARAM_BWD);
  HIP_TRY(gst::launch_param_backward(a, ctx->stream));
  return GST_OK;
}

int gst_set_plan_jump(gst_ctx* ctx, int reps) {
  if (!ctx) return fail(GST_EINVAL, "ctx is NULL");
  if (reps != 0 && (reps < 2 || reps > 16 || (reps & (reps - 1)) != 0))
    return fail(GST_EINVAL, "jump repetitions must be 0 or a power of two from 2 to 16");
  ctx->plan_jump = reps;
  return GST_OK;
}

int gst_profile_enable(gst_ctx* ctx, int enable) {
  if (!ctx) return fail(GST_EINVAL, "ctx is NULL");
  ctx->prof.on = enable != 0;
  return GST_OK;
}

int gst_profile_only(gst_ctx* ctx, const char* kernel) {
  if (!ctx) return fail(GST_EINVAL, "ctx is NULL");
  if (!kernel) {
    ctx->prof.only = -1;
    return GST_OK;
  }
  for (int f = 0; f < FAM_N; ++f)
    if (std::strcmp(kernel, kFamilyNames[f]) == 0) {
      ctx->prof.only = f;
      return GST_OK;
    }
  return fail(GST_EINVAL, std::string("unknown kernel family ") + kernel);
}

int gst_profile_read(gst_ctx* ctx, const char* kernel, double* total_ms, int64_t* launches) {
  if (!ctx || !kernel) return fail(GST_EINVAL, "NULL argument");
  int fam = -1;
  for (int f = 0; f < FAM_N; ++f)
    if (std::strcmp(kernel, kFamilyNames[f]) == 0) fam = f;
  if (fam < 0) return fail(GST_EINVAL, std::string("unknown kernel family ") + kernel);
  HIP_TRY(hipSetDevice(ctx->device));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  for (auto& p : ctx->prof.pending) {
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, p.a, p.b));
    ctx->prof.total_ms[p.family] += ms;
    ctx->prof.launches[p.family] += 1;
    if (p.owner) {
      ctx->prof.pool.push_back(p.a);
      ctx->prof.pool.push_back(p.b);
    }
  }
  ctx->prof.pending.clear();
  if (total_ms) *total_ms = ctx->prof.total_ms[fam];
  if (launches) *launches = ctx->prof.launches[fam];
  return GST_OK;
}

int gst_req_create_host(gst_ctx* ctx, int n_qubits, int n_gates, int n_outcomes, const gst_seqlist* sl,
                        const int32_t* counts_host, gst_req** out) {
  if (!ctx || !out) return fail(GST_EINVAL, "NULL argument");
  const int D = dim_of(n_qubits);
  if (!D) return fail(GST_EINVAL, "n_qubits must be 1, 2 or 3");
  if (n_gates < 1 || n_gates > gst_max_gates(n_qubits)) return fail(GST_EINVAL, "n_gates out of range");
  if (n_outcomes < 1 || n_outcomes > std::min(D, 16)) return fail(GST_EINVAL, "n_outcomes must be in 1..min(D, 16)");
  int rc = check_seqs(sl);
  if (rc) return rc;
  const int64_t S = sl->n_seq;
  if (S > 0 && sl->offsets[0] != 0) return fail(GST_EINVAL, "offsets[0] != 0");
  int64_t max_len = 0;
  for (int64_t s = 0; s < S; ++s) {
    const int64_t L = sl->offsets[s + 1] - sl->offsets[s];
    if (L < 0) return fail(GST_EINVAL, "offsets decrease");
    max_len = std::max(max_len, L);
  }
  const int64_t n_steps = S > 0 ? sl->offsets[S] : 0;
  for (int64_t t = 0; t < n_steps; ++t)
    if (sl->gate_idx[t] >= n_gates) return fail(GST_EINDEX, "gate index >= n_gates at step " + std::to_string(t));
  double total_counts = 0.0;
  if (counts_host)
    for (int64_t x = 0; x < S * n_outcomes; ++x) {
      if (counts_host[x] < 0) return fail(GST_EINVAL, "negative count");
      total_counts += counts_host[x];
    }
  HIP_TRY(hipSetDevice(ctx->device));
  std::unique_ptr<gst_req> r(new (std::nothrow) gst_req());
  if (!r) return fail(GST_ENOMEM, "host allocation failed");
  r->ctx = ctx;
  r->n_qubits = n_qubits;
  r->D = D;
  r->M = n_outcomes;
  r->K = n_gates;
  r->S = S;
  r->max_len = max_len;
  r->total_counts = total_counts;
  // batch tiles: sequences by length (descending, stable), cut into tiles of
  // the one- and two-qubit tile kernels (three-qubit requests use their own
  // tiles below)
  std::vector<int64_t> order;
  const int64_t tile_seqs = D == 64 ? std::max<int64_t>(S, 1) : tile_seqs_of_group(ctx, tile_group(D, n_gates), S);
  gst::cut_tiles(sl->offsets, S, tile_seqs, &order, &r->tile_q, &r->tile_cost);
  if (D == 64) {
    r->tile_q.clear();
    r->tile_cost.clear();
  }
  std::vector<gst::BatchTile> tiles = gst::batch_tiles({&r->tile_q}, {&r->tile_cost}, {0});
  const int64_t Pw = gst::slab_width(D, n_outcomes, n_gates);
  // three-qubit requests: tiles of 16 sequences for the chain kernel, and the
  // step positions of each gate (ascending) cut into chunks for the
  // gate-gradient kernel
  std::vector<int64_t> pos64, cbeg64, cend64, gcp64;
  // three-qubit lists with deep sharing: the grouped-chain plan instead
  gst::Plan64 p64;
  const bool use_p64 = D == 64 && S > 0 && gst::build_plan64(sl->offsets, sl->gate_idx, S, n_gates,
                                                              gst::Plan64Options(), &p64);
  if (D == 64 && !use_p64) {
    r->tile_seqs64 = ctx->tune_tile[3] > 0 ? ctx->tune_tile[3] : 16;
    r->n_tiles64 = (S + r->tile_seqs64 - 1) / r->tile_seqs64;
    std::vector<int64_t> gp((size_t)n_gates + 1, 0);
    for (int64_t t = 0; t < n_steps; ++t) gp[sl->gate_idx[t] + 1] += 1;
    for (int k = 0; k < n_gates; ++k) gp[k + 1] += gp[k];
    pos64.resize((size_t)n_steps);
    std::vector<int64_t> fill(gp.begin(), gp.end() - 1);
    for (int64_t t = 0; t < n_steps; ++t) pos64[fill[sl->gate_idx[t]]++] = t;
    gcp64.assign((size_t)n_gates + 1, 0);
    for (int k = 0; k < n_gates; ++k) {
      gcp64[k] = (int64_t)cbeg64.size();
      for (int64_t b = gp[k]; b < gp[k + 1]; b += gst::GEMM64_CHUNK) {
        cbeg64.push_back(b);
        cend64.push_back(std::min(b + gst::GEMM64_CHUNK, gp[k + 1]));
      }
    }
    gcp64[n_gates] = (int64_t)cbeg64.size();
    r->n_chunks64 = (int64_t)cbeg64.size();
    r->eval_ws_bytes = (size_t)n_steps * 64 * 8 * 2 + 256;
  }
  const int64_t Pc64 = 1 + 64 + (int64_t)n_outcomes * 64;
  Carver cv;
  const size_t o_off = cv.take<int64_t>(S + 1), o_g = cv.take<uint8_t>(std::max<int64_t>(n_steps, 1)),
               o_c = cv.take<int32_t>(counts_host ? S * n_outcomes : 1), o_ord = cv.take<int64_t>(S + 1),
               o_sl = cv.take<double>((size_t)std::max<int64_t>(r->n_tiles(), 1) * Pw),
               o_t = cv.take<gst::BatchTile>(tiles.size() + 1), o_q = cv.take<unsigned>(kQueueWords + 2),
               o_p64 = cv.take<int64_t>(pos64.size() + 1), o_cb64 = cv.take<int64_t>(cbeg64.size() + 1),
               o_ce64 = cv.take<int64_t>(cend64.size() + 1), o_gc64 = cv.take<int64_t>(gcp64.size() + 1),
               o_ts64 = cv.take<double>((size_t)std::max<int64_t>(r->n_tiles64, 1) * (D == 64 ? Pc64 : 1)),
               o_cs64 = cv.take<double>((size_t)std::max<int64_t>(r->n_chunks64, 1) * (D == 64 ? 4096 : 1)),
               o_pt64 = cv.take<double>(D == 64 ? (size_t)gst::reduce_parts((int)std::max<int64_t>(r->n_tiles64, 1)) *
                                                      Pc64 : 1);
  rc = r->data.reserve(cv.off + 256, ctx->stream);
  if (rc) return rc;
  char* base = reinterpret_cast<char*>(r->data.p);
  r->offsets = reinterpret_cast<int64_t*>(base + o_off);
  r->gates = reinterpret_cast<uint8_t*>(base + o_g);
  r->counts = counts_host ? reinterpret_cast<int32_t*>(base + o_c) : nullptr;
  r->order = reinterpret_cast<int64_t*>(base + o_ord);
  r->tile_slab = reinterpret_cast<double*>(base + o_sl);
  r->tiles = reinterpret_cast<gst::BatchTile*>(base + o_t);
  r->queue = reinterpret_cast<unsigned*>(base + o_q);
  r->n_steps = n_steps;
  if (D == 64) {
    r->pos64 = reinterpret_cast<int64_t*>(base + o_p64);
    r->chunk_beg64 = reinterpret_cast<int64_t*>(base + o_cb64);
    r->chunk_end64 = reinterpret_cast<int64_t*>(base + o_ce64);
    r->gate_chunk_ptr64 = reinterpret_cast<int64_t*>(base + o_gc64);
    r->tile_slab64 = reinterpret_cast<double*>(base + o_ts64);
    r->chunk_slab64 = reinterpret_cast<double*>(base + o_cs64);
    r->part64 = reinterpret_cast<double*>(base + o_pt64);
    if (!pos64.empty()) HIP_TRY(hipMemcpy(r->pos64, pos64.data(), pos64.size() * 8, hipMemcpyHostToDevice));
    if (!cbeg64.empty()) {
      HIP_TRY(hipMemcpy(r->chunk_beg64, cbeg64.data(), cbeg64.size() * 8, hipMemcpyHostToDevice));
      HIP_TRY(hipMemcpy(r->chunk_end64, cend64.data(), cend64.size() * 8, hipMemcpyHostToDevice));
    }
    HIP_TRY(hipMemcpy(r->gate_chunk_ptr64, gcp64.data(), gcp64.size() * 8, hipMemcpyHostToDevice));
    // an empty list has no tiles: its single partial row stays zero
    if (r->n_tiles64 == 0) HIP_TRY(hipMemset(r->tile_slab64, 0, (size_t)Pc64 * 8));
  }
  if (!tiles.empty())
    HIP_TRY(hipMemcpy(r->tiles, tiles.data(), tiles.size() * sizeof(gst::BatchTile), hipMemcpyHostToDevice));
  std::vector<int64_t> zero_off(1, 0);
  HIP_TRY(hipMemcpy(r->offsets, S > 0 ? sl->offsets : zero_off.data(), (size_t)(S + 1) * 8, hipMemcpyHostToDevice));
  if (n_steps > 0) HIP_TRY(hipMemcpy(r->gates, sl->gate_idx, (size_t)n_steps, hipMemcpyHostToDevice));
  if (counts_host && S > 0) HIP_TRY(hipMemcpy(r->counts, counts_host, (size_t)S * n_outcomes * 4, hipMemcpyHostToDevice));
  if (S > 0) HIP_TRY(hipMemcpy(r->order, order.data(), (size_t)S * 8, hipMemcpyHostToDevice));
  if (S > 0 && D <= 16) {
    gst::HostPlan hp;
    gst::PlanOptions opt;
    opt.jump = ctx->plan_jump;
    if (gst::build_plan(sl->offsets, sl->gate_idx, S, n_gates, opt, &hp)) {
      rc = upload_plan(r.get(), hp, counts_host);
      if (rc) return rc;
    }
  }
  if (use_p64) {
    rc = upload_plan64(r.get(), p64, counts_host);
    if (rc) return rc;
  }
  r->resident_bytes = r->data.bytes + r->plan.buf.bytes + r->plan64.buf.bytes;
  (void)o_off;
  *out = r.release();
  return GST_OK;
}

// Device-pointer form: the list (and counts) are copied to the host in stream
// order, then the request is built exactly as from host arrays.
int gst_req_create(gst_ctx* ctx, int n_qubits, int n_gates, int n_outcomes, const gst_seqlist* sl,
                   const int32_t* counts, gst_req** out) {
  if (!ctx || !out) return fail(GST_EINVAL, "NULL argument");
  const int D = dim_of(n_qubits);
  if (!D) return fail(GST_EINVAL, "n_qubits must be 1, 2 or 3");
  if (n_gates < 1 || n_gates > gst_max_gates(n_qubits)) return fail(GST_EINVAL, "n_gates out of range");
  if (n_outcomes < 1 || n_outcomes > std::min(D, 16)) return fail(GST_EINVAL, "n_outcomes must be in 1..min(D, 16)");
  int rc = check_seqs(sl);
  if (rc) return rc;
  HIP_TRY(hipSetDevice(ctx->device));
  const int64_t S = sl->n_seq;
  std::vector<int64_t> off((size_t)S + 1, 0);
  if (S > 0) {
    HIP_TRY(hipMemcpyAsync(off.data(), sl->offsets, off.size() * 8, hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
  }
  if (off[0] != 0) return fail(GST_EINVAL, "offsets[0] != 0");
  for (int64_t s = 0; s < S; ++s)
    if (off[s + 1] < off[s]) return fail(GST_EINVAL, "offsets decrease");
  const int64_t n_steps = off[(size_t)S];
  std::vector<uint8_t> g((size_t)std::max<int64_t>(n_steps, 1), 0);
  std::vector<int32_t> c;
  if (n_steps > 0) HIP_TRY(hipMemcpyAsync(g.data(), sl->gate_idx, (size_t)n_steps, hipMemcpyDeviceToHost, ctx->stream));
  if (counts && S > 0) {
    c.resize((size_t)S * n_outcomes);
    HIP_TRY(hipMemcpyAsync(c.data(), counts, c.size() * 4, hipMemcpyDeviceToHost, ctx->stream));
  }
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  gst_seqlist h{S, off.data(), g.data(), -1};
  const int32_t zero = 0;
  return gst_req_create_host(ctx, n_qubits, n_gates, n_outcomes, &h,
                             counts ? (c.empty() ? &zero : c.data()) : nullptr, out);
}

int gst_req_footprint(const gst_req* req, size_t* bytes) {
  if (!req || !bytes) return fail(GST_EINVAL, "NULL argument");
  *bytes = req->resident_bytes + std::max(req->ws.bytes, req->eval_ws_bytes);
  return GST_OK;
}


static gst::BatchReq batch_req_of(const gst_req* r, const gst_gateset* th, int mode, const double* w,
                                  double* probs, bool want_grad) {
  gst::BatchReq q{};
  q.rho = th->rho;
  q.E = th->effects;
  q.G = th->gates;
  q.off = r->offsets;
  q.gates = r->gates;
  q.order = r->order;
  q.counts = r->counts;
  q.W = w;
  q.probs = probs;
  q.slab = r->tile_slab;
  q.M = r->M;
  q.K = r->K;
  q.mode = mode;
  q.want_grad = want_grad ? 1 : 0;
  return q;
}

// A request without a sharing plan: its tiles through the batched kernel
// (the same kernels and summation order as inside any batch).
static int run_tiles(gst_req* r, const gst_gateset* th, int mode, const double* w, double* probs, double* objective,
                     double* grad) {
  gst_ctx* ctx = r->ctx;
  const int64_t nt = r->n_tiles();  // 0 for an empty list: the reduce then writes zeros
  const bool want_grad = grad != nullptr;
  const int g = tile_group(r->D, r->K);
  const int grid = group_grid(ctx, g, r->K, nt);
  const size_t ck_bytes = want_grad ? group_ckpt_doubles(g, grid, r->max_len) * 8 : 0;
  // checkpoints in the context workspace: calls on a context are stream
  // ordered, so every request can share it
  int rc = ctx->ws.reserve(ck_bytes + 256, ctx->stream);
  if (rc) return rc;
  gst::BatchLaunch l{};
  l.D = r->D;
  l.kmax = r->K;
  l.reqs = nullptr;
  l.one = batch_req_of(r, th, mode, w, probs, want_grad);
  l.tiles = r->tiles;
  l.n_tiles = (int)nt;
  l.queue = r->queue;
  l.ckpt = want_grad ? reinterpret_cast<double*>(ctx->ws.p) : nullptr;
  l.ckpt_per_team = group_ckpt_stride(g, r->max_len);
  l.status = ctx->status;
  l.req_nonpos = reinterpret_cast<unsigned long long*>(r->queue + kQueueWords);
  HIP_TRY(gst::launch_queue_reset(r->queue, l.req_nonpos, 1, ctx->stream));
  if (grid > 0) {
    ProfScope ps(ctx, group_family(g));
    HIP_TRY(group_launch(g, l, grid, ctx->stream));
  }
  if (objective || grad) {
    ProfScope ps(ctx, FAM_TILES_RED);
    gst::BatchReduce red{};
    red.items = nullptr;
    red.one.req = 0;
    red.one.n_tiles = (int)nt;
    red.one.P = gst::slab_width(r->D, r->M, r->K);
    red.one.slab = r->tile_slab;
    red.one.objective = objective;
    red.one.grad = grad;
    red.req_nonpos = l.req_nonpos;
    HIP_TRY(gst::launch_batch_reduce(red, (int)((red.one.P + 63) / 64), gst::batch_reduce_chunks(nt), ctx->stream));
  }
  return GST_OK;
}

// A three-qubit request: chain kernel over its tiles, gate-gradient kernel
// over the recorded steps, ordered reduction.  `nonpos` (optional) receives
// the count of p <= 0 with N > 0 of this evaluation.
static int run64(gst_req* r, const gst_gateset* th, int mode, const double* w, double* probs, double* objective,
                 double* grad, unsigned long long* nonpos = nullptr) {
  if (r->plan64.used) return run_plan64(r, th, mode, w, probs, objective, grad, nonpos);
  gst_ctx* ctx = r->ctx;
  const bool want_grad = grad != nullptr;
  unsigned long long* np = nonpos ? nonpos : reinterpret_cast<unsigned long long*>(r->queue + kQueueWords);
  if (want_grad) {
    // per-step records in the context workspace (calls on a context are stream ordered)
    int rc = ctx->ws.reserve(r->eval_ws_bytes, ctx->stream);
    if (rc) return rc;
  }
  double* rec_b = want_grad ? reinterpret_cast<double*>(ctx->ws.p) : nullptr;
  double* rec_f = want_grad ? rec_b + (size_t)r->n_steps * 64 : nullptr;
  HIP_TRY(gst::launch_queue_reset(r->queue, np, 1, ctx->stream));
  gst::Chain64Launch a{};
  a.M = r->M;
  a.K = r->K;
  a.rho = th->rho;
  a.E = th->effects;
  a.G = th->gates;
  a.off = r->offsets;
  a.gates = r->gates;
  a.order = r->order;
  a.counts = r->counts;
  a.W = w;
  a.probs = probs;
  a.mode = mode;
  a.want_grad = want_grad ? 1 : 0;
  a.S = r->S;
  a.tile_seqs = (int)r->tile_seqs64;
  a.n_tiles = r->n_tiles64;
  a.queue = r->queue;
  a.rec_b = rec_b;
  a.rec_f = rec_f;
  a.slab = r->tile_slab64;
  a.status = ctx->status;
  a.nonpos = np;
  const int grid = (int)std::min<int64_t>(
      r->n_tiles64, (int64_t)capped(gst::chain64_blocks_per_cu(r->K), ctx->tune_bpc[3]) * ctx->n_cu);
  if (grid > 0) {
    ProfScope ps(ctx, FAM_CHAIN64);
    HIP_TRY(gst::launch_chain64(a, grid, ctx->stream));
  }
  if (want_grad && r->n_chunks64 > 0) {
    ProfScope ps(ctx, FAM_GEMM64);
    gst::Gemm64Launch g{};
    g.rec_b = rec_b;
    g.rec_f = rec_f;
    g.pos = r->pos64;
    g.chunk_beg = r->chunk_beg64;
    g.chunk_end = r->chunk_end64;
    g.slab = r->chunk_slab64;
    g.n_chunks = (int)r->n_chunks64;
    HIP_TRY(gst::launch_gemm64(g, ctx->stream));
  }
  if (objective || grad) {
    ProfScope ps(ctx, FAM_REDUCE64);
    // [objective | rho | E] from the tile partials (two ordered stages) ...
    const int64_t Pc = 1 + 64 + (int64_t)r->M * 64;
    HIP_TRY(gst::launch_reduce(r->tile_slab64, (int)std::max<int64_t>(r->n_tiles64, 1), Pc, objective, grad,
                               nullptr, 64, r->part64, ctx->stream));
    // ... and the gate columns from the chunk partials
    gst::Reduce64Launch red{};
    red.M = r->M;
    red.K = r->K;
    red.chunk_slab = r->chunk_slab64;
    red.gate_chunk_ptr = r->gate_chunk_ptr64;
    red.grad = grad;
    red.nonpos = np;
    HIP_TRY(gst::launch_reduce64(red, ctx->stream));
  }
  return GST_OK;
}

static int req_run(gst_req* r, const gst_gateset* th, int mode, const double* w, double* probs, double* objective,
                   double* grad) {
  if (!r) return fail(GST_EINVAL, "req is NULL");
  int D = 0;
  int rc = check_gateset(th, &D);
  if (rc) return rc;
  if (th->n_qubits != r->n_qubits || th->n_gates != r->K || th->n_outcomes != r->M)
    return fail(GST_EINVAL, "gate set does not match the request");
  if (mode == gst::MODE_LOGLIK && !r->counts) return fail(GST_EINVAL, "request has no counts");
  gst_ctx* ctx = r->ctx;
  HIP_TRY(hipSetDevice(ctx->device));
  if (r->D == 64) return run64(r, th, mode, w, probs, objective, grad);
  if (r->plan.used) return run_plan(r, th, mode, w, probs, objective, grad);
  return run_tiles(r, th, mode, w, probs, objective, grad);
}

int gst_req_eval(gst_req* req, const gst_gateset* theta, double* probs, double* objective, double* grad) {
  if (!objective) return fail(GST_EINVAL, "objective is NULL");
  return req_run(req, theta, gst::MODE_LOGLIK, nullptr, probs, objective, grad);
}

int gst_req_probs(gst_req* req, const gst_gateset* theta, double* probs) {
  if (!probs && req && req->S > 0) return fail(GST_EINVAL, "probs is NULL");
  return req_run(req, theta, gst::MODE_PROBS, nullptr, probs, nullptr, nullptr);
}

int gst_req_vjp(gst_req* req, const gst_gateset* theta, const double* w, double* grad) {
  if (!grad || (req && req->S > 0 && !w)) return fail(GST_EINVAL, "NULL argument");
  return req_run(req, theta, gst::MODE_VJP, w, nullptr, nullptr, grad);
}

// Enqueue the batched launch sequence on `stream`.  Per-kernel profiling
// scopes are recorded only for eager runs on the context stream.
static int batch_enqueue(gst_batch* b, hipStream_t stream, bool eager) {
  gst_ctx* ctx = b->ctx;
  gst_ctx* pc = eager ? ctx : nullptr;
  if (!b->reqs.empty())
    HIP_TRY(gst::launch_queue_reset(b->launch[0].queue, b->req_nonpos, (int)b->reqs.size(), stream));
  for (int g = 0; g < 6; ++g) {
    if (b->n_tiles[g] == 0) continue;
    ProfScope ps(pc, group_family(g));
    HIP_TRY(group_launch(g, b->launch[g], b->grid_of[g], stream));
  }
  if (b->n_items > 0) {
    ProfScope ps(pc, FAM_TILES_RED);
    HIP_TRY(gst::launch_batch_reduce(b->red, b->n_items, b->red_chunks, stream));
  }
  for (const gst_batch::PlanGroup& pg : b->pgroup) {
    if (pg.n == 0) continue;
    for (int l = 0; l < pg.n_levels; ++l) {
      ProfScope ps(pc, FAM_TRUNK_FWD);
      HIP_TRY(gst::launch_trunk_fwd_batch(pg.dev, pg.D, pg.n, l, pg.fwd_grid[l], pg.K_max, pg.jl_max, stream));
    }
    {
      ProfScope ps(pc, FAM_LEAF);
      HIP_TRY(gst::launch_items_batch(pg.dev, pg.D, pg.n, pg.item_grid, pg.K_max, pg.M_max, stream));
    }
    if (pg.any_grad) {
      for (int l = pg.n_levels - 1; l >= 0; --l) {
        {
          ProfScope ps(pc, FAM_INJECT);
          HIP_TRY(gst::launch_inject_batch(pg.dev, pg.n, l, pg.inj_grid[l], stream));
        }
        ProfScope ps(pc, FAM_TRUNK_BWD);
        HIP_TRY(gst::launch_trunk_bwd_batch(pg.dev, pg.D, pg.n, l, pg.bwd_grid[l], pg.K_max, pg.jl_max, stream));
      }
      if (pg.fill_grid > 0) {
        ProfScope ps(pc, FAM_FILL);
        HIP_TRY(gst::launch_fill_rev_batch(pg.dev, pg.D, pg.n, pg.fill_grid, pg.K_max, pg.M_max, stream));
      }
      ProfScope ps(pc, FAM_GEMM);
      HIP_TRY(gst::launch_grad_gemm_batch(pg.dev, pg.D, pg.n, pg.gemm_grid, stream));
    }
    if (pg.any_slab) {
      ProfScope ps(pc, FAM_REDUCE);
      HIP_TRY(gst::launch_reduce_plan_batch(pg.dev, pg.n, pg.red_x, pg.red_parts, stream));
    }
  }
  const gst_batch::P64Group& g = b->p64;
  if (g.n > 0) {
    // the three-qubit grouped-chain plans, in the order of the standalone sequence
    HIP_TRY(gst::launch_gate_prep64_batch(g.dev, g.n, g.K_max, stream));
    {
      ProfScope ps(pc, FAM_P64_FWD);
      for (int l = 0; l < g.n_levels; ++l) {
        HIP_TRY(gst::launch_plan64_fwd_batch(g.dev, g.n, l, g.grid_long[l], true, stream));
        HIP_TRY(gst::launch_plan64_fwd_batch(g.dev, g.n, l, g.grid_short[l], false, stream));
      }
    }
    {
      ProfScope ps(pc, FAM_P64_READ);
      HIP_TRY(gst::launch_readout64_batch(g.dev, g.n, g.ro_grid, stream));
    }
    if (g.any_grad) {
      {
        ProfScope ps(pc, FAM_P64_BWD);
        for (int l = g.n_levels - 1; l >= 0; --l) {
          HIP_TRY(gst::launch_plan64_bwd_batch(g.dev, g.n, l, g.grid_long[l], true, stream));
          HIP_TRY(gst::launch_plan64_bwd_batch(g.dev, g.n, l, g.grid_short[l], false, stream));
        }
      }
      {
        ProfScope ps(pc, FAM_GEMM64);
        HIP_TRY(gst::launch_gemm64_ts_batch(g.dev, g.n, g.gemm_grid, stream));
      }
      HIP_TRY(gst::launch_root64_batch(g.dev, g.n, stream));
    }
    if (g.any_slab) {
      ProfScope ps(pc, FAM_REDUCE64);
      HIP_TRY(gst::launch_slab_sum64_batch(g.dev, g.n, g.red_x, g.red_parts, stream));
      if (g.any_grad) HIP_TRY(gst::launch_reduce64_batch(g.dev, g.n, g.r64_x, stream));
    }
  }
  return GST_OK;
}

int gst_batch_create(gst_ctx* ctx, int n, gst_req* const* reqs, const gst_gateset* thetas, double* const* probs,
                     double* const* objectives, double* const* grads, int capture_graph, gst_batch** out) {
  if (!ctx || !out || n < 0 || (n > 0 && (!reqs || !thetas))) return fail(GST_EINVAL, "NULL argument");
  HIP_TRY(hipSetDevice(ctx->device));
  std::unique_ptr<gst_batch> b(new (std::nothrow) gst_batch());
  if (!b) return fail(GST_ENOMEM, "host allocation failed");
  b->ctx = ctx;
  std::vector<gst::BatchReq> rq;
  // per tile kernel: the requests' tile cuts
  std::vector<const std::vector<int64_t>*> group_q[6], group_cost[6];
  std::vector<int> group_req[6];
  std::vector<gst::BatchReduceItem> items;
  std::vector<int> plan_x[2];  // batched plan requests per D
  std::vector<int> p64_x;      // batched three-qubit grouped-chain plans
  for (int x = 0; x < n; ++x) {
    gst_req* r = reqs[x];
    if (!r || r->ctx != ctx) return fail(GST_EINVAL, "request missing or from another context");
    // a request's partial sums and workspace are its own: it can run once per launch
    if (std::find(b->reqs.begin(), b->reqs.end(), r) != b->reqs.end())
      return fail(GST_EINVAL, "request listed twice in one batch");
    int D = 0;
    int rc = check_gateset(&thetas[x], &D);
    if (rc) return rc;
    if (thetas[x].n_qubits != r->n_qubits || thetas[x].n_gates != r->K || thetas[x].n_outcomes != r->M)
      return fail(GST_EINVAL, "gate set does not match its request");
    double* po = probs ? probs[x] : nullptr;
    double* ob = objectives ? objectives[x] : nullptr;
    double* gr = grads ? grads[x] : nullptr;
    if (ob && !r->counts) return fail(GST_EINVAL, "objective requested for a request without counts");
    if (!ob && gr) return fail(GST_EINVAL, "gradient requested without the objective");
    b->reqs.push_back(r);
    b->thetas.push_back(thetas[x]);
    b->probs.push_back(po);
    b->objectives.push_back(ob);
    b->grads.push_back(gr);
    if (r->D == 64) {
      if (r->plan64.used)
        p64_x.push_back(x);
      else
        b->plan_reqs.push_back(x);
      rq.push_back(gst::BatchReq{});
      continue;
    }
    if (r->plan.used) {
      plan_x[D == 16 ? 1 : 0].push_back(x);
      rq.push_back(gst::BatchReq{});
      continue;
    }
    gst::BatchReq q{};
    q.rho = thetas[x].rho;
    q.E = thetas[x].effects;
    q.G = thetas[x].gates;
    q.off = r->offsets;
    q.gates = r->gates;
    q.order = r->order;
    q.counts = r->counts;
    q.W = nullptr;
    q.probs = po;
    q.slab = r->tile_slab;
    q.M = r->M;
    q.K = r->K;
    q.mode = ob ? gst::MODE_LOGLIK : gst::MODE_PROBS;
    q.want_grad = gr != nullptr;
    rq.push_back(q);
    b->kmax = std::max(b->kmax, r->K);
    b->max_len = std::max(b->max_len, r->max_len);
    group_q[tile_group(D, r->K)].push_back(&r->tile_q);
    group_cost[tile_group(D, r->K)].push_back(&r->tile_cost);
    group_req[tile_group(D, r->K)].push_back(x);
    if (ob) {
      const int64_t P = gst::slab_width(D, r->M, r->K);
      b->red_chunks = std::max(b->red_chunks, gst::batch_reduce_chunks(r->n_tiles()));
      for (int64_t c0 = 0; c0 < P; c0 += 64) {
        gst::BatchReduceItem it{};
        it.req = x;
        it.n_tiles = (int)r->n_tiles();
        it.P = P;
        it.col0 = c0;
        it.slab = r->tile_slab;
        it.objective = ob;
        it.grad = gr;
        items.push_back(it);
      }
    }
  }
  // longest tiles first (balance); execution order does not change results.
  // Every tile writes row `local` of its own request's slab: checked here
  // against the cuts before anything is launched.
  std::vector<gst::BatchTile> tiles[6];
  std::vector<const std::vector<int64_t>*> cut_of_req((size_t)n, nullptr);
  for (int x = 0; x < n; ++x)
    if (!b->reqs[x]->plan.used && b->reqs[x]->D != 64) cut_of_req[x] = &b->reqs[x]->tile_q;
  int64_t ck_doubles = 0;
  for (int g = 0; g < 6; ++g) {
    tiles[g] = gst::batch_tiles(group_q[g], group_cost[g], group_req[g]);
    b->n_tiles[g] = (int)tiles[g].size();
    b->grid_of[g] = group_grid(ctx, g, b->kmax, b->n_tiles[g]);
    // the groups run one after another on the stream and share the checkpoints
    ck_doubles = std::max<int64_t>(ck_doubles, (int64_t)group_ckpt_doubles(g, b->grid_of[g], b->max_len));
  }
  {
    std::vector<gst::BatchTile> all;
    for (int g = 0; g < 6; ++g) all.insert(all.end(), tiles[g].begin(), tiles[g].end());
    const std::string bad = gst::check_batch_tiles(all, cut_of_req);
    if (!bad.empty()) return fail(GST_EINVAL, "internal: batch tile list: " + bad);
  }
  b->n_items = (int)items.size();
  // batched plans: each request's launch arguments, its scratch region in
  // plan_ws, and its level tables (trunk ranges, reverse head rows, slot ranges)
  std::vector<PlanSetup> psetup[2];
  std::vector<int64_t> lvl_tab[2];
  std::vector<size_t> ws_at[2], lvl_at[2];
  size_t ws_total = 0;
  for (int gi = 0; gi < 2; ++gi) {
    gst_batch::PlanGroup& pg = b->pgroup[gi];
    pg.D = gi == 1 ? 16 : 4;
    pg.n = (int)plan_x[gi].size();
    psetup[gi].resize(pg.n);
    for (int y = 0; y < pg.n; ++y) {
      const int x = plan_x[gi][y];
      gst_req* r = b->reqs[x];
      const gst::HostPlan& P = r->plan.host;
      PlanSetup& st = psetup[gi][y];
      plan_setup(r, &b->thetas[x], b->objectives[x] ? gst::MODE_LOGLIK : gst::MODE_PROBS, nullptr, b->probs[x],
                 b->objectives[x], b->grads[x], nullptr, &st);
      ws_at[gi].push_back(ws_total);
      ws_total += (st.ws_bytes() + 255) / 256 * 256;
      lvl_at[gi].push_back(lvl_tab[gi].size());
      for (int l = 0; l <= P.n_levels; ++l) lvl_tab[gi].push_back(P.trunk_level_ptr[l]);
      for (int l = 0; l < P.n_levels; ++l) lvl_tab[gi].push_back(st.tb_at[l]);
      for (int l = 0; l <= P.n_levels; ++l) lvl_tab[gi].push_back(r->plan.inj_level_ptr[l]);
      pg.K_max = std::max(pg.K_max, r->K);
      pg.M_max = std::max(pg.M_max, r->M);
      pg.jl_max = std::max(pg.jl_max, P.jump_levels);
      if (P.n_levels > pg.n_levels) {
        pg.n_levels = P.n_levels;
        pg.fwd_grid.resize(pg.n_levels, 0);
        pg.bwd_grid.resize(pg.n_levels, 0);
        pg.inj_grid.resize(pg.n_levels, 0);
      }
      for (int l = 0; l < P.n_levels; ++l) {
        pg.fwd_grid[l] = std::max(pg.fwd_grid[l], st.tb_blocks[l]);
        if (st.want_grad) {
          pg.bwd_grid[l] = std::max(pg.bwd_grid[l], st.tb_blocks[l]);
          const int64_t ns = r->plan.inj_level_ptr[l + 1] - r->plan.inj_level_ptr[l];
          pg.inj_grid[l] = std::max(pg.inj_grid[l], (int)std::min<int64_t>(ns, 65536));
        }
      }
      if (st.want_grad) {
        pg.any_grad = true;
        pg.gemm_grid = (int)std::max<int64_t>(pg.gemm_grid, st.g.n_chunks);
      }
      if (st.need_slab) {
        pg.any_slab = true;
        pg.red_x = (int)std::max<int64_t>(pg.red_x, (st.red.P + 63) / 64);
        pg.red_parts = std::max(pg.red_parts, st.red.n_part);
      }
    }
  }
  // The batch fills the GPU with all requests' work at once, so each request's
  // item chunks and fill tasks go to fewer workgroups than alone (each
  // workgroup stages the gate set once for more work); the chunks keep their
  // head rows, so the sums are those of the standalone evaluation.
  for (int gi = 0; gi < 2; ++gi) {
    gst_batch::PlanGroup& pg = b->pgroup[gi];
    if (pg.n == 0) continue;
    int64_t total = 0;
    for (const PlanSetup& st : psetup[gi]) total += (st.a.n_items + gst::kItemChunk - 1) / gst::kItemChunk;
    const int64_t resident = (int64_t)ctx->n_cu * gst::item_blocks_per_cu(pg.D, pg.K_max, pg.M_max);
    const int64_t per_wg = std::max<int64_t>(1, total / std::max<int64_t>(1, 4 * resident));
    for (PlanSetup& st : psetup[gi]) {
      const int64_t nc = (st.a.n_items + gst::kItemChunk - 1) / gst::kItemChunk;
      st.a.item_blocks = (int)std::max<int64_t>(1, std::min<int64_t>(st.a.item_blocks, (nc + per_wg - 1) / per_wg));
      if (st.a.fill_blocks > 0)
        st.a.fill_blocks = (int)std::max<int64_t>(1, (st.a.fill_blocks + per_wg - 1) / per_wg);
      pg.item_grid = std::max(pg.item_grid, st.a.item_blocks + st.a.fill_blocks);
      if (st.want_grad && st.a.n_fill > 0) pg.fill_grid = std::max(pg.fill_grid, st.a.fill_blocks);
    }
  }
  if (ws_total > 0) {
    int rc = b->plan_ws.reserve(ws_total, ctx->stream);
    if (rc) return rc;
  }
  Carver cv;
  size_t o_t[6], o_pa[2], o_pi[2], o_pg[2], o_pr[2], o_pl[2];
  const size_t o_rq = cv.take<gst::BatchReq>(rq.size() + 1);
  for (int g = 0; g < 6; ++g) o_t[g] = cv.take<gst::BatchTile>(tiles[g].size() + 1);
  const size_t o_it = cv.take<gst::BatchReduceItem>(items.size() + 1), o_q = cv.take<unsigned>(16 * 6),
               o_np = cv.take<unsigned long long>(rq.size() + 1), o_ck = cv.take<double>((size_t)ck_doubles + 1),
               o_p64 = cv.take<gst::Plan64Req>(p64_x.size() + 1);
  for (int gi = 0; gi < 2; ++gi) {
    o_pa[gi] = cv.take<gst::PlanArgs>(psetup[gi].size() + 1);
    o_pi[gi] = cv.take<gst::InjectLaunch>(psetup[gi].size() + 1);
    o_pg[gi] = cv.take<gst::GemmLaunch>(psetup[gi].size() + 1);
    o_pr[gi] = cv.take<gst::PlanReduce>(psetup[gi].size() + 1);
    o_pl[gi] = cv.take<int64_t>(lvl_tab[gi].size() + 1);
  }
  int rc = b->desc.reserve(cv.off + 256, ctx->stream);
  if (rc) return rc;
  char* base = reinterpret_cast<char*>(b->desc.p);
  for (int gi = 0; gi < 2; ++gi) {
    gst_batch::PlanGroup& pg = b->pgroup[gi];
    if (pg.n == 0) continue;
    const int64_t* lvl = reinterpret_cast<const int64_t*>(base + o_pl[gi]);
    std::vector<gst::PlanArgs> va(pg.n);
    std::vector<gst::InjectLaunch> vi(pg.n);
    std::vector<gst::GemmLaunch> vg(pg.n);
    std::vector<gst::PlanReduce> vr(pg.n);
    for (int y = 0; y < pg.n; ++y) {
      PlanSetup& st = psetup[gi][y];
      const int x = plan_x[gi][y];
      const int L = b->reqs[x]->plan.host.n_levels;
      st.bind((char*)b->plan_ws.p + ws_at[gi][y]);
      st.a.req_nonpos = reinterpret_cast<unsigned long long*>(base + o_np) + x;
      st.a.lvl_trunk = lvl + lvl_at[gi][y];
      st.a.lvl_head = lvl + lvl_at[gi][y] + (L + 1);
      st.in.lvl_inj = lvl + lvl_at[gi][y] + (2 * L + 1);
      va[y] = st.a;
      vi[y] = st.in;
      vg[y] = st.g;
      vr[y] = st.red;
    }
    HIP_TRY(hipMemcpy(base + o_pa[gi], va.data(), va.size() * sizeof(gst::PlanArgs), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(base + o_pi[gi], vi.data(), vi.size() * sizeof(gst::InjectLaunch), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(base + o_pg[gi], vg.data(), vg.size() * sizeof(gst::GemmLaunch), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(base + o_pr[gi], vr.data(), vr.size() * sizeof(gst::PlanReduce), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(base + o_pl[gi], lvl_tab[gi].data(), lvl_tab[gi].size() * 8, hipMemcpyHostToDevice));
    pg.dev.args = reinterpret_cast<const gst::PlanArgs*>(base + o_pa[gi]);
    pg.dev.inject = reinterpret_cast<const gst::InjectLaunch*>(base + o_pi[gi]);
    pg.dev.gemm = reinterpret_cast<const gst::GemmLaunch*>(base + o_pg[gi]);
    pg.dev.reduce = reinterpret_cast<const gst::PlanReduce*>(base + o_pr[gi]);
  }
  if (!rq.empty()) HIP_TRY(hipMemcpy(base + o_rq, rq.data(), rq.size() * sizeof(gst::BatchReq), hipMemcpyHostToDevice));
  for (int g = 0; g < 6; ++g)
    if (!tiles[g].empty())
      HIP_TRY(hipMemcpy(base + o_t[g], tiles[g].data(), tiles[g].size() * sizeof(gst::BatchTile), hipMemcpyHostToDevice));
  if (!items.empty())
    HIP_TRY(hipMemcpy(base + o_it, items.data(), items.size() * sizeof(gst::BatchReduceItem), hipMemcpyHostToDevice));
  unsigned* queues = reinterpret_cast<unsigned*>(base + o_q);
  b->req_nonpos = reinterpret_cast<unsigned long long*>(base + o_np);
  for (int g = 0; g < 6; ++g) {
    gst::BatchLaunch& l = b->launch[g];
    l.D = g == 0 ? 16 : 4;
    l.kmax = b->kmax;
    l.reqs = reinterpret_cast<const gst::BatchReq*>(base + o_rq);
    l.tiles = reinterpret_cast<const gst::BatchTile*>(base + o_t[g]);
    l.n_tiles = b->n_tiles[g];
    l.queue = queues + 16 * g;
    l.ckpt = reinterpret_cast<double*>(base + o_ck);
    l.ckpt_per_team = group_ckpt_stride(g, b->max_len);
    l.status = ctx->status;
    l.req_nonpos = b->req_nonpos;
  }
  b->red.items = reinterpret_cast<const gst::BatchReduceItem*>(base + o_it);
  b->red.req_nonpos = b->req_nonpos;
  if (!p64_x.empty()) {
    // each request's standalone arguments; the launch grids are the largest
    // of the requests' own
    gst_batch::P64Group& g = b->p64;
    std::vector<gst::Plan64Req> v;
    for (int x : p64_x) {
      gst_req* r = b->reqs[x];
      const DevicePlan64& d = r->plan64;
      const int mode = b->objectives[x] ? gst::MODE_LOGLIK : gst::MODE_PROBS;
      v.push_back(plan64_req(r, &b->thetas[x], mode, nullptr, b->probs[x], b->objectives[x], b->grads[x],
                             b->req_nonpos + x));
      const gst::Plan64Req& q = v.back();
      const int L = d.host.n_levels;
      g.K_max = std::max(g.K_max, r->K);
      g.n_levels = std::max(g.n_levels, L);
      g.grid_long.resize((size_t)g.n_levels, 0);
      g.grid_short.resize((size_t)g.n_levels, 0);
      for (int l = 0; l < L; ++l) {
        const int t = (int)(d.level_tile_ptr[l + 1] - d.level_tile_ptr[l]);
        int& grid = d.level_long[l] ? g.grid_long[l] : g.grid_short[l];
        grid = std::max(grid, t);
      }
      g.ro_grid = std::max(g.ro_grid, q.ro_blocks);
      if (q.want_grad) {
        g.any_grad = true;
        g.gemm_grid = std::max(g.gemm_grid, q.gemm.n_chunks);
        if (q.r64.grad) g.r64_x = std::max(g.r64_x, r->K * 64);  // K gate tiles of 4096 entries, 64 per workgroup
      }
      if (q.slab) {
        g.any_slab = true;
        g.red_x = std::max(g.red_x, (int)((q.P + 63) / 64));
        g.red_parts = std::max(g.red_parts, q.red_parts);
      }
    }
    g.n = (int)v.size();
    HIP_TRY(hipMemcpy(base + o_p64, v.data(), v.size() * sizeof(gst::Plan64Req), hipMemcpyHostToDevice));
    g.dev = reinterpret_cast<const gst::Plan64Req*>(base + o_p64);
  }
  if (capture_graph && !b->reqs.empty()) {
    HIP_TRY(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
    HIP_TRY(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
    rc = batch_enqueue(b.get(), b->cap_stream, false);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(b->cap_stream, &g);
    if (rc) return rc;
    if (e != hipSuccess) return fail(GST_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    b->graph = g;
    HIP_TRY(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
  }
  *out = b.release();
  return GST_OK;
}

int gst_batch_run(gst_batch* b) {
  if (!b) return fail(GST_EINVAL, "batch is NULL");
  gst_ctx* ctx = b->ctx;
  HIP_TRY(hipSetDevice(ctx->device));
  {
    // While profiling, the launch sequence runs eagerly so that every kernel
    // is bracketed by its own events; otherwise the captured graph replays.
    ProfScope ps(ctx, FAM_BATCH);
    if (b->exec && !ctx->prof.on) {
      HIP_TRY(hipGraphLaunch(b->exec, ctx->stream));
    } else {
      int rc = batch_enqueue(b, ctx->stream, true);
      if (rc) return rc;
    }
  }
  for (int x : b->plan_reqs) {
    gst_req* r = b->reqs[x];
    const int mode = b->objectives[x] ? gst::MODE_LOGLIK : gst::MODE_PROBS;
    int rc = run64(r, &b->thetas[x], mode, nullptr, b->probs[x], b->objectives[x], b->grads[x], b->req_nonpos + x);
    if (rc) return rc;
  }
  return GST_OK;
}

int gst_batch_nonpos(gst_batch* b, int64_t* counts) {
  if (!b || !counts) return fail(GST_EINVAL, "NULL argument");
  HIP_TRY(hipSetDevice(b->ctx->device));
  HIP_TRY(hipStreamSynchronize(b->ctx->stream));
  std::vector<unsigned long long> v(b->reqs.size());
  if (!v.empty()) HIP_TRY(hipMemcpy(v.data(), b->req_nonpos, v.size() * 8, hipMemcpyDeviceToHost));
  for (size_t x = 0; x < v.size(); ++x) counts[x] = (int64_t)v[x];
  return GST_OK;
}

int gst_batch_destroy(gst_batch* b) {
  if (!b) return GST_OK;
  (void)hipSetDevice(b->ctx->device);
  (void)hipStreamSynchronize(b->ctx->stream);
  delete b;
  return GST_OK;
}

int gst_req_plan_info(const gst_req* req, int64_t* info, int n) {
  if (!req || !info || n < 1) return fail(GST_EINVAL, "NULL argument");
  const gst::HostPlan& P = req->plan.host;
  int64_t chain = 0, chain_max = 0;
  for (int64_t t = 0; t < P.n_trunks(); ++t) {
    int64_t c = 0;
    for (int64_t sg = P.seg_ptr[t]; sg < P.seg_ptr[t + 1]; ++sg) {
      const int per = (int)(P.seg_pattern[sg] & 0xffu);
      c += (int64_t)P.seg_count[sg] * (per == 0 ? 1 : per);
    }
    chain += c;
    chain_max = std::max(chain_max, c);
  }
  const gst::Plan64& Q = req->plan64.host;
  const bool q = req->plan64.used;
  int64_t vals[16] = {req->plan.used || q ? 1 : 0, q ? Q.sum_len : P.sum_len, q ? Q.n_nodes : P.n_nodes,
                      P.n_trunks(), P.trunk_steps(), P.item_steps(), q ? Q.n_levels : P.n_levels,
                      (int64_t)P.inj_loc.size(), chain, chain_max, P.n_jump_trunks(), P.n_fill(),
                      q ? 1 : 0, q ? Q.n_tiles() : 0, q ? Q.n_chains : 0, q ? Q.n_rows : 0};
  for (int x = 0; x < n && x < 16; ++x) info[x] = vals[x];
  return GST_OK;
}

int gst_req_destroy(gst_req* req) {
  if (!req) return GST_OK;
  (void)hipSetDevice(req->ctx->device);
  (void)hipStreamSynchronize(req->ctx->stream);
  delete req;
  return GST_OK;
}

}  // extern "C"

namespace {

// Context-level calls with a three-qubit gate set: the list (and counts) are
// read back to the host and evaluated as a temporary resident request, whose
// per-gate step positions the gate-gradient kernel needs.
int plain_eval64(gst_ctx* ctx, const gst_gateset* gs, const gst_seqlist* sl, int mode, const int32_t* counts,
                 const double* w, double* probs, double* objective, double* grad) {
  const int64_t S = sl->n_seq;
  std::vector<int64_t> off((size_t)S + 1, 0);
  if (S > 0) HIP_TRY(hipMemcpyAsync(off.data(), sl->offsets, off.size() * 8, hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  if (off[0] != 0) return fail(GST_EINVAL, "offsets[0] != 0");
  for (int64_t s = 0; s < S; ++s)
    if (off[s + 1] < off[s]) return fail(GST_EINVAL, "offsets decrease");
  std::vector<uint8_t> g((size_t)std::max<int64_t>(off[S], 1));
  if (off[S] > 0) HIP_TRY(hipMemcpyAsync(g.data(), sl->gate_idx, (size_t)off[S], hipMemcpyDeviceToHost, ctx->stream));
  std::vector<int32_t> c;
  if (mode == gst::MODE_LOGLIK) {
    c.resize((size_t)std::max<int64_t>(S * gs->n_outcomes, 1));
    if (S > 0)
      HIP_TRY(hipMemcpyAsync(c.data(), counts, (size_t)S * gs->n_outcomes * 4, hipMemcpyDeviceToHost, ctx->stream));
  }
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  gst_seqlist hs{S, off.data(), g.data(), -1};
  gst_req* r = nullptr;
  int rc = gst_req_create_host(ctx, gs->n_qubits, gs->n_gates, gs->n_outcomes, &hs,
                               mode == gst::MODE_LOGLIK ? c.data() : nullptr, &r);
  if (rc) return rc;
  rc = req_run(r, gs, mode, w, probs, objective, grad);
  gst_req_destroy(r);  // waits for the stream first
  return rc;
}

}  // namespace

// ---------------------------------------------------------------------------
// The fit: LGST, gauge optimization, iterative MLGST
// ---------------------------------------------------------------------------
int gst_lgst(int n_qubits, int n_outcomes, int n_gates, int64_t n_seq, const int64_t* offsets, const uint8_t* gate_idx,
             const int32_t* counts, int n_prep, const int64_t* prep_offsets, const uint8_t* prep_gates, int n_meas,
             const int64_t* meas_offsets, const uint8_t* meas_gates, double* rho, double* effects, double* gates) {
  const int D = dim_of(n_qubits);
  if (!D) return fail(GST_EINVAL, "n_qubits must be 1, 2 or 3");
  if (n_outcomes < 1 || n_gates < 1 || n_gates > 255 || n_seq < 0) return fail(GST_EINVAL, "sizes out of range");
  if (n_prep < D || (int64_t)n_meas * n_outcomes < D)
    return fail(GST_EINVAL, "LGST needs at least D preparation fiducials and D measurement rows");
  if (!offsets || !counts || !prep_offsets || !meas_offsets || !rho || !effects || !gates || (n_seq > 0 && !gate_idx))
    return fail(GST_EINVAL, "NULL argument");
  const uint8_t empty = 0;
  std::vector<double> AB, Bk;
  int j0 = -1, i0 = -1;
  int rc = gst::lgst_matrices(n_seq, offsets, gate_idx ? gate_idx : &empty, counts, n_outcomes, n_gates, n_prep,
                              prep_offsets, prep_gates ? prep_gates : &empty, n_meas, meas_offsets,
                              meas_gates ? meas_gates : &empty, &AB, &Bk, &j0, &i0);
  if (rc == -1) return fail(GST_EINVAL, "a fiducial pair (with or without a gate between) is not in the list");
  if (rc == -2) return fail(GST_EINVAL, "both fiducial lists must contain the empty word");
  if (rc == -3) return fail(GST_EINVAL, "an LGST sequence has no counts");
  rc = gst::lgst_estimate(D, n_outcomes, n_gates, n_prep, n_meas, AB.data(), Bk.data(), j0, i0, rho, effects, gates);
  if (rc == -4) return fail(GST_EINVAL, "the SVD of the AB matrix did not converge");
  if (rc == -5) return fail(GST_EINVAL, "the AB matrix has rank below D (fiducials not informationally complete)");
  return GST_OK;
}

int gst_gauge_optimize(int n_qubits, int n_outcomes, int n_gates, double* rho, double* effects, double* gates,
                       const double* target_rho, const double* target_effects, const double* target_gates,
                       double spam_weight, double gtol, double* gauge, double* objective) {
  const int D = dim_of(n_qubits);
  if (!D || n_qubits > 2) return fail(GST_EINVAL, "gauge optimization takes one or two qubits");
  if (n_outcomes < 1 || n_gates < 1 || !(spam_weight >= 0.0) || !(gtol > 0.0)) return fail(GST_EINVAL, "bad argument");
  if (!rho || !effects || !gates || !target_rho || !target_effects || !target_gates) return fail(GST_EINVAL, "NULL argument");
  const int M = n_outcomes, K = n_gates;
  const size_t DD = (size_t)D * D;
  std::vector<double> X(DD, 0.0), Xi(DD), t(DD);
  if (!gst::gauge_linear_start(D, M, K, rho, effects, gates, target_rho, target_effects, target_gates, spam_weight,
                               X.data()))
    return fail(GST_EINVAL, "the linear gauge problem is singular");
  auto f = [&](const double* x, double* g) {
    return gst::gauge_objective(D, M, K, x, rho, effects, gates, target_rho, target_effects, target_gates, spam_weight, g);
  };
  gst::LbfgsResult r = gst::lbfgs((int)DD, X.data(), f, 10, gtol, 20000);
  if (!gst::invert(D, X.data(), Xi.data())) return fail(GST_EINVAL, "the gauge optimization reached a singular matrix");
  // rho <- X rho, E <- E X^-1, G <- X G X^-1
  std::vector<double> v(D);
  for (int i = 0; i < D; ++i) {
    double s = 0.0;
    for (int j = 0; j < D; ++j) s += X[(size_t)i * D + j] * rho[j];
    v[i] = s;
  }
  std::copy(v.begin(), v.end(), rho);
  for (int m = 0; m < M; ++m) {
    for (int j = 0; j < D; ++j) {
      double s = 0.0;
      for (int i = 0; i < D; ++i) s += effects[(size_t)m * D + i] * Xi[(size_t)i * D + j];
      v[j] = s;
    }
    std::copy(v.begin(), v.end(), effects + (size_t)m * D);
  }
  for (int k = 0; k < K; ++k) {
    double* g = gates + k * DD;
    for (int i = 0; i < D; ++i)
      for (int j = 0; j < D; ++j) {
        double s = 0.0;
        for (int q = 0; q < D; ++q) s += g[(size_t)i * D + q] * Xi[(size_t)q * D + j];
        t[(size_t)i * D + j] = s;
      }
    for (int i = 0; i < D; ++i)
      for (int j = 0; j < D; ++j) {
        double s = 0.0;
        for (int q = 0; q < D; ++q) s += X[(size_t)i * D + q] * t[(size_t)q * D + j];
        g[(size_t)i * D + j] = s;
      }
  }
  if (gauge) std::copy(X.begin(), X.end(), gauge);
  if (objective) *objective = r.f;
  return GST_OK;
}

int gst_mlgst(gst_ctx* ctx, int n_stages, gst_req* const* stages, int mode, const double* targets, double* theta,
              const gst_fit_options* opt, gst_fit_report* reports) {
  if (!ctx || n_stages < 1 || !stages || !theta || !opt) return fail(GST_EINVAL, "NULL argument");
  if (mode != GST_PARAM_TP && mode != GST_PARAM_CPTP)
    return fail(GST_EINVAL, "MLGST needs the TP or CPTP parameterization (the likelihood of the full one is unbounded)");
  if (opt->max_iter < 1 || !(opt->gtol > 0.0) || opt->memory < 1 || opt->memory > 100)
    return fail(GST_EINVAL, "options out of range");
  const gst_req* r0 = stages[0];
  for (int s = 0; s < n_stages; ++s)
    if (!stages[s] || stages[s]->ctx != ctx || stages[s]->n_qubits != r0->n_qubits || stages[s]->M != r0->M ||
        stages[s]->K != r0->K)
      return fail(GST_EINVAL, "every stage must be a request of this context with the same sizes");
  const int nq = r0->n_qubits, D = r0->D, M = r0->M, K = r0->K;
  int64_t n = 0;
  int rc = gst_param_count(mode, nq, M, K, &n);
  if (rc) return rc;
  gst_diag dg;
  if ((rc = gst_sync(ctx, &dg))) return rc;  // errors of earlier calls are reported, not absorbed
  HIP_TRY(hipSetDevice(ctx->device));
  // device: theta | rho | E | G | grad_full | objective | grad_theta
  const int64_t P = D + (int64_t)M * D + (int64_t)K * D * D;
  DevBuf buf;
  if ((rc = buf.reserve((size_t)(n + P + P + 1 + n) * sizeof(double), ctx->stream))) return rc;
  double* th_d = reinterpret_cast<double*>(buf.p);
  double* rho_d = th_d + n;
  double* E_d = rho_d + D;
  double* G_d = E_d + (int64_t)M * D;
  double* gf_d = G_d + (int64_t)K * D * D;
  double* obj_d = gf_d + P;
  double* gth_d = obj_d + 1;
  double* pin = nullptr;  // [n] theta out, [1 + n] objective and gradient in
  HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&pin), (size_t)(2 * n + 1) * sizeof(double), hipHostMallocDefault));
  std::unique_ptr<double, void (*)(double*)> pin_guard(pin, [](double* q) { (void)hipHostFree(q); });
  const gst_gateset gs{nq, K, M, rho_d, E_d, G_d};
  int err = GST_OK;
  for (int s = 0; s < n_stages && err == GST_OK; ++s) {
    gst_req* req = stages[s];
    const double scale = 1.0 / std::max(1.0, req->total_counts);
    auto f = [&](const double* x, double* g) -> double {
      if (err) return INFINITY;
      std::memcpy(pin, x, (size_t)n * sizeof(double));
      int e = GST_OK;
      if (hipMemcpyAsync(th_d, pin, (size_t)n * 8, hipMemcpyHostToDevice, ctx->stream) != hipSuccess) e = GST_EDEVICE;
      if (!e) e = gst_param_forward(ctx, mode, nq, M, K, th_d, targets, rho_d, E_d, G_d);
      if (!e) e = gst_req_eval(req, &gs, nullptr, obj_d, gf_d);
      if (!e) e = gst_param_backward(ctx, mode, nq, M, K, th_d, targets, gf_d, gth_d);
      if (!e && hipMemcpyAsync(pin + n, obj_d, (size_t)(1 + n) * 8, hipMemcpyDeviceToHost, ctx->stream) != hipSuccess)
        e = GST_EDEVICE;
      if (!e && hipStreamSynchronize(ctx->stream) != hipSuccess) e = GST_EDEVICE;
      if (e) {
        err = e;
        return INFINITY;
      }
      const double F = pin[n];
      if (!std::isfinite(F)) return INFINITY;  // some p <= 0 with N > 0: the step was too long
      for (int64_t i = 0; i < n; ++i) g[i] = pin[n + 1 + i] * scale;
      return F * scale;
    };
    // TP: a start with some p <= 0 where N > 0 (the previous stage's estimate need
    // not be completely positive) is moved inward by depolarizing every gate with
    // the smallest strength 2^-10, 2^-9, ..., 1/2 that makes the likelihood finite
    // CPTP: gates and state are physical, only the effects (complete, not
    // constrained positive) can give p < 0; they are mixed with the uniform POVM
    // 1/M by the smallest such strength instead
    double shrink = 0.0;
    {
      std::vector<double> gtmp((size_t)n), th0(theta, theta + n), trial((size_t)n);
      if (!std::isfinite(f(theta, gtmp.data())) && !err) {
        const int64_t g0 = (D - 1) + (int64_t)(M - 1) * D;  // TP: first gate parameter
        const int64_t e0 = D, e1 = D + (int64_t)(M - 1) * D;  // CPTP: the free effects
        const double u0 = std::sqrt(std::sqrt((double)D)) / M;  // vec(1)/M, component 0
        for (int k = 10; k >= 1; --k) {
          const double delta = std::ldexp(1.0, -k);
          for (int64_t i = 0; i < n; ++i) {
            if (mode == GST_PARAM_TP)
              trial[i] = i < g0 ? th0[i] : th0[i] * (1.0 - delta);
            else
              trial[i] = (i >= e0 && i < e1) ? (1.0 - delta) * th0[i] + delta * ((i - e0) % D == 0 ? u0 : 0.0)
                                             : th0[i];
          }
          if (std::isfinite(f(trial.data(), gtmp.data()))) {
            std::copy(trial.begin(), trial.end(), theta);
            shrink = delta;
            break;
          }
          if (err) break;
        }
      }
    }
    const gst::LbfgsResult r = gst::lbfgs((int)n, theta, f, opt->memory, opt->gtol, opt->max_iter);
    if (!err && !std::isfinite(r.f)) err = GST_ENONPOS;  // the stage's start has p <= 0 where N > 0
    if (reports) {
      reports[s].iterations = r.iterations;
      reports[s].evaluations = r.evaluations;
      reports[s].status = r.status;
      reports[s].objective = r.f / scale;
      reports[s].grad_max = r.gmax;
      reports[s].shrink = shrink;
    }
  }
  (void)gst_sync(ctx, &dg);  // the counters hold only the fit's own rejected steps
  if (err == GST_ENONPOS) return fail(err, "the starting parameters give p <= 0 where N > 0");
  if (err) return fail(err, "an evaluation failed during the fit");
  return GST_OK;
}

// ---------------------------------------------------------------------------
// Post-fit metrics
// ---------------------------------------------------------------------------
int gst_avg_gate_fidelity(int n_qubits, int n_gates, const double* gates, const double* targets, double* f_avg) {
  const int D = dim_of(n_qubits);
  if (!D || n_gates < 1) return fail(GST_EINVAL, "sizes out of range");
  if (!gates || !targets || !f_avg) return fail(GST_EINVAL, "NULL argument");
  for (int k = 0; k < n_gates; ++k)
    f_avg[k] = gst::avg_gate_fidelity(D, gates + (size_t)k * D * D, targets + (size_t)k * D * D);
  return GST_OK;
}

int gst_diamond_unitary(int dim, const double* U, const double* V, double* dist) {
  if (dim < 1 || dim > 64) return fail(GST_EINVAL, "dim must be in 1..64");
  if (!U || !V || !dist) return fail(GST_EINVAL, "NULL argument");
  const double d = gst::diamond_unitary(dim, U, V);
  if (d < 0) return fail(GST_EINVAL, "the eigenvalues of U^dagger V did not converge");
  *dist = d;
  return GST_OK;
}

int gst_hamiltonian_decomposition_target(int n_qubits, const double* G, const double* U, double* h, double* angle,
                                         double* gamma) {
  const int D = dim_of(n_qubits);
  if (!D || n_qubits > 2) return fail(GST_EINVAL, "n_qubits must be 1 or 2");
  if (!G || !U || !h) return fail(GST_EINVAL, "NULL argument");
  double g = 0.0;
  if (gst::hamiltonian_decomposition_toward(n_qubits, G, U, h, &g))
    return fail(GST_EINVAL, "the target's eigen-decomposition did not converge");
  if (gamma) *gamma = g;
  if (angle) {
    double s = 0.0;
    for (int k = 0; k < D; ++k) s += h[k] * h[k];
    *angle = std::sqrt(s);
  }
  return GST_OK;
}

int gst_hamiltonian_decomposition(int n_qubits, const double* G, double* h, double* angle, double* gamma) {
  const int D = dim_of(n_qubits);
  if (!D) return fail(GST_EINVAL, "n_qubits must be 1, 2 or 3");
  if (!G || !h) return fail(GST_EINVAL, "NULL argument");
  double g = 0.0;
  if (gst::hamiltonian_decomposition(n_qubits, G, h, &g))
    return fail(GST_EINVAL, "no real principal logarithm (an eigenvalue on the closed negative real axis)");
  if (gamma) *gamma = g;
  if (angle) {
    double s = 0.0;
    for (int k = 0; k < D; ++k) s += h[k] * h[k];
    *angle = std::sqrt(s);
  }
  return GST_OK;
}
