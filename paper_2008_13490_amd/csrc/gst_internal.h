// Internal declarations shared by the host-side library code and the kernels.
#pragma once
#include <stdint.h>
#include <hip/hip_ext.h>

#include <vector>

#include "../../include/gst.h"
#include "gst_param_tables.h"
#include "gst_tiles.h"
#include <hip/hip_runtime.h>

namespace gst {

// Kernel timing.  While a LaunchTimer is installed on the calling thread,
// every launch asks it for a pair of HIP events that the runtime stamps with
// the kernel's own start and end (hipExtLaunchKernelGGL), so that no marker
// is queued between kernels.
struct LaunchTimer {
  virtual bool events(hipEvent_t* start, hipEvent_t* stop) = 0;
  virtual ~LaunchTimer() = default;
};
LaunchTimer*& launch_timer();  // per thread; null = no timing

template <typename F, typename... Args>
inline void gst_launch(F kernel, dim3 grid, dim3 block, size_t lds, hipStream_t stream, Args... args) {
  hipEvent_t a = nullptr, b = nullptr;
  if (LaunchTimer* t = launch_timer())
    if (!t->events(&a, &b)) a = b = nullptr;
  hipExtLaunchKernelGGL(kernel, grid, block, (uint32_t)lds, stream, a, b, 0u, args...);
}


// Evaluation modes of the sequence kernel.
enum Mode : int { MODE_PROBS = 0, MODE_LOGLIK = 1, MODE_VJP = 2 };

// One launch of the sequence ("leaf") kernel.  A work item is one sequence:
// the chain starts at a stored anchor state (or at rho) and applies the
// gates gate_idx[beg .. end) in time order; the readout belongs to sequence
// `seq` (row of counts / probs / w).
struct LeafLaunch {
  int D, M, K;                 // D = 4^n (4, 16 or 64)
  const double* rho;           // [D]
  const double* E;             // [M][D]
  const double* G;             // [K][D][D]
  int64_t n_items;
  // item table; if items == nullptr, item q is sequence q of (off, gates)
  const int64_t* off;          // [S+1]
  const uint8_t* gates;        // [off[S]]
  const int64_t* items;        // [n_items][4]: seq, beg, end, anchor node (-1 = rho) or null
  const double* anchor_states; // [n_nodes][D] states of stored trie nodes
  double* anchor_adj;          // [n_items][D] adjoint at the anchor (trie mode) or null
  const int32_t* counts;       // [S][M]  (MODE_LOGLIK)
  const double* W;             // [S][M]  (MODE_VJP)
  double* probs;               // [S][M] or null
  int mode;
  int want_grad;
  int max_len;                 // longest chain of any item
  double* slab;                // [gridDim.x][P], P = 1 + D + M*D + K*D*D
  double* ckpt;                // checkpoint scratch, ckpt_per_team doubles per team
  int64_t ckpt_per_team;
  unsigned long long* status;  // [0] bad gate indices, [1] p <= 0 with N > 0
};

// Kernels of the shared-prefix plan.  Row conventions:
//   state arena FA: row 0 = rho, row 1 + j = state after trunk step j,
//                   row 1 + nTS + x = state before item step x;
//   adjoint arena BA: row j = adjoint after trunk step j,
//                     row nTS + x = adjoint after item step x.
// Items per chunk of the item kernel: each chunk has its own row of partial
// sums, so a request's sums do not depend on how many workgroups run them.
constexpr int kItemChunk = 32;

struct PlanArgs {
  int D, M, K;
  const double* rho;
  const double* E;
  const double* G;
  int64_t nTS;                   // trunk steps
  // trunks (level range t_begin..t_end)
  int64_t t_begin, t_end;
  const int64_t* trunk_ptr;      // [n_trunks + 1]
  const int64_t* trunk_anchor;   // [n_trunks] location (state after trunk step), -1 = rho
  const int32_t* trunk_src;      // [n_trunks] source-arena row of the adjoint at the anchor, -1 = rho
  // each trunk's chain as ops: bits 0..6 gate index, or jump level with bit 7
  // set; bits 8..15 the steps the op spans; op_slot = injection slot of the
  // state after the op (-1 none)
  const int64_t* op_ptr;         // [n_trunks + 1]
  const uint32_t* op_desc;
  const int32_t* op_slot;
  // items
  int64_t n_items;
  const int64_t* items;          // [n_items][4] seq, beg, end, anchor location
  const int64_t* item_step_ptr;  // [n_items + 1]
  const uint8_t* gates;          // sequence gate indices (beg/end index into it)
  const int32_t* item_src;       // [n_items] source-arena row of the item's adjoint, -1 = rho
  const uint8_t* item_kv;        // [n_items][16] the first 16 gate indices of each item's word (0 past its end)
  const int32_t* item_cnt;       // [n_items][M] the counts in item order (requests with counts)
  const int32_t* counts;
  const double* W;
  double* probs;
  int mode;
  int want_grad;
  // arenas and injections: the adjoints arriving at stored states are rows
  // of the source arena, slot by slot; inj holds each slot's sum
  double* FA;
  double* BA;
  double* src_adj;               // [source rows][D]
  const double* inj;             // [n_inj][D]
  double* slab;                  // [blocks][1 + D + M*D]: objective, dL/drho, dL/dE
  unsigned long long* status;
  unsigned long long* req_nonpos;  // optional per-request count of p <= 0 with N > 0
  // germ-power jumps (segments of period 0): each trunk's jump pattern (0 =
  // none), whose product powers the trunk kernels build in LDS
  const uint32_t* trunk_jpat;
  const uint8_t* trunk_jg3;
  const uint8_t* trunk_jlev;     // the jump levels each trunk builds
  int jump_levels;               // the most any trunk builds (sizes the LDS)
  double* jump_t;                // [n_trunks][jump_levels][16][16]: the forward sweep's jump
                                 // matrices, transposed, for the reverse sweep
  int item_blocks;               // item workgroups; the item launch adds the forward fill workgroups
  // fill tasks: states (forward) or adjoints (reverse) inside each jump
  int64_t n_fill;
  const int64_t* fill_first;
  const int64_t* fill_in;
  const int32_t* fill_n;
  const uint32_t* fill_pattern;
  const uint8_t* fill_gate3;
  // batched launches only: the levels, the trunk range of each ([n_levels + 1],
  // device), the first head row of each level's reverse trunk workgroups
  // ([n_levels]), and the forward fill workgroups of the item launch
  int n_levels;
  const int64_t* lvl_trunk;
  const int64_t* lvl_head;
  int fill_blocks;
};

// inj[slot] = the sum of source-arena rows inj_ptr[slot] .. inj_ptr[slot + 1]
// - 1 (the adjoints of the items and trunks anchored at the slot's state).
struct InjectLaunch {
  int D;
  int64_t s_begin, s_end;
  const int64_t* inj_ptr;
  const double* src_adj;    // [source rows][D]
  double* inj;              // [n_inj][D]
  // batched launches only: levels (0 = no reverse sweep) and the slot range of
  // each ([n_levels + 1], device)
  int n_levels;
  const int64_t* lvl_inj;
};

// dG from the reverse-sweep records: chunk c adds, for gate chunk_gate[c],
// sum over records r in [chunk_beg[c], chunk_end[c]) of BA[rec_b[r]] FA[rec_f[r]]^T.
struct GemmLaunch {
  int D, M, K;
  int64_t n_chunks;
  const int64_t* chunk_gate;
  const int64_t* chunk_beg;
  const int64_t* chunk_end;
  const int64_t* rec_b;
  const int64_t* rec_f;
  const double* FA;
  const double* BA;
  double* tiles;  // [n_chunks][D*D]: the chunk's contribution to its gate's gradient tile
};

// Ordered sum of the sharing plan's partial results.  Head rows hold
// [objective | dL/drho | dL/dE] (width H = 1 + D + M*D); each gradient chunk
// holds one D x D tile of gate chunk_gate, the chunks of gate k being rows
// chunk_ptr[k] .. chunk_ptr[k+1] of `tiles`.  Output column x of the width
// P = H + K*D*D result (0: objective, x >= 1: grad[x-1]) adds the rows of its
// own region in two fixed stages.  `part` holds n_part * P doubles.
struct PlanReduce {
  int D, M, K;
  int n_head;
  const double* head;
  const double* tiles;
  int64_t chunk_ptr[9];  // K + 1 entries; K <= max_gates_for(D) <= 8
  int64_t P;
  int n_part;  // reduce_parts of the largest region
  double* part;
  double* objective;
  double* grad;
};

// Batched evaluation of many requests (persistent kernel, tile queue).
struct BatchReq {
  const double* rho;
  const double* E;
  const double* G;
  const int64_t* off;
  const uint8_t* gates;
  const int64_t* order;    // sequence order (by length, descending) or null
  const int32_t* counts;
  const double* W;
  double* probs;
  double* slab;            // [n_tiles][P] of this request
  int M, K, mode, want_grad;
};
struct BatchLaunch {
  int D;
  int kmax;
  const BatchReq* reqs;            // null: every tile belongs to `one`
  BatchReq one;
  const BatchTile* tiles;
  int n_tiles;
  unsigned* queue;
  double* ckpt;
  int64_t ckpt_per_team;
  unsigned long long* status;
  unsigned long long* req_nonpos;  // [n_req]
};
struct BatchReduceItem {
  int req;
  int n_tiles;
  int64_t P;
  int64_t col0;
  double* slab;  // [n_tiles][P]; stage 1 leaves the chunk sums in the first row of each chunk
  double* objective;
  double* grad;
};
struct BatchReduce {
  const BatchReduceItem* items;    // null: block b reduces columns [64b, 64b+64) of `one`
  BatchReduceItem one;
  const unsigned long long* req_nonpos;
};
size_t batch_lds(int kmax);
// One-qubit requests with K <= 4 gates: one chain per lane, a wave per tile
// of 64 sequences (gst_lane1q.hip).  ckpt_per_team of the launch is the
// checkpoint stride of one wave.
bool lane1q_supported(int K);
int lane1q_ckpt_per_wave(int64_t max_len);
int lane1q_blocks_per_cu(int K);
hipError_t launch_lane1q(const BatchLaunch& a, int K, int n_blocks, hipStream_t stream);
// Resident workgroups per CU of the batched kernel (occupancy with its LDS).
int batch_blocks_per_cu(int D, int kmax);
hipError_t launch_batch(const BatchLaunch& a, int n_blocks, hipStream_t stream);
hipError_t launch_queue_reset(unsigned* q, unsigned long long* req_nonpos, int n_req, hipStream_t stream);
// Chunks of the two-stage tile-slab sum for a request of n_tiles tiles; the
// launch takes the largest over its items.
int batch_reduce_chunks(int64_t n_tiles);
hipError_t launch_batch_reduce(const BatchReduce& a, int n_items, int max_chunks, hipStream_t stream);

// Three-qubit gate sets (D = 64): one chain per wave, the gate set in LDS,
// per-step records for the gate gradient (see gst_kernels64.hip).
constexpr int CHAIN64_WAVES = 8;        // waves per workgroup of the chain kernel
constexpr int64_t GEMM64_CHUNK = 8192;  // positions per chunk of the gate-gradient kernel
struct Chain64Launch {
  int M, K;
  const double* rho;        // [64]
  const double* E;          // [M][64]
  const double* G;          // [K][64][64]
  const int64_t* off;       // [S+1]
  const uint8_t* gates;     // [sum L]
  const int64_t* order;     // sequences by length, descending
  const int32_t* counts;    // [S][M] (MODE_LOGLIK)
  const double* W;          // [S][M] (MODE_VJP)
  double* probs;            // [S][M] or null
  int mode, want_grad;
  int64_t S;
  int tile_seqs;            // sequences per tile (consecutive in `order`)
  int64_t n_tiles;
  unsigned* queue;          // tile counter, zero before the launch
  double* rec_b;            // [sum L][64]: adjoint after each step (want_grad)
  double* rec_f;            // [sum L][64]: state before each step (want_grad)
  double* slab;             // [n_tiles][1 + 64 + 64 M]
  unsigned long long* status;
  unsigned long long* nonpos;
};
struct Gemm64Launch {
  const double* rec_b;
  const double* rec_f;
  const int64_t* row_b;      // optional: rows of rec_b and rec_f of each record (else pos for both)
  const int64_t* row_f;
  const int64_t* pos;        // step positions grouped by gate, ascending within a gate
  const int64_t* chunk_beg;  // [n_chunks] ranges in pos (one gate each)
  const int64_t* chunk_end;
  double* slab;              // [n_chunks][4096]
  int n_chunks;
};
struct Reduce64Launch {            // gate columns only
  int M, K;
  const double* chunk_slab;        // [n_chunks][4096]
  const int64_t* gate_chunk_ptr;   // [K + 1] chunk range of each gate
  double* grad;
  const unsigned long long* nonpos;
};
// Three-qubit sharing plan with grouped chains (gst_plan64.h): tiles of
// sixteen chains with one word, stepped together on the matrix cores.
struct Plan64Launch {
  const double* GA;          // [K][4][16][64]: A operands of G, GA[k][w][kk][l] = G[k][16w + l%16][4kk + l/16]
  const double* GAT;         // [K][4][16][64]: the same for G^T
  int64_t t_begin;           // first tile of the launch (one workgroup per tile)
  const int64_t* tile_row0;
  const int32_t* tile_len;
  const int64_t* tile_word;
  const int64_t* tile_ev;
  const int64_t* col_anchor; // [n_tiles][16]
  const int64_t* col_chain;  // [n_tiles][16]
  const uint8_t* words;
  const int64_t* ev_ptr;
  const uint8_t* ev_cend;    // [tile-steps][16]: byte c < 15 the step's events of columns <= c, byte 15 the most of one column
  const int64_t* ev_src;     // < 2^31
  double* FA;                // [n_rows][64], row 0 = rho
  double* BA;                // [n_rows][64]
  double* INJ;               // [n_slots + n_chains][64]
  int64_t n_slots;
  int K;                     // gates (<= 5)
};
// dG over tile-steps: chunk c adds, for its gate, over its tile-steps (tile,
// t), sum over the tile's 16 columns of BA[row(c, t)] FA[row(c, t - 1)]^T (row
// t - 1 = -1: the column's anchor).
struct Gemm64TsLaunch {
  const double* BA;
  const double* FA;
  const int64_t* tile_row0;
  const int64_t* col_anchor;
  const int64_t* ts_tile;
  const int32_t* ts_step;
  const int64_t* chunk_beg;
  const int64_t* chunk_end;
  double* slab;              // [n_chunks][4096]
  int n_chunks;
};
constexpr int GEMM64_TS_CHUNK_MAX = 64;  // tile-steps per chunk at most (staged in LDS)
hipError_t launch_gemm64_ts(const Gemm64TsLaunch& a, hipStream_t stream);
constexpr int READOUT64_WAVES = 4;
struct Readout64Launch {
  int M;
  const double* E;
  const double* FA;
  int64_t n_slots;
  const int64_t* slot_row;
  const int64_t* slot_ptr;
  const int64_t* slot_seq;
  const int64_t* slot_pack;  // [n_slots][4]: node row, first sequence, slot_ptr[s], slot_ptr[s + 1]
  const int32_t* slot_cnt;   // [n_slots][M]: the first sequence's counts
  const int32_t* counts;
  const double* W;
  double* probs;
  int mode, want_grad;
  double* INJ;               // seeds: rows 0 .. n_slots-1
  double* slab;              // [waves][1 + 64 + 64 M]
  unsigned long long* status;
  unsigned long long* nonpos;
};
struct Root64Launch {        // the adjoint of rho: root seed + chains anchored at rho (ascending)
  const double* INJ;
  int64_t root_slot;         // -1 none
  int64_t n_slots;
  const int64_t* root_chains;
  int n_root_chains;
  double* out;               // [64]
};
hipError_t launch_gate_prep64(const double* G, const double* rho, int K, double* GA, double* GAT, double* FA,
                              hipStream_t stream);
hipError_t launch_plan64_fwd(const Plan64Launch& a, int n_tiles, bool reg_gates, hipStream_t stream);
hipError_t launch_plan64_bwd(const Plan64Launch& a, int n_tiles, bool reg_gates, hipStream_t stream);
hipError_t launch_readout64(const Readout64Launch& a, int n_blocks, hipStream_t stream);
hipError_t launch_root64(const Root64Launch& a, hipStream_t stream);
int readout64_blocks_per_cu();

size_t chain64_lds(int K);
int chain64_blocks_per_cu(int K);
hipError_t launch_chain64(const Chain64Launch& a, int n_blocks, hipStream_t stream);
hipError_t launch_gemm64(const Gemm64Launch& a, hipStream_t stream);
hipError_t launch_reduce64(const Reduce64Launch& a, hipStream_t stream);

// One request of a batched launch of three-qubit grouped-chain plans: the
// arguments of its standalone launch sequence.  The batched kernels take
// request blockIdx.y (z for the slab sum), copy its arguments to registers and
// run the standalone kernels' bodies on its own grid; workgroups beyond that
// grid exit, so every request gets the bits of its standalone evaluation.
struct Plan64Req {
  Plan64Launch tiles;         // t_begin unused: the level ranges below
  const int64_t* level_tile;  // [n_levels + 1] tile ranges of the levels
  const uint8_t* level_long;  // [n_levels] 1: the level keeps the gates in registers
  int n_levels;
  int want_grad;
  const double* G;            // the gate set and rho, for the operand layouts
  const double* rho;
  Readout64Launch ro;
  int ro_blocks;
  Gemm64TsLaunch gemm;        // n_chunks = 0: no gradient GEMM
  Root64Launch root;
  // the ordered sum of the readout's wave rows (slab = null: none)
  const double* slab;
  int n_slabs, red_parts, red_per;
  int64_t P;                  // 1 + 64 + 64 M
  double* part;
  double* objective;
  double* grad;
  const double* extra_rho;    // the root adjoint, with the gradient
  Reduce64Launch r64;         // r64.grad = null: no gate columns
};
hipError_t launch_gate_prep64_batch(const Plan64Req* reqs, int n, int K_max, hipStream_t stream);
hipError_t launch_plan64_fwd_batch(const Plan64Req* reqs, int n, int level, int grid_x, bool reg_gates,
                                   hipStream_t stream);
hipError_t launch_readout64_batch(const Plan64Req* reqs, int n, int grid_x, hipStream_t stream);
hipError_t launch_plan64_bwd_batch(const Plan64Req* reqs, int n, int level, int grid_x, bool reg_gates,
                                   hipStream_t stream);
hipError_t launch_gemm64_ts_batch(const Plan64Req* reqs, int n, int grid_x, hipStream_t stream);
hipError_t launch_root64_batch(const Plan64Req* reqs, int n, hipStream_t stream);
hipError_t launch_slab_sum64_batch(const Plan64Req* reqs, int n, int grid_x, int parts_max, hipStream_t stream);
hipError_t launch_reduce64_batch(const Plan64Req* reqs, int n, int grid_x, hipStream_t stream);

hipError_t launch_trunk_fwd(const PlanArgs& a, hipStream_t stream);
hipError_t launch_trunk_bwd(const PlanArgs& a, hipStream_t stream);
hipError_t launch_items(const PlanArgs& a, int n_blocks, hipStream_t stream);
// Workgroups of the item launch: one per 16 items, at most max_blocks (> 0);
// item_blocks_per_cu is the kernel's occupancy.  The launch adds
// fill_blocks_for(n_fill) workgroups of forward fill tasks when it has them.
int item_blocks_for(int64_t n_items, int64_t max_blocks);
int item_blocks_per_cu(int D, int K, int M);
int fill_blocks_for(int64_t n_fill);
int trunk_blocks_for(int64_t n_trunks);
hipError_t launch_inject(const InjectLaunch& a, hipStream_t stream);
hipError_t launch_grad_gemm(const GemmLaunch& a, hipStream_t stream);
hipError_t launch_reduce_plan(const PlanReduce& a, hipStream_t stream);

// The plans of n requests with the same D in one launch per kernel: request y
// takes args[y], inject[y], gemm[y], reduce[y] (device arrays).  Each launch
// spans the most workgroups any request's standalone launch has (grid_x);
// K_max and jl_max size the LDS.  The sequence is: trunk_fwd per level
// ascending, items, then (inject, trunk_bwd) per level descending, fill_rev,
// grad_gemm, reduce.
struct PlanBatch {
  const PlanArgs* args;
  const InjectLaunch* inject;
  const GemmLaunch* gemm;
  const PlanReduce* reduce;
};
hipError_t launch_trunk_fwd_batch(const PlanBatch& b, int D, int n, int level, int grid_x, int K_max, int jl_max,
                                  hipStream_t stream);
hipError_t launch_items_batch(const PlanBatch& b, int D, int n, int grid_x, int K_max, int M_max,
                              hipStream_t stream);
hipError_t launch_inject_batch(const PlanBatch& b, int n, int level, int grid_x, hipStream_t stream);
hipError_t launch_trunk_bwd_batch(const PlanBatch& b, int D, int n, int level, int grid_x, int K_max, int jl_max,
                                  hipStream_t stream);
hipError_t launch_fill_rev_batch(const PlanBatch& b, int D, int n, int grid_x, int K_max, int M_max,
                                 hipStream_t stream);
hipError_t launch_grad_gemm_batch(const PlanBatch& b, int D, int n, int grid_x, hipStream_t stream);
hipError_t launch_reduce_plan_batch(const PlanBatch& b, int n, int grid_x, int parts, hipStream_t stream);
// Predictions of repeated gate applications: V = block-start states
// [n_pairs][Q][D], probs [n_pairs][r_max + 1][M]; pair = preparation * n_gates + gate.
struct PredictLaunch {
  int D, M, K;
  const double* rho;
  const double* E;
  const double* G;
  int n_pairs, n_gates;
  const int64_t* prep_off;    // [n_prep + 1]
  const uint8_t* prep_gates;
  const int32_t* gate_of;     // [n_gates]
  int r_max, levels, Q;       // blocks of 2^(levels-1) repetitions, Q blocks
  double* V;
  double* probs;
};
// The block-start chain (V), then the blocks with their readouts (probs).
hipError_t launch_predict_chain(const PredictLaunch& a, hipStream_t stream);
hipError_t launch_predict_fill(const PredictLaunch& a, hipStream_t stream);
hipError_t launch_tv_distance(const double* p, const double* q, int64_t n, int M, double* out, hipStream_t stream);

// Parameterizations of the gate set (TP and CPTP estimation modes).  theta and
// grad_theta in the layout of gst.h; grad_full = [rho | effects | gates].
struct ParamLaunch {
  int mode;          // 1 = TP, 2 = CPTP
  int n, D, d, M, K;
  double sqrt_d, inv_sqrt_d;
  const double* theta;
  const double* targets;    // CPTP: G0 [K][D][D]
  const double* grad_full;  // backward
  double* rho;              // forward outputs
  double* E;
  double* G;
  double* grad_theta;       // backward output
  const double* ty;         // CPTP structure tables of the generator (D <= 16):
  const double* tzr;        //   y [D][D], z [D (j)][D][D] (real and imaginary parts)
  const double* tzi;
};
hipError_t launch_param_forward(const ParamLaunch& a, hipStream_t stream);
hipError_t launch_param_backward(const ParamLaunch& a, hipStream_t stream);

// reverse fill tasks (adjoints inside the jumps into BA)
hipError_t launch_fill_rev(const PlanArgs& a, hipStream_t stream);
int fill_blocks_for(int64_t n_fill);

// The allocation-free evaluation (gst_noalloc.hip): the scratch array's address
// on `device`, resolved once per device (0 or a gst_status), and gst_loglik on a
// given scratch buffer (gst_api.cpp).
int scratch_bind(int device);
int ctx_device(const gst_ctx* ctx);
int loglik_into_scratch(gst_ctx* ctx, const gst_gateset* gs, const gst_seqlist* sl, const int32_t* counts,
                        double* probs, double* objective, double* grad, void* scratch, size_t scratch_bytes);

__host__ __device__ inline int64_t slab_width(int D, int M, int K) { return 1 + D + (int64_t)M * D + (int64_t)K * D * D; }

hipError_t launch_leaf(const LeafLaunch& a, int n_blocks, hipStream_t stream);
int leaf_blocks_for(int D, int64_t n_items);
int leaf_ckpt_interval(int D);
int leaf_teams_per_block(int D);
int max_gates_for(int D);

// out[p] = sum of slab[w][p] over w (fixed two-stage order) plus extra_rho on
// the rho entries; writes objective (p = 0) and the gradient (p >= 1).  The
// kernels write +inf into their objective partial for p <= 0 with N > 0; the
// objective is then +inf and grad is left untouched.  `part` holds
// reduce_parts(n_slabs) * P doubles of scratch.
int reduce_parts(int n_slabs);
hipError_t launch_reduce(const double* slab, int n_slabs, int64_t P, double* objective, double* grad,
                         const double* extra_rho, int D, double* part, hipStream_t stream);

}  // namespace gst
