// Internal declarations shared by the host-side library code and the kernels.
#pragma once
#include <stdint.h>
#include <hip/hip_runtime.h>

namespace gst {

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

__host__ __device__ inline int64_t slab_width(int D, int M, int K) { return 1 + D + (int64_t)M * D + (int64_t)K * D * D; }

hipError_t launch_leaf(const LeafLaunch& a, int n_blocks, hipStream_t stream);
int leaf_blocks_for(int D, int64_t n_items);
int leaf_ckpt_interval(int D);
int leaf_teams_per_block(int D);
int max_gates_for(int D);

// out[p] = sum_w slab[w][p] in ascending w; writes objective (p = 0) and the
// gradient (p >= 1).  When status[1] > 0 the objective is +inf and grad is
// left untouched.
hipError_t launch_reduce(const double* slab, int n_slabs, int64_t P, double* objective,
                         double* grad, const unsigned long long* status, hipStream_t stream);

}  // namespace gst
