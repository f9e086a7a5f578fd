// Kernels for three-qubit gate sets (D = 64).
//
// Thesis Sec. 6.3.1: p[s][m] = e_m^T G[s_L] ... G[s_1] rho, the multinomial
// log-likelihood of the counts and its gradient.
//
// Layout on the chip
//   * One chain per wave: lane i holds component i of the state.  A step is
//     the 64 fused multiply-adds acc = fma(G[k][i][j], f[j], acc), j
//     ascending from acc = 0 (the order of the plain definition, so states
//     and probabilities are bit-identical to a sequential loop).  f[j] is
//     broadcast inside its 16-lane row by DPP row_newbcast; the four rows
//     reach every lane through four row copies (ds_bpermute).
//   * The whole gate set sits in LDS (K <= 5 gates of 32 KB).  Inside a gate
//     the column pairs of row i are XOR-permuted by i mod 32, so the row
//     reads of the forward product (lane i reads row i) and the column reads
//     of the adjoint product (lane j reads column j) are both free of bank
//     conflicts.
//   * With the LDS full, the gradient of the gates is not accumulated on
//     chip: the chain kernel writes, for every step of every sequence, the
//     state before the step and the adjoint after it (one 512-byte row each,
//     at the step's position in the sequence list), and a second kernel adds
//     dG_k = sum b f^T over the positions of gate k with FP64 MFMA 16x16x4
//     tiles, in fixed chunks.  A third kernel adds the per-tile and per-chunk
//     partial sums in a fixed order.
//   * Work is cut into tiles of consecutive sequences of the length-sorted
//     order; each wave takes tiles from an atomic counter and writes one row
//     of partial sums per tile, so results do not depend on scheduling.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "gst_device.h"
#include "gst_internal.h"
#include "gst_plan64.h"

namespace gst {
namespace {

constexpr int N64 = 64;
constexpr int GATE64 = N64 * N64;  // doubles per gate in LDS

// Position (in doubles) of G[i][j] inside a gate: column pairs XOR-permuted
// by the row.
__device__ __forceinline__ int swz(int i, int j) { return i * N64 + ((((j >> 1) ^ (i & 31)) << 1) | (j & 1)); }

// x of lane 16 r + (l & 15), in every lane l.
__device__ __forceinline__ double row_copy(double x, int r, int lane) { return __shfl(x, 16 * r + (lane & 15)); }

// Row i of gate Gk dotted with x, columns ascending from 0 (bit-exact chain).
__device__ __forceinline__ double mv_row(const double* Gk, int i, double x) {
  const double* row = Gk + i * N64;
  const int s = i & 31;
  double acc = 0.0;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const double xr = row_copy(x, r, i);
    Row16 R;
    R.a0 = *reinterpret_cast<const double2*>(row + 2 * ((8 * r + 0) ^ s));
    R.a1 = *reinterpret_cast<const double2*>(row + 2 * ((8 * r + 1) ^ s));
    R.a2 = *reinterpret_cast<const double2*>(row + 2 * ((8 * r + 2) ^ s));
    R.a3 = *reinterpret_cast<const double2*>(row + 2 * ((8 * r + 3) ^ s));
    R.a4 = *reinterpret_cast<const double2*>(row + 2 * ((8 * r + 4) ^ s));
    R.a5 = *reinterpret_cast<const double2*>(row + 2 * ((8 * r + 5) ^ s));
    R.a6 = *reinterpret_cast<const double2*>(row + 2 * ((8 * r + 6) ^ s));
    R.a7 = *reinterpret_cast<const double2*>(row + 2 * ((8 * r + 7) ^ s));
    acc = dot16_from(acc, xr, R);
  }
  return acc;
}

// Column j of gate Gk dotted with x (the adjoint product G^T x): four
// independent partial chains, one per row block, added in a fixed order.
__device__ __forceinline__ double mv_col(const double* Gk, int j, double x) {
  double part[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const double xr = row_copy(x, r, j);
    Row16 R;
    const int i0 = 16 * r;
    R.a0 = double2{Gk[swz(i0 + 0, j)], Gk[swz(i0 + 1, j)]};
    R.a1 = double2{Gk[swz(i0 + 2, j)], Gk[swz(i0 + 3, j)]};
    R.a2 = double2{Gk[swz(i0 + 4, j)], Gk[swz(i0 + 5, j)]};
    R.a3 = double2{Gk[swz(i0 + 6, j)], Gk[swz(i0 + 7, j)]};
    R.a4 = double2{Gk[swz(i0 + 8, j)], Gk[swz(i0 + 9, j)]};
    R.a5 = double2{Gk[swz(i0 + 10, j)], Gk[swz(i0 + 11, j)]};
    R.a6 = double2{Gk[swz(i0 + 12, j)], Gk[swz(i0 + 13, j)]};
    R.a7 = double2{Gk[swz(i0 + 14, j)], Gk[swz(i0 + 15, j)]};
    part[r] = dot16(xr, R);
  }
  return (part[0] + part[1]) + (part[2] + part[3]);
}

// E row m (global memory) dotted with x, columns ascending from 0.
__device__ __forceinline__ double mv_global_row(const double* __restrict__ row, int lane, double x) {
  const auto* g = as_global(row);
  double acc = 0.0;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const double xr = row_copy(x, r, lane);
    const auto* q = g + 16 * r;
    Row16 R;
    R.a0 = double2{q[0], q[1]};
    R.a1 = double2{q[2], q[3]};
    R.a2 = double2{q[4], q[5]};
    R.a3 = double2{q[6], q[7]};
    R.a4 = double2{q[8], q[9]};
    R.a5 = double2{q[10], q[11]};
    R.a6 = double2{q[12], q[13]};
    R.a7 = double2{q[14], q[15]};
    acc = dot16_from(acc, xr, R);
  }
  return acc;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int sh = 1; sh < 64; sh <<= 1) v += __shfl_xor(v, sh);
  return v;
}

__global__ __launch_bounds__(CHAIN64_WAVES * 64) void chain64_kernel(const Chain64Launch a) {
  extern __shared__ double G_lds[];
  const int tid = threadIdx.x, lane = tid & 63;
  const int K = a.K, M = a.M;
  for (int x = tid; x < K * GATE64; x += CHAIN64_WAVES * 64) {
    const int k = x >> 12, i = (x >> 6) & 63, j = x & 63;
    G_lds[k * GATE64 + swz(i, j)] = a.G[x];
  }
  __syncthreads();
  const auto* g_off = as_global(a.off);
  const auto* g_order = as_global(a.order);
  const auto* g_gates = as_global(a.gates);
  const auto* g_counts = as_global(a.counts);
  const auto* g_W = as_global(a.W);
  auto* g_probs = as_global(a.probs);
  auto* g_rec_b = as_global(a.rec_b);
  auto* g_rec_f = as_global(a.rec_f);
  const bool grad = a.want_grad != 0;
  const double rho_i = a.rho[lane];
  const int mrow = lane < M ? lane : M - 1;       // lanes >= M compute a discarded readout
  const double* Erow = a.E + (size_t)mrow * N64;
  unsigned bad = 0, nonpos = 0;
  for (;;) {
    int tile = 0;
    if (lane == 0) tile = (int)atomicAdd(a.queue, 1u);
    tile = __builtin_amdgcn_readfirstlane(tile);
    if (tile >= a.n_tiles) break;
    double obj = 0.0, drho = 0.0;
    double dE[16];
#pragma unroll
    for (int m = 0; m < 16; ++m) dE[m] = 0.0;
    const int64_t q0 = (int64_t)tile * a.tile_seqs;
    const int64_t q1 = q0 + a.tile_seqs < a.S ? q0 + a.tile_seqs : a.S;
    for (int64_t q = q0; q < q1; ++q) {
      const int64_t seq = g_order[q];
      const int64_t beg = g_off[seq];
      const int L = (int)(g_off[seq + 1] - beg);
      double f = rho_i;
      // ---- forward: gate indices of 64 steps per load, broadcast by readlane ----
      for (int t0 = 0; t0 < L; t0 += 64) {
        const int n = L - t0 < 64 ? L - t0 : 64;
        const int kv = lane < n ? (int)g_gates[beg + t0 + lane] : 0;
        for (int x = 0; x < n; ++x) {
          int k = __builtin_amdgcn_readlane(kv, x);
          if (k >= K) {
            bad += lane == 0;
            k = 0;
          }
          if (grad) g_rec_f[(beg + t0 + x) * N64 + lane] = f;
          f = mv_row(G_lds + k * GATE64, lane, f);
        }
      }
      // ---- readout: lane m < M holds p_m ----
      const double p = mv_global_row(Erow, lane, f);
      double dp = 0.0;
      if (lane < M) {
        const int64_t o = seq * M + lane;
        if (a.probs) g_probs[o] = p;
        if (a.mode == MODE_LOGLIK) {
          const int32_t N = g_counts[o];
          if (N > 0) {
            if (p <= 0.0) {
              ++nonpos;
              obj = INFINITY;  // -N log p with p <= 0; no term is ever -inf
            } else {
              obj -= (double)N * log(p);
              dp = -(double)N / p;
            }
          }
        } else if (a.mode == MODE_VJP) {
          dp = g_W[o];
        }
      }
      if (!grad) continue;
      // ---- effect gradient dE[m][j] += dp_m f_j and seed b_j = sum_m E[m][j] dp_m ----
      double b = 0.0;
#pragma unroll
      for (int m = 0; m < 16; ++m) {
        if (m < M) {
          const double dpm = __shfl(dp, m);
          dE[m] = fma(dpm, f, dE[m]);
          b = fma(a.E[(size_t)m * N64 + lane], dpm, b);
        }
      }
      // ---- reverse sweep: record (b after step, state before step) ----
      for (int c0 = ((L - 1) / 64) * 64; c0 >= 0 && L > 0; c0 -= 64) {
        const int n = L - c0 < 64 ? L - c0 : 64;
        int kv = lane < n ? (int)g_gates[beg + c0 + lane] : 0;
        if (kv >= K) kv = 0;  // counted in the forward sweep
        for (int x = n - 1; x >= 0; --x) {
          const int k = __builtin_amdgcn_readlane(kv, x);
          g_rec_b[(beg + c0 + x) * N64 + lane] = b;
          b = mv_col(G_lds + k * GATE64, lane, b);
        }
      }
      drho += b;
    }
    // ---- this tile's partial sums ----
    const int64_t Pc = 1 + N64 + (int64_t)M * N64;
    double* out = a.slab + (int64_t)tile * Pc;
    const double o = wave_sum(obj);
    if (lane == 0) out[0] = o;
    out[1 + lane] = drho;
#pragma unroll
    for (int m = 0; m < 16; ++m)
      if (m < M) out[1 + N64 + m * N64 + lane] = dE[m];
  }
  if (lane == 0 && bad) atomicAdd(a.status + 0, (unsigned long long)bad);
  const unsigned np = (unsigned)wave_sum((double)nonpos);
  if (lane == 0 && np) {
    atomicAdd(a.status + 1, (unsigned long long)np);
    atomicAdd(a.nonpos, (unsigned long long)np);
  }
}

// dG_k partial over one chunk of positions of gate k: wave w owns rows
// 16w .. 16w+15 (four 16x16 tiles); four positions per MFMA, in order.
__global__ __launch_bounds__(256) void gemm64_kernel(const Gemm64Launch a) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int z = lane >> 4, ii = lane & 15;
  const int c = blockIdx.x;
  const int64_t r0 = a.chunk_beg[c], r1 = a.chunk_end[c];
  const auto* g_pos = as_global(a.pos);
  const auto* g_b = as_global(a.rec_b);
  const auto* g_f = as_global(a.rec_f);
  d4 acc[4];
#pragma unroll
  for (int tc = 0; tc < 4; ++tc) acc[tc] = d4{0.0, 0.0, 0.0, 0.0};
  const auto* g_rb = as_global(a.row_b);
  const auto* g_rf = as_global(a.row_f);
  for (int64_t r = r0; r < r1; r += 4) {
    const bool v = r + z < r1;
    const int64_t idx = v ? r + z : r0;
    const int64_t pb = a.row_b ? g_rb[idx] : g_pos[idx];
    const int64_t pf = a.row_b ? g_rf[idx] : pb;
    const double av = v ? g_b[pb * N64 + 16 * w + ii] : 0.0;
    double bv[4];
#pragma unroll
    for (int tc = 0; tc < 4; ++tc) bv[tc] = v ? g_f[pf * N64 + 16 * tc + ii] : 0.0;
#pragma unroll
    for (int tc = 0; tc < 4; ++tc) acc[tc] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv[tc], acc[tc], 0, 0, 0);
  }
  // tile element C[r][cc] sits in lane 16*(r&3)+cc, register r>>2
  double* out = a.slab + (int64_t)c * GATE64;
#pragma unroll
  for (int tc = 0; tc < 4; ++tc)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = 4 * v + (lane >> 4), cc = lane & 15;
      out[(16 * w + r) * N64 + 16 * tc + cc] = acc[tc][v];
    }
}

// Gate columns of the gradient: entry e of dG_k is the sum of the chunk
// partials of gate k, added in order with four interleaved partial sums.
// (The tile columns [objective | rho | E] go through the two-stage ordered
// reduction of the other kernels.)
__device__ __forceinline__ void reduce64_body(const Reduce64Launch& a, int64_t bx) {
  __shared__ double red[4][64];
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int64_t y = bx * 64 + tx;  // index into [K][4096]
  const int64_t Y = (int64_t)a.K * GATE64;
  double v = 0.0;
  if (y < Y) {
    const int k = (int)(y / GATE64);
    const int64_t e = y % GATE64;
    for (int64_t c = a.gate_chunk_ptr[k] + ty; c < a.gate_chunk_ptr[k + 1]; c += 4) v += a.chunk_slab[c * GATE64 + e];
  }
  red[ty][tx] = v;
  __syncthreads();
  if (ty != 0 || y >= Y) return;
  v = (red[0][tx] + red[1][tx]) + (red[2][tx] + red[3][tx]);
  const bool nonpos = a.nonpos && *a.nonpos != 0;
  if (a.grad && !nonpos) a.grad[1 + N64 + (int64_t)a.M * N64 - 1 + y] = v;
}

__global__ __launch_bounds__(256) void reduce64_kernel(const Reduce64Launch a) { reduce64_body(a, blockIdx.x); }

// ---------------------------------------------------------------------------
// The grouped-chain plan (gst_plan64.h).
//
// A tile holds sixteen chains with one gate word.  Its states form a 64 x 16
// block V; a step is V <- G V, one FP64 MFMA product.  Wave w of the tile's
// workgroup computes rows 16w .. 16w+15 with sixteen 16x16x4 MFMAs over the
// inner index in ascending blocks of four; each MFMA adds its four products
// one after another in ascending order, so every entry is the chain of fused
// multiply-adds acc = fma(G[i][j], v[j], acc), j = 0 .. 63 from acc = 0 (the
// plain definition's order: probabilities are bit-identical to it).  The block
// lives in LDS in the operand order of the MFMA (Vs[kk][lane] = V[4kk +
// lane/16][lane%16]), which is also the order in which the products come out,
// so a step writes its rows straight back for the next one.  The A operands
// come from a copy of the gate set rearranged once per evaluation so that every
// operand load reads 512 consecutive bytes; the next step's operands are
// loaded while the current step runs.
// ---------------------------------------------------------------------------

// GA[k][w][kk][l] = G[k][16w + l%16][4kk + l/16]; GAT the same for G^T.  Block 0
// also writes rho into row 0 of the state arena.
__device__ __forceinline__ void gate_prep64_body(const double* G, const double* rho, double* GA, double* GAT,
                                                 double* FA, int k) {
  const double* g = G + (int64_t)k * GATE64;
  for (int x = threadIdx.x; x < GATE64; x += 256) {
    const int w = x >> 10, kk = (x >> 6) & 15, l = x & 63;
    GA[(int64_t)k * GATE64 + x] = g[(16 * w + (l & 15)) * N64 + 4 * kk + (l >> 4)];
    GAT[(int64_t)k * GATE64 + x] = g[(4 * kk + (l >> 4)) * N64 + 16 * w + (l & 15)];
  }
  if (k == 0 && threadIdx.x < N64) FA[threadIdx.x] = rho[threadIdx.x];
}

__global__ __launch_bounds__(256) void gate_prep64_kernel(const double* G, const double* rho, double* GA,
                                                          double* GAT, double* FA) {
  gate_prep64_body(G, rho, GA, GAT, FA, blockIdx.x);
}

// Workgroup barrier for the LDS exchange of a step: waits for this wave's LDS
// operations only, so the global stores of the step and the operand loads of
// the next step stay in flight across it (a full __syncthreads() would wait for
// them as well).  The memory clobber keeps the compiler from moving LDS
// accesses across it.
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

__device__ __forceinline__ void load_ops(double (&dst)[16], const double* base, int lane) {
  const auto* g = as_global(base);
#pragma unroll
  for (int kk = 0; kk < 16; ++kk) dst[kk] = g[kk * 64 + lane];
}

// A tile's gate word and events are staged in LDS a chunk of steps at a time,
// so that the loop over the steps reads nothing from global memory whose value
// it needs at once: the only global loads in the loop are the next step's
// operands (the gate, and in the reverse sweep the vectors added at the next
// node), issued a whole step ahead.
constexpr int CH_STEPS = 256;   // steps per staged chunk
constexpr int CH_EVENTS = 1024; // events per staged chunk (a node has at most EV_NODE)
constexpr int EV_NODE = kMaxNodeEvents;  // events of one node at most: its seed and a chain per child
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));  // a step's row of the column table

// A tile-step's 16 states in LDS: element (row 4k + r4, column c) at
// k * VST + 16 r4 + c, which is where lane 16 r4 + c of an MFMA reads its B
// operand of block k and writes row 4 v + r4 of its output block; the blocks
// are padded by two doubles so that the row-wise reads below spread over the
// banks.
constexpr int VST = 66;

// Where a step's gate operands come from.  RegGates: a wave's operand blocks of
// all K <= 5 gates (16 doubles per lane each) stay in registers for the whole
// sweep and a step picks its gate by a uniform branch, so the vector memory
// path carries only the stored states, not 32 KB of gate operands per
// tile-step; for the levels with long chains.  LoadGates: the operands of the
// next step are loaded while the current one runs; for levels of short
// chains, where loading all K gates up front would cost more than the steps.
struct RegGates {
  static constexpr bool kReg = true;
  double g[5][16];
  __device__ __forceinline__ void init(const double* base, int K, int w, int l) {
#pragma unroll
    for (int k = 0; k < 5; ++k)
      if (k < K) load_ops(g[k], base + ((int64_t)k * 4 + w) * 1024, l);
  }
  __device__ __forceinline__ void start(const double*, int, int, int) {}
  // the wave's 16 x 64 block of gate k times B, sixteen MFMAs in ascending k
  __device__ __forceinline__ d4 product(const double*, int k, int, const double* B, int w, int l) {
    (void)w;
    d4 acc = {0.0, 0.0, 0.0, 0.0};
    switch (k) {
#define GST_P64_CASE(K)                                                                    \
  case K:                                                                                  \
    _Pragma("unroll") for (int kk = 0; kk < 16; ++kk)                                      \
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(g[K][kk], B[kk * VST + l], acc, 0, 0, 0);  \
    break;
      GST_P64_CASE(0) GST_P64_CASE(1) GST_P64_CASE(2) GST_P64_CASE(3)
      default:
        GST_P64_CASE(4)
#undef GST_P64_CASE
    }
    return acc;
  }
};

struct LoadGates {
  static constexpr bool kReg = false;
  double an[16];
  __device__ __forceinline__ void init(const double*, int, int, int) {}
  __device__ __forceinline__ void start(const double* base, int k, int w, int l) {
    load_ops(an, base + ((int64_t)k * 4 + w) * 1024, l);
  }
  // operands of gate k (loaded a step ago); each register takes gate k_next's
  // operand (< 0: none) as soon as its MFMA has read it, so one set of 16
  // registers serves both
  __device__ __forceinline__ d4 product(const double* base, int k, int k_next, const double* B, int w, int l) {
    (void)k;
    d4 acc = {0.0, 0.0, 0.0, 0.0};
    if (k_next >= 0) {
      const auto* g = as_global(base + ((int64_t)k_next * 4 + w) * 1024);
#pragma unroll
      for (int kk = 0; kk < 16; ++kk) {
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(an[kk], B[kk * VST + l], acc, 0, 0, 0);
        an[kk] = g[kk * 64 + l];
      }
    } else {
#pragma unroll
      for (int kk = 0; kk < 16; ++kk) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(an[kk], B[kk * VST + l], acc, 0, 0, 0);
    }
    return acc;
  }
};


// Writes the tile-step's 16 adjoints (columns c = 0..15) to 16 consecutive
// arena rows, two doubles per lane and store, so that every wave store covers
// 1 KB of consecutive memory; non-temporal, since only the gradient GEMM reads
// them (held in the L2 they would be written back at the kernel's end).

__device__ __forceinline__ void store_tile_rows(const double* V, double* out, int tid) {
  auto* g = as_global(reinterpret_cast<d2*>(out));
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int f = 2 * (tid + 256 * h);  // column f >> 6, doubles (f & 63) and the next
    const int cc = f >> 6, j = f & 63;
    d2 v;
    v.x = V[(j >> 2) * VST + (j & 3) * 16 + cc];
    v.y = V[((j + 1) >> 2) * VST + ((j + 1) & 3) * 16 + cc];
    __builtin_nontemporal_store(v, &g[f >> 1]);
  }
}

template <class Gates>
__device__ __forceinline__ void plan64_fwd_body(const Plan64Launch& a, int64_t tile) {
  __shared__ double Vs[2][16 * VST];
  __shared__ uint8_t Ws[CH_STEPS + 1];
  const int tid = threadIdx.x, l = tid & 63, w = tid >> 6;
  const int c = l & 15, r4 = l >> 4;
  const int64_t anc = a.col_anchor[tile * 16 + c];
  const auto* fa = as_global(a.FA);
  Gates gs;
  gs.init(a.GA, a.K, w, l);
#pragma unroll
  for (int v = 0; v < 4; ++v) Vs[0][(4 * w + v) * VST + l] = fa[anc * N64 + 4 * (4 * w + v) + r4];
  const int len = uniform(a.tile_len[tile]);
  const auto* word = as_global(a.words + a.tile_word[tile]);
  const int64_t row0 = a.tile_row0[tile];
  int cur = 0;
  for (int t0 = 0; t0 < len; t0 += CH_STEPS) {
    const int n = len - t0 < CH_STEPS ? len - t0 : CH_STEPS;
    // word[t0 .. t0 + n], the last one the first gate of the next chunk
    for (int x = tid; x <= n && t0 + x < len; x += 256) Ws[x] = word[t0 + x];
    lds_barrier();
    if (t0 == 0) gs.start(a.GA, uniform(Ws[0]), w, l);
    for (int x = 0; x < n; ++x) {
      const int t = t0 + x;
      const d4 acc = gs.product(a.GA, uniform(Ws[x]), t + 1 < len ? uniform(Ws[x + 1]) : -1, Vs[cur], w, l);
      // rows 16w + 4v + r4 of column c: operand block kk = 4w + v of the next step
      // (stored straight from the registers: measured faster here than the
      // row-wise stores through LDS that the reverse sweep uses)
      auto* dst = as_global(a.FA + (row0 + (int64_t)t * 16 + c) * N64 + 16 * w + r4);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        Vs[cur ^ 1][(4 * w + v) * VST + l] = acc[v];
        dst[4 * v] = acc[v];
      }
      lds_barrier();
      cur ^= 1;
    }
  }
}

template <class Gates>
__global__ __launch_bounds__(256) void plan64_fwd_kernel(const Plan64Launch a) {
  plan64_fwd_body<Gates>(a, a.t_begin + blockIdx.x);
}

// Rows 4(4w + v) + r4 of the INJ rows that events of one node add to column c:
// up to EV_NODE rows, a window of them in fixed registers, added later in the
// events' order.
// The node is step x of the staged chunk: its events are Ev[Es[x] ..
// Es[x + 1]), ascending by column, and the step's row of the column table says
// where column c's lie, so no lane scans the others'.  The loads run over the
// most events of one column at this step (a uniform count); a lane with fewer
// loads rows of the step's other events, which `n` masks out where they are
// added.
template <int W>
struct NodeAdds {
  double r[W][4];
  int n;     // this column's events at the node
  int most;  // the most events of one column at the node (uniform)
};

// Events e0 .. e0 + W - 1 of the node (a window of W rows; a node has up to
// EV_NODE, so a window smaller than that is loaded in several rounds).
template <int W>
__device__ __forceinline__ void load_node_adds(NodeAdds<W>& q, const int32_t* Es, const int32_t* Ev, const u32x4* Cc,
                                               int x, int e0, int c, int w, int r4, const double* inj) {
  const auto* g = as_global(inj);
  const int jb = uniform(Es[x]), tot = uniform(Es[x + 1]) - jb;
  const auto* row = reinterpret_cast<const uint8_t*>(Cc + x);
  q.most = uniform((int)row[15]);
  const int lo = c > 0 ? (int)row[c - 1] : 0, hi = c < 15 ? (int)row[c] : tot;
  q.n = hi - lo;
  int src[W];
#pragma unroll
  for (int e = 0; e < W; ++e) {
    const int j = jb + (lo + e0 + e < tot ? lo + e0 + e : tot - 1);
    src[e] = Ev[j < 0 ? 0 : (j < CH_EVENTS ? j : CH_EVENTS - 1)];
  }
#pragma unroll
  for (int e = 0; e < W; ++e)
#pragma unroll
    for (int v = 0; v < 4; ++v) q.r[e][v] = 0.0;
#pragma unroll
  for (int e = 0; e < W; ++e)
    if (e0 + e < q.most)
#pragma unroll
      for (int v = 0; v < 4; ++v) q.r[e][v] = g[(int64_t)src[e] * N64 + 4 * (4 * w + v) + r4];
}

// Adds the window's events to `add` in their order (absent ones add zero); the
// first window starts the sum with its first row, so the node's sum is the same
// chain of additions whatever the window.
template <int W>
__device__ __forceinline__ double node_add(const NodeAdds<W>& q, int e0, double add, int v) {
#pragma unroll
  for (int e = 0; e < W; ++e) {
    const double r = e0 + e < q.n ? q.r[e][v] : 0.0;
    add = (e0 == 0 && e == 0) ? r : add + r;
  }
  return add;
}

// A node's events summed: the first window loaded earlier (q), the others now.
template <int W>
__device__ __forceinline__ void node_sum(NodeAdds<W>& q, const int32_t* Es, const int32_t* Ev, const u32x4* Cc, int x,
                                         int c, int w, int r4, const double* inj, double (&add)[4]) {
#pragma unroll
  for (int v = 0; v < 4; ++v) add[v] = node_add(q, 0, 0.0, v);
  for (int e0 = W; e0 < q.most; e0 += W) {
    load_node_adds(q, Es, Ev, Cc, x, e0, c, w, r4, inj);
#pragma unroll
    for (int v = 0; v < 4; ++v) add[v] = node_add(q, e0, add[v], v);
  }
}

// Reverse sweep of a tile.  b_t, the adjoint of the node after step t, is
// G_{t+1}^T b_{t+1} plus the node's seed and the adjoints of the chains anchored
// there (in that order, summed first); it is stored, and G_t^T b_t with the
// events of node t-1 added becomes b_{t-1}.  The events' rows are loaded while
// the step's product runs, the next gate's operands a step ahead.  At the end each
// chain delivers G_0^T b_0 to its anchor.
template <class Gates, int EVW>
__device__ __forceinline__ void plan64_bwd_body(const Plan64Launch& a, int64_t tile) {
  __shared__ double Bs[2][16 * VST];
  __shared__ uint8_t Ws[CH_STEPS + 1];
  __shared__ int32_t Es[CH_STEPS + 2];
  __shared__ int32_t Ev[CH_EVENTS];
  __shared__ u32x4 Cc[CH_STEPS + 1];
  __shared__ unsigned long long Em[5];  // bit x: step s0 + x of the chunk has events
  const int tid = threadIdx.x, l = tid & 63, w = tid >> 6;
  const int c = l & 15, r4 = l >> 4;
  const int len = uniform(a.tile_len[tile]);
  const auto* word = as_global(a.words + a.tile_word[tile]);
  const int64_t row0 = a.tile_row0[tile];
  const int64_t tev = a.tile_ev[tile];
  const auto* evp = as_global(a.ev_ptr + tev);
  const auto* cend = as_global(reinterpret_cast<const u32x4*>(a.ev_cend) + tev);
  const auto* evs = as_global(a.ev_src);
  Gates gs;
  gs.init(a.GAT, a.K, w, l);
  int cur = 0;
  for (int t1 = len; t1 > 0;) {
    // chunk [t0, t1) with at most CH_STEPS steps and CH_EVENTS events
    // (and the events of step t0 - 1, added at the end of step t0)
    int t0 = t1 - CH_STEPS > 0 ? t1 - CH_STEPS : 0;
    const int64_t e1 = uniform64(evp[t1]);
    while (t1 - t0 > 1 && uniform64(evp[t0 > 0 ? t0 - 1 : 0]) + CH_EVENTS < e1) t0 = t1 - (t1 - t0) / 2;
    const int s0 = t0 > 0 ? t0 - 1 : 0;
    const int64_t e0 = uniform64(evp[s0]);
    const int n = t1 - t0;
    // Ws[x] = word[t0 - 1 + x] (x = 0 only if t0 > 0); Es[x] = events before
    // step s0 + x; Cc[x] = the column table of step s0 + x
    for (int x = tid; x <= n; x += 256)
      if (x > 0 || t0 > 0) Ws[x] = word[t0 - 1 + x];
    for (int x = tid; x <= t1 - s0; x += 256) Es[x] = (int32_t)(evp[s0 + x] - e0);
    for (int x = tid; x < t1 - s0; x += 256) Cc[x] = cend[s0 + x];
    for (int j = tid; j < (int)(e1 - e0); j += 256) Ev[j] = (int32_t)evs[e0 + j];
    {
      // which of the chunk's steps have events: a step without any skips the
      // lookup (the steps s0 .. t1 - 1, at most CH_STEPS + 1)
      const int xa = tid, xb = tid + 256;
      const bool fa = xa < t1 - s0 && evp[s0 + xa + 1] > evp[s0 + xa];
      const bool fb = xb < t1 - s0 && evp[s0 + xb + 1] > evp[s0 + xb];
      const unsigned long long ba = __ballot(fa), bb = __ballot(fb);
      if (l == 0) {
        Em[w] = ba;
        if (w == 0) Em[4] = bb;
      }
    }
    lds_barrier();
    const unsigned long long em0 = uniform64((int64_t)Em[0]), em1 = uniform64((int64_t)Em[1]),
                             em2 = uniform64((int64_t)Em[2]), em3 = uniform64((int64_t)Em[3]),
                             em4 = uniform64((int64_t)Em[4]);
    auto has_events = [&](int xs) {
      const int wi = xs >> 6;
      const unsigned long long b = wi == 0 ? em0 : wi == 1 ? em1 : wi == 2 ? em2 : wi == 3 ? em3 : em4;
      return ((b >> (xs & 63)) & 1ull) != 0;
    };
    if (t1 == len) {
      // b of the last node: its events alone
      NodeAdds<EVW> q;
      load_node_adds(q, Es, Ev, Cc, t1 - 1 - s0, 0, c, w, r4, a.INJ);
      double add[4];
      node_sum(q, Es, Ev, Cc, t1 - 1 - s0, c, w, r4, a.INJ, add);
#pragma unroll
      for (int v = 0; v < 4; ++v) Bs[0][(4 * w + v) * VST + l] = add[v];
      gs.start(a.GAT, uniform(Ws[n]), w, l);
      lds_barrier();
    }
    for (int x = n - 1; x >= 0; --x) {
      const int t = t0 + x;
      NodeAdds<EVW> q;  // events of node t - 1 (the first window before the product)
      q.n = 0;
      q.most = 0;
      const bool ev = t > 0 && has_events(t - 1 - s0);
      if (ev) load_node_adds(q, Es, Ev, Cc, t - 1 - s0, 0, c, w, r4, a.INJ);
      const d4 acc = gs.product(a.GAT, uniform(Ws[x + 1]), t > 0 ? uniform(Ws[x]) : -1, Bs[cur], w, l);
      store_tile_rows(Bs[cur], a.BA + (row0 + (int64_t)t * 16) * N64, tid);
      if (ev) {
        double add[4];
        node_sum(q, Es, Ev, Cc, t - 1 - s0, c, w, r4, a.INJ, add);
#pragma unroll
        for (int v = 0; v < 4; ++v) Bs[cur ^ 1][(4 * w + v) * VST + l] = acc[v] + add[v];
      } else {
#pragma unroll
        for (int v = 0; v < 4; ++v) Bs[cur ^ 1][(4 * w + v) * VST + l] = acc[v] + 0.0;
      }
      lds_barrier();
      cur ^= 1;
    }
    t1 = t0;
  }
  const int64_t ch = a.col_chain[tile * 16 + c];
  if (ch >= 0) {
    auto* out = as_global(a.INJ + (a.n_slots + ch) * N64 + r4);
#pragma unroll
    for (int v = 0; v < 4; ++v) out[4 * (4 * w + v)] = Bs[cur][(4 * w + v) * VST + l];
  }
}

// Event windows: the long level keeps all of a node's rows at once (a tile per
// CU either way), the levels of short chains three (occupancy).
template <class Gates>
__global__ __launch_bounds__(256) void plan64_bwd_kernel(const Plan64Launch a) {
  plan64_bwd_body<Gates, Gates::kReg ? EV_NODE : 3>(a, a.t_begin + blockIdx.x);
}

// The gate gradient of the grouped-chain plan: one workgroup per chunk of
// tile-steps of one gate, wave w owning rows 16w .. 16w+15 of dG.  A tile-step
// contributes sum_c b_c f_c^T over its sixteen columns: four MFMAs over the
// columns per 16 x 16 output tile, operands read straight from the arenas
// (a tile-step's adjoint rows are consecutive, and so are its state rows
// except at step 0, where they are the columns' anchors).  The chunk's rows
// are looked up once, into LDS, and each tile-step's operands are loaded
// while the previous one's MFMAs run, so that a tile-step waits for one
// memory round trip at most instead of a chain of dependent ones.
constexpr int TS_CHUNK_MAX = GEMM64_TS_CHUNK_MAX;

struct TsOps {
  double av[4];     // adjoint rows 4kb + z, elements 16w + ii
  double bv[4][4];  // state rows of the same columns, elements 16tc + ii
};

__device__ __forceinline__ void load_ts(TsOps& o, const double* BA, const double* FA, int64_t rb, const int64_t* rf,
                                        int w, int z, int ii) {
  const auto* g_b = as_global(BA);
  const auto* g_f = as_global(FA);
#pragma unroll
  for (int kb = 0; kb < 4; ++kb) {
    const int col = 4 * kb + z;
    o.av[kb] = g_b[(rb + col) * N64 + 16 * w + ii];
    const int64_t r = rf[col];
#pragma unroll
    for (int tc = 0; tc < 4; ++tc) o.bv[kb][tc] = g_f[r * N64 + 16 * tc + ii];
  }
}

constexpr int TS_SST = 80;  // padded row stride (doubles) of the staged rows: a half-wave's operand reads hit distinct banks

// The 32 rows of tile-step x (16 adjoint rows, then the 16 state rows before
// them), 16 bytes per thread and load, a row per 32 consecutive threads.
__device__ __forceinline__ void load_ts_rows(d2 (&rg)[4], const double* BA, const double* FA, int64_t rb,
                                             const int64_t* rf, int tid) {
  const auto* gb = as_global(reinterpret_cast<const d2*>(BA));
  const auto* gf = as_global(reinterpret_cast<const d2*>(FA));
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int item = tid + 256 * i, row = (item >> 5) & 15, j = item & 31;
    rg[i] = item < 512 ? gb[(rb + row) * (N64 / 2) + j] : gf[rf[row] * (N64 / 2) + j];
  }
}

__device__ __forceinline__ void store_ts_rows(const d2 (&rg)[4], double* Sb, double* Sf, int tid) {
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int item = tid + 256 * i, row = (item >> 5) & 15, j = item & 31;
    double* dst = (item < 512 ? Sb : Sf) + row * TS_SST + 2 * j;
    *reinterpret_cast<d2*>(dst) = rg[i];
  }
}

__device__ __forceinline__ void gemm64_ts_body(const Gemm64TsLaunch& a, int64_t ch) {
  __shared__ int64_t Rb[TS_CHUNK_MAX];       // adjoint row of column 0 at each tile-step
  __shared__ int64_t Rf[TS_CHUNK_MAX][16];   // the columns' state rows before it
  __shared__ double Sb[2][16 * TS_SST];      // a tile-step's adjoint rows, double-buffered
  __shared__ double Sf[2][16 * TS_SST];      // its state rows
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int z = lane >> 4, ii = lane & 15;
  const int64_t x0 = a.chunk_beg[ch];
  const int n = (int)(a.chunk_end[ch] - x0);  // <= TS_CHUNK_MAX (checked on the host)
  for (int e = tid; e < n * 16; e += 256) {
    const int x = e >> 4, c = e & 15;
    const int64_t tile = a.ts_tile[x0 + x];
    const int t = a.ts_step[x0 + x];
    const int64_t r0 = a.tile_row0[tile] + (int64_t)t * 16;
    if (c == 0) Rb[x] = r0;
    Rf[x][c] = t > 0 ? r0 - 16 + c : a.col_anchor[tile * 16 + c];
  }
  __syncthreads();
  d4 acc[4];
#pragma unroll
  for (int tc = 0; tc < 4; ++tc) acc[tc] = d4{0.0, 0.0, 0.0, 0.0};
  d2 rg[4];
  if (n > 0) {
    load_ts_rows(rg, a.BA, a.FA, Rb[0], Rf[0], tid);
    store_ts_rows(rg, Sb[0], Sf[0], tid);
  }
  lds_barrier();
  for (int x = 0; x < n; ++x) {
    const int cur = x & 1;
    if (x + 1 < n) load_ts_rows(rg, a.BA, a.FA, Rb[x + 1], Rf[x + 1], tid);
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) {
      const int row = 4 * kb + z;
      const double av = Sb[cur][row * TS_SST + 16 * w + ii];
#pragma unroll
      for (int tc = 0; tc < 4; ++tc)
        acc[tc] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, Sf[cur][row * TS_SST + 16 * tc + ii], acc[tc], 0, 0, 0);
    }
    if (x + 1 < n) store_ts_rows(rg, Sb[cur ^ 1], Sf[cur ^ 1], tid);
    lds_barrier();
  }
  double* out = a.slab + ch * GATE64;
#pragma unroll
  for (int tc = 0; tc < 4; ++tc)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = 4 * v + (lane >> 4), cc = lane & 15;
      out[(16 * w + r) * N64 + 16 * tc + cc] = acc[tc][v];
    }
}

__global__ __launch_bounds__(256) void gemm64_ts_kernel(const Gemm64TsLaunch a) { gemm64_ts_body(a, blockIdx.x); }

// Readouts per seed slot (the sequences ending at one node): p = E f, the
// objective, dL/dp, the seed E^T (sum of the slot's dL/dp), and dL/dE, for
// sixteen slots at a time on the matrix cores.  A wave takes the slot groups
// wv, wv + (waves of the launch), ... and, per group:
//   P^T = F^T E^T      (16 slots x 16 outcomes, K = 64: the slots' states as
//                       the A operand, E in registers as the B operand)
//   per (slot, outcome), in P's output layout: the objective terms and dL/dp
//   dE += D^T F        (outcomes x states, K = 16 slots)
//   S^T = D E          (slots x states, K = outcomes: the seeds)
// where D holds dL/dp (slots x outcomes).  F and D change layout through a
// small LDS tile per wave.  Lane l = 16 r4 + c owns, in an output block, rows
// 4v + r4 (v = 0..3) of column c.  Each wave writes one partial row
// [objective | 0 | dL/dE]; every sum has a fixed order.
constexpr int RO_FST = 66;  // padded row stride (doubles) of a wave's staged states
constexpr int RO_DST = 17;  // the same for its dL/dp tile

// Workgroup blk of n_blocks (the waves' slot groups depend on the count, so a
// request's sums are the same in any launch that gives it n_blocks workgroups).
__device__ __forceinline__ void readout64_body(const Readout64Launch& a, int64_t blk, int64_t n_blocks) {
  __shared__ double Fs[READOUT64_WAVES][16 * RO_FST];
  __shared__ double Ds[READOUT64_WAVES][16 * RO_DST];
  const int l = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int c = l & 15, r4 = l >> 4;
  const int64_t wv = blk * READOUT64_WAVES + w;
  const int64_t nw = n_blocks * READOUT64_WAVES;
  const int M = a.M;
  const auto* gE = as_global(a.E);
  const auto* g_pack = as_global(a.slot_pack);
  const auto* g_cnt = as_global(a.slot_cnt);
  const auto* g_seq = as_global(a.slot_seq);
  const auto* g_counts = as_global(a.counts);
  const auto* g_W = as_global(a.W);
  auto* g_probs = as_global(a.probs);
  const bool grad = a.want_grad != 0;
  // E as B operands: eP[kk] = E[c][4kk + r4] for P^T, eS[kk][tc] = E[4kk + r4][16tc + c] for S^T
  double eP[16], eS[4][4];
#pragma unroll
  for (int kk = 0; kk < 16; ++kk) eP[kk] = c < M ? gE[c * N64 + 4 * kk + r4] : 0.0;
#pragma unroll
  for (int kk = 0; kk < 4; ++kk)
#pragma unroll
    for (int tc = 0; tc < 4; ++tc) eS[kk][tc] = 4 * kk + r4 < M ? gE[(4 * kk + r4) * N64 + 16 * tc + c] : 0.0;
  d4 dE[4];
#pragma unroll
  for (int tc = 0; tc < 4; ++tc) dE[tc] = d4{0.0, 0.0, 0.0, 0.0};
  double obj = 0.0;
  unsigned nonpos = 0;
  double* Fw = Fs[w];
  double* Dw = Ds[w];
  const int64_t n_groups = (a.n_slots + 15) / 16;
  for (int64_t gi = wv; gi < n_groups; gi += nw) {
    // slot 16 gi + c: its state row, the A operand of P^T (elements 4kk + r4)
    const int64_t sc = gi * 16 + c;
    const int64_t rowc = g_pack[4 * (sc < a.n_slots ? sc : 0)];
    // the sixteen rows read whole (two rows of 512 B per load, 16 B per lane)
    // into the wave's tile, then the A operand from there
    {
      const auto* fa2 = as_global(reinterpret_cast<const d2*>(a.FA));
      d2 rv[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int64_t rr = __shfl(rowc, 2 * i + (l >> 5));
        rv[i] = fa2[rr * (N64 / 2) + (l & 31)];
      }
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int i = 0; i < 8; ++i) *reinterpret_cast<d2*>(&Fw[(2 * i + (l >> 5)) * RO_FST + 2 * (l & 31)]) = rv[i];
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    }
    double fA[16];
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) fA[kk] = Fw[c * RO_FST + 4 * kk + r4];
    // slots 16 gi + 4v + r4 of the output rows: first sequence, sequence range,
    // the first sequence's count (or weight) of outcome c
    int64_t seq0[4], q0[4], q1[4];
    double n0[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t s = gi * 16 + 4 * v + r4;
      const bool valid = s < a.n_slots;
      const int64_t b = 4 * (valid ? s : 0);
      seq0[v] = g_pack[b + 1];
      q0[v] = g_pack[b + 2];
      q1[v] = valid ? g_pack[b + 3] : q0[v];
      n0[v] = 0.0;
      if (a.mode == MODE_LOGLIK && valid && c < M) n0[v] = (double)g_cnt[s * M + c];
    }
    if (a.mode == MODE_VJP) {
#pragma unroll
      for (int v = 0; v < 4; ++v) n0[v] = q1[v] > q0[v] && c < M ? g_W[seq0[v] * M + c] : 0.0;
    }
    d4 p = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) p = __builtin_amdgcn_mfma_f64_16x16x4f64(fA[kk], eP[kk], p, 0, 0, 0);
    double dps[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      dps[v] = 0.0;
      if (c >= M) continue;
      for (int64_t q = q0[v]; q < q1[v]; ++q) {
        const int64_t seq = q == q0[v] ? seq0[v] : g_seq[q];
        const int64_t o = seq * M + c;
        if (a.probs) g_probs[o] = p[v];
        if (a.mode == MODE_LOGLIK) {
          const double N = q == q0[v] ? n0[v] : (double)g_counts[o];
          if (N > 0.0) {
            if (p[v] <= 0.0) {
              ++nonpos;
              obj = INFINITY;
            } else {
              obj -= N * log(p[v]);
              dps[v] += -N / p[v];
            }
          }
        } else if (a.mode == MODE_VJP) {
          dps[v] += q == q0[v] ? n0[v] : g_W[o];
        }
      }
    }
    if (!grad) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) Dw[(4 * v + r4) * RO_DST + c] = dps[v];
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    // dE += D^T F: A = dps (outcome c, slot 4kk + r4), B = F[slot 4kk + r4][16tc + c]
#pragma unroll
    for (int kk = 0; kk < 4; ++kk)
#pragma unroll
      for (int tc = 0; tc < 4; ++tc)
        dE[tc] = __builtin_amdgcn_mfma_f64_16x16x4f64(dps[kk], Fw[(4 * kk + r4) * RO_FST + 16 * tc + c], dE[tc], 0, 0,
                                                      0);
    // S^T = D E: A = D[slot c][outcome 4kk + r4], B = eS
    double dA[4];
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) dA[kk] = Dw[c * RO_DST + 4 * kk + r4];
    d4 st[4];
#pragma unroll
    for (int tc = 0; tc < 4; ++tc) {
      st[tc] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) st[tc] = __builtin_amdgcn_mfma_f64_16x16x4f64(dA[kk], eS[kk][tc], st[tc], 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t s = gi * 16 + 4 * v + r4;
      if (s < a.n_slots) {
        auto* out = as_global(a.INJ + s * N64 + c);
#pragma unroll
        for (int tc = 0; tc < 4; ++tc) out[16 * tc] = st[tc][v];
      }
    }
    // the tiles are rewritten by the next group
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  }
  if (a.slab) {
    const int64_t Pc = 1 + N64 + (int64_t)M * N64;
    double* out = a.slab + wv * Pc;
    const double o = wave_sum(obj);
    if (l == 0) out[0] = o;
    out[1 + l] = 0.0;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int m = 4 * v + r4;
      if (m < M)
#pragma unroll
        for (int tc = 0; tc < 4; ++tc) out[1 + N64 + m * N64 + 16 * tc + c] = dE[tc][v];
    }
  }
  const unsigned np = (unsigned)wave_sum((double)nonpos);
  if (l == 0 && np) {
    atomicAdd(a.status + 1, (unsigned long long)np);
    atomicAdd(a.nonpos, (unsigned long long)np);
  }
}

__global__ __launch_bounds__(READOUT64_WAVES * 64) void readout64_kernel(const Readout64Launch a) {
  readout64_body(a, blockIdx.x, gridDim.x);
}

__device__ __forceinline__ void root64_body(const Root64Launch& a) {
  const int j = threadIdx.x;
  double v = a.root_slot >= 0 ? a.INJ[a.root_slot * N64 + j] : 0.0;
  for (int i = 0; i < a.n_root_chains; ++i) v += a.INJ[(a.n_slots + a.root_chains[i]) * N64 + j];
  a.out[j] = v;
}

__global__ __launch_bounds__(64) void root64_kernel(const Root64Launch a) { root64_body(a); }

// ---------------------------------------------------------------------------
// Batched forms of the grouped-chain plan kernels: request blockIdx.y (z for
// the slab sum), its arguments read before anything is stored, its own grid.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void gate_prep64_batch(const Plan64Req* r) {
  const Plan64Req& q = r[blockIdx.y];
  if ((int)blockIdx.x >= q.tiles.K) return;
  // the tile kernels read the operand layouts (const there); the prep writes them
  gate_prep64_body(q.G, q.rho, const_cast<double*>(q.tiles.GA), const_cast<double*>(q.tiles.GAT), q.tiles.FA,
                   blockIdx.x);
}

template <class Gates>
__global__ __launch_bounds__(256) void plan64_fwd_batch(const Plan64Req* r, int level, int want_long) {
  const Plan64Req& q = r[blockIdx.y];
  if (level >= q.n_levels || (int)q.level_long[level] != want_long) return;
  const int64_t t0 = q.level_tile[level], t1 = q.level_tile[level + 1];
  if ((int64_t)blockIdx.x >= t1 - t0) return;
  const Plan64Launch a = q.tiles;
  plan64_fwd_body<Gates>(a, t0 + blockIdx.x);
}

template <class Gates>
__global__ __launch_bounds__(256) void plan64_bwd_batch(const Plan64Req* r, int level, int want_long) {
  const Plan64Req& q = r[blockIdx.y];
  if (!q.want_grad || level >= q.n_levels || (int)q.level_long[level] != want_long) return;
  const int64_t t0 = q.level_tile[level], t1 = q.level_tile[level + 1];
  if ((int64_t)blockIdx.x >= t1 - t0) return;
  const Plan64Launch a = q.tiles;
  // several requests' long levels share the CUs: a window of two rows lets two
  // of their tiles share a CU
  plan64_bwd_body<Gates, Gates::kReg ? 2 : 3>(a, t0 + blockIdx.x);
}

__global__ __launch_bounds__(READOUT64_WAVES * 64) void readout64_batch(const Plan64Req* r) {
  const Plan64Req& q = r[blockIdx.y];
  const int nb = q.ro_blocks;
  if ((int)blockIdx.x >= nb) return;
  const Readout64Launch a = q.ro;
  readout64_body(a, blockIdx.x, nb);
}

__global__ __launch_bounds__(256) void gemm64_ts_batch(const Plan64Req* r) {
  const Plan64Req& q = r[blockIdx.y];
  if (!q.want_grad || (int)blockIdx.x >= q.gemm.n_chunks) return;
  const Gemm64TsLaunch a = q.gemm;
  gemm64_ts_body(a, blockIdx.x);
}

__global__ __launch_bounds__(64) void root64_batch(const Plan64Req* r) {
  const Plan64Req& q = r[blockIdx.y];
  if (!q.want_grad) return;
  const Root64Launch a = q.root;
  root64_body(a);
}

__global__ __launch_bounds__(256) void slab_sum64_stage1_batch(const Plan64Req* r) {
  const Plan64Req& q = r[blockIdx.z];
  if (!q.slab || (int64_t)blockIdx.x * 64 >= q.P || (int)blockIdx.y >= q.red_parts) return;
  slab_sum_stage1(q.slab, q.n_slabs, q.P, q.red_per, q.part, blockIdx.x, blockIdx.y);
}

__global__ __launch_bounds__(256) void slab_sum64_stage2_batch(const Plan64Req* r) {
  const Plan64Req& q = r[blockIdx.y];
  if (!q.slab || (int64_t)blockIdx.x * 64 >= q.P) return;
  slab_sum_stage2(q.part, q.red_parts, q.P, q.objective, q.grad, q.extra_rho, N64, blockIdx.x);
}

__global__ __launch_bounds__(256) void reduce64_batch(const Plan64Req* r) {
  const Plan64Req& q = r[blockIdx.y];
  if (!q.want_grad || !q.r64.grad || (int64_t)blockIdx.x * 64 >= (int64_t)q.r64.K * GATE64) return;
  const Reduce64Launch a = q.r64;
  reduce64_body(a, blockIdx.x);
}

}  // namespace

hipError_t launch_gate_prep64(const double* G, const double* rho, int K, double* GA, double* GAT, double* FA,
                              hipStream_t stream) {
  if (K < 1) return hipErrorInvalidValue;
  gst_launch(gate_prep64_kernel, dim3(K), dim3(256), 0, stream, G, rho, GA, GAT, FA);
  return hipGetLastError();
}

hipError_t launch_gemm64_ts(const Gemm64TsLaunch& a, hipStream_t stream) {
  if (a.n_chunks <= 0) return hipSuccess;
  gst_launch(gemm64_ts_kernel, dim3(a.n_chunks), dim3(256), 0, stream, a);
  return hipGetLastError();
}

hipError_t launch_plan64_fwd(const Plan64Launch& a, int n_tiles, bool reg_gates, hipStream_t stream) {
  if (n_tiles <= 0) return hipSuccess;
  if (a.K < 1 || a.K > 5) return hipErrorInvalidValue;
  if (reg_gates)
    gst_launch(plan64_fwd_kernel<RegGates>, dim3(n_tiles), dim3(256), 0, stream, a);
  else
    gst_launch(plan64_fwd_kernel<LoadGates>, dim3(n_tiles), dim3(256), 0, stream, a);
  return hipGetLastError();
}

hipError_t launch_plan64_bwd(const Plan64Launch& a, int n_tiles, bool reg_gates, hipStream_t stream) {
  if (n_tiles <= 0) return hipSuccess;
  if (a.K < 1 || a.K > 5) return hipErrorInvalidValue;
  if (reg_gates)
    gst_launch(plan64_bwd_kernel<RegGates>, dim3(n_tiles), dim3(256), 0, stream, a);
  else
    gst_launch(plan64_bwd_kernel<LoadGates>, dim3(n_tiles), dim3(256), 0, stream, a);
  return hipGetLastError();
}

int readout64_blocks_per_cu() {
  int n = 0;
  const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, readout64_kernel, READOUT64_WAVES * 64, 0);
  return (e == hipSuccess && n > 0) ? n : 1;
}

hipError_t launch_readout64(const Readout64Launch& a, int n_blocks, hipStream_t stream) {
  if (n_blocks <= 0 || a.M < 1 || a.M > 16) return hipErrorInvalidValue;
  gst_launch(readout64_kernel, dim3(n_blocks), dim3(READOUT64_WAVES * 64), 0, stream, a);
  return hipGetLastError();
}

hipError_t launch_root64(const Root64Launch& a, hipStream_t stream) {
  gst_launch(root64_kernel, dim3(1), dim3(64), 0, stream, a);
  return hipGetLastError();
}

size_t chain64_lds(int K) { return (size_t)K * GATE64 * sizeof(double); }

int chain64_blocks_per_cu(int K) {
  int n = 0;
  const hipError_t e =
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, chain64_kernel, CHAIN64_WAVES * 64, chain64_lds(K));
  return (e == hipSuccess && n > 0) ? n : 1;
}

hipError_t launch_chain64(const Chain64Launch& a, int n_blocks, hipStream_t stream) {
  if (a.K < 1 || a.K > 5 || a.M < 1 || a.M > 16) return hipErrorInvalidValue;
  gst_launch(chain64_kernel, dim3(n_blocks), dim3(CHAIN64_WAVES * 64), chain64_lds(a.K), stream, a);
  return hipGetLastError();
}

hipError_t launch_gemm64(const Gemm64Launch& a, hipStream_t stream) {
  if (a.n_chunks <= 0) return hipSuccess;
  gst_launch(gemm64_kernel, dim3(a.n_chunks), dim3(256), 0, stream, a);
  return hipGetLastError();
}

hipError_t launch_gate_prep64_batch(const Plan64Req* reqs, int n, int K_max, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  if (K_max < 1 || K_max > 5) return hipErrorInvalidValue;
  gst_launch(gate_prep64_batch, dim3(K_max, n), dim3(256), 0, stream, reqs);
  return hipGetLastError();
}

hipError_t launch_plan64_fwd_batch(const Plan64Req* reqs, int n, int level, int grid_x, bool reg_gates,
                                   hipStream_t stream) {
  if (n <= 0 || grid_x <= 0) return hipSuccess;
  if (reg_gates)
    gst_launch(plan64_fwd_batch<RegGates>, dim3(grid_x, n), dim3(256), 0, stream, reqs, level, 1);
  else
    gst_launch(plan64_fwd_batch<LoadGates>, dim3(grid_x, n), dim3(256), 0, stream, reqs, level, 0);
  return hipGetLastError();
}

hipError_t launch_plan64_bwd_batch(const Plan64Req* reqs, int n, int level, int grid_x, bool reg_gates,
                                   hipStream_t stream) {
  if (n <= 0 || grid_x <= 0) return hipSuccess;
  if (reg_gates)
    gst_launch(plan64_bwd_batch<RegGates>, dim3(grid_x, n), dim3(256), 0, stream, reqs, level, 1);
  else
    gst_launch(plan64_bwd_batch<LoadGates>, dim3(grid_x, n), dim3(256), 0, stream, reqs, level, 0);
  return hipGetLastError();
}

hipError_t launch_readout64_batch(const Plan64Req* reqs, int n, int grid_x, hipStream_t stream) {
  if (n <= 0 || grid_x <= 0) return hipSuccess;
  gst_launch(readout64_batch, dim3(grid_x, n), dim3(READOUT64_WAVES * 64), 0, stream, reqs);
  return hipGetLastError();
}

hipError_t launch_gemm64_ts_batch(const Plan64Req* reqs, int n, int grid_x, hipStream_t stream) {
  if (n <= 0 || grid_x <= 0) return hipSuccess;
  gst_launch(gemm64_ts_batch, dim3(grid_x, n), dim3(256), 0, stream, reqs);
  return hipGetLastError();
}

hipError_t launch_root64_batch(const Plan64Req* reqs, int n, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  gst_launch(root64_batch, dim3(1, n), dim3(64), 0, stream, reqs);
  return hipGetLastError();
}

hipError_t launch_slab_sum64_batch(const Plan64Req* reqs, int n, int grid_x, int parts_max, hipStream_t stream) {
  if (n <= 0 || grid_x <= 0) return hipSuccess;
  if (parts_max < 1 || parts_max > 64) return hipErrorInvalidValue;
  gst_launch(slab_sum64_stage1_batch, dim3(grid_x, parts_max, n), dim3(256), 0, stream, reqs);
  gst_launch(slab_sum64_stage2_batch, dim3(grid_x, n), dim3(256), 0, stream, reqs);
  return hipGetLastError();
}

hipError_t launch_reduce64_batch(const Plan64Req* reqs, int n, int grid_x, hipStream_t stream) {
  if (n <= 0 || grid_x <= 0) return hipSuccess;
  gst_launch(reduce64_batch, dim3(grid_x, n), dim3(256), 0, stream, reqs);
  return hipGetLastError();
}

hipError_t launch_reduce64(const Reduce64Launch& a, hipStream_t stream) {
  const int64_t Y = (int64_t)a.K * GATE64;
  if (Y == 0 || !a.grad) return hipSuccess;
  gst_launch(reduce64_kernel, dim3((unsigned)((Y + 63) / 64)), dim3(256), 0, stream, a);
  return hipGetLastError();
}

}  // namespace gst
