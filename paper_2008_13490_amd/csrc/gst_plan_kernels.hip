// Kernels of the shared-prefix plan (one- and two-qubit gate sets).
//
// Thesis Eq. GSTFullFiducialsGerms: sequences F_q g^l F_p share F_p g^l.  The
// plan (gst_plan.h) splits the evaluation into
//   trunk_fwd_kernel  long shared prefixes, one 16-lane team each; every state
//                     is stored in the state arena FA (the forward products are
//                     the same operations as in the plain evaluation, so the
//                     probabilities stay bit-identical);
//   item_kernel       every sequence from its deepest stored state: the rest of
//                     its word, readout, objective, seeds and the reverse sweep
//                     of that rest; states before and adjoints after each step
//                     go to the arenas;
//   inject_kernel     adjoints arriving at each stored state, summed in a
//                     fixed order;
//   trunk_bwd_kernel  reverse sweep of the trunks, adding the injected
//                     adjoints; adjoints after each step go to the arena;
//   grad_gemm_kernel  dG_k = sum over all steps with gate k of b f^T, as FP64
//                     MFMA 16x16x4 rank-4 updates over the stored pairs.
// The two chains (forward and reverse) are latency bound; the gradient GEMM
// runs over all stored steps at once.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "gst_device.h"
#include "gst_internal.h"

namespace gst {
namespace {

__device__ __forceinline__ double load_state(const double* FA, int64_t row, int D, int i) {
  return i < D ? FA[row * D + i] : 0.0;
}

// ---------------------------------------------------------------------------
// Trunk kernels: one trunk per wave.  The chains are latency bound.  Each
// trunk's gate word comes as periodic segments (a pattern of 1..4 gates
// repeated; germ powers are exactly this), so the rows of a segment's gates are
// loaded into registers once and the steps of the segment run with no memory
// access other than the store of the result.  Lanes 16..63 repeat the work of
// lanes 0..15 (same rows, same inputs); only lanes 0..D-1 store.
// ---------------------------------------------------------------------------
constexpr int SEGW = 64;  // segment descriptors held at a time (one per lane)

// Doubles of LDS in front of the per-wave staging of injected vectors (the
// gate set, its transpose, the effects and rho).
__host__ __device__ inline size_t trunk_head_doubles(int K) {
  return (size_t)2 * K * GATE_STRIDE + 2 * 16 * ROW + 16;
}

// Item and fill workgroups hold only the gate set (no checkpoint stash); the
// head-row reduction reuses it afterwards.
__host__ __device__ inline size_t item_lds_bytes(int K) {
  const size_t a = trunk_head_doubles(K) * 8, r = (size_t)WAVES * (1 + 16 + 256) * 8;
  return (a > r ? a : r) + 64;
}

// Per wave after the staging area: the trunk's jump matrices, `levels` of
// them in the gate layout.
__host__ __device__ inline size_t trunk_jump_doubles(int K, int wave, int levels) {
  return trunk_head_doubles(K) + (size_t)WAVES * SEGW * 16 + (size_t)wave * levels * GATE_STRIDE;
}

__host__ __device__ inline size_t trunk_lds_bytes(int K, int levels) {
  const size_t a = trunk_jump_doubles(K, WAVES, levels) * 8 + 64;
  const size_t r = lds_red_bytes(K);
  return a > r ? a : r;
}

struct Seg {
  int start, count, per, g0, g1, g2, g3;
};

// Descriptors of up to 64 consecutive segments, lane j holding segment
// base + j: one batch of loads per 64 segments instead of a dependent load
// at the start of every segment (segments can be a single step long).
struct SegLanes {
  int start, count, pat, g3;
  int64_t slot;
};

__device__ __forceinline__ SegLanes load_seg_lanes(const PlanArgs& a, int64_t sg, int64_t sg_end, bool want_slot) {
  SegLanes d{0, 0, 0, 0, -1};
  if (sg < sg_end) {
    d.start = a.seg_start[sg];
    d.count = a.seg_count[sg];
    d.pat = (int)a.seg_pattern[sg];
    d.g3 = (int)a.seg_gate3[sg];
    if (want_slot) d.slot = a.seg_inj[sg];
  }
  return d;
}

__device__ __forceinline__ Seg seg_of(const SegLanes& d, int x) {
  Seg g;
  const uint32_t pat = (uint32_t)__builtin_amdgcn_readlane(d.pat, x);
  g.start = __builtin_amdgcn_readlane(d.start, x);
  g.count = __builtin_amdgcn_readlane(d.count, x);
  g.per = (int)(pat & 0xffu);
  g.g0 = (int)((pat >> 8) & 0xffu);
  g.g1 = (int)((pat >> 16) & 0xffu);
  g.g2 = (int)((pat >> 24) & 0xffu);
  g.g3 = __builtin_amdgcn_readlane(d.g3, x);
  return g;
}

// C = A B for 16 x 16 matrices in the gate layout, by one wave: column c of
// C is A times column c of B, a dot16 per 16-lane team, four columns per team.
__device__ __forceinline__ void wave_matmul(double* C, const double* A, const double* B, int lane) {
  const int i = lane & 15, t = lane >> 4;
  const Row16 Ar = load_row(A + i * ROW);
  double y[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) y[u] = dot16(B[i * ROW + 4 * u + t], Ar);
#pragma unroll
  for (int u = 0; u < 4; ++u) C[i * ROW + 4 * u + t] = y[u];
  wave_sync();
}

// The trunk's jump matrices into the wave's slots js[e * GATE_STRIDE]: slot 0
// = G_{g_per-1} ... G_{g_0} of the pattern (reverse: its transpose G_{g_0}^T
// ... G_{g_per-1}^T, from the transposed gate set), slot e = slot e-1 squared.
__device__ void build_jumps(double* js, const double* gates, uint32_t pat, int g3, int levels, bool rev,
                            int lane) {
  const int per = (int)(pat & 0xffu);
  const int g[4] = {(int)((pat >> 8) & 0xffu), (int)((pat >> 16) & 0xffu), (int)((pat >> 24) & 0xffu), g3};
  const int i = lane & 15, t = lane >> 4;
  if (per == 1) {
#pragma unroll
    for (int u = 0; u < 4; ++u) js[i * ROW + 4 * u + t] = gates[g[0] * GATE_STRIDE + i * ROW + 4 * u + t];
    wave_sync();
  } else {
    const double* src = gates + g[rev ? per - 1 : 0] * GATE_STRIDE;
    for (int k = 1; k < per; ++k) {  // the last product lands in slot 0
      double* dst = js + (((per - 1 - k) & 1) ? GATE_STRIDE : 0);
      wave_matmul(dst, gates + g[rev ? per - 1 - k : k] * GATE_STRIDE, src, lane);
      src = dst;
    }
  }
  for (int e = 1; e < levels; ++e)
    wave_matmul(js + e * GATE_STRIDE, js + (e - 1) * GATE_STRIDE, js + (e - 1) * GATE_STRIDE, lane);
}

template <int D>
__global__ __launch_bounds__(256) void trunk_fwd_kernel(const PlanArgs a) {
  extern __shared__ double lds_raw[];
  const int K = a.K;
  const Lds s = carve(lds_raw, K);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, i = lane & 15;
  stage_gateset<D>(s, a.G, a.E, a.rho, K, a.M);
  if (blockIdx.x == 0 && tid < D) a.FA[tid] = a.rho[tid];
  const double* gl = s.Gs + i * ROW;
  double* js = lds_raw + trunk_jump_doubles(K, wave, a.jump_levels);
  for (int64_t t = a.t_begin + (int64_t)blockIdx.x * WAVES + wave; t < a.t_end; t += (int64_t)gridDim.x * WAVES) {
    const int64_t beg = a.trunk_ptr[t];
    const int64_t anc = a.trunk_anchor[t];
    const uint32_t jp = (uint32_t)__builtin_amdgcn_readfirstlane((int)a.trunk_jpat[t]);
    if (jp != 0u) build_jumps(js, s.Gs, jp, a.trunk_jg3[t], a.jump_levels, false, lane);
    double f = anc >= 0 ? load_state(a.FA, 1 + anc, D, i) : s.rho[i];
    double* out = a.FA + (1 + beg) * D + i;
    const bool st = (D == 16) || lane < D;  // rows 1..3 store the same values as row 0
    const int64_t sg0 = a.seg_ptr[t], sg1 = a.seg_ptr[t + 1];
    for (int64_t cb = sg0; cb < sg1; cb += SEGW) {
    const SegLanes d = load_seg_lanes(a, cb + lane, sg1, false);
    const int n = (int)(sg1 - cb < SEGW ? sg1 - cb : SEGW);
    for (int x = 0; x < n; ++x) {
      const Seg g = seg_of(d, x);
      if (g.per == 0) {  // count jumps of g.g0 steps by jump matrix g.g1; the state after each is stored
        const Row16 RC = load_row(js + g.g1 * GATE_STRIDE + i * ROW);
        const int64_t stride = g.g0;
        double* o = out + (g.start + stride - 1) * D;
        for (int c = 0; c < g.count; ++c) {
          f = dot16(f, RC);
          if (st) o[0] = f;
          o += stride * D;
        }
        continue;
      }
      double* o = out + (int64_t)g.start * D;
      const Row16 R0 = load_row(gl + g.g0 * GATE_STRIDE);
      if (g.per == 1) {
        for (int c = 0; c < g.count; ++c) {
          f = dot16(f, R0);
          if (st) o[0] = f;
          o += D;
        }
      } else if (g.per == 2) {
        const Row16 R1 = load_row(gl + g.g1 * GATE_STRIDE);
        for (int c = 0; c < g.count; ++c) {
          f = dot16(f, R0);
          if (st) o[0] = f;
          f = dot16(f, R1);
          if (st) o[D] = f;
          o += 2 * D;
        }
      } else if (g.per == 3) {
        const Row16 R1 = load_row(gl + g.g1 * GATE_STRIDE);
        const Row16 R2 = load_row(gl + g.g2 * GATE_STRIDE);
        for (int c = 0; c < g.count; ++c) {
          f = dot16(f, R0);
          if (st) o[0] = f;
          f = dot16(f, R1);
          if (st) o[D] = f;
          f = dot16(f, R2);
          if (st) o[2 * D] = f;
          o += 3 * D;
        }
      } else {
        const Row16 R1 = load_row(gl + g.g1 * GATE_STRIDE);
        const Row16 R2 = load_row(gl + g.g2 * GATE_STRIDE);
        const Row16 R3 = load_row(gl + g.g3 * GATE_STRIDE);
        for (int c = 0; c < g.count; ++c) {
          f = dot16(f, R0);
          if (st) o[0] = f;
          f = dot16(f, R1);
          if (st) o[D] = f;
          f = dot16(f, R2);
          if (st) o[2 * D] = f;
          f = dot16(f, R3);
          if (st) o[3 * D] = f;
          o += 4 * D;
        }
      }
    }
    }
  }
}

// ---------------------------------------------------------------------------
// items: one sequence per team, from its anchor state
// ---------------------------------------------------------------------------
template <int D, bool REV>
__device__ void run_fills(const PlanArgs& a, const Lds& s, int64_t blk, int64_t n_blk);

// Workgroups from a.item_blocks on run the forward fill tasks instead (they
// need only the trunk states, like the items).
template <int D>
__global__ __launch_bounds__(256) void item_kernel(const PlanArgs a) {
  extern __shared__ double lds_raw[];
  const int K = a.K, M = a.M;
  const Lds s = carve(lds_raw, K);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, i = lane & 15, team = lane >> 4;
  stage_gateset<D>(s, a.G, a.E, a.rho, K, M);
  if ((int)blockIdx.x >= a.item_blocks) {
    run_fills<D, false>(a, s, (int64_t)blockIdx.x - a.item_blocks, (int64_t)gridDim.x - a.item_blocks);
    return;
  }
  const bool grad = a.want_grad != 0;
  double obj = 0.0, drho = 0.0;
  double dE[16];
#pragma unroll
  for (int m = 0; m < 16; ++m) dE[m] = 0.0;
  unsigned nonpos = 0;
  const int64_t n_groups = (a.n_items + TPW - 1) / TPW;
  for (int64_t grp = (int64_t)blockIdx.x * WAVES + wave; grp < n_groups; grp += (int64_t)a.item_blocks * WAVES) {
    const int64_t q = grp * TPW + team;
    const bool has = q < a.n_items;
    int64_t seq = 0, beg = 0, end = 0, anc = -1, isp = 0;
    if (has) {
      const int64_t* it = a.items + 4 * q;
      seq = it[0];
      beg = it[1];
      end = it[2];
      anc = it[3];
      isp = a.item_step_ptr[q];
    }
    const int L = (int)(end - beg);
    const int Lw = wave_max4(L);
    const uint8_t* word = a.gates + beg;
    double* fa = a.FA + (1 + a.nTS + isp) * D;  // state before item step x: fa[x*D + i]
    double* ba = a.BA + (a.nTS + isp) * D;      // adjoint after item step x
    double f = anc >= 0 ? load_state(a.FA, 1 + anc, D, i) : s.rho[i];

    // ---- forward over the rest of the word ----
    for (int t0 = 0; t0 < Lw; t0 += 16) {
      const int kv = (t0 + i < L) ? (int)word[t0 + i] : 0;
#define GST_IF(R)                                                        \
  if (t0 + R < Lw) {                                                     \
    const int x = t0 + R;                                                \
    const int k = bcast_i32<R>(kv);                                      \
    if (grad && x < L && i < D) fa[(int64_t)x * D + i] = f;              \
    const double fn = dot16(f, load_row(s.Gs + k * GATE_STRIDE + i * ROW)); \
    f = x < L ? fn : f;                                                  \
  }
      GST_IF(0) GST_IF(1) GST_IF(2) GST_IF(3) GST_IF(4) GST_IF(5) GST_IF(6) GST_IF(7)
      GST_IF(8) GST_IF(9) GST_IF(10) GST_IF(11) GST_IF(12) GST_IF(13) GST_IF(14) GST_IF(15)
#undef GST_IF
    }

    // ---- readout, objective, seeds ----
    const double p = dot16(f, load_row(s.Es + i * ROW));
    double dp = 0.0;
    if (has && i < M) {
      const int64_t o = seq * M + i;
      if (a.probs) a.probs[o] = p;
      if (a.mode == MODE_LOGLIK) {
        const int32_t N = a.counts[o];
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
        dp = a.W[o];
      }
    }
    if (!grad) continue;
#define GST_DE(R) \
  if (R < M) dE[R] = fma(bcast_f64<R>(dp), f, dE[R]);
    GST_DE(0) GST_DE(1) GST_DE(2) GST_DE(3) GST_DE(4) GST_DE(5) GST_DE(6) GST_DE(7)
    GST_DE(8) GST_DE(9) GST_DE(10) GST_DE(11) GST_DE(12) GST_DE(13) GST_DE(14) GST_DE(15)
#undef GST_DE
    double b = dot16(dp, load_row(s.ETs + i * ROW));

    // ---- reverse sweep of the rest of the word ----
    const int nb = (Lw + 15) / 16;
    for (int c = nb - 1; c >= 0; --c) {
      const int t0 = c * 16;
      const int kv = (t0 + i < L) ? (int)word[t0 + i] : 0;
#define GST_IB(R)                                                         \
  if (t0 + R < Lw) {                                                      \
    const int x = t0 + R;                                                 \
    const int k = bcast_i32<R>(kv);                                       \
    if (x < L && i < D) ba[(int64_t)x * D + i] = b;                       \
    const double bn = dot16(b, load_row(s.GTs + k * GATE_STRIDE + i * ROW)); \
    b = x < L ? bn : b;                                                   \
  }
      GST_IB(15) GST_IB(14) GST_IB(13) GST_IB(12) GST_IB(11) GST_IB(10) GST_IB(9) GST_IB(8)
      GST_IB(7) GST_IB(6) GST_IB(5) GST_IB(4) GST_IB(3) GST_IB(2) GST_IB(1) GST_IB(0)
#undef GST_IB
    }
    if (has && i < D) a.item_adj[q * D + i] = b;
    if (has && anc < 0) drho += b;
  }
  if (nonpos) {
    atomicAdd(a.status + 1, (unsigned long long)nonpos);
    if (a.req_nonpos) atomicAdd(a.req_nonpos, (unsigned long long)nonpos);
  }
  if (a.mode != MODE_LOGLIK && !grad) return;
  d4 none[KMAX];
  write_slab<D>(lds_raw, obj, drho, dE, none, M, 0, a.slab + (int64_t)blockIdx.x * slab_width(D, M, 0));
}

// ---------------------------------------------------------------------------
// trunk reverse sweep, one trunk per wave: segments in reverse, G^T rows of a
// segment in registers; adjoints injected at stored states (a descending list
// per trunk, staged in LDS) are added on the way back
// ---------------------------------------------------------------------------
template <int D>
__global__ __launch_bounds__(256) void trunk_bwd_kernel(const PlanArgs a) {
  extern __shared__ double lds_raw[];
  const int K = a.K;
  const Lds s = carve(lds_raw, K);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, i = lane & 15;
  stage_gateset<D>(s, a.G, a.E, a.rho, K, a.M);
  const double* gl = s.GTs + i * ROW;
  double* inj_st = lds_raw + trunk_head_doubles(K) + (size_t)wave * SEGW * 16;
  double* js = lds_raw + trunk_jump_doubles(K, wave, a.jump_levels);
  double drho = 0.0;
  for (int64_t t = a.t_begin + (int64_t)blockIdx.x * WAVES + wave; t < a.t_end; t += (int64_t)gridDim.x * WAVES) {
    const int64_t beg = a.trunk_ptr[t];
    const uint32_t jp = (uint32_t)__builtin_amdgcn_readfirstlane((int)a.trunk_jpat[t]);
    if (jp != 0u) build_jumps(js, s.GTs, jp, a.trunk_jg3[t], a.jump_levels, true, lane);
    double* ba = a.BA + beg * D + i;
    const bool st = (D == 16) || lane < D;
    const int64_t sg0 = a.seg_ptr[t], sg1 = a.seg_ptr[t + 1];
    double b = 0.0;
#define GST_TBSTEP(RT, J)                    \
  {                                          \
    if (st) ba[(int64_t)(J) * D] = b;        \
    b = dot16(b, RT);                  \
  }
    // segments in reverse, 64 at a time: their descriptors in registers and
    // their injected vectors (the adjoint arriving at the state after each
    // segment's last step) staged in this wave's LDS, all loaded up front
    for (int64_t ce = sg1; ce > sg0; ce -= SEGW) {
    const int64_t cb = ce - SEGW > sg0 ? ce - SEGW : sg0;
    const int n = (int)(ce - cb);
    const SegLanes d = load_seg_lanes(a, cb + lane, ce, true);
    wave_sync();  // the previous chunk's vectors have been read
#pragma unroll 4
    for (int q = 0; q < SEGW / 4; ++q) {
      const int x = 4 * q + (lane >> 4);
      const int64_t slot = __shfl(d.slot, x);
      const double v = (x < n && slot >= 0 && i < D) ? a.inj[slot * D + i] : 0.0;
      inj_st[x * 16 + i] = v;
    }
    wave_sync();
    for (int x = n - 1; x >= 0; --x) {
      const Seg g = seg_of(d, x);
      b += inj_st[x * 16 + i];  // adjoint arriving at the state after the segment's last step
      if (g.per == 0) {  // jumps in reverse with the transposed matrix
        const Row16 RC = load_row(js + g.g1 * GATE_STRIDE + i * ROW);
        const int stride = g.g0;
        for (int c = g.count - 1; c >= 0; --c) GST_TBSTEP(RC, g.start + (c + 1) * stride - 1)
        continue;
      }
      const Row16 R0 = load_row(gl + g.g0 * GATE_STRIDE);
      if (g.per == 1) {
        for (int c = g.count - 1; c >= 0; --c) GST_TBSTEP(R0, g.start + c)
      } else if (g.per == 2) {
        const Row16 R1 = load_row(gl + g.g1 * GATE_STRIDE);
        for (int c = g.count - 1; c >= 0; --c) {
          const int j0 = g.start + 2 * c;
          GST_TBSTEP(R1, j0 + 1)
          GST_TBSTEP(R0, j0)
        }
      } else if (g.per == 3) {
        const Row16 R1 = load_row(gl + g.g1 * GATE_STRIDE);
        const Row16 R2 = load_row(gl + g.g2 * GATE_STRIDE);
        for (int c = g.count - 1; c >= 0; --c) {
          const int j0 = g.start + 3 * c;
          GST_TBSTEP(R2, j0 + 2)
          GST_TBSTEP(R1, j0 + 1)
          GST_TBSTEP(R0, j0)
        }
      } else {
        const Row16 R1 = load_row(gl + g.g1 * GATE_STRIDE);
        const Row16 R2 = load_row(gl + g.g2 * GATE_STRIDE);
        const Row16 R3 = load_row(gl + g.g3 * GATE_STRIDE);
        for (int c = g.count - 1; c >= 0; --c) {
          const int j0 = g.start + 4 * c;
          GST_TBSTEP(R3, j0 + 3)
          GST_TBSTEP(R2, j0 + 2)
          GST_TBSTEP(R1, j0 + 1)
          GST_TBSTEP(R0, j0)
        }
      }
    }
    }
#undef GST_TBSTEP
    if (lane < D) a.trunk_adj[t * D + i] = b;
    if (a.trunk_anchor[t] < 0) drho += b;
  }
  // lanes 16..63 repeat lanes 0..15: only row 0 contributes
  if (lane >= 16) drho = 0.0;
  double dE[16];
#pragma unroll
  for (int m = 0; m < 16; ++m) dE[m] = 0.0;
  d4 none[KMAX];
  write_slab<D>(lds_raw, 0.0, drho, dE, none, a.M, 0, a.slab + (int64_t)blockIdx.x * slab_width(D, a.M, 0));
}

// ---------------------------------------------------------------------------
// fill tasks: the states (forward) or adjoints (reverse) inside one jump, one
// task per 16-lane team, from the stored value at the jump's start (forward)
// or end (reverse).  Step j of a task applies gate pattern[j % period].
// ---------------------------------------------------------------------------
template <int D, bool REV>
__device__ void run_fills(const PlanArgs& a, const Lds& s, int64_t blk, int64_t n_blk) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, i = lane & 15, team = lane >> 4;
  const double* gl = (REV ? s.GTs : s.Gs) + i * ROW;
  const int64_t n_groups = (a.n_fill + TPW - 1) / TPW;
  for (int64_t grp = blk * WAVES + wave; grp < n_groups; grp += n_blk * WAVES) {
    const int64_t q = grp * TPW + team;
    const bool has = q < a.n_fill;
    int64_t first = 0, in = 0;
    int n = 1;
    uint32_t pat = 1u;
    int g3 = 0;
    if (has) {
      first = a.fill_first[q];
      in = a.fill_in[q];
      n = a.fill_n[q];
      pat = a.fill_pattern[q];
      g3 = a.fill_gate3[q];
    }
    const int per = (int)(pat & 0xffu);
    const int nw = wave_max4(n);
    const bool st = has && i < D;
    auto gate = [&](int j) {
      const int ph = j % per;
      return ph == 0 ? (int)((pat >> 8) & 0xffu) : ph == 1 ? (int)((pat >> 16) & 0xffu)
                                                 : ph == 2 ? (int)((pat >> 24) & 0xffu) : g3;
    };
    if (!REV) {
      // states after steps 0 .. n-2 (the one after step n-1 is the jump's)
      double f = load_state(a.FA, in, D, i);
      double* o = a.FA + (1 + first) * D + i;
      Row16 R = load_row(gl + gate(0) * GATE_STRIDE);
      for (int j = 0; j + 1 < nw; ++j) {
        const Row16 Rn = load_row(gl + gate(j + 1) * GATE_STRIDE);
        f = dot16(f, R);
        if (st && j + 1 < n) o[(int64_t)j * D] = f;
        R = Rn;
      }
    } else {
      // adjoints after steps n-2 .. 0, from the one after step n-1
      double b = st ? a.BA[(first + n - 1) * D + i] : 0.0;
      double* o = a.BA + first * D + i;
      Row16 R = load_row(gl + gate(nw - 1) * GATE_STRIDE);
      for (int j = nw - 1; j >= 1; --j) {
        const Row16 Rn = load_row(gl + gate(j - 1) * GATE_STRIDE);
        const double nb = dot16(b, R);
        if (j < n) {
          b = nb;
          if (st) o[(int64_t)(j - 1) * D] = b;
        }
        R = Rn;
      }
    }
  }
}

// reverse fill tasks (the forward ones run in the item kernel's extra workgroups)
template <int D>
__global__ __launch_bounds__(256) void fill_rev_kernel(const PlanArgs a) {
  extern __shared__ double lds_raw[];
  const Lds s = carve(lds_raw, a.K);
  stage_gateset<D>(s, a.G, a.E, a.rho, a.K, a.M);
  run_fills<D, true>(a, s, blockIdx.x, gridDim.x);
}

// One wave per injection slot: four groups of 16 lanes take every fourth
// source (two independent partial sums each), then the groups are combined
// in a fixed order.
__global__ __launch_bounds__(64) void inject_kernel(const InjectLaunch a) {
  const int D = a.D;
  const int lane = threadIdx.x, g = lane >> 4, i = lane & 15;
  for (int64_t slot = a.s_begin + blockIdx.x; slot < a.s_end; slot += gridDim.x) {
    const int64_t z0 = a.inj_ptr[slot], z1 = a.inj_ptr[slot + 1];
    double v0 = 0.0, v1 = 0.0;
    if (i < D) {
      int64_t z = z0 + g;
      for (; z + 4 < z1; z += 8) {
        const int64_t s0 = a.inj_src[z], s1 = a.inj_src[z + 4];
        v0 += s0 >= 0 ? a.item_adj[s0 * D + i] : a.trunk_adj[(-s0 - 1) * D + i];
        v1 += s1 >= 0 ? a.item_adj[s1 * D + i] : a.trunk_adj[(-s1 - 1) * D + i];
      }
      if (z < z1) {
        const int64_t s0 = a.inj_src[z];
        v0 += s0 >= 0 ? a.item_adj[s0 * D + i] : a.trunk_adj[(-s0 - 1) * D + i];
      }
    }
    double v = v0 + v1;
    v += __shfl_xor(v, 16);
    v += __shfl_xor(v, 32);
    if (lane < D) a.inj[slot * D + i] = v;
  }
}

// ---------------------------------------------------------------------------
// gradient GEMM over the stored (adjoint, state) pairs, one chunk of records
// of one gate per workgroup; four records per MFMA 16x16x4
// ---------------------------------------------------------------------------
template <int D>
__global__ __launch_bounds__(256) void grad_gemm_kernel(const GemmLaunch a) {
  __shared__ double tile[WAVES][256];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, i = lane & 15, z = lane >> 4;
  const int64_t c = blockIdx.x;
  const int64_t r0 = a.chunk_beg[c], r1 = a.chunk_end[c];
  const int k = (int)a.chunk_gate[c];
  d4 acc = {0.0, 0.0, 0.0, 0.0};
  // records r0 + 16*u + 4*wave + z, u = 0..7 (chunks hold at most 128 records)
  int64_t rb[8], rf[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int64_t r = r0 + 16 * u + 4 * wave + z;
    rb[u] = r < r1 ? a.rec_b[r] : -1;
    rf[u] = r < r1 ? a.rec_f[r] : -1;
  }
  double av[8], bv[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    av[u] = (rb[u] >= 0 && i < D) ? a.BA[rb[u] * D + i] : 0.0;
    bv[u] = (rf[u] >= 0 && i < D) ? a.FA[rf[u] * D + i] : 0.0;
  }
#pragma unroll
  for (int u = 0; u < 8; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv[u], acc, 0, 0, 0);
#pragma unroll
  for (int v = 0; v < 4; ++v) tile[wave][(4 * v + (lane >> 4)) * 16 + (lane & 15)] = acc[v];
  __syncthreads();
  if (tid < D * D) {
    const int r = tid / D, cc = tid % D;
    a.tiles[c * D * D + tid] =
        (tile[0][r * 16 + cc] + tile[1][r * 16 + cc]) + (tile[2][r * 16 + cc] + tile[3][r * 16 + cc]);
  }
}

// ---------------------------------------------------------------------------
// ordered sum of head rows and per-gate chunk tiles (two stages, fixed order)
// ---------------------------------------------------------------------------
struct Rows {
  const double* src;  // row 0, this column
  int64_t stride;
  int64_t n;
};

__device__ inline int parts_of(int64_t n) {
  const int64_t g = (n + 15) / 16;
  return g < 1 ? 1 : (g > 64 ? 64 : (int)g);
}

__device__ inline Rows rows_of(const PlanReduce& a, int64_t x) {
  const int64_t H = 1 + a.D + (int64_t)a.M * a.D, DD = (int64_t)a.D * a.D;
  if (x < H) return Rows{a.head + x, H, a.n_head};
  const int64_t y = x - H, k = y / DD;
  const int64_t c0 = a.chunk_ptr[k], c1 = a.chunk_ptr[k + 1];
  return Rows{a.tiles + c0 * DD + (y - k * DD), DD, c1 - c0};
}

// Block (x, g): rows [g*per, (g+1)*per) of each column's region, four
// interleaved partial sums combined in a fixed order.
__global__ __launch_bounds__(256) void plan_reduce_stage1(const PlanReduce a) {
  __shared__ double red[4][64];
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int64_t x = (int64_t)blockIdx.x * 64 + tx;
  const int g = blockIdx.y;
  double v = 0.0;
  int G = 0;
  if (x < a.P) {
    const Rows R = rows_of(a, x);
    G = parts_of(R.n);
    const int64_t per = (R.n + G - 1) / G, w0 = g * per, w1 = min(R.n, w0 + per);
    if (g < G)
      for (int64_t w = w0 + ty; w < w1; w += 4) v += R.src[w * R.stride];
  }
  red[ty][tx] = v;
  __syncthreads();
  if (ty == 0 && x < a.P && g < G) a.part[(int64_t)g * a.P + x] = (red[0][tx] + red[1][tx]) + (red[2][tx] + red[3][tx]);
}

// Column x adds its region's stage-1 partials in ascending g.  A +inf
// objective partial marks p <= 0 with N > 0: the objective is then +inf and
// the gradient is not written.
__global__ __launch_bounds__(256) void plan_reduce_stage2(const PlanReduce a) {
  __shared__ double red[4][64];
  __shared__ int nonpos_sh;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int64_t x = (int64_t)blockIdx.x * 64 + tx;
  double v = 0.0;
  if (x < a.P) {
    const int G = parts_of(rows_of(a, x).n);
    for (int g = ty; g < G; g += 4) v += a.part[(int64_t)g * a.P + x];
  }
  red[ty][tx] = v;
  if (ty == 1) {
    const bool inf = tx < parts_of(a.n_head) && isinf(a.part[(int64_t)tx * a.P]);
    const bool any = __ballot(inf) != 0ull;
    if (tx == 0) nonpos_sh = any ? 1 : 0;
  }
  __syncthreads();
  const bool nonpos = nonpos_sh != 0;
  if (ty != 0 || x >= a.P) return;
  v = (red[0][tx] + red[1][tx]) + (red[2][tx] + red[3][tx]);
  if (x == 0) {
    if (a.objective) *a.objective = nonpos ? INFINITY : v;
  } else if (a.grad && !nonpos) {
    a.grad[x - 1] = v;
  }
}

}  // namespace

int fill_blocks_for(int64_t n_fill) {
  const int64_t b = (n_fill + WAVES * TPW - 1) / (WAVES * TPW);
  return (int)(b < 1 ? 1 : (b > 1024 ? 1024 : b));
}

int item_blocks_for(int64_t n_items) {
  int64_t b = (n_items + WAVES * TPW - 1) / (WAVES * TPW);
  if (b < 1) b = 1;
  if (b > 1024) b = 1024;  // four resident workgroups per CU
  return (int)b;
}

int trunk_blocks_for(int64_t n) {
  int64_t b = (n + WAVES - 1) / WAVES;
  return (int)(b < 1 ? 1 : (b > 4096 ? 4096 : b));
}

hipError_t launch_trunk_fwd(const PlanArgs& a, hipStream_t stream) {
  const int blocks = trunk_blocks_for(a.t_end - a.t_begin);
  const size_t bytes = trunk_lds_bytes(a.K, a.jump_levels);
  if (a.D == 16)
    hipLaunchKernelGGL(trunk_fwd_kernel<16>, dim3(blocks), dim3(256), bytes, stream, a);
  else if (a.D == 4)
    hipLaunchKernelGGL(trunk_fwd_kernel<4>, dim3(blocks), dim3(256), bytes, stream, a);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_trunk_bwd(const PlanArgs& a, hipStream_t stream) {
  const int blocks = trunk_blocks_for(a.t_end - a.t_begin);
  const size_t bytes = trunk_lds_bytes(a.K, a.jump_levels);
  if (a.D == 16)
    hipLaunchKernelGGL(trunk_bwd_kernel<16>, dim3(blocks), dim3(256), bytes, stream, a);
  else if (a.D == 4)
    hipLaunchKernelGGL(trunk_bwd_kernel<4>, dim3(blocks), dim3(256), bytes, stream, a);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_items(const PlanArgs& a, int n_blocks, hipStream_t stream) {
  if (a.item_blocks != n_blocks) return hipErrorInvalidValue;
  const size_t bytes = item_lds_bytes(a.K);
  const unsigned grid = (unsigned)n_blocks + (a.want_grad && a.n_fill > 0 ? (unsigned)fill_blocks_for(a.n_fill) : 0u);
  if (a.D == 16)
    hipLaunchKernelGGL(item_kernel<16>, dim3(grid), dim3(256), bytes, stream, a);
  else if (a.D == 4)
    hipLaunchKernelGGL(item_kernel<4>, dim3(grid), dim3(256), bytes, stream, a);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_inject(const InjectLaunch& a, hipStream_t stream) {
  const int64_t n = a.s_end - a.s_begin;
  if (n <= 0) return hipSuccess;
  const int blocks = (int)(n < 65536 ? n : 65536);
  hipLaunchKernelGGL(inject_kernel, dim3(blocks), dim3(64), 0, stream, a);
  return hipGetLastError();
}

hipError_t launch_fill_rev(const PlanArgs& a, hipStream_t stream) {
  if (a.n_fill <= 0) return hipSuccess;
  const int blocks = fill_blocks_for(a.n_fill);
  const size_t bytes = item_lds_bytes(a.K);
  if (a.D == 16)
    hipLaunchKernelGGL(fill_rev_kernel<16>, dim3((unsigned)blocks), dim3(256), bytes, stream, a);
  else if (a.D == 4)
    hipLaunchKernelGGL(fill_rev_kernel<4>, dim3((unsigned)blocks), dim3(256), bytes, stream, a);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_reduce_plan(const PlanReduce& a, hipStream_t stream) {
  if (a.P <= 0 || a.n_part < 1 || a.n_part > 64 || a.K < 0 || a.K > 8) return hipErrorInvalidValue;
  const unsigned xb = (unsigned)((a.P + 63) / 64);
  hipLaunchKernelGGL(plan_reduce_stage1, dim3(xb, (unsigned)a.n_part), dim3(256), 0, stream, a);
  hipLaunchKernelGGL(plan_reduce_stage2, dim3(xb), dim3(256), 0, stream, a);
  return hipGetLastError();
}

hipError_t launch_grad_gemm(const GemmLaunch& a, hipStream_t stream) {
  if (a.n_chunks <= 0) return hipSuccess;
  if (a.D == 16)
    hipLaunchKernelGGL(grad_gemm_kernel<16>, dim3((unsigned)a.n_chunks), dim3(256), 0, stream, a);
  else if (a.D == 4)
    hipLaunchKernelGGL(grad_gemm_kernel<4>, dim3((unsigned)a.n_chunks), dim3(256), 0, stream, a);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace gst
