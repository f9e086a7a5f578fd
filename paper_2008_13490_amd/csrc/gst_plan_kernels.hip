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
//                     go to the arenas, the adjoint at its start state to the
//                     source arena (the sources of one stored state are
//                     consecutive rows there);
//   inject_kernel     adjoints arriving at each stored state, summed in a
//                     fixed order;
//   trunk_bwd_kernel  reverse sweep of the trunks, adding the injected
//                     adjoints; adjoints after each step go to the arena;
//   grad_gemm_kernel  dG_k = sum over all steps with gate k of b f^T, as FP64
//                     MFMA 16x16x4 rank-4 updates over the stored pairs.
// The two chains (forward and reverse) are latency bound; the gradient GEMM
// runs over all stored steps at once.  The records that only the gradient GEMM
// reads (the items' states and adjoints, the states and adjoints filled inside
// jumps) are stored non-temporally: written through to memory instead of
// being held in the L2, whose write-back at the end of each kernel otherwise
// lengthens the item and fill launches.
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
// Trunk kernels: one trunk per workgroup of a single wave, so that the wave has
// its CU's LDS bandwidth to itself.  A trunk's chain is a flat list of ops,
// each a gate step or a germ-power jump; the rows of the next op are read
// from LDS while the current op's product runs.  The chains are latency
// bound.  Lanes 16..63 repeat the work of lanes 0..15 (same rows, same
// inputs); only lanes 0..D-1 store.
// ---------------------------------------------------------------------------
constexpr int OPW = 64;  // op descriptors held at a time (one per lane)

// Doubles of LDS in front of the staging of injected vectors (the gate set,
// its transpose, the effects and rho).
__host__ __device__ inline size_t trunk_head_doubles(int K) {
  return (size_t)2 * K * GATE_STRIDE + 2 * 16 * ROW + 16;
}

// A head row [objective | dL/drho | dL/dE]: every 16-lane team leaves its
// partial sums in LDS (no shuffles across teams, `hw` doubles per team: 17 +
// 16 M with the effects, 17 without), and the workgroup adds the team partials
// in a fixed order.
__host__ __device__ inline int head_stride(int M) { return 17 + 16 * M; }
__host__ __device__ inline size_t head_red_bytes(int n_waves, int M) {
  return (size_t)n_waves * TPW * head_stride(M) * 8;
}

template <int D, bool WITH_E, int NW>
__device__ void write_head(double* red, int hw, double obj, double drho, const double (&dE)[16], int M, double* out) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, i = lane & 15, team = lane >> 4;
  lds_sync();  // the previous contents of `red` have been read (no wait for global stores)
  double* mine = red + (size_t)(wave * TPW + team) * hw;
  double o = obj;
#pragma unroll
  for (int sh = 1; sh < 16; sh <<= 1) o += __shfl_xor(o, sh);
  if (i == 0) mine[0] = o;
  mine[1 + i] = drho;
  if (WITH_E) {
#pragma unroll
    for (int m = 0; m < 16; ++m)
      if (m < M) mine[17 + m * 16 + i] = dE[m];
  }
  lds_sync();
  const int H = 1 + D + M * D;
  for (int x = tid; x < H; x += blockDim.x) {
    int src = -1;
    if (x < 1 + D) {
      src = x;
    } else if (WITH_E) {
      const int y = x - 1 - D;
      src = 17 + (y / D) * 16 + (y % D);
    }
    double v = 0.0;
    if (src >= 0) {
#pragma unroll
      for (int p = 0; p < NW * TPW; ++p) v += red[p * hw + src];
    }
    out[x] = v;
  }
}

// A chunk's items staged in LDS: per item its descriptor (sequence, word
// begin and end, anchor, first record row), its start state, its counts and
// the first 16 gate indices of its word.
constexpr int IST_DESC = 6;
__host__ __device__ inline size_t item_stage_bytes() {
  return (size_t)kItemChunk * (IST_DESC * 8 + 16 * 8 + 16 * 4 + 16 * 4);
}

// Item and fill workgroups hold the gate set and, behind it, the head-row
// reduction of the item chunks and the staged chunk.
__host__ __device__ inline size_t item_lds_bytes(int K, int M) {
  return trunk_head_doubles(K) * 8 + head_red_bytes(WAVES, M) + item_stage_bytes() + 64;
}

// A trunk workgroup holds only what it uses: the gates (forward) or their
// transposes (reverse) at the start, rho, the staged injected vectors
// (reverse), and the trunk's jump matrices in the gate layout (at least two
// slots: the germ product alternates between slots 0 and 1).  Fewer bytes let
// more trunk workgroups share a CU when many requests run at once.
__device__ __forceinline__ Lds carve_trunk(double* base, int K) {
  Lds l;
  l.Gs = base;
  l.GTs = base;  // one of the two is staged
  l.Es = nullptr;
  l.ETs = nullptr;
  l.rho = base + (size_t)K * GATE_STRIDE;
  l.stash = nullptr;
  l.sk = nullptr;
  return l;
}
__host__ __device__ inline size_t trunk_inj_doubles(int K) { return (size_t)K * GATE_STRIDE + 16; }
__host__ __device__ inline size_t trunk_jump_doubles(int K) { return trunk_inj_doubles(K) + (size_t)OPW * 16; }

__host__ __device__ inline size_t trunk_lds_bytes(int K, int levels) {
  const size_t a = (trunk_jump_doubles(K) + (size_t)(levels > 2 ? levels : 2) * GATE_STRIDE) * 8 + 64;
  const size_t r = head_red_bytes(1, 0);
  return a > r ? a : r;
}

// Lane i's row of the matrix of op `od`: a gate (of the gate set or its
// transpose) or a jump matrix slot.
__device__ __forceinline__ const double* op_row(const double* gates, const double* js, uint32_t od, int i) {
  const double* base = (od & 0x80u) ? js : gates;
  return base + (od & 0x7fu) * GATE_STRIDE + i * ROW;
}

__device__ __forceinline__ uint32_t lane_u32(uint32_t v, int x) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, x);
}

// A trunk's descriptors, read by every lane (uniform addresses; the fourth
// jump gate is taken from the aligned word holding it, so that all of them
// are word loads).
struct TrunkMeta {
  int64_t beg, end, anchor, o0, o1;
  uint32_t jp;
  int jg3, jlev;
  int32_t src;
};
__device__ __forceinline__ TrunkMeta trunk_meta(const PlanArgs& a, int64_t t) {
  TrunkMeta m;
  m.beg = a.trunk_ptr[t];
  m.end = a.trunk_ptr[t + 1];
  m.anchor = a.trunk_anchor[t];
  m.o0 = a.op_ptr[t];
  m.o1 = a.op_ptr[t + 1];
  m.jp = a.trunk_jpat[t];
  m.jg3 = (int)((reinterpret_cast<const uint32_t*>(a.trunk_jg3)[t >> 2] >> (8 * (t & 3))) & 0xffu);
  m.jlev = (int)((reinterpret_cast<const uint32_t*>(a.trunk_jlev)[t >> 2] >> (8 * (t & 3))) & 0xffu);
  m.src = a.trunk_src[t];
  return m;
}

// Op descriptors of ops ob .. ob + 63, lane x holding op ob + x; lanes past
// the trunk's last op o1 - 1 read that op again (they are never used).  The
// loads are not masked, so nothing waits for them before their first use.
__device__ __forceinline__ uint32_t op_descs(const PlanArgs& a, int64_t ob, int64_t o1, int lane) {
  return a.op_desc[ob + lane < o1 ? ob + lane : o1 - 1];
}

// Trunks t_begin + blk, t_begin + blk + nblk, ... of [t_begin, t_end).  The
// loads a chain needs are issued early: the trunk's descriptors, first ops
// and anchor state (before the gate set is staged, for the workgroup's first
// trunk), and each batch's successor before the batch's chain.
template <int D>
__device__ __forceinline__ void trunk_fwd_body(const PlanArgs& a, int64_t t_begin, int64_t t_end, int64_t blk,
                                               int64_t nblk) {
  extern __shared__ double lds_raw[];
  const int K = a.K;
  const Lds s = carve_trunk(lds_raw, K);
  const int lane = threadIdx.x & 63, i = lane & 15;
  int64_t t = t_begin + blk;
  TrunkMeta m{};
  // the trunk's first ops and its anchor state (a deeper trunk's, or rho:
  // rho's address stands in for the load when there is none)
  uint32_t dl = 0u;
  double fa = 0.0;
  auto first_ops = [&]() {
    if (m.o1 > m.o0) dl = op_descs(a, m.o0, m.o1, lane);
    fa = (m.anchor >= 0 ? a.FA + (1 + m.anchor) * D : a.rho)[i < D ? i : 0];
  };
  if (t < t_end) {
    m = trunk_meta(a, t);
    first_ops();
  }
  stage_gateset<D, 64, STAGE_G>(s, a.G, a.E, a.rho, K, a.M);
  if (blk == 0 && lane < D) a.FA[lane] = a.rho[lane];
  double* js = lds_raw + trunk_jump_doubles(K);
  const bool st = (D == 16) || lane < D;  // rows 1..3 store the same values as row 0
  for (; t < t_end; t += nblk) {
    if (t != t_begin + blk) {
      m = trunk_meta(a, t);
      first_ops();
    }
    const int64_t o0 = m.o0, o1 = m.o1;
    const uint32_t jp = (uint32_t)__builtin_amdgcn_readfirstlane((int)m.jp);
    if (jp != 0u) {
      build_jumps(js, s.Gs, jp, (uint8_t)m.jg3, m.jlev, false, lane);
      // the transposes for the reverse sweep (element (r, c) of slot e is
      // element (c, r) of the forward matrix); lane (i, q) writes rows 4v + q
      double* jt = a.jump_t + (size_t)t * a.jump_levels * 256;
      for (int e = 0; e < m.jlev; ++e)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = 4 * v + (lane >> 4);
          jt[e * 256 + r * 16 + i] = js[e * GATE_STRIDE + i * ROW + r];
        }
    }
    double f = m.anchor >= 0 ? (i < D ? fa : 0.0) : s.rho[i];
    double* out = a.FA + (1 + m.beg) * D + i;  // state after trunk step j: out[j*D]
    int64_t pos = 0;                           // steps done
    for (int64_t ob = o0; ob < o1; ob += OPW) {
      const int n = (int)(o1 - ob < OPW ? o1 - ob : OPW);
      const uint32_t dc = dl;
      if (ob + OPW < o1) dl = op_descs(a, ob + OPW, o1, lane);  // the next batch, during this chain
      // three ops per iteration, the rows of the next two ops in flight
      auto rows = [&](int x) { return load_row(op_row(s.Gs, js, lane_u32(dc, x < n ? x : n - 1), i)); };
      auto step = [&](const Row16& R, int x) {
        f = dot16(f, R);
        pos += (lane_u32(dc, x) >> 8) & 0xffu;
        if (st) out[(pos - 1) * D] = f;
      };
      Row16 R0 = rows(0), R1 = rows(1);
      int x = 0;
      for (; x + 3 <= n; x += 3) {
        const Row16 R2 = rows(x + 2);
        step(R0, x);
        R0 = rows(x + 3);
        step(R1, x + 1);
        R1 = rows(x + 4);
        step(R2, x + 2);
      }
      if (x < n) step(R0, x);
      if (x + 1 < n) step(R1, x + 1);
    }
  }
}

template <int D>
__global__ __launch_bounds__(64) void trunk_fwd_kernel(const PlanArgs a) {
  trunk_fwd_body<D>(a, a.t_begin, a.t_end, blockIdx.x, gridDim.x);
}

// ---------------------------------------------------------------------------
// items: one sequence per team, from its anchor state
// ---------------------------------------------------------------------------
// A team's fill task: its descriptors (loaded first, with a clamped index)
// and the stored value it starts from (loaded once they are in).
struct FillTask {
  int64_t first, in;
  int n, g3;
  uint32_t pat;
  double v;
};
__device__ __forceinline__ FillTask fill_task_desc(const PlanArgs& a, int64_t grp, int team) {
  FillTask t;
  const int64_t q = grp * TPW + team, qc = q < a.n_fill ? q : a.n_fill - 1;
  t.first = a.fill_first[qc];
  t.in = a.fill_in[qc];
  t.n = a.fill_n[qc];
  t.pat = a.fill_pattern[qc];
  t.g3 = a.fill_gate3[qc];
  t.v = 0.0;
  return t;
}
template <int D, bool REV>
__device__ __forceinline__ void fill_task_start(const PlanArgs& a, FillTask& t, int i) {
  const int c = i < D ? i : 0;
  t.v = REV ? a.BA[(t.first + t.n - 1) * D + c] : a.FA[t.in * D + c];
}

template <int D, bool REV>
__device__ void run_fills(const PlanArgs& a, const Lds& s, int64_t blk, int64_t n_blk, FillTask t0);

// Workgroups from a.item_blocks on run the forward fill tasks instead (they
// need only the trunk states, like the items).
// Workgroup blk of nblk: the first a.item_blocks take items, the rest fill tasks.
template <int D>
__device__ __forceinline__ void item_body(const PlanArgs& a, int64_t blk, int64_t nblk) {
  extern __shared__ double lds_raw[];
  const int K = a.K, M = a.M;
  const Lds s = carve(lds_raw, K);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, i = lane & 15, team = lane >> 4;
  const int64_t n_chunks = (a.n_items + kItemChunk - 1) / kItemChunk;
  // A chunk's item-indexed data (descriptor fields, counts, the first gates
  // of each word) is loaded into registers with clamped indices, nothing
  // waiting for it until it is stored to LDS: the first chunk's before the
  // gate set is staged, each next chunk's while the current one runs.
  int64_t dq = 0;
  int32_t nq[2] = {0, 0};
  uint32_t kq[2] = {0u, 0u};
  auto load_q = [&](int64_t chunk) {
    const int64_t q0 = chunk * kItemChunk, ql = a.n_items - 1;
    if (tid < kItemChunk * IST_DESC) {
      const int it = tid / IST_DESC, c = tid % IST_DESC;
      const int64_t q = q0 + it < ql ? q0 + it : ql;
      dq = c < 4 ? a.items[4 * q + c] : (c == 4 ? a.item_step_ptr[q] : (int64_t)a.item_src[q]);
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int x = tid + WAVES * 64 * u, it = x >> 4, c = x & 15;
      const int64_t q = q0 + it < ql ? q0 + it : ql;
      if (a.item_cnt) nq[u] = a.item_cnt[q * M + (c < M ? c : M - 1)];
      kq[u] = a.item_kv[q * 16 + c];
    }
  };
  FillTask t0{};
  if ((int)blk < a.item_blocks && blk < n_chunks) load_q(blk);
  if ((int)blk >= a.item_blocks && a.n_fill > 0) t0 = fill_task_desc(a, (blk - a.item_blocks) * WAVES + wave, team);
  stage_gateset<D>(s, a.G, a.E, a.rho, K, M);
  if ((int)blk >= a.item_blocks) {
    run_fills<D, false>(a, s, blk - a.item_blocks, nblk - a.item_blocks, t0);
    return;
  }
  const bool grad = a.want_grad != 0;
  const bool need_head = a.mode == MODE_LOGLIK || grad;
  double* red = lds_raw + trunk_head_doubles(K);
  const int hw = head_stride(M);
  double obj = 0.0, drho = 0.0;
  double dE[16];
#pragma unroll
  for (int m = 0; m < 16; ++m) dE[m] = 0.0;
  unsigned nonpos = 0;
  // The items are cut into chunks of kItemChunk (two rounds of one item per
  // team), each with its own head row, whatever the number of workgroups:
  // workgroup blk takes chunks blk, blk + item_blocks, ...  A chunk's item
  // data is staged in LDS by the whole workgroup first (the item-indexed
  // data, then the start states its descriptors point to), so that an item's
  // chain starts from LDS instead of from dependent global round trips of its
  // own.
  static_assert(kItemChunk == 2 * WAVES * TPW, "an item chunk is two rounds of the workgroup's teams");
  int64_t* st_desc = reinterpret_cast<int64_t*>(red + (size_t)WAVES * TPW * hw);  // [kItemChunk][IST_DESC]
  double* st_f = reinterpret_cast<double*>(st_desc + kItemChunk * IST_DESC);      // [kItemChunk][16]
  int32_t* st_n = reinterpret_cast<int32_t*>(st_f + kItemChunk * 16);             // [kItemChunk][16]
  int32_t* st_kv = st_n + kItemChunk * 16;                                        // [kItemChunk][16]
  for (int64_t chunk = blk; chunk < n_chunks; chunk += a.item_blocks) {
    const int64_t q0 = chunk * kItemChunk;
    // the item-indexed data (the previous chunk's staged data has been read:
    // write_head ends with a barrier, and so does the staging below)
    if (tid < kItemChunk * IST_DESC) {
      const int it = tid / IST_DESC, c = tid % IST_DESC;
      st_desc[tid] = q0 + it < a.n_items ? dq : ((c == 3 || c == 5) ? -1 : 0);
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int x = tid + WAVES * 64 * u, it = x >> 4, c = x & 15;
      const bool has_it = q0 + it < a.n_items;
      st_n[x] = (a.mode == MODE_LOGLIK && a.item_cnt && has_it && c < M) ? nq[u] : 0;
      st_kv[x] = has_it ? (int)kq[u] : 0;
    }
    lds_sync();
    // start states: item `it`, component `c`
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int x = tid + WAVES * 64 * u, it = x >> 4, c = x & 15;
      const int64_t anc = st_desc[it * IST_DESC + 3];
      st_f[x] = anc >= 0 ? load_state(a.FA, 1 + anc, D, c) : s.rho[c];
    }
    if (chunk + a.item_blocks < n_chunks) load_q(chunk + a.item_blocks);
    lds_sync();
    for (int r = 0; r < 2; ++r) {
    const int it = r * (WAVES * TPW) + wave * TPW + team;
    const int64_t q = q0 + it;
    const bool has = q < a.n_items;
    const int64_t seq = st_desc[it * IST_DESC + 0], beg = st_desc[it * IST_DESC + 1];
    const int64_t end = st_desc[it * IST_DESC + 2], anc = st_desc[it * IST_DESC + 3];
    const int64_t isp = st_desc[it * IST_DESC + 4], zrow = st_desc[it * IST_DESC + 5];
    const int32_t Nq = st_n[it * 16 + i];
    const int L = (int)(end - beg);
    const int Lw = wave_max4(L);
    const uint8_t* word = a.gates + beg;
    double* fa = a.FA + (1 + a.nTS + isp) * D;  // state before item step x: fa[x*D + i]
    double* ba = a.BA + (a.nTS + isp) * D;      // adjoint after item step x
    double f = st_f[it * 16 + i];
    const int kv0 = st_kv[it * 16 + i];

    // ---- forward over the rest of the word ----
    for (int t0 = 0; t0 < Lw; t0 += 16) {
      const int kv = t0 == 0 ? kv0 : ((t0 + i < L) ? (int)word[t0 + i] : 0);
#define GST_IF(R)                                                        \
  if (t0 + R < Lw) {                                                     \
    const int x = t0 + R;                                                \
    const int k = bcast_i32<R>(kv);                                      \
    if (grad && x < L && i < D) __builtin_nontemporal_store(f, &fa[(int64_t)x * D + i]);            \
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
        const int32_t N = Nq;
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
    if (grad) {
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
        const int kv = t0 == 0 ? kv0 : ((t0 + i < L) ? (int)word[t0 + i] : 0);
#define GST_IB(R)                                                         \
  if (t0 + R < Lw) {                                                      \
    const int x = t0 + R;                                                 \
    const int k = bcast_i32<R>(kv);                                       \
    if (x < L && i < D) __builtin_nontemporal_store(b, &ba[(int64_t)x * D + i]);                  \
    const double bn = dot16(b, load_row(s.GTs + k * GATE_STRIDE + i * ROW)); \
    b = x < L ? bn : b;                                                   \
  }
        GST_IB(15) GST_IB(14) GST_IB(13) GST_IB(12) GST_IB(11) GST_IB(10) GST_IB(9) GST_IB(8)
        GST_IB(7) GST_IB(6) GST_IB(5) GST_IB(4) GST_IB(3) GST_IB(2) GST_IB(1) GST_IB(0)
#undef GST_IB
      }
      if (has && i < D && zrow >= 0) a.src_adj[zrow * D + i] = b;
      if (has && anc < 0) drho += b;
    }
    }
    if (need_head) {  // the chunk's head row
      write_head<D, true, WAVES>(red, hw, obj, drho, dE, M, a.slab + chunk * slab_width(D, M, 0));
      obj = 0.0;
      drho = 0.0;
#pragma unroll
      for (int m = 0; m < 16; ++m) dE[m] = 0.0;
    } else {
      lds_sync();  // the staged chunk has been read
    }
  }
  if (nonpos) {
    atomicAdd(a.status + 1, (unsigned long long)nonpos);
    if (a.req_nonpos) atomicAdd(a.req_nonpos, (unsigned long long)nonpos);
  }
}

template <int D>
__global__ __launch_bounds__(256) void item_kernel(const PlanArgs a) {
  item_body<D>(a, blockIdx.x, gridDim.x);
}

// ---------------------------------------------------------------------------
// trunk reverse sweep, one trunk per workgroup of a single wave: ops in
// reverse with the transposed rows; the adjoints injected at stored states
// (64 ops at a time, staged in LDS) are added on the way back
// ---------------------------------------------------------------------------
// Trunks t_begin + blk, ... as in the forward; workgroup blk writes head row
// blk of `slab`.  Batches of 64 ops run from the trunk's end; the loads are
// issued ahead: the trunk's descriptors and the ops of its first two batches
// (before the gate set is staged, for the workgroup's first trunk), the first
// batch's injected vectors before the jump matrices are built, and during the
// chain of batch k the vectors of batch k + 1 and the ops of batch k + 2.
template <int D>
__device__ __forceinline__ void trunk_bwd_body(const PlanArgs& a, int64_t t_begin, int64_t t_end, int64_t blk,
                                               int64_t nblk, double* slab) {
  extern __shared__ double lds_raw[];
  const int K = a.K;
  const Lds s = carve_trunk(lds_raw, K);
  const int lane = threadIdx.x & 63, i = lane & 15;
  int64_t t = t_begin + blk;
  TrunkMeta m{};
  // batch k of the trunk: ops max(o0, o1 - 64 (k + 1)) .. o1 - 64 k - 1
  auto batch_ob = [&](int64_t oe) { return oe - OPW > m.o0 ? oe - OPW : m.o0; };
  auto slots = [&](int64_t ob, int64_t oe) { return a.op_slot[ob + lane < oe ? ob + lane : oe - 1]; };
  // the ops of the trunk's first two batches
  uint32_t dl = 0u, dl1 = 0u;
  int32_t sl = -1, sl1 = -1;
  auto first_ops = [&]() {
    const int64_t ob = batch_ob(m.o1);
    if (m.o1 > m.o0) {
      dl = op_descs(a, ob, m.o1, lane);
      sl = slots(ob, m.o1);
    }
    if (ob > m.o0) {
      dl1 = op_descs(a, batch_ob(ob), ob, lane);
      sl1 = slots(batch_ob(ob), ob);
    }
  };
  // the forward sweep's transposed jump matrices of the trunk (at most five
  // levels), lane (i, q) holding rows 4v + q
  double jtv[5][4];
  auto load_jt = [&](const TrunkMeta& mm, int64_t tt) {
    const double* jt = a.jump_t + (size_t)tt * a.jump_levels * 256;
#pragma unroll
    for (int e = 0; e < 5; ++e)
#pragma unroll
      for (int v = 0; v < 4; ++v) jtv[e][v] = jt[(e < mm.jlev ? e : 0) * 256 + (4 * v + (lane >> 4)) * 16 + i];
  };
  if (t < t_end) {
    m = trunk_meta(a, t);
    first_ops();
    if (m.jp != 0u) load_jt(m, t);
  }
  stage_gateset<D, 64, STAGE_GT>(s, a.G, a.E, a.rho, K, a.M);
  double* inj_st = lds_raw + trunk_inj_doubles(K);
  double* js = lds_raw + trunk_jump_doubles(K);
  const bool st = (D == 16) || lane < D;
  double drho = 0.0;
  for (; t < t_end; t += nblk) {
    if (t != t_begin + blk) {
      m = trunk_meta(a, t);
      first_ops();
    }
    const int64_t o0 = m.o0, o1 = m.o1;
    // the injected vector of the op at lane x of a batch, read whole by that
    // lane (its slot is the lane's own), unmasked: `use` says whether the op
    // receives one
    auto inj_load = [&](int64_t ob, int64_t oe, int32_t sl, d2 (&v)[D / 2], bool& use) {
      use = lane < oe - ob && sl >= 0;
      const d2* src = reinterpret_cast<const d2*>(a.inj + (use ? (int64_t)sl * D : 0));
#pragma unroll
      for (int c = 0; c < D / 2; ++c) v[c] = src[c];
    };
    int64_t oe = o1, ob = batch_ob(oe);
    // the first batch's vectors load while the jump matrices are built
    d2 v[D / 2];
    bool use = false;
    if (oe > o0) inj_load(ob, oe, sl, v, use);
    const uint32_t jp = (uint32_t)__builtin_amdgcn_readfirstlane((int)m.jp);
    if (jp != 0u) {  // the forward sweep's jump matrices, transposed, into the slots
      if (t != t_begin + blk) load_jt(m, t);
      for (int e = 0; e < m.jlev; ++e)
#pragma unroll
        for (int v = 0; v < 4; ++v) js[e * GATE_STRIDE + (4 * v + (lane >> 4)) * ROW + i] = jtv[e < 5 ? e : 0][v];
      wave_sync();
    }
    double* ba = a.BA + m.beg * D + i;  // adjoint after trunk step j: ba[j*D]
    int64_t pos = m.end - m.beg;
    double b = 0.0;
    for (; oe > o0; oe = ob, ob = batch_ob(ob)) {
      const int n = (int)(oe - ob);
      wave_sync();  // the previous batch's vectors have been read
      d2* row = reinterpret_cast<d2*>(inj_st + lane * 16);  // row x of op x
#pragma unroll
      for (int c = 0; c < 8; ++c) row[c] = (use && c < D / 2) ? v[c < D / 2 ? c : 0] : d2{0.0, 0.0};
      wave_sync();
      // ahead: the next batch's vectors, the ops of the one after
      const uint32_t dc = dl;
      if (ob > o0) {
        const int64_t ob1 = batch_ob(ob);
        inj_load(ob1, ob, sl1, v, use);
        dl = dl1;
        if (ob1 > o0) {
          dl1 = op_descs(a, batch_ob(ob1), ob1, lane);
          sl1 = slots(batch_ob(ob1), ob1);
        }
      }
      // three ops per iteration (descending), the rows of the next two in flight
      auto rows = [&](int x) { return load_row(op_row(s.GTs, js, lane_u32(dc, x >= 0 ? x : 0), i)); };
      auto step = [&](const Row16& R, int x) {
        b += inj_st[x * 16 + i];
        if (st) ba[(pos - 1) * D] = b;
        b = dot16(b, R);
        pos -= (lane_u32(dc, x) >> 8) & 0xffu;
      };
      Row16 R0 = rows(n - 1), R1 = rows(n - 2);
      int x = n - 1;
      for (; x >= 2; x -= 3) {
        const Row16 R2 = rows(x - 2);
        step(R0, x);
        R0 = rows(x - 3);
        step(R1, x - 1);
        R1 = rows(x - 4);
        step(R2, x - 2);
      }
      if (x >= 0) step(R0, x);
      if (x >= 1) step(R1, x - 1);
    }
    if (lane < D && m.src >= 0) a.src_adj[(int64_t)m.src * D + i] = b;
    if (m.anchor < 0) drho += b;
  }
  // lanes 16..63 repeat lanes 0..15: only row 0 contributes
  if (lane >= 16) drho = 0.0;
  const double no_dE[16] = {};
  write_head<D, false, 1>(lds_raw, head_stride(0), 0.0, drho, no_dE, a.M, slab + blk * slab_width(D, a.M, 0));
}

template <int D>
__global__ __launch_bounds__(64) void trunk_bwd_kernel(const PlanArgs a) {
  trunk_bwd_body<D>(a, a.t_begin, a.t_end, blockIdx.x, gridDim.x, a.slab);
}

// ---------------------------------------------------------------------------
// fill tasks: the states (forward) or adjoints (reverse) inside one jump, one
// task per 16-lane team, from the stored value at the jump's start (forward)
// or end (reverse).  Step j of a task applies gate pattern[j % period].
// ---------------------------------------------------------------------------
// Workgroup blk of n_blk runs groups blk * WAVES + wave, + n_blk * WAVES, ...;
// `t0` is the first group's task, its descriptors already loaded.
template <int D, bool REV>
__device__ void run_fills(const PlanArgs& a, const Lds& s, int64_t blk, int64_t n_blk, FillTask t0) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, i = lane & 15, team = lane >> 4;
  const double* gl = (REV ? s.GTs : s.Gs) + i * ROW;
  const int64_t n_groups = (a.n_fill + TPW - 1) / TPW;
  FillTask t = t0;
  for (int64_t grp = blk * WAVES + wave; grp < n_groups; grp += n_blk * WAVES) {
    if (grp != blk * WAVES + wave) t = fill_task_desc(a, grp, team);
    fill_task_start<D, REV>(a, t, i);
    const bool has = grp * TPW + team < a.n_fill;
    const int64_t first = t.first, in = t.in;
    const int n = has ? t.n : 1;
    const uint32_t pat = has ? t.pat : (t.pat & 0xffu);
    const int g3 = t.g3;
    (void)in;
    // the four tasks of a wave share their period (the plan groups them):
    // the pattern rows stay in registers and the phase is uniform
    const int per = __builtin_amdgcn_readfirstlane((int)(pat & 0xffu));
    const int nw = wave_max4(n);
    const bool st = has && i < D;
    const Row16 R0 = load_row(gl + (int)((pat >> 8) & 0xffu) * GATE_STRIDE);
    Row16 R1 = R0, R2 = R0, R3 = R0;
    if (per > 1) R1 = load_row(gl + (int)((pat >> 16) & 0xffu) * GATE_STRIDE);
    if (per > 2) R2 = load_row(gl + (int)((pat >> 24) & 0xffu) * GATE_STRIDE);
    if (per > 3) R3 = load_row(gl + g3 * GATE_STRIDE);
    auto apply = [&](double v, int ph) {
      if (ph == 0) return dot16(v, R0);
      if (ph == 1) return dot16(v, R1);
      if (ph == 2) return dot16(v, R2);
      return dot16(v, R3);
    };
    if (!REV) {
      // states after steps 0 .. n-2 (the one after step n-1 is the jump's);
      // step j applies pattern gate j % per
      double f = i < D ? t.v : 0.0;
      double* o = a.FA + (1 + first) * D + i;
      int ph = 0;
      for (int j = 0; j + 1 < nw; ++j) {
        f = apply(f, ph);
        if (st && j + 1 < n) __builtin_nontemporal_store(f, &o[(int64_t)j * D]);
        ph = ph + 1 == per ? 0 : ph + 1;
      }
    } else {
      // adjoints after steps n-2 .. 0, from the one after step n-1
      double b = st ? t.v : 0.0;
      double* o = a.BA + first * D + i;
      int ph = (nw - 1) % per;
      for (int j = nw - 1; j >= 1; --j) {
        const double nb = apply(b, ph);
        if (j < n) {
          b = nb;
          if (st) __builtin_nontemporal_store(b, &o[(int64_t)(j - 1) * D]);
        }
        ph = ph == 0 ? per - 1 : ph - 1;
      }
    }
  }
}

// reverse fill tasks (the forward ones run in the item kernel's extra workgroups)
template <int D>
__global__ __launch_bounds__(256) void fill_rev_kernel(const PlanArgs a) {
  extern __shared__ double lds_raw[];
  const Lds s = carve(lds_raw, a.K);
  // the first group's descriptors load while the gate set is staged
  const FillTask t0 = fill_task_desc(a, (int64_t)blockIdx.x * WAVES + (threadIdx.x >> 6), (threadIdx.x & 63) >> 4);
  stage_gateset<D, 256, STAGE_GT>(s, a.G, a.E, a.rho, a.K, a.M);
  run_fills<D, true>(a, s, blockIdx.x, gridDim.x, t0);
}

// One wave per injection slot: its sources are consecutive rows of the
// source arena; four groups of 16 lanes take every fourth row, the first
// eight rows of each group loaded at once, and the group sums are combined
// in a fixed order.
__device__ __forceinline__ void inject_body(const InjectLaunch& a, int64_t s_begin, int64_t s_end, int64_t blk,
                                            int64_t nblk) {
  const int D = a.D;
  const int lane = threadIdx.x, g = lane >> 4, i = lane & 15;
  for (int64_t slot = s_begin + blk; slot < s_end; slot += nblk) {
    const int64_t z0 = a.inj_ptr[slot], z1 = a.inj_ptr[slot + 1];
    double t[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int64_t z = z0 + g + 4 * u;
      t[u] = a.src_adj[(z < z1 && i < D) ? z * D + i : 0];
    }
    double v = 0.0;
#pragma unroll
    for (int u = 0; u < 8; ++u) v += (z0 + g + 4 * u < z1 && i < D) ? t[u] : 0.0;
    for (int64_t z = z0 + g + 32; z < z1; z += 4) v += i < D ? a.src_adj[z * D + i] : 0.0;
    v += __shfl_xor(v, 16);
    v += __shfl_xor(v, 32);
    if (lane < D) a.inj[slot * D + i] = v;
  }
}

__global__ __launch_bounds__(64) void inject_kernel(const InjectLaunch a) {
  inject_body(a, a.s_begin, a.s_end, blockIdx.x, gridDim.x);
}

// ---------------------------------------------------------------------------
// gradient GEMM over the stored (adjoint, state) pairs, one chunk of records
// of one gate per workgroup; four records per MFMA 16x16x4
// ---------------------------------------------------------------------------
template <int D>
__device__ __forceinline__ void grad_gemm_body(const GemmLaunch& a, int64_t c) {
  __shared__ double tile[WAVES][256];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, i = lane & 15, z = lane >> 4;
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

template <int D>
__global__ __launch_bounds__(256) void grad_gemm_kernel(const GemmLaunch a) {
  grad_gemm_body<D>(a, blockIdx.x);
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
__device__ __forceinline__ void reduce_stage1_body(const PlanReduce& a, int64_t bx, int g) {
  __shared__ double red[4][64];
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int64_t x = bx * 64 + tx;
  double v = 0.0;
  int G = 0;
  if (x < a.P) {
    const Rows R = rows_of(a, x);
    G = parts_of(R.n);
    const int64_t per = (R.n + G - 1) / G, w0 = g * per, w1 = min(R.n, w0 + per);
    if (g < G)
      for (int64_t w = w0 + ty; w < w1; w += 32) {  // rows w, w+4, ..., eight loads in flight
        double t[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int64_t ww = w + 4 * u;
          const double val = R.src[(ww < w1 ? ww : w1 - 1) * R.stride];
          t[u] = ww < w1 ? val : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) v += t[u];
      }
  }
  red[ty][tx] = v;
  __syncthreads();
  if (ty == 0 && x < a.P && g < G) a.part[(int64_t)g * a.P + x] = (red[0][tx] + red[1][tx]) + (red[2][tx] + red[3][tx]);
}

__global__ __launch_bounds__(256) void plan_reduce_stage1(const PlanReduce a) {
  reduce_stage1_body(a, blockIdx.x, blockIdx.y);
}

// Column x adds its region's stage-1 partials in ascending g.  A +inf
// objective partial marks p <= 0 with N > 0: the objective is then +inf and
// the gradient is not written.
__device__ __forceinline__ void reduce_stage2_body(const PlanReduce& a, int64_t bx) {
  __shared__ double red[4][64];
  __shared__ int nonpos_sh;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int64_t x = bx * 64 + tx;
  double v = 0.0;
  if (x < a.P) {  // partials g = ty, ty+4, ... (at most 16), all loads in flight
    const int G = parts_of(rows_of(a, x).n);
    double t[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int g = ty + 4 * u;
      const double val = a.part[(int64_t)(g < G ? g : 0) * a.P + x];
      t[u] = g < G ? val : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) v += t[u];
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

__global__ __launch_bounds__(256) void plan_reduce_stage2(const PlanReduce a) { reduce_stage2_body(a, blockIdx.x); }

// ---------------------------------------------------------------------------
// Batched forms: the plans of several requests in one launch per kernel.
// Request blockIdx.y takes its launch arguments from a device array (copied to
// registers before anything is stored); its workgroups are blockIdx.x < the
// count of its standalone launch, split the same way (so its results are the
// same bits as alone), and the others exit.  A request without the gradient
// skips the reverse kernels; one with fewer levels skips the extra ones.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int64_t trunk_blocks_of(int64_t n) { return n < 1 ? 1 : (n > 65535 ? 65535 : n); }

template <int D>
__global__ __launch_bounds__(64) void trunk_fwd_batch(const PlanBatch b, int level) {
  const PlanArgs a = b.args[blockIdx.y];
  if (level >= a.n_levels) return;
  const int64_t t0 = a.lvl_trunk[level], t1 = a.lvl_trunk[level + 1];
  const int64_t n = trunk_blocks_of(t1 - t0);
  if ((int64_t)blockIdx.x >= n) return;
  trunk_fwd_body<D>(a, t0, t1, blockIdx.x, n);
}

template <int D>
__global__ __launch_bounds__(256) void item_batch(const PlanBatch b) {
  const PlanArgs a = b.args[blockIdx.y];
  const int64_t n = (int64_t)a.item_blocks + a.fill_blocks;
  if ((int64_t)blockIdx.x >= n) return;
  item_body<D>(a, blockIdx.x, n);
}

template <int D>
__global__ __launch_bounds__(64) void trunk_bwd_batch(const PlanBatch b, int level) {
  const PlanArgs a = b.args[blockIdx.y];
  if (!a.want_grad || level >= a.n_levels) return;
  const int64_t t0 = a.lvl_trunk[level], t1 = a.lvl_trunk[level + 1];
  const int64_t n = trunk_blocks_of(t1 - t0);
  if ((int64_t)blockIdx.x >= n) return;
  trunk_bwd_body<D>(a, t0, t1, blockIdx.x, n, a.slab + a.lvl_head[level] * slab_width(D, a.M, 0));
}

__global__ __launch_bounds__(64) void inject_batch(const PlanBatch b, int level) {
  const InjectLaunch in = b.inject[blockIdx.y];
  if (level >= in.n_levels) return;
  const int64_t s0 = in.lvl_inj[level], s1 = in.lvl_inj[level + 1];
  const int64_t n = s1 - s0 < 65536 ? s1 - s0 : 65536;
  if ((int64_t)blockIdx.x >= n) return;
  inject_body(in, s0, s1, blockIdx.x, n);
}

template <int D>
__global__ __launch_bounds__(256) void fill_rev_batch(const PlanBatch b) {
  const PlanArgs a = b.args[blockIdx.y];
  if (!a.want_grad || a.n_fill <= 0 || (int64_t)blockIdx.x >= a.fill_blocks) return;
  extern __shared__ double lds_raw[];
  const Lds s = carve(lds_raw, a.K);
  const FillTask t0 = fill_task_desc(a, (int64_t)blockIdx.x * WAVES + (threadIdx.x >> 6), (threadIdx.x & 63) >> 4);
  stage_gateset<D, 256, STAGE_GT>(s, a.G, a.E, a.rho, a.K, a.M);
  run_fills<D, true>(a, s, blockIdx.x, a.fill_blocks, t0);
}

template <int D>
__global__ __launch_bounds__(256) void grad_gemm_batch(const PlanBatch b) {
  const GemmLaunch g = b.gemm[blockIdx.y];
  if ((int64_t)blockIdx.x >= g.n_chunks) return;
  grad_gemm_body<D>(g, blockIdx.x);
}

__global__ __launch_bounds__(256) void reduce_stage1_batch(const PlanBatch b) {
  const PlanReduce& r = b.reduce[blockIdx.z];  // chunk_ptr is indexed at run time: no register copy
  if (r.P <= 0 || (int64_t)blockIdx.x * 64 >= r.P || (int)blockIdx.y >= r.n_part) return;
  reduce_stage1_body(r, blockIdx.x, blockIdx.y);
}

__global__ __launch_bounds__(256) void reduce_stage2_batch(const PlanBatch b) {
  const PlanReduce& r = b.reduce[blockIdx.z];  // chunk_ptr is indexed at run time: no register copy
  if (r.P <= 0 || (int64_t)blockIdx.x * 64 >= r.P) return;
  reduce_stage2_body(r, blockIdx.x);
}

}  // namespace

int fill_blocks_for(int64_t n_fill) {
  const int64_t b = (n_fill + WAVES * TPW - 1) / (WAVES * TPW);
  return (int)(b < 1 ? 1 : (b > 1024 ? 1024 : b));
}

int item_blocks_per_cu(int D, int K, int M) {
  int n = 0;
  const size_t bytes = item_lds_bytes(K, M);
  const hipError_t e = D == 16 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, item_kernel<16>, 256, bytes)
                               : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, item_kernel<4>, 256, bytes);
  return (e == hipSuccess && n > 0) ? n : 1;
}

int item_blocks_for(int64_t n_items, int64_t max_blocks) {
  int64_t b = (n_items + kItemChunk - 1) / kItemChunk;
  if (b < 1) b = 1;
  if (max_blocks > 0 && b > max_blocks) b = max_blocks;  // the workgroups then take several chunks each
  return (int)b;
}

int trunk_blocks_for(int64_t n) {
  return (int)(n < 1 ? 1 : (n > 65535 ? 65535 : n));  // one single-wave workgroup per trunk
}

hipError_t launch_trunk_fwd(const PlanArgs& a, hipStream_t stream) {
  const int blocks = trunk_blocks_for(a.t_end - a.t_begin);
  const size_t bytes = trunk_lds_bytes(a.K, a.jump_levels);
  if (a.D == 16)
    gst_launch(trunk_fwd_kernel<16>, dim3(blocks), dim3(64), bytes, stream, a);
  else if (a.D == 4)
    gst_launch(trunk_fwd_kernel<4>, dim3(blocks), dim3(64), bytes, stream, a);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_trunk_bwd(const PlanArgs& a, hipStream_t stream) {
  const int blocks = trunk_blocks_for(a.t_end - a.t_begin);
  const size_t bytes = trunk_lds_bytes(a.K, a.jump_levels);
  if (a.D == 16)
    gst_launch(trunk_bwd_kernel<16>, dim3(blocks), dim3(64), bytes, stream, a);
  else if (a.D == 4)
    gst_launch(trunk_bwd_kernel<4>, dim3(blocks), dim3(64), bytes, stream, a);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_items(const PlanArgs& a, int n_blocks, hipStream_t stream) {
  if (a.item_blocks != n_blocks) return hipErrorInvalidValue;
  const size_t bytes = item_lds_bytes(a.K, a.M);
  const unsigned grid = (unsigned)n_blocks + (a.want_grad && a.n_fill > 0 ? (unsigned)fill_blocks_for(a.n_fill) : 0u);
  if (a.D == 16)
    gst_launch(item_kernel<16>, dim3(grid), dim3(256), bytes, stream, a);
  else if (a.D == 4)
    gst_launch(item_kernel<4>, dim3(grid), dim3(256), bytes, stream, a);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_inject(const InjectLaunch& a, hipStream_t stream) {
  const int64_t n = a.s_end - a.s_begin;
  if (n <= 0) return hipSuccess;
  const int blocks = (int)(n < 65536 ? n : 65536);
  gst_launch(inject_kernel, dim3(blocks), dim3(64), 0, stream, a);
  return hipGetLastError();
}

hipError_t launch_fill_rev(const PlanArgs& a, hipStream_t stream) {
  if (a.n_fill <= 0) return hipSuccess;
  const int blocks = fill_blocks_for(a.n_fill);
  const size_t bytes = item_lds_bytes(a.K, a.M);
  if (a.D == 16)
    gst_launch(fill_rev_kernel<16>, dim3((unsigned)blocks), dim3(256), bytes, stream, a);
  else if (a.D == 4)
    gst_launch(fill_rev_kernel<4>, dim3((unsigned)blocks), dim3(256), bytes, stream, a);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_reduce_plan(const PlanReduce& a, hipStream_t stream) {
  if (a.P <= 0 || a.n_part < 1 || a.n_part > 64 || a.K < 0 || a.K > 8) return hipErrorInvalidValue;
  const unsigned xb = (unsigned)((a.P + 63) / 64);
  gst_launch(plan_reduce_stage1, dim3(xb, (unsigned)a.n_part), dim3(256), 0, stream, a);
  gst_launch(plan_reduce_stage2, dim3(xb), dim3(256), 0, stream, a);
  return hipGetLastError();
}

hipError_t launch_grad_gemm(const GemmLaunch& a, hipStream_t stream) {
  if (a.n_chunks <= 0) return hipSuccess;
  if (a.D == 16)
    gst_launch(grad_gemm_kernel<16>, dim3((unsigned)a.n_chunks), dim3(256), 0, stream, a);
  else if (a.D == 4)
    gst_launch(grad_gemm_kernel<4>, dim3((unsigned)a.n_chunks), dim3(256), 0, stream, a);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

#define GST_BATCH_D(kern, ...)                                             \
  do {                                                                     \
    if (D == 16)                                                           \
      gst_launch(kern<16>, __VA_ARGS__);                                   \
    else if (D == 4)                                                       \
      gst_launch(kern<4>, __VA_ARGS__);                                    \
    else                                                                   \
      return hipErrorInvalidValue;                                         \
  } while (0)

hipError_t launch_trunk_fwd_batch(const PlanBatch& b, int D, int n, int level, int grid_x, int K_max, int jl_max,
                                  hipStream_t stream) {
  if (n <= 0 || grid_x <= 0) return hipSuccess;
  GST_BATCH_D(trunk_fwd_batch, dim3((unsigned)grid_x, (unsigned)n), dim3(64), trunk_lds_bytes(K_max, jl_max), stream,
              b, level);
  return hipGetLastError();
}

hipError_t launch_items_batch(const PlanBatch& b, int D, int n, int grid_x, int K_max, int M_max,
                              hipStream_t stream) {
  if (n <= 0 || grid_x <= 0) return hipSuccess;
  GST_BATCH_D(item_batch, dim3((unsigned)grid_x, (unsigned)n), dim3(256), item_lds_bytes(K_max, M_max), stream, b);
  return hipGetLastError();
}

hipError_t launch_inject_batch(const PlanBatch& b, int n, int level, int grid_x, hipStream_t stream) {
  if (n <= 0 || grid_x <= 0) return hipSuccess;
  gst_launch(inject_batch, dim3((unsigned)grid_x, (unsigned)n), dim3(64), 0, stream, b, level);
  return hipGetLastError();
}

hipError_t launch_trunk_bwd_batch(const PlanBatch& b, int D, int n, int level, int grid_x, int K_max, int jl_max,
                                  hipStream_t stream) {
  if (n <= 0 || grid_x <= 0) return hipSuccess;
  GST_BATCH_D(trunk_bwd_batch, dim3((unsigned)grid_x, (unsigned)n), dim3(64), trunk_lds_bytes(K_max, jl_max), stream,
              b, level);
  return hipGetLastError();
}

hipError_t launch_fill_rev_batch(const PlanBatch& b, int D, int n, int grid_x, int K_max, int M_max,
                                 hipStream_t stream) {
  if (n <= 0 || grid_x <= 0) return hipSuccess;
  GST_BATCH_D(fill_rev_batch, dim3((unsigned)grid_x, (unsigned)n), dim3(256), item_lds_bytes(K_max, M_max), stream,
              b);
  return hipGetLastError();
}

hipError_t launch_grad_gemm_batch(const PlanBatch& b, int D, int n, int grid_x, hipStream_t stream) {
  if (n <= 0 || grid_x <= 0) return hipSuccess;
  GST_BATCH_D(grad_gemm_batch, dim3((unsigned)grid_x, (unsigned)n), dim3(256), 0, stream, b);
  return hipGetLastError();
}

hipError_t launch_reduce_plan_batch(const PlanBatch& b, int n, int grid_x, int parts, hipStream_t stream) {
  if (n <= 0 || grid_x <= 0) return hipSuccess;
  if (parts < 1 || parts > 64) return hipErrorInvalidValue;
  gst_launch(reduce_stage1_batch, dim3((unsigned)grid_x, (unsigned)parts, (unsigned)n), dim3(256), 0, stream, b);
  gst_launch(reduce_stage2_batch, dim3((unsigned)grid_x, 1u, (unsigned)n), dim3(256), 0, stream, b);
  return hipGetLastError();
}

#undef GST_BATCH_D

}  // namespace gst
