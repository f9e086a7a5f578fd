// Kernels for one- and two-qubit gate sets (D = 4 or 16).
//
// Thesis Sec. 6.3.1: p[s][m] = e_m^T G[s_L] ... G[s_1] rho, the multinomial
// log-likelihood of the counts and its gradient (chain rule of the product).
//
// Layout on the chip
//   * A team of 16 lanes (one DPP row) owns one chain; lane i holds component
//     i of the current state (rows i >= D are zero padding for one qubit).
//     A wave runs four chains, a workgroup of four waves sixteen.
//   * The gate set lives in LDS twice: G (rows) for the forward product and
//     G^T (rows = columns of G) for the adjoint, rows padded to 18 doubles so
//     that the 16-byte reads of a team hit distinct banks.
//   * One step of a forward chain is, in lane i, 16 fused multiply-adds
//     acc = fma(G[k][i][j], f[j], acc), j ascending from acc = 0, with f[j]
//     broadcast from lane j of the row by DPP row_newbcast inside
//     v_fmac_f64.  This is the order of the plain definition of the product,
//     so states and probabilities are bit-identical to a sequential loop.
//   * Reverse sweeps run b <- G^T b and stash the pairs (b_t, f_{t-1}) with
//     their gate index in the wave's LDS stash.  After every segment of C
//     steps the wave accumulates dG_k += sum b_t f_{t-1}^T with FP64 MFMA
//     16x16x4 tiles (one tile per gate, in registers); steps are grouped by
//     gate so every MFMA is a rank-4 update of one gate.
//   * Each workgroup writes one slab of partial results; a last kernel adds
//     the slabs in ascending order (deterministic).
//
// Kernels
//   leaf_kernel      one sequence per team: forward chain, readout, objective,
//                    seeds, reverse sweep (segments recomputed from
//                    checkpoints in HBM), dG through the LDS stash
//   reduce_kernel    sums the slabs
// (the kernels of the shared-prefix plan are in gst_plan_kernels.hip)
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "gst_device.h"
#include "gst_internal.h"

namespace gst {
namespace {

struct Item {
  int64_t seq, beg, end, anchor;
};

__device__ __forceinline__ Item load_item(const LeafLaunch& a, int64_t q) {
  Item it;
  if (a.items) {
    const int64_t* p = a.items + 4 * q;
    it.seq = p[0];
    it.beg = p[1];
    it.end = p[2];
    it.anchor = p[3];
  } else {
    it.seq = q;
    it.beg = a.off[q];
    it.end = a.off[q + 1];
    it.anchor = -1;
  }
  return it;
}

// ---------------------------------------------------------------------------
// leaf kernel: one work item (sequence) per 16-lane team
// ---------------------------------------------------------------------------
template <int D>
__global__ __launch_bounds__(256) void leaf_kernel(const LeafLaunch a) {
  extern __shared__ double lds_raw[];
  const int K = a.K, M = a.M;
  const Lds s = carve(lds_raw, K);
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int i = lane & 15;
  const int team = lane >> 4;
  stage_gateset<D>(s, a.G, a.E, a.rho, K, M);

  double* st_b = s.stash + (size_t)wave * 2 * ENT * 16;
  double* st_f = st_b + ENT * 16;
  uint8_t* st_k = s.sk + wave * ENT;

  const bool grad = a.want_grad != 0;
  const int64_t gteam = ((int64_t)blockIdx.x * WAVES + wave) * TPW + team;
  double* ck = a.ckpt ? a.ckpt + gteam * a.ckpt_per_team : nullptr;

  d4 acc[KMAX];
#pragma unroll
  for (int k = 0; k < KMAX; ++k) acc[k] = d4{0.0, 0.0, 0.0, 0.0};
  double obj = 0.0, drho = 0.0;
  double dE[16];
#pragma unroll
  for (int m = 0; m < 16; ++m) dE[m] = 0.0;
  unsigned bad = 0, nonpos = 0;

  const int64_t n_groups = (a.n_items + TPW - 1) / TPW;
  const int64_t wave_id = (int64_t)blockIdx.x * WAVES + wave;
  const int64_t n_waves = (int64_t)gridDim.x * WAVES;

  for (int64_t grp = wave_id; grp < n_groups; grp += n_waves) {
    const int64_t q = grp * TPW + team;
    const bool has = q < a.n_items;
    const Item it = has ? load_item(a, q) : Item{0, 0, 0, -1};
    const int L = (int)(it.end - it.beg);
    int Lw = L;
    Lw = max(Lw, __shfl_xor(Lw, 16));
    Lw = max(Lw, __shfl_xor(Lw, 32));
    const uint8_t* word = a.gates + it.beg;

    double f;
    if (it.anchor >= 0)
      f = i < D ? a.anchor_states[it.anchor * D + i] : 0.0;
    else
      f = s.rho[i];

    // ---- forward chain (checkpoint every C steps); gate indices are
    // loaded one chunk of 16 steps ahead ----
    int kv_next = i < L ? (int)word[i] : 0;
    for (int t0 = 0; t0 < Lw; t0 += 16) {
      int kv = kv_next;
      kv_next = t0 + 16 + i < L ? (int)word[t0 + 16 + i] : 0;
      if (t0 + i < L && kv >= K) {
        ++bad;
        kv = 0;
      }
#define GST_FWD_STEP(R)                                        \
  if (t0 + R < Lw) {                                           \
    const int t = t0 + R;                                      \
    const int k = bcast_i32<R>(kv);                            \
    if (grad && (R % C) == 0 && t < L) ck[(t / C) * 16 + i] = f; \
    const double fn = dot16_bcast(f, grow(s, k, i));           \
    f = t < L ? fn : f;                                        \
  }
      GST_FWD_STEP(0) GST_FWD_STEP(1) GST_FWD_STEP(2) GST_FWD_STEP(3)
      GST_FWD_STEP(4) GST_FWD_STEP(5) GST_FWD_STEP(6) GST_FWD_STEP(7)
      GST_FWD_STEP(8) GST_FWD_STEP(9) GST_FWD_STEP(10) GST_FWD_STEP(11)
      GST_FWD_STEP(12) GST_FWD_STEP(13) GST_FWD_STEP(14) GST_FWD_STEP(15)
#undef GST_FWD_STEP
    }

    // ---- readout: lane m < M holds p_m ----
    const double p = dot16_bcast(f, reinterpret_cast<const double2*>(s.Es + i * ROW));
    double dp = 0.0;
    if (has && i < M) {
      const int64_t o = it.seq * M + i;
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

    // ---- SPAM adjoints: dE[m] += dp_m f ; seed b = sum_m dp_m e_m ----
#define GST_DE(R) \
  if (R < M) dE[R] = fma(bcast_f64<R>(dp), f, dE[R]);
    GST_DE(0) GST_DE(1) GST_DE(2) GST_DE(3) GST_DE(4) GST_DE(5) GST_DE(6) GST_DE(7)
    GST_DE(8) GST_DE(9) GST_DE(10) GST_DE(11) GST_DE(12) GST_DE(13) GST_DE(14) GST_DE(15)
#undef GST_DE
    // ---- reverse sweep, one segment of C steps at a time ----
    // (a segment's gate indices and checkpoint are loaded one segment ahead)
    const int nseg = (L + C - 1) / C;
    int nsegw = nseg;
    nsegw = max(nsegw, __shfl_xor(nsegw, 16));
    nsegw = max(nsegw, __shfl_xor(nsegw, 32));
    int kv_nx = 0;
    double ck_nx = 0.0;
    if (nsegw >= 1 && nsegw - 1 < nseg) {
      if (i < C && (nsegw - 1) * C + i < L) kv_nx = word[(nsegw - 1) * C + i];
      ck_nx = ck[(nsegw - 1) * 16 + i];
    }
    double b = dot16_bcast(dp, reinterpret_cast<const double2*>(s.ETs + i * ROW));
    for (int c = nsegw - 1; c >= 0; --c) {
      const bool act = c < nseg;
      const int base = c * C;
      int kv = kv_nx;
      if (kv >= K) kv = 0;  // counted in the forward sweep
      double fs[C];
      fs[0] = act ? ck_nx : 0.0;
      kv_nx = 0;
      ck_nx = 0.0;
      if (c >= 1 && c - 1 < nseg) {
        if (i < C && (c - 1) * C + i < L) kv_nx = word[(c - 1) * C + i];
        ck_nx = ck[(c - 1) * 16 + i];
      }
#define GST_REC(R)                                                   \
  {                                                                  \
    const int k = bcast_i32<R - 1>(kv);                              \
    fs[R] = dot16_bcast(fs[R - 1], grow(s, k, i));                   \
  }
      GST_REC(1) GST_REC(2) GST_REC(3) GST_REC(4) GST_REC(5) GST_REC(6) GST_REC(7)
#undef GST_REC
#define GST_BWD(R)                                                   \
  {                                                                  \
    const bool v = act && (base + R < L);                            \
    const int k = bcast_i32<R>(kv);                                  \
    const int e = team * C + R;                                      \
    st_b[e * 16 + i] = b;                                            \
    st_f[e * 16 + i] = fs[R];                                        \
    if (i == 0) st_k[e] = v ? (uint8_t)k : (uint8_t)0xFF;            \
    const double bn = dot16_bcast(b, gtrow(s, k, i));                \
    b = v ? bn : b;                                                  \
  }
      GST_BWD(7) GST_BWD(6) GST_BWD(5) GST_BWD(4) GST_BWD(3) GST_BWD(2) GST_BWD(1) GST_BWD(0)
#undef GST_BWD
      wave_sync();
      flush_stash(st_b, st_f, st_k, K, acc, lane);
      wave_sync();
    }
    if (a.anchor_adj) {
      if (has && i < D) a.anchor_adj[q * D + i] = it.anchor >= 0 ? b : 0.0;
      if (has && it.anchor < 0) drho += b;
    } else if (has) {
      drho += b;
    }
  }

  if (bad) atomicAdd(a.status + 0, (unsigned long long)bad);
  if (nonpos) atomicAdd(a.status + 1, (unsigned long long)nonpos);
  if (!grad && a.mode != MODE_LOGLIK) return;
  write_slab<D>(lds_raw, obj, drho, dE, acc, M, K, a.slab + (int64_t)blockIdx.x * slab_width(D, M, K));
}

// Slab sums in two deterministic stages (bodies in gst_device.h).
__global__ __launch_bounds__(256) void reduce_stage1(const double* __restrict__ slab, int n_slabs, int64_t P,
                                                     int per, double* __restrict__ part) {
  slab_sum_stage1(slab, n_slabs, P, per, part, blockIdx.x, blockIdx.y);
}

__global__ __launch_bounds__(256) void reduce_stage2(const double* __restrict__ part, int n_part, int64_t P,
                                                     double* objective, double* grad,
                                                     const double* __restrict__ extra_rho, int D) {
  slab_sum_stage2(part, n_part, P, objective, grad, extra_rho, D, blockIdx.x);
}

}  // namespace

int leaf_ckpt_interval(int) { return C; }
int leaf_teams_per_block(int) { return WAVES * TPW; }
int max_gates_for(int D) { return D <= 16 ? KMAX : (D == 64 ? 5 : 0); }  // D = 64: the gate set fills the LDS

int leaf_blocks_for(int D, int64_t n_items) {
  (void)D;
  const int64_t per_block = WAVES * TPW;
  int64_t b = (n_items + per_block - 1) / per_block;
  if (b < 1) b = 1;
  if (b > 2048) b = 2048;
  return (int)b;
}

hipError_t launch_leaf(const LeafLaunch& a, int n_blocks, hipStream_t stream) {
  const size_t bytes = lds_bytes(a.K);
  if (a.D == 16)
    gst_launch(leaf_kernel<16>, dim3(n_blocks), dim3(256), bytes, stream, a);
  else if (a.D == 4)
    gst_launch(leaf_kernel<4>, dim3(n_blocks), dim3(256), bytes, stream, a);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

int reduce_parts(int n_slabs) {
  int g = (n_slabs + 15) / 16;
  return g < 1 ? 1 : (g > 64 ? 64 : g);
}

hipError_t launch_reduce(const double* slab, int n_slabs, int64_t P, double* objective, double* grad,
                         const double* extra_rho, int D, double* part, hipStream_t stream) {
  const int G = reduce_parts(n_slabs);
  const int per = (n_slabs + G - 1) / G;
  gst_launch(reduce_stage1, dim3((unsigned)((P + 63) / 64), G), dim3(256), 0, stream, slab, n_slabs, P, per,
                     part);
  gst_launch(reduce_stage2, dim3((unsigned)((P + 63) / 64)), dim3(256), 0, stream, part, G, P, objective, grad,
                     extra_rho, D);
  return hipGetLastError();
}

}  // namespace gst
