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
// trunk forward: one trunk per team
// ---------------------------------------------------------------------------
template <int D>
__global__ __launch_bounds__(256) void trunk_fwd_kernel(const PlanArgs a) {
  extern __shared__ double lds_raw[];
  const int K = a.K;
  const Lds s = carve(lds_raw, K);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, i = lane & 15, team = lane >> 4;
  stage_gateset<D>(s, a.G, a.E, a.rho, K, a.M);
  const int64_t nT = a.t_end - a.t_begin;
  const int64_t n_groups = (nT + TPW - 1) / TPW;
  for (int64_t grp = (int64_t)blockIdx.x * WAVES + wave; grp < n_groups; grp += (int64_t)gridDim.x * WAVES) {
    const int64_t t = a.t_begin + grp * TPW + team;
    const bool has = t < a.t_end;
    const int64_t beg = has ? a.trunk_ptr[t] : 0;
    const int L = has ? (int)(a.trunk_ptr[t + 1] - beg) : 0;
    const int Lw = wave_max4(L);
    const int64_t anc = has ? a.trunk_anchor[t] : -1;
    double f = load_state(a.FA, anc >= 0 ? 1 + anc : 0, D, i);
    const uint8_t* word = a.trunk_gates + beg;
    double* out = a.FA + (1 + beg) * D;
    int kv = i < L ? (int)word[i] : 0;
    Row16 cur = load_row(s.Gs + bcast_i32<0>(kv) * GATE_STRIDE + i * ROW);
    for (int t0 = 0; t0 < Lw; t0 += 16) {
      const int kvn = (t0 + 16 + i < L) ? (int)word[t0 + 16 + i] : 0;
#define GST_TF(R)                                                                    \
  if (t0 + R < Lw) {                                                                 \
    const int j = t0 + R;                                                            \
    const int kn = (R < 15) ? bcast_i32<(R + 1) & 15>(kv) : bcast_i32<0>(kvn);       \
    const Row16 nxt = load_row(s.Gs + kn * GATE_STRIDE + i * ROW);                   \
    const double fn = dot16(f, cur);                                                 \
    f = j < L ? fn : f;                                                              \
    if (j < L && i < D) out[(int64_t)j * D + i] = f;                                 \
    cur = nxt;                                                                       \
  }
      GST_TF(0) GST_TF(1) GST_TF(2) GST_TF(3) GST_TF(4) GST_TF(5) GST_TF(6) GST_TF(7)
      GST_TF(8) GST_TF(9) GST_TF(10) GST_TF(11) GST_TF(12) GST_TF(13) GST_TF(14) GST_TF(15)
#undef GST_TF
      kv = kvn;
    }
  }
}

// ---------------------------------------------------------------------------
// items: one sequence per team, from its anchor state
// ---------------------------------------------------------------------------
template <int D>
__global__ __launch_bounds__(256) void item_kernel(const PlanArgs a) {
  extern __shared__ double lds_raw[];
  const int K = a.K, M = a.M;
  const Lds s = carve(lds_raw, K);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, i = lane & 15, team = lane >> 4;
  stage_gateset<D>(s, a.G, a.E, a.rho, K, M);
  const bool grad = a.want_grad != 0;
  double obj = 0.0;
  double dE[16];
#pragma unroll
  for (int m = 0; m < 16; ++m) dE[m] = 0.0;
  unsigned nonpos = 0;
  const int64_t n_groups = (a.n_items + TPW - 1) / TPW;
  for (int64_t grp = (int64_t)blockIdx.x * WAVES + wave; grp < n_groups; grp += (int64_t)gridDim.x * WAVES) {
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
    double f = load_state(a.FA, anc >= 0 ? 1 + anc : 0, D, i);

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
    double b = dot16_split(dp, load_row(s.ETs + i * ROW));

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
    const double bn = dot16_split(b, load_row(s.GTs + k * GATE_STRIDE + i * ROW)); \
    b = x < L ? bn : b;                                                   \
  }
      GST_IB(15) GST_IB(14) GST_IB(13) GST_IB(12) GST_IB(11) GST_IB(10) GST_IB(9) GST_IB(8)
      GST_IB(7) GST_IB(6) GST_IB(5) GST_IB(4) GST_IB(3) GST_IB(2) GST_IB(1) GST_IB(0)
#undef GST_IB
    }
    if (has && i < D) a.item_adj[q * D + i] = b;
  }
  if (nonpos) atomicAdd(a.status + 1, (unsigned long long)nonpos);
  if (a.mode != MODE_LOGLIK && !grad) return;
  d4 zero[KMAX];
#pragma unroll
  for (int k = 0; k < KMAX; ++k) zero[k] = d4{0.0, 0.0, 0.0, 0.0};
  write_slab<D>(lds_raw, obj, 0.0, dE, zero, M, K, a.slab);
}

// ---------------------------------------------------------------------------
// trunk reverse sweep
// ---------------------------------------------------------------------------
template <int D>
__global__ __launch_bounds__(256) void trunk_bwd_kernel(const PlanArgs a) {
  extern __shared__ double lds_raw[];
  const int K = a.K;
  const Lds s = carve(lds_raw, K);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, i = lane & 15, team = lane >> 4;
  stage_gateset<D>(s, a.G, a.E, a.rho, K, a.M);
  const int64_t nT = a.t_end - a.t_begin;
  const int64_t n_groups = (nT + TPW - 1) / TPW;
  for (int64_t grp = (int64_t)blockIdx.x * WAVES + wave; grp < n_groups; grp += (int64_t)gridDim.x * WAVES) {
    const int64_t t = a.t_begin + grp * TPW + team;
    const bool has = t < a.t_end;
    const int64_t beg = has ? a.trunk_ptr[t] : 0;
    const int L = has ? (int)(a.trunk_ptr[t + 1] - beg) : 0;
    const int Lw = wave_max4(L);
    const int nb = (Lw + 15) / 16;
    const uint8_t* word = a.trunk_gates + beg;
    const int32_t* injs = a.trunk_inj + beg;
    double* ba = a.BA + beg * D;
    double b = 0.0;
    // Software pipeline over 16-step blocks, walked from the end: gate
    // indices and injection slots are loaded two blocks ahead, the injected
    // vectors one block ahead of their use.
    auto ld_idx = [&](int c, int& kvo, int& jvo) {
      kvo = 0;
      jvo = -1;
      if (c >= 0 && c * 16 + i < L) {
        kvo = word[c * 16 + i];
        jvo = injs[c * 16 + i];
      }
    };
    int kv_c, jv_c, kv_n, jv_n;
    ld_idx(nb - 1, kv_c, jv_c);
    ld_idx(nb - 2, kv_n, jv_n);
    double ij_c[16], ij_n[16];
#define GST_LDI(DST, JV, R)                                                       \
  {                                                                               \
    const int slot = bcast_i32<R>(JV);                                            \
    DST[R] = (slot >= 0 && i < D) ? a.inj[(int64_t)slot * D + i] : 0.0;           \
  }
#define GST_LDI16(DST, JV)                                                                      \
  GST_LDI(DST, JV, 0) GST_LDI(DST, JV, 1) GST_LDI(DST, JV, 2) GST_LDI(DST, JV, 3)              \
  GST_LDI(DST, JV, 4) GST_LDI(DST, JV, 5) GST_LDI(DST, JV, 6) GST_LDI(DST, JV, 7)              \
  GST_LDI(DST, JV, 8) GST_LDI(DST, JV, 9) GST_LDI(DST, JV, 10) GST_LDI(DST, JV, 11)            \
  GST_LDI(DST, JV, 12) GST_LDI(DST, JV, 13) GST_LDI(DST, JV, 14) GST_LDI(DST, JV, 15)
    GST_LDI16(ij_c, jv_c)
    for (int c = nb - 1; c >= 0; --c) {
      const int t0 = c * 16;
      // loads for later blocks
      GST_LDI16(ij_n, jv_n)
      int kv_nn, jv_nn;
      ld_idx(c - 2, kv_nn, jv_nn);
      // the block runs from its last valid step down to step 0
      const int rstart = min(15, Lw - 1 - t0);
      Row16 cur = load_row(s.GTs + __shfl(kv_c, (lane & 48) | rstart, 64) * GATE_STRIDE + i * ROW);
#define GST_TB(R)                                                                     \
  if (R <= rstart) {                                                                  \
    const int j = t0 + R;                                                             \
    const bool v = j < L;                                                             \
    const int kn = bcast_i32<(R + 15) & 15>(kv_c);                                    \
    const Row16 nxt = load_row(s.GTs + kn * GATE_STRIDE + i * ROW);                   \
    if (v) b += ij_c[R];                                                              \
    if (v && i < D) ba[(int64_t)j * D + i] = b;                                       \
    const double bn = dot16_split(b, cur);                                            \
    b = v ? bn : b;                                                                   \
    cur = nxt;                                                                        \
  }
      GST_TB(15) GST_TB(14) GST_TB(13) GST_TB(12) GST_TB(11) GST_TB(10) GST_TB(9) GST_TB(8)
      GST_TB(7) GST_TB(6) GST_TB(5) GST_TB(4) GST_TB(3) GST_TB(2) GST_TB(1) GST_TB(0)
#undef GST_TB
      kv_c = kv_n;
      kv_n = kv_nn;
      jv_n = jv_nn;
#pragma unroll
      for (int r = 0; r < 16; ++r) ij_c[r] = ij_n[r];
    }
#undef GST_LDI16
#undef GST_LDI
    if (has && i < D) a.trunk_adj[t * D + i] = b;
  }
}

__global__ void inject_kernel(const InjectLaunch a) {
  const int D = a.D;
  const int64_t n = (a.s_end - a.s_begin) * D;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x) {
    const int64_t slot = a.s_begin + x / D;
    const int i = (int)(x % D);
    double v = 0.0;
    for (int64_t z = a.inj_ptr[slot]; z < a.inj_ptr[slot + 1]; ++z) {
      const int64_t src = a.inj_src[z];
      v += src >= 0 ? a.item_adj[src * D + i] : a.trunk_adj[(-src - 1) * D + i];
    }
    a.inj[slot * D + i] = v;
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
  // records r0 + 16*g + 4*wave + z for g = 0, 1, ...
  for (int64_t base = r0 + 4 * wave; base < r1; base += 4 * 4 * WAVES) {
    double av[4], bv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t r = base + u * 4 * WAVES + z;
      av[u] = 0.0;
      bv[u] = 0.0;
      if (r < r1 && i < D) {
        av[u] = a.BA[a.rec_b[r] * D + i];
        bv[u] = a.FA[a.rec_f[r] * D + i];
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv[u], acc, 0, 0, 0);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) tile[wave][(4 * v + (lane >> 4)) * 16 + (lane & 15)] = acc[v];
  __syncthreads();
  const int64_t P = slab_width(D, a.M, a.K);
  double* out = a.slab + c * P;
  const int64_t g0 = 1 + D + (int64_t)a.M * D + (int64_t)k * D * D;
  for (int64_t x = tid; x < P; x += blockDim.x) {
    double v = 0.0;
    if (x >= g0 && x < g0 + D * D) {
      const int y = (int)(x - g0), r = y / D, cc = y % D;
      v = (tile[0][r * 16 + cc] + tile[1][r * 16 + cc]) + (tile[2][r * 16 + cc] + tile[3][r * 16 + cc]);
    }
    out[x] = v;
  }
}

}  // namespace

int item_blocks_for(int64_t n_items) {
  int64_t b = (n_items + WAVES * TPW - 1) / (WAVES * TPW);
  if (b < 1) b = 1;
  if (b > 1024) b = 1024;
  return (int)b;
}

static int trunk_blocks(int64_t n) {
  int64_t b = (n + WAVES * TPW - 1) / (WAVES * TPW);
  return (int)(b < 1 ? 1 : (b > 2048 ? 2048 : b));
}

hipError_t launch_trunk_fwd(const PlanArgs& a, hipStream_t stream) {
  const int blocks = trunk_blocks(a.t_end - a.t_begin);
  const size_t bytes = lds_main_bytes(a.K);
  if (a.D == 16)
    hipLaunchKernelGGL(trunk_fwd_kernel<16>, dim3(blocks), dim3(256), bytes, stream, a);
  else if (a.D == 4)
    hipLaunchKernelGGL(trunk_fwd_kernel<4>, dim3(blocks), dim3(256), bytes, stream, a);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_trunk_bwd(const PlanArgs& a, hipStream_t stream) {
  const int blocks = trunk_blocks(a.t_end - a.t_begin);
  const size_t bytes = lds_main_bytes(a.K);
  if (a.D == 16)
    hipLaunchKernelGGL(trunk_bwd_kernel<16>, dim3(blocks), dim3(256), bytes, stream, a);
  else if (a.D == 4)
    hipLaunchKernelGGL(trunk_bwd_kernel<4>, dim3(blocks), dim3(256), bytes, stream, a);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_items(const PlanArgs& a, int n_blocks, hipStream_t stream) {
  const size_t bytes = lds_bytes(a.K);
  if (a.D == 16)
    hipLaunchKernelGGL(item_kernel<16>, dim3(n_blocks), dim3(256), bytes, stream, a);
  else if (a.D == 4)
    hipLaunchKernelGGL(item_kernel<4>, dim3(n_blocks), dim3(256), bytes, stream, a);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_inject(const InjectLaunch& a, hipStream_t stream) {
  const int64_t n = (a.s_end - a.s_begin) * a.D;
  if (n <= 0) return hipSuccess;
  int blocks = (int)((n + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(inject_kernel, dim3(blocks), dim3(256), 0, stream, a);
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
