// Sequence kernel for one- and two-qubit gate sets (D = 4 or 16).
//
// Thesis Sec. 6.3.1: p[s][m] = e_m^T G[s_L] ... G[s_1] rho, the multinomial
// log-likelihood of the counts and its gradient (chain rule of the product).
//
// Layout on the chip
//   * A team of 16 lanes (one DPP row) owns one chain; lane i holds component
//     i of the current state f (rows i >= D are zero padding for one qubit).
//     A wave runs four chains, a workgroup of four waves sixteen.
//   * The gate set lives in LDS twice: G (rows) for the forward product and
//     G^T (rows = columns of G) for the adjoint, rows padded to 18 doubles so
//     that the 16-byte reads of a team hit distinct banks.
//   * One step of the forward chain is, in lane i, 16 fused multiply-adds
//     acc = fma(G[k][i][j], f[j], acc), j ascending from acc = 0, with f[j]
//     broadcast from lane j of the row by DPP row_newbcast inside
//     v_fmac_f64.  This is the order of the plain definition, so the states
//     and the probabilities are bit-identical to a sequential evaluation.
//   * The reverse sweep recomputes each segment of C steps from a checkpoint
//     (HBM scratch, one per C steps), runs b <- G^T b and stashes the pairs
//     (b_t, f_{t-1}) and the gate index in the wave's LDS stash.  After each
//     segment the wave accumulates dG_k += sum b_t f_{t-1}^T with FP64 MFMA
//     16x16x4 tiles, one tile per gate, held in registers; steps are grouped by
//     gate so that every MFMA is a real rank-4 update.
//   * At the end the four waves add their tiles, adjoints and objective in a
//     fixed order and write one slab of partial results per workgroup; a
//     second kernel adds the slabs in ascending order.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "gst_internal.h"

namespace gst {
namespace {

constexpr int TEAM = 16;           // lanes per chain
constexpr int WAVES = 4;           // waves per workgroup
constexpr int TPW = 64 / TEAM;     // chains per wave
constexpr int ROW = 18;            // padded LDS row stride in doubles
constexpr int GATE_STRIDE = 16 * ROW;  // doubles per gate matrix in LDS
constexpr int KMAX = 8;            // gates accumulated on chip
constexpr int C = 8;               // checkpoint interval (steps per segment)

typedef double d4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// cross-lane helpers
// ---------------------------------------------------------------------------
template <int J>
__device__ __forceinline__ int bcast_i32(int v) {
  return __builtin_amdgcn_update_dpp(0, v, 0x150 + J, 0xF, 0xF, false);
}

template <int J>
__device__ __forceinline__ double bcast_f64(double v) {
  long long x = __double_as_longlong(v);
  int lo = __builtin_amdgcn_update_dpp(0, (int)x, 0x150 + J, 0xF, 0xF, false);
  int hi = __builtin_amdgcn_update_dpp(0, (int)(x >> 32), 0x150 + J, 0xF, 0xF, false);
  return __longlong_as_double((long long)(unsigned)lo | ((long long)hi << 32));
}

// acc = sum_j fma(r[j], x@lane j of this row, acc) for j = 0..15, ascending,
// starting from acc = 0.  x is read through DPP row_newbcast; the leading
// s_nop covers the VALU-write -> DPP-read hazard on x.
__device__ __forceinline__ double dot16_bcast(double x, const double2* __restrict__ row) {
  const double2 a0 = row[0], a1 = row[1], a2 = row[2], a3 = row[3];
  const double2 a4 = row[4], a5 = row[5], a6 = row[6], a7 = row[7];
  double acc = 0.0;
  asm volatile(
      "s_nop 1\n\t"
      "v_fmac_f64_dpp %0, %1, %2 row_newbcast:0 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %0, %1, %3 row_newbcast:1 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %0, %1, %4 row_newbcast:2 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %0, %1, %5 row_newbcast:3 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %0, %1, %6 row_newbcast:4 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %0, %1, %7 row_newbcast:5 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %0, %1, %8 row_newbcast:6 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %0, %1, %9 row_newbcast:7 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %0, %1, %10 row_newbcast:8 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %0, %1, %11 row_newbcast:9 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %0, %1, %12 row_newbcast:10 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %0, %1, %13 row_newbcast:11 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %0, %1, %14 row_newbcast:12 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %0, %1, %15 row_newbcast:13 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %0, %1, %16 row_newbcast:14 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %0, %1, %17 row_newbcast:15 row_mask:0xf bank_mask:0xf"
      : "+v"(acc)
      : "v"(x), "v"(a0.x), "v"(a0.y), "v"(a1.x), "v"(a1.y), "v"(a2.x), "v"(a2.y), "v"(a3.x),
        "v"(a3.y), "v"(a4.x), "v"(a4.y), "v"(a5.x), "v"(a5.y), "v"(a6.x), "v"(a6.y), "v"(a7.x),
        "v"(a7.y));
  return acc;
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// LDS layout (doubles): Gs[K][16][ROW] | GTs[K][16][ROW] | Es[16][ROW] | ETs[16][ROW] |
//                       rho[16] | stash per wave: b[TPW*C][16], f[TPW*C][16] | stash gates (bytes)
struct Lds {
  double* Gs;
  double* GTs;
  double* Es;
  double* ETs;
  double* rho;
  double* stash;   // WAVES * 2 * TPW*C*16
  uint8_t* sk;     // WAVES * TPW*C
};

__host__ __device__ inline size_t lds_bytes(int K) {
  size_t d = (size_t)2 * K * GATE_STRIDE + 2 * 16 * ROW + 16 + (size_t)WAVES * 2 * TPW * C * 16;
  return d * 8 + (size_t)WAVES * TPW * C;
}

__device__ __forceinline__ Lds carve(double* base, int K) {
  Lds l;
  l.Gs = base;
  l.GTs = l.Gs + (size_t)K * GATE_STRIDE;
  l.Es = l.GTs + (size_t)K * GATE_STRIDE;
  l.ETs = l.Es + 16 * ROW;
  l.rho = l.ETs + 16 * ROW;
  l.stash = l.rho + 16;
  l.sk = reinterpret_cast<uint8_t*>(l.stash + (size_t)WAVES * 2 * TPW * C * 16);
  return l;
}

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
// the kernel
// ---------------------------------------------------------------------------
template <int D>
__global__ __launch_bounds__(256) void leaf_kernel(const LeafLaunch a) {
  extern __shared__ double lds_raw[];
  const int K = a.K, M = a.M;
  Lds s = carve(lds_raw, K);
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int i = lane & 15;          // component owned by this lane
  const int team = lane >> 4;       // chain slot inside the wave

  // ---- stage the gate set (zero-padded to 16 x 16) ----
  for (int x = tid; x < K * 16 * ROW; x += blockDim.x) {
    const int k = x / (16 * ROW), r = (x / ROW) % 16, c = x % ROW;
    double g = 0.0, gt = 0.0;
    if (r < D && c < D) {
      g = a.G[((size_t)k * D + r) * D + c];
      gt = a.G[((size_t)k * D + c) * D + r];
    }
    s.Gs[x] = g;
    s.GTs[x] = gt;
  }
  for (int x = tid; x < 16 * ROW; x += blockDim.x) {
    const int r = x / ROW, c = x % ROW;
    s.Es[x] = (r < M && c < D) ? a.E[(size_t)r * D + c] : 0.0;
    s.ETs[x] = (c < M && r < D) ? a.E[(size_t)c * D + r] : 0.0;
  }
  if (tid < 16) s.rho[tid] = tid < D ? a.rho[tid] : 0.0;
  __syncthreads();

  double* st_b = s.stash + (size_t)wave * 2 * TPW * C * 16;
  double* st_f = st_b + TPW * C * 16;
  uint8_t* st_k = s.sk + wave * TPW * C;

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
    // ---- the four items of this wave ----
    const int64_t q = grp * TPW + team;
    const bool has = q < a.n_items;
    Item it = has ? load_item(a, q) : Item{0, 0, 0, -1};
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

    // ---- forward chain ----
    for (int t0 = 0; t0 < Lw; t0 += 16) {
      int kv = 0;
      if (t0 + i < L) {
        kv = word[t0 + i];
        if (kv >= K) {
          ++bad;
          kv = 0;
        }
      }
#define GST_FWD_STEP(R)                                                             \
  if (t0 + R < Lw) {                                                                \
    const int t = t0 + R;                                                           \
    const int k = bcast_i32<R>(kv);                                                 \
    if (grad && (R % C) == 0 && t < L) ck[(t / C) * 16 + i] = f;                    \
    const double fn = dot16_bcast(f, reinterpret_cast<const double2*>(s.Gs + k * GATE_STRIDE + i * ROW)); \
    f = t < L ? fn : f;                                                             \
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
#define GST_DE(R) if (R < M) dE[R] = fma(bcast_f64<R>(dp), f, dE[R]);
    GST_DE(0) GST_DE(1) GST_DE(2) GST_DE(3) GST_DE(4) GST_DE(5) GST_DE(6) GST_DE(7)
    GST_DE(8) GST_DE(9) GST_DE(10) GST_DE(11) GST_DE(12) GST_DE(13) GST_DE(14) GST_DE(15)
#undef GST_DE
    double b = dot16_bcast(dp, reinterpret_cast<const double2*>(s.ETs + i * ROW));

    // ---- reverse sweep, one segment of C steps at a time ----
    const int nseg = (L + C - 1) / C;
    int nsegw = nseg;
    nsegw = max(nsegw, __shfl_xor(nsegw, 16));
    nsegw = max(nsegw, __shfl_xor(nsegw, 32));
    for (int c = nsegw - 1; c >= 0; --c) {
      const bool act = c < nseg;
      const int base = c * C;
      int kv = 0;
      if (act && i < C && base + i < L) {
        kv = word[base + i];
        if (kv >= K) kv = 0;  // already counted in the forward sweep
      }
      double fs[C];
      fs[0] = act ? ck[c * 16 + i] : 0.0;
      // recompute f_{base+1} .. f_{base+C-1}
#define GST_REC(R)                                                                     \
  {                                                                                    \
    const int k = bcast_i32<R - 1>(kv);                                                \
    fs[R] = dot16_bcast(fs[R - 1], reinterpret_cast<const double2*>(s.Gs + k * GATE_STRIDE + i * ROW)); \
  }
      GST_REC(1) GST_REC(2) GST_REC(3) GST_REC(4) GST_REC(5) GST_REC(6) GST_REC(7)
#undef GST_REC
      // backward over the segment
#define GST_BWD(R)                                                                     \
  {                                                                                    \
    const bool v = act && (base + R < L);                                              \
    const int k = bcast_i32<R>(kv);                                                    \
    const int e = team * C + R;                                                        \
    st_b[e * 16 + i] = b;                                                              \
    st_f[e * 16 + i] = fs[R];                                                          \
    if (i == 0) st_k[e] = v ? (uint8_t)k : (uint8_t)0xFF;                              \
    const double bn = dot16_bcast(b, reinterpret_cast<const double2*>(s.GTs + k * GATE_STRIDE + i * ROW)); \
    b = v ? bn : b;                                                                    \
  }
      GST_BWD(7) GST_BWD(6) GST_BWD(5) GST_BWD(4) GST_BWD(3) GST_BWD(2) GST_BWD(1) GST_BWD(0)
#undef GST_BWD
      wave_sync();
      // ---- dG_k += sum over stashed steps with gate k of b f^T (MFMA 16x16x4) ----
      const int ent = TPW * C;  // <= 64
      const int my_k = lane < ent ? (int)st_k[lane] : 0xFF;
#pragma unroll
      for (int k = 0; k < KMAX; ++k) {
        if (k < K) {
          unsigned long long mask = __ballot(my_k == k);
          while (mask) {
            int e4[4];
#pragma unroll
            for (int z = 0; z < 4; ++z) {
              if (mask) {
                const int bit = __ffsll((long long)mask) - 1;
                e4[z] = bit;
                mask &= mask - 1;
              } else {
                e4[z] = -1;
              }
            }
            const int sel = lane >> 4;
            const int e = sel == 0 ? e4[0] : sel == 1 ? e4[1] : sel == 2 ? e4[2] : e4[3];
            const double av = e >= 0 ? st_b[e * 16 + i] : 0.0;
            const double bv = e >= 0 ? st_f[e * 16 + i] : 0.0;
            acc[k] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[k], 0, 0, 0);
          }
        }
      }
      wave_sync();
    }
    // adjoint at the anchor
    if (a.anchor_adj) {
      if (has && i < D) a.anchor_adj[q * D + i] = b;
    } else if (has) {
      drho += b;
    }
  }

  // ---- combine the four chains of each wave, then the four waves ----
  if (bad) atomicAdd(a.status + 0, (unsigned long long)bad);
  if (nonpos) atomicAdd(a.status + 1, (unsigned long long)nonpos);
  if (!grad && a.mode != MODE_LOGLIK) return;

  __syncthreads();  // LDS is reused from here on
  double* red = lds_raw;  // [WAVES][P16] with P16 = 1 + 16 + 16*16 + K*256
  const int P16 = 1 + 16 + 256 + K * 256;
  double* mine = red + (size_t)wave * P16;
  // objective: lanes m < M of each team
  double o = obj;
#pragma unroll
  for (int sh = 1; sh < 64; sh <<= 1) o += __shfl_xor(o, sh);
  // drho and dE: sum over the four teams (lanes i, 16+i, 32+i, 48+i)
  double dr = drho;
  dr += __shfl_xor(dr, 16);
  dr += __shfl_xor(dr, 32);
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    dE[m] += __shfl_xor(dE[m], 16);
    dE[m] += __shfl_xor(dE[m], 32);
  }
  if (lane == 0) mine[0] = o;
  if (lane < 16) {
    mine[1 + lane] = dr;
#pragma unroll
    for (int m = 0; m < 16; ++m) mine[17 + m * 16 + lane] = dE[m];
  }
  // tiles: C[r][cc] at lane 16*(r&3)+cc, register r>>2
#pragma unroll
  for (int k = 0; k < KMAX; ++k) {
    if (k < K) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = 4 * v + (lane >> 4), cc = lane & 15;
        mine[273 + k * 256 + r * 16 + cc] = acc[k][v];
      }
    }
  }
  __syncthreads();
  const int64_t P = slab_width(D, M, K);
  double* out = a.slab + (int64_t)blockIdx.x * P;
  for (int x = tid; x < P; x += blockDim.x) {
    int src;
    if (x == 0) {
      src = 0;
    } else if (x < 1 + D) {
      src = x;
    } else if (x < 1 + D + M * D) {
      const int y = x - 1 - D;
      src = 17 + (y / D) * 16 + (y % D);
    } else {
      const int y = x - 1 - D - M * D;
      const int k = y / (D * D), r = (y / D) % D, cc = y % D;
      src = 273 + k * 256 + r * 16 + cc;
    }
    double v = red[src];
    v += red[P16 + src];
    v += red[2 * P16 + src];
    v += red[3 * P16 + src];
    out[x] = v;
  }
}

__global__ void reduce_kernel(const double* __restrict__ slab, int n_slabs, int64_t P,
                              double* objective, double* grad,
                              const unsigned long long* __restrict__ status) {
  const bool nonpos = status && status[1] != 0;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < P;
       x += (int64_t)gridDim.x * blockDim.x) {
    double v = 0.0;
    for (int w = 0; w < n_slabs; ++w) v += slab[(int64_t)w * P + x];
    if (x == 0) {
      if (objective) *objective = nonpos ? INFINITY : v;
    } else if (grad && !nonpos) {
      grad[x - 1] = v;
    }
  }
}

}  // namespace

int leaf_ckpt_interval(int) { return C; }
int leaf_teams_per_block(int) { return WAVES * TPW; }
int max_gates_for(int D) { return D <= 16 ? KMAX : 0; }

int leaf_blocks_for(int D, int64_t n_items) {
  (void)D;
  const int64_t per_block = WAVES * TPW;
  int64_t b = (n_items + per_block - 1) / per_block;
  if (b < 1) b = 1;
  if (b > 2048) b = 2048;
  return (int)b;
}

hipError_t launch_leaf(const LeafLaunch& a, int n_blocks, hipStream_t stream) {
  const size_t lds = lds_bytes(a.K);
  const size_t red = (size_t)WAVES * (1 + 16 + 256 + (size_t)a.K * 256) * 8;
  const size_t bytes = lds > red ? lds : red;
  if (a.D == 16) {
    hipLaunchKernelGGL(leaf_kernel<16>, dim3(n_blocks), dim3(256), bytes, stream, a);
  } else if (a.D == 4) {
    hipLaunchKernelGGL(leaf_kernel<4>, dim3(n_blocks), dim3(256), bytes, stream, a);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_reduce(const double* slab, int n_slabs, int64_t P, double* objective,
                         double* grad, const unsigned long long* status, hipStream_t stream) {
  int blocks = (int)((P + 255) / 256);
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(reduce_kernel, dim3(blocks), dim3(256), 0, stream, slab, n_slabs, P, objective,
                     grad, status);
  return hipGetLastError();
}

}  // namespace gst
