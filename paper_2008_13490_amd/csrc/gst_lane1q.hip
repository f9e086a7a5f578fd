// One-qubit gate sets (D = 4) with one chain per lane.
//
// A one-qubit state has four components, too few to spread over a 16-lane
// DPP row without idle lanes; here every lane owns a whole chain (its four
// components in registers), a wave runs 64 sequences at once and takes
// tiles of 64 consecutive sequences of a request's length-sorted order from
// the work queue.
//
//   * Forward step, per lane: f'_i = fma(G[k][i][3], f_3, fma(.., fma(G[k][i][0],
//     f_0, 0))), columns ascending from zero as in the plain definition, so
//     states and probabilities are bit-identical to a sequential loop.  The
//     gate rows come from the wave's copy of the gate set in LDS (16 doubles
//     per gate; lanes that apply the same gate read the same address).
//   * Checkpoints every 8 steps in HBM (coalesced across the wave); the
//     reverse sweep recomputes a segment from its checkpoint into the wave's
//     LDS, applies b <- G^T b and accumulates dG_k += b f^T in per-lane
//     registers for all gates (the update of the gates a lane does not apply
//     adds zeros).
//   * At the end of a tile the wave adds its 64 lanes in a fixed butterfly
//     order and writes the tile's row of partial sums (the slab layout of the
//     other kernels), so a request's result does not depend on which wave ran
//     which tile, nor on the other requests of a batch.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "gst_device.h"
#include "gst_internal.h"

namespace gst {
namespace {

constexpr int CL = 8;         // steps per reverse segment (checkpoint interval)
constexpr int SLOT = 64 + 16 + 4;  // doubles of LDS per wave: G[4][4][4], E[4][4], rho[4]

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int sh = 32; sh >= 1; sh >>= 1) v += __shfl_xor(v, sh);
  return v;
}

// f' = G f with the plain column order; g = the 16 entries of one gate.
__device__ __forceinline__ void apply(const double* g, double (&f)[4]) {
  const double2* r = reinterpret_cast<const double2*>(g);
  const double2 a0 = r[0], a1 = r[1], a2 = r[2], a3 = r[3], a4 = r[4], a5 = r[5], a6 = r[6], a7 = r[7];
  const double x0 = fma(a1.y, f[3], fma(a1.x, f[2], fma(a0.y, f[1], fma(a0.x, f[0], 0.0))));
  const double x1 = fma(a3.y, f[3], fma(a3.x, f[2], fma(a2.y, f[1], fma(a2.x, f[0], 0.0))));
  const double x2 = fma(a5.y, f[3], fma(a5.x, f[2], fma(a4.y, f[1], fma(a4.x, f[0], 0.0))));
  const double x3 = fma(a7.y, f[3], fma(a7.x, f[2], fma(a6.y, f[1], fma(a6.x, f[0], 0.0))));
  f[0] = x0;
  f[1] = x1;
  f[2] = x2;
  f[3] = x3;
}

// b' = G^T b.
__device__ __forceinline__ void apply_t(const double* g, double (&b)[4]) {
  const double2* r = reinterpret_cast<const double2*>(g);
  const double2 a0 = r[0], a1 = r[1], a2 = r[2], a3 = r[3], a4 = r[4], a5 = r[5], a6 = r[6], a7 = r[7];
  const double y0 = fma(a6.x, b[3], fma(a4.x, b[2], fma(a2.x, b[1], a0.x * b[0])));
  const double y1 = fma(a6.y, b[3], fma(a4.y, b[2], fma(a2.y, b[1], a0.y * b[0])));
  const double y2 = fma(a7.x, b[3], fma(a5.x, b[2], fma(a3.x, b[1], a1.x * b[0])));
  const double y3 = fma(a7.y, b[3], fma(a5.y, b[2], fma(a3.y, b[1], a1.y * b[0])));
  b[0] = y0;
  b[1] = y1;
  b[2] = y2;
  b[3] = y3;
}

// Gate indices of steps [t, t + 8) of a word packed into 64 bits (byte x =
// step t + x; steps at or past L read as 0).  `base` always exists.
__device__ __forceinline__ uint64_t load_pack(const __attribute__((address_space(1))) uint8_t* word, int t, int L,
                                              const __attribute__((address_space(1))) uint8_t* base) {
  uint64_t k = 0;
#pragma unroll
  for (int x = 0; x < CL; ++x) {
    const bool in = t + x < L;
    const uint64_t v = *(in ? word + t + x : base);
    k |= (in ? v : 0ull) << (8 * x);
  }
  return k;
}

template <int K>
__global__ __launch_bounds__(256, 2) void lane1q_kernel(const BatchLaunch a) {
  extern __shared__ double lds1[];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double* Gw = lds1 + wave * SLOT;
  double* Ew = Gw + 64;
  // states of the current reverse segment: [x][lane][4]
  double* fsl = lds1 + 4 * SLOT + (size_t)wave * CL * 64 * 4;
  const int64_t gwave = (int64_t)blockIdx.x * 4 + wave;
  double* ck = a.ckpt + gwave * a.ckpt_per_team;
  double* rw = Ew + 16;
  int staged = -1;
  unsigned bad = 0, nonpos = 0;
  for (;;) {
    int tile = 0;
    if (lane == 0) tile = (int)atomicAdd(a.queue, 1u);
    tile = __builtin_amdgcn_readfirstlane(tile);
    if (tile >= a.n_tiles) break;
    const BatchTile T = a.tiles[tile];
    const BatchReq R = a.reqs ? a.reqs[T.req] : a.one;
    const int M = R.M;
    if (T.req != staged) {
      wave_sync();
      Gw[lane] = lane < K * 16 ? R.G[lane] : 0.0;
      if (lane < 16) Ew[lane] = lane < M * 4 ? R.E[lane] : 0.0;
      if (lane < 4) rw[lane] = R.rho[lane];
      staged = T.req;
      wave_sync();
    }
    const auto* g_off = as_global(R.off);
    const auto* g_order = as_global(R.order);
    const auto* g_gates = as_global(R.gates);
    const auto* g_counts = as_global(R.counts);
    const auto* g_W = as_global(R.W);
    auto* g_probs = as_global(R.probs);
    const bool grad = R.want_grad != 0;
    double obj = 0.0;
    unsigned tile_nonpos = 0;
    double drho[4] = {0.0, 0.0, 0.0, 0.0};
    double dE[4][4];
    double dG[K][16];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int j = 0; j < 4; ++j) dE[m][j] = 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int e = 0; e < 16; ++e) dG[k][e] = 0.0;
    for (int64_t qb = T.q0; qb < T.q1; qb += 64) {
      const int64_t q = qb + lane;
      const bool has = q < T.q1;
      const int64_t seq = has ? (R.order ? g_order[q] : q) : 0;
      const int64_t beg = has ? g_off[seq] : 0;
      const int L = has ? (int)(g_off[seq + 1] - beg) : 0;
      int Lw = L;
#pragma unroll
      for (int sh = 32; sh >= 1; sh >>= 1) Lw = max(Lw, __shfl_xor(Lw, sh));
      const auto* word = g_gates + beg;
      double f[4] = {rw[0], rw[1], rw[2], rw[3]};
      // ---- forward, a segment of eight steps at a time; its gate indices
      // are loaded one segment ahead ----
      uint64_t kn = load_pack(word, 0, L, g_gates);
      for (int t0 = 0; t0 < Lw; t0 += CL) {
        const uint64_t kc = kn;
        kn = load_pack(word, t0 + CL, L, g_gates);
        if (grad && t0 < L) {
          double* c = ck + (int64_t)(t0 / CL) * 256 + lane * 4;
          reinterpret_cast<double4*>(c)[0] = double4{f[0], f[1], f[2], f[3]};
        }
#pragma unroll 1
        for (int x = 0; x < CL; ++x) {
          int k = (int)((kc >> (8 * x)) & 0xFF);
          if (k >= K) {
            bad += t0 + x < L;
            k = 0;
          }
          double n[4] = {f[0], f[1], f[2], f[3]};
          apply(Gw + k * 16, n);
          if (t0 + x < L) {
#pragma unroll
            for (int j = 0; j < 4; ++j) f[j] = n[j];
          }
        }
      }
      // ---- readout, objective, seeds ----
      double dp[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        if (m < M) {
          const double* e = Ew + m * 4;
          const double p = fma(e[3], f[3], fma(e[2], f[2], fma(e[1], f[1], fma(e[0], f[0], 0.0))));
          if (has) {
            const int64_t o = seq * M + m;
            if (R.probs) g_probs[o] = p;
            if (R.mode == MODE_LOGLIK) {
              const int32_t N = g_counts[o];
              if (N > 0) {
                if (p <= 0.0) {
                  ++tile_nonpos;
                  obj = INFINITY;  // -N log p with p <= 0; no term is ever -inf
                } else {
                  obj -= (double)N * log(p);
                  dp[m] = -(double)N / p;
                }
              }
            } else if (R.mode == MODE_VJP) {
              dp[m] = g_W[o];
            }
          }
        }
      }
      if (!grad) continue;
      double b[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        if (m < M) {
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            dE[m][j] = fma(dp[m], f[j], dE[m][j]);
            b[j] = fma(Ew[m * 4 + j], dp[m], b[j]);
          }
        }
      }
      // ---- reverse sweep, one segment at a time: recompute its states from
      // the checkpoint into LDS, then walk it backwards ----
      const int nseg = (L + CL - 1) / CL;
      int nsegw = nseg;
#pragma unroll
      for (int sh = 32; sh >= 1; sh >>= 1) nsegw = max(nsegw, __shfl_xor(nsegw, sh));
      for (int c = nsegw - 1; c >= 0; --c) {
        const bool act = c < nseg;
        const int base = c * CL;
        uint64_t kc = act ? load_pack(word, base, L, g_gates) : 0ull;
        double s[4];
        {
          const double* cp = ck + (int64_t)c * 256 + lane * 4;
          const double4 v = act ? reinterpret_cast<const double4*>(cp)[0] : double4{0.0, 0.0, 0.0, 0.0};
          s[0] = v.x;
          s[1] = v.y;
          s[2] = v.z;
          s[3] = v.w;
        }
#pragma unroll 1
        for (int x = 0; x < CL; ++x) {
          double4* dst = reinterpret_cast<double4*>(fsl + ((size_t)x * 64 + lane) * 4);
          *dst = double4{s[0], s[1], s[2], s[3]};
          int k = (int)((kc >> (8 * x)) & 0xFF);
          apply(Gw + (k < K ? k : 0) * 16, s);
        }
#pragma unroll 1
        for (int x = CL - 1; x >= 0; --x) {
          const bool v = act && base + x < L;
          int k = (int)((kc >> (8 * x)) & 0xFF);
          k = k < K ? k : 0;
          const double4 fv = *reinterpret_cast<const double4*>(fsl + ((size_t)x * 64 + lane) * 4);
          const double fx[4] = {fv.x, fv.y, fv.z, fv.w};
          // dG_k += b fx^T for the gate of this step (the others add zeros)
#pragma unroll
          for (int kk = 0; kk < K; ++kk) {
            const bool on = v && k == kk;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const double bi = on ? b[i] : 0.0;
#pragma unroll
              for (int j = 0; j < 4; ++j) dG[kk][i * 4 + j] = fma(bi, fx[j], dG[kk][i * 4 + j]);
            }
          }
          double nb[4] = {b[0], b[1], b[2], b[3]};
          apply_t(Gw + k * 16, nb);
          if (v) {
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = nb[j];
          }
        }
      }
      if (has) {
#pragma unroll
        for (int j = 0; j < 4; ++j) drho[j] += b[j];
      }
    }
    {
      const double tn = wsum((double)tile_nonpos);
      if (lane == 0 && tn > 0) atomicAdd(a.req_nonpos + (a.reqs ? T.req : 0), (unsigned long long)tn);
      nonpos += tile_nonpos;
    }
    if (!grad && R.mode != MODE_LOGLIK) continue;
    // ---- the tile's partial sums: [objective | rho (4) | E (M*4) | G (K*16)] ----
    double* out = R.slab + (int64_t)T.local * slab_width(4, M, K);
    {
      const double sm = wsum(obj);
      if (lane == 0) out[0] = sm;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const double sm = wsum(drho[j]);
      if (lane == 0) out[1 + j] = sm;
    }
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      if (m < M) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const double sm = wsum(dE[m][j]);
          if (lane == 0) out[5 + m * 4 + j] = sm;
        }
      }
    }
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const double sm = wsum(dG[k][e]);
        if (lane == 0) out[5 + M * 4 + k * 16 + e] = sm;
      }
  }
  // nonpos and bad-index counts are per lane
  const double nb = wsum((double)bad), np = wsum((double)nonpos);
  if (lane == 0) {
    if (nb > 0) atomicAdd(a.status + 0, (unsigned long long)nb);
    if (np > 0) atomicAdd(a.status + 1, (unsigned long long)np);
  }
}

}  // namespace

// Per-lane kernel for one-qubit requests with K <= 4 (registers of dG).
bool lane1q_supported(int K) { return K >= 1 && K <= 4; }

size_t lane1q_lds() { return ((size_t)4 * SLOT + (size_t)4 * CL * 64 * 4) * sizeof(double); }

int lane1q_ckpt_per_wave(int64_t max_len) { return (int)(((max_len + CL - 1) / CL + 1) * 256); }

int lane1q_blocks_per_cu(int K) {
  int n = 0;
  hipError_t e = hipErrorInvalidValue;
  switch (K) {
    case 1: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, lane1q_kernel<1>, 256, lane1q_lds()); break;
    case 2: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, lane1q_kernel<2>, 256, lane1q_lds()); break;
    case 3: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, lane1q_kernel<3>, 256, lane1q_lds()); break;
    case 4: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, lane1q_kernel<4>, 256, lane1q_lds()); break;
    default: break;
  }
  return (e == hipSuccess && n > 0) ? n : 1;
}

hipError_t launch_lane1q(const BatchLaunch& a, int K, int n_blocks, hipStream_t stream) {
  switch (K) {
    case 1: gst_launch(lane1q_kernel<1>, dim3(n_blocks), dim3(256), lane1q_lds(), stream, a); break;
    case 2: gst_launch(lane1q_kernel<2>, dim3(n_blocks), dim3(256), lane1q_lds(), stream, a); break;
    case 3: gst_launch(lane1q_kernel<3>, dim3(n_blocks), dim3(256), lane1q_lds(), stream, a); break;
    case 4: gst_launch(lane1q_kernel<4>, dim3(n_blocks), dim3(256), lane1q_lds(), stream, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace gst
