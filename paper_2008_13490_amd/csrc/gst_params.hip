// Parameterizations of the gate set: the TP and CPTP estimation modes.
//
// Thesis Sec. 6.3.2 runs the fit with fully unconstrained maps, with
// trace-preserving maps, or with CPTP channels (the quantum operations of
// Sec. 2.4).  These kernels map a parameter vector theta to the full
// parameterization (rho, effects, gates as Pauli transfer matrices) and carry
// the full gradient back to theta.
//
// TP: row 0 of every gate is e_0, rho[0] = 1/sqrt(d), and the last effect is
// vec(1) minus the others.  CPTP: G_k = exp(L_k) G0_k (Eq.
// GateDecompositionLindbladCorrespondence) with L_k the transfer matrix of a
// generator in the form of Eq. masterequation: -i [H, .] with
// H = sum_k h_k P_k / 2 (Eq. GateDecompositionHamiltonian) plus
// sum_jk C_jk (P_j . P_k - {P_k P_j, .} / 2) with C = T T^dagger; rho is
// A A^dagger / tr(A A^dagger); effects as TP.
//
// The matrix exponential is a degree-16 Taylor polynomial of L / 2^s by
// Horner's rule followed by s squarings, on the FP64 matrix cores (one wave).
// The backward pass needs the adjoint of the exponential's derivative: for the
// trace inner product it is the derivative at L^T, read off the upper-right
// block of exp([[L^T, X], [0, L^T]]) with X = dF/dG G0^T, computed by the same
// scheme on block upper-triangular matrices.  From dF/dL the parameters'
// gradient follows by the structure tables (h) and by C = T T^dagger:
// dF/dT = (conj(Chat) + Chat^T) T with Chat_jk = sum_ab dF/dL_ab z_ab(j).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "gst_device.h"
#include "gst_internal.h"

namespace gst {

namespace {

constexpr int TAYLOR = 16;  // degree of the Taylor polynomial, for ||X|| <= 1/2

// ---------------------------------------------------------------------------
// TP: affine maps, one thread per output entry
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void tp_forward_kernel(const ParamLaunch a) {
  const int D = a.D, M = a.M;
  const int64_t n_rho = D, n_e = (int64_t)M * D, n_g = (int64_t)a.K * D * D;
  const double* eth = a.theta + (D - 1);
  const double* gth = eth + (int64_t)(M - 1) * D;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n_rho + n_e + n_g;
       x += (int64_t)gridDim.x * blockDim.x) {
    if (x < n_rho) {
      a.rho[x] = x == 0 ? a.inv_sqrt_d : a.theta[x - 1];
    } else if (x < n_rho + n_e) {
      const int64_t y = x - n_rho;
      const int m = (int)(y / D), c = (int)(y % D);
      double v;
      if (m < M - 1) {
        v = eth[(int64_t)m * D + c];
      } else {
        v = c == 0 ? a.sqrt_d : 0.0;
        for (int mm = 0; mm < M - 1; ++mm) v = v - eth[(int64_t)mm * D + c];
      }
      a.E[y] = v;
    } else {
      const int64_t y = x - n_rho - n_e;
      const int64_t k = y / ((int64_t)D * D);
      const int r = (int)((y / D) % D), c = (int)(y % D);
      a.G[y] = r == 0 ? (c == 0 ? 1.0 : 0.0) : gth[k * D * (D - 1) + (int64_t)(r - 1) * D + c];
    }
  }
}

__global__ __launch_bounds__(256) void tp_backward_kernel(const ParamLaunch a) {
  const int D = a.D, M = a.M;
  const int64_t n_rho = D - 1, n_e = (int64_t)(M - 1) * D, n_g = (int64_t)a.K * D * (D - 1);
  const double* gr = a.grad_full;
  const double* ge = gr + D;
  const double* gg = ge + (int64_t)M * D;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n_rho + n_e + n_g;
       x += (int64_t)gridDim.x * blockDim.x) {
    double v;
    if (x < n_rho) {
      v = gr[x + 1];
    } else if (x < n_rho + n_e) {
      const int64_t y = x - n_rho;
      v = ge[y] - ge[(int64_t)(M - 1) * D + y % D];
    } else {
      const int64_t y = x - n_rho - n_e;
      const int64_t k = y / ((int64_t)D * (D - 1));
      v = gg[k * D * D + D + y % ((int64_t)D * (D - 1))];
    }
    a.grad_theta[x] = v;
  }
}

// ---------------------------------------------------------------------------
// CPTP
// ---------------------------------------------------------------------------
// entry [r][c] of the Pauli product P_i (n qubits, qubit 0 the most significant bit)
__device__ inline void pauli_entry(int i, int r, int c, int n, double* re, double* im) {
  double pr = 1.0, pi = 0.0;
  for (int q = 0; q < n; ++q) {
    const int sh = n - 1 - q;
    const int s = (i >> (2 * sh)) & 3, rb = (r >> sh) & 1, cb = (c >> sh) & 1;
    double er = 0.0, ei = 0.0;
    if (s == 0) er = rb == cb ? 1.0 : 0.0;
    else if (s == 1) er = rb != cb ? 1.0 : 0.0;
    else if (s == 2) ei = rb != cb ? (rb == 0 ? -1.0 : 1.0) : 0.0;
    else er = rb == cb ? (rb == 0 ? 1.0 : -1.0) : 0.0;
    const double nr = pr * er - pi * ei, ni = pr * ei + pi * er;
    pr = nr;
    pi = ni;
  }
  *re = pr;
  *im = pi;
}

// lower-triangular complex d x d matrix A of the state parameters
__device__ inline void load_cholesky(const double* x, int d, double (*Ar)[4], double (*Ai)[4]) {
  for (int j = 0; j < 4; ++j)
    for (int k = 0; k < 4; ++k) {
      Ar[j][k] = 0.0;
      Ai[j][k] = 0.0;
    }
  int p = d;
  for (int j = 0; j < d; ++j) {
    Ar[j][j] = x[j];
    for (int k = 0; k < j; ++k) {
      Ar[j][k] = x[p];
      Ai[j][k] = x[p + 1];
      p += 2;
    }
  }
}

// rho = A A^dagger / t, t = tr(A A^dagger)
__device__ inline void cholesky_state(const double* x, int d, double (*Ar)[4], double (*Ai)[4], double (*Rr)[4],
                                      double (*Ri)[4], double* t) {
  load_cholesky(x, d, Ar, Ai);
  double tr = 0.0;
  for (int r = 0; r < d; ++r)
    for (int c = 0; c < d; ++c) {
      double sr = 0.0, si = 0.0;
      for (int l = 0; l < d; ++l) {  // A_rl conj(A_cl)
        sr = fma(Ar[r][l], Ar[c][l], sr);
        sr = fma(Ai[r][l], Ai[c][l], sr);
        si = fma(Ai[r][l], Ar[c][l], si);
        si = fma(-Ar[r][l], Ai[c][l], si);
      }
      Rr[r][c] = sr;
      Ri[r][c] = si;
      if (r == c) tr += sr;
    }
  for (int r = 0; r < d; ++r)
    for (int c = 0; c < d; ++c) {
      Rr[r][c] /= tr;
      Ri[r][c] /= tr;
    }
  *t = tr;
}

// LDS of a gate workgroup (doubles)
struct GateLds {
  double* Tr;  // [16][16] T (row j = Pauli label j + 1)
  double* Ti;
  double* Cr;  // [16][16] C = T T^dagger, later Chat
  double* Ci;
  double* hs;  // [16] h by Pauli label (hs[0] = 0)
  double* L;   // [16][ROW] the generator (zero-padded)
  double* LT;  // [16][ROW] its transpose
  double* W[6];  // [16][ROW] work matrices
  double* red;   // [16]
};

__device__ inline GateLds carve_gate(double* base) {
  GateLds s;
  s.Tr = base;
  s.Ti = s.Tr + 256;
  s.Cr = s.Ti + 256;
  s.Ci = s.Cr + 256;
  s.hs = s.Ci + 256;
  s.L = s.hs + 16;
  s.LT = s.L + GATE_STRIDE;
  for (int w = 0; w < 6; ++w) s.W[w] = s.LT + (1 + w) * GATE_STRIDE;
  s.red = s.W[5] + GATE_STRIDE;
  return s;
}
constexpr size_t GATE_LDS_DOUBLES = 4 * 256 + 16 + 8 * (size_t)GATE_STRIDE + 16;

// T and h from the gate's parameters, C = T T^dagger, then L (and L^T) from the
// structure tables.  All 256 threads; ends with a barrier.
template <int D>
__device__ void build_generator(const ParamLaunch& a, const double* tg, const GateLds& s) {
  constexpr int m = D - 1;
  const int tid = threadIdx.x;
  {
    const int j = tid >> 4, k = tid & 15;
    double tr = 0.0, ti = 0.0;
    if (j < m && k < m) {
      if (j == k) {
        tr = tg[m + j];
      } else if (k < j) {
        const int p = 2 * m + 2 * (j * (j - 1) / 2 + k);
        tr = tg[p];
        ti = tg[p + 1];
      }
    }
    s.Tr[tid] = tr;
    s.Ti[tid] = ti;
    if (tid < 16) s.hs[tid] = (tid >= 1 && tid < D) ? tg[tid - 1] : 0.0;
  }
  __syncthreads();
  {
    const int j = tid >> 4, k = tid & 15;
    double cr = 0.0, ci = 0.0;
    if (j < m && k < m) {
      const int lmax = j < k ? j : k;
      for (int l = 0; l <= lmax; ++l) {  // T_jl conj(T_kl)
        const double ar = s.Tr[j * 16 + l], ai = s.Ti[j * 16 + l], br = s.Tr[k * 16 + l], bi = s.Ti[k * 16 + l];
        cr = fma(ar, br, cr);
        cr = fma(ai, bi, cr);
        ci = fma(ai, br, ci);
        ci = fma(-ar, bi, ci);
      }
    }
    s.Cr[tid] = cr;
    s.Ci[tid] = ci;
  }
  __syncthreads();
  {
    const int r = tid >> 4, c = tid & 15;
    double l = 0.0;
    if (r < D && c < D) {
      const int rc = r ^ c;
      if (rc) l = s.hs[rc] * a.ty[r * D + c];
      const double* zr = a.tzr + (size_t)(r * D + c) * D;
      const double* zi = a.tzi + (size_t)(r * D + c) * D;
      for (int j = 1; j < D; ++j) {
        const int k = rc ^ j;
        if (k == 0) continue;
        const double cr = s.Cr[(j - 1) * 16 + (k - 1)], ci = s.Ci[(j - 1) * 16 + (k - 1)];
        l = fma(cr, zr[j], l);
        l = fma(-ci, zi[j], l);
      }
    }
    s.L[r * ROW + c] = l;
    s.LT[c * ROW + r] = l;
    if (c < ROW - 16) {
      s.L[r * ROW + 16 + c] = 0.0;
      s.LT[r * ROW + 16 + c] = 0.0;
    }
  }
  __syncthreads();
}

// Register result of A B (16 x 16, LDS, stride ROW) on the matrix cores: lane l
// holds C[4v + (l >> 4)][l & 15] in acc[v].
__device__ inline d4 mm_acc(const double* A, const double* B, d4 acc, int lane) {
  const int i = lane & 15, t = lane >> 4;
  double x[4], y[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    x[k] = A[i * ROW + 4 * k + t];
    y[k] = B[(4 * k + t) * ROW + i];
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(x[k], y[k], acc, 0, 0, 0);
  return acc;
}

__device__ inline void store_acc(double* C, d4 acc, int lane) {
  const int i = lane & 15, t = lane >> 4;
#pragma unroll
  for (int v = 0; v < 4; ++v) C[(4 * v + t) * ROW + i] = acc[v];
}

// s >= 0 with max(||L||_1, ||L||_inf) / 2^s <= 1/2, by the lanes of one wave
__device__ inline int scaling_of(const double* L, int lane) {
  const int i = lane & 15;
  double cs = 0.0, rs = 0.0;
  for (int r = 0; r < 16; ++r) {
    cs += fabs(L[r * ROW + i]);
    rs += fabs(L[i * ROW + r]);
  }
  double m = fmax(cs, rs);
#pragma unroll
  for (int o = 1; o < 16; o <<= 1) m = fmax(m, __shfl_xor(m, o, 16));
  int s = 0;
  while (m > 0.5 && s < 64) {
    m *= 0.5;
    ++s;
  }
  return __builtin_amdgcn_readfirstlane(s);
}

// X <- scale * src (entrywise; zero padding kept), one wave
__device__ inline void scaled_copy(double* X, const double* src, double scale, int lane) {
  for (int x = lane; x < 16 * ROW; x += 64) X[x] = src[x] * scale;
}

// exp(L) (L in LDS, padded) into the returned buffer among W[0..1]; one wave.
__device__ double* expm_wave(const GateLds& s, int lane) {
  const int i = lane & 15, t = lane >> 4;
  const int sc = scaling_of(s.L, lane);
  double* X = s.W[2];
  scaled_copy(X, s.L, ldexp(1.0, -sc), lane);
  double* P = s.W[0];
  double* Pn = s.W[1];
  for (int x = lane; x < 16 * ROW; x += 64) P[x] = (x / ROW == x % ROW) ? 1.0 : 0.0;
  wave_sync();
  for (int k = TAYLOR; k >= 1; --k) {
    const d4 q = mm_acc(X, P, d4{0.0, 0.0, 0.0, 0.0}, lane);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = 4 * v + t;
      Pn[r * ROW + i] = (r == i ? 1.0 : 0.0) + q[v] / (double)k;
    }
    wave_sync();
    double* tmp = P;
    P = Pn;
    Pn = tmp;
  }
  for (int e = 0; e < sc; ++e) {
    store_acc(Pn, mm_acc(P, P, d4{0.0, 0.0, 0.0, 0.0}, lane), lane);
    wave_sync();
    double* tmp = P;
    P = Pn;
    Pn = tmp;
  }
  return P;
}

template <int D>
__global__ __launch_bounds__(256) void cptp_forward_kernel(const ParamLaunch a) {
  extern __shared__ double lds_raw[];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int M = a.M, d = a.d;
  const double* eth = a.theta + D;
  const double* gth = eth + (int64_t)(M - 1) * D;
  if (blockIdx.x == a.K) {  // state and effects
    if (tid < D) {
      double Ar[4][4], Ai[4][4], Rr[4][4], Ri[4][4], t;
      cholesky_state(a.theta, d, Ar, Ai, Rr, Ri, &t);
      double acc = 0.0;  // Re tr(P_i rho)
      for (int r = 0; r < d; ++r)
        for (int c = 0; c < d; ++c) {
          double pr, pi;
          pauli_entry(tid, r, c, a.n, &pr, &pi);
          acc = fma(pr, Rr[c][r], acc);
          acc = fma(-pi, Ri[c][r], acc);
        }
      a.rho[tid] = acc * a.inv_sqrt_d;
    }
    for (int x = tid; x < M * D; x += blockDim.x) {
      const int mm = x / D, c = x % D;
      double v;
      if (mm < M - 1) {
        v = eth[x];
      } else {
        v = c == 0 ? a.sqrt_d : 0.0;
        for (int q = 0; q < M - 1; ++q) v = v - eth[q * D + c];
      }
      a.E[x] = v;
    }
    return;
  }
  const int g = blockIdx.x;
  const GateLds s = carve_gate(lds_raw);
  build_generator<D>(a, gth + (int64_t)g * D * (D - 1), s);
  // target into W[3] (zero-padded)
  double* G0 = s.W[3];
  {
    const int r = tid >> 4, c = tid & 15;
    G0[r * ROW + c] = (r < D && c < D) ? a.targets[((int64_t)g * D + r) * D + c] : 0.0;
    if (c < ROW - 16) G0[r * ROW + 16 + c] = 0.0;
  }
  __syncthreads();
  if (wave == 0) {
    const double* Ex = expm_wave(s, lane);
    const d4 acc = mm_acc(Ex, G0, d4{0.0, 0.0, 0.0, 0.0}, lane);
    const int i = lane & 15, t = lane >> 4;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = 4 * v + t;
      if (r < D && i < D) a.G[((int64_t)g * D + r) * D + i] = acc[v];
    }
  }
}

template <int D>
__global__ __launch_bounds__(256) void cptp_backward_kernel(const ParamLaunch a) {
  extern __shared__ double lds_raw[];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int M = a.M, d = a.d;
  const double* gr = a.grad_full;
  const double* ge = gr + D;
  const double* gg = ge + (int64_t)M * D;
  const int64_t e_off = D, g_off = D + (int64_t)(M - 1) * D;
  if (blockIdx.x == a.K) {
    if (tid < D) {
      // Q = sum_i gr_i P_i / sqrt(d); Q' = (Q - tr(Q rho)) / t; Gamma = 2 Q' A
      double Ar[4][4], Ai[4][4], Rr[4][4], Ri[4][4], t;
      cholesky_state(a.theta, d, Ar, Ai, Rr, Ri, &t);
      double Qr[4][4], Qi[4][4];
      for (int r = 0; r < d; ++r)
        for (int c = 0; c < d; ++c) {
          double sr = 0.0, si = 0.0;
          for (int i = 0; i < D; ++i) {
            double pr, pi;
            pauli_entry(i, r, c, a.n, &pr, &pi);
            sr = fma(gr[i], pr, sr);
            si = fma(gr[i], pi, si);
          }
          Qr[r][c] = sr * a.inv_sqrt_d;
          Qi[r][c] = si * a.inv_sqrt_d;
        }
      double q = 0.0;  // Re tr(Q rho)
      for (int r = 0; r < d; ++r)
        for (int c = 0; c < d; ++c) {
          q = fma(Qr[r][c], Rr[c][r], q);
          q = fma(-Qi[r][c], Ri[c][r], q);
        }
      for (int r = 0; r < d; ++r) {
        Qr[r][r] -= q;
        for (int c = 0; c < d; ++c) {
          Qr[r][c] /= t;
          Qi[r][c] /= t;
        }
      }
      // this thread's parameter: a diagonal entry or one half of a pair
      int j = 0, l = 0, part = 0;
      if (tid < d) {
        j = l = tid;
      } else {
        const int p = (tid - d) >> 1;
        part = (tid - d) & 1;
        j = 1;
        while ((j * (j + 1)) / 2 <= p) ++j;
        l = p - (j * (j - 1)) / 2;
      }
      double gre = 0.0, gim = 0.0;  // (2 Q' A)_jl
      for (int k = 0; k < d; ++k) {
        gre = fma(Qr[j][k], Ar[k][l], gre);
        gre = fma(-Qi[j][k], Ai[k][l], gre);
        gim = fma(Qr[j][k], Ai[k][l], gim);
        gim = fma(Qi[j][k], Ar[k][l], gim);
      }
      a.grad_theta[tid] = 2.0 * (part ? gim : gre);
    }
    for (int x = tid; x < (M - 1) * D; x += blockDim.x) a.grad_theta[e_off + x] = ge[x] - ge[(M - 1) * D + x % D];
    return;
  }
  const int g = blockIdx.x;
  const GateLds s = carve_gate(lds_raw);
  build_generator<D>(a, a.theta + g_off + (int64_t)g * D * (D - 1), s);
  // W[3] = dF/dG, W[4] = G0^T
  {
    const int r = tid >> 4, c = tid & 15;
    const bool in = r < D && c < D;
    s.W[3][r * ROW + c] = in ? gg[((int64_t)g * D + r) * D + c] : 0.0;
    s.W[4][c * ROW + r] = in ? a.targets[((int64_t)g * D + r) * D + c] : 0.0;
    if (c < ROW - 16) {
      s.W[3][r * ROW + 16 + c] = 0.0;
      s.W[4][r * ROW + 16 + c] = 0.0;
    }
  }
  __syncthreads();
  if (wave == 0) {
    const int i = lane & 15, t = lane >> 4;
    const int sc = scaling_of(s.L, lane);
    const double f = ldexp(1.0, -sc);
    // A = L^T / 2^s into W[2]; Xs = (dF/dG G0^T) / 2^s into W[5]
    scaled_copy(s.W[2], s.LT, f, lane);
    {
      const d4 x = mm_acc(s.W[3], s.W[4], d4{0.0, 0.0, 0.0, 0.0}, lane);
      wave_sync();
#pragma unroll
      for (int v = 0; v < 4; ++v) s.W[5][(4 * v + t) * ROW + i] = x[v] * f;
    }
    // block Horner: P11 in W[0] / W[1], P12 in W[3] / W[4] (dF/dG and G0^T are done)
    double* P11 = s.W[0];
    double* N11 = s.W[1];
    double* P12 = s.W[3];
    double* N12 = s.W[4];
    for (int x = lane; x < 16 * ROW; x += 64) {
      P11[x] = (x / ROW == x % ROW) ? 1.0 : 0.0;
      P12[x] = 0.0;
    }
    wave_sync();
    const double* Am = s.W[2];
    const double* Xs = s.W[5];
    for (int k = TAYLOR; k >= 1; --k) {
      const d4 q11 = mm_acc(Am, P11, d4{0.0, 0.0, 0.0, 0.0}, lane);
      const d4 q12 = mm_acc(Xs, P11, mm_acc(Am, P12, d4{0.0, 0.0, 0.0, 0.0}, lane), lane);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = 4 * v + t;
        N11[r * ROW + i] = (r == i ? 1.0 : 0.0) + q11[v] / (double)k;
        N12[r * ROW + i] = q12[v] / (double)k;
      }
      wave_sync();
      double* tmp = P11;
      P11 = N11;
      N11 = tmp;
      tmp = P12;
      P12 = N12;
      N12 = tmp;
    }
    for (int e = 0; e < sc; ++e) {
      const d4 q11 = mm_acc(P11, P11, d4{0.0, 0.0, 0.0, 0.0}, lane);
      const d4 q12 = mm_acc(P12, P11, mm_acc(P11, P12, d4{0.0, 0.0, 0.0, 0.0}, lane), lane);
      store_acc(N11, q11, lane);
      store_acc(N12, q12, lane);
      wave_sync();
      double* tmp = P11;
      P11 = N11;
      N11 = tmp;
      tmp = P12;
      P12 = N12;
      N12 = tmp;
    }
    // dF/dL into L's slot
    for (int x = lane; x < 16 * ROW; x += 64) s.L[x] = P12[x];
  }
  __syncthreads();
  const double* Lb = s.L;
  double* out = a.grad_theta + g_off + (int64_t)g * D * (D - 1);
  constexpr int m = D - 1;
  // dF/dh_k = sum_a dF/dL[a][a^k] y[a][a^k]
  if (tid < m) {
    const int k = tid + 1;
    double v = 0.0;
    for (int r = 0; r < D; ++r) v = fma(Lb[r * ROW + (r ^ k)], a.ty[r * D + (r ^ k)], v);
    out[tid] = v;
  }
  // Chat_jk = sum_a dF/dL[a][b] z[a][b][j], b = a ^ j ^ k  (into Cr / Ci)
  {
    const int j = tid >> 4, k = tid & 15;
    double cr = 0.0, ci = 0.0;
    if (j < m && k < m) {
      const int jl = j + 1, kl = k + 1;
      for (int r = 0; r < D; ++r) {
        const int c = r ^ jl ^ kl;
        const size_t x = (size_t)(r * D + c) * D + jl;
        cr = fma(Lb[r * ROW + c], a.tzr[x], cr);
        ci = fma(Lb[r * ROW + c], a.tzi[x], ci);
      }
    }
    __syncthreads();  // C is no longer needed
    s.Cr[tid] = cr;
    s.Ci[tid] = ci;
  }
  __syncthreads();
  // Gamma_jl = sum_{k >= l} (conj(Chat_jk) + Chat_kj) T_kl for l <= j
  {
    const int j = tid >> 4, l = tid & 15;
    if (j < m && l <= j) {
      double gre = 0.0, gim = 0.0;
      for (int k = l; k < m; ++k) {
        const double wr = s.Cr[j * 16 + k] + s.Cr[k * 16 + j];
        const double wi = s.Ci[k * 16 + j] - s.Ci[j * 16 + k];
        const double tr = s.Tr[k * 16 + l], ti = s.Ti[k * 16 + l];
        gre = fma(wr, tr, gre);
        gre = fma(-wi, ti, gre);
        gim = fma(wr, ti, gim);
        gim = fma(wi, tr, gim);
      }
      if (l == j) {
        out[m + j] = gre;
      } else {
        const int p = 2 * m + 2 * (j * (j - 1) / 2 + l);
        out[p] = gre;
        out[p + 1] = gim;
      }
    }
  }
}

}  // namespace

static int tp_blocks(int64_t n) {
  const int64_t b = (n + 255) / 256;
  return (int)(b < 4096 ? (b > 0 ? b : 1) : 4096);
}

hipError_t launch_param_forward(const ParamLaunch& a, hipStream_t stream) {
  if (a.mode == 1) {
    const int64_t n = a.D + (int64_t)a.M * a.D + (int64_t)a.K * a.D * a.D;
    gst_launch(tp_forward_kernel, dim3(tp_blocks(n)), dim3(256), 0, stream, a);
    return hipGetLastError();
  }
  if (a.mode != 2 || a.d > 4) return hipErrorInvalidValue;
  const size_t bytes = GATE_LDS_DOUBLES * 8;
  if (a.D == 16)
    gst_launch(cptp_forward_kernel<16>, dim3(a.K + 1), dim3(256), bytes, stream, a);
  else
    gst_launch(cptp_forward_kernel<4>, dim3(a.K + 1), dim3(256), bytes, stream, a);
  return hipGetLastError();
}

hipError_t launch_param_backward(const ParamLaunch& a, hipStream_t stream) {
  if (a.mode == 1) {
    const int64_t n = (a.D - 1) + (int64_t)(a.M - 1) * a.D + (int64_t)a.K * a.D * (a.D - 1);
    gst_launch(tp_backward_kernel, dim3(tp_blocks(n)), dim3(256), 0, stream, a);
    return hipGetLastError();
  }
  if (a.mode != 2 || a.d > 4) return hipErrorInvalidValue;
  const size_t bytes = GATE_LDS_DOUBLES * 8;
  if (a.D == 16)
    gst_launch(cptp_backward_kernel<16>, dim3(a.K + 1), dim3(256), bytes, stream, a);
  else
    gst_launch(cptp_backward_kernel<4>, dim3(a.K + 1), dim3(256), bytes, stream, a);
  return hipGetLastError();
}

}  // namespace gst
