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
// dF/dT = (conj(Chat) + Chat^T) T with Chat_jk = sum_ab dF/dL_ab z_j(a, b).
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

// lower-triangular complex d x d matrix A of the state parameters (d fixed at
// compile time, loops unrolled: the small matrices stay in registers)
template <int d>
__device__ inline void load_cholesky(const double* x, double (&Ar)[d][d], double (&Ai)[d][d]) {
#pragma unroll
  for (int j = 0; j < d; ++j)
#pragma unroll
    for (int k = 0; k < d; ++k) {
      Ar[j][k] = 0.0;
      Ai[j][k] = 0.0;
    }
#pragma unroll
  for (int j = 0; j < d; ++j) {
    Ar[j][j] = x[j];
#pragma unroll
    for (int k = 0; k < j; ++k) {
      const int p = d + 2 * (j * (j - 1) / 2 + k);
      Ar[j][k] = x[p];
      Ai[j][k] = x[p + 1];
    }
  }
}

// rho = A A^dagger / t, t = tr(A A^dagger)
template <int d>
__device__ inline void cholesky_state(const double* x, double (&Ar)[d][d], double (&Ai)[d][d], double (&Rr)[d][d],
                                      double (&Ri)[d][d], double* t) {
  load_cholesky<d>(x, Ar, Ai);
  double tr = 0.0;
#pragma unroll
  for (int r = 0; r < d; ++r)
#pragma unroll
    for (int c = 0; c < d; ++c) {
      double sr = 0.0, si = 0.0;
#pragma unroll
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
#pragma unroll
  for (int r = 0; r < d; ++r)
#pragma unroll
    for (int c = 0; c < d; ++c) {
      Rr[r][c] /= tr;
      Ri[r][c] /= tr;
    }
  *t = tr;
}

// state coordinates v_i = Re tr(P_i rho) / sqrt(d) and the effects (TP form)
template <int D, int d>
__device__ void spam_forward(const ParamLaunch& a) {
  const int tid = threadIdx.x, M = a.M;
  const double* eth = a.theta + D;
  if (tid < D) {
    double Ar[d][d], Ai[d][d], Rr[d][d], Ri[d][d], t;
    cholesky_state<d>(a.theta, Ar, Ai, Rr, Ri, &t);
    double acc = 0.0;
#pragma unroll
    for (int r = 0; r < d; ++r)
#pragma unroll
      for (int c = 0; c < d; ++c) {
        double pr, pi;
        pauli_entry(tid, r, c, d == 2 ? 1 : 2, &pr, &pi);
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
}

// Q = sum_i gr_i P_i / sqrt(d); Q' = (Q - tr(Q rho)) / t; dF/dA = 2 Q' A (entries
// below the diagonal as real and imaginary parts); the effects' differences
template <int D, int d>
__device__ void spam_backward(const ParamLaunch& a) {
  const int tid = threadIdx.x, M = a.M;
  const double* gr = a.grad_full;
  const double* ge = gr + D;
  if (tid < D) {
    double Ar[d][d], Ai[d][d], Rr[d][d], Ri[d][d], t;
    cholesky_state<d>(a.theta, Ar, Ai, Rr, Ri, &t);
    double g[D];
#pragma unroll
    for (int i = 0; i < D; ++i) g[i] = gr[i];
    double Qr[d][d], Qi[d][d];
#pragma unroll
    for (int r = 0; r < d; ++r)
#pragma unroll
      for (int c = 0; c < d; ++c) {
        double sr = 0.0, si = 0.0;
#pragma unroll
        for (int i = 0; i < D; ++i) {
          double pr, pi;
          pauli_entry(i, r, c, d == 2 ? 1 : 2, &pr, &pi);
          sr = fma(g[i], pr, sr);
          si = fma(g[i], pi, si);
        }
        Qr[r][c] = sr * a.inv_sqrt_d;
        Qi[r][c] = si * a.inv_sqrt_d;
      }
    double q = 0.0;  // Re tr(Q rho)
#pragma unroll
    for (int r = 0; r < d; ++r)
#pragma unroll
      for (int c = 0; c < d; ++c) {
        q = fma(Qr[r][c], Rr[c][r], q);
        q = fma(-Qi[r][c], Ri[c][r], q);
      }
#pragma unroll
    for (int r = 0; r < d; ++r) {
      Qr[r][r] -= q;
#pragma unroll
      for (int c = 0; c < d; ++c) {
        Qr[r][c] /= t;
        Qi[r][c] /= t;
      }
    }
    double out = 0.0;
#pragma unroll
    for (int j = 0; j < d; ++j)
#pragma unroll
      for (int l = 0; l <= j; ++l) {
        double gre = 0.0, gim = 0.0;  // (Q' A)_jl
#pragma unroll
        for (int k = 0; k < d; ++k) {
          gre = fma(Qr[j][k], Ar[k][l], gre);
          gre = fma(-Qi[j][k], Ai[k][l], gre);
          gim = fma(Qr[j][k], Ai[k][l], gim);
          gim = fma(Qi[j][k], Ar[k][l], gim);
        }
        const int p = d + 2 * (j * (j - 1) / 2 + l);
        if (l == j && tid == j) out = 2.0 * gre;
        if (l < j && tid == p) out = 2.0 * gre;
        if (l < j && tid == p + 1) out = 2.0 * gim;
      }
    a.grad_theta[tid] = out;
  }
  for (int x = tid; x < (M - 1) * D; x += blockDim.x) a.grad_theta[D + x] = ge[x] - ge[(M - 1) * D + x % D];
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
      // all table loads in flight together (z by j, then entry: coalesced)
      double zr[D], zi[D];
#pragma unroll
      for (int j = 1; j < D; ++j) {
        zr[j] = a.tzr[(size_t)j * D * D + r * D + c];
        zi[j] = a.tzi[(size_t)j * D * D + r * D + c];
      }
      const double y = a.ty[r * D + c];
      if (rc) l = s.hs[rc] * y;
      // the term j = r^c has a zero coefficient (k = 0): it adds exact zeros
#pragma unroll
      for (int j = 1; j < D; ++j) {
        const int k = rc ^ j;
        const int kk = k ? k - 1 : 0;
        const double cr = s.Cr[(j - 1) * 16 + kk], ci = s.Ci[(j - 1) * 16 + kk];
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

// Operands of the 16x16x4 FP64 MFMA in registers.  The product's layout (lane l
// holds C[4v + (l >> 4)][l & 15] in register v) is the layout of the right
// operand B (step k reads B[4k + (l >> 4)][l & 15]), so a chain of left
// multiplications P <- X P keeps P in registers; the left operand (lane l:
// A[l & 15][4k + (l >> 4)]) is loaded from LDS once.
struct Frag {
  double v[4];
};

__device__ inline Frag load_left(const double* A, double scale, int lane) {
  const int i = lane & 15, t = lane >> 4;
  Frag f;
#pragma unroll
  for (int k = 0; k < 4; ++k) f.v[k] = A[i * ROW + 4 * k + t] * scale;
  return f;
}

__device__ inline d4 mfma_left(const Frag& A, const Frag& B, d4 acc) {
#pragma unroll
  for (int k = 0; k < 4; ++k) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(A.v[k], B.v[k], acc, 0, 0, 0);
  return acc;
}

__device__ inline void store_frag(double* C, const Frag& f, int lane) {
  const int i = lane & 15, t = lane >> 4;
#pragma unroll
  for (int v = 0; v < 4; ++v) C[(4 * v + t) * ROW + i] = f.v[v];
}

__device__ inline Frag identity_frag(int lane) {
  const int i = lane & 15, t = lane >> 4;
  Frag f;
#pragma unroll
  for (int v = 0; v < 4; ++v) f.v[v] = (4 * v + t == i) ? 1.0 : 0.0;
  return f;
}

// exp(L) (L in LDS, padded) as a right-operand fragment; one wave.  Horner's
// rule for the Taylor polynomial of X = L / 2^s runs in registers; the s
// squarings go through the LDS buffer W (P is needed as a left operand there).
__device__ Frag expm_wave(const double* L, double* W, int lane) {
  const int i = lane & 15, t = lane >> 4;
  const int sc = scaling_of(L, lane);
  const Frag X = load_left(L, ldexp(1.0, -sc), lane);
  Frag P = identity_frag(lane);
  for (int k = TAYLOR; k >= 1; --k) {
    const double rk = 1.0 / (double)k;  // uniform: off the chain of dependent products
    const d4 q = mfma_left(X, P, d4{0.0, 0.0, 0.0, 0.0});
#pragma unroll
    for (int v = 0; v < 4; ++v) P.v[v] = fma(q[v], rk, 4 * v + t == i ? 1.0 : 0.0);
  }
  for (int e = 0; e < sc; ++e) {
    store_frag(W, P, lane);
    wave_sync();
    const d4 q = mfma_left(load_left(W, 1.0, lane), P, d4{0.0, 0.0, 0.0, 0.0});
    wave_sync();  // W is rewritten by the next squaring
#pragma unroll
    for (int v = 0; v < 4; ++v) P.v[v] = q[v];
  }
  return P;
}

template <int D>
__global__ __launch_bounds__(256) void cptp_forward_kernel(const ParamLaunch a) {
  extern __shared__ double lds_raw[];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const double* gth = a.theta + D + (int64_t)(a.M - 1) * D;
  if (blockIdx.x == a.K) {  // state and effects
    spam_forward<D, D == 16 ? 4 : 2>(a);
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
    const Frag Ex = expm_wave(s.L, s.W[0], lane);
    store_frag(s.W[1], Ex, lane);
    wave_sync();
    const d4 acc = mm_acc(s.W[1], G0, d4{0.0, 0.0, 0.0, 0.0}, lane);
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
  const double* gg = a.grad_full + D + (int64_t)a.M * D;
  const int64_t g_off = D + (int64_t)(a.M - 1) * D;
  if (blockIdx.x == a.K) {  // state and effects
    spam_backward<D, D == 16 ? 4 : 2>(a);
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
    // X = dF/dG G0^T into W[5] (a left operand below)
    store_acc(s.W[5], mm_acc(s.W[3], s.W[4], d4{0.0, 0.0, 0.0, 0.0}, lane), lane);
    wave_sync();
    const Frag A = load_left(s.LT, f, lane);   // L^T / 2^s
    const Frag Xs = load_left(s.W[5], f, lane);
    // block Horner: [[P11, P12], [0, P11]] <- I + [[A, Xs], [0, A]] [[P11, P12], [0, P11]] / k
    Frag P11 = identity_frag(lane), P12;
#pragma unroll
    for (int v = 0; v < 4; ++v) P12.v[v] = 0.0;
    for (int k = TAYLOR; k >= 1; --k) {
      const double rk = 1.0 / (double)k;
      const d4 q11 = mfma_left(A, P11, d4{0.0, 0.0, 0.0, 0.0});
      const d4 q12 = mfma_left(Xs, P11, mfma_left(A, P12, d4{0.0, 0.0, 0.0, 0.0}));
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        P11.v[v] = fma(q11[v], rk, 4 * v + t == i ? 1.0 : 0.0);
        P12.v[v] = q12[v] * rk;
      }
    }
    // squarings: P11 <- P11 P11, P12 <- P11 P12 + P12 P11
    for (int e = 0; e < sc; ++e) {
      store_frag(s.W[0], P11, lane);
      store_frag(s.W[1], P12, lane);
      wave_sync();
      const Frag L11 = load_left(s.W[0], 1.0, lane), L12 = load_left(s.W[1], 1.0, lane);
      wave_sync();
      const d4 q11 = mfma_left(L11, P11, d4{0.0, 0.0, 0.0, 0.0});
      const d4 q12 = mfma_left(L12, P11, mfma_left(L11, P12, d4{0.0, 0.0, 0.0, 0.0}));
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        P11.v[v] = q11[v];
        P12.v[v] = q12[v];
      }
    }
    // dF/dL into L's slot
    store_frag(s.L, P12, lane);
  }
  __syncthreads();
  const double* Lb = s.L;
  double* out = a.grad_theta + g_off + (int64_t)g * D * (D - 1);
  constexpr int m = D - 1;
  // dF/dh_k = sum_a dF/dL[a][a^k] y[a][a^k]
  if (tid < m) {
    const int k = tid + 1;
    double y[D];
#pragma unroll
    for (int r = 0; r < D; ++r) y[r] = a.ty[r * D + (r ^ k)];
    double v = 0.0;
#pragma unroll
    for (int r = 0; r < D; ++r) v = fma(Lb[r * ROW + (r ^ k)], y[r], v);
    out[tid] = v;
  }
  // Chat_jk = sum_a dF/dL[a][b] z[j][a][b], b = a ^ j ^ k  (into Cr / Ci)
  {
    const int j = tid >> 4, k = tid & 15;
    double cr = 0.0, ci = 0.0;
    if (j < m && k < m) {
      const int jl = j + 1, kl = k + 1;
      double zr[D], zi[D];
#pragma unroll
      for (int r = 0; r < D; ++r) {
        const size_t x = (size_t)jl * D * D + r * D + (r ^ jl ^ kl);
        zr[r] = a.tzr[x];
        zi[r] = a.tzi[x];
      }
#pragma unroll
      for (int r = 0; r < D; ++r) {
        const double lb = Lb[r * ROW + (r ^ jl ^ kl)];
        cr = fma(lb, zr[r], cr);
        ci = fma(lb, zi[r], ci);
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
