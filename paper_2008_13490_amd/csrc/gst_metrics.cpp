// Post-fit metrics of the estimates: thesis Sec. 6.1 (average gate fidelity,
// App. G), App. H (diamond distance of unitaries), App. J (gate
// decompositions and effective Hamiltonians).
#include "gst_metrics.h"

#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "gst_fit_core.h"
#include "gst_param_tables.h"

namespace gst {

double avg_gate_fidelity(int D, const double* R, const double* RU) {
  double tr = 0.0;  // Tr(RU^T R) = sum_ab RU_ab R_ab
  for (int x = 0; x < D * D; ++x) tr += RU[x] * R[x];
  const double N = sqrt((double)D);
  return (tr + N * R[0]) / (N * (N + 1.0));
}

namespace {

// cyclic Jacobi for the real symmetric n x n matrix A (destroyed): eigenvectors
// in the columns of V
bool jacobi_sym(int n, std::vector<double>& A, std::vector<double>& V) {
  V.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        const double a = A[(size_t)i * n + j] * A[(size_t)i * n + j];
        tot += a;
        if (i != j) off += a;
      }
    if (off <= 1e-30 * tot || off == 0.0) return true;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = A[(size_t)p * n + q];
        if (apq == 0.0) continue;
        const double app = A[(size_t)p * n + p], aqq = A[(size_t)q * n + q];
        const double theta = (aqq - app) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {  // columns p, q
          const double akp = A[(size_t)k * n + p], akq = A[(size_t)k * n + q];
          A[(size_t)k * n + p] = c * akp - s * akq;
          A[(size_t)k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {  // rows p, q
          const double apk = A[(size_t)p * n + k], aqk = A[(size_t)q * n + k];
          A[(size_t)p * n + k] = c * apk - s * aqk;
          A[(size_t)q * n + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          const double vkp = V[(size_t)k * n + p], vkq = V[(size_t)k * n + q];
          V[(size_t)k * n + p] = c * vkp - s * vkq;
          V[(size_t)k * n + q] = s * vkp + c * vkq;
        }
      }
  }
  return false;
}

// i-k-j order: each C[i][j] still accumulates k in ascending order, and the
// inner loop runs over contiguous rows
void mm(int n, const double* A, const double* B, double* C) {
  for (int i = 0; i < n; ++i) {
    double* c = C + (size_t)i * n;
    for (int j = 0; j < n; ++j) c[j] = 0.0;
    for (int k = 0; k < n; ++k) {
      const double a = A[(size_t)i * n + k];
      const double* b = B + (size_t)k * n;
      for (int j = 0; j < n; ++j) c[j] += a * b[j];
    }
  }
}

double fro(int n, const double* A) {
  double s = 0.0;
  for (int x = 0; x < n * n; ++x) s += A[x] * A[x];
  return sqrt(s);
}

}  // namespace

bool unitary_eigenvalues(int d, const double* W, double* re, double* im) {
  // C = (W + W^dagger)/2 + c (W - W^dagger)/(2i): Hermitian, with W's eigenvectors
  const double c = 0.6180339887498949;
  std::vector<double> Cr((size_t)d * d), Ci((size_t)d * d);
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j) {
      const double wr = W[2 * (i * d + j)], wi = W[2 * (i * d + j) + 1];
      const double tr = W[2 * (j * d + i)], ti = -W[2 * (j * d + i) + 1];  // (W^dagger)_ij
      // (W + W^dagger)/2
      double hr = 0.5 * (wr + tr), hi = 0.5 * (wi + ti);
      // (W - W^dagger)/(2i) = -i (W - W^dagger)/2
      const double dr = 0.5 * (wr - tr), di = 0.5 * (wi - ti);
      hr += c * di;
      hi += -c * dr;
      Cr[(size_t)i * d + j] = hr;
      Ci[(size_t)i * d + j] = hi;
    }
  const int n = 2 * d;
  std::vector<double> S((size_t)n * n), V;
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j) {
      S[(size_t)i * n + j] = Cr[(size_t)i * d + j];
      S[(size_t)i * n + d + j] = -Ci[(size_t)i * d + j];
      S[(size_t)(d + i) * n + j] = Ci[(size_t)i * d + j];
      S[(size_t)(d + i) * n + d + j] = Cr[(size_t)i * d + j];
    }
  if (!jacobi_sym(n, S, V)) return false;
  for (int col = 0; col < n; ++col) {
    // v = x + i y; lambda = v^dagger W v / v^dagger v
    double nr = 0.0, ni = 0.0, den = 0.0;
    for (int i = 0; i < d; ++i) {
      const double xi = V[(size_t)i * n + col], yi = V[(size_t)(d + i) * n + col];
      den += xi * xi + yi * yi;
      double wvr = 0.0, wvi = 0.0;  // (W v)_i
      for (int j = 0; j < d; ++j) {
        const double xj = V[(size_t)j * n + col], yj = V[(size_t)(d + j) * n + col];
        const double wr = W[2 * (i * d + j)], wi = W[2 * (i * d + j) + 1];
        wvr += wr * xj - wi * yj;
        wvi += wr * yj + wi * xj;
      }
      nr += xi * wvr + yi * wvi;  // conj(v_i) (W v)_i
      ni += xi * wvi - yi * wvr;
    }
    re[col] = nr / den;
    im[col] = ni / den;
  }
  return true;
}

double diamond_unitary(int d, const double* U, const double* V) {
  // W = U^dagger V
  std::vector<double> W((size_t)2 * d * d, 0.0);
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j) {
      double sr = 0.0, si = 0.0;
      for (int k = 0; k < d; ++k) {
        const double ur = U[2 * (k * d + i)], ui = -U[2 * (k * d + i) + 1];  // conj(U_ki)
        const double vr = V[2 * (k * d + j)], vi = V[2 * (k * d + j) + 1];
        sr += ur * vr - ui * vi;
        si += ur * vi + ui * vr;
      }
      W[2 * (i * d + j)] = sr;
      W[2 * (i * d + j) + 1] = si;
    }
  std::vector<double> lr(2 * d), li(2 * d);
  if (!unitary_eigenvalues(d, W.data(), lr.data(), li.data())) return -1.0;
  const int m = 2 * d;
  std::vector<double> ph(m);
  const double two_pi = 2.0 * M_PI;
  for (int x = 0; x < m; ++x) {
    double a = atan2(li[x], lr[x]);
    if (a < 0) a += two_pi;
    ph[x] = a;
  }
  std::sort(ph.begin(), ph.end());
  bool inside = true;
  for (int x = 0; x < m; ++x) {
    const double gap = x + 1 < m ? ph[x + 1] - ph[x] : ph[0] + two_pi - ph[x];
    if (gap > M_PI) inside = false;
  }
  if (inside) return 1.0;
  double best = 0.0;
  for (int j = 0; j < m; ++j)
    for (int k = j + 1; k < m; ++k) best = std::max(best, hypot(lr[j] - lr[k], li[j] - li[k]));
  return 0.5 * best;
}

void expm_real(int D, const double* L, double* E) {
  const size_t DD = (size_t)D * D;
  double nrm = 0.0;
  for (int i = 0; i < D; ++i) {
    double r = 0.0;
    for (int j = 0; j < D; ++j) r += fabs(L[(size_t)i * D + j]);
    nrm = std::max(nrm, r);
  }
  int s = 0;
  while (nrm > 0.5 && s < 64) {
    nrm *= 0.5;
    ++s;
  }
  const double f = ldexp(1.0, -s);
  std::vector<double> X(DD), P(DD, 0.0), T(DD);
  for (size_t x = 0; x < DD; ++x) X[x] = L[x] * f;
  for (int i = 0; i < D; ++i) P[(size_t)i * D + i] = 1.0;
  for (int k = 18; k >= 1; --k) {  // Horner: P = 1 + X P / k
    mm(D, X.data(), P.data(), T.data());
    for (size_t x = 0; x < DD; ++x) P[x] = T[x] / k;
    for (int i = 0; i < D; ++i) P[(size_t)i * D + i] += 1.0;
  }
  for (int e = 0; e < s; ++e) {
    mm(D, P.data(), P.data(), T.data());
    P.swap(T);
  }
  memcpy(E, P.data(), DD * sizeof(double));
}

bool logm_real(int D, const double* G, double* L) {
  const size_t DD = (size_t)D * D;
  std::vector<double> A(G, G + DD), Y(DD), Z(DD), Yi(DD), Zi(DD), X(DD), P(DD), T(DD), S(DD, 0.0);
  int k = 0;
  auto dist_to_one = [&](const std::vector<double>& M) {
    double s = 0.0;
    for (int i = 0; i < D; ++i)
      for (int j = 0; j < D; ++j) {
        const double v = M[(size_t)i * D + j] - (i == j ? 1.0 : 0.0);
        s += v * v;
      }
    return sqrt(s);
  };
  while (dist_to_one(A) > 0.25) {
    if (++k > 40) return false;
    // Denman-Beavers: Y -> A^(1/2), Z -> A^(-1/2)
    Y = A;
    std::fill(Z.begin(), Z.end(), 0.0);
    for (int i = 0; i < D; ++i) Z[(size_t)i * D + i] = 1.0;
    bool conv = false;
    for (int it = 0; it < 100; ++it) {
      if (!invert(D, Y.data(), Yi.data()) || !invert(D, Z.data(), Zi.data())) return false;
      double change = 0.0, size = 0.0;
      for (size_t x = 0; x < DD; ++x) {
        const double yn = 0.5 * (Y[x] + Zi[x]);
        change += (yn - Y[x]) * (yn - Y[x]);
        size += yn * yn;
        Z[x] = 0.5 * (Z[x] + Yi[x]);
        Y[x] = yn;
      }
      if (change <= 1e-30 * size) {
        conv = true;
        break;
      }
    }
    if (!conv) return false;
    A = Y;
  }
  // log(1 + X) = sum_j (-1)^(j+1) X^j / j, ||X||_F <= 1/4
  for (int i = 0; i < D; ++i)
    for (int j = 0; j < D; ++j) X[(size_t)i * D + j] = A[(size_t)i * D + j] - (i == j ? 1.0 : 0.0);
  P = X;
  for (int j = 1; j <= 40; ++j) {
    const double c = (j % 2 ? 1.0 : -1.0) / j;
    for (size_t x = 0; x < DD; ++x) S[x] += c * P[x];
    mm(D, P.data(), X.data(), T.data());
    P.swap(T);
  }
  const double f = ldexp(1.0, k);
  for (size_t x = 0; x < DD; ++x) L[x] = S[x] * f;
  // check exp(L) = G
  expm_real(D, L, T.data());
  for (size_t x = 0; x < DD; ++x) T[x] -= G[x];
  return fro(D, T.data()) <= 1e-9 * fro(D, G);
}

int hamiltonian_decomposition(int n, const double* G, double* h, double* gamma) {
  const int D = 1 << (2 * n);
  const size_t DD = (size_t)D * D;
  std::vector<double> L(DD), LH(DD, 0.0), E(DD);
  if (!logm_real(D, G, L.data())) return -1;
  std::vector<double> y, zr, zi;
  param_tables(n, &y, &zr, &zi);  // L^H[a][b] = h_{a^b} y[a][b]
  h[0] = 0.0;
  for (int k = 1; k < D; ++k) {
    double num = 0.0, den = 0.0;
    for (int a = 0; a < D; ++a) {
      const double s = y[(size_t)a * D + (a ^ k)];
      num += L[(size_t)a * D + (a ^ k)] * s;
      den += fabs(s);
    }
    h[k] = den != 0.0 ? num / den : 0.0;
  }
  for (int a = 0; a < D; ++a)
    for (int b = 0; b < D; ++b)
      if (a != b) LH[(size_t)a * D + b] = h[a ^ b] * y[(size_t)a * D + b];
  expm_real(D, LH.data(), E.data());
  for (size_t x = 0; x < DD; ++x) E[x] -= G[x];
  *gamma = fro(D, E.data());
  return 0;
}

namespace {

// The Pauli products P_k (unnormalized, qubit 0 the leftmost factor) as
// interleaved complex d x d matrices.
std::vector<double> pauli_products(int n) {
  const int d = 1 << n, D = d * d;
  static const double S[4][8] = {{1, 0, 0, 0, 0, 0, 1, 0},   // I
                                 {0, 0, 1, 0, 1, 0, 0, 0},   // X
                                 {0, 0, 0, -1, 0, 1, 0, 0},  // Y
                                 {1, 0, 0, 0, 0, 0, -1, 0}}; // Z
  std::vector<double> P((size_t)D * d * d * 2, 0.0);
  for (int k = 0; k < D; ++k)
    for (int r = 0; r < d; ++r)
      for (int c = 0; c < d; ++c) {
        double re = 1.0, im = 0.0;
        for (int q = 0; q < n; ++q) {
          const int a = (k >> (2 * (n - 1 - q))) & 3;
          const int br = (r >> (n - 1 - q)) & 1, bc = (c >> (n - 1 - q)) & 1;
          const double sr = S[a][(br * 2 + bc) * 2], si = S[a][(br * 2 + bc) * 2 + 1];
          const double nr = re * sr - im * si, ni = re * si + im * sr;
          re = nr;
          im = ni;
        }
        const size_t at = (((size_t)k * d + r) * d + c) * 2;
        P[at] = re;
        P[at + 1] = im;
      }
  return P;
}

// Frechet derivative of exp at A in direction E: the upper-right block of exp([[A, E], [0, A]]).
void expm_frechet(int D, const double* A, const double* E, double* Z) {
  const int D2 = 2 * D;
  std::vector<double> B((size_t)D2 * D2, 0.0), X((size_t)D2 * D2);
  for (int i = 0; i < D; ++i)
    for (int j = 0; j < D; ++j) {
      B[(size_t)i * D2 + j] = A[(size_t)i * D + j];
      B[(size_t)(i + D) * D2 + j + D] = A[(size_t)i * D + j];
      B[(size_t)i * D2 + j + D] = E[(size_t)i * D + j];
    }
  expm_real(D2, B.data(), X.data());
  for (int i = 0; i < D; ++i)
    for (int j = 0; j < D; ++j) Z[(size_t)i * D + j] = X[(size_t)i * D2 + j + D];
}

}  // namespace

bool target_hamiltonian(int n, const double* U, double* h) {
  const int d = 1 << n, D = d * d, d2 = 2 * d;
  // A = (U + U^dagger) / 2 + c (U - U^dagger) / (2i), Hermitian with the
  // eigenvectors of U; its real embedding [[X, -Y], [Y, X]] (A = X + iY)
  const double c = 0.6180339887498949;
  std::vector<double> Sm((size_t)d2 * d2), V((size_t)d2 * d2);
  for (int r = 0; r < d; ++r)
    for (int q = 0; q < d; ++q) {
      const double ur = U[((size_t)r * d + q) * 2], ui = U[((size_t)r * d + q) * 2 + 1];
      const double vr = U[((size_t)q * d + r) * 2], vi = -U[((size_t)q * d + r) * 2 + 1];  // (U^dagger)[r][q]
      const double xr = 0.5 * (ur + vr) + c * 0.5 * (ui - vi);  // (U - U^dagger) / (2i) = -i (U - U^dagger) / 2
      const double xi = 0.5 * (ui + vi) - c * 0.5 * (ur - vr);
      Sm[(size_t)r * d2 + q] = xr;
      Sm[(size_t)(r + d) * d2 + q + d] = xr;
      Sm[(size_t)r * d2 + q + d] = -xi;
      Sm[(size_t)(r + d) * d2 + q] = xi;
    }
  if (!jacobi_sym(d2, Sm, V)) return false;
  std::vector<double> mu(d2);
  for (int a = 0; a < d2; ++a) mu[a] = Sm[(size_t)a * d2 + a];
  // H = -sum over eigenvalue clusters of theta Pi (Pi the cluster's complex projector)
  std::vector<double> H((size_t)d * d * 2, 0.0);
  std::vector<char> done(d2, 0);
  for (int a = 0; a < d2; ++a) {
    if (done[a]) continue;
    std::vector<int> cl;
    for (int b = a; b < d2; ++b)
      if (!done[b] && fabs(mu[b] - mu[a]) <= 1e-8) {
        cl.push_back(b);
        done[b] = 1;
      }
    // real projector onto the cluster's eigenvectors; Pi = its [0:d][0:d] + i [d:2d][0:d] blocks
    std::vector<double> Pr((size_t)d * d, 0.0), Pi((size_t)d * d, 0.0);
    for (int b : cl)
      for (int r = 0; r < d; ++r)
        for (int q = 0; q < d; ++q) {
          Pr[(size_t)r * d + q] += V[(size_t)r * d2 + b] * V[(size_t)q * d2 + b];
          Pi[(size_t)r * d + q] += V[(size_t)(r + d) * d2 + b] * V[(size_t)q * d2 + b];
        }
    double m = 0.0;
    for (int r = 0; r < d; ++r) m += Pr[(size_t)r * d + r];
    // lambda = Tr(Pi U) / m
    double lr = 0.0, li = 0.0;
    for (int r = 0; r < d; ++r)
      for (int q = 0; q < d; ++q) {
        const double ar = Pr[(size_t)r * d + q], ai = Pi[(size_t)r * d + q];
        const double ur = U[((size_t)q * d + r) * 2], ui = U[((size_t)q * d + r) * 2 + 1];
        lr += ar * ur - ai * ui;
        li += ar * ui + ai * ur;
      }
    double theta = atan2(li / m, lr / m);
    if (theta <= -M_PI + 1e-12) theta = M_PI;  // the principal argument of -1 is pi
    for (size_t x = 0; x < (size_t)d * d; ++x) {
      H[2 * x] -= theta * Pr[x];
      H[2 * x + 1] -= theta * Pi[x];
    }
  }
  // h_k = 2 Re Tr(P_k H) / d
  const std::vector<double> P = pauli_products(n);
  h[0] = 0.0;
  for (int k = 1; k < D; ++k) {
    double t = 0.0;
    for (int r = 0; r < d; ++r)
      for (int q = 0; q < d; ++q) {
        const size_t p = (((size_t)k * d + r) * d + q) * 2, x = ((size_t)q * d + r) * 2;
        t += P[p] * H[x] - P[p + 1] * H[x + 1];
      }
    h[k] = 2.0 * t / d;
  }
  return true;
}

int hamiltonian_decomposition_toward(int n, const double* G, const double* U, double* h, double* gamma) {
  const int D = 1 << (2 * n);
  const size_t DD = (size_t)D * D;
  if (!target_hamiltonian(n, U, h)) return -1;
  std::vector<double> y, zr, zi;
  param_tables(n, &y, &zr, &zi);  // L^H[a][b] = h_{a^b} y[a][b]
  std::vector<double> L(DD), E(DD), R(DD), LT(DD), Z(DD);
  auto build = [&](const double* x) {
    std::fill(L.begin(), L.end(), 0.0);
    for (int a = 0; a < D; ++a)
      for (int b = 0; b < D; ++b)
        if (a != b) L[(size_t)a * D + b] = x[(a ^ b) - 1] * y[(size_t)a * D + b];
  };
  // f = ||G - exp(L^H)||_F^2; df/dh_k = -2 sum_a Z[a][a^k] y[a][a^k], Z = Dexp_{L^T}(G - exp(L))
  auto f = [&](const double* x, double* g) -> double {
    build(x);
    expm_real(D, L.data(), E.data());
    double v = 0.0;
    for (size_t q = 0; q < DD; ++q) {
      R[q] = G[q] - E[q];
      v += R[q] * R[q];
    }
    for (int a = 0; a < D; ++a)
      for (int b = 0; b < D; ++b) LT[(size_t)a * D + b] = L[(size_t)b * D + a];
    expm_frechet(D, LT.data(), R.data(), Z.data());
    for (int k = 1; k < D; ++k) {
      double s = 0.0;
      for (int a = 0; a < D; ++a) s += Z[(size_t)a * D + (a ^ k)] * y[(size_t)a * D + (a ^ k)];
      g[k - 1] = -2.0 * s;
    }
    return v;
  };
  std::vector<double> x(h + 1, h + D);
  lbfgs(D - 1, x.data(), f, 20, 1e-14, 2000);
  h[0] = 0.0;
  for (int k = 1; k < D; ++k) h[k] = x[k - 1];
  build(x.data());
  expm_real(D, L.data(), E.data());
  for (size_t q = 0; q < DD; ++q) E[q] -= G[q];
  *gamma = fro(D, E.data());
  return 0;
}

}  // namespace gst
