// The fit around the likelihood, host side: thesis Sec. 6.3.1 (the GST gauge,
// linear-inversion estimates from the matrix AB of bare-experiment
// frequencies, iterative refinement, gauge optimization).
#include "gst_fit_core.h"

#include <math.h>
#include <string.h>

#include <algorithm>
#include <deque>
#include <map>
#include <string>

namespace gst {

bool svd_jacobi(int m, int n, const double* A, double* U, double* S, double* V) {
  // columns of W = A V are rotated pairwise until orthogonal
  std::vector<double> W(A, A + (size_t)m * n), Vm((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) Vm[(size_t)i * n + i] = 1.0;
  bool done = false;
  for (int sweep = 0; sweep < 80 && !done; ++sweep) {
    done = true;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        double a = 0.0, b = 0.0, g = 0.0;
        for (int r = 0; r < m; ++r) {
          const double wp = W[(size_t)r * n + p], wq = W[(size_t)r * n + q];
          a += wp * wp;
          b += wq * wq;
          g += wp * wq;
        }
        if (g == 0.0 || fabs(g) <= 1e-15 * sqrt(a * b)) continue;
        done = false;
        const double zeta = (b - a) / (2.0 * g);
        const double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
        for (int r = 0; r < m; ++r) {
          const double wp = W[(size_t)r * n + p], wq = W[(size_t)r * n + q];
          W[(size_t)r * n + p] = c * wp - s * wq;
          W[(size_t)r * n + q] = s * wp + c * wq;
        }
        for (int r = 0; r < n; ++r) {
          const double vp = Vm[(size_t)r * n + p], vq = Vm[(size_t)r * n + q];
          Vm[(size_t)r * n + p] = c * vp - s * vq;
          Vm[(size_t)r * n + q] = s * vp + c * vq;
        }
      }
  }
  if (!done) return false;
  std::vector<double> sig(n);
  std::vector<int> order(n);
  for (int j = 0; j < n; ++j) {
    double s2 = 0.0;
    for (int r = 0; r < m; ++r) s2 += W[(size_t)r * n + j] * W[(size_t)r * n + j];
    sig[j] = sqrt(s2);
    order[j] = j;
  }
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return sig[x] > sig[y]; });
  for (int c = 0; c < n; ++c) {
    const int j = order[c];
    S[c] = sig[j];
    for (int r = 0; r < m; ++r) U[(size_t)r * n + c] = sig[j] > 0 ? W[(size_t)r * n + j] / sig[j] : 0.0;
    for (int r = 0; r < n; ++r) V[(size_t)r * n + c] = Vm[(size_t)r * n + j];
  }
  return true;
}

bool invert(int n, const double* A, double* Ai) {
  std::vector<double> L(A, A + (size_t)n * n);
  std::vector<int> piv(n);
  for (int i = 0; i < n; ++i) piv[i] = i;
  for (int k = 0; k < n; ++k) {
    int p = k;
    for (int r = k + 1; r < n; ++r)
      if (fabs(L[(size_t)r * n + k]) > fabs(L[(size_t)p * n + k])) p = r;
    if (L[(size_t)p * n + k] == 0.0) return false;
    if (p != k) {
      for (int c = 0; c < n; ++c) std::swap(L[(size_t)p * n + c], L[(size_t)k * n + c]);
      std::swap(piv[p], piv[k]);
    }
    for (int r = k + 1; r < n; ++r) {
      const double f = L[(size_t)r * n + k] / L[(size_t)k * n + k];
      L[(size_t)r * n + k] = f;
      for (int c = k + 1; c < n; ++c) L[(size_t)r * n + c] -= f * L[(size_t)k * n + c];
    }
  }
  // solve L U x = P e_j for each column j
  for (int j = 0; j < n; ++j) {
    std::vector<double> x(n);
    for (int i = 0; i < n; ++i) {
      double v = piv[i] == j ? 1.0 : 0.0;
      for (int c = 0; c < i; ++c) v -= L[(size_t)i * n + c] * x[c];
      x[i] = v;
    }
    for (int i = n - 1; i >= 0; --i) {
      double v = x[i];
      for (int c = i + 1; c < n; ++c) v -= L[(size_t)i * n + c] * x[c];
      x[i] = v / L[(size_t)i * n + i];
    }
    for (int i = 0; i < n; ++i) Ai[(size_t)i * n + j] = x[i];
  }
  return true;
}

bool solve(int n, const double* A, const double* b, double* x) {
  std::vector<double> L(A, A + (size_t)n * n), y(b, b + n);
  for (int k = 0; k < n; ++k) {
    int p = k;
    for (int r = k + 1; r < n; ++r)
      if (fabs(L[(size_t)r * n + k]) > fabs(L[(size_t)p * n + k])) p = r;
    if (L[(size_t)p * n + k] == 0.0) return false;
    if (p != k) {
      for (int c = 0; c < n; ++c) std::swap(L[(size_t)p * n + c], L[(size_t)k * n + c]);
      std::swap(y[p], y[k]);
    }
    const double* rk = &L[(size_t)k * n];
    for (int r = k + 1; r < n; ++r) {
      double* rr = &L[(size_t)r * n];
      const double f = rr[k] / rk[k];
      if (f == 0.0) continue;
      for (int c = k + 1; c < n; ++c) rr[c] -= f * rk[c];
      y[r] -= f * y[k];
    }
  }
  for (int i = n - 1; i >= 0; --i) {
    double v = y[i];
    for (int c = i + 1; c < n; ++c) v -= L[(size_t)i * n + c] * x[c];
    x[i] = v / L[(size_t)i * n + i];
  }
  return true;
}

int lgst_matrices(int64_t S, const int64_t* offsets, const uint8_t* gates, const int32_t* counts, int M, int K,
                  int n_prep, const int64_t* prep_off, const uint8_t* prep_gates, int n_meas, const int64_t* meas_off,
                  const uint8_t* meas_gates, std::vector<double>* AB, std::vector<double>* Bk, int* j0, int* i0) {
  std::map<std::string, int64_t> rows;  // first occurrence of each word
  for (int64_t s = 0; s < S; ++s)
    rows.emplace(std::string(reinterpret_cast<const char*>(gates + offsets[s]), (size_t)(offsets[s + 1] - offsets[s])),
                 s);
  auto word = [](const int64_t* off, const uint8_t* g, int i) {
    return std::string(reinterpret_cast<const char*>(g + off[i]), (size_t)(off[i + 1] - off[i]));
  };
  *j0 = *i0 = -1;
  for (int j = 0; j < n_prep; ++j)
    if (prep_off[j + 1] == prep_off[j] && *j0 < 0) *j0 = j;
  for (int i = 0; i < n_meas; ++i)
    if (meas_off[i + 1] == meas_off[i] && *i0 < 0) *i0 = i;
  if (*j0 < 0 || *i0 < 0) return -2;
  const size_t R = (size_t)M * n_meas;
  AB->assign(R * n_prep, 0.0);
  Bk->assign((size_t)K * R * n_prep, 0.0);
  auto fill = [&](const std::string& w, double* dst, size_t stride) -> int {
    auto it = rows.find(w);
    if (it == rows.end()) return -1;
    const int32_t* c = counts + it->second * M;
    double tot = 0.0;
    for (int m = 0; m < M; ++m) tot += c[m];
    if (tot <= 0.0) return -3;
    for (int m = 0; m < M; ++m) dst[m * stride] = c[m] / tot;
    return 0;
  };
  for (int i = 0; i < n_meas; ++i)
    for (int j = 0; j < n_prep; ++j) {
      const std::string fp = word(prep_off, prep_gates, j), fq = word(meas_off, meas_gates, i);
      int rc = fill(fp + fq, AB->data() + (size_t)M * i * n_prep + j, n_prep);
      if (rc) return rc;
      for (int k = 0; k < K; ++k) {
        rc = fill(fp + std::string(1, (char)k) + fq, Bk->data() + (size_t)k * R * n_prep + (size_t)M * i * n_prep + j,
                  n_prep);
        if (rc) return rc;
      }
    }
  return 0;
}

int lgst_estimate(int D, int M, int K, int n_prep, int n_meas, const double* AB, const double* Bk, int j0, int i0,
                  double* rho, double* E, double* G) {
  const int R = M * n_meas, P = n_prep;
  std::vector<double> U((size_t)R * P), Sv(P), V((size_t)P * P);
  if (!svd_jacobi(R, P, AB, U.data(), Sv.data(), V.data())) return -4;
  // truncate to D columns and fix the signs
  std::vector<double> Ud((size_t)R * D), Vd((size_t)P * D);
  for (int c = 0; c < D; ++c) {
    int arg = 0;
    for (int r = 1; r < P; ++r)
      if (fabs(V[(size_t)r * P + c]) > fabs(V[(size_t)arg * P + c])) arg = r;
    const double sg = V[(size_t)arg * P + c] < 0 ? -1.0 : 1.0;
    for (int r = 0; r < R; ++r) Ud[(size_t)r * D + c] = sg * U[(size_t)r * P + c];
    for (int r = 0; r < P; ++r) Vd[(size_t)r * D + c] = sg * V[(size_t)r * P + c];
  }
  // X -> U^T X V for an R x P matrix X (D x D result)
  auto project = [&](const double* X, double* out) {
    std::vector<double> XV((size_t)R * D, 0.0);
    for (int r = 0; r < R; ++r)
      for (int c = 0; c < D; ++c) {
        double s = 0.0;
        for (int q = 0; q < P; ++q) s += X[(size_t)r * P + q] * Vd[(size_t)q * D + c];
        XV[(size_t)r * D + c] = s;
      }
    for (int a = 0; a < D; ++a)
      for (int c = 0; c < D; ++c) {
        double s = 0.0;
        for (int r = 0; r < R; ++r) s += Ud[(size_t)r * D + a] * XV[(size_t)r * D + c];
        out[(size_t)a * D + c] = s;
      }
  };
  std::vector<double> Ahat((size_t)D * D), Ainv((size_t)D * D), Pk((size_t)D * D);
  project(AB, Ahat.data());
  if (!invert(D, Ahat.data(), Ainv.data())) return -5;
  for (int k = 0; k < K; ++k) {
    project(Bk + (size_t)k * R * P, Pk.data());
    for (int a = 0; a < D; ++a)
      for (int c = 0; c < D; ++c) {
        double s = 0.0;
        for (int q = 0; q < D; ++q) s += Ainv[(size_t)a * D + q] * Pk[(size_t)q * D + c];
        G[((size_t)k * D + a) * D + c] = s;
      }
  }
  std::vector<double> ub(D, 0.0);
  for (int a = 0; a < D; ++a) {
    double s = 0.0;
    for (int r = 0; r < R; ++r) s += Ud[(size_t)r * D + a] * AB[(size_t)r * P + j0];
    ub[a] = s;
  }
  for (int a = 0; a < D; ++a) {
    double s = 0.0;
    for (int q = 0; q < D; ++q) s += Ainv[(size_t)a * D + q] * ub[q];
    rho[a] = s;
  }
  for (int J = 0; J < M; ++J)
    for (int c = 0; c < D; ++c) {
      double s = 0.0;
      for (int q = 0; q < P; ++q) s += AB[(size_t)(J + M * i0) * P + q] * Vd[(size_t)q * D + c];
      E[(size_t)J * D + c] = s;
    }
  return 0;
}

namespace {
// C = A B (n x n row-major)
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
void transpose(int n, const double* A, double* At) {
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) At[(size_t)j * n + i] = A[(size_t)i * n + j];
}
}  // namespace

double gauge_objective(int D, int M, int K, const double* X, const double* rho, const double* E, const double* G,
                       const double* rT, const double* ET, const double* GT, double w, double* grad) {
  const size_t DD = (size_t)D * D;
  std::vector<double> Xi(DD), XiT(DD), gX(DD, 0.0), t1(DD), t2(DD), Y(DD), R(DD), YT(DD), RXiT(DD), B(DD);
  if (!invert(D, X, Xi.data())) return INFINITY;
  transpose(D, Xi.data(), XiT.data());
  double f = 0.0;
  for (int k = 0; k < K; ++k) {
    const double* g = G + k * DD;
    mm(D, g, Xi.data(), t1.data());  // g X^-1
    mm(D, X, t1.data(), Y.data());   // Y = X g X^-1
    for (size_t x = 0; x < DD; ++x) {
      R[x] = Y[x] - GT[k * DD + x];
      f += R[x] * R[x];
    }
    // 2 (R (g X^-1)^T - Y^T R X^-T)
    transpose(D, t1.data(), t2.data());
    mm(D, R.data(), t2.data(), B.data());
    for (size_t x = 0; x < DD; ++x) gX[x] += 2.0 * B[x];
    transpose(D, Y.data(), YT.data());
    mm(D, R.data(), XiT.data(), RXiT.data());
    mm(D, YT.data(), RXiT.data(), B.data());
    for (size_t x = 0; x < DD; ++x) gX[x] -= 2.0 * B[x];
  }
  // state: r = X rho - rho_T, gradient 2 w r rho^T
  std::vector<double> r(D);
  for (int i = 0; i < D; ++i) {
    double s = 0.0;
    for (int j = 0; j < D; ++j) s += X[(size_t)i * D + j] * rho[j];
    r[i] = s - rT[i];
    f += w * r[i] * r[i];
  }
  for (int i = 0; i < D; ++i)
    for (int j = 0; j < D; ++j) gX[(size_t)i * D + j] += 2.0 * w * r[i] * rho[j];
  // effects: q = X^-T e - e_T, gradient -2 w (X^-T e) (X^-1 q)^T
  std::vector<double> u(D), q(D), v(D);
  for (int m = 0; m < M; ++m) {
    const double* e = E + (size_t)m * D;
    for (int i = 0; i < D; ++i) {
      double s = 0.0;
      for (int j = 0; j < D; ++j) s += XiT[(size_t)i * D + j] * e[j];
      u[i] = s;
      q[i] = s - ET[(size_t)m * D + i];
      f += w * q[i] * q[i];
    }
    for (int i = 0; i < D; ++i) {
      double s = 0.0;
      for (int j = 0; j < D; ++j) s += Xi[(size_t)i * D + j] * q[j];
      v[i] = s;
    }
    for (int i = 0; i < D; ++i)
      for (int j = 0; j < D; ++j) gX[(size_t)i * D + j] -= 2.0 * w * u[i] * v[j];
  }
  if (grad) memcpy(grad, gX.data(), DD * sizeof(double));
  return f;
}

bool gauge_linear_start(int D, int M, int K, const double* rho, const double* E, const double* G, const double* rT,
                        const double* ET, const double* GT, double w, double* X) {
  const int n = D * D;
  std::vector<double> N((size_t)n * n, 0.0), rhs(n, 0.0);
  std::vector<int> idx;
  std::vector<double> val;
  // adds the row (idx, val) with right-hand side b to the normal equations
  auto add_row = [&](double b) {
    for (size_t p = 0; p < idx.size(); ++p) {
      rhs[idx[p]] += val[p] * b;
      for (size_t q = 0; q < idx.size(); ++q) N[(size_t)idx[p] * n + idx[q]] += val[p] * val[q];
    }
  };
  for (int k = 0; k < K; ++k) {
    const double* g = G + (size_t)k * n;
    const double* t = GT + (size_t)k * n;
    for (int a = 0; a < D; ++a)
      for (int b = 0; b < D; ++b) {
        // (X g)_ab - (t X)_ab = sum_c X_ac g_cb - sum_c t_ac X_cb
        idx.clear();
        val.clear();
        for (int c = 0; c < D; ++c) {
          idx.push_back(a * D + c);
          val.push_back(g[(size_t)c * D + b]);
          idx.push_back(c * D + b);
          val.push_back(-t[(size_t)a * D + c]);
        }
        add_row(0.0);
      }
  }
  const double sw = sqrt(w);
  for (int i = 0; i < D; ++i) {  // (X rho)_i = rho_T,i
    idx.clear();
    val.clear();
    for (int j = 0; j < D; ++j) {
      idx.push_back(i * D + j);
      val.push_back(sw * rho[j]);
    }
    add_row(sw * rT[i]);
  }
  for (int m = 0; m < M; ++m)
    for (int j = 0; j < D; ++j) {  // (X^T t_m)_j = e_m,j
      idx.clear();
      val.clear();
      for (int i = 0; i < D; ++i) {
        idx.push_back(i * D + j);
        val.push_back(sw * ET[(size_t)m * D + i]);
      }
      add_row(sw * E[(size_t)m * D + j]);
    }
  return solve(n, N.data(), rhs.data(), X);
}

LbfgsResult lbfgs(int n, double* x, const std::function<double(const double*, double*)>& f, int m, double gtol,
                  int max_iter) {
  LbfgsResult res;
  std::vector<double> g(n), q(n), d(n), xn(n), gn(n);
  double fx = f(x, g.data());
  res.evaluations = 1;
  if (!std::isfinite(fx)) {  // no descent from a point where f is undefined
    res.status = 2;
    res.f = fx;
    return res;
  }
  std::deque<std::vector<double>> Ss, Ys;
  auto gmax_of = [&](const std::vector<double>& v) {
    double a = 0.0;
    for (double z : v) a = std::max(a, fabs(z));
    return a;
  };
  auto dot = [&](const std::vector<double>& a, const std::vector<double>& b) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
  };
  res.status = 1;
  for (int it = 0; it < max_iter; ++it) {
    if (gmax_of(g) <= gtol) {
      res.status = 0;
      break;
    }
    // two-loop recursion
    q = g;
    const int k = (int)Ss.size();
    std::vector<double> alpha(k);
    for (int j = k - 1; j >= 0; --j) {
      alpha[j] = dot(Ss[j], q) / dot(Ys[j], Ss[j]);
      for (int i = 0; i < n; ++i) q[i] -= alpha[j] * Ys[j][i];
    }
    if (k) {
      const double gam = dot(Ss[k - 1], Ys[k - 1]) / dot(Ys[k - 1], Ys[k - 1]);
      for (int i = 0; i < n; ++i) q[i] *= gam;
    }
    for (int j = 0; j < k; ++j) {
      const double b = dot(Ys[j], q) / dot(Ys[j], Ss[j]);
      for (int i = 0; i < n; ++i) q[i] += (alpha[j] - b) * Ss[j][i];
    }
    for (int i = 0; i < n; ++i) d[i] = -q[i];
    const double gd = dot(g, d);
    if (!(gd < 0.0)) {
      res.status = 2;
      break;
    }
    // strong Wolfe line search: bracket by doubling from the unit step, then
    // bisect; a step whose objective is not finite counts as too long
    auto phi = [&](double a, double* dphi) {
      for (int i = 0; i < n; ++i) xn[i] = x[i] + a * d[i];
      const double v = f(xn.data(), gn.data());
      ++res.evaluations;
      *dphi = dot(gn, d);
      return v;
    };
    const double c1 = 1e-4, c2 = 0.9;
    double a_prev = 0.0, f_prev = fx, a = 1.0, fn = 0.0, dn = 0.0;
    double lo = 0.0, hi = 0.0, f_lo = fx;
    bool found = false, zoom = false;
    for (int ls = 0; ls < 60 && !found && !zoom; ++ls) {
      fn = phi(a, &dn);
      if (!std::isfinite(fn) || fn > fx + c1 * a * gd || (ls > 0 && fn >= f_prev)) {
        lo = a_prev, f_lo = f_prev, hi = a, zoom = true;
      } else if (fabs(dn) <= -c2 * gd) {
        found = true;
      } else if (dn >= 0.0) {
        lo = a, f_lo = fn, hi = a_prev, zoom = true;
      } else {
        a_prev = a, f_prev = fn, a *= 2.0;
      }
    }
    for (int z = 0; z < 60 && zoom && !found; ++z) {
      a = 0.5 * (lo + hi);
      fn = phi(a, &dn);
      if (!std::isfinite(fn) || fn > fx + c1 * a * gd || fn >= f_lo) {
        hi = a;
      } else {
        if (fabs(dn) <= -c2 * gd) {
          found = true;
          break;
        }
        if (dn * (hi - lo) >= 0.0) hi = lo;
        lo = a, f_lo = fn;
      }
    }
    if (!found) {
      // the best point with sufficient decrease, if any
      if (lo > 0.0 && std::isfinite(f_lo) && f_lo <= fx + c1 * lo * gd && f_lo < fx) {
        a = lo;
        fn = phi(a, &dn);
      } else {
        res.status = 2;
        break;
      }
    }
    std::vector<double> s(n), y(n);
    for (int i = 0; i < n; ++i) {
      s[i] = xn[i] - x[i];
      y[i] = gn[i] - g[i];
    }
    if (dot(s, y) > 1e-300) {
      Ss.push_back(s);
      Ys.push_back(y);
      if ((int)Ss.size() > m) {
        Ss.pop_front();
        Ys.pop_front();
      }
    }
    memcpy(x, xn.data(), (size_t)n * sizeof(double));
    g = gn;
    fx = fn;
    res.iterations = it + 1;
  }
  res.f = fx;
  res.gmax = gmax_of(g);
  return res;
}

}  // namespace gst
