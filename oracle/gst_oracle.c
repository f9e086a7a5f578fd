/*
 * gst_oracle.c -- plain CPU reference for the GST likelihood path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header or table with the HIP path.
 *
 * What it computes (thesis Sec. 6.3.1):
 *   p[s][m] = e_m^T G[s_L] ... G[s_1] rho              (Eqs. GSTBornRuleVectorized,
 *                                                        GSTFullFiducialsGerms; s_1 acts first)
 *   F       = - sum_{s,m: N>0} N[s][m] log p[s][m]     (negative multinomial log-likelihood
 *                                                        of the counts, without the data-only
 *                                                        multinomial constant; 0 log 0 := 0)
 *   dF/dtheta for theta = (rho, E_0..E_{M-1}, G_0..G_{K-1}), every entry
 *                                                       (the full parameterization whose size
 *                                                        the thesis counts as 1616 for 2 qubits)
 *
 * The probability is the plain definition evaluated right to left: each new
 * state component is a dot product accumulated with one fused multiply-add per
 * term, in ascending column order, starting from zero.  The gradient is the
 * chain rule of that product, applied sequence by sequence; the per-sequence
 * contributions are added in ascending sequence order.  Every quantity is
 * IEEE binary64; compile with -ffp-contract=off so that no other
 * contraction is introduced.
 *
 * Also (thesis Eq. statisticaldistance): the statistical distance
 *   D = 1/2 sum_J |p_J - q_J|  of two outcome distributions, row by row.
 *
 * Layouts: rho[D]; E[M][D] (row m = e_m); G[K][D][D] row-major with
 * G[k][i][j] = Tr(P_i G_k(P_j))/d; offsets[S+1] int64, gates[offsets[S]] uint8
 * in time order; counts[S][M] int32; probs[S][M]; gradient
 * [rho (D) | E (M*D) | G (K*D*D)].
 *
 * Return codes: 0 ok, -1 invalid argument, -2 gate index out of range,
 * -3 a probability <= 0 where the count is > 0 (objective set to +inf; the
 * number of such entries is written to *n_nonpos).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_EINDEX (-2)
#define OR_ENONPOS (-3)

static int check_lists(int D, int M, int K, int64_t S, const int64_t* off, const uint8_t* gates,
                       int64_t* max_len) {
  if (D < 1 || M < 1 || K < 1 || K > 255 || S < 0 || !off) return OR_EINVAL;
  if (off[0] != 0) return OR_EINVAL;
  int64_t mx = 0;
  for (int64_t s = 0; s < S; ++s) {
    int64_t L = off[s + 1] - off[s];
    if (L < 0) return OR_EINVAL;
    if (L > mx) mx = L;
  }
  if (off[S] > 0 && !gates) return OR_EINVAL;
  for (int64_t t = 0; t < off[S]; ++t)
    if (gates[t] >= K) return OR_EINDEX;
  *max_len = mx;
  return OR_OK;
}

/* f_out = G f_in, one fused multiply-add per term, columns ascending. */
static void apply_gate(int D, const double* G, const double* f_in, double* f_out) {
  for (int i = 0; i < D; ++i) {
    double acc = 0.0;
    for (int j = 0; j < D; ++j) acc = fma(G[(size_t)i * D + j], f_in[j], acc);
    f_out[i] = acc;
  }
}

/* <e_m, f>, same accumulation rule. */
static double dot(int D, const double* e, const double* f) {
  double acc = 0.0;
  for (int j = 0; j < D; ++j) acc = fma(e[j], f[j], acc);
  return acc;
}

/* states[t] for t = 0..L of sequence s (states[0] = rho). */
static void forward(int D, const double* rho, const double* G, const uint8_t* word, int64_t L,
                    double* states) {
  memcpy(states, rho, sizeof(double) * (size_t)D);
  for (int64_t t = 1; t <= L; ++t)
    apply_gate(D, G + (size_t)word[t - 1] * D * D, states + (size_t)(t - 1) * D,
               states + (size_t)t * D);
}

int oracle_probs(int D, int M, int K, const double* rho, const double* E, const double* G,
                 int64_t S, const int64_t* off, const uint8_t* gates, double* probs) {
  int64_t mx = 0;
  int rc = check_lists(D, M, K, S, off, gates, &mx);
  if (rc) return rc;
  if (!rho || !E || !G || (S > 0 && !probs)) return OR_EINVAL;
  double* st = (double*)malloc(sizeof(double) * (size_t)D * (size_t)(mx + 1));
  if (!st) return OR_EINVAL;
  for (int64_t s = 0; s < S; ++s) {
    int64_t L = off[s + 1] - off[s];
    forward(D, rho, G, gates + off[s], L, st);
    const double* fL = st + (size_t)L * D;
    for (int m = 0; m < M; ++m) probs[s * M + m] = dot(D, E + (size_t)m * D, fL);
  }
  free(st);
  return OR_OK;
}

/*
 * Reverse sweep of one sequence given its states and the adjoint seed
 * dp[m] = dLoss/dp[s][m]:
 *   dE[m] += dp[m] f_L;   b = sum_m dp[m] e_m;
 *   for t = L..1:  dG[s_t] += b f_{t-1}^T ;  b = G[s_t]^T b;
 *   drho += b.
 */
static void backward(int D, int M, const double* E, const double* G, const uint8_t* word,
                     int64_t L, const double* states, const double* dp, double* b, double* nb,
                     double* grho, double* gE, double* gG) {
  const double* fL = states + (size_t)L * D;
  for (int m = 0; m < M; ++m)
    for (int j = 0; j < D; ++j) gE[(size_t)m * D + j] += dp[m] * fL[j];
  for (int j = 0; j < D; ++j) {
    double acc = 0.0;
    for (int m = 0; m < M; ++m) acc += dp[m] * E[(size_t)m * D + j];
    b[j] = acc;
  }
  for (int64_t t = L; t >= 1; --t) {
    const int k = word[t - 1];
    const double* Gk = G + (size_t)k * D * D;
    double* dGk = gG + (size_t)k * D * D;
    const double* fprev = states + (size_t)(t - 1) * D;
    for (int i = 0; i < D; ++i)
      for (int j = 0; j < D; ++j) dGk[(size_t)i * D + j] += b[i] * fprev[j];
    for (int j = 0; j < D; ++j) {
      double acc = 0.0;
      for (int i = 0; i < D; ++i) acc += Gk[(size_t)i * D + j] * b[i];
      nb[j] = acc;
    }
    memcpy(b, nb, sizeof(double) * (size_t)D);
  }
  for (int j = 0; j < D; ++j) grho[j] += b[j];
}

/*
 * Objective, probabilities and gradient.  probs and grad may be NULL.
 * The gradient is written (not accumulated) and is only meaningful when the
 * return code is 0.
 */
int oracle_loglik(int D, int M, int K, const double* rho, const double* E, const double* G,
                  int64_t S, const int64_t* off, const uint8_t* gates, const int32_t* counts,
                  double* probs, double* objective, double* grad, int64_t* n_nonpos) {
  int64_t mx = 0;
  int rc = check_lists(D, M, K, S, off, gates, &mx);
  if (rc) return rc;
  if (!rho || !E || !G || !objective || (S > 0 && !counts)) return OR_EINVAL;
  for (int64_t i = 0; i < S * M; ++i)
    if (counts[i] < 0) return OR_EINVAL;
  const size_t np = (size_t)D + (size_t)M * D + (size_t)K * D * D;
  double* st = (double*)malloc(sizeof(double) * (size_t)D * (size_t)(mx + 3) + sizeof(double) * 2 * M);
  if (!st) return OR_EINVAL;
  double* b = st + (size_t)D * (size_t)(mx + 1);
  double* nb = b + D;
  double* p = nb + D;
  double* dp = p + M;
  if (grad) memset(grad, 0, sizeof(double) * np);
  double F = 0.0;
  int64_t bad = 0;
  for (int64_t s = 0; s < S; ++s) {
    int64_t L = off[s + 1] - off[s];
    const uint8_t* word = gates + off[s];
    forward(D, rho, G, word, L, st);
    const double* fL = st + (size_t)L * D;
    double Fs = 0.0;
    for (int m = 0; m < M; ++m) {
      p[m] = dot(D, E + (size_t)m * D, fL);
      if (probs) probs[s * M + m] = p[m];
      const int32_t N = counts[s * M + m];
      if (N > 0) {
        if (p[m] <= 0.0) {
          ++bad;
          dp[m] = 0.0;
        } else {
          Fs -= (double)N * log(p[m]);
          dp[m] = -(double)N / p[m];
        }
      } else {
        dp[m] = 0.0;
      }
    }
    F += Fs;
    if (grad) backward(D, M, E, G, word, L, st, dp, b, nb, grad, grad + D, grad + D + (size_t)M * D);
  }
  free(st);
  if (n_nonpos) *n_nonpos = bad;
  if (bad) {
    *objective = INFINITY;
    return OR_ENONPOS;
  }
  *objective = F;
  return OR_OK;
}

/* Vector-Jacobian product: grad = sum_{s,m} W[s][m] dp[s][m]/dtheta. */
int oracle_vjp(int D, int M, int K, const double* rho, const double* E, const double* G,
               int64_t S, const int64_t* off, const uint8_t* gates, const double* W, double* grad) {
  int64_t mx = 0;
  int rc = check_lists(D, M, K, S, off, gates, &mx);
  if (rc) return rc;
  if (!rho || !E || !G || !grad || (S > 0 && !W)) return OR_EINVAL;
  const size_t np = (size_t)D + (size_t)M * D + (size_t)K * D * D;
  double* st = (double*)malloc(sizeof(double) * (size_t)D * (size_t)(mx + 3));
  if (!st) return OR_EINVAL;
  double* b = st + (size_t)D * (size_t)(mx + 1);
  double* nb = b + D;
  memset(grad, 0, sizeof(double) * np);
  for (int64_t s = 0; s < S; ++s) {
    int64_t L = off[s + 1] - off[s];
    const uint8_t* word = gates + off[s];
    forward(D, rho, G, word, L, st);
    backward(D, M, E, G, word, L, st, W + s * M, b, nb, grad, grad + D, grad + D + (size_t)M * D);
  }
  free(st);
  return OR_OK;
}

/*
 * Same probabilities in extended precision (long double, x87 64-bit
 * mantissa) with plain multiply-add: bounds the binary64 oracle's own
 * rounding when a difference has to be attributed.
 */
int oracle_probs_extended(int D, int M, int K, const double* rho, const double* E, const double* G,
                          int64_t S, const int64_t* off, const uint8_t* gates, double* probs) {
  int64_t mx = 0;
  int rc = check_lists(D, M, K, S, off, gates, &mx);
  if (rc) return rc;
  if (!rho || !E || !G || (S > 0 && !probs)) return OR_EINVAL;
  long double* f = (long double*)malloc(sizeof(long double) * 2 * (size_t)D);
  if (!f) return OR_EINVAL;
  long double* g = f + D;
  for (int64_t s = 0; s < S; ++s) {
    for (int j = 0; j < D; ++j) f[j] = rho[j];
    for (int64_t t = off[s]; t < off[s + 1]; ++t) {
      const double* Gk = G + (size_t)gates[t] * D * D;
      for (int i = 0; i < D; ++i) {
        long double acc = 0.0L;
        for (int j = 0; j < D; ++j) acc += (long double)Gk[(size_t)i * D + j] * f[j];
        g[i] = acc;
      }
      memcpy(f, g, sizeof(long double) * (size_t)D);
    }
    for (int m = 0; m < M; ++m) {
      long double acc = 0.0L;
      for (int j = 0; j < D; ++j) acc += (long double)E[(size_t)m * D + j] * f[j];
      probs[s * M + m] = (double)acc;
    }
  }
  free(f);
  return OR_OK;
}

/* Statistical distance (total variation distance), Eq. statisticaldistance:
 * out[i] = 1/2 * sum_{j ascending} |p[i][j] - q[i][j]| for i < n, rows of m. */
int oracle_tv_distance(int64_t n, int m, const double* p, const double* q, double* out) {
  if (n < 0 || m < 1 || (n > 0 && (!p || !q || !out))) return OR_EINVAL;
  for (int64_t i = 0; i < n; ++i) {
    double acc = 0.0;
    for (int j = 0; j < m; ++j) acc += fabs(p[i * m + j] - q[i * m + j]);
    out[i] = 0.5 * acc;
  }
  return OR_OK;
}
