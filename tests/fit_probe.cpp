// C entries for the CPU tests of the fit's host code (LGST, gauge objective,
// L-BFGS).
#include <math.h>
#include <string.h>

#include <vector>

#include "gst_fit_core.h"

extern "C" {

int probe_svd(int m, int n, const double* A, double* U, double* S, double* V) {
  return gst::svd_jacobi(m, n, A, U, S, V) ? 0 : -1;
}

int probe_lgst(int D, int M, int K, int64_t S, const int64_t* off, const uint8_t* gates, const int32_t* counts,
               int n_prep, const int64_t* poff, const uint8_t* pg, int n_meas, const int64_t* moff, const uint8_t* mg,
               double* rho, double* E, double* G) {
  std::vector<double> AB, Bk;
  int j0, i0;
  int rc = gst::lgst_matrices(S, off, gates, counts, M, K, n_prep, poff, pg, n_meas, moff, mg, &AB, &Bk, &j0, &i0);
  if (rc) return rc;
  return gst::lgst_estimate(D, M, K, n_prep, n_meas, AB.data(), Bk.data(), j0, i0, rho, E, G);
}

double probe_gauge_objective(int D, int M, int K, const double* X, const double* rho, const double* E,
                             const double* G, const double* rT, const double* ET, const double* GT, double w,
                             double* grad) {
  return gst::gauge_objective(D, M, K, X, rho, E, G, rT, ET, GT, w, grad);
}

// minimizes the gauge objective from X (in place); returns the objective
double probe_gauge_opt(int D, int M, int K, double* X, const double* rho, const double* E, const double* G,
                       const double* rT, const double* ET, const double* GT, double w, double gtol, int* iters) {
  if (!X) return -1.0;
  auto f = [&](const double* x, double* g) { return gst::gauge_objective(D, M, K, x, rho, E, G, rT, ET, GT, w, g); };
  gst::LbfgsResult r = gst::lbfgs(D * D, X, f, 10, gtol, 5000);
  *iters = r.iterations;
  return r.f;
}

int probe_gauge_start(int D, int M, int K, const double* rho, const double* E, const double* G, const double* rT,
                      const double* ET, const double* GT, double w, double* X) {
  return gst::gauge_linear_start(D, M, K, rho, E, G, rT, ET, GT, w, X) ? 0 : -1;
}

double probe_rosenbrock(double* x, int* iters) {
  auto f = [](const double* v, double* g) {
    const double a = v[0], b = v[1];
    g[0] = -2 * (1 - a) - 400 * a * (b - a * a);
    g[1] = 200 * (b - a * a);
    return (1 - a) * (1 - a) + 100 * (b - a * a) * (b - a * a);
  };
  gst::LbfgsResult r = gst::lbfgs(2, x, f, 10, 1e-10, 5000);
  *iters = r.iterations;
  return r.f;
}
}
