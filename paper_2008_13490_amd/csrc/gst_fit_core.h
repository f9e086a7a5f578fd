// The fit around the likelihood, host side (plain C++): linear-inversion GST,
// gauge optimization and the limited-memory BFGS minimizer that iterative
// MLGST runs over the GPU evaluations.
#pragma once
#include <stdint.h>

#include <functional>
#include <vector>

namespace gst {

// One-sided Jacobi SVD of the row-major m x n matrix A (m >= n): A = U diag(S) V^T,
// U m x n, V n x n (row-major), S descending.  Returns false if the sweeps do
// not converge.
bool svd_jacobi(int m, int n, const double* A, double* U, double* S, double* V);

// Inverse of the row-major n x n matrix A by LU with partial pivoting; false if
// a pivot is zero.
bool invert(int n, const double* A, double* Ai);

// x = A^-1 b by LU with partial pivoting (row-major A); false if a pivot is zero.
bool solve(int n, const double* A, const double* b, double* x);

// The bare-experiment frequency matrices of LGST, found by word in the list:
// AB [M n_meas][n_prep] (row J + M i: outcome J after measurement fiducial i),
// Bk [K][M n_meas][n_prep] with gate k between the fiducials (time order: the
// preparation fiducial first).  j0 / i0: the positions of the empty fiducials.
// Returns 0, or -1 if a word is missing from the list, -2 if a fiducial list
// has no empty word, -3 if a listed sequence has no counts.
int lgst_matrices(int64_t S, const int64_t* offsets, const uint8_t* gates, const int32_t* counts, int M, int K,
                  int n_prep, const int64_t* prep_off, const uint8_t* prep_gates, int n_meas, const int64_t* meas_off,
                  const uint8_t* meas_gates, std::vector<double>* AB, std::vector<double>* Bk, int* j0, int* i0);

// LGST estimates from the matrices: AB = U S V^T truncated to rank D, each
// singular pair signed so that the largest-magnitude entry of its V column is
// positive; Ahat = U^T AB V, G_k = Ahat^-1 U^T B_k V, rho = Ahat^-1 U^T AB[:, j0],
// E_J = AB[J + M i0, :] V.  Returns 0, -4 if the SVD fails, -5 if Ahat is singular.
int lgst_estimate(int D, int M, int K, int n_prep, int n_meas, const double* AB, const double* Bk, int j0, int i0,
                  double* rho, double* E, double* G);

// sum_k ||X G_k X^-1 - T_k||_F^2 + w (||X rho - rho_T||^2 + sum_m ||X^-T e_m - e_T,m||^2)
// and its gradient with respect to the entries of X (row-major); +inf if X is singular.
double gauge_objective(int D, int M, int K, const double* X, const double* rho, const double* E, const double* G,
                       const double* rT, const double* ET, const double* GT, double w, double* grad);

// X minimizing the quadratic sum_k ||X G_k - T_k X||_F^2 + w (||X rho - rho_T||^2
// + sum_m ||X^T e_T,m - e_m||^2) (the gauge relations multiplied through by X),
// by the normal equations; the start of the gauge optimization.  false if the
// normal matrix is singular.
bool gauge_linear_start(int D, int M, int K, const double* rho, const double* E, const double* G, const double* rT,
                        const double* ET, const double* GT, double w, double* X);

struct LbfgsResult {
  int iterations = 0;
  int evaluations = 0;
  double f = 0.0;
  double gmax = 0.0;  // max |gradient| at the result
  int status = 0;     // 0 gradient tolerance met, 1 iteration limit, 2 line search could not decrease f
};

// Limited-memory BFGS: two-loop recursion with memory m and initial scaling
// s^T y / y^T y; strong Wolfe line search (c1 = 1e-4, c2 = 0.9) that brackets
// by doubling from the unit step and then bisects (at most 60 trials each); a
// step whose objective is not finite counts as too long; pairs with s^T y <= 0
// are skipped.  f(x, grad) returns the objective and writes the gradient.
LbfgsResult lbfgs(int n, double* x, const std::function<double(const double*, double*)>& f, int m, double gtol,
                  int max_iter);

}  // namespace gst
