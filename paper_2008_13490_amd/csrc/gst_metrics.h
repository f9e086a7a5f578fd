// Post-fit metrics of the estimates (host side, plain C++).
#pragma once

namespace gst {

// Average gate fidelity (thesis Eq. gatemetricsaveragegatefidelity) of the
// operation with transfer matrix R against the unitary channel with transfer
// matrix RU (both D x D row-major, normalized Pauli basis, D = N^2):
// (Tr(RU^T R) + N R[0][0]) / (N (N + 1)); for R of rho -> M rho M^dagger this is
// Eq. gatemetricsaveragegatefidelityEvaluation.
double avg_gate_fidelity(int D, const double* R, const double* RU);

// Eigenvalues of the d x d unitary W (row-major, interleaved real and
// imaginary parts): 2d values (each eigenvalue at least twice), from the
// eigenvectors of a Hermitian combination of W and W^dagger (real symmetric
// embedding, cyclic Jacobi) and their Rayleigh quotients.  false if Jacobi
// does not converge.
bool unitary_eigenvalues(int d, const double* W, double* re, double* im);

// Diamond distance of the unitary channels of U and V (App. H, Eq.
// appdiamondunitaryResult): 1 if the origin lies in the convex hull of the
// eigenvalues of U^dagger V, else half their largest distance.  -1 on failure.
double diamond_unitary(int d, const double* U, const double* V);

// exp(L) of a real D x D matrix (Taylor polynomial of L / 2^s, s squarings).
void expm_real(int D, const double* L, double* E);

// The real principal logarithm of G (inverse scaling and squaring: Denman-
// Beavers square roots until ||A - 1||_F <= 1/4, Taylor series of log(1 + X),
// times 2^k), checked by ||exp(L) - G||_F <= 1e-9 ||G||_F.  false where it does
// not exist (eigenvalues on the closed negative real axis) or the check fails.
bool logm_real(int D, const double* G, double* L);

// App. J: h (D entries, h[0] = 0) of the projection of log G onto the transfer
// matrices of -i[H, .], H = sum_k h_k P_k / 2 (Eq. GateDecompositionHamiltonianProjection),
// and gamma = ||G - exp(L^H)||_F (Eq. GateDecompositionHamiltonianProjectionError).
// 0, or -1 without a real principal logarithm.
int hamiltonian_decomposition(int n, const double* G, double* h, double* gamma);

// h (h_0 = 0) of the target's Hamiltonian H = i log U (U the d x d unitary,
// row-major, interleaved real and imaginary parts; each eigenvalue's argument
// in (-pi, pi]), so that U = exp(-iH) up to a global phase, H = sum_k h_k P_k / 2.
// false if the eigen-decomposition fails.
bool target_hamiltonian(int n, const double* U, double* h);

// App. J for gates with or without a real principal logarithm: h minimizing
// gamma(h) = ||G - exp(L^H(h))||_F (L-BFGS, gradient from the Frechet
// derivative of exp) starting from the target's Hamiltonian; gamma at the
// result.  0, or -1 if the target's eigen-decomposition fails.
int hamiltonian_decomposition_toward(int n, const double* G, const double* U, double* h, double* gamma);

}  // namespace gst
