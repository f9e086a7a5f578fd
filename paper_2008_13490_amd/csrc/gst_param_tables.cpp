// Structure tables of the CPTP generator (host side).
//
// For n qubits (D = 4^n), in the normalized Pauli basis with entries
// X[a][b] = tr(P_a X(P_b)) / d:
//   * the map -i [H, .], H = sum_k h_k P_k / 2 (thesis Eq. GateDecompositionHamiltonian),
//     has entries h_{a^b} y[a][b] (P_k P_b is a multiple of P_a only for k = a^b);
//   * the map sum_jk C_jk (P_j . P_k - {P_k P_j, .} / 2) (the dissipator of Eq.
//     masterequation with coefficient matrix C) has entries
//     sum_j Re(C_{j, a^b^j} z[j][a][b]) (zero where a^b^j = 0).
// Pauli labels multiply by XOR of their per-qubit codes (I, X, Y, Z = 0..3);
// the phases follow from sigma_x sigma_y = i sigma_z and its cyclic versions.
#include "gst_param_tables.h"

#include <complex>

namespace gst {
namespace {

using cplx = std::complex<double>;

// sigma_p sigma_q = phase * sigma_{p ^ q} for one qubit (I, X, Y, Z = 0..3)
cplx phase1(int p, int q) {
  if (p == 0 || q == 0 || p == q) return 1.0;
  // X Y = i Z, Y Z = i X, Z X = i Y; the reversed orders carry -i
  const bool cyclic = (p == 1 && q == 2) || (p == 2 && q == 3) || (p == 3 && q == 1);
  return cyclic ? cplx(0.0, 1.0) : cplx(0.0, -1.0);
}

// phase of the product P_{x_0} P_{x_1} ... (a multiple of a Pauli product)
cplx phase_of(const std::vector<int>& xs, int n) {
  cplx ph = 1.0;
  int label = 0;
  for (int x : xs) {
    for (int q = 0; q < n; ++q) {
      const int sh = 2 * (n - 1 - q);
      ph *= phase1((label >> sh) & 3, (x >> sh) & 3);
    }
    label ^= x;
  }
  return ph;
}

}  // namespace

void param_tables(int n, std::vector<double>* y, std::vector<double>* zr, std::vector<double>* zi) {
  const int D = 1 << (2 * n);
  y->assign((size_t)D * D, 0.0);
  zr->assign((size_t)D * D * D, 0.0);
  zi->assign((size_t)D * D * D, 0.0);
  for (int a = 0; a < D; ++a)
    for (int b = 0; b < D; ++b) {
      const int k = a ^ b;
      // tr(P_a (-i/2) [P_k, P_b]) / d, the products being multiples of the identity
      if (k) {
        const cplx v = cplx(0.0, -0.5) * (phase_of({a, k, b}, n) - phase_of({a, b, k}, n));
        (*y)[(size_t)a * D + b] = v.real();
      }
      for (int j = 1; j < D; ++j) {
        const int kk = a ^ b ^ j;
        if (kk == 0) continue;
        // (tr(P_a P_j P_b P_k) - tr(P_a P_k P_j P_b) / 2 - tr(P_a P_b P_k P_j) / 2) / d
        const cplx v = phase_of({a, j, b, kk}, n) - 0.5 * phase_of({a, kk, j, b}, n) -
                       0.5 * phase_of({a, b, kk, j}, n);
        (*zr)[((size_t)j * D + a) * D + b] = v.real();
        (*zi)[((size_t)j * D + a) * D + b] = v.imag();
      }
    }
}


}  // namespace gst
