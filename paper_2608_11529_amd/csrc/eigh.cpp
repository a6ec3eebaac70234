// Eigenpairs of a small complex Hermitian matrix by cyclic Jacobi rotations
// (host only).  The block Davidson solver of the reference states uses it
// for its projected matrix, whose order stays below a few hundred.
//
// Each rotation first turns the phase of column q so that A[p][q] becomes
// real, A <- D^H A D with D = diag(1, .., e^{-i phi}, ..), then applies the
// real symmetric Jacobi rotation that zeroes it; the product of the unitary
// factors accumulates the eigenvectors.  Sweeps repeat until the
// off-diagonal Frobenius norm falls below 1e-15 of the matrix norm.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdint>
#include <numeric>
#include <vector>

#include "mrpt2.h"

namespace {
using cd = std::complex<double>;
}

extern "C" mrpt2_status mrpt2_hermitian_eigh(int32_t n, const double* a, double* w, double* v) {
  if (n < 1 || !a || !w || !v) return MRPT2_ERR_ARG;
  const size_t N = (size_t)n;
  std::vector<cd> A(N * N), V(N * N, cd(0.0, 0.0));
  for (size_t i = 0; i < N * N; ++i) A[i] = cd(a[2 * i], a[2 * i + 1]);
  for (size_t i = 0; i < N; ++i) {
    A[i * N + i] = cd(A[i * N + i].real(), 0.0);
    V[i * N + i] = 1.0;
  }
  double fro = 0.0;
  for (size_t i = 0; i < N * N; ++i) fro += std::norm(A[i]);
  fro = std::sqrt(fro);
  if (!std::isfinite(fro)) return MRPT2_ERR_NUMERIC;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (size_t p = 0; p < N; ++p)
      for (size_t q = p + 1; q < N; ++q) off += std::norm(A[p * N + q]);
    if (std::sqrt(2.0 * off) <= 1e-15 * fro || fro == 0.0) break;
    for (size_t p = 0; p < N; ++p) {
      for (size_t q = p + 1; q < N; ++q) {
        const cd z = A[p * N + q];
        const double r = std::abs(z);
        if (r == 0.0) continue;
        const cd ph = z / r;                       // e^{i phi}
        const cd phc = std::conj(ph);
        // column q times e^{-i phi}, row q times e^{+i phi}
        for (size_t k = 0; k < N; ++k) {
          A[k * N + q] *= phc;
          V[k * N + q] *= phc;
        }
        for (size_t k = 0; k < N; ++k) A[q * N + k] *= ph;
        // real rotation zeroing the now real A[p][q] = r
        const double app = A[p * N + p].real(), aqq = A[q * N + q].real();
        const double tau = (aqq - app) / (2.0 * r);
        const double t = (tau >= 0.0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
        const double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
        for (size_t k = 0; k < N; ++k) {          // columns p, q
          const cd akp = A[k * N + p], akq = A[k * N + q];
          A[k * N + p] = c * akp - s * akq;
          A[k * N + q] = s * akp + c * akq;
          const cd vkp = V[k * N + p], vkq = V[k * N + q];
          V[k * N + p] = c * vkp - s * vkq;
          V[k * N + q] = s * vkp + c * vkq;
        }
        for (size_t k = 0; k < N; ++k) {          // rows p, q
          const cd apk = A[p * N + k], aqk = A[q * N + k];
          A[p * N + k] = c * apk - s * aqk;
          A[q * N + k] = s * apk + c * aqk;
        }
        A[p * N + q] = 0.0;
        A[q * N + p] = 0.0;
        A[p * N + p] = cd(A[p * N + p].real(), 0.0);
        A[q * N + q] = cd(A[q * N + q].real(), 0.0);
      }
    }
  }
  // ascending eigenvalues; eigenvector j in column j of v (row-major n x n)
  std::vector<size_t> idx(N);
  std::iota(idx.begin(), idx.end(), 0);
  std::vector<double> d(N);
  for (size_t i = 0; i < N; ++i) d[i] = A[i * N + i].real();
  std::sort(idx.begin(), idx.end(), [&](size_t x, size_t y) { return d[x] < d[y]; });
  for (size_t j = 0; j < N; ++j) {
    w[j] = d[idx[j]];
    for (size_t k = 0; k < N; ++k) {
      v[2 * (k * N + j)] = V[k * N + idx[j]].real();
      v[2 * (k * N + j) + 1] = V[k * N + idx[j]].imag();
    }
  }
  return MRPT2_OK;
}
