/* Test infrastructure (oracle): the Epstein-Nesbet sum over the external
 * determinants with two virtual electrons, written out as plain loops.
 *
 * For one set of core holes and a block of n_s external active strings s,
 * the external determinants are K = (core - holes) + alpha_s + {a, b} with
 * virtual spinors a < b.  Their first-order numerators (Sec. 2.3, eq. pt2en)
 * are
 *     sigma_K = sum_k coef[s][k] X[k][a][b],
 * the sum running over the couplings of string s (CSR lists: indices k of
 * the integral matrices X[k][a][b] = <ab||x_k y_k> and the coefficients
 * sign * C_L of the reference determinants L), and the Epstein-Nesbet
 * diagonal (eq. zeroh) is
 *     H_KK = e0[s] + va[s][a] + va[s][b] + Wvv[a][b].
 * The function returns
 *     sum_{s, a < b, amask[a], bmask[b]} |sigma_K|^2 g(E0 - H_KK) / norm,
 * with g(d) = 1/d, or with the imaginary level shift of Sec. 2.6 the real part
 * of 1/(d + i b/d).  Each (s, a) row is summed over b in order; the rows are
 * combined with Neumaier's compensated summation in a fixed order, so the
 * result does not depend on the number of threads.
 *
 * No part of the GPU library is shared with this file.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

static double weight(double d, double b) {
  if (b == 0.0) return 1.0 / d;
  const double eps = b / d;
  return d / (d * d + eps * eps);
}

double oracle_vv_block(int64_t n_s, int64_t nv, const int64_t* ptr, const int64_t* kidx,
                       const double complex* cval, const double complex* X, const double* e0,
                       const double* va, const double* Wvv, const unsigned char* amask,
                       const unsigned char* bmask, double E0, double norm, double b) {
  const int64_t nrow = n_s * nv;
  double* rows = (double*)malloc((size_t)(nrow > 0 ? nrow : 1) * sizeof(double));
  if (!rows) return NAN;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t r = 0; r < nrow; ++r) {
    const int64_t s = r / nv, a = r % nv;
    double acc = 0.0;
    if (amask[a]) {
      for (int64_t bb = a + 1; bb < nv; ++bb) {
        if (!bmask[bb]) continue;
        double complex sig = 0.0;
        for (int64_t e = ptr[s]; e < ptr[s + 1]; ++e)
          sig += cval[e] * X[(kidx[e] * nv + a) * nv + bb];
        const double hkk = e0[s] + va[s * nv + a] + va[s * nv + bb] + Wvv[a * nv + bb];
        const double re = creal(sig), im = cimag(sig);
        acc += (re * re + im * im) * weight(E0 - hkk, b);
      }
    }
    rows[r] = acc / norm;
  }
  double sum = 0.0, comp = 0.0;
  for (int64_t r = 0; r < nrow; ++r) {
    const double x = rows[r], t = sum + x;
    if (fabs(sum) >= fabs(x)) comp += (sum - t) + x;
    else comp += (x - t) + sum;
    sum = t;
  }
  free(rows);
  return sum + comp;
}
