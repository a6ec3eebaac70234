// Host-only driver of the plan builder and of the Hermitian eigensolver, for
// a build with the address and undefined-behaviour sanitizers (test
// infrastructure).  It reads plan descriptors from a file of records
// (int32 n_inst, then n_inst mrpt2_desc structures), builds every plan,
// describes every work block of every class (at most 20000 per class,
// evenly spaced), and solves random Hermitian matrices of orders 1..40
// checking the residual of each eigenpair.  One line per plan: status and
// the external determinant count per instance.
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "plan.hpp"

extern "C" mrpt2_status mrpt2_hermitian_eigh(int32_t n, const double* a, double* w, double* v);

int main(int argc, char** argv) {
  if (argc < 2) return 2;
  FILE* f = std::fopen(argv[1], "rb");
  if (!f) return 2;
  int32_t n = 0;
  while (std::fread(&n, sizeof(n), 1, f) == 1) {
    std::vector<mrpt2_desc> d((size_t)(n > 0 ? n : 1));
    if (n > 0 && std::fread(d.data(), sizeof(mrpt2_desc), (size_t)n, f) != (size_t)n) return 2;
    mrpt2::Plan P;
    std::string err;
    const mrpt2_status st = mrpt2::build_plan(d.data(), n, nullptr, &P, &err);
    std::printf("plan %d", (int)st);
    if (st == MRPT2_OK) {
      for (const auto& ip : P.inst) {
        std::printf(" %lld", (long long)ip.info.n_ext);
        for (int k = 0; k < MRPT2_N_CLASS; ++k) {
          const auto& cp = ip.cls[k];
          const int64_t nb = (cp.strings.empty() || cp.n_rows == 0) ? 0 : cp.n_blocks;
          const int64_t step = nb > 20000 ? nb / 20000 : 1;
          for (int64_t b = 0; b < nb; b += step) {
            mrpt2_block o;
            mrpt2::class_block(ip, k, b, &o);
            if (o.s_lo < 0 || o.s_hi > (int64_t)cp.strings.size() || o.s_lo > o.s_hi) {
              std::printf(" bad-block");
              return 1;
            }
          }
        }
      }
    }
    std::printf("\n");
  }
  std::fclose(f);
  std::srand(7);
  for (int m = 1; m <= 40; ++m) {
    std::vector<std::complex<double>> A((size_t)m * m);
    for (int i = 0; i < m; ++i)
      for (int j = 0; j <= i; ++j) {
        const double re = std::rand() / (double)RAND_MAX - 0.5, im = (i == j) ? 0.0 : std::rand() / (double)RAND_MAX - 0.5;
        A[(size_t)i * m + j] = {re, im};
        A[(size_t)j * m + i] = {re, -im};
      }
    std::vector<double> w((size_t)m), v((size_t)2 * m * m);
    if (mrpt2_hermitian_eigh(m, reinterpret_cast<const double*>(A.data()), w.data(), v.data()) != MRPT2_OK) return 1;
    const auto* V = reinterpret_cast<const std::complex<double>*>(v.data());
    double worst = 0.0;
    for (int k = 0; k < m; ++k)
      for (int i = 0; i < m; ++i) {
        std::complex<double> r = -w[k] * V[(size_t)i * m + k];
        for (int j = 0; j < m; ++j) r += A[(size_t)i * m + j] * V[(size_t)j * m + k];
        worst = std::max(worst, std::abs(r));
      }
    if (!(worst < 1e-10)) {
      std::printf("eigh residual %g at order %d\n", worst, m);
      return 1;
    }
  }
  std::printf("eigh ok\n");
  return 0;
}
