// Kernels of the block Davidson solver for the lowest eigenvectors of the
// reference-space Hamiltonian H_PP (complex Hermitian, dense, [n][n]).
// A set of vectors is stored one vector per row: X[j][i], i < n.
#include "kernels.hpp"

namespace mrpt2 {

constexpr int DV_COLS = 8;      // vectors per H X launch

// W[c0 + j] = H X[c0 + j], j < nc <= DV_COLS: one wave per row of H, the
// row read once for all nc vectors.  grid (ceil(n / 4)), block 256.
__global__ void __launch_bounds__(256) k_dv_hx(const double2* __restrict__ H, const double2* __restrict__ X,
                                                double2* __restrict__ W, int n, int c0, int nc) {
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + wv;
  if (i >= n) return;                     // whole wave
  double2 acc[DV_COLS];
#pragma unroll
  for (int j = 0; j < DV_COLS; ++j) acc[j] = make_double2(0.0, 0.0);
  const double2* h = H + (int64_t)i * n;
  for (int t = lane; t < n; t += 64) {
    const double2 hv = h[t];
#pragma unroll
    for (int j = 0; j < DV_COLS; ++j)
      if (j < nc) acc[j] = cfma(hv, X[(int64_t)(c0 + j) * n + t], acc[j]);
  }
#pragma unroll
  for (int j = 0; j < DV_COLS; ++j) {
    double x = acc[j].x, y = acc[j].y;
    for (int off = 32; off > 0; off >>= 1) {
      x += __shfl_down(x, off, 64);
      y += __shfl_down(y, off, 64);
    }
    if (lane == 0 && j < nc) W[(int64_t)(c0 + j) * n + i] = make_double2(x, y);
  }
}

// G[a * nb + b] = sum_i conj(A[a0 + a][i]) B[b0 + b][i], one block per (a, b),
// reduced in a fixed order.  grid (na * nb), block 256.
__global__ void __launch_bounds__(256) k_dv_dots(const double2* __restrict__ A, int a0, const double2* __restrict__ B,
                                                  int b0, int nb, int n, double2* __restrict__ G) {
  __shared__ double sx[256], sy[256];
  const int a = blockIdx.x / nb, b = blockIdx.x % nb;
  const double2* x = A + (int64_t)(a0 + a) * n;
  const double2* y = B + (int64_t)(b0 + b) * n;
  double re = 0.0, im = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) {
    const double2 u = x[i], v = y[i];
    re = fma(u.x, v.x, fma(u.y, v.y, re));
    im = fma(u.x, v.y, fma(-u.y, v.x, im));
  }
  sx[threadIdx.x] = re;
  sy[threadIdx.x] = im;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      sx[threadIdx.x] += sx[threadIdx.x + o];
      sy[threadIdx.x] += sy[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) G[blockIdx.x] = make_double2(sx[0], sy[0]);
}

// Y[y0 + j][i] = beta Y[y0 + j][i] + alpha sum_{a < nx} X[x0 + a][i] M[a * ldm + j],
// j < grid.y.  Y must not overlap the rows of X that are read.
// grid (ceil(n / 256), nout), block 256.
__global__ void __launch_bounds__(256) k_dv_comb(const double2* __restrict__ X, int x0, int nx,
                                                  const double2* __restrict__ M, int ldm, double2* Y, int y0,
                                                  double alpha, double beta, int n) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= n) return;
  double2 acc = make_double2(0.0, 0.0);
  for (int a = 0; a < nx; ++a) acc = cfma(X[(int64_t)(x0 + a) * n + i], M[a * ldm + j], acc);
  double2* y = Y + (int64_t)(y0 + j) * n + i;
  const double2 old = beta != 0.0 ? *y : make_double2(0.0, 0.0);
  *y = make_double2(fma(alpha, acc.x, beta * old.x), fma(alpha, acc.y, beta * old.y));
}

// Diagonal-preconditioned residuals, T[t0 + j][i] = R[j][i] / (theta_j - H_ii),
// with the denominator kept at least 1e-8 in magnitude; dg[i] = Re H_ii (the
// dense solver's diagonal or the direct solver's active-space energies, the
// latter having no stored H).  grid (ceil(n/256), nr).
__global__ void __launch_bounds__(256) k_dv_prec(const double* __restrict__ dg, const double2* __restrict__ R,
                                                  const double* __restrict__ theta, double2* T, int t0, int n) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= n) return;
  double den = theta[j] - dg[i];
  if (fabs(den) < 1e-8) den = den < 0.0 ? -1e-8 : 1e-8;
  const double2 r = R[(int64_t)j * n + i];
  T[(int64_t)(t0 + j) * n + i] = make_double2(r.x / den, r.y / den);
}

// X[x0 + j][i] *= s[j] (complex).  grid (ceil(n / 256), nx).
__global__ void __launch_bounds__(256) k_dv_scale(double2* X, int x0, const double2* __restrict__ s, int n) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  double2* x = X + (int64_t)(x0 + blockIdx.y) * n + i;
  *x = cmul(*x, s[blockIdx.y]);
}

// d[i] = Re H_ii.  grid (ceil(n / 256)).
__global__ void __launch_bounds__(256) k_dv_diag(const double2* __restrict__ H, double* d, int n) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) d[i] = H[(int64_t)i * n + i].x;
}

// Direct sigma-build in P: W[c0 + j] = (H_PP - E_core) X[c0 + j], j < nc,
// without a stored H_PP.  Row i applies its excitation list (the reference
// strings one or two active replacements away) with elements from the
// Slater-Condon rules (hpp_element, as the dense H_PP) and adds its diagonal
// (the active-space energy).  One wave per row, the list entries spread over
// the lanes; every element serves all nc vectors.  grid (ceil(n / 4)),
// block 256.
__global__ void __launch_bounds__(256) k_dv_hx_direct(const Inst* __restrict__ insts, int inst,
                                                       const double2* __restrict__ X, double2* __restrict__ W,
                                                       int n, int c0, int nc) {
  const Dev& d = inst_at(insts, inst).d;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + wv;
  if (i >= n) return;                     // whole wave
  const uint64_t bi = d.pstrings[i];
  double2 acc[DV_COLS];
#pragma unroll
  for (int j = 0; j < DV_COLS; ++j) acc[j] = make_double2(0.0, 0.0);
  const int64_t e1 = d.plist_ptr[i + 1];
  for (int64_t e = d.plist_ptr[i] + lane; e < e1; e += 64) {
    const int t = d.plist_col[e];
    const double2 hv = hpp_element(d, bi, d.pstrings[t]);
#pragma unroll
    for (int j = 0; j < DV_COLS; ++j)
      if (j < nc) acc[j] = cfma(hv, X[(int64_t)(c0 + j) * n + t], acc[j]);
  }
  if (lane == 0) {
    const double e = act_energy(d, bi);
#pragma unroll
    for (int j = 0; j < DV_COLS; ++j)
      if (j < nc) {
        const double2 x = X[(int64_t)(c0 + j) * n + i];
        acc[j] = make_double2(fma(e, x.x, acc[j].x), fma(e, x.y, acc[j].y));
      }
  }
#pragma unroll
  for (int j = 0; j < DV_COLS; ++j) {
    double x = acc[j].x, y = acc[j].y;
    for (int off = 32; off > 0; off >>= 1) {
      x += __shfl_down(x, off, 64);
      y += __shfl_down(y, off, 64);
    }
    if (lane == 0 && j < nc) W[(int64_t)(c0 + j) * n + i] = make_double2(x, y);
  }
}

// Diagonal of H_PP - E_core (the active-space energies), for the direct
// solver's starting vectors and preconditioner.  grid (ceil(n / 256)).
__global__ void __launch_bounds__(256) k_dv_diag_direct(const Inst* __restrict__ insts, int inst, double* dg,
                                                         int n) {
  const Dev& d = inst_at(insts, inst).d;
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) dg[i] = act_energy(d, d.pstrings[i]);
}

}  // namespace mrpt2
