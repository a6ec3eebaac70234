// One-pass tables over the Cholesky factors (frozen-core fold, core Fock
// matrix, pair energies) and the complex FP64 MFMA integral builds.
#include "kernels.hpp"

namespace mrpt2 {

// Slab of the factor columns of every occupied-type spinor x (frozen core,
// core, active): slab[x][pc][L] = sqrt|w| B[L][n_fc + pc][x], and the scaled
// diagonals dg[L][p] = sqrt|w| Re B[L][p][p].  The mixed form also writes the
// FP32 copy slab32 of the virtual rows (pc >= n_o) of the non-frozen x, with
// the column multiplied by i where w < 0: a product of two such entries then
// carries the weight's sign, with the rounding of the unrotated product.
// Grid (ceil(rank/64), n_corr) per factor set, block 256.
__device__ __forceinline__ void pack_body(const Dev& d, int t, const uint3 bid) {
  const double2* __restrict__ B = d.sets.B[t];
  const int l0 = d.sets.l0[t], rank = d.sets.rank[t];
  __shared__ double2 tile[64][17];
  const int pc = bid.y;
  const int Lb = bid.x * 64;
  const int row = d.n_fc + pc;
  for (int x0 = 0; x0 < d.n_occ; x0 += 16) {
    for (int e = threadIdx.x; e < 64 * 16; e += 256) {
      const int li = e >> 4, xi = e & 15;
      const int L = Lb + li, x = x0 + xi;
      double2 v = make_double2(0.0, 0.0);
      if (L < rank && x < d.n_occ) v = fac_at(d.sets, B, L, row, x, d.n);
      tile[li][xi] = v;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 64 * 16; e += 256) {
      const int xi = e >> 6, li = e & 63;
      const int L = Lb + li, x = x0 + xi;
      if (L < rank && x < d.n_occ) {
        const double s = d.scale[l0 + L];
        const double2 v = tile[li][xi];
        d.slab[((int64_t)x * d.n_corr + pc) * d.n_l + l0 + L] = make_double2(s * v.x, s * v.y);
        if (d.slab32 && x >= d.n_fc && pc >= d.n_o) {
          const int64_t o = ((int64_t)(x - d.n_fc) * d.n_v + (pc - d.n_o)) * d.n_l2 + l0 + L;
          const float re = (float)(s * v.x), im = (float)(s * v.y);
          d.slab32[o] = d.sign[l0 + L] < 0.0 ? make_float2(-im, re) : make_float2(re, im);
          if (l0 + L + 1 == d.n_l && d.n_l2 > d.n_l) d.slab32[o + 1] = make_float2(0.f, 0.f);
        }
      }
    }
    __syncthreads();
  }
}

// grid (ceil(n/256), rank)
__device__ __forceinline__ void diag_body(const Dev& d, int t, const uint3 bid) {
  const double2* __restrict__ B = d.sets.B[t];
  const int l0 = d.sets.l0[t], rank = d.sets.rank[t];
  const int p = bid.x * 256 + threadIdx.x;
  const int L = bid.y;
  if (p >= d.n || L >= rank) return;
  d.dg[(int64_t)(l0 + L) * d.n + p] = d.scale[l0 + L] * fac_at(d.sets, B, L, p, p, d.n).x;
}

// Pair energies W_pq = (pp|qq) - (pq|qp) over all spinors, streaming every
// factor once: (pq|qp) = sum_L w_L |B_pq|^2 for Hermitian B.  W is
// symmetric: with packed factors only q >= p is read (rows of the stored
// triangle, contiguous in q) and each entry is also written to (q, p).
// grid (ceil(n/256), n), block 256.  Sets flag on non-finite results.
__device__ __forceinline__ void wpass_body(const Dev& d, int* flag, const uint3 bid) {
  const SetPtrs& sp = d.sets;
  const int q = bid.x * 256 + threadIdx.x;
  const int p = bid.y;
  if (q >= d.n || (sp.packed && q < p)) return;
  double coul = 0.0, exch = 0.0;
  for (int t = 0; t < sp.n_sets; ++t) {
    const double2* __restrict__ B = sp.B[t] + (sp.packed ? tri_off(p, q, d.n) : (int64_t)p * d.n + q);
    const int64_t stride = fac_stride(sp, d.n);
    const int l0 = sp.l0[t];
    const int rank = sp.rank[t];
    int L = 0;
    for (; L + 4 <= rank; L += 4) {
      double2 v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = B[(int64_t)(L + u) * stride];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int Lg = l0 + L + u;
        const double sg = d.sign[Lg], sc = d.scale[Lg];
        exch = fma(sg * sc * sc, cabs2(v[u]), exch);
        coul = fma(sg * d.dg[(int64_t)Lg * d.n + p], d.dg[(int64_t)Lg * d.n + q], coul);
      }
    }
    for (; L < rank; ++L) {
      const double2 v = B[(int64_t)L * stride];
      const int Lg = l0 + L;
      const double sg = d.sign[Lg], sc = d.scale[Lg];
      exch = fma(sg * sc * sc, cabs2(v), exch);
      coul = fma(sg * d.dg[(int64_t)Lg * d.n + p], d.dg[(int64_t)Lg * d.n + q], coul);
    }
  }
  double w = (p == q) ? 0.0 : coul - exch;
  if (!isfinite(w) || !isfinite(coul + exch)) {
    *flag = 1;
    w = 0.0;
  }
  d.W[(int64_t)p * d.n + q] = w;
  if (sp.packed && q != p) d.W[(int64_t)q * d.n + p] = w;
}

// Orbital energies in the field of the frozen and correlated core:
// eps_p = h_pp + sum_{j in core, j != p} W_pj (frozen core included).
__device__ __forceinline__ void eps_body(const Dev& d, int* flag, const uint3 bid) {
  const double2* __restrict__ h = d.h;
  const int pc = bid.x * 256 + threadIdx.x;
  if (pc >= d.n_corr) return;
  const int g = d.n_fc + pc;
  double e = h[(int64_t)g * d.n + g].x;
  for (int j = 0; j < d.n_fc + d.n_c; ++j)
    if (j != g) e += d.W[(int64_t)g * d.n + j];
  if (!isfinite(e) || !isfinite(h[(int64_t)g * d.n + g].y)) *flag = 1;
  d.eps[pc] = e;
}

// dsum[L] = sum over frozen and correlated core j of dg[L][j].
__device__ __forceinline__ void dsum_body(const Dev& d, const uint3 bid) {
  const int L = bid.x * 256 + threadIdx.x;
  if (L >= d.n_l) return;
  double s = 0.0;
  for (int j = 0; j < d.n_fc + d.n_c; ++j) s += d.dg[(int64_t)L * d.n + j];
  d.dsum[L] = s;
}

// Core Fock matrix f_pq = h_pq + sum_{j in core} [(pq|jj) - (pj|jq)] for p
// active or virtual and q core or active (frozen-core fold of Sec. 2 plus the
// correlated core): the Coulomb part sum_L w_L B_pq^L dsum_L per entry, the
// exchange part from the per-core-spinor partials fx (fockx_body), summed in
// core order.  grid (n_o, n_a + n_v), one wavefront per entry.
__device__ __forceinline__ void fock_body(const Dev& d, const uint3 bid) {
  const double2* __restrict__ h = d.h;
  const int qo = bid.x;
  const int pr = bid.y;
  const int lane = threadIdx.x;
  const int pcorr = d.n_c + pr;
  double2 acc = make_double2(0.0, 0.0);
  const double2* Bq = d.slab + ((int64_t)(d.n_fc + qo) * d.n_corr + pcorr) * d.n_l;
  for (int L = lane; L < d.n_l; L += 64) {
    const double s = d.sign[L] * d.dsum[L];
    acc.x = fma(s, Bq[L].x, acc.x);
    acc.y = fma(s, Bq[L].y, acc.y);
  }
  for (int off = 32; off > 0; off >>= 1) {
    acc.x += __shfl_down(acc.x, off, 64);
    acc.y += __shfl_down(acc.y, off, 64);
  }
  if (lane == 0) {
    const int np = d.n_a + d.n_v;
    for (int j = 0; j < d.n_fc + d.n_c; ++j) {
      const double2 x = d.fx[((int64_t)j * np + pr) * d.n_o + qo];
      acc.x -= x.x;
      acc.y -= x.y;
    }
    const int gp = d.n_fc + pcorr, gq = d.n_fc + qo;
    const double2 hv = h[(int64_t)gp * d.n + gq];
    d.f[(int64_t)pr * d.n_o + qo] = make_double2(hv.x + acc.x, hv.y + acc.y);
  }
}

// ---- complex FP64 MFMA tile: C[64][64] = sum_k a(r,k) b(c,k) ----------------
typedef double d4 __attribute__((ext_vector_type(4)));
constexpr int KC = 16;
constexpr int KP = KC + 1;

// v_mfma_f64_16x16x4f64 operand layout: lane l holds A[l%16][l/16] and
// B[l/16][l%16]; the result D[i][j] sits in lane j + 16 (i%4), register i/4.
// A complex product uses two real MFMAs per pair of complex k:
//   Re += [ar, -ai] . [br; bi],   Im += [ai, ar] . [br; bi].
// TA = double4: the A operand is staged as (re, im, -im, re) per complex k, so
// that the lanes holding the second real k of a pair read the (-im, re) half
// and every operand comes straight from LDS (no per-step selects; twice the
// LDS of the A stage, which costs occupancy where many small blocks run).
// TA = double2: staged as (re, im), the lanes select their parts.
// BCOL: b(c, k) is read with c fastest across threads (operands stored k-major).
// ZERO = false adds to the accumulators instead of starting from zero.
template <bool BCOL = false, bool ZERO = true, class TA, class FA, class FB>
__device__ __forceinline__ void cgemm64(FA fa, FB fb, int K, TA* sA, double2* sB,
                                        d4 (&accR)[2][2], d4 (&accI)[2][2]) {
  constexpr bool PAIR = sizeof(TA) == 32;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wr = (wv >> 1) * 32, wc = (wv & 1) * 32;
  if (ZERO) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        accR[i][j] = d4{0.0, 0.0, 0.0, 0.0};
        accI[i][j] = d4{0.0, 0.0, 0.0, 0.0};
      }
  }
  const int kq = lane >> 4;           // 0..3
  const int kcl = kq >> 1, comp = kq & 1;
  for (int k0 = 0; k0 < K; k0 += KC) {
    for (int e = tid; e < 64 * KC; e += 256) {
      const int r = e / KC, kk = e % KC;
      const bool in = (k0 + kk) < K;
      const double2 v = in ? fa(r, k0 + kk) : make_double2(0.0, 0.0);
      if constexpr (PAIR) sA[r * KP + kk] = make_double4(v.x, v.y, -v.y, v.x);
      else sA[r * KP + kk] = v;
      if (!BCOL) sB[r * KP + kk] = in ? fb(r, k0 + kk) : make_double2(0.0, 0.0);
    }
    if (BCOL)
      for (int e = tid; e < 64 * KC; e += 256) {
        const int c = e & 63, kk = e >> 6;
        sB[c * KP + kk] = (k0 + kk) < K ? fb(c, k0 + kk) : make_double2(0.0, 0.0);
      }
    __syncthreads();
#pragma unroll 2
    for (int ks = 0; ks < KC; ks += 2) {
      const int kc = ks + kcl;
      double ar[2], ai[2], bb[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        if constexpr (PAIR) {
          const double2 v = ((const double2*)&sA[(wr + i * 16 + (lane & 15)) * KP + kc])[comp];
          ar[i] = v.x;
          ai[i] = v.y;
        } else {
          const double2 v = sA[(wr + i * 16 + (lane & 15)) * KP + kc];
          ar[i] = comp ? -v.y : v.x;
          ai[i] = comp ? v.x : v.y;
        }
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) bb[j] = ((const double*)&sB[(wc + j * 16 + (lane & 15)) * KP + kc])[comp];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          accR[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i], bb[j], accR[i][j], 0, 0, 0);
          accI[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[i], bb[j], accI[i][j], 0, 0, 0);
        }
    }
    __syncthreads();
  }
}

// Row/column of accumulator element (i, j, reg) for this lane.
__device__ __forceinline__ int acc_row(int i, int r) {
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  return (wv >> 1) * 32 + i * 16 + (lane >> 4) + 4 * r;
}
__device__ __forceinline__ int acc_col(int j) {
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  return (wv & 1) * 32 + j * 16 + (lane & 15);
}

// Exchange part of the core Fock block, one core spinor j (frozen or
// correlated) at a time: fx[j][p][q] = sum_L w_L B_pj^L B_jq^L
// = sum_L sign_L slab[j][p][L] conj(slab[j][q][L]) (B Hermitian), for p active
// or virtual and q core or active: a complex GEMM with K = n_l on FP64 MFMA.
// grid (ceil((n_a + n_v)/64) * ceil(n_o/64), n_fc + n_c), block 256.
__device__ __forceinline__ void fockx_body(const Dev& d, const uint3 bid) {
  __shared__ double2 sA[64 * KP];
  __shared__ double2 sB[64 * KP];
  const int np = d.n_a + d.n_v;
  const int npt = (np + 63) / 64;
  const int p0 = (int)(bid.x % npt) * 64, q0 = (int)(bid.x / npt) * 64;
  const int j = bid.y;
  const int nl = d.n_l;
  const double2* Sp = d.slab + ((int64_t)j * d.n_corr + d.n_c) * nl;   // rows p (correlated n_c + p)
  const double2* Sq = d.slab + (int64_t)j * d.n_corr * nl;             // rows q (correlated q)
  const double* sg = d.sign;
  auto fa = [&](int r, int k) -> double2 {
    const int p = p0 + r;
    if (p >= np) return make_double2(0.0, 0.0);
    const double2 v = Sp[(int64_t)p * nl + k];
    return make_double2(sg[k] * v.x, sg[k] * v.y);
  };
  auto fb = [&](int c, int k) -> double2 {
    const int q = q0 + c;
    if (q >= d.n_o) return make_double2(0.0, 0.0);
    const double2 v = Sq[(int64_t)q * nl + k];
    return make_double2(v.x, -v.y);
  };
  d4 accR[2][2], accI[2][2];
  cgemm64(fa, fb, nl, sA, sB, accR, accI);
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int jj = 0; jj < 2; ++jj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int p = p0 + acc_row(i, r), q = q0 + acc_col(jj);
        if (p < np && q < d.n_o)
          d.fx[((int64_t)j * np + p) * d.n_o + q] = make_double2(accR[i][jj][r], accI[i][jj][r]);
      }
}

// Antisymmetrised virtual-pair integrals for every occupied pair x < y
// (core or active):  A[xy][a][b] = <ab||xy> = (ax|by) - (ay|bx)
//   = sum_L w_L (B_ax B_by - B_ay B_bx),
// stored per 64 x 64 tile (I, J), I <= J, of virtual pairs, K = 2 n_l.
// One tile per block (instances with few virtual tiles, where the 128 x 128
// form below would leave many of its waves idle).
// grid (n_tp, n_pairs), block 256.
__device__ __forceinline__ void abuild_body(const Dev& d, const uint3 bid) {
  __shared__ double2 sA[64 * KP];
  __shared__ double2 sB[64 * KP];
  const int64_t tp = bid.x;
  int64_t pr = bid.y;
  int xo = 0;
  while (pr >= d.n_o - 1 - xo) {
    pr -= d.n_o - 1 - xo;
    ++xo;
  }
  const int yo = xo + 1 + (int)pr;
  const int I = d.tile_pairs[2 * tp], J = d.tile_pairs[2 * tp + 1];
  const int nl = d.n_l;
  const double2* Sx = d.slab + ((int64_t)(d.n_fc + xo) * d.n_corr + d.n_o) * nl;
  const double2* Sy = d.slab + ((int64_t)(d.n_fc + yo) * d.n_corr + d.n_o) * nl;
  const double* sg = d.sign;
  const int nv = d.n_v;
  auto fa = [&](int r, int k) -> double2 {
    const int a = I * 64 + r;
    if (a >= nv) return make_double2(0.0, 0.0);
    const int L = k < nl ? k : k - nl;
    const double2 v = (k < nl ? Sx : Sy)[(int64_t)a * nl + L];
    return make_double2(sg[L] * v.x, sg[L] * v.y);
  };
  auto fb = [&](int r, int k) -> double2 {
    const int b = J * 64 + r;
    if (b >= nv) return make_double2(0.0, 0.0);
    if (k < nl) return Sy[(int64_t)b * nl + k];
    const double2 v = Sx[(int64_t)b * nl + (k - nl)];
    return make_double2(-v.x, -v.y);
  };
  d4 accR[2][2], accI[2][2];
  cgemm64(fa, fb, 2 * nl, sA, sB, accR, accI);
  double2* out = d.A + ((int64_t)bid.y * d.n_tp + tp) * 4096;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        out[acc_row(i, r) * 64 + acc_col(j)] = make_double2(accR[i][j][r], accI[i][j][r]);
}

// They are built in 128 x 128 blocks of virtual pairs: the block covers
// the four tiles (I, J) = (2 I2 + u, 2 J2 + v), u, v in {0, 1}, I2 <= J2, and
// each of its eight waves computes a 64 x 32 half of one tile on FP64 MFMA
// (four by two 16 x 16 products, real and imaginary parts).  Twice the
// arithmetic per staged operand of the 64 x 64 form: each stage of AK complex
// k stages 256 rows for 128 x 128 products.  The next stage's operands are
// fetched into registers while the current one is multiplied, so the global
// latency hides behind the MFMA work; waves whose tile lies below the diagonal
// (I > J) or past the last virtual tile only help to stage.
// grid (n2 (n2 + 1) / 2 with n2 = ceil(n_vt / 2), n_pairs), block 512.
constexpr int AK = 16;              // complex k per stage
constexpr int AKP = AK + 1;         // padded LDS row (double2)

__device__ __forceinline__ void abuild128_body(const Dev& d, const uint3 bid) {
  // A staged as (re, im, -im, re): the lanes of the second k of a pair read the
  // (-im, re) half, so each MFMA operand comes straight from LDS
  __shared__ double4 sA[128 * AKP];
  __shared__ double2 sB[128 * AKP];
  const int nvt = d.n_vt, nvt2 = (nvt + 1) >> 1;
  int I2 = 0;
  int64_t rem = bid.x;
  while (rem >= nvt2 - I2) {
    rem -= nvt2 - I2;
    ++I2;
  }
  const int J2 = I2 + (int)rem;
  int64_t pr = bid.y;
  int xo = 0;
  while (pr >= d.n_o - 1 - xo) {
    pr -= d.n_o - 1 - xo;
    ++xo;
  }
  const int yo = xo + 1 + (int)pr;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int u = wv >> 2, cq = wv & 3;                 // row half, column quarter of the block
  const int I = 2 * I2 + u, J = 2 * J2 + (cq >> 1);
  const bool active = (I <= J) && (J < nvt);
  const int nl = d.n_l, nv = d.n_v;
  const int K = 2 * nl;
  const double2* __restrict__ Sx = d.slab + ((int64_t)(d.n_fc + xo) * d.n_corr + d.n_o) * nl;
  const double2* __restrict__ Sy = d.slab + ((int64_t)(d.n_fc + yo) * d.n_corr + d.n_o) * nl;
  const double* __restrict__ sg = d.sign;
  const int a0 = I2 * 128, b0 = J2 * 128;
  // staging: element e = tid + 512 q (q < 4) of each operand is row e / AK,
  // k e % AK.  The raw values are fetched into registers and scaled (sign of
  // the factor, minus of the exchange half) only when stored, so nothing
  // waits for the fetch before the stage's products.
  double2 ra[4], rb[4];
  double rs[4];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 512 * q;
      const int r = e / AK, k = k0 + e % AK;
      const bool first = k < nl;
      const int L = first ? k : k - nl;
      const int a = a0 + r, b = b0 + r;
      ra[q] = make_double2(0.0, 0.0);
      rb[q] = make_double2(0.0, 0.0);
      rs[q] = 0.0;
      if (k < K) {
        rs[q] = sg[L];
        if (a < nv) ra[q] = (first ? Sx : Sy)[(int64_t)a * nl + L];
        if (b < nv) rb[q] = (first ? Sy : Sx)[(int64_t)b * nl + L];
      }
    }
  };
  d4 accR[4][2], accI[4][2];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      accR[i][j] = d4{0.0, 0.0, 0.0, 0.0};
      accI[i][j] = d4{0.0, 0.0, 0.0, 0.0};
    }
  const int kq = lane >> 4, kcl = kq >> 1, comp = kq & 1;
  const int rowA = u * 64 + (lane & 15), rowB = cq * 32 + (lane & 15);
  fetch(0);
  for (int k0 = 0; k0 < K; k0 += AK) {
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 512 * q;
      const double m = (k0 + e % AK) < nl ? 1.0 : -1.0;
      const double xr = rs[q] * ra[q].x, xi = rs[q] * ra[q].y;
      sA[(e / AK) * AKP + e % AK] = make_double4(xr, xi, -xi, xr);
      sB[(e / AK) * AKP + e % AK] = make_double2(m * rb[q].x, m * rb[q].y);
    }
    __syncthreads();
    if (k0 + AK < K) fetch(k0 + AK);
    if (active) {
#pragma unroll 2
      for (int ks = 0; ks < AK; ks += 2) {
        const int kc = ks + kcl;
        double ar[4], ai[4], bb[2];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const double2 v = ((const double2*)&sA[(rowA + i * 16) * AKP + kc])[comp];
          ar[i] = v.x;
          ai[i] = v.y;
        }
#pragma unroll
        for (int j = 0; j < 2; ++j) bb[j] = ((const double*)&sB[(rowB + j * 16) * AKP + kc])[comp];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j) {
            accR[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i], bb[j], accR[i][j], 0, 0, 0);
            accI[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[i], bb[j], accI[i][j], 0, 0, 0);
          }
      }
    }
  }
  if (!active) return;
  const int64_t tp = (int64_t)I * nvt - (int64_t)I * (I - 1) / 2 + (J - I);
  double2* out = d.A + ((int64_t)bid.y * d.n_tp + tp) * 4096 + (cq & 1) * 32;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        out[(i * 16 + (lane >> 4) + 4 * r) * 64 + j * 16 + (lane & 15)] = make_double2(accR[i][j][r], accI[i][j][r]);
}

// ---- mixed precision: complex FP32 MFMA with FP64 carry ---------------------
typedef float f4 __attribute__((ext_vector_type(4)));
constexpr int KC32 = 32;            // complex k per stage
constexpr int KP32 = KC32 + 1;

// v_mfma_f32_16x16x4f32: lane l holds A[l%16][l/16] and B[l/16][l%16]; the
// result D[i][j] sits in lane j + 16 (i/4), register i%4.  Products and the
// sums over one stage (KC32 complex k) are FP32; every stage's partial sums
// are added into FP64 accumulators, so the FP32 rounding of a sum grows
// with the stage length only.
//
// Complex FP32 GEMM with three real products per complex product (Gauss):
// P1 = sum a_re b_re, P2 = sum a_im b_im, P3 = sum (a_re + a_im)(b_re + b_im)
// over a stage, Re = P1 - P2 and Im = P3 - P1 - P2 formed in FP64 when each
// stage's partial sums are carried; a quarter fewer MFMAs than the four-product
// form.  The operands are staged as three real planes (re, im, re + im) per
// matrix, four complex k per MFMA.  The loaders return two complex FP32
// operands (k, k+1) for even k; each stage's loads are issued two stages
// ahead and complete behind the MFMAs of the stages in between.
template <class FA, class FB>
__device__ __forceinline__ void cgemm64_f32_3m(FA fa, FB fb, int K, float* sA, float* sB,
                                               double (&accR)[2][2][4], double (&accI)[2][2][4]) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wr = (wv >> 1) * 32, wc = (wv & 1) * 32;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        accR[i][j][r] = 0.0;
        accI[i][j][r] = 0.0;
      }
  constexpr int HP = KC32 / 2;                // operand pairs per staged row
  constexpr int PER = 64 * HP / 256;          // pairs per thread and operand
  constexpr int PL = 64 * KP32;               // floats of one plane
  float4 ra0[PER], rb0[PER], ra1[PER], rb1[PER];
  auto fetch = [&](float4 (&ra)[PER], float4 (&rb)[PER], int k0) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = tid + 256 * u;
      const int r = e / HP, k = k0 + 2 * (e % HP);
      ra[u] = k < K ? fa(r, k) : make_float4(0.f, 0.f, 0.f, 0.f);
      rb[u] = k < K ? fb(r, k) : make_float4(0.f, 0.f, 0.f, 0.f);
    }
  };
  auto stage = [&](float4 (&ra)[PER], float4 (&rb)[PER], int k0) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = tid + 256 * u;
      const int o = (e / HP) * KP32 + 2 * (e % HP);
      sA[o] = ra[u].x;
      sA[o + 1] = ra[u].z;
      sA[PL + o] = ra[u].y;
      sA[PL + o + 1] = ra[u].w;
      sA[2 * PL + o] = ra[u].x + ra[u].y;
      sA[2 * PL + o + 1] = ra[u].z + ra[u].w;
      sB[o] = rb[u].x;
      sB[o + 1] = rb[u].z;
      sB[PL + o] = rb[u].y;
      sB[PL + o + 1] = rb[u].w;
      sB[2 * PL + o] = rb[u].x + rb[u].y;
      sB[2 * PL + o + 1] = rb[u].z + rb[u].w;
    }
    __syncthreads();
    if (k0 + 2 * KC32 < K) fetch(ra, rb, k0 + 2 * KC32);
    f4 p1[2][2], p2[2][2], p3[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        p1[i][j] = f4{0.f, 0.f, 0.f, 0.f};
        p2[i][j] = f4{0.f, 0.f, 0.f, 0.f};
        p3[i][j] = f4{0.f, 0.f, 0.f, 0.f};
      }
#pragma unroll 1
    for (int ks = 0; ks < KC32; ks += 4) {
      const int kc = ks + (lane >> 4);
      float a[3][2], b[3][2];
#pragma unroll
      for (int q = 0; q < 3; ++q) {
#pragma unroll
        for (int i = 0; i < 2; ++i) a[q][i] = sA[q * PL + (wr + i * 16 + (lane & 15)) * KP32 + kc];
#pragma unroll
        for (int j = 0; j < 2; ++j) b[q][j] = sB[q * PL + (wc + j * 16 + (lane & 15)) * KP32 + kc];
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          p1[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[0][i], b[0][j], p1[i][j], 0, 0, 0);
          p2[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[1][i], b[1][j], p2[i][j], 0, 0, 0);
          p3[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[2][i], b[2][j], p3[i][j], 0, 0, 0);
        }
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const double x1 = (double)p1[i][j][r], x2 = (double)p2[i][j][r];
          accR[i][j][r] += x1 - x2;
          accI[i][j][r] += ((double)p3[i][j][r] - x1) - x2;
        }
    __syncthreads();
  };
  fetch(ra0, rb0, 0);
  if (KC32 < K) fetch(ra1, rb1, KC32);
  for (int k0 = 0; k0 < K; k0 += 2 * KC32) {
    stage(ra0, rb0, k0);
    if (k0 + KC32 < K) stage(ra1, rb1, k0 + KC32);
  }
}

__device__ __forceinline__ int acc_row_f32(int i, int r) {
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  return (wv >> 1) * 32 + i * 16 + 4 * (lane >> 4) + r;
}

// Complex FP32-MFMA product (four real products per complex product) for
// FP64 operands given element by element: each is rounded to FP32 when
// staged (b with c fastest across threads), the sums over one stage of KC32
// complex k are FP32 and are added into FP64 accumulators.  Result layout
// acc_row_f32, acc_col.
template <class FA, class FB>
__device__ __forceinline__ void cgemm64_f32c(FA fa, FB fb, int K, float2* sA, float2* sB,
                                             double (&accR)[2][2][4], double (&accI)[2][2][4]) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wr = (wv >> 1) * 32, wc = (wv & 1) * 32;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        accR[i][j][r] = 0.0;
        accI[i][j][r] = 0.0;
      }
  const int kq = lane >> 4;
  const int kcl = kq >> 1, comp = kq & 1;
  for (int k0 = 0; k0 < K; k0 += KC32) {
    for (int e = tid; e < 64 * KC32; e += 256) {
      const int r = e / KC32, kk = e % KC32;
      const double2 v = (k0 + kk) < K ? fa(r, k0 + kk) : make_double2(0.0, 0.0);
      sA[r * KP32 + kk] = make_float2((float)v.x, (float)v.y);
    }
    for (int e = tid; e < 64 * KC32; e += 256) {
      const int c = e & 63, kk = e >> 6;
      const double2 v = (k0 + kk) < K ? fb(c, k0 + kk) : make_double2(0.0, 0.0);
      sB[c * KP32 + kk] = make_float2((float)v.x, (float)v.y);
    }
    __syncthreads();
    f4 pR[2][2], pI[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        pR[i][j] = f4{0.f, 0.f, 0.f, 0.f};
        pI[i][j] = f4{0.f, 0.f, 0.f, 0.f};
      }
#pragma unroll 4
    for (int ks = 0; ks < KC32; ks += 2) {
      const int kc = ks + kcl;
      float ar[2], ai[2], bb[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const float2 v = sA[(wr + i * 16 + (lane & 15)) * KP32 + kc];
        ar[i] = comp ? -v.y : v.x;
        ai[i] = comp ? v.x : v.y;
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const float2 v = sB[(wc + j * 16 + (lane & 15)) * KP32 + kc];
        bb[j] = comp ? v.y : v.x;
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          pR[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[i], bb[j], pR[i][j], 0, 0, 0);
          pI[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(ai[i], bb[j], pI[i][j], 0, 0, 0);
        }
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          accR[i][j][r] += (double)pR[i][j][r];
          accI[i][j][r] += (double)pI[i][j][r];
        }
    __syncthreads();
  }
}

// Mixed-precision form of k_abuild: the same integrals and output layout,
// from the FP32 slab.
__device__ __forceinline__ void abuild_f32_body(const Dev& d, const uint3 bid) {
  __shared__ float sA[3 * 64 * KP32];
  __shared__ float sB[3 * 64 * KP32];
  const int64_t tp = bid.x;
  int64_t pr = bid.y;
  int xo = 0;
  while (pr >= d.n_o - 1 - xo) {
    pr -= d.n_o - 1 - xo;
    ++xo;
  }
  const int yo = xo + 1 + (int)pr;
  const int I = d.tile_pairs[2 * tp], J = d.tile_pairs[2 * tp + 1];
  // K runs over [x-columns, y-columns] of the FP32 slab (rows of n_l2 pairs,
  // zero-padded): A[a][k] = (S_x[a] | S_y[a]), B[b][k] = (S_y[b] | -S_x[b]);
  // the factor signs are carried by the slab itself.
  const int nl2 = d.n_l2;
  const float4* Sx = (const float4*)(d.slab32 + (int64_t)xo * d.n_v * nl2);
  const float4* Sy = (const float4*)(d.slab32 + (int64_t)yo * d.n_v * nl2);
  const int nv = d.n_v;
  const int h2 = nl2 >> 1;
  auto fa = [&](int r, int k) -> float4 {
    const int a = I * 64 + r;
    if (a >= nv) return make_float4(0.f, 0.f, 0.f, 0.f);
    const int kp = k >> 1;
    return kp < h2 ? Sx[(int64_t)a * h2 + kp] : Sy[(int64_t)a * h2 + kp - h2];
  };
  auto fb = [&](int r, int k) -> float4 {
    const int b = J * 64 + r;
    if (b >= nv) return make_float4(0.f, 0.f, 0.f, 0.f);
    const int kp = k >> 1;
    if (kp < h2) return Sy[(int64_t)b * h2 + kp];
    const float4 v = Sx[(int64_t)b * h2 + kp - h2];
    return make_float4(-v.x, -v.y, -v.z, -v.w);
  };
  double accR[2][2][4], accI[2][2][4];
  cgemm64_f32_3m(fa, fb, 2 * nl2, sA, sB, accR, accI);
  double2* out = d.A + ((int64_t)bid.y * d.n_tp + tp) * 4096;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        out[acc_row_f32(i, r) * 64 + acc_col(j)] = make_double2(accR[i][j][r], accI[i][j][r]);
}

// Integrals with one active or virtual and one active spinor against two
// occupied ones: G[x][p][y][q] = (px|qy), x, y core or active, p active or
// virtual, q active.  One GEMM: rows (x, p), columns (y, q), K = n_l.
// grid (ceil(N/64), ceil(M/64)), block 256.
__device__ __forceinline__ void gbuild_body(const Dev& d, const uint3 bid) {
  __shared__ double2 sA[64 * KP];
  __shared__ double2 sB[64 * KP];
  const int npr = d.n_a + d.n_v;
  const int64_t M = (int64_t)d.n_o * npr;
  const int64_t N = (int64_t)d.n_o * d.n_a;
  const int64_t m0 = (int64_t)bid.y * 64, n0 = (int64_t)bid.x * 64;
  const int nl = d.n_l;
  const double* sg = d.sign;
  auto fa = [&](int r, int k) -> double2 {
    const int64_t m = m0 + r;
    if (m >= M) return make_double2(0.0, 0.0);
    const int xo = (int)(m / npr), p = (int)(m % npr);
    const double2 v = d.slab[((int64_t)(d.n_fc + xo) * d.n_corr + d.n_c + p) * nl + k];
    return make_double2(sg[k] * v.x, sg[k] * v.y);
  };
  auto fb = [&](int r, int k) -> double2 {
    const int64_t nn = n0 + r;
    if (nn >= N) return make_double2(0.0, 0.0);
    const int yo = (int)(nn / d.n_a), q = (int)(nn % d.n_a);
    return d.slab[((int64_t)(d.n_fc + yo) * d.n_corr + d.n_c + q) * nl + k];
  };
  d4 accR[2][2], accI[2][2];
  cgemm64(fa, fb, nl, sA, sB, accR, accI);
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t m = m0 + acc_row(i, r), nn = n0 + acc_col(j);
        if (m < M && nn < N) d.G[m * N + nn] = make_double2(accR[i][j][r], accI[i][j][r]);
      }
}

}  // namespace mrpt2
