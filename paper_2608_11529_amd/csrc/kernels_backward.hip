// Adjoint of the MRPT2 energy: dE2/dh, dE2/dB (every factor set) and dE2/dC.
//
// With t_K = sigma_K / Delta_K and N = ||C||^2,
//   E2 = sum_K |sigma_K|^2 / (N Delta_K),
// the gradient (convention dE/dRe z + i dE/dIm z) of each determinant's term is
//   sigma-bar_K = 2 t_K / N,   Delta-bar_K = -|t_K|^2 / N,
// and E2 itself carries -E2/N per unit of N.  The first-order vector is never
// stored: each pass recomputes sigma_K and Delta_K for the determinants it
// owns.  Per class two passes share the work:
//   row pass    (one thread per row, every string): the adjoints of the
//               couplings X (or the pair integrals A), of the row constants
//               of Delta (eps, W of core/virtual spinors) and of the string
//               tables Uc, Uv, contracted with the string occupations;
//   string pass (one thread per string, a range of rows): the adjoint of the
//               coefficients through each coupling, and of T (and so of E0
//               and of the active-space energy of the string).
// The table adjoints are then carried back through the forward steps: the
// reference energy (H_PP), the coupling build, the pair and occupied-block
// integrals (complex FP64 MFMA, transposed), the core Fock block, the orbital
// energies and the pair energies W, and the last pass writes every factor's
// gradient once, Hermitian-projected: (G + G^H) / 2.
//
// Accumulations that many threads share use FP64 atomics; their order is not
// fixed, so the gradient is reproducible to rounding, not bit for bit.
#include "kernels.hpp"
#include "plan.hpp"

namespace mrpt2 {

__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ void catomic(double2* p, double2 v) {
  atomicAdd(&p->x, v.x);
  atomicAdd(&p->y, v.y);
}
__device__ __forceinline__ int64_t gidx(const Dev& d, int xo, int pr, int yo, int qa) {
  return (((int64_t)xo * (d.n_a + d.n_v) + pr) * d.n_o + yo) * d.n_a + qa;
}

// Region clear.  grid (gx), block 256, grid-stride.
__device__ __forceinline__ void bzero_body(const GradDev& g, const uint3 bid, int64_t nblk) {
  const double4 z = make_double4(0.0, 0.0, 0.0, 0.0);
  for (int64_t i = (int64_t)bid.x * 256 + threadIdx.x; i < g.n_zero; i += nblk * 256) g.zero[i] = z;
}

// Sum of v over a block of 256 threads in a fixed order (each wave by a fixed
// butterfly, then the four waves in order); every thread of the block must
// call it.  The adjoint's row passes write E2 per block with it, so the E2 of
// the adjoint call repeats bit for bit.
__device__ __forceinline__ double block_sum256(double v) {
  __shared__ double sw[4];
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if ((threadIdx.x & 63) == 0) sw[threadIdx.x >> 6] = v;
  __syncthreads();
  const double t = ((sw[0] + sw[1]) + sw[2]) + sw[3];
  __syncthreads();
  return t;
}

// ---- row decoding shared by the two passes ----------------------------------
struct Row {
  int c0, c1, a, b;
  int64_t rab;
  bool valid;
};

template <int H, int V>
__device__ __forceinline__ Row decode_row(const Dev& d, const ClassDev& cd, int64_t r) {
  Row w;
  w.c0 = w.c1 = w.a = w.b = -1;
  w.rab = 0;
  w.valid = r < cd.n_rows;
  if (!w.valid) r = cd.n_rows - 1;
  if (V == 2) {
    const int64_t per = d.n_tp * 4096;
    const int64_t hole = r / per;
    w.rab = r % per;
    const int64_t tp = w.rab >> 12;
    const int la = (int)((w.rab >> 6) & 63), lb = (int)(w.rab & 63);
    w.a = d.tile_pairs[2 * tp] * 64 + la;
    w.b = d.tile_pairs[2 * tp + 1] * 64 + lb;
    if (!(w.a < w.b && w.b < d.n_v)) {
      w.valid = false;
      w.a = 0;
      w.b = d.n_v > 1 ? 1 : 0;
    }
    if (H == 1) w.c0 = (int)hole;
    if (H == 2) {
      w.c0 = d.hole_pairs[2 * hole];
      w.c1 = d.hole_pairs[2 * hole + 1];
    }
  } else {
    int64_t hi = r;
    if (V == 1) {
      w.a = (int)(r % d.n_v);
      hi = r / d.n_v;
    }
    if (H == 1) w.c0 = (int)hi;
    if (H == 2) {
      w.c0 = d.hole_pairs[2 * hi];
      w.c1 = d.hole_pairs[2 * hi + 1];
    }
  }
  return w;
}

// Row constant of Delta (the part that does not depend on the string).
template <int H, int V>
__device__ __forceinline__ double row_const(const Dev& d, const Row& w) {
  const int64_t gfc = d.n_fc, gv = d.n_fc + d.n_o;
  double qr = 0.0;
  if (H >= 1) qr += d.eps[w.c0];
  if (H == 2) qr += d.eps[w.c1] - d.W[(gfc + w.c0) * d.n + gfc + w.c1];
  if (V >= 1) qr -= d.eps[d.n_o + w.a];
  if (V == 2) qr -= d.eps[d.n_o + w.b] + d.W[(gv + w.a) * d.n + gv + w.b];
  if (H >= 1 && V >= 1) {
    qr += d.W[(gfc + w.c0) * d.n + gv + w.a];
    if (V == 2) qr += d.W[(gfc + w.c0) * d.n + gv + w.b];
    if (H == 2) {
      qr += d.W[(gfc + w.c1) * d.n + gv + w.a];
      if (V == 2) qr += d.W[(gfc + w.c1) * d.n + gv + w.b];
    }
  }
  return qr;
}

// Offset of a coupling in row r from its key (see the plan's coupling keys):
// into A (v = 2: occupied pair of the row and the pattern, then the row's
// place in the tile pair) or X (v < 2: pattern j, row r).
template <int H, int V>
__device__ __forceinline__ int64_t coupling_off(const Dev& d, const ClassDev& cd, int32_t key, const Row& w,
                                                int64_t r) {
  key &= 0x7fffffff;
  if (V == 2) {
    int64_t pair;
    if (H == 2) pair = occ_pair(w.c0, w.c1, d.n_o);
    else if (H == 1) pair = occ_pair(w.c0, d.n_c + key, d.n_o);
    else pair = key;
    return pair * d.n_tp * 4096 + w.rab;
  }
  return (int64_t)key * cd.n_rows + r;
}

template <int H, int V>
__device__ __forceinline__ double string_delta(const ClassDev& cd, const Dev& d, int64_t s, const Row& w) {
  double del = cd.T[s];
  if (H >= 1) del += cd.Uc[s * d.n_c + w.c0];
  if (H == 2) del += cd.Uc[s * d.n_c + w.c1];
  if (V >= 1) del -= cd.Uv[s * d.n_v + w.a];
  if (V == 2) del -= cd.Uv[s * d.n_v + w.b];
  return del;
}

// The same from the transposed tables (string-owned passes: lanes = strings,
// so the loads of a wave are contiguous).
template <int H, int V>
__device__ __forceinline__ double string_delta_t(const ClassDev& cd, const ClassGrad& cg, int64_t s,
                                                 const Row& w) {
  const int64_t S = cd.n_str;
  double del = cd.T[s];
  if (H >= 1) del += cg.UcT[(int64_t)w.c0 * S + s];
  if (H == 2) del += cg.UcT[(int64_t)w.c1 * S + s];
  if (V >= 1) del -= cg.UvT[(int64_t)w.a * S + s];
  if (V == 2) del -= cg.UvT[(int64_t)w.b * S + s];
  return del;
}

// sign * C_beta per coupling of a class.  grid (ceil(n_conn / 256)).
__device__ __forceinline__ void becoef_body(const Dev& d, const ClassDev& cd, const ClassGrad& cg,
                                            const uint3 bid) {
  const int64_t e = (int64_t)bid.x * 256 + threadIdx.x;
  if (e >= cd.n_conn) return;
  const int32_t cb = cd.conn[2 * e];
  double2 cv = d.c[cb & 0x7fffffff];
  if (cb < 0) cv = make_double2(-cv.x, -cv.y);
  cg.ecoef[e] = cv;
}

// ---- row pass ------------------------------------------------------------------
// One thread per row; the block walks the strings of its chunk (all strings
// unless the class has few rows).  Accumulates, per row:
//   couplings:  Xbar[j][r] += sigma-bar * conj(sign C_beta)
//   q  = sum_s Delta-bar             (row constant of Delta)
//   y_t = sum_{s containing t} Delta-bar   (tables Uc, Uv: W of the row's
//         core holes and virtual spinors with active spinor t)
// then adds q and y into the adjoints of eps and W.  The coupling lists are
// the same for every thread of the block, so their loads are uniform.
// grid (ceil(rows / 256), string chunks), block 256, dynamic LDS n_a * 256 doubles.
template <int H, int V>
__device__ __forceinline__ void brow_body(const Dev& d, const ClassDev& cd, const GradDev& g, const ClassGrad& cg,
                                          const uint3 bid) {
  extern __shared__ double sY[];
  const int tid = threadIdx.x;
  const int64_t r = (int64_t)bid.x * 256 + tid;
  const Row w = decode_row<H, V>(d, cd, r);
  const int64_t rr = w.valid ? r : cd.n_rows - 1;
  const int na = d.n_a;
  for (int t = 0; t < na; ++t) sY[t * 256 + tid] = 0.0;
  const double qr = row_const<H, V>(d, w);
  const double N = d.scal[1];
  const double twoN = 2.0 / N, oneN = 1.0 / N;
  double2* Xb = (V == 2) ? g.Ab : cg.Xb;
  const double2* X = (V == 2) ? d.A : cd.X;
  const double2* __restrict__ ec = cg.ecoef;
  const int32_t* __restrict__ ek = cd.ekey;
  double q = 0.0, e2 = 0.0;
  const double b2 = d.ls_b2;
  const int64_t S = cd.n_str;
  // strings [s_lo, s_hi) of this block; with several string chunks the
  // coupling adjoints of a row are shared and added atomically
  const int nsc = cg.row_split;
  const int64_t chunk = (S + nsc - 1) / nsc;
  const int64_t s_lo = (int64_t)bid.y * chunk, s_hi = min(S, s_lo + chunk);
  const bool shared_rows = nsc > 1;
  // several string chunks: the chunk's own slice of partials where the plan
  // gave them (plain adds, summed in order by bxbred_body), else atomics
  double2* Xbw = Xb;
  bool atomic = shared_rows;
  if (V < 2 && shared_rows && cg.Xbp) {
    Xbw = cg.Xbp + (int64_t)bid.y * cd.n_pat * cd.n_rows;
    atomic = false;
  }
  for (int64_t s = s_lo; s < s_hi; ++s) {
    const int e0 = cd.conn_ptr[s], e1 = cd.conn_ptr[s + 1];
    if (e1 == e0) continue;
    double2 sig = make_double2(0.0, 0.0);
    int e = e0;
    for (; e + 4 <= e1; e += 4) {
      double2 xv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) xv[u] = X[coupling_off<H, V>(d, cd, ek[e + u], w, rr)];
#pragma unroll
      for (int u = 0; u < 4; ++u) sig = cfma(ec[e + u], xv[u], sig);
    }
    for (; e < e1; ++e) sig = cfma(ec[e], X[coupling_off<H, V>(d, cd, ek[e], w, rr)], sig);
    const double del = string_delta<H, V>(cd, d, s, w) + qr;
    double gw, gp;
    en_weight_d(del, b2, gw, gp);
    const double2 sb = make_double2(twoN * gw * sig.x, twoN * gw * sig.y);
    const double dl = oneN * gp * cabs2(sig);
    if (w.valid) {
      e2 = fma(gw, cabs2(sig), e2);
      for (e = e0; e < e1; ++e) {
        double2* p = Xbw + coupling_off<H, V>(d, cd, ek[e], w, rr);
        const double2 v = cmul(sb, cconj(ec[e]));
        if (atomic) catomic(p, v);
        else *p = cadd(*p, v);
      }
      q += dl;
      uint64_t x = cd.strings[s];
      while (x) {
        const int tt = __builtin_ctzll(x);
        x &= x - 1;
        sY[tt * 256 + tid] += dl;
      }
    }
  }
  const double e2b = block_sum256(e2);
  if (tid == 0) cd.part[(int64_t)bid.y * ((cd.n_rows + 255) / 256) + bid.x] = e2b;
  if (!w.valid) return;
  const int64_t n = d.n, gfc = d.n_fc, gv = d.n_fc + d.n_o, ga = d.n_fc + d.n_c;
  double* Wb = g.Wb;
  // row constant: eps and W of holes and virtual spinors
  if (H >= 1) atomicAdd(&g.epsb[w.c0], q);
  if (H == 2) {
    atomicAdd(&g.epsb[w.c1], q);
    atomicAdd(&Wb[(gfc + w.c0) * n + gfc + w.c1], -q);
  }
  if (V >= 1) atomicAdd(&g.epsb[d.n_o + w.a], -q);
  if (V == 2) {
    atomicAdd(&g.epsb[d.n_o + w.b], -q);
    atomicAdd(&Wb[(gv + w.a) * n + gv + w.b], -q);
  }
  if (H >= 1 && V >= 1) {
    atomicAdd(&Wb[(gfc + w.c0) * n + gv + w.a], q);
    if (V == 2) atomicAdd(&Wb[(gfc + w.c0) * n + gv + w.b], q);
    if (H == 2) {
      atomicAdd(&Wb[(gfc + w.c1) * n + gv + w.a], q);
      if (V == 2) atomicAdd(&Wb[(gfc + w.c1) * n + gv + w.b], q);
    }
  }
  // string tables: Uc[s][c] = sum_{t in s} W[c][t], Uv[s][a] = sum_{t in s} W[a][t]
  for (int t = 0; t < na; ++t) {
    const double y = sY[t * 256 + tid];
    if (y == 0.0) continue;
    if (H >= 1) atomicAdd(&Wb[(gfc + w.c0) * n + ga + t], y);
    if (H == 2) atomicAdd(&Wb[(gfc + w.c1) * n + ga + t], y);
    if (V >= 1) atomicAdd(&Wb[(gv + w.a) * n + ga + t], -y);
    if (V == 2) atomicAdd(&Wb[(gv + w.b) * n + ga + t], -y);
  }
}

// Coupling adjoints of a class from the string chunks' private slices, summed
// in chunk order.  grid (ceil(n_pat n_rows / 256)), block 256.
__device__ __forceinline__ void bxbred_body(const ClassDev& cd, const ClassGrad& cg, const uint3 bid) {
  const int64_t i = (int64_t)bid.x * 256 + threadIdx.x;
  const int64_t m = (int64_t)cd.n_pat * cd.n_rows;
  if (i >= m) return;
  double2 v = make_double2(0.0, 0.0);
  for (int p = 0; p < cg.row_split; ++p) v = cadd(v, cg.Xbp[(int64_t)p * m + i]);
  cg.Xb[i] = v;
}

// ---- string pass -------------------------------------------------------------
// One thread per string, rows [part * rows_per_part, ...) taken RCH at a time
// so that each coupling's integrals for those rows are independent loads.
// Accumulates, per string and part:  cbe[e] = sum_r sign conj(X[j_e][r])
// sigma-bar (coefficient adjoint through coupling e), and Tb[s] = sum_r
// Delta-bar.  grid (ceil(S / 256), parts), block 256.
constexpr int RCH = 8;

template <int H, int V>
__device__ __forceinline__ void bstr_body(const Dev& d, const ClassDev& cd, const GradDev& g, const ClassGrad& cg,
                                          const uint3 bid) {
  const int64_t S = cd.n_str;
  int64_t s = (int64_t)bid.x * 256 + threadIdx.x;
  const bool live = s < S;
  if (!live) s = S - 1;
  const int part = bid.y;
  const int64_t r0 = (int64_t)part * cg.rows_per_part;
  const int64_t r1 = min(cd.n_rows, r0 + cg.rows_per_part);
  const int e0 = cd.conn_ptr[s], e1 = cd.conn_ptr[s + 1];
  const double N = d.scal[1];
  const double twoN = 2.0 / N, oneN = 1.0 / N;
  const double2* X = (V == 2) ? d.A : cd.X;
  const double2* __restrict__ ec = cg.ecoef;
  const int32_t* __restrict__ ek = cd.ekey;
  double2* cbe = cg.cbe + (int64_t)part * cd.n_conn;
  double tq = 0.0;
  const double b2 = d.ls_b2;
  for (int64_t rc = r0; rc < r1; rc += RCH) {
    Row w[RCH];
    int64_t rk[RCH];
    bool any = false;
#pragma unroll
    for (int k = 0; k < RCH; ++k) {
      rk[k] = rc + k < r1 ? rc + k : r1 - 1;
      w[k] = decode_row<H, V>(d, cd, rk[k]);
      w[k].valid = w[k].valid && (rc + k < r1);
      any = any || w[k].valid;
    }
    if (!any || e1 == e0) continue;
    double2 sig[RCH];
#pragma unroll
    for (int k = 0; k < RCH; ++k) sig[k] = make_double2(0.0, 0.0);
    for (int e = e0; e < e1; ++e) {
      const double2 cv = ec[e];
      const int32_t key = ek[e];
      double2 xv[RCH];
#pragma unroll
      for (int k = 0; k < RCH; ++k) xv[k] = X[coupling_off<H, V>(d, cd, key, w[k], rk[k])];
#pragma unroll
      for (int k = 0; k < RCH; ++k) sig[k] = cfma(cv, xv[k], sig[k]);
    }
    double2 sb[RCH];
#pragma unroll
    for (int k = 0; k < RCH; ++k) {
      // one-virtual classes read the transposed tables (contiguous across the
      // wave); two-virtual rows of a chunk share cache lines of Uv[s]
      const double sd = V <= 1 ? string_delta_t<H, V>(cd, cg, s, w[k]) : string_delta<H, V>(cd, d, s, w[k]);
      const double del = sd + row_const<H, V>(d, w[k]);
      double gw, gp;
      en_weight_d(del, b2, gw, gp);
      if (!w[k].valid) gw = gp = 0.0;
      sb[k] = make_double2(twoN * gw * sig[k].x, twoN * gw * sig[k].y);
      tq += oneN * gp * cabs2(sig[k]);
    }
    if (live) {
      for (int e = e0; e < e1; ++e) {
        const int32_t key = ek[e];
        double2 xv[RCH];
#pragma unroll
        for (int k = 0; k < RCH; ++k) xv[k] = X[coupling_off<H, V>(d, cd, key, w[k], rk[k])];
        double2 acc = make_double2(0.0, 0.0);
#pragma unroll
        for (int k = 0; k < RCH; ++k) acc = cadd(acc, cmul(cconj(xv[k]), sb[k]));
        if (key < 0) acc = make_double2(-acc.x, -acc.y);
        cbe[e] = cadd(cbe[e], acc);
      }
    }
  }
  if (live) cg.Tb[(int64_t)part * S + s] = tq;
}

// ---- class (2,2) ------------------------------------------------------------------
// sigma_K = <ab||cc'> C_alpha, Delta = G(alpha) + Y_a(alpha) + Y_b(alpha) - W_ab as in
// the forward kernel, w = 1/Delta, cw = |C_alpha|^2.  Two kernels share the work.
//
// Row-owned (the forward kernel's layout; each thread 4 x 4 (a, b) of a tile,
// strings staged in LDS): S1 = sum_alpha cw w and S2 = sum_alpha cw w^2, four
// fractions merged per reciprocal, give
//   Abar[cc'][ab] = (2/N) A S1  (written once)  and the row constants'
//   adjoint -(1/N) |A|^2 S2  (eps and W of c, c', a, b; W_ab).
// grid (C(n_c,2), n_tp), block 256.
__device__ __forceinline__ void b22a_body(const Dev& d, const ClassDev& cd, const GradDev& g, const uint3 bid) {
  __shared__ double sYa[AC22][64];
  __shared__ double sYb[AC22][64];
  __shared__ double sG[AC22];
  __shared__ double sCw[AC22];
  __shared__ double ya0[64], yb0[64];
  __shared__ double red[256];
  const int hp = bid.x, tp = bid.y;   // core pairs fastest: blocks of one tile pair share its tables in L2
  const int c0 = d.hole_pairs[2 * hp], c1 = d.hole_pairs[2 * hp + 1];
  const int I = d.tile_pairs[2 * tp], J = d.tile_pairs[2 * tp + 1];
  const int tid = threadIdx.x, ta = tid & 15, tb = tid >> 4;
  const int nv = d.n_v, nc = d.n_c;
  const int64_t n = d.n, gfc = d.n_fc, gv = d.n_fc + d.n_o;
  const double* __restrict__ W = d.W;
  if (tid < 64) {
    const int a = I * 64 + tid;
    ya0[tid] = (a < nv) ? -d.eps[d.n_o + a] + W[(gfc + c0) * n + gv + a] + W[(gfc + c1) * n + gv + a] : -1.0;
  } else if (tid < 128) {
    const int b = J * 64 + tid - 64;
    yb0[tid - 64] = (b < nv) ? -d.eps[d.n_o + b] + W[(gfc + c0) * n + gv + b] + W[(gfc + c1) * n + gv + b] : -1.0;
  }
  const double gconst = d.eps[c0] + d.eps[c1] - W[(gfc + c0) * n + gfc + c1];
  double wab[4][4], S1[4][4], S2[4][4];
  bool ok[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int a = I * 64 + ta + 16 * i, b = J * 64 + tb + 16 * j;
      ok[i][j] = (a < b) && (b < nv);
      wab[i][j] = ok[i][j] ? W[(gv + a) * n + gv + b] : 0.0;
      S1[i][j] = S2[i][j] = 0.0;
    }
  const int np = d.n_p;
  for (int s0 = 0; s0 < np; s0 += AC22) {
    __syncthreads();
    for (int e = tid; e < AC22 * 64; e += 256) {
      const int al = e >> 6, l = e & 63;
      const int s = s0 + al;
      const int a = I * 64 + l, b = J * 64 + l;
      double ya = ya0[l], yb = yb0[l];
      if (s < np) {
        if (a < nv) ya -= cd.Uv[(int64_t)s * nv + a];
        if (b < nv) yb -= cd.Uv[(int64_t)s * nv + b];
      }
      sYa[al][l] = ya;
      sYb[al][l] = yb;
    }
    if (tid < AC22) {
      const int s = s0 + tid;
      if (s < np) {
        sG[tid] = cd.T[s] + cd.Uc[(int64_t)s * nc + c0] + cd.Uc[(int64_t)s * nc + c1] + gconst;
        sCw[tid] = cabs2(d.c[s]);
      } else {
        sG[tid] = 1e30;
        sCw[tid] = 0.0;
      }
    }
    __syncthreads();
#pragma unroll 1
    for (int al = 0; al < AC22; al += 4) {
      double gk[4], cw[4], za[4][4], yb[4][4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        gk[k] = sG[al + k];
        cw[k] = sCw[al + k];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int k = 0; k < 4; ++k) za[i][k] = gk[k] + sYa[al + k][ta + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int k = 0; k < 4; ++k) yb[j][k] = sYb[al + k][tb + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const double d0 = (za[i][0] + yb[j][0]) - wab[i][j];
          const double d1 = (za[i][1] + yb[j][1]) - wab[i][j];
          const double d2 = (za[i][2] + yb[j][2]) - wab[i][j];
          const double d3 = (za[i][3] + yb[j][3]) - wab[i][j];
          const double p01 = d0 * d1, p23 = d2 * d3;
          const double r = rcp_nr(p01 * p23);
          const double q0 = d1 * p23, q1 = d0 * p23, q2 = d3 * p01, q3 = d2 * p01;
          const double n1 = fma(cw[0], q0, fma(cw[1], q1, fma(cw[2], q2, cw[3] * q3)));
          const double n2 = fma(cw[0] * q0, q0, fma(cw[1] * q1, q1, fma(cw[2] * q2, q2, cw[3] * q3 * q3)));
          S1[i][j] = fma(n1, r, S1[i][j]);
          S2[i][j] = fma(n2, r * r, S2[i][j]);
        }
    }
  }
  // pair-integral adjoint tile and row constants
  const double N = d.scal[1], oneN = 1.0 / N, twoN = 2.0 / N;
  const double2* Ablk = d.A + ((int64_t)occ_pair(c0, c1, d.n_o) * d.n_tp + tp) * 4096;
  double2* Ab = g.Ab + ((int64_t)occ_pair(c0, c1, d.n_o) * d.n_tp + tp) * 4096;
  double rowa[4] = {0.0, 0.0, 0.0, 0.0}, colb[4] = {0.0, 0.0, 0.0, 0.0};
  double e2 = 0.0;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (ok[i][j]) {
        const int li = (ta + 16 * i) * 64 + tb + 16 * j;
        const double2 av = Ablk[li];
        e2 = fma(cabs2(av), S1[i][j], e2);
        Ab[li] = make_double2(twoN * S1[i][j] * av.x, twoN * S1[i][j] * av.y);
        const double gq = -oneN * cabs2(av) * S2[i][j];   // sum over alpha of Delta-bar
        const int a = I * 64 + ta + 16 * i, b = J * 64 + tb + 16 * j;
        atomicAdd(&g.Wb[(gv + a) * n + gv + b], -gq);
        rowa[i] += gq;
        colb[j] += gq;
      }
  const double e2b = block_sum256(e2);
  if (tid == 0) cd.part[(int64_t)tp * cd.n_holes + hp] = e2b;
  __syncthreads();
  double* sRC = &sYa[0][0];   // row sums [0..63], column sums [64..127]
  if (tid < 128) sRC[tid] = 0.0;
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 4; ++i) atomicAdd(&sRC[ta + 16 * i], rowa[i]);
#pragma unroll
  for (int j = 0; j < 4; ++j) atomicAdd(&sRC[64 + tb + 16 * j], colb[j]);
  __syncthreads();
  if (tid < 128) {
    const int x = tid & 63;
    const double v = sRC[tid];
    const int vv = (tid < 64 ? I : J) * 64 + x;
    if (vv < nv && v != 0.0) {
      atomicAdd(&g.epsb[d.n_o + vv], -v);
      atomicAdd(&g.Wb[(gfc + c0) * n + gv + vv], v);
      atomicAdd(&g.Wb[(gfc + c1) * n + gv + vv], v);
    }
    red[tid] = v;
  }
  __syncthreads();
  if (tid == 0) {
    double tot = 0.0;
    for (int x = 0; x < 64; ++x) tot += red[x];
    atomicAdd(&g.epsb[c0], tot);
    atomicAdd(&g.epsb[c1], tot);
    atomicAdd(&g.Wb[(gfc + c0) * n + gfc + c1], -tot);
  }
}

// String-owned (one thread per reference string alpha; the block walks all
// tile pairs for a group of core pairs, in sub-tiles whose |A|^2 and W_ab are
// staged in LDS and read by every thread):
//   R1(alpha) = sum |A|^2 w        -> Cbar_alpha = (2/N) C_alpha R1,
//   Tbar(alpha) = -(1/N) cw sum |A|^2 w^2,
//   Uv tables: per virtual a (b), x(alpha, a) = cw sum_{c c', b (a)} |A|^2 w^2
//   is kept in a private LDS slot per thread, then contracted with the string
//   occupations, W[a][t] += (1/N) sum_alpha [t in alpha] x(alpha, a), into a
//   per-block partial of W (reduced by the next kernel);
//   Uc: per core pair likewise with -1/N, straight into W.
// The sub-tiles are B22S x B22S; blocks of B22T threads keep the LDS slab of
// per-thread values small enough for four blocks (sixteen waves) per CU.
// grid (ceil(n_p / B22T), ceil(C(n_c,2) / group)), block B22T.
constexpr int B22T = 256;
constexpr int B22S = 16;
constexpr int B22HP = 8;                   // at most this many core pairs per part (LDS slab of the Uc sums)
// Row stride of the per-thread LDS columns: one double of padding puts the 16
// rows that the contraction reads at once (one per lane group) in distinct banks.
constexpr int B22P = B22T + 1;

// Contract one B22S-row slab of per-thread values with the string occupations:
// wpart[v0 + x][t] += sum_l [t in str_l] buf[x][l], rows x < B22S, t < n_a.
// A 16 x 256 by 256 x 64 product with a 0/1 right factor, on FP64 MFMA:
// wave w takes the spinors t = 16 w ... 16 w + 15 (16 x 16 x 4 products over
// the 256 strings; lane l supplies buf[l % 16][k + l / 16] and the bit of
// spinor 16 w + l % 16 in string k + l / 16, and holds the result rows
// l / 16 + 4 r of column l % 16).  No barrier inside.
static_assert(B22S == 16, "the contraction's MFMA tile has 16 rows");
__device__ __forceinline__ void b22_contract(const double* buf, const uint64_t* sStr, double* wpart, int v0, int nv,
                                             int na) {
  typedef double d4c __attribute__((ext_vector_type(4)));
  const int lane = threadIdx.x & 63, t0 = 16 * (threadIdx.x >> 6);
  if (t0 >= na) return;                      // wave-uniform
  const int m = lane & 15, kq = lane >> 4;
  d4c acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
  for (int l0 = 0; l0 < B22T; l0 += 4) {
    const int l = l0 + kq;
    const double a = buf[m * B22P + l];
    const double b = ((sStr[l] >> (t0 + m)) & 1ull) ? 1.0 : 0.0;
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
  }
  const int t = t0 + m;
  if (t < na) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int vv = v0 + kq + 4 * r;
      if (vv < nv) wpart[(int64_t)vv * na + t] += acc[r];
    }
  }
}

// String tables transposed for the generic string-owned pass of the
// one-virtual classes, whose lanes are strings: out[x][s] = in[s][x] with
// in = Uv (which = 0, x < n_v) or Uc (which = 1, x < n_c).  32 x 32 tiles
// through LDS.
// grid (ceil(S / 32), ceil(m / 32)), block 256.
__device__ __forceinline__ void btrans_body(const Dev& d, const ClassDev& cd, const ClassGrad& cg, int which,
                                            const uint3 bid) {
  __shared__ double tile[32][33];
  const int64_t S = cd.n_str;
  const int m = which ? d.n_c : d.n_v;
  const double* in = which ? cd.Uc : cd.Uv;
  double* out = which ? cg.UcT : cg.UvT;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const int64_t s0 = (int64_t)bid.x * 32;
  const int x0 = bid.y * 32;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int64_t s = s0 + ty + 8 * k;
    const int x = x0 + tx;
    tile[ty + 8 * k][tx] = (s < S && x < m) ? in[s * m + x] : 0.0;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int x = x0 + ty + 8 * k;
    const int64_t s = s0 + tx;
    if (s < S && x < m) out[(int64_t)x * S + s] = tile[tx][ty + 8 * k];
  }
}

__device__ __forceinline__ void b22b_body(const Dev& d, const ClassDev& cd, const GradDev& g, const ClassGrad& cg,
                                          const uint3 bid, int64_t nsblk) {
  __shared__ double sBuf[B22S * B22P];   // per-thread column: a side, then b side of a sub-tile
  __shared__ double sA2[B22S][B22S];
  __shared__ double sWab[B22S][B22S];
  __shared__ double sWc[2][B22S];        // W[c][v] + W[c'][v] of the sub-tile's a (0) and b (1)
  __shared__ double sEa[B22S];           // eps of the sub-tile's a
  __shared__ double sQ2[B22HP][B22T];    // per core pair of the part and string: sum of |A|^2 w^2 (Uc tables)
  __shared__ uint64_t sStr[B22T];
  const int tid = threadIdx.x;
  const int np = d.n_p, nv = d.n_v, nc = d.n_c, na = d.n_a;
  int s = bid.x * B22T + tid;
  const bool live = s < np;
  if (!live) s = np - 1;
  const int64_t nhp = cd.n_holes;
  const int64_t hp0 = (int64_t)bid.y * cg.rows_per_part, hp1 = min(nhp, hp0 + cg.rows_per_part);
  const int64_t n = d.n, gfc = d.n_fc, gv = d.n_fc + d.n_o, ga = d.n_fc + d.n_c;
  const double* __restrict__ W = d.W;
  const double N = d.scal[1], oneN = 1.0 / N;
  const double cw = live ? cabs2(d.c[s]) : 0.0;
  const uint64_t str = live ? d.pstrings[s] : 0ull;
  sStr[tid] = str;
#pragma unroll
  for (int h = 0; h < B22HP; ++h) sQ2[h][tid] = 0.0;
  const double Ts = cd.T[s];
  const double* Uvs = cd.Uv + (int64_t)s * nv;
  const double* Ucs = cd.Uc + (int64_t)s * nc;
  double* wpart = cg.wpart + ((int64_t)bid.y * nsblk + bid.x) * nv * na;
  double R1 = 0.0, T2 = 0.0;
  constexpr int NB = B22S;
  for (int64_t tp = 0; tp < d.n_tp; ++tp) {
    const int I = d.tile_pairs[2 * tp], J = d.tile_pairs[2 * tp + 1];
    for (int ha = 0; ha < 64; ha += B22S) {
      const int a0 = I * 64 + ha;
      if (a0 >= nv || J * 64 + 63 <= a0) continue;
      for (int hb = 0; hb < 64; hb += NB) {
        const int b0 = J * 64 + hb;
        if (b0 >= nv || b0 + NB - 1 <= a0) continue;
#pragma unroll
        for (int la = 0; la < B22S; ++la) sBuf[la * B22P + tid] = 0.0;
        double vb[NB], ybs[NB];
#pragma unroll
        for (int lb = 0; lb < NB; ++lb) {
          vb[lb] = 0.0;
          const int b = b0 + lb;
          ybs[lb] = (b < nv) ? -d.eps[d.n_o + b] - Uvs[b] : 0.0;   // the string's part of the b side
        }
        for (int64_t hp = hp0; hp < hp1; ++hp) {
          const int c0 = d.hole_pairs[2 * hp], c1 = d.hole_pairs[2 * hp + 1];
          const double2* Ablk = d.A + ((int64_t)occ_pair(c0, c1, d.n_o) * d.n_tp + tp) * 4096;
          __syncthreads();
          for (int e = tid; e < B22S * NB; e += B22T) {
            const int la = e / NB, lb = e % NB;
            const int a = a0 + la, b = b0 + lb;
            const bool ok = (a < b) && (b < nv);
            // outside a < b < n_v: zero weight and a denominator near -1e30,
            // whose fraction vanishes (products of four such stay finite)
            sA2[la][lb] = ok ? cabs2(Ablk[(ha + la) * 64 + hb + lb]) : 0.0;
            sWab[la][lb] = ok ? W[(gv + a) * n + gv + b] : -1e30;
          }
          if (tid < 2 * B22S) {
            const int side = tid / B22S, l = tid % B22S;
            const int v = (side ? b0 : a0) + l;
            sWc[side][l] = v < nv ? W[(gfc + c0) * n + gv + v] + W[(gfc + c1) * n + gv + v] : 0.0;
            if (side == 0) sEa[l] = v < nv ? d.eps[d.n_o + v] : 0.0;
          }
          __syncthreads();
          const double Gc = Ts + Ucs[c0] + Ucs[c1] + d.eps[c0] + d.eps[c1] - W[(gfc + c0) * n + gfc + c1];
          double yb[NB];
#pragma unroll
          for (int lb = 0; lb < NB; ++lb) yb[lb] = ybs[lb] + sWc[1][lb];
          double q2c = 0.0;
          for (int la = 0; la < B22S; ++la) {
            const int a = a0 + la;
            if (a >= nv || b0 + NB - 1 <= a) break;
            const double base = Gc - sEa[la] - Uvs[a] + sWc[0][la];
            double va = 0.0;
#pragma unroll
            for (int lb = 0; lb < NB; lb += 4) {
              double dd[4], a2[4];
#pragma unroll
              for (int k = 0; k < 4; ++k) {
                a2[k] = sA2[la][lb + k];
                dd[k] = (base + yb[lb + k]) - sWab[la][lb + k];
              }
              const double p01 = dd[0] * dd[1], p23 = dd[2] * dd[3];
              const double r = rcp_nr(p01 * p23);
              const double r01 = r * p23, r23 = r * p01;
              double w[4];
              w[0] = r01 * dd[1];
              w[1] = r01 * dd[0];
              w[2] = r23 * dd[3];
              w[3] = r23 * dd[2];
#pragma unroll
              for (int k = 0; k < 4; ++k) {
                R1 = fma(a2[k], w[k], R1);
                const double t2 = a2[k] * w[k] * w[k];
                va += t2;
                vb[lb + k] += t2;
              }
            }
            q2c += va;
            sBuf[la * B22P + tid] += cw * va;
          }
          T2 += q2c;
          sQ2[hp - hp0][tid] += cw * q2c;   // own column
        }
        // the sub-tile's a side, then its b side, contracted with the occupations
        __syncthreads();
        b22_contract(sBuf, sStr, wpart, a0, nv, na);
        __syncthreads();
#pragma unroll
        for (int lb = 0; lb < NB; ++lb) sBuf[lb * B22P + tid] = cw * vb[lb];
        __syncthreads();
        b22_contract(sBuf, sStr, wpart, b0, nv, na);
        __syncthreads();
      }
    }
  }
  if (live) {
    cg.Tb[(int64_t)bid.y * np + s] = -oneN * cw * T2;
    cg.r1[(int64_t)bid.y * np + s] = R1;
  }
  // Uc tables of the part's core pairs: W[c][t] -= (1/N) sum_alpha [t in alpha] cw q2
  __syncthreads();
  const int nh = (int)(hp1 - hp0);
  for (int e = tid; e < nh * 64; e += B22T) {
    const int h = e >> 6, t = e & 63;
    if (t >= na) continue;
    double v = 0.0;
    for (int l = 0; l < B22T; ++l)
      if ((sStr[l] >> t) & 1ull) v += sQ2[h][l];
    if (v != 0.0) {
      const int c0 = d.hole_pairs[2 * (hp0 + h)], c1 = d.hole_pairs[2 * (hp0 + h) + 1];
      atomicAdd(&g.Wb[(gfc + c0) * n + ga + t], -oneN * v);
      atomicAdd(&g.Wb[(gfc + c1) * n + ga + t], -oneN * v);
    }
  }
}

// Uv tables of class (2,2): W[a][t] += (1/N) sum over the string-owned kernel's
// blocks of their partials.  grid (ceil(n_v n_a / 256)).
__device__ __forceinline__ void b22w_body(const Dev& d, const ClassDev& cd, const GradDev& g, const ClassGrad& cg,
                                          const uint3 bid, int64_t nblk) {
  const int64_t i = (int64_t)bid.x * 256 + threadIdx.x;
  const int64_t per = (int64_t)d.n_v * d.n_a;
  if (i >= per) return;
  double v = 0.0;
  for (int64_t b = 0; b < nblk; ++b) v += cg.wpart[b * per + i];
  const int a = (int)(i / d.n_a), t = (int)(i % d.n_a);
  const int64_t gv = d.n_fc + d.n_o, ga = d.n_fc + d.n_c;
  if (v != 0.0) g.Wb[(gv + a) * d.n + ga + t] += v / d.scal[1];
}

// Per-string adjoints of class (2,2) from the per-block partials: Tbar (as in
// the generic case) and Cbar_alpha = (2/N) C_alpha sum R1.  grid (ceil(np/256)).
__device__ __forceinline__ void b22fin_body(const Dev& d, const ClassDev& cd, const GradDev& g,
                                            const ClassGrad& cg, const uint3 bid) {
  __shared__ double red[256];
  const int np = d.n_p;
  const int64_t s = (int64_t)bid.x * 256 + threadIdx.x;
  double T = 0.0;
  if (s < np) {
    double R = 0.0;
    for (int p = 0; p < cg.parts; ++p) {
      T += cg.Tb[(int64_t)p * np + s];
      R += cg.r1[(int64_t)p * np + s];
    }
    const double ea = -T;
    const int64_t n = d.n, ga = d.n_fc + d.n_c;
    uint64_t x = cd.strings[s];
    while (x) {
      const int t = __builtin_ctzll(x);
      x &= x - 1;
      atomicAdd(&g.epsb[d.n_c + t], ea);
      uint64_t y = x;
      while (y) {
        const int u = __builtin_ctzll(y);
        y &= y - 1;
        atomicAdd(&g.Wb[(ga + t) * n + ga + u], ea);
      }
    }
    const double k = 2.0 / d.scal[1] * R;
    const double2 c = d.c[s];
    catomic(&g.cb[s], make_double2(k * c.x, k * c.y));
  }
  red[threadIdx.x] = T;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(&g.scal[0], red[0]);
}

// ---- class (1,2) ---------------------------------------------------------------------
// sigma_K = sum_j D[s][j] X_j with X_j = <ab||c t_j> (dense coefficients), and
//   Delta = T + eps_c + Uc_c - eps_a - Uv_a - eps_b - Uv_b - W_ab + W_ca + W_cb.
// Row pass (the forward kernel's layout, one thread per (a, b) of a 16 x 16
// sub-tile, couplings and their adjoints in registers): Abar for the core-active
// pairs, the row constants, and the Uv tables.  For the tables each thread
// keeps y[t] = sum over the strings containing active spinor t of its
// Delta-bar (YREG: in registers, else in its own LDS column; the string's
// occupation is wave-uniform, so the update loop is scalar); the sums over b
// (table of a) and over a (table of b) are taken once per block at the end.
// Strings are staged CH at a time (64 where the LDS holds it, else 32).
// grid (n_c, 16 n_tp), block 256, dynamic LDS (n_a + 1) * 256 doubles.

__device__ __forceinline__ double xsum16(double v) {   // sum over the 16 lanes sharing tid >> 4
  v += __shfl_xor(v, 1, 64);
  v += __shfl_xor(v, 2, 64);
  v += __shfl_xor(v, 4, 64);
  v += __shfl_xor(v, 8, 64);
  return v;
}
__device__ __forceinline__ double xsum4(double v) {    // sum over lanes l, l^16, l^32, l^48
  v += __shfl_xor(v, 16, 64);
  v += __shfl_xor(v, 32, 64);
  return v;
}
__device__ __forceinline__ uint64_t uniform64(uint64_t x) {   // a wave-uniform value into scalar registers
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(x >> 32));
  return ((uint64_t)hi << 32) | lo;
}

// Xbar_j += sigma-bar_k conj(D_kj) with the group's coefficients held as for
// row_sig (kernels.hpp), in the operand order of the LDS form.
template <int MJ, int GS, int J0, int K>
__device__ __forceinline__ void b12r_xb_k(const double2 (&C)[GS * MJ / 16], const double2 (&sbv)[GS],
                                          double2 (&Xb)[MJ]) {
  constexpr int E = K * MJ + J0, M = E >> 4, L = E & 15;
  fmac_row<L, false>(Xb[J0].x, C[M].y, sbv[K].y);
  fmac_row<L, false>(Xb[J0].x, C[M].x, sbv[K].x);
  fmac_row<L, true>(Xb[J0].y, C[M].y, sbv[K].x);
  fmac_row<L, false>(Xb[J0].y, C[M].x, sbv[K].y);
  if constexpr (K + 1 < GS) b12r_xb_k<MJ, GS, J0, K + 1>(C, sbv, Xb);
}
template <int MJ, int GS, int J0>
__device__ __forceinline__ void b12r_xb(uint32_t um, const double2 (&C)[GS * MJ / 16], const double2 (&sbv)[GS],
                                        double2 (&Xb)[MJ]) {
  if (um & (1u << J0)) b12r_xb_k<MJ, GS, J0, 0>(C, sbv, Xb);
  if constexpr (J0 + 1 < MJ) b12r_xb<MJ, GS, J0 + 1>(um, C, sbv, Xb);
}

template <int MJ, int GS, bool YREG, int CH>
__device__ __forceinline__ void b12r_body(const Dev& d, const ClassDev& cd, const GradDev& g, const ClassGrad& cg,
                                          const uint3 bid) {
  extern __shared__ double sY[];            // [n_a][256]
  __shared__ double sUa[CH][16];
  __shared__ double sUb[CH][16];
  __shared__ double sG[CH];
  __shared__ double2 sD[CH][MJ];
  __shared__ uint32_t sM[CH];
  __shared__ uint64_t sStr[CH];
  __shared__ uint64_t sOcc[CH];           // up to 8 occupied spinors per string, one byte each
  __shared__ double sRow[16], sCol[16];
  const int tps = bid.y;                    // cores fastest: blocks of one sub-tile share its tables
  const int tp = tps >> 4, sub = tps & 15;
  const int sa = sub >> 2, sb = sub & 3;
  const int c = bid.x;
  const int I = d.tile_pairs[2 * tp], Jt = d.tile_pairs[2 * tp + 1];
  if (I == Jt && sa > sb) return;            // sub-tile below the diagonal: no rows
  const int tid = threadIdx.x, ia = tid >> 4, ib = tid & 15;
  const int la = sa * 16 + ia, lb = sb * 16 + ib;
  const int nv = d.n_v, nc = d.n_c, na = d.n_a;
  int a = I * 64 + la, b = Jt * 64 + lb;
  const bool valid = (a < b) && (b < nv);
  if (!valid) {
    a = 0;
    b = nv > 1 ? 1 : 0;
  }
  const int J = cd.n_pat;
  const int64_t n = d.n, gfc = d.n_fc, gv = d.n_fc + d.n_o, ga = d.n_fc + d.n_c;
  const double* __restrict__ W = d.W;
  const double rowc = -d.eps[d.n_o + a] - d.eps[d.n_o + b] - W[(gv + a) * n + gv + b] + W[(gfc + c) * n + gv + a] +
                      W[(gfc + c) * n + gv + b];
  const double N = d.scal[1], oneN = 1.0 / N, twoN = 2.0 / N;
  double2 X[MJ], Xb[MJ];
#pragma unroll
  for (int j = 0; j < MJ; ++j) {
    X[j] = make_double2(0.0, 0.0);
    Xb[j] = make_double2(0.0, 0.0);
    if (j < J) {
      const int64_t pr = occ_pair(c, nc + cd.pat[j].a0, d.n_o);
      X[j] = d.A[(pr * d.n_tp + tp) * 4096 + la * 64 + lb];
    }
  }
  constexpr int NY = YREG ? MJ : 1;
  double y[NY];
#pragma unroll
  for (int t = 0; t < NY; ++t) y[t] = 0.0;
  if (!YREG)
    for (int t = 0; t < na; ++t) sY[t * 256 + tid] = 0.0;
  const double epsc = d.eps[c];
  double q = 0.0, e2 = 0.0;
  const int64_t S = cd.n_str;
  for (int64_t s0 = 0; s0 < S; s0 += CH) {
    __syncthreads();
    for (int e = tid; e < CH * 16; e += 256) {
      const int sl = e >> 4, l = e & 15;
      const int64_t s = s0 + sl;
      const int aa = I * 64 + sa * 16 + l, bb = Jt * 64 + sb * 16 + l;
      sUa[sl][l] = (s < S && aa < nv) ? cd.Uv[s * nv + aa] : 0.0;
      sUb[sl][l] = (s < S && bb < nv) ? cd.Uv[s * nv + bb] : 0.0;
    }
    for (int e = tid; e < CH * MJ; e += 256) {
      const int sl = e / MJ, j = e % MJ;
      const int64_t s = s0 + sl;
      sD[sl][j] = (s < S && j < J) ? cd.D[s * J + j] : make_double2(0.0, 0.0);
    }
    if (tid < CH) {
      const int64_t s = s0 + tid;
      sG[tid] = (s < S) ? cd.T[s] + cd.Uc[s * nc + c] + epsc : 1e30;
      sM[tid] = (s < S) ? cd.mask[s] : 0u;
      const uint64_t str = (s < S) ? cd.strings[s] : 0ull;
      sStr[tid] = str;
      // the string's occupied spinors, padded with row n_a of sY (a row that
      // is never read); all ones marks a string with more than 8
      uint64_t ol = ~0ull;
      if (__builtin_popcountll(str) <= 8) {
        ol = 0;
        uint64_t x = str;
        for (int i = 0; i < 8; ++i) {
          const uint64_t t = x ? (uint64_t)__builtin_ctzll(x) : (uint64_t)na;
          x &= x - 1;
          ol |= t << (8 * i);
        }
      }
      sOcc[tid] = ol;
    }
    __syncthreads();
#pragma unroll 1
    for (int sl = 0; sl < CH; sl += GS) {
      uint32_t um = 0;
#pragma unroll
      for (int k = 0; k < GS; ++k) um |= sM[sl + k];
      um = __builtin_amdgcn_readfirstlane(um);
      double2 sg[GS];
#pragma unroll
      for (int k = 0; k < GS; ++k) sg[k] = make_double2(0.0, 0.0);
      static_assert((GS * MJ) % 16 == 0, "a group's coefficients fill whole rows");
      double2 C[GS * MJ / 16];
      {
        const double2* cgrp = &sD[sl][0];    // the group's GS MJ coefficients, contiguous
#pragma unroll
        for (int m = 0; m < GS * MJ / 16; ++m) C[m] = cgrp[(tid & 15) + 16 * m];
      }
      row_sig<MJ, GS, 0>(um, C, X, sg);
      double dd[GS];
#pragma unroll
      for (int k = 0; k < GS; ++k) dd[k] = valid ? (sG[sl + k] + rowc) - sUa[sl + k][ia] - sUb[sl + k][ib] : 1.0;
      double w[GS];
      if (GS == 4) {
        const double p01 = dd[0] * dd[1], p23 = dd[2 % GS] * dd[3 % GS];
        const double r = rcp_nr(p01 * p23);
        const double r01 = r * p23, r23 = r * p01;
        w[0] = r01 * dd[1];
        w[1] = r01 * dd[0];
        w[2 % GS] = r23 * dd[3 % GS];
        w[3 % GS] = r23 * dd[2 % GS];
      } else {
        const double r = rcp_nr(dd[0] * dd[1 % GS]);
        w[0] = r * dd[1 % GS];
        w[1 % GS] = r * dd[0];
      }
      double2 sbv[GS];
      double dl[GS];
#pragma unroll
      for (int k = 0; k < GS; ++k) {
        const double2 t = make_double2(sg[k].x * w[k], sg[k].y * w[k]);
        sbv[k] = valid ? make_double2(twoN * t.x, twoN * t.y) : make_double2(0.0, 0.0);
        dl[k] = valid ? -oneN * cabs2(t) : 0.0;
        e2 += valid ? cabs2(sg[k]) * w[k] : 0.0;
        q += dl[k];
      }
      // Xbar_j += sigma-bar conj(D_j); the coefficients are read again
      // rather than held through the denominators (the registers are short;
      // the empty asm with a memory clobber keeps the two reads apart)
      asm volatile("" ::: "memory");
      {
        const double2* cgrp = &sD[sl][0];
#pragma unroll
        for (int m = 0; m < GS * MJ / 16; ++m) C[m] = cgrp[(tid & 15) + 16 * m];
      }
      b12r_xb<MJ, GS, 0>(um, C, sbv, Xb);
#pragma unroll
      for (int k = 0; k < GS; ++k) {
        const uint64_t str = uniform64(sStr[sl + k]);
        if (YREG) {
#pragma unroll
          for (int t = 0; t < NY; ++t)
            if ((str >> t) & 1ull) y[t] += dl[k];
        } else {
          const uint64_t ol = uniform64(sOcc[sl + k]);
          if (ol != ~0ull) {
            // eight adds at addresses taken from the byte list, no bit scan
#pragma unroll
            for (int i = 0; i < 8; ++i) atomicAdd(&sY[(int)((ol >> (8 * i)) & 0xff) * 256 + tid], dl[k]);
          } else {
            uint64_t x = str;
            while (x) {
              const int t = __builtin_ctzll(x);
              x &= x - 1;
              atomicAdd(&sY[t * 256 + tid], dl[k]);
            }
          }
        }
      }
    }
  }
  // pair-integral adjoints of this row (each written once)
  if (valid) {
#pragma unroll
    for (int j = 0; j < MJ; ++j)
      if (j < J) {
        const int64_t pr = occ_pair(c, nc + cd.pat[j].a0, d.n_o);
        g.Ab[(pr * d.n_tp + tp) * 4096 + la * 64 + lb] = Xb[j];
      }
    atomicAdd(&g.Wb[(gv + a) * n + gv + b], -q);
  }
  if (YREG) {
#pragma unroll
    for (int t = 0; t < NY; ++t)
      if (t < na) sY[t * 256 + tid] = y[t];
  }
  const double e2b = block_sum256(e2);
  if (tid == 0) cd.part[(int64_t)bid.y * nc + c] = e2b;
  // row constants: eps and W of c, a, b
  __syncthreads();
  if (tid < 16) {
    sRow[tid] = 0.0;
    sCol[tid] = 0.0;
  }
  __syncthreads();
  const double qr = xsum16(q);
  if (ib == 0) sRow[ia] = qr;
  const double qc = xsum4(q);
  if ((tid & 63) < 16) atomicAdd(&sCol[ib], qc);
  __syncthreads();
  if (tid < 32) {
    const bool isa = tid < 16;
    const int x = tid & 15;
    const double v = isa ? sRow[x] : sCol[x];
    const int vv = isa ? I * 64 + sa * 16 + x : Jt * 64 + sb * 16 + x;
    if (vv < nv && v != 0.0) {
      atomicAdd(&g.epsb[d.n_o + vv], -v);
      atomicAdd(&g.Wb[(gfc + c) * n + gv + vv], v);
    }
    if (tid == 0) {
      double tot = 0.0;
      for (int y = 0; y < 16; ++y) tot += sRow[y];
      atomicAdd(&g.epsb[c], tot);
    }
  }
  // Uv tables of the sub-tile's a (sum over b) and b (sum over a)
  for (int e = tid; e < na * 32; e += 256) {
    const int t = e >> 5, x = e & 31;
    const double* yt = sY + t * 256;
    double v = 0.0;
    int vv;
    if (x < 16) {
      for (int y = 0; y < 16; ++y) v += yt[x * 16 + y];
      vv = I * 64 + sa * 16 + x;
    } else {
      for (int y = 0; y < 16; ++y) v += yt[y * 16 + x - 16];
      vv = Jt * 64 + sb * 16 + x - 16;
    }
    if (vv < nv && v != 0.0) atomicAdd(&g.Wb[(gv + vv) * n + ga + t], -v);
  }
}

// String pass of class (1,2): one thread per string (its dense coefficients
// and their adjoints in registers), the couplings of one a-row (64 b of a
// tile) staged in LDS at a time.  Per part (core c, group of tile pairs):
//   Dbar[s][j] = sum_rows conj(X_j) sigma-bar,   Tbar[s] = sum_rows Delta-bar,
// and the Uc table of c: W[c][t] += sum_s [t in s] Tbar_part[s].
// grid (ceil(S/256), n_c * groups), block 256.
template <int MJ>
__device__ __forceinline__ void b12s_wide(const Dev& d, const ClassDev& cd, const GradDev& g, const ClassGrad& cg,
                                          const uint3 bid, double2 (*sX)[MJ]) {
  __shared__ double sQ[64];
  __shared__ double sZ[64];
  const int tid = threadIdx.x;
  const int64_t S = cd.n_str;
  int64_t s = (int64_t)bid.x * 256 + tid;
  const bool live = s < S;
  if (!live) s = S - 1;
  const int part = bid.y;
  const int ngr = (int)((d.n_tp + cg.rows_per_part - 1) / cg.rows_per_part);
  const int c = part / ngr;
  const int64_t tp0 = (int64_t)(part % ngr) * cg.rows_per_part;
  const int64_t tp1 = min(d.n_tp, tp0 + cg.rows_per_part);
  const int J = cd.n_pat;
  const int nv = d.n_v, nc = d.n_c, na = d.n_a;
  const int64_t n = d.n, gfc = d.n_fc, gv = d.n_fc + d.n_o, ga = d.n_fc + d.n_c;
  const double N = d.scal[1], oneN = 1.0 / N, twoN = 2.0 / N;
  double2 D[MJ], Db[MJ];
#pragma unroll
  for (int j = 0; j < MJ; ++j) {
    D[j] = (j < J) ? cd.D[s * J + j] : make_double2(0.0, 0.0);
    Db[j] = make_double2(0.0, 0.0);
  }
  uint32_t um = live ? cd.mask[s] : 0u;
  for (int o = 1; o < 64; o <<= 1) um |= __shfl_xor(um, o, 64);
  um = __builtin_amdgcn_readfirstlane(um);   // wave-uniform: scalar branches below
  const double Gs = cd.T[s] + cd.Uc[s * nc + c] + d.eps[c];
  const double* Uvs = cd.Uv + s * nv;
  double tq = 0.0;
  if (tid < 64) sZ[tid] = 0.0;
  __syncthreads();
  for (int64_t tp = tp0; tp < tp1; ++tp) {
    const int I = d.tile_pairs[2 * tp], Jt = d.tile_pairs[2 * tp + 1];
    for (int la = 0; la < 64; ++la) {
      const int a = I * 64 + la;
      if (a >= nv || Jt * 64 + 63 <= a) break;
      __syncthreads();
      for (int e = tid; e < 64 * MJ; e += 256) {
        const int j = e >> 6, lb = e & 63;
        const int b = Jt * 64 + lb;
        double2 v = make_double2(0.0, 0.0);
        if (j < J && b > a && b < nv) {
          const int64_t pr = occ_pair(c, nc + cd.pat[j].a0, d.n_o);
          v = d.A[(pr * d.n_tp + tp) * 4096 + la * 64 + lb];
        }
        sX[lb][j] = v;
      }
      if (tid < 64) {
        const int b = Jt * 64 + tid;
        sQ[tid] = (b > a && b < nv) ? -d.eps[d.n_o + a] - d.eps[d.n_o + b] - d.W[(gv + a) * n + gv + b] +
                                          d.W[(gfc + c) * n + gv + a] + d.W[(gfc + c) * n + gv + b]
                                    : 0.0;
      }
      __syncthreads();
      const double ga_s = Gs - Uvs[a];
      const int lb0 = max(0, a + 1 - Jt * 64);
      const int lb1 = min(64, nv - Jt * 64);
      // four consecutive b share one reciprocal (products of the denominators)
      for (int lb = lb0; lb < lb1; lb += 4) {
        double2 sg[4];
        double dd[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int l = min(lb + k, lb1 - 1);
          sg[k] = make_double2(0.0, 0.0);
#pragma unroll
          for (int j = 0; j < MJ; ++j)
            if (um & (1u << j)) sg[k] = cfma(D[j], sX[l][j], sg[k]);
          dd[k] = ga_s + sQ[l] - Uvs[Jt * 64 + l];
        }
        const double p01 = dd[0] * dd[1], p23 = dd[2] * dd[3];
        const double r = rcp_nr(p01 * p23);
        const double r01 = r * p23, r23 = r * p01;
        double w[4];
        w[0] = r01 * dd[1];
        w[1] = r01 * dd[0];
        w[2] = r23 * dd[3];
        w[3] = r23 * dd[2];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          if (lb + k >= lb1) break;
          const double2 t = make_double2(sg[k].x * w[k], sg[k].y * w[k]);
          const double2 sbv = make_double2(twoN * t.x, twoN * t.y);
          tq -= oneN * cabs2(t);
#pragma unroll
          for (int j = 0; j < MJ; ++j)
            if (um & (1u << j)) {   // Dbar_j += sigma-bar conj(X_j)
              const double2 xv = sX[lb + k][j];
              Db[j].x = fma(sbv.x, xv.x, fma(sbv.y, xv.y, Db[j].x));
              Db[j].y = fma(sbv.y, xv.x, fma(-sbv.x, xv.y, Db[j].y));
            }
        }
      }
    }
  }
  if (live) {
    double2* out = cg.dbp + ((int64_t)part * S + s) * J;
#pragma unroll
    for (int j = 0; j < MJ; ++j)
      if (j < J) out[j] = Db[j];
    cg.Tb[(int64_t)part * S + s] = tq;
    uint64_t x = cd.strings[s];
    while (x) {
      const int t = __builtin_ctzll(x);
      x &= x - 1;
      atomicAdd(&sZ[t], tq);
    }
  }
  __syncthreads();
  if (tid < na && sZ[tid] != 0.0) atomicAdd(&g.Wb[(gfc + c) * n + ga + tid], sZ[tid]);
}

// The same pass when the block's strings couple through at most MQ patterns
// (the union of their masks, the usual case: strings come ordered by mask):
// only those patterns' couplings are staged, the coefficients and their
// adjoints sit compacted in MQ registers, and each coupling read from LDS
// serves both sigma and the coefficient adjoint of its determinant (one
// reciprocal per determinant instead of one per four; half the LDS reads).
// Slots beyond the block's nq patterns hold zero coefficients and couplings,
// so the per-determinant loops run over all MQ slots without branches (MQ is
// nq rounded up to an even count by the caller).
template <int MQ>
__device__ __forceinline__ void b12s_compact(const Dev& d, const ClassDev& cd, const GradDev& g, const ClassGrad& cg,
                                             const uint3 bid, uint32_t um, double2 (*sX)[MQ]) {
  __shared__ double sQ[64];
  __shared__ double sZ[64];
  const int tid = threadIdx.x;
  const int64_t S = cd.n_str;
  int64_t s = (int64_t)bid.x * 256 + tid;
  const bool live = s < S;
  if (!live) s = S - 1;
  const int part = bid.y;
  const int ngr = (int)((d.n_tp + cg.rows_per_part - 1) / cg.rows_per_part);
  const int c = part / ngr;
  const int64_t tp0 = (int64_t)(part % ngr) * cg.rows_per_part;
  const int64_t tp1 = min(d.n_tp, tp0 + cg.rows_per_part);
  const int J = cd.n_pat;
  const int nv = d.n_v, nc = d.n_c, na = d.n_a;
  const int64_t n = d.n, gfc = d.n_fc, gv = d.n_fc + d.n_o, ga = d.n_fc + d.n_c;
  const double N = d.scal[1], oneN = 1.0 / N, twoN = 2.0 / N;
  // the block's patterns, in order: jl[q], q < nq
  int jl[MQ];
  const int nq = __builtin_popcount(um);
  {
    uint32_t m = um;
#pragma unroll
    for (int q = 0; q < MQ; ++q) {
      jl[q] = m ? __builtin_ctz(m) : 0;
      m &= m - 1;
    }
  }
  double2 Dc[MQ], Dbc[MQ];
#pragma unroll
  for (int q = 0; q < MQ; ++q) {
    Dc[q] = q < nq ? cd.D[s * J + jl[q]] : make_double2(0.0, 0.0);
    Dbc[q] = make_double2(0.0, 0.0);
  }
  int64_t prq[MQ];   // occupied pair of (c, the pattern's active spinor)
#pragma unroll
  for (int q = 0; q < MQ; ++q) prq[q] = q < nq ? occ_pair(c, nc + cd.pat[jl[q]].a0, d.n_o) : 0;
  const double Gs = cd.T[s] + cd.Uc[s * nc + c] + d.eps[c];
  const double* Uvs = cd.Uv + s * nv;
  double tq = 0.0;
  if (tid < 64) sZ[tid] = 0.0;
  __syncthreads();
  for (int64_t tp = tp0; tp < tp1; ++tp) {
    const int I = d.tile_pairs[2 * tp], Jt = d.tile_pairs[2 * tp + 1];
    for (int la = 0; la < 64; ++la) {
      const int a = I * 64 + la;
      if (a >= nv || Jt * 64 + 63 <= a) break;
      __syncthreads();
      for (int e = tid; e < 64 * MQ; e += 256) {
        const int q = e >> 6, lb = e & 63;
        const int b = Jt * 64 + lb;
        double2 v = make_double2(0.0, 0.0);
        int64_t pr = 0;
#pragma unroll
        for (int u = 0; u < MQ; ++u)
          if (u == q) pr = prq[u];
        if (q < nq && b > a && b < nv) v = d.A[(pr * d.n_tp + tp) * 4096 + la * 64 + lb];
        sX[lb][q] = v;
      }
      if (tid < 64) {
        const int b = Jt * 64 + tid;
        sQ[tid] = (b > a && b < nv) ? -d.eps[d.n_o + a] - d.eps[d.n_o + b] - d.W[(gv + a) * n + gv + b] +
                                          d.W[(gfc + c) * n + gv + a] + d.W[(gfc + c) * n + gv + b]
                                    : 0.0;
      }
      __syncthreads();
      const double ga_s = Gs - Uvs[a];
      const int lb0 = max(0, a + 1 - Jt * 64);
      const int lb1 = min(64, nv - Jt * 64);
      for (int l = lb0; l < lb1; ++l) {
        double2 xv[MQ];
        double2 sg = make_double2(0.0, 0.0);
#pragma unroll
        for (int q = 0; q < MQ; ++q) {
          xv[q] = sX[l][q];
          sg = cfma(Dc[q], xv[q], sg);
        }
        const double w = rcp_nr(ga_s + sQ[l] - Uvs[Jt * 64 + l]);
        const double2 t = make_double2(sg.x * w, sg.y * w);
        const double2 sbv = make_double2(twoN * t.x, twoN * t.y);
        tq -= oneN * cabs2(t);
#pragma unroll
        for (int q = 0; q < MQ; ++q) {   // Dbar_j += sigma-bar conj(X_j)
          Dbc[q].x = fma(sbv.x, xv[q].x, fma(sbv.y, xv[q].y, Dbc[q].x));
          Dbc[q].y = fma(sbv.y, xv[q].x, fma(-sbv.x, xv[q].y, Dbc[q].y));
        }
      }
    }
  }
  if (live) {
    double2* out = cg.dbp + ((int64_t)part * S + s) * J;
#pragma unroll
    for (int q = 0; q < MQ; ++q)
      if (q < nq) out[jl[q]] = Dbc[q];
    cg.Tb[(int64_t)part * S + s] = tq;
    uint64_t x = cd.strings[s];
    while (x) {
      const int t = __builtin_ctzll(x);
      x &= x - 1;
      atomicAdd(&sZ[t], tq);
    }
  }
  __syncthreads();
  if (tid < na && sZ[tid] != 0.0) atomicAdd(&g.Wb[(gfc + c) * n + ga + tid], sZ[tid]);
}

// String pass of class (1,2): the compact form when the block's strings couple
// through at most 12 patterns, else the wide form.
template <int MJ>
__device__ __forceinline__ void b12s_body(const Dev& d, const ClassDev& cd, const GradDev& g, const ClassGrad& cg,
                                          const uint3 bid) {
  __shared__ uint32_t sUm;
  const int64_t S = cd.n_str;
  const int64_t s = (int64_t)bid.x * 256 + threadIdx.x;
  if (threadIdx.x == 0) sUm = 0u;
  __syncthreads();
  if (s < S) atomicOr(&sUm, cd.mask[s]);
  __syncthreads();
  const uint32_t um = __builtin_amdgcn_readfirstlane(sUm);
  // one LDS buffer for whichever form runs
  constexpr int MB = MJ > 12 ? MJ : 12;
  __shared__ double2 sXb[64 * MB];
  const int nq = __builtin_popcount(um);
  if (MJ > 12 && nq > 12) b12s_wide<MJ>(d, cd, g, cg, bid, (double2(*)[MJ])sXb);
  else if (nq <= 4) b12s_compact<4>(d, cd, g, cg, bid, um, (double2(*)[4])sXb);
  else if (nq <= 6) b12s_compact<6>(d, cd, g, cg, bid, um, (double2(*)[6])sXb);
  else if (MJ <= 8 || nq <= 8) b12s_compact<8>(d, cd, g, cg, bid, um, (double2(*)[8])sXb);
  else if (nq <= 10) b12s_compact<10>(d, cd, g, cg, bid, um, (double2(*)[10])sXb);
  else b12s_compact<12>(d, cd, g, cg, bid, um, (double2(*)[12])sXb);
}

// ---- class (0,2) ---------------------------------------------------------------------
// sigma[s][b] = sum_k Md[s][k] A[sup_k][a][b] over a tile of at most 64 strings
// and the 64 b of a tile pair (the forward contraction on FP64 MFMA), with
//   Delta = T[s] - eps_a - eps_b - W_ab - Uv[s][a] - Uv[s][b].
// Two passes recompute sigma block by block; both keep every sum in a fixed
// order and write only entries they own, so the result repeats bit for bit:
//   row pass    (block: one a of a tile pair, every string tile):
//               Abar[sup_k][a][b] += sum_s conj(Md[s][k]) sigma-bar[s][b], a second
//               complex MFMA product with sigma-bar staged in LDS, added into
//               the block's own entries of Abar; the row constants (eps_a,
//               eps_b, W_ab) from the column sums of Delta-bar;
//   string pass (block: one string tile, 64 of its support columns, one part
//               of the (tile pair, a) rows): Mbar[s][k] = sum_b sigma-bar[s][b]
//               conj(A[sup_k][a][b]) accumulated on MFMA over the part's rows,
//               then per coupling cbe[e] = sign_e Mbar[s][ccol_e]; Tbar[s]; and
//               u[s][v] = sum of Delta-bar over the string's determinants with
//               virtual spinor v (a or b), for the Uv tables (b02w_body).

// sigma of one (string tile t, row (tp, la)) block on MFMA, then in place the
// adjoint sigma-bar = (2/N) sigma / Delta and dl = Delta-bar = -|sigma|^2 /
// (N Delta^2), zero outside the valid (string, a < b < n_v) entries, and adds
// |sigma|^2 / Delta of the valid entries to e2.  Ends with a barrier (the MFMA
// staging's last).
__device__ __forceinline__ void b02_tile(const Dev& d, const ClassDev& cd, int64_t t, int64_t tp, int la,
                                         double4* sA, double2* sB, d4 (&aR)[2][2], d4 (&aI)[2][2],
                                         double (&dl)[2][2][4], double& e2) {
  const int s0 = cd.tile_s0[t], s1 = cd.tile_s0[t + 1];
  const int k0 = cd.tile_k0[t], K = cd.tile_k0[t + 1] - k0;
  const double2* M = cd.Md + (int64_t)64 * k0;
  const int32_t* sup = cd.tile_sup + k0;
  const double2* Ar = d.A + tp * 4096 + la * 64;
  auto fa = [&](int r, int k) -> double2 { return M[r * K + k]; };
  auto fb = [&](int r, int k) -> double2 {
    const int pr = sup[k];
    return pr < 0 ? make_double2(0.0, 0.0) : Ar[(int64_t)pr * d.n_tp * 4096 + r];
  };
  cgemm64<true>(fa, fb, K, sA, sB, aR, aI);
  const int I = d.tile_pairs[2 * tp], Jt = d.tile_pairs[2 * tp + 1];
  const int nv = d.n_v;
  const int a = I * 64 + la;
  const int64_t gv = d.n_fc + d.n_o;
  const double ea = d.eps[d.n_o + a];
  const double N = d.scal[1], oneN = 1.0 / N, twoN = 2.0 / N;
  double rowc[2];
  bool bok[2];
  int bb[2];
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int b = Jt * 64 + acc_col(j);
    bok[j] = (a < b) && (b < nv);
    bb[j] = bok[j] ? b : a;
    rowc[j] = bok[j] ? -ea - d.eps[d.n_o + b] - d.W[(gv + a) * d.n + gv + b] : 0.0;
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int s = s0 + acc_row(i, r);
      const bool sok = s < s1;
      const int64_t so = (int64_t)(sok ? s : s0) * nv;
      const double Ts = cd.T[sok ? s : s0], ua = cd.Uv[so + a];
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const bool ok = sok && bok[j];
        const double del = (Ts + rowc[j]) - ua - cd.Uv[so + bb[j]];
        const double gw = ok ? rcp_nr(del) : 0.0;
        const double sx = aR[i][j][r], sy = aI[i][j][r];
        aR[i][j][r] = twoN * gw * sx;
        aI[i][j][r] = twoN * gw * sy;
        dl[i][j][r] = -oneN * gw * gw * fma(sx, sx, sy * sy);
        e2 = fma(gw, fma(sx, sx, sy * sy), e2);
      }
    }
}

// Row pass.  grid (64 n_tp) (block = tp * 64 + la), block 256.
__device__ __forceinline__ void b02r_body(const Dev& d, const ClassDev& cd, const GradDev& g, const uint3 bid) {
  __shared__ double4 sA[64 * KP];
  __shared__ double2 sB[64 * KP];
  __shared__ double2 sS[64 * 65];          // sigma-bar [string][b]
  __shared__ double sQ[2][64];
  const int64_t tp = bid.x >> 6;
  const int la = bid.x & 63;
  const int I = d.tile_pairs[2 * tp], Jt = d.tile_pairs[2 * tp + 1];
  const int nv = d.n_v;
  const int a = I * 64 + la;
  if (a + 1 >= nv || a >= Jt * 64 + 63) return;   // no valid (a, b) in this block
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int64_t n = d.n, gv = d.n_fc + d.n_o;
  double2* Abr = g.Ab + tp * 4096 + la * 64;
  double q[2] = {0.0, 0.0};
  double e2 = 0.0;
  for (int64_t t = 0; t < cd.n_tiles; ++t) {
    const int k0 = cd.tile_k0[t], K = cd.tile_k0[t + 1] - k0;
    if (K == 0) continue;
    d4 aR[2][2], aI[2][2];
    double dl[2][2][4];
    b02_tile(d, cd, t, tp, la, sA, sB, aR, aI, dl, e2);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          sS[acc_row(i, r) * 65 + acc_col(j)] = make_double2(aR[i][j][r], aI[i][j][r]);
          q[j] += dl[i][j][r];
        }
    __syncthreads();
    const double2* M = cd.Md + (int64_t)64 * k0;
    const int32_t* sup = cd.tile_sup + k0;
    for (int kt0 = 0; kt0 < K; kt0 += 64) {
      auto fa = [&](int r, int s) -> double2 {   // conj(Md[s][kt0 + r])
        const int k = kt0 + r;
        if (k >= K) return make_double2(0.0, 0.0);
        const double2 v = M[s * K + k];
        return make_double2(v.x, -v.y);
      };
      auto fb = [&](int c, int s) -> double2 { return sS[s * 65 + c]; };
      d4 oR[2][2], oI[2][2];
      cgemm64<true>(fa, fb, 64, sA, sB, oR, oI);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int k = kt0 + acc_row(i, r);
          const int pr = k < K ? sup[k] : -1;
          if (pr < 0) continue;
#pragma unroll
          for (int j = 0; j < 2; ++j) {
            const int lb = acc_col(j), b = Jt * 64 + lb;
            if (a < b && b < nv) {
              double2* p = Abr + (int64_t)pr * d.n_tp * 4096 + lb;
              const double2 o = *p;
              *p = make_double2(o.x + oR[i][j][r], o.y + oI[i][j][r]);
            }
          }
        }
    }
  }
  const double e2b = block_sum256(e2);
  if (tid == 0) cd.part[bid.x] = e2b;
  // row constants: per column b the sum over strings of Delta-bar
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const double v = xsum4(q[j]);
    if ((lane >> 4) == 0) sQ[wv >> 1][acc_col(j)] = v;
  }
  __syncthreads();
  if (tid < 64) {
    const int b = Jt * 64 + tid;
    double qb = sQ[0][tid] + sQ[1][tid];
    if (!(a < b && b < nv)) qb = 0.0;
    if (qb != 0.0) {
      atomicAdd(&g.epsb[d.n_o + b], -qb);
      atomicAdd(&g.Wb[(gv + a) * n + gv + b], -qb);
    }
    double tot = qb;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) tot += __shfl_xor(tot, o, 64);
    if (tid == 0 && tot != 0.0) atomicAdd(&g.epsb[d.n_o + a], -tot);
  }
}

// String pass.  grid (n_tiles * nkb (tile, block of 64 support columns), parts),
// nkb = the widest tile's support in 64-column blocks; block 256.
__device__ __forceinline__ void b02s_body(const Dev& d, const ClassDev& cd, const GradDev& g, const ClassGrad& cg,
                                          const uint3 bid, int nkb) {
  __shared__ double4 sA[64 * KP];
  __shared__ double2 sB[64 * KP];
  __shared__ double2 sS[64 * 65];          // sigma-bar [string][b], at the end Mbar [string][column]
  __shared__ double sRow[2][64];
  const int64_t t = bid.x / nkb;
  const int kt0 = (int)(bid.x % nkb) * 64;
  const bool first = kt0 == 0;             // the first column block also owns Tbar and u
  const int part = bid.y;
  const int s0 = cd.tile_s0[t], s1 = cd.tile_s0[t + 1];
  const int k0 = cd.tile_k0[t], K = cd.tile_k0[t + 1] - k0;
  if (kt0 > 0 && kt0 >= K) return;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int nv = d.n_v;
  const int64_t S = cd.n_str;
  const int64_t nrow = 64 * d.n_tp;
  const int64_t r0 = (int64_t)part * cg.rows_per_part, r1 = min(nrow, r0 + cg.rows_per_part);
  const int32_t* sup = cd.tile_sup + k0;
  double* u2 = cg.u2 + (int64_t)part * S * nv;
  d4 mR[2][2], mI[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      mR[i][j] = d4{0.0, 0.0, 0.0, 0.0};
      mI[i][j] = d4{0.0, 0.0, 0.0, 0.0};
    }
  double tq[2][4], ub[2][2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      tq[i][r] = 0.0;
#pragma unroll
      for (int j = 0; j < 2; ++j) ub[i][j][r] = 0.0;
    }
  // b side of u: sums over the rows of one tile pair, added when the tile pair changes
  auto flush_ub = [&](int64_t tpc) {
    const int Jc = d.tile_pairs[2 * tpc + 1];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int s = s0 + acc_row(i, r);
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const int b = Jc * 64 + acc_col(j);
          if (s < s1 && b < nv && ub[i][j][r] != 0.0) u2[(int64_t)s * nv + b] += ub[i][j][r];
          ub[i][j][r] = 0.0;
        }
      }
  };
  int64_t cur = -1;
  for (int64_t row = r0; row < r1; ++row) {
    const int64_t tp = row >> 6;
    const int la = (int)(row & 63);
    const int I = d.tile_pairs[2 * tp], Jt = d.tile_pairs[2 * tp + 1];
    const int a = I * 64 + la;
    if (a + 1 >= nv || a >= Jt * 64 + 63 || K == 0) continue;
    if (first && tp != cur) {
      if (cur >= 0) flush_ub(cur);
      cur = tp;
    }
    d4 aR[2][2], aI[2][2];
    double dl[2][2][4];
    double e2u = 0.0;   // E2 is the row pass's
    b02_tile(d, cd, t, tp, la, sA, sB, aR, aI, dl, e2u);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const double v = dl[i][0][r] + dl[i][1][r];
        if (first) {
          tq[i][r] += v;
          const double va = xsum16(v);   // a side: the string's sum over this wave's 32 columns
          if ((lane & 15) == 0) sRow[wv & 1][acc_row(i, r)] = va;
        }
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          sS[acc_row(i, r) * 65 + acc_col(j)] = make_double2(aR[i][j][r], aI[i][j][r]);
          if (first) ub[i][j][r] += dl[i][j][r];
        }
      }
    __syncthreads();
    if (first && tid < 64) {
      const int s = s0 + tid;
      const double va = sRow[0][tid] + sRow[1][tid];
      if (s < s1 && va != 0.0) u2[(int64_t)s * nv + a] += va;
    }
    const double2* Ar = d.A + tp * 4096 + la * 64;
    auto fa = [&](int r, int b) -> double2 { return sS[r * 65 + b]; };
    auto fb = [&](int c, int b) -> double2 {   // conj(A[sup_{kt0 + c}][a][b])
      const int k = kt0 + c;
      const int pr = k < K ? sup[k] : -1;
      if (pr < 0) return make_double2(0.0, 0.0);
      const double2 v = Ar[(int64_t)pr * d.n_tp * 4096 + b];
      return make_double2(v.x, -v.y);
    };
    cgemm64<false, false>(fa, fb, 64, sA, sB, mR, mI);
  }
  if (first) {
    if (cur >= 0) flush_ub(cur);
    // Tbar: per string the sum over the part's determinants
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const double v = xsum16(tq[i][r]);
        if ((lane & 15) == 0) sRow[wv & 1][acc_row(i, r)] = v;
      }
    __syncthreads();
    if (tid < 64 && s0 + tid < s1) cg.Tb[(int64_t)part * S + s0 + tid] = sRow[0][tid] + sRow[1][tid];
  }
  // coupling adjoints of the tile's strings through the columns of this block
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) sS[acc_row(i, r) * 65 + acc_col(j)] = make_double2(mR[i][j][r], mI[i][j][r]);
  __syncthreads();
  double2* cbe = cg.cbe + (int64_t)part * cd.n_conn;
  for (int sl = tid >> 2; sl < 64; sl += 64) {
    const int s = s0 + sl;
    if (s >= s1) continue;
    for (int e = cd.conn_ptr[s] + (tid & 3); e < cd.conn_ptr[s + 1]; e += 4) {
      const int c = cd.ccol[e] - kt0;
      if (c < 0 || c >= 64) continue;
      const double2 v = sS[sl * 65 + c];
      cbe[e] = cd.conn[2 * e] < 0 ? make_double2(-v.x, -v.y) : v;
    }
  }
}

// Uv tables of class (0,2): W[v][t] -= sum_s [t in s] sum_parts u[s][v].
// grid (ceil(n_v / 256), string chunks), block 256, dynamic LDS n_a * 256 doubles.
__device__ __forceinline__ void b02w_body(const Dev& d, const ClassDev& cd, const GradDev& g, const ClassGrad& cg,
                                          const uint3 bid, int nchunk) {
  extern __shared__ double sY[];
  const int tid = threadIdx.x;
  const int nv = d.n_v, na = d.n_a;
  const int v = bid.x * 256 + tid;
  const bool live = v < nv;
  const int64_t S = cd.n_str;
  for (int t = 0; t < na; ++t) sY[t * 256 + tid] = 0.0;
  const int64_t chunk = (S + nchunk - 1) / nchunk;
  const int64_t s_lo = (int64_t)bid.y * chunk, s_hi = min(S, s_lo + chunk);
  const int64_t per = S * nv;
  for (int64_t s = s_lo; s < s_hi; ++s) {
    double u = 0.0;
    if (live)
      for (int p = 0; p < cg.parts; ++p) u += cg.u2[p * per + s * nv + v];
    uint64_t x = uniform64(cd.strings[s]);
    while (x) {
      const int t = __builtin_ctzll(x);
      x &= x - 1;
      sY[t * 256 + tid] += u;
    }
  }
  if (!live) return;
  const int64_t gv = d.n_fc + d.n_o, ga = d.n_fc + d.n_c;
  for (int t = 0; t < na; ++t) {
    const double y = sY[t * 256 + tid];
    if (y != 0.0) atomicAdd(&g.Wb[(gv + v) * d.n + ga + t], -y);
  }
}

// ---- per-string adjoints -------------------------------------------------------
// T[s] = (E0 - E_core) - E_act(s):  dE0 += Tbar[s];  E_act(s) = sum_{t in s} eps_t
// + sum_{t<u in s} W_tu receives -Tbar[s].  Coupling adjoints go to C.
// Thread i handles string i (if i < S) and coupling i (if i < n_conn).
// grid (ceil(max(S, n_conn) / 256)), block 256.
__device__ __forceinline__ void bstrfin_body(const Dev& d, const ClassDev& cd, const GradDev& g,
                                             const ClassGrad& cg, const uint3 bid) {
  __shared__ double red[256];
  const int64_t S = cd.n_str;
  const int64_t i = (int64_t)bid.x * 256 + threadIdx.x;
  double T = 0.0;
  if (i < S) {
    for (int p = 0; p < cg.parts; ++p) T += cg.Tb[(int64_t)p * S + i];
    const double ea = -T;
    const int64_t n = d.n, ga = d.n_fc + d.n_c;
    uint64_t x = cd.strings[i];
    while (x) {
      const int t = __builtin_ctzll(x);
      x &= x - 1;
      atomicAdd(&g.epsb[d.n_c + t], ea);
      uint64_t y = x;
      while (y) {
        const int u = __builtin_ctzll(y);
        y &= y - 1;
        atomicAdd(&g.Wb[(ga + t) * n + ga + u], ea);
      }
    }
  }
  if (i < cd.n_conn) {
    const int32_t cb = cd.conn[2 * i];
    double2 v = make_double2(0.0, 0.0);
    if (cg.dbp) {          // dense coefficients: Cbar_beta += sign Dbar[s][j]
      // string of coupling i: the last s with conn_ptr[s] <= i
      int64_t lo = 0, hi = S - 1;
      while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (cd.conn_ptr[mid] <= i) lo = mid;
        else hi = mid - 1;
      }
      const int j = cd.conn[2 * i + 1];
      for (int p = 0; p < cg.parts; ++p) v = cadd(v, cg.dbp[((int64_t)p * S + lo) * cd.n_pat + j]);
      if (cb < 0) v = make_double2(-v.x, -v.y);
    } else {
      for (int p = 0; p < cg.parts; ++p) v = cadd(v, cg.cbe[(int64_t)p * cd.n_conn + i]);
    }
    catomic(&g.cb[cb & 0x7fffffff], v);
  }
  red[threadIdx.x] = T;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(&g.scal[0], red[0]);
}

// ---- reference energy ------------------------------------------------------------
// E0 - E_core = Re(C^H H~ C) / N: the adjoint of H~[i][j] is
// Ebar C_i conj(C_j) / N, carried into f, G, eps and W by the Slater-Condon
// rules of the forward build.  grid (ceil(np/16), ceil(np/16)), block 256.
__device__ __forceinline__ void bhpp_body(const Dev& d, const GradDev& g, const uint3 bid) {
  const int j = bid.x * 16 + (threadIdx.x & 15);
  const int i = bid.y * 16 + (threadIdx.x >> 4);
  if (i >= d.n_p || j >= d.n_p) return;
  const uint64_t bi = d.pstrings[i], bj = d.pstrings[j];
  const uint64_t cre = bi & ~bj, ann = bj & ~bi;
  const int nd = __popcll(cre);
  if (nd > 2) return;
  const double sc = g.scal[0] / d.scal[1];
  const double2 ci = d.c[i], cj = d.c[j];
  double2 hb = cmul(ci, cconj(cj));
  hb = make_double2(sc * hb.x, sc * hb.y);
  const int nc = d.n_c;
  const int64_t n = d.n, ga = d.n_fc + d.n_c;
  auto below = [](uint64_t s, int p) { return __popcll(s & ((1ull << p) - 1)) & 1; };
  if (nd == 0) {
    const double ea = hb.x;
    uint64_t x = bi;
    while (x) {
      const int t = __builtin_ctzll(x);
      x &= x - 1;
      atomicAdd(&g.epsb[nc + t], ea);
      uint64_t y = x;
      while (y) {
        const int u = __builtin_ctzll(y);
        y &= y - 1;
        atomicAdd(&g.Wb[(ga + t) * n + ga + u], ea);
      }
    }
  } else if (nd == 1) {
    const int p = __builtin_ctzll(cre), q = __builtin_ctzll(ann);
    int par = below(bj, q);
    const uint64_t mid = bj & ~(1ull << q);
    par ^= below(mid, p);
    const double2 xb = par ? make_double2(-hb.x, -hb.y) : hb;
    catomic(&g.fb[(int64_t)p * d.n_o + nc + q], xb);
    uint64_t x = mid;
    while (x) {
      const int w = __builtin_ctzll(x);
      x &= x - 1;
      catomic(&g.Gb[gidx(d, nc + q, p, nc + w, w)], xb);
      catomic(&g.Gb[gidx(d, nc + w, p, nc + q, w)], make_double2(-xb.x, -xb.y));
    }
  } else {
    const int q1 = __builtin_ctzll(ann), q2 = 63 - __builtin_clzll(ann);
    const int p1 = __builtin_ctzll(cre), p2 = 63 - __builtin_clzll(cre);
    uint64_t s = bj;
    int par = below(s, q1);
    s &= ~(1ull << q1);
    par ^= below(s, q2);
    s &= ~(1ull << q2);
    par ^= below(s, p1);
    s |= 1ull << p1;
    par ^= below(s, p2);
    const double2 xb = par ? make_double2(-hb.x, -hb.y) : hb;
    catomic(&g.Gb[gidx(d, nc + q1, p2, nc + q2, p1)], xb);
    catomic(&g.Gb[gidx(d, nc + q2, p2, nc + q1, p1)], make_double2(-xb.x, -xb.y));
  }
}

// ---- couplings of the classes with at most one virtual electron ------------------
// Transpose of the coupling build: Xbar[j][r] into f and G.
// grid (ceil(rows/256), n_pat), block 256.
__device__ __forceinline__ void bxbuild_body(const Dev& d, const ClassDev& cd, const GradDev& g,
                                             const ClassGrad& cg, const uint3 bid) {
  const int64_t r = bid.x * 256ll + threadIdx.x;
  const int j = bid.y;
  if (r >= cd.n_rows) return;
  const double2 xb = cg.Xb[(int64_t)j * cd.n_rows + r];
  if (xb.x == 0.0 && xb.y == 0.0) return;
  int c0, c1, a;
  decode_small_row(d, cd, r, &c0, &c1, &a);
  const Pattern pt = cd.pat[j];
  const int nc = d.n_c, na = d.n_a;
  const double2 mxb = make_double2(-xb.x, -xb.y);
  if (pt.kind == PAT_SINGLE) {
    const int qo = (cd.h == 1) ? c0 : nc + pt.a0;
    const int pr = (cd.v == 1) ? na + a : pt.r0;
    catomic(&g.fb[(int64_t)pr * d.n_o + qo], xb);
  } else if (pt.kind == PAT_SPECT) {
    const int qo = (cd.h == 1) ? c0 : nc + pt.a0;
    const int pr = (cd.v == 1) ? na + a : pt.r0;
    const int w = pt.w;
    catomic(&g.Gb[gidx(d, qo, pr, nc + w, w)], xb);
    catomic(&g.Gb[gidx(d, nc + w, pr, qo, w)], mxb);
  } else {
    int q, s;
    if (cd.h == 2) { q = c0; s = c1; }
    else if (cd.h == 1) { q = c0; s = nc + pt.a0; }
    else { q = nc + pt.a0; s = nc + pt.a1; }
    int rr, pr;
    if (cd.v == 1) { rr = pt.r0; pr = na + a; }
    else { rr = pt.r0; pr = pt.r1; }
    catomic(&g.Gb[gidx(d, q, pr, s, rr)], xb);
    catomic(&g.Gb[gidx(d, s, pr, q, rr)], mxb);
  }
}

// ---- pair integrals: A[xy][ab] = sum_L w_L (S_x[a] S_y[b] - S_y[a] S_x[b]) ----------
// with S_x[a][L] = sqrt|w_L| B[L][a][x].  With Atilde_xy[a][b] = Abar_xy[a][b]
// - Abar_xy[b][a] (zero where A is not stored) and Atilde_yx = Atilde_xy^T,
//   Sbar_x[a][L] = sign_L sum_{y != x} sum_b Atilde_xy[a][b] conj(S_y[b][L]),
// one complex FP64 MFMA GEMM per occupied x with K = (n_o - 1) n_v.
// grid (ceil(n_l/64), ceil(n_v/64) * n_o), block 256.
__device__ __forceinline__ void bagemm_body(const Dev& d, const GradDev& g, const uint3 bid) {
  // K runs over (y != x, b) in stages of one y and 16 consecutive b, so that
  // the Abar operand is read as contiguous runs of the tile-major adjoint:
  // D[a][b] = Abar[a][b] - Abar[b][a] of the pair (x, y) (sign flipped for
  // y < x), the first term row-wise from tile (I, J'), the second from tile
  // (J', I) with a fastest and transposed through LDS.
  __shared__ double2 sA[64 * KP];
  __shared__ double2 sB[64 * KP];
  const int nvt = (d.n_v + 63) / 64;
  const int x = bid.y / nvt;
  const int I = bid.y % nvt, a0 = I * 64;
  const int L0 = bid.x * 64;
  const int nv = d.n_v, nl = d.n_l, no = d.n_o;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wr = (wv >> 1) * 32, wc = (wv & 1) * 32;
  const int kq = lane >> 4, kcl = kq >> 1, comp = kq & 1;
  d4 accR[2][2], accI[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      accR[i][j] = d4{0.0, 0.0, 0.0, 0.0};
      accI[i][j] = d4{0.0, 0.0, 0.0, 0.0};
    }
  auto tpi = [&](int i0, int j0) -> int64_t {   // tile pair (i0 <= j0)
    return (int64_t)i0 * nvt - (int64_t)i0 * (i0 - 1) / 2 + (j0 - i0);
  };
  for (int y = 0; y < no; ++y) {
    if (y == x) continue;
    const int64_t pr = x < y ? occ_pair(x, y, no) : occ_pair(y, x, no);
    const double sgn = x < y ? 1.0 : -1.0;
    const double2* Sy = d.slab + ((int64_t)(d.n_fc + y) * d.n_corr + no) * nl;
    for (int b0 = 0; b0 < nv; b0 += KC) {
      const int Jb = b0 >> 6, lb0 = b0 & 63;    // the 16 b lie in one tile (64 = 4 x 16)
      // D term 1: Abar[a][b] from tile (I, Jb), rows a, 16 consecutive b
      for (int e = tid; e < 64 * KC; e += 256) {
        const int r = e / KC, kk = e % KC;
        const int a = a0 + r, bb = b0 + kk;
        double2 v = make_double2(0.0, 0.0);
        if (I <= Jb && a < nv && bb < nv) v = g.Ab[(pr * d.n_tp + tpi(I, Jb)) * 4096 + r * 64 + lb0 + kk];
        sA[r * KP + kk] = make_double2(sgn * v.x, sgn * v.y);
      }
      // B operand: conj(S_y[b][L]), L fastest
      for (int e = tid; e < 64 * KC; e += 256) {
        const int c = e & 63, kk = e >> 6;
        const int L = L0 + c, bb = b0 + kk;
        sB[c * KP + kk] = (L < nl && bb < nv) ? cconj(Sy[(int64_t)bb * nl + L]) : make_double2(0.0, 0.0);
      }
      __syncthreads();
      // D term 2: - Abar[b][a] from tile (Jb, I), 16 rows b, a fastest
      if (Jb <= I) {
        for (int e = tid; e < 64 * KC; e += 256) {
          const int r = e & 63, kk = e >> 6;
          const int a = a0 + r, bb = b0 + kk;
          if (a < nv && bb < nv) {
            const double2 v = g.Ab[(pr * d.n_tp + tpi(Jb, I)) * 4096 + (lb0 + kk) * 64 + r];
            const double2 u = sA[r * KP + kk];
            sA[r * KP + kk] = make_double2(u.x - sgn * v.x, u.y - sgn * v.y);
          }
        }
        __syncthreads();
      }
#pragma unroll 2
      for (int ks = 0; ks < KC; ks += 2) {
        const int kc = ks + kcl;
        double ar[2], ai[2], bq[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          const double2 v = sA[(wr + i * 16 + (lane & 15)) * KP + kc];
          ar[i] = comp ? -v.y : v.x;
          ai[i] = comp ? v.x : v.y;
        }
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const double2 v = sB[(wc + j * 16 + (lane & 15)) * KP + kc];
          bq[j] = comp ? v.y : v.x;
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j) {
            accR[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i], bq[j], accR[i][j], 0, 0, 0);
            accI[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[i], bq[j], accI[i][j], 0, 0, 0);
          }
      }
      __syncthreads();
    }
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int a = a0 + acc_row(i, r), L = L0 + acc_col(j);
        if (a < nv && L < nl) {
          double2* p = g.slabb + ((int64_t)(d.n_fc + x) * d.n_corr + no + a) * nl + L;
          const double sg = d.sign[L];
          *p = cadd(*p, make_double2(sg * accR[i][j][r], sg * accI[i][j][r]));
        }
      }
}

// The same GEMM in 128 x 128 blocks (the 128 virtual a of two tiles, 128
// Cholesky columns), eight waves each computing a 64 x 32 part on FP64 MFMA:
// twice the products per staged operand of the 64 x 64 block.  Used where the
// blocks are nearly full (large n_v and N_L).
// grid (ceil(n_l/128), ceil(n_vt/2) * n_o), block 512.
__device__ __forceinline__ void bagemm128_body(const Dev& d, const GradDev& g, const uint3 bid) {
  __shared__ double4 sA[128 * KP];   // (re, im, -im, re): MFMA operands straight from LDS
  __shared__ double2 sB[128 * KP];
  const int nvt = (d.n_v + 63) / 64, nvt2 = (nvt + 1) / 2;
  const int x = bid.y / nvt2;
  const int I2 = bid.y % nvt2, a0 = I2 * 128;
  const int L0 = bid.x * 128;
  const int nv = d.n_v, nl = d.n_l, no = d.n_o;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int u = wv >> 2, cq = wv & 3;       // row half (64 a), column quarter (32 L)
  const int kq = lane >> 4, kcl = kq >> 1, comp = kq & 1;
  const int rowA = u * 64 + (lane & 15), rowB = cq * 32 + (lane & 15);
  d4 accR[4][2], accI[4][2];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      accR[i][j] = d4{0.0, 0.0, 0.0, 0.0};
      accI[i][j] = d4{0.0, 0.0, 0.0, 0.0};
    }
  auto tpi = [&](int i0, int j0) -> int64_t {   // tile pair (i0 <= j0)
    return (int64_t)i0 * nvt - (int64_t)i0 * (i0 - 1) / 2 + (j0 - i0);
  };
  // Stages run over (y != x, b0); the raw operands of the next stage are
  // fetched into registers while the current stage's products run (one block
  // per CU: nothing else would hide the fetch), and scaled when stored.
  // Element e = tid + 512 q (q < 4): term 1 and B at (r, kk) = (e / KC, e % KC),
  // term 2 at (r, kk) = (e % 128, e / 128) (a fastest, coalesced).
  double2 f1[4], fbv[4], f2[4];
  auto fetch = [&](int y, int b0) {
    const int64_t pr = x < y ? occ_pair(x, y, no) : occ_pair(y, x, no);
    const double2* Sy = d.slab + ((int64_t)(d.n_fc + y) * d.n_corr + no) * nl;
    const double2* Abp = g.Ab + pr * d.n_tp * 4096;
    const int Jb = b0 >> 6, lb0 = b0 & 63;    // the 16 b lie in one tile
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 512 * q;
      {
        const int r = e / KC, kk = e % KC;
        const int a = a0 + r, I = a >> 6, bb = b0 + kk;
        f1[q] = (I <= Jb && a < nv && bb < nv) ? Abp[tpi(I, Jb) * 4096 + (r & 63) * 64 + lb0 + kk]
                                                : make_double2(0.0, 0.0);
      }
      {
        const int c = e & 127, kk = e >> 7;
        const int L = L0 + c, bb = b0 + kk;
        fbv[q] = (L < nl && bb < nv) ? Sy[(int64_t)bb * nl + L] : make_double2(0.0, 0.0);
      }
      {
        const int r = e & 127, kk = e >> 7;
        const int a = a0 + r, I = a >> 6, bb = b0 + kk;
        f2[q] = (Jb <= I && a < nv && bb < nv) ? Abp[tpi(Jb, I) * 4096 + (lb0 + kk) * 64 + (r & 63)]
                                                : make_double2(0.0, 0.0);
      }
    }
  };
  auto next = [&](int& y, int& b0) {           // the stage after (y, b0); y = no at the end
    b0 += KC;
    if (b0 >= nv) {
      b0 = 0;
      ++y;
      if (y == x) ++y;
    }
  };
  int y = x == 0 ? 1 : 0, b0 = 0;
  if (y < no) fetch(y, b0);
  while (y < no) {
    const double sgn = x < y ? 1.0 : -1.0;
    const int Jb = b0 >> 6;
    const bool term2 = Jb <= 2 * I2 + 1;
    __syncthreads();                          // the previous stage's products are done
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 512 * q;
      {
        const int r = e / KC, kk = e % KC;
        const double2 v = f1[q];
        sA[r * KP + kk] = make_double4(sgn * v.x, sgn * v.y, -sgn * v.y, sgn * v.x);
      }
      {
        const int c = e & 127, kk = e >> 7;
        sB[c * KP + kk] = cconj(fbv[q]);
      }
    }
    // D term 2: - Abar[b][a] from tile (Jb, I), Jb <= I
    if (term2) {
      __syncthreads();
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int e = tid + 512 * q;
        const int r = e & 127, kk = e >> 7;
        const double2 v = f2[q];
        if (v.x != 0.0 || v.y != 0.0) {
          const double4 w = sA[r * KP + kk];
          const double nx = w.x - sgn * v.x, ny = w.y - sgn * v.y;
          sA[r * KP + kk] = make_double4(nx, ny, -ny, nx);
        }
      }
    }
    __syncthreads();
    int yn = y, bn = b0;
    next(yn, bn);
    if (yn < no) fetch(yn, bn);               // in flight during the products
#pragma unroll 2
    for (int ks = 0; ks < KC; ks += 2) {
      const int kc = ks + kcl;
      double ar[4], ai[4], bq[2];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const double2 v = ((const double2*)&sA[(rowA + i * 16) * KP + kc])[comp];
        ar[i] = v.x;
        ai[i] = v.y;
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) bq[j] = ((const double*)&sB[(rowB + j * 16) * KP + kc])[comp];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          accR[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i], bq[j], accR[i][j], 0, 0, 0);
          accI[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[i], bq[j], accI[i][j], 0, 0, 0);
        }
    }
    y = yn;
    b0 = bn;
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int a = a0 + u * 64 + i * 16 + (lane >> 4) + 4 * r, L = L0 + cq * 32 + j * 16 + (lane & 15);
        if (a < nv && L < nl) {
          double2* p = g.slabb + ((int64_t)(d.n_fc + x) * d.n_corr + no + a) * nl + L;
          const double sg = d.sign[L];
          *p = cadd(*p, make_double2(sg * accR[i][j][r], sg * accI[i][j][r]));
        }
      }
}

// Mixed form of bagemm_body: the same stages, the operands rounded to FP32
// as staged into three real planes (re, im, re + im) each, the product
// formed by three real FP32 MFMA products per complex product (Gauss, as in
// the forward pair-integral build) and each stage's sums carried into FP64.
__device__ __forceinline__ void bagemm_f32_body(const Dev& d, const GradDev& g, const uint3 bid) {
  constexpr int PL = 64 * KP;                 // floats of one plane
  __shared__ float sA[3 * PL];
  __shared__ float sB[3 * PL];
  const int nvt = (d.n_v + 63) / 64;
  const int x = bid.y / nvt;
  const int I = bid.y % nvt, a0 = I * 64;
  const int L0 = bid.x * 64;
  const int nv = d.n_v, nl = d.n_l, no = d.n_o;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wr = (wv >> 1) * 32, wc = (wv & 1) * 32;
  double accR[2][2][4], accI[2][2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        accR[i][j][r] = 0.0;
        accI[i][j][r] = 0.0;
      }
  auto tpi = [&](int i0, int j0) -> int64_t {   // tile pair (i0 <= j0)
    return (int64_t)i0 * nvt - (int64_t)i0 * (i0 - 1) / 2 + (j0 - i0);
  };
  for (int y = 0; y < no; ++y) {
    if (y == x) continue;
    const int64_t pr = x < y ? occ_pair(x, y, no) : occ_pair(y, x, no);
    const double sgn = x < y ? 1.0 : -1.0;
    const double2* Sy = d.slab + ((int64_t)(d.n_fc + y) * d.n_corr + no) * nl;
    for (int b0 = 0; b0 < nv; b0 += KC) {
      const int Jb = b0 >> 6, lb0 = b0 & 63;
      // D = Abar[a][b] - Abar[b][a] in FP64, then rounded once into the planes
      double2 dv[64 * KC / 256];
#pragma unroll
      for (int u = 0; u < 64 * KC / 256; ++u) {
        const int e = tid + 256 * u;
        const int r = e / KC, kk = e % KC;
        const int a = a0 + r, bb = b0 + kk;
        double2 v = make_double2(0.0, 0.0);
        if (a < nv && bb < nv) {
          if (I <= Jb) {
            const double2 t = g.Ab[(pr * d.n_tp + tpi(I, Jb)) * 4096 + r * 64 + lb0 + kk];
            v = make_double2(sgn * t.x, sgn * t.y);
          }
          if (Jb <= I) {
            const double2 t = g.Ab[(pr * d.n_tp + tpi(Jb, I)) * 4096 + (lb0 + kk) * 64 + r];
            v = make_double2(v.x - sgn * t.x, v.y - sgn * t.y);
          }
        }
        dv[u] = v;
      }
#pragma unroll
      for (int u = 0; u < 64 * KC / 256; ++u) {
        const int e = tid + 256 * u;
        const int o = (e / KC) * KP + e % KC;
        const float re = (float)dv[u].x, im = (float)dv[u].y;
        sA[o] = re;
        sA[PL + o] = im;
        sA[2 * PL + o] = re + im;
      }
      // B operand: conj(S_y[b][L]), L fastest
      for (int e = tid; e < 64 * KC; e += 256) {
        const int c = e & 63, kk = e >> 6;
        const int L = L0 + c, bb = b0 + kk;
        const double2 v = (L < nl && bb < nv) ? cconj(Sy[(int64_t)bb * nl + L]) : make_double2(0.0, 0.0);
        const float re = (float)v.x, im = (float)v.y;
        const int o = c * KP + kk;
        sB[o] = re;
        sB[PL + o] = im;
        sB[2 * PL + o] = re + im;
      }
      __syncthreads();
      f4 p1[2][2], p2[2][2], p3[2][2];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          p1[i][j] = f4{0.f, 0.f, 0.f, 0.f};
          p2[i][j] = f4{0.f, 0.f, 0.f, 0.f};
          p3[i][j] = f4{0.f, 0.f, 0.f, 0.f};
        }
#pragma unroll
      for (int ks = 0; ks < KC; ks += 4) {
        const int kc = ks + (lane >> 4);
        float av[3][2], bv[3][2];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
#pragma unroll
          for (int i = 0; i < 2; ++i) av[q][i] = sA[q * PL + (wr + i * 16 + (lane & 15)) * KP + kc];
#pragma unroll
          for (int j = 0; j < 2; ++j) bv[q][j] = sB[q * PL + (wc + j * 16 + (lane & 15)) * KP + kc];
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j) {
            p1[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[0][i], bv[0][j], p1[i][j], 0, 0, 0);
            p2[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[1][i], bv[1][j], p2[i][j], 0, 0, 0);
            p3[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[2][i], bv[2][j], p3[i][j], 0, 0, 0);
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
    }
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int a = a0 + acc_row_f32(i, r), L = L0 + acc_col(j);
        if (a < nv && L < nl) {
          double2* p = g.slabb + ((int64_t)(d.n_fc + x) * d.n_corr + no + a) * nl + L;
          const double sg = d.sign[L];
          *p = cadd(*p, make_double2(sg * accR[i][j][r], sg * accI[i][j][r]));
        }
      }
}

// ---- occupied-block integrals: G[m][k] = sum_L w_L P[m][L] Q[k][L] -----------------
// m = (x, p) over occupied x and active/virtual p, k = (y, q) over occupied y and
// active q, P[m] = S_x[p], Q[k] = S_y[q].
//   Pbar[m][L] = sign_L sum_k Gbar[m][k] conj(Q[k][L])   (which = 0)
//   Qbar[k][L] = sign_L sum_m Gbar[m][k] conj(P[m][L])   (which = 1)
// grid (ceil(n_l/64), ceil(rows/64)), block 256.
__device__ __forceinline__ void bggemm_body(const Dev& d, const GradDev& g, int which, const uint3 bid) {
  __shared__ double2 sA[64 * KP];
  __shared__ double2 sB[64 * KP];
  const int npr = d.n_a + d.n_v;
  const int64_t M = (int64_t)d.n_o * npr, N = (int64_t)d.n_o * d.n_a;
  const int64_t R = which ? N : M, K = which ? M : N;
  const int64_t m0 = (int64_t)bid.y * 64;
  const int L0 = bid.x * 64;
  const int nl = d.n_l;
  auto prow = [&](int64_t m) -> int64_t {    // slab row of P[m]
    return ((int64_t)(d.n_fc + m / npr) * d.n_corr + d.n_c + m % npr);
  };
  auto qrow = [&](int64_t k) -> int64_t {    // slab row of Q[k]
    return ((int64_t)(d.n_fc + k / d.n_a) * d.n_corr + d.n_c + k % d.n_a);
  };
  auto fa = [&](int r, int k) -> double2 {
    const int64_t m = m0 + r;
    if (m >= R) return make_double2(0.0, 0.0);
    return which ? g.Gb[(int64_t)k * N + m] : g.Gb[m * N + k];
  };
  auto fb = [&](int c, int k) -> double2 {
    const int L = L0 + c;
    if (L >= nl) return make_double2(0.0, 0.0);
    return cconj(d.slab[(which ? prow(k) : qrow(k)) * nl + L]);
  };
  d4 accR[2][2], accI[2][2];
  cgemm64(fa, fb, (int)K, sA, sB, accR, accI);
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t m = m0 + acc_row(i, r);
        const int L = L0 + acc_col(j);
        if (m < R && L < nl) {
          double2* p = g.slabb + (which ? qrow(m) : prow(m)) * nl + L;
          const double sg = d.sign[L];
          *p = cadd(*p, make_double2(sg * accR[i][j][r], sg * accI[i][j][r]));
        }
      }
}

// ---- core Fock block -------------------------------------------------------------
// f[p][q] = h_pq + sum_L w_L dsum_L B_pq - sum_{j core} sum_L w_L B_pj conj(B_qj)
// in slab form (p active/virtual row pr, q core/active qo).  Adjoint into the
// slab entries of frozen/core columns j and of column q.
// grid (n_occ, n_corr), block 64 (threads over L).
__device__ __forceinline__ void bfock_body(const Dev& d, const GradDev& g, const uint3 bid) {
  const int x = bid.x;        // slab column (global occupied index)
  const int pc = bid.y;       // slab row (correlated index)
  const int nl = d.n_l, no = d.n_o, nc = d.n_c, npr = d.n_a + d.n_v;
  const bool core_col = x < d.n_fc + nc;
  const bool coul = x >= d.n_fc && pc >= nc;
  if (!core_col && !coul) return;
  const double2* fb = g.fb;
  for (int L = threadIdx.x; L < nl; L += 64) {
    double2 acc = make_double2(0.0, 0.0);
    if (core_col) {
      if (pc >= nc) {            // B_pj with p = pr: -sum_q fbar[pr][q] S_j[q]
        const int pr = pc - nc;
        for (int qo = 0; qo < no; ++qo)
          acc = csub(acc, cmul(fb[(int64_t)pr * no + qo], d.slab[((int64_t)x * d.n_corr + qo) * nl + L]));
      }
      if (pc < no) {             // B_qj with q = pc: -sum_p conj(fbar[p][q]) S_j[p]
        for (int pr = 0; pr < npr; ++pr)
          acc = csub(acc, cmul(cconj(fb[(int64_t)pr * no + pc]), d.slab[((int64_t)x * d.n_corr + nc + pr) * nl + L]));
      }
    }
    if (coul) {
      const double2 f = fb[(int64_t)(pc - nc) * no + (x - d.n_fc)];
      acc = cadd(acc, make_double2(d.dsum[L] * f.x, d.dsum[L] * f.y));
    }
    const double sg = d.sign[L];
    double2* p = g.slabb + ((int64_t)x * d.n_corr + pc) * nl + L;
    *p = cadd(*p, make_double2(sg * acc.x, sg * acc.y));
  }
}

// dsumbar[L] = sign_L sum_{p, q} Re(conj(fbar[p][q]) S_q[p][L]).  grid (ceil(n_l/256)).
__device__ __forceinline__ void bdsum_body(const Dev& d, const GradDev& g, const uint3 bid) {
  const int L = bid.x * 256 + threadIdx.x;
  if (L >= d.n_l) return;
  const int no = d.n_o, npr = d.n_a + d.n_v;
  double acc = 0.0;
  for (int qo = 0; qo < no; ++qo)
    for (int pr = 0; pr < npr; ++pr) {
      const double2 f = g.fb[(int64_t)pr * no + qo];
      const double2 v = d.slab[((int64_t)(d.n_fc + qo) * d.n_corr + d.n_c + pr) * d.n_l + L];
      acc += f.x * v.x + f.y * v.y;
    }
  g.dsumb[L] = d.sign[L] * acc;
}

// h receives fbar (active/virtual x core/active block) and epsbar (diagonal);
// eps_p = h_pp + sum_{j core, j != p} W_pj gives Wbar[p][j] += epsbar[p].
// grid (ceil(n_corr / 256), 1 + n_o): row 0 handles eps, rows 1.. the f column qo.
__device__ __forceinline__ void bhfe_body(const Dev& d, const GradDev& g, const uint3 bid) {
  const int i = bid.x * 256 + threadIdx.x;
  const int64_t n = d.n;
  if (bid.y == 0) {
    if (i >= d.n_corr) return;
    const int64_t gg = d.n_fc + i;
    const double e = g.epsb[i];
    atomicAdd(&g.hb[gg * n + gg].x, e);
    for (int j = 0; j < d.n_fc + d.n_c; ++j)
      if (j != gg) g.Wb[gg * n + j] += e;
  } else {
    const int qo = bid.y - 1;
    const int npr = d.n_a + d.n_v;
    if (i >= npr) return;
    const int64_t gp = d.n_fc + d.n_c + i, gq = d.n_fc + qo;
    catomic(g.hb + gp * n + gq, g.fb[(int64_t)i * d.n_o + qo]);
  }
}

// Wsym = Wbar + Wbar^T.  grid (ceil(n/256), n).
__device__ __forceinline__ void bwsym_body(const Dev& d, const GradDev& g, const uint3 bid) {
  const int q = bid.x * 256 + threadIdx.x;
  const int p = bid.y;
  if (q >= d.n) return;
  const int64_t n = d.n;
  g.Wsym[p * n + q] = (p == q) ? 0.0 : g.Wb[p * n + q] + g.Wb[(int64_t)q * n + p];
}

// dgbar[L][p] = sign_L sum_q Wsym[q][p] dg[L][q] + [p frozen/core] dsumbar[L]
// (W_pq Coulomb part sign_L dg_p dg_q; dsum_L = sum_{j core} dg[L][j]).
// grid (ceil(n/256), n_l).
__device__ __forceinline__ void bdg_body(const Dev& d, const GradDev& g, const uint3 bid) {
  const int p = bid.x * 256 + threadIdx.x;
  const int L = bid.y;
  if (p >= d.n) return;
  const int64_t n = d.n;
  const double* dg = d.dg + (int64_t)L * n;
  double acc = 0.0;
  for (int q = 0; q < d.n; ++q) acc = fma(g.Wsym[(int64_t)q * n + p], dg[q], acc);
  acc *= d.sign[L];
  if (p < d.n_fc + d.n_c) acc += g.dsumb[L];
  g.dgb[(int64_t)L * n + p] = acc;
}

// ---- factor gradients ----------------------------------------------------------------
// Raw gradient of factor L of set t at (p, q):
//   R = -2 sign s^2 Wbar[p][q] B[p][q]          (p != q; exchange part of W)
//     + [p == q] s dgbar[L][p]                  (diagonals)
//     + [q occupied type, p correlated] s slabbar[q][p - n_fc][L]
// written as gradE2 (R(p,q) + conj(R(q,p))) / 2.  32 x 32 tiles through LDS.
// In the packed layout the stored entry (p, q), p < q, stands for both
// triangles, so its gradient is gradE2 (R(p,q) + conj(R(q,p))), and a real
// diagonal entry's is gradE2 Re R(p,p).
// grid (ceil(n/32), ceil(n/32) * rank), block 256 (32 x 8).
__device__ __forceinline__ double2 raw_dB(const Dev& d, const GradDev& g, int Lg, int p, int q, double2 b) {
  const double s = d.scale[Lg], sg = d.sign[Lg];
  double2 r = make_double2(0.0, 0.0);
  const int64_t n = d.n;
  if (p != q) {
    const double c = -2.0 * sg * s * s * g.Wb[(int64_t)p * n + q];
    r = make_double2(c * b.x, c * b.y);
  } else {
    r.x = s * g.dgb[(int64_t)Lg * n + p];
  }
  if (q < d.n_occ && p >= d.n_fc) {
    const double2 v = g.slabb[((int64_t)q * d.n_corr + (p - d.n_fc)) * d.n_l + Lg];
    r = cadd(r, make_double2(s * v.x, s * v.y));
  }
  return r;
}

__device__ __forceinline__ void bdB_body(const Dev& d, const GradDev& g, int t, const uint3 bid) {
  __shared__ double2 tT[32][33];
  const int nt = (d.n + 31) / 32;
  const int L = bid.y / nt;
  const int P0 = (bid.y % nt) * 32, Q0 = bid.x * 32;
  const int Lg = d.sets.l0[t] + L;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const int64_t n = d.n;
  if (d.sets.packed) {
    if (P0 > Q0 + 31) return;                  // tile entirely below the diagonal
    double2* out = g.out_dB[t] + (int64_t)L * fac_stride(d.sets, d.n);
    const double ge = *g.grad_e2;
    for (int k = ty; k < 32; k += 8) {
      const int p = P0 + k, q = Q0 + tx;
      if (p > q || q >= d.n) continue;
      const double2 b = fac_at(d.sets, d.sets.B[t], L, p, q, d.n);
      const double2 a = raw_dB(d, g, Lg, p, q, b);
      double2 v;
      if (p == q) {
        v = make_double2(ge * a.x, 0.0);
      } else {
        const double2 c = raw_dB(d, g, Lg, q, p, make_double2(b.x, -b.y));
        v = make_double2(ge * (a.x + c.x), ge * (a.y - c.y));
      }
      out[tri_off(p, q, d.n)] = v;
    }
    return;
  }
  const double2* B = d.sets.B[t] + (int64_t)L * d.n * d.n;
  double2* out = g.out_dB[t] + (int64_t)L * d.n * d.n;
  // transposed partner: R(q, p) for q in [Q0, Q0+32), p in [P0, P0+32)
  for (int k = ty; k < 32; k += 8) {
    const int q = Q0 + k, p = P0 + tx;
    double2 v = make_double2(0.0, 0.0);
    if (q < d.n && p < d.n) v = raw_dB(d, g, Lg, q, p, B[(int64_t)q * n + p]);
    tT[k][tx] = v;
  }
  __syncthreads();
  const double ge = *g.grad_e2;
  for (int k = ty; k < 32; k += 8) {
    const int p = P0 + k, q = Q0 + tx;
    if (p < d.n && q < d.n) {
      const double2 a = raw_dB(d, g, Lg, p, q, B[(int64_t)p * n + q]);
      const double2 c = tT[tx][k];
      out[(int64_t)p * n + q] = make_double2(0.5 * ge * (a.x + c.x), 0.5 * ge * (a.y - c.y));
    }
  }
}

// dh = gradE2 (hbar + hbar^H) / 2.  grid (ceil(n/256), n).
__device__ __forceinline__ void bdh_body(const Dev& d, const GradDev& g, const uint3 bid) {
  const int q = bid.x * 256 + threadIdx.x;
  const int p = bid.y;
  if (q >= d.n) return;
  const int64_t n = d.n;
  const double2 a = g.hb[(int64_t)p * n + q], c = g.hb[(int64_t)q * n + p];
  const double ge = *g.grad_e2;
  g.out_dh[(int64_t)p * n + q] = make_double2(0.5 * ge * (a.x + c.x), 0.5 * ge * (a.y - c.y));
}

// dC = gradE2 [cbar + Ebar (2/N)(sigma_P - E0 C) - (2 E2 / N) C].  grid (ceil(np/256)).
__device__ __forceinline__ void bdc_body(const Dev& d, const GradDev& g, const uint3 bid) {
  const int i = bid.x * 256 + threadIdx.x;
  if (i >= d.n_p) return;
  const double N = d.scal[1], E0 = d.scal[0];
  const double eb = g.scal[0], e2 = g.scal[1];
  const double2 c = d.c[i], sp = d.sigp[i];
  const double k1 = 2.0 * eb / N, k2 = -2.0 * e2 / N;
  double2 v = g.cb[i];
  v.x += k1 * (sp.x - E0 * c.x) + k2 * c.x;
  v.y += k1 * (sp.y - E0 * c.y) + k2 * c.y;
  const double ge = *g.grad_e2;
  g.out_dc[i] = make_double2(ge * v.x, ge * v.y);
  if (i == 0 && g.out_e2) *g.out_e2 = e2;
}

}  // namespace mrpt2
