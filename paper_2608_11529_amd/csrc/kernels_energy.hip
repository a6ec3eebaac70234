// Reference-space energy, per-string denominator tables, the sigma
// contraction with the Epstein-Nesbet epilogue, and the reductions.
#include <type_traits>

#include "kernels.hpp"
#include "plan.hpp"

namespace mrpt2 {

__device__ __forceinline__ int popc64(uint64_t x) { return __popcll(x); }

// Sign of a_p or a+_p on string s (active bits below p).
__device__ __forceinline__ int below_parity(uint64_t s, int p) { return popc64(s & ((1ull << p) - 1)) & 1; }

// Active-space energy of string al relative to the core energy:
// sum_{t in al} eps_t + sum_{t<u in al} W_tu.
__device__ double act_energy(const Dev& d, uint64_t al) {
  double e = 0.0;
  uint64_t x = al;
  while (x) {
    const int t = __builtin_ctzll(x);
    x &= x - 1;
    const int gt = d.n_fc + d.n_c + t;
    e += d.eps[d.n_c + t];
    uint64_t y = x;
    while (y) {
      const int u = __builtin_ctzll(y);
      y &= y - 1;
      e += d.W[(int64_t)gt * d.n + d.n_fc + d.n_c + u];
    }
  }
  return e;
}

// Element <bi|H|bj> of the reference-space Hamiltonian minus the core
// energy, by the Slater-Condon rules within the active space (core and frozen
// core folded into f).  bi = bra, bj = ket (active strings).
__device__ __forceinline__ double2 hpp_element(const Dev& d, uint64_t bi, uint64_t bj) {
  const uint64_t cre = bi & ~bj, ann = bj & ~bi;
  const int nd = popc64(cre);
  double2 v = make_double2(0.0, 0.0);
  const int nc = d.n_c;
  if (nd == 0) {
    v.x = act_energy(d, bi);
  } else if (nd == 1) {
    const int p = __builtin_ctzll(cre), q = __builtin_ctzll(ann);
    // ket a_q then a+_p
    int par = below_parity(bj, q);
    const uint64_t mid = bj & ~(1ull << q);
    par ^= below_parity(mid, p);
    v = d.f[(int64_t)p * d.n_o + nc + q];
    uint64_t x = mid;
    while (x) {
      const int w = __builtin_ctzll(x);
      x &= x - 1;
      v = cadd(v, csub(Gv(d, nc + q, p, nc + w, w), Gv(d, nc + w, p, nc + q, w)));
    }
    if (par) v = make_double2(-v.x, -v.y);
  } else if (nd == 2) {
    const int q1 = __builtin_ctzll(ann), q2 = 63 - __builtin_clzll(ann);
    const int p1 = __builtin_ctzll(cre), p2 = 63 - __builtin_clzll(cre);
    // ket a_q1, a_q2, a+_p1, a+_p2: value (p2 q1|p1 q2) - (p2 q2|p1 q1)
    uint64_t s = bj;
    int par = below_parity(s, q1);
    s &= ~(1ull << q1);
    par ^= below_parity(s, q2);
    s &= ~(1ull << q2);
    par ^= below_parity(s, p1);
    s |= 1ull << p1;
    par ^= below_parity(s, p2);
    v = csub(Gv(d, nc + q1, p2, nc + q2, p1), Gv(d, nc + q2, p2, nc + q1, p1));
    if (par) v = make_double2(-v.x, -v.y);
  }
  return v;
}

// Dense reference-space Hamiltonian minus the core energy.  Row i = bra,
// column j = ket.  grid (ceil(np/16), ceil(np/16)), block (16, 16).
__device__ __forceinline__ void hpp_body(const Dev& d, double2* __restrict__ out, const uint3 bid) {
  const int j = bid.x * 16 + (threadIdx.x & 15);
  const int i = bid.y * 16 + (threadIdx.x >> 4);
  if (i >= d.n_p || j >= d.n_p) return;
  out[(int64_t)i * d.n_p + j] = hpp_element(d, d.pstrings[i], d.pstrings[j]);
}

// sigma_P = H~ C, one wavefront per row.  grid (np), block 64.
__device__ __forceinline__ void sigp_body(const Dev& d, const uint3 bid) {
  const double2* __restrict__ hpp = d.hpp;
  const int i = bid.x;
  const int lane = threadIdx.x;
  double2 acc = make_double2(0.0, 0.0);
  for (int j = lane; j < d.n_p; j += 64) acc = cfma(hpp[(int64_t)i * d.n_p + j], d.c[j], acc);
  for (int off = 32; off > 0; off >>= 1) {
    acc.x += __shfl_down(acc.x, off, 64);
    acc.y += __shfl_down(acc.y, off, 64);
  }
  if (lane == 0) d.sigp[i] = acc;
}

// E0 - E_core = Re(C^H H~ C) / C^H C and ||C||^2.  One block, fixed order.
__device__ __forceinline__ void e0_body(const Dev& d, int* flag) {
  __shared__ double sn[256], sd[256];
  double num = 0.0, den = 0.0;
  for (int i = threadIdx.x; i < d.n_p; i += 256) {
    const double2 c = d.c[i], s = d.sigp[i];
    num += c.x * s.x + c.y * s.y;
    den += cabs2(c);
  }
  sn[threadIdx.x] = num;
  sd[threadIdx.x] = den;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      sn[threadIdx.x] += sn[threadIdx.x + o];
      sd[threadIdx.x] += sd[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double e0 = sn[0] / sd[0];
    if (!isfinite(e0) || !(sd[0] > 0.0)) *flag = 1;
    d.scal[0] = e0;
    d.scal[1] = sd[0];
  }
}

// T[s] = (E0 - E_core) - E_act(alpha_s); Uc[s][c] = sum_{t in alpha_s} W_ct;
// Uv[s][a] = sum_{t in alpha_s} W_at.  grid (S, ceil(max(n_c, n_v)/256)).
__device__ __forceinline__ void class_tables_body(const Dev& d, const ClassDev& cd, const uint3 bid) {
  const int64_t s = bid.x;
  const uint64_t al = cd.strings[s];
  const int p = bid.y * 256 + threadIdx.x;
  if (bid.y == 0 && threadIdx.x == 0) cd.T[s] = d.scal[0] - act_energy(d, al);
  const int ga = d.n_fc + d.n_c;   // first active global index
  if (cd.h > 0 && p < d.n_c) {
    double u = 0.0;
    uint64_t x = al;
    while (x) {
      const int t = __builtin_ctzll(x);
      x &= x - 1;
      u += d.W[(int64_t)(d.n_fc + p) * d.n + ga + t];
    }
    cd.Uc[s * d.n_c + p] = u;
  }
  if (cd.v > 0 && p < d.n_v) {
    double u = 0.0;
    uint64_t x = al;
    while (x) {
      const int t = __builtin_ctzll(x);
      x &= x - 1;
      u += d.W[(int64_t)(d.n_fc + d.n_o + p) * d.n + ga + t];
    }
    cd.Uv[s * d.n_v + p] = u;
  }
}

// Row r of a class with v <= 1: holes index * n_v^v + virtual.
__device__ __forceinline__ void decode_small_row(const Dev& d, const ClassDev& cd, int64_t r, int* c0,
                                                 int* c1, int* a) {
  int64_t hi = r;
  *a = -1;
  if (cd.v == 1) {
    *a = (int)(r % d.n_v);
    hi = r / d.n_v;
  }
  *c0 = -1;
  *c1 = -1;
  if (cd.h == 1) *c0 = (int)hi;
  if (cd.h == 2) {
    *c0 = d.hole_pairs[2 * hi];
    *c1 = d.hole_pairs[2 * hi + 1];
  }
}

// Coupling integrals of the classes with at most one virtual electron, per
// pattern and row; the operator order of the plan fixes the integral slots:
// rank-2 K = a+_p a+_r a_s a_q L gives (pq|rs) - (ps|rq) with q, s the
// annihilations in order (core first) and r, p the creations in order
// (active first, virtual last); rank-1 K = a+_p a_q L gives f_pq (one-body
// pattern) or (pq|ww) - (pw|wq) (spectator w).  G(x;p;y;q) = (px|qy).
// grid (ceil(rows/256), n_pat).
__device__ __forceinline__ void xbuild_body(const Dev& d, const ClassDev& cd, const uint3 bid) {
  const int64_t r = bid.x * 256ll + threadIdx.x;
  const int j = bid.y;
  if (r >= cd.n_rows) return;
  int c0, c1, a;
  decode_small_row(d, cd, r, &c0, &c1, &a);
  const Pattern pt = cd.pat[j];
  const int nc = d.n_c, na = d.n_a;
  double2 x = make_double2(0.0, 0.0);
  // q = first annihilation (occupied index), p = last creation (act/virt row)
  if (pt.kind == PAT_SINGLE) {
    const int qo = (cd.h == 1) ? c0 : nc + pt.a0;
    const int pr = (cd.v == 1) ? na + a : pt.r0;
    x = d.f[(int64_t)pr * d.n_o + qo];
  } else if (pt.kind == PAT_SPECT) {
    const int qo = (cd.h == 1) ? c0 : nc + pt.a0;
    const int pr = (cd.v == 1) ? na + a : pt.r0;
    const int w = pt.w;
    x = csub(Gv(d, qo, pr, nc + w, w), Gv(d, nc + w, pr, qo, w));
  } else {
    // annihilations in order
    int q, s;
    if (cd.h == 2) { q = c0; s = c1; }
    else if (cd.h == 1) { q = c0; s = nc + pt.a0; }
    else { q = nc + pt.a0; s = nc + pt.a1; }
    // creations in order: active ascending then virtual; r first, p last
    int rr, pr;
    if (cd.v == 1) { rr = pt.r0; pr = na + a; }
    else { rr = pt.r0; pr = pt.r1; }
    x = csub(Gv(d, q, pr, s, rr), Gv(d, s, pr, q, rr));
  }
  cd.X[(int64_t)j * cd.n_rows + r] = x;
}

constexpr int SIG_THREADS = 256;

// Sigma contraction and Epstein-Nesbet epilogue for one class:
//   sigma[r, s] = sum_{(beta, j, sign) in list(s)} sign C_beta X[j, r]
//   Delta = (E0 - E_core) - (H_KK - E_core)
//         = T[s] + sum_{c in holes} (eps_c + Uc[s][c]) - sum_{a in virt} (eps_a + Uv[s][a])
//           - W_cc' - W_ab + sum_{c, a} W_ca
//   partial += |sigma|^2 g(Delta)   (divided by ||C||^2 at the end)
// with g = 1/Delta, or its level-shifted form (en_weight).
// One thread per row, a chunk of strings per block.  grid (rb * nsc).
template <int H, int V>
__device__ __forceinline__ void sigma_body(const Dev& d, const ClassDev& cd, int* flag, const uint3 bid) {
  __shared__ double red[SIG_THREADS];
  const int64_t rb = bid.x / cd.nsc;
  const int sc = bid.x % cd.nsc;
  const int64_t chunk = (cd.n_str + cd.nsc - 1) / cd.nsc;
  const int64_t s_lo = sc * chunk;
  const int64_t s_hi = min(cd.n_str, s_lo + chunk);
  int64_t r = rb * SIG_THREADS + threadIdx.x;
  bool valid = r < cd.n_rows;
  if (!valid) r = cd.n_rows - 1;
  int c0 = -1, c1 = -1, a = -1, b = -1;
  int64_t rab = 0, hole = 0;
  const int nc = d.n_c;
  if (V == 2) {
    const int64_t per = d.n_tp * 4096;
    hole = r / per;
    rab = r % per;
    const int64_t tp = rab >> 12;
    const int la = (int)((rab >> 6) & 63), lb = (int)(rab & 63);
    a = d.tile_pairs[2 * tp] * 64 + la;
    b = d.tile_pairs[2 * tp + 1] * 64 + lb;
    if (!(a < b && b < d.n_v)) {
      valid = false;            // padding or lower triangle: keep table reads in range
      a = 0;
      b = d.n_v > 1 ? 1 : 0;
    }
    if (H == 1) c0 = (int)hole;
    if (H == 2) {
      c0 = d.hole_pairs[2 * hole];
      c1 = d.hole_pairs[2 * hole + 1];
    }
  } else {
    decode_small_row(d, cd, r, &c0, &c1, &a);
  }
  // row constant
  double qr = 0.0;
  const int gfc = d.n_fc, gv = d.n_fc + d.n_o;
  if (H >= 1) qr += d.eps[c0];
  if (H == 2) qr += d.eps[c1] - d.W[(int64_t)(gfc + c0) * d.n + gfc + c1];
  if (V >= 1) qr -= d.eps[d.n_o + a];
  if (V == 2) qr -= d.eps[d.n_o + b] + d.W[(int64_t)(gv + a) * d.n + gv + b];
  if (H >= 1 && V >= 1) {
    qr += d.W[(int64_t)(gfc + c0) * d.n + gv + a];
    if (V == 2) qr += d.W[(int64_t)(gfc + c0) * d.n + gv + b];
    if (H == 2) {
      qr += d.W[(int64_t)(gfc + c1) * d.n + gv + a];
      if (V == 2) qr += d.W[(int64_t)(gfc + c1) * d.n + gv + b];
    }
  }
  double acc = 0.0;
  bool bad = false;
  const double b2 = d.ls_b2;
  for (int64_t s = s_lo; s < s_hi; ++s) {
    const int e0 = cd.conn_ptr[s], e1 = cd.conn_ptr[s + 1];
    double2 sig = make_double2(0.0, 0.0);
    for (int e = e0; e < e1; ++e) {
      const int32_t cb = cd.conn[2 * e];
      const int j = cd.conn[2 * e + 1];
      double2 cv = d.c[cb & 0x7fffffff];
      if (cb < 0) cv = make_double2(-cv.x, -cv.y);
      double2 xv;
      if (V == 2) {
        const Pattern pt = cd.pat[j];
        int64_t pair;
        if (H == 2) pair = occ_pair(c0, c1, d.n_o);
        else if (H == 1) pair = occ_pair(c0, nc + pt.a0, d.n_o);
        else pair = occ_pair(nc + pt.a0, nc + pt.a1, d.n_o);
        xv = d.A[pair * d.n_tp * 4096 + rab];
      } else {
        xv = cd.X[(int64_t)j * cd.n_rows + r];
      }
      sig = cfma(cv, xv, sig);
    }
    double del = cd.T[s] + qr;
    if (H >= 1) del += cd.Uc[s * nc + c0];
    if (H == 2) del += cd.Uc[s * nc + c1];
    if (V >= 1) del -= cd.Uv[s * d.n_v + a];
    if (V == 2) del -= cd.Uv[s * d.n_v + b];
    if (e1 > e0) {
      const double t = cabs2(sig) * en_weight(del, b2);
      if (valid) {
        // an exactly vanishing denominator leaves eq. pt2en undefined; under
        // the level shift the weight Delta^3/(Delta^4 + b^2) is 0 there
        if ((b2 == 0.0 && !(del != 0.0)) || !isfinite(t)) bad = true;
        acc += t;
      }
    }
  }
  if (bad) *flag = 2;
  red[threadIdx.x] = valid ? acc : 0.0;
  __syncthreads();
  for (int o = SIG_THREADS / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) cd.part[bid.x] = red[0];
}


// Class (2,2): K = core - {c, c'} + alpha + {a, b}, alpha in P.  Its only
// connected reference determinant is core + alpha, so
//   sigma_K = <ab||cc'> C_alpha  and  |sigma_K|^2 = |<ab||cc'>|^2 |C_alpha|^2,
// and the class is a sum over (c<c', a<b) of |<ab||cc'>|^2 times
// S_ab = sum_alpha |C_alpha|^2 / Delta(a, b, alpha), with
//   Delta = G(alpha) + Y_a(alpha) + Y_b(alpha) - W_ab,
//   G = T(alpha) + eps_c + Uc_c(alpha) + eps_c' + Uc_c'(alpha) - W_cc',
//   Y_a = -eps_a - Uv_a(alpha) + W_ca + W_c'a.
// Pure FP64 vector work: each thread owns a 4 x 4 block of (a, b) of a
// 64 x 64 tile and walks alpha four at a time, merging the four fractions
// c1/d1 + ... + c4/d4 into one numerator and denominator (pairwise products)
// so that a single reciprocal serves four determinants.  Merging four rather
// than eight keeps the kernel within 168 VGPRs and, with 32-string LDS
// chunks, at three waves per SIMD, which outweighs the extra reciprocals.
// grid (C(n_c, 2), n_tp), block 256.
constexpr int AC22 = 64;            // strings per LDS chunk of the (2,2) adjoint kernels
constexpr int E22C = 32;            // strings per LDS chunk of e22 (36 KB: three blocks per CU)

// LS: the imaginary level shift of Sec. 2.6, each fraction cw/Delta becoming
// cw Delta^3 / (Delta^4 + b^2) before the merge (padding strings then take a
// moderate denominator so that the merged products stay finite).
template <bool LS>
__device__ __forceinline__ void e22_body(const Dev& d, const ClassDev& cd, int* flag, const uint3 bid) {
  __shared__ double sYa[E22C][64];
  __shared__ double sYb[E22C][64];
  __shared__ double sG[E22C];
  __shared__ double sCw[E22C];
  __shared__ double ya0[64], yb0[64];
  __shared__ double red[256];
  const int hp = bid.x, tp = bid.y;   // core pairs fastest: blocks of one tile pair share its tables in L2
  const int c0 = d.hole_pairs[2 * hp], c1 = d.hole_pairs[2 * hp + 1];
  const int I = d.tile_pairs[2 * tp], J = d.tile_pairs[2 * tp + 1];
  const int tid = threadIdx.x, ta = tid & 15, tb = tid >> 4;
  const int nv = d.n_v, nc = d.n_c;
  const int64_t gfc = d.n_fc, gv = d.n_fc + d.n_o;
  const double* __restrict__ W = d.W;
  if (tid < 64) {
    const int a = I * 64 + tid;
    ya0[tid] = (a < nv) ? -d.eps[d.n_o + a] + W[(gfc + c0) * d.n + gv + a] + W[(gfc + c1) * d.n + gv + a] : -1.0;
  } else if (tid < 128) {
    const int b = J * 64 + tid - 64;
    yb0[tid - 64] = (b < nv) ? -d.eps[d.n_o + b] + W[(gfc + c0) * d.n + gv + b] + W[(gfc + c1) * d.n + gv + b] : -1.0;
  }
  const double gconst = d.eps[c0] + d.eps[c1] - W[(gfc + c0) * d.n + gfc + c1];
  double wab[4][4], acc[4][4];
  bool ok[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int a = I * 64 + ta + 16 * i, b = J * 64 + tb + 16 * j;
      ok[i][j] = (a < b) && (b < nv);
      wab[i][j] = ok[i][j] ? W[(gv + a) * d.n + gv + b] : 0.0;
      acc[i][j] = 0.0;
    }
  const int np = d.n_p;
  const double* __restrict__ Uv = cd.Uv;
  const double* __restrict__ Uc = cd.Uc;
  const double lsb2 = d.ls_b2;
  (void)lsb2;
  for (int a0 = 0; a0 < np; a0 += E22C) {
    __syncthreads();
    for (int e = tid; e < E22C * 64; e += 256) {
      const int al = e >> 6, l = e & 63;
      const int s = a0 + al;
      const int a = I * 64 + l, b = J * 64 + l;
      double ya = ya0[l], yb = yb0[l];
      if (s < np) {
        if (a < nv) ya -= Uv[(int64_t)s * nv + a];
        if (b < nv) yb -= Uv[(int64_t)s * nv + b];
      }
      sYa[al][l] = ya;
      sYb[al][l] = yb;
    }
    if (tid < E22C) {
      const int s = a0 + tid;
      if (s < np) {
        sG[tid] = cd.T[s] + Uc[(int64_t)s * nc + c0] + Uc[(int64_t)s * nc + c1] + gconst;
        sCw[tid] = cabs2(d.c[s]);
      } else {
        sG[tid] = LS ? 1e6 : 1e30;   // padding: vanishing weight, harmless denominator
        sCw[tid] = 0.0;
      }
    }
    __syncthreads();
#pragma unroll 1
    for (int al = 0; al < E22C; al += 4) {
      double g[4], cw[4], za[4][4], yb[4][4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        g[k] = sG[al + k];
        cw[k] = sCw[al + k];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int k = 0; k < 4; ++k) za[i][k] = g[k] + sYa[al + k][ta + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int k = 0; k < 4; ++k) yb[j][k] = sYb[al + k][tb + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          // sum_k cw_k / d_k over four strings as one fraction: pairwise
          // numerators and denominators, one reciprocal
          double n2[2], q2[2];
#pragma unroll
          for (int k = 0; k < 2; ++k) {
            const double da = (za[i][2 * k] + yb[j][2 * k]) - wab[i][j];
            const double db = (za[i][2 * k + 1] + yb[j][2 * k + 1]) - wab[i][j];
            if constexpr (LS) {
              const double a2 = da * da, b2 = db * db;
              const double qa = fma(a2, a2, lsb2), qb = fma(b2, b2, lsb2);
              n2[k] = fma(cw[2 * k] * da * a2, qb, cw[2 * k + 1] * db * b2 * qa);
              q2[k] = qa * qb;
            } else {
              n2[k] = fma(cw[2 * k], db, cw[2 * k + 1] * da);
              q2[k] = da * db;
            }
          }
          const double num = fma(n2[0], q2[1], n2[1] * q2[0]);
          acc[i][j] = fma(num, rcp_nr(q2[0] * q2[1]), acc[i][j]);
        }
    }
  }
  // weights |<ab||cc'>|^2 from the pair-integral tile
  const double2* Ablk = d.A + ((int64_t)occ_pair(c0, c1, d.n_o) * d.n_tp + tp) * 4096;
  double sum = 0.0;
  bool bad = false;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (ok[i][j]) {
        const double t = cabs2(Ablk[(ta + 16 * i) * 64 + tb + 16 * j]) * acc[i][j];
        if (!isfinite(t)) bad = true;
        sum += t;
      }
    }
  if (bad) *flag = 2;
  red[tid] = sum;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (tid < o) red[tid] += red[tid + o];
    __syncthreads();
  }
  if (tid == 0) cd.part[(int64_t)hp * d.n_tp + tp] = red[0];
}

// Dense coefficients of a class with few patterns: D[s][j] = sum of sign C_beta
// over the excitation list of string s with pattern j, and the bit mask of the
// patterns present.  grid (ceil(S / 256)).
__device__ __forceinline__ void dense_coef_body(const Dev& d, const ClassDev& cd, const uint3 bid) {
  const int64_t s = bid.x * 256ll + threadIdx.x;
  if (s >= cd.n_str) return;
  const int J = cd.n_pat;
  double2* row = cd.D + s * J;
  for (int j = 0; j < J; ++j) row[j] = make_double2(0.0, 0.0);
  uint32_t m = 0;
  for (int e = cd.conn_ptr[s]; e < cd.conn_ptr[s + 1]; ++e) {
    const int32_t cb = cd.conn[2 * e];
    const int j = cd.conn[2 * e + 1];
    double2 cv = d.c[cb & 0x7fffffff];
    if (cb < 0) cv = make_double2(-cv.x, -cv.y);
    row[j] = cadd(row[j], cv);
    m |= 1u << j;
  }
  cd.mask[s] = m;
}

// Class (1,2): K = core - {c} + alpha' + {a, b}, reached from
// L = core + alpha' + {t} by a_c a_t -> a+_b a+_a:
//   sigma_K = sum_t <ab||ct> D[alpha'][t],
//   Delta   = T + eps_c + Uc_c - eps_a - Uv_a - eps_b - Uv_b - W_ab + W_ca + W_cb.
// Each thread owns two (a, b) of a 16 x 32 region of a 64 x 64 virtual tile
// pair (b and b + 16), the couplings <ab||ct> of both in registers; strings
// are walked in chunks staged in LDS, patterns present in a string selected
// by a wave-uniform mask, and four fractions |sigma|^2 / Delta merged per
// reciprocal.  Every coefficient read from LDS feeds both pairs, which halves
// the LDS traffic per determinant (the LDS read bandwidth, not the FP64
// arithmetic, limited the one-pair form).  Partial sums stay per 16 x 16
// sub-tile.  grid (n_c, 8 n_tp), block 256.
// F32 (mixed form): the couplings and coefficients are rounded to FP32 and
// sigma is summed in FP32 (a few terms per determinant; the mixed form's
// pair integrals carry FP32 rounding already), which halves the LDS bytes of
// every coefficient read; |sigma|^2, the denominators and the sums stay FP64.
constexpr int SC12 = 64;

__device__ __forceinline__ float2 cfma(float2 a, float2 b, float2 c) {
  return make_float2(fmaf(a.x, b.x, fmaf(-a.y, b.y, c.x)), fmaf(a.x, b.y, fmaf(a.y, b.x, c.y)));
}
__device__ __forceinline__ double cabs2_64(double2 a) { return cabs2(a); }
__device__ __forceinline__ double cabs2_64(float2 a) {
  const double x = a.x, y = a.y;
  return fma(x, x, y * y);
}
template <class CV>
__device__ __forceinline__ CV to_cv(double2 v) {
  if constexpr (sizeof(CV) == 8) return make_float2((float)v.x, (float)v.y);
  else return v;
}

// sigma of four strings for the two (a, b) of a thread, pattern j = J0 and
// every later pattern present in the group's mask um; the coefficient of
// (string k, pattern j) is entry e = k MJ + j of the group's 4 MJ staged
// coefficients, held by lane e mod 16 of every row in C[e / 16].  The
// products run in the order of cfma (same rounding).
template <int MJ, int J0, int K>
__device__ __forceinline__ void e12_row_k(const double2 (&C)[MJ / 4], const double2 (&X)[2][MJ],
                                          double2 (&sg)[2][4]) {
  constexpr int E = K * MJ + J0, M = E >> 4, L = E & 15;
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    fmac_row<L, true>(sg[p][K].x, C[M].y, X[p][J0].y);
    fmac_row<L, false>(sg[p][K].x, C[M].x, X[p][J0].x);
    fmac_row<L, false>(sg[p][K].y, C[M].y, X[p][J0].x);
    fmac_row<L, false>(sg[p][K].y, C[M].x, X[p][J0].y);
  }
  if constexpr (K + 1 < 4) e12_row_k<MJ, J0, K + 1>(C, X, sg);
}
template <int MJ, int J0>
__device__ __forceinline__ void e12_row_fmas(uint32_t um, const double2 (&C)[MJ / 4], const double2 (&X)[2][MJ],
                                             double2 (&sg)[2][4]) {
  if (um & (1u << J0)) e12_row_k<MJ, J0, 0>(C, X, sg);
  if constexpr (J0 + 1 < MJ) e12_row_fmas<MJ, J0 + 1>(um, C, X, sg);
}

template <int MJ, bool LS, bool F32 = false>
__device__ __forceinline__ void e12_body(const Dev& d, const ClassDev& cd, int* flag, const uint3 bid) {
  typedef typename std::conditional<F32, float2, double2>::type CV;
  __shared__ double sUa[SC12][16];
  __shared__ double sUb[SC12][32];
  __shared__ double sG[SC12];
  __shared__ CV sD[SC12][MJ];
  __shared__ uint32_t sM[SC12];
  __shared__ double red[2][256];
  const int tps = bid.y;                    // cores fastest: blocks of one region share its tables
  const int tp = tps >> 3, reg = tps & 7;
  const int sa = reg >> 1, sb2 = reg & 1;   // 16-row band sa, 32-column band sb2
  const int c = bid.x;
  const int I = d.tile_pairs[2 * tp], Jt = d.tile_pairs[2 * tp + 1];
  const int64_t pbase = (int64_t)c * d.n_tp * 16 + (int64_t)tp * 16 + sa * 4 + 2 * sb2;
  if (I == Jt && sa > 2 * sb2 + 1) {        // both sub-tiles entirely below the diagonal
    if (threadIdx.x < 2) cd.part[pbase + threadIdx.x] = 0.0;
    return;
  }
  const int tid = threadIdx.x;
  const int la = sa * 16 + (tid >> 4);
  const int nv = d.n_v, nc = d.n_c;
  const int J = cd.n_pat;
  const int64_t gfc = d.n_fc, gv = d.n_fc + d.n_o;
  const double* __restrict__ W = d.W;
  const int a0 = I * 64 + la;
  const int a = a0 < nv ? a0 : 0;
  int lb[2];
  bool valid[2];
  double rowc[2];
  CV X[2][MJ];
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    lb[p] = sb2 * 32 + 16 * p + (tid & 15);
    int b = Jt * 64 + lb[p];
    valid[p] = (a0 < b) && (b < nv);
    if (!valid[p]) b = nv > 1 ? 1 : 0;
    const int aa = valid[p] ? a : 0;
    rowc[p] = -d.eps[d.n_o + aa] - d.eps[d.n_o + b] - W[(gv + aa) * d.n + gv + b] + W[(gfc + c) * d.n + gv + aa] +
              W[(gfc + c) * d.n + gv + b];
#pragma unroll
    for (int j = 0; j < MJ; ++j) {
      X[p][j] = to_cv<CV>(make_double2(0.0, 0.0));
      if (j < J) {
        const int64_t pr = occ_pair(c, nc + cd.pat[j].a0, d.n_o);
        X[p][j] = to_cv<CV>(d.A[(pr * d.n_tp + tp) * 4096 + la * 64 + lb[p]]);
      }
    }
  }
  const double epsc = d.eps[c];
  const int64_t S = cd.n_str;
  const double lsb2 = d.ls_b2;
  (void)lsb2;
  double acc[2] = {0.0, 0.0};
  const int ia = tid >> 4, ib = tid & 15;
  for (int64_t s0 = 0; s0 < S; s0 += SC12) {
    __syncthreads();
    for (int e = tid; e < SC12 * 16; e += 256) {
      const int sl = e >> 4, l = e & 15;
      const int64_t s = s0 + sl;
      const int aa = I * 64 + sa * 16 + l;
      sUa[sl][l] = (s < S && aa < nv) ? cd.Uv[s * nv + aa] : 0.0;
    }
    for (int e = tid; e < SC12 * 32; e += 256) {
      const int sl = e >> 5, l = e & 31;
      const int64_t s = s0 + sl;
      const int bb = Jt * 64 + sb2 * 32 + l;
      sUb[sl][l] = (s < S && bb < nv) ? cd.Uv[s * nv + bb] : 0.0;
    }
    for (int e = tid; e < SC12 * MJ; e += 256) {
      const int sl = e / MJ, j = e % MJ;
      const int64_t s = s0 + sl;
      sD[sl][j] = to_cv<CV>((s < S && j < J) ? cd.D[s * J + j] : make_double2(0.0, 0.0));
    }
    if (tid < SC12) {
      const int64_t s = s0 + tid;
      sG[tid] = (s < S) ? cd.T[s] + cd.Uc[s * nc + c] + epsc : (LS ? 1e6 : 1e30);
      sM[tid] = (s < S) ? cd.mask[s] : 0u;
    }
    __syncthreads();
#pragma unroll 1
    for (int sl = 0; sl < SC12; sl += 4) {
      CV sg[2][4];
      // strings are ordered by pattern mask, so the union of four masks is
      // usually a single mask; absent couplings carry zero coefficients
      const uint32_t um = sM[sl] | sM[sl + 1] | sM[sl + 2] | sM[sl + 3];
#pragma unroll
      for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int k = 0; k < 4; ++k) sg[p][k] = to_cv<CV>(make_double2(0.0, 0.0));
      if constexpr (F32) {
#pragma unroll
        for (int j = 0; j < MJ; ++j)
          if (um & (1u << j)) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
              const CV dv = sD[sl + k][j];
              sg[0][k] = cfma(dv, X[0][j], sg[0][k]);
              sg[1][k] = cfma(dv, X[1][j], sg[1][k]);
            }
          }
      } else {
        // the group's 4 MJ coefficients are contiguous in sD: lane l of each
        // row loads entries l, l + 16, ... (MJ is a multiple of 4)
        static_assert(MJ % 4 == 0, "pattern slots in multiples of four");
        const double2* cg = &sD[sl][0];
        double2 C[MJ / 4];
#pragma unroll
        for (int m = 0; m < MJ / 4; ++m) C[m] = cg[(tid & 15) + 16 * m];
        e12_row_fmas<MJ, 0>(um, C, X, sg);
      }
      double g4[4], ua[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        g4[k] = sG[sl + k];
        ua[k] = sUa[sl + k][ia];
      }
#pragma unroll
      for (int p = 0; p < 2; ++p) {
        double w[4], dd[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          w[k] = cabs2_64(sg[p][k]);
          dd[k] = (g4[k] + rowc[p]) - ua[k] - sUb[sl + k][ib + 16 * p];
          if constexpr (LS) {
            const double d2 = dd[k] * dd[k];
            w[k] *= dd[k] * d2;
            dd[k] = fma(d2, d2, lsb2);
          }
        }
        const double n01 = fma(w[0], dd[1], w[1] * dd[0]);
        const double q01 = dd[0] * dd[1];
        const double n23 = fma(w[2], dd[3], w[3] * dd[2]);
        const double q23 = dd[2] * dd[3];
        acc[p] = fma(fma(n01, q23, n23 * q01), rcp_nr(q01 * q23), acc[p]);
      }
    }
  }
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    if (valid[p] && !isfinite(acc[p])) *flag = 2;
    red[p][tid] = valid[p] ? acc[p] : 0.0;
  }
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (tid < o) {
      red[0][tid] += red[0][tid + o];
      red[1][tid] += red[1][tid + o];
    }
    __syncthreads();
  }
  if (tid < 2) cd.part[pbase + tid] = red[tid][0];
}


// Class (2,1): K = core - {c, c'} + alpha + {a}, reached from
// L = core + alpha - {u} by a_c a_c' -> a+_a a+_u:
//   sigma_K = sum_u X[u][(c c', a)] D[alpha][u]   (X = <au||cc'>, xbuild),
//   Delta   = T + eps_c + Uc_c + eps_c' + Uc_c' - W_cc' - eps_a - Uv_a + W_ca + W_c'a.
// One thread per (core pair, a) with the couplings of its row in registers;
// strings walked in chunks staged in LDS, the patterns present in four
// strings selected by a wave-uniform mask (strings ordered by pattern mask),
// four fractions merged per reciprocal.  The generic kernel read every
// coupling of every determinant from memory.  grid (C(n_c, 2), ceil(n_v / 256)),
// block 256: core pairs fastest, so that the blocks sharing a range of
// virtual spinors (the same string-table columns) run together.
constexpr int SC21 = 16;

template <int MJ, bool LS>
__device__ __forceinline__ void e21_body(const Dev& d, const ClassDev& cd, int* flag, const uint3 bid) {
  __shared__ double sUv[SC21][256];
  __shared__ double2 sD[SC21][MJ];
  __shared__ double sG[SC21];
  __shared__ uint32_t sM[SC21];
  __shared__ double red[256];
  const int hp = bid.x, at = bid.y;
  const int c0 = d.hole_pairs[2 * hp], c1 = d.hole_pairs[2 * hp + 1];
  const int tid = threadIdx.x;
  const int nv = d.n_v, nc = d.n_c;
  const int a0 = at * 256 + tid;
  const bool valid = a0 < nv;
  const int a = valid ? a0 : 0;
  const int64_t r = (int64_t)hp * nv + a;
  const int J = cd.n_pat;
  const int64_t gfc = d.n_fc, gv = d.n_fc + d.n_o;
  const double* __restrict__ W = d.W;
  const double rowc = -d.eps[d.n_o + a] + W[(gfc + c0) * d.n + gv + a] + W[(gfc + c1) * d.n + gv + a];
  const double gconst = d.eps[c0] + d.eps[c1] - W[(gfc + c0) * d.n + gfc + c1];
  double2 X[MJ];
#pragma unroll
  for (int j = 0; j < MJ; ++j) X[j] = (j < J) ? cd.X[(int64_t)j * cd.n_rows + r] : make_double2(0.0, 0.0);
  const int64_t S = cd.n_str;
  const double lsb2 = d.ls_b2;
  (void)lsb2;
  double acc = 0.0;
  for (int64_t s0 = 0; s0 < S; s0 += SC21) {
    __syncthreads();
    for (int e = tid; e < SC21 * 256; e += 256) {
      const int sl = e >> 8, l = e & 255;
      const int64_t s = s0 + sl;
      const int aa = at * 256 + l;
      sUv[sl][l] = (s < S && aa < nv) ? cd.Uv[s * nv + aa] : 0.0;
    }
    for (int e = tid; e < SC21 * MJ; e += 256) {
      const int sl = e / MJ, j = e % MJ;
      const int64_t s = s0 + sl;
      sD[sl][j] = (s < S && j < J) ? cd.D[s * J + j] : make_double2(0.0, 0.0);
    }
    if (tid < SC21) {
      const int64_t s = s0 + tid;
      sG[tid] = (s < S) ? cd.T[s] + cd.Uc[s * nc + c0] + cd.Uc[s * nc + c1] + gconst : (LS ? 1e6 : 1e30);
      sM[tid] = (s < S) ? cd.mask[s] : 0u;
    }
    __syncthreads();
#pragma unroll 1
    for (int sl = 0; sl < SC21; sl += 4) {
      double2 sg[4];
      const uint32_t um = sM[sl] | sM[sl + 1] | sM[sl + 2] | sM[sl + 3];
#pragma unroll
      for (int k = 0; k < 4; ++k) sg[k] = make_double2(0.0, 0.0);
      // the group's 4 MJ coefficients, contiguous in sD: lane l of each row
      // loads entries l, l + 16, ..., the products take them by row broadcast
      double2 C[MJ / 4];
      {
        const double2* cg = &sD[sl][0];
#pragma unroll
        for (int m = 0; m < MJ / 4; ++m) C[m] = cg[(tid & 15) + 16 * m];
      }
      row_sig<MJ, 4, 0>(um, C, X, sg);
      double w[4], dd[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        w[k] = cabs2(sg[k]);
        dd[k] = (sG[sl + k] + rowc) - sUv[sl + k][tid];
        if constexpr (LS) {
          const double d2 = dd[k] * dd[k];
          w[k] *= dd[k] * d2;
          dd[k] = fma(d2, d2, lsb2);
        }
      }
      const double n01 = fma(w[0], dd[1], w[1] * dd[0]);
      const double q01 = dd[0] * dd[1];
      const double n23 = fma(w[2], dd[3], w[3] * dd[2]);
      const double q23 = dd[2] * dd[3];
      acc = fma(fma(n01, q23, n23 * q01), rcp_nr(q01 * q23), acc);
    }
  }
  if (valid && !isfinite(acc)) *flag = 2;
  red[tid] = valid ? acc : 0.0;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (tid < o) red[tid] += red[tid + o];
    __syncthreads();
  }
  if (tid == 0) cd.part[(int64_t)at * cd.n_holes + hp] = red[0];
}


// Class (0,2): K = core + alpha'' + {a, b}, reached from
// L = core + alpha'' + {t, w} by a_t a_w -> a+_b a+_a:
//   sigma_K = sum_{t<w} <ab||tw> sign C_L,
//   Delta   = T - eps_a - Uv_a - eps_b - Uv_b - W_ab.
// The strings come in tiles of at most 64 of one occupation category (plan
// order); a tile's coefficients sign C_L form a dense block Md[s][col] over
// the tile's support columns (its strings' active pairs), so that sigma over
// a tile and 64 virtual pairs is one complex GEMM with K = support size.

// Dense coefficient blocks, one thread per tile row.  grid (n_tiles), block 64.
__device__ __forceinline__ void e02coef_body(const Dev& d, const ClassDev& cd, const uint3 bid) {
  const int64_t t = bid.x;
  const int r = threadIdx.x;
  const int s0 = cd.tile_s0[t], s1 = cd.tile_s0[t + 1];
  const int k0 = cd.tile_k0[t], K = cd.tile_k0[t + 1] - k0;
  double2* row = cd.Md + (int64_t)64 * k0 + (int64_t)r * K;
  for (int k = 0; k < K; ++k) row[k] = make_double2(0.0, 0.0);
  const int s = s0 + r;
  if (s >= s1) return;
  for (int e = cd.conn_ptr[s]; e < cd.conn_ptr[s + 1]; ++e) {
    const int32_t cb = cd.conn[2 * e];
    double2 cv = d.c[cb & 0x7fffffff];
    if (cb < 0) cv = make_double2(-cv.x, -cv.y);
    const int k = cd.ccol[e];
    row[k] = make_double2(row[k].x + cv.x, row[k].y + cv.y);
  }
}

// sigma for (tile, virtual a, 64 virtual b of a tile pair) on FP64 MFMA, then
// |sigma|^2 / Delta summed over the valid (string, a < b) entries, four
// fractions per reciprocal.  grid (n_tiles, 64 n_tp): tiles fastest, so that
// the blocks sharing one row of pair integrals run together.  block 256.
// F32 (mixed form): the contraction on FP32 MFMA with FP64 accumulation per
// 32-term stage; denominators and sums stay FP64.
template <bool F32, bool LS>
__device__ __forceinline__ void e02_body(const Dev& d, const ClassDev& cd, int* flag, const uint3 bid) {
  // float2 slots of each staging buffer (the FP64 A operand is staged as
  // (re, im, -im, re))
  constexpr int SHA = F32 ? 64 * KP32 : 4 * 64 * KP, SHB = F32 ? 64 * KP32 : 2 * 64 * KP;
  __shared__ __align__(32) float2 sA[SHA];
  __shared__ __align__(32) float2 sB[SHB];
  __shared__ double red[256];
  const int64_t t = bid.x;
  const int64_t tp = bid.y >> 6;
  const int la = (int)(bid.y & 63);
  const int64_t blk = (int64_t)bid.y * cd.n_tiles + t;
  const int I = d.tile_pairs[2 * tp], Jt = d.tile_pairs[2 * tp + 1];
  const int nv = d.n_v;
  const int a = I * 64 + la;
  if (a + 1 >= nv || a >= Jt * 64 + 63) {      // no valid (a, b) in this block
    if (threadIdx.x == 0) cd.part[blk] = 0.0;
    return;
  }
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
  double accR[2][2][4], accI[2][2][4];
  if constexpr (F32) {
    cgemm64_f32c(fa, fb, K, sA, sB, accR, accI);
  } else {
    d4 aR[2][2], aI[2][2];
    cgemm64<true>(fa, fb, K, (double4*)sA, (double2*)sB, aR, aI);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          accR[i][j][r] = aR[i][j][r];
          accI[i][j][r] = aI[i][j][r];
        }
  }
  auto arow = [](int i, int r) { return F32 ? acc_row_f32(i, r) : acc_row(i, r); };
  const int64_t gv = d.n_fc + d.n_o;
  const double ea = d.eps[d.n_o + a];
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
  double acc = 0.0;
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    double Ts[4], ua[4];
    bool sok[4];
    int64_t so[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int s = s0 + arow(i, r);
      sok[r] = s < s1;
      const int sv = sok[r] ? s : s0;
      so[r] = (int64_t)sv * nv;
      Ts[r] = cd.T[sv];
      ua[r] = cd.Uv[so[r] + a];
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      double w[4], dd[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const bool ok = sok[r] && bok[j];
        const double del = (Ts[r] + rowc[j]) - ua[r] - cd.Uv[so[r] + bb[j]];
        w[r] = ok ? accR[i][j][r] * accR[i][j][r] + accI[i][j][r] * accI[i][j][r] : 0.0;
        dd[r] = ok ? del : 1.0;
        if constexpr (LS) {
          const double d2 = dd[r] * dd[r];
          w[r] *= dd[r] * d2;
          dd[r] = fma(d2, d2, d.ls_b2);
        }
      }
      const double n01 = fma(w[0], dd[1], w[1] * dd[0]);
      const double q01 = dd[0] * dd[1];
      const double n23 = fma(w[2], dd[3], w[3] * dd[2]);
      const double q23 = dd[2] * dd[3];
      acc = fma(fma(n01, q23, n23 * q01), rcp_nr(q01 * q23), acc);
    }
  }
  if (!isfinite(acc)) *flag = 2;
  const int tid = threadIdx.x;
  red[tid] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (tid < o) red[tid] += red[tid + o];
    __syncthreads();
  }
  if (tid == 0) cd.part[blk] = red[0];
}

// Per-class sum of partials (Neumaier-compensated, fixed order) divided by
// ||C||^2; out[k] for k < 9, out[9] = E2, out[10] = E0 - E_core,
// out[11] = ||C||^2; e2 receives E2.  A non-finite E2 (an exactly zero
// denominator, an overflow) sets the error flag.  One block.
__device__ __forceinline__ void finish_body(const Dev& d, const ClassDev* cds, int* flag) {
  __shared__ double ss[256], sc[256];
  __shared__ double cls[MRPT2_N_CLASS];
  double* out = d.out_parts;
  for (int k = 0; k < MRPT2_N_CLASS; ++k) {
    double s = 0.0, comp = 0.0;
    const int64_t nk = cds[k].n_part;
    const double* pk = cds[k].part;
    for (int64_t i = threadIdx.x; i < nk; i += 256) {
      const double x = pk[i];
      const double t = s + x;
      comp += (fabs(s) >= fabs(x)) ? (s - t) + x : (x - t) + s;
      s = t;
    }
    ss[threadIdx.x] = s;
    sc[threadIdx.x] = comp;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if (threadIdx.x < o) {
        const double a = ss[threadIdx.x], b = ss[threadIdx.x + o];
        const double t = a + b;
        const double e = (fabs(a) >= fabs(b)) ? (a - t) + b : (b - t) + a;
        ss[threadIdx.x] = t;
        sc[threadIdx.x] += sc[threadIdx.x + o] + e;
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) cls[k] = (ss[0] + sc[0]) / d.scal[1];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double s = 0.0, comp = 0.0;
    for (int k = 0; k < MRPT2_N_CLASS; ++k) {
      const double x = cls[k];
      const double t = s + x;
      comp += (fabs(s) >= fabs(x)) ? (s - t) + x : (x - t) + s;
      s = t;
    }
    const double tot = s + comp;
    if (!isfinite(tot)) *flag = 2;
    if (out) {
      for (int k = 0; k < MRPT2_N_CLASS; ++k) out[k] = cls[k];
      out[9] = tot;
      out[10] = d.scal[0];
      out[11] = d.scal[1];
    }
    *d.out_e2 = tot;
  }
}

__global__ void k_clear_flag(int* flag) {
  if (threadIdx.x == 0) *flag = 0;
}

}  // namespace mrpt2
