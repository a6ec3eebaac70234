// Device kernels of the MRPT2 energy (gfx950).
//
// Index conventions (n_fc frozen core, n_c core, n_a active, n_v virtual):
//   global spinor g in [0, n): frozen core, core, active, virtual;
//   correlated index pc = g - n_fc;
//   occupied index xo in [0, n_o): core then active (n_o = n_c + n_a);
//   active/virtual row index pr in [0, n_a + n_v): active then virtual.
// Complex numbers are double2 (x = re, y = im).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mrpt2 {

// ---- complex helpers -------------------------------------------------------
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cfma(double2 a, double2 b, double2 c) {
  return make_double2(fma(a.x, b.x, fma(-a.y, b.y, c.x)), fma(a.x, b.y, fma(a.y, b.x, c.y)));
}
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double cabs2(double2 a) { return fma(a.x, a.x, a.y * a.y); }

// FP64 multiply-add acc += (+-c_L) x, where c_L is the value c held by lane L
// of the thread's row of 16 lanes (DPP row broadcast on the first operand):
// coefficients loaded once per row feed all 64 lanes without an LDS
// broadcast read per use.  Callers pass c straight from a memory load: a
// vector instruction writing c shortly before would need wait states ahead
// of the DPP read, which the inline assembly does not insert.
template <int L, bool NEG>
__device__ __forceinline__ void fmac_row(double& acc, double c, double x) {
  if constexpr (NEG)
    asm("v_fmac_f64_dpp %0, -%1, %2 row_newbcast:%3 row_mask:0xf bank_mask:0xf" : "+v"(acc) : "v"(c), "v"(x), "n"(L));
  else
    asm("v_fmac_f64_dpp %0, %1, %2 row_newbcast:%3 row_mask:0xf bank_mask:0xf" : "+v"(acc) : "v"(c), "v"(x), "n"(L));
}

// sigma_k += D_kj X_j for the GS strings of a group and one row of couplings
// X (patterns J0 and later present in the group's mask um): coefficient
// (string k, pattern j), entry e = k MJ + j of the group's GS MJ, is held by
// lane e mod 16 of every row in C[e / 16] and reaches the products by DPP
// row broadcast (fmac_row), in the order of cfma.
template <int MJ, int GS, int J0, int K>
__device__ __forceinline__ void row_sig_k(const double2 (&C)[GS * MJ / 16], const double2 (&X)[MJ],
                                           double2 (&sg)[GS]) {
  constexpr int E = K * MJ + J0, M = E >> 4, L = E & 15;
  fmac_row<L, true>(sg[K].x, C[M].y, X[J0].y);
  fmac_row<L, false>(sg[K].x, C[M].x, X[J0].x);
  fmac_row<L, false>(sg[K].y, C[M].y, X[J0].x);
  fmac_row<L, false>(sg[K].y, C[M].x, X[J0].y);
  if constexpr (K + 1 < GS) row_sig_k<MJ, GS, J0, K + 1>(C, X, sg);
}
template <int MJ, int GS, int J0>
__device__ __forceinline__ void row_sig(uint32_t um, const double2 (&C)[GS * MJ / 16], const double2 (&X)[MJ],
                                         double2 (&sg)[GS]) {
  if (um & (1u << J0)) row_sig_k<MJ, GS, J0, 0>(C, X, sg);
  if constexpr (J0 + 1 < MJ) row_sig<MJ, GS, J0 + 1>(um, C, X, sg);
}
// Reciprocal: hardware estimate (about 2^-24 relative) refined by one
// Newton-Raphson step, r1 = r0 (2 - d r0), giving relative error below 2^-47
// with a one-sided bias, far under the energy tolerances used here.
__device__ __forceinline__ double rcp_nr(double d) {
  double r = __builtin_amdgcn_rcp(d);
  double e = fma(-d, r, 1.0);
  return fma(r, e, r);
}

// Epstein-Nesbet weight g of one external determinant as a function of
// Delta = E0 - H_KK, and its derivative g'.  Without a level shift g = 1/Delta.
// With the imaginary level shift of Sec. 2.6 the denominator becomes
// Delta + i b/Delta and its inverse is taken by the real part:
//   g  = Delta^3 / (Delta^4 + b^2),
//   g' = Delta^2 (3 b^2 - Delta^4) / (Delta^4 + b^2)^2.
// b2 = b^2 is uniform over a launch, so the branch does not diverge.
__device__ __forceinline__ double en_weight(double del, double b2) {
  if (b2 == 0.0) return rcp_nr(del);
  const double d2 = del * del;
  return del * d2 * rcp_nr(fma(d2, d2, b2));
}
__device__ __forceinline__ void en_weight_d(double del, double b2, double& g, double& gp) {
  if (b2 == 0.0) {
    const double iv = rcp_nr(del);
    g = iv;
    gp = -iv * iv;
    return;
  }
  const double d2 = del * del, d4 = d2 * d2, iq = rcp_nr(d4 + b2);
  g = del * d2 * iq;
  gp = d2 * fma(3.0, b2, -d4) * iq * iq;
}

// ---- per-instance device view -------------------------------------------------
struct SetPtrs {
  const double2* B[4];
  int rank[4];
  int l0[4];
  int n_sets;
  int packed;      // 1: each B[L] stored as its upper triangle by rows
};

// Offset of entry (p, q), p <= q, in a row-major packed upper triangle of an
// n x n matrix.
__device__ __forceinline__ int64_t tri_off(int p, int q, int n) {
  return (int64_t)p * n - (int64_t)p * (p - 1) / 2 + (q - p);
}
// Entries per factor matrix in the caller's layout.
__device__ __forceinline__ int64_t fac_stride(const SetPtrs& sp, int n) {
  return sp.packed ? (int64_t)n * (n + 1) / 2 : (int64_t)n * n;
}
// Factor entry B[L][p][q] of one set (Hermitian; the packed layout keeps the
// upper triangle, the lower is its conjugate, a diagonal entry is real).
__device__ __forceinline__ double2 fac_at(const SetPtrs& sp, const double2* B, int L, int p, int q, int n) {
  if (!sp.packed) return B[((int64_t)L * n + p) * n + q];
  const double2* M = B + (int64_t)L * ((int64_t)n * (n + 1) / 2);
  if (p < q) return M[tri_off(p, q, n)];
  if (p > q) {
    const double2 v = M[tri_off(q, p, n)];
    return make_double2(v.x, -v.y);
  }
  return make_double2(M[tri_off(p, p, n)].x, 0.0);
}

struct Dev {
  int n_fc, n_c, n_a, n_v, n_o, n_occ, n_corr, n, n_l, n_p;
  int n_vt;
  int64_t n_tp, n_pairs;
  const double* sign;        // [n_l]
  const double* scale;       // [n_l]
  const uint64_t* pstrings;  // [n_p]
  const int64_t* plist_ptr;  // [n_p + 1] excitation lists of P (CSR)
  const int32_t* plist_col;  // reference strings one or two active replacements away
  const int32_t* hole_pairs; // [C(n_c,2)][2]
  const int32_t* tile_pairs; // [n_tp][2]
  double* dg;                // [n_l][n]   scale * Re B[L][p][p]
  double2* slab;             // [n_occ][n_corr][n_l]   scale * B[L][n_fc+pc][x]
  float2* slab32;            // mixed form only, else null: [n_o][n_v][n_l2], FP32
                             // slab of the virtual rows of the occupied x >= n_fc,
                             // times i where the factor weight is negative; the
                             // rows are padded with zero to the even n_l2
  int n_l2;                  // n_l rounded up to even
  double* W;                 // [n][n]
  double* eps;               // [n_corr]
  double2* f;                // [n_a+n_v][n_o]
  double2* fx;               // [n_fc+n_c][n_a+n_v][n_o] exchange partials of f per core spinor
  double2* G;                // [n_o][n_a+n_v][n_o][n_a]
  double2* A;                // [n_pairs][n_tp][64][64]
  double2* hpp;              // [n_p][n_p]
  double2* sigp;             // [n_p]
  double* scal;              // [0] = E0 - E_core, [1] = ||C||^2
  double ls_b2;              // square of the imaginary level-shift constant b (0: none)
  double dstat_thresh;       // denominator statistics: count |Delta| below this
  double2* dstat_out;        // [9] per class (min |Delta|, count below the threshold)
  double* dsum;              // [n_l]
  // inputs and outputs of the current call
  const double2* h;          // [n][n]
  const double2* c;          // [n_p]
  SetPtrs sets;              // factor sets
  double* out_parts;         // [12] or null
  double* out_e2;            // [1]
  double2* out_hpp;          // reference-Hamiltonian output (or null)
};

struct Pattern;

struct ClassDev {
  int h, v, n_pat;
  int64_t n_str, n_rows, n_holes, n_conn;
  const uint64_t* strings;
  const int32_t* conn_ptr;
  const int32_t* conn;
  const Pattern* pat;
  const int32_t* ekey;   // per coupling: integral key | sign << 31
  double* T;     // [S]
  double* Uc;    // [S][n_c]
  double* Uv;    // [S][n_v]
  double2* X;    // [n_pat][n_rows] (v < 2)
  double* part;  // partial sums
  int64_t n_part;  // partial sums written by the class's kernel
  int nsc;       // string chunks
  double2* D;    // [S][n_pat] dense coefficients (classes with few patterns)
  uint32_t* mask;  // [S] nonzero patterns per string
  // class (0,2): string tiles and their dense coefficient blocks
  int64_t n_tiles;
  const int32_t* tile_s0;   // [n_tiles + 1]
  const int32_t* tile_k0;   // [n_tiles + 1]
  const int32_t* tile_sup;  // [tile_k0[n_tiles]] occupied-pair index or -1
  const int32_t* ccol;      // [n_conn]
  double2* Md;              // tile t: [64][K_t] at 64 * tile_k0[t]
  double2* dstat;           // denominator statistics per (row block, string chunk)
  int64_t n_dstat;
};

// Adjoint (backward) state of one instance: gradients of E2 with respect to
// the intermediate tables, accumulated in the gradient workspace, and the
// caller's output buffers.
struct GradDev {
  double* scal;        // [0] dE2/d(E0 - E_core), [1] E2 of the recomputed forward pass
  double* Wb;          // [n][n]      adjoint of W
  double* Wsym;        // [n][n]      Wb + Wb^T
  double* epsb;        // [n_corr]    adjoint of eps
  double2* fb;         // f layout    adjoint of the core Fock block
  double2* Gb;         // G layout    adjoint of (px|qy)
  double2* Ab;         // A layout    adjoint of <ab||xy>
  double2* slabb;      // slab layout adjoint of the scaled factor columns
  double* dgb;         // [n_l][n]    adjoint of the scaled diagonals
  double* dsumb;       // [n_l]       adjoint of dsum
  double2* hb;         // [n][n]      adjoint of h (before projection)
  double2* cb;         // [n_p]       adjoint of C from the external space
  double4* zero;       // region cleared before the adjoint kernels
  int64_t n_zero;      // its size in 32-byte units
  const double* grad_e2;   // upstream gradient dL/dE2 (device scalar)
  double2* out_dh;     // [n][n]
  double2* out_dc;     // [n_p]
  double2* out_dB[4];  // per factor set [rank][n][n]
  double* out_e2;      // E2 of the forward pass (or null)
};

struct ClassGrad {
  double2* Xb;         // [n_pat][n_rows] adjoint of X (v < 2)
  double2* Xbp;        // [row_split][n_pat][n_rows] its private partials per string chunk, or null
  double* Tb;          // [parts][S]  per-part sums of dE2/dDelta over each string
  double2* cbe;        // [parts][n_conn] per-part coefficient adjoints per coupling
  double* r1;          // [parts][S] class (2,2): per-part sums of |A|^2 / Delta per string
  double2* dbp;        // [parts][S][n_pat] dense-coefficient adjoints (class (1,2)) or null
  double2* ecoef;      // [n_conn] sign * C_beta per coupling
  double* wpart;       // class (2,2): per-block partials of the Uv adjoint [blocks][n_v][n_a]
  double* UvT;         // generic one-virtual classes: string tables transposed for the
  double* UcT;         // string-owned pass, Uv^T [n_v][S] (v = 1), Uc^T [n_c][S] (h >= 1)
  double* u2;          // class (0,2): per part, per string and virtual spinor, sums of Delta-bar [parts][S][n_v]
  int64_t wblocks;     // number of those blocks (string blocks x parts)
  int row_split;       // string chunks of the row-owned pass (> 1: shared rows, atomics)
  int parts;           // row parts of the string-owned pass
  int64_t rows_per_part;   // rows per part (tile pairs per part for class (1,2))
};

// Everything a kernel needs about one instance (uploaded once per call).
// Descriptors sit kInstStride bytes apart in device memory.
struct Inst {
  Dev d;
  ClassDev cls[9];
  GradDev g;
  ClassGrad cg[9];
};
constexpr size_t kInstStride = 4096;

__device__ __forceinline__ const Inst& inst_at(const Inst* base, int i) {
  return *reinterpret_cast<const Inst*>(reinterpret_cast<const char*>(base) + (size_t)i * kInstStride);
}

// One instance's share of a batched launch: its grid (gx x gy blocks) starts
// at flat block blk0 of the launch; arg is kernel specific (factor set).
struct Job {
  int32_t inst, gx, gy, arg;
  int64_t blk0;
};

// Job of flat block b: the last job whose first block is <= b.
__device__ __forceinline__ int find_job(const Job* __restrict__ jobs, int n, int64_t b) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].blk0 <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ int64_t occ_pair(int x, int y, int n_o) {  // x < y
  return (int64_t)x * n_o - (int64_t)x * (x + 1) / 2 + (y - x - 1);
}

__device__ __forceinline__ double2 Gv(const Dev& d, int xo, int pr, int yo, int qa) {
  return d.G[(((int64_t)xo * (d.n_a + d.n_v) + pr) * d.n_o + yo) * d.n_a + qa];
}

}  // namespace mrpt2
