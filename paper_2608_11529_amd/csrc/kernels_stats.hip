// Denominator statistics of the external space (Sec. 2.6: an intruder state
// is an external determinant whose E0 - H_KK comes close to zero, where the
// terms of eq. pt2en blow up and a level shift is needed).
#include "kernels.hpp"

namespace mrpt2 {

// Smallest value and sum over a block of 256 threads.
__device__ __forceinline__ void block_min_sum256(double& mn, double& cnt) {
  __shared__ double sm[4], sc[4];
  for (int o = 32; o > 0; o >>= 1) {
    mn = fmin(mn, __shfl_xor(mn, o, 64));
    cnt += __shfl_xor(cnt, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    sm[threadIdx.x >> 6] = mn;
    sc[threadIdx.x >> 6] = cnt;
  }
  __syncthreads();
  mn = fmin(fmin(sm[0], sm[1]), fmin(sm[2], sm[3]));
  cnt = ((sc[0] + sc[1]) + sc[2]) + sc[3];
  __syncthreads();
}

// One class: each thread owns a row of the class's (row x string) grid
// (core holes and virtual spinors) and walks its block's chunk of strings;
// Delta = E0 - H_KK is the row constant plus the string tables, as in the
// energy kernels.  Each block writes the smallest |Delta| of its determinants
// and how many lie below the threshold (counts are exact in a double).
// Two-virtual classes: the block's 256 rows are one hole tuple, one virtual
// tile pair, four a and 64 b, so each chunk of strings stages the string
// parts of Delta (T + Uc, Uv of the four a and of the 64 b) in LDS.
// grid (ceil(rows / 256), string chunks), block 256.
constexpr int DSC = 64;   // strings per LDS chunk of the two-virtual statistics pass

template <int H, int V>
__device__ __forceinline__ void dstat_body(const Dev& d, const ClassDev& cd, int nchunk, const uint3 bid) {
  const int64_t r = (int64_t)bid.x * 256 + threadIdx.x;
  const Row w = decode_row<H, V>(d, cd, r);
  const double qr = row_const<H, V>(d, w);
  const int64_t S = cd.n_str, per = (S + nchunk - 1) / nchunk;
  const int64_t s0 = (int64_t)bid.y * per, s1 = s0 + per < S ? s0 + per : S;
  const double th = d.dstat_thresh;
  double mn = __builtin_huge_val(), cnt = 0.0;
  if constexpr (V == 2) {
    __shared__ double sG[DSC], sUa[DSC][4], sUb[DSC][64];
    const int tid = threadIdx.x, ia = tid >> 6, ib = tid & 63;
    const int64_t rab0 = ((int64_t)bid.x * 256) % (d.n_tp * 4096);
    const int64_t tp = rab0 >> 12;
    const int la0 = (int)((rab0 >> 6) & 63);
    const int a0 = d.tile_pairs[2 * tp] * 64 + la0, b0 = d.tile_pairs[2 * tp + 1] * 64;
    const int nv = d.n_v, nc = d.n_c;
    for (int64_t c0 = s0; c0 < s1; c0 += DSC) {
      __syncthreads();
      for (int e = tid; e < DSC * 64; e += 256) {
        const int sl = e >> 6, l = e & 63;
        const int64_t s = c0 + sl;
        sUb[sl][l] = (s < s1 && b0 + l < nv) ? cd.Uv[s * nv + b0 + l] : 0.0;
      }
      {
        const int sl = tid >> 2, l = tid & 3;
        const int64_t s = c0 + sl;
        sUa[sl][l] = (s < s1 && a0 + l < nv) ? cd.Uv[s * nv + a0 + l] : 0.0;
      }
      if (tid < DSC) {
        const int64_t s = c0 + tid;
        double gs = __builtin_huge_val();      // padding: |Delta| = inf counts nowhere
        if (s < s1) {
          gs = cd.T[s];
          if (H >= 1) gs += cd.Uc[s * nc + w.c0];
          if (H == 2) gs += cd.Uc[s * nc + w.c1];
        }
        sG[tid] = gs;
      }
      __syncthreads();
      if (w.valid) {
        const int ns = (int)(s1 - c0 < DSC ? s1 - c0 : DSC);
        for (int sl = 0; sl < ns; ++sl) {
          const double a = fabs(((sG[sl] + qr) - sUa[sl][ia]) - sUb[sl][ib]);
          mn = fmin(mn, a);
          cnt += a < th ? 1.0 : 0.0;
        }
      }
    }
  } else if (w.valid) {
    for (int64_t s = s0; s < s1; ++s) {
      const double a = fabs(string_delta<H, V>(cd, d, s, w) + qr);
      mn = fmin(mn, a);
      cnt += a < th ? 1.0 : 0.0;
    }
  }
  block_min_sum256(mn, cnt);
  if (threadIdx.x == 0) {
    const int64_t nbx = (cd.n_rows + 255) / 256;
    cd.dstat[(int64_t)bid.y * nbx + bid.x] = make_double2(mn, cnt);
  }
}

// Per class of one instance: the blocks' values folded into (min |Delta|,
// count).  grid (1), block 256.
__device__ __forceinline__ void dstatfin_body(const Dev& d, const ClassDev* cls) {
  for (int k = 0; k < 9; ++k) {
    const ClassDev& cd = cls[k];
    double mn = __builtin_huge_val(), cnt = 0.0;
    for (int64_t i = threadIdx.x; i < cd.n_dstat; i += 256) {
      const double2 v = cd.dstat[i];
      mn = fmin(mn, v.x);
      cnt += v.y;
    }
    block_min_sum256(mn, cnt);
    if (threadIdx.x == 0) d.dstat_out[k] = make_double2(mn, cnt);
  }
}

}  // namespace mrpt2
