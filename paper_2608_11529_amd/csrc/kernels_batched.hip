// Batched launch wrappers: one launch covers every instance of a plan.  Each
// flat block finds its job (instance, grid, argument) in the plan's job
// table, rebuilds its block coordinates within that instance's grid, and runs
// the kernel body on the instance's descriptor.
#include "kernels.hpp"

namespace mrpt2 {

#define MRPT2_JOB                                                                              \
  const int job_ = find_job(jobs, njobs, (int64_t)blockIdx.x);                                 \
  const Job jb = jobs[job_];                                                                   \
  const int64_t lb_ = (int64_t)blockIdx.x - jb.blk0;                                           \
  const uint3 bid = make_uint3((uint32_t)(lb_ % jb.gx), (uint32_t)(lb_ / jb.gx), 0u);         \
  const Inst& I = inst_at(insts, jb.inst);

#define MRPT2_ARGS const Inst* __restrict__ insts, const Job* __restrict__ jobs, int njobs, int* flag, int karg

__global__ void __launch_bounds__(256) k_b_pack(MRPT2_ARGS) {
  MRPT2_JOB
  pack_body(I.d, jb.arg, bid);
}
__global__ void __launch_bounds__(256) k_b_diag(MRPT2_ARGS) {
  MRPT2_JOB
  diag_body(I.d, jb.arg, bid);
}
__global__ void __launch_bounds__(256) k_b_wpass(MRPT2_ARGS) {
  MRPT2_JOB
  wpass_body(I.d, flag, bid);
}
__global__ void __launch_bounds__(256) k_b_eps(MRPT2_ARGS) {
  MRPT2_JOB
  eps_body(I.d, flag, bid);
}
__global__ void __launch_bounds__(256) k_b_dsum(MRPT2_ARGS) {
  MRPT2_JOB
  dsum_body(I.d, bid);
}
__global__ void __launch_bounds__(256) k_b_fockx(MRPT2_ARGS) {
  MRPT2_JOB
  fockx_body(I.d, bid);
}
__global__ void __launch_bounds__(64) k_b_fock(MRPT2_ARGS) {
  MRPT2_JOB
  fock_body(I.d, bid);
}
__global__ void __launch_bounds__(256) k_b_gbuild(MRPT2_ARGS) {
  MRPT2_JOB
  gbuild_body(I.d, bid);
}
__global__ void __launch_bounds__(256) k_b_hpp(MRPT2_ARGS) {
  MRPT2_JOB
  hpp_body(I.d, karg ? I.d.out_hpp : I.d.hpp, bid);
}
__global__ void __launch_bounds__(64) k_b_sigp(MRPT2_ARGS) {
  MRPT2_JOB
  sigp_body(I.d, bid);
}
__global__ void __launch_bounds__(256) k_b_e0(MRPT2_ARGS) {
  MRPT2_JOB
  (void)bid;
  e0_body(I.d, flag);
}
// two waves per SIMD (252 VGPRs, no AGPR accumulators) instead of one
__global__ void __launch_bounds__(256) k_b_abuild(MRPT2_ARGS) {
  MRPT2_JOB
  abuild_body(I.d, bid);
}
__global__ void __launch_bounds__(512) k_b_abuild128(MRPT2_ARGS) {
  MRPT2_JOB
  abuild128_body(I.d, bid);
}
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 8))) k_b_abuild_f32(MRPT2_ARGS) {
  MRPT2_JOB
  abuild_f32_body(I.d, bid);
}
__global__ void __launch_bounds__(256) k_b_class_tables(MRPT2_ARGS) {
  MRPT2_JOB
  class_tables_body(I.d, I.cls[jb.arg], bid);
}
__global__ void __launch_bounds__(256) k_b_xbuild(MRPT2_ARGS) {
  MRPT2_JOB
  xbuild_body(I.d, I.cls[jb.arg], bid);
}
__global__ void __launch_bounds__(256) k_b_dense_coef(MRPT2_ARGS) {
  MRPT2_JOB
  dense_coef_body(I.d, I.cls[jb.arg], bid);
}
// three waves per SIMD: 168 VGPRs (a few spills) beat two waves at 176
template <bool LS>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 8))) k_b_e22(MRPT2_ARGS) {
  MRPT2_JOB
  e22_body<LS>(I.d, I.cls[0], flag, bid);
}
template <int MJ, bool LS>
__global__ void __launch_bounds__(256) k_b_e21(MRPT2_ARGS) {
  MRPT2_JOB
  e21_body<MJ, LS>(I.d, I.cls[3], flag, bid);
}
template <int MJ, bool LS, bool F32 = false>
__global__ void __launch_bounds__(256) k_b_e12(MRPT2_ARGS) {
  MRPT2_JOB
  e12_body<MJ, LS, F32>(I.d, I.cls[1], flag, bid);
}
template <bool F32, bool LS>
__global__ void __launch_bounds__(256) k_b_e02(MRPT2_ARGS) {
  MRPT2_JOB
  e02_body<F32, LS>(I.d, I.cls[2], flag, bid);
}
__global__ void __launch_bounds__(64) k_b_e02coef(MRPT2_ARGS) {
  MRPT2_JOB
  e02coef_body(I.d, I.cls[jb.arg], bid);
}
template <int H, int V, int K>
__global__ void __launch_bounds__(SIG_THREADS) k_b_sigma(MRPT2_ARGS) {
  MRPT2_JOB
  sigma_body<H, V>(I.d, I.cls[K], flag, bid);
}
__global__ void __launch_bounds__(256) k_b_finish(MRPT2_ARGS) {
  MRPT2_JOB
  (void)bid;
  finish_body(I.d, I.cls, flag);
}

// ---- adjoint ----
__global__ void __launch_bounds__(256) k_b_bzero(MRPT2_ARGS) {
  MRPT2_JOB
  bzero_body(I.g, bid, jb.gx);
}
template <int H, int V, int K>
__global__ void __launch_bounds__(256) k_b_brow(MRPT2_ARGS) {
  MRPT2_JOB
  brow_body<H, V>(I.d, I.cls[K], I.g, I.cg[K], bid);
}
template <int H, int V, int K>
__global__ void __launch_bounds__(256) k_b_bstr(MRPT2_ARGS) {
  MRPT2_JOB
  bstr_body<H, V>(I.d, I.cls[K], I.g, I.cg[K], bid);
}
__global__ void __launch_bounds__(256) k_b_becoef(MRPT2_ARGS) {
  MRPT2_JOB
  becoef_body(I.d, I.cls[jb.arg], I.cg[jb.arg], bid);
}
__global__ void __launch_bounds__(256) k_b_b22a(MRPT2_ARGS) {
  MRPT2_JOB
  b22a_body(I.d, I.cls[0], I.g, bid);
}
__global__ void __launch_bounds__(256) k_b_btrans(MRPT2_ARGS) {
  MRPT2_JOB
  btrans_body(I.d, I.cls[jb.arg >> 1], I.cg[jb.arg >> 1], jb.arg & 1, bid);
}
__global__ void __launch_bounds__(B22T) k_b_b22b(MRPT2_ARGS) {
  MRPT2_JOB
  b22b_body(I.d, I.cls[0], I.g, I.cg[0], bid, jb.gx);
}
__global__ void __launch_bounds__(256) k_b_b22w(MRPT2_ARGS) {
  MRPT2_JOB
  b22w_body(I.d, I.cls[0], I.g, I.cg[0], bid, I.cg[0].wblocks);
}
__global__ void __launch_bounds__(256) k_b_b22fin(MRPT2_ARGS) {
  MRPT2_JOB
  b22fin_body(I.d, I.cls[0], I.g, I.cg[0], bid);
}
template <int MJ, int CH = 32>
__global__ void __launch_bounds__(256, (MJ == 20 ? 2 : 1)) k_b_b12r(MRPT2_ARGS) {
  MRPT2_JOB
  // four strings per group up to 20 patterns (two beyond: registers); the
  // per-spinor table sums in registers up to 16 patterns, else in LDS
  b12r_body<MJ, (MJ > 20 ? 2 : 4), (MJ <= 16), CH>(I.d, I.cls[1], I.g, I.cg[1], bid);
}
template <int MJ>
__global__ void __launch_bounds__(256) k_b_b12s(MRPT2_ARGS) {
  MRPT2_JOB
  b12s_body<MJ>(I.d, I.cls[1], I.g, I.cg[1], bid);
}
__global__ void __launch_bounds__(256) k_b_b02r(MRPT2_ARGS) {
  MRPT2_JOB
  b02r_body(I.d, I.cls[2], I.g, bid);
}
__global__ void __launch_bounds__(256) k_b_b02s(MRPT2_ARGS) {
  MRPT2_JOB
  b02s_body(I.d, I.cls[2], I.g, I.cg[2], bid, (int)(jb.gx / I.cls[2].n_tiles));
}
__global__ void __launch_bounds__(256) k_b_b02w(MRPT2_ARGS) {
  MRPT2_JOB
  b02w_body(I.d, I.cls[2], I.g, I.cg[2], bid, jb.gy);
}
__global__ void __launch_bounds__(256) k_b_bsfin(MRPT2_ARGS) {
  MRPT2_JOB
  bstrfin_body(I.d, I.cls[jb.arg], I.g, I.cg[jb.arg], bid);
}
__global__ void __launch_bounds__(256) k_b_bhpp(MRPT2_ARGS) {
  MRPT2_JOB
  bhpp_body(I.d, I.g, bid);
}
__global__ void __launch_bounds__(256) k_b_bxb(MRPT2_ARGS) {
  MRPT2_JOB
  bxbuild_body(I.d, I.cls[jb.arg], I.g, I.cg[jb.arg], bid);
}
template <int H, int V>
__global__ void __launch_bounds__(256) k_b_dstat(MRPT2_ARGS) {
  MRPT2_JOB
  dstat_body<H, V>(I.d, I.cls[jb.arg], jb.gy, bid);
}
__global__ void __launch_bounds__(256) k_b_dstatfin(MRPT2_ARGS) {
  MRPT2_JOB
  (void)bid;
  dstatfin_body(I.d, I.cls);
}
__global__ void __launch_bounds__(256) k_b_bxbred(MRPT2_ARGS) {
  MRPT2_JOB
  bxbred_body(I.cls[jb.arg], I.cg[jb.arg], bid);
}
__global__ void __launch_bounds__(512) k_b_bag128(MRPT2_ARGS) {
  MRPT2_JOB
  bagemm128_body(I.d, I.g, bid);
}
__global__ void __launch_bounds__(256) k_b_bag(MRPT2_ARGS) {
  MRPT2_JOB
  bagemm_body(I.d, I.g, bid);
}
// three waves per SIMD (168 VGPRs, a few spills) beat two at 196 registers
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 8))) k_b_bagf(MRPT2_ARGS) {
  MRPT2_JOB
  bagemm_f32_body(I.d, I.g, bid);
}
__global__ void __launch_bounds__(256) k_b_bgg(MRPT2_ARGS) {
  MRPT2_JOB
  bggemm_body(I.d, I.g, jb.arg, bid);
}
__global__ void __launch_bounds__(64) k_b_bfock(MRPT2_ARGS) {
  MRPT2_JOB
  bfock_body(I.d, I.g, bid);
}
__global__ void __launch_bounds__(256) k_b_bdsum(MRPT2_ARGS) {
  MRPT2_JOB
  bdsum_body(I.d, I.g, bid);
}
__global__ void __launch_bounds__(256) k_b_bhfe(MRPT2_ARGS) {
  MRPT2_JOB
  bhfe_body(I.d, I.g, bid);
}
__global__ void __launch_bounds__(256) k_b_bwsym(MRPT2_ARGS) {
  MRPT2_JOB
  bwsym_body(I.d, I.g, bid);
}
__global__ void __launch_bounds__(256) k_b_bdg(MRPT2_ARGS) {
  MRPT2_JOB
  bdg_body(I.d, I.g, bid);
}
__global__ void __launch_bounds__(256) k_b_bdb(MRPT2_ARGS) {
  MRPT2_JOB
  bdB_body(I.d, I.g, jb.arg, bid);
}
__global__ void __launch_bounds__(256) k_b_bdh(MRPT2_ARGS) {
  MRPT2_JOB
  bdh_body(I.d, I.g, bid);
}
__global__ void __launch_bounds__(256) k_b_bdc(MRPT2_ARGS) {
  MRPT2_JOB
  bdc_body(I.d, I.g, bid);
}

#undef MRPT2_JOB

}  // namespace mrpt2
