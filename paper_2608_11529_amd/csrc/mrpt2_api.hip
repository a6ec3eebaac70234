// C interface: plan management and the launch sequence of one energy
// evaluation (tables -> reference energy -> integral builds -> per-class
// sigma contraction with the Epstein-Nesbet epilogue -> reductions).  Every
// launch covers all instances of the plan (batched form); the sequence is
// fixed by the plan, so it can be captured into a HIP graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <mutex>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "kernels.hpp"
#include "mrpt2.h"
#include "plan.hpp"

#include "kernels_tables.hip"
#include "kernels_energy.hip"
#include "kernels_backward.hip"
#include "kernels_stats.hip"
#include "kernels_batched.hip"
#include "kernels_davidson.hip"

struct mrpt2_plan_s {
  mrpt2::Plan p;
};

using namespace mrpt2;

static_assert(sizeof(Inst) <= kInstBytes, "instance descriptor exceeds its reserved bytes");
static_assert(kInstStride == kInstBytes, "host and device descriptor strides differ");
static_assert(sizeof(Job) == sizeof(JobH), "job layout differs between host and device");

namespace {

#define HIPCHK(x)                                \
  do {                                           \
    if ((x) != hipSuccess) return MRPT2_ERR_HIP; \
  } while (0)

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

Dev make_dev(const InstancePlan& ip, const char* pers, char* work, const mrpt2_inputs* in) {
  Dev d{};
  d.n_fc = ip.n_fc;
  d.n_c = ip.n_c;
  d.n_a = ip.n_a;
  d.n_v = ip.n_v;
  d.n_o = ip.n_o;
  d.n_occ = ip.n_occ;
  d.n_corr = ip.n_corr;
  d.n = ip.n;
  d.n_l = ip.n_l;
  d.n_p = (int)ip.pstrings.size();
  d.n_vt = ip.n_vt;
  d.n_tp = ip.n_tp;
  d.n_pairs = ip.n_pairs;
  const char* P = pers + ip.persistent_base;
  char* W = work + ip.workspace_base;
  d.sign = (const double*)(P + ip.off_sign);
  d.scale = (const double*)(P + ip.off_scale);
  d.pstrings = (const uint64_t*)(P + ip.off_pstrings);
  d.plist_ptr = (const int64_t*)(P + ip.off_plist_ptr);
  d.plist_col = (const int32_t*)(P + ip.off_plist_col);
  d.hole_pairs = (const int32_t*)(P + ip.off_hole_pairs);
  d.tile_pairs = (const int32_t*)(P + ip.off_tile_pairs);
  d.dg = (double*)(W + ip.off_dg);
  d.slab = (double2*)(W + ip.off_slab);
  d.n_l2 = ip.n_l + (ip.n_l & 1);
  d.slab32 = (ip.d.precision == MRPT2_MIXED && ip.n_v >= 2) ? (float2*)(W + ip.off_slab32) : nullptr;
  d.W = (double*)(W + ip.off_W);
  d.eps = (double*)(W + ip.off_eps);
  d.f = (double2*)(W + ip.off_f);
  d.fx = (double2*)(W + ip.off_fx);
  d.G = (double2*)(W + ip.off_G);
  d.A = (double2*)(W + ip.off_A);
  d.hpp = (double2*)(W + ip.off_hpp);
  d.sigp = (double2*)(W + ip.off_sigp);
  d.scal = (double*)(W + ip.off_scal);
  d.ls_b2 = ip.d.level_shift_b * ip.d.level_shift_b;
  d.dsum = (double*)(W + ip.off_dsum);
  d.dstat_out = (double2*)(W + ip.off_dstat_out);
  d.h = (const double2*)in->h;
  d.c = (const double2*)in->c;
  int l0 = 0;
  d.sets.n_sets = ip.d.n_sets;
  d.sets.packed = ip.d.layout == MRPT2_LAYOUT_PACKED ? 1 : 0;
  for (int t = 0; t < ip.d.n_sets; ++t) {
    d.sets.B[t] = (const double2*)in->B[t];
    d.sets.rank[t] = ip.d.rank[t];
    d.sets.l0[t] = l0;
    l0 += ip.d.rank[t];
  }
  return d;
}

ClassDev make_class(const InstancePlan& ip, int k, const char* pers, char* work) {
  const ClassPlan& cp = ip.cls[k];
  const char* P = pers + ip.persistent_base;
  char* W = work + ip.workspace_base;
  ClassDev c{};
  c.h = cp.h;
  c.v = cp.v;
  c.n_pat = (int)cp.patterns.size();
  c.n_str = (int64_t)cp.strings.size();
  c.n_rows = cp.n_rows;
  c.n_holes = cp.n_holes;
  c.n_conn = cp.n_conn;
  c.strings = (const uint64_t*)(P + cp.off_strings);
  c.conn_ptr = (const int32_t*)(P + cp.off_conn_ptr);
  c.conn = (const int32_t*)(P + cp.off_conn);
  c.pat = (const Pattern*)(P + cp.off_pat);
  c.ekey = (const int32_t*)(P + cp.off_ekey);
  c.T = (double*)(W + cp.off_T);
  c.Uc = (double*)(W + cp.off_Uc);
  c.Uv = (double*)(W + cp.off_Uv);
  c.X = (double2*)(W + cp.off_X);
  c.D = (double2*)(W + cp.off_D);
  c.mask = (uint32_t*)(W + cp.off_mask);
  c.n_tiles = cp.n_tiles;
  c.tile_s0 = (const int32_t*)(P + cp.off_tile_s0);
  c.tile_k0 = (const int32_t*)(P + cp.off_tile_k0);
  c.tile_sup = (const int32_t*)(P + cp.off_tile_sup);
  c.ccol = (const int32_t*)(P + cp.off_ccol);
  c.Md = (double2*)(W + cp.off_Md);
  c.dstat = (double2*)(W + cp.off_dstat);
  c.n_dstat = cp.n_dstat;
  c.part = (double*)(W + ip.off_part_class[k]);
  c.n_part = (cp.strings.empty() || cp.n_rows == 0) ? 0 : cp.n_blocks;
  const int64_t rb = cdiv(cp.n_rows, 256);
  c.nsc = rb > 0 ? (int)(sigma_blocks(ip, k) / rb) : 1;
  return c;
}

GradDev make_grad(const InstancePlan& ip, char* gw, const mrpt2_grads* out, const double* grad_e2, double* e2) {
  GradDev g{};
  char* G = gw + ip.grad_base;
  g.scal = (double*)(G + ip.off_gs);
  g.Wb = (double*)(G + ip.off_Wb);
  g.Wsym = (double*)(G + ip.off_Wsym);
  g.epsb = (double*)(G + ip.off_epsb);
  g.fb = (double2*)(G + ip.off_fb);
  g.Gb = (double2*)(G + ip.off_Gb);
  g.Ab = (double2*)(G + ip.off_Ab);
  g.slabb = (double2*)(G + ip.off_slabb);
  g.dgb = (double*)(G + ip.off_dgb);
  g.dsumb = (double*)(G + ip.off_dsumb);
  g.hb = (double2*)(G + ip.off_hb);
  g.cb = (double2*)(G + ip.off_cb);
  g.zero = (double4*)G;
  g.n_zero = (int64_t)(ip.grad_bytes / 32);
  g.grad_e2 = grad_e2;
  g.out_dh = (double2*)out->dh;
  g.out_dc = (double2*)out->dc;
  for (int t = 0; t < ip.d.n_sets; ++t) g.out_dB[t] = (double2*)out->dB[t];
  g.out_e2 = e2;
  return g;
}

ClassGrad make_class_grad(const InstancePlan& ip, int k, char* gw) {
  const ClassPlan& cp = ip.cls[k];
  char* G = gw + ip.grad_base;
  ClassGrad c{};
  c.Xb = (double2*)(G + cp.off_Xb);
  c.Xbp = cp.xb_private ? (double2*)(G + cp.off_Xbp) : nullptr;
  c.Tb = (double*)(G + cp.off_Tb);
  c.cbe = (double2*)(G + cp.off_cbe);
  c.r1 = (double*)(G + cp.off_r1);
  c.dbp = cp.kernel_bwd == KERN_E12 ? (double2*)(G + cp.off_dbp) : nullptr;
  c.row_split = cp.row_split;
  c.ecoef = (double2*)(G + cp.off_ecoef);
  c.wpart = (double*)(G + cp.off_wpart);
  c.u2 = (double*)(G + cp.off_u2);
  c.UvT = (double*)(G + cp.off_UvT);
  c.UcT = (double*)(G + cp.off_UcT);
  c.wblocks = cp.kernel_bwd == KERN_E22 ? (int64_t)cp.parts * ((int64_t)(cp.strings.size() + B22T - 1) / B22T) : 0;
  c.parts = cp.parts;
  c.rows_per_part = cp.rows_per_part;
  return c;
}

struct Timer {
  hipEvent_t ev[2 * 128];
  int slot[128];
  int n = 0;
  bool on = false;
  hipStream_t st = nullptr;
  void begin(int s) {
    if (!on || s < 0 || n >= 128) return;
    slot[n] = s;
    hipEventRecord(ev[2 * n], st);
  }
  void end(int s) {
    if (!on || s < 0 || n >= 128) return;
    hipEventRecord(ev[2 * n + 1], st);
    ++n;
  }
};

mrpt2_status check_regions(const Plan& p, const void* pers, void* work, size_t wbytes) {
  if (!pers || !work) return MRPT2_ERR_ARG;
  if (wbytes < p.workspace_bytes) return MRPT2_ERR_WORKSPACE;
  if (((uintptr_t)pers & 255) || ((uintptr_t)work & 255)) return MRPT2_ERR_ARG;
  return MRPT2_OK;
}

// Pinned staging for `sets` descriptor sets.  Growing it waits for the
// stream, so that no queued copy still reads the old buffer.
mrpt2_status ensure_pinned(Plan& P, size_t sets, hipStream_t st) {
  const size_t need = kInstBytes * P.inst.size() * sets;
  if (P.pinned && P.pinned_bytes >= need) return MRPT2_OK;
  if (P.pinned) {
    HIPCHK(hipStreamSynchronize(st));
    HIPCHK(hipHostFree(P.pinned));
    P.pinned = nullptr;
    P.pinned_bytes = 0;
  }
  HIPCHK(hipHostMalloc(&P.pinned, need, hipHostMallocDefault));
  P.pinned_bytes = need;
  return MRPT2_OK;
}

// Fill the instance descriptors in pinned host memory and copy them to the
// workspace (asynchronously, on stream).  They are staged in descriptor set
// `slot`: a multi-state call fills one set per state before the stream has
// copied the earlier ones.
// Descriptors of every instance written into host memory `stage`.
mrpt2_status fill_insts(const Plan& P, const mrpt2_inputs* in, const char* pers, char* work, char* stage,
                        double* e2, double* parts, double* hpp_out, int only, char* gw,
                        const mrpt2_grads* grads, const double* grad_e2) {
  const size_t bytes = kInstBytes * P.inst.size();
  std::memset(stage, 0, bytes);
  for (size_t i = 0; i < P.inst.size(); ++i) {
    if (only >= 0 && (int)i != only) continue;
    const mrpt2_inputs* ini = in + (only >= 0 ? 0 : i);
    const InstancePlan& ip = P.inst[i];
    if (!ini->h || (only < 0 && !ini->c)) return MRPT2_ERR_ARG;
    for (int t = 0; t < ip.d.n_sets; ++t)
      if (ip.d.rank[t] > 0 && !ini->B[t]) return MRPT2_ERR_ARG;
    Inst* I = (Inst*)(stage + kInstBytes * i);
    I->d = make_dev(ip, pers, work, ini);
    I->d.out_e2 = e2 ? e2 + i : nullptr;
    I->d.out_parts = parts ? parts + 12 * i : nullptr;
    I->d.out_hpp = (double2*)hpp_out;
    I->d.dstat_thresh = P.dstat_thresh;
    for (int k = 0; k < MRPT2_N_CLASS; ++k) I->cls[k] = make_class(ip, k, pers, work);
    if (gw) {
      const mrpt2_grads* go = grads + i;
      if (!go->dh || !go->dc || !grad_e2) return MRPT2_ERR_ARG;
      for (int t = 0; t < ip.d.n_sets; ++t)
        if (ip.d.rank[t] > 0 && !go->dB[t]) return MRPT2_ERR_ARG;
      I->g = make_grad(ip, gw, go, grad_e2 + i, e2 ? e2 + i : nullptr);
      I->d.out_e2 = I->g.scal + 1;
      I->d.out_parts = nullptr;
      for (int k = 0; k < MRPT2_N_CLASS; ++k) {
        I->cg[k] = make_class_grad(ip, k, gw);
        // the adjoint's E2 comes from its row passes' block sums
        I->cls[k].part = (double*)(gw + ip.grad_base + ip.cls[k].off_e2part);
        I->cls[k].n_part = ip.cls[k].n_e2part;
      }
    }
  }
  return MRPT2_OK;
}

mrpt2_status upload_insts(Plan& P, const mrpt2_inputs* in, const char* pers, char* work, hipStream_t st,
                          double* e2, double* parts, double* hpp_out, int only, char* gw = nullptr,
                          const mrpt2_grads* grads = nullptr, const double* grad_e2 = nullptr,
                          int slot = 0) {
  const size_t bytes = kInstBytes * P.inst.size();
  mrpt2_status ps = ensure_pinned(P, (size_t)slot + 1, st);
  if (ps != MRPT2_OK) return ps;
  char* stage = (char*)P.pinned + bytes * slot;
  // The staging buffer is reused by every call on this plan: before the
  // first descriptor set of a call is rewritten, the previous call's last
  // copy from it must have run (an asynchronous call may still have it
  // queued).  Under stream capture the copy is a graph node that reads the
  // buffer at every replay, so the captured plan is reserved for its graph
  // and nothing is waited for or recorded.
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  HIPCHK(hipStreamIsCapturing(st, &cap));
  const bool capturing = cap != hipStreamCaptureStatusNone;
  if (!capturing && slot == 0 && P.staged_recorded) HIPCHK(hipEventSynchronize(P.staged));
  ps = fill_insts(P, in, pers, work, stage, e2, parts, hpp_out, only, gw, grads, grad_e2);
  if (ps != MRPT2_OK) return ps;
  HIPCHK(hipMemcpyAsync(work + P.off_insts, stage, bytes, hipMemcpyHostToDevice, st));
  if (!capturing) {
    if (!P.staged) HIPCHK(hipEventCreateWithFlags(&P.staged, hipEventDisableTiming));
    HIPCHK(hipEventRecord(P.staged, st));
    P.staged_recorded = true;
  }
  return MRPT2_OK;
}

// Launches whose results depend on the reference vector (sigma_P, E0, the
// per-string tables that hold E0, the coefficient blocks, the sigma
// contractions and the sums).  Everything else in the energy sequence
// depends only on h and the factors.
bool depends_on_c(int kid) {
  switch (kid) {
    case K_SIGP: case K_E0: case K_CTAB: case K_DCOEF: case K_E02COEF: case K_E22:
    case K_E12_8: case K_E12_16: case K_E12_20: case K_E12_24: case K_E12_32: case K_E02: case K_E02F:
    case K_E12F_8: case K_E12F_16: case K_E12F_20: case K_E12F_24: case K_E12F_32:
    case K_E22S: case K_E12S_8: case K_E12S_16: case K_E12S_20: case K_E12S_24: case K_E12S_32: case K_E02S:
    case K_E02FS: case K_E21_8: case K_E21_16: case K_E21_20: case K_E21_24: case K_E21_32: case K_E21S_8:
    case K_E21S_16: case K_E21S_20: case K_E21S_24: case K_E21S_32:
    case K_SIG22: case K_SIG12: case K_SIG02: case K_SIG21: case K_SIG11: case K_SIG01:
    case K_SIG20: case K_SIG10: case K_SIG00: case K_FINISH:
      return true;
    default:
      return false;
  }
}

enum RunPart { RUN_ALL = 0, RUN_SHARED = 1, RUN_PER_STATE = 2 };

// Enqueue a launch sequence.
mrpt2_status run(const Plan& P, const std::vector<Launch>& seq, const char* pers, char* work, hipStream_t st,
                 Timer& tm, RunPart part = RUN_ALL) {
  const Inst* insts = (const Inst*)(work + P.off_insts);
  const Job* jobs_all = (const Job*)(pers + P.off_jobs);
  int* flag = (int*)(work + P.off_flag);
  for (const Launch& L : seq) {
    if (part != RUN_ALL && depends_on_c(L.kid) != (part == RUN_PER_STATE)) continue;
    const Job* jobs = jobs_all + L.job0;
    const dim3 g((unsigned)L.nblocks), b256(256), b64(64);
    const int nj = L.njobs, ka = L.arg;
    tm.begin(L.stage);
    switch (L.kid) {
      case K_CLEAR: hipLaunchKernelGGL(k_clear_flag, dim3(1), dim3(64), 0, st, flag); break;
      case K_PACK: hipLaunchKernelGGL(k_b_pack, g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_DIAG: hipLaunchKernelGGL(k_b_diag, g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_WPASS: hipLaunchKernelGGL(k_b_wpass, g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_EPS: hipLaunchKernelGGL(k_b_eps, g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_DSUM: hipLaunchKernelGGL(k_b_dsum, g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_FOCK: hipLaunchKernelGGL(k_b_fock, g, b64, 0, st, insts, jobs, nj, flag, ka); break;
      case K_FOCKX: hipLaunchKernelGGL(k_b_fockx, g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_GBUILD: hipLaunchKernelGGL(k_b_gbuild, g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_HPP: hipLaunchKernelGGL(k_b_hpp, g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_SIGP: hipLaunchKernelGGL(k_b_sigp, g, b64, 0, st, insts, jobs, nj, flag, ka); break;
      case K_E0: hipLaunchKernelGGL(k_b_e0, g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_ABUILD: hipLaunchKernelGGL(k_b_abuild128, g, dim3(512), 0, st, insts, jobs, nj, flag, ka); break;
      case K_ABUILD64: hipLaunchKernelGGL(k_b_abuild, g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_ABUILD32: hipLaunchKernelGGL(k_b_abuild_f32, g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_CTAB: hipLaunchKernelGGL(k_b_class_tables, g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_XBUILD: hipLaunchKernelGGL(k_b_xbuild, g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_DCOEF: hipLaunchKernelGGL(k_b_dense_coef, g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_E22: hipLaunchKernelGGL(k_b_e22<false>, g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_E12_8: hipLaunchKernelGGL((k_b_e12<8, false>), g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_E12_16: hipLaunchKernelGGL((k_b_e12<16, false>), g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_E12_20: hipLaunchKernelGGL((k_b_e12<20, false>), g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_E21_8: hipLaunchKernelGGL((k_b_e21<8, false>), g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_E21_16: hipLaunchKernelGGL((k_b_e21<16, false>), g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_E21_20: hipLaunchKernelGGL((k_b_e21<20, false>), g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_E21_24: hipLaunchKernelGGL((k_b_e21<24, false>), g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_E21_32: hipLaunchKernelGGL((k_b_e21<32, false>), g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_E21S_8: hipLaunchKernelGGL((k_b_e21<8, true>), g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_E21S_16: hipLaunchKernelGGL((k_b_e21<16, true>), g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_E21S_20: hipLaunchKernelGGL((k_b_e21<20, true>), g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_E21S_24: hipLaunchKernelGGL((k_b_e21<24, true>), g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_E21S_32: hipLaunchKernelGGL((k_b_e21<32, true>), g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_E12_24: hipLaunchKernelGGL((k_b_e12<24, false>), g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_E12_32: hipLaunchKernelGGL((k_b_e12<32, false>), g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_E12F_8: hipLaunchKernelGGL((k_b_e12<8, false, true>), g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_E12F_16: hipLaunchKernelGGL((k_b_e12<16, false, true>), g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_E12F_20: hipLaunchKernelGGL((k_b_e12<20, false, true>), g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_E12F_24: hipLaunchKernelGGL((k_b_e12<24, false, true>), g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_E12F_32: hipLaunchKernelGGL((k_b_e12<32, false, true>), g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_E02: hipLaunchKernelGGL((k_b_e02<false, false>), g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_E02F: hipLaunchKernelGGL((k_b_e02<true, false>), g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_E22S: hipLaunchKernelGGL(k_b_e22<true>, g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_E12S_8: hipLaunchKernelGGL((k_b_e12<8, true>), g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_E12S_16: hipLaunchKernelGGL((k_b_e12<16, true>), g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_E12S_20: hipLaunchKernelGGL((k_b_e12<20, true>), g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_E12S_24: hipLaunchKernelGGL((k_b_e12<24, true>), g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_E12S_32: hipLaunchKernelGGL((k_b_e12<32, true>), g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_E02S: hipLaunchKernelGGL((k_b_e02<false, true>), g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_E02FS: hipLaunchKernelGGL((k_b_e02<true, true>), g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_E02COEF: hipLaunchKernelGGL(k_b_e02coef, g, b64, 0, st, insts, jobs, nj, flag, ka); break;
      case K_SIG22: hipLaunchKernelGGL((k_b_sigma<2, 2, 0>), g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_SIG12: hipLaunchKernelGGL((k_b_sigma<1, 2, 1>), g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_SIG02: hipLaunchKernelGGL((k_b_sigma<0, 2, 2>), g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_SIG21: hipLaunchKernelGGL((k_b_sigma<2, 1, 3>), g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_SIG11: hipLaunchKernelGGL((k_b_sigma<1, 1, 4>), g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_SIG01: hipLaunchKernelGGL((k_b_sigma<0, 1, 5>), g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_SIG20: hipLaunchKernelGGL((k_b_sigma<2, 0, 6>), g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_SIG10: hipLaunchKernelGGL((k_b_sigma<1, 0, 7>), g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_SIG00: hipLaunchKernelGGL((k_b_sigma<0, 0, 8>), g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_FINISH: hipLaunchKernelGGL(k_b_finish, g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_DSTAT22: hipLaunchKernelGGL((k_b_dstat<2, 2>), g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_DSTAT12: hipLaunchKernelGGL((k_b_dstat<1, 2>), g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_DSTAT02: hipLaunchKernelGGL((k_b_dstat<0, 2>), g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_DSTAT21: hipLaunchKernelGGL((k_b_dstat<2, 1>), g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_DSTAT11: hipLaunchKernelGGL((k_b_dstat<1, 1>), g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_DSTAT01: hipLaunchKernelGGL((k_b_dstat<0, 1>), g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_DSTAT20: hipLaunchKernelGGL((k_b_dstat<2, 0>), g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_DSTAT10: hipLaunchKernelGGL((k_b_dstat<1, 0>), g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_DSTAT00: hipLaunchKernelGGL((k_b_dstat<0, 0>), g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_DSTATFIN: hipLaunchKernelGGL(k_b_dstatfin, g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_BZERO: hipLaunchKernelGGL(k_b_bzero, g, b256, 0, st, insts, jobs, nj, flag, ka); break;
#define MRPT2_BROW(ID, H, V, K)                                                                    \
  case ID:                                                                                        \
    if (L.dyn_lds > 65536 &&                                                                      \
        hipFuncSetAttribute((const void*)k_b_brow<H, V, K>, hipFuncAttributeMaxDynamicSharedMemorySize, \
                            (int)L.dyn_lds) != hipSuccess)                                        \
      return MRPT2_ERR_HIP;                                                                       \
    hipLaunchKernelGGL((k_b_brow<H, V, K>), g, b256, L.dyn_lds, st, insts, jobs, nj, flag, ka);   \
    break;
      MRPT2_BROW(K_BROW22, 2, 2, 0)
      MRPT2_BROW(K_BROW12, 1, 2, 1)
      MRPT2_BROW(K_BROW02, 0, 2, 2)
      MRPT2_BROW(K_BROW21, 2, 1, 3)
      MRPT2_BROW(K_BROW11, 1, 1, 4)
      MRPT2_BROW(K_BROW01, 0, 1, 5)
      MRPT2_BROW(K_BROW20, 2, 0, 6)
      MRPT2_BROW(K_BROW10, 1, 0, 7)
      MRPT2_BROW(K_BROW00, 0, 0, 8)
#undef MRPT2_BROW
      case K_BSTR22: hipLaunchKernelGGL((k_b_bstr<2, 2, 0>), g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_BSTR12: hipLaunchKernelGGL((k_b_bstr<1, 2, 1>), g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_BSTR02: hipLaunchKernelGGL((k_b_bstr<0, 2, 2>), g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_BSTR21: hipLaunchKernelGGL((k_b_bstr<2, 1, 3>), g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_BSTR11: hipLaunchKernelGGL((k_b_bstr<1, 1, 4>), g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_BSTR01: hipLaunchKernelGGL((k_b_bstr<0, 1, 5>), g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_BSTR20: hipLaunchKernelGGL((k_b_bstr<2, 0, 6>), g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_BSTR10: hipLaunchKernelGGL((k_b_bstr<1, 0, 7>), g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_BSTR00: hipLaunchKernelGGL((k_b_bstr<0, 0, 8>), g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_BSFIN: hipLaunchKernelGGL(k_b_bsfin, g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_BECOEF: hipLaunchKernelGGL(k_b_becoef, g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_B22A: hipLaunchKernelGGL(k_b_b22a, g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_B22WR: hipLaunchKernelGGL(k_b_b22w, g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_B02R: hipLaunchKernelGGL(k_b_b02r, g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_B02S: hipLaunchKernelGGL(k_b_b02s, g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_B02W:
        if (L.dyn_lds > 65536 &&
            hipFuncSetAttribute((const void*)k_b_b02w, hipFuncAttributeMaxDynamicSharedMemorySize, (int)L.dyn_lds) !=
                hipSuccess)
          return MRPT2_ERR_HIP;
        hipLaunchKernelGGL(k_b_b02w, g, b256, L.dyn_lds, st, insts, jobs, nj, flag, ka);
        break;
      case K_B22B:
        static_assert(B22T == kB22Threads && B22HP == kB22PairsPerPart, "(2,2) string-pass shape");
        hipLaunchKernelGGL(k_b_b22b, g, dim3(B22T), 0, st, insts, jobs, nj, flag, ka);
        break;
      case K_BTRANS: hipLaunchKernelGGL(k_b_btrans, g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_B22FIN: hipLaunchKernelGGL(k_b_b22fin, g, b256, 0, st, insts, jobs, nj, flag, ka); break;
#define MRPT2_B12R(ID, MJ, ...)                                                                    \
  case ID:                                                                                        \
    if (L.dyn_lds > 65536 &&                                                                      \
        hipFuncSetAttribute((const void*)k_b_b12r<MJ __VA_ARGS__>,                                \
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)L.dyn_lds) != hipSuccess) \
      return MRPT2_ERR_HIP;                                                                       \
    hipLaunchKernelGGL((k_b_b12r<MJ __VA_ARGS__>), g, b256, L.dyn_lds, st, insts, jobs, nj, flag, ka); \
    break;
      MRPT2_B12R(K_B12R_8, 8)
      MRPT2_B12R(K_B12R_16, 16)
      MRPT2_B12R(K_B12R_24, 24)
      MRPT2_B12R(K_B12R_20, 20)
      MRPT2_B12R(K_B12R_20W, 20, , 64)
      case K_B12S_20: hipLaunchKernelGGL((k_b_b12s<20>), g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      MRPT2_B12R(K_B12R_32, 32)
#undef MRPT2_B12R
      case K_B12S_8: hipLaunchKernelGGL((k_b_b12s<8>), g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_B12S_16: hipLaunchKernelGGL((k_b_b12s<16>), g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_B12S_24: hipLaunchKernelGGL((k_b_b12s<24>), g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_B12S_32: hipLaunchKernelGGL((k_b_b12s<32>), g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_BHPP: hipLaunchKernelGGL(k_b_bhpp, g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_BXB: hipLaunchKernelGGL(k_b_bxb, g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_BAG: hipLaunchKernelGGL(k_b_bag, g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_BAG128: hipLaunchKernelGGL(k_b_bag128, g, dim3(512), 0, st, insts, jobs, nj, flag, ka); break;
      case K_BXBRED: hipLaunchKernelGGL(k_b_bxbred, g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_BAGF: hipLaunchKernelGGL(k_b_bagf, g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_BGG: hipLaunchKernelGGL(k_b_bgg, g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_BFOCK: hipLaunchKernelGGL(k_b_bfock, g, b64, 0, st, insts, jobs, nj, flag, ka); break;
      case K_BDSUM: hipLaunchKernelGGL(k_b_bdsum, g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_BHFE: hipLaunchKernelGGL(k_b_bhfe, g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_BWSYM: hipLaunchKernelGGL(k_b_bwsym, g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_BDG: hipLaunchKernelGGL(k_b_bdg, g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_BDB: hipLaunchKernelGGL(k_b_bdb, g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_BDH: hipLaunchKernelGGL(k_b_bdh, g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      case K_BDC: hipLaunchKernelGGL(k_b_bdc, g, b256, 0, st, insts, jobs, nj, flag, ka); break;
      default: return MRPT2_ERR_ARG;
    }
    tm.end(L.stage);
    HIPCHK(hipGetLastError());
  }
  return MRPT2_OK;
}

mrpt2_status read_flag(const Plan& P, const void* workspace, hipStream_t st) {
  int hflag = 0;
  HIPCHK(hipMemcpyAsync(&hflag, (const char*)workspace + P.off_flag, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  return hflag ? MRPT2_ERR_NUMERIC : MRPT2_OK;
}

// ---- block Davidson for the reference states --------------------------------
// Device buffers (one region, caller-owned): H_PP [n][n], the basis V and its
// image W = H V [mmax][n] each, restart copies of both, the Ritz vectors X and
// residuals R [k][n], and small matrices.
struct DvLayout {
  int mmax = 0;
  size_t H = 0, V = 0, W = 0, Vt = 0, Wt = 0, X = 0, R = 0, G = 0, M = 0, th = 0, sc = 0, dg = 0, total = 0;
};

DvLayout dv_layout(int64_t n, int k, bool dense = true) {
  DvLayout L;
  L.mmax = (int)std::min<int64_t>(n, std::max(6 * k, 30));
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += (bytes + 255) / 256 * 256;
    return o;
  };
  const size_t vec = (size_t)n * 16, mm = (size_t)L.mmax;
  L.H = take(dense ? (size_t)n * vec : 0);
  L.V = take(mm * vec);
  L.W = take(mm * vec);
  L.Vt = take(mm * vec);
  L.Wt = take(mm * vec);
  L.X = take((size_t)k * vec);
  L.R = take((size_t)k * vec);
  L.G = take(mm * mm * 16);
  L.M = take(mm * mm * 16);
  L.th = take(mm * 8);
  L.sc = take(mm * 16);
  L.dg = take((size_t)n * 8);
  L.total = off;
  return L;
}

// Synchronous small copies on the solver's stream (the host buffers are
// ordinary memory and are reused right after).
mrpt2_status dv_copy(void* dst, const void* src, size_t bytes, hipMemcpyKind kind, hipStream_t st) {
  HIPCHK(hipMemcpyAsync(dst, src, bytes, kind, st));
  HIPCHK(hipStreamSynchronize(st));
  return MRPT2_OK;
}

#define DVCHK(x)                          \
  do {                                    \
    const mrpt2_status s_ = (x);          \
    if (s_ != MRPT2_OK) return s_;        \
  } while (0)

// The k lowest eigenpairs of the n x n Hermitian matrix at L.H (already in
// place).  Returns MRPT2_ERR_NUMERIC when max_iter iterations leave a
// residual norm above tol (the current Ritz pairs are still written).
// With n > mmax = max(6k, 30), a restart keeps q >= 2k Ritz vectors (the
// restart happens at m > mmax - k >= 5k), so the basis never holds fewer
// than k vectors.
// dinst: the instance descriptors for the direct sigma-build in P (H_PP not
// stored), or null for the dense H_PP in the solver region.
mrpt2_status davidson(char* base, const DvLayout& L, int64_t n64, int k, double tol, int max_iter,
                      hipStream_t st, double* c_out, double* e_out, int32_t* iters, const Inst* dinst = nullptr,
                      int di = 0) {
  using cd = std::complex<double>;
  const int n = (int)n64, mmax = L.mmax;
  double2* H = (double2*)(base + L.H);
  double2* V = (double2*)(base + L.V);
  double2* W = (double2*)(base + L.W);
  double2* Vt = (double2*)(base + L.Vt);
  double2* Wt = (double2*)(base + L.Wt);
  double2* X = (double2*)(base + L.X);
  double2* R = (double2*)(base + L.R);
  double2* G = (double2*)(base + L.G);
  double2* M = (double2*)(base + L.M);
  double* th = (double*)(base + L.th);
  double2* sc = (double2*)(base + L.sc);
  double* dg = (double*)(base + L.dg);
  const dim3 b256(256);
  const unsigned nb = (unsigned)cdiv(n, 256);
  // initial basis: unit vectors at the k lowest diagonal elements
  if (dinst) hipLaunchKernelGGL(k_dv_diag_direct, dim3(nb), b256, 0, st, dinst, di, dg, n);
  else hipLaunchKernelGGL(k_dv_diag, dim3(nb), b256, 0, st, H, dg, n);
  std::vector<double> d(n);
  DVCHK(dv_copy(d.data(), dg, (size_t)n * 8, hipMemcpyDeviceToHost, st));
  std::vector<int> idx(n);
  std::iota(idx.begin(), idx.end(), 0);
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return d[a] < d[b]; });
  // a space that fits in the basis starts complete (the first Rayleigh-Ritz
  // step is then exact and no restart can shrink the basis below k vectors)
  const int m0 = n <= mmax ? n : k;
  {
    std::vector<cd> v0((size_t)m0 * n, cd(0.0, 0.0));
    for (int j = 0; j < m0; ++j) v0[(size_t)j * n + idx[j]] = 1.0;
    DVCHK(dv_copy(V, v0.data(), v0.size() * 16, hipMemcpyHostToDevice, st));
  }
  int m = m0, nnew = m0;
  std::vector<cd> S((size_t)mmax * mmax, cd(0.0, 0.0)), g((size_t)mmax * mmax), Y((size_t)mmax * mmax),
      mh((size_t)mmax * mmax);
  std::vector<double> w(mmax), rn(k);
  bool conv = false;
  int it = 0;
  for (it = 1; it <= max_iter; ++it) {
    for (int c = m - nnew; c < m; c += DV_COLS) {
      if (dinst)
        hipLaunchKernelGGL(k_dv_hx_direct, dim3((unsigned)cdiv(n, 4)), b256, 0, st, dinst, di, V, W, n, c,
                           std::min(DV_COLS, m - c));
      else
        hipLaunchKernelGGL(k_dv_hx, dim3((unsigned)cdiv(n, 4)), b256, 0, st, H, V, W, n, c, std::min(DV_COLS, m - c));
    }
    hipLaunchKernelGGL(k_dv_dots, dim3((unsigned)(m * nnew)), b256, 0, st, V, 0, W, m - nnew, nnew, n, G);
    HIPCHK(hipGetLastError());
    DVCHK(dv_copy(g.data(), G, (size_t)m * nnew * 16, hipMemcpyDeviceToHost, st));
    for (int a = 0; a < m; ++a)
      for (int b = 0; b < nnew; ++b) {
        const int col = m - nnew + b;
        S[(size_t)a * mmax + col] = g[(size_t)a * nnew + b];
        if (a < m - nnew) S[(size_t)col * mmax + a] = std::conj(g[(size_t)a * nnew + b]);
      }
    for (int a = m - nnew; a < m; ++a)          // Hermitian part of the new block
      for (int b = a; b < m; ++b) {
        const cd h = 0.5 * (S[(size_t)a * mmax + b] + std::conj(S[(size_t)b * mmax + a]));
        S[(size_t)a * mmax + b] = h;
        S[(size_t)b * mmax + a] = std::conj(h);
      }
    // Rayleigh-Ritz on the projected matrix
    std::vector<cd> sm((size_t)m * m);
    for (int a = 0; a < m; ++a)
      for (int b = 0; b < m; ++b) sm[(size_t)a * m + b] = S[(size_t)a * mmax + b];
    DVCHK(mrpt2_hermitian_eigh(m, (const double*)sm.data(), w.data(), (double*)Y.data()));
    // Ritz vectors X = V Y_k, residuals R = W Y_k - X diag(theta)
    for (int a = 0; a < m; ++a)
      for (int j = 0; j < k; ++j) mh[(size_t)a * k + j] = Y[(size_t)a * m + j];
    DVCHK(dv_copy(M, mh.data(), (size_t)m * k * 16, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_dv_comb, dim3(nb, k), b256, 0, st, V, 0, m, M, k, X, 0, 1.0, 0.0, n);
    hipLaunchKernelGGL(k_dv_comb, dim3(nb, k), b256, 0, st, W, 0, m, M, k, R, 0, 1.0, 0.0, n);
    for (int a = 0; a < k; ++a)
      for (int j = 0; j < k; ++j) mh[(size_t)a * k + j] = a == j ? cd(-w[j], 0.0) : cd(0.0, 0.0);
    DVCHK(dv_copy(M, mh.data(), (size_t)k * k * 16, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_dv_comb, dim3(nb, k), b256, 0, st, X, 0, k, M, k, R, 0, 1.0, 1.0, n);
    hipLaunchKernelGGL(k_dv_dots, dim3((unsigned)(k * k)), b256, 0, st, R, 0, R, 0, k, n, G);
    HIPCHK(hipGetLastError());
    DVCHK(dv_copy(g.data(), G, (size_t)k * k * 16, hipMemcpyDeviceToHost, st));
    std::vector<int> open;
    for (int j = 0; j < k; ++j) {
      rn[j] = std::sqrt(std::max(0.0, g[(size_t)j * k + j].real()));
      if (!std::isfinite(rn[j]) || !std::isfinite(w[j])) return MRPT2_ERR_NUMERIC;
      if (rn[j] > tol) open.push_back(j);
    }
    if (open.empty()) {
      conv = true;
      break;
    }
    if (it == max_iter) break;
    const int nu = (int)open.size();
    if (m + nu > mmax) {
      // restart on the q lowest Ritz vectors (X and R stay valid)
      const int q = std::min(std::min(m, std::max(2 * k, mmax / 2)), mmax - nu);
      for (int a = 0; a < m; ++a)
        for (int j = 0; j < q; ++j) mh[(size_t)a * q + j] = Y[(size_t)a * m + j];
      DVCHK(dv_copy(M, mh.data(), (size_t)m * q * 16, hipMemcpyHostToDevice, st));
      hipLaunchKernelGGL(k_dv_comb, dim3(nb, q), b256, 0, st, V, 0, m, M, q, Vt, 0, 1.0, 0.0, n);
      hipLaunchKernelGGL(k_dv_comb, dim3(nb, q), b256, 0, st, W, 0, m, M, q, Wt, 0, 1.0, 0.0, n);
      HIPCHK(hipMemcpyAsync(V, Vt, (size_t)q * n * 16, hipMemcpyDeviceToDevice, st));
      HIPCHK(hipMemcpyAsync(W, Wt, (size_t)q * n * 16, hipMemcpyDeviceToDevice, st));
      std::fill(S.begin(), S.end(), cd(0.0, 0.0));
      for (int j = 0; j < q; ++j) S[(size_t)j * mmax + j] = w[j];
      m = q;
    }
    // preconditioned residuals, orthonormalised (two Gram-Schmidt passes)
    // against the basis and the directions accepted before them
    std::vector<double> ths(nu);
    for (int u = 0; u < nu; ++u) ths[u] = w[open[u]];
    DVCHK(dv_copy(th, ths.data(), (size_t)nu * 8, hipMemcpyHostToDevice, st));
    int acc = 0;
    for (int u = 0; u < nu; ++u) {
      const int row = m + acc;
      hipLaunchKernelGGL(k_dv_prec, dim3(nb, 1), b256, 0, st, dg, R + (size_t)open[u] * n, th + u, V, row, n);
      hipLaunchKernelGGL(k_dv_dots, dim3(1), b256, 0, st, V, row, V, row, 1, n, G);
      HIPCHK(hipGetLastError());
      cd pre;
      DVCHK(dv_copy(&pre, G, 16, hipMemcpyDeviceToHost, st));
      for (int pass = 0; pass < 2; ++pass) {
        hipLaunchKernelGGL(k_dv_dots, dim3((unsigned)row), b256, 0, st, V, 0, V, row, 1, n, G);
        hipLaunchKernelGGL(k_dv_comb, dim3(nb, 1), b256, 0, st, V, 0, row, G, 1, V, row, -1.0, 1.0, n);
      }
      hipLaunchKernelGGL(k_dv_dots, dim3(1), b256, 0, st, V, row, V, row, 1, n, G);
      HIPCHK(hipGetLastError());
      cd post;
      DVCHK(dv_copy(&post, G, 16, hipMemcpyDeviceToHost, st));
      const double p0 = std::sqrt(std::max(0.0, pre.real())), p1 = std::sqrt(std::max(0.0, post.real()));
      if (!(p1 > 1e-8 * p0) || !(p1 > 1e-300)) continue;      // no new direction
      const cd inv(1.0 / p1, 0.0);
      DVCHK(dv_copy(sc, &inv, 16, hipMemcpyHostToDevice, st));
      hipLaunchKernelGGL(k_dv_scale, dim3(nb, 1), b256, 0, st, V, row, sc, n);
      ++acc;
    }
    nnew = acc;
    m += acc;
    if (nnew == 0) break;
  }
  // Ritz vectors: unit norm, largest component real and positive
  std::vector<cd> x((size_t)k * n);
  DVCHK(dv_copy(x.data(), X, x.size() * 16, hipMemcpyDeviceToHost, st));
  for (int j = 0; j < k; ++j) {
    cd* v = x.data() + (size_t)j * n;
    double nrm = 0.0, best = -1.0;
    int at = 0;
    for (int i = 0; i < n; ++i) {
      nrm += std::norm(v[i]);
      if (std::abs(v[i]) > best) {
        best = std::abs(v[i]);
        at = i;
      }
    }
    const cd f = std::conj(v[at]) / (std::abs(v[at]) * std::sqrt(nrm));
    for (int i = 0; i < n; ++i) v[i] *= f;
    e_out[j] = w[j];
  }
  DVCHK(dv_copy(c_out, x.data(), x.size() * 16, hipMemcpyHostToDevice, st));
  if (iters) *iters = std::min(it, max_iter);
  return conv ? MRPT2_OK : MRPT2_ERR_NUMERIC;
}

mrpt2_status energy_enqueue(mrpt2_plan_t plan, const mrpt2_inputs* in, const void* persistent, void* workspace,
                            size_t workspace_bytes, hipStream_t st, double* e2, double* parts, Timer& tm) {
  if (!plan || !in || !e2) return MRPT2_ERR_ARG;
  Plan& P = plan->p;
  mrpt2_status s = check_regions(P, persistent, workspace, workspace_bytes);
  if (s != MRPT2_OK) return s;
  s = upload_insts(P, in, (const char*)persistent, (char*)workspace, st, e2, parts, nullptr, -1);
  if (s != MRPT2_OK) return s;
  return run(P, P.energy, (const char*)persistent, (char*)workspace, st, tm);
}

}  // namespace

// ---- a workspace the library owns, for callers that cannot allocate --------
// File-scope device array: every GPU the library runs on holds its own copy
// until the process ends.  In host code its name is not a device address;
// the address is taken once per device with hipGetSymbolAddress and used
// wherever the array's memory is needed.
static __device__ __align__(256) char scratch[MRPT2_STATIC_WORKSPACE_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's array (taken on the first call
// on that device, with that device current).
mrpt2_status scratch_address(void** out) {
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return MRPT2_ERR_ARG;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return MRPT2_ERR_HIP;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return MRPT2_OK;
}

}  // namespace

extern "C" {

mrpt2_status mrpt2_plan(const mrpt2_desc* desc, int32_t n_inst, mrpt2_plan_t* out) {
  return mrpt2_plan_tuned(desc, n_inst, nullptr, out);
}

mrpt2_status mrpt2_plan_tuned(const mrpt2_desc* desc, int32_t n_inst, const mrpt2_tuning* tuning,
                              mrpt2_plan_t* out) {
  if (!out) return MRPT2_ERR_ARG;
  *out = nullptr;
  mrpt2_plan_s* p = new (std::nothrow) mrpt2_plan_s();
  if (!p) return MRPT2_ERR_ARG;
  std::string err;
  mrpt2_status st;
  try {
    st = build_plan(desc, n_inst, tuning, &p->p, &err);
  } catch (...) {
    st = MRPT2_ERR_SHAPE;
  }
  if (st != MRPT2_OK) {
    delete p;
    return st;
  }
  *out = p;
  return MRPT2_OK;
}

mrpt2_status mrpt2_plan_sizes(mrpt2_plan_t plan, size_t* pers, size_t* work) {
  if (!plan || !pers || !work) return MRPT2_ERR_ARG;
  *pers = plan->p.persistent_bytes;
  *work = plan->p.workspace_bytes;
  return MRPT2_OK;
}

mrpt2_status mrpt2_plan_upload(mrpt2_plan_t plan, void* pers, size_t bytes, hipStream_t st) {
  if (!plan || !pers) return MRPT2_ERR_ARG;
  if (bytes < plan->p.persistent_bytes) return MRPT2_ERR_WORKSPACE;
  if ((uintptr_t)pers & 255) return MRPT2_ERR_ARG;
  HIPCHK(hipMemcpyAsync(pers, plan->p.host_blob.data(), plan->p.persistent_bytes, hipMemcpyHostToDevice, st));
  return MRPT2_OK;
}

mrpt2_status mrpt2_plan_info(mrpt2_plan_t plan, int32_t inst, mrpt2_info* info) {
  if (!plan || !info || inst < 0 || inst >= (int)plan->p.inst.size()) return MRPT2_ERR_ARG;
  *info = plan->p.inst[inst].info;
  return MRPT2_OK;
}

mrpt2_status mrpt2_plan_ref_strings(mrpt2_plan_t plan, int32_t inst, uint64_t* bits) {
  if (!plan || !bits || inst < 0 || inst >= (int)plan->p.inst.size()) return MRPT2_ERR_ARG;
  const auto& v = plan->p.inst[inst].pstrings;
  std::memcpy(bits, v.data(), v.size() * 8);
  return MRPT2_OK;
}

mrpt2_status mrpt2_energy(mrpt2_plan_t plan, const mrpt2_inputs* in, const void* persistent, void* workspace,
                          size_t workspace_bytes, hipStream_t st, double* e2, double* parts) {
  Timer tm;
  mrpt2_status s = energy_enqueue(plan, in, persistent, workspace, workspace_bytes, st, e2, parts, tm);
  if (s != MRPT2_OK) return s;
  return read_flag(plan->p, workspace, st);
}

mrpt2_status mrpt2_energy_static(mrpt2_plan_t plan, const mrpt2_inputs* in, const void* persistent,
                                 hipStream_t st, double* e2, double* parts) {
  if (!plan || !in || !e2 || !persistent) return MRPT2_ERR_ARG;
  Plan& P = plan->p;
  if (P.workspace_bytes > (size_t)MRPT2_STATIC_WORKSPACE_BYTES) return MRPT2_ERR_WORKSPACE;
  if ((uintptr_t)persistent & 255) return MRPT2_ERR_ARG;
  void* work = nullptr;
  mrpt2_status s = scratch_address(&work);
  if (s != MRPT2_OK) return s;
  // descriptors staged in the plan's host buffer (sized when the plan was
  // built) and copied from there; the call ends with a stream
  // synchronisation, so the next call finds the buffer free
  s = fill_insts(P, in, (const char*)persistent, (char*)work, P.static_stage.data(), e2, parts, nullptr, -1,
                 nullptr, nullptr, nullptr);
  if (s != MRPT2_OK) return s;
  HIPCHK(hipMemcpyAsync((char*)work + P.off_insts, P.static_stage.data(), kInstBytes * P.inst.size(),
                        hipMemcpyHostToDevice, st));
  Timer tm;
  s = run(P, P.energy, (const char*)persistent, (char*)work, st, tm);
  if (s != MRPT2_OK) return s;
  return read_flag(P, work, st);
}

mrpt2_status mrpt2_static_workspace_bytes(size_t* bytes) {
  if (!bytes) return MRPT2_ERR_ARG;
  *bytes = (size_t)MRPT2_STATIC_WORKSPACE_BYTES;
  return MRPT2_OK;
}

mrpt2_status mrpt2_energy_roots(mrpt2_plan_t plan, const mrpt2_inputs* in, int32_t n_roots,
                                const void* persistent, void* workspace, size_t workspace_bytes,
                                hipStream_t st, double* e2, double* parts) {
  if (!plan || !in || !e2 || n_roots < 1) return MRPT2_ERR_ARG;
  Plan& P = plan->p;
  mrpt2_status s = check_regions(P, persistent, workspace, workspace_bytes);
  if (s != MRPT2_OK) return s;
  const size_t n = P.inst.size();
  for (size_t i = 0; i < n; ++i)
    if (!in[i].c) return MRPT2_ERR_ARG;
  s = ensure_pinned(P, (size_t)n_roots, st);
  if (s != MRPT2_OK) return s;
  std::vector<mrpt2_inputs> rin(in, in + n);
  Timer tm;
  for (int r = 0; r < n_roots; ++r) {
    for (size_t i = 0; i < n; ++i) rin[i].c = in[i].c + 2 * (size_t)r * P.inst[i].pstrings.size();
    s = upload_insts(P, rin.data(), (const char*)persistent, (char*)workspace, st, e2 + (size_t)r * n,
                     parts ? parts + (size_t)12 * r * n : nullptr, nullptr, -1, nullptr, nullptr, nullptr, r);
    if (s != MRPT2_OK) return s;
    if (r == 0) {
      s = run(P, P.energy, (const char*)persistent, (char*)workspace, st, tm, RUN_SHARED);
      if (s != MRPT2_OK) return s;
    }
    s = run(P, P.energy, (const char*)persistent, (char*)workspace, st, tm, RUN_PER_STATE);
    if (s != MRPT2_OK) return s;
  }
  return read_flag(P, workspace, st);
}

mrpt2_status mrpt2_energy_async(mrpt2_plan_t plan, const mrpt2_inputs* in, const void* persistent,
                                void* workspace, size_t workspace_bytes, hipStream_t st, double* e2,
                                double* parts) {
  Timer tm;
  return energy_enqueue(plan, in, persistent, workspace, workspace_bytes, st, e2, parts, tm);
}

mrpt2_status mrpt2_check(mrpt2_plan_t plan, const void* workspace, hipStream_t st) {
  if (!plan || !workspace) return MRPT2_ERR_ARG;
  return read_flag(plan->p, workspace, st);
}

mrpt2_status mrpt2_energy_timed(mrpt2_plan_t plan, const mrpt2_inputs* in, const void* persistent,
                                void* workspace, size_t workspace_bytes, hipStream_t st, double* e2,
                                double* parts, float* stage_ms) {
  if (!stage_ms) return MRPT2_ERR_ARG;
  Timer tm;
  tm.on = true;
  tm.st = st;
  for (int i = 0; i < 256; ++i)
    if (hipEventCreate(&tm.ev[i]) != hipSuccess) return MRPT2_ERR_HIP;
  mrpt2_status s = energy_enqueue(plan, in, persistent, workspace, workspace_bytes, st, e2, parts, tm);
  if (s == MRPT2_OK) s = read_flag(plan->p, workspace, st);
  for (int i = 0; i < ST_N; ++i) stage_ms[i] = 0.0f;
  if (s == MRPT2_OK || s == MRPT2_ERR_NUMERIC) {
    for (int i = 0; i < tm.n; ++i) {
      float ms = 0.0f;
      if (hipEventElapsedTime(&ms, tm.ev[2 * i], tm.ev[2 * i + 1]) == hipSuccess) stage_ms[tm.slot[i]] += ms;
    }
  }
  for (int i = 0; i < 256; ++i) hipEventDestroy(tm.ev[i]);
  return s;
}

mrpt2_status mrpt2_delta_stats(mrpt2_plan_t plan, const mrpt2_inputs* in, const void* persistent, void* workspace,
                               size_t workspace_bytes, hipStream_t st, double thresh, double* min_abs_delta,
                               int64_t* n_below) {
  if (!plan || !in || !min_abs_delta || !(thresh >= 0.0) || !std::isfinite(thresh)) return MRPT2_ERR_ARG;
  Plan& P = plan->p;
  mrpt2_status s = check_regions(P, persistent, workspace, workspace_bytes);
  if (s != MRPT2_OK) return s;
  P.dstat_thresh = thresh;
  s = upload_insts(P, in, (const char*)persistent, (char*)workspace, st, nullptr, nullptr, nullptr, -1);
  if (s != MRPT2_OK) return s;
  Timer tm;
  s = run(P, P.stats, (const char*)persistent, (char*)workspace, st, tm);
  if (s != MRPT2_OK) return s;
  s = read_flag(P, workspace, st);
  if (s != MRPT2_OK) return s;
  for (size_t i = 0; i < P.inst.size(); ++i) {
    double2 v[MRPT2_N_CLASS];
    HIPCHK(hipMemcpyAsync(v, (const char*)workspace + P.inst[i].workspace_base + P.inst[i].off_dstat_out,
                          sizeof(v), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (int k = 0; k < MRPT2_N_CLASS; ++k) {
      const bool empty = P.inst[i].cls[k].n_dstat == 0;
      min_abs_delta[i * MRPT2_N_CLASS + k] = empty ? HUGE_VAL : v[k].x;
      if (n_below) n_below[i * MRPT2_N_CLASS + k] = empty ? 0 : (int64_t)v[k].y;
    }
  }
  return MRPT2_OK;
}

mrpt2_status mrpt2_plan_backward_size(mrpt2_plan_t plan, size_t* grad_workspace_bytes) {
  if (!plan || !grad_workspace_bytes) return MRPT2_ERR_ARG;
  *grad_workspace_bytes = plan->p.grad_bytes;
  return MRPT2_OK;
}

static mrpt2_status backward_enqueue(mrpt2_plan_t plan, const mrpt2_inputs* in, const void* persistent,
                                     void* workspace, size_t workspace_bytes, void* grad_workspace,
                                     size_t grad_workspace_bytes, const double* grad_e2, const mrpt2_grads* grads,
                                     hipStream_t st, double* e2, Timer& tm) {
  if (!plan || !in || !grads || !grad_e2 || !grad_workspace) return MRPT2_ERR_ARG;
  Plan& P = plan->p;
  mrpt2_status s = check_regions(P, persistent, workspace, workspace_bytes);
  if (s != MRPT2_OK) return s;
  if (grad_workspace_bytes < P.grad_bytes) return MRPT2_ERR_WORKSPACE;
  if ((uintptr_t)grad_workspace & 255) return MRPT2_ERR_ARG;
  s = upload_insts(P, in, (const char*)persistent, (char*)workspace, st, e2, nullptr, nullptr, -1,
                   (char*)grad_workspace, grads, grad_e2);
  if (s != MRPT2_OK) return s;
  return run(P, P.backward, (const char*)persistent, (char*)workspace, st, tm);
}

mrpt2_status mrpt2_energy_backward(mrpt2_plan_t plan, const mrpt2_inputs* in, const void* persistent,
                                   void* workspace, size_t workspace_bytes, void* grad_workspace,
                                   size_t grad_workspace_bytes, const double* grad_e2, const mrpt2_grads* grads,
                                   hipStream_t st, double* e2) {
  Timer tm;
  mrpt2_status s = backward_enqueue(plan, in, persistent, workspace, workspace_bytes, grad_workspace,
                                    grad_workspace_bytes, grad_e2, grads, st, e2, tm);
  if (s != MRPT2_OK) return s;
  return read_flag(plan->p, workspace, st);
}

mrpt2_status mrpt2_energy_backward_async(mrpt2_plan_t plan, const mrpt2_inputs* in, const void* persistent,
                                         void* workspace, size_t workspace_bytes, void* grad_workspace,
                                         size_t grad_workspace_bytes, const double* grad_e2,
                                         const mrpt2_grads* grads, hipStream_t st, double* e2) {
  Timer tm;
  return backward_enqueue(plan, in, persistent, workspace, workspace_bytes, grad_workspace, grad_workspace_bytes,
                          grad_e2, grads, st, e2, tm);
}

mrpt2_status mrpt2_energy_backward_timed(mrpt2_plan_t plan, const mrpt2_inputs* in, const void* persistent,
                                         void* workspace, size_t workspace_bytes, void* grad_workspace,
                                         size_t grad_workspace_bytes, const double* grad_e2,
                                         const mrpt2_grads* grads, hipStream_t st, double* e2, float* stage_ms) {
  if (!stage_ms) return MRPT2_ERR_ARG;
  Timer tm;
  tm.on = true;
  tm.st = st;
  for (int i = 0; i < 256; ++i)
    if (hipEventCreate(&tm.ev[i]) != hipSuccess) return MRPT2_ERR_HIP;
  mrpt2_status s = backward_enqueue(plan, in, persistent, workspace, workspace_bytes, grad_workspace,
                                    grad_workspace_bytes, grad_e2, grads, st, e2, tm);
  if (s == MRPT2_OK) s = read_flag(plan->p, workspace, st);
  for (int i = 0; i < ST_NB; ++i) stage_ms[i] = 0.0f;
  if (s == MRPT2_OK || s == MRPT2_ERR_NUMERIC) {
    for (int i = 0; i < tm.n; ++i) {
      float ms = 0.0f;
      if (hipEventElapsedTime(&ms, tm.ev[2 * i], tm.ev[2 * i + 1]) == hipSuccess) stage_ms[tm.slot[i]] += ms;
    }
  }
  for (int i = 0; i < 256; ++i) hipEventDestroy(tm.ev[i]);
  return s;
}

mrpt2_status mrpt2_reference_hamiltonian(mrpt2_plan_t plan, int32_t inst, const mrpt2_inputs* in,
                                         const void* persistent, void* workspace, size_t workspace_bytes,
                                         hipStream_t st, double* hpp) {
  if (!plan || !in || !hpp || inst < 0 || inst >= (int)plan->p.inst.size()) return MRPT2_ERR_ARG;
  Plan& P = plan->p;
  mrpt2_status s = check_regions(P, persistent, workspace, workspace_bytes);
  if (s != MRPT2_OK) return s;
  s = upload_insts(P, in, (const char*)persistent, (char*)workspace, st, nullptr, nullptr, hpp, inst);
  if (s != MRPT2_OK) return s;
  Timer tm;
  s = run(P, P.reference[inst], (const char*)persistent, (char*)workspace, st, tm);
  if (s != MRPT2_OK) return s;
  return read_flag(P, workspace, st);
}

mrpt2_status mrpt2_reference_states_size(mrpt2_plan_t plan, int32_t inst, int32_t n_states, size_t* bytes) {
  if (!plan || !bytes || inst < 0 || inst >= (int)plan->p.inst.size() || n_states < 1) return MRPT2_ERR_ARG;
  const int64_t n = (int64_t)plan->p.inst[inst].pstrings.size();
  if (n_states > n) return MRPT2_ERR_ARG;
  *bytes = dv_layout(n, n_states).total;
  return MRPT2_OK;
}

mrpt2_status mrpt2_reference_states(mrpt2_plan_t plan, int32_t inst, const mrpt2_inputs* in, int32_t n_states,
                                    double tol, int32_t max_iter, const void* persistent, void* workspace,
                                    size_t workspace_bytes, void* dv, size_t dv_bytes, hipStream_t st,
                                    double* c_out, double* e_out, int32_t* iterations) {
  if (!plan || !in || !dv || !c_out || !e_out || inst < 0 || inst >= (int)plan->p.inst.size() || n_states < 1 ||
      max_iter < 1 || !(tol > 0.0))
    return MRPT2_ERR_ARG;
  Plan& P = plan->p;
  const int64_t n = (int64_t)P.inst[inst].pstrings.size();
  if (n_states > n || n > INT32_MAX / 4) return MRPT2_ERR_ARG;
  mrpt2_status s = check_regions(P, persistent, workspace, workspace_bytes);
  if (s != MRPT2_OK) return s;
  const DvLayout L = dv_layout(n, n_states);
  if (dv_bytes < L.total) return MRPT2_ERR_WORKSPACE;
  if ((uintptr_t)dv & 255) return MRPT2_ERR_ARG;
  char* base = (char*)dv;
  // H_PP - E_core from the Slater-Condon rules (as mrpt2_reference_hamiltonian)
  s = upload_insts(P, in, (const char*)persistent, (char*)workspace, st, nullptr, nullptr, (double*)(base + L.H), inst);
  if (s != MRPT2_OK) return s;
  Timer tm;
  s = run(P, P.reference[inst], (const char*)persistent, (char*)workspace, st, tm);
  if (s != MRPT2_OK) return s;
  s = read_flag(P, workspace, st);
  if (s != MRPT2_OK) return s;
  return davidson(base, L, n, n_states, tol, max_iter, st, c_out, e_out, iterations);
}

// Tables of one instance (factor pass, orbital energies, pair energies,
// occupied-block integrals; no H_PP) for the direct sigma-build in P.
static mrpt2_status reference_tables(Plan& P, int32_t inst, const mrpt2_inputs* in, const void* persistent,
                                     void* workspace, size_t workspace_bytes, hipStream_t st) {
  mrpt2_status s = check_regions(P, persistent, workspace, workspace_bytes);
  if (s != MRPT2_OK) return s;
  s = upload_insts(P, in, (const char*)persistent, (char*)workspace, st, nullptr, nullptr, nullptr, inst);
  if (s != MRPT2_OK) return s;
  Timer tm;
  s = run(P, P.reference_tables[inst], (const char*)persistent, (char*)workspace, st, tm);
  if (s != MRPT2_OK) return s;
  return read_flag(P, workspace, st);
}

mrpt2_status mrpt2_reference_sigma(mrpt2_plan_t plan, int32_t inst, const mrpt2_inputs* in, int32_t n_vec,
                                   const double* x, const void* persistent, void* workspace,
                                   size_t workspace_bytes, hipStream_t st, double* y) {
  if (!plan || !in || !x || !y || x == y || n_vec < 1 || inst < 0 || inst >= (int)plan->p.inst.size())
    return MRPT2_ERR_ARG;
  Plan& P = plan->p;
  const int64_t n = (int64_t)P.inst[inst].pstrings.size();
  if (n > INT32_MAX / 4) return MRPT2_ERR_ARG;
  mrpt2_status s = reference_tables(P, inst, in, persistent, workspace, workspace_bytes, st);
  if (s != MRPT2_OK) return s;
  const Inst* insts = (const Inst*)((const char*)workspace + P.off_insts);
  for (int c = 0; c < n_vec; c += DV_COLS)
    hipLaunchKernelGGL(k_dv_hx_direct, dim3((unsigned)cdiv(n, 4)), dim3(256), 0, st, insts, inst, (const double2*)x,
                       (double2*)y, (int)n, c, std::min(DV_COLS, n_vec - c));
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(st));
  return MRPT2_OK;
}

mrpt2_status mrpt2_reference_states_direct_size(mrpt2_plan_t plan, int32_t inst, int32_t n_states,
                                                size_t* bytes) {
  if (!plan || !bytes || inst < 0 || inst >= (int)plan->p.inst.size() || n_states < 1) return MRPT2_ERR_ARG;
  const int64_t n = (int64_t)plan->p.inst[inst].pstrings.size();
  if (n_states > n) return MRPT2_ERR_ARG;
  *bytes = dv_layout(n, n_states, false).total;
  return MRPT2_OK;
}

mrpt2_status mrpt2_reference_states_direct(mrpt2_plan_t plan, int32_t inst, const mrpt2_inputs* in,
                                           int32_t n_states, double tol, int32_t max_iter, const void* persistent,
                                           void* workspace, size_t workspace_bytes, void* dv, size_t dv_bytes,
                                           hipStream_t st, double* c_out, double* e_out, int32_t* iterations) {
  if (!plan || !in || !dv || !c_out || !e_out || inst < 0 || inst >= (int)plan->p.inst.size() || n_states < 1 ||
      max_iter < 1 || !(tol > 0.0))
    return MRPT2_ERR_ARG;
  Plan& P = plan->p;
  const int64_t n = (int64_t)P.inst[inst].pstrings.size();
  if (n_states > n || n > INT32_MAX / 4) return MRPT2_ERR_ARG;
  const DvLayout L = dv_layout(n, n_states, false);
  if (dv_bytes < L.total) return MRPT2_ERR_WORKSPACE;
  if ((uintptr_t)dv & 255) return MRPT2_ERR_ARG;
  mrpt2_status s = reference_tables(P, inst, in, persistent, workspace, workspace_bytes, st);
  if (s != MRPT2_OK) return s;
  const Inst* insts = (const Inst*)((const char*)workspace + P.off_insts);
  return davidson((char*)dv, L, n, n_states, tol, max_iter, st, c_out, e_out, iterations, insts, inst);
}

mrpt2_status mrpt2_plan_class_blocks(mrpt2_plan_t plan, int32_t inst, int32_t cls, int64_t* n_blocks) {
  if (!plan || !n_blocks || inst < 0 || inst >= (int)plan->p.inst.size() || cls < 0 || cls >= MRPT2_N_CLASS)
    return MRPT2_ERR_ARG;
  const ClassPlan& cp = plan->p.inst[inst].cls[cls];
  *n_blocks = (cp.strings.empty() || cp.n_rows == 0) ? 0 : cp.n_blocks;
  return MRPT2_OK;
}

mrpt2_status mrpt2_plan_class_block(mrpt2_plan_t plan, int32_t inst, int32_t cls, int64_t block,
                                    mrpt2_block* out) {
  int64_t nb = 0;
  mrpt2_status s = mrpt2_plan_class_blocks(plan, inst, cls, &nb);
  if (s != MRPT2_OK) return s;
  if (!out || block < 0 || block >= nb) return MRPT2_ERR_ARG;
  class_block(plan->p.inst[inst], cls, block, out);
  return MRPT2_OK;
}

mrpt2_status mrpt2_plan_class_strings(mrpt2_plan_t plan, int32_t inst, int32_t cls, uint64_t* bits) {
  if (!plan || !bits || inst < 0 || inst >= (int)plan->p.inst.size() || cls < 0 || cls >= MRPT2_N_CLASS)
    return MRPT2_ERR_ARG;
  const auto& v = plan->p.inst[inst].cls[cls].strings;
  if (!v.empty()) std::memcpy(bits, v.data(), v.size() * 8);
  return MRPT2_OK;
}

mrpt2_status mrpt2_class_partials(mrpt2_plan_t plan, int32_t inst, int32_t cls, const void* workspace,
                                  hipStream_t st, double* out) {
  int64_t nb = 0;
  mrpt2_status s = mrpt2_plan_class_blocks(plan, inst, cls, &nb);
  if (s != MRPT2_OK) return s;
  if (!workspace || !out) return MRPT2_ERR_ARG;
  const InstancePlan& ip = plan->p.inst[inst];
  const char* src = (const char*)workspace + ip.workspace_base + ip.off_part_class[cls];
  if (nb > 0) {
    HIPCHK(hipMemcpyAsync(out, src, (size_t)nb * 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
  }
  return MRPT2_OK;
}

void mrpt2_plan_destroy(mrpt2_plan_t plan) {
  if (!plan) return;
  if (plan->p.pinned) (void)hipHostFree(plan->p.pinned);
  if (plan->p.staged) (void)hipEventDestroy(plan->p.staged);
  delete plan;
}

const char* mrpt2_status_string(mrpt2_status s) {
  switch (s) {
    case MRPT2_OK: return "ok";
    case MRPT2_ERR_ARG: return "invalid argument";
    case MRPT2_ERR_SHAPE: return "inconsistent or unsupported sizes";
    case MRPT2_ERR_UNSUPPORTED: return "unsupported option";
    case MRPT2_ERR_WORKSPACE: return "persistent or workspace region too small";
    case MRPT2_ERR_HIP: return "HIP runtime error";
    case MRPT2_ERR_NUMERIC: return "non-finite input or zero denominator";
  }
  return "unknown status";
}

}  // extern "C"
