// C interface: plan management and the launch sequence of one energy
// evaluation (tables -> reference energy -> integral builds -> per-class
// sigma contraction with the Epstein-Nesbet epilogue -> reductions).
#include <hip/hip_runtime.h>

#include <cstring>
#include <new>
#include <string>

#include "kernels.hpp"
#include "mrpt2.h"
#include "plan.hpp"

#include "kernels_tables.hip"
#include "kernels_energy.hip"

struct mrpt2_plan_s {
  mrpt2::Plan p;
};

using namespace mrpt2;

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
  d.hole_pairs = (const int32_t*)(P + ip.off_hole_pairs);
  d.tile_pairs = (const int32_t*)(P + ip.off_tile_pairs);
  d.dg = (double*)(W + ip.off_dg);
  d.slab = (double2*)(W + ip.off_slab);
  d.W = (double*)(W + ip.off_W);
  d.eps = (double*)(W + ip.off_eps);
  d.f = (double2*)(W + ip.off_f);
  d.G = (double2*)(W + ip.off_G);
  d.A = (double2*)(W + ip.off_A);
  d.hpp = (double2*)(W + ip.off_hpp);
  d.sigp = (double2*)(W + ip.off_sigp);
  d.scal = (double*)(W + ip.off_scal);
  d.dsum = (double*)(W + ip.off_dsum);
  d.c = in ? (const double2*)in->c : nullptr;
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
  c.strings = (const uint64_t*)(P + cp.off_strings);
  c.conn_ptr = (const int32_t*)(P + cp.off_conn_ptr);
  c.conn = (const int32_t*)(P + cp.off_conn);
  c.pat = (const Pattern*)(P + cp.off_pat);
  c.T = (double*)(W + cp.off_T);
  c.Uc = (double*)(W + cp.off_Uc);
  c.Uv = (double*)(W + cp.off_Uv);
  c.X = (double2*)(W + cp.off_X);
  c.D = (double2*)(W + cp.off_D);
  c.mask = (uint32_t*)(W + cp.off_mask);
  c.part = (double*)(W + ip.off_part_class[k]);
  const int64_t rb = cdiv(cp.n_rows, 256);
  c.nsc = rb > 0 ? (int)(sigma_blocks(ip, k) / rb) : 1;
  return c;
}

// Steps shared by the energy and the reference Hamiltonian: factor slabs,
// pair energies, orbital energies, core Fock matrix, occupied integrals.
// Timing slots of mrpt2_energy_timed (milliseconds, summed over instances).
enum {
  ST_TABLES = 0, ST_GBUILD = 1, ST_REF = 2, ST_ABUILD = 3, ST_SIGMA0 = 4,       // 4..12 sigma per class
  ST_PREP0 = 13,                                                               // 13..21 class tables + couplings
  ST_FINISH = 22, ST_N = 23
};

struct Timer {
  hipEvent_t ev[2 * ST_N * 8];
  int slot[ST_N * 8];
  int n = 0;
  bool on = false;
  hipStream_t st;
  int open_slot = -1;
  void begin(int s) {
    if (!on || n >= ST_N * 8) return;
    slot[n] = s;
    hipEventRecord(ev[2 * n], st);
    open_slot = n;
  }
  void end() {
    if (!on || open_slot < 0) return;
    hipEventRecord(ev[2 * open_slot + 1], st);
    ++n;
    open_slot = -1;
  }
};

mrpt2_status tables(const InstancePlan& ip, const mrpt2_inputs* in, Dev& d, hipStream_t st, int* flag,
                    Timer* tm) {
  SetPtrs sp{};
  sp.n_sets = ip.d.n_sets;
  int l0 = 0;
  for (int t = 0; t < ip.d.n_sets; ++t) {
    const int rank = ip.d.rank[t];
    const double2* B = (const double2*)in->B[t];
    if (rank > 0 && !B) return MRPT2_ERR_ARG;
    sp.B[t] = B;
    sp.rank[t] = rank;
    sp.l0[t] = l0;
    if (rank > 0) {
      hipLaunchKernelGGL(k_pack, dim3(cdiv(rank, 64), ip.n_corr), dim3(256), 0, st, d, B, l0, rank);
      hipLaunchKernelGGL(k_diag, dim3(cdiv(ip.n, 256), rank), dim3(256), 0, st, d, B, l0, rank);
    }
    l0 += rank;
  }
  hipLaunchKernelGGL(k_wpass, dim3(cdiv(ip.n, 256), ip.n), dim3(256), 0, st, d, sp, flag);
  hipLaunchKernelGGL(k_eps, dim3(cdiv(ip.n_corr, 256)), dim3(256), 0, st, d, (const double2*)in->h, flag);
  hipLaunchKernelGGL(k_dsum, dim3(cdiv(ip.n_l, 256)), dim3(256), 0, st, d);
  if (ip.n_o > 0 && ip.n_a + ip.n_v > 0)
    hipLaunchKernelGGL(k_fock, dim3(ip.n_o, ip.n_a + ip.n_v), dim3(64), 0, st, d, (const double2*)in->h);
  tm->end();
  tm->begin(ST_GBUILD);
  if (ip.n_a > 0) {
    const int64_t M = (int64_t)ip.n_o * (ip.n_a + ip.n_v), N = (int64_t)ip.n_o * ip.n_a;
    hipLaunchKernelGGL(k_gbuild, dim3(cdiv(N, 64), cdiv(M, 64)), dim3(256), 0, st, d);
  }
  tm->end();
  HIPCHK(hipGetLastError());
  return MRPT2_OK;
}

mrpt2_status check_regions(const Plan& p, const void* pers, void* work, size_t wbytes) {
  if (!pers || !work) return MRPT2_ERR_ARG;
  if (wbytes < p.workspace_bytes) return MRPT2_ERR_WORKSPACE;
  if (((uintptr_t)pers & 255) || ((uintptr_t)work & 255)) return MRPT2_ERR_ARG;
  return MRPT2_OK;
}

mrpt2_status run_energy(mrpt2_plan_t plan, const mrpt2_inputs* in, const void* persistent, void* workspace,
                        size_t workspace_bytes, hipStream_t st, double* e2, double* parts, Timer& tm) {
  if (!plan || !in || !e2) return MRPT2_ERR_ARG;
  const Plan& P = plan->p;
  mrpt2_status s = check_regions(P, persistent, workspace, workspace_bytes);
  if (s != MRPT2_OK) return s;
  const char* pers = (const char*)persistent;
  char* work = (char*)workspace;
  int* flag = (int*)(work + P.off_flag);
  hipLaunchKernelGGL(k_clear_flag, dim3(1), dim3(64), 0, st, flag);
  for (size_t ii = 0; ii < P.inst.size(); ++ii) {
    const InstancePlan& ip = P.inst[ii];
    const mrpt2_inputs* ini = in + ii;
    if (!ini->h || !ini->c) return MRPT2_ERR_ARG;
    Dev d = make_dev(ip, pers, work, ini);
    tm.begin(ST_TABLES);
    s = tables(ip, ini, d, st, flag, &tm);
    if (s != MRPT2_OK) return s;
    const int np = (int)ip.pstrings.size();
    tm.begin(ST_REF);
    hipLaunchKernelGGL(k_hpp, dim3(cdiv(np, 16), cdiv(np, 16)), dim3(16, 16), 0, st, d, d.hpp);
    hipLaunchKernelGGL(k_sigp, dim3(np), dim3(64), 0, st, d, (const double2*)d.hpp);
    hipLaunchKernelGGL(k_e0, dim3(1), dim3(256), 0, st, d, flag);
    tm.end();
    if (ip.n_v >= 2 && ip.n_pairs > 0) {
      tm.begin(ST_ABUILD);
      if (ip.d.precision == MRPT2_MIXED)
        hipLaunchKernelGGL(k_abuild_f32, dim3(ip.n_tp, ip.n_pairs), dim3(256), 0, st, d);
      else
        hipLaunchKernelGGL(k_abuild, dim3(ip.n_tp, ip.n_pairs), dim3(256), 0, st, d);
      tm.end();
    }
    PartList pl{};
    for (int k = 0; k < MRPT2_N_CLASS; ++k) {
      const ClassPlan& cp = ip.cls[k];
      ClassDev cd = make_class(ip, k, pers, work);
      pl.p[k] = cd.part;
      pl.n[k] = 0;
      if (cp.strings.empty() || cp.n_rows == 0) continue;
      const int mx = std::max(ip.n_c, ip.n_v);
      tm.begin(ST_PREP0 + k);
      hipLaunchKernelGGL(k_class_tables, dim3(cd.n_str, cdiv(std::max(mx, 1), 256)), dim3(256), 0, st, d, cd);
      if (cp.v < 2 && cd.n_pat > 0)
        hipLaunchKernelGGL(k_xbuild, dim3(cdiv(cp.n_rows, 256), cd.n_pat), dim3(256), 0, st, d, cd);
      tm.end();
      const int64_t nb = sigma_blocks(ip, k);
      pl.n[k] = nb;
      dim3 g(nb), b(256);
      tm.begin(ST_SIGMA0 + k);
      pl.n[k] = cp.n_blocks;
      if (cp.kernel == KERN_E22) {
        // dedicated vector kernel: one block per (virtual tile pair, core pair)
        hipLaunchKernelGGL(k_e22, dim3(ip.n_tp, cp.n_holes), dim3(256), 0, st, d, cd, flag);
        tm.end();
        continue;
      }
      if (cp.kernel == KERN_E12) {
        // one core hole, two virtual electrons: coefficients densified per
        // string, couplings held in registers; one block per (tile pair, core)
        hipLaunchKernelGGL(k_dense_coef, dim3(cdiv(cd.n_str, 256)), dim3(256), 0, st, d, cd);
        const dim3 g12(ip.n_tp * 16, cp.n_holes);
        if (cd.n_pat <= 8) hipLaunchKernelGGL((k_e12<8>), g12, dim3(256), 0, st, d, cd, flag);
        else if (cd.n_pat <= 16) hipLaunchKernelGGL((k_e12<16>), g12, dim3(256), 0, st, d, cd, flag);
        else if (cd.n_pat <= 24) hipLaunchKernelGGL((k_e12<24>), g12, dim3(256), 0, st, d, cd, flag);
        else hipLaunchKernelGGL((k_e12<32>), g12, dim3(256), 0, st, d, cd, flag);
        tm.end();
        continue;
      }
      if (cp.kernel == KERN_E02) {
        // no core hole, two virtual electrons: couplings of a 32-row block in LDS
        if (hipFuncSetAttribute((const void*)k_e02, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)kE02MaxLds) != hipSuccess)
          return MRPT2_ERR_HIP;
        hipLaunchKernelGGL(k_e02, dim3(ip.n_tp * 128), dim3(256), (size_t)cd.n_pat * 512, st, d, cd, flag);
        tm.end();
        continue;
      }
      switch (k) {
        case 0: hipLaunchKernelGGL((k_sigma<2, 2>), g, b, 0, st, d, cd, flag); break;
        case 1: hipLaunchKernelGGL((k_sigma<1, 2>), g, b, 0, st, d, cd, flag); break;
        case 2: hipLaunchKernelGGL((k_sigma<0, 2>), g, b, 0, st, d, cd, flag); break;
        case 3: hipLaunchKernelGGL((k_sigma<2, 1>), g, b, 0, st, d, cd, flag); break;
        case 4: hipLaunchKernelGGL((k_sigma<1, 1>), g, b, 0, st, d, cd, flag); break;
        case 5: hipLaunchKernelGGL((k_sigma<0, 1>), g, b, 0, st, d, cd, flag); break;
        case 6: hipLaunchKernelGGL((k_sigma<2, 0>), g, b, 0, st, d, cd, flag); break;
        case 7: hipLaunchKernelGGL((k_sigma<1, 0>), g, b, 0, st, d, cd, flag); break;
        default: hipLaunchKernelGGL((k_sigma<0, 0>), g, b, 0, st, d, cd, flag); break;
      }
      tm.end();
    }
    tm.begin(ST_FINISH);
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(256), 0, st, d, pl, parts ? parts + 12 * ii : nullptr, e2 + ii);
    tm.end();
    HIPCHK(hipGetLastError());
  }
  int hflag = 0;
  HIPCHK(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  return hflag ? MRPT2_ERR_NUMERIC : MRPT2_OK;
}

}  // namespace

extern "C" {

mrpt2_status mrpt2_plan(const mrpt2_desc* desc, int32_t n_inst, mrpt2_plan_t* out) {
  if (!out) return MRPT2_ERR_ARG;
  *out = nullptr;
  mrpt2_plan_s* p = new (std::nothrow) mrpt2_plan_s();
  if (!p) return MRPT2_ERR_ARG;
  std::string err;
  mrpt2_status st;
  try {
    st = build_plan(desc, n_inst, &p->p, &err);
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
  tm.on = false;
  return run_energy(plan, in, persistent, workspace, workspace_bytes, st, e2, parts, tm);
}

mrpt2_status mrpt2_energy_timed(mrpt2_plan_t plan, const mrpt2_inputs* in, const void* persistent,
                                void* workspace, size_t workspace_bytes, hipStream_t st, double* e2,
                                double* parts, float* stage_ms) {
  if (!stage_ms) return MRPT2_ERR_ARG;
  Timer tm;
  tm.on = true;
  tm.st = st;
  const int nev = 2 * ST_N * 8;
  for (int i = 0; i < nev; ++i)
    if (hipEventCreate(&tm.ev[i]) != hipSuccess) return MRPT2_ERR_HIP;
  mrpt2_status s = run_energy(plan, in, persistent, workspace, workspace_bytes, st, e2, parts, tm);
  for (int i = 0; i < ST_N; ++i) stage_ms[i] = 0.0f;
  if (s == MRPT2_OK || s == MRPT2_ERR_NUMERIC) {
    for (int i = 0; i < tm.n; ++i) {
      float ms = 0.0f;
      if (hipEventElapsedTime(&ms, tm.ev[2 * i], tm.ev[2 * i + 1]) == hipSuccess) stage_ms[tm.slot[i]] += ms;
    }
  }
  for (int i = 0; i < nev; ++i) hipEventDestroy(tm.ev[i]);
  return s;
}

mrpt2_status mrpt2_reference_hamiltonian(mrpt2_plan_t plan, int32_t inst, const mrpt2_inputs* in,
                                         const void* persistent, void* workspace, size_t workspace_bytes,
                                         hipStream_t st, double* hpp) {
  if (!plan || !in || !hpp || inst < 0 || inst >= (int)plan->p.inst.size()) return MRPT2_ERR_ARG;
  const Plan& P = plan->p;
  mrpt2_status s = check_regions(P, persistent, workspace, workspace_bytes);
  if (s != MRPT2_OK) return s;
  char* work = (char*)workspace;
  int* flag = (int*)(work + P.off_flag);
  const InstancePlan& ip = P.inst[inst];
  if (!in->h) return MRPT2_ERR_ARG;
  Dev d = make_dev(ip, (const char*)persistent, work, in);
  hipLaunchKernelGGL(k_clear_flag, dim3(1), dim3(64), 0, st, flag);
  Timer tm;
  s = tables(ip, in, d, st, flag, &tm);
  if (s != MRPT2_OK) return s;
  const int np = (int)ip.pstrings.size();
  hipLaunchKernelGGL(k_hpp, dim3(cdiv(np, 16), cdiv(np, 16)), dim3(16, 16), 0, st, d, (double2*)hpp);
  HIPCHK(hipGetLastError());
  int hflag = 0;
  HIPCHK(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  return hflag ? MRPT2_ERR_NUMERIC : MRPT2_OK;
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

void mrpt2_plan_destroy(mrpt2_plan_t plan) { delete plan; }

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
