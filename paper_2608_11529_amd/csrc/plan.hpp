// Host-side plan: STP-DAS string spaces, excitation lists and the device
// memory layout of one MRPT2 energy evaluation.
#pragma once
#include <cstdint>
#include <string>
#include <unordered_map>
#include <vector>

#include "mrpt2.h"

namespace mrpt2 {

constexpr int kTile = 64;           // virtual tile edge of the pair-integral blocks
constexpr int kMaxAct = 64;         // active spinors fit one 64-bit string
constexpr int kMaxDenseJ = 32;      // patterns held in registers by the dense-coefficient kernels

// Excitation classes, indexed as in mrpt2_info.
constexpr int kClassH[MRPT2_N_CLASS] = {2, 1, 0, 2, 1, 0, 2, 1, 0};
constexpr int kClassV[MRPT2_N_CLASS] = {2, 2, 2, 1, 1, 1, 0, 0, 0};

// Pattern kinds: how the active part of an external string is reached from a
// reference string, and which integral multiplies the coefficient.
enum PatKind : int32_t {
  PAT_DOUBLE = 0,   // rank-2: active annihilations A, creations R
  PAT_SINGLE = 1,   // rank-1 one-body part (f^core)
  PAT_SPECT = 2     // rank-1 two-body part with spectator w
};

// One pattern: up to two active annihilations (a0 < a1), up to two active
// creations (r0 < r1), a spectator w.  -1 marks an unused slot.
struct Pattern {
  int32_t kind, a0, a1, r0, r1, w, pad0, pad1;
};

struct ClassPlan {
  int h = 0, v = 0;
  std::vector<uint64_t> strings;       // active strings of external dets
  std::vector<Pattern> patterns;
  std::vector<int32_t> conn_ptr;       // CSR over strings
  std::vector<int32_t> conn;           // pairs (beta | sign<<31, pattern id)
  std::vector<int32_t> ekey;           // per coupling: integral key (see coupling_key) | sign<<31
  int64_t n_holes = 0;                 // C(n_c, h)
  int64_t n_rows = 0;                  // rows of the sigma matrix (holes x virtual tuples)
  int64_t n_ext = 0;                   // exact determinant count
  int64_t n_conn = 0;
  // device offsets (bytes) within the instance's persistent region
  size_t off_strings = 0, off_conn_ptr = 0, off_conn = 0, off_pat = 0, off_ekey = 0;
  // device offsets within the instance's workspace
  size_t off_T = 0, off_Uc = 0, off_Uv = 0, off_X = 0, off_D = 0, off_mask = 0;
  // gradient workspace offsets (adjoint): coupling adjoints, string-pass partials
  size_t off_Xb = 0, off_Tb = 0, off_cbe = 0, off_r1 = 0, off_dbp = 0, off_ecoef = 0, off_wpart = 0;
  size_t off_UvT = 0, off_UcT = 0, off_u2 = 0;
  size_t off_e2part = 0;               // adjoint: per row-pass block, its share of E2
  size_t off_Xbp = 0;                  // private coupling-adjoint partials per string chunk (or 0 bytes)
  bool xb_private = false;
  int64_t n_e2part = 0;
  int parts = 1;                       // row parts of the string-owned adjoint pass
  int64_t rows_per_part = 0;           // rows per part (tile pairs per part for the (1,2) kernels)
  int row_split = 1;                   // string chunks of the generic row-owned adjoint pass
  bool dense_coef = false;             // coefficients as a dense [S][n_pat] table + masks
  // class (0,2) contraction kernel: tiles of at most 64 consecutive strings of
  // one occupation category; a tile's support is the union of the active
  // pairs its strings couple through
  std::vector<int32_t> tile_s0;        // [n_tiles + 1] first string of each tile
  std::vector<int32_t> tile_k0;        // [n_tiles + 1] first support column (counts padded to even)
  std::vector<int32_t> tile_sup;       // per support column: occupied-pair index of the active pair, or -1
  std::vector<int32_t> ccol;           // per coupling: its column in the support of the string's tile
  int64_t n_tiles = 0;
  size_t off_tile_s0 = 0, off_tile_k0 = 0, off_tile_sup = 0, off_ccol = 0, off_Md = 0;
  int kernel = 0;                      // KERN_* below (sigma contraction)
  int kernel_bwd = 0;                  // KERN_* of the adjoint passes (generic under a level shift)
  // launch-shape targets (mrpt2_tuning; 0 = built-in rule)
  int64_t sigma_target = 0, bwd_target = 0, bwd_row_target = 0;
  int64_t n_blocks = 0;                // partial sums written by the class's kernel
  // denominator statistics: (row block, string chunk) values in the workspace
  size_t off_dstat = 0;
  int dstat_chunks = 1;
  int64_t n_dstat = 0;
};

struct InstancePlan {
  mrpt2_desc d{};
  int n_fc = 0, n_c = 0, n_a = 0, n_v = 0, n_e = 0;
  int n = 0, n_corr = 0, n_o = 0, n_occ = 0, n_l = 0;
  int n_vt = 0;                       // virtual tiles
  int pair_tile = 0;                  // FP64 pair-integral blocks: 64, 128 or 0 (rule)
  int64_t n_tp = 0;                   // virtual tile pairs I <= J
  int64_t n_pairs = 0;                // occupied pairs x < y (core + active)
  std::vector<std::vector<int>> pcats;
  std::vector<uint64_t> pstrings;
  std::unordered_map<uint64_t, int32_t> pindex;
  std::vector<int64_t> plist_ptr;     // [N_P + 1] excitation lists of P (CSR)
  std::vector<int32_t> plist_col;     // reference strings one or two replacements away
  ClassPlan cls[MRPT2_N_CLASS];
  std::vector<int32_t> hole_pairs;    // (c, c') for c < c'
  std::vector<int32_t> tile_pairs;    // (I, J) for I <= J
  std::vector<double> set_sign;       // per Cholesky vector: sign of its weight
  std::vector<double> set_scale;      // per Cholesky vector: sqrt|weight|
  // persistent layout
  size_t off_plist_ptr = 0, off_plist_col = 0;
  size_t off_pstrings = 0, off_hole_pairs = 0, off_tile_pairs = 0, off_sign = 0, off_scale = 0;
  size_t persistent_bytes = 0, persistent_base = 0;
  // workspace layout
  size_t off_fx = 0;
  size_t off_dg = 0, off_slab = 0, off_slab32 = 0, off_W = 0, off_eps = 0, off_f = 0, off_G = 0, off_A = 0;
  size_t off_hpp = 0, off_sigp = 0, off_scal = 0, off_dsum = 0, off_part = 0;
  size_t off_dstat_out = 0;           // [9] (min |Delta|, count) of mrpt2_delta_stats
  size_t workspace_bytes = 0, workspace_base = 0;
  // gradient workspace layout (adjoint)
  size_t off_gs = 0, off_Wb = 0, off_Wsym = 0, off_epsb = 0, off_fb = 0, off_Gb = 0, off_Ab = 0;
  size_t off_slabb = 0, off_dgb = 0, off_dsumb = 0, off_hb = 0, off_cb = 0;
  size_t grad_bytes = 0, grad_base = 0;
  int64_t n_part = 0;                 // partial-sum slots
  size_t off_part_class[MRPT2_N_CLASS]{};
  int64_t n_part_class[MRPT2_N_CLASS]{};
  mrpt2_info info{};
  std::vector<char> host_blob;        // persistent region image
};

// Kernels of the launch sequence.  Every launch covers all instances: a job
// per instance (and factor set or class where needed) gives its grid; the
// kernel finds its job from the flat block index.
enum KernelId : int {
  K_CLEAR, K_PACK, K_DIAG, K_WPASS, K_EPS, K_DSUM, K_FOCK, K_GBUILD, K_HPP, K_SIGP, K_E0,
  K_ABUILD, K_ABUILD32, K_CTAB, K_XBUILD, K_DCOEF, K_E22, K_E12_8, K_E12_16, K_E12_24, K_E12_32,
  K_E02, K_E02F, K_E02COEF, K_E22S, K_E12S_8, K_E12S_16, K_E12S_24, K_E12S_32, K_E02S, K_E02FS, K_SIG22, K_SIG12, K_SIG02, K_SIG21, K_SIG11, K_SIG01, K_SIG20, K_SIG10, K_SIG00, K_FINISH,
  // adjoint
  K_BZERO, K_BROW22, K_BROW12, K_BROW02, K_BROW21, K_BROW11, K_BROW01, K_BROW20, K_BROW10, K_BROW00,
  K_BSTR22, K_BSTR12, K_BSTR02, K_BSTR21, K_BSTR11, K_BSTR01, K_BSTR20, K_BSTR10, K_BSTR00,
  K_BSFIN, K_BHPP, K_BXB, K_BAG, K_BAGF, K_BGG, K_BFOCK, K_BDSUM, K_BHFE, K_BWSYM, K_BDG, K_BDB, K_BDH, K_BDC,
  K_BECOEF, K_BTRANS, K_B22A, K_B22B, K_B22WR, K_B22FIN, K_B12R_8, K_B12R_16, K_B12R_24, K_B12R_32, K_B12S_8, K_B12S_16, K_B12S_24, K_B12S_32,
  K_B12R_20, K_B12S_20, K_E12_20, K_E12S_20,
  // class (2,1) dense-coefficient kernel, pattern widths 8, 16, 20, 24, 32 (then level-shifted)
  K_E21_8, K_E21_16, K_E21_20, K_E21_24, K_E21_32, K_E21S_8, K_E21S_16, K_E21S_20, K_E21S_24, K_E21S_32,
  K_FOCKX, K_ABUILD64,
  // class (0,2) adjoint on MFMA: row pass, string pass, Uv tables
  K_B02R, K_B02S, K_B02W,
  K_BAG128, K_BXBRED,
  // denominator statistics (one per class, same order), then the fold
  K_DSTAT22, K_DSTAT12, K_DSTAT02, K_DSTAT21, K_DSTAT11, K_DSTAT01, K_DSTAT20, K_DSTAT10, K_DSTAT00,
  K_DSTATFIN,
  K_B12R_20W,                          // the 20-pattern (1,2) row pass with 64-string chunks
  // class (1,2) of the mixed form: sigma summed in FP32
  K_E12F_8, K_E12F_16, K_E12F_24, K_E12F_32, K_E12F_20
};

// Timing slots (mrpt2_energy_timed).
enum StageId : int {
  ST_NONE = -1, ST_TABLES = 0, ST_GBUILD = 1, ST_REF = 2, ST_ABUILD = 3, ST_SIGMA0 = 4,
  ST_PREP0 = 13, ST_FINISH = 22, ST_N = 23,
  // adjoint (mrpt2_energy_backward_timed): per-class row and string passes, then the chain
  ST_BROW0 = 23, ST_BSTR0 = 32, ST_BFIN = 41, ST_BHPP = 42, ST_BXB = 43, ST_BPAIR = 44, ST_BOCC = 45,
  ST_BTAB = 46, ST_BOUT = 47, ST_BZERO = 48, ST_NB = 49
};

struct JobH {                         // host image of the device Job
  int32_t inst, gx, gy, arg;
  int64_t blk0;
};

struct Launch {
  int kid = 0;
  int stage = ST_NONE;
  int64_t job0 = 0;                   // first job (index into the job table)
  int njobs = 0;
  int64_t nblocks = 0;
  size_t dyn_lds = 0;
  int arg = 0;                        // kernel-wide argument (hpp: write the caller's buffer)
};

constexpr size_t kInstBytes = 4096;   // device bytes reserved per instance descriptor

struct Plan {
  std::vector<InstancePlan> inst;
  size_t persistent_bytes = 0;
  size_t workspace_bytes = 0;
  size_t off_flag = 0;                // device error flag in the workspace
  size_t off_insts = 0;               // instance descriptors in the workspace
  size_t off_jobs = 0;                // job table in the persistent region
  std::vector<JobH> jobs;
  std::vector<Launch> energy;         // launch sequence of mrpt2_energy (all instances)
  std::vector<Launch> backward;       // launch sequence of mrpt2_energy_backward
  std::vector<Launch> stats;          // launch sequence of mrpt2_delta_stats
  double dstat_thresh = 0.0;          // threshold of the current mrpt2_delta_stats call
  size_t grad_bytes = 0;              // gradient workspace of mrpt2_energy_backward
  std::vector<std::vector<Launch>> reference;  // per instance: tables + H_PP
  std::vector<std::vector<Launch>> reference_tables;  // per instance: tables only
  std::vector<char> host_blob;
  std::vector<char> static_stage;     // host staging of the descriptors for mrpt2_energy_static
  void* pinned = nullptr;             // host staging of the instance descriptors
  size_t pinned_bytes = 0;            // its size (one descriptor set per state of a multi-state call)
  hipEvent_t staged = nullptr;        // recorded after each copy from the pinned staging buffer
  bool staged_recorded = false;
};

// Kernel that evaluates a class.
enum ClassKernel : int { KERN_GENERIC = 0, KERN_E22 = 1, KERN_E12 = 2, KERN_E02 = 3, KERN_E21 = 4 };
constexpr int kStrTile = 64;                // strings per tile of the (0,2) contraction kernel
constexpr int kB22Threads = 256;            // strings per block of the (2,2) string-owned adjoint kernel
constexpr int kB22PairsPerPart = 8;         // its largest group of core pairs per block

struct Plan;
// Launch sequences and job table of a plan whose instances are built.
void build_launches(Plan* P);

// Description of partial-sum block b of class k (see mrpt2_block).
void class_block(const InstancePlan& ip, int k, int64_t b, mrpt2_block* out);

// Builds the plan; returns MRPT2_OK or an error with a message in *err.
mrpt2_status build_plan(const mrpt2_desc* d, int n_inst, const mrpt2_tuning* tuning, Plan* out, std::string* err);

// Number of rows per string chunk and the blocks used by the sparse-sigma
// kernel of class k (shared by plan and launcher so the partial-sum slots
// match the launch).
int64_t sigma_blocks(const InstancePlan& ip, int k);

}  // namespace mrpt2
