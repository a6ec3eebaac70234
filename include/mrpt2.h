/*
 * mrpt2.h - C interface of the MI355X Epstein-Nesbet MRPT2 energy library.
 *
 * Computes the second-order energy of four-component multireference
 * perturbation theory in the small-tensor-product distributed active space
 * (STP-DAS) organisation (Majumder, Upadhyay, Beck, Oele, Li):
 *
 *   E2 = sum_{K in Q} |<K|H|Psi0>|^2 / (E0 - H_KK)          (eq. pt2, eq. pt2en)
 *
 * with the Epstein-Nesbet zeroth-order Hamiltonian (eq. zeroh: full H inside
 * the primary space P, diagonal H_KK on the external space Q), P built from
 * DAS configuration categories (Sec. 2.4), Q = every single and double
 * excitation of P that is not in P (Sec. 2.3), frozen core folded into the
 * one-electron operator and frozen virtuals removed (Sec. 2.5).
 *
 * Conventions (all arrays row-major; complex numbers interleaved (re, im)
 * as pairs of doubles):
 *  - Spinor order: frozen core | core | active (DAS subspaces in order) |
 *    kept virtuals.  n = n_frozen_core + n_core + n_active + n_virt.
 *    Frozen virtuals are never passed.
 *  - H = sum h_pq a+_p a_q + 1/2 sum (pq|rs) a+_p a+_r a_s a_q with
 *    (pq|rs) = sum_t weight[t] sum_L B_t[L,p,q] B_t[L,r,s]; h and every
 *    B_t[L] must be Hermitian.  One factor set per two-electron operator
 *    (Dirac-Coulomb, Gaunt, gauge), each with a real signed weight.
 *  - Determinant phase: |D> = a+_{p1} ... a+_{pN} |0> with p1 < ... < pN.
 *    The reference coefficient vector C follows the order returned by
 *    mrpt2_plan_ref_strings.  Psi0 = C / ||C||; E0 is its Rayleigh quotient,
 *    so C need not be normalised.
 *  - All large arrays are device pointers owned by the caller.  The library
 *    never allocates device memory: the caller provides a persistent region
 *    (plan tables, uploaded once) and a workspace region (scratch).
 *  - Every call returns a status; nothing aborts or throws across the ABI.
 *
 * Thread safety: a plan is immutable after mrpt2_plan; concurrent calls on
 * one plan need separate workspaces.
 */
#ifndef MRPT2_H
#define MRPT2_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MRPT2_MAX_SUB 16
#define MRPT2_MAX_SETS 4
#define MRPT2_N_CLASS 9

typedef enum {
  MRPT2_OK = 0,
  MRPT2_ERR_ARG = 1,          /* null pointer, bad count or value */
  MRPT2_ERR_SHAPE = 2,        /* sizes inconsistent or beyond limits */
  MRPT2_ERR_UNSUPPORTED = 3,  /* option not implemented */
  MRPT2_ERR_WORKSPACE = 4,    /* persistent/workspace region too small */
  MRPT2_ERR_HIP = 5,          /* a HIP runtime call failed */
  MRPT2_ERR_NUMERIC = 6       /* non-finite input or a zero denominator */
} mrpt2_status;

typedef enum { MRPT2_FP64 = 0, MRPT2_MIXED = 1 } mrpt2_precision;

/* Storage of the Cholesky factors B_t[L] (and of their gradients dB_t):
 *  MRPT2_LAYOUT_FULL    complex [rank_t][n][n], every entry;
 *  MRPT2_LAYOUT_PACKED  complex [rank_t][n (n + 1) / 2]: the upper triangle
 *    of each Hermitian B_t[L] by rows, entry (p, q) with p <= q at
 *    p n - p (p - 1) / 2 + (q - p); the lower triangle is its conjugate and
 *    the imaginary part of a diagonal entry is ignored.  Halves the factor
 *    memory and its one HBM pass.  The gradient in this layout is taken with
 *    respect to the stored entries themselves: 2 P_pq off the diagonal and
 *    P_pp on it, P being the Hermitian-projected gradient of the full
 *    layout. */
typedef enum { MRPT2_LAYOUT_FULL = 0, MRPT2_LAYOUT_PACKED = 1 } mrpt2_layout;

/* Problem description (one instance).  Sec. 2.4: the primary space holds
 * the active occupations whose per-subspace electron counts m_k satisfy
 * sum m_k = n_act_elec and sum_k max(0, m_k - sub_base[k]) <= max_hops
 * (max_hops >= n_act_elec gives a complete active space). */
typedef struct {
  int32_t n_frozen_core;            /* frozen core spinors (folded, Sec. 2.5) */
  int32_t n_core;                   /* correlated core spinors */
  int32_t n_virt;                   /* kept virtual spinors */
  int32_t n_sub;                    /* DAS subspaces, 0..MRPT2_MAX_SUB (0: single
                                       determinant reference) */
  int32_t sub_size[MRPT2_MAX_SUB];  /* spinors per subspace */
  int32_t sub_base[MRPT2_MAX_SUB];  /* base electron count per subspace */
  int32_t max_hops;                 /* inter-subspace hop limit of P */
  int32_t n_act_elec;               /* active electrons */
  int32_t q_mode;                   /* 0: Q = all S+D not in P (Sec. 2.3);
                                       1: only those with a core hole or a
                                       virtual electron (Sec. 2.4 listing) */
  int32_t n_sets;                   /* factor sets, 1..MRPT2_MAX_SETS */
  int32_t rank[MRPT2_MAX_SETS];     /* Cholesky vectors per set */
  double weight[MRPT2_MAX_SETS];    /* real signed weight per set */
  int32_t precision;                /* mrpt2_precision */
  double level_shift_b;             /* imaginary level shift b (Sec. 2.6), in
                                       Eh^2: every inverse denominator 1/Delta
                                       becomes Re 1/(Delta + i b/Delta) =
                                       Delta^3/(Delta^4 + b^2), in E2 and in
                                       its gradient; only b^2 enters.  0 gives
                                       eq. pt2 exactly.  A nonzero b runs the
                                       adjoint of every excitation class on the
                                       generic passes (slower). */
  int32_t layout;                   /* mrpt2_layout of B and dB */
} mrpt2_desc;

/* Sizes and exact algorithmic work of one instance. */
typedef struct {
  int32_t n_orb;                    /* n (spinors passed in h, B) */
  int32_t n_corr;                   /* correlated spinors */
  int32_t n_chol;                   /* total Cholesky vectors */
  int64_t n_ref;                    /* N_P */
  int64_t n_ext;                    /* N_Q */
  int64_t n_ext_class[MRPT2_N_CLASS];  /* per class, order (h,v) =
      (2,2),(1,2),(0,2),(2,1),(1,1),(0,1),(2,0),(1,0),(0,0) */
  int64_t n_strings_class[MRPT2_N_CLASS];
  int64_t n_conn_class[MRPT2_N_CLASS];
  double flop_integral;             /* algorithmic flops of the integral builds */
  double flop_sigma;                /* algorithmic flops of the sigma contractions
                                       (nonzero couplings only; the (2,2) class
                                       has none) */
  double bytes_factors;             /* bytes of all factor sets (one HBM pass) */
  int32_t n_patterns_class[MRPT2_N_CLASS];  /* distinct coupling patterns per
      class: for (1,2) the active spinors t of the reference determinants
      core + alpha' + t it couples to, which sizes the dense-coefficient
      kernels (up to 8, 16, 24 or 32 patterns; more run the generic kernel) */
  int64_t n_ref_couplings;          /* off-diagonal entries of the excitation
      lists of P (pairs of reference determinants one or two active
      replacements apart), which the direct sigma-build in P applies */
  int32_t kernel_class[MRPT2_N_CLASS];      /* sigma kernel of each class:
      0 generic (excitation lists), 1 class (2,2) string sums, 2 class (1,2)
      dense coefficients, 3 class (0,2) string tiles on MFMA, 4 class (2,1)
      dense coefficients */
} mrpt2_info;

/* Inputs of one instance (device pointers). */
typedef struct {
  const double* h;                     /* complex [n][n] */
  const double* B[MRPT2_MAX_SETS];     /* complex [rank_t][n][n], or
                                          [rank_t][n (n + 1) / 2] packed */
  const double* c;                     /* complex [N_P], plan order */
} mrpt2_inputs;

/* Gradient outputs of one instance (device pointers, caller-owned, overwritten). */
typedef struct {
  double* dh;                          /* complex [n][n] */
  double* dB[MRPT2_MAX_SETS];          /* complex, in the layout of B */
  double* dc;                          /* complex [N_P], plan order */
} mrpt2_grads;

typedef struct mrpt2_plan_s* mrpt2_plan_t;

/* Build the plan for n_inst instances (host only; no device work).
 * Enumerates the DAS categories, reference and external strings by
 * excitation class (Sec. 2.4), excitation lists and the work decomposition.
 * Errors: MRPT2_ERR_ARG for null pointers, n_inst < 1 or a level_shift_b
 * that is not finite, MRPT2_ERR_SHAPE for inconsistent sizes (electrons vs
 * subspaces, more than 64 active spinors, N_P >= 2^24), MRPT2_ERR_UNSUPPORTED
 * for an unknown precision or factor layout.  On error *out is NULL. */
mrpt2_status mrpt2_plan(const mrpt2_desc* desc, int32_t n_inst, mrpt2_plan_t* out);

/* Launch shapes of one instance's work decomposition, per excitation class
 * (class order as in mrpt2_info); 0 keeps the built-in rule.  Each value is a
 * target block count:
 *   sigma_blocks    the generic sigma kernel (classes without a dedicated
 *                   kernel): rows in blocks of 256, the strings split into
 *                   ceil(target / row blocks) chunks (default 8192);
 *   bwd_blocks      the string-owned adjoint pass: (string block, row part)
 *                   blocks (default 2048); more parts cost gradient workspace;
 *   bwd_row_blocks  the generic row-owned adjoint pass when it has fewer than
 *                   512 row blocks: strings split into
 *                   ceil(target / row blocks) chunks (default 2048).
 * and one per instance:
 *   pair_tile       edge of the output blocks of the FP64 virtual-pair
 *                   integral build: 128 (eight waves, four 64 x 64 tiles per
 *                   block) or 64 (one tile per block); 0 keeps the built-in
 *                   rule (128 where at least 90 % of the 128 x 128 blocks'
 *                   tiles lie on or above the diagonal and inside n_virt);
 *                   the mixed form has one block shape and ignores it.
 * The values change launch grids and partial-sum layouts, never the result
 * beyond summation order.  Tables of them are written by the package's
 * autotuner (timed sweeps per class and size bucket). */
typedef struct {
  int32_t sigma_blocks[MRPT2_N_CLASS];
  int32_t bwd_blocks[MRPT2_N_CLASS];
  int32_t bwd_row_blocks[MRPT2_N_CLASS];
  int32_t pair_tile;
} mrpt2_tuning;

/* mrpt2_plan with launch shapes: tuning is a host array of n_inst entries
 * (or NULL for the built-in rules).  Negative values, and a pair_tile other
 * than 0, 64 or 128, are MRPT2_ERR_ARG. */
mrpt2_status mrpt2_plan_tuned(const mrpt2_desc* desc, int32_t n_inst, const mrpt2_tuning* tuning,
                              mrpt2_plan_t* out);

/* Bytes of the persistent region (plan tables) and of the workspace needed by
 * mrpt2_energy.  Both must be 256-byte aligned device allocations. */
mrpt2_status mrpt2_plan_sizes(mrpt2_plan_t plan, size_t* persistent_bytes, size_t* workspace_bytes);

/* Copy the plan tables to the caller's persistent region (async on stream;
 * the host source stays valid for the life of the plan). */
mrpt2_status mrpt2_plan_upload(mrpt2_plan_t plan, void* persistent, size_t bytes, hipStream_t stream);

mrpt2_status mrpt2_plan_info(mrpt2_plan_t plan, int32_t inst, mrpt2_info* info);

/* Active parts of the reference determinants, in the order C must follow:
 * bit t of bits[i] set = active spinor t (0-based within the active block)
 * occupied in reference determinant i.  bits has N_P entries (host). */
mrpt2_status mrpt2_plan_ref_strings(mrpt2_plan_t plan, int32_t inst, uint64_t* bits);

/* E2 for every instance.  in: n_inst input sets (host array of structs whose
 * pointers are device pointers).  e2: device double[n_inst] (written).
 * parts: optional device double[n_inst][12] = per-class E2 (class order as
 * in mrpt2_info), then E0 - E_core (reference energy relative to the core
 * energy), then ||C||^2.  Enqueued on stream; the call synchronises the
 * stream once to read the device error flag.  Errors: MRPT2_ERR_WORKSPACE if
 * the regions are too small or not uploaded, MRPT2_ERR_NUMERIC if an input
 * is not finite or a denominator is zero (the energies are then not valid),
 * MRPT2_ERR_HIP for launch or runtime failures. */
mrpt2_status mrpt2_energy(mrpt2_plan_t plan, const mrpt2_inputs* in,
                          const void* persistent, void* workspace, size_t workspace_bytes,
                          hipStream_t stream, double* e2, double* parts);

/* State-specific E2 of several reference states per instance (the state
 * index m of eq. pt2: E2_m with E0_m = <Psi_m|H|Psi_m> and the first-order
 * vector of Psi_m, each state with its own denominators).  in[i].c points to
 * n_roots coefficient vectors of instance i, complex [n_roots][N_P] in plan
 * order (each normalised or not; the norm is divided out as in
 * mrpt2_energy).  The steps that do not depend on the reference vector (the
 * factor tables, the occupied-block and virtual-pair integrals, H_PP and the
 * couplings) run once per call; the reference energy, the per-string
 * denominator tables, the sigma contractions and the sums run once per state.
 * e2: device double[n_roots][n_inst]; parts: optional device
 * double[n_roots][n_inst][12] laid out as in mrpt2_energy.  Root m gives the
 * same numbers as mrpt2_energy called with c = root m.  Synchronises the
 * stream once at the end.  Errors as mrpt2_energy; MRPT2_ERR_ARG for
 * n_roots < 1 or a NULL c. */
mrpt2_status mrpt2_energy_roots(mrpt2_plan_t plan, const mrpt2_inputs* in, int32_t n_roots,
                                const void* persistent, void* workspace, size_t workspace_bytes,
                                hipStream_t stream, double* e2, double* parts);

/* mrpt2_energy without its final synchronisation: every step (a small
 * host-to-device copy of the instance descriptors from library-owned pinned
 * memory, then one batched launch per stage covering all instances) is
 * enqueued on `stream`, so the call can be captured into a HIP graph and
 * replayed.  Replays re-copy the descriptors staged by the captured call
 * (same input and output pointers); any later call on the same plan restages
 * them, so a plan whose calls are captured should be reserved for that graph,
 * and make one ordinary call before the capture (the staging buffer is
 * allocated on a plan's first call).  The device error flag stays in the
 * workspace; read it with mrpt2_check.  Two asynchronous calls with different
 * inputs on one plan must be separated by a stream synchronisation (they
 * share the pinned descriptor buffer). */
mrpt2_status mrpt2_energy_async(mrpt2_plan_t plan, const mrpt2_inputs* in,
                                const void* persistent, void* workspace, size_t workspace_bytes,
                                hipStream_t stream, double* e2, double* parts);

/* Synchronise `stream` and report the error flag of the last evaluation on
 * this workspace: MRPT2_OK or MRPT2_ERR_NUMERIC. */
mrpt2_status mrpt2_check(mrpt2_plan_t plan, const void* workspace, hipStream_t stream);

/* mrpt2_energy with its stages timed by HIP events recorded on `stream`.
 * stage_ms (host float[23], milliseconds summed over instances):
 * [0] factor tables (slabs, pair energies, orbital energies, core Fock),
 * [1] occupied-integral build, [2] reference energy, [3] virtual-pair
 * integral build, [4 + k] sigma contraction and epilogue of class k,
 * [13 + k] denominator tables and couplings of class k, [22] reduction.
 * Same errors as mrpt2_energy; MRPT2_ERR_ARG if stage_ms is NULL. */
mrpt2_status mrpt2_energy_timed(mrpt2_plan_t plan, const mrpt2_inputs* in,
                                const void* persistent, void* workspace, size_t workspace_bytes,
                                hipStream_t stream, double* e2, double* parts, float* stage_ms);

/* Dense reference-space Hamiltonian minus the core energy,
 * H_PP - E_core * 1, for instance inst (complex [N_P][N_P], device, written)
 * - the matrix whose lowest eigenvector is the reference state.  Uses the
 * same workspace as mrpt2_energy; c in `in` is not read. */
mrpt2_status mrpt2_reference_hamiltonian(mrpt2_plan_t plan, int32_t inst, const mrpt2_inputs* in,
                                         const void* persistent, void* workspace,
                                         size_t workspace_bytes, hipStream_t stream, double* hpp);

/* Bytes of the device region mrpt2_reference_states needs for n_states
 * states of instance inst (holds H_PP, 16 N_P^2 bytes, and the search space). */
mrpt2_status mrpt2_reference_states_size(mrpt2_plan_t plan, int32_t inst, int32_t n_states, size_t* bytes);

/* The n_states lowest eigenpairs of the reference-space Hamiltonian minus the
 * core energy, H_PP - E_core (eq. zeroh inside P: the CI problem in the
 * primary space that yields Psi0 and the states E2_m refers to), on the
 * device.  H_PP is assembled from the Slater-Condon rules as in
 * mrpt2_reference_hamiltonian (into dv), then a block Davidson solver runs:
 * the search space starts from the unit vectors of the n_states lowest
 * diagonal elements; each iteration applies H_PP to the new directions (a
 * dense Hermitian product, one wavefront per row), solves the projected
 * matrix on the host (mrpt2_hermitian_eigh), forms Ritz vectors and
 * residuals, and adds the residuals divided by (theta - diag H_PP),
 * orthonormalised twice against the search space; the space restarts from
 * the lowest Ritz vectors when full.
 * dv: device region of mrpt2_reference_states_size bytes, 256-byte aligned.
 * tol: bound on every residual norm ||H x - theta x|| (x of unit norm, Eh).
 * c_out: device complex [n_states][N_P] (written; plan order, unit norm, the
 * largest component real and positive); e_out: host double[n_states]
 * (written, ascending); iterations: host int (optional, written).
 * Errors: MRPT2_ERR_ARG for bad arguments or n_states > N_P,
 * MRPT2_ERR_WORKSPACE if dv_bytes is too small, MRPT2_ERR_NUMERIC if
 * max_iter iterations leave a residual above tol (the Ritz pairs reached are
 * written) or a value is not finite. */
mrpt2_status mrpt2_reference_states(mrpt2_plan_t plan, int32_t inst, const mrpt2_inputs* in, int32_t n_states,
                                    double tol, int32_t max_iter, const void* persistent, void* workspace,
                                    size_t workspace_bytes, void* dv, size_t dv_bytes, hipStream_t stream,
                                    double* c_out, double* e_out, int32_t* iterations);

/* Direct sigma-build in P (Sec. 2.4, the sigma of eq. sumsigma restricted
 * to the primary space): Y = (H_PP - E_core) X for n_vec vectors without
 * storing H_PP.  The plan keeps, for every reference determinant, the list
 * of reference determinants reached from it by one or two replacements of
 * active spinors (mrpt2_info.n_ref_couplings entries in all); each row
 * applies its list with elements from the Slater-Condon rules on the
 * integral tables (the same rules as mrpt2_reference_hamiltonian) and adds
 * its diagonal.  x, y: device complex [n_vec][N_P] (plan order), distinct.
 * The tables are rebuilt from h and B in workspace first.  Synchronises
 * stream; MRPT2_ERR_NUMERIC on non-finite tables. */
mrpt2_status mrpt2_reference_sigma(mrpt2_plan_t plan, int32_t inst, const mrpt2_inputs* in, int32_t n_vec,
                                   const double* x, const void* persistent, void* workspace,
                                   size_t workspace_bytes, hipStream_t stream, double* y);

/* mrpt2_reference_states with the direct sigma-build in P instead of a
 * stored H_PP: the solver region (mrpt2_reference_states_direct_size) holds
 * only the search space, its image, their restart copies, Ritz vectors,
 * residuals and small matrices, O(N_P) per vector, so reference spaces far
 * beyond a dense H_PP fit.  Same arguments, results and errors. */
mrpt2_status mrpt2_reference_states_direct_size(mrpt2_plan_t plan, int32_t inst, int32_t n_states, size_t* bytes);
mrpt2_status mrpt2_reference_states_direct(mrpt2_plan_t plan, int32_t inst, const mrpt2_inputs* in,
                                           int32_t n_states, double tol, int32_t max_iter, const void* persistent,
                                           void* workspace, size_t workspace_bytes, void* dv, size_t dv_bytes,
                                           hipStream_t stream, double* c_out, double* e_out, int32_t* iterations);

/* Eigenpairs of a complex Hermitian n x n matrix (host memory, row-major,
 * interleaved complex; only its Hermitian part is used) by cyclic Jacobi
 * rotations: w (host double[n]) ascending, v (host complex [n][n]) with
 * eigenvector j in column j.  Used for the projected matrix of the Davidson
 * solver; meant for n up to a few hundred.  Errors: MRPT2_ERR_ARG,
 * MRPT2_ERR_NUMERIC for non-finite input. */
mrpt2_status mrpt2_hermitian_eigh(int32_t n, const double* a, double* w, double* v);

/* Denominator statistics of the external space (Sec. 2.6: an intruder state
 * is an external determinant K whose E0 - H_KK comes close to zero, where
 * its term of eq. pt2en blows up and the level shift is meant to act): for
 * every instance and excitation class, the smallest |E0 - H_KK| over the
 * class's determinants and the number of them with |E0 - H_KK| < thresh
 * (the unshifted denominators, whatever the plan's level shift).  Runs the
 * factor tables, the occupied-block integrals, the reference energy and the
 * per-string denominator tables on `workspace` (not the pair integrals or
 * any sigma contraction), then one pass over each class's (row x string)
 * grid.  in: as mrpt2_energy (c is read for E0).  min_abs_delta: host
 * double[n_inst][9], class order as in mrpt2_info, +inf for an empty class
 * (written); n_below: host int64[n_inst][9] or NULL (written).  Synchronises
 * the stream.  Errors as mrpt2_energy; MRPT2_ERR_ARG for a NULL
 * min_abs_delta or a thresh that is negative or not finite. */
mrpt2_status mrpt2_delta_stats(mrpt2_plan_t plan, const mrpt2_inputs* in, const void* persistent, void* workspace,
                               size_t workspace_bytes, hipStream_t stream, double thresh, double* min_abs_delta,
                               int64_t* n_below);

/* Bytes of the gradient workspace of mrpt2_energy_backward (256-byte aligned
 * device allocation, caller-owned). */
mrpt2_status mrpt2_plan_backward_size(mrpt2_plan_t plan, size_t* grad_workspace_bytes);

/* Gradient of E2 (eq. pt2en with the Epstein-Nesbet partition, eq. zeroh)
 * with respect to every input, for every instance: the adjoint of the energy
 * evaluation, derived from its steps (the paper gives no gradient).
 * The forward pass is recomputed first on `workspace` (same contents as after
 * mrpt2_energy); the first-order vector sigma_K / (E0 - H_KK) is recomputed
 * per block and never stored.  grad_e2: device [n_inst], the upstream
 * gradient dL/dE2 per instance; the outputs are dL/dh, dL/dB_t, dL/dc.
 * Convention: for a complex input z the output is dL/dRe z + i dL/dIm z.  h
 * and every B_t[L] are Hermitian parameters, so dh and dB_t[L] are projected,
 * (G + G^H) / 2; dc is unconstrained (it is orthogonal to c and to i c, as E2
 * depends only on the ray of c).  Layouts as in mrpt2_inputs (interleaved
 * complex FP64, row-major); dB_t must be given for every set with rank > 0.
 * e2: device [n_inst] receiving E2 of the recomputed forward pass, or NULL.
 * The gradient workspace is cleared by the call; accumulation order is not
 * fixed (FP64 atomics), so results are reproducible to rounding.  The
 * arithmetic is FP64 in both precisions of the plan (the mixed form uses its
 * FP32-MFMA pair integrals in the recomputed forward pass).  Synchronises the
 * stream once to read the error flag.  Errors: MRPT2_ERR_ARG for null
 * pointers or misaligned regions, MRPT2_ERR_WORKSPACE if a region is too
 * small, MRPT2_ERR_NUMERIC for a non-finite input or zero denominator,
 * MRPT2_ERR_HIP for launch or runtime failures. */
mrpt2_status mrpt2_energy_backward(mrpt2_plan_t plan, const mrpt2_inputs* in, const void* persistent,
                                   void* workspace, size_t workspace_bytes, void* grad_workspace,
                                   size_t grad_workspace_bytes, const double* grad_e2,
                                   const mrpt2_grads* grads, hipStream_t stream, double* e2);

/* mrpt2_energy_backward without its final synchronisation: the descriptor
 * copy and every launch (the forward recomputation included) are enqueued on
 * `stream`, so one captured HIP graph holds the forward pass and the adjoint
 * of every instance.  The capture rules of mrpt2_energy_async apply; read the
 * error flag with mrpt2_check. */
mrpt2_status mrpt2_energy_backward_async(mrpt2_plan_t plan, const mrpt2_inputs* in, const void* persistent,
                                         void* workspace, size_t workspace_bytes, void* grad_workspace,
                                         size_t grad_workspace_bytes, const double* grad_e2,
                                         const mrpt2_grads* grads, hipStream_t stream, double* e2);

/* mrpt2_energy_backward with its stages timed by HIP events on `stream`:
 * stage_ms (host, 49 floats) receives milliseconds per stage: 0..22 as in
 * mrpt2_energy_timed (the recomputed forward pass), 23 + k and 32 + k the
 * row-owned and string-owned adjoint passes of class k, then 41 per-string
 * adjoints, 42 reference energy, 43 coupling build, 44 pair integrals, 45
 * occupied-block integrals, 46 Fock/orbital/pair-energy tables, 47 output
 * gradients, 48 workspace clear.  Same errors as mrpt2_energy_backward;
 * MRPT2_ERR_ARG if stage_ms is NULL. */
mrpt2_status mrpt2_energy_backward_timed(mrpt2_plan_t plan, const mrpt2_inputs* in, const void* persistent,
                                         void* workspace, size_t workspace_bytes, void* grad_workspace,
                                         size_t grad_workspace_bytes, const double* grad_e2,
                                         const mrpt2_grads* grads, hipStream_t stream, double* e2,
                                         float* stage_ms);

/* Work decomposition of one excitation class: mrpt2_energy writes one
 * partial sum per block, sum over the block's external determinants of
 * |sigma_K|^2 / (E0 - H_KK) (not yet divided by ||C||^2).  A block covers
 * either (kind 0) the core holes `hole[0..n_holes)`, lowest virtual in
 * [a_lo, a_hi), second virtual in [b_lo, b_hi) (b > a; two-virtual classes),
 * or (kind 1) the rows [row_lo, row_hi) with row = hole_index * n_virt^v + a
 * (hole_index in lexicographic order of the hole sets), and in both cases the
 * class strings [s_lo, s_hi) in mrpt2_plan_class_strings order.  Virtual
 * indices are 0-based within the kept virtuals, core indices within the
 * correlated core.  For checking sampled parts of a large sum. */
typedef struct {
  int32_t kind;
  int32_t n_holes;
  int32_t hole[2];
  int32_t a_lo, a_hi, b_lo, b_hi;
  int64_t row_lo, row_hi;
  int64_t s_lo, s_hi;
} mrpt2_block;

mrpt2_status mrpt2_plan_class_blocks(mrpt2_plan_t plan, int32_t inst, int32_t cls, int64_t* n_blocks);
mrpt2_status mrpt2_plan_class_block(mrpt2_plan_t plan, int32_t inst, int32_t cls, int64_t block,
                                    mrpt2_block* out);
/* Active strings of the external determinants of class cls (host, in the
 * order the blocks refer to; same bit convention as the reference strings). */
mrpt2_status mrpt2_plan_class_strings(mrpt2_plan_t plan, int32_t inst, int32_t cls, uint64_t* bits);
/* Copy the block partial sums of class cls from the last mrpt2_energy on
 * this workspace to host memory (n_blocks doubles); synchronises stream. */
mrpt2_status mrpt2_class_partials(mrpt2_plan_t plan, int32_t inst, int32_t cls, const void* workspace,
                                  hipStream_t stream, double* out);

/* ---- energy without caller-provided workspace ------------------------------
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation):
 * mrpt2_energy with the workspace replaced by a device array the library
 * owns, MRPT2_STATIC_WORKSPACE_BYTES per GPU, held from the library's load
 * until the process ends.  The call allocates nothing (no device, pinned or
 * heap memory): plan tables (persistent region, uploaded by
 * mrpt2_plan_upload), inputs and outputs are the caller's, as for
 * mrpt2_energy, and the instance descriptors are staged in host memory the
 * plan reserved when it was built.  Plans whose workspace (mrpt2_plan_sizes)
 * exceeds the array are rejected with MRPT2_ERR_WORKSPACE before any work.
 * The array is shared by every call on that GPU and keeps the last call's
 * contents (nothing in the energy sequence reads it before writing it):
 * calls that overlap on one GPU race, so calls on one device must be
 * serialised by the caller (one stream, or synchronisation between streams).
 * The call ends with a synchronisation of stream (error flag), like
 * mrpt2_energy.  Outputs: e2 [n_inst], parts [n_inst][12] (nullable), device
 * pointers.  mrpt2_static_workspace_bytes reports the array's size. */
#define MRPT2_STATIC_WORKSPACE_BYTES (64ull << 20)
mrpt2_status mrpt2_energy_static(mrpt2_plan_t plan, const mrpt2_inputs* in, const void* persistent,
                                 hipStream_t stream, double* e2, double* parts);
mrpt2_status mrpt2_static_workspace_bytes(size_t* bytes);

void mrpt2_plan_destroy(mrpt2_plan_t plan);
const char* mrpt2_status_string(mrpt2_status s);

#ifdef __cplusplus
}
#endif
#endif
