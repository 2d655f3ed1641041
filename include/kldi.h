/*
 * kldi.h -- C ABI of libkldi: block-filtered exchange-correlation (EXC) integration on AMD MI355X
 * (gfx950).
 *
 * The library evaluates, for a Kohn-Sham density matrix D in a contracted cartesian Gaussian basis
 * on an atom-centred quadrature grid {(r_i, w_i)}:
 *     Phi_{mu i} = chi_mu(r_i)                                    (paper Sec. II-A, eq. phi_def)
 *     X = D Phi,  rho_i = sum_mu Phi_{mu i} X_{mu i}              (eq. r_equals_dphi; Appendix A,
 *                                                                  "The density matrix")
 *     grad rho_i = 2 sum_mu grad Phi_{mu i} X_{mu i},  sigma_i = |grad rho_i|^2      (GGA)
 *     E_xc = sum_i w_i f(rho_i, sigma_i)                          (Appendix A, "Numerical
 *                                                                  integration grids")
 *     Z_{mu i} = w_i (v_rho,i Phi_{mu i} / 2 + 2 v_sigma,i grad rho_i . grad Phi_{mu i})
 *     Vxc = Phi Z^T + Z Phi^T                                     (eq. fxc_matrix_form with b = 1
 *                                                                  and W = diag(w v^xc), eq. w_def;
 *                                                                  for LDA Vxc = Phi W Phi^T)
 * as block-structured matrix products (Sec. III): the grid and the AOs are reordered (Sec. III-B.2),
 * cut into AO tiles x grid blocks (Sec. III-B.1), tiles whose max-abs summary is below t_b are
 * dropped (eqs. block_summary_A .. retained_blocks_B), and inside each product only the block
 * pairs with a_pq * b_qr >= t_d are executed (eqs. block_pair_filter .. executed_block_pairs),
 * enumerated by prefix-sum compaction (Appendix D, Alg. parallel_where).
 *
 * Conventions for every call:
 *  - Every function returns a kldi_status: KLDI_OK (0) on success, a negative code otherwise; the
 *    matching message is available from kldi_last_error() (thread-local).  No C++ exception
 *    crosses the ABI.
 *  - Units: bohr for positions, bohr^-2 for exponents, hartree for energies.
 *  - Basis and grid arguments are HOST pointers; they are read during kldi_plan_create only and
 *    copied; the caller keeps ownership.  D, rho, E_xc and Vxc of kldi_eval are DEVICE pointers
 *    (HIP global memory on the current device) owned by the caller.
 *  - All public floating-point data is FP64 whatever the internal precision.  Matrices are dense,
 *    row-major, n_ao x n_ao, in the caller's AO order; rho is in the caller's grid order.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  kldi_eval only enqueues
 *    work; results are ready after the stream is synchronised.  Part of an FP32 evaluation runs on a
 *    stream of the plan forked from `stream` and joined back into it, so ordering on `stream` holds;
 *    evaluations of one plan on different streams at the same time are not supported.
 *  - Arguments are validated before any launch.  A plan is not re-entrant: concurrent kldi_eval
 *    calls on one plan race on its workspaces.
 */
#ifndef KLDI_H
#define KLDI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  KLDI_OK = 0,
  KLDI_E_ARG = -1,          /* invalid argument (NULL pointer, bad size, bad enum, ...)          */
  KLDI_E_OOM = -2,          /* device memory for the plan's workspaces could not be allocated    */
  KLDI_E_HIP = -3,          /* a HIP runtime call failed                                          */
  KLDI_E_UNSUPPORTED = -4,  /* valid request this library does not implement                     */
  KLDI_E_STATE = -5,        /* call out of order                                                  */
  KLDI_E_NONFINITE = -6     /* non-finite entry found in D (reported by kldi_eval_check)          */
} kldi_status;

/* Exchange-correlation functional (spin-unpolarised, total density).  The paper uses M06-2X via
 * Libxc (Sec. IV, "Numerical settings"); this library implements the published forms below. */
typedef enum {
  KLDI_XC_LDA_X = 1,        /* Slater exchange f = -(3/4)(3/pi)^(1/3) rho^(4/3)                  */
  KLDI_XC_PBE = 2,          /* PBE exchange + PW92 correlation + PBE gradient correction          */
  KLDI_XC_PBE_X = 3,        /* PBE exchange only                                                   */
  /* Meta-GGA (the kinetic-energy density path of the paper's M06-2X, whose parameters are not
   * available here): MVS exchange (Sun, Perdew, Ruzsinszky 2015), F_x(s, alpha), alpha = (tau - tau_W) /
   * tau_unif, tau = 1/2 sum D grad chi . grad chi; FP64 plans only (KLDI_E_UNSUPPORTED otherwise). */
  KLDI_XC_MVS = 4,          /* MVS exchange + PBE correlation                                      */
  KLDI_XC_MVS_X = 5         /* MVS exchange only                                                   */
} kldi_xc;

/* Working precision of the block GEMMs.  The functional, rho accumulation across tiles, E_xc and
 * the Vxc accumulation across grid segments are FP64 in every mode. */
typedef enum {
  KLDI_PREC_FP64 = 0,       /* FP64 operands, FP64 MFMA (v_mfma_f64_16x16x4)                     */
  KLDI_PREC_FP32 = 1,       /* FP32 operands, FP32 MFMA accumulate, FP64 flush                    */
  /* Split-precision products on BF16 MFMA (v_mfma_f32_16x16x32_bf16, FP32 accumulation within one
   * 32-AO K tile, FP64 flush) for the X = D Phi product: each FP64 operand is written as a sum of
   * BF16 pieces v = v_0 + v_1 (+ v_2), each piece the BF16 rounding of what the earlier ones leave,
   * and the products of pieces whose orders add up to at most 1 (X3) or 2 (X6) are summed.  The
   * Vxc product runs as in KLDI_PREC_FP32. */
  KLDI_PREC_BF16X3 = 3,     /* two pieces, 3 products: about 16 significant bits per product      */
  KLDI_PREC_BF16X6 = 4      /* three pieces, 6 products: about 24 significant bits per product    */
} kldi_prec;

/* Contracted cartesian Gaussian basis (Appendix A, "Gaussian basis functions"):
 *   chi(r) = N_rel * dx^lx dy^ly dz^lz * sum_k prim_coef[k] exp(-prim_exp[k] |r - R_atom|^2),
 * N_rel = sqrt((2l-1)!! / ((2lx-1)!! (2ly-1)!! (2lz-1)!!)), applied by the library.  prim_coef
 * includes the normalisation of the x^l component.  AO order = shell order, components of a shell
 * lexicographic (x, y, z; xx, xy, xz, yy, yz, zz).  l <= 2. */
typedef struct {
  int32_t n_atoms;
  const double *atom_xyz;        /* [n_atoms * 3]                                                 */
  int32_t n_shells;
  const int32_t *shell_atom;     /* [n_shells], 0 <= atom < n_atoms                               */
  const int32_t *shell_l;        /* [n_shells], 0..2                                              */
  const int32_t *shell_prim_ptr; /* [n_shells + 1], CSR offsets into prim_exp/prim_coef, strictly
                                    increasing, first entry 0                                     */
  const double *prim_exp;        /* [shell_prim_ptr[n_shells]], > 0                              */
  const double *prim_coef;       /* [shell_prim_ptr[n_shells]]                                    */
} kldi_basis;

/* Quadrature grid (Sec. II-A: {(r_i, w_i)}).  point_atom is the atom whose atom-centred grid
 * generated the point; it is the "associated atom" of the Morton grouping (Sec. III-B.2). */
typedef struct {
  int64_t n_points;              /* >= 1                                                          */
  const double *xyz;             /* [n_points * 3]                                                */
  const double *weight;          /* [n_points]                                                    */
  const int32_t *point_atom;     /* [n_points], 0 <= atom < n_atoms                               */
} kldi_grid;

/* How the block-GEMM stages distribute their work items (tasks of Sec. III-D) over the GPU. */
typedef enum {
  KLDI_SCHED_GRID = 0,      /* grid blocks (X) / Vxc segments dealt round-robin over the 8 XCDs,
                               Vxc items in decreasing estimated cost; one workgroup per item      */
  KLDI_SCHED_QUEUE = 1      /* 8 per-XCD queues of about equal estimated cost (items of a queue
                               share L2), each ordered by decreasing cost; one workgroup per item.
                               Plans of more than 1024 grid blocks refuse it (KLDI_E_UNSUPPORTED):
                               it has been verified only on smaller plans                          */
} kldi_schedule;

typedef struct {
  double t_b;                    /* block-retention threshold (eq. block_filter_A), >= 0          */
  double t_d;                    /* block-pair execution threshold (eq. block_pair_filter), >= 0  */
  double rho_cut;                /* points with rho <= rho_cut get f = v = 0, >= 0                 */
  int32_t grid_block;            /* G, points per screening block: 128 or 256.  Both screen and
                                    filter per G-point block (S_Phi, a_pq, b_pr, z_qr at that
                                    granularity); the kernels compute in 128-point blocks, the
                                    two halves of a 256-point block sharing its retained tiles
                                    and summaries                                                 */
  int32_t ao_block;              /* d, AOs per tile; the library supports 32                       */
  int32_t prec;                  /* kldi_prec                                                     */
  int32_t xc;                    /* kldi_xc                                                       */
  int32_t v_segment;             /* grid blocks per Vxc work item (the K extent of its tile);
                                    0 = chosen by the plan                                         */
  int32_t chunk_tiles;           /* max retained tiles whose Phi/Z are held at once (the grid is
                                    processed in chunks of whole Vxc segments); 0 = fit to memory */
  int32_t schedule;              /* kldi_schedule                                                 */
  const int32_t *shell_order;    /* NULL: basis functions in the atom order (atoms by the Morton key
                                    of their centres, each atom's shells in input order); else host
                                    array [n_shells], the internal sequence of (caller) shells, e.g.
                                    from kldi_overlap_order; read at plan time; single-molecule plans */
} kldi_opts;

typedef struct kldi_plan kldi_plan;

typedef struct {
  int32_t n_ao, n_tiles;               /* AOs and AO tiles (d AOs each, last one padded)          */
  int64_t n_points, n_blocks;          /* grid points and grid blocks (G each, last one padded)   */
  int64_t n_candidate_tiles;           /* (tile, block) pairs passing the shell-radius pre-filter */
  int64_t n_retained_tiles;            /* |S_Phi|: (tile, block) pairs with max-abs >= t_b        */
  double retained_fraction;            /* n_retained_tiles / (n_tiles * n_blocks)                 */
  int32_t max_tiles_per_block;         /* max over blocks of |S_r|                                */
  int32_t v_segment;                   /* grid blocks per Vxc segment                             */
  int64_t n_v_items;                   /* Vxc work items (chunk pair x segment)                  */
  int64_t workspace_bytes;             /* device bytes held by the plan                           */
  int32_t n_grid_chunks;               /* chunks of grid blocks per evaluation                    */
  double plan_ms;                      /* wall time of kldi_plan_create                           */
  int32_t n_mol;                       /* molecules (1 for kldi_plan_create)                      */
  int32_t schedule;                    /* kldi_schedule in use                                    */
  int32_t graph;                       /* 1 if evaluations replay a captured graph                */
  int64_t n_x_items;                   /* X = D Phi work items (grid block x chunk of 4 tiles)     */
} kldi_plan_info_t;

typedef struct {
  int64_t n_pairs_x;                   /* executed (p, q, r) tile triples of X = D Phi            */
  int64_t n_pairs_v;                   /* executed (p, q, r) tile triples of M = Phi Z^T          */
  double gemm_flops;                   /* 2 d^2 G (n_pairs_x + n_pairs_v): algorithmic GEMM work  */
  int32_t nonfinite_d;                 /* 1 if D held a NaN or Inf                                */
  int64_t n_points_mlp;                /* grid points evaluated by an attached functional surrogate */
  int64_t n_pairs_v_diag;              /* of n_pairs_v, the diagonal triples (p, p, r) that an FP32
                                          plan runs on FP64 MFMA (0 for FP64 plans, whose Vxc product
                                          is FP64 throughout)                                         */
} kldi_eval_stats_t;

/* Stages of one evaluation, for kldi_eval_timing. */
typedef enum {
  KLDI_STAGE_DPREP = 0,     /* D to internal tiles + block summaries a_pq                          */
  KLDI_STAGE_BASIS = 1,     /* Phi on retained tiles                                               */
  KLDI_STAGE_XGEMM = 2,     /* X = D Phi block GEMMs with the rho / grad rho epilogue              */
  KLDI_STAGE_XFUNC = 3,     /* rho reduction, functional, E_xc partials, Z on retained tiles       */
  KLDI_STAGE_VGEMM = 4,     /* M = Phi Z^T block GEMMs over grid segments                         */
  KLDI_STAGE_VFINAL = 5,    /* FP64 segment reduction, symmetrise, un-permute, E_xc sum           */
  KLDI_N_STAGES = 6
} kldi_stage;

/* Fills *opts with defaults: t_b = t_d = 1e-10, rho_cut = 1e-14, G = 128, d = 32, FP64, LDA,
 * v_segment and chunk_tiles chosen by the plan, KLDI_SCHED_GRID. */
void kldi_opts_default(kldi_opts *opts);

/* Builds the geometry-level structure reused across evaluations (Sec. III-B.3: reordering and
 * filtering once per geometry): Morton grid order and atom-grouped AO order (Sec. III-B.2,
 * eq. morton_code), grid blocks and AO tiles, shell cut-off radii, the exact block maxima of Phi
 * (and grad Phi for GGA) on the device, the retained set S_Phi with its block-compressed column
 * lists BCS(C) (Appendix C), the Vxc work list, and all device workspaces.
 * basis, grid, opts: host pointers (copied).  stream: hipStream_t or NULL.  *out receives the
 * plan, owned by the caller and released with kldi_plan_destroy.
 * Errors: KLDI_E_ARG (validation), KLDI_E_UNSUPPORTED (grid_block not 128 or 256, ao_block != 32, or more
 * than 512 retained AO tiles, i.e. 16,384 AOs, in one grid block), KLDI_E_OOM, KLDI_E_HIP.  On error
 * *out is set to NULL and nothing is leaked.  A plan with no retained tile (thresholds above every block
 * maximum) is valid: its evaluations return exact zeros. */
kldi_status kldi_plan_create(const kldi_basis *basis, const kldi_grid *grid, const kldi_opts *opts,
                             void *stream, kldi_plan **out);

/* Batching form: one plan over n_mol independent molecules (basis[m], grid[m], host arrays of n_mol
 * structs, each as for kldi_plan_create; opts shared).  All molecules live in one index space: every
 * stage of kldi_eval runs once over all of them (one launch per stage), so uneven molecules share the
 * GPU the way the tasks of one molecule do (Sec. III-D: independent tasks, one final reduction per
 * output).  Packed caller layout, offsets from kldi_batch_layout: D and Vxc of molecule m are the
 * n_ao(m) x n_ao(m) row-major blocks at d_off[m]; rho of molecule m starts at pt_off[m]; E_xc is
 * exc[m].  Errors as kldi_plan_create; n_mol >= 1. */
kldi_status kldi_batch_create(int32_t n_mol, const kldi_basis *basis, const kldi_grid *grid, const kldi_opts *opts,
                              void *stream, kldi_plan **out);

/* Offsets of the packed layout (host arrays of n_mol + 1, any may be NULL): ao_off (first AO of each
 * molecule in the stacked AO index; ao_off[n_mol] = total AOs), d_off (first element of D / Vxc),
 * pt_off (first grid point). */
kldi_status kldi_batch_layout(const kldi_plan *plan, int64_t *ao_off, int64_t *d_off, int64_t *pt_off);

/* Graph mode (enable != 0): kldi_eval launches one small kernel that records its buffers and clears
 * the counters, then replays a HIP graph captured from the plan's own launches (captured on first use,
 * recaptured after kldi_plan_attach_mlp or kldi_plan_autotune).  Results are identical to the
 * launch-by-launch path.  Per-stage timing is not recorded in graph mode. */
kldi_status kldi_plan_graph(kldi_plan *plan, int32_t enable);

typedef struct {
  int32_t v_segment;                   /* chosen grid blocks per Vxc work item                      */
  int32_t schedule;                    /* chosen kldi_schedule                                       */
  double ms;                           /* mean ms per evaluation of the chosen configuration          */
  int32_t n_tried;                     /* configurations timed; 0 when taken from the in-process cache */
} kldi_tune_t;

/* Autotuner: times evaluations of this plan with D_dev (device, packed as for kldi_eval) for each
 * candidate Vxc tile depth (v_segment in {8, 16, 32, 64} whose FP64 partials fit in memory) and each
 * kldi_schedule the plan's size admits (KLDI_SCHED_QUEUE up to 1024 grid blocks), reps timed evaluations each after one warm-up, keeps the fastest, and records it in
 * an in-process cache keyed by the plan's shape (molecules, AOs, blocks, retained tiles, functional,
 * precision) that later plans of the same shape reuse without timing.  Synchronises `stream`.
 * Writes the choice to *out (host, may be NULL).  reps >= 1; reps = 0 only consults the cache. */
kldi_status kldi_plan_autotune(kldi_plan *plan, const double *D_dev, int32_t reps, void *stream, kldi_tune_t *out);

/* Releases the plan and its device memory (synchronises its device).  NULL is a no-op. */
kldi_status kldi_plan_destroy(kldi_plan *plan);

/* Copies the plan's sizes and structure statistics to *out (host). */
kldi_status kldi_plan_info(const kldi_plan *plan, kldi_plan_info_t *out);

/* Single-molecule plans only (KLDI_E_UNSUPPORTED for batches).
 * Copies the plan's structure to caller-allocated HOST arrays (any may be NULL):
 *   ao_perm[n_ao]             internal AO index -> caller AO index
 *   pt_perm[n_points]         internal point index -> caller point index
 *   retained[n_tiles*n_blocks] 1 if (tile p, block r) is in S_Phi, at [r * n_tiles + p]
 *   phi_max[n_tiles*n_blocks]  max |Phi| of tile (p, r) if retained, else 0, at [r * n_tiles + p]
 * For tests and diagnostics (Sec. III-B.2 orders, eq. retained_blocks_B). */
kldi_status kldi_plan_structure(const kldi_plan *plan, int32_t *ao_perm, int64_t *pt_perm,
                                uint8_t *retained, double *phi_max);

/* One EXC evaluation on a ready plan (Sec. III-C): per-evaluation pair screening and
 * compaction, basis evaluation on retained tiles, X = D Phi block GEMMs with the rho / grad rho
 * epilogue, the functional, Z, the M = Phi Z^T block GEMMs, the FP64 reduction over grid
 * segments, symmetrisation and un-permutation.
 *   D_dev   [n_ao*n_ao] FP64, device, symmetric, caller AO order (read during the call only)
 *   rho_dev [n_points]  FP64, device, caller grid order, or NULL
 *   exc_dev [n_mol]     FP64, device: E_xc (one value per molecule of a batch)
 *   vxc_dev [n_ao*n_ao] FP64, device, symmetric, caller AO order, or NULL (then the M products are
 *                       skipped)
 * Only enqueues work on `stream`.  Errors: KLDI_E_ARG (NULL plan/D/exc), KLDI_E_HIP. */
kldi_status kldi_eval(kldi_plan *plan, const double *D_dev, double *rho_dev, double *exc_dev,
                      double *vxc_dev, void *stream);

/* Synchronises `stream` and copies the counters of the last kldi_eval on this plan to *out
 * (host): executed block-pair counts (the n_P of Sec. III-D), the algorithmic GEMM FLOPs they
 * imply, and whether D held a non-finite value (then returns KLDI_E_NONFINITE). */
kldi_status kldi_eval_check(kldi_plan *plan, kldi_eval_stats_t *out, void *stream);

/* rho and sigma = |grad rho|^2 on the grid for D (the density part of kldi_eval: screening, basis,
 * X = D Phi, the rho / grad rho epilogue), in caller grid order.  rho_dev, sigma_dev: [n_points]
 * FP64 device arrays, either may be NULL (not both).  sigma is |grad rho|^2 for GGA plans and 0 for
 * LDA plans.  Used, e.g., to sample the (rho, sigma) points a functional surrogate is trained on. */
kldi_status kldi_eval_grid(kldi_plan *plan, const double *D_dev, double *rho_dev, double *sigma_dev, void *stream);

/* The library's exchange-correlation functional on device arrays: f (energy per volume), v_rho =
 * df/drho and v_sigma = df/dsigma at n points, zero where rho <= rho_cut.  sigma_dev and
 * vsigma_dev may be NULL for KLDI_XC_LDA_X.  FP64 device pointers. */
kldi_status kldi_xc_eval(int32_t xc, const double *rho_dev, const double *sigma_dev, int64_t n, double rho_cut,
                         double *f_dev, double *vrho_dev, double *vsigma_dev, void *stream);

/* ---- functional surrogate (learned form; not in the paper) ---------------------------------------
 * A 2-64-64-64-3 SiLU network maps x = (n(log rho), n(log sigma)) -- n(.) the affine map of the
 * training range box onto [-1, 1], sigma floored at 1e-30 -- to three standardised heads whose
 * de-standardised values are f / rho^(4/3), v_rho / rho^(1/3) and v_sigma * rho^(4/3).  Parameters
 * (8707) are ordered W1[64][2], b1[64], W2[64][64], b2, W3[64][64], b3, W4[3][64], b4[3], W row-major
 * [out][in].  Training (FP32 master weights, Adam) and inference (BF16 weights, FP32 accumulation)
 * run in the library's own kernels.  The three heads are independent: the surrogate's v_rho, v_sigma
 * are not exact derivatives of its f. */
typedef struct kldi_mlp kldi_mlp;

typedef struct {
  uint64_t seed;                       /* parameter initialisation: U(+-1/sqrt(fan_in)), zero biases */
} kldi_mlp_cfg;

typedef struct {
  int32_t epochs;                      /* passes over the training points                          */
  int32_t batch;                       /* points per Adam step (> 0)                               */
  double lr;                           /* Adam step size (beta1 0.9, beta2 0.999, eps 1e-8)        */
  uint64_t seed;                       /* order of the points in each epoch                         */
  int32_t xc;                          /* functional providing the targets (KLDI_XC_PBE or _PBE_X)  */
  double rho_min;                      /* points below are not trained on and fall back later      */
} kldi_train_cfg;

kldi_status kldi_mlp_create(const kldi_mlp_cfg *cfg, kldi_mlp **out);
kldi_status kldi_mlp_destroy(kldi_mlp *mlp);                       /* NULL is a no-op */

/* Trains on n (rho, sigma) points (FP64 device arrays).  Points with rho < rho_min are dropped; the
 * range box is the min/max of log rho and log sigma over the rest; targets are cfg->xc evaluated by
 * the library, standardised by their mean and standard deviation.  loss_host[epochs] (host, may be
 * NULL) receives the mean standardised squared error of each epoch.  Synchronises `stream`. */
kldi_status kldi_mlp_train(kldi_mlp *mlp, const double *rho_dev, const double *sigma_dev, int64_t n,
                           const kldi_train_cfg *cfg, double *loss_host, void *stream);

/* f, v_rho, v_sigma at n points (FP64 device arrays) from the network where it covers the point
 * (rho >= rho_min, features inside the box), else from the analytic functional it was trained on.
 * used_dev[n] (device, may be NULL) receives 1 where the network was used.  KLDI_E_STATE before the
 * network has been trained (it has no range box or target statistics yet). */
kldi_status kldi_mlp_forward(const kldi_mlp *mlp, const double *rho_dev, const double *sigma_dev, int64_t n,
                             double *f_dev, double *vrho_dev, double *vsigma_dev, int32_t *used_dev, void *stream);

/* Loss and gradient of the training kernels for one batch, for checks: x_dev [n*2] features and
 * t_dev [n*3] standardised targets (FP32 device arrays), 1 <= n <= 1048576.  *loss_host = mean
 * squared error, grad_host[8707] = its gradient (host). */
kldi_status kldi_mlp_loss_grad(kldi_mlp *mlp, const float *x_dev, const float *t_dev, int64_t n, double *loss_host,
                               float *grad_host, void *stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, step size lr > 0) on one batch, for checks of
 * the update: the gradient of the batch exactly as kldi_mlp_loss_grad returns it, then the moment
 * and parameter update of the training kernels (FP32 master weights; the BF16 copy is refreshed).
 * x_dev, t_dev as for kldi_mlp_loss_grad; *loss_host (host, may be NULL) = the batch loss before the
 * step.  Advances the network's step count, which sets the bias corrections 1 - beta^k.
 * Synchronises `stream`. */
kldi_status kldi_mlp_step(kldi_mlp *mlp, const float *x_dev, const float *t_dev, int64_t n, double lr,
                          double *loss_host, void *stream);

/* Allocation-free form of kldi_mlp_step, for callers that cannot allocate device memory (code under
 * HIP graph capture, tight training loops, harnesses that forbid hipMalloc).  The same kernels and
 * results as kldi_mlp_step (identical parameters, moments and loss), but the per-workgroup partial
 * gradients live in a static device array of the library (8.9 MB, one per GPU, held until the process
 * ends) instead of memory allocated per call, so: n <= 16384 points per call (larger n is rejected
 * with KLDI_E_ARG); calls that overlap on one GPU (concurrent streams, threads) race on that array
 * and must be serialised by the caller; nothing is allocated and the stream is not synchronised.
 * *loss_dev (device, may be NULL) receives the batch loss before the step.  The step count used for
 * the bias corrections advances on the host at each call. */
kldi_status kldi_mlp_step_static(kldi_mlp *mlp, const float *x_dev, const float *t_dev, int64_t n, double lr,
                                 double *loss_dev, void *stream);

/* Basis-function order by overlap-signature clustering (Sec. III-B.2, "Locality-Preserving
 * Reordering"; appendix on reordering details, eqs. overlap_signature, cosine_similarity,
 * cosine_distance).  Row i of the overlap matrix is the signature of basis function i; functions are
 * compared by the cosine distance of their signatures; average-linkage agglomerative clustering
 * merges clusters until one remains, each merge joining the leaf sequences of its two sub-trees (the
 * earlier-formed first) with each sub-tree taken forward or reversed so that the two leaves that
 * meet are the closest of the four possible junctions.  The leaf order of the tree is the basis
 * permutation.
 *   S_host          [n_ao * n_ao] host, the symmetric overlap matrix in caller AO order (row-major;
 *                   n_ao follows from basis->shell_l), finite with no zero row
 *   ao_order_out    [n_ao] host or NULL: the leaf order (caller AO indices)
 *   shell_order_out [n_shells] host: the order the library applies (a shell's components stay
 *                   together): shells sorted stably by the first leaf position of any component;
 *                   pass it as kldi_opts.shell_order
 * Host work only, O(n_ao^2) memory and O(n_ao^3 / threads) time for the signature products.
 * Errors: KLDI_E_ARG, KLDI_E_OOM. */
kldi_status kldi_overlap_order(const kldi_basis *basis, const double *S_host, int32_t *ao_order_out,
                               int32_t *shell_order_out);

/* Host copies of the parameters (FP32 master, [8707]) and of the training statistics (box[4],
 * tmean[3], tstd[3]); any pointer may be NULL.  set_params (host) overwrites the parameters. */
kldi_status kldi_mlp_params(kldi_mlp *mlp, float *get_params, const float *set_params, double *box, double *tmean,
                            double *tstd);

/* Evaluations of a GGA plan then use the trained network in place of the analytic functional where
 * it covers a point (NULL detaches).  The plan keeps a view of the network's device memory (weights,
 * range box, target statistics), so training the network again after attaching is seen by the next
 * evaluation and by replays of a captured graph; the network must outlive the plan's use of it.
 * Errors: KLDI_E_UNSUPPORTED (LDA plan), KLDI_E_STATE (network not trained), KLDI_E_ARG (network
 * trained on another functional than the plan's). */
kldi_status kldi_plan_attach_mlp(kldi_plan *plan, const kldi_mlp *mlp);

/* Turns per-stage timing on (enable != 0) or off and clears the accumulated samples.  While on,
 * each kldi_eval records HIP events between its stages on its stream (up to 256 evaluations are
 * kept; older ones are overwritten). */
kldi_status kldi_plan_timing(kldi_plan *plan, int32_t enable);

/* Synchronises the recorded events and writes the mean duration in ms of each stage over the
 * evaluations timed since kldi_plan_timing(plan, 1) to stage_ms[KLDI_N_STAGES] (host), and their
 * number to *n_evals (host, may be NULL).  Stages that did not run (no Vxc requested) read 0. */
kldi_status kldi_eval_timing(kldi_plan *plan, double *stage_ms, int32_t *n_evals);

/* Nuclear gradient of E_xc with the grid held fixed (the EXC gradient of Sec. IV-B, Fig. 5(b); the grid
 * points and weights do not move with the atoms, a reading: the paper does not say).  The basis
 * functions of atom A move with R_A, so
 *   dE_xc/dR_Aa = -2 sum_{mu on A} sum_nu D_{mu nu} K^a_{mu nu},
 *   K^a = (d_a Phi) W^T + Q^a Phi^T,  W = w v_rho Phi + sum_b c_b d_b Phi,  Q^a = sum_b c_b d_a d_b Phi,
 * c_b = 2 w v_sigma d_b rho (zero for LDA), evaluated like the energy: Phi on retained tiles, rho and
 * the functional as kldi_eval, and each product A B^T of the Vxc shape on the tile triples (p, q, r)
 * whose operands are retained at grid block r, whose D block is retained (a_pq >= t_b) and whose
 * contribution bound a_pq max|A_pr| max|B_qr| reaches t_d (the pair filter of eq. block_pair_filter for
 * the three factors; a reading: the paper states no filter for the gradient).
 *   D_dev     as for kldi_eval (device, n_ao x n_ao, caller order)
 *   grad_dev  [n_atoms * 3] device, caller atom order, (x, y, z) per atom, Eh/bohr
 *   exc_dev   1 double on the device, or NULL: E_xc of the same evaluation
 * Single-molecule plans with KLDI_PREC_FP64 or KLDI_PREC_FP32, 128-point blocks and the analytic
 * functional (else KLDI_E_UNSUPPORTED).  FP32 plans run the X product and the gradient products on FP32
 * MFMA with FP64 running sums (the products' operands rounded to FP32, 32 points summed in FP32) and
 * contract with D in FP64.
 * Allocates its workspaces on the plan on first use (KLDI_E_OOM if they do not fit); only enqueues
 * work on `stream`. */
kldi_status kldi_eval_grad(kldi_plan *plan, const double *D_dev, double *grad_dev, double *exc_dev, void *stream);

/* Thread-local description of the last error on this thread ("" if none). */
const char *kldi_last_error(void);

/* ABI version, currently 3. */
int32_t kldi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* KLDI_H */
