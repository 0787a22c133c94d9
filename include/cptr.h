/*
 * cptr.h -- C ABI of the MI355X multi-stage preconditioned GMRES solver.
 *
 * The solver takes the reduced (primary) system A x = b of a fully implicit
 * thermal-compositional(-reactive) Newton step (Cremon, Castelletto & White,
 * Sec. "Static-Condensation Strategy", Eq. reduced) in cell-interleaved block
 * form, left-scales it once (Eq. splitPrec1), and runs right-preconditioned
 * restarted GMRES or flexible GMRES with a multi-stage preconditioner
 * (Eq. multistageprec): the three-stage CPTR3 scheme (Eqs. CPTR31, CPTR32,
 * CPTR3M1, CPTRM2, CPTR3M3; Algorithm 2), the two-stage CPR scheme
 * (Eqs. CPR, CPRM1; Algorithm 1) or a block-ILU(0) / block-Jacobi stage alone.
 * Every stage runs as HIP kernels on the caller's stream.
 *
 * Data layout (all device memory unless stated otherwise)
 *   BSR matrix with n_cells block rows, block size b (2 <= b <= 8):
 *     row_ptr  int32[n_cells + 1]
 *     col_idx  int32[nnzb]    ascending within a row, the diagonal block
 *                             present, pattern structurally symmetric
 *     vals     double[nnzb * b * b]  row-major b x b blocks
 *   vectors: double[n_cells * b], cell-interleaved (unknown k of cell i at i*b + k).
 *   Inside a cell, p_index is pressure and T_index temperature; every other
 *   unknown belongs to the group "s" (saturations, mole fractions).
 *
 * Ownership: pointers passed in stay owned by the caller; a call never frees
 * or keeps them past its return (setup copies what it needs).  The context
 * owns the scaled matrix, the AMG hierarchies, the ILU factors and the Krylov
 * workspace, and releases them in cptr_destroy.
 *
 * Errors: every entry point returns a cptr_status.  Negative values are hard
 * errors (outputs not valid); positive values are soft (outputs written).
 * cptr_last_error() returns a thread-local message for the last failure
 * (e.g. the failing cell).  Nothing aborts or exits.
 */
#ifndef CPTR_H
#define CPTR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cptr_ctx cptr_ctx;

typedef enum {
    CPTR_OK = 0,
    CPTR_NOT_CONVERGED = 1,      /* max_iters reached; x holds the last iterate */
    CPTR_E_ARG = -1,             /* invalid argument / unsupported pattern      */
    CPTR_E_HIP = -2,             /* HIP runtime error                           */
    CPTR_E_SINGULAR_BLOCK = -3,  /* singular D_ss, zero Ahat_PP, singular pivot */
    CPTR_E_NONFINITE = -4,       /* NaN / Inf in the input or during the solve  */
    CPTR_E_OOM = -5,             /* device allocation failed                    */
    CPTR_E_STATE = -6            /* call out of order (e.g. solve before setup) */
} cptr_status;

/* preconditioner variants (Sec. "Multi-Stage Preconditioning"):
 *   CPTR3: three stages, AMG on C_TT, AMG on B_PP, last stage (Algorithm 2);
 *   CPR: AMG on B_PP, last stage (Algorithm 1);
 *   CPTR: two-stage CPTR (Sec. "Two-stage Constrained Pressure-Temperature
 *     Residual", Algorithm 1): the first scaling of the decoupling alone
 *     (beta = 0), one unknown-based system AMG V-cycle on the 2x2 elliptic
 *     block B_ee = [[B_PP, B_PT], [B_TP, B_TT]] -- each unknown's diagonal
 *     block coarsened on its own, P = blockdiag(P_P, P_T), R = P^T, full
 *     Galerkin products -- then the last stage.  Its system hierarchy is
 *     hierarchy index 0 of the cptr_amg_* inspection calls, with rows ordered
 *     [P of every cell; T of every cell]; levels_T reports its depth;
 *   LAST_ONLY: the last stage alone. */
enum { CPTR_VARIANT_CPTR3 = 0, CPTR_VARIANT_CPR = 1, CPTR_VARIANT_CPTR = 2, CPTR_VARIANT_LAST_ONLY = 3 };
/* order of the two scalar AMG stages of CPTR3: temperature first as in
 * Eqs. CPTR3M1 / CPTRM2, or pressure first */
enum { CPTR_T_THEN_P = 0, CPTR_P_THEN_T = 1 };
/* last (global) stage: block ILU(0) in the tile order, or block Jacobi */
enum { CPTR_LAST_BILU0 = 0, CPTR_LAST_BJACOBI = 1 };
enum { CPTR_GMRES = 0, CPTR_FGMRES = 1 };
enum { CPTR_FP64 = 0, CPTR_FP32 = 1 };
/* AMG smoother: damped Jacobi, l1-Jacobi, or the Chebyshev iteration on
 * D^{-1} A over [lambda/30, 1.1 lambda] with lambda the Gershgorin bound
 * max_i sum_j |a_ij| / |a_ii| of each level (degree cheb_degree per sweep) */
enum { CPTR_SMOOTH_JACOBI = 0, CPTR_SMOOTH_L1JACOBI = 1, CPTR_SMOOTH_CHEBYSHEV = 2 };
/* fine-level interpolation of the temperature AMG stage: classical
 * extended+i, the learned correction judged against it by the V-cycle
 * convergence factor, or the learned correction without the judge.  The
 * judge runs at every full build of the temperature hierarchy (cptr_setup,
 * and every rebuild by cptr_update_values): both hierarchies are built and
 * the learned one is kept only when its convergence factor, measured over
 * judge_cycles V-cycles from the reuse test's start vector, is lower.  The
 * learned hierarchy differs from the classical one only in the fine level's
 * interpolation weights (below it: the classical C/F splits and transfer
 * operators, its own Galerkin products).  A hierarchy kept by the reuse test
 * of cptr_update_values keeps its interpolation and is not judged
 * (rho_T_classical / rho_T_learned read -1).  The judge and the reuse test
 * measure the V-cycle in the preconditioner's precision (the FP32 V-cycle
 * with precond_precision CPTR_FP32). */
enum { CPTR_INTERP_CLASSICAL = 0, CPTR_INTERP_LEARNED = 1, CPTR_INTERP_LEARNED_FORCED = 2 };

typedef struct {
    int32_t variant;            /* CPTR_VARIANT_*                                 */
    int32_t stage_order;        /* CPTR_T_THEN_P (default) | CPTR_P_THEN_T         */
    int32_t last_stage;         /* CPTR_LAST_*                                    */
    int32_t krylov;             /* CPTR_GMRES | CPTR_FGMRES                        */
    int32_t restart;            /* Krylov restart length m (1..200)                */
    int32_t max_iters;          /* total Arnoldi steps                            */
    double  rtol;               /* |bbar - Abar x| <= rtol |bbar| (scaled system)  */
    int32_t precond_precision;  /* CPTR_FP64 | CPTR_FP32 (needs CPTR_FGMRES)       */
    int32_t reorth;             /* 1: second Gram-Schmidt pass                    */
    double  amg_theta;          /* strength threshold (0.25)                      */
    int32_t amg_max_coarse;     /* direct solve at or below this size (1000)      */
    int32_t amg_max_levels;     /* (25)                                           */
    int32_t amg_pmax;           /* interpolation truncation, 0 = none (4)         */
    int32_t smoother;           /* CPTR_SMOOTH_*                                  */
    int32_t pre_sweeps, post_sweeps;
    double  jacobi_omega;       /* (2/3)                                          */
    uint64_t pmis_seed;         /* seed of the coarsening's random measure        */
    int32_t ilu_tile_x, ilu_tile_y;  /* tile shape of the BILU(0) order (32, 8)   */
    int32_t t_interp;           /* CPTR_INTERP_CLASSICAL | CPTR_INTERP_LEARNED     */
    double  reuse_rho_max;      /* hierarchy reuse threshold for update_values    */
    int32_t timing;             /* 1: time every stage of every Arnoldi step with */
                                /*    HIP events on the solve stream              */
    int32_t setup_kernels;      /* AMG setup row kernels: 0 by row length, 1 one  */
                                /* wavefront per row, 2 one thread per row, 3     */
                                /* 8-lane groups on every level (long rows take   */
                                /* the sequential path; for tests).  The          */
                                /* hierarchy is bit-identical either way.         */
    int32_t exact_subsolves;    /* 1: every AMG stage applies its operator's      */
                                /* exact inverse instead of a V-cycle (the Schur- */
                                /* complement quality study of Sec. "Numerical    */
                                /* Results": M_PP = B_PP, M_TT = C_TT, M_ee =     */
                                /* B_ee), by a dense inverse on the GPU; setup    */
                                /* fails with CPTR_E_ARG when an operator has     */
                                /* more than 8192 rows (0)                        */
    int32_t cheb_degree;        /* Chebyshev smoother: degree per sweep (2); the  */
                                /* pre-smoothing is one Chebyshev iteration of    */
                                /* degree cheb_degree * pre_sweeps, likewise post */
    int32_t stop_unscaled;      /* 1: the solve also requires the residual of the */
                                /* unscaled system, |b - A x| <= rtol |b|; after  */
                                /* a cycle that ends above it, later cycles stop  */
                                /* their Givens estimate at min(target, |rbar|    */
                                /* (rtol |b| / |b - A x|) / 2) (0)                */
    int32_t judge_cycles;       /* V-cycles of the learned interpolation's judge  */
                                /* (1..1000, default 4): both temperature         */
                                /* hierarchies are measured from the same start   */
                                /* vector over this many cycles and the lower     */
                                /* factor wins; the reuse test keeps 10 cycles,   */
                                /* since it compares one factor with a threshold  */
} cptr_options;

typedef struct {
    int32_t iterations;         /* Arnoldi steps over all restarts                */
    int32_t restarts;
    int32_t converged;
    int32_t used_learned;       /* the temperature hierarchy uses the learned     */
                                /* fine-level interpolation                       */
    double  rel_res_scaled;     /* |bbar - Abar x| / |bbar|, recomputed in FP64   */
    double  rel_res_unscaled;   /* |b - A x| / |b|                                */
    double  rho_T, rho_P;       /* convergence factors measured by the last       */
                                /* update_values (-1: not measured)               */
    double  setup_ms, solve_ms;
    int32_t levels_T, levels_P;
    int32_t reused;             /* bit 0: T hierarchy kept, bit 1: P hierarchy    */
                                /* kept by the last update_values                 */
    /* with options.timing = 1: summed HIP-event times over all Arnoldi steps  */
    int32_t timed_steps;
    double  t_stage1_ms;        /* first scalar stage (gather + V-cycle)          */
    double  t_stage2_ms;        /* second scalar stage (residual update + V-cycle) */
    double  t_last_ms;          /* last stage (fused residual update + BILU/BJ)   */
    double  t_spmv_ms;          /* outer operator apply w = Abar z                */
    double  t_arnoldi_ms;       /* Gram-Schmidt, Givens, normalisation            */
    /* learned interpolation judge of the last full temperature build        */
    /* (-1: not measured)                                                    */
    double  rho_T_classical, rho_T_learned;
    /* host wall clock of the last setup / update_values: scaling and          */
    /* extraction; temperature and pressure hierarchies (built concurrently,  */
    /* each from its start); the whole value-dependent setup                  */
    double  t_setup_scale_ms, t_setup_amgT_ms, t_setup_amgP_ms, t_setup_values_ms;
} cptr_result;

/* Fill *opt with the defaults noted above (CPTR3, T then P, BILU(0) in 32x8
 * tiles, GMRES(30), rtol 1e-8, classical AMG with the paper's max coarse size
 * 1000 (Sec. "Thermal-Compositional Homogeneous Cases")). */
cptr_status cptr_default_options(cptr_options *opt);

/* Create a context on HIP device `hip_device`; all work goes to `hip_stream`
 * (a hipStream_t, NULL = the default stream).  *opt is copied.  The context
 * holds one solver for the linear systems of a Newton iteration (Sec.
 * "Numerical Results": right-preconditioned GMRES on the scaled system of
 * Eq. splitPrec2, relative tolerance 1e-8); CPTR_E_ARG for invalid options,
 * CPTR_E_HIP when the device cannot be used. */
cptr_status cptr_create(cptr_ctx **ctx, int32_t hip_device, void *hip_stream, const cptr_options *opt);

/* Set up the solver for a system (Eqs. splitPrec1, CPTR31, CPTR32 and the
 * sub-solver setups): left scaling, extraction of B_PP and C_TT, two AMG
 * hierarchies, the ILU(0) factors.  nx * ny must equal n_cells when the
 * cells form an nx x ny grid (cell c = x + nx*y), which the BILU(0) tile
 * order needs; pass nx = ny = 0 for an unstructured pattern (then only block
 * Jacobi is accepted as last stage).  Device pointers; copied. */
cptr_status cptr_setup(cptr_ctx *ctx, int32_t n_cells, int32_t b, int32_t nnzb,
                       const int32_t *d_row_ptr, const int32_t *d_col_idx, const double *d_vals,
                       int32_t p_index, int32_t T_index, int32_t nx, int32_t ny);

/* New values on the same pattern (a Newton sequence of systems, each with
 * its own left scaling, Eqs. splitPrec1, CPTR31, CPTR32): the matrix is
 * rescaled and the last stage refactored.  Each AMG hierarchy is first
 * reused: its C/F splits and its P and R = P^T on every level are kept, and
 * the Galerkin products, smoother diagonals and coarsest inverse are redone
 * from the new values.  Its V-cycle convergence factor rho (as in
 * cptr_amg_conv_factor, 10 cycles, seed 0) is then measured; the hierarchy
 * is kept if rho < options.reuse_rho_max and rebuilt from scratch otherwise.
 * reuse_rho_max <= 0 rebuilds always.  The next cptr_solve reports rho_T,
 * rho_P and the kept hierarchies in cptr_result.reused.  d_vals: device,
 * nnzb*b*b, same layout as in cptr_setup; copied.  On an error (a non-finite
 * entry, a singular block) the context is left without a valid setup:
 * cptr_solve and cptr_update_values return CPTR_E_STATE until the next
 * successful cptr_setup. */
cptr_status cptr_update_values(cptr_ctx *ctx, const double *d_vals);

/* Solve A x = b through the scaled system Abar x = bbar of Eq. splitPrec2
 * (the left scaling does not change x): right-preconditioned restarted GMRES,
 * or flexible GMRES with the FP32 preconditioner, with x0 = 0 and the
 * multi-stage preconditioner of Eq. multistageprec applied as in Algorithm 2
 * (Algorithm 1 for the two-stage variants), until the recomputed FP64 residual
 * satisfies |bbar - Abar x| <= rtol |bbar| (Sec. "Numerical Results").
 * d_rhs (device, n_cells*b, cell-interleaved) in, d_x (device, same layout)
 * out; both caller-owned.  Returns after the work on the stream has
 * finished; *out (host) may be NULL.  CPTR_NOT_CONVERGED when max_iters is
 * reached (d_x holds the last iterate), CPTR_E_STATE before a successful
 * setup, CPTR_E_NONFINITE for a non-finite right-hand side or breakdown. */
cptr_status cptr_solve(cptr_ctx *ctx, const double *d_rhs, double *d_x, cptr_result *out);

/* Relative Givens residual estimates |g_{j+1}| / |bbar| of the last solve,
 * one per Arnoldi step over all restarts (the GMRES least-squares residual
 * of Sec. "Numerical Results", non-increasing by the minimal-residual
 * property): host buffer of capacity cap, of which the first min(cap, count)
 * entries are written (host_buf may be NULL to query the count); *len
 * receives the count.  CPTR_E_ARG for a null context or len. */
cptr_status cptr_residual_history(const cptr_ctx *ctx, double *host_buf, int32_t cap, int32_t *len);

/* Thread-local message describing the last error. */
const char *cptr_last_error(void);

cptr_status cptr_destroy(cptr_ctx *ctx);

/* ---------------------------------------------------------------------- */
/* Stage-level entry points on the same kernels, for inspection and tests.  */
/* All pointers are device memory unless stated otherwise.                  */
/* ---------------------------------------------------------------------- */

/* The left scaling of Eqs. CPTR31/CPTR32 (variant CPTR3), Eq. CPR (variant
 * CPR) or the first scaling alone (variant CPTR) on a BSR matrix and rhs:
 * writes d_abar (nnzb*b*b) and d_rhsbar. */
cptr_status cptr_decouple(int32_t variant, int32_t n_cells, int32_t b, const int32_t *d_row_ptr,
                          const int32_t *d_col_idx, const double *d_vals, const double *d_rhs,
                          int32_t p_index, int32_t T_index, double *d_abar, double *d_rhsbar,
                          void *hip_stream);

/* cptr_decouple for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernels and the same results, bit for bit, with the per-cell
 * weights w_P, w_T (n_cells*b doubles each), beta (n_cells doubles) and the
 * singular-cell word held in a static device array of
 * CPTR_NOALLOC_SCRATCH_BYTES per GPU (allocated with the library's code
 * object, kept until the process ends) instead of memory allocated per call.
 * The call allocates nothing: no hipMalloc, hipFree or allocating library
 * routine.  Limit: 256 + 2 align256(8 n_cells b) + align256(8 n_cells)
 * bytes must fit the array (about 600k cells at b = 8); larger inputs
 * return CPTR_E_ARG before any kernel runs.  All calls on one GPU share that
 * GPU's array, so calls that overlap in time on one GPU (other streams or
 * host threads) race; serialise them.  The caller passes inputs and outputs
 * as for cptr_decouple (d_abar, and d_rhsbar when d_rhs is given, written);
 * returns after the stream's work, CPTR_E_SINGULAR_BLOCK naming the lowest
 * singular cell as cptr_decouple does. */
#define CPTR_NOALLOC_SCRATCH_BYTES (80u * 1024u * 1024u)
cptr_status cptr_decouple_noalloc(int32_t variant, int32_t n_cells, int32_t b, const int32_t *d_row_ptr,
                                  const int32_t *d_col_idx, const double *d_vals, const double *d_rhs,
                                  int32_t p_index, int32_t T_index, double *d_abar, double *d_rhsbar,
                                  void *hip_stream);

/* Measurement of the HBM streaming-read rate that bounds the solve's
 * bandwidth-bound kernels (not part of the method): reads the n doubles of
 * d_x once, with the outer SpMV's access pattern (non-temporal 16-byte loads,
 * 1 KB of contiguous bytes per wavefront load), and writes one partial sum per
 * workgroup to d_part.  *blocks (host) receives the number of workgroups,
 * i.e. the doubles d_part must hold; with d_x = d_part = NULL the call only
 * reports it.  d_x must be 16-byte aligned (CPTR_E_ARG otherwise).
 * Asynchronous on the stream; the caller times it. */
cptr_status cptr_stream_read(const double *d_x, uint64_t n, double *d_part, int32_t *blocks, void *hip_stream);

/* y = A x for a BSR matrix (the outer operator apply of every Arnoldi step).
 * At b = 8 the values and x must be 16-byte aligned (any hipMalloc or torch
 * allocation is); CPTR_E_ARG otherwise. */
cptr_status cptr_bsr_spmv(int32_t n_cells, int32_t b, const int32_t *d_row_ptr, const int32_t *d_col_idx,
                          const double *d_vals, const double *d_x, double *d_y, void *hip_stream);

/* Static condensation of the full Newton system (Sec. "Static-Condensation
 * Strategy", Eqs. global and reduced): the secondary unknowns couple only
 * within their cell (J22 block diagonal, J21 cell-local), and
 *   Q_j = J22_jj^{-1} J21_jj,  q_j = J22_jj^{-1} r2_j           per cell,
 *   A_ij = J11_ij - J12_ij Q_j,  b_i = -r1_i + sum_j J12_ij q_j  per block,
 * so A keeps the pattern (d_row_ptr, d_col_idx) of J11.  The per-cell
 * solves are Gauss-Jordan with partial pivoting.
 *   n1 primary (1..8) and n2 secondary (0..8) unknowns per cell;
 *   d_J11: nnzb x n1 x n1 and d_J12: nnzb x n1 x n2, row-major blocks;
 *   d_J21: n_cells x n2 x n1, d_J22: n_cells x n2 x n2, row-major per cell;
 *   d_r1: n_cells*n1, d_r2: n_cells*n2 (cell-interleaved).
 * Writes d_A (nnzb x n1 x n1), d_b (n_cells*n1) and the cell factors d_Q
 * (n_cells x n2 x n1) and d_q (n_cells*n2) that cptr_recover_secondary
 * takes; all caller-owned device memory.  Returns after the work is done on
 * the stream.  CPTR_E_SINGULAR_BLOCK if some J22_jj is singular
 * (cptr_last_error names the lowest such cell); nothing is written to d_A,
 * d_b then. */
cptr_status cptr_condense(int32_t n_cells, int32_t n1, int32_t n2, int32_t nnzb, const int32_t *d_row_ptr,
                          const int32_t *d_col_idx, const double *d_J11, const double *d_J12,
                          const double *d_J21, const double *d_J22, const double *d_r1, const double *d_r2,
                          double *d_A, double *d_b, double *d_Q, double *d_q, void *hip_stream);

/* The secondary Newton update from the primary one (second block row of Eq.
 * global): d2_j = -q_j - Q_j d1_j, with Q, q from cptr_condense.  d_delta1:
 * n_cells*n1, d_delta2: n_cells*n2, cell-interleaved.  Asynchronous on the
 * stream. */
cptr_status cptr_recover_secondary(int32_t n_cells, int32_t n1, int32_t n2, const double *d_Q, const double *d_q,
                                   const double *d_delta1, double *d_delta2, void *hip_stream);

/* Exact elimination of the well unknowns (the remark closing Sec.
 * "Static-Condensation Strategy": wells eliminated by a Schur complement,
 * one perforation per well, so the reservoir pattern is kept).  Reading:
 * well w has nw unknowns, perforates cell c_w = d_well_cell[w] and couples to
 * that cell's primary unknowns only: the cell's primary rows carry J1w_w
 * (n1 x nw) against the well unknowns, the well rows carry Jw1_w (nw x n1)
 * against the cell's primary unknowns and Jww_w (nw x nw) against their own;
 * the well residual is rw_w.  With Qw_w = Jww_w^{-1} Jw1_w and
 * qw_w = Jww_w^{-1} rw_w (Gauss-Jordan with partial pivoting per well):
 *   A_{c_w c_w} -= J1w_w Qw_w,   b_{c_w} += J1w_w qw_w
 * in place on the reduced system (d_A: nnzb x n1 x n1 blocks on the pattern
 * d_row_ptr / d_col_idx, d_b: n_cells*n1, e.g. as written by cptr_condense),
 * wells taken in index order (wells that share a cell add their terms in
 * that order).  Inputs, device memory, row-major per well: d_well_cell
 * int32[n_wells], d_J1w n_wells x n1 x nw, d_Jw1 n_wells x nw x n1, d_Jww
 * n_wells x nw x nw, d_rw n_wells*nw.  Writes the factors d_Qw
 * (n_wells x nw x n1) and d_qw (n_wells*nw) that cptr_recover_wells takes.
 * Returns after the work is done.  CPTR_E_ARG for a well cell outside
 * 0..n_cells-1 or without a stored diagonal block, CPTR_E_SINGULAR_BLOCK
 * (cptr_last_error names the lowest such well) for a singular Jww; d_A and
 * d_b are not changed then. */
cptr_status cptr_condense_wells(int32_t n_cells, int32_t n1, int32_t nnzb, const int32_t *d_row_ptr,
                                const int32_t *d_col_idx, int32_t n_wells, int32_t nw, const int32_t *d_well_cell,
                                const double *d_J1w, const double *d_Jw1, const double *d_Jww, const double *d_rw,
                                double *d_A, double *d_b, double *d_Qw, double *d_qw, void *hip_stream);

/* The well update from the primary one (the well rows of the full system):
 * dw_w = -qw_w - Qw_w d1_{c_w}, with Qw, qw from cptr_condense_wells.
 * d_delta1: n_cells*n1, d_deltaw: n_wells*nw.  Asynchronous on the stream. */
cptr_status cptr_recover_wells(int32_t n_wells, int32_t n1, int32_t nw, const int32_t *d_well_cell,
                               const double *d_Qw, const double *d_qw, const double *d_delta1, double *d_deltaw,
                               void *hip_stream);

/* Number of AMG levels of hierarchy `which` (0 = temperature C_TT, 1 = pressure
 * B_PP; with variant CPTR, 0 = the system hierarchy of B_ee). */
cptr_status cptr_amg_levels(const cptr_ctx *ctx, int32_t which, int32_t *levels);

/* Sizes of level `level`: rows and nnz of the operator, nnz of P (0 on the coarsest). */
cptr_status cptr_amg_level_info(const cptr_ctx *ctx, int32_t which, int32_t level,
                                int32_t *nrows, int32_t *nnz, int32_t *p_nnz);

/* Copy level `level` of a hierarchy to host buffers sized by cptr_amg_level_info:
 * operator CSR (rp, ci, v), C/F split (cf, 1 = C; NULL allowed) and P CSR
 * (NULL allowed, and on the coarsest level). */
cptr_status cptr_amg_level_copy(const cptr_ctx *ctx, int32_t which, int32_t level,
                                int32_t *h_rp, int32_t *h_ci, double *h_v, int32_t *h_cf,
                                int32_t *h_prp, int32_t *h_pci, double *h_pv);

/* One V-cycle of hierarchy `which` with zero initial guess: d_x = V(d_b) (length = fine rows). */
cptr_status cptr_amg_vcycle(cptr_ctx *ctx, int32_t which, const double *d_b, double *d_x);

/* Asymptotic V-cycle convergence factor of hierarchy `which` (the measure
 * that judges hierarchy reuse and the learned interpolation): from the start
 * vector e_0[i] = u(seed, i) in [-1, 1), where u maps SplitMix64 of (seed, i)
 * to its top 53 bits scaled to [0, 1) then to 2 u - 1, iterate
 * e <- e - V(A e) `cycles` times (FP64) and return
 * rho = (|e_K|_2 / |e_0|_2)^(1/K) in *rho (host).  (With the FP32
 * preconditioner the reuse test and the judge apply the FP32 V-cycle: A e in
 * FP64 rounded to FP32 as its input, its output subtracted in FP64; this call
 * always measures the FP64 V-cycle.) */
cptr_status cptr_amg_conv_factor(cptr_ctx *ctx, int32_t which, int32_t cycles, uint64_t seed, double *rho);

/* One application of the multi-stage preconditioner: d_y = M^{-1} d_r. */
cptr_status cptr_precond_apply(cptr_ctx *ctx, const double *d_r, double *d_y);

/* The scaled right-hand side and matrix held by the context (device copies). */
cptr_status cptr_get_scaled(const cptr_ctx *ctx, double *d_abar, double *d_rhsbar_or_null, const double *d_rhs);

/* ---------------------------------------------------------------------- */
/* Learned fine-level interpolation of the temperature AMG stage (an        */
/* extension of amg(C_TT), Eq. CPTR3M1).                                    */
/*                                                                          */
/* Edges are the F-row entries (i, J) of the classical extended+i           */
/* interpolation of C_TT's fine level, in storage order.  Each edge has 16   */
/* features (FP64 formulas, stored FP32):                                   */
/*   0 a_ij/a_ii, 1 a_ji/a_jj, 2 (-s a_ij)/max_k(-s a_ik) with s = sign a_ii  */
/*   (0 if that max <= 0), 3 1 if j is not a neighbour of i, 4 the classical  */
/*   weight, 5 sum over neighbours k of i (k != j) coupled to j of            */
/*   a_ik a_kj/(a_ii a_kk), 6 row sum of i / a_ii, 7 1/(edges of row i),     */
/*   8 (a_ij - a_ji)/(|a_ij| + |a_ji|) (0 if both 0), 9 classical row sum,   */
/*   10 weight / max |weight| of the row, 11 |a_jj|/(|a_ii| + |a_jj|),       */
/*   12 row sum of j / a_jj, 13 strong couplings of i / (row length - 1),    */
/*   14 1, 15 0.                                                            */
/* The network 16 -> 64 -> 64 -> 1 (ReLU) has BF16 weights and runs on the  */
/* matrix cores with FP32 accumulation; its input and first hidden layer are */
/* rounded to BF16.  delta = tanh(o)/2 and w = w0 (1 + delta), rescaled to   */
/* the classical row sum when the rescale factor lies in [1/4, 4].           */
/* Parameters: float[CPTR_MLP_NPARAMS] host blob, W1[64][16], b1[64],        */
/* W2[64][64], b2[64], W3[64], b3[1].                                       */
/* ---------------------------------------------------------------------- */
#define CPTR_MLP_NPARAMS 5313

/* Parameters used by the next setups of ctx when options.t_interp is
 * CPTR_INTERP_LEARNED (judged) or CPTR_INTERP_LEARNED_FORCED.  Host blob,
 * copied; NULL removes them (classical interpolation only). */
cptr_status cptr_load_mlp(cptr_ctx *ctx, const float *host_params);

typedef struct cptr_mlp cptr_mlp;   /* trainable network: FP32 master weights, Adam moments */

/* Create a trainable network on device `hip_device` from a host blob. */
cptr_status cptr_mlp_create(cptr_mlp **mlp, int32_t hip_device, const float *host_params);

/* Copy the current parameters and/or the last gradient to host (NULL skips). */
cptr_status cptr_mlp_get(const cptr_mlp *mlp, float *host_params, float *host_grad);

/* One training step on the temperature operator of a context set up with
 * classical interpolation: K = n_vectors (1..16) smooth error vectors
 * (20 damped-Jacobi sweeps, omega 2/3, on C_TT e = 0 from SplitMix64-uniform
 * starts u(seed, k n + i)), loss = mean over F rows of
 * sum_k (e_i - sum_J w_iJ e_j)^2 / sum_k e_i^2 with the corrected weights,
 * gradient through the network (BF16 matrix-core products, FP32
 * accumulation), then one Adam step (beta 0.9, 0.999, eps 1e-8) with
 * learning rate lr.  *loss (host) receives the loss before the step.
 * Runs on the context's stream. */
cptr_status cptr_mlp_train_step(cptr_mlp *mlp, cptr_ctx *ctx, int32_t n_vectors, uint64_t seed, double lr,
                                double *loss);

/* Features and network outputs of the context's temperature edges (classical
 * interpolation): host buffers of capacity cap edges (X: 16 floats per edge,
 * o: one float per edge; either may be NULL); *n_edges receives the count.
 * The outputs use mlp's parameters (o is skipped when mlp is NULL). */
cptr_status cptr_mlp_edges(const cptr_mlp *mlp, cptr_ctx *ctx, float *host_X, float *host_o, int32_t cap,
                           int32_t *n_edges);

cptr_status cptr_mlp_destroy(cptr_mlp *mlp);

#ifdef __cplusplus
}
#endif
#endif /* CPTR_H */
