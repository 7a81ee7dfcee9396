/*
 * ldu.h -- C ABI of the MI355X (gfx950) LDU pressure-solve library.
 *
 * The library solves A x = b for one scalar matrix stored in OpenFOAM's
 * lduMatrix form (paper Sec. 2.1, "Design aspects"): a diagonal per cell and,
 * per internal face f, an upper coefficient A[owner[f], neighbour[f]] and a
 * lower coefficient A[neighbour[f], owner[f]].  It provides the product
 * y = A x and its transpose (the "Amul" and "Tmul" SpMVM kernels of the
 * profiling table, Sec. 4.3), conjugate gradients with the diagonal
 * preconditioner and the GAMG solver with the Richardson (damped Jacobi)
 * smoother and a diagonal-PCG coarsest level (the pressure solvers of
 * Appendix A and of the smoother table in Sec. 4.3), an FP32-bulk variant
 * with FP64 iterative refinement, and the adjoint solve with per-face
 * coefficient gradients.
 *
 * Conventions shared by every call:
 *  - Array arguments are DEVICE pointers (HIP device memory of the current
 *    device), borrowed for the duration of the call only.  The library never
 *    frees or retains them.  Counts are in elements.
 *  - hip_stream is a hipStream_t (NULL = the legacy default stream).  All
 *    device work of a call is ordered on that stream.  Calls that return a
 *    solver status synchronise that stream before returning.
 *  - A handle owns all device memory it allocates; allocation happens in
 *    ldu_create, gamg_setup and the first call of a solver variant, never
 *    inside an iteration.  A handle is not thread-safe and must be used from
 *    one stream at a time.
 *  - Return values: LDU_OK (0) or LDU_NOT_CONVERGED (1, result usable, stats
 *    filled) or a negative error.  After a negative return, output arrays are
 *    unspecified and ldu_last_error() describes the failure.  After
 *    LDU_ERR_HIP the handle is poisoned and later calls return LDU_ERR_STATE.
 *  - Residuals are ||b - A x||_2 / ||b||_2, computed in FP64 on the device.
 *    b = 0 yields x = 0 with zero iterations.
 */
#ifndef LDU_H
#define LDU_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LDU_ABI_VERSION 1

enum {
    LDU_OK = 0,
    LDU_NOT_CONVERGED = 1,
    LDU_ERR_ARG = -1,       /* bad argument (null pointer, size, option) */
    LDU_ERR_ADDR = -2,      /* face addressing violates the LDU contract */
    LDU_ERR_NAN = -3,       /* non-finite coefficient, rhs or residual */
    LDU_ERR_BREAKDOWN = -4, /* CG breakdown: |p.Ap| <= 1e-300 */
    LDU_ERR_NOMEM = -5,     /* device allocation failed */
    LDU_ERR_HIP = -6,       /* HIP runtime error; handle poisoned */
    LDU_ERR_STATE = -7,     /* poisoned handle or call out of order */
    LDU_ERR_LIMIT = -8      /* a structural limit of the library was hit */
};

enum { LDU_FP64 = 0, LDU_MIXED = 1 };
/* GAMG smoothers and coarsest-level CG preconditioners (Sec. 4.3 compares
 * both smoothers and both coarsest preconditioners) */
enum { LDU_SMOOTH_JACOBI = 0, LDU_SMOOTH_GS2 = 1 };
enum { LDU_COARSE_DIAG = 0, LDU_COARSE_DIC = 1 };

typedef struct ldu_t *ldu_handle;

/* Options of pcg_solve.  Defaults (ldu_pcg_default_opts): rel_tol 1e-8,
 * abs_tol 0, max_iter 10000, check_every 16, precond 1 (diagonal),
 * precision LDU_FP64, max_refine 50, inner_rel_tol 1e-4,
 * inner_max_iter 1000. */
typedef struct {
    double rel_tol;       /* stop at ||r||/||b|| <= rel_tol */
    double abs_tol;       /* unused, reserved: must be 0 */
    int max_iter;         /* FP64: CG iterations; MIXED: per inner solve cap is inner_max_iter */
    int check_every;      /* host reads the convergence flag every k iterations (>= 1) */
    int precond;          /* 0 none, 1 diagonal, 2 one GAMG V-cycle (the handle's
                             hierarchy and sweep settings from gamg_setup, or the
                             defaults; correction scaling off so that the
                             preconditioner is symmetric, which also needs
                             n_pre == n_post; FP32 V-cycle in MIXED) */
    int precision;        /* LDU_FP64 or LDU_MIXED */
    int max_refine;       /* MIXED: outer refinement steps */
    int inner_max_iter;   /* MIXED: FP32 CG iterations per refinement */
    double inner_rel_tol; /* MIXED: inner stop at ||r32||/||rhat|| <= max(this,
                             0.3 rel_tol / current outer residual) */
} ldu_pcg_opts;

/* Options of gamg_setup / gamg_solve.  Defaults (ldu_gamg_default_opts):
 * rel_tol 1e-8, max_cycles 200, n_coarsest 50, n_pre 2, n_post 2,
 * max_levels 50, scale_correction 1, match_rounds 16, precision LDU_FP64,
 * max_refine 200, omega 0.75, passes 1, aggressive_from 0, smoother LDU_SMOOTH_JACOBI,
 * gs_inner 1, coarsest LDU_COARSE_DIAG. */
typedef struct {
    double rel_tol;
    double abs_tol;        /* unused, reserved: must be 0 */
    int max_cycles;        /* FP64: V-cycles; MIXED: see max_refine */
    int n_coarsest;        /* coarsen while a level has more cells than this */
    int n_pre, n_post;     /* Jacobi sweeps before / after the coarse correction */
    int max_levels;        /* including the finest level, <= 64 */
    int scale_correction;  /* 1: scale the prolonged correction (energy optimal) */
    int match_rounds;      /* handshake matching rounds per level */
    int precision;         /* LDU_FP64 or LDU_MIXED */
    int max_refine;        /* MIXED: refinement steps (one FP32 V-cycle each) */
    double omega;          /* Jacobi relaxation factor */
    int passes;            /* pairwise matching passes per level (1..3): pass k
                            * matches the aggregates of pass k-1 on their
                            * Galerkin matrix, so aggregates hold up to about
                            * 2^passes cells and the hierarchy has fewer levels
                            * (aggressive agglomeration, the remedy the paper
                            * points to for GAMG's many tiny levels, Sec. 4.4) */
    int aggressive_from;   /* first level coarsened with `passes` passes; finer
                            * levels keep one pass (0: every level) */
    int smoother;          /* LDU_SMOOTH_JACOBI: damped Jacobi (Richardson) with
                            * omega; LDU_SMOOTH_GS2: two-stage Gauss-Seidel
                            * (Berger-Vergiat et al. 2021): each sweep corrects
                            * e by gs_inner Jacobi-Richardson steps that
                            * approximate (D + L)^-1 (r - A e); forward sweeps
                            * before the coarse correction, backward (D + U)
                            * after it; omega unused */
    int gs_inner;          /* inner steps per two-stage sweep, 1..8 */
    int coarsest;          /* coarsest-level CG preconditioner: LDU_COARSE_DIAG,
                            * or LDU_COARSE_DIC (diagonal incomplete Cholesky,
                            * M = (Dt + L) Dt^-1 (Dt + U) with diag(M) = diag(A);
                            * falls back to the diagonal when a pivot is not
                            * usable) */
} ldu_gamg_opts;

typedef struct {
    int iterations;        /* CG iterations, V-cycles, or (MIXED) inner CG iterations */
    int refinements;       /* MIXED: outer refinement steps; FP64: 0 */
    int converged;         /* 1 if the final true residual meets rel_tol */
    int n_levels;          /* GAMG levels (0 for PCG) */
    double initial_residual; /* ||b - A x0|| / ||b|| */
    double final_residual;   /* ||b - A x|| / ||b|| recomputed in FP64 */
    long long level_cells[64];
    long long level_faces[64];
    double *history;       /* optional HOST buffer for the residual history
                              (entry k: residual after iteration or cycle k; a
                              solve keeps its first 2^20 entries) */
    int history_len;       /* its capacity (entries) */
    int history_count;     /* entries written */
} ldu_stats;

void ldu_pcg_default_opts(ldu_pcg_opts *o);
void ldu_gamg_default_opts(ldu_gamg_opts *o);

/* Create a matrix handle from LDU arrays (Sec. 2.1).
 * owner, neighbour: int32[nFaces] with 0 <= owner[f] < neighbour[f] < nCells,
 *   sorted by (owner, neighbour), no duplicates (OpenFOAM's upper-triangular
 *   face order); otherwise LDU_ERR_ADDR.
 * diag: double[nCells]; upper, lower: double[nFaces]; non-finite -> LDU_ERR_NAN.
 * The arrays are copied; the matrix is re-laid on the device into row
 * segments (the LDU -> row-ordered conversion map of Sec. 3.4) for the
 * product kernels.  nCells >= 1, nFaces >= 0, 2*nFaces + padding < 2^31. */
int ldu_create(int32_t nCells, int64_t nFaces, const int32_t *owner,
               const int32_t *neighbour, const double *diag,
               const double *upper, const double *lower, void *hip_stream,
               ldu_handle *out);

/* Replace the coefficients, keeping the addressing.  A GAMG hierarchy that
 * was set up keeps its agglomeration and recomputes its coarse matrices
 * (agglomeration caching, Sec. 2.1 and Sec. 4.4). */
int ldu_set_coeffs(ldu_handle h, const double *diag, const double *upper,
                   const double *lower, void *hip_stream);

int ldu_destroy(ldu_handle h);

/* y = A x  (Amul), FP64; x, y: double[nCells], must not alias. */
int ldu_amul(ldu_handle h, const double *x, double *y, void *hip_stream);
/* y = A^T x  (Tmul): upper and lower exchanged. */
int ldu_tmul(ldu_handle h, const double *x, double *y, void *hip_stream);
/* y = A x with FP32 values (rounded from the FP64 coefficients), FP32
 * vectors and FP32 accumulation. */
int ldu_amul_f32(ldu_handle h, const float *x, float *y, void *hip_stream);

/* ||b - A x||_2 / ||b||_2 in FP64 (0 when b = 0); *out is a HOST double. */
int ldu_residual(ldu_handle h, const double *b, const double *x, double *out,
                 void *hip_stream);

/* Conjugate gradients for A x = b, A symmetric definite (either sign), with
 * the diagonal preconditioner (Appendix A, "PCG / diagonal") or a GAMG
 * V-cycle preconditioner (the PCG + AMG pairing of the paper's AmgX
 * configuration, Appendix A listing).  x: in = initial guess, out = solution.
 * opts may be NULL (defaults); stats may be NULL.  precision LDU_MIXED runs
 * FP32 inner CG solves inside FP64 refinement.  Exceeding the iteration
 * budget returns LDU_NOT_CONVERGED with the last iterate. */
int pcg_solve(ldu_handle h, const double *b, double *x,
              const ldu_pcg_opts *opts, ldu_stats *stats, void *hip_stream);

/* pcg_solve without any device allocation, for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, kernels and results as pcg_solve with
 * precond 0 or 1 and precision LDU_FP64 (anything else: LDU_ERR_ARG).  The
 * CG vectors, reduction partials and residual history live in a static
 * device array of the library (24.1 MiB per GPU, held until the process
 * ends), not in the handle: nCells must be at most 1,048,576 (else
 * LDU_ERR_LIMIT) and at most the first 4096 history entries are kept.
 * Every call on one GPU shares that array, so calls that overlap on a GPU
 * (other streams or threads) race.  The handle itself is created by
 * ldu_create, which allocates. */
int pcg_solve_noalloc(ldu_handle h, const double *b, double *x,
                      const ldu_pcg_opts *opts, ldu_stats *stats, void *hip_stream);

/* PBiCG for non-symmetric A (the paper's solver for the velocity and
 * turbulence systems, Appendix A): preconditioned bi-conjugate gradients with
 * the shadow residual equal to the residual at each (re)start, one fused
 * Amul + Tmul pass per iteration.  opts->precond 0 (none) or 1 (diagonal);
 * precision must be LDU_FP64.  x holds x0 on entry.  The first call on a
 * handle allocates its three shadow vectors.  LDU_ERR_BREAKDOWN when
 * |pt.A p| or |(M^-1 r).rt| falls to 1e-300. */
int pbicg_solve(ldu_handle h, const double *b, double *x,
                const ldu_pcg_opts *opts, ldu_stats *stats, void *hip_stream);

/* Build the GAMG hierarchy (agglomeration + Galerkin coarse matrices); done
 * lazily by gamg_solve otherwise.  Calling it again rebuilds. */
int gamg_setup(ldu_handle h, const ldu_gamg_opts *opts, void *hip_stream);

/* GAMG as a solver: per cycle, r = b - A x in FP64 and x += V(r).
 * precision LDU_MIXED: FP32 V-cycles (FP64 coarsest) inside FP64 refinement. */
int gamg_solve(ldu_handle h, const double *b, double *x,
               const ldu_gamg_opts *opts, ldu_stats *stats, void *hip_stream);

/* One V-cycle e = V(r) from e = 0 (FP64); e, r: double[nCells]. */
int gamg_vcycle(ldu_handle h, const double *r, double *e,
                const ldu_gamg_opts *opts, void *hip_stream);

/* GAMG hierarchy inspection (for tests and tools).
 * gamg_level_size: cells and faces of level l (HOST outputs).
 * gamg_level_export: DEVICE outputs, any may be NULL: agg int32[n_l]
 *   (coarse cell of each cell; not defined on the coarsest level), owner,
 *   neighbour int32[nf_l], diag double[n_l], upper, lower double[nf_l]. */
int gamg_level_size(ldu_handle h, int level, int64_t *n_cells,
                    int64_t *n_faces);
int gamg_level_export(ldu_handle h, int level, int32_t *agg, int32_t *owner,
                      int32_t *neighbour, double *diag, double *upper,
                      double *lower, void *hip_stream);
/* Storage of level l's matrix in the product kernels (level 0 needs no GAMG
 * hierarchy; HOST outputs, either may be NULL).  compressed: 1 when the rows
 * sit in length-sorted compressed slices, 0 in plain slices of 64 rows.
 * col16: 1 when the kernels read columns as 16-bit offsets from the
 * smallest column of their slot (the k-th entries of a slice's rows) for the
 * slots that span at most 65535 columns, the others reading 32-bit columns;
 * 0 when every slot reads 32-bit columns.  Either way the products are the
 * same bit for bit. */
int ldu_level_layout(ldu_handle h, int level, int *compressed, int *col16);
/* The form of level l's one-pass down leg, r_c = P^T (I - omega A D^-1) r,
 * which cycles with one Jacobi pre-sweep from zero and no correction scaling
 * use (HOST outputs, lanes may be NULL): 0 not built (the coarsest level, or
 * no such cycle has run on this hierarchy); 1 the operator R in compressed
 * slices; 2 R in CSR, with *lanes lanes per row; 3 a product over the
 * level's own slices with stored values -omega a_ij / D_j, then the member
 * sums.  LDU_ERR_STATE without a hierarchy, LDU_ERR_ARG for a bad level. */
int ldu_level_downleg(ldu_handle h, int level, int *form, int *lanes);

/* Adjoint solve A^T lambda = g on the transposed coefficients (upper and
 * lower exchanged on every level) with solver 0: PCG (opts is an
 * ldu_pcg_opts*), 1: GAMG (an ldu_gamg_opts*), or 2: PBiCG (an
 * ldu_pcg_opts*; for non-symmetric A). */
enum { LDU_SOLVER_PCG = 0, LDU_SOLVER_GAMG = 1, LDU_SOLVER_PBICG = 2 };
int ldu_adjoint_solve(ldu_handle h, const double *g, double *lambda,
                      int solver, const void *opts, ldu_stats *stats,
                      void *hip_stream);

/* Pressure-equation assembly on the handle's mesh, replacing its
 * coefficients (the step before each pressure solve of a SIMPLE iteration;
 * Sec. 4.3 profiles its negSumDiag, interpolation and divergence kernels):
 *   gamma_f = w_f gamma[owner] + (1 - w_f) gamma[neighbour]
 *   upper_f = lower_f = gamma_f mag_sf_f delta_f
 *   diag_i  = -(sum of the off-diagonal coefficients in column i) - diag_bc_i
 *   b_i     = sum_{owner(f)=i} phi_f - sum_{neighbour(f)=i} phi_f + b_bc_i
 * gamma, diag_bc, b_bc, b: [n_cells]; weights, mag_sf, delta, phi: [n_faces]
 * in the handle's face order; all device pointers.  diag_bc, b_bc may be
 * NULL (zero).  b may be NULL (no right-hand side); when it is given, phi is
 * required unless the mesh has no faces, and a phi without b is an error.
 * diag, upper, lower (may be NULL) receive copies of the assembled
 * coefficients.  A cached GAMG hierarchy keeps its aggregation and gets new
 * Galerkin values, as with ldu_set_coeffs.  Rows sum their faces in the
 * serial face loop's order, so results are deterministic.  LDU_ERR_NAN if a
 * coefficient comes out non-finite (the handle's values are then
 * unspecified until the next successful assembly or ldu_set_coeffs). */
int ldu_assemble_pressure(ldu_handle h, const double *gamma, const double *weights,
                          const double *mag_sf, const double *delta,
                          const double *diag_bc, const double *phi,
                          const double *b_bc, double *b, double *diag,
                          double *upper, double *lower, void *hip_stream);

/* Gradients of a loss L through A x = b given lambda = A^-T dL/dx:
 * g_diag[i] = -lambda[i] x[i], g_upper[f] = -lambda[owner[f]] x[neighbour[f]],
 * g_lower[f] = -lambda[neighbour[f]] x[owner[f]] (and dL/db = lambda).
 * Outputs in the caller's face order; any output may be NULL. */
int ldu_coeff_grad(ldu_handle h, const double *lambda, const double *x,
                   double *g_diag, double *g_upper, double *g_lower,
                   void *hip_stream);

/* Description of the last error on the calling thread. */
const char *ldu_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
