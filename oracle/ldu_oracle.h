/*
 * Serial FP64 CPU oracle for the LDU pressure solve.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the plain, slow reference that
 * the GPU library is checked against.  Only the test suite, the smoke check
 * and the benchmark's CPU-baseline leg may load it; the product path never
 * calls it.  It shares no code, header or constant table with the GPU path.
 *
 * Matrix storage is OpenFOAM's lduMatrix form (paper Sec. 2.1): diag[n] plus,
 * for each internal face f, upper[f] = A[owner[f], neighbour[f]] and
 * lower[f] = A[neighbour[f], owner[f]], faces sorted by (owner, neighbour)
 * with owner < neighbour.
 *
 * Parity status of each routine is recorded in the header comment of the
 * routine in ldu_oracle.c.
 */
#ifndef LDU_ORACLE_H
#define LDU_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_OK 0
#define ORC_NOT_CONVERGED 1
#define ORC_ERR_ARG (-1)
#define ORC_ERR_ADDR (-2)
#define ORC_ERR_NAN (-3)
#define ORC_ERR_BREAKDOWN (-4)

/* addressing and value checks */
int orc_validate(int32_t n, int64_t nf, const int32_t *own, const int32_t *nb,
                 const double *diag, const double *upper, const double *lower);

/* y = A x and y = A^T x, FP64 */
void orc_amul(int32_t n, int64_t nf, const int32_t *own, const int32_t *nb,
              const double *diag, const double *upper, const double *lower,
              const double *x, double *y);
void orc_tmul(int32_t n, int64_t nf, const int32_t *own, const int32_t *nb,
              const double *diag, const double *upper, const double *lower,
              const double *x, double *y);
/* y = A x with every value, product and sum in IEEE single precision */
void orc_amul_f32(int32_t n, int64_t nf, const int32_t *own, const int32_t *nb,
                  const float *diag, const float *upper, const float *lower,
                  const float *x, float *y);

/* diagonal- (precond=1) or un-preconditioned (precond=0) CG, FP64.
 * x holds x0 on entry.  hist (may be NULL) receives ||r_k||/||b|| for
 * k = 0..iters and must hold max_iter+2 entries.  transpose=1 solves A^T x=b. */
int orc_pcg(int32_t n, int64_t nf, const int32_t *own, const int32_t *nb,
            const double *diag, const double *upper, const double *lower,
            const double *b, double *x, double tol, int max_iter, int precond,
            int transpose, int *iters, double *hist, double *true_res);

/* FP32 inner CG with FP64 iterative refinement (outer loop in FP64) */
int orc_pcg_mixed(int32_t n, int64_t nf, const int32_t *own, const int32_t *nb,
                  const double *diag, const double *upper, const double *lower,
                  const double *b, double *x, double tol, int max_refine,
                  double inner_tol, int inner_max_iter, int transpose,
                  int *refinements, int *inner_iters, double *hist,
                  double *true_res);

/* PBiCG (non-symmetric A): precond 0 none, 1 diagonal; transpose solves
 * A^T x = b */
int orc_pbicg(int32_t n, int64_t nf, const int32_t *own, const int32_t *nb,
              const double *diag, const double *upper, const double *lower,
              const double *b, double *x, double tol, int max_iter, int precond,
              int transpose, int *iters, double *hist, double *true_res);

/* ---- GAMG: pairwise agglomeration hierarchy, V-cycle, solve ---- */
typedef struct orc_gamg orc_gamg;

orc_gamg *orc_gamg_build(int32_t n, int64_t nf, const int32_t *own,
                         const int32_t *nb, const double *diag,
                         const double *upper, const double *lower,
                         int n_coarsest, int max_levels, int match_rounds);
/* passes > 1: aggressive agglomeration (pairwise matching repeated on the
 * Galerkin matrix of the previous pass, aggregates composed per level) */
orc_gamg *orc_gamg_build2(int32_t n, int64_t nf, const int32_t *own,
                          const int32_t *nb, const double *diag,
                          const double *upper, const double *lower,
                          int n_coarsest, int max_levels, int match_rounds,
                          int passes);
/* as build2, with the extra passes only on levels >= aggressive_from (the
 * finer levels keep pairwise agglomeration) */
orc_gamg *orc_gamg_build3(int32_t n, int64_t nf, const int32_t *own,
                          const int32_t *nb, const double *diag,
                          const double *upper, const double *lower,
                          int n_coarsest, int max_levels, int match_rounds,
                          int passes, int aggressive_from);
void orc_gamg_free(orc_gamg *h);
/* cycle variants: smoother (Jacobi, or two-stage Gauss-Seidel with gs_inner
 * inner steps) and the coarsest-level CG preconditioner (diagonal or DIC) */
enum { ORC_SMOOTH_JACOBI = 0, ORC_SMOOTH_GS2 = 1 };
enum { ORC_COARSE_DIAG = 0, ORC_COARSE_DIC = 1 };
int orc_gamg_set_cycle(orc_gamg *h, int smoother, int gs_inner, int coarsest_pc);
/* one two-stage Gauss-Seidel sweep on A e = r (e in/out; from_zero ignores
 * e's input); backward uses the upper triangle */
void orc_gs2_sweep(int32_t n, int64_t nf, const int32_t *own, const int32_t *nb,
                   const double *diag, const double *upper, const double *lower,
                   const double *r, double *e, int from_zero, int backward,
                   int inner);
/* the same sweep in FP32 (the smoother of the mixed-precision V-cycle) */
void orc_gs2_sweep32(int32_t n, int64_t nf, const int32_t *own, const int32_t *nb,
                     const float *diag, const float *upper, const float *lower,
                     const float *r, float *e, int from_zero, int backward,
                     int inner);
/* DIC pivots Dt (dt may be NULL) and z = M^-1 r (r, z may be NULL); returns 1
 * when every pivot is usable, 0 when the diagonal fallback applies */
int orc_dic(int32_t n, int64_t nf, const int32_t *own, const int32_t *nb,
            const double *diag, const double *upper, const double *lower,
            double *dt, const double *r, double *z);
/* new level-0 coefficients; aggregation kept, coarse matrices recomputed */
void orc_gamg_set_values(orc_gamg *h, const double *diag, const double *upper,
                         const double *lower);
int orc_gamg_nlevels(const orc_gamg *h);
void orc_gamg_level_size(const orc_gamg *h, int level, int64_t *n, int64_t *nf);
/* agg may be NULL; it is only defined for levels below the coarsest */
void orc_gamg_level_export(const orc_gamg *h, int level, int32_t *agg,
                           int32_t *own, int32_t *nb, double *diag,
                           double *upper, double *lower);
/* matching state of one level (partner, leftover join target), for tests */
void orc_gamg_level_match(const orc_gamg *h, int level, int32_t *partner,
                          int32_t *join);

/* one V-cycle e = V(0, r) (e is output only) */
int orc_gamg_vcycle(const orc_gamg *h, const double *r, double *e, int n_pre,
                    int n_post, double omega, int scale, int transpose);
/* the same V-cycle in FP32 (coarsest level solved in FP64), as the mixed-
 * precision solvers apply it */
int orc_gamg_vcycle32(const orc_gamg *h, const float *r, float *e, int n_pre,
                      int n_post, double omega, int scale, int transpose);
int orc_gamg_solve(const orc_gamg *h, const double *b, double *x, double tol,
                   int max_cycles, int n_pre, int n_post, double omega,
                   int scale, int transpose, int *cycles, double *hist,
                   double *true_res);
/* CG preconditioned by one V-cycle per iteration (scaling off) */
int orc_pcg_gamg(const orc_gamg *h, const double *b, double *x, double tol,
                 int max_iter, int n_pre, int n_post, double omega,
                 int transpose, int *iters, double *hist, double *true_res);
/* FP64 refinement around an inner FP32 CG preconditioned by an FP32 V-cycle */
int orc_pcg_gamg_mixed(const orc_gamg *h, const double *b, double *x, double tol,
                       int max_refine, double inner_tol, int inner_max_iter,
                       int n_pre, int n_post, double omega, int transpose,
                       int *refinements, int *inner_iters, double *hist,
                       double *true_res);
/* FP32 V-cycle (coarsest level in FP64) inside FP64 refinement */
int orc_gamg_mixed(const orc_gamg *h, const double *b, double *x, double tol,
                   int max_refine, int n_pre, int n_post, double omega,
                   int scale, int transpose, int *refinements, double *hist,
                   double *true_res);

/* per-face / per-cell gradients of L(x) with lambda = A^-T dL/dx:
 * g_diag = -lambda o x, g_upper[f] = -lambda[own] x[nb],
 * g_lower[f] = -lambda[nb] x[own] */
void orc_coeff_grad(int32_t n, int64_t nf, const int32_t *own,
                    const int32_t *nb, const double *lambda, const double *x,
                    double *g_diag, double *g_upper, double *g_lower);

/* pressure-equation assembly: linear interpolation of gamma to the faces,
 * fvm::laplacian coefficients, negSumDiag, divergence of phi (phi, b_bc, b
 * may be NULL; diag_bc may be NULL) */
void orc_assemble_pressure(int32_t n, int64_t nf, const int32_t *own,
                           const int32_t *nb, const double *gamma,
                           const double *w, const double *mag_sf,
                           const double *delta, const double *diag_bc,
                           const double *phi, const double *b_bc, double *diag,
                           double *upper, double *lower, double *b);

#ifdef __cplusplus
}
#endif
#endif
