/*
 * Serial FP64 CPU oracle for the LDU pressure solve -- TEST INFRASTRUCTURE.
 *
 * Plain, slow and written to be checked by eye against the definitions it
 * cites.  Build with -O2 -ffp-contract=off (no fused multiply-add, no
 * re-association), so every expression below rounds exactly as written.
 *
 * The paper names the solvers it runs (lduMatrix Amul/Tmul, PCG with the
 * diagonal preconditioner, GAMG with the Richardson i.e. damped-Jacobi
 * smoother and a diagonal-PCG coarsest solve; Sec. 4.3 profiling table and
 * smoother table, Appendix A solver tables) but does not define them; each
 * routine here is the textbook method, and each choice the paper leaves open
 * is stated where it is made.
 *
 * Parity pins (tests that fix each routine independently of itself) live in
 * tests/test_oracle_*.py.  Routines without an independent pin say
 * "parity unpinned" below.
 */
#include "ldu_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* small helpers                                                             */
/* ------------------------------------------------------------------------ */

static void *xcalloc(size_t n, size_t sz) {
    void *p = calloc(n ? n : 1, sz);
    if (!p) abort();
    return p;
}

static double dot(int32_t n, const double *a, const double *b) {
    double s = 0.0;
    for (int32_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

static double dot_f32(int32_t n, const float *a, const float *b) {
    /* single-precision vectors, products and sum in double */
    double s = 0.0;
    for (int32_t i = 0; i < n; ++i) s += (double)a[i] * (double)b[i];
    return s;
}

/* ------------------------------------------------------------------------ */
/* validation: OpenFOAM upper-triangular face order (Sec. 2.1)               */
/* ------------------------------------------------------------------------ */

int orc_validate(int32_t n, int64_t nf, const int32_t *own, const int32_t *nb,
                 const double *diag, const double *upper, const double *lower) {
    if (n < 0 || nf < 0) return ORC_ERR_ARG;
    for (int64_t f = 0; f < nf; ++f) {
        if (own[f] < 0 || own[f] >= nb[f] || nb[f] >= n) return ORC_ERR_ADDR;
        if (f > 0) {
            if (own[f] < own[f - 1]) return ORC_ERR_ADDR;
            if (own[f] == own[f - 1] && nb[f] <= nb[f - 1]) return ORC_ERR_ADDR;
        }
    }
    if (diag)
        for (int32_t i = 0; i < n; ++i)
            if (!isfinite(diag[i])) return ORC_ERR_NAN;
    for (int64_t f = 0; f < nf; ++f) {
        if (upper && !isfinite(upper[f])) return ORC_ERR_NAN;
        if (lower && !isfinite(lower[f])) return ORC_ERR_NAN;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Amul / Tmul: the lduMatrix face-loop product (Sec. 4.3, "SpMVM (Amul +    */
/* Tmul)" in the kernel time breakdown).                                      */
/*   y = diag o x;  for each face f in order:                                 */
/*       y[nb] += lower*x[own];  y[own] += upper*x[nb]                        */
/* Tmul is the same loop with upper and lower exchanged (A^T).               */
/* Pins: dense matvec, closed-form eigenpairs, dense transpose.              */
/* ------------------------------------------------------------------------ */

void orc_amul(int32_t n, int64_t nf, const int32_t *own, const int32_t *nb,
              const double *diag, const double *upper, const double *lower,
              const double *x, double *y) {
    for (int32_t i = 0; i < n; ++i) y[i] = diag[i] * x[i];
    for (int64_t f = 0; f < nf; ++f) {
        y[nb[f]] += lower[f] * x[own[f]];
        y[own[f]] += upper[f] * x[nb[f]];
    }
}

void orc_tmul(int32_t n, int64_t nf, const int32_t *own, const int32_t *nb,
              const double *diag, const double *upper, const double *lower,
              const double *x, double *y) {
    orc_amul(n, nf, own, nb, diag, lower, upper, x, y);
}

void orc_amul_f32(int32_t n, int64_t nf, const int32_t *own, const int32_t *nb,
                  const float *diag, const float *upper, const float *lower,
                  const float *x, float *y) {
    for (int32_t i = 0; i < n; ++i) y[i] = diag[i] * x[i];
    for (int64_t f = 0; f < nf; ++f) {
        y[nb[f]] += lower[f] * x[own[f]];
        y[own[f]] += upper[f] * x[nb[f]];
    }
}

/* a matrix view; transpose is handled by exchanging upper and lower */
typedef struct {
    int32_t n;
    int64_t nf;
    const int32_t *own, *nb;
    const double *diag, *up, *lo;
} omat;

static omat make_mat(int32_t n, int64_t nf, const int32_t *own,
                     const int32_t *nb, const double *diag, const double *upper,
                     const double *lower, int transpose) {
    omat m = {n, nf, own, nb, diag, transpose ? lower : upper,
              transpose ? upper : lower};
    return m;
}

static void mat_mul(const omat *m, const double *x, double *y) {
    orc_amul(m->n, m->nf, m->own, m->nb, m->diag, m->up, m->lo, x, y);
}

/* r = b - A x */
static void residual(const omat *m, const double *b, const double *x,
                     double *r) {
    mat_mul(m, x, r);
    for (int32_t i = 0; i < m->n; ++i) r[i] = b[i] - r[i];
}

/* ------------------------------------------------------------------------ */
/* CG with the diagonal preconditioner (Appendix A: "PCG / diagonal" for p). */
/* Hestenes-Stiefel recurrences:                                              */
/*   r = b - A x0; z = D^-1 r; p = z; rho = r.z                               */
/*   repeat: q = A p; alpha = rho/(p.q); x += alpha p; r -= alpha q;          */
/*           stop if ||r||/||b|| <= tol;                                       */
/*           z = D^-1 r; rho' = r.z; beta = rho'/rho; p = z + beta p          */
/* On exit the true residual b - A x is recomputed; if it is above tol the    */
/* iteration restarts from it while iterations remain.                        */
/* Pins: dense solve, finite termination on closed-form eigenvectors,         */
/* manufactured solution.                                                     */
/* ------------------------------------------------------------------------ */

typedef struct {
    double *r, *z, *p, *q;
} cg_work;

/* preconditioner z = M^-1 r: 0 identity, 1 diagonal, or a callback */
typedef void (*precond_fn)(void *ctx, const double *r, double *z);

static void apply_precond(const omat *m, int precond, precond_fn fn, void *ctx,
                          const double *r, double *z) {
    if (fn) {
        fn(ctx, r, z);
        return;
    }
    for (int32_t i = 0; i < m->n; ++i) z[i] = precond ? r[i] / m->diag[i] : r[i];
}

/* one CG run from the residual already in w->r; returns ORC_OK when the
 * recursive residual reached tol, ORC_NOT_CONVERGED when *total hit max_iter */
static int cg_run_pc(const omat *m, int precond, precond_fn fn, void *ctx,
                     double *x, cg_work *w, double bnorm, double tol,
                     int max_iter, int *total, double *hist) {
    const int32_t n = m->n;
    double *r = w->r, *z = w->z, *p = w->p, *q = w->q;
    apply_precond(m, precond, fn, ctx, r, z);
    for (int32_t i = 0; i < n; ++i) p[i] = z[i];
    double rho = dot(n, r, z);
    while (*total < max_iter) {
        mat_mul(m, p, q);
        double pq = dot(n, p, q);
        if (!isfinite(pq) || fabs(pq) <= 1e-300) return ORC_ERR_BREAKDOWN;
        double alpha = rho / pq;
        for (int32_t i = 0; i < n; ++i) x[i] = x[i] + alpha * p[i];
        for (int32_t i = 0; i < n; ++i) r[i] = r[i] - alpha * q[i];
        *total += 1;
        double res = sqrt(dot(n, r, r)) / bnorm;
        if (hist) hist[*total] = res;
        if (!isfinite(res)) return ORC_ERR_NAN;
        if (res <= tol) return ORC_OK;
        apply_precond(m, precond, fn, ctx, r, z);
        double rho_new = dot(n, r, z);
        double beta = rho_new / rho;
        rho = rho_new;
        for (int32_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
    }
    return ORC_NOT_CONVERGED;
}

static int cg_run(const omat *m, int precond, double *x, cg_work *w,
                  double bnorm, double tol, int max_iter, int *total,
                  double *hist) {
    return cg_run_pc(m, precond, NULL, NULL, x, w, bnorm, tol, max_iter, total,
                     hist);
}

/* CG driver with restarts from the true residual (shared by every
 * preconditioner) */
static int cg_solve(const omat *m, int precond, precond_fn fn, void *ctx,
                    const double *b, double *x, double tol, int max_iter,
                    int *iters, double *hist, double *true_res) {
    const int32_t n = m->n;
    int total = 0;
    double bnorm = sqrt(dot(n, b, b));
    if (iters) *iters = 0;
    if (bnorm == 0.0) {
        for (int32_t i = 0; i < n; ++i) x[i] = 0.0;
        if (hist) hist[0] = 0.0;
        if (true_res) *true_res = 0.0;
        return ORC_OK;
    }
    cg_work w;
    w.r = xcalloc(n, sizeof(double));
    w.z = xcalloc(n, sizeof(double));
    w.p = xcalloc(n, sizeof(double));
    w.q = xcalloc(n, sizeof(double));
    residual(m, b, x, w.r);
    double res = sqrt(dot(n, w.r, w.r)) / bnorm;
    if (hist) hist[0] = res;
    int st = ORC_OK;
    if (!isfinite(res)) {
        st = ORC_ERR_NAN;
    } else {
        while (res > tol) {
            st = cg_run_pc(m, precond, fn, ctx, x, &w, bnorm, tol, max_iter,
                           &total, hist);
            if (st < 0) break;
            residual(m, b, x, w.r); /* true residual, restart point */
            res = sqrt(dot(n, w.r, w.r)) / bnorm;
            if (res <= tol) { st = ORC_OK; break; }
            if (total >= max_iter) { st = ORC_NOT_CONVERGED; break; }
        }
    }
    if (iters) *iters = total;
    if (true_res) *true_res = res;
    free(w.r); free(w.z); free(w.p); free(w.q);
    return st;
}

int orc_pcg(int32_t n, int64_t nf, const int32_t *own, const int32_t *nb,
            const double *diag, const double *upper, const double *lower,
            const double *b, double *x, double tol, int max_iter, int precond,
            int transpose, int *iters, double *hist, double *true_res) {
    omat m = make_mat(n, nf, own, nb, diag, upper, lower, transpose);
    return cg_solve(&m, precond, NULL, NULL, b, x, tol, max_iter, iters, hist,
                    true_res);
}

/* ------------------------------------------------------------------------ */
/* PBiCG: preconditioned bi-conjugate gradients for non-symmetric A, the     */
/* paper's solver for the U, k and omega systems (Appendix A solver tables), */
/* which is why its profile lists Amul + Tmul together (Sec. 4.3).  Textbook */
/* form (Fletcher 1976; Saad, Alg. 7.3 with a preconditioner), shadow        */
/* residual taken equal to the initial residual:                              */
/*   r = b - A x; rt = r; z = M^-1 r; zt = M^-T rt; p = z; pt = zt;           */
/*   rho = z.rt                                                               */
/*   repeat: q = A p; qt = A^T pt; sigma = pt.q; alpha = rho/sigma;           */
/*           x += alpha p; r -= alpha q; rt -= alpha qt;                      */
/*           stop if ||r||/||b|| <= tol;                                      */
/*           z = M^-1 r; zt = M^-T rt; rho' = z.rt; beta = rho'/rho;          */
/*           p = z + beta p; pt = zt + beta pt                                */
/* M is the diagonal (M^-T = M^-1) or the identity.  Breakdown when |sigma|  */
/* or |rho'| <= 1e-300 or either is not finite.  On exit the true residual   */
/* is recomputed, and the iteration restarts from it (with a new shadow      */
/* residual) while it is above tol and iterations remain.                    */
/* Pins: dense non-symmetric solves; on symmetric A it reproduces PCG.       */
/* ------------------------------------------------------------------------ */

static void apply_diag(const omat *m, int precond, const double *r, double *z) {
    for (int32_t i = 0; i < m->n; ++i) z[i] = precond ? r[i] / m->diag[i] : r[i];
}

/* y = A^T x for the matrix view m */
static void mat_mul_t(const omat *m, const double *x, double *y) {
    orc_amul(m->n, m->nf, m->own, m->nb, m->diag, m->lo, m->up, x, y);
}

int orc_pbicg(int32_t n, int64_t nf, const int32_t *own, const int32_t *nb,
              const double *diag, const double *upper, const double *lower,
              const double *b, double *x, double tol, int max_iter, int precond,
              int transpose, int *iters, double *hist, double *true_res) {
    omat m = make_mat(n, nf, own, nb, diag, upper, lower, transpose);
    int total = 0;
    if (iters) *iters = 0;
    double bnorm = sqrt(dot(n, b, b));
    if (bnorm == 0.0) {
        for (int32_t i = 0; i < n; ++i) x[i] = 0.0;
        if (hist) hist[0] = 0.0;
        if (true_res) *true_res = 0.0;
        return ORC_OK;
    }
    double *r = xcalloc((size_t)n + 1, sizeof(double));
    double *rt = xcalloc((size_t)n + 1, sizeof(double));
    double *z = xcalloc((size_t)n + 1, sizeof(double));
    double *zt = xcalloc((size_t)n + 1, sizeof(double));
    double *p = xcalloc((size_t)n + 1, sizeof(double));
    double *pt = xcalloc((size_t)n + 1, sizeof(double));
    double *q = xcalloc((size_t)n + 1, sizeof(double));
    double *qt = xcalloc((size_t)n + 1, sizeof(double));
    residual(&m, b, x, r);
    double res = sqrt(dot(n, r, r)) / bnorm;
    if (hist) hist[0] = res;
    int st = ORC_OK;
    if (!isfinite(res)) st = ORC_ERR_NAN;
    while (st == ORC_OK && res > tol) {
        /* (re)start from the current residual with the shadow rt = r */
        int run = ORC_NOT_CONVERGED;
        memcpy(rt, r, (size_t)n * sizeof(double));
        apply_diag(&m, precond, r, z);
        apply_diag(&m, precond, rt, zt);
        memcpy(p, z, (size_t)n * sizeof(double));
        memcpy(pt, zt, (size_t)n * sizeof(double));
        double rho = dot(n, z, rt);
        while (total < max_iter) {
            mat_mul(&m, p, q);
            mat_mul_t(&m, pt, qt);
            double sigma = dot(n, pt, q);
            if (!isfinite(sigma) || fabs(sigma) <= 1e-300) { run = ORC_ERR_BREAKDOWN; break; }
            double alpha = rho / sigma;
            for (int32_t i = 0; i < n; ++i) x[i] = x[i] + alpha * p[i];
            for (int32_t i = 0; i < n; ++i) r[i] = r[i] - alpha * q[i];
            for (int32_t i = 0; i < n; ++i) rt[i] = rt[i] - alpha * qt[i];
            total += 1;
            double rr = sqrt(dot(n, r, r)) / bnorm;
            if (hist) hist[total] = rr;
            if (!isfinite(rr)) { run = ORC_ERR_NAN; break; }
            if (rr <= tol) { run = ORC_OK; break; }
            apply_diag(&m, precond, r, z);
            apply_diag(&m, precond, rt, zt);
            double rho_new = dot(n, z, rt);
            if (!isfinite(rho_new) || fabs(rho_new) <= 1e-300) { run = ORC_ERR_BREAKDOWN; break; }
            double beta = rho_new / rho;
            rho = rho_new;
            for (int32_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
            for (int32_t i = 0; i < n; ++i) pt[i] = zt[i] + beta * pt[i];
        }
        if (run < 0) { st = run; break; }
        residual(&m, b, x, r); /* true residual, restart point */
        res = sqrt(dot(n, r, r)) / bnorm;
        if (!isfinite(res)) { st = ORC_ERR_NAN; break; }
        if (res <= tol) break;
        if (total >= max_iter) { st = ORC_NOT_CONVERGED; break; }
    }
    if (iters) *iters = total;
    if (true_res) *true_res = res;
    free(r); free(rt); free(z); free(zt); free(p); free(pt); free(q); free(qt);
    return st;
}

/* ------------------------------------------------------------------------ */
/* Mixed precision: FP32 inner CG inside FP64 iterative refinement.          */
/* Not in the paper (a precision variant of its PCG).  Outer loop:           */
/*   r = b - A64 x (FP64); while ||r||/||b|| > tol:                           */
/*     s = max|r|; rhat = fp32(r/s); d = inner(rhat); x += s*fp64(d);        */
/*     r = b - A64 x                                                          */
/* Inner CG: FP32 values, vectors, products and axpys; the dot products are  */
/* accumulated in FP64 and alpha, beta are formed in FP64, then rounded to   */
/* FP32 for the updates.  Stops at ||r||/||rhat|| <= max(inner_tol,          */
/* 0.3 tol/res) (res: the outer relative residual) or after inner_max_iter   */
/* iterations.                                                                */
/* Pin: refinement converges to the FP64 solution (tests), FP32 Amul error   */
/* bound.                                                                     */
/* ------------------------------------------------------------------------ */

typedef struct {
    int32_t n;
    int64_t nf;
    const int32_t *own, *nb;
    float *diag, *up, *lo;
} fmat;

static fmat make_fmat(const omat *m) {
    fmat f;
    f.n = m->n;
    f.nf = m->nf;
    f.own = m->own;
    f.nb = m->nb;
    f.diag = xcalloc(m->n, sizeof(float));
    f.up = xcalloc(m->nf, sizeof(float));
    f.lo = xcalloc(m->nf, sizeof(float));
    for (int32_t i = 0; i < m->n; ++i) f.diag[i] = (float)m->diag[i];
    for (int64_t k = 0; k < m->nf; ++k) {
        f.up[k] = (float)m->up[k];
        f.lo[k] = (float)m->lo[k];
    }
    return f;
}

static void free_fmat(fmat *f) {
    free(f->diag); free(f->up); free(f->lo);
}

static void fmat_mul(const fmat *m, const float *x, float *y) {
    orc_amul_f32(m->n, m->nf, m->own, m->nb, m->diag, m->up, m->lo, x, y);
}

/* inner FP32 CG from d = 0 on A32 d = rhat to ||r|| <= inner_tol ||rhat||;
 * returns iterations done */
static int pcg32_inner(const fmat *m, const float *rhat, float *d,
                       double inner_tol, int inner_max) {
    const int32_t n = m->n;
    float *r = xcalloc(n, sizeof(float));
    float *z = xcalloc(n, sizeof(float));
    float *p = xcalloc(n, sizeof(float));
    float *q = xcalloc(n, sizeof(float));
    for (int32_t i = 0; i < n; ++i) { d[i] = 0.0f; r[i] = rhat[i]; }
    double r0 = sqrt(dot_f32(n, r, r));
    int it = 0;
    if (r0 > 0.0) {
        for (int32_t i = 0; i < n; ++i) z[i] = r[i] / m->diag[i];
        for (int32_t i = 0; i < n; ++i) p[i] = z[i];
        double rho = dot_f32(n, r, z);
        while (it < inner_max) {
            fmat_mul(m, p, q);
            double pq = dot_f32(n, p, q);
            if (!isfinite(pq) || fabs(pq) <= 1e-300) break;
            float af = (float)(rho / pq);
            for (int32_t i = 0; i < n; ++i) d[i] = d[i] + af * p[i];
            for (int32_t i = 0; i < n; ++i) r[i] = r[i] - af * q[i];
            ++it;
            if (sqrt(dot_f32(n, r, r)) <= inner_tol * r0) break;
            for (int32_t i = 0; i < n; ++i) z[i] = r[i] / m->diag[i];
            double rho_new = dot_f32(n, r, z);
            float bf = (float)(rho_new / rho);
            rho = rho_new;
            for (int32_t i = 0; i < n; ++i) p[i] = z[i] + bf * p[i];
        }
    }
    free(r); free(z); free(p); free(q);
    return it;
}

/* shared FP64 refinement driver; inner(ctx, rhat, d, tol_now) fills d.
 * tol_now = max(inner_tol, 0.3 tol / res): an inner solve stops once its
 * relative reduction would bring the outer residual below tol with a safety
 * factor of 0.3, or at the fixed inner tolerance, whichever is looser. */
typedef int (*inner_fn)(void *ctx, const float *rhat, float *d, double tol_now);

static double inner_target(double inner_tol, double tol, double res) {
    double t = 0.3 * tol / res;
    return t > inner_tol ? t : inner_tol;
}

static int refine(const omat *m, const double *b, double *x, double tol,
                  int max_refine, inner_fn inner, void *ctx, int *refinements,
                  int *inner_total, double *hist, double *true_res) {
    const int32_t n = m->n;
    double bnorm = sqrt(dot(n, b, b));
    if (refinements) *refinements = 0;
    if (inner_total) *inner_total = 0;
    if (bnorm == 0.0) {
        for (int32_t i = 0; i < n; ++i) x[i] = 0.0;
        if (hist) hist[0] = 0.0;
        if (true_res) *true_res = 0.0;
        return ORC_OK;
    }
    double *r = xcalloc(n, sizeof(double));
    float *rhat = xcalloc(n, sizeof(float));
    float *d = xcalloc(n, sizeof(float));
    residual(m, b, x, r);
    double res = sqrt(dot(n, r, r)) / bnorm;
    if (hist) hist[0] = res;
    int k = 0, st = ORC_OK;
    while (res > tol) {
        if (!isfinite(res)) { st = ORC_ERR_NAN; break; }
        if (k >= max_refine) { st = ORC_NOT_CONVERGED; break; }
        double s = 0.0;
        for (int32_t i = 0; i < n; ++i) s = fabs(r[i]) > s ? fabs(r[i]) : s;
        for (int32_t i = 0; i < n; ++i) rhat[i] = (float)(r[i] / s);
        int it = inner(ctx, rhat, d, res);
        if (inner_total) *inner_total += it;
        for (int32_t i = 0; i < n; ++i) x[i] = x[i] + s * (double)d[i];
        ++k;
        residual(m, b, x, r);
        res = sqrt(dot(n, r, r)) / bnorm;
        if (hist) hist[k] = res;
    }
    if (refinements) *refinements = k;
    if (true_res) *true_res = res;
    free(r); free(rhat); free(d);
    return st;
}

typedef struct {
    const fmat *m;
    double tol, outer_tol;
    int max_iter;
} pcg32_ctx;

static int pcg32_inner_cb(void *ctx, const float *rhat, float *d, double res) {
    pcg32_ctx *c = (pcg32_ctx *)ctx;
    return pcg32_inner(c->m, rhat, d, inner_target(c->tol, c->outer_tol, res),
                       c->max_iter);
}

int orc_pcg_mixed(int32_t n, int64_t nf, const int32_t *own, const int32_t *nb,
                  const double *diag, const double *upper, const double *lower,
                  const double *b, double *x, double tol, int max_refine,
                  double inner_tol, int inner_max_iter, int transpose,
                  int *refinements, int *inner_iters, double *hist,
                  double *true_res) {
    omat m = make_mat(n, nf, own, nb, diag, upper, lower, transpose);
    fmat fm = make_fmat(&m);
    pcg32_ctx c = {&fm, inner_tol, tol, inner_max_iter};
    int st = refine(&m, b, x, tol, max_refine, pcg32_inner_cb, &c, refinements,
                    inner_iters, hist, true_res);
    free_fmat(&fm);
    return st;
}

/* ------------------------------------------------------------------------ */
/* GAMG (Appendix A: "GAMG / Richardson" for p; Sec. 4.3: Richardson i.e.    */
/* damped Jacobi on every level, diagonal-PCG at the coarsest level; the     */
/* profiled steps agglomerateMatrix, restrictField, prolongField, scale,     */
/* Vcycle).  The paper keeps OpenFOAM's serial coarsening and does not state */
/* it; this oracle uses a parallel-friendly pairwise matching, defined as:   */
/*                                                                            */
/*  weight of face f between i and j: the squared diagonally scaled strength  */
/*  w_f = (0.5*(|upper_f| + |lower_f|))^2 / |diag_i diag_j|                    */
/*  order of candidate neighbours j of cell i: larger w first, then larger    */
/*  tie key h(min(i,j), max(i,j)) (SplitMix64 output function of the packed   */
/*  pair, Steele, Lea & Flood 2014), then smaller j.                          */
/*  round: every unmatched cell picks its best unmatched neighbour; cells     */
/*  that pick each other become a pair.  Rounds repeat until one adds no pair */
/*  or match_rounds rounds have run.                                          */
/*  leftovers: an unmatched cell with a matched neighbour joins the aggregate */
/*  of its best matched neighbour (decided from the matched state only);      */
/*  otherwise it stays a singleton.                                           */
/*  numbering: each aggregate has a seed (the smaller cell of the pair, or    */
/*  the singleton); coarse index = rank of the seed among all seeds.          */
/*  stop: n <= n_coarsest, or n_coarse > 0.95 n, or max_levels levels.        */
/* Galerkin coarse operator (agglomerateMatrix) with piecewise-constant      */
/* prolongation P: A_c = P^T A P in LDU form, coarse faces = distinct         */
/* aggregate pairs sorted by (a, b); each coarse value is summed over fine    */
/* faces in ascending face order, the coarse diagonal over member cells in    */
/* ascending order and then over internal faces in ascending order.          */
/* Pins: brute-force matching definition, dense P^T A P, symmetry and zero   */
/* row sums preserved, dense two-level V-cycle formula, convergence to the   */
/* dense solution.                                                            */
/* ------------------------------------------------------------------------ */

typedef struct {
    int32_t n;
    int64_t nf;
    int32_t *own, *nb;
    double *diag, *up, *lo;
    float *diag32, *up32, *lo32;
    int32_t *agg;     /* to the next level; NULL on the coarsest */
    int32_t *partner; /* matching state, NULL on the coarsest */
    int32_t *join;
    int singular;     /* coarsest only: A 1 = 0 to rounding */
} olevel;

#define ORC_MAX_LEVELS 64

struct orc_gamg {
    int nlev;
    olevel lev[ORC_MAX_LEVELS];
    int smoother;    /* ORC_SMOOTH_JACOBI or ORC_SMOOTH_GS2 */
    int gs_inner;    /* two-stage Gauss-Seidel: inner Jacobi-Richardson steps */
    int coarsest_pc; /* ORC_COARSE_DIAG or ORC_COARSE_DIC */
};

static uint64_t splitmix64_out(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static uint64_t tie_key(int32_t i, int32_t j) {
    uint64_t lo = (uint64_t)(uint32_t)(i < j ? i : j);
    uint64_t hi = (uint64_t)(uint32_t)(i < j ? j : i);
    return splitmix64_out((lo << 32) | hi);
}

/* squared strength of the coupling between cells i and j through face f:
 * (|upper_f| + |lower_f|)^2 / 4 divided by |diag_i diag_j| (the coupling
 * relative to the diagonals; no square root, so it rounds identically
 * everywhere).  A zero diagonal product falls back to the unscaled value. */
static double strength2(double up, double lo, double di, double dj) {
    double s = 0.5 * (fabs(up) + fabs(lo));
    double den = fabs(di) * fabs(dj);
    return den > 0.0 ? (s * s) / den : s * s;
}

/* is candidate (w1,h1,j1) better than (w2,h2,j2)? */
static int better(double w1, uint64_t h1, int32_t j1, double w2, uint64_t h2,
                  int32_t j2) {
    if (w1 != w2) return w1 > w2;
    if (h1 != h2) return h1 > h2;
    return j1 < j2;
}

/* cell adjacency: for cell i, entries start[i]..start[i+1] of (cell, face) */
typedef struct {
    int64_t *start;
    int32_t *cell;
    int64_t *face;
} adjacency;

static adjacency build_adjacency(const olevel *L) {
    adjacency a;
    a.start = xcalloc((size_t)L->n + 1, sizeof(int64_t));
    a.cell = xcalloc((size_t)(2 * L->nf), sizeof(int32_t));
    a.face = xcalloc((size_t)(2 * L->nf), sizeof(int64_t));
    for (int64_t f = 0; f < L->nf; ++f) {
        a.start[L->own[f] + 1]++;
        a.start[L->nb[f] + 1]++;
    }
    for (int32_t i = 0; i < L->n; ++i) a.start[i + 1] += a.start[i];
    int64_t *fill = xcalloc((size_t)L->n, sizeof(int64_t));
    for (int64_t f = 0; f < L->nf; ++f) {
        int32_t o = L->own[f], b = L->nb[f];
        a.cell[a.start[o] + fill[o]] = b;
        a.face[a.start[o] + fill[o]++] = f;
        a.cell[a.start[b] + fill[b]] = o;
        a.face[a.start[b] + fill[b]++] = f;
    }
    free(fill);
    return a;
}

static void free_adjacency(adjacency *a) {
    free(a->start); free(a->cell); free(a->face);
}

/* best neighbour j of i with (partner[j] < 0) == want_unmatched; -1 if none */
static int32_t best_neighbour(const olevel *L, const adjacency *a, int32_t i,
                              const int32_t *partner, int want_unmatched) {
    int32_t best = -1;
    double bw = 0.0;
    uint64_t bh = 0;
    for (int64_t k = a->start[i]; k < a->start[i + 1]; ++k) {
        int32_t j = a->cell[k];
        int unmatched = partner[j] < 0;
        if (unmatched != want_unmatched) continue;
        int64_t f = a->face[k];
        double w = strength2(L->up[f], L->lo[f], L->diag[i], L->diag[j]);
        uint64_t h = tie_key(i, j);
        if (best < 0 || better(w, h, j, bw, bh, best)) {
            best = j;
            bw = w;
            bh = h;
        }
    }
    return best;
}

/* pairwise agglomeration of level L; fills L->agg/partner/join, returns n_c */
static int32_t agglomerate(olevel *L, int match_rounds) {
    const int32_t n = L->n;
    adjacency a = build_adjacency(L);
    int32_t *partner = xcalloc(n, sizeof(int32_t));
    int32_t *pick = xcalloc(n, sizeof(int32_t));
    int32_t *join = xcalloc(n, sizeof(int32_t));
    for (int32_t i = 0; i < n; ++i) partner[i] = -1;
    for (int round = 0; round < match_rounds; ++round) {
        for (int32_t i = 0; i < n; ++i)
            pick[i] = partner[i] < 0 ? best_neighbour(L, &a, i, partner, 1) : -1;
        int added = 0;
        for (int32_t i = 0; i < n; ++i) {
            int32_t j = pick[i];
            if (j >= 0 && pick[j] == i) {
                partner[i] = j;
                added = 1;
            }
        }
        if (!added) break;
    }
    for (int32_t i = 0; i < n; ++i)
        join[i] = partner[i] < 0 ? best_neighbour(L, &a, i, partner, 0) : -1;
    /* seeds and their ranks */
    int32_t *rank = pick; /* reuse */
    int32_t nc = 0;
    for (int32_t i = 0; i < n; ++i) {
        int seed = (partner[i] >= 0 && i < partner[i]) ||
                   (partner[i] < 0 && join[i] < 0);
        rank[i] = seed ? nc++ : -1;
    }
    int32_t *agg = xcalloc(n, sizeof(int32_t));
    for (int32_t i = 0; i < n; ++i) {
        if (partner[i] >= 0) {
            agg[i] = rank[i < partner[i] ? i : partner[i]];
        } else if (join[i] < 0) {
            agg[i] = rank[i];
        } else {
            int32_t j = join[i], pj = partner[j];
            agg[i] = rank[j < pj ? j : pj];
        }
    }
    free(pick);
    free_adjacency(&a);
    L->agg = agg;
    L->partner = partner;
    L->join = join;
    return nc;
}

static int cmp_i64(const void *a, const void *b) {
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return (x > y) - (x < y);
}

/* C = P^T A P for the aggregation agg (agglomerateMatrix) */
static void galerkin(const olevel *F, int32_t nc, olevel *C) {
    int64_t nkeys = 0;
    int64_t *keys = xcalloc((size_t)F->nf, sizeof(int64_t));
    for (int64_t f = 0; f < F->nf; ++f) {
        int32_t a = F->agg[F->own[f]], b = F->agg[F->nb[f]];
        if (a == b) continue;
        int64_t lo = a < b ? a : b, hi = a < b ? b : a;
        keys[nkeys++] = lo * (int64_t)nc + hi;
    }
    qsort(keys, (size_t)nkeys, sizeof(int64_t), cmp_i64);
    int64_t ncf = 0;
    for (int64_t k = 0; k < nkeys; ++k)
        if (k == 0 || keys[k] != keys[k - 1]) keys[ncf++] = keys[k];
    C->n = nc;
    C->nf = ncf;
    C->own = xcalloc((size_t)ncf, sizeof(int32_t));
    C->nb = xcalloc((size_t)ncf, sizeof(int32_t));
    C->up = xcalloc((size_t)ncf, sizeof(double));
    C->lo = xcalloc((size_t)ncf, sizeof(double));
    C->diag = xcalloc((size_t)nc, sizeof(double));
    for (int64_t c = 0; c < ncf; ++c) {
        C->own[c] = (int32_t)(keys[c] / nc);
        C->nb[c] = (int32_t)(keys[c] % nc);
    }
    for (int64_t f = 0; f < F->nf; ++f) {
        int32_t a = F->agg[F->own[f]], b = F->agg[F->nb[f]];
        if (a == b) continue;
        int64_t key = (a < b ? (int64_t)a * nc + b : (int64_t)b * nc + a);
        int64_t *hit = bsearch(&key, keys, (size_t)ncf, sizeof(int64_t), cmp_i64);
        int64_t c = hit - keys;
        if (a < b) {
            C->up[c] += F->up[f];
            C->lo[c] += F->lo[f];
        } else {
            C->up[c] += F->lo[f];
            C->lo[c] += F->up[f];
        }
    }
    for (int32_t i = 0; i < F->n; ++i) C->diag[F->agg[i]] += F->diag[i];
    for (int64_t f = 0; f < F->nf; ++f) {
        int32_t a = F->agg[F->own[f]], b = F->agg[F->nb[f]];
        if (a == b) C->diag[a] += (F->up[f] + F->lo[f]);
    }
    free(keys);
}

static void level_f32(olevel *L) {
    L->diag32 = xcalloc((size_t)L->n, sizeof(float));
    L->up32 = xcalloc((size_t)L->nf, sizeof(float));
    L->lo32 = xcalloc((size_t)L->nf, sizeof(float));
    for (int32_t i = 0; i < L->n; ++i) L->diag32[i] = (float)L->diag[i];
    for (int64_t f = 0; f < L->nf; ++f) {
        L->up32[f] = (float)L->up[f];
        L->lo32[f] = (float)L->lo[f];
    }
}

/* singular coarsest level: every row sum of A is zero to rounding */
static void set_singular(olevel *C) {
    double *one = xcalloc((size_t)C->n, sizeof(double));
    double *y = xcalloc((size_t)C->n, sizeof(double));
    for (int32_t i = 0; i < C->n; ++i) one[i] = 1.0;
    orc_amul(C->n, C->nf, C->own, C->nb, C->diag, C->up, C->lo, one, y);
    C->singular = C->n > 0;
    for (int32_t i = 0; i < C->n; ++i)
        if (!(fabs(y[i]) <= 1e-12 * fabs(C->diag[i]))) C->singular = 0;
    free(one); free(y);
}

/* free the arrays of a level */
static void free_level(olevel *L) {
    free(L->own); free(L->nb); free(L->diag); free(L->up); free(L->lo);
    free(L->diag32); free(L->up32); free(L->lo32);
    free(L->agg); free(L->partner); free(L->join);
    memset(L, 0, sizeof(*L));
}

/* aggregation of level L by `passes` rounds of pairwise agglomeration: pass
 * k matches the cells of the Galerkin matrix of pass k-1 (a temporary used
 * only for its coupling strengths), and the aggregates compose.  One pass is
 * plain pairwise agglomeration.  Returns the number of aggregates and leaves
 * the composed map in L->agg (partner/join describe the first pass). */
static int32_t agglomerate_passes(olevel *L, int match_rounds, int passes) {
    int32_t nc = agglomerate(L, match_rounds);
    if (passes <= 1 || nc <= 1) return nc;
    olevel T;
    memset(&T, 0, sizeof T);
    galerkin(L, nc, &T);
    int32_t nc2 = agglomerate_passes(&T, match_rounds, passes - 1);
    for (int32_t i = 0; i < L->n; ++i) L->agg[i] = T.agg[L->agg[i]];
    free_level(&T);
    return nc2;
}

orc_gamg *orc_gamg_build(int32_t n, int64_t nf, const int32_t *own,
                         const int32_t *nb, const double *diag,
                         const double *upper, const double *lower,
                         int n_coarsest, int max_levels, int match_rounds) {
    return orc_gamg_build2(n, nf, own, nb, diag, upper, lower, n_coarsest,
                           max_levels, match_rounds, 1);
}

orc_gamg *orc_gamg_build2(int32_t n, int64_t nf, const int32_t *own,
                          const int32_t *nb, const double *diag,
                          const double *upper, const double *lower,
                          int n_coarsest, int max_levels, int match_rounds,
                          int passes) {
    return orc_gamg_build3(n, nf, own, nb, diag, upper, lower, n_coarsest,
                           max_levels, match_rounds, passes, 0);
}

orc_gamg *orc_gamg_build3(int32_t n, int64_t nf, const int32_t *own,
                          const int32_t *nb, const double *diag,
                          const double *upper, const double *lower,
                          int n_coarsest, int max_levels, int match_rounds,
                          int passes, int aggressive_from) {
    orc_gamg *h = xcalloc(1, sizeof(orc_gamg));
    h->smoother = ORC_SMOOTH_JACOBI;
    h->gs_inner = 1;
    h->coarsest_pc = ORC_COARSE_DIAG;
    if (max_levels > ORC_MAX_LEVELS) max_levels = ORC_MAX_LEVELS;
    if (max_levels < 1) max_levels = 1;
    olevel *L0 = &h->lev[0];
    L0->n = n;
    L0->nf = nf;
    L0->own = xcalloc((size_t)nf, sizeof(int32_t));
    L0->nb = xcalloc((size_t)nf, sizeof(int32_t));
    L0->diag = xcalloc((size_t)n, sizeof(double));
    L0->up = xcalloc((size_t)nf, sizeof(double));
    L0->lo = xcalloc((size_t)nf, sizeof(double));
    memcpy(L0->own, own, (size_t)nf * sizeof(int32_t));
    memcpy(L0->nb, nb, (size_t)nf * sizeof(int32_t));
    memcpy(L0->diag, diag, (size_t)n * sizeof(double));
    memcpy(L0->up, upper, (size_t)nf * sizeof(double));
    memcpy(L0->lo, lower, (size_t)nf * sizeof(double));
    h->nlev = 1;
    while (h->nlev < max_levels) {
        olevel *L = &h->lev[h->nlev - 1];
        if (L->n <= n_coarsest) break;
        int32_t nc = agglomerate_passes(L, match_rounds,
                                        h->nlev - 1 >= aggressive_from ? passes : 1);
        if (100 * (int64_t)nc > 95 * (int64_t)L->n) {
            free(L->agg); free(L->partner); free(L->join);
            L->agg = L->partner = L->join = NULL;
            break;
        }
        galerkin(L, nc, &h->lev[h->nlev]);
        h->nlev++;
    }
    for (int l = 0; l < h->nlev; ++l) level_f32(&h->lev[l]);
    set_singular(&h->lev[h->nlev - 1]);
    return h;
}

/* new fine-level coefficients on a cached hierarchy: the aggregation of
 * every level is kept and each coarse matrix is recomputed by the Galerkin
 * product (OpenFOAM's cached GAMG agglomeration) */
void orc_gamg_set_values(orc_gamg *h, const double *diag, const double *upper,
                         const double *lower) {
    olevel *L0 = &h->lev[0];
    memcpy(L0->diag, diag, (size_t)L0->n * sizeof(double));
    memcpy(L0->up, upper, (size_t)L0->nf * sizeof(double));
    memcpy(L0->lo, lower, (size_t)L0->nf * sizeof(double));
    for (int l = 0; l + 1 < h->nlev; ++l) {
        olevel *F = &h->lev[l], *C = &h->lev[l + 1];
        free(C->own); free(C->nb); free(C->diag); free(C->up); free(C->lo);
        galerkin(F, C->n, C);
    }
    for (int l = 0; l < h->nlev; ++l) {
        olevel *L = &h->lev[l];
        free(L->diag32); free(L->up32); free(L->lo32);
        level_f32(L);
    }
    set_singular(&h->lev[h->nlev - 1]);
}

int orc_gamg_set_cycle(orc_gamg *h, int smoother, int gs_inner, int coarsest_pc) {
    if ((smoother != ORC_SMOOTH_JACOBI && smoother != ORC_SMOOTH_GS2) || gs_inner < 1 ||
        (coarsest_pc != ORC_COARSE_DIAG && coarsest_pc != ORC_COARSE_DIC))
        return ORC_ERR_ARG;
    h->smoother = smoother;
    h->gs_inner = gs_inner;
    h->coarsest_pc = coarsest_pc;
    return ORC_OK;
}

void orc_gamg_free(orc_gamg *h) {
    if (!h) return;
    for (int l = 0; l < h->nlev; ++l) free_level(&h->lev[l]);
    free(h);
}

int orc_gamg_nlevels(const orc_gamg *h) { return h->nlev; }

void orc_gamg_level_size(const orc_gamg *h, int level, int64_t *n,
                         int64_t *nf) {
    *n = h->lev[level].n;
    *nf = h->lev[level].nf;
}

void orc_gamg_level_export(const orc_gamg *h, int level, int32_t *agg,
                           int32_t *own, int32_t *nb, double *diag,
                           double *upper, double *lower) {
    const olevel *L = &h->lev[level];
    if (agg && L->agg) memcpy(agg, L->agg, (size_t)L->n * sizeof(int32_t));
    if (own) memcpy(own, L->own, (size_t)L->nf * sizeof(int32_t));
    if (nb) memcpy(nb, L->nb, (size_t)L->nf * sizeof(int32_t));
    if (diag) memcpy(diag, L->diag, (size_t)L->n * sizeof(double));
    if (upper) memcpy(upper, L->up, (size_t)L->nf * sizeof(double));
    if (lower) memcpy(lower, L->lo, (size_t)L->nf * sizeof(double));
}

void orc_gamg_level_match(const orc_gamg *h, int level, int32_t *partner,
                          int32_t *join) {
    const olevel *L = &h->lev[level];
    if (partner && L->partner)
        memcpy(partner, L->partner, (size_t)L->n * sizeof(int32_t));
    if (join && L->join) memcpy(join, L->join, (size_t)L->n * sizeof(int32_t));
}

/* ---- V-cycle ----------------------------------------------------------- */

#define COARSEST_TOL 1e-10

static omat level_mat(const olevel *L, int transpose) {
    return make_mat(L->n, L->nf, L->own, L->nb, L->diag, L->up, L->lo,
                    transpose);
}

/* ---- DIC (diagonal incomplete Cholesky) for the coarsest CG ------------ */
/* The paper's alternative coarsest-level preconditioner (Sec. 4.3, smoother */
/* and coarse-preconditioner table).  Textbook diagonal-modified ILU(0):      */
/*   M = (Dt + L) Dt^-1 (Dt + U), with L, U the strictly lower / upper parts  */
/*   of A and Dt chosen so that diag(M) = diag(A):                            */
/*   Dt_i = A_ii - sum_{j<i} A_ij A_ji / Dt_j   (ascending j);                */
/* for symmetric A this is the incomplete Cholesky of OpenFOAM's DIC.  A      */
/* pivot that is not finite, or not of the sign of A_ii with magnitude above  */
/* 1e-12 |A_ii|, marks the factorization unusable and the level falls back to */
/* the diagonal preconditioner.                                               */
/* Apply z = M^-1 r:                                                          */
/*   forward  y_i = (r_i - sum_{j<i} A_ij y_j) / Dt_i,       i ascending      */
/*   backward z_i = y_i - (sum_{j>i} A_ij z_j) / Dt_i,        i descending    */
/* each row sum taken in ascending column order.                              */
/* ------------------------------------------------------------------------ */

typedef struct {
    int32_t n;
    int64_t *lstart, *ustart; /* row i: lower entries [lstart[i], lstart[i+1]) */
    int32_t *lcol, *ucol;
    double *lval, *uval;
    const double *diag;
    double *dt;               /* Dt, the modified pivots */
    int ok;
} dic_fact;

static void dic_build(const omat *m, dic_fact *F) {
    const int32_t n = m->n;
    const int64_t nf = m->nf;
    F->n = n;
    F->diag = m->diag;
    F->lstart = xcalloc((size_t)n + 1, sizeof(int64_t));
    F->ustart = xcalloc((size_t)n + 1, sizeof(int64_t));
    F->lcol = xcalloc((size_t)nf + 1, sizeof(int32_t));
    F->ucol = xcalloc((size_t)nf + 1, sizeof(int32_t));
    F->lval = xcalloc((size_t)nf + 1, sizeof(double));
    F->uval = xcalloc((size_t)nf + 1, sizeof(double));
    F->dt = xcalloc((size_t)n + 1, sizeof(double));
    /* row-wise lists: row nb[f] holds (own[f], lo[f]) in L; row own[f] holds
     * (nb[f], up[f]) in U.  Faces are sorted by (owner, neighbour), so filling
     * in face order leaves every row in ascending column order. */
    for (int64_t f = 0; f < nf; ++f) {
        F->lstart[m->nb[f] + 1]++;
        F->ustart[m->own[f] + 1]++;
    }
    for (int32_t i = 0; i < n; ++i) {
        F->lstart[i + 1] += F->lstart[i];
        F->ustart[i + 1] += F->ustart[i];
    }
    int64_t *lc = xcalloc((size_t)n + 1, sizeof(int64_t));
    int64_t *uc = xcalloc((size_t)n + 1, sizeof(int64_t));
    for (int64_t f = 0; f < nf; ++f) {
        const int32_t o = m->own[f], b = m->nb[f];
        const int64_t pl = F->lstart[b] + lc[b]++;
        F->lcol[pl] = o;
        F->lval[pl] = m->lo[f];
        const int64_t pu = F->ustart[o] + uc[o]++;
        F->ucol[pu] = b;
        F->uval[pu] = m->up[f];
    }
    free(lc); free(uc);
    /* pivots: A_ji for a lower entry (i, j) is the upper entry of row j at
     * column i, i.e. the same face */
    F->ok = 1;
    for (int32_t i = 0; i < n; ++i) {
        double d = m->diag[i];
        for (int64_t k = F->lstart[i]; k < F->lstart[i + 1]; ++k) {
            const int32_t j = F->lcol[k];
            double aji = 0.0;
            for (int64_t q = F->ustart[j]; q < F->ustart[j + 1]; ++q)
                if (F->ucol[q] == i) aji = F->uval[q];
            d = d - (F->lval[k] * aji) / F->dt[j];
        }
        F->dt[i] = d;
        if (!isfinite(d) || !(fabs(d) > 1e-12 * fabs(m->diag[i])) ||
            (d > 0.0) != (m->diag[i] > 0.0))
            F->ok = 0;
    }
}

static void dic_free(dic_fact *F) {
    free(F->lstart); free(F->ustart); free(F->lcol); free(F->ucol);
    free(F->lval); free(F->uval); free(F->dt);
}

static void dic_apply(void *ctx, const double *r, double *z) {
    const dic_fact *F = (const dic_fact *)ctx;
    const int32_t n = F->n;
    if (!F->ok) {
        for (int32_t i = 0; i < n; ++i) z[i] = r[i] / F->diag[i];
        return;
    }
    for (int32_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int64_t k = F->lstart[i]; k < F->lstart[i + 1]; ++k)
            s += F->lval[k] * z[F->lcol[k]];
        z[i] = (r[i] - s) / F->dt[i];
    }
    for (int32_t i = n - 1; i >= 0; --i) {
        double s = 0.0;
        for (int64_t k = F->ustart[i]; k < F->ustart[i + 1]; ++k)
            s += F->uval[k] * z[F->ucol[k]];
        z[i] = z[i] - s / F->dt[i];
    }
}

/* coarsest level: PCG (diagonal, or DIC when asked) from 0 to
 * ||r|| <= 1e-10 ||rhs|| or max(2n, 100) iterations; a singular level first
 * projects its rhs to zero mean (the constant null space of a pure
 * zero-gradient operator) */
static void coarsest_solve(const orc_gamg *h, const olevel *L, const double *r,
                           double *e, int transpose) {
    const int32_t n = L->n;
    omat m = level_mat(L, transpose);
    double *rhs = xcalloc(n, sizeof(double));
    for (int32_t i = 0; i < n; ++i) rhs[i] = r[i];
    if (L->singular) {
        double s = 0.0;
        for (int32_t i = 0; i < n; ++i) s += rhs[i];
        double mean = s / (double)n;
        for (int32_t i = 0; i < n; ++i) rhs[i] = rhs[i] - mean;
    }
    for (int32_t i = 0; i < n; ++i) e[i] = 0.0;
    double bn = sqrt(dot(n, rhs, rhs));
    if (bn > 0.0) {
        cg_work w;
        w.r = rhs;
        w.z = xcalloc(n, sizeof(double));
        w.p = xcalloc(n, sizeof(double));
        w.q = xcalloc(n, sizeof(double));
        int total = 0;
        int max_it = 2 * n > 100 ? 2 * n : 100;
        if (h->coarsest_pc == ORC_COARSE_DIC) {
            dic_fact F;
            dic_build(&m, &F);
            cg_run_pc(&m, 1, dic_apply, &F, e, &w, bn, COARSEST_TOL, max_it, &total,
                      NULL);
            dic_free(&F);
        } else {
            cg_run(&m, 1, e, &w, bn, COARSEST_TOL, max_it, &total, NULL);
        }
        free(w.z); free(w.p); free(w.q);
    }
    free(rhs);
}

typedef struct {
    int n_pre, n_post, scale, transpose;
    double omega;
} vparams;

/* e_new = e + omega*(r - A e)/diag, simultaneous over all cells */
static void jacobi_sweep(const omat *m, const double *r, double *e,
                         double *y, double omega) {
    mat_mul(m, e, y);
    for (int32_t i = 0; i < m->n; ++i)
        y[i] = e[i] + omega * (r[i] - y[i]) / m->diag[i];
    memcpy(e, y, (size_t)m->n * sizeof(double));
}

/* y = L x (strictly lower part: row nb[f], column own[f]) or y = U x
 * (strictly upper: row own[f], column nb[f]); each row sums its terms in
 * ascending column order, which is face order for a face list sorted by
 * (owner, neighbour) */
static void tri_mul(const omat *m, int upper, const double *x, double *y) {
    for (int32_t i = 0; i < m->n; ++i) y[i] = 0.0;
    for (int64_t f = 0; f < m->nf; ++f) {
        if (upper) y[m->own[f]] += m->up[f] * x[m->nb[f]];
        else y[m->nb[f]] += m->lo[f] * x[m->own[f]];
    }
}

/* ---- two-stage Gauss-Seidel smoother ------------------------------------ */
/* The paper's second GPU smoother (Sec. 4.3), after Berger-Vergiat et al.    */
/* (2021): a Gauss-Seidel sweep e += (D + L)^-1 (r - A e) whose triangular    */
/* solve is replaced by `inner` Jacobi-Richardson steps                       */
/*   t = r - A e;  g = D^-1 t;  repeat inner times: g = D^-1 (t - L g);       */
/*   e = e + g.                                                               */
/* Forward sweeps (L) pre-smooth, backward sweeps (U, i.e. (D + U)^-1) post-  */
/* smooth, so a V-cycle with n_pre = n_post is symmetric for symmetric A.     */
/* A sweep from e = 0 takes t = r and sets e = g.  No damping.                */
/* ------------------------------------------------------------------------ */
static void gs2_sweep(const omat *m, const double *r, double *e, int from_zero,
                      int backward, int inner, double *t, double *g,
                      double *y) {
    const int32_t n = m->n;
    if (from_zero) memcpy(t, r, (size_t)n * sizeof(double));
    else residual(m, r, e, t);
    for (int32_t i = 0; i < n; ++i) g[i] = t[i] / m->diag[i];
    for (int k = 0; k < inner; ++k) {
        tri_mul(m, backward, g, y);
        for (int32_t i = 0; i < n; ++i) g[i] = (t[i] - y[i]) / m->diag[i];
    }
    for (int32_t i = 0; i < n; ++i) e[i] = from_zero ? g[i] : e[i] + g[i];
}

static void vcycle(const orc_gamg *h, int l, const double *r, double *e,
                   const vparams *vp) {
    const olevel *L = &h->lev[l];
    if (l == h->nlev - 1) {
        coarsest_solve(h, L, r, e, vp->transpose);
        return;
    }
    const int32_t n = L->n;
    const olevel *C = &h->lev[l + 1];
    omat m = level_mat(L, vp->transpose);
    const int gs = h->smoother == ORC_SMOOTH_GS2;
    double *y = xcalloc(n, sizeof(double));
    double *t = xcalloc(n, sizeof(double));
    double *c = xcalloc(n, sizeof(double));
    double *g = xcalloc(n, sizeof(double));
    double *rc = xcalloc(C->n, sizeof(double));
    double *ec = xcalloc(C->n, sizeof(double));
    /* pre-smoothing from e = 0 (Jacobi: the first sweep is omega*r/diag) */
    if (gs) {
        for (int32_t i = 0; i < n; ++i) e[i] = 0.0;
        for (int s = 0; s < vp->n_pre; ++s)
            gs2_sweep(&m, r, e, s == 0, 0, h->gs_inner, t, g, y);
    } else {
        for (int32_t i = 0; i < n; ++i)
            e[i] = vp->n_pre > 0 ? vp->omega * r[i] / m.diag[i] : 0.0;
        for (int s = 1; s < vp->n_pre; ++s) jacobi_sweep(&m, r, e, y, vp->omega);
    }
    /* residual after smoothing, restricted by summation (restrictField) */
    residual(&m, r, e, t);
    for (int32_t i = 0; i < n; ++i) rc[L->agg[i]] += t[i];
    vcycle(h, l + 1, rc, ec, vp);
    /* prolongation by injection (prolongField) and correction scaling */
    for (int32_t i = 0; i < n; ++i) c[i] = ec[L->agg[i]];
    double s = 1.0;
    if (vp->scale) {
        mat_mul(&m, c, y);
        double ct = dot(n, c, t);
        double cac = dot(n, c, y);
        if (isfinite(cac) && fabs(cac) > 1e-300) s = ct / cac;
    }
    for (int32_t i = 0; i < n; ++i) e[i] = e[i] + s * c[i];
    for (int k = 0; k < vp->n_post; ++k) {
        if (gs) gs2_sweep(&m, r, e, 0, 1, h->gs_inner, t, g, y);
        else jacobi_sweep(&m, r, e, y, vp->omega);
    }
    free(y); free(t); free(c); free(g); free(rc); free(ec);
}

/* single steps exposed for the pins: one two-stage Gauss-Seidel sweep, and
 * the DIC pivots / preconditioner application on one matrix */
void orc_gs2_sweep(int32_t n, int64_t nf, const int32_t *own, const int32_t *nb,
                   const double *diag, const double *upper, const double *lower,
                   const double *r, double *e, int from_zero, int backward,
                   int inner) {
    omat m = make_mat(n, nf, own, nb, diag, upper, lower, 0);
    double *t = xcalloc((size_t)n + 1, sizeof(double));
    double *g = xcalloc((size_t)n + 1, sizeof(double));
    double *y = xcalloc((size_t)n + 1, sizeof(double));
    gs2_sweep(&m, r, e, from_zero, backward, inner, t, g, y);
    free(t); free(g); free(y);
}

int orc_dic(int32_t n, int64_t nf, const int32_t *own, const int32_t *nb,
            const double *diag, const double *upper, const double *lower,
            double *dt, const double *r, double *z) {
    omat m = make_mat(n, nf, own, nb, diag, upper, lower, 0);
    dic_fact F;
    dic_build(&m, &F);
    if (dt) memcpy(dt, F.dt, (size_t)n * sizeof(double));
    if (r && z) dic_apply(&F, r, z);
    const int ok = F.ok;
    dic_free(&F);
    return ok;
}

int orc_gamg_vcycle(const orc_gamg *h, const double *r, double *e, int n_pre,
                    int n_post, double omega, int scale, int transpose) {
    vparams vp = {n_pre, n_post, scale, transpose, omega};
    vcycle(h, 0, r, e, &vp);
    return ORC_OK;
}

/* GAMG as a standalone solver: per cycle r = b - A x (FP64); stop when
 * ||r||/||b|| <= tol; otherwise x += V(0, r). */
int orc_gamg_solve(const orc_gamg *h, const double *b, double *x, double tol,
                   int max_cycles, int n_pre, int n_post, double omega,
                   int scale, int transpose, int *cycles, double *hist,
                   double *true_res) {
    const olevel *L = &h->lev[0];
    const int32_t n = L->n;
    omat m = level_mat(L, transpose);
    vparams vp = {n_pre, n_post, scale, transpose, omega};
    if (cycles) *cycles = 0;
    double bnorm = sqrt(dot(n, b, b));
    if (bnorm == 0.0) {
        for (int32_t i = 0; i < n; ++i) x[i] = 0.0;
        if (hist) hist[0] = 0.0;
        if (true_res) *true_res = 0.0;
        return ORC_OK;
    }
    double *r = xcalloc(n, sizeof(double));
    double *e = xcalloc(n, sizeof(double));
    int st = ORC_NOT_CONVERGED;
    double res = 0.0;
    for (int k = 0;; ++k) {
        residual(&m, b, x, r);
        res = sqrt(dot(n, r, r)) / bnorm;
        if (hist) hist[k] = res;
        if (!isfinite(res)) { st = ORC_ERR_NAN; break; }
        if (cycles) *cycles = k;
        if (res <= tol) { st = ORC_OK; break; }
        if (k >= max_cycles) { st = ORC_NOT_CONVERGED; break; }
        vcycle(h, 0, r, e, &vp);
        for (int32_t i = 0; i < n; ++i) x[i] = x[i] + e[i];
    }
    if (true_res) *true_res = res;
    free(r); free(e);
    return st;
}

/* CG preconditioned by one V-cycle per iteration (correction scaling off, so
 * that the preconditioner is a fixed symmetric operator for symmetric A and
 * n_pre = n_post): the solver / preconditioner pairing of the paper's AmgX
 * configuration (Appendix A listing: PCG with an AMG V-cycle preconditioner)
 * applied to this GAMG hierarchy. */
typedef struct {
    const orc_gamg *h;
    vparams vp;
} vpc_ctx;

static void vcycle_precond(void *ctx, const double *r, double *z) {
    vpc_ctx *c = (vpc_ctx *)ctx;
    vcycle(c->h, 0, r, z, &c->vp);
}

int orc_pcg_gamg(const orc_gamg *h, const double *b, double *x, double tol,
                 int max_iter, int n_pre, int n_post, double omega,
                 int transpose, int *iters, double *hist, double *true_res) {
    omat m = level_mat(&h->lev[0], transpose);
    vpc_ctx c = {h, {n_pre, n_post, 0, transpose, omega}};
    return cg_solve(&m, 2, vcycle_precond, &c, b, x, tol, max_iter, iters,
                    hist, true_res);
}

/* ---- FP32 V-cycle with an FP64 coarsest level (mixed form) -------------- */

static void level_fmat(const olevel *L, int transpose, fmat *m) {
    m->n = L->n;
    m->nf = L->nf;
    m->own = L->own;
    m->nb = L->nb;
    m->diag = L->diag32;
    m->up = transpose ? L->lo32 : L->up32;
    m->lo = transpose ? L->up32 : L->lo32;
}

static void jacobi_sweep32(const fmat *m, const float *r, float *e, float *y,
                           float omega) {
    fmat_mul(m, e, y);
    for (int32_t i = 0; i < m->n; ++i)
        y[i] = e[i] + omega * (r[i] - y[i]) / m->diag[i];
    memcpy(e, y, (size_t)m->n * sizeof(float));
}

static void tri_mul32(const fmat *m, int upper, const float *x, float *y) {
    for (int32_t i = 0; i < m->n; ++i) y[i] = 0.0f;
    for (int64_t f = 0; f < m->nf; ++f) {
        if (upper) y[m->own[f]] += m->up[f] * x[m->nb[f]];
        else y[m->nb[f]] += m->lo[f] * x[m->own[f]];
    }
}

/* the two-stage Gauss-Seidel sweep in FP32 (same steps as gs2_sweep) */
static void gs2_sweep32(const fmat *m, const float *r, float *e, int from_zero,
                        int backward, int inner, float *t, float *g, float *y) {
    const int32_t n = m->n;
    if (from_zero) {
        memcpy(t, r, (size_t)n * sizeof(float));
    } else {
        fmat_mul(m, e, t);
        for (int32_t i = 0; i < n; ++i) t[i] = r[i] - t[i];
    }
    for (int32_t i = 0; i < n; ++i) g[i] = t[i] / m->diag[i];
    for (int k = 0; k < inner; ++k) {
        tri_mul32(m, backward, g, y);
        for (int32_t i = 0; i < n; ++i) g[i] = (t[i] - y[i]) / m->diag[i];
    }
    for (int32_t i = 0; i < n; ++i) e[i] = from_zero ? g[i] : e[i] + g[i];
}

void orc_gs2_sweep32(int32_t n, int64_t nf, const int32_t *own, const int32_t *nb,
                     const float *diag, const float *upper, const float *lower,
                     const float *r, float *e, int from_zero, int backward,
                     int inner) {
    fmat m = {n, nf, own, nb, (float *)diag, (float *)upper, (float *)lower};
    float *t = xcalloc((size_t)n + 1, sizeof(float));
    float *g = xcalloc((size_t)n + 1, sizeof(float));
    float *y = xcalloc((size_t)n + 1, sizeof(float));
    gs2_sweep32(&m, r, e, from_zero, backward, inner, t, g, y);
    free(t); free(g); free(y);
}

static void vcycle32(const orc_gamg *h, int l, const float *r, float *e,
                     const vparams *vp) {
    const olevel *L = &h->lev[l];
    const int32_t n = L->n;
    if (l == h->nlev - 1) {
        double *rd = xcalloc(n, sizeof(double));
        double *ed = xcalloc(n, sizeof(double));
        for (int32_t i = 0; i < n; ++i) rd[i] = (double)r[i];
        coarsest_solve(h, L, rd, ed, vp->transpose);
        for (int32_t i = 0; i < n; ++i) e[i] = (float)ed[i];
        free(rd); free(ed);
        return;
    }
    const olevel *C = &h->lev[l + 1];
    fmat m;
    level_fmat(L, vp->transpose, &m);
    const float omega = (float)vp->omega;
    const int gs = h->smoother == ORC_SMOOTH_GS2;
    float *y = xcalloc(n, sizeof(float));
    float *t = xcalloc(n, sizeof(float));
    float *c = xcalloc(n, sizeof(float));
    float *g = xcalloc(n, sizeof(float));
    float *rc = xcalloc(C->n, sizeof(float));
    float *ec = xcalloc(C->n, sizeof(float));
    if (gs) {
        for (int32_t i = 0; i < n; ++i) e[i] = 0.0f;
        for (int s = 0; s < vp->n_pre; ++s)
            gs2_sweep32(&m, r, e, s == 0, 0, h->gs_inner, t, g, y);
    } else {
        for (int32_t i = 0; i < n; ++i)
            e[i] = vp->n_pre > 0 ? omega * r[i] / m.diag[i] : 0.0f;
        for (int s = 1; s < vp->n_pre; ++s) jacobi_sweep32(&m, r, e, y, omega);
    }
    fmat_mul(&m, e, t);
    for (int32_t i = 0; i < n; ++i) t[i] = r[i] - t[i];
    for (int32_t i = 0; i < n; ++i) rc[L->agg[i]] += t[i];
    vcycle32(h, l + 1, rc, ec, vp);
    for (int32_t i = 0; i < n; ++i) c[i] = ec[L->agg[i]];
    float sf = 1.0f;
    if (vp->scale) {
        fmat_mul(&m, c, y);
        double ct = dot_f32(n, c, t);
        double cac = dot_f32(n, c, y);
        if (isfinite(cac) && fabs(cac) > 1e-300) sf = (float)(ct / cac);
    }
    for (int32_t i = 0; i < n; ++i) e[i] = e[i] + sf * c[i];
    for (int k = 0; k < vp->n_post; ++k) {
        if (gs) gs2_sweep32(&m, r, e, 0, 1, h->gs_inner, t, g, y);
        else jacobi_sweep32(&m, r, e, y, omega);
    }
    free(y); free(t); free(c); free(g); free(rc); free(ec);
}

int orc_gamg_vcycle32(const orc_gamg *h, const float *r, float *e, int n_pre,
                      int n_post, double omega, int scale, int transpose) {
    vparams vp = {n_pre, n_post, scale, transpose, omega};
    vcycle32(h, 0, r, e, &vp);
    return ORC_OK;
}

typedef struct {
    const orc_gamg *h;
    vparams vp;
} vc32_ctx;

static int vcycle32_cb(void *ctx, const float *rhat, float *d, double res) {
    vc32_ctx *c = (vc32_ctx *)ctx;
    (void)res;
    vcycle32(c->h, 0, rhat, d, &c->vp);
    return 1;
}

/* inner FP32 CG preconditioned by one FP32 V-cycle (scaling off), from d = 0
 * on A32 d = rhat; FP64 dot products, alpha and beta rounded to FP32 */
typedef struct {
    const orc_gamg *h;
    vparams vp;
    double tol, outer_tol;
    int max_iter;
} vpc32_ctx;

static int pcg32_vcycle_inner(void *ctx, const float *rhat, float *d, double res) {
    vpc32_ctx *c = (vpc32_ctx *)ctx;
    const double tol_now = inner_target(c->tol, c->outer_tol, res);
    fmat m;
    level_fmat(&c->h->lev[0], c->vp.transpose, &m);
    const int32_t n = m.n;
    float *r = xcalloc(n, sizeof(float));
    float *z = xcalloc(n, sizeof(float));
    float *p = xcalloc(n, sizeof(float));
    float *q = xcalloc(n, sizeof(float));
    for (int32_t i = 0; i < n; ++i) { d[i] = 0.0f; r[i] = rhat[i]; }
    double r0 = sqrt(dot_f32(n, r, r));
    int it = 0;
    if (r0 > 0.0) {
        vcycle32(c->h, 0, r, z, &c->vp);
        for (int32_t i = 0; i < n; ++i) p[i] = z[i];
        double rho = dot_f32(n, r, z);
        while (it < c->max_iter) {
            fmat_mul(&m, p, q);
            double pq = dot_f32(n, p, q);
            if (!isfinite(pq) || fabs(pq) <= 1e-300) break;
            float af = (float)(rho / pq);
            for (int32_t i = 0; i < n; ++i) d[i] = d[i] + af * p[i];
            for (int32_t i = 0; i < n; ++i) r[i] = r[i] - af * q[i];
            ++it;
            if (sqrt(dot_f32(n, r, r)) <= tol_now * r0) break;
            vcycle32(c->h, 0, r, z, &c->vp);
            double rho_new = dot_f32(n, r, z);
            float bf = (float)(rho_new / rho);
            rho = rho_new;
            for (int32_t i = 0; i < n; ++i) p[i] = z[i] + bf * p[i];
        }
    }
    free(r); free(z); free(p); free(q);
    return it;
}

int orc_pcg_gamg_mixed(const orc_gamg *h, const double *b, double *x, double tol,
                       int max_refine, double inner_tol, int inner_max_iter,
                       int n_pre, int n_post, double omega, int transpose,
                       int *refinements, int *inner_iters, double *hist,
                       double *true_res) {
    omat m = level_mat(&h->lev[0], transpose);
    vpc32_ctx c = {h, {n_pre, n_post, 0, transpose, omega}, inner_tol, tol,
                   inner_max_iter};
    return refine(&m, b, x, tol, max_refine, pcg32_vcycle_inner, &c, refinements,
                  inner_iters, hist, true_res);
}

int orc_gamg_mixed(const orc_gamg *h, const double *b, double *x, double tol,
                   int max_refine, int n_pre, int n_post, double omega,
                   int scale, int transpose, int *refinements, double *hist,
                   double *true_res) {
    omat m = level_mat(&h->lev[0], transpose);
    vc32_ctx c = {h, {n_pre, n_post, scale, transpose, omega}};
    return refine(&m, b, x, tol, max_refine, vcycle32_cb, &c, refinements,
                  NULL, hist, true_res);
}

/* ------------------------------------------------------------------------ */
/* Adjoint gradients.  Not in the paper.  For A x = b and a loss L(x), with  */
/* lambda = A^-T dL/dx: dL/db = lambda and dL/dA_ij = -lambda_i x_j, which   */
/* in LDU storage is -lambda o x for diag, -lambda[own] x[nb] for upper and  */
/* -lambda[nb] x[own] for lower.  Pin: central finite differences and dense  */
/* brute force (tests).                                                      */
/* ------------------------------------------------------------------------ */

void orc_coeff_grad(int32_t n, int64_t nf, const int32_t *own,
                    const int32_t *nb, const double *lambda, const double *x,
                    double *g_diag, double *g_upper, double *g_lower) {
    for (int32_t i = 0; i < n; ++i) g_diag[i] = -(lambda[i] * x[i]);
    for (int64_t f = 0; f < nf; ++f) {
        g_upper[f] = -(lambda[own[f]] * x[nb[f]]);
        g_lower[f] = -(lambda[nb[f]] * x[own[f]]);
    }
}

/* ------------------------------------------------------------------------ */
/* Pressure-equation assembly, the step before the solve in every SIMPLE     */
/* iteration (Sec. 4.3 profile: lduMatrix::negSumDiag, the interpolation and */
/* divergence kernels; the pressure-assembly rows of the scaling tables):    */
/*   gamma_f = w_f gamma[own] + (1 - w_f) gamma[nb]   (linear interpolation) */
/*   upper_f = lower_f = gamma_f |S_f| delta_f         (fvm::laplacian)       */
/*   diag_i  = -(off-diagonal sum of column i) - diag_bc_i   (negSumDiag:    */
/*             diag[own] -= lower_f, diag[nb] -= upper_f, in face order)     */
/*   b_i     = sum_{own(f)=i} phi_f - sum_{nb(f)=i} phi_f + b_bc_i  (fvc::div) */
/* The _bc terms carry the boundary faces (Dirichlet coefficients, boundary  */
/* fluxes).  phi, b_bc and b may be NULL (no right-hand side).               */
/* Pins: closed-form 7-point stencil, zero column sums, telescoping          */
/* divergence, exact interpolation of linear fields.                         */
/* ------------------------------------------------------------------------ */
void orc_assemble_pressure(int32_t n, int64_t nf, const int32_t *own,
                           const int32_t *nb, const double *gamma,
                           const double *w, const double *mag_sf,
                           const double *delta, const double *diag_bc,
                           const double *phi, const double *b_bc, double *diag,
                           double *upper, double *lower, double *b) {
    for (int64_t f = 0; f < nf; ++f) {
        const double gf = w[f] * gamma[own[f]] + (1.0 - w[f]) * gamma[nb[f]];
        upper[f] = gf * mag_sf[f] * delta[f];
        lower[f] = upper[f];
    }
    for (int32_t i = 0; i < n; ++i) diag[i] = 0.0;
    for (int64_t f = 0; f < nf; ++f) {
        diag[own[f]] -= lower[f];
        diag[nb[f]] -= upper[f];
    }
    if (diag_bc)
        for (int32_t i = 0; i < n; ++i) diag[i] = diag[i] - diag_bc[i];
    if (phi && b) {
        for (int32_t i = 0; i < n; ++i) b[i] = 0.0;
        for (int64_t f = 0; f < nf; ++f) {
            b[own[f]] += phi[f];
            b[nb[f]] -= phi[f];
        }
        if (b_bc)
            for (int32_t i = 0; i < n; ++i) b[i] = b[i] + b_bc[i];
    }
}
