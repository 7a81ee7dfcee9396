// Amul / Tmul and the conjugate-gradient solvers.
//
// Amul is the sparse product of the lduMatrix (the "SpMVM (Amul + Tmul)" row of
// the kernel time breakdown, Sec. 4.3).  It is HBM-bound (about 0.15 flop per
// byte), so it is a pure streaming kernel: no matrix cores, coalesced 64-wide
// streams of columns and values, the x gather served from L2, and an
// atomic-free row ownership (each row is summed by exactly one lane).
//
// PCG with the diagonal preconditioner (Appendix A) runs as three fused
// kernels per iteration, with every scalar (rho, alpha, beta, residual) kept in
// device memory and a device "done" flag that freezes the iteration at the
// first iterate meeting the tolerance; the host only reads the scalars every
// check_every iterations, instead of synchronising after each kernel as the
// paper's executor does (Sec. 4.3, CUDA API statistics).
#include "device.hpp"

#include <cmath>

namespace ldu {

// ---------------------------------------------------------------- products
// NT: the result is stored nontemporally (level 0 above kStreamNtCells)
template <bool CMP, typename T, bool NT = false>
__global__ void __launch_bounds__(kBlock) k_amul(SellView<T> A, const T *__restrict__ x,
                                                 T *__restrict__ y) {
    const int lane = threadIdx.x & 63;
    for_each_slice<product_cap<CMP, T>()>(A.nslices, [&](int64_t s) {
        const int64_t p = s * kWave + lane;
        if (p < A.n) {
            const int32_t i = sv_row<CMP>(A, p);
            vst<NT>(y + i, sell_row<CMP>(A, s, lane, i, Direct<T>{x}));
        }
    });
}

void launch_amul(const SellView<double> &A, const double *x, double *y, hipStream_t st) {
    const int G = stream_grid_slices(A.nslices);
    if (A.pdeg) k_amul<true, double><<<G, kBlock, 0, st>>>(A, x, y);
    else if (A.n > kStreamNtCells) k_amul<false, double, true><<<G, kBlock, 0, st>>>(A, x, y);
    else k_amul<false, double><<<G, kBlock, 0, st>>>(A, x, y);
    HIP_CHECK(hipGetLastError());
}
void launch_amul32(const SellView<float> &A, const float *x, float *y, hipStream_t st) {
    const int G = stream_grid_slices(A.nslices);
    if (A.pdeg) k_amul<true, float><<<G, kBlock, 0, st>>>(A, x, y);
    else k_amul<false, float><<<G, kBlock, 0, st>>>(A, x, y);
    HIP_CHECK(hipGetLastError());
}

// ---------------------------------------------------------------- scalars
__global__ void k_init_scalars(DevScalars *ds, double tol, int max_iter) {
    DevScalars z{};
    z.tol = tol;
    z.max_iter = max_iter;
    *ds = z;
}
__global__ void k_set_done(DevScalars *ds, int done) { ds->done = done; }
void set_done(ldu_t *h, int done, hipStream_t st) {
    k_set_done<<<1, 1, 0, st>>>(h->dev, done);
    HIP_CHECK(hipGetLastError());
}

void set_scalars_for_solve(ldu_t *h, double tol, int max_iter, hipStream_t st) {
    k_init_scalars<<<1, 1, 0, st>>>(h->dev, tol, max_iter);
    HIP_CHECK(hipGetLastError());
}

void read_scalars(ldu_t *h, hipStream_t st) {
    HIP_CHECK(hipMemcpyAsync(h->host, h->dev, sizeof(DevScalars), hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipStreamSynchronize(st));
}

void ensure_hist(ldu_t *h, int64_t entries) {
    // the device history keeps the first kMaxHistory entries of a solve; the
    // epilogues write entry k only while k < hist_cap
    if (entries > kMaxHistory) entries = kMaxHistory;
    if (entries < 1) entries = 1;
    if (entries <= h->hist_cap) return;
    if (h->hist) h->arena.release(h->hist);
    h->hist = nullptr;
    h->hist_cap = 0;
    h->hist = h->arena.get<double>((size_t)entries);
    h->hist_cap = (int)entries;
}

void copy_history(ldu_t *h, ldu_stats *stats, int count, hipStream_t st) {
    if (!stats) return;
    stats->history_count = 0;
    if (!stats->history || stats->history_len <= 0 || count <= 0) return;
    int m = count < stats->history_len ? count : stats->history_len;
    if (m > h->hist_cap) m = h->hist_cap;
    HIP_CHECK(hipMemcpyAsync(stats->history, h->hist, sizeof(double) * m,
                             hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipStreamSynchronize(st));
    stats->history_count = m;
}

// ---------------------------------------------------------------- residual
// r = b - A x, plus ||r||^2, ||b||^2 and, when P is set, p = D^-1 r (or r)
// and rho = r.p; MAXABS adds ||r||_inf.  Epilogue modes:
//   kResPlain  : scalars only (true residual, CG (re)start)
//   kResCycle  : GAMG/refinement outer loop, honours and sets the done flag
enum { kResPlain = 0, kResCycle = 1 };

template <bool CMP, bool P, bool MAXABS>
__global__ void __launch_bounds__(kBlock)
k_residual(SellView<double> A, const double *__restrict__ b, const double *__restrict__ x,
           double *__restrict__ r, double *__restrict__ p, int precond, int gated,
           double *partials, const DevScalars *ds) {
    if (gated && ds->done) return;
    const int lane = threadIdx.x & 63;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};  // rr, bb, rho, maxabs
    for_each_slice<product_cap<CMP, double>()>(A.nslices, [&](int64_t s) {
        const int64_t pos = s * kWave + lane;
        if (pos < A.n) {
            const int32_t i = sv_row<CMP>(A, pos);
            const double bi = b[i];
            const double ri = bi - sell_row<CMP>(A, s, lane, i, Direct<double>{x});
            r[i] = ri;
            acc[0] += ri * ri;
            acc[1] += bi * bi;
            if (P) {
                const double zi = precond ? ri / A.diag[i] : ri;
                p[i] = zi;
                acc[2] += ri * zi;
            }
            if (MAXABS) acc[3] = fmax(acc[3], fabs(ri));
        }
    });
    block_partials<4, 1>(acc, partials);
}

// epilogue of the residual: scalars, history entry and, for the outer loop
// of GAMG and of the refinement (kResCycle), the convergence decision
struct EpiResidual {
    int mode, write_hist, has_p;
    double *hist;
    int hist_cap;
    __device__ bool active(const DevScalars *ds) const {
        return mode != kResCycle || !ds->done;
    }
    __device__ void operator()(const double *t, DevScalars *ds) const {
        ds->rr = t[0];
        ds->bb = t[1];
        ds->bnorm = sqrt(t[1]);
        ds->maxabs = t[3];
        if (has_p) ds->rho = t[2];
        ds->x_pending = 0;  // a (re)start owes no solution update
        // b = 0 gives 0; a non-finite b or x gives a non-finite residual
        // (a NaN norm of b must not read as b = 0)
        const double res = ds->bnorm == 0.0 ? 0.0 : sqrt(t[0]) / ds->bnorm;
        ds->res = res;
        const int it = ds->iters;
        if (write_hist && hist && it < hist_cap) hist[it] = res;
        if (mode == kResCycle) {
            if (!isfinite(res)) {
                ds->status = LDU_ERR_NAN;
                ds->done = kFailed;
            } else if (res <= ds->tol) {
                ds->done = kConverged;
            } else if (it >= ds->max_iter) {
                ds->done = kMaxIter;
            } else {
                ds->iters = it + 1;
            }
        }
    }
};

template <bool P, bool MAXABS>
static void launch_residual(ldu_t *h, const SellView<double> &A, const double *b, const double *x,
                            double *r, double *p, int precond, int mode, bool write_hist,
                            hipStream_t st) {
    const int G = stream_grid_slices(A.nslices);
    if (A.pdeg)
        k_residual<true, P, MAXABS><<<G, kBlock, 0, st>>>(A, b, x, r, p, precond,
                                                          mode == kResCycle, h->partials, h->dev);
    else
        k_residual<false, P, MAXABS><<<G, kBlock, 0, st>>>(A, b, x, r, p, precond,
                                                           mode == kResCycle, h->partials, h->dev);
    launch_finalize<4, 1>(h->partials, G, h->dev,
                          EpiResidual{mode, write_hist ? 1 : 0, P ? 1 : 0, h->hist, h->hist_cap}, st);
    HIP_CHECK(hipGetLastError());
}

void launch_residual_cycle(ldu_t *h, const SellView<double> &A, const double *b,
                           const double *x, double *r, bool maxabs, int grid,
                           hipStream_t st) {
    (void)grid;
    if (maxabs) launch_residual<false, true>(h, A, b, x, r, nullptr, 0, kResCycle, true, st);
    else launch_residual<false, false>(h, A, b, x, r, nullptr, 0, kResCycle, true, st);
}

void launch_residual_plain(ldu_t *h, const SellView<double> &A, const double *b,
                           const double *x, double *r, bool write_hist, int grid,
                           hipStream_t st) {
    (void)grid;
    launch_residual<false, false>(h, A, b, x, r, nullptr, 0, kResPlain, write_hist, st);
}

double residual_norm(ldu_t *h, const Level &L, bool tr, const double *b, const double *x,
                     double *r_out, hipStream_t st) {
    launch_residual<false, false>(h, L.A.view(tr), b, x, r_out, nullptr, 0, kResPlain, false, st);
    read_scalars(h, st);
    return h->host->res;
}

// ---------------------------------------------------------------- PCG, FP64
// q = A p and p.q -> alpha = rho / p.q
template <bool CMP, bool NT = false>
__global__ void __launch_bounds__(kBlock)
k_pcg_q(SellView<double> A, const double *__restrict__ p, double *__restrict__ q,
        double *partials, const DevScalars *ds) {
    if (ds->done) return;
    const int lane = threadIdx.x & 63;
    double acc[1] = {0.0};
    for_each_slice<product_cap<CMP, double>()>(A.nslices, [&](int64_t s) {
        const int64_t pos = s * kWave + lane;
        if (pos < A.n) {
            const int32_t i = sv_row<CMP>(A, pos);
            const double qi = sell_row<CMP>(A, s, lane, i, Direct<double>{p});
            vst<NT>(q + i, qi);
            acc[0] += p[i] * qi;
        }
    });
    block_partials<1>(acc, partials);
}

struct EpiAlpha {
    __device__ bool active(const DevScalars *ds) const { return !ds->done; }
    __device__ void operator()(const double *t, DevScalars *ds) const {
        const double pq = t[0];
        ds->pq = pq;
        if (!isfinite(pq) || fabs(pq) <= 1e-300) {
            ds->status = LDU_ERR_BREAKDOWN;
            ds->done = kFailed;
        } else {
            ds->alpha = ds->rho / pq;
            ds->x_pending = 1;
        }
    }
};

void launch_pcg_q(ldu_t *h, const SellView<double> &A, const double *p, double *q, int grid,
                  hipStream_t st) {
    if (A.pdeg) k_pcg_q<true><<<grid, kBlock, 0, st>>>(A, p, q, h->partials, h->dev);
    else if (A.n > kStreamNtCells)
        k_pcg_q<false, true><<<grid, kBlock, 0, st>>>(A, p, q, h->partials, h->dev);
    else k_pcg_q<false><<<grid, kBlock, 0, st>>>(A, p, q, h->partials, h->dev);
    launch_finalize<1>(h->partials, grid, h->dev, EpiAlpha{}, st);
}

// r -= alpha q; ||r||^2 and r.D^-1 r.  The iteration's x += alpha p waits
// for the direction update, which reads p anyway (k_pcg_p), or, when the
// solve stops in between, for k_x_pending: one read of p per iteration
// instead of two.
template <bool NT>
__global__ void __launch_bounds__(kBlock)
k_pcg_update(int32_t n, int64_t S, const double *__restrict__ D, double *__restrict__ r,
             const double *__restrict__ q, int precond, double *partials,
             const DevScalars *ds) {
    if (ds->done) return;
    const double alpha = ds->alpha;
    const int lane = threadIdx.x & 63;
    double acc[2] = {0.0, 0.0};
    for_each_slice(S, [&](int64_t s) {
        const int64_t i = s * kWave + lane;
        if (i < n) {
            const double ri = vld<NT>(r + i) - alpha * vld<NT>(q + i);
            vst<NT>(r + i, ri);
            const double zi = precond ? ri / vld<NT>(D + i) : ri;
            acc[0] += ri * ri;
            acc[1] += ri * zi;
        }
    });
    block_partials<2>(acc, partials);
}

// iteration count, residual history and convergence test after the x, r
// update; with_beta: also beta = rho'/rho from the second sum
struct EpiConverge {
    double *hist;
    int hist_cap;
    int with_beta;
    __device__ bool active(const DevScalars *ds) const { return !ds->done; }
    __device__ void operator()(const double *t, DevScalars *ds) const {
        const int it = ds->iters + 1;
        ds->iters = it;
        ds->rr = t[0];
        const double res = sqrt(t[0]) / ds->bnorm;
        ds->res = res;
        if (hist && it < hist_cap) hist[it] = res;
        if (!isfinite(res)) {
            ds->status = LDU_ERR_NAN;
            ds->done = kFailed;
        } else if (res <= ds->tol) {
            ds->done = kConverged;
        } else if (it >= ds->max_iter) {
            ds->done = kMaxIter;
        } else if (with_beta) {
            ds->beta = t[1] / ds->rho;
            ds->rho = t[1];
            ds->x_pending = 0;  // k_pcg_p applies it next
        }
    }
};

void launch_converge(ldu_t *h, int grid, bool with_beta, hipStream_t st) {
    if (with_beta) launch_finalize<2>(h->partials, grid, h->dev, EpiConverge{h->hist, h->hist_cap, 1}, st);
    else launch_finalize<1>(h->partials, grid, h->dev, EpiConverge{h->hist, h->hist_cap, 0}, st);
}

// x += alpha p (the iteration's solution update, deferred from
// k_pcg_update); p = D^-1 r + beta p.  p keeps the default cache policy even
// where the other vectors stream nontemporally (NT): the CG product gathers
// it next (c4's diagonal PCG: 1.05 -> 1.02 s per right-hand side).
template <bool NT>
__global__ void __launch_bounds__(kBlock)
k_pcg_p(int32_t n, int64_t S, const double *__restrict__ D, const double *__restrict__ r,
        double *__restrict__ x, double *__restrict__ p, int precond, const DevScalars *ds) {
    if (ds->done) return;
    const double alpha = ds->alpha, beta = ds->beta;
    const int lane = threadIdx.x & 63;
    for_each_slice(S, [&](int64_t s) {
        const int64_t i = s * kWave + lane;
        if (i < n) {
            const double pi = p[i];
            vst<NT>(x + i, vld<NT>(x + i) + alpha * pi);
            const double ri = vld<NT>(r + i);
            const double zi = precond ? ri / vld<NT>(D + i) : ri;
            p[i] = zi + beta * pi;
        }
    });
}

// x += alpha p when the stopped solve's last iteration still owes it: alpha
// was formed (x_pending) but the direction update that applies it did not
// run.  The same expression as in the direction updates.
__global__ void __launch_bounds__(kBlock)
k_x_pending(int32_t n, int64_t S, double *__restrict__ x, const double *__restrict__ p,
            const DevScalars *ds) {
    if (!ds->x_pending) return;
    const double alpha = ds->alpha;
    const int lane = threadIdx.x & 63;
    for_each_slice(S, [&](int64_t s) {
        const int64_t i = s * kWave + lane;
        if (i < n) x[i] = x[i] + alpha * p[i];
    });
}

void launch_x_pending(ldu_t *h, double *x, int32_t n, int64_t S, int grid, hipStream_t st) {
    k_x_pending<<<grid, kBlock, 0, st>>>(n, S, x, h->p, h->dev);
    HIP_CHECK(hipGetLastError());
}

__global__ void k_fill(double *a, int64_t n, double v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        a[i] = v;
}
static void fill(double *a, int64_t n, double v, hipStream_t st) {
    int64_t g = (n + kBlock - 1) / kBlock;
    g = g > 4096 ? 4096 : (g < 1 ? 1 : g);
    k_fill<<<(unsigned)g, kBlock, 0, st>>>(a, n, v);
}
void zero_vector(double *a, int64_t n, hipStream_t st) {
    fill(a, n, 0.0, st);
    HIP_CHECK(hipStreamSynchronize(st));
}

static void fill_stats_common(ldu_stats *stats) {
    if (!stats) return;
    stats->refinements = 0;
    stats->n_levels = 0;
    stats->history_count = 0;
}

int pcg_fp64(ldu_t *h, const double *b, double *x, const ldu_pcg_opts &o, bool tr,
             ldu_stats *stats, hipStream_t st, bool own_hist) {
    const Level &L = h->L0;
    const SellView<double> A = L.A.view(tr);
    const int n = L.n;
    const int64_t S = L.A.nslices;
    const int G = stream_grid_slices(S);
    const int precond = o.precond ? 1 : 0;
    const bool nt = n > kStreamNtCells;
    if (own_hist) ensure_hist(h, (int64_t)o.max_iter + 2);
    fill_stats_common(stats);
    set_scalars_for_solve(h, o.rel_tol, o.max_iter, st);
    launch_residual<true, false>(h, A, b, x, h->r, h->p, precond, kResPlain, true, st);
    read_scalars(h, st);
    DevScalars &hs = *h->host;
    if (stats) stats->initial_residual = hs.res;
    if (hs.bnorm == 0.0) {
        fill(x, n, 0.0, st);
        HIP_CHECK(hipStreamSynchronize(st));
        if (stats) {
            stats->iterations = 0;
            stats->converged = 1;
            stats->initial_residual = stats->final_residual = 0.0;
        }
        copy_history(h, stats, 1, st);
        return LDU_OK;
    }
    if (!std::isfinite(hs.res)) throw Error(LDU_ERR_NAN, "non-finite initial residual");
    double res = hs.res;
    int status = LDU_OK;
    const int every = o.check_every > 0 ? o.check_every : 16;
    while (res > o.rel_tol) {
        for (;;) {
            for (int k = 0; k < every; ++k) {
                launch_pcg_q(h, A, h->p, h->q, G, st);
                if (nt)
                    k_pcg_update<true><<<G, kBlock, 0, st>>>(n, S, A.diag, h->r, h->q, precond,
                                                             h->partials, h->dev);
                else
                    k_pcg_update<false><<<G, kBlock, 0, st>>>(n, S, A.diag, h->r, h->q, precond,
                                                              h->partials, h->dev);
                launch_converge(h, G, true, st);
                if (nt)
                    k_pcg_p<true><<<G, kBlock, 0, st>>>(n, S, A.diag, h->r, x, h->p, precond,
                                                        h->dev);
                else
                    k_pcg_p<false><<<G, kBlock, 0, st>>>(n, S, A.diag, h->r, x, h->p, precond,
                                                         h->dev);
            }
            HIP_CHECK(hipGetLastError());
            read_scalars(h, st);
            if (hs.done != kRunning) break;
        }
        // the stopping iteration's x += alpha p (none when alpha itself failed)
        launch_x_pending(h, x, n, S, G, st);
        if (hs.done == kFailed) {
            status = hs.status;
            break;
        }
        // true residual; restart from it if the recursive one drifted
        launch_residual<true, false>(h, A, b, x, h->r, h->p, precond, kResPlain, false, st);
        read_scalars(h, st);
        res = hs.res;
        if (!std::isfinite(res)) { status = LDU_ERR_NAN; break; }
        if (res <= o.rel_tol) { status = LDU_OK; break; }
        if (hs.iters >= o.max_iter) { status = LDU_NOT_CONVERGED; break; }
        k_set_done<<<1, 1, 0, st>>>(h->dev, kRunning);
    }
    const int iters = hs.iters;
    if (stats) {
        stats->iterations = iters;
        stats->final_residual = res;
        stats->converged = (status == LDU_OK);
    }
    copy_history(h, stats, iters + 1, st);
    return status;
}

// ---------------------------------------------------------------- PBiCG
// Preconditioned bi-conjugate gradients for non-symmetric A (the paper's
// solver for the velocity and turbulence systems, whose profile pairs Amul
// with Tmul).  Shadow residual rt = r at every (re)start; M = D or I.
//   q = A p, qt = A^T pt, sigma = pt.q;  alpha = rho / sigma
//   x += alpha p; r -= alpha q; rt -= alpha qt;  ||r||^2, rho' = (M^-1 r).rt
//   beta = rho' / rho;  p = M^-1 r + beta p;  pt = M^-1 rt + beta pt

// rt = r, pt = p (the residual kernel has set r, p = M^-1 r and rho = r.p)
__global__ void __launch_bounds__(kBlock)
k_bicg_start(int32_t n, int64_t S, const double *__restrict__ r, const double *__restrict__ p,
             double *__restrict__ rt, double *__restrict__ pt, const DevScalars *ds) {
    if (ds->done) return;
    const int lane = threadIdx.x & 63;
    for_each_slice(S, [&](int64_t s) {
        const int64_t i = s * kWave + lane;
        if (i < n) {
            rt[i] = r[i];
            pt[i] = p[i];
        }
    });
}

// q = A p and qt = A^T pt in one pass over the shared column structure
// (valT holds A^T at the same positions); sigma = pt . q
template <bool CMP>
__global__ void __launch_bounds__(kBlock)
k_bicg_q(SellView<double> A, const double *__restrict__ valT, const double *__restrict__ p,
         const double *__restrict__ pt, double *__restrict__ q, double *__restrict__ qt,
         double *partials, const DevScalars *ds) {
    if (ds->done) return;
    SellView<double> At = A;
    At.val = valT;
    const int lane = threadIdx.x & 63;
    double acc[1] = {0.0};
    for_each_slice<product_cap<CMP, double>()>(A.nslices, [&](int64_t s) {
        const int64_t pos = s * kWave + lane;
        if (pos < A.n) {
            const int32_t i = sv_row<CMP>(A, pos);
            const double qi = sell_row<CMP>(A, s, lane, i, Direct<double>{p});
            const double qti = sell_row<CMP>(At, s, lane, i, Direct<double>{pt});
            q[i] = qi;
            qt[i] = qti;
            acc[0] += pt[i] * qi;
        }
    });
    block_partials<1>(acc, partials);
}

// x += alpha p; r -= alpha q; rt -= alpha qt; ||r||^2 and (M^-1 r) . rt
__global__ void __launch_bounds__(kBlock)
k_bicg_update(int32_t n, int64_t S, const double *__restrict__ D, double *__restrict__ x,
              double *__restrict__ r, double *__restrict__ rt, const double *__restrict__ p,
              const double *__restrict__ q, const double *__restrict__ qt, int precond,
              double *partials, const DevScalars *ds) {
    if (ds->done) return;
    const double alpha = ds->alpha;
    const int lane = threadIdx.x & 63;
    double acc[2] = {0.0, 0.0};
    for_each_slice(S, [&](int64_t s) {
        const int64_t i = s * kWave + lane;
        if (i < n) {
            x[i] = x[i] + alpha * p[i];
            const double ri = r[i] - alpha * q[i];
            const double rti = rt[i] - alpha * qt[i];
            r[i] = ri;
            rt[i] = rti;
            const double zi = precond ? ri / D[i] : ri;
            acc[0] += ri * ri;
            acc[1] += zi * rti;
        }
    });
    block_partials<2>(acc, partials);
}

// convergence as for CG, then beta, with breakdown when rho' vanishes
struct EpiBicg {
    double *hist;
    int hist_cap;
    __device__ bool active(const DevScalars *ds) const { return !ds->done; }
    __device__ void operator()(const double *t, DevScalars *ds) const {
        const int it = ds->iters + 1;
        ds->iters = it;
        ds->rr = t[0];
        const double res = sqrt(t[0]) / ds->bnorm;
        ds->res = res;
        if (hist && it < hist_cap) hist[it] = res;
        if (!isfinite(res)) {
            ds->status = LDU_ERR_NAN;
            ds->done = kFailed;
        } else if (res <= ds->tol) {
            ds->done = kConverged;
        } else if (it >= ds->max_iter) {
            ds->done = kMaxIter;
        } else if (!isfinite(t[1]) || fabs(t[1]) <= 1e-300) {
            ds->status = LDU_ERR_BREAKDOWN;
            ds->done = kFailed;
        } else {
            ds->beta = t[1] / ds->rho;
            ds->rho = t[1];
        }
    }
};

// p = M^-1 r + beta p; pt = M^-1 rt + beta pt
__global__ void __launch_bounds__(kBlock)
k_bicg_p(int32_t n, int64_t S, const double *__restrict__ D, const double *__restrict__ r,
         const double *__restrict__ rt, double *__restrict__ p, double *__restrict__ pt,
         int precond, const DevScalars *ds) {
    if (ds->done) return;
    const double beta = ds->beta;
    const int lane = threadIdx.x & 63;
    for_each_slice(S, [&](int64_t s) {
        const int64_t i = s * kWave + lane;
        if (i < n) {
            const double zi = precond ? r[i] / D[i] : r[i];
            const double zti = precond ? rt[i] / D[i] : rt[i];
            p[i] = zi + beta * p[i];
            pt[i] = zti + beta * pt[i];
        }
    });
}

int pbicg_fp64(ldu_t *h, const double *b, double *x, const ldu_pcg_opts &o, bool tr,
               ldu_stats *stats, hipStream_t st) {
    const Level &L = h->L0;
    const SellView<double> A = L.A.view(tr);
    const double *valT = tr ? L.A.val : L.A.valT;
    const int n = L.n;
    const int64_t S = L.A.nslices;
    const int G = stream_grid_slices(S);
    const int precond = o.precond ? 1 : 0;
    if (!h->rt) {  // shadow vectors, allocated on the handle's first PBiCG solve
        h->rt = h->arena.get<double>(n);
        h->pt = h->arena.get<double>(n);
        h->qt = h->arena.get<double>(n);
    }
    ensure_hist(h, (int64_t)o.max_iter + 2);
    fill_stats_common(stats);
    set_scalars_for_solve(h, o.rel_tol, o.max_iter, st);
    launch_residual<true, false>(h, A, b, x, h->r, h->p, precond, kResPlain, true, st);
    read_scalars(h, st);
    DevScalars &hs = *h->host;
    if (stats) stats->initial_residual = hs.res;
    if (hs.bnorm == 0.0) {
        fill(x, n, 0.0, st);
        HIP_CHECK(hipStreamSynchronize(st));
        if (stats) {
            stats->iterations = 0;
            stats->converged = 1;
            stats->initial_residual = stats->final_residual = 0.0;
        }
        copy_history(h, stats, 1, st);
        return LDU_OK;
    }
    if (!std::isfinite(hs.res)) throw Error(LDU_ERR_NAN, "non-finite initial residual");
    double res = hs.res;
    int status = LDU_OK;
    const int every = o.check_every > 0 ? o.check_every : 16;
    while (res > o.rel_tol) {
        k_bicg_start<<<G, kBlock, 0, st>>>(n, S, h->r, h->p, h->rt, h->pt, h->dev);
        for (;;) {
            for (int k = 0; k < every; ++k) {
                if (A.pdeg)
                    k_bicg_q<true><<<G, kBlock, 0, st>>>(A, valT, h->p, h->pt, h->q, h->qt,
                                                         h->partials, h->dev);
                else
                    k_bicg_q<false><<<G, kBlock, 0, st>>>(A, valT, h->p, h->pt, h->q, h->qt,
                                                          h->partials, h->dev);
                launch_finalize<1>(h->partials, G, h->dev, EpiAlpha{}, st);
                k_bicg_update<<<G, kBlock, 0, st>>>(n, S, A.diag, x, h->r, h->rt, h->p, h->q,
                                                    h->qt, precond, h->partials, h->dev);
                launch_finalize<2>(h->partials, G, h->dev, EpiBicg{h->hist, h->hist_cap}, st);
                k_bicg_p<<<G, kBlock, 0, st>>>(n, S, A.diag, h->r, h->rt, h->p, h->pt, precond,
                                               h->dev);
            }
            HIP_CHECK(hipGetLastError());
            read_scalars(h, st);
            if (hs.done != kRunning) break;
        }
        if (hs.done == kFailed) {
            status = hs.status;
            break;
        }
        // true residual; restart from it (new shadow) if the recursive one drifted
        launch_residual<true, false>(h, A, b, x, h->r, h->p, precond, kResPlain, false, st);
        read_scalars(h, st);
        res = hs.res;
        if (!std::isfinite(res)) { status = LDU_ERR_NAN; break; }
        if (res <= o.rel_tol) { status = LDU_OK; break; }
        if (hs.iters >= o.max_iter) { status = LDU_NOT_CONVERGED; break; }
        k_set_done<<<1, 1, 0, st>>>(h->dev, kRunning);
    }
    const int iters = hs.iters;
    if (stats) {
        stats->iterations = iters;
        stats->final_residual = res;
        stats->converged = (status == LDU_OK);
    }
    copy_history(h, stats, iters + 1, st);
    return status;
}

// ---------------------------------------------------------------- PCG, mixed
// Outer FP64 refinement with inner FP32 CG.  Inner dot products accumulate
// in FP64; alpha and beta are formed in FP64 and rounded to FP32.

// rhat = fp32(r / s), d = 0, z = rhat / D32, p = z; ||rhat||^2 and rhat.z
__global__ void __launch_bounds__(kBlock)
k_mx_start(int32_t n, int64_t S, const double *__restrict__ r, const float *__restrict__ D,
           float *__restrict__ r32, float *__restrict__ d32, float *__restrict__ p32,
           double *partials, const DevScalars *ds) {
    if (ds->done) return;
    const double sc = ds->maxabs;
    const int lane = threadIdx.x & 63;
    double acc[2] = {0.0, 0.0};
    for_each_slice(S, [&](int64_t s) {
        const int64_t i = s * kWave + lane;
        if (i < n) {
            const float ri = (float)(r[i] / sc);
            const float zi = ri / D[i];
            r32[i] = ri;
            d32[i] = 0.0f;
            p32[i] = zi;
            acc[0] += (double)ri * (double)ri;
            acc[1] += (double)ri * (double)zi;
        }
    });
    block_partials<2>(acc, partials);
}

// start of an inner solve: ||rhat||, rho, and the inner target
// max(inner_tol, 0.3 tol / res) for the current outer residual res
struct EpiMxStart {
    int has_rho;
    __device__ bool active(const DevScalars *ds) const { return !ds->done; }
    __device__ void operator()(const double *t, DevScalars *ds) const {
        ds->scale = ds->maxabs;
        ds->r0 = sqrt(t[0]);
        if (has_rho) ds->rho = t[1];
        ds->inner_iters = 0;
        ds->inner_done = !(ds->r0 > 0.0);
        const double target = 0.3 * ds->tol / ds->res;
        ds->inner_now = target > ds->inner_tol ? target : ds->inner_tol;
    }
};

template <bool CMP>
__global__ void __launch_bounds__(kBlock)
k_mx_q(SellView<float> A, const float *__restrict__ p, float *__restrict__ q, double *partials,
       const DevScalars *ds) {
    if (vc_skip(ds)) return;
    const int lane = threadIdx.x & 63;
    double acc[1] = {0.0};
    for_each_slice(A.nslices, [&](int64_t s) {
        const int64_t pos = s * kWave + lane;
        if (pos < A.n) {
            const int32_t i = sv_row<CMP>(A, pos);
            const float qi = sell_row<CMP>(A, s, lane, i, Direct<float>{p});
            q[i] = qi;
            acc[0] += (double)p[i] * (double)qi;
        }
    });
    block_partials<1>(acc, partials);
}

struct EpiMxAlpha {
    __device__ bool active(const DevScalars *ds) const { return !vc_skip(ds); }
    __device__ void operator()(const double *t, DevScalars *ds) const {
        const double pq = t[0];
        if (!isfinite(pq) || fabs(pq) <= 1e-300) ds->inner_done = 1;
        else ds->alpha = ds->rho / pq;
    }
};

template <bool DIAGZ>
__global__ void __launch_bounds__(kBlock)
k_mx_update(int32_t n, int64_t S, const float *__restrict__ D, float *__restrict__ d,
            float *__restrict__ r, const float *__restrict__ p, const float *__restrict__ q,
            double *partials, const DevScalars *ds) {
    if (vc_skip(ds)) return;
    const float af = (float)ds->alpha;
    const int lane = threadIdx.x & 63;
    double acc[2] = {0.0, 0.0};
    for_each_slice(S, [&](int64_t s) {
        const int64_t i = s * kWave + lane;
        if (i < n) {
            const float di = d[i] + af * p[i];
            const float ri = r[i] - af * q[i];
            d[i] = di;
            r[i] = ri;
            acc[0] += (double)ri * (double)ri;
            if (DIAGZ) {
                const float zi = ri / D[i];
                acc[1] += (double)ri * (double)zi;
            }
        }
    });
    block_partials<2>(acc, partials);
}

struct EpiMxInner {
    int with_beta;
    __device__ bool active(const DevScalars *ds) const { return !vc_skip(ds); }
    __device__ void operator()(const double *t, DevScalars *ds) const {
        const int it = ds->inner_iters + 1;
        ds->inner_iters = it;
        if (sqrt(t[0]) <= ds->inner_now * ds->r0 || it >= ds->inner_max) {
            ds->inner_done = 1;
        } else if (with_beta) {
            ds->beta = t[1] / ds->rho;
            ds->rho = t[1];
        }
    }
};

__global__ void __launch_bounds__(kBlock)
k_mx_p(int32_t n, int64_t S, const float *__restrict__ D, const float *__restrict__ r,
       float *__restrict__ p, const DevScalars *ds) {
    if (vc_skip(ds)) return;
    const float bf = (float)ds->beta;
    const int lane = threadIdx.x & 63;
    for_each_slice(S, [&](int64_t s) {
        const int64_t i = s * kWave + lane;
        if (i < n) p[i] = r[i] / D[i] + bf * p[i];
    });
}

void launch_mx_q(ldu_t *h, const SellView<float> &A32, int G, hipStream_t st) {
    if (A32.pdeg) k_mx_q<true><<<G, kBlock, 0, st>>>(A32, h->p32, h->q32, h->partials, h->dev);
    else k_mx_q<false><<<G, kBlock, 0, st>>>(A32, h->p32, h->q32, h->partials, h->dev);
    launch_finalize<1>(h->partials, G, h->dev, EpiMxAlpha{}, st);
}

// d += alpha p; r -= alpha q; ||r||^2 and the inner convergence test (the
// preconditioned direction comes from outside)
void launch_mx_update_plain(ldu_t *h, int32_t n, int64_t S, int G, hipStream_t st) {
    k_mx_update<false><<<G, kBlock, 0, st>>>(n, S, nullptr, h->d32, h->r32, h->p32, h->q32,
                                             h->partials, h->dev);
    launch_finalize<2>(h->partials, G, h->dev, EpiMxInner{0}, st);
}

// x += s * fp64(d)
__global__ void __launch_bounds__(kBlock)
k_mx_refine(int32_t n, int64_t S, const float *__restrict__ d, double *__restrict__ x,
            const DevScalars *ds) {
    if (ds->done) return;
    const double sc = ds->scale;
    const int lane = threadIdx.x & 63;
    for_each_slice(S, [&](int64_t s) {
        const int64_t i = s * kWave + lane;
        if (i < n) x[i] = x[i] + sc * (double)d[i];
    });
}

__global__ void k_mx_set_inner(DevScalars *ds, double inner_tol, int inner_max) {
    ds->inner_tol = inner_tol;
    ds->inner_max = inner_max;
}
void set_inner(ldu_t *h, double inner_tol, int inner_max, hipStream_t st) {
    k_mx_set_inner<<<1, 1, 0, st>>>(h->dev, inner_tol, inner_max);
}
void launch_mx_refine(ldu_t *h, double *x, int32_t n, int64_t S, int G, hipStream_t st) {
    k_mx_refine<<<G, kBlock, 0, st>>>(n, S, h->d32, x, h->dev);
}

int pcg_mixed(ldu_t *h, const double *b, double *x, const ldu_pcg_opts &o, bool tr,
              ldu_stats *stats, hipStream_t st) {
    Level &L = h->L0;
    ensure_f32(L, h->arena, st);
    const SellView<double> A = L.A.view(tr);
    const SellView<float> A32 = L.A.view32(tr);
    const int n = L.n;
    const int64_t S = L.A.nslices;
    const int G = stream_grid_slices(S);
    ensure_hist(h, (int64_t)o.max_refine + 2);
    fill_stats_common(stats);
    set_scalars_for_solve(h, o.rel_tol, o.max_refine, st);
    k_mx_set_inner<<<1, 1, 0, st>>>(h->dev, o.inner_rel_tol, o.inner_max_iter);
    launch_residual<false, true>(h, A, b, x, h->r, nullptr, 0, kResCycle, true, st);
    read_scalars(h, st);
    DevScalars &hs = *h->host;
    if (stats) stats->initial_residual = hs.res;
    if (hs.bnorm == 0.0) {
        fill(x, n, 0.0, st);
        HIP_CHECK(hipStreamSynchronize(st));
        if (stats) {
            stats->iterations = 0;
            stats->converged = 1;
            stats->initial_residual = stats->final_residual = 0.0;
        }
        copy_history(h, stats, 1, st);
        return LDU_OK;
    }
    const int every = o.check_every > 0 ? o.check_every : 16;
    long long inner_total = 0;
    while (hs.done == kRunning) {
        k_mx_start<<<G, kBlock, 0, st>>>(n, S, h->r, A32.diag, h->r32, h->d32, h->p32,
                                         h->partials, h->dev);
        launch_finalize<2>(h->partials, G, h->dev, EpiMxStart{1}, st);
        for (;;) {
            for (int k = 0; k < every; ++k) {
                if (A32.pdeg)
                    k_mx_q<true><<<G, kBlock, 0, st>>>(A32, h->p32, h->q32, h->partials, h->dev);
                else
                    k_mx_q<false><<<G, kBlock, 0, st>>>(A32, h->p32, h->q32, h->partials, h->dev);
                launch_finalize<1>(h->partials, G, h->dev, EpiMxAlpha{}, st);
                k_mx_update<true><<<G, kBlock, 0, st>>>(n, S, A32.diag, h->d32, h->r32,
                                                        h->p32, h->q32, h->partials, h->dev);
                launch_finalize<2>(h->partials, G, h->dev, EpiMxInner{1}, st);
                k_mx_p<<<G, kBlock, 0, st>>>(n, S, A32.diag, h->r32, h->p32, h->dev);
            }
            HIP_CHECK(hipGetLastError());
            read_scalars(h, st);
            if (hs.inner_done) break;
        }
        inner_total += hs.inner_iters;
        k_mx_refine<<<G, kBlock, 0, st>>>(n, S, h->d32, x, h->dev);
        launch_residual<false, true>(h, A, b, x, h->r, nullptr, 0, kResCycle, true, st);
        read_scalars(h, st);
    }
    int status = LDU_OK;
    if (hs.done == kFailed) status = hs.status;
    else if (hs.done == kMaxIter) status = LDU_NOT_CONVERGED;
    if (stats) {
        stats->iterations = (int)inner_total;
        stats->refinements = hs.iters;
        stats->final_residual = hs.res;
        stats->converged = (status == LDU_OK);
    }
    copy_history(h, stats, hs.iters + 1, st);
    return status;
}

// ---------------------------------------------------------------- adjoint gradients
__global__ void k_coeff_grad(int32_t n, int64_t nf, const int32_t *__restrict__ own,
                             const int32_t *__restrict__ nb, const double *__restrict__ lam,
                             const double *__restrict__ x, double *gd, double *gu, double *gl) {
    const int64_t m = nf > n ? nf : n;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < m;
         k += (int64_t)gridDim.x * blockDim.x) {
        if (gd && k < n) gd[k] = -(lam[k] * x[k]);
        if (k < nf) {
            const int32_t o = own[k], b = nb[k];
            if (gu) gu[k] = -(lam[o] * x[b]);
            if (gl) gl[k] = -(lam[b] * x[o]);
        }
    }
}

void launch_coeff_grad(const Level &L, const double *lam, const double *x, double *gd,
                       double *gu, double *gl, hipStream_t st) {
    const int64_t m = L.nf > L.n ? L.nf : L.n;
    int64_t g = (m + kBlock - 1) / kBlock;
    g = g > 8192 ? 8192 : (g < 1 ? 1 : g);
    k_coeff_grad<<<(unsigned)g, kBlock, 0, st>>>(L.n, L.nf, L.own, L.nb, lam, x, gd, gu, gl);
    HIP_CHECK(hipGetLastError());
}

}  // namespace ldu
