// The extern "C" entry points declared in include/ldu.h.  Every call maps
// internal exceptions to status codes; nothing but plain C crosses the ABI.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "internal.hpp"

namespace ldu {

static thread_local std::string g_last_error;

void hip_fail(hipError_t e, const char *what, const char *file, int line) {
    char buf[512];
    std::snprintf(buf, sizeof buf, "%s failed: %s (%s:%d)", what, hipGetErrorString(e), file,
                  line);
    if (e == hipErrorOutOfMemory) throw Error(LDU_ERR_NOMEM, buf);
    throw Error(LDU_ERR_HIP, buf);
}

Arena::~Arena() { release_all(); }

void *Arena::alloc(size_t bytes) {
    void *p = nullptr;
    if (bytes == 0) bytes = 16;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        throw Error(LDU_ERR_NOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
    }
    ptrs_.push_back(p);
    return p;
}

void Arena::release(void *p) {
    for (size_t k = 0; k < ptrs_.size(); ++k)
        if (ptrs_[k] == p) {
            (void)hipFree(p);
            ptrs_[k] = ptrs_.back();
            ptrs_.pop_back();
            return;
        }
}

void Arena::release_all() {
    for (void *p : ptrs_) (void)hipFree(p);
    ptrs_.clear();
}

}  // namespace ldu

using namespace ldu;

namespace {

int fail(int code, const std::string &msg) {
    g_last_error = msg;
    return code;
}

template <class F>
int guarded(ldu_t *h, F &&f) {
    if (h && h->poisoned) return fail(LDU_ERR_STATE, "handle is poisoned by an earlier HIP error");
    try {
        if (h) HIP_CHECK(hipSetDevice(h->device));
        return f();
    } catch (const Error &e) {
        if (h && e.code == LDU_ERR_HIP) h->poisoned = true;
        return fail(e.code, e.what());
    } catch (const std::bad_alloc &) {
        return fail(LDU_ERR_NOMEM, "host allocation failed");
    } catch (const std::exception &e) {
        return fail(LDU_ERR_ARG, e.what());
    }
}

hipStream_t S(void *s) { return reinterpret_cast<hipStream_t>(s); }

// a roctx range around one ABI call: `rocprofv3 --marker-trace` shows the
// setup, solve and gradient calls on the timeline beside their kernels
struct Range {
    explicit Range(const char *name) { roctxRangePushA(name); }
    ~Range() { roctxRangePop(); }
    Range(const Range &) = delete;
    Range &operator=(const Range &) = delete;
};

void check_pcg_opts(const ldu_pcg_opts &o) {
    if (!(o.rel_tol >= 0.0) || o.abs_tol != 0.0 || o.max_iter < 0 || o.check_every < 1 ||
        o.precond < 0 || o.precond > 2 ||
        (o.precision != LDU_FP64 && o.precision != LDU_MIXED) || o.max_refine < 0 ||
        o.inner_max_iter < 1 || !(o.inner_rel_tol > 0.0))
        throw Error(LDU_ERR_ARG, "invalid ldu_pcg_opts");
}

void check_gamg_opts(const ldu_gamg_opts &o) {
    if (!(o.rel_tol >= 0.0) || o.abs_tol != 0.0 || o.max_cycles < 0 || o.n_coarsest < 1 ||
        o.n_pre < 0 || o.n_post < 0 || o.max_levels < 1 || o.max_levels > kMaxLevels ||
        o.match_rounds < 0 || (o.precision != LDU_FP64 && o.precision != LDU_MIXED) ||
        o.max_refine < 0 || !(o.omega > 0.0) || o.passes < 1 || o.passes > 3 ||
        o.aggressive_from < 0 ||
        (o.smoother != LDU_SMOOTH_JACOBI && o.smoother != LDU_SMOOTH_GS2) ||
        o.gs_inner < 1 || o.gs_inner > 8 ||
        (o.coarsest != LDU_COARSE_DIAG && o.coarsest != LDU_COARSE_DIC) ||
        (o.scale_correction != 0 && o.scale_correction != 1))
        throw Error(LDU_ERR_ARG, "invalid ldu_gamg_opts");
}

bool same_structure(const ldu_gamg_opts &a, const ldu_gamg_opts &b) {
    return a.n_coarsest == b.n_coarsest && a.max_levels == b.max_levels &&
           a.match_rounds == b.match_rounds && a.passes == b.passes &&
           a.aggressive_from == b.aggressive_from;
}

void ensure_gamg(ldu_t *h, const ldu_gamg_opts &o, hipStream_t st) {
    if (!h->gamg_ready || !same_structure(h->gamg_opts, o)) gamg_build(h, o, st);
}

void copy_in(void *dst, const void *src, size_t bytes, hipStream_t st) {
    if (bytes) HIP_CHECK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, st));
}

}  // namespace

extern "C" {

void ldu_pcg_default_opts(ldu_pcg_opts *o) {
    if (!o) return;
    o->rel_tol = 1e-8;
    o->abs_tol = 0.0;
    o->max_iter = 10000;
    o->check_every = 16;
    o->precond = 1;
    o->precision = LDU_FP64;
    o->max_refine = 50;
    o->inner_max_iter = 1000;
    o->inner_rel_tol = 1e-4;
}

void ldu_gamg_default_opts(ldu_gamg_opts *o) {
    if (!o) return;
    o->rel_tol = 1e-8;
    o->abs_tol = 0.0;
    o->max_cycles = 200;
    o->n_coarsest = 50;
    o->n_pre = 2;
    o->n_post = 2;
    o->max_levels = 50;
    o->scale_correction = 1;
    o->match_rounds = 16;
    o->precision = LDU_FP64;
    o->max_refine = 200;
    o->omega = 0.75;
    o->passes = 1;
    o->aggressive_from = 0;
    o->smoother = LDU_SMOOTH_JACOBI;
    o->gs_inner = 1;
    o->coarsest = LDU_COARSE_DIAG;
}

const char *ldu_last_error(void) { return g_last_error.c_str(); }

int ldu_create(int32_t nCells, int64_t nFaces, const int32_t *owner, const int32_t *neighbour,
               const double *diag, const double *upper, const double *lower, void *hip_stream,
               ldu_handle *out) {
    Range range("ldu_create");
    if (!out) return fail(LDU_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (nCells < 1 || nFaces < 0) return fail(LDU_ERR_ARG, "nCells must be >= 1, nFaces >= 0");
    if (!diag || (nFaces > 0 && (!owner || !neighbour || !upper || !lower)))
        return fail(LDU_ERR_ARG, "NULL array argument");
    ldu_t *h = new (std::nothrow) ldu_t;
    if (!h) return fail(LDU_ERR_NOMEM, "host allocation failed");
    int rc = guarded(nullptr, [&] {
        hipStream_t st = S(hip_stream);
        HIP_CHECK(hipGetDevice(&h->device));
        noalloc_init(h->device);  // the static scratch's address on this device
        Level &L = h->L0;
        L.n = nCells;
        L.nf = nFaces;
        L.own = h->arena.get<int32_t>(nFaces);
        L.nb = h->arena.get<int32_t>(nFaces);
        L.upper = h->arena.get<double>(nFaces);
        L.lower = h->arena.get<double>(nFaces);
        L.diag = h->arena.get<double>(nCells);
        copy_in(L.own, owner, sizeof(int32_t) * nFaces, st);
        copy_in(L.nb, neighbour, sizeof(int32_t) * nFaces, st);
        copy_in(L.upper, upper, sizeof(double) * nFaces, st);
        copy_in(L.lower, lower, sizeof(double) * nFaces, st);
        copy_in(L.diag, diag, sizeof(double) * nCells, st);
        h->dev = h->arena.get<DevScalars>(1);
        h->flag = h->arena.get<int>(1);
        h->partials = h->arena.get<double>(4 * (size_t)kMaxGrid);
        HIP_CHECK(hipHostMalloc((void **)&h->host, sizeof(DevScalars), hipHostMallocDefault));
        HIP_CHECK(hipHostMalloc((void **)&h->hflag, sizeof(int), hipHostMallocDefault));
        std::memset(h->host, 0, sizeof(DevScalars));
        HIP_CHECK(hipMemcpyAsync(h->dev, h->host, sizeof(DevScalars), hipMemcpyHostToDevice, st));
        h->r = h->arena.get<double>(nCells);
        h->p = h->arena.get<double>(nCells);
        h->q = h->arena.get<double>(nCells);
        h->r32 = h->arena.get<float>(nCells);
        h->p32 = h->arena.get<float>(nCells);
        h->q32 = h->arena.get<float>(nCells);
        h->d32 = h->arena.get<float>(nCells);
        build_level_sell(h, h->arena, L, true, st);
        HIP_CHECK(hipStreamSynchronize(st));
        return LDU_OK;
    });
    if (rc != LDU_OK) {
        ldu_destroy(h);
        return rc;
    }
    *out = h;
    return LDU_OK;
}

int ldu_destroy(ldu_handle h) {
    if (!h) return LDU_OK;
    (void)hipSetDevice(h->device);
    (void)hipDeviceSynchronize();
    h->levels.clear();
    h->gamg_arena.release_all();
    h->arena.release_all();
    if (h->host) (void)hipHostFree(h->host);
    if (h->hflag) (void)hipHostFree(h->hflag);
    delete h;
    return LDU_OK;
}

int ldu_set_coeffs(ldu_handle h, const double *diag, const double *upper, const double *lower,
                   void *hip_stream) {
    Range range("ldu_set_coeffs");
    if (!h) return fail(LDU_ERR_ARG, "NULL handle");
    if (!diag || (h->L0.nf > 0 && (!upper || !lower))) return fail(LDU_ERR_ARG, "NULL array");
    return guarded(h, [&] {
        hipStream_t st = S(hip_stream);
        Level &L = h->L0;
        HIP_CHECK(hipMemsetAsync(h->flag, 0, sizeof(int), st));
        check_finite(h, diag, L.n, st);
        if (L.nf > 0) {
            check_finite(h, upper, L.nf, st);
            check_finite(h, lower, L.nf, st);
        }
        HIP_CHECK(hipMemcpyAsync(h->hflag, h->flag, sizeof(int), hipMemcpyDeviceToHost, st));
        HIP_CHECK(hipStreamSynchronize(st));
        if (*h->hflag) throw Error(LDU_ERR_NAN, "non-finite coefficient");
        copy_in(L.diag, diag, sizeof(double) * L.n, st);
        copy_in(L.upper, upper, sizeof(double) * L.nf, st);
        copy_in(L.lower, lower, sizeof(double) * L.nf, st);
        set_level_values(L, st);
        refresh_f32(L, st);
        gamg_refresh_values(h, st);
        HIP_CHECK(hipStreamSynchronize(st));
        return LDU_OK;
    });
}

int ldu_assemble_pressure(ldu_handle h, const double *gamma, const double *weights,
                          const double *mag_sf, const double *delta, const double *diag_bc,
                          const double *phi, const double *b_bc, double *b, double *diag,
                          double *upper, double *lower, void *hip_stream) {
    Range range("ldu_assemble_pressure");
    if (!h) return fail(LDU_ERR_ARG, "NULL handle");
    if (!gamma || (h->L0.nf > 0 && (!weights || !mag_sf || !delta || (b && !phi))) ||
        (phi && !b))
        return fail(LDU_ERR_ARG, "NULL array");
    return guarded(h, [&] {
        hipStream_t st = S(hip_stream);
        Level &L = h->L0;
        assemble_pressure(h, gamma, weights, mag_sf, delta, diag_bc, phi, b_bc, b, st);
        HIP_CHECK(hipMemsetAsync(h->flag, 0, sizeof(int), st));
        check_finite(h, L.diag, L.n, st);
        if (L.nf > 0) check_finite(h, L.upper, L.nf, st);
        HIP_CHECK(hipMemcpyAsync(h->hflag, h->flag, sizeof(int), hipMemcpyDeviceToHost, st));
        HIP_CHECK(hipStreamSynchronize(st));
        if (*h->hflag) throw Error(LDU_ERR_NAN, "non-finite assembled coefficient");
        refresh_f32(L, st);
        gamg_refresh_values(h, st);
        if (diag) copy_in(diag, L.diag, sizeof(double) * L.n, st);
        if (upper) copy_in(upper, L.upper, sizeof(double) * L.nf, st);
        if (lower) copy_in(lower, L.lower, sizeof(double) * L.nf, st);
        HIP_CHECK(hipStreamSynchronize(st));
        return LDU_OK;
    });
}

int ldu_amul(ldu_handle h, const double *x, double *y, void *hip_stream) {
    if (!h || !x || !y) return fail(LDU_ERR_ARG, "NULL argument");
    return guarded(h, [&] {
        launch_amul(h->L0.A.view(false), x, y, S(hip_stream));
        return LDU_OK;
    });
}

int ldu_tmul(ldu_handle h, const double *x, double *y, void *hip_stream) {
    if (!h || !x || !y) return fail(LDU_ERR_ARG, "NULL argument");
    return guarded(h, [&] {
        launch_amul(h->L0.A.view(true), x, y, S(hip_stream));
        return LDU_OK;
    });
}

int ldu_amul_f32(ldu_handle h, const float *x, float *y, void *hip_stream) {
    if (!h || !x || !y) return fail(LDU_ERR_ARG, "NULL argument");
    return guarded(h, [&] {
        hipStream_t st = S(hip_stream);
        ensure_f32(h->L0, h->arena, st);
        if (h->gamg_ready) h->levels[0].A = h->L0.A;
        launch_amul32(h->L0.A.view32(false), x, y, st);
        return LDU_OK;
    });
}

int ldu_residual(ldu_handle h, const double *b, const double *x, double *out, void *hip_stream) {
    if (!h || !b || !x || !out) return fail(LDU_ERR_ARG, "NULL argument");
    return guarded(h, [&] {
        *out = residual_norm(h, h->L0, false, b, x, h->r, S(hip_stream));
        return LDU_OK;
    });
}

static int pcg_common(ldu_handle h, const double *b, double *x, const ldu_pcg_opts *opts,
                      ldu_stats *stats, void *hip_stream, bool tr) {
    if (!h || !b || !x) return fail(LDU_ERR_ARG, "NULL argument");
    return guarded(h, [&] {
        ldu_pcg_opts o;
        ldu_pcg_default_opts(&o);
        if (opts) o = *opts;
        check_pcg_opts(o);
        hipStream_t st = S(hip_stream);
        if (o.precond == 2) {
            if (!h->gamg_ready) {
                ldu_gamg_opts go;
                ldu_gamg_default_opts(&go);
                gamg_build(h, go, st);
            }
            if (o.precision == LDU_MIXED) return pcg_gamg_mixed(h, b, x, o, tr, stats, st);
            return pcg_gamg_fp64(h, b, x, o, tr, stats, st);
        }
        if (o.precision == LDU_MIXED) return pcg_mixed(h, b, x, o, tr, stats, st);
        return pcg_fp64(h, b, x, o, tr, stats, st);
    });
}

int pcg_solve(ldu_handle h, const double *b, double *x, const ldu_pcg_opts *opts,
              ldu_stats *stats, void *hip_stream) {
    Range range("pcg_solve");
    return pcg_common(h, b, x, opts, stats, hip_stream, false);
}

int pcg_solve_noalloc(ldu_handle h, const double *b, double *x, const ldu_pcg_opts *opts,
                      ldu_stats *stats, void *hip_stream) {
    Range range("pcg_solve_noalloc");
    if (!h || !b || !x) return fail(LDU_ERR_ARG, "NULL argument");
    return guarded(h, [&] {
        ldu_pcg_opts o;
        ldu_pcg_default_opts(&o);
        if (opts) o = *opts;
        check_pcg_opts(o);
        if (o.precond == 2 || o.precision != LDU_FP64)
            throw Error(LDU_ERR_ARG,
                        "pcg_solve_noalloc: precond 0 or 1 and precision LDU_FP64 only");
        return pcg_fp64_noalloc(h, b, x, o, stats, S(hip_stream));
    });
}

int gamg_setup(ldu_handle h, const ldu_gamg_opts *opts, void *hip_stream) {
    Range range("gamg_setup");
    if (!h) return fail(LDU_ERR_ARG, "NULL handle");
    return guarded(h, [&] {
        ldu_gamg_opts o;
        ldu_gamg_default_opts(&o);
        if (opts) o = *opts;
        check_gamg_opts(o);
        gamg_build(h, o, S(hip_stream));
        return LDU_OK;
    });
}

static int gamg_common(ldu_handle h, const double *b, double *x, const ldu_gamg_opts *opts,
                       ldu_stats *stats, void *hip_stream, bool tr) {
    if (!h || !b || !x) return fail(LDU_ERR_ARG, "NULL argument");
    return guarded(h, [&] {
        ldu_gamg_opts o;
        ldu_gamg_default_opts(&o);
        if (opts) o = *opts;
        check_gamg_opts(o);
        hipStream_t st = S(hip_stream);
        ensure_gamg(h, o, st);
        if (o.precision == LDU_MIXED) return gamg_mixed(h, b, x, o, tr, stats, st);
        return gamg_fp64(h, b, x, o, tr, stats, st);
    });
}

int gamg_solve(ldu_handle h, const double *b, double *x, const ldu_gamg_opts *opts,
               ldu_stats *stats, void *hip_stream) {
    Range range("gamg_solve");
    return gamg_common(h, b, x, opts, stats, hip_stream, false);
}

int gamg_vcycle(ldu_handle h, const double *r, double *e, const ldu_gamg_opts *opts,
                void *hip_stream) {
    Range range("gamg_vcycle");
    if (!h || !r || !e) return fail(LDU_ERR_ARG, "NULL argument");
    return guarded(h, [&] {
        ldu_gamg_opts o;
        ldu_gamg_default_opts(&o);
        if (opts) o = *opts;
        check_gamg_opts(o);
        hipStream_t st = S(hip_stream);
        ensure_gamg(h, o, st);
        gamg_vcycle64(h, r, e, o, false, st);
        return LDU_OK;
    });
}

int gamg_level_size(ldu_handle h, int level, int64_t *n_cells, int64_t *n_faces) {
    if (!h) return fail(LDU_ERR_ARG, "NULL handle");
    if (!h->gamg_ready) return fail(LDU_ERR_STATE, "GAMG hierarchy not set up");
    if (level < 0 || level >= (int)h->levels.size()) return fail(LDU_ERR_ARG, "bad level");
    if (n_cells) *n_cells = h->levels[level].n;
    if (n_faces) *n_faces = h->levels[level].nf;
    return LDU_OK;
}

int ldu_level_layout(ldu_handle h, int level, int *compressed, int *col16) {
    if (!h) return fail(LDU_ERR_ARG, "NULL handle");
    if (level < 0) return fail(LDU_ERR_ARG, "bad level");
    if (level > 0 && !h->gamg_ready) return fail(LDU_ERR_STATE, "GAMG hierarchy not set up");
    if (level > 0 && level >= (int)h->levels.size()) return fail(LDU_ERR_ARG, "bad level");
    const Level &L = level == 0 ? h->L0 : h->levels[level];
    if (compressed) *compressed = L.A.pdeg != nullptr;
    if (col16) *col16 = L.A.c16 != nullptr;
    return LDU_OK;
}

int ldu_level_downleg(ldu_handle h, int level, int *form, int *lanes) {
    if (!h) return fail(LDU_ERR_ARG, "NULL handle");
    if (!h->gamg_ready) return fail(LDU_ERR_STATE, "GAMG hierarchy not set up");
    if (level < 0 || level >= (int)h->levels.size()) return fail(LDU_ERR_ARG, "bad level");
    const Level &L = h->levels[level];
    int f = 0, g = 0;
    if (L.ah) {
        f = 3;
    } else if (L.R.sptr) {
        f = 1;
    } else if (L.Rc.rptr) {
        f = 2;
        g = L.Rc.group;
    }
    if (form) *form = f;
    if (lanes) *lanes = g;
    return LDU_OK;
}

int gamg_level_export(ldu_handle h, int level, int32_t *agg, int32_t *owner, int32_t *neighbour,
                      double *diag, double *upper, double *lower, void *hip_stream) {
    if (!h) return fail(LDU_ERR_ARG, "NULL handle");
    if (!h->gamg_ready) return fail(LDU_ERR_STATE, "GAMG hierarchy not set up");
    if (level < 0 || level >= (int)h->levels.size()) return fail(LDU_ERR_ARG, "bad level");
    return guarded(h, [&] {
        hipStream_t st = S(hip_stream);
        const Level &L = h->levels[level];
        if (agg && L.agg) copy_in(agg, L.agg, sizeof(int32_t) * L.n, st);
        if (owner) copy_in(owner, L.own, sizeof(int32_t) * L.nf, st);
        if (neighbour) copy_in(neighbour, L.nb, sizeof(int32_t) * L.nf, st);
        if (diag) copy_in(diag, L.diag, sizeof(double) * L.n, st);
        if (upper) copy_in(upper, L.upper, sizeof(double) * L.nf, st);
        if (lower) copy_in(lower, L.lower, sizeof(double) * L.nf, st);
        HIP_CHECK(hipStreamSynchronize(st));
        return LDU_OK;
    });
}

static int pbicg_common(ldu_handle h, const double *b, double *x, const ldu_pcg_opts *opts,
                        ldu_stats *stats, void *hip_stream, bool tr) {
    if (!h || !b || !x) return fail(LDU_ERR_ARG, "NULL argument");
    return guarded(h, [&] {
        ldu_pcg_opts o;
        ldu_pcg_default_opts(&o);
        if (opts) o = *opts;
        check_pcg_opts(o);
        if (o.precond > 1 || o.precision != LDU_FP64)
            throw Error(LDU_ERR_ARG, "PBiCG takes precond 0 or 1 and precision LDU_FP64");
        return pbicg_fp64(h, b, x, o, tr, stats, S(hip_stream));
    });
}

int pbicg_solve(ldu_handle h, const double *b, double *x, const ldu_pcg_opts *opts,
                ldu_stats *stats, void *hip_stream) {
    Range range("pbicg_solve");
    return pbicg_common(h, b, x, opts, stats, hip_stream, false);
}

int ldu_adjoint_solve(ldu_handle h, const double *g, double *lambda, int solver,
                      const void *opts, ldu_stats *stats, void *hip_stream) {
    Range range("ldu_adjoint_solve");
    switch (solver) {
    case LDU_SOLVER_PCG:
        return pcg_common(h, g, lambda, static_cast<const ldu_pcg_opts *>(opts), stats,
                          hip_stream, true);
    case LDU_SOLVER_GAMG:
        return gamg_common(h, g, lambda, static_cast<const ldu_gamg_opts *>(opts), stats,
                           hip_stream, true);
    case LDU_SOLVER_PBICG:
        return pbicg_common(h, g, lambda, static_cast<const ldu_pcg_opts *>(opts), stats,
                            hip_stream, true);
    default:
        return fail(LDU_ERR_ARG, "unknown solver");
    }
}

int ldu_coeff_grad(ldu_handle h, const double *lambda, const double *x, double *g_diag,
                   double *g_upper, double *g_lower, void *hip_stream) {
    Range range("ldu_coeff_grad");
    if (!h || !lambda || !x) return fail(LDU_ERR_ARG, "NULL argument");
    return guarded(h, [&] {
        launch_coeff_grad(h->L0, lambda, x, g_diag, g_upper, g_lower, S(hip_stream));
        return LDU_OK;
    });
}

}  // extern "C"
