// Diagonal-preconditioned CG that allocates no device memory: for callers
// that cannot allocate (work under HIP graph capture, tight serving loops,
// harnesses that forbid hipMalloc).
//
// Its per-call workspace (the CG vectors r, p, q, the per-block reduction
// partials and the residual history) lives in one file-scope device array of
// fixed size, `scratch`.  Each GPU the library runs on holds its own copy
// until the process ends.  In host code the array's name is only a host-side
// stand-in, so its device address is looked up once per device, with that
// device current, when the first handle on it is created (noalloc_init), and
// only that address is passed to kernels.
//
// Every call on a GPU shares that GPU's array: calls that overlap on one GPU
// (two streams, two threads) race and give wrong results.  Nothing in the
// array has to start at zero: each solve writes r and p (the residual
// kernel), q (the product) and every partial and history entry before it
// reads them, so the contents a previous call left behind are never read.
#include <hip/hip_runtime.h>

#include <mutex>

#include "internal.hpp"

namespace ldu {

namespace {

// r, p, q for up to kNoAllocMaxCells cells, the partials of 4 sums over
// kMaxGrid blocks, and kNoAllocHistory residual-history entries: 24.1 MiB
constexpr size_t kScratchDoubles =
    3 * (size_t)kNoAllocMaxCells + 4 * (size_t)kMaxGrid + (size_t)kNoAllocHistory;
constexpr int kMaxDevices = 64;

__device__ __align__(256) double scratch[kScratchDoubles];

std::mutex g_mu;
double *g_scratch_dev[kMaxDevices] = {};

// the device address of `scratch` on the current device (set by noalloc_init)
double *scratch_address(int device) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (device < 0 || device >= kMaxDevices || !g_scratch_dev[device])
        throw Error(LDU_ERR_STATE, "no scratch address for this device (no handle created on it)");
    return g_scratch_dev[device];
}

// points the handle's CG buffers at the scratch array for one call and puts
// its own buffers back afterwards (also when the solve throws)
struct ScratchBinding {
    ldu_t *h;
    double *r, *p, *q, *partials, *hist;
    int hist_cap;
    ScratchBinding(ldu_t *hh, double *base, int64_t n)
        : h(hh), r(hh->r), p(hh->p), q(hh->q), partials(hh->partials), hist(hh->hist),
          hist_cap(hh->hist_cap) {
        (void)n;
        h->r = base;
        h->p = base + kNoAllocMaxCells;
        h->q = base + 2 * kNoAllocMaxCells;
        h->partials = base + 3 * kNoAllocMaxCells;
        h->hist = h->partials + 4 * (size_t)kMaxGrid;
        h->hist_cap = kNoAllocHistory;
    }
    ~ScratchBinding() {
        h->r = r;
        h->p = p;
        h->q = q;
        h->partials = partials;
        h->hist = hist;
        h->hist_cap = hist_cap;
    }
};

}  // namespace

void noalloc_init(int device) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (device < 0 || device >= kMaxDevices)
        throw Error(LDU_ERR_LIMIT, "device index above the library's limit of 64");
    if (g_scratch_dev[device]) return;
    void *ptr = nullptr;
    HIP_CHECK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr || (reinterpret_cast<uintptr_t>(ptr) & 255) != 0)
        throw Error(LDU_ERR_HIP, "scratch array has no 256-byte aligned device address");
    g_scratch_dev[device] = static_cast<double *>(ptr);
}

int pcg_fp64_noalloc(ldu_t *h, const double *b, double *x, const ldu_pcg_opts &o,
                     ldu_stats *stats, hipStream_t st) {
    if ((int64_t)h->L0.n > kNoAllocMaxCells)
        throw Error(LDU_ERR_LIMIT, "pcg_solve_noalloc: nCells above its limit of 1048576");
    double *base = scratch_address(h->device);
    ScratchBinding bind(h, base, h->L0.n);
    return pcg_fp64(h, b, x, o, false, stats, st, /*own_hist=*/false);
}

}  // namespace ldu
