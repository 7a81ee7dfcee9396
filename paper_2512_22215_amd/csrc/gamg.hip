// GAMG: pairwise agglomeration, Galerkin coarse matrices and the V-cycle.
//
// The paper runs OpenFOAM's GAMG for the pressure equation with the
// Richardson (damped Jacobi) smoother on every level and a diagonal-PCG
// coarsest solve, its fastest combination (Sec. 4.3, smoother table;
// Appendix A), and profiles agglomerateMatrix, restrictField, prolongField,
// scale and Vcycle (Sec. 4.3, kernel time breakdown).  It keeps OpenFOAM's
// serial CPU coarsening.  Here the coarsening is a parallel handshake
// matching with a strict total order on faces:
//   weight w_f = ((|upper_f| + |lower_f|) / 2)^2 / |diag_i diag_j| (the
//   squared coupling relative to the diagonals, which stays level under
//   geometric mesh grading), ties broken by a SplitMix64 hash of the face's
//   (min, max) cell pair, then by the smaller cell index;
//   each round, every unmatched cell picks its best unmatched neighbour and
//   mutual picks pair up; rounds stop when one adds no pair or after
//   match_rounds; an unmatched cell then joins the aggregate of its best
//   matched neighbour (no cascading) or stays a singleton; aggregates are
//   numbered by their seed cell (pair minimum or singleton).
// The result depends only on the matrix, not on the order in which threads
// run, and equals the greedy matching in that face order.
//
// Galerkin coarse matrices A_c = P^T A P (piecewise-constant P) are formed in
// LDU form with coarse faces sorted by (a, b); each coarse value is summed
// over its fine faces in ascending face order, and each coarse diagonal over
// member cells in ascending order and then over the aggregate's internal
// faces in ascending order.  Summation order is fixed, so the hierarchy is
// bitwise reproducible.
#include "device.hpp"

#include <algorithm>
#include <cmath>

namespace ldu {

__device__ __forceinline__ uint64_t splitmix64_out(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
__device__ __forceinline__ uint64_t tie_key(int32_t i, int32_t j) {
    const uint64_t lo = (uint32_t)(i < j ? i : j), hi = (uint32_t)(i < j ? j : i);
    return splitmix64_out((lo << 32) | hi);
}
// squared diagonally scaled coupling strength (no square root: it rounds the
// same way on every device)
__device__ __forceinline__ double strength2(double a, double at, double di, double dj) {
    const double s = 0.5 * (fabs(a) + fabs(at));
    const double den = fabs(di) * fabs(dj);
    return den > 0.0 ? (s * s) / den : s * s;
}
__device__ __forceinline__ bool better(double w1, uint64_t h1, int32_t j1, double w2,
                                       uint64_t h2, int32_t j2) {
    if (w1 != w2) return w1 > w2;
    if (h1 != h2) return h1 > h2;
    return j1 < j2;
}

static unsigned grid_n(int64_t n) {
    int64_t g = (n + kBlock - 1) / kBlock;
    g = g > 8192 ? 8192 : (g < 1 ? 1 : g);
    return (unsigned)g;
}
#define GRID_STRIDE(i, n)                                                         \
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < (n); \
         i += (int64_t)gridDim.x * blockDim.x)

// best neighbour of row i among those whose matched state equals want_matched
__device__ int32_t best_neighbour(const Sell &A, int32_t i, const int32_t *partner,
                                  bool want_matched) {
    const int64_t ps = A.iperm ? (int64_t)A.iperm[i] : (int64_t)i;
    const int w = row_len(A, ps);
    int32_t best = -1;
    double bw = 0.0;
    uint64_t bh = 0;
    for (int k = 0; k < w; ++k) {
        const int64_t pos = entry_at(A, ps, k);
        const int32_t c = A.col[pos];
        if (c == i) continue;  // padding
        if ((partner[c] >= 0) != want_matched) continue;
        const double wt = strength2(A.val[pos], A.valT[pos], A.diag[i], A.diag[c]);
        const uint64_t hk = tie_key(i, c);
        if (best < 0 || better(wt, hk, c, bw, bh, best)) {
            best = c;
            bw = wt;
            bh = hk;
        }
    }
    return best;
}

// flags[0] = pair added this round, flags[1] = matching finished
__global__ void k_match_init(int32_t n, int32_t *partner, int *flags) {
    GRID_STRIDE(i, n) partner[i] = -1;
    if (blockIdx.x == 0 && threadIdx.x == 0) { flags[0] = 0; flags[1] = 0; }
}
__global__ void k_match_pick(Sell A, const int32_t *partner, int32_t *pick, const int *flags) {
    if (flags[1]) return;
    GRID_STRIDE(i, A.n) {
        pick[i] = partner[i] < 0 ? best_neighbour(A, (int32_t)i, partner, false) : -1;
    }
}
__global__ void k_match_pair(int32_t n, const int32_t *pick, int32_t *partner, int *flags) {
    if (flags[1]) return;
    GRID_STRIDE(i, n) {
        const int32_t j = pick[i];
        if (j >= 0 && pick[j] == (int32_t)i) {
            partner[i] = j;
            flags[0] = 1;
        }
    }
}
__global__ void k_match_round_end(int *flags) {
    if (!flags[1] && !flags[0]) flags[1] = 1;
    flags[0] = 0;
}
__global__ void k_match_leftover(Sell A, const int32_t *partner, int32_t *join, int32_t *seed) {
    GRID_STRIDE(i, A.n) {
        const int32_t p = partner[i];
        const int32_t jn = p < 0 ? best_neighbour(A, (int32_t)i, partner, true) : -1;
        join[i] = jn;
        seed[i] = ((p >= 0 && (int32_t)i < p) || (p < 0 && jn < 0)) ? 1 : 0;
    }
}
__global__ void k_match_assign(int32_t n, const int32_t *partner, const int32_t *join,
                               const int32_t *rank, int32_t *agg) {
    GRID_STRIDE(i, n) {
        const int32_t p = partner[i];
        int32_t a;
        if (p >= 0) {
            a = rank[(int32_t)i < p ? (int32_t)i : p];
        } else if (join[i] < 0) {
            a = rank[i];
        } else {
            const int32_t j = join[i], pj = partner[j];
            a = rank[j < pj ? j : pj];
        }
        agg[i] = a;
    }
}

// aggregate member lists, ascending cell order
__global__ void k_agg_count(int32_t n, const int32_t *agg, int32_t *cnt) {
    GRID_STRIDE(i, n) atomicAdd(&cnt[agg[i]], 1);
}
__global__ void k_agg_fill(int32_t n, const int32_t *agg, const int32_t *start, int32_t *cursor,
                           int32_t *cells) {
    GRID_STRIDE(i, n) {
        const int32_t a = agg[i];
        cells[start[a] + atomicAdd(&cursor[a], 1)] = (int32_t)i;
    }
}
__global__ void k_agg_sort(int32_t nc, const int32_t *start, int32_t *cells) {
    GRID_STRIDE(a, nc) {
        const int32_t lo = start[a], hi = start[a + 1];
        for (int32_t k = lo + 1; k < hi; ++k) {
            const int32_t v = cells[k];
            int32_t m = k - 1;
            while (m >= lo && cells[m] > v) { cells[m + 1] = cells[m]; --m; }
            cells[m + 1] = v;
        }
    }
}

// coarse row a: the sorted distinct aggregates b > a adjacent to a
__device__ int coarse_row(const Sell &A, const int32_t *agg, const int32_t *start,
                          const int32_t *cells, int32_t a, int32_t *list, int *overflow) {
    int m = 0;
    for (int32_t k = start[a]; k < start[a + 1]; ++k) {
        const int32_t i = cells[k];
        const int64_t ps = A.iperm ? (int64_t)A.iperm[i] : (int64_t)i;
        const int w = row_len(A, ps);
        for (int e = 0; e < w; ++e) {
            const int32_t c = A.col[entry_at(A, ps, e)];
            if (c == i) continue;
            const int32_t b = agg[c];
            if (b <= a) continue;
            int pos = m;  // insertion into the sorted unique list
            while (pos > 0 && list[pos - 1] > b) --pos;
            if (pos > 0 && list[pos - 1] == b) continue;
            if (m >= kMaxCoarseRow) { *overflow = 1; return m; }
            for (int q = m; q > pos; --q) list[q] = list[q - 1];
            list[pos] = b;
            ++m;
        }
    }
    return m;
}
__global__ void k_coarse_count(Sell A, int32_t nc, const int32_t *agg, const int32_t *start,
                               const int32_t *cells, int32_t *cnt, int *overflow) {
    int32_t list[kMaxCoarseRow];
    GRID_STRIDE(a, nc) cnt[a] = coarse_row(A, agg, start, cells, (int32_t)a, list, overflow);
}
__global__ void k_coarse_fill(Sell A, int32_t nc, const int32_t *agg, const int32_t *start,
                              const int32_t *cells, const int32_t *cptr, int32_t *cown,
                              int32_t *cnb, int *overflow) {
    int32_t list[kMaxCoarseRow];
    GRID_STRIDE(a, nc) {
        const int m = coarse_row(A, agg, start, cells, (int32_t)a, list, overflow);
        for (int k = 0; k < m; ++k) {
            cown[cptr[a] + k] = (int32_t)a;
            cnb[cptr[a] + k] = list[k];
        }
    }
}

// coarse face values: fine faces between aggregates a < b in ascending order
__global__ void k_coarse_values(int64_t ncf, const int32_t *cown, const int32_t *cnb,
                                const int32_t *agg, const int32_t *start, const int32_t *cells,
                                const int64_t *ownStart, const int32_t *fnb,
                                const double *fup, const double *flo, double *cup,
                                double *clo) {
    GRID_STRIDE(c, ncf) {
        const int32_t a = cown[c], b = cnb[c];
        int32_t ka = start[a], kb = start[b];
        const int32_t ea = start[a + 1], eb = start[b + 1];
        double up = 0.0, lo = 0.0;
        while (ka < ea || kb < eb) {  // merge the two member lists
            int32_t i;
            bool in_a;
            if (kb >= eb || (ka < ea && cells[ka] < cells[kb])) { i = cells[ka++]; in_a = true; }
            else { i = cells[kb++]; in_a = false; }
            const int32_t other = in_a ? b : a;
            for (int64_t f = ownStart[i]; f < ownStart[i + 1]; ++f) {
                if (agg[fnb[f]] != other) continue;
                if (in_a) { up += fup[f]; lo += flo[f]; }
                else { up += flo[f]; lo += fup[f]; }
            }
        }
        cup[c] = up;
        clo[c] = lo;
    }
}

// The same visits recorded once (count, then fill), so that new fine values
// only need a pass over the lists: each sum keeps its order and its bits.
// LIST = false counts, LIST = true writes at the counted offsets.
template <bool LIST>
__global__ void k_coarse_facelist(int64_t ncf, const int32_t *cown, const int32_t *cnb,
                                  const int32_t *agg, const int32_t *start,
                                  const int32_t *cells, const int64_t *ownStart,
                                  const int32_t *fnb, int64_t *count, const int64_t *offs,
                                  int32_t *list) {
    GRID_STRIDE(c, ncf) {
        const int32_t a = cown[c], b = cnb[c];
        int32_t ka = start[a], kb = start[b];
        const int32_t ea = start[a + 1], eb = start[b + 1];
        int64_t m = LIST ? offs[c] : 0;
        while (ka < ea || kb < eb) {
            int32_t i;
            bool in_a;
            if (kb >= eb || (ka < ea && cells[ka] < cells[kb])) { i = cells[ka++]; in_a = true; }
            else { i = cells[kb++]; in_a = false; }
            const int32_t other = in_a ? b : a;
            for (int64_t f = ownStart[i]; f < ownStart[i + 1]; ++f) {
                if (agg[fnb[f]] != other) continue;
                if (LIST) list[m] = in_a ? (int32_t)f : ~(int32_t)f;
                ++m;
            }
        }
        if (!LIST) count[c] = m;
    }
}
template <bool LIST>
__global__ void k_coarse_celllist(int32_t nc, const int32_t *agg, const int32_t *start,
                                  const int32_t *cells, const int64_t *ownStart,
                                  const int32_t *fnb, int64_t *count, const int64_t *offs,
                                  int32_t *list) {
    GRID_STRIDE(a, nc) {
        int64_t m = LIST ? offs[a] : 0;
        for (int32_t k = start[a]; k < start[a + 1]; ++k) {
            const int32_t i = cells[k];
            for (int64_t f = ownStart[i]; f < ownStart[i + 1]; ++f) {
                if (agg[fnb[f]] != (int32_t)a) continue;
                if (LIST) list[m] = (int32_t)f;
                ++m;
            }
        }
        if (!LIST) count[a] = m;
    }
}

// coarse values from the recorded lists (the sums of k_coarse_values and
// k_coarse_diag, term for term)
__global__ void k_coarse_values_list(int64_t ncf, const int64_t *__restrict__ cfs,
                                     const int32_t *__restrict__ cff,
                                     const double *__restrict__ fup,
                                     const double *__restrict__ flo, double *__restrict__ cup,
                                     double *__restrict__ clo) {
    GRID_STRIDE(c, ncf) {
        double up = 0.0, lo = 0.0;
        for (int64_t k = cfs[c]; k < cfs[c + 1]; ++k) {
            const int32_t g = cff[k];
            if (g >= 0) { up += fup[g]; lo += flo[g]; }
            else { up += flo[~g]; lo += fup[~g]; }
        }
        cup[c] = up;
        clo[c] = lo;
    }
}
__global__ void k_coarse_diag_list(int32_t nc, const int32_t *__restrict__ start,
                                   const int32_t *__restrict__ cells,
                                   const int64_t *__restrict__ cis,
                                   const int32_t *__restrict__ cif,
                                   const double *__restrict__ fdiag,
                                   const double *__restrict__ fup,
                                   const double *__restrict__ flo, double *__restrict__ cdiag) {
    GRID_STRIDE(a, nc) {
        double d = 0.0;
        for (int32_t k = start[a]; k < start[a + 1]; ++k) d += fdiag[cells[k]];
        for (int64_t k = cis[a]; k < cis[a + 1]; ++k) {
            const int32_t f = cif[k];
            d += (fup[f] + flo[f]);
        }
        cdiag[a] = d;
    }
}

__global__ void k_coarse_diag(int32_t nc, const int32_t *agg, const int32_t *start,
                              const int32_t *cells, const int64_t *ownStart, const int32_t *fnb,
                              const double *fdiag, const double *fup, const double *flo,
                              double *cdiag) {
    GRID_STRIDE(a, nc) {
        double d = 0.0;
        for (int32_t k = start[a]; k < start[a + 1]; ++k) d += fdiag[cells[k]];
        for (int32_t k = start[a]; k < start[a + 1]; ++k) {
            const int32_t i = cells[k];
            for (int64_t f = ownStart[i]; f < ownStart[i + 1]; ++f)
                if (agg[fnb[f]] == (int32_t)a) d += (fup[f] + flo[f]);
        }
        cdiag[a] = d;
    }
}

// singular level: |(A 1)_i| <= 1e-12 |diag_i| for every row
__global__ void k_singular(Sell A, int *flag) {
    GRID_STRIDE(i, A.n) {
        const int64_t ps = A.iperm ? (int64_t)A.iperm[i] : (int64_t)i;
        const int64_t s = ps >> 6, lane = ps & 63;
        const SellView<double> v = A.view(false);
        struct One { __device__ double operator()(int32_t) const { return 1.0; } };
        const double y = sell_row_any(v, s, (int)lane, (int32_t)i, One{});
        if (!(fabs(y) <= 1e-12 * fabs(A.diag[i]))) atomicAnd(flag, 0);
    }
}

// ---------------------------------------------------------------- setup
// FP32 copies of every level's values; level 0's live with the handle
static void ensure_f32_levels(ldu_t *h, hipStream_t st) {
    ensure_f32(h->L0, h->arena, st);
    h->levels[0].A = h->L0.A;
    for (size_t l = 1; l < h->levels.size(); ++l) ensure_f32(h->levels[l], h->gamg_arena, st);
}

static void alloc_work(Level &L, Arena &ar) {
    L.r = ar.get<double>(L.n);
    L.e = ar.get<double>(L.n);
    L.e2 = ar.get<double>(L.n);
    L.t = ar.get<double>(L.n);
}

static void coarse_values(ldu_t *h, Level &F, Level &C, hipStream_t st) {
    if (F.cfStart) {  // recorded visits (hierarchy levels)
        if (C.nf > 0)
            k_coarse_values_list<<<grid_n(C.nf), kBlock, 0, st>>>(C.nf, F.cfStart, F.cfFace,
                                                                   F.upper, F.lower, C.upper,
                                                                   C.lower);
        k_coarse_diag_list<<<grid_n(C.n), kBlock, 0, st>>>(C.n, F.aggStart, F.aggCells,
                                                           F.ciStart, F.ciFace, F.diag, F.upper,
                                                           F.lower, C.diag);
    } else {  // the aggressive passes' temporary matrices
        if (C.nf > 0)
            k_coarse_values<<<grid_n(C.nf), kBlock, 0, st>>>(C.nf, C.own, C.nb, F.agg,
                                                              F.aggStart, F.aggCells, F.ownStart,
                                                              F.nb, F.upper, F.lower, C.upper,
                                                              C.lower);
        k_coarse_diag<<<grid_n(C.n), kBlock, 0, st>>>(C.n, F.agg, F.aggStart, F.aggCells,
                                                      F.ownStart, F.nb, F.diag, F.upper, F.lower,
                                                      C.diag);
    }
    HIP_CHECK(hipGetLastError());
}

// record the fine faces each coarse value and diagonal sums (count, scan, fill)
static void coarse_lists(Level &F, const Level &C, Arena &ar, hipStream_t st) {
    Arena tmp;
    int64_t *cnt = tmp.get<int64_t>((size_t)C.nf + 1);
    F.cfStart = ar.get<int64_t>((size_t)C.nf + 1);
    if (C.nf > 0)
        k_coarse_facelist<false><<<grid_n(C.nf), kBlock, 0, st>>>(
            C.nf, C.own, C.nb, F.agg, F.aggStart, F.aggCells, F.ownStart, F.nb, cnt, nullptr,
            nullptr);
    exclusive_scan_i64(cnt, F.cfStart, C.nf, tmp, st);
    int64_t *cntc = tmp.get<int64_t>((size_t)C.n + 1);
    F.ciStart = ar.get<int64_t>((size_t)C.n + 1);
    k_coarse_celllist<false><<<grid_n(C.n), kBlock, 0, st>>>(
        C.n, F.agg, F.aggStart, F.aggCells, F.ownStart, F.nb, cntc, nullptr, nullptr);
    exclusive_scan_i64(cntc, F.ciStart, C.n, tmp, st);
    int64_t nff = 0, nif = 0;
    HIP_CHECK(hipMemcpyAsync(&nff, F.cfStart + C.nf, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipMemcpyAsync(&nif, F.ciStart + C.n, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipStreamSynchronize(st));
    F.cfFace = ar.get<int32_t>((size_t)nff + 1);
    F.ciFace = ar.get<int32_t>((size_t)nif + 1);
    if (C.nf > 0)
        k_coarse_facelist<true><<<grid_n(C.nf), kBlock, 0, st>>>(
            C.nf, C.own, C.nb, F.agg, F.aggStart, F.aggCells, F.ownStart, F.nb, nullptr,
            F.cfStart, F.cfFace);
    k_coarse_celllist<true><<<grid_n(C.n), kBlock, 0, st>>>(
        C.n, F.agg, F.aggStart, F.aggCells, F.ownStart, F.nb, nullptr, F.ciStart, F.ciFace);
    HIP_CHECK(hipGetLastError());
    HIP_CHECK(hipStreamSynchronize(st));
}

__global__ void k_set_int(int *p, int v) { *p = v; }

static void detect_singular(ldu_t *h, Level &L, hipStream_t st) {
    k_set_int<<<1, 1, 0, st>>>(h->flag, 1);
    k_singular<<<grid_n(L.n), kBlock, 0, st>>>(L.A, h->flag);
    HIP_CHECK(hipMemcpyAsync(h->hflag, h->flag, sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipStreamSynchronize(st));
    L.singular = (*h->hflag != 0) && L.n > 0;
}

// member lists of F's aggregation (F.agg, F.nc): aggStart and aggCells in
// ascending cell order
static void agg_lists(Level &F, Arena &ar, hipStream_t st) {
    Arena tmp;
    const int32_t n = F.n, nc = F.nc;
    const unsigned g = grid_n(n);
    int32_t *cnt = tmp.get<int32_t>(nc);
    int32_t *cursor = tmp.get<int32_t>(nc);
    HIP_CHECK(hipMemsetAsync(cnt, 0, sizeof(int32_t) * nc, st));
    HIP_CHECK(hipMemsetAsync(cursor, 0, sizeof(int32_t) * nc, st));
    k_agg_count<<<g, kBlock, 0, st>>>(n, F.agg, cnt);
    F.aggStart = ar.get<int32_t>((size_t)nc + 1);
    scan_counts_i32(cnt, F.aggStart, nc, tmp, st);
    F.aggCells = ar.get<int32_t>(n);
    k_agg_fill<<<g, kBlock, 0, st>>>(n, F.agg, F.aggStart, cursor, F.aggCells);
    k_agg_sort<<<grid_n(nc), kBlock, 0, st>>>(nc, F.aggStart, F.aggCells);
    HIP_CHECK(hipGetLastError());
    HIP_CHECK(hipStreamSynchronize(st));
}

// one pairwise matching pass over level F: F.agg (in ar) and F.nc; the member
// lists go to lists_ar
static int32_t agglomerate(ldu_t *h, Level &F, int match_rounds, Arena &ar, Arena &lists_ar,
                           hipStream_t st) {
    const int32_t n = F.n;
    Arena tmp;
    int32_t *partner = tmp.get<int32_t>(n);
    int32_t *pick = tmp.get<int32_t>(n);
    int32_t *join = tmp.get<int32_t>(n);
    int32_t *seed = tmp.get<int32_t>(n);
    int32_t *rank = tmp.get<int32_t>((size_t)n + 1);
    int *flags = tmp.get<int>(2);
    const unsigned g = grid_n(n);
    k_match_init<<<g, kBlock, 0, st>>>(n, partner, flags);
    for (int round = 0; round < match_rounds; ++round) {
        k_match_pick<<<g, kBlock, 0, st>>>(F.A, partner, pick, flags);
        k_match_pair<<<g, kBlock, 0, st>>>(n, pick, partner, flags);
        k_match_round_end<<<1, 1, 0, st>>>(flags);
    }
    k_match_leftover<<<g, kBlock, 0, st>>>(F.A, partner, join, seed);
    scan_counts_i32(seed, rank, n, tmp, st);
    int32_t nc = 0;
    HIP_CHECK(hipMemcpyAsync(&nc, rank + n, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipStreamSynchronize(st));
    F.nc = nc;
    F.agg = ar.get<int32_t>(n);
    k_match_assign<<<g, kBlock, 0, st>>>(n, partner, join, rank, F.agg);
    HIP_CHECK(hipGetLastError());
    agg_lists(F, lists_ar, st);
    return nc;
}

__global__ void k_compose(int32_t n, const int32_t *__restrict__ outer, int32_t *agg) {
    GRID_STRIDE(i, n) agg[i] = outer[agg[i]];
}

static void galerkin(ldu_t *h, Level &F, Level &C, Arena &ar, hipStream_t st);

// aggregation of level F by `passes` pairwise matching passes: pass k matches
// the aggregates of pass k-1 on their Galerkin matrix (a temporary, used only
// for its coupling strengths) and the aggregate maps compose.  One pass is
// plain pairwise agglomeration.
static int32_t agglomerate_passes(ldu_t *h, Level &F, int match_rounds, int passes, Arena &ar,
                                  hipStream_t st) {
    if (passes <= 1) return agglomerate(h, F, match_rounds, ar, ar, st);
    Arena tmp;
    const int32_t nc = agglomerate(h, F, match_rounds, ar, tmp, st);
    if (nc <= 1) {
        agg_lists(F, ar, st);
        return nc;
    }
    Level T;
    galerkin(h, F, T, tmp, st);
    build_level_sell(h, tmp, T, false, st);
    const int32_t nc2 = agglomerate_passes(h, T, match_rounds, passes - 1, tmp, st);
    k_compose<<<grid_n(F.n), kBlock, 0, st>>>(F.n, T.agg, F.agg);
    HIP_CHECK(hipGetLastError());
    F.nc = nc2;
    agg_lists(F, ar, st);
    return nc2;
}

static void galerkin(ldu_t *h, Level &F, Level &C, Arena &ar, hipStream_t st) {
    Arena tmp;
    const int32_t nc = F.nc;
    int32_t *cnt = tmp.get<int32_t>(nc);
    int32_t *cptr = tmp.get<int32_t>((size_t)nc + 1);
    int *overflow = tmp.get<int>(1);
    HIP_CHECK(hipMemsetAsync(overflow, 0, sizeof(int), st));
    k_coarse_count<<<grid_n(nc), kBlock, 0, st>>>(F.A, nc, F.agg, F.aggStart, F.aggCells, cnt,
                                                  overflow);
    scan_counts_i32(cnt, cptr, nc, tmp, st);
    int32_t ncf = 0;
    int ovf = 0;
    HIP_CHECK(hipMemcpyAsync(&ncf, cptr + nc, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipMemcpyAsync(&ovf, overflow, sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipStreamSynchronize(st));
    if (ovf) throw Error(LDU_ERR_LIMIT, "coarse level row exceeds the supported width");
    C.n = nc;
    C.nf = ncf;
    C.own = ar.get<int32_t>(ncf);
    C.nb = ar.get<int32_t>(ncf);
    C.upper = ar.get<double>(ncf);
    C.lower = ar.get<double>(ncf);
    C.diag = ar.get<double>(nc);
    k_coarse_fill<<<grid_n(nc), kBlock, 0, st>>>(F.A, nc, F.agg, F.aggStart, F.aggCells, cptr,
                                                 C.own, C.nb, overflow);
    HIP_CHECK(hipGetLastError());
    coarse_values(h, F, C, st);
    HIP_CHECK(hipStreamSynchronize(st));
}

static void ensure_rop(ldu_t *h, const ldu_gamg_opts &o, hipStream_t st);
static void refresh_rop(ldu_t *h, hipStream_t st);

void gamg_build(ldu_t *h, const ldu_gamg_opts &o, hipStream_t st) {
    h->gamg_ready = false;
    h->levels.clear();
    h->gamg_arena.release_all();
    Arena &ar = h->gamg_arena;
    h->levels.push_back(h->L0);
    h->levels[0].agg = h->levels[0].aggStart = h->levels[0].aggCells = nullptr;
    h->levels[0].cfStart = h->levels[0].ciStart = nullptr;
    h->levels[0].cfFace = h->levels[0].ciFace = nullptr;
    const int maxl = std::min(std::max(o.max_levels, 1), kMaxLevels);
    while ((int)h->levels.size() < maxl) {
        const size_t l = h->levels.size() - 1;
        if (h->levels[l].n <= o.n_coarsest) break;
        const int passes = (int)l >= o.aggressive_from ? o.passes : 1;
        const int32_t nc = agglomerate_passes(h, h->levels[l], o.match_rounds, passes, ar, st);
        if (100 * (int64_t)nc > 95 * (int64_t)h->levels[l].n) {
            h->levels[l].agg = nullptr;
            break;
        }
        Level C;
        galerkin(h, h->levels[l], C, ar, st);
        coarse_lists(h->levels[l], C, ar, st);  // for value refreshes on this structure
        build_level_sell(h, ar, C, false, st);
        h->levels.push_back(C);
    }
    if (h->levels.back().n > kMaxCoarsest && h->levels.back().nf > 0) {
        h->levels.clear();
        h->gamg_arena.release_all();
        throw Error(LDU_ERR_LIMIT, "coarsest GAMG level has more than 8192 cells; raise max_levels");
    }
    for (auto &L : h->levels) alloc_work(L, ar);
    h->coarse_work = ar.get<double>(5 * (size_t)h->levels.back().n);
    h->dic_dt = ar.get<double>(h->levels.back().n);
    h->dic_ready = false;

    if (h->L0.A.val32) ensure_f32_levels(h, st);
    detect_singular(h, h->levels.back(), st);
    h->gamg_opts = o;
    h->gamg_ready = true;
    // a Jacobi cycle with one pre-sweep will run its down leg through R (the
    // CG + V-cycle solve turns correction scaling off): build it with the
    // hierarchy
    if (o.smoother == LDU_SMOOTH_JACOBI && o.n_pre == 1) {
        ldu_gamg_opts q = o;
        q.scale_correction = 0;
        ensure_rop(h, q, st);
    }
}

// new level-0 values: recompute every coarse matrix on the cached structure
void gamg_refresh_values(ldu_t *h, hipStream_t st) {
    if (!h->gamg_ready) return;
    h->levels[0].A = h->L0.A;
    for (size_t l = 0; l + 1 < h->levels.size(); ++l) {
        Level &F = h->levels[l], &C = h->levels[l + 1];
        coarse_values(h, F, C, st);
        set_level_values(C, st);
        refresh_f32(C, st);
    }
    detect_singular(h, h->levels.back(), st);
    h->dic_ready = false;
    refresh_rop(h, st);
}

// DIC pivots of the coarsest level (diagonal incomplete Cholesky; the paper's
// other coarsest-level preconditioner, Sec. 4.3 smoother table):
//   Dt_i = A_ii - sum_{j<i} A_ij A_ji / Dt_j, ascending j,
// with A_ji read from the transposed values at the same position.  Serial in
// one thread: the level has a few dozen rows, and this runs once per set of
// coefficients.  ok = 0 when a pivot is not finite, changes sign against
// A_ii, or falls below 1e-12 |A_ii|; the solve then uses the diagonal.
__global__ void k_dic_factor(Sell A, double *dt, int *ok) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    int good = 1;
    for (int32_t i = 0; i < A.n; ++i) {
        const int64_t ps = A.iperm ? (int64_t)A.iperm[i] : (int64_t)i;
        const int w = row_len(A, ps);
        double d = A.diag[i];
        for (int k = 0; k < w; ++k) {
            const int64_t e = entry_at(A, ps, k);
            const int32_t c = A.col[e];
            if (c < i) d = d - (A.val[e] * A.valT[e]) / dt[c];
        }
        dt[i] = d;
        if (!isfinite(d) || !(fabs(d) > 1e-12 * fabs(A.diag[i])) || ((d > 0.0) != (A.diag[i] > 0.0)))
            good = 0;
    }
    *ok = good;
}

static void ensure_dic(ldu_t *h, hipStream_t st) {
    if (h->dic_ready) return;
    Level &L = h->levels.back();
    k_dic_factor<<<1, 1, 0, st>>>(L.A, h->dic_dt, h->flag);
    HIP_CHECK(hipGetLastError());
    HIP_CHECK(hipMemcpyAsync(h->hflag, h->flag, sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipStreamSynchronize(st));
    h->dic_ok = *h->hflag != 0;
    h->dic_ready = true;
}

// ---------------------------------------------------------------- V-cycle kernels
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_vc_first(int32_t n, int64_t S, const T *__restrict__ r, const T *__restrict__ D,
           T *__restrict__ e, T omega, const DevScalars *ds) {
    if (vc_skip(ds)) return;
    const int lane = threadIdx.x & 63;
    for_each_slice(S, [&](int64_t s) {
        const int64_t i = s * kWave + lane;
        if (i < n) e[i] = omega * r[i] / D[i];
    });
}

template <typename T>
__global__ void __launch_bounds__(kBlock)
k_vc_zero(int32_t n, int64_t S, T *__restrict__ e, const DevScalars *ds) {
    if (vc_skip(ds)) return;
    const int lane = threadIdx.x & 63;
    for_each_slice(S, [&](int64_t s) {
        const int64_t i = s * kWave + lane;
        if (i < n) e[i] = T(0);
    });
}

// e_out = e + omega (r - A e) / D; DOT also accumulates the block partials of
// rdot . e_out (the preconditioned CG's r . z, saving a pass over both)
// The finer level's unscaled correction e_f += P e_c, applied by the kernel
// that produces e_c: row a adds its value to the members of aggregate a.
constexpr int kCorrBatch = 8;  // aggregate members a fused correction handles at once

template <typename T>
struct FineCorr {
    T *e;
    const int32_t *start, *cells;
    __device__ __forceinline__ void operator()(int32_t a, T v) const {
        apply(start[a], start[a + 1], v);
    }
    // members k0..k1-1 of the aggregate (bounds loaded ahead by the caller),
    // kCorrBatch at a time: their indices, then their values, are loaded
    // together before any store (the members are distinct cells), so an
    // aggregate of several passes costs a few round trips, not one per member
    __device__ __forceinline__ void apply(int32_t k0, int32_t k1, T v) const {
        for (int32_t k = k0; k < k1; k += kCorrBatch) {
            int32_t j[kCorrBatch];
            T ev[kCorrBatch];
#pragma unroll
            for (int u = 0; u < kCorrBatch; ++u)
                if (k + u < k1) j[u] = cells[k + u];
#pragma unroll
            for (int u = 0; u < kCorrBatch; ++u)
                if (k + u < k1) ev[u] = e[j[u]];
#pragma unroll
            for (int u = 0; u < kCorrBatch; ++u)
                if (k + u < k1) e[j[u]] = ev[u] + v;
        }
    }
};

// e_out = e + omega (r - A e) / D; DOT also accumulates the block partials of
// rdot . e_out (the preconditioned CG's r . z, saving a pass over both); CORR
// also applies the finer level's correction with e_out
template <bool CMP, bool DOT, bool CORR, typename T>
__global__ void __launch_bounds__(kBlock)
k_vc_jacobi(SellView<T> A, const T *__restrict__ r, const T *__restrict__ e,
            T *__restrict__ eo, T omega, const T *__restrict__ rdot, double *partials,
            FineCorr<T> fc, const DevScalars *ds) {
    if (vc_skip(ds)) return;
    const int lane = threadIdx.x & 63;
    double acc[1] = {0.0};
    // with CORR the aggregate bounds of row i are loaded before the row's
    // product, so their round trip overlaps its gathers
    auto finish = [&](int32_t i, T y, T ri, T di, T ei, int32_t k0, int32_t k1) {
        const T zi = ei + omega * (ri - y) / di;
        eo[i] = zi;
        if constexpr (DOT) acc[0] += (double)rdot[i] * (double)zi;
        if constexpr (CORR) fc.apply(k0, k1, zi);
    };
    if constexpr (CMP) {
        // the row's own values (r, D, e) are loaded before its entries, so
        // their round trip overlaps the entry loads and gathers
        for_each_cmp_slice(A, [&](int64_t, const CmpHead &hd) {
            if (hd.row >= 0) {
                const int32_t i = hd.row;
                int32_t k0 = 0, k1 = 0;
                if constexpr (CORR) {
                    k0 = fc.start[i];
                    k1 = fc.start[i + 1];
                }
                const T ri = r[i], di = A.diag[i], ei = e[i];
                T y = di * ei;  // the row's order: diagonal, then columns
                cmp_entries_at<kCmpBatch>(A, hd.b0, hd.w, lane, Direct<T>{e},
                                          [&](int32_t, T v, T xv) { y = y + v * xv; });
                finish(i, y, ri, di, ei, k0, k1);
            }
        });
    } else {
        for_each_slice<product_cap<CMP, T>()>(A.nslices, [&](int64_t s) {
            const int64_t p = s * kWave + lane;
            if (p < A.n) {
                const int32_t i = (int32_t)p;
                int32_t k0 = 0, k1 = 0;
                if constexpr (CORR) {
                    k0 = fc.start[i];
                    k1 = fc.start[i + 1];
                }
                const T y = sell_row<CMP>(A, s, lane, i, Direct<T>{e});
                // the CG's last sweep (DOT) reads r and D nontemporally: the
                // iteration reads neither again before its next CG product
                if constexpr (DOT)
                    finish(i, y, vld<true>(r + i), vld<true>(A.diag + i), e[i], k0, k1);
                else
                    finish(i, y, r[i], A.diag[i], e[i], k0, k1);
            }
        });
    }
    if constexpr (DOT) block_partials<1>(acc, partials);
}

// t = r - A e
template <bool CMP, typename T>
__global__ void __launch_bounds__(kBlock)
k_vc_resid(SellView<T> A, const T *__restrict__ r, const T *__restrict__ e,
           T *__restrict__ t, const DevScalars *ds) {
    if (vc_skip(ds)) return;
    const int lane = threadIdx.x & 63;
    for_each_slice<product_cap<CMP, T>()>(A.nslices, [&](int64_t s) {
        const int64_t p = s * kWave + lane;
        if (p < A.n) {
            const int32_t i = sv_row<CMP>(A, p);
            t[i] = r[i] - sell_row<CMP>(A, s, lane, i, Direct<T>{e});
        }
    });
}

// one inner step of the two-stage Gauss-Seidel sweep (Berger-Vergiat et al.
// 2021, the paper's second GPU smoother, Sec. 4.3):
//   g_i = (t_i - sum_{j in tri(i)} A_ij src_j) / D_i
// over the strictly lower (forward sweep) or strictly upper (backward sweep)
// part of row i; src_j = t_j / D_j on the first step (SRC_T), else the
// previous step's g.  mode 0 stores g; mode 1 sets e = g (a sweep from
// zero); mode 2 adds g to e.
template <typename T>
struct DivDiag {
    const T *t, *D;
    __device__ __forceinline__ T operator()(int32_t j) const { return t[j] / D[j]; }
};

template <bool CMP, bool UPPER, bool SRC_T, typename T>
__global__ void __launch_bounds__(kBlock)
k_vc_gs(SellView<T> A, const T *__restrict__ t, const T *__restrict__ g, T *__restrict__ out,
        int mode, const DevScalars *ds) {
    if (vc_skip(ds)) return;
    const int lane = threadIdx.x & 63;
    for_each_slice<product_cap<CMP, T>()>(A.nslices, [&](int64_t s) {
        const int64_t p = s * kWave + lane;
        if (p < A.n) {
            const int32_t i = sv_row<CMP>(A, p);
            T y;
            if constexpr (SRC_T) y = sell_tri<CMP, UPPER>(A, s, lane, i, DivDiag<T>{t, A.diag});
            else y = sell_tri<CMP, UPPER>(A, s, lane, i, Direct<T>{g});
            const T gi = (t[i] - y) / A.diag[i];
            out[i] = mode == 2 ? out[i] + gi : gi;
        }
    });
}

// r_c[a] = sum of t over the members of aggregate a, ascending cell order
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_vc_restrict(int32_t nc, const int32_t *__restrict__ start, const int32_t *__restrict__ cells,
              const T *__restrict__ t, T *__restrict__ rc, T *__restrict__ ec_first,
              const T *__restrict__ Dc, T omega, const DevScalars *ds) {
    if (vc_skip(ds)) return;
    GRID_STRIDE(a, nc) {
        const T dc = ec_first ? Dc[a] : T(1);  // loaded ahead of the member sums
        T s = T(0);
        const int32_t k1 = start[a + 1];
        for (int32_t k = start[a]; k < k1; k += kCorrBatch) {  // loads of a batch together
            int32_t j[kCorrBatch];
            T tv[kCorrBatch];
#pragma unroll
            for (int u = 0; u < kCorrBatch; ++u)
                if (k + u < k1) j[u] = cells[k + u];
#pragma unroll
            for (int u = 0; u < kCorrBatch; ++u)
                if (k + u < k1) tv[u] = t[j[u]];
#pragma unroll
            for (int u = 0; u < kCorrBatch; ++u)
                if (k + u < k1) s += tv[u];
        }
        rc[a] = s;
        // the coarse level's first Jacobi sweep from zero, e_c = omega r_c / D_c
        if (ec_first) ec_first[a] = omega * s / dc;
    }
}

// ---------------------------------------------------------------- restriction operator
// The down leg of a cycle whose pre-smoothing is one Jacobi sweep from zero,
// e = omega D^-1 r, followed by the residual and its restriction (the
// agglomeration's summation, Sec. 4.3):
//   r_c = P^T (r - A e) = P^T (I - omega A D^-1) r = R r,
//   R_cj = sum over the members i of c, ascending, of (1 - omega) when
//          j = i and -omega a_ij / D_j for the entries a_ij of row i.
// One pass over R replaces the residual kernel (which writes t) and the
// restriction (which reads it back through the member lists); the two are
// equal up to rounding.  valT holds R for A^T (a_ji).
// A large plain-slice level (a fine mesh) keeps the two steps but folds the
// sweep into its own slices: t = (I - omega A D^-1) r is a product over the
// level's layout, 16-bit columns included, with the values -omega a_ij / D_j
// (Ah), and the member sums of t follow.  R's rows there would gather from
// members of several orientations at once (a pair along z reaches two mesh
// planes, a pair along x one), so each of their gathers touches about three
// times as many cache lines per entry as the level's own rows do.

// entries a coarse row gathers before merging: its members' row entries and
// their diagonals
__global__ void k_rop_count(int32_t nc, const int32_t *__restrict__ start,
                            const int32_t *__restrict__ cells, Sell A, int64_t *cnt) {
    GRID_STRIDE(c, nc) {
        int64_t m = 0;
        for (int32_t k = start[c]; k < start[c + 1]; ++k) {
            const int32_t i = cells[k];
            const int64_t ps = A.iperm ? (int64_t)A.iperm[i] : (int64_t)i;
            const int w = row_len(A, ps);
            m += 1;
            for (int q = 0; q < w; ++q) m += A.col[entry_at(A, ps, q)] != i;  // padding: col i
        }
        cnt[c] = m;
    }
}

// a member row's entries in column order, with the diagonal at its place:
// (col, src) with src the entry's position in the level's slices, or -1 for
// the diagonal; valid is false past the end
struct RowCursor {
    int32_t i = 0, col = 0;
    int64_t ps = 0, src = 0;
    int w = 0, q = 0;
    bool diag = false, valid = false;
    __device__ void init(const Sell &A, int32_t row) {
        i = row;
        ps = A.iperm ? (int64_t)A.iperm[row] : (int64_t)row;
        w = row_len(A, ps);
        q = 0;
        diag = false;
        next(A);
    }
    __device__ void next(const Sell &A) {
        while (q < w) {
            const int64_t e = entry_at(A, ps, q);
            const int32_t j = A.col[e];
            if (j == i) {  // padding points at the row
                ++q;
                continue;
            }
            if (!diag && j > i) break;
            col = j;
            src = e;
            ++q;
            valid = true;
            return;
        }
        if (!diag) {
            col = i;
            src = -1;
            diag = true;
            valid = true;
            return;
        }
        valid = false;
    }
};

// per coarse row: the member contributions in member order, each member's in
// column order, as (column, source) pairs (source: the entry's position in
// the level's slices, or -1 for a member's own diagonal), ordered by column
// with equal columns in member order: a merge of the two rows of a pair, or a
// stable insertion sort of the concatenated rows of a larger aggregate.
// rdeg: the number of distinct columns.
__global__ void k_rop_gather(int32_t nc, const int32_t *__restrict__ start,
                             const int32_t *__restrict__ cells, Sell A,
                             const int64_t *__restrict__ tstart, int32_t *tcol, int64_t *tsrc,
                             int32_t *rdeg) {
    GRID_STRIDE(c, nc) {
        const int64_t o = tstart[c];
        int m = 0;
        auto push = [&](int32_t j, int64_t src) {
            tcol[o + m] = j;
            tsrc[o + m] = src;
            ++m;
        };
        const int32_t k0 = start[c], k1 = start[c + 1];
        if (k1 - k0 <= 2) {
            RowCursor a, b;
            a.init(A, cells[k0]);
            if (k1 - k0 == 2) b.init(A, cells[k0 + 1]);
            while (a.valid || b.valid) {
                if (a.valid && (!b.valid || a.col <= b.col)) {
                    push(a.col, a.src);
                    a.next(A);
                } else {
                    push(b.col, b.src);
                    b.next(A);
                }
            }
            int u = 0;
            for (int t = 0; t < m; ++t) u += t == 0 || tcol[o + t] != tcol[o + t - 1];
            rdeg[c] = u;
            continue;
        }
        for (int32_t k = k0; k < k1; ++k) {
            const int32_t i = cells[k];
            const int64_t ps = A.iperm ? (int64_t)A.iperm[i] : (int64_t)i;
            const int w = row_len(A, ps);
            bool diag = false;
            for (int q = 0; q < w; ++q) {
                const int64_t e = entry_at(A, ps, q);
                const int32_t j = A.col[e];
                if (j == i) continue;
                if (!diag && j > i) {
                    push(i, -1);
                    diag = true;
                }
                push(j, e);
            }
            if (!diag) push(i, -1);
        }
        int u = 0;
        for (int a = 0; a < m; ++a) {
            const int32_t kc = tcol[o + a];
            const int64_t ks = tsrc[o + a];
            int b = a - 1;
            while (b >= 0 && tcol[o + b] > kc) {
                tcol[o + b + 1] = tcol[o + b];
                tsrc[o + b + 1] = tsrc[o + b];
                --b;
            }
            tcol[o + b + 1] = kc;
            tsrc[o + b + 1] = ks;
        }
        for (int a = 0; a < m; ++a) u += a == 0 || tcol[o + a] != tcol[o + a - 1];
        rdeg[c] = u;
    }
}

// R's columns, and for each entry of R the run of its sources in the sorted
// pairs (start, count): compressed slices
__global__ void k_rop_link_sell(int32_t nc, Sell R, const int64_t *__restrict__ tstart,
                                const int32_t *__restrict__ tcol, int64_t *rs0, int32_t *rsn) {
    GRID_STRIDE(c, nc) {
        const int64_t ps = R.iperm[c], o = tstart[c], o1 = tstart[c + 1];
        int q = 0;
        for (int64_t a = o; a < o1;) {
            int64_t b = a + 1;
            while (b < o1 && tcol[b] == tcol[a]) ++b;
            const int64_t e = entry_at(R, ps, q++);
            R.col[e] = tcol[a];
            rs0[e] = a;
            rsn[e] = (int32_t)(b - a);
            a = b;
        }
    }
}

// the same for CSR
__global__ void k_rop_link_csr(int32_t nc, Csr R, const int64_t *__restrict__ tstart,
                               const int32_t *__restrict__ tcol, int64_t *rs0, int32_t *rsn) {
    GRID_STRIDE(c, nc) {
        const int64_t o = tstart[c], o1 = tstart[c + 1];
        int64_t e = R.rptr[c];
        for (int64_t a = o; a < o1;) {
            int64_t b = a + 1;
            while (b < o1 && tcol[b] == tcol[a]) ++b;
            R.col[e] = tcol[a];
            rs0[e] = a;
            rsn[e] = (int32_t)(b - a);
            ++e;
            a = b;
        }
    }
}

__global__ void k_widen(int32_t n, const int32_t *__restrict__ a, int64_t *__restrict__ b) {
    GRID_STRIDE(i, n) b[i] = a[i];
}

// values of R (and of its A^T form) from the level's coefficients: each entry
// sums its sources in member order, (1 - omega) for a diagonal and
// -omega a / D_j for an entry a of column j
template <class M>
__global__ void k_rop_values(int64_t nnz, M R, const int64_t *__restrict__ rs0,
                             const int32_t *__restrict__ rsn, const int64_t *__restrict__ src,
                             const double *__restrict__ aval, const double *__restrict__ avalT,
                             const double *__restrict__ D, double omega) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz;
         e += (int64_t)gridDim.x * blockDim.x) {
        const double dj = D[R.col[e]];
        double v = 0.0, vT = 0.0;
        for (int64_t k = rs0[e]; k < rs0[e] + rsn[e]; ++k) {
            const int64_t q = src[k];
            if (q < 0) {
                v = v + (1.0 - omega);
                vT = vT + (1.0 - omega);
            } else {
                v = v + (-omega * aval[q]) / dj;
                vT = vT + (-omega * avalT[q]) / dj;
            }
        }
        R.val[e] = v;
        R.valT[e] = vT;
    }
}

__global__ void k_rop_f32(const double *a, float *b, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        b[i] = (float)a[i];
}

// Ah = -omega A D^-1 at the positions of a plain-slice level's entries (the
// same expression as a source of R's values); padding (value 0) stays 0
__global__ void k_ahat_values(int64_t nnz, const int32_t *__restrict__ col,
                              const double *__restrict__ val, const double *__restrict__ valT,
                              const double *__restrict__ D, double omega, double *__restrict__ ah,
                              double *__restrict__ ahT) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz;
         e += (int64_t)gridDim.x * blockDim.x) {
        const double dj = D[col[e]];
        ah[e] = (-omega * val[e]) / dj;
        ahT[e] = (-omega * valT[e]) / dj;
    }
}

// t = (I - omega A D^-1) r over a plain-slice level whose values are Ah:
// row i is (1 - omega) r_i plus its entries in column order
template <bool C16, typename T>
__global__ void __launch_bounds__(kBlock)
k_vc_ahat(SellView<T> Ah, const T *__restrict__ r, T *__restrict__ t, T c0,
          const DevScalars *ds) {
    if (vc_skip(ds)) return;
    const int lane = threadIdx.x & 63;
    for_each_slice<product_cap<false, T>()>(Ah.nslices, [&](int64_t s) {
        const int64_t p = s * kWave + lane;
        if (p < Ah.n) {
            T y = c0 * r[p];
            plain_entries<C16, 8>(Ah, s, lane, Direct<T>{r},
                                  [&](int32_t, T v, T xv) { y = y + v * xv; });
            t[p] = y;
        }
    });
}

// cycles whose down leg R replaces: Jacobi, one pre-sweep, no correction
// scaling (which needs the residual itself)
static bool rop_cycle(const ldu_gamg_opts &o) {
    return o.smoother == LDU_SMOOTH_JACOBI && o.n_pre == 1 && !o.scale_correction;
}

// entries a lane of the compressed-slice R product loads before its gathers:
// R's rows are longer than the level's own (47 entries on the c3 headline's
// level 1), so it takes larger batches than kCmpBatch (FP64 solves with 24,
// 32 and 48 entries: 147.2, 146.0 and 148.0 ms; mixed ones: 116.4, 115.5
// and 114.3 ms)
template <typename T>
constexpr int kRBatch = sizeof(T) == 8 ? 32 : 48;

// r_c = R r (row c: columns ascending, from zero), and the coarse level's
// first Jacobi sweep from zero e_c = omega r_c / D_c when ec_first is given
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_vc_rrestrict_cmp(SellView<T> R, const T *__restrict__ r, T *__restrict__ rc,
               T *__restrict__ ec_first, const T *__restrict__ Dc, T omega,
               const DevScalars *ds) {
    if (vc_skip(ds)) return;
    const int lane = threadIdx.x & 63;
    for_each_cmp_slice(R, [&](int64_t, const CmpHead &hd) {
        if (hd.row >= 0) {
            const int32_t c = hd.row;
            // the coarse diagonal is loaded before the row, so its round
            // trip overlaps the row's gathers
            const T dc = ec_first ? Dc[c] : T(1);
            T acc = T(0);
            cmp_entries_at<kRBatch<T>>(R, hd.b0, hd.w, lane, Direct<T>{r},
                                       [&](int32_t, T v, T xv) { acc = acc + v * xv; });
            rc[c] = acc;
            if (ec_first) ec_first[c] = omega * acc / dc;
        }
    });
}

// r_c = R r, and the coarse level's first Jacobi sweep from zero
// e_c = omega r_c / D_c when ec_first is given.  G lanes share a row: lane g
// of the group sums the row's entries g, g + G, g + 2G, ... in order, then
// the group adds its G partial sums by a fixed butterfly (every lane ends
// with the same total).  A wave covers 64 / G consecutive rows.  The order
// is fixed, so results are reproducible; it is not the row's column order,
// which R's results never had to follow (R's rows are sums the oracle forms
// in two steps, residual then restriction).
template <int G, typename T>
__global__ void __launch_bounds__(kBlock)
k_vc_rrestrict_csr(CsrView<T> R, const T *__restrict__ r, T *__restrict__ rc,
               T *__restrict__ ec_first, const T *__restrict__ Dc, T omega,
               const DevScalars *ds) {
    if (vc_skip(ds)) return;
    constexpr int RPW = kWave / G;
    constexpr int U = kCsrBatch;
    const int lane = threadIdx.x & 63;
    const int g = lane % G;
    const int64_t chunks = (R.n + RPW - 1) / RPW;
    for_each_slice(chunks, [&](int64_t s) {
        const int64_t c = s * RPW + lane / G;
        T acc = T(0), dc = T(1);
        if (c < R.n) {
            // the coarse diagonal is loaded before the row, so its round
            // trip overlaps the row's gathers
            if (ec_first && g == 0) dc = Dc[c];
            const int64_t e1 = R.rptr[c + 1];
            for (int64_t k0 = R.rptr[c] + g; k0 < e1; k0 += (int64_t)G * U) {
                int32_t cc[U];
                T vv[U], xv[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int64_t k = k0 + (int64_t)u * G;
                    if (k < e1) {
                        cc[u] = __builtin_nontemporal_load(R.col + k);
                        vv[u] = __builtin_nontemporal_load(R.val + k);
                    }
                }
#pragma unroll
                for (int u = 0; u < U; ++u)
                    if (k0 + (int64_t)u * G < e1) xv[u] = r[cc[u]];
#pragma unroll
                for (int u = 0; u < U; ++u)
                    if (k0 + (int64_t)u * G < e1) acc = acc + vv[u] * xv[u];
            }
        }
#pragma unroll
        for (int off = G / 2; off > 0; off >>= 1) acc = acc + __shfl_xor(acc, off);
        if (c < R.n && g == 0) {
            rc[c] = acc;
            if (ec_first) ec_first[c] = omega * acc / dc;
        }
    });
}

template <typename T>
static void launch_rrestrict_csr(const CsrView<T> &R, const T *r, T *rc, T *ec_first, const T *Dc,
                             T omega, const DevScalars *ds, hipStream_t st) {
    const int64_t chunks = (R.n + kWave / R.group - 1) / (kWave / R.group);
    const int G = stream_grid_slices(chunks);
    switch (R.group) {
    case 1: k_vc_rrestrict_csr<1, T><<<G, kBlock, 0, st>>>(R, r, rc, ec_first, Dc, omega, ds); break;
    case 2: k_vc_rrestrict_csr<2, T><<<G, kBlock, 0, st>>>(R, r, rc, ec_first, Dc, omega, ds); break;
    case 4: k_vc_rrestrict_csr<4, T><<<G, kBlock, 0, st>>>(R, r, rc, ec_first, Dc, omega, ds); break;
    case 8: k_vc_rrestrict_csr<8, T><<<G, kBlock, 0, st>>>(R, r, rc, ec_first, Dc, omega, ds); break;
    default: k_vc_rrestrict_csr<16, T><<<G, kBlock, 0, st>>>(R, r, rc, ec_first, Dc, omega, ds);
    }
}

// c = P e_c; s = (c . t) / (c . A c), or 1 when c.Ac is ~0
template <bool CMP, typename T>
__global__ void __launch_bounds__(kBlock)
k_vc_scale(SellView<T> A, const T *__restrict__ ec, const int32_t *__restrict__ agg,
           const T *__restrict__ t, double *partials, const DevScalars *ds) {
    if (vc_skip(ds)) return;
    const int lane = threadIdx.x & 63;
    double acc[2] = {0.0, 0.0};
    for_each_slice<product_cap<CMP, T>()>(A.nslices, [&](int64_t s) {
        const int64_t p = s * kWave + lane;
        if (p < A.n) {
            const int32_t i = sv_row<CMP>(A, p);
            const T ac = sell_row<CMP>(A, s, lane, i, ViaAgg<T>{ec, agg});
            const T ci = ec[agg[i]];
            acc[0] += (double)ci * (double)t[i];
            acc[1] += (double)ci * (double)ac;
        }
    });
    block_partials<2>(acc, partials);
}

struct EpiScale {
    __device__ bool active(const DevScalars *ds) const { return !vc_skip(ds); }
    __device__ void operator()(const double *v, DevScalars *ds) const {
        ds->s = (isfinite(v[1]) && fabs(v[1]) > 1e-300) ? v[0] / v[1] : 1.0;
    }
};

// e += s c.  With rfirst, e is the first Jacobi sweep from zero, formed here
// as omega r / D (the same expression as k_vc_first) instead of being read.
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_vc_correct(int32_t n, int64_t S, const T *__restrict__ ec, const int32_t *__restrict__ agg,
             T *__restrict__ e, int use_s, const T *__restrict__ rfirst,
             const T *__restrict__ D, T omega, const DevScalars *ds) {
    if (vc_skip(ds)) return;
    const T sc = use_s ? (T)ds->s : T(1);
    const int lane = threadIdx.x & 63;
    for_each_slice(S, [&](int64_t s) {
        const int64_t i = s * kWave + lane;
        if (i < n) {
            const T e0 = rfirst ? omega * rfirst[i] / D[i] : e[i];
            e[i] = e0 + sc * ec[agg[i]];
        }
    });
}

// coarsest level: diagonal PCG in FP64 by one workgroup, from e = 0 to
// ||r|| <= tol ||rhs|| or max_it iterations; a singular level first
// projects its rhs to zero mean.  w: 3 n doubles of scratch (r, p, q).
template <int K, int NW>
__device__ __forceinline__ void bcast_sum(double (&v)[K]) {
    if constexpr (NW == 1) {
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] = wave_sum(v[k]);  // every lane gets the sum
    } else {
        __shared__ double out[K];
        block_reduce<K>(v);
        if (threadIdx.x == 0) {
#pragma unroll
            for (int k = 0; k < K; ++k) out[k] = v[k];
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] = out[k];
        __syncthreads();
    }
}

// LDS holds the coarsest CG vectors when 5 n doubles fit (dynamic shared memory)
constexpr int kLdsCoarse = 1536;

// a barrier also in the one-wavefront case (there it costs next to nothing
// and orders the LDS stores of one lane before other lanes' loads)
template <int NW>
__device__ __forceinline__ void csync() {
    __syncthreads();
}

// DIC preconditioner z = M^-1 r by forward and backward substitution in row
// form, serially (one thread): y_i = (r_i - sum_{j<i} A_ij y_j) / Dt_i for
// ascending i, then z_i = y_i - (sum_{j>i} A_ij z_j) / Dt_i for descending i,
// each row sum in column order
__device__ void dic_serial(const SellView<double> &A, const double *__restrict__ dt,
                           const double *__restrict__ r, double *__restrict__ z) {
    const int32_t n = A.n;
    for (int32_t i = 0; i < n; ++i) {
        const int64_t ps = sv_pos(A, i);
        const int w = row_len(A, ps);
        double sum = 0.0;
        for (int k = 0; k < w; ++k) {
            const int64_t e = entry_at(A, ps, k);
            const int32_t c = A.col[e];
            if (c < i) sum = sum + A.val[e] * z[c];
        }
        z[i] = (r[i] - sum) / dt[i];
    }
    for (int32_t i = n - 1; i >= 0; --i) {
        const int64_t ps = sv_pos(A, i);
        const int w = row_len(A, ps);
        double sum = 0.0;
        for (int k = 0; k < w; ++k) {
            const int64_t e = entry_at(A, ps, k);
            const int32_t c = A.col[e];
            if (c > i) sum = sum + A.val[e] * z[c];
        }
        z[i] = z[i] - sum / dt[i];
    }
}

template <typename TI, int NW>
__device__ void coarsest_body(const SellView<double> &A, const TI *__restrict__ rhs,
                              TI *__restrict__ eo, double *__restrict__ w, int singular,
                              double tol, int max_it, const double *__restrict__ dt) {
    constexpr int NT = NW * kWave;
    const int32_t n = A.n;
    double *r = w, *p = w + n, *q = w + 2 * (int64_t)n, *x = w + 3 * (int64_t)n,
           *z = w + 4 * (int64_t)n;
    for (int32_t i = threadIdx.x; i < n; i += NT) {
        r[i] = (double)rhs[i];
        x[i] = 0.0;
    }
    csync<NW>();
    if (singular) {
        double m[1] = {0.0};
        for (int32_t i = threadIdx.x; i < n; i += NT) m[0] += r[i];
        bcast_sum<1, NW>(m);
        const double mean = m[0] / (double)n;
        for (int32_t i = threadIdx.x; i < n; i += NT) r[i] = r[i] - mean;
        csync<NW>();
    }
    // z = M^-1 r (diagonal, or DIC when dt is given); r is complete on entry
    auto precond = [&]() {
        if (dt) {
            if (threadIdx.x == 0) dic_serial(A, dt, r, z);
        } else {
            for (int32_t i = threadIdx.x; i < n; i += NT) z[i] = r[i] / A.diag[i];
        }
        csync<NW>();
    };
    double b2[1] = {0.0};
    for (int32_t i = threadIdx.x; i < n; i += NT) b2[0] += r[i] * r[i];
    bcast_sum<1, NW>(b2);
    const double bn = sqrt(b2[0]);
    if (bn > 0.0) {
        precond();
        double rz[1] = {0.0};
        for (int32_t i = threadIdx.x; i < n; i += NT) {
            p[i] = z[i];
            rz[0] += r[i] * z[i];
        }
        bcast_sum<1, NW>(rz);
        double rho = rz[0];
        for (int it = 0; it < max_it; ++it) {
            double pq[1] = {0.0};
            for (int32_t i = threadIdx.x; i < n; i += NT) {
                const int64_t ps = sv_pos(A, i);
                const double qi = sell_row_any(A, ps >> 6, (int)(ps & 63), i, Direct<double>{p});
                q[i] = qi;
                pq[0] += p[i] * qi;
            }
            bcast_sum<1, NW>(pq);
            if (!isfinite(pq[0]) || fabs(pq[0]) <= 1e-300) break;
            const double alpha = rho / pq[0];
            double rr[1] = {0.0};
            for (int32_t i = threadIdx.x; i < n; i += NT) {
                x[i] = x[i] + alpha * p[i];
                const double ri = r[i] - alpha * q[i];
                r[i] = ri;
                rr[0] += ri * ri;
            }
            bcast_sum<1, NW>(rr);
            if (sqrt(rr[0]) / bn <= tol) break;
            precond();
            double rzn[1] = {0.0};
            for (int32_t i = threadIdx.x; i < n; i += NT) rzn[0] += r[i] * z[i];
            bcast_sum<1, NW>(rzn);
            const double beta = rzn[0] / rho;
            rho = rzn[0];
            for (int32_t i = threadIdx.x; i < n; i += NT) p[i] = z[i] + beta * p[i];
            csync<NW>();
        }
    }
    csync<NW>();
    for (int32_t i = threadIdx.x; i < n; i += NT) eo[i] = (TI)x[i];
}

__device__ __forceinline__ double readlane_f64(double v, int j) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), j);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), j);
    return __hiloint2double(hi, lo);
}


// coarsest level of at most 64 cells with rows of at most kWaveRow entries:
// one wavefront, one row per lane, the row's entries held in LDS
// (entry-major, so lanes read distinct banks) and the search direction in
// LDS.  Row i sums diag_i p_i first and then its entries in column order, as
// the sparse kernels do.  The first kRegRow entries of a row also stay in
// registers for the whole solve, so a product issues all their gathers of p
// at once instead of one LDS round trip per entry.
constexpr int kWaveRow = 48;
constexpr int kRegRow = 16;

// LDS ordering for one wavefront: its LDS operations execute in order, so a
// fence against compiler reordering is all a lane-to-lane exchange needs
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

struct CoarsestLds {
    int32_t cL[kWaveRow * kWave];
    double vL[kWaveRow * kWave];
    double p[kWave];
};

// the one-wavefront coarsest CG, run by the 64 lanes of one wave (the
// caller's other waves, if any, do not take part)
__device__ void coarsest_wave_body(const SellView<double> &A, const double *__restrict__ rhs_d,
                                   const float *__restrict__ rhs_f, double *__restrict__ eo_d,
                                   float *__restrict__ eo_f, int singular, double tol,
                                   int max_it, const double *__restrict__ dt,
                                   const FineCorr<double> &fcd, const FineCorr<float> &fcf,
                                   CoarsestLds &sm) {
    int32_t *cL = sm.cL;
    double *vL = sm.vL;
    double *p = sm.p;
    const int32_t n = A.n;
    const int i = threadIdx.x;
    double di = 1.0, ri = 0.0, rdt = 0.0;
    int m = 0, nl = 0;  // entries of row i, and how many lie left of the diagonal
    if (i < n) {
        const int64_t ps = sv_pos(A, i);
        const int w = row_len(A, ps);
        for (int k = 0; k < w; ++k) {
            const int64_t e = entry_at(A, ps, k);
            const int32_t c = A.col[e];
            if (c == i) continue;  // padding entries point at the row
            cL[m * kWave + i] = c;
            vL[m * kWave + i] = A.val[e];
            nl += c < i;
            ++m;
        }
        di = A.diag[i];
        ri = rhs_d ? rhs_d[i] : (double)rhs_f[i];
        if (dt) rdt = 1.0 / dt[i];
    }
    wave_lds_sync();
    int32_t cR[kRegRow];
    double vR[kRegRow];
#pragma unroll
    for (int k = 0; k < kRegRow; ++k) {
        cR[k] = k < m ? cL[k * kWave + i] : 0;
        vR[k] = k < m ? vL[k * kWave + i] : 0.0;
    }
    // z = M^-1 r: the diagonal, or the DIC factor by column-oriented
    // substitution: at step j lane j's value is final and is broadcast, and
    // every row holding column j takes its term (lower entries in ascending
    // column order on the way down, upper entries in descending order on the
    // way up)
    auto precond = [&](double rv) -> double {
        if (!dt) return (i < n) ? rv / di : 0.0;
        double acc = 0.0, y = 0.0;
        int kk = 0;
        for (int j = 0; j < n; ++j) {
            const double cand = (rv - acc) * rdt;
            const double yj = readlane_f64(cand, j);
            if (i == j) y = cand;
            if (kk < nl && cL[kk * kWave + i] == j) {
                acc = acc + vL[kk * kWave + i] * yj;
                ++kk;
            }
        }
        acc = 0.0;
        double zv = 0.0;
        kk = m - 1;
        for (int j = n - 1; j >= 0; --j) {
            const double cand = y - acc * rdt;
            const double zj = readlane_f64(cand, j);
            if (i == j) zv = cand;
            if (kk >= nl && cL[kk * kWave + i] == j) {
                acc = acc + vL[kk * kWave + i] * zj;
                --kk;
            }
        }
        return (i < n) ? zv : 0.0;
    };
    if (singular) {
        const double mean = wave_sum(ri) / (double)n;
        if (i < n) ri = ri - mean;
    }
    double xi = 0.0;
    const double bn = sqrt(wave_sum(ri * ri));
    if (bn > 0.0) {
        double pi = precond(ri);
        double rho = wave_sum(ri * pi);
        for (int it = 0; it < max_it; ++it) {
            p[i] = pi;
            wave_lds_sync();
            double qi = 0.0;
            if (i < n) {
                double pv[kRegRow];
#pragma unroll
                for (int k = 0; k < kRegRow; ++k) pv[k] = k < m ? p[cR[k]] : 0.0;
                qi = di * pi;
#pragma unroll
                for (int k = 0; k < kRegRow; ++k)
                    if (k < m) qi = qi + vR[k] * pv[k];
                for (int k = kRegRow; k < m; ++k)
                    qi = qi + vL[k * kWave + i] * p[cL[k * kWave + i]];
            }
            wave_lds_sync();
            const double pq = wave_sum(pi * qi);
            if (!isfinite(pq) || fabs(pq) <= 1e-300) break;
            const double alpha = rho / pq;
            xi = xi + alpha * pi;
            ri = ri - alpha * qi;
            const double zi = precond(ri);
            const double rr = wave_sum(ri * ri);
            const double rz = wave_sum(ri * zi);
            if (sqrt(rr) / bn <= tol) break;
            const double beta = rz / rho;
            rho = rz;
            pi = zi + beta * pi;
        }
    }
    if (i < n) {  // the result, and the finer level's correction with it
        if (eo_d) {
            eo_d[i] = xi;
            if (fcd.e) fcd(i, xi);
        } else {
            const float v = (float)xi;
            eo_f[i] = v;
            if (fcf.e) fcf(i, v);
        }
    }
}

__global__ void __launch_bounds__(kWave)
k_coarsest_wave(SellView<double> A, const double *__restrict__ rhs_d,
                const float *__restrict__ rhs_f, double *__restrict__ eo_d,
                float *__restrict__ eo_f, int singular, double tol, int max_it,
                const double *__restrict__ dt, FineCorr<double> fcd, FineCorr<float> fcf,
                const DevScalars *ds) {
    __shared__ CoarsestLds sm;
    if (vc_skip(ds)) return;
    coarsest_wave_body(A, rhs_d, rhs_f, eo_d, eo_f, singular, tol, max_it, dt, fcd, fcf, sm);
}

// coarsest-level launch for larger levels: one 256-thread block
template <typename TI, int NW>
__global__ void __launch_bounds__(kBlock)
k_coarsest(SellView<double> A, const TI *__restrict__ rhs, TI *__restrict__ eo,
           double *__restrict__ w, int singular, double tol, int max_it,
           const double *__restrict__ dt, const DevScalars *ds) {
    extern __shared__ double lds_w[];
    if (vc_skip(ds)) return;
    coarsest_body<TI, NW>(A, rhs, eo, A.n <= kLdsCoarse ? lds_w : w, singular, tol, max_it, dt);
}

// x += e (GAMG correction of the outer FP64 loop)
__global__ void __launch_bounds__(kBlock)
k_add(int32_t n, int64_t S, const double *__restrict__ e, double *__restrict__ x,
      const DevScalars *ds) {
    if (ds->done) return;
    const int lane = threadIdx.x & 63;
    for_each_slice(S, [&](int64_t s) {
        const int64_t i = s * kWave + lane;
        if (i < n) x[i] = x[i] + e[i];
    });
}

// mixed: rhat = fp32(r / ||r||_inf)
__global__ void __launch_bounds__(kBlock)
k_cast_scaled(int32_t n, int64_t S, const double *__restrict__ r, float *__restrict__ r32,
              DevScalars *ds) {
    if (ds->done) return;
    const double sc = ds->maxabs;
    const int lane = threadIdx.x & 63;
    for_each_slice(S, [&](int64_t s) {
        const int64_t i = s * kWave + lane;
        if (i < n) r32[i] = (float)(r[i] / sc);
    });
    if (blockIdx.x == 0 && threadIdx.x == 0) ds->scale = sc;
}

__global__ void __launch_bounds__(kBlock)
k_refine_add(int32_t n, int64_t S, const float *__restrict__ d, double *__restrict__ x,
             const DevScalars *ds) {
    if (ds->done) return;
    const double sc = ds->scale;
    const int lane = threadIdx.x & 63;
    for_each_slice(S, [&](int64_t s) {
        const int64_t i = s * kWave + lane;
        if (i < n) x[i] = x[i] + sc * (double)d[i];
    });
}

template <bool CMP, typename T>
static void launch_jacobi_l(const SellView<T> &A, const T *r, const T *e, T *eo, T omega,
                            const T *rdot, double *partials, const FineCorr<T> &fc,
                            const DevScalars *ds, int G, hipStream_t st) {
    if (rdot && fc.e)
        k_vc_jacobi<CMP, true, true, T><<<G, kBlock, 0, st>>>(A, r, e, eo, omega, rdot, partials, fc, ds);
    else if (rdot)
        k_vc_jacobi<CMP, true, false, T><<<G, kBlock, 0, st>>>(A, r, e, eo, omega, rdot, partials, fc, ds);
    else if (fc.e)
        k_vc_jacobi<CMP, false, true, T><<<G, kBlock, 0, st>>>(A, r, e, eo, omega, rdot, partials, fc, ds);
    else
        k_vc_jacobi<CMP, false, false, T><<<G, kBlock, 0, st>>>(A, r, e, eo, omega, rdot, partials, fc, ds);
}

// one Jacobi sweep; with rdot, also the block partials of rdot . e_out; with
// fc.e, also the finer level's correction
template <typename T>
static void launch_jacobi(const SellView<T> &A, const T *r, const T *e, T *eo, T omega,
                          const T *rdot, double *partials, const FineCorr<T> &fc,
                          const DevScalars *ds, int G, hipStream_t st) {
    if (A.pdeg) launch_jacobi_l<true, T>(A, r, e, eo, omega, rdot, partials, fc, ds, G, st);
    else launch_jacobi_l<false, T>(A, r, e, eo, omega, rdot, partials, fc, ds, G, st);
}

template <bool CMP, bool UPPER, typename T>
static void launch_gs_step(const SellView<T> &A, const T *t, const T *g, T *out, int mode,
                           const DevScalars *ds, int G, hipStream_t st) {
    if (g) k_vc_gs<CMP, UPPER, false, T><<<G, kBlock, 0, st>>>(A, t, g, out, mode, ds);
    else k_vc_gs<CMP, UPPER, true, T><<<G, kBlock, 0, st>>>(A, t, g, out, mode, ds);
}

// one two-stage Gauss-Seidel sweep on A e = r: t = r - A e (t = r from
// zero), `inner` triangular Jacobi-Richardson steps through the ping-pong
// buffers w0, w1, the last one updating e in place (each row reads only t,
// the previous step and its own e entry)
template <typename T>
static void gs_sweep(const SellView<T> &A, const T *r, T *e, T *t, T *w0, T *w1, bool from_zero,
                     bool backward, int inner, const DevScalars *ds, int G, hipStream_t st) {
    const T *tt = r;
    if (!from_zero) {
        if (A.pdeg) k_vc_resid<true, T><<<G, kBlock, 0, st>>>(A, r, e, t, ds);
        else k_vc_resid<false, T><<<G, kBlock, 0, st>>>(A, r, e, t, ds);
        tt = t;
    }
    const T *g = nullptr;
    for (int k = 0; k < inner; ++k) {
        const bool last = k + 1 == inner;
        T *out = last ? e : (k % 2 == 0 ? w0 : w1);
        const int mode = last ? (from_zero ? 1 : 2) : 0;
        if (A.pdeg) {
            if (backward) launch_gs_step<true, true, T>(A, tt, g, out, mode, ds, G, st);
            else launch_gs_step<true, false, T>(A, tt, g, out, mode, ds, G, st);
        } else {
            if (backward) launch_gs_step<false, true, T>(A, tt, g, out, mode, ds, G, st);
            else launch_gs_step<false, false, T>(A, tt, g, out, mode, ds, G, st);
        }
        g = out;
    }
}

// ---------------------------------------------------------------- V-cycle driver
struct VCtx {
    ldu_t *h;
    const ldu_gamg_opts *o;
    bool tr;
    hipStream_t st;
    double *cw;        // coarsest scratch, 5 n_coarsest doubles
    const double *dt;  // coarsest DIC pivots, or null for the diagonal
};

template <typename T>
static SellView<T> lview(const Level &L, bool tr);
template <>
SellView<double> lview<double>(const Level &L, bool tr) { return L.A.view(tr); }
template <>
SellView<float> lview<float>(const Level &L, bool tr) { return L.A.view32(tr); }

template <typename T>
static SellView<T> rview(const Level &L, bool tr);
template <>
SellView<double> rview<double>(const Level &L, bool tr) { return L.R.view(tr); }
template <>
SellView<float> rview<float>(const Level &L, bool tr) { return L.R.view32(tr); }
template <typename T>
static CsrView<T> rcview(const Level &L, bool tr);
template <>
CsrView<double> rcview<double>(const Level &L, bool tr) { return L.Rc.view(tr); }
template <>
CsrView<float> rcview<float>(const Level &L, bool tr) { return L.Rc.view32(tr); }
// R's values of this precision exist (either layout)
template <typename T>
static const T *ahval(const Level &L, bool tr);
template <>
const double *ahval<double>(const Level &L, bool tr) { return tr ? L.ahT : L.ah; }
template <>
const float *ahval<float>(const Level &L, bool tr) { return tr ? L.ahT32 : L.ah32; }
template <typename T>
static bool has_rop(const Level &L, bool tr) {
    return rview<T>(L, tr).val != nullptr || rcview<T>(L, tr).val != nullptr ||
           ahval<T>(L, tr) != nullptr;
}

template <typename T>
static T *lvec(Level &L, int which);
template <>
double *lvec<double>(Level &L, int which) {
    return which == 0 ? L.r : which == 1 ? L.e : which == 2 ? L.e2 : which == 3 ? L.t : L.w;
}
template <>
float *lvec<float>(Level &L, int which) {
    return which == 0 ? L.r32 : which == 1 ? L.e32 : which == 2 ? L.e232 : which == 3 ? L.t32
                                                                                     : L.w32;
}

constexpr int kFuseCorrRows = 1 << 17;


// One V-cycle e = V(l, r); returns the buffer holding e.  With rdot, the
// last level-l kernel also leaves the block partials of rdot . e in
// h->partials and *dotted is set (only when that kernel is a Jacobi sweep).
// e_ready: the caller's restriction already stored the first Jacobi sweep
// e = omega r / D in this level's e.  fc: the finer level's unscaled
// correction e_f += P e, applied here by the kernel that produces e when it
// can (*corrected tells the caller).
template <typename T>
static T *vcycle(const VCtx &c, size_t l, const T *r, const T *rdot = nullptr,
                 bool *dotted = nullptr, bool e_ready = false, FineCorr<T> fc = {},
                 bool *corrected = nullptr) {
    if (dotted) *dotted = false;
    if (corrected) *corrected = false;
    ldu_t *h = c.h;
    Level &L = h->levels[l];
    hipStream_t st = c.st;
    T *e = lvec<T>(L, 1), *e2 = lvec<T>(L, 2), *t = lvec<T>(L, 3);
    if (l + 1 == h->levels.size()) {
        const int maxit = std::max(2 * L.n, 100);
        const size_t lds = L.n <= kLdsCoarse ? sizeof(double) * 5 * L.n : 0;
        if (L.n <= kWave && L.max_row <= kWaveRow) {
            const bool f64 = sizeof(T) == sizeof(double);
            FineCorr<double> fcd{};
            FineCorr<float> fcf{};
            if (f64) fcd = {(double *)fc.e, fc.start, fc.cells};
            else fcf = {(float *)fc.e, fc.start, fc.cells};
            k_coarsest_wave<<<1, kWave, 0, st>>>(
                L.A.view(c.tr), f64 ? (const double *)r : nullptr,
                f64 ? nullptr : (const float *)r, f64 ? (double *)e : nullptr,
                f64 ? nullptr : (float *)e, L.singular, kCoarsestTol, maxit, c.dt, fcd, fcf,
                h->dev);
            if (corrected && fc.e) *corrected = true;
        } else
            k_coarsest<T, kWavesPerBlock><<<1, kBlock, lds, st>>>(L.A.view(c.tr), r, e, c.cw,
                                                                 L.singular, kCoarsestTol,
                                                                 maxit, c.dt, h->dev);
        HIP_CHECK(hipGetLastError());
        return e;
    }
    const SellView<T> A = lview<T>(L, c.tr);
    const int64_t S = L.A.nslices;
    const int G = stream_grid_slices(S);
    const T omega = (T)c.o->omega;
    const bool gs = c.o->smoother == LDU_SMOOTH_GS2;
    T *w1 = lvec<T>(L, 4);
    const bool rop = rop_cycle(*c.o) && L.r_ready && L.r_omega == c.o->omega &&
                     has_rop<T>(L, c.tr);
    // without correction scaling, on levels small enough to be bound by launch
    // latency, the coarse level applies e += P e_c itself (a scatter through
    // the member lists: on large levels the gather form of k_vc_correct moves
    // fewer bytes)
    const bool fuse_corr = !c.o->scale_correction && L.n <= kFuseCorrRows;
    // with the one-pass down leg nothing reads the first sweep before the
    // correction, which then forms it itself
    const bool defer_first = rop && !e_ready && !fuse_corr;
    if (gs) {  // forward two-stage Gauss-Seidel sweeps, the first from e = 0
        if (c.o->n_pre == 0) k_vc_zero<T><<<G, kBlock, 0, st>>>(L.n, S, e, h->dev);
        for (int k = 0; k < c.o->n_pre; ++k)
            gs_sweep<T>(A, r, e, t, e2, w1, k == 0, false, c.o->gs_inner, h->dev, G, st);
    } else {
        if (c.o->n_pre == 0) k_vc_zero<T><<<G, kBlock, 0, st>>>(L.n, S, e, h->dev);
        else if (!e_ready && !defer_first)
            k_vc_first<T><<<G, kBlock, 0, st>>>(L.n, S, r, A.diag, e, omega, h->dev);
        for (int k = 1; k < c.o->n_pre; ++k) {
            launch_jacobi<T>(A, r, e, e2, omega, nullptr, nullptr, {}, h->dev, G, st);
            std::swap(e, e2);
        }
    }
    Level &C = h->levels[l + 1];
    T *rc = lvec<T>(C, 0);
    // the coarse level's first Jacobi sweep rides on the restriction, unless
    // the coarse level will form it in its own correction (a large
    // non-coarsest level whose down leg also runs through R)
    const bool c_defers = l + 2 < h->levels.size() && rop && C.r_ready &&
                          C.r_omega == c.o->omega && has_rop<T>(C, c.tr) &&
                          C.n > kFuseCorrRows;
    const bool c_first = !gs && c.o->n_pre > 0 && l + 2 < h->levels.size() && !c_defers;
    T *ec_first = c_first ? lvec<T>(C, 1) : nullptr;
    if (rop) {
        if (L.ah) {  // t = (I - omega A D^-1) r over the level's slices, then its member sums
            SellView<T> Ah = A;
            Ah.val = ahval<T>(L, c.tr);
            if (Ah.c16)
                k_vc_ahat<true, T><<<G, kBlock, 0, st>>>(Ah, r, t, T(1) - omega, h->dev);
            else
                k_vc_ahat<false, T><<<G, kBlock, 0, st>>>(Ah, r, t, T(1) - omega, h->dev);
            k_vc_restrict<T><<<grid_n(C.n), kBlock, 0, st>>>(C.n, L.aggStart, L.aggCells, t, rc,
                                                            ec_first, lview<T>(C, c.tr).diag,
                                                            omega, h->dev);
        } else if (L.R.sptr) {  // residual and restriction in one pass over R (t is not formed)
            const SellView<T> R = rview<T>(L, c.tr);
            k_vc_rrestrict_cmp<T><<<stream_grid_slices(R.nslices), kBlock, 0, st>>>(
                R, r, rc, ec_first, lview<T>(C, c.tr).diag, omega, h->dev);
        } else {
            launch_rrestrict_csr<T>(rcview<T>(L, c.tr), r, rc, ec_first, lview<T>(C, c.tr).diag,
                                    omega, h->dev, st);
        }
    } else {
        if (A.pdeg) k_vc_resid<true, T><<<G, kBlock, 0, st>>>(A, r, e, t, h->dev);
        else k_vc_resid<false, T><<<G, kBlock, 0, st>>>(A, r, e, t, h->dev);
        k_vc_restrict<T><<<grid_n(C.n), kBlock, 0, st>>>(C.n, L.aggStart, L.aggCells, t, rc,
                                                        ec_first, lview<T>(C, c.tr).diag, omega,
                                                        h->dev);
    }
    bool done_corr = false;
    const T *ec = vcycle<T>(c, l + 1, rc, nullptr, nullptr, c_first,
                            fuse_corr ? FineCorr<T>{e, L.aggStart, L.aggCells} : FineCorr<T>{},
                            &done_corr);
    if (c.o->scale_correction) {
        if (A.pdeg) k_vc_scale<true, T><<<G, kBlock, 0, st>>>(A, ec, L.agg, t, h->partials, h->dev);
        else k_vc_scale<false, T><<<G, kBlock, 0, st>>>(A, ec, L.agg, t, h->partials, h->dev);
        launch_finalize<2>(h->partials, G, h->dev, EpiScale{}, st);
    }
    if (!done_corr)
        k_vc_correct<T><<<G, kBlock, 0, st>>>(L.n, S, ec, L.agg, e, c.o->scale_correction,
                                             defer_first ? r : nullptr, A.diag, omega, h->dev);
    for (int k = 0; k < c.o->n_post; ++k) {
        const bool last = k + 1 == c.o->n_post;
        if (gs) {  // backward sweeps: the V-cycle stays symmetric
            gs_sweep<T>(A, r, e, t, e2, w1, false, true, c.o->gs_inner, h->dev, G, st);
        } else {  // the last sweep may take the caller's dot product and correction
            launch_jacobi<T>(A, r, e, e2, omega, last ? rdot : nullptr, h->partials,
                             last ? fc : FineCorr<T>{}, h->dev, G, st);
            std::swap(e, e2);
            if (last && rdot && dotted) *dotted = true;
            if (last && fc.e && corrected) *corrected = true;
        }
    }
    HIP_CHECK(hipGetLastError());
    return e;
}

static void ensure_work32(ldu_t *h, hipStream_t st) {
    ensure_f32_levels(h, st);
    for (auto &L : h->levels) {
        if (!L.r32) {
            L.r32 = h->gamg_arena.get<float>(L.n);
            L.e32 = h->gamg_arena.get<float>(L.n);
            L.e232 = h->gamg_arena.get<float>(L.n);
            L.t32 = h->gamg_arena.get<float>(L.n);
        }
    }
}

// buffers and factors a cycle needs beyond the hierarchy: the second
// ping-pong vector of the two-stage smoother (three or more inner steps) and
// the DIC pivots of the coarsest level
// R's structure for level l (once per hierarchy): its slices and, per
// entry, the run of sources its value sums
static void rop_structure(ldu_t *h, size_t l, hipStream_t st) {
    Level &L = h->levels[l];
    const Level &C = h->levels[l + 1];
    if (!L.A.pdeg && C.n > kCsrMaxRows) {  // a large plain-slice level: Ah over its own slices
        L.ah = h->gamg_arena.get<double>(L.A.nnz);
        L.ahT = h->gamg_arena.get<double>(L.A.nnz);
        L.r_ready = false;
        return;
    }
    Arena tmp;
    int64_t *cnt = tmp.get<int64_t>(C.n);
    int64_t *tstart = tmp.get<int64_t>(C.n + 1);
    k_rop_count<<<grid_n(C.n), kBlock, 0, st>>>(C.n, L.aggStart, L.aggCells, L.A, cnt);
    exclusive_scan_i64(cnt, tstart, C.n, tmp, st);
    int64_t total = 0;
    HIP_CHECK(hipMemcpyAsync(&total, tstart + C.n, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipStreamSynchronize(st));
    int32_t *tcol = tmp.get<int32_t>(total);
    L.r_src = h->gamg_arena.get<int64_t>(total);
    int32_t *rdeg = tmp.get<int32_t>(C.n);
    k_rop_gather<<<grid_n(C.n), kBlock, 0, st>>>(C.n, L.aggStart, L.aggCells, L.A, tstart, tcol,
                                                L.r_src, rdeg);
    if (C.n > kCsrMaxRows) {
        build_sliced_rows(L.R, C.n, rdeg, h->gamg_arena, st);
        L.r_src0 = h->gamg_arena.get<int64_t>(L.R.nnz);
        L.r_srcn = h->gamg_arena.get<int32_t>(L.R.nnz);
        k_rop_link_sell<<<grid_n(C.n), kBlock, 0, st>>>(C.n, L.R, tstart, tcol, L.r_src0,
                                                        L.r_srcn);
    } else {
        Csr &R = L.Rc;
        R = Csr{};
        R.n = C.n;
        R.rptr = h->gamg_arena.get<int64_t>((size_t)C.n + 1);
        int64_t *rdeg64 = tmp.get<int64_t>(C.n);
        k_widen<<<grid_n(C.n), kBlock, 0, st>>>(C.n, rdeg, rdeg64);
        exclusive_scan_i64(rdeg64, R.rptr, C.n, tmp, st);
        HIP_CHECK(hipMemcpyAsync(&R.nnz, R.rptr + C.n, sizeof(int64_t), hipMemcpyDeviceToHost,
                                 st));
        HIP_CHECK(hipStreamSynchronize(st));
        R.col = h->gamg_arena.get<int32_t>(R.nnz);
        R.val = h->gamg_arena.get<double>(R.nnz);
        R.valT = h->gamg_arena.get<double>(R.nnz);
        // lanes per row: the power of two nearest mean length / entries per lane
        const double per = (double)R.nnz / std::max<int32_t>(C.n, 1) / kCsrEntriesPerLane;
        int g = 1;
        while (g < 16 && 2.0 * g <= per * 1.41421356) g *= 2;
        R.group = g;
        L.r_src0 = h->gamg_arena.get<int64_t>(R.nnz);
        L.r_srcn = h->gamg_arena.get<int32_t>(R.nnz);
        k_rop_link_csr<<<grid_n(C.n), kBlock, 0, st>>>(C.n, R, tstart, tcol, L.r_src0, L.r_srcn);
    }
    HIP_CHECK(hipGetLastError());
    HIP_CHECK(hipStreamSynchronize(st));  // tmp is released after this point
    L.r_ready = false;
}

// R's values (and their FP32 copies, when present) for the given omega
static void rop_values(Level &L, double omega, hipStream_t st) {
    if (L.ah) {
        const int64_t nnz = L.A.nnz;
        k_ahat_values<<<grid_n(nnz), kBlock, 0, st>>>(nnz, L.A.col, L.A.val, L.A.valT, L.A.diag,
                                                      omega, L.ah, L.ahT);
        if (L.ah32) {
            k_rop_f32<<<grid_n(nnz), kBlock, 0, st>>>(L.ah, L.ah32, nnz);
            k_rop_f32<<<grid_n(nnz), kBlock, 0, st>>>(L.ahT, L.ahT32, nnz);
        }
        HIP_CHECK(hipGetLastError());
        L.r_omega = omega;
        L.r_ready = true;
        return;
    }
    auto fill = [&](auto &R) {
        k_rop_values<<<grid_n(R.nnz), kBlock, 0, st>>>(R.nnz, R, L.r_src0, L.r_srcn, L.r_src,
                                                      L.A.val, L.A.valT, L.A.diag, omega);
        if (R.val32) {
            k_rop_f32<<<grid_n(R.nnz), kBlock, 0, st>>>(R.val, R.val32, R.nnz);
            k_rop_f32<<<grid_n(R.nnz), kBlock, 0, st>>>(R.valT, R.valT32, R.nnz);
        }
    };
    if (L.R.sptr) fill(L.R);
    else fill(L.Rc);
    HIP_CHECK(hipGetLastError());
    L.r_omega = omega;
    L.r_ready = true;
}

// R for every level but the coarsest, for the cycles whose down leg it
// replaces: structure once per hierarchy, values again after new
// coefficients or another omega, FP32 copies once the FP32 path is in use
static void ensure_rop(ldu_t *h, const ldu_gamg_opts &o, hipStream_t st) {
    if (!rop_cycle(o)) return;
    const bool f32 = h->L0.A.val32 != nullptr;
    for (size_t l = 0; l + 1 < h->levels.size(); ++l) {
        Level &L = h->levels[l];
        if (!L.R.sptr && !L.Rc.rptr && !L.ah) rop_structure(h, l, st);
        const bool fresh = L.r_ready && L.r_omega == o.omega;
        if (!fresh) rop_values(L, o.omega, st);
        auto f32_copies = [&](auto &R) {
            if (!f32 || R.val32) return;  // values are current: only the FP32 copies are new
            R.val32 = h->gamg_arena.get<float>(R.nnz);
            R.valT32 = h->gamg_arena.get<float>(R.nnz);
            k_rop_f32<<<grid_n(R.nnz), kBlock, 0, st>>>(R.val, R.val32, R.nnz);
            k_rop_f32<<<grid_n(R.nnz), kBlock, 0, st>>>(R.valT, R.valT32, R.nnz);
        };
        if (L.ah) {
            if (f32 && !L.ah32) {
                L.ah32 = h->gamg_arena.get<float>(L.A.nnz);
                L.ahT32 = h->gamg_arena.get<float>(L.A.nnz);
                k_rop_f32<<<grid_n(L.A.nnz), kBlock, 0, st>>>(L.ah, L.ah32, L.A.nnz);
                k_rop_f32<<<grid_n(L.A.nnz), kBlock, 0, st>>>(L.ahT, L.ahT32, L.A.nnz);
            }
        } else if (L.R.sptr) {
            f32_copies(L.R);
        } else {
            f32_copies(L.Rc);
        }
        HIP_CHECK(hipGetLastError());
    }
}

// new level coefficients: R's values follow at once (same omega)
static void refresh_rop(ldu_t *h, hipStream_t st) {
    for (size_t l = 0; l + 1 < h->levels.size(); ++l)
        if ((h->levels[l].R.sptr || h->levels[l].Rc.rptr || h->levels[l].ah) &&
            h->levels[l].r_ready)
            rop_values(h->levels[l], h->levels[l].r_omega, st);
}

static VCtx make_ctx(ldu_t *h, const ldu_gamg_opts &o, bool tr, hipStream_t st) {
    ensure_rop(h, o, st);
    if (o.smoother == LDU_SMOOTH_GS2 && o.gs_inner >= 3) {
        for (auto &L : h->levels) {
            if (!L.w) L.w = h->gamg_arena.get<double>(L.n);
            if (!L.w32) L.w32 = h->gamg_arena.get<float>(L.n);
        }
    }
    const double *dt = nullptr;
    if (o.coarsest == LDU_COARSE_DIC) {
        ensure_dic(h, st);
        if (h->dic_ok) dt = h->dic_dt;
    }
    return VCtx{h, &o, tr, st, h->coarse_work, dt};
}

static void fill_level_stats(ldu_t *h, ldu_stats *stats) {
    if (!stats) return;
    stats->n_levels = (int)h->levels.size();
    for (int l = 0; l < 64; ++l) {
        const bool in = l < (int)h->levels.size();
        stats->level_cells[l] = in ? h->levels[l].n : 0;
        stats->level_faces[l] = in ? h->levels[l].nf : 0;
    }
}

void gamg_vcycle64(ldu_t *h, const double *r, double *e, const ldu_gamg_opts &o, bool tr,
                   hipStream_t st) {
    set_scalars_for_solve(h, 0.0, 0, st);
    VCtx c = make_ctx(h, o, tr, st);
    double *res = vcycle<double>(c, 0, r);
    HIP_CHECK(hipMemcpyAsync(e, res, sizeof(double) * h->L0.n, hipMemcpyDeviceToDevice, st));
    HIP_CHECK(hipStreamSynchronize(st));
}

static int finish_status(const DevScalars &hs) {
    if (hs.done == kFailed) return hs.status;
    if (hs.done == kMaxIter) return LDU_NOT_CONVERGED;
    return LDU_OK;
}

int gamg_fp64(ldu_t *h, const double *b, double *x, const ldu_gamg_opts &o, bool tr,
              ldu_stats *stats, hipStream_t st) {
    Level &L = h->levels[0];
    const SellView<double> A = L.A.view(tr);
    const int64_t S = L.A.nslices;
    const int G = stream_grid_slices(S);
    ensure_hist(h, (int64_t)o.max_cycles + 2);
    fill_level_stats(h, stats);
    if (stats) { stats->refinements = 0; stats->history_count = 0; }
    set_scalars_for_solve(h, o.rel_tol, o.max_cycles, st);
    VCtx c = make_ctx(h, o, tr, st);
    launch_residual_cycle(h, A, b, x, h->r, false, G, st);
    read_scalars(h, st);
    DevScalars &hs = *h->host;
    if (stats) stats->initial_residual = hs.res;
    if (hs.bnorm == 0.0) {
        zero_vector(x, L.n, st);
        if (stats) {
            stats->iterations = 0;
            stats->converged = 1;
            stats->initial_residual = stats->final_residual = 0.0;
        }
        copy_history(h, stats, 1, st);
        return LDU_OK;
    }
    while (hs.done == kRunning) {
        const double *e = vcycle<double>(c, 0, h->r);
        k_add<<<G, kBlock, 0, st>>>(L.n, S, e, x, h->dev);
        launch_residual_cycle(h, A, b, x, h->r, false, G, st);
        read_scalars(h, st);
    }
    const int status = finish_status(hs);
    if (stats) {
        stats->iterations = hs.iters;
        stats->final_residual = hs.res;
        stats->converged = (status == LDU_OK);
    }
    copy_history(h, stats, hs.iters + 1, st);
    return status;
}

// ---------------------------------------------------------------- CG + V-cycle
// CG preconditioned by one V-cycle per iteration, correction scaling off so
// that the preconditioner is one fixed symmetric operator: the pairing of the
// paper's AmgX configuration (Appendix A listing: PCG with an AMG V-cycle
// preconditioner) on this GAMG hierarchy.

// p = z; rho = r.z
__global__ void __launch_bounds__(kBlock)
k_pg_start(int32_t n, int64_t S, const double *__restrict__ r, const double *__restrict__ z,
           double *__restrict__ p, double *partials, const DevScalars *ds) {
    if (ds->done) return;
    const int lane = threadIdx.x & 63;
    double acc[1] = {0.0};
    for_each_slice(S, [&](int64_t s) {
        const int64_t i = s * kWave + lane;
        if (i < n) {
            const double zi = z[i];
            p[i] = zi;
            acc[0] += r[i] * zi;
        }
    });
    block_partials<1>(acc, partials);
}

struct EpiRho {
    __device__ bool active(const DevScalars *ds) const { return !ds->done; }
    __device__ void operator()(const double *t, DevScalars *ds) const {
        ds->rho = t[0];
        ds->x_pending = 0;
    }
};

// r -= alpha q; ||r||^2.  The iteration's x += alpha p waits for the
// direction update, which reads p anyway (k_pg_p), or, when the solve stops
// in between, for k_x_pending: one read of p per iteration instead of two.
template <bool NT>
__global__ void __launch_bounds__(kBlock)
k_pg_update(int32_t n, int64_t S, double *__restrict__ r, const double *__restrict__ q,
            double *partials, const DevScalars *ds) {
    if (ds->done) return;
    const double alpha = ds->alpha;
    const int lane = threadIdx.x & 63;
    double acc[1] = {0.0};
    for_each_slice(S, [&](int64_t s) {
        const int64_t i = s * kWave + lane;
        if (i < n) {
            const double ri = vld<NT>(r + i) - alpha * vld<NT>(q + i);
            vst<NT>(r + i, ri);
            acc[0] += ri * ri;
        }
    });
    block_partials<1>(acc, partials);
}


// rho' = r.z; beta = rho'/rho
__global__ void __launch_bounds__(kBlock)
k_pg_rz(int32_t n, int64_t S, const double *__restrict__ r, const double *__restrict__ z,
        double *partials, const DevScalars *ds) {
    if (ds->done) return;
    const int lane = threadIdx.x & 63;
    double acc[1] = {0.0};
    for_each_slice(S, [&](int64_t s) {
        const int64_t i = s * kWave + lane;
        if (i < n) acc[0] += r[i] * z[i];
    });
    block_partials<1>(acc, partials);
}

struct EpiBeta {
    __device__ bool active(const DevScalars *ds) const { return !ds->done; }
    __device__ void operator()(const double *t, DevScalars *ds) const {
        ds->beta = t[0] / ds->rho;
        ds->rho = t[0];
        ds->x_pending = 0;  // k_pg_p applies it next
    }
};

// x += alpha p (the iteration's solution update, deferred from k_pg_update);
// p = z + beta p.  x and z are not read again before the next iteration's
// direction update, so they stream past the caches (nontemporal) at every
// size, while p keeps the default policy at every size: the new p, which the
// CG product gathers next, then stays in the Infinity Cache (the c3 CG
// product went from 133 to 122 us).
__global__ void __launch_bounds__(kBlock)
k_pg_p(int32_t n, int64_t S, double *__restrict__ x, const double *__restrict__ z,
       double *__restrict__ p, const DevScalars *ds) {
    if (ds->done) return;
    const double alpha = ds->alpha, beta = ds->beta;
    const int lane = threadIdx.x & 63;
    for_each_slice(S, [&](int64_t s) {
        const int64_t i = s * kWave + lane;
        if (i < n) {
            const double pi = p[i];
            vst<true>(x + i, vld<true>(x + i) + alpha * pi);
            p[i] = vld<true>(z + i) + beta * pi;
        }
    });
}

int pcg_gamg_fp64(ldu_t *h, const double *b, double *x, const ldu_pcg_opts &o, bool tr,
                  ldu_stats *stats, hipStream_t st) {
    ldu_gamg_opts go = h->gamg_opts;
    go.scale_correction = 0;
    Level &L = h->levels[0];
    const SellView<double> A = L.A.view(tr);
    const int n = L.n;
    const int64_t S = L.A.nslices;
    const int G = stream_grid_slices(S);
    const bool nt = n > kStreamNtCells;
    ensure_hist(h, (int64_t)o.max_iter + 2);
    fill_level_stats(h, stats);
    if (stats) { stats->refinements = 0; stats->history_count = 0; }
    set_scalars_for_solve(h, o.rel_tol, o.max_iter, st);
    VCtx c = make_ctx(h, go, tr, st);
    launch_residual_plain(h, A, b, x, h->r, true, G, st);
    read_scalars(h, st);
    DevScalars &hs = *h->host;
    if (stats) stats->initial_residual = hs.res;
    if (hs.bnorm == 0.0) {
        zero_vector(x, n, st);
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
        const double *z = vcycle<double>(c, 0, h->r);
        k_pg_start<<<G, kBlock, 0, st>>>(n, S, h->r, z, h->p, h->partials, h->dev);
        launch_finalize<1>(h->partials, G, h->dev, EpiRho{}, st);
        for (;;) {
            for (int k = 0; k < every; ++k) {
                launch_pcg_q(h, A, h->p, h->q, G, st);
                if (nt)
                    k_pg_update<true><<<G, kBlock, 0, st>>>(n, S, h->r, h->q, h->partials,
                                                            h->dev);
                else
                    k_pg_update<false><<<G, kBlock, 0, st>>>(n, S, h->r, h->q, h->partials,
                                                             h->dev);
                launch_converge(h, G, false, st);
                bool dotted = false;
                z = vcycle<double>(c, 0, h->r, h->r, &dotted);
                if (!dotted) k_pg_rz<<<G, kBlock, 0, st>>>(n, S, h->r, z, h->partials, h->dev);
                launch_finalize<1>(h->partials, G, h->dev, EpiBeta{}, st);
                k_pg_p<<<G, kBlock, 0, st>>>(n, S, x, z, h->p, h->dev);
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
        launch_residual_plain(h, A, b, x, h->r, false, G, st);
        read_scalars(h, st);
        res = hs.res;
        if (!std::isfinite(res)) { status = LDU_ERR_NAN; break; }
        if (res <= o.rel_tol) { status = LDU_OK; break; }
        if (hs.iters >= o.max_iter) { status = LDU_NOT_CONVERGED; break; }
        set_done(h, kRunning, st);
    }
    if (stats) {
        stats->iterations = hs.iters;
        stats->final_residual = res;
        stats->converged = (status == LDU_OK);
    }
    copy_history(h, stats, hs.iters + 1, st);
    return status;
}

// FP32 inner CG preconditioned by an FP32 V-cycle (FP64 coarsest), inside FP64
// refinement; inner dot products in FP64, alpha/beta rounded to FP32

// rhat = fp32(r / ||r||_inf), d = 0; ||rhat||^2
__global__ void __launch_bounds__(kBlock)
k_mxg_start(int32_t n, int64_t S, const double *__restrict__ r, float *__restrict__ r32,
            float *__restrict__ d32, double *partials, const DevScalars *ds) {
    if (ds->done) return;
    const double sc = ds->maxabs;
    const int lane = threadIdx.x & 63;
    double acc[2] = {0.0, 0.0};
    for_each_slice(S, [&](int64_t s) {
        const int64_t i = s * kWave + lane;
        if (i < n) {
            const float ri = (float)(r[i] / sc);
            r32[i] = ri;
            d32[i] = 0.0f;
            acc[0] += (double)ri * (double)ri;
        }
    });
    block_partials<2>(acc, partials);
}

// p = z; rho = r.z (FP32 vectors, FP64 sum)
__global__ void __launch_bounds__(kBlock)
k_mxg_p0(int32_t n, int64_t S, const float *__restrict__ r, const float *__restrict__ z,
         float *__restrict__ p, double *partials, const DevScalars *ds) {
    if (vc_skip(ds)) return;
    const int lane = threadIdx.x & 63;
    double acc[1] = {0.0};
    for_each_slice(S, [&](int64_t s) {
        const int64_t i = s * kWave + lane;
        if (i < n) {
            p[i] = z[i];
            acc[0] += (double)r[i] * (double)z[i];
        }
    });
    block_partials<1>(acc, partials);
}

struct EpiMxRho {
    __device__ bool active(const DevScalars *ds) const { return !vc_skip(ds); }
    __device__ void operator()(const double *t, DevScalars *ds) const { ds->rho = t[0]; }
};

// rho' = r.z -> beta (FP64), then p = z + fp32(beta) p in the next kernel
__global__ void __launch_bounds__(kBlock)
k_mxg_rz(int32_t n, int64_t S, const float *__restrict__ r, const float *__restrict__ z,
         double *partials, const DevScalars *ds) {
    if (vc_skip(ds)) return;
    const int lane = threadIdx.x & 63;
    double acc[1] = {0.0};
    for_each_slice(S, [&](int64_t s) {
        const int64_t i = s * kWave + lane;
        if (i < n) acc[0] += (double)r[i] * (double)z[i];
    });
    block_partials<1>(acc, partials);
}

struct EpiMxBeta {
    __device__ bool active(const DevScalars *ds) const { return !vc_skip(ds); }
    __device__ void operator()(const double *t, DevScalars *ds) const {
        ds->beta = t[0] / ds->rho;
        ds->rho = t[0];
    }
};

__global__ void __launch_bounds__(kBlock)
k_mxg_p(int32_t n, int64_t S, const float *__restrict__ z, float *__restrict__ p,
        const DevScalars *ds) {
    if (vc_skip(ds)) return;
    const float bf = (float)ds->beta;
    const int lane = threadIdx.x & 63;
    for_each_slice(S, [&](int64_t s) {
        const int64_t i = s * kWave + lane;
        if (i < n) p[i] = z[i] + bf * p[i];
    });
}

struct EpiMxgStart {
    __device__ bool active(const DevScalars *ds) const { return !ds->done; }
    __device__ void operator()(const double *t, DevScalars *ds) const {
        ds->scale = ds->maxabs;
        ds->r0 = sqrt(t[0]);
        ds->inner_iters = 0;
        ds->inner_done = !(ds->r0 > 0.0);
        const double target = 0.3 * ds->tol / ds->res;
        ds->inner_now = target > ds->inner_tol ? target : ds->inner_tol;
    }
};

int pcg_gamg_mixed(ldu_t *h, const double *b, double *x, const ldu_pcg_opts &o, bool tr,
                   ldu_stats *stats, hipStream_t st) {
    ensure_work32(h, st);
    ldu_gamg_opts go = h->gamg_opts;
    go.scale_correction = 0;
    Level &L = h->levels[0];
    const SellView<double> A = L.A.view(tr);
    const SellView<float> A32 = L.A.view32(tr);
    const int n = L.n;
    const int64_t S = L.A.nslices;
    const int G = stream_grid_slices(S);
    ensure_hist(h, (int64_t)o.max_refine + 2);
    fill_level_stats(h, stats);
    if (stats) stats->history_count = 0;
    set_scalars_for_solve(h, o.rel_tol, o.max_refine, st);
    set_inner(h, o.inner_rel_tol, o.inner_max_iter, st);
    VCtx c = make_ctx(h, go, tr, st);
    launch_residual_cycle(h, A, b, x, h->r, true, G, st);
    read_scalars(h, st);
    DevScalars &hs = *h->host;
    if (stats) stats->initial_residual = hs.res;
    if (hs.bnorm == 0.0) {
        zero_vector(x, n, st);
        if (stats) {
            stats->iterations = 0;
            stats->refinements = 0;
            stats->converged = 1;
            stats->initial_residual = stats->final_residual = 0.0;
        }
        copy_history(h, stats, 1, st);
        return LDU_OK;
    }
    const int every = o.check_every > 0 ? o.check_every : 16;
    long long inner_total = 0;
    while (hs.done == kRunning) {
        k_mxg_start<<<G, kBlock, 0, st>>>(n, S, h->r, h->r32, h->d32, h->partials, h->dev);
        launch_finalize<2>(h->partials, G, h->dev, EpiMxgStart{}, st);
        const float *z = vcycle<float>(c, 0, h->r32);
        k_mxg_p0<<<G, kBlock, 0, st>>>(n, S, h->r32, z, h->p32, h->partials, h->dev);
        launch_finalize<1>(h->partials, G, h->dev, EpiMxRho{}, st);
        for (;;) {
            for (int k = 0; k < every; ++k) {
                launch_mx_q(h, A32, G, st);
                launch_mx_update_plain(h, n, S, G, st);
                bool dotted = false;  // the last level-0 sweep may take r.z itself
                z = vcycle<float>(c, 0, h->r32, h->r32, &dotted);
                if (!dotted) k_mxg_rz<<<G, kBlock, 0, st>>>(n, S, h->r32, z, h->partials, h->dev);
                launch_finalize<1>(h->partials, G, h->dev, EpiMxBeta{}, st);
                k_mxg_p<<<G, kBlock, 0, st>>>(n, S, z, h->p32, h->dev);
            }
            HIP_CHECK(hipGetLastError());
            read_scalars(h, st);
            if (hs.inner_done) break;
        }
        inner_total += hs.inner_iters;
        launch_mx_refine(h, x, n, S, G, st);
        launch_residual_cycle(h, A, b, x, h->r, true, G, st);
        read_scalars(h, st);
    }
    const int status = finish_status(hs);
    if (stats) {
        stats->iterations = (int)inner_total;
        stats->refinements = hs.iters;
        stats->final_residual = hs.res;
        stats->converged = (status == LDU_OK);
    }
    copy_history(h, stats, hs.iters + 1, st);
    return status;
}

int gamg_mixed(ldu_t *h, const double *b, double *x, const ldu_gamg_opts &o, bool tr,
               ldu_stats *stats, hipStream_t st) {
    ensure_work32(h, st);
    Level &L = h->levels[0];
    const SellView<double> A = L.A.view(tr);
    const int64_t S = L.A.nslices;
    const int G = stream_grid_slices(S);
    ensure_hist(h, (int64_t)o.max_refine + 2);
    fill_level_stats(h, stats);
    if (stats) stats->history_count = 0;
    set_scalars_for_solve(h, o.rel_tol, o.max_refine, st);
    VCtx c = make_ctx(h, o, tr, st);
    launch_residual_cycle(h, A, b, x, h->r, true, G, st);
    read_scalars(h, st);
    DevScalars &hs = *h->host;
    if (stats) stats->initial_residual = hs.res;
    if (hs.bnorm == 0.0) {
        zero_vector(x, L.n, st);
        if (stats) {
            stats->iterations = 0;
            stats->refinements = 0;
            stats->converged = 1;
            stats->initial_residual = stats->final_residual = 0.0;
        }
        copy_history(h, stats, 1, st);
        return LDU_OK;
    }
    while (hs.done == kRunning) {
        k_cast_scaled<<<G, kBlock, 0, st>>>(L.n, S, h->r, L.r32, h->dev);
        const float *d = vcycle<float>(c, 0, L.r32);
        k_refine_add<<<G, kBlock, 0, st>>>(L.n, S, d, x, h->dev);
        launch_residual_cycle(h, A, b, x, h->r, true, G, st);
        read_scalars(h, st);
    }
    const int status = finish_status(hs);
    if (stats) {
        stats->iterations = hs.iters;
        stats->refinements = hs.iters;
        stats->final_residual = hs.res;
        stats->converged = (status == LDU_OK);
    }
    copy_history(h, stats, hs.iters + 1, st);
    return status;
}

}  // namespace ldu
