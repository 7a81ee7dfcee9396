// LDU -> sliced-ELLPACK re-layout, value maps and scans (setup kernels).
//
// The paper's external-solver path converts OpenFOAM's LDU arrays to a
// row-ordered (CSR) matrix through a permutation map computed once and reused
// when the values change (Sec. 3.4).  Here the same idea produces the
// row-segmented layout the product kernels stream: per row its "lower"
// entries (faces where the row is the neighbour, i.e. OpenFOAM's losort
// order) followed by its "upper" entries (faces it owns), column-sorted, and
// two face -> position maps (slotU, slotL) so that new coefficients are
// scattered in place without redoing the structure.
#include "device.hpp"

#include <algorithm>

namespace ldu {

// ---------------------------------------------------------------- scans
constexpr int kScanItems = 8;
constexpr int kScanChunk = kBlock * kScanItems;

template <typename T>
__device__ T block_exclusive_scan(T v, T *total) {
    __shared__ T sm[kBlock];
    sm[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < kBlock; off <<= 1) {
        T a = (threadIdx.x >= (unsigned)off) ? sm[threadIdx.x - off] : T(0);
        __syncthreads();
        sm[threadIdx.x] += a;
        __syncthreads();
    }
    T incl = sm[threadIdx.x];
    *total = sm[kBlock - 1];
    __syncthreads();
    return incl - v;
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_scan_partial(const T *in, int64_t n, T *bsum) {
    const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanItems;
    T s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k)
        if (base + k < n) s += in[base + k];
    T tot;
    block_exclusive_scan<T>(s, &tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// exclusive scan of nb block sums by one block (in place), total -> bsum[nb]
template <typename T>
__global__ void __launch_bounds__(kBlock) k_scan_sums(T *bsum, int64_t nb) {
    const int64_t per = (nb + kBlock - 1) / kBlock;
    const int64_t lo = (int64_t)threadIdx.x * per;
    T s = 0;
    for (int64_t k = lo; k < lo + per && k < nb; ++k) s += bsum[k];
    T tot;
    T off = block_exclusive_scan<T>(s, &tot);
    for (int64_t k = lo; k < lo + per && k < nb; ++k) {
        T v = bsum[k];
        bsum[k] = off;
        off += v;
    }
    if (threadIdx.x == 0) bsum[nb] = tot;
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_scan_final(const T *in, int64_t n, const T *bsum, T *out) {
    const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanItems;
    T v[kScanItems];
    T s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = (base + k < n) ? in[base + k] : T(0);
        s += v[k];
    }
    T tot;
    T off = block_exclusive_scan<T>(s, &tot) + bsum[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < n) out[base + k] = off;
        off += v[k];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[n] = bsum[gridDim.x];
}

template <typename T>
static void exclusive_scan(const T *in, T *out, int64_t n, Arena &tmp, hipStream_t st) {
    const int64_t nb = (n + kScanChunk - 1) / kScanChunk;
    if (nb == 0) {
        HIP_CHECK(hipMemsetAsync(out, 0, sizeof(T), st));
        return;
    }
    T *bsum = tmp.get<T>(nb + 1);
    k_scan_partial<T><<<(unsigned)nb, kBlock, 0, st>>>(in, n, bsum);
    k_scan_sums<T><<<1, kBlock, 0, st>>>(bsum, nb);
    k_scan_final<T><<<(unsigned)nb, kBlock, 0, st>>>(in, n, bsum, out);
    HIP_CHECK(hipGetLastError());
}

void exclusive_scan_i64(const int64_t *in, int64_t *out, int64_t n, Arena &tmp,
                        hipStream_t st) {
    exclusive_scan<int64_t>(in, out, n, tmp, st);
}
void scan_counts_i32(const int32_t *cnt, int32_t *out, int64_t n, Arena &tmp,
                     hipStream_t st) {
    exclusive_scan<int32_t>(cnt, out, n, tmp, st);
}

// ---------------------------------------------------------------- checks
__global__ void k_validate(int32_t n, int64_t nf, const int32_t *own, const int32_t *nb,
                           int *flag) {
    for (int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; f < nf;
         f += (int64_t)gridDim.x * blockDim.x) {
        const int32_t o = own[f], b = nb[f];
        bool bad = o < 0 || o >= b || b >= n;
        if (f > 0) {
            const int32_t po = own[f - 1], pb = nb[f - 1];
            bad = bad || o < po || (o == po && b <= pb);
        }
        if (bad) atomicOr(flag, 1);
    }
}

__global__ void k_check_finite(const double *a, int64_t n, int *flag) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        if (!isfinite(a[i])) atomicOr(flag, 2);
}

static unsigned grid_for(int64_t n) {
    int64_t g = (n + kBlock - 1) / kBlock;
    if (g > 8192) g = 8192;
    return (unsigned)(g < 1 ? 1 : g);
}

void check_finite(ldu_t *h, const double *a, int64_t n, hipStream_t st) {
    if (n > 0) k_check_finite<<<grid_for(n), kBlock, 0, st>>>(a, n, h->flag);
}

// ---------------------------------------------------------------- structure
// ownStart[i] = first face with owner >= i (faces are sorted by owner)
__global__ void k_own_start(int32_t n, int64_t nf, const int32_t *own, int64_t *ownStart) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i <= n;
         i += (int64_t)gridDim.x * blockDim.x) {
        int64_t lo = 0, hi = nf;
        while (lo < hi) {
            int64_t mid = (lo + hi) >> 1;
            if (own[mid] < i) lo = mid + 1; else hi = mid;
        }
        ownStart[i] = lo;
    }
}

__global__ void k_count_lower(int64_t nf, const int32_t *nb, int32_t *cntL) {
    for (int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; f < nf;
         f += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(&cntL[nb[f]], 1);
}

__global__ void k_degree(int32_t n, const int64_t *ownStart, const int32_t *cntL, int32_t *deg) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        deg[i] = cntL[i] + (int32_t)(ownStart[i + 1] - ownStart[i]);
}

// entries of slice s = 64 x (longest row stored in the slice)
__global__ void k_slice_entries(int32_t n, int64_t S, const int32_t *deg, const int32_t *perm,
                                int64_t *entries) {
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < S;
         s += (int64_t)gridDim.x * blockDim.x) {
        int64_t w = 0;
        for (int l = 0; l < kWave; ++l) {
            const int64_t p = s * kWave + l;
            if (p < n) {
                const int64_t d = deg[perm ? perm[p] : p];
                w = d > w ? d : w;
            }
        }
        entries[s] = w * kWave;
    }
}

// compressed slices: inside each slice of 64 rows, order the rows by length
// (longest first, ties by row index); positions past n hold no row (-1)
__global__ void k_slice_sort(int32_t n, int64_t S, const int32_t *deg, int32_t *perm,
                             int32_t *iperm, int32_t *pdeg) {
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < S * kWave;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t s0 = (q >> 6) << 6;
        const int l = (int)(q & 63);
        const int32_t dl = q < n ? deg[q] : -1;
        int rank = 0;
        for (int j = 0; j < kWave; ++j) {
            const int32_t dj = (s0 + j) < n ? deg[s0 + j] : -1;
            rank += (dj > dl) || (dj == dl && j < l);
        }
        perm[s0 + rank] = q < n ? (int32_t)q : -1;
        pdeg[s0 + rank] = dl > 0 ? dl : 0;
        if (q < n) iperm[q] = (int32_t)(s0 + rank);
    }
}

// entries of a compressed slice (sum of its row lengths) and the length of
// its offset table (longest row + 1)
__global__ void k_slice_sizes(int64_t S, const int32_t *pdeg, int64_t *entries, int32_t *tlen) {
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < S;
         s += (int64_t)gridDim.x * blockDim.x) {
        int64_t e = 0;
        for (int l = 0; l < kWave; ++l) e += pdeg[s * kWave + l];
        entries[s] = e;
        tlen[s] = pdeg[s * kWave] + 1;
    }
}

// otab[tptr[s] + k] = entries of slice s in its columns 0..k-1
__global__ void k_slice_table(int64_t S, const int32_t *pdeg, const int32_t *tptr, int32_t *otab) {
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < S;
         s += (int64_t)gridDim.x * blockDim.x) {
        const int w = pdeg[s * kWave];
        int32_t off = 0;
        for (int k = 0; k <= w; ++k) {
            otab[tptr[s] + k] = off;
            int cnt = 0;
            for (int l = 0; l < kWave; ++l) cnt += pdeg[s * kWave + l] > k;
            off += cnt;
        }
    }
}

// max of a[0..n) (values >= 0) into *out, which the caller zeroes: one
// partial per block, combined by an integer atomic max (order-independent)
__global__ void __launch_bounds__(kBlock) k_max_i32(const int32_t *a, int64_t n, int32_t *out) {
    __shared__ int32_t sm[kBlock];
    int32_t m = 0;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock)
        m = a[i] > m ? a[i] : m;
    sm[threadIdx.x] = m;
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
        if (threadIdx.x < (unsigned)off && sm[threadIdx.x + off] > sm[threadIdx.x])
            sm[threadIdx.x] = sm[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicMax(out, sm[0]);
}

__global__ void k_fill_i32(int32_t *a, int64_t n, int32_t v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        a[i] = v;
}

// storage index of entry k of row i (plain or compressed slices)
struct Slots {
    const int64_t *sptr;
    const int32_t *iperm, *tptr, *otab;
    __device__ __forceinline__ int64_t operator()(int64_t i, int64_t k) const {
        const int64_t p = iperm ? (int64_t)iperm[i] : i;
        const int64_t s = p >> 6;
        if (otab) return sptr[s] + otab[tptr[s] + k] + (p & 63);
        return sptr[s] + k * kWave + (p & 63);
    }
};

__global__ void k_fill_upper(int64_t nf, const int32_t *own, const int32_t *nb,
                             const int64_t *ownStart, const int32_t *cntL, Slots slot,
                             int32_t *col, int64_t *slotU) {
    for (int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; f < nf;
         f += (int64_t)gridDim.x * blockDim.x) {
        const int32_t i = own[f];
        const int64_t pos = slot(i, cntL[i] + (f - ownStart[i]));
        col[pos] = nb[f];
        slotU[f] = pos;
    }
}

// lower entries land in arbitrary order within their row; k_sort_lower
// orders them by column, which makes the final layout deterministic
__global__ void k_fill_lower(int64_t nf, const int32_t *own, const int32_t *nb, Slots slot,
                             int32_t *cursor, int32_t *col, int64_t *faceAt) {
    for (int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; f < nf;
         f += (int64_t)gridDim.x * blockDim.x) {
        const int32_t j = nb[f];
        const int k = atomicAdd(&cursor[j], 1);
        const int64_t pos = slot(j, k);
        col[pos] = own[f];
        faceAt[pos] = f;
    }
}

__global__ void k_sort_lower(int32_t n, Slots slot, const int32_t *cntL, int32_t *col,
                             int64_t *faceAt, int64_t *slotL) {
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * blockDim.x) {
        const int m = cntL[j];
        for (int a = 1; a < m; ++a) {  // insertion sort by column
            const int64_t pa = slot(j, a);
            const int32_t c = col[pa];
            const int64_t fa = faceAt[pa];
            int b = a - 1;
            while (b >= 0 && col[slot(j, b)] > c) {
                const int64_t pb = slot(j, b), pn = slot(j, b + 1);
                col[pn] = col[pb];
                faceAt[pn] = faceAt[pb];
                --b;
            }
            const int64_t pn = slot(j, b + 1);
            col[pn] = c;
            faceAt[pn] = fa;
        }
        for (int a = 0; a < m; ++a) {
            const int64_t pa = slot(j, a);
            slotL[faceAt[pa]] = pa;
        }
    }
}

// plain slices: padding entries point at their own row with value 0
// (positions past n: row 0)
__global__ void k_fill_pad(int32_t n, int64_t S, const int64_t *sptr, const int32_t *deg,
                           int32_t *col, double *val, double *valT) {
    const int64_t rows = S * kWave;
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < rows;
         p += (int64_t)gridDim.x * blockDim.x) {
        const int64_t s = p >> 6;
        const int64_t w = (sptr[s + 1] - sptr[s]) >> 6;
        const int64_t d = (p < n) ? deg[p] : 0;
        for (int64_t k = d; k < w; ++k) {
            const int64_t pos = sptr[s] + k * kWave + (p & 63);
            col[pos] = (p < n) ? (int32_t)p : 0;
            val[pos] = 0.0;
            valT[pos] = 0.0;
        }
    }
}

__global__ void k_set_values(int64_t nf, const int64_t *slotU, const int64_t *slotL,
                             const double *upper, const double *lower, double *val,
                             double *valT) {
    for (int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; f < nf;
         f += (int64_t)gridDim.x * blockDim.x) {
        const double u = upper[f], l = lower[f];
        const int64_t pu = slotU[f], pl = slotL[f];
        val[pu] = u;
        val[pl] = l;
        valT[pu] = l;
        valT[pl] = u;
    }
}

// slot bases for 16-bit columns: the smallest column of each slot, and a
// flag when some slot spans more than 65535 columns
__device__ __forceinline__ void slot_span(const int64_t *sptr, const int32_t *pdeg,
                                          const int32_t *tptr, const int32_t *otab, int64_t s,
                                          int k, int64_t &e0, int &cnt, int64_t &bi) {
    if (pdeg) {
        const int32_t *ot = otab + tptr[s];
        e0 = sptr[s] + ot[k];
        cnt = ot[k + 1] - ot[k];
        bi = tptr[s] + k;
    } else {
        e0 = sptr[s] + (int64_t)k * kWave;
        cnt = kWave;
        bi = (sptr[s] >> 6) + k;
    }
}

__global__ void k_col16_bases(int64_t S, const int64_t *sptr, const int32_t *pdeg,
                              const int32_t *tptr, const int32_t *otab, const int32_t *col,
                              int32_t *cbase, unsigned long long *narrow) {
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < S;
         s += (int64_t)gridDim.x * blockDim.x) {
        const int w = pdeg ? pdeg[s * kWave] : (int)((sptr[s + 1] - sptr[s]) >> 6);
        for (int k = 0; k < w; ++k) {
            int64_t e0, bi;
            int cnt;
            slot_span(sptr, pdeg, tptr, otab, s, k, e0, cnt, bi);
            int32_t lo = col[e0], hi = col[e0];
            for (int l = 1; l < cnt; ++l) {
                const int32_t c = col[e0 + l];
                lo = c < lo ? c : lo;
                hi = c > hi ? c : hi;
            }
            const bool fits = (int64_t)hi - lo <= 65535;
            cbase[bi] = fits ? lo : -1;  // -1: this slot reads the 32-bit columns
            if (fits) atomicAdd(narrow, 1ull);
        }
    }
}

__global__ void k_col16_fill(int64_t S, const int64_t *sptr, const int32_t *pdeg,
                             const int32_t *tptr, const int32_t *otab, const int32_t *col,
                             const int32_t *cbase, uint16_t *c16) {
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < S;
         s += (int64_t)gridDim.x * blockDim.x) {
        const int w = pdeg ? pdeg[s * kWave] : (int)((sptr[s + 1] - sptr[s]) >> 6);
        for (int k = 0; k < w; ++k) {
            int64_t e0, bi;
            int cnt;
            slot_span(sptr, pdeg, tptr, otab, s, k, e0, cnt, bi);
            const int32_t b = cbase[bi];
            for (int l = 0; l < cnt; ++l) c16[e0 + l] = b >= 0 ? (uint16_t)(col[e0 + l] - b) : 0;
        }
    }
}

// 16-bit columns for the slots narrow enough, on a level that has any
static void build_col16(Sell &A, int64_t nslots, Arena &ar, Arena &tmp, hipStream_t st) {
    A.c16 = nullptr;
    A.cbase = nullptr;
    // plain slices only: in compressed slices the slot bases cost more than
    // the narrower columns save (measured on the Galerkin levels)
    if (A.nnz == 0 || nslots == 0 || A.pdeg) return;
    int32_t *cbase = ar.get<int32_t>(nslots);
    unsigned long long *narrow = tmp.get<unsigned long long>(1);
    HIP_CHECK(hipMemsetAsync(narrow, 0, sizeof(unsigned long long), st));
    k_col16_bases<<<grid_for(A.nslices), kBlock, 0, st>>>(A.nslices, A.sptr, A.pdeg, A.tptr,
                                                         A.otab, A.col, cbase, narrow);
    unsigned long long hnarrow = 0;
    HIP_CHECK(hipMemcpyAsync(&hnarrow, narrow, sizeof(hnarrow), hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipStreamSynchronize(st));
    if (hnarrow == 0) return;
    uint16_t *c16 = ar.get<uint16_t>(A.nnz);
    k_col16_fill<<<grid_for(A.nslices), kBlock, 0, st>>>(A.nslices, A.sptr, A.pdeg, A.tptr,
                                                        A.otab, A.col, cbase, c16);
    HIP_CHECK(hipGetLastError());
    A.c16 = c16;
    A.cbase = cbase;
}

__global__ void k_to_f32(const double *a, float *b, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        b[i] = (float)a[i];
}

void build_level_sell(ldu_t *h, Arena &ar, Level &L, bool validate, hipStream_t st) {
    const int32_t n = L.n;
    const int64_t nf = L.nf;
    const int64_t S = slices_of(n);
    Arena tmp;
    if (validate) {
        HIP_CHECK(hipMemsetAsync(h->flag, 0, sizeof(int), st));
        if (nf > 0)
            k_validate<<<grid_for(nf), kBlock, 0, st>>>(n, nf, L.own, L.nb, h->flag);
        check_finite(h, L.diag, n, st);
        check_finite(h, L.upper, nf, st);
        check_finite(h, L.lower, nf, st);
        HIP_CHECK(hipMemcpyAsync(h->hflag, h->flag, sizeof(int), hipMemcpyDeviceToHost, st));
        HIP_CHECK(hipStreamSynchronize(st));
        if (*h->hflag & 1) throw Error(LDU_ERR_ADDR, "face addressing violates 0 <= owner < neighbour < nCells, sorted by (owner, neighbour), no duplicates");
        if (*h->hflag & 2) throw Error(LDU_ERR_NAN, "non-finite coefficient");
    }
    L.ownStart = ar.get<int64_t>(n + 1);
    k_own_start<<<grid_for(n + 1), kBlock, 0, st>>>(n, nf, L.own, L.ownStart);
    int32_t *cntL = tmp.get<int32_t>(n);
    HIP_CHECK(hipMemsetAsync(cntL, 0, sizeof(int32_t) * n, st));
    if (nf > 0) k_count_lower<<<grid_for(nf), kBlock, 0, st>>>(nf, L.nb, cntL);
    int32_t *deg = tmp.get<int32_t>(n);
    k_degree<<<grid_for(n), kBlock, 0, st>>>(n, L.ownStart, cntL, deg);
    int64_t *entries = tmp.get<int64_t>(S);
    L.A.sptr = ar.get<int64_t>(S + 1);
    k_slice_entries<<<grid_for(S), kBlock, 0, st>>>(n, S, deg, nullptr, entries);
    exclusive_scan_i64(entries, L.A.sptr, S, tmp, st);
    int64_t nnz = 0;
    HIP_CHECK(hipMemcpyAsync(&nnz, L.A.sptr + S, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipStreamSynchronize(st));
    L.A.perm = L.A.iperm = L.A.pdeg = L.A.tptr = L.A.otab = nullptr;
    int64_t nslots = nnz / kWave;  // plain slices: one slot per 64 entries
    if (nnz * 100 > 103 * std::max<int64_t>(2 * nf, kWave)) {
        // rows of uneven length: compressed slices, lanes ordered by length
        L.A.perm = ar.get<int32_t>(S * kWave);
        L.A.iperm = ar.get<int32_t>(n);
        L.A.pdeg = ar.get<int32_t>(S * kWave);
        k_slice_sort<<<grid_for(S * kWave), kBlock, 0, st>>>(n, S, deg, L.A.perm, L.A.iperm,
                                                             L.A.pdeg);
        int32_t *tlen = tmp.get<int32_t>(S);
        k_slice_sizes<<<grid_for(S), kBlock, 0, st>>>(S, L.A.pdeg, entries, tlen);
        exclusive_scan_i64(entries, L.A.sptr, S, tmp, st);
        L.A.tptr = ar.get<int32_t>(S + 1);
        scan_counts_i32(tlen, L.A.tptr, S, tmp, st);
        int32_t ntab = 0;
        HIP_CHECK(hipMemcpyAsync(&ntab, L.A.tptr + S, sizeof(int32_t), hipMemcpyDeviceToHost,
                                 st));
        HIP_CHECK(hipMemcpyAsync(&nnz, L.A.sptr + S, sizeof(int64_t), hipMemcpyDeviceToHost,
                                 st));
        HIP_CHECK(hipStreamSynchronize(st));
        L.A.otab = ar.get<int32_t>(ntab);
        nslots = ntab;
        k_slice_table<<<grid_for(S), kBlock, 0, st>>>(S, L.A.pdeg, L.A.tptr, L.A.otab);
    }
    {  // longest row, for kernels that stage a whole row
        int32_t *dmax = tmp.get<int32_t>(1);
        k_fill_i32<<<1, kBlock, 0, st>>>(dmax, 1, 0);
        k_max_i32<<<grid_for(n), kBlock, 0, st>>>(deg, n, dmax);
        HIP_CHECK(hipMemcpyAsync(&L.max_row, dmax, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        HIP_CHECK(hipStreamSynchronize(st));
    }
    L.A.n = n;
    L.A.nslices = S;
    L.A.nnz = nnz;
    L.A.col = ar.get<int32_t>(nnz);
    L.A.val = ar.get<double>(nnz);
    L.A.valT = ar.get<double>(nnz);
    L.A.diag = L.diag;
    L.slotU = ar.get<int64_t>(nf);
    L.slotL = ar.get<int64_t>(nf);
    if (nf > 0) {
        const Slots slot{L.A.sptr, L.A.iperm, L.A.tptr, L.A.otab};
        k_fill_upper<<<grid_for(nf), kBlock, 0, st>>>(nf, L.own, L.nb, L.ownStart, cntL, slot,
                                                     L.A.col, L.slotU);
        int32_t *cursor = tmp.get<int32_t>(n);
        int64_t *faceAt = tmp.get<int64_t>(nnz);
        HIP_CHECK(hipMemsetAsync(cursor, 0, sizeof(int32_t) * n, st));
        k_fill_lower<<<grid_for(nf), kBlock, 0, st>>>(nf, L.own, L.nb, slot, cursor, L.A.col,
                                                     faceAt);
        k_sort_lower<<<grid_for(n), kBlock, 0, st>>>(n, slot, cntL, L.A.col, faceAt, L.slotL);
    }
    if (!L.A.pdeg)
        k_fill_pad<<<grid_for(S * kWave), kBlock, 0, st>>>(n, S, L.A.sptr, deg, L.A.col, L.A.val,
                                                          L.A.valT);
    HIP_CHECK(hipGetLastError());
    build_col16(L.A, nslots, ar, tmp, st);
    set_level_values(L, st);
    HIP_CHECK(hipStreamSynchronize(st));  // tmp is released after this point
}

// compressed slices for n rows of the given lengths (device array): the
// lane order, slice starts and offset tables, and uninitialised col, val and
// valT arrays of the total entry count (no diagonal)
void build_sliced_rows(Sell &A, int32_t n, const int32_t *deg, Arena &ar, hipStream_t st) {
    Arena tmp;
    const int64_t S = slices_of(n);
    A = Sell{};
    A.n = n;
    A.nslices = S;
    A.perm = ar.get<int32_t>(S * kWave);
    A.iperm = ar.get<int32_t>(n);
    A.pdeg = ar.get<int32_t>(S * kWave);
    k_slice_sort<<<grid_for(S * kWave), kBlock, 0, st>>>(n, S, deg, A.perm, A.iperm, A.pdeg);
    int64_t *entries = tmp.get<int64_t>(S);
    int32_t *tlen = tmp.get<int32_t>(S);
    k_slice_sizes<<<grid_for(S), kBlock, 0, st>>>(S, A.pdeg, entries, tlen);
    A.sptr = ar.get<int64_t>(S + 1);
    exclusive_scan_i64(entries, A.sptr, S, tmp, st);
    A.tptr = ar.get<int32_t>(S + 1);
    scan_counts_i32(tlen, A.tptr, S, tmp, st);
    int32_t ntab = 0;
    int64_t nnz = 0;
    HIP_CHECK(hipMemcpyAsync(&ntab, A.tptr + S, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipMemcpyAsync(&nnz, A.sptr + S, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipStreamSynchronize(st));
    A.otab = ar.get<int32_t>(ntab);
    k_slice_table<<<grid_for(S), kBlock, 0, st>>>(S, A.pdeg, A.tptr, A.otab);
    A.nnz = nnz;
    A.col = ar.get<int32_t>(nnz);
    A.val = ar.get<double>(nnz);
    A.valT = ar.get<double>(nnz);
    HIP_CHECK(hipGetLastError());
    HIP_CHECK(hipStreamSynchronize(st));  // tmp is released after this point
}

void set_level_values(Level &L, hipStream_t st) {
    if (L.nf > 0)
        k_set_values<<<grid_for(L.nf), kBlock, 0, st>>>(L.nf, L.slotU, L.slotL, L.upper,
                                                        L.lower, L.A.val, L.A.valT);
    HIP_CHECK(hipGetLastError());
}

void refresh_f32(Level &L, hipStream_t st) {
    if (!L.A.val32) return;
    k_to_f32<<<grid_for(L.A.nnz), kBlock, 0, st>>>(L.A.val, L.A.val32, L.A.nnz);
    k_to_f32<<<grid_for(L.A.nnz), kBlock, 0, st>>>(L.A.valT, L.A.valT32, L.A.nnz);
    k_to_f32<<<grid_for(L.n), kBlock, 0, st>>>(L.diag, L.A.diag32, L.n);
    HIP_CHECK(hipGetLastError());
}

void ensure_f32(Level &L, Arena &ar, hipStream_t st) {
    if (L.A.val32) return;
    L.A.val32 = ar.get<float>(L.A.nnz);
    L.A.valT32 = ar.get<float>(L.A.nnz);
    L.A.diag32 = ar.get<float>(L.n);
    refresh_f32(L, st);
}

}  // namespace ldu
