// Device-side building blocks shared by the kernels of the library.
//
// - for_each_slice: XCD-aware work distribution.  MI355X dispatches
//   consecutive workgroups round-robin over its 8 XCDs, each with its own L2.
//   Large grids are therefore split into 8 contiguous row ranges, one per
//   XCD, and the workgroups of an XCD sweep their range front to back; the
//   +-nx*ny neighbour band of a cell is then read from the L2 that fetched it
//   instead of the L2 of another XCD.
// - deterministic reductions: a fixed butterfly inside the wavefront, a fixed
//   order across the 4 wavefronts of a block, one partial per block, and a
//   one-block finalize kernel that sums the partials in a fixed order.
//   Results are bitwise reproducible run to run; no floating-point atomics.
// - sell_row: one row of a sliced-ELLPACK product, diagonal first and then
//   the entries in column order, each product rounded before its addition
//   (the library is compiled without FMA contraction), which is exactly the
//   rounding sequence of the lduMatrix face loop for that row.
#pragma once

#include "internal.hpp"

namespace ldu {

// The slices a wave walks, for a grid of G blocks: with G a multiple of 8
// (and at least 64) block b works in XCD b % 8's contiguous eighth of the
// slices [lo, hi), starting at group j with stride Gx groups of
// kWavesPerBlock slices; wave w of the block takes slice lo + g * 4 + w.
struct SliceWalkRange {
    int64_t lo, hi, j, Gx;
    int w;
};
__device__ __forceinline__ SliceWalkRange slice_walk_range(int64_t S, int G) {
    const int nx = (G >= 64 && (G & 7) == 0) ? 8 : 1;
    const int64_t x = blockIdx.x % nx;
    const int64_t R = (S + nx - 1) / nx;
    SliceWalkRange r;
    r.lo = x * R;
    r.hi = (r.lo + R < S) ? r.lo + R : S;
    r.j = blockIdx.x / nx;
    r.Gx = G / nx;
    r.w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
    return r;
}

// true once the solve has stopped (done) or the current inner solve of a
// mixed-precision solve has (inner_done, always 0 in FP64 solves): the
// kernels of an iteration then return at once.  Both flags are read unconditionally (bitwise or), so
// their two scalar loads share one round trip at kernel start instead of
// running in sequence.
__device__ __forceinline__ bool vc_skip(const DevScalars *ds) {
    return (ds->done | ds->inner_done) != 0;
}

template <int CAP = 0, class F>
__device__ __forceinline__ void for_each_slice(int64_t S, F &&f) {
    int G = gridDim.x;
    if (CAP > 0 && G > CAP) {  // only the first CAP blocks walk slices
        if ((int)blockIdx.x >= CAP) return;
        G = CAP;
    }
    const SliceWalkRange r = slice_walk_range(S, G);
    for (int64_t g = r.j; r.lo + g * kWavesPerBlock < r.hi; g += r.Gx) {
        const int64_t s = r.lo + g * kWavesPerBlock + r.w;
        if (s < r.hi) f(s);
    }
}

// active-block cap of a product kernel over level matrix A (see
// kPlainF64ProductBlocks); 0: every block walks slices
template <bool CMP, typename T>
constexpr int product_cap() {
    return (!CMP && sizeof(T) == 8) ? kPlainF64ProductBlocks : 0;
}

// Wavefront reductions with DPP lane moves (no LDS round trips): pairs and
// quads (quad_perm), the 16-lane rows (row_ror 4, 8), then row 0 into row 1
// and row 2 into row 3 (row_bcast 15), rows 0-1 into rows 2-3 (row_bcast
// 31); lane 63 ends with the total, which every lane then reads.  The order
// is fixed, so results are reproducible.  A lane the move does not write
// keeps `old` (0 for sums, its own value for maxima).
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ double dpp_move(double v, double old) {
    const int lo = __builtin_amdgcn_update_dpp(__double2loint(old), __double2loint(v), CTRL,
                                               ROW_MASK, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(__double2hiint(old), __double2hiint(v), CTRL,
                                               ROW_MASK, 0xf, false);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double lane63(double v) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double wave_sum(double v) {
    v = v + dpp_move<0xB1>(v, 0.0);        // quad_perm [1,0,3,2]
    v = v + dpp_move<0x4E>(v, 0.0);        // quad_perm [2,3,0,1]
    v = v + dpp_move<0x124>(v, 0.0);       // row_ror 4
    v = v + dpp_move<0x128>(v, 0.0);       // row_ror 8
    v = v + dpp_move<0x142, 0xa>(v, 0.0);  // row_bcast 15
    v = v + dpp_move<0x143, 0xc>(v, 0.0);  // row_bcast 31
    return lane63(v);
}
__device__ __forceinline__ double wave_max(double v) {
    v = fmax(v, dpp_move<0xB1>(v, v));
    v = fmax(v, dpp_move<0x4E>(v, v));
    v = fmax(v, dpp_move<0x124>(v, v));
    v = fmax(v, dpp_move<0x128>(v, v));
    v = fmax(v, dpp_move<0x142, 0xa>(v, v));
    v = fmax(v, dpp_move<0x143, 0xc>(v, v));
    return lane63(v);
}

// block-wide reduction of K values (slots >= K - M take the max, the others
// the sum); the result is valid in thread 0
template <int K, int M = 0>
__device__ __forceinline__ void block_reduce(double (&v)[K]) {
    __shared__ double sm[K][kWavesPerBlock];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = (k >= K - M) ? wave_max(v[k]) : wave_sum(v[k]);
    __syncthreads();
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) sm[k][w] = v[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k)
            v[k] = (k >= K - M) ? fmax(fmax(sm[k][0], sm[k][1]), fmax(sm[k][2], sm[k][3]))
                                : ((sm[k][0] + sm[k][1]) + sm[k][2]) + sm[k][3];
    }
}

// grid-wide reductions in two launches: every block of the producer kernel
// stores its block total in partials[k * kMaxGrid + block] (plain stores; the
// kernel boundary makes them visible), then k_finalize, one block, sums the
// partials in a fixed order and runs the epilogue.  A single-kernel variant
// needs an agent-scope release per block, which on this chip writes back L2
// and cost ~60% of a streaming kernel's time.
template <int K, int M = 0>
__device__ __forceinline__ void block_partials(double (&v)[K], double *partials) {
    block_reduce<K, M>(v);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) partials[k * kMaxGrid + blockIdx.x] = v[k];
    }
}

template <int K, int M, class Epi>
__global__ void __launch_bounds__(kBlock)
k_finalize(const double *__restrict__ partials, int nblocks, DevScalars *ds, Epi epi) {
    if (!epi.active(ds)) return;
    double s[K];
#pragma unroll
    for (int k = 0; k < K; ++k) s[k] = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += kBlock) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const double p = partials[k * kMaxGrid + b];
            s[k] = (k >= K - M) ? fmax(s[k], p) : s[k] + p;
        }
    }
    block_reduce<K, M>(s);
    if (threadIdx.x == 0) epi(s, ds);
}

template <int K, int M = 0, class Epi>
inline void launch_finalize(double *partials, int nblocks, DevScalars *ds, const Epi &epi,
                            hipStream_t st) {
    k_finalize<K, M, Epi><<<1, kBlock, 0, st>>>(partials, nblocks, ds, epi);
}

// Loads and stores of the level-0 vector streams.  NT: nontemporal, for
// vectors too large to stay in the 256 MB Infinity Cache between kernels
// (kStreamNtCells); below that the plain forms keep them there.
template <bool NT, typename T>
__device__ __forceinline__ T vld(const T *p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}
template <bool NT, typename T>
__device__ __forceinline__ void vst(T *p, T v) {
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

// row stored at slice position p, and the slice position of row i
template <bool CMP, typename T>
__device__ __forceinline__ int32_t sv_row(const SellView<T> &A, int64_t p) {
    if constexpr (CMP) return A.perm[p];
    else return (int32_t)p;
}
template <typename T>
__device__ __forceinline__ int64_t sv_pos(const SellView<T> &A, int32_t i) {
    return A.iperm ? (int64_t)A.iperm[i] : (int64_t)i;
}

// x accessors for the product kernels
template <typename T>
struct Direct {
    const T *x;
    __device__ __forceinline__ T operator()(int32_t j) const { return x[j]; }
};
template <typename T>
struct ViaAgg {  // prolonged vector c_j = ec[agg[j]]
    const T *ec;
    const int32_t *agg;
    __device__ __forceinline__ T operator()(int32_t j) const { return ec[agg[j]]; }
};

// Offsets of a compressed slice's entries.  Rows are sorted by length
// within the slice (longest first), so the entries of column k are those of
// the first cnt_k lanes, cnt_k = #{lanes with length > k}, stored after the
// entries of columns 0..k-1.  A wave that holds the whole slice (every lane
// with entries active) counts cnt_k with a ballot and keeps the running
// offset in a scalar register: no offset table loads on the dependent path
// from the slice header to the gathers.  Row-per-lane callers, whose lanes
// belong to different slices, read the slice's offset table instead (TABLE).
struct SliceOffsets {
    int64_t off = 0;
    __device__ __forceinline__ int64_t next(bool has) {
        const int64_t o = off;
        off += __popcll(__ballot(has));
        return o;
    }
};

// A wave's walk over the slots of a plain slice s (slot k: the k-th entries
// of the slice's rows; the slot count is the slice width, wave-uniform, so
// the slot bases come from scalar loads).  C16: columns are the slot base
// plus a 16-bit offset.
template <bool C16, typename T>
struct PlainWalk {
    const int32_t *cp;
    const uint16_t *hp;
    const T *vp;
    const int32_t *bp;
    int w;

    __device__ __forceinline__ PlainWalk(const SellView<T> &A, int64_t s, int lane) {
        const int64_t b0 = A.sptr[s];
        cp = A.col + b0 + lane;
        hp = C16 ? A.c16 + b0 + lane : nullptr;
        vp = A.val + b0 + lane;
        w = (int)((A.sptr[s + 1] - b0) >> 6);
        bp = C16 ? A.cbase + (b0 >> 6) : nullptr;
    }
    // stored column (16-bit offset or 32-bit column), slot base and value of
    // slot k; the column is formed later (column()), so that the vector
    // loads of a whole batch are in flight before the first wait on them.
    // The base is a scalar load per slot: those of one slice share a scalar
    // cache line.  (Reading a fixed batch of bases per step instead measured
    // slower, with more HBM traffic.)  A slot too wide for 16-bit offsets has
    // base -1 and reads the 32-bit columns (a wave-uniform branch).
    __device__ __forceinline__ void load(int k, int32_t &raw, int32_t &base, T &v) const {
        const int64_t o = (int64_t)k * kWave;
        if constexpr (C16) {
            base = bp[k];
            if (base >= 0) raw = (int32_t)__builtin_nontemporal_load(hp + o);
            else raw = __builtin_nontemporal_load(cp + o);
        } else {
            base = 0;
            raw = __builtin_nontemporal_load(cp + o);
        }
        v = __builtin_nontemporal_load(vp + o);
    }
    static __device__ __forceinline__ int32_t column(int32_t raw, int32_t base) {
        return C16 && base >= 0 ? base + raw : raw;
    }
};

template <bool C16, int B, typename T, class XA, class F>
__device__ __forceinline__ void plain_entries(const SellView<T> &A, int64_t s, int lane,
                                              const XA &xa, F &&f) {
    const PlainWalk<C16, T> pw(A, s, lane);
    for (int k = 0; k < pw.w; k += B) {
        int32_t c[B], cb[B];
        T v[B];
#pragma unroll
        for (int u = 0; u < B; ++u)
            if (k + u < pw.w) pw.load(k + u, c[u], cb[u], v[u]);
        T xv[B];
#pragma unroll
        for (int u = 0; u < B; ++u) {
            if (k + u < pw.w) {
                c[u] = PlainWalk<C16, T>::column(c[u], cb[u]);
                xv[u] = xa(c[u]);
            }
        }
#pragma unroll
        for (int u = 0; u < B; ++u)
            if (k + u < pw.w) f(c[u], v[u], xv[u]);
    }
}

// the entries of a compressed-slice row whose slice starts at b0 and whose
// length is w (see cmp_entries)
template <int B, typename T, class XA, class F>
__device__ __forceinline__ void cmp_entries_at(const SellView<T> &A, int64_t b0, int w, int lane,
                                               const XA &xa, F &&f) {
    const int32_t *cp = A.col + b0 + lane;
    const T *vp = A.val + b0 + lane;
    SliceOffsets so;
    for (int k = 0; k < w; k += B) {
        int32_t c[B];
        T v[B];
#pragma unroll
        for (int u = 0; u < B; ++u) {
            const bool has = k + u < w;
            const int64_t o = so.next(has);
            if (has) {
                c[u] = __builtin_nontemporal_load(cp + o);
                v[u] = __builtin_nontemporal_load(vp + o);
            }
        }
        T xv[B];
#pragma unroll
        for (int u = 0; u < B; ++u)
            if (k + u < w) xv[u] = xa(c[u]);
#pragma unroll
        for (int u = 0; u < B; ++u)
            if (k + u < w) f(c[u], v[u], xv[u]);
    }
}

// the off-diagonal entries of the row at slice position 64 s + lane, loaded
// B at a time: f(column, value, x[column]) for each, in column order.  Plain
// slices walk their slots with PlainWalk; compressed slices loop per lane to
// the row's own length, with ballot-counted offsets.
template <int B, typename T, class XA, class F>
__device__ __forceinline__ void cmp_entries(const SellView<T> &A, int64_t s, int lane,
                                            const XA &xa, F &&f) {
    cmp_entries_at<B>(A, A.sptr[s], A.pdeg[s * kWave + lane], lane, xa, f);
}

// The header of a compressed slice as one lane needs it: the slice start, and
// the length and row index of the lane's row (0 and -1 past the level's last
// row: pdeg and perm cover whole slices).
struct CmpHead {
    int64_t b0 = 0;
    int w = 0;
    int32_t row = -1;
};

template <typename T>
__device__ __forceinline__ CmpHead cmp_head(const SellView<T> &A, int64_t s, int lane) {
    CmpHead h;
    const int64_t p = s * kWave + lane;
    h.b0 = A.sptr[s];
    h.w = A.pdeg[p];
    h.row = A.perm[p];
    return h;
}

// for_each_slice over compressed slices, software-pipelined: the header of a
// wave's next slice is loaded before the current slice is processed, so its
// round trip overlaps the current slice's entry loads and gathers.
// f(s, head); lanes whose head.row is -1 hold no row.
template <typename T, class F>
__device__ __forceinline__ void for_each_cmp_slice(const SellView<T> &A, F &&f) {
    const int lane = threadIdx.x & 63;
    const SliceWalkRange r = slice_walk_range(A.nslices, gridDim.x);
    CmpHead h;
    {
        const int64_t s0 = r.lo + r.j * kWavesPerBlock + r.w;
        if (s0 < r.hi) h = cmp_head(A, s0, lane);
    }
    for (int64_t g = r.j; r.lo + g * kWavesPerBlock < r.hi; g += r.Gx) {
        const int64_t s = r.lo + g * kWavesPerBlock + r.w;
        const int64_t sn = s + r.Gx * kWavesPerBlock;
        CmpHead hn;
        if (sn < r.hi) hn = cmp_head(A, sn, lane);
        if (s < r.hi) f(s, h);
        h = hn;
    }
}

template <bool CMP, int B, typename T, class XA, class F>
__device__ __forceinline__ void row_entries(const SellView<T> &A, int64_t s, int lane,
                                            const XA &xa, F &&f) {
    if constexpr (CMP) {
        cmp_entries<B>(A, s, lane, xa, f);
    } else {
        if (A.c16) plain_entries<true, B>(A, s, lane, xa, f);
        else plain_entries<false, B>(A, s, lane, xa, f);
    }
}

// (A x)_i for the row i stored at position 64 s + lane of slice s; CMP
// selects the compressed-slice layout at compile time (each layout gets its
// own kernels, so the plain one keeps its register budget and occupancy).
// Without TABLE every lane of the slice that holds a row must be active;
// TABLE serves row-per-lane callers (lanes in different slices) from the
// 32-bit columns and the offset table.
template <bool CMP, typename T, class XA, bool TABLE = false>
__device__ __forceinline__ T sell_row(const SellView<T> &A, int64_t s, int lane,
                                      int32_t i, const XA &xa) {
    if constexpr (!TABLE) {
        T acc = A.diag[i] * xa(i);
        row_entries<CMP, CMP ? kCmpBatch : 8>(A, s, lane, xa, [&](int32_t, T v, T xv) {
            acc = acc + v * xv;
        });
        return acc;
    } else {
        const int64_t b0 = A.sptr[s];
        T acc = A.diag[i] * xa(i);
        const int32_t *cp = A.col + b0 + lane;
        const T *vp = A.val + b0 + lane;
        int w;
        const int32_t *ot = nullptr;
        if constexpr (CMP) {
            w = A.pdeg[s * kWave + lane];
            ot = A.otab + A.tptr[s];
        } else {
            w = (int)((A.sptr[s + 1] - b0) >> 6);
        }
        for (int k = 0; k < w; ++k) {
            const int64_t o = CMP ? (int64_t)ot[k] : (int64_t)k * kWave;
            acc = acc + vp[o] * xa(cp[o]);
        }
        return acc;
    }
}

// strictly lower (UPPER false: columns < i) or strictly upper (columns > i)
// part of row i applied to x, summed from zero in column order; padding
// entries (column == i) drop out with the mask.  Every lane of the slice
// that holds a row must be active.
template <bool CMP, bool UPPER, typename T, class XA>
__device__ __forceinline__ T sell_tri(const SellView<T> &A, int64_t s, int lane, int32_t i,
                                      const XA &xa) {
    T acc = T(0);
    row_entries<CMP, 8>(A, s, lane, xa, [&](int32_t c, T v, T xv) {
        if (UPPER ? c > i : c < i) acc = acc + v * xv;
    });
    return acc;
}

// either layout, decided at run time, for row-per-lane callers (setup
// kernels, the block coarsest solve)
template <typename T, class XA>
__device__ __forceinline__ T sell_row_any(const SellView<T> &A, int64_t s, int lane, int32_t i,
                                          const XA &xa) {
    return A.pdeg ? sell_row<true, T, XA, true>(A, s, lane, i, xa)
                  : sell_row<false, T, XA, true>(A, s, lane, i, xa);
}

// entry count of the row at slice position p, and the storage index of its
// k-th entry (either layout)
template <class M>
__device__ __forceinline__ int row_len(const M &A, int64_t p) {
    if (A.pdeg) return A.pdeg[p];
    const int64_t s = p >> 6;
    return (int)((A.sptr[s + 1] - A.sptr[s]) >> 6);  // includes padding (col == row)
}
template <class M>
__device__ __forceinline__ int64_t entry_at(const M &A, int64_t p, int k) {
    const int64_t s = p >> 6, lane = p & 63;
    if (A.pdeg) return A.sptr[s] + A.otab[A.tptr[s] + k] + lane;
    return A.sptr[s] + (int64_t)k * kWave + lane;
}

}  // namespace ldu
