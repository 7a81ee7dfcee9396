// Bandwidth ceilings of plain HBM streams, timed beside the solver kernels:
// a read-only sum, a copy, and an update shaped like the CG's x/r step
// (x += a p; r -= a q: four reads and two writes per cell).  They carry no
// index streams and no gathers, so what they reach is what a streaming
// kernel can draw from HBM on this device; the solver kernels are compared
// with it as well as with the vendor peak.
//
// Shape (the fastest of a sweep over grid-stride and chunked loops, 4-16
// loads in flight per thread, plain and nontemporal accesses, on MI355X):
// each block walks chunks of U x 256 16-byte elements, chunk c, c + grid,
// ...; thread t of the block loads elements t, t + 256, ... of the chunk, so
// one wave's loads cover contiguous 1 KiB runs and a thread keeps U loads in
// flight.  NT selects nontemporal loads and stores, which stream past the
// caches: faster for arrays well above the 256 MB Infinity Cache, slower for
// arrays that fit it.  Tails shorter than a 16-byte element are handled by
// the first thread.  Nothing is allocated: the read kernel writes one
// partial per block into the caller's array.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "ldu_bench.h"

namespace {

constexpr int kThreads = 256;

typedef double v2d __attribute__((ext_vector_type(2)));

template <bool NT>
__device__ __forceinline__ v2d ld2(const v2d *p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}
template <bool NT>
__device__ __forceinline__ void st2(v2d *p, v2d v) {
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

int grid_of(int blocks) {
    if (blocks <= 0) return 2048;
    return blocks > LDU_STREAM_MAX_BLOCKS ? LDU_STREAM_MAX_BLOCKS : blocks;
}

// chunks of U * kThreads elements; f(element index, u) for each of a
// thread's U elements of a full chunk, g(element index) for a partial one
template <int U, class F, class G>
__device__ __forceinline__ void for_each_chunk(int64_t n2, F &&f, G &&g) {
    const int64_t ch = (int64_t)U * kThreads;
    for (int64_t c = blockIdx.x; c * ch < n2; c += gridDim.x) {
        const int64_t b = c * ch + threadIdx.x;
        if (b + (int64_t)(U - 1) * kThreads < n2) {
            f(b);
        } else {
            for (int u = 0; u < U; ++u)
                if (b + (int64_t)u * kThreads < n2) g(b + (int64_t)u * kThreads);
        }
    }
}

template <bool NT>
__global__ void __launch_bounds__(kThreads) k_read(const v2d *__restrict__ a, int64_t n2,
                                                   const double *__restrict__ tail, int ntail,
                                                   double *out) {
    constexpr int U = 8;
    double s0 = 0.0, s1 = 0.0;
    for_each_chunk<U>(
        n2,
        [&](int64_t b) {
            v2d v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) v[u] = ld2<NT>(a + b + u * kThreads);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                s0 += v[u].x;
                s1 += v[u].y;
            }
        },
        [&](int64_t j) {
            const v2d v = a[j];
            s0 += v.x;
            s1 += v.y;
        });
    if (blockIdx.x == 0 && threadIdx.x == 0)
        for (int k = 0; k < ntail; ++k) s0 += tail[k];
    __shared__ double sm[kThreads];
    sm[threadIdx.x] = s0 + s1;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sm[threadIdx.x] += sm[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = sm[0];
}

template <bool NT>
__global__ void __launch_bounds__(kThreads) k_copy(const v2d *__restrict__ a, v2d *__restrict__ b,
                                                   int64_t n2, const double *__restrict__ ta,
                                                   double *__restrict__ tb, int ntail) {
    constexpr int U = 8;
    for_each_chunk<U>(
        n2,
        [&](int64_t j) {
            v2d v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) v[u] = ld2<NT>(a + j + u * kThreads);
#pragma unroll
            for (int u = 0; u < U; ++u) st2<NT>(b + j + u * kThreads, v[u]);
        },
        [&](int64_t j) { b[j] = a[j]; });
    if (blockIdx.x == 0 && threadIdx.x == 0)
        for (int k = 0; k < ntail; ++k) tb[k] = ta[k];
}

template <bool NT>
__global__ void __launch_bounds__(kThreads)
k_cg_update(v2d *__restrict__ x, v2d *__restrict__ r, const v2d *__restrict__ p,
            const v2d *__restrict__ q, double alpha, int64_t n2, double *__restrict__ tx,
            double *__restrict__ tr, const double *__restrict__ tp,
            const double *__restrict__ tq, int ntail) {
    constexpr int U = 2;
    for_each_chunk<U>(
        n2,
        [&](int64_t b) {
            v2d xv[U], rv[U], pv[U], qv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t j = b + u * kThreads;
                xv[u] = ld2<NT>(x + j);
                rv[u] = ld2<NT>(r + j);
                pv[u] = ld2<NT>(p + j);
                qv[u] = ld2<NT>(q + j);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t j = b + u * kThreads;
                st2<NT>(x + j, xv[u] + alpha * pv[u]);
                st2<NT>(r + j, rv[u] - alpha * qv[u]);
            }
        },
        [&](int64_t j) {
            x[j] = x[j] + alpha * p[j];
            r[j] = r[j] - alpha * q[j];
        });
    if (blockIdx.x == 0 && threadIdx.x == 0)
        for (int k = 0; k < ntail; ++k) {
            tx[k] = tx[k] + alpha * tp[k];
            tr[k] = tr[k] - alpha * tq[k];
        }
}

bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

int launched() { return hipGetLastError() == hipSuccess ? 0 : -6; }

hipStream_t S(void *s) { return reinterpret_cast<hipStream_t>(s); }

}  // namespace

extern "C" {

int ldu_stream_read(const double *a, int64_t n, double *partials, int blocks, int nontemporal,
                    void *hip_stream) {
    if (!a || !partials || n < 0 || !aligned16(a)) return -1;
    const int G = grid_of(blocks);
    const int64_t n2 = n / 2;
    const v2d *a2 = reinterpret_cast<const v2d *>(a);
    if (nontemporal)
        k_read<true><<<G, kThreads, 0, S(hip_stream)>>>(a2, n2, a + 2 * n2, (int)(n - 2 * n2),
                                                        partials);
    else
        k_read<false><<<G, kThreads, 0, S(hip_stream)>>>(a2, n2, a + 2 * n2, (int)(n - 2 * n2),
                                                         partials);
    return launched();
}

int ldu_stream_copy(const double *a, double *b, int64_t n, int blocks, int nontemporal,
                    void *hip_stream) {
    if (!a || !b || n < 0 || !aligned16(a) || !aligned16(b)) return -1;
    const int G = grid_of(blocks);
    const int64_t n2 = n / 2;
    const v2d *a2 = reinterpret_cast<const v2d *>(a);
    v2d *b2 = reinterpret_cast<v2d *>(b);
    if (nontemporal)
        k_copy<true><<<G, kThreads, 0, S(hip_stream)>>>(a2, b2, n2, a + 2 * n2, b + 2 * n2,
                                                        (int)(n - 2 * n2));
    else
        k_copy<false><<<G, kThreads, 0, S(hip_stream)>>>(a2, b2, n2, a + 2 * n2, b + 2 * n2,
                                                         (int)(n - 2 * n2));
    return launched();
}

int ldu_stream_cg_update(double *x, double *r, const double *p, const double *q, double alpha,
                         int64_t n, int blocks, int nontemporal, void *hip_stream) {
    if (!x || !r || !p || !q || n < 0 || !aligned16(x) || !aligned16(r) || !aligned16(p) ||
        !aligned16(q))
        return -1;
    const int G = grid_of(blocks);
    const int64_t n2 = n / 2;
    v2d *x2 = reinterpret_cast<v2d *>(x), *r2 = reinterpret_cast<v2d *>(r);
    const v2d *p2 = reinterpret_cast<const v2d *>(p), *q2 = reinterpret_cast<const v2d *>(q);
    const int nt = (int)(n - 2 * n2);
    if (nontemporal)
        k_cg_update<true><<<G, kThreads, 0, S(hip_stream)>>>(x2, r2, p2, q2, alpha, n2, x + 2 * n2,
                                                             r + 2 * n2, p + 2 * n2, q + 2 * n2, nt);
    else
        k_cg_update<false><<<G, kThreads, 0, S(hip_stream)>>>(
            x2, r2, p2, q2, alpha, n2, x + 2 * n2, r + 2 * n2, p + 2 * n2, q + 2 * n2, nt);
    return launched();
}

}  // extern "C"
