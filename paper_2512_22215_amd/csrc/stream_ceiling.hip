// Bandwidth ceilings of plain HBM streams, timed beside the solver kernels:
// a read-only sum, a copy, and an update shaped like the CG's x/r step
// (x += a p; r -= a q: four reads and two writes per cell).  They carry no
// index streams and no gathers, so what they reach is what a streaming
// kernel can draw from HBM on this device; the solver kernels are compared
// with it as well as with the vendor peak.
//
// Each thread moves 16 bytes per load (double2) and keeps UNROLL loads in
// flight over a grid-stride loop; tails shorter than a double2 are handled
// by the first thread.  Nothing is allocated: the read kernel writes one
// partial per block into the caller's array.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "ldu_bench.h"

namespace {

constexpr int kThreads = 256;
constexpr int kUnroll = 4;

int grid_of(int blocks) {
    if (blocks <= 0) return 2048;
    return blocks > LDU_STREAM_MAX_BLOCKS ? LDU_STREAM_MAX_BLOCKS : blocks;
}

__global__ void __launch_bounds__(kThreads) k_read(const double2 *__restrict__ a, int64_t n2,
                                                   const double *__restrict__ tail, int ntail,
                                                   double *out) {
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    double s0 = 0.0, s1 = 0.0;
    int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x;
    for (; i + (kUnroll - 1) * stride < n2; i += kUnroll * stride) {
        double2 v[kUnroll];
#pragma unroll
        for (int k = 0; k < kUnroll; ++k) v[k] = a[i + k * stride];
#pragma unroll
        for (int k = 0; k < kUnroll; ++k) {
            s0 += v[k].x;
            s1 += v[k].y;
        }
    }
    for (; i < n2; i += stride) {
        const double2 v = a[i];
        s0 += v.x;
        s1 += v.y;
    }
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

__global__ void __launch_bounds__(kThreads) k_copy(const double2 *__restrict__ a,
                                                   double2 *__restrict__ b, int64_t n2,
                                                   const double *__restrict__ ta,
                                                   double *__restrict__ tb, int ntail) {
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x;
    for (; i + (kUnroll - 1) * stride < n2; i += kUnroll * stride) {
        double2 v[kUnroll];
#pragma unroll
        for (int k = 0; k < kUnroll; ++k) v[k] = a[i + k * stride];
#pragma unroll
        for (int k = 0; k < kUnroll; ++k) b[i + k * stride] = v[k];
    }
    for (; i < n2; i += stride) b[i] = a[i];
    if (blockIdx.x == 0 && threadIdx.x == 0)
        for (int k = 0; k < ntail; ++k) tb[k] = ta[k];
}

__device__ __forceinline__ void cg_step(double2 &x, double2 &r, const double2 p,
                                        const double2 q, double alpha) {
    x.x = x.x + alpha * p.x;
    x.y = x.y + alpha * p.y;
    r.x = r.x - alpha * q.x;
    r.y = r.y - alpha * q.y;
}

__global__ void __launch_bounds__(kThreads)
k_cg_update(double2 *__restrict__ x, double2 *__restrict__ r, const double2 *__restrict__ p,
            const double2 *__restrict__ q, double alpha, int64_t n2, double *__restrict__ tx,
            double *__restrict__ tr, const double *__restrict__ tp,
            const double *__restrict__ tq, int ntail) {
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x;
    for (; i + stride < n2; i += 2 * stride) {
        double2 xv[2], rv[2], pv[2], qv[2];
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            xv[k] = x[i + k * stride];
            rv[k] = r[i + k * stride];
            pv[k] = p[i + k * stride];
            qv[k] = q[i + k * stride];
        }
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            cg_step(xv[k], rv[k], pv[k], qv[k], alpha);
            x[i + k * stride] = xv[k];
            r[i + k * stride] = rv[k];
        }
    }
    for (; i < n2; i += stride) {
        double2 xv = x[i], rv = r[i];
        cg_step(xv, rv, p[i], q[i], alpha);
        x[i] = xv;
        r[i] = rv;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0)
        for (int k = 0; k < ntail; ++k) {
            tx[k] = tx[k] + alpha * tp[k];
            tr[k] = tr[k] - alpha * tq[k];
        }
}

bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

int launched() { return hipGetLastError() == hipSuccess ? 0 : -6; }

}  // namespace

extern "C" {

int ldu_stream_read(const double *a, int64_t n, double *partials, int blocks,
                    void *hip_stream) {
    if (!a || !partials || n < 0 || !aligned16(a)) return -1;
    const int G = grid_of(blocks);
    const int64_t n2 = n / 2;
    k_read<<<G, kThreads, 0, reinterpret_cast<hipStream_t>(hip_stream)>>>(
        reinterpret_cast<const double2 *>(a), n2, a + 2 * n2, (int)(n - 2 * n2), partials);
    return launched();
}

int ldu_stream_copy(const double *a, double *b, int64_t n, int blocks, void *hip_stream) {
    if (!a || !b || n < 0 || !aligned16(a) || !aligned16(b)) return -1;
    const int G = grid_of(blocks);
    const int64_t n2 = n / 2;
    k_copy<<<G, kThreads, 0, reinterpret_cast<hipStream_t>(hip_stream)>>>(
        reinterpret_cast<const double2 *>(a), reinterpret_cast<double2 *>(b), n2, a + 2 * n2,
        b + 2 * n2, (int)(n - 2 * n2));
    return launched();
}

int ldu_stream_cg_update(double *x, double *r, const double *p, const double *q, double alpha,
                         int64_t n, int blocks, void *hip_stream) {
    if (!x || !r || !p || !q || n < 0 || !aligned16(x) || !aligned16(r) || !aligned16(p) ||
        !aligned16(q))
        return -1;
    const int G = grid_of(blocks);
    const int64_t n2 = n / 2;
    k_cg_update<<<G, kThreads, 0, reinterpret_cast<hipStream_t>(hip_stream)>>>(
        reinterpret_cast<double2 *>(x), reinterpret_cast<double2 *>(r),
        reinterpret_cast<const double2 *>(p), reinterpret_cast<const double2 *>(q), alpha, n2,
        x + 2 * n2, r + 2 * n2, p + 2 * n2, q + 2 * n2, (int)(n - 2 * n2));
    return launched();
}

}  // extern "C"
