/*
 * ldu_bench.h -- bandwidth-ceiling kernels exported by libldu.so beside the
 * solver ABI of ldu.h.  They are measurement aids, not part of the solve:
 * each streams plain double arrays with no index stream and no gathers, so
 * its achieved rate is the HBM ceiling a streaming solver kernel is compared
 * with (the product and vector kernels of Sec. 4.3's profile are all
 * streaming).
 *
 * Arguments are DEVICE pointers (16-byte aligned, as torch allocations are),
 * n counts doubles, blocks is the grid size (<= 0: 2048; at most
 * LDU_STREAM_MAX_BLOCKS), nontemporal != 0 streams with nontemporal loads
 * and stores (past the caches), hip_stream a hipStream_t.  The calls only launch:
 * time them with events on hip_stream.  Return 0, -1 for a bad argument, -6
 * when the launch failed.  Nothing is allocated.
 */
#ifndef LDU_BENCH_H
#define LDU_BENCH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LDU_STREAM_MAX_BLOCKS 8192

/* read-only: partials[b] = sum of the doubles block b read (8 n bytes) */
int ldu_stream_read(const double *a, int64_t n, double *partials, int blocks,
                    int nontemporal, void *hip_stream);
/* b = a (16 n bytes) */
int ldu_stream_copy(const double *a, double *b, int64_t n, int blocks,
                    int nontemporal, void *hip_stream);
/* x += alpha p; r -= alpha q (48 n bytes: four reads, two writes), the
 * vector update of a CG iteration */
int ldu_stream_cg_update(double *x, double *r, const double *p, const double *q,
                         double alpha, int64_t n, int blocks, int nontemporal,
                         void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif
