/*
 * kc_peaks.h -- on-device peak microbenchmarks of one MI355X (gfx950), the
 * denominators the k-clique counting kernels are measured against: an HBM copy,
 * an LDS read stream (128-bit reads), an int32 VALU loop and a 64-bit AND +
 * popcount loop (the counting kernels' intersection step).
 *
 * Each call launches its kernel `iters` times on hip_stream (NULL = the default
 * stream), times the launches with HIP events on that stream, synchronises it,
 * and returns the mean milliseconds per launch in *ms and the work of one launch
 * (bytes or operations) in *work.  Returns 0, or the hipError_t of the first HIP
 * call that failed (nothing is launched after it); -1 for a bad argument.
 */
#ifndef KC_PEAKS_H
#define KC_PEAKS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Copy `bytes` (a multiple of 16, both pointers 16-byte aligned device memory)
 * from src to dst: *work = 2 * bytes (read + write). */
int kcp_hbm_copy(const void *src, void *dst, size_t bytes, int32_t iters, void *hip_stream, float *ms, double *work);

/* Every thread of `blocks` blocks of 256 threads reads 128-bit LDS words, `reps`
 * per thread (rounded down to a multiple of 4, at least 4): *work = blocks * 256 *
 * reps * 16 bytes. */
int kcp_lds_read(int32_t blocks, int32_t reps, int32_t iters, void *hip_stream, float *ms, double *work);

/* Every thread of `blocks` blocks of 256 threads runs `reps` rounds of 16
 * independent int32 add/xor operations: *work = blocks * 256 * reps * 16 ops. */
int kcp_valu_int32(int32_t blocks, int32_t reps, int32_t iters, void *hip_stream, float *ms, double *work);

/* Every thread of `blocks` blocks of 256 threads runs `reps` rounds of 8
 * independent popcount(a & b) of 64-bit words accumulated into counters:
 * *work = blocks * 256 * reps * 8 words (each 2 ANDs and 2 popcounts in int32). */
int kcp_and_popcount(int32_t blocks, int32_t reps, int32_t iters, void *hip_stream, float *ms, double *work);

#ifdef __cplusplus
}
#endif

#endif /* KC_PEAKS_H */
