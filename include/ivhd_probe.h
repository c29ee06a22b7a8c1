/*
 * ivhd_probe.h -- measurement helper of the MI355X IVHD library (not part of
 * the method).
 *
 * The loop's step kernel is bound by random 8-byte position gathers, and
 * the first pass of its atomic mode by one 64-bit integer atomic per random
 * edge.  These calls perform such accesses alone, so that a benchmark can
 * measure the chip's rates for a given footprint and count and set the
 * kernels' times beside them.  Conventions as in ivhd.h (device pointers
 * owned by the caller, stream as void*, status return, ivhd_last_error()).
 */
#ifndef IVHD_PROBE_H
#define IVHD_PROBE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ivhd_probe_gather: d_dst[t] = d_src[d_idx[t]] for t < n, rows of two
 * floats: d_src float32 [n_src][2], d_idx int32 [n] with entries in
 * [0, n_src) (not checked: the caller guarantees the range), d_dst float32
 * [n][2].  One thread per row, loads and stores of 8 bytes.  n >= 0,
 * n_src >= 1.  Asynchronous.                                                */
int ivhd_probe_gather(const float *d_src, int64_t n_src, const int32_t *d_idx, int64_t n, float *d_dst,
                      void *stream);

/* ivhd_probe_atomic: d_acc[d_idx[t]] += 2^32 + 1 for t < n (both 32-bit
 * halves of the word count the hits), one 64-bit integer atomic per index,
 * the access of one random-edge reaction in the atomic mode: d_acc uint64
 * [n_acc], d_idx int32 [n] with entries in [0, n_acc) (not checked: the
 * caller guarantees the range).  n >= 0, n_acc >= 1.  Asynchronous.         */
int ivhd_probe_atomic(uint64_t *d_acc, int64_t n_acc, const int32_t *d_idx, int64_t n, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* IVHD_PROBE_H */
