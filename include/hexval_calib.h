/* hexval_calib.h: machine ceilings of the current GPU, measured with kernels
 * of known work (libhexval_calib.so).  They put the achievable HBM read rate
 * and FP64 vector rate beside the vendor's peak figures when the roofline
 * fractions of the library's first passes are read.  Not part of the check
 * itself.
 *
 * Conventions: every call runs on the current device and the default stream,
 * synchronously; pointers are device pointers the caller owns; the return
 * value is 0 on success, 1 for a bad argument, 2 for a HIP error, 3 when a
 * small internal allocation fails.  One untimed launch precedes the timed
 * ones. */
#ifndef HEXVAL_CALIB_H
#define HEXVAL_CALIB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Reads the first bytes (rounded down to 16) of buf once per launch, 16 bytes
 * per lane access, four accesses in flight per lane; *ms = mean time per
 * launch over reps launches.  Read rate = bytes / ms. */
int hexval_calib_read(const void* buf, int64_t bytes, int reps, float* ms);

/* Copies bytes (rounded down to 16) from src to dst per launch; buffers must
 * not overlap.  Traffic per launch = 2 * bytes. */
int hexval_calib_copy(void* dst, const void* src, int64_t bytes, int reps, float* ms);

/* Eight independent FP64 FMA chains of iters steps on every lane of
 * 8 blocks of 256 per compute unit; *flops = FP64 operations per launch (FMA
 * counted as 2), *ms = mean time per launch, *clock_mhz = the shader clock
 * during one launch (its cycle counter against the constant 100 MHz one). */
int hexval_calib_fp64(int64_t iters, int reps, float* ms, double* flops, double* clock_mhz);

#ifdef __cplusplus
}
#endif

#endif
