/*
 * rt_ceilings.h -- measured hardware ceilings that bound the packet march
 * (librt_ceilings.so, built beside librt_mcrt.so).
 *
 * The march is a gather of absorber densities plus a scatter-add of float64
 * deposits into per-cell accumulators (Partl et al. 2011, Sec. 2: the photons
 * absorbed in every crossed cell are added to that cell).  Its ceilings are
 * the HBM bandwidth, the rate of float64 atomic adds into device memory, and
 * the rate of float64 atomic adds into LDS, where the tiled march gathers a
 * tile's deposits.  Each call runs one microbenchmark on the caller's stream,
 * times it with HIP events and returns the rate; nothing is allocated: every
 * buffer is the caller's device memory.
 *
 * Every call returns 0 on success, -1 for an invalid argument (nothing runs)
 * and -3 for a HIP error.  Calls synchronise the stream.
 */
#ifndef RT_CEILINGS_H
#define RT_CEILINGS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Device copy of `bytes` (a multiple of 16, > 0) from d_src to d_dst, repeated
 * reps times after one untimed run; *gbs = 2 * bytes * reps / time / 1e9
 * (bytes read plus bytes written).  Buffers must not overlap and must be
 * 16-byte aligned. */
int32_t rtc_hbm_copy(void *d_dst, const void *d_src, size_t bytes, int32_t reps, void *hip_stream,
                     double *gbs);

/* Device read of `bytes` (a multiple of 16, > 0) from d_src, reps times; each
 * block writes one float to d_sink (at least 65536 floats).  *gbs = bytes *
 * reps / time / 1e9. */
int32_t rtc_hbm_read(const void *d_src, size_t bytes, int32_t reps, float *d_sink, void *hip_stream,
                     double *gbs);

/* Float64 atomic adds (the hardware add, no return value) into d_buf[0..n):
 * `updates` adds in all, lane t's k-th add at a hashed index, so addresses
 * spread over the whole buffer.  A small buffer stays in the L2 caches, a
 * large one reaches HBM.  *rate = updates / time (per second).  d_buf's final
 * contents are the number of adds that hit each element. */
int32_t rtc_global_atomic_f64(double *d_buf, size_t n, int64_t updates, void *hip_stream, double *rate);

/* Float64 atomic adds into LDS, as the tiled march deposits: every block of
 * 256 threads holds 512 cells x `acc` doubles (acc in 1..4) and each lane adds
 * to a hashed cell, `acc` adds per cell visit, laid out cell-major
 * (soa = 0: the acc values of a cell adjacent) or value-major (soa = 1:
 * value k of every cell in a plane of its own).  `updates` adds in all over
 * blocks x CUs; *rate = updates / time.  d_sink (at least 65536 doubles)
 * receives one sum per block so that nothing is optimised away. */
int32_t rtc_lds_atomic_f64(int32_t acc, int32_t soa, int64_t updates, double *d_sink, void *hip_stream,
                           double *rate);

#ifdef __cplusplus
}
#endif
#endif /* RT_CEILINGS_H */
