/*
 * microbench.h -- C ABI of the device microbenchmarks (part of librmc.so).
 *
 * These are not steps of the method.  They measure the ceilings the
 * transport kernels are priced against: LDS atomic throughput for the
 * LDS-staged FP64 tally, random-address FP64 atomics in L2/HBM for the
 * whole-grid tally, HBM copy bandwidth, and FP32 FMA issue rate.
 *
 * Conventions as in mcrad.h: pointers ending in _d are caller-owned device
 * memory; calls only enqueue on `stream` (the caller times them with events
 * on that stream); arguments are checked on the host and a bad one returns
 * MC_ERR_INVALID_ARG before anything is enqueued.
 *
 * Random addresses come from a 32-bit integer hash of (thread id, seed,
 * iteration); every address is reduced into range by a multiply-high, so no
 * access leaves the buffer.
 */
#ifndef MICROBENCH_H
#define MICROBENCH_H

#include <stddef.h>
#include <stdint.h>

#include "mcrad.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MB_LDS_ADD_F64 = 0,      /* one FP64 add (ds_add_f64) per lane at a random 8-byte slot */
    MB_LDS_ADD_F32 = 1,      /* one FP32 add (ds_add_f32) per lane at a random 4-byte slot */
    MB_LDS_ADD_U64 = 2,      /* one 64-bit integer add (ds_add_u64) per lane at a random slot */
    MB_LDS_ADD_U32 = 3,      /* one 32-bit integer add (ds_add_u32) per lane at a random slot */
    MB_LDS_ADD_F64_ROW33 = 4, /* each lane picks a random row of 33 FP64 slots and adds to all 33:
                                 the pattern of a tally flush at N = 16 */
    MB_LDS_ADD_U64_ROW33 = 5, /* the same with 64-bit integer adds (ds_add_u64): the fixed-point
                                 tally flush; one address computation per 33 adds */
    MB_LDS_ADD_U64_PRE = 6    /* each lane draws 8 random slots once and adds to each of them in
                                 every iteration: 64-bit integer adds with no address arithmetic */
} mb_lds_kind;

/* LDS atomic throughput.  n_blocks workgroups of `block` threads (a multiple
 * of 64, at most 1024), each with lds_bytes of dynamic LDS (at least 1 KiB,
 * at most 160 KiB, a multiple of 8; for the row kind at least 33 x 8 bytes)
 * zeroed at start; each thread makes `iters` iterations of the kind's adds.
 * Lane-operations: n_blocks * block * iters (x 33 for the row kinds, x 8 for
 * MB_LDS_ADD_U64_PRE).  sink_d: FP64 [n_blocks], the sum of each workgroup's
 * LDS array after the adds (each add is of 1, so it equals block * iters
 * times that factor).
 * clk_d: NULL or uint64 [4]: workgroup 0 records the shader clock counter
 * (variable frequency) at its start and end in [0], [1] and the constant-rate
 * counter (mb_wall_clock_khz) in [2], [3], which gives the clock under load. */
mc_status mb_lds_atomics(int kind, uint32_t lds_bytes, uint32_t block, uint32_t n_blocks, uint32_t iters, uint32_t seed,
                         double *sink_d, uint64_t *clk_d, void *stream);

/* Random-address FP64 atomic add (global_atomic_add_f64, no return) on
 * buf_d[n_elem], 1 <= n_elem < 2^32: n_blocks workgroups of 256 threads,
 * `iters` adds each.  buf_d is accumulated into, not cleared. */
mc_status mb_global_atomics_f64(double *buf_d, uint64_t n_elem, uint32_t n_blocks, uint32_t iters, uint32_t seed,
                                void *stream);

/* FP64 atomic adds of 1.0 (global_atomic_add_f64, no return) to buf_d
 * [n_rows][row_len] in the pattern of the tail finisher's flush: the lanes of
 * a wave take consecutive elements of rows drawn at random, so one wave
 * instruction covers 64 / row_len rows.  n_blocks workgroups of 256 threads,
 * `iters` adds per thread; 1 <= row_len <= 4096, n_rows * row_len < 2^32.
 * buf_d is accumulated into, not cleared. */
mc_status mb_global_atomics_rows_f64(double *buf_d, uint32_t n_rows, uint32_t row_len, uint32_t n_blocks,
                                     uint32_t iters, uint32_t seed, void *stream);

/* Device copy dst_d[i] = src_d[i] of n16 16-byte elements (both 16-byte
 * aligned, not overlapping): bytes moved through HBM = 32 * n16. */
mc_status mb_copy(const void *src_d, void *dst_d, uint64_t n16, void *stream);

/* FP32 FMA issue rate: n_blocks workgroups of 256 threads, each thread runs
 * 8 independent chains of `iters` fused multiply-adds (non-packed v_fma_f32,
 * 2 flops each).  sink_d: FP32 [n_blocks * 256].  clk_d as above. */
mc_status mb_fma_f32(float *sink_d, uint32_t n_blocks, uint32_t iters, uint64_t *clk_d, void *stream);

/* Rate of the constant-rate counter of device `device`, kHz. */
mc_status mb_wall_clock_khz(int device, int *khz);

#ifdef __cplusplus
}
#endif
#endif /* MICROBENCH_H */
