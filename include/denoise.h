/*
 * denoise.h -- C ABI of the BF16 matrix-core kernels of the learned denoiser
 * (part of librmc.so).  The denoiser maps harmonic coefficient maps from few
 * packets to maps from many packets; its convolutions run here.
 *
 * Conventions as in mcrad.h: pointers ending in _d are caller-owned device
 * memory; calls only enqueue on `stream`; errors are status codes checked on
 * the host before anything is enqueued.  BF16 tensors are raw 16-bit
 * patterns (uint16_t).  Activations are channels last, [n][h][w][c], with c
 * a multiple of 8 and 16-byte aligned rows (pad with zero channels); weights
 * [co][3][3][ci].  Products are exact in FP32 and summed in FP32 on the
 * MFMA units (v_mfma_f32_16x16x32_bf16); the order of the sums differs from
 * a sequential loop.  Invalid shapes or alignment: MC_ERR_INVALID_ARG.
 */
#ifndef DENOISE_H
#define DENOISE_H

#include <stdint.h>

#include "mcrad.h"

#ifdef __cplusplus
extern "C" {
#endif

/* 3x3 convolution, stride 1, zero padding 1:
 *   y[n][h][w][co] = bias[co] + sum_{ky,kx,ci} w[co][ky][kx][ci] x[n][h+ky-1][w+kx-1][ci]
 * x_d: BF16 [n][h][w][ci], ci % 8 == 0, 16-byte aligned; w_d: BF16
 * [co][3][3][ci], 16-byte aligned; bias_d: FP32 [co] or NULL; y_d: FP32
 * [n][h][w][co] (overwritten; 16-byte aligned when co % 4 == 0).  The
 * gradient with respect to x is this same call on the upstream gradient with
 * the weights flipped in both spatial directions and ci/co swapped. */
mc_status dn_conv3x3_fwd(const uint16_t *x_d, const uint16_t *w_d, const float *bias_d, float *y_d, int n, int ci,
                         int co, int h, int w, void *stream);

/* Weight gradient of dn_conv3x3_fwd:
 *   gw[co][ky][kx][ci] = sum_{n,h,w} gy[n][h][w][co] x[n][h+ky-1][w+kx-1][ci]
 * x_d: BF16 [n][h][w][ci]; gy_d: BF16 [n][h][w][co]; ci and co multiples of
 * 8, both 16-byte aligned; gw_d: FP32 [co][3][3][ci] (overwritten; partial
 * sums over pixel slices are added with FP32 atomics, so the last bits
 * depend on their order). */
mc_status dn_conv3x3_wgrad(const uint16_t *x_d, const uint16_t *gy_d, float *gw_d, int n, int ci, int co, int h, int w,
                           void *stream);

#ifdef __cplusplus
}
#endif
#endif /* DENOISE_H */
