// denoise.hip -- BF16 matrix-core kernels of the learned denoiser: 3x3
// convolution (stride 1, zero padding 1) as an implicit GEMM on the MFMA
// units with FP32 accumulation, and its weight gradient.  The input
// gradient is the forward kernel applied to the flipped, transposed weights.
//
// Layouts: activations NCHW, BF16 (raw 16-bit patterns); weights
// [co][ci][3][3] BF16; outputs and weight gradients FP32.
//
// GEMM view of the forward pass: D[co][p] = sum_k W[co][k] X[k][p] with
// k = ci*9 + ky*3 + kx and p = (n*H + y)*W + x, X[k][p] = x[n][ci][y+ky-1][x+kx-1]
// (zero outside).  A workgroup of four waves computes a 64 x 64 tile of D;
// each wave a 32 x 32 quarter as 2 x 2 blocks of v_mfma_f32_16x16x16_bf16,
// whose lane layout (checked on the device) is: A[m][k] with m = lane % 16,
// k = 4 (lane / 16) + i; B[k][n] with n = lane % 16, k = 4 (lane / 16) + i;
// D[m][n] with n = lane % 16, m = 4 (lane / 16) + i, i = 0..3.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "mcrad.h"
#include "denoise.h"

namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kTM = 64, kTN = 64, kTK = 16;   // tile of D and K step
constexpr int kPadA = kTK + 4;                // LDS row pitch (shorts) of the A tile
constexpr int kPadB = kTN + 4;                // LDS row pitch (shorts) of the B tile

// im2col element X[k][p] of a [n][c][h][w] BF16 tensor (0 outside the image)
__device__ __forceinline__ unsigned short im2col(const unsigned short *x, int C, int H, int W, int k, int p,
                                                 int K, int P) {
    if (k >= K || p >= P) return 0;
    const int c = k / 9, r = k - c * 9, ky = r / 3, kx = r - ky * 3;
    const int xx = p % W, t = p / W, yy = t % H, n = t / H;
    const int sy = yy + ky - 1, sx = xx + kx - 1;
    if (sy < 0 || sy >= H || sx < 0 || sx >= W) return 0;
    return x[(((size_t)n * C + c) * H + sy) * W + sx];
}

// y[n][co][h][w] = bias[co] + sum_{ci,ky,kx} w[co][ci][ky][kx] x[n][ci][h+ky-1][w+kx-1]
__global__ void __launch_bounds__(256) k_conv3x3_fwd(const unsigned short *x, const unsigned short *w,
                                                     const float *bias, float *y, int N, int Ci, int Co, int H,
                                                     int W) {
    __shared__ unsigned short sA[kTM][kPadA];   // weights: [co][k]
    __shared__ unsigned short sB[kTK][kPadB];   // im2col:  [k][p]
    const int K = Ci * 9, P = N * H * W;
    const int m0 = blockIdx.y * kTM, p0 = blockIdx.x * kTN;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;   // this wave's quarter
    f32x4 acc[2][2];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += kTK) {
        // stage the tiles: 1024 elements each, 4 per thread
        for (int e = tid; e < kTM * kTK; e += 256) {
            const int r = e / kTK, c = e % kTK;
            const int co = m0 + r, k = k0 + c;
            sA[r][c] = (co < Co && k < K) ? w[(size_t)co * K + k] : (unsigned short)0;
        }
        for (int e = tid; e < kTK * kTN; e += 256) {
            const int r = e / kTN, c = e % kTN;
            sB[r][c] = im2col(x, Ci, H, W, k0 + r, p0 + c, K, P);
        }
        __syncthreads();
        bf16x4 fa[2], fb[2];
        for (int a = 0; a < 2; ++a)
            for (int i = 0; i < 4; ++i) fa[a][i] = (short)sA[wm + 16 * a + lane % 16][4 * (lane / 16) + i];
        for (int b = 0; b < 2; ++b)
            for (int i = 0; i < 4; ++i) fb[b][i] = (short)sB[4 * (lane / 16) + i][wn + 16 * b + lane % 16];
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(fa[a], fb[b], acc[a][b], 0, 0, 0);
        __syncthreads();
    }
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int i = 0; i < 4; ++i) {
                const int co = m0 + wm + 16 * a + 4 * (lane / 16) + i;
                const int p = p0 + wn + 16 * b + lane % 16;
                if (co < Co && p < P) {
                    const int xx = p % W, t = p / W, yy = t % H, n = t / H;
                    y[(((size_t)n * Co + co) * H + yy) * W + xx] = acc[a][b][i] + (bias ? bias[co] : 0.f);
                }
            }
}

// gw[co][k] += sum_p gy[co][p] X[k][p] over this workgroup's slice of pixels
// (the GEMM's K dimension is the pixel index; slices add with FP32 atomics).
__global__ void __launch_bounds__(256) k_conv3x3_wgrad(const unsigned short *x, const unsigned short *gy, float *gw,
                                                       int N, int Ci, int Co, int H, int W, int p_per_slice) {
    __shared__ unsigned short sA[kTM][kPadA];   // gy:     [co][p]
    __shared__ unsigned short sB[kTK][kPadB];   // im2col^T: [p][k]
    const int K = Ci * 9, P = N * H * W, HW = H * W;
    const int m0 = blockIdx.y * kTM, k0 = blockIdx.x * kTN;
    const int pa = blockIdx.z * p_per_slice, pb = min(P, pa + p_per_slice);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    f32x4 acc[2][2];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int q0 = pa; q0 < pb; q0 += kTK) {
        for (int e = tid; e < kTM * kTK; e += 256) {
            const int r = e / kTK, c = e % kTK;
            const int co = m0 + r, p = q0 + c;
            unsigned short v = 0;
            if (co < Co && p < pb) {
                const int n = p / HW, s = p - n * HW;
                v = gy[((size_t)n * Co + co) * HW + s];
            }
            sA[r][c] = v;
        }
        for (int e = tid; e < kTK * kTN; e += 256) {
            const int r = e / kTN, c = e % kTN;
            const int p = q0 + r;
            sB[r][c] = p < pb ? im2col(x, Ci, H, W, k0 + c, p, K, P) : (unsigned short)0;
        }
        __syncthreads();
        bf16x4 fa[2], fb[2];
        for (int a = 0; a < 2; ++a)
            for (int i = 0; i < 4; ++i) fa[a][i] = (short)sA[wm + 16 * a + lane % 16][4 * (lane / 16) + i];
        for (int b = 0; b < 2; ++b)
            for (int i = 0; i < 4; ++i) fb[b][i] = (short)sB[4 * (lane / 16) + i][wn + 16 * b + lane % 16];
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(fa[a], fb[b], acc[a][b], 0, 0, 0);
        __syncthreads();
    }
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int i = 0; i < 4; ++i) {
                const int co = m0 + wm + 16 * a + 4 * (lane / 16) + i;
                const int k = k0 + wn + 16 * b + lane % 16;
                if (co < Co && k < K && acc[a][b][i] != 0.f) atomicAdd(gw + (size_t)co * K + k, acc[a][b][i]);
            }
}

__global__ void k_zero_f32(float *p, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0.f;
}

bool dims_ok(int n, int ci, int co, int h, int w) {
    if (n < 1 || ci < 1 || co < 1 || h < 1 || w < 1) return false;
    const long long P = (long long)n * h * w;
    return P <= (1ll << 30) && (long long)ci * 9 <= (1 << 24) && co <= (1 << 24);
}

}  // namespace

extern "C" {

mc_status dn_conv3x3_fwd(const uint16_t *x_d, const uint16_t *w_d, const float *bias_d, float *y_d, int n, int ci,
                         int co, int h, int w, void *stream) {
    if (!x_d || !w_d || !y_d || !dims_ok(n, ci, co, h, w)) return MC_ERR_INVALID_ARG;
    const long long P = (long long)n * h * w;
    const dim3 grid((unsigned)((P + kTN - 1) / kTN), (unsigned)((co + kTM - 1) / kTM));
    if (grid.y > 65535) return MC_ERR_UNSUPPORTED;
    hipLaunchKernelGGL(k_conv3x3_fwd, grid, dim3(256), 0, reinterpret_cast<hipStream_t>(stream), x_d, w_d, bias_d, y_d,
                       n, ci, co, h, w);
    return hipGetLastError() == hipSuccess ? MC_OK : MC_ERR_DEVICE;
}

mc_status dn_conv3x3_wgrad(const uint16_t *x_d, const uint16_t *gy_d, float *gw_d, int n, int ci, int co, int h, int w,
                           void *stream) {
    if (!x_d || !gy_d || !gw_d || !dims_ok(n, ci, co, h, w)) return MC_ERR_INVALID_ARG;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const long long K = (long long)ci * 9, P = (long long)n * h * w;
    const size_t nw = (size_t)co * K;
    hipLaunchKernelGGL(k_zero_f32, dim3((unsigned)std::min<size_t>((nw + 255) / 256, 4096)), dim3(256), 0, s, gw_d, nw);
    const unsigned gx = (unsigned)((K + kTN - 1) / kTN), gyd = (unsigned)((co + kTM - 1) / kTM);
    // enough pixel slices to fill the device, each a multiple of the K step
    const long long tiles = (long long)gx * gyd;
    long long slices = std::max<long long>(1, std::min<long long>(1024 / std::max<long long>(tiles, 1) + 1,
                                                                   (P + 1023) / 1024));
    slices = std::min<long long>(slices, 65535);
    long long per = (P + slices - 1) / slices;
    per = (per + kTK - 1) / kTK * kTK;
    slices = (P + per - 1) / per;
    if (gyd > 65535) return MC_ERR_UNSUPPORTED;
    hipLaunchKernelGGL(k_conv3x3_wgrad, dim3(gx, gyd, (unsigned)slices), dim3(256), 0, s, x_d, gy_d, gw_d, n, ci, co, h,
                       w, (int)per);
    return hipGetLastError() == hipSuccess ? MC_OK : MC_ERR_DEVICE;
}

}  // extern "C"
