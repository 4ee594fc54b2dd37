// denoise.hip -- BF16 matrix-core kernels of the learned denoiser: 3x3
// convolution (stride 1, zero padding 1) as an implicit GEMM on the gfx950
// MFMA units with FP32 accumulation, and its weight gradient.  The input
// gradient is the forward kernel applied to the flipped, transposed weights.
//
// Layouts (channels last, so that the GEMM's reduction index -- the input
// channel -- is contiguous): activations [n][h][w][c] BF16 (raw 16-bit
// patterns) with c a multiple of 8; weights [co][3][3][ci] BF16; outputs and
// weight gradients FP32 ([n][h][w][co] and [co][3][3][ci]).
//
// Forward GEMM: D[co][p] = sum_{tap, ci} W[co][tap][ci] X[p + off(tap)][ci]
// for the pixels p of an 8 x 8 block of one image.  The reduction runs over
// chunks of 32 input channels (the K of v_mfma_f32_16x16x32_bf16) and, within
// a chunk, over the nine taps: for a tap, B is the chunk's halo tile read at
// that tap's offset, so each input pixel is loaded from HBM once per chunk.
// A workgroup of four waves computes 64 output channels x 64 pixels (each
// wave a 32 x 32 quarter, 2 x 2 MFMA blocks).  Operands are staged in LDS,
// double buffered: while the waves multiply chunk c out of one buffer, the
// 16-byte global loads of chunk c + 1 are in flight into registers, which
// then fill the other buffer (one barrier per chunk).
//
// MFMA lane layout of v_mfma_f32_16x16x32_bf16 (checked on the device):
// A[m][k] with m = lane % 16, k = 8 (lane / 16) + i, i = 0..7; B[k][n] with
// n = lane % 16, k = 8 (lane / 16) + i; D[m][n] with n = lane % 16,
// m = 4 (lane / 16) + i, i = 0..3.  A lane's eight k values of A or B are
// eight consecutive channels in LDS: one 16-byte read.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "mcrad.h"
#include "denoise.h"

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int kCiC = 32;                   // input channels per chunk (the MFMA K)
constexpr int kTCo = 64;                   // output channels per workgroup
constexpr int kTY = 8, kTX = 8;            // output pixels per workgroup
constexpr int kHY = kTY + 2, kHX = kTX + 2;
constexpr int kPitch = kCiC + 8;           // LDS pitch (BF16) of one pixel's or one (co, tap)'s chunk: 80 bytes
constexpr int kXVec = kHY * kHX * (kCiC / 8);      // 16-byte vectors of a halo tile chunk (400)
constexpr int kWVec = kTCo * 9 * (kCiC / 8);       // 16-byte vectors of a weight chunk (2304)
constexpr int kThreads = 256;
constexpr int kXPer = (kXVec + kThreads - 1) / kThreads;   // 2
constexpr int kWPer = kWVec / kThreads;                    // 9
static_assert(kWVec % kThreads == 0, "weight chunk split");
constexpr int kXBuf = kHY * kHX * kPitch;  // BF16 elements of one X buffer
constexpr int kWBuf = kTCo * 9 * kPitch;   // BF16 elements of one W buffer
constexpr size_t kFwdLds = 2 * (size_t)(kXBuf + kWBuf) * sizeof(uint16_t);

__device__ __forceinline__ u32x4 load16(const uint16_t *p) {
    return *reinterpret_cast<const u32x4 *>(p);
}

// BF16 element q (0..7) of a 16-byte vector
__device__ __forceinline__ uint16_t half_of(const u32x4 v, int q) {
    return (uint16_t)(v[q >> 1] >> (16 * (q & 1)));
}

// Global loads of one chunk (input channels c0 .. c0 + 31) into registers;
// zeros outside the image, past the last channel or past the last output channel.
__device__ __forceinline__ void fwd_fetch(const uint16_t *x, const uint16_t *w, int img, int ty0, int tx0, int co0,
                                          int c0, int Ci, int Co, int H, int W, u32x4 (&rx)[kXPer],
                                          u32x4 (&rw)[kWPer]) {
    const int tid = threadIdx.x;
#pragma unroll
    for (int j = 0; j < kXPer; ++j) {
        const int v = tid + j * kThreads;
        u32x4 val = {0u, 0u, 0u, 0u};
        if (v < kXVec) {
            const int pix = v >> 2, part = v & 3;
            const int hy = pix / kHX, hx = pix - hy * kHX;
            const int gy = ty0 + hy - 1, gx = tx0 + hx - 1, c = c0 + 8 * part;
            if (gy >= 0 && gy < H && gx >= 0 && gx < W && c < Ci)
                val = load16(x + (((size_t)img * H + gy) * W + gx) * Ci + c);
        }
        rx[j] = val;
    }
#pragma unroll
    for (int j = 0; j < kWPer; ++j) {
        const int v = tid + j * kThreads;
        const int row = v >> 2, part = v & 3;   // row = co_l * 9 + tap
        const int col = row / 9, tap = row - col * 9;
        const int co = co0 + col, c = c0 + 8 * part;
        u32x4 val = {0u, 0u, 0u, 0u};
        if (co < Co && c < Ci) val = load16(w + ((size_t)co * 9 + tap) * Ci + c);
        rw[j] = val;
    }
}

__device__ __forceinline__ void fwd_stash(uint16_t *sx, uint16_t *sw, const u32x4 (&rx)[kXPer],
                                          const u32x4 (&rw)[kWPer]) {
    const int tid = threadIdx.x;
#pragma unroll
    for (int j = 0; j < kXPer; ++j) {
        const int v = tid + j * kThreads;
        if (v < kXVec) *reinterpret_cast<u32x4 *>(sx + (v >> 2) * kPitch + 8 * (v & 3)) = rx[j];
    }
#pragma unroll
    for (int j = 0; j < kWPer; ++j) {
        const int v = tid + j * kThreads;
        *reinterpret_cast<u32x4 *>(sw + (v >> 2) * kPitch + 8 * (v & 3)) = rw[j];
    }
}

// y[img][gy][gx][co] = bias[co] + sum_{tap, ci} w[co][tap][ci] x[img][gy + ky - 1][gx + kx - 1][ci]
__global__ void __launch_bounds__(kThreads) k_conv3x3_fwd(const uint16_t *__restrict__ x,
                                                          const uint16_t *__restrict__ w,
                                                          const float *__restrict__ bias, float *__restrict__ y,
                                                          int Ci, int Co, int H, int W, int tiles_x, int tiles_y) {
    extern __shared__ uint16_t smem[];   // [2][kXBuf] halo tiles, then [2][kWBuf] weight chunks
    const int t = blockIdx.x;
    const int img = t / (tiles_x * tiles_y), tt = t - img * tiles_x * tiles_y;
    const int ty0 = (tt / tiles_x) * kTY, tx0 = (tt % tiles_x) * kTX;
    const int co0 = blockIdx.y * kTCo;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;   // this wave's quarter: channels, pixels
    const int kg = lane >> 4, l16 = lane & 15;
    f32x4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    // pixel (py, px) of each B block of this lane in the 8 x 8 tile
    int bpy[2], bpx[2];
#pragma unroll
    for (int b = 0; b < 2; ++b) {
        const int p = wn + 16 * b + l16;
        bpy[b] = p >> 3;
        bpx[b] = p & 7;
    }
    u32x4 rx[kXPer], rw[kWPer];
    const int nchunk = (Ci + kCiC - 1) / kCiC;
    fwd_fetch(x, w, img, ty0, tx0, co0, 0, Ci, Co, H, W, rx, rw);
    fwd_stash(smem, smem + 2 * kXBuf, rx, rw);
    __syncthreads();
    for (int c = 0; c < nchunk; ++c) {
        const int cur = c & 1;
        if (c + 1 < nchunk) fwd_fetch(x, w, img, ty0, tx0, co0, (c + 1) * kCiC, Ci, Co, H, W, rx, rw);
        const uint16_t *X = smem + cur * kXBuf, *Wt = smem + 2 * kXBuf + cur * kWBuf;
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) {
            const int ky = tap / 3, kx = tap - 3 * ky;
            bf16x8 fa[2], fb[2];
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                const u32x4 v = load16(Wt + ((wm + 16 * a + l16) * 9 + tap) * kPitch + 8 * kg);
                fa[a] = __builtin_bit_cast(bf16x8, v);
            }
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const u32x4 v = load16(X + ((bpy[b] + ky) * kHX + bpx[b] + kx) * kPitch + 8 * kg);
                fb[b] = __builtin_bit_cast(bf16x8, v);
            }
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[a], fb[b], acc[a][b], 0, 0, 0);
        }
        if (c + 1 < nchunk) fwd_stash(smem + (cur ^ 1) * kXBuf, smem + 2 * kXBuf + (cur ^ 1) * kWBuf, rx, rw);
        __syncthreads();
    }
    // D[m][n]: m = 4 kg + i (output channel), n = l16 (pixel)
    const bool vec = (Co & 3) == 0;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int gy = ty0 + bpy[b], gx = tx0 + bpx[b];
            const int co = co0 + wm + 16 * a + 4 * kg;
            if (gy >= H || gx >= W || co >= Co) continue;
            float *dst = y + (((size_t)img * H + gy) * W + gx) * Co + co;
            f32x4 v = acc[a][b];
#pragma unroll
            for (int i = 0; i < 4; ++i) v[i] += (bias && co + i < Co) ? bias[co + i] : 0.f;
            if (vec) {
                *reinterpret_cast<f32x4 *>(dst) = v;
            } else {
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    if (co + i < Co) dst[i] = v[i];
            }
        }
}

// ---- weight gradient
// gw[co][tap][ci] = sum_p gy[p][co] x[p + off(tap)][ci].  GEMM per tap with
// M = output channels, N = input channels, K = pixels.  A workgroup holds 64
// output channels x one chunk of 32 input channels x the nine taps and runs
// over a slice of 8 x 8 pixel tiles; per tile it stages gy transposed
// ([co][pixel]) and the input halo transposed into three copies shifted by
// kx ([kx][ci][row][8 pixels]), so that a lane's eight consecutive pixels of
// either operand are one aligned 16-byte LDS read.  Each wave owns 16 output
// channels: per 32-pixel K step its A fragment serves 2 x 9 MFMAs.  Partial
// sums over the pixel slices are added with FP32 atomics.
constexpr int kGP = 64 + 8;                            // LDS pitch (BF16) of a gy^T row: 64 pixels
constexpr int kGVec = kTY * kTX * (kTCo / 8);          // 16-byte vectors of the gy tile (512)
constexpr int kXTRow = kTX;                            // BF16 per [kx][ci][row] run: 8 pixels
constexpr size_t kWgradLds = ((size_t)kTCo * kGP + 3ull * kCiC * kHY * kXTRow) * sizeof(uint16_t);

__global__ void __launch_bounds__(kThreads) k_conv3x3_wgrad(const uint16_t *__restrict__ x,
                                                            const uint16_t *__restrict__ gy, float *__restrict__ gw,
                                                            int Ci, int Co, int H, int W, int tiles_x, int tiles_y,
                                                            int n_tiles, int tiles_per_slice) {
    extern __shared__ uint16_t smem[];
    uint16_t *sg = smem;                      // [64 co][kGP]
    uint16_t *sxT = smem + kTCo * kGP;        // [3 kx][32 ci][kHY rows][8 px]
    const int c0 = blockIdx.x * kCiC, co0 = blockIdx.y * kTCo;
    const int t0 = blockIdx.z * tiles_per_slice, t1 = min(n_tiles, t0 + tiles_per_slice);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int kg = lane >> 4, l16 = lane & 15;
    f32x4 acc[9][2];
#pragma unroll
    for (int tap = 0; tap < 9; ++tap)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[tap][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int t = t0; t < t1; ++t) {
        const int img = t / (tiles_x * tiles_y), tt = t - img * tiles_x * tiles_y;
        const int ty0 = (tt / tiles_x) * kTY, tx0 = (tt % tiles_x) * kTX;
        // gy tile, transposed: 512 vectors of 8 output channels of one pixel
        u32x4 rg[kGVec / kThreads];
#pragma unroll
        for (int j = 0; j < kGVec / kThreads; ++j) {
            const int v = tid + j * kThreads;
            const int p = v >> 3, part = v & 7;
            const int py = p >> 3, px = p & 7;
            const int yy = ty0 + py, xx = tx0 + px, co = co0 + 8 * part;
            u32x4 val = {0u, 0u, 0u, 0u};
            if (yy < H && xx < W && co < Co) val = load16(gy + (((size_t)img * H + yy) * W + xx) * Co + co);
            rg[j] = val;
        }
        // input halo: 400 vectors of 8 input channels of one pixel
        u32x4 rx[kXPer];
#pragma unroll
        for (int j = 0; j < kXPer; ++j) {
            const int v = tid + j * kThreads;
            u32x4 val = {0u, 0u, 0u, 0u};
            if (v < kXVec) {
                const int pix = v >> 2, part = v & 3;
                const int hy = pix / kHX, hx = pix - hy * kHX;
                const int yy = ty0 + hy - 1, xx = tx0 + hx - 1, c = c0 + 8 * part;
                if (yy >= 0 && yy < H && xx >= 0 && xx < W && c < Ci)
                    val = load16(x + (((size_t)img * H + yy) * W + xx) * Ci + c);
            }
            rx[j] = val;
        }
        __syncthreads();   // the previous tile's fragments have been read
#pragma unroll
        for (int j = 0; j < kGVec / kThreads; ++j) {
            const int v = tid + j * kThreads;
            const int p = v >> 3, part = v & 7;
#pragma unroll
            for (int q = 0; q < 8; ++q) sg[(8 * part + q) * kGP + p] = half_of(rg[j], q);
        }
#pragma unroll
        for (int j = 0; j < kXPer; ++j) {
            const int v = tid + j * kThreads;
            if (v >= kXVec) continue;
            const int pix = v >> 2, part = v & 3;
            const int hy = pix / kHX, hx = pix - hy * kHX;
#pragma unroll
            for (int kx = 0; kx < 3; ++kx) {
                const int px = hx - kx;   // this halo column is pixel px of the copy shifted by kx
                if (px < 0 || px >= kTX) continue;
#pragma unroll
                for (int q = 0; q < 8; ++q)
                    sxT[((kx * kCiC + 8 * part + q) * kHY + hy) * kXTRow + px] = half_of(rx[j], q);
            }
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < 2; ++s) {   // K steps: tile rows 4s .. 4s + 3, lane group kg takes row 4s + kg
            const int row = 4 * s + kg;
            const bf16x8 fa = __builtin_bit_cast(bf16x8, load16(sg + (16 * wave + l16) * kGP + 8 * row));
#pragma unroll
            for (int tap = 0; tap < 9; ++tap) {
                const int ky = tap / 3, kx = tap - 3 * ky;
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    const bf16x8 fb = __builtin_bit_cast(
                        bf16x8, load16(sxT + ((kx * kCiC + 16 * b + l16) * kHY + row + ky) * kXTRow));
                    acc[tap][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa, fb, acc[tap][b], 0, 0, 0);
                }
            }
        }
    }
    // D[m][n]: m = 4 kg + i (output channel within the wave's 16), n = l16 (+16 b) input channel
#pragma unroll
    for (int tap = 0; tap < 9; ++tap)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int ci = c0 + 16 * b + l16;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int co = co0 + 16 * wave + 4 * kg + i;
                if (co < Co && ci < Ci && acc[tap][b][i] != 0.f)
                    atomicAdd(gw + ((size_t)co * 9 + tap) * Ci + ci, acc[tap][b][i]);
            }
        }
}

__global__ void k_zero_f32(float *p, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0.f;
}

bool dims_ok(int n, int ci, int co, int h, int w) {
    if (n < 1 || ci < 1 || co < 1 || h < 1 || w < 1) return false;
    const long long tiles = (long long)n * ((h + kTY - 1) / kTY) * ((w + kTX - 1) / kTX);
    const long long P = (long long)n * h * w;
    return P <= (1ll << 30) && tiles < (1ll << 31) && ci <= (1 << 16) && co <= (1 << 16);
}

bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

mc_status set_lds(const void *fn, size_t bytes) {
    return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) == hipSuccess
               ? MC_OK
               : MC_ERR_DEVICE;
}

}  // namespace

extern "C" {

mc_status dn_conv3x3_fwd(const uint16_t *x_d, const uint16_t *w_d, const float *bias_d, float *y_d, int n, int ci,
                         int co, int h, int w, void *stream) {
    if (!x_d || !w_d || !y_d || !dims_ok(n, ci, co, h, w) || (ci & 7) || !aligned16(x_d) || !aligned16(w_d) ||
        ((co & 3) == 0 && !aligned16(y_d)))
        return MC_ERR_INVALID_ARG;
    const int tx = (w + kTX - 1) / kTX, ty = (h + kTY - 1) / kTY;
    const long long tiles = (long long)n * tx * ty;
    const unsigned gco = (unsigned)((co + kTCo - 1) / kTCo);
    if (gco > 65535) return MC_ERR_UNSUPPORTED;
    mc_status st = set_lds(reinterpret_cast<const void *>(k_conv3x3_fwd), kFwdLds);
    if (st != MC_OK) return st;
    hipLaunchKernelGGL(k_conv3x3_fwd, dim3((unsigned)tiles, gco), dim3(kThreads), kFwdLds,
                       reinterpret_cast<hipStream_t>(stream), x_d, w_d, bias_d, y_d, ci, co, h, w, tx, ty);
    return hipGetLastError() == hipSuccess ? MC_OK : MC_ERR_DEVICE;
}

mc_status dn_conv3x3_wgrad(const uint16_t *x_d, const uint16_t *gy_d, float *gw_d, int n, int ci, int co, int h, int w,
                           void *stream) {
    if (!x_d || !gy_d || !gw_d || !dims_ok(n, ci, co, h, w) || (ci & 7) || (co & 7) || !aligned16(x_d) ||
        !aligned16(gy_d))
        return MC_ERR_INVALID_ARG;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const size_t nw = (size_t)co * 9 * ci;
    hipLaunchKernelGGL(k_zero_f32, dim3((unsigned)std::min<size_t>((nw + 255) / 256, 4096)), dim3(256), 0, s, gw_d, nw);
    const int tx = (w + kTX - 1) / kTX, ty = (h + kTY - 1) / kTY;
    const long long tiles = (long long)n * tx * ty;
    const unsigned gx = (unsigned)((ci + kCiC - 1) / kCiC), gyd = (unsigned)((co + kTCo - 1) / kTCo);
    if (gyd > 65535) return MC_ERR_UNSUPPORTED;
    // enough pixel slices to give the device ~2048 workgroups
    const long long blocks = (long long)gx * gyd;
    long long slices = std::max<long long>(1, std::min<long long>(tiles, (2048 + blocks - 1) / blocks));
    slices = std::min<long long>(slices, 65535);
    const long long per = (tiles + slices - 1) / slices;
    slices = (tiles + per - 1) / per;
    mc_status st = set_lds(reinterpret_cast<const void *>(k_conv3x3_wgrad), kWgradLds);
    if (st != MC_OK) return st;
    hipLaunchKernelGGL(k_conv3x3_wgrad, dim3(gx, gyd, (unsigned)slices), dim3(kThreads), kWgradLds, s, x_d, gy_d, gw_d,
                       ci, co, h, w, tx, ty, (int)tiles, (int)per);
    return hipGetLastError() == hipSuccess ? MC_OK : MC_ERR_DEVICE;
}

}  // extern "C"
