// microbench.hip -- device ceilings the transport kernels are priced against:
// LDS atomics (the LDS-staged FP64 tally), random-address FP64 atomics in
// L2/HBM (the whole-grid tally), HBM copy bandwidth and FP32 FMA issue rate.
// Declared in include/microbench.h.
#include <hip/hip_runtime.h>

#include "mcrad.h"
#include "microbench.h"

namespace {

__device__ __forceinline__ uint32_t mb_hash(uint32_t x) {
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

// a uniform index in [0, n) for n < 2^32
__device__ __forceinline__ uint32_t mb_pick(uint32_t h, uint32_t n) {
    return (uint32_t)(((uint64_t)h * n) >> 32);
}

constexpr uint32_t kMaxLds = 160u * 1024u;
constexpr int kRow = 33;

template <int KIND>
__global__ void __launch_bounds__(1024) k_lds_atomics(uint32_t lds_bytes, uint32_t iters, uint32_t seed, double *sink,
                                                      uint64_t *clk) {
    extern __shared__ __align__(16) unsigned char lds[];
    const bool rec = clk != nullptr && blockIdx.x == 0 && threadIdx.x == 0;
    uint64_t c0 = 0, w0 = 0;
    if (rec) {
        c0 = clock64();
        w0 = wall_clock64();
    }
    uint32_t *w32 = reinterpret_cast<uint32_t *>(lds);
    for (uint32_t i = threadIdx.x; i < lds_bytes / 4u; i += blockDim.x) w32[i] = 0u;
    __syncthreads();
    const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t h = mb_hash(gid ^ (seed * 0x9e3779b9u));
    uint32_t pre[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) pre[c] = mb_pick(mb_hash(h + 0x632be5abu * (c + 1)), lds_bytes / 8u);
    for (uint32_t it = 0; it < iters; ++it) {
        h = h * 1664525u + 1013904223u;
        const uint32_t r = mb_hash(h);
        if constexpr (KIND == MB_LDS_ADD_F64) {
            atomicAdd(reinterpret_cast<double *>(lds) + mb_pick(r, lds_bytes / 8u), 1.0);
        } else if constexpr (KIND == MB_LDS_ADD_F32) {
            atomicAdd(reinterpret_cast<float *>(lds) + mb_pick(r, lds_bytes / 4u), 1.0f);
        } else if constexpr (KIND == MB_LDS_ADD_U64) {
            atomicAdd(reinterpret_cast<unsigned long long *>(lds) + mb_pick(r, lds_bytes / 8u), 1ull);
        } else if constexpr (KIND == MB_LDS_ADD_U32) {
            atomicAdd(reinterpret_cast<uint32_t *>(lds) + mb_pick(r, lds_bytes / 4u), 1u);
        } else if constexpr (KIND == MB_LDS_ADD_F64_ROW33) {
            double *row = reinterpret_cast<double *>(lds) + (size_t)mb_pick(r, lds_bytes / (8u * kRow)) * kRow;
#pragma unroll
            for (int c = 0; c < kRow; ++c) atomicAdd(row + c, 1.0);
        } else if constexpr (KIND == MB_LDS_ADD_U64_ROW33) {
            unsigned long long *row =
                reinterpret_cast<unsigned long long *>(lds) + (size_t)mb_pick(r, lds_bytes / (8u * kRow)) * kRow;
#pragma unroll
            for (int c = 0; c < kRow; ++c) atomicAdd(row + c, 1ull);
        } else {   // MB_LDS_ADD_U64_PRE: eight addresses drawn once per lane, reused in turn
            (void)r;
            unsigned long long *base = reinterpret_cast<unsigned long long *>(lds);
#pragma unroll
            for (int c = 0; c < 8; ++c) atomicAdd(base + pre[c], 1ull);
        }
    }
    __syncthreads();
    // The workgroup's total, block * iters adds of 1 (x 33 for rows): every
    // thread sums a strided share, the waves reduce theirs, and the wave sums
    // meet in the first words of LDS.  All partial sums are integers below
    // 2^53, so they are exact in any order.  (Summed by one thread, the 144
    // KiB of a 1024-thread workgroup cost ~0.3 ms, a third of a launch.)
    double v = 0.0;
    if constexpr (KIND == MB_LDS_ADD_F32 || KIND == MB_LDS_ADD_U32) {
        for (uint32_t i = threadIdx.x; i < lds_bytes / 4u; i += blockDim.x)
            v += KIND == MB_LDS_ADD_F32 ? (double)reinterpret_cast<float *>(lds)[i] : (double)w32[i];
    } else {
        constexpr bool integer = KIND == MB_LDS_ADD_U64 || KIND == MB_LDS_ADD_U64_ROW33 || KIND == MB_LDS_ADD_U64_PRE;
        for (uint32_t i = threadIdx.x; i < lds_bytes / 8u; i += blockDim.x)
            v += integer ? (double)reinterpret_cast<unsigned long long *>(lds)[i] : reinterpret_cast<double *>(lds)[i];
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    __syncthreads();   // every thread has read its share before the wave sums overwrite LDS
    double *wsum = reinterpret_cast<double *>(lds);
    if ((threadIdx.x & 63u) == 0) wsum[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (uint32_t w = 0; w < blockDim.x / 64u; ++w) t += wsum[w];
        sink[blockIdx.x] = t;
    }
    if (rec) {
        clk[0] = c0;
        clk[1] = clock64();
        clk[2] = w0;
        clk[3] = wall_clock64();
    }
}

__global__ void __launch_bounds__(256) k_global_atomics_f64(double *buf, uint32_t n, uint32_t iters, uint32_t seed) {
    const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t h = mb_hash(gid ^ (seed * 0x9e3779b9u));
    for (uint32_t it = 0; it < iters; ++it) {
        h = h * 1664525u + 1013904223u;
        unsafeAtomicAdd(buf + mb_pick(mb_hash(h), n), 1.0);
    }
}

// The finisher's pattern: each wave adds to runs of row_len consecutive
// doubles (one pixel's K sums) of random rows, consecutive lanes on
// consecutive elements, so one wave instruction covers about two rows.
__global__ void __launch_bounds__(256) k_global_atomics_rows_f64(double *buf, uint32_t n_rows, uint32_t row_len,
                                                                 uint32_t iters, uint32_t seed) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint32_t ws = mb_hash(wave ^ (seed * 0x9e3779b9u));
    for (uint32_t it = 0; it < iters; ++it) {
        const uint32_t e = lane + 64u * it;
        const uint32_t v = e / row_len, c = e - v * row_len;
        const uint32_t row = mb_pick(mb_hash(ws + v * 0x85ebca6bu), n_rows);
        __hip_atomic_fetch_add((__attribute__((address_space(1))) double *)(buf + (size_t)row * row_len + c), 1.0,
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// each workgroup copies one contiguous chunk of 4 x 256 16-byte elements:
// four independent loads in flight per thread, then their stores
__global__ void __launch_bounds__(256) k_copy16(const u32x4 *__restrict__ src, u32x4 *__restrict__ dst, uint64_t n) {
    const uint64_t base = (uint64_t)blockIdx.x * 1024u + threadIdx.x;
    u32x4 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
        if (base + u * 256u < n) v[u] = src[base + u * 256u];
#pragma unroll
    for (int u = 0; u < 4; ++u)
        if (base + u * 256u < n) dst[base + u * 256u] = v[u];
}

__global__ void __launch_bounds__(256) k_fma_f32(float *sink, uint32_t iters, uint64_t *clk) {
    const bool rec = clk != nullptr && blockIdx.x == 0 && threadIdx.x == 0;
    uint64_t c0 = 0, w0 = 0;
    if (rec) {
        c0 = clock64();
        w0 = wall_clock64();
    }
    const float x = (float)threadIdx.x * 1e-3f;
    float a[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) a[j] = x + (float)j;
    const float m = 0.999f, c = 1e-4f;
    for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
        for (int j = 0; j < 8; ++j) a[j] = __builtin_fmaf(a[j], m, c);
    }
    float s = 0.f;
#pragma unroll
    for (int j = 0; j < 8; ++j) s += a[j];
    sink[blockIdx.x * blockDim.x + threadIdx.x] = s;
    if (rec) {
        clk[0] = c0;
        clk[1] = clock64();
        clk[2] = w0;
        clk[3] = wall_clock64();
    }
}

template <int KIND>
mc_status launch_lds(uint32_t lds_bytes, uint32_t block, uint32_t n_blocks, uint32_t iters, uint32_t seed, double *sink,
                     uint64_t *clk, hipStream_t s) {
    if (hipFuncSetAttribute(reinterpret_cast<const void *>(&k_lds_atomics<KIND>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes) != hipSuccess)
        return MC_ERR_DEVICE;
    hipLaunchKernelGGL(k_lds_atomics<KIND>, dim3(n_blocks), dim3(block), lds_bytes, s, lds_bytes, iters, seed, sink, clk);
    return hipGetLastError() == hipSuccess ? MC_OK : MC_ERR_DEVICE;
}

}  // namespace

extern "C" {

mc_status mb_lds_atomics(int kind, uint32_t lds_bytes, uint32_t block, uint32_t n_blocks, uint32_t iters, uint32_t seed,
                         double *sink_d, uint64_t *clk_d, void *stream) {
    if (!sink_d || block == 0 || block > 1024 || block % 64 != 0 || n_blocks == 0 || iters == 0 || lds_bytes < 1024 ||
        lds_bytes > kMaxLds || lds_bytes % 8 != 0)
        return MC_ERR_INVALID_ARG;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    switch (kind) {
        case MB_LDS_ADD_F64: return launch_lds<MB_LDS_ADD_F64>(lds_bytes, block, n_blocks, iters, seed, sink_d, clk_d, s);
        case MB_LDS_ADD_F32: return launch_lds<MB_LDS_ADD_F32>(lds_bytes, block, n_blocks, iters, seed, sink_d, clk_d, s);
        case MB_LDS_ADD_U64: return launch_lds<MB_LDS_ADD_U64>(lds_bytes, block, n_blocks, iters, seed, sink_d, clk_d, s);
        case MB_LDS_ADD_U32: return launch_lds<MB_LDS_ADD_U32>(lds_bytes, block, n_blocks, iters, seed, sink_d, clk_d, s);
        case MB_LDS_ADD_F64_ROW33:
            return launch_lds<MB_LDS_ADD_F64_ROW33>(lds_bytes, block, n_blocks, iters, seed, sink_d, clk_d, s);
        case MB_LDS_ADD_U64_ROW33:
            return launch_lds<MB_LDS_ADD_U64_ROW33>(lds_bytes, block, n_blocks, iters, seed, sink_d, clk_d, s);
        case MB_LDS_ADD_U64_PRE:
            return launch_lds<MB_LDS_ADD_U64_PRE>(lds_bytes, block, n_blocks, iters, seed, sink_d, clk_d, s);
        default: return MC_ERR_INVALID_ARG;
    }
}

mc_status mb_global_atomics_f64(double *buf_d, uint64_t n_elem, uint32_t n_blocks, uint32_t iters, uint32_t seed,
                                void *stream) {
    if (!buf_d || n_elem == 0 || n_elem >= (1ull << 32) || n_blocks == 0 || iters == 0) return MC_ERR_INVALID_ARG;
    hipLaunchKernelGGL(k_global_atomics_f64, dim3(n_blocks), dim3(256), 0, reinterpret_cast<hipStream_t>(stream), buf_d,
                       (uint32_t)n_elem, iters, seed);
    return hipGetLastError() == hipSuccess ? MC_OK : MC_ERR_DEVICE;
}

mc_status mb_global_atomics_rows_f64(double *buf_d, uint32_t n_rows, uint32_t row_len, uint32_t n_blocks,
                                     uint32_t iters, uint32_t seed, void *stream) {
    if (!buf_d || n_rows == 0 || row_len == 0 || row_len > 4096 || (uint64_t)n_rows * row_len >= (1ull << 32) ||
        n_blocks == 0 || iters == 0 || (uint64_t)iters * 64u >= (1ull << 32))
        return MC_ERR_INVALID_ARG;
    hipLaunchKernelGGL(k_global_atomics_rows_f64, dim3(n_blocks), dim3(256), 0, reinterpret_cast<hipStream_t>(stream),
                       buf_d, n_rows, row_len, iters, seed);
    return hipGetLastError() == hipSuccess ? MC_OK : MC_ERR_DEVICE;
}

mc_status mb_copy(const void *src_d, void *dst_d, uint64_t n16, void *stream) {
    if (!src_d || !dst_d || n16 == 0 || (reinterpret_cast<uintptr_t>(src_d) & 15u) ||
        (reinterpret_cast<uintptr_t>(dst_d) & 15u))
        return MC_ERR_INVALID_ARG;
    const uintptr_t a = reinterpret_cast<uintptr_t>(src_d), b = reinterpret_cast<uintptr_t>(dst_d);
    if (a < b + 16u * n16 && b < a + 16u * n16) return MC_ERR_INVALID_ARG;   // overlap
    const uint64_t blocks = (n16 + 1023u) / 1024u;
    if (blocks > 0x7FFFFFFFull) return MC_ERR_INVALID_ARG;
    hipLaunchKernelGGL(k_copy16, dim3((unsigned)blocks), dim3(256), 0,
                       reinterpret_cast<hipStream_t>(stream), reinterpret_cast<const u32x4 *>(src_d),
                       reinterpret_cast<u32x4 *>(dst_d), n16);
    return hipGetLastError() == hipSuccess ? MC_OK : MC_ERR_DEVICE;
}

mc_status mb_fma_f32(float *sink_d, uint32_t n_blocks, uint32_t iters, uint64_t *clk_d, void *stream) {
    if (!sink_d || n_blocks == 0 || iters == 0) return MC_ERR_INVALID_ARG;
    hipLaunchKernelGGL(k_fma_f32, dim3(n_blocks), dim3(256), 0, reinterpret_cast<hipStream_t>(stream), sink_d, iters,
                       clk_d);
    return hipGetLastError() == hipSuccess ? MC_OK : MC_ERR_DEVICE;
}

mc_status mb_wall_clock_khz(int device, int *khz) {
    if (!khz) return MC_ERR_INVALID_ARG;
    return hipDeviceGetAttribute(khz, hipDeviceAttributeWallClockRate, device) == hipSuccess ? MC_OK : MC_ERR_DEVICE;
}

}  // extern "C"
