// mcrad.hip -- forward / adjoint radiance Monte Carlo with a harmonic angular
// tally on AMD Instinct MI355X (gfx950), behind the C ABI of include/mcrad.h.
//
// Method: Hochuli, Powell, Arridge & Cox, "Quantitative photoacoustic
// tomography using forward and adjoint Monte Carlo models of radiance"
// (arXiv:1608.05238).  Sec. 3: packet launch, free path, absorption
// weighting, 2D Henyey-Greenstein scattering, threshold termination.
// Sec. 3.1: harmonic tally.  Sec. 4: adjoint RTE.  Sec. 5: gradients.
// Sec. 6: adjoint source, signed weights, normalisation by packet count.
//
// GPU design (one process, one GPU):
//  * one lane per packet, persistent waves that refill dead lanes from a
//    global packet counter with one wave-aggregated atomic;
//  * FP32 transport in pixel-local coordinates (pixel index + offset in
//    [0,1]), so precision does not degrade with the grid size;
//  * the per-visit harmonic sum is accumulated in registers and flushed once
//    per pixel visit:
//      - LDS mode: the whole FP32 tally [npix][K] sits in LDS (small grids),
//        flushed to the FP64 tally with coalesced atomics when the workgroup
//        ends;
//      - global mode: flushing lanes stage their K-vectors in LDS and the
//        wave issues them as contiguous runs of atomics into an FP32 tally
//        [npix][K] in HBM (one or two cache lines per visit instead of K
//        scattered lines), folded into FP64 after every chunk of packets.
//  * no MFMA: the transport is not a dense contraction.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <mutex>
#include <vector>

#include "mcrad.h"

namespace {

constexpr int kMaxSrc = 8;
constexpr int kMaxProf = 2 * (2 * MC_NHARM_MAX + 1);  // profile coefficients over all sources
constexpr int kBlock = 256;                            // global mode: threads per workgroup (4 waves)
constexpr int kWaves = kBlock / 64;
constexpr int kBlockLds = 512;                         // LDS mode: threads sharing one LDS tally copy
constexpr uint64_t kChunk = 1ull << 22;                // packets per launch
constexpr size_t kLdsTallyMax = 144 * 1024;            // LDS bytes for the in-LDS tally mode
constexpr float kPi = 3.14159265358979323846f;
constexpr uint32_t kMaxInteractions = 1u << 24;         // hard cap per packet (guards invalid media)

enum : int { EV_LAUNCH = 0, EV_CROSS = 1, EV_SCATTER = 2, EV_ESCAPE = 3, EV_KILL = 4, EV_NONE = 5 };

struct SrcDev {
    int kind, lambertian, prof_off, n_prof;
    double x0, z0, x1, z1;      // mm
    float dir_x, dir_z;
    double cum;                 // inclusive prefix of the sampling measure
};

struct Params {
    int nx, nz, npix, nsrc;
    float dx;
    int adjoint;
    uint32_t tag, flags;
    uint64_t seed, pid0, npk;   // packet range of this launch
    float wth, rm, inv_rm;
    double total;
    const float4 *med;          // {mua dx, mus dx, 1/(mua dx), 1/(mus dx)}
    const float *g;
    const double *map;          // MAP source values (sign)
    const double *cdf;          // MAP: inclusive prefix of |map|
    float *t32;                 // global mode FP32 tally [npix][K]
    double *t64;                // FP64 tally [npix][K]
    unsigned long long *counter;
    double *led;                // 5 doubles
    unsigned long long *ledc;   // 4 counters
    SrcDev src[kMaxSrc];
    float prof[kMaxProf];
};

// ------------------------------------------------------------------ Philox
// Philox4x32-10 (Salmon et al., SC'11): 10 rounds of two 32x32->64-bit
// products; key bumped by the Weyl constants between rounds.
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint32_t lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
        const uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
    }
    return c;
}

__device__ __forceinline__ uint4 rng_block(const Params &P, uint64_t pid, uint32_t j) {
    return philox4x32_10(make_uint4(j, P.tag, (uint32_t)pid, (uint32_t)(pid >> 32)),
                         (uint32_t)P.seed, (uint32_t)(P.seed >> 32));
}

// u in (0,1): top 23 bits centred in their cell; exact in FP32.
__device__ __forceinline__ float u01(uint32_t x) { return (float)(x >> 9) * 0x1p-23f + 0x1p-24f; }

// ------------------------------------------------------------------ packet
struct Packet {
    int ix, iz;
    float fx, fz;      // offset inside the pixel, pixel units
    float sx, sz;      // direction (sin t, cos t)
    float isx, isz;    // reciprocals (inf for a zero component)
    float w, w0abs;
    float tau;         // optical depth left on the current free path
    float uh, ur;      // HG and roulette uniforms of the current block
    uint32_t k;        // current block index
    uint64_t pid;
    bool alive;
};

struct LedgerRegs {
    double launched = 0, absorbed = 0, escaped = 0, gain = 0, loss = 0;
    uint32_t packets = 0, segments = 0, visits = 0, scatters = 0;
};

template <int NH>
__device__ __forceinline__ void harmonics(float sx, float sz, float *h) {
    // h = [1, cos t .. cos Nt, sin t .. sin Nt] from z = cos t + i sin t
    h[0] = 1.f;
    float re = sz, im = sx;
#pragma unroll
    for (int n = 1; n <= NH; ++n) {
        h[n] = re;
        h[NH + n] = im;
        const float nre = re * sz - im * sx;
        const float nim = re * sx + im * sz;
        re = nre;
        im = nim;
    }
}

// Angular profile p(t) = c0/2pi + (1/pi) sum (c_n cos nt + s_n sin nt).
__device__ __forceinline__ float profile(const Params &P, const SrcDev &s, float sx, float sz) {
    const float *c = P.prof + s.prof_off;
    float p = c[0] * (0.5f / kPi);
    float re = sz, im = sx;
    for (int n = 1; n <= s.n_prof; ++n) {
        p += (c[n] * re + c[s.n_prof + n] * im) * (1.f / kPi);
        const float nre = re * sz - im * sx;
        const float nim = re * sx + im * sz;
        re = nre;
        im = nim;
    }
    return p;
}

__device__ __forceinline__ void set_dir(Packet &p, float sx, float sz) {
    p.sx = sx;
    p.sz = sz;
    p.isx = sx != 0.f ? 1.f / sx : INFINITY;
    p.isz = sz != 0.f ? 1.f / sz : INFINITY;
}

// Draw block k: free path (optical depth) and the uniforms used at its end.
__device__ __forceinline__ void new_leg(const Params &P, Packet &p) {
    const uint4 r = rng_block(P, p.pid, p.k);
    p.tau = -logf(u01(r.x));
    p.uh = u01(r.y);
    p.ur = u01(r.z);
}

// Snap distance (pixels) for points given on the outer boundary: a float
// coordinate of a point on the boundary is only known to a few ulp of its
// magnitude, i.e. to ~n 2^-24 pixels.
__host__ __device__ __forceinline__ double boundary_snap(int n) { return 1e-6 + 4.0 * n * 0x1p-24; }

// Pixel of a point given in pixel units; points on a face moving towards the
// lower index belong to the lower pixel; points within boundary_snap() of the
// outer boundary are taken to be on it.
__device__ __forceinline__ void locate1(double a, int n, float s, int &i, float &f) {
    const double tol = boundary_snap(n);
    if (fabs(a) < tol) a = 0.0;
    if (fabs(a - n) < tol) a = n;
    double fl = floor(a);
    int ii = (int)fl;
    if (a == fl && s < 0.f) ii -= 1;
    i = ii;
    f = (float)(a - ii);
}

// Launch (Sec. 3; Sec. 6 for the volumetric signed source).  Returns false
// if the packet starts outside the grid (it then escapes at once).
template <int NH>
__device__ bool launch(const Params &P, uint64_t pid, Packet &p, float *h, LedgerRegs &L) {
    const uint4 r = rng_block(P, pid, 0);
    const float u0 = u01(r.x), u1 = u01(r.y), u2 = u01(r.z), u3 = u01(r.w);
    int s = 0;
    if (P.nsrc > 1) {
        const double t = (double)u0 * P.total;
        while (s < P.nsrc - 1 && !(P.src[s].cum > t)) ++s;
    }
    const SrcDev &S = P.src[s];
    const float flip = P.adjoint ? -1.f : 1.f;
    double ax, az;   // position in pixel units
    float sx, sz, w0 = 1.f;
    if (S.kind == MC_SRC_PENCIL || S.kind == MC_SRC_LINE) {
        const double lu = S.kind == MC_SRC_LINE ? (double)u1 : 0.0;
        ax = (S.x0 + lu * (S.x1 - S.x0)) / (double)P.dx;
        az = (S.z0 + lu * (S.z1 - S.z0)) / (double)P.dx;
        sx = flip * S.dir_x;
        sz = flip * S.dir_z;
        if (S.kind == MC_SRC_LINE && S.lambertian) {   // sin(alpha) uniform on (-1,1)
            const float sa = 2.f * u2 - 1.f, ca = sqrtf(fmaxf(0.f, 1.f - sa * sa));
            const float nx_ = sx * ca + sz * sa, nz_ = sz * ca - sx * sa;
            sx = nx_;
            sz = nz_;
        }
    } else if (S.kind == MC_SRC_POINT) {
        ax = S.x0 / (double)P.dx;
        az = S.z0 / (double)P.dx;
        sincospif(2.f * u2 - 1.f, &sx, &sz);
        w0 = 2.f * kPi * profile(P, S, sx, sz);
    } else {   // MAP: pixel with probability |q_i| / sum |q|, uniform inside it
        const double t = (double)u0 * P.cdf[P.npix - 1];
        int lo = 0, hi = P.npix - 1;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (P.cdf[mid] > t) hi = mid; else lo = mid + 1;
        }
        const int ixs = lo % P.nx, izs = lo / P.nx;
        ax = ixs + (double)u1;
        az = izs + (double)u2;
        sincospif(2.f * u3 - 1.f, &sx, &sz);
        w0 = (P.map[lo] < 0.0 ? -2.f : 2.f) * kPi * profile(P, S, sx, sz);
    }
    p.pid = pid;
    p.k = 1;
    p.w = w0;
    p.w0abs = fabsf(w0);
    set_dir(p, sx, sz);
    L.launched += w0;
    L.packets += 1;
    locate1(ax, P.nx, sx, p.ix, p.fx);
    locate1(az, P.nz, sz, p.iz, p.fz);
    if (p.ix < 0 || p.ix >= P.nx || p.iz < 0 || p.iz >= P.nz) {
        L.escaped += w0;
        p.alive = false;
        return false;
    }
    p.alive = true;
    harmonics<NH>(sx, sz, h);
    new_leg(P, p);
    return true;
}

// One segment: run to the next pixel face or to the end of the free path,
// depositing the track length weighted by the decaying weight (Sec. 3).
// Returns EV_CROSS, EV_ESCAPE or EV_SCATTER; T (pixel units) and the pixel
// of the segment are returned through the references.
__device__ __forceinline__ int step(const Params &P, Packet &p, float &T, float &dw, int &pix) {
    pix = p.iz * P.nx + p.ix;
    const float4 m = P.med[pix];
    const float dfx = p.sx > 0.f ? (1.f - p.fx) * p.isx : (p.sx < 0.f ? -p.fx * p.isx : INFINITY);
    const float dfz = p.sz > 0.f ? (1.f - p.fz) * p.isz : (p.sz < 0.f ? -p.fz * p.isz : INFINITY);
    const float d = fminf(dfx, dfz);
    const float od = m.y * d;
    const bool scat = od > p.tau;
    const float l = scat ? p.tau * m.w : d;
    dw = -p.w * expm1f(-m.x * l);     // weight absorbed on the segment
    T = m.x > 0.f ? dw * m.z : p.w * l;
    p.w -= dw;
    if (scat) {
        p.fx = fminf(fmaxf(p.fx + l * p.sx, 0.f), 1.f);
        p.fz = fminf(fmaxf(p.fz + l * p.sz, 0.f), 1.f);
        return EV_SCATTER;
    }
    p.tau -= od;
    if (dfx <= dfz) {
        if (p.sx > 0.f) { p.ix += 1; p.fx = 0.f; } else { p.ix -= 1; p.fx = 1.f; }
    } else {
        p.fx = fminf(fmaxf(p.fx + l * p.sx, 0.f), 1.f);
    }
    if (dfz <= dfx) {
        if (p.sz > 0.f) { p.iz += 1; p.fz = 0.f; } else { p.iz -= 1; p.fz = 1.f; }
    } else {
        p.fz = fminf(fmaxf(p.fz + l * p.sz, 0.f), 1.f);
    }
    if (p.ix < 0 || p.ix >= P.nx || p.iz < 0 || p.iz >= P.nz) return EV_ESCAPE;
    return EV_CROSS;
}

// Scatter site: termination test on |W| (Sec. 3, Sec. 6), then the 2D HG
// deflection (eq. scattering_angle) written without atan/tan: with
// a = (1+g) cos(pi(u-1/2)), b = (1-g) sin(pi(u-1/2)), tan(dt/2) = b/a, so
// cos dt = (a^2-b^2)/(a^2+b^2), sin dt = 2ab/(a^2+b^2).  Returns false if
// the packet was killed.
template <int NH>
__device__ __forceinline__ bool scatter(const Params &P, Packet &p, float *h, LedgerRegs &L) {
    if (p.k >= kMaxInteractions) {
        L.loss += p.w;
        p.alive = false;
        return false;
    }
    if (fabsf(p.w) < P.wth * p.w0abs) {
        if ((P.flags & MC_FLAG_LITERAL_TRUNCATION) || !(p.ur < P.inv_rm)) {
            L.loss += p.w;
            p.alive = false;
            return false;
        }
        L.gain += (double)((P.rm - 1.f) * p.w);
        p.w *= P.rm;
    }
    const float g = P.g[p.iz * P.nx + p.ix];
    float sp, cp;
    sincospif(p.uh - 0.5f, &sp, &cp);
    const float a = (1.f + g) * cp, b = (1.f - g) * sp;
    const float inv = 1.f / (a * a + b * b);
    const float cd = (a * a - b * b) * inv, sd = 2.f * a * b * inv;
    float nx_ = p.sx * cd + p.sz * sd;
    float nz_ = p.sz * cd - p.sx * sd;
    const float rn = rsqrtf(nx_ * nx_ + nz_ * nz_);
    nx_ *= rn;
    nz_ *= rn;
    set_dir(p, nx_, nz_);
    harmonics<NH>(nx_, nz_, h);
    L.scatters += 1;
    p.k += 1;
    new_leg(P, p);
    return true;
}

__device__ __forceinline__ void ledger_flush(const Params &P, LedgerRegs &L) {
    double v[5] = {L.launched, L.absorbed, L.escaped, L.gain, L.loss};
    unsigned long long c[4] = {L.packets, L.segments, L.visits, L.scatters};
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
        for (int i = 0; i < 5; ++i) v[i] += __shfl_xor(v[i], off);
#pragma unroll
        for (int i = 0; i < 4; ++i) c[i] += __shfl_xor(c[i], off);
    }
    if (__lane_id() == 0) {
        for (int i = 0; i < 5; ++i) atomicAdd(P.led + i, v[i]);
        for (int i = 0; i < 4; ++i) atomicAdd(P.ledc + i, c[i]);
    }
}

// ------------------------------------------------------------------ transport kernel
// LDS_TALLY: the FP32 tally [npix][K] lives in LDS for the workgroup's life.
// Otherwise flushes go to the FP32 HBM tally through per-wave LDS staging.
template <int NH, bool LDS_TALLY>
__global__ void __launch_bounds__(LDS_TALLY ? kBlockLds : kBlock) k_transport(Params P) {
    constexpr int K = 2 * NH + 1;
    extern __shared__ float smem[];
    const int lane = __lane_id();
    const int wave = threadIdx.x >> 6;
    float *stage = smem + wave * 64 * K;                              // global mode
    int *stage_pix = reinterpret_cast<int *>(smem + kWaves * 64 * K) + wave * 64;

    if (LDS_TALLY) {
        for (int i = threadIdx.x; i < P.npix * K; i += blockDim.x) smem[i] = 0.f;
        __syncthreads();
    }

    Packet p;
    p.alive = false;
    float h[K], acc[K];
#pragma unroll
    for (int j = 0; j < K; ++j) acc[j] = 0.f;
    LedgerRegs L;
    bool more = true;
    const unsigned long long lt_mask = (1ull << lane) - 1ull;

    for (;;) {
        // refill dead lanes with one wave-aggregated atomic on the packet counter
        if (more) {
            const unsigned long long dead = __ballot(!p.alive);
            if (dead) {
                const int ndead = __popcll(dead);
                const int leader = __ffsll((long long)dead) - 1;
                unsigned long long base = 0;
                if (lane == leader) base = atomicAdd(P.counter, (unsigned long long)ndead);
                base = __shfl(base, leader);
                if (base + ndead >= P.npk) more = false;
                if (!p.alive) {
                    const unsigned long long my = base + __popcll(dead & lt_mask);
                    if (my < P.npk) launch<NH>(P, P.pid0 + my, p, h, L);
                }
            }
        }
        if (!__ballot(p.alive)) {
            if (!more) break;
            continue;
        }
        bool flush = false;
        int pix = 0;
        if (p.alive) {
            float T, dw;
            const int ev = step(P, p, T, dw, pix);
#pragma unroll
            for (int j = 0; j < K; ++j) acc[j] = fmaf(T, h[j], acc[j]);
            L.absorbed += (double)dw;
            L.segments += 1;
            if (ev == EV_SCATTER) {
                if (!scatter<NH>(P, p, h, L)) flush = true;
            } else {
                flush = true;
                if (ev == EV_ESCAPE) {
                    L.escaped += p.w;
                    p.alive = false;
                }
            }
            if (flush) L.visits += 1;
        }
        if (LDS_TALLY) {
            if (flush) {
                float *t = smem + pix * K;
#pragma unroll
                for (int j = 0; j < K; ++j) {
                    atomicAdd(t + j, acc[j]);
                    acc[j] = 0.f;
                }
            }
        } else {
            const unsigned long long fm = __ballot(flush);
            if (fm) {
                const int nf = __popcll(fm);
                if (flush) {
                    const int slot = __popcll(fm & lt_mask);
                    float *st = stage + slot * K;
#pragma unroll
                    for (int j = 0; j < K; ++j) {
                        st[j] = acc[j];
                        acc[j] = 0.f;
                    }
                    stage_pix[slot] = pix;
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                const int total = nf * K;
                for (int e = lane; e < total; e += 64) {
                    const int v = e / K;
                    const int j = e - v * K;
                    const float val = stage[e];
                    if (val != 0.f) unsafeAtomicAdd(P.t32 + (size_t)stage_pix[v] * K + j, val);
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            }
        }
    }
    ledger_flush(P, L);
    if (LDS_TALLY) {
        __syncthreads();
        for (int i = threadIdx.x; i < P.npix * K; i += blockDim.x) {
            const float v = smem[i];
            if (v != 0.f) unsafeAtomicAdd(P.t64 + i, (double)v);
        }
    }
}

// ------------------------------------------------------------------ trace kernel
// Runs the listed packets one after the other through the same device
// functions as k_transport and records every event.
template <int NH>
__global__ void k_trace(Params P, const uint64_t *pids, int n_pids, mc_event *ev, size_t cap,
                        unsigned long long *n_ev) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    constexpr int K = 2 * NH + 1;
    float h[K];
    LedgerRegs L;
    size_t n = 0;
    auto rec = [&](const Packet &p, int type, int k, int ix, int iz, float w, float t) {
        if (n < cap) {
            mc_event e;
            e.pid = p.pid;
            e.k = k;
            e.type = type;
            e.ix = ix;
            e.iz = iz;
            e.x = ((float)p.ix + p.fx) * P.dx;
            e.z = ((float)p.iz + p.fz) * P.dx;
            e.sx = p.sx;
            e.sz = p.sz;
            e.w = w;
            e.t = t * P.dx;
            ev[n] = e;
        }
        ++n;
    };
    for (int q = 0; q < n_pids; ++q) {
        Packet p;
        const bool in = launch<NH>(P, pids[q], p, h, L);
        rec(p, EV_LAUNCH, 0, p.ix, p.iz, p.w, 0.f);
        if (!in) {
            rec(p, EV_ESCAPE, 0, p.ix, p.iz, p.w, 0.f);
            continue;
        }
        while (p.alive) {
            const int ix = p.ix, iz = p.iz, k = (int)p.k;
            float T, dw;
            int pix;
            const int e = step(P, p, T, dw, pix);
            if (e == EV_SCATTER) {
                if (scatter<NH>(P, p, h, L)) rec(p, EV_SCATTER, k, ix, iz, p.w, T);
                else rec(p, EV_KILL, k, ix, iz, p.w, T);
            } else if (e == EV_ESCAPE) {
                p.alive = false;
                rec(p, EV_ESCAPE, k, ix, iz, p.w, T);
            } else {
                rec(p, EV_CROSS, k, ix, iz, p.w, T);
            }
        }
    }
    *n_ev = n;
}

// ------------------------------------------------------------------ setup / post kernels
__global__ void k_setup_medium(int npix, float dx, const float *mua, const float *mus, float4 *med) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npix) return;
    const float a = mua[i] * dx, s = mus[i] * dx;
    med[i] = make_float4(a, s, a > 0.f ? 1.f / a : 0.f, s > 0.f ? 1.f / s : 0.f);
}

__global__ void k_fill_zero(uint32_t *p, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

// Single-block inclusive scan of |map| in FP64 (fixed order: each thread a
// contiguous run, then a sequential pass over the 1024 run totals).
__global__ void __launch_bounds__(1024) k_map_cdf(int n, const double *map, double *cdf) {
    __shared__ double part[1024];
    const int t = threadIdx.x;
    const int per = (n + 1023) / 1024;
    const int a = t * per, b = min(n, a + per);
    double s = 0;
    for (int i = a; i < b; ++i) s += fabs(map[i]);
    part[t] = s;
    __syncthreads();
    if (t == 0) {
        double acc = 0;
        for (int i = 0; i < 1024; ++i) {
            const double v = part[i];
            part[i] = acc;
            acc += v;
        }
    }
    __syncthreads();
    s = part[t];
    for (int i = a; i < b; ++i) {
        s += fabs(map[i]);
        cdf[i] = s;
    }
}

__global__ void k_fold(size_t n, float *t32, double *t64) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const float v = t32[i];
        if (v != 0.f) {
            t64[i] += (double)v;
            t32[i] = 0.f;
        }
    }
}

// Normalise (Sec. 6: divide by the packet count; times the source measure and
// the track-length-to-fluence factor 1/(dx Np) in pixel units) and transpose
// [npix][K] -> [K][npix]; the adjoint output reads the mirrored direction,
// (-1)^n on orders n >= 1.
__global__ void k_normalise(int npix, int N, int adjoint, double scale, const double *t64, double *out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npix) return;
    const int K = 2 * N + 1;
    for (int c = 0; c < K; ++c) {
        const int n = c <= N ? c : c - N;
        const double f = (adjoint && (n & 1)) ? -scale : scale;
        out[(size_t)c * npix + i] = t64[(size_t)i * K + c] * f;
    }
}

__global__ void k_ledger_out(const double *led, const unsigned long long *ledc, double scale, mc_ledger *out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    out->launched = led[0];
    out->absorbed = led[1];
    out->escaped = led[2];
    out->roulette_gain = led[3];
    out->roulette_loss = led[4];
    out->scale = scale;
    out->packets = ledc[0];
    out->segments = ledc[1];
    out->visits = ledc[2];
    out->scatters = ledc[3];
}

// Residual (Sec. 2, Sec. 6) with a deterministic single-block reduction of eps.
__global__ void __launch_bounds__(1024) k_residual(int npix, double area, const float *mua, const double *a0,
                                                   const double *hmeas, double *qs, double *eps) {
    __shared__ double red[1024];
    double s = 0;
    for (int i = threadIdx.x; i < npix; i += 1024) {
        const double m = mua[i];
        const double r = hmeas[i] - m * a0[i];
        if (qs) qs[i] = m * r;
        s += r * r;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 512; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *eps = 0.5 * area * red[0];
}

// Gradients (Sec. 5: eqs. grad_2D_abs_integral3, scattering_gradient3).
__global__ void k_gradient(int npix, int N, double area, const float *mua, const float *g, const double *fwd,
                           const double *adj, const double *hmeas, double *dmua, double *dmus) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npix) return;
    const double a0 = fwd[i], a0s = adj[i];
    const double r = hmeas[i] - (double)mua[i] * a0;
    const double gi = g[i];
    double all = 0, wg = 0, gn = 1;
    for (int n = 1; n <= N; ++n) {
        gn *= gi;
        const double pr = fwd[(size_t)n * npix + i] * adj[(size_t)n * npix + i] +
                          fwd[(size_t)(N + n) * npix + i] * adj[(size_t)(N + n) * npix + i];
        all += pr;
        wg += pr * (1.0 - gn);
    }
    const double ip = 0.31830988618379067154;   // 1/pi
    if (dmua) dmua[i] = area * (-a0 * r + a0 * a0s * (0.5 * ip) + all * ip);
    if (dmus) dmus[i] = area * (wg * ip);
}

__global__ void __launch_bounds__(1024) k_detect(int npix, int N, double area, const double *c, const double *d,
                                                 double *out) {
    __shared__ double red[1024];
    const double ip = 0.31830988618379067154;
    double s = 0;
    for (int i = threadIdx.x; i < npix; i += 1024) {
        double v = c[i] * d[i] * (0.5 * ip);
        for (int n = 1; n <= N; ++n)
            v += (c[(size_t)n * npix + i] * d[(size_t)n * npix + i] +
                  c[(size_t)(N + n) * npix + i] * d[(size_t)(N + n) * npix + i]) * ip;
        s += v;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 512; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = area * red[0];
}

__global__ void k_philox_fill(uint64_t seed, uint32_t tag, uint64_t pid0, uint64_t n, uint32_t j, uint32_t *out) {
    const uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t pid = pid0 + i;
    const uint4 r = philox4x32_10(make_uint4(j, tag, (uint32_t)pid, (uint32_t)(pid >> 32)), (uint32_t)seed,
                                  (uint32_t)(seed >> 32));
    out[4 * i + 0] = r.x;
    out[4 * i + 1] = r.y;
    out[4 * i + 2] = r.z;
    out[4 * i + 3] = r.w;
}

// ------------------------------------------------------------------ dispatch tables
using TransportFn = void (*)(Params);
using TraceFn = void (*)(Params, const uint64_t *, int, mc_event *, size_t, unsigned long long *);

template <int NH>
struct Table {
    static void fill(TransportFn *lds, TransportFn *glb, TraceFn *tr) {
        lds[NH] = k_transport<NH, true>;
        glb[NH] = k_transport<NH, false>;
        tr[NH] = k_trace<NH>;
        if constexpr (NH > 0) Table<NH - 1>::fill(lds, glb, tr);
    }
};

struct Kernels {
    TransportFn lds[MC_NHARM_MAX + 1], glb[MC_NHARM_MAX + 1];
    TraceFn tr[MC_NHARM_MAX + 1];
    Kernels() { Table<MC_NHARM_MAX>::fill(lds, glb, tr); }
};

const Kernels &kernels() {
    static Kernels k;
    return k;
}

// ------------------------------------------------------------------ host helpers
size_t align_up(size_t v) { return (v + 255) & ~size_t(255); }

// Optional timing of the transport launches with HIP events recorded on the
// launch stream (enabled by mc_profile_enable; read by mc_profile_read).
struct Profile {
    std::mutex mu;
    bool on = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
    double ms = 0;
    uint64_t launches = 0;
};
Profile &profile_state() {
    static Profile p;
    return p;
}

struct Layout {
    size_t med, cdf, t64, t32, led, ledc, counters, total;
    uint64_t n_chunks;
    bool lds_mode;
};

bool lds_fits(int npix, int K) {
    return (size_t)npix * K * sizeof(float) <= kLdsTallyMax;
}

Layout layout(const mc_medium *m, const mc_source *src, const mc_run *run) {
    Layout L{};
    const size_t npix = (size_t)m->nx * m->nz;
    const int K = 2 * run->n_harm + 1;
    L.lds_mode = lds_fits((int)npix, K);
    L.n_chunks = (run->n_packets + kChunk - 1) / kChunk;
    size_t off = 0;
    L.med = off;
    off = align_up(off + npix * sizeof(float4));
    L.cdf = off;
    if (src[0].kind == MC_SRC_MAP) off = align_up(off + npix * sizeof(double));
    L.t64 = off;
    off = align_up(off + npix * K * sizeof(double));
    L.t32 = off;
    if (!L.lds_mode) off = align_up(off + npix * K * sizeof(float));
    L.led = off;
    off = align_up(off + 8 * sizeof(double));
    L.ledc = off;
    off = align_up(off + 8 * sizeof(unsigned long long));
    L.counters = off;
    off = align_up(off + L.n_chunks * sizeof(unsigned long long));
    L.total = off;
    return L;
}

mc_status validate(const mc_medium *m, const mc_source *src, int n_src, const mc_run *run) {
    if (!m || !src || !run) return MC_ERR_INVALID_ARG;
    if (m->nx <= 0 || m->nz <= 0 || !(m->dx > 0.f) || !m->mua_d || !m->mus_d || !m->g_d) return MC_ERR_INVALID_ARG;
    if ((int64_t)m->nx * m->nz > (1 << 26)) return MC_ERR_UNSUPPORTED;
    if (run->n_harm < 0 || run->n_harm > MC_NHARM_MAX || run->n_packets == 0) return MC_ERR_INVALID_ARG;
    if (!(run->roulette_m > 1.f) || !(run->w_threshold >= 0.f)) return MC_ERR_INVALID_ARG;
    if (n_src < 1 || n_src > kMaxSrc) return MC_ERR_INVALID_ARG;
    const double W = (double)m->nx * m->dx, H = (double)m->nz * m->dx;
    const double tx = boundary_snap(m->nx) * m->dx, tz = boundary_snap(m->nz) * m->dx;
    int prof_total = 0;
    for (int s = 0; s < n_src; ++s) {
        const mc_source &q = src[s];
        if (q.kind < MC_SRC_PENCIL || q.kind > MC_SRC_MAP) return MC_ERR_INVALID_ARG;
        if (q.kind == MC_SRC_MAP) {
            if (n_src != 1 || !q.map_d) return MC_ERR_INVALID_ARG;
        } else {
            if (!(q.power > 0)) return MC_ERR_INVALID_ARG;
            const int np = q.kind == MC_SRC_LINE ? 2 : 1;
            const double pts[2][2] = {{q.x0, q.z0}, {q.x1, q.z1}};
            for (int k = 0; k < np; ++k)
                if (!(pts[k][0] >= -tx && pts[k][0] <= W + tx && pts[k][1] >= -tz && pts[k][1] <= H + tz))
                    return MC_ERR_INVALID_ARG;
            if (q.kind != MC_SRC_POINT && q.kind != MC_SRC_MAP && std::fabs(std::hypot((double)q.dir_x, (double)q.dir_z) - 1.0) > 1e-5)
                return MC_ERR_INVALID_ARG;
        }
        if (q.kind == MC_SRC_POINT || q.kind == MC_SRC_MAP) {
            if (q.prof_h) {
                if (q.n_prof < 0 || q.n_prof > MC_NHARM_MAX) return MC_ERR_INVALID_ARG;
                prof_total += 2 * q.n_prof + 1;
            } else {
                prof_total += 1;
            }
        }
    }
    if (prof_total > kMaxProf) return MC_ERR_UNSUPPORTED;
    return MC_OK;
}

// Build kernel parameters.  map_total: sum |map| (MAP source) computed on
// the host for the normalisation; the device CDF is built separately.
void fill_params(Params &P, const mc_medium *m, const mc_source *src, int n_src, const mc_run *run, int adjoint,
                 double map_abs_sum) {
    std::memset(&P, 0, sizeof(P));
    P.nx = m->nx;
    P.nz = m->nz;
    P.npix = m->nx * m->nz;
    P.nsrc = n_src;
    P.dx = m->dx;
    P.adjoint = adjoint;
    P.tag = run->stream_tag;
    P.flags = run->flags;
    P.seed = run->seed;
    P.wth = run->w_threshold;
    P.rm = run->roulette_m;
    P.inv_rm = 1.f / run->roulette_m;
    P.g = m->g_d;
    double total = 0;
    int poff = 0;
    const double A = (double)m->dx * m->dx;
    for (int s = 0; s < n_src; ++s) {
        const mc_source &q = src[s];
        SrcDev &d = P.src[s];
        d.kind = q.kind;
        d.lambertian = q.lambertian;
        d.x0 = q.x0; d.z0 = q.z0; d.x1 = q.x1; d.z1 = q.z1;
        d.dir_x = q.dir_x; d.dir_z = q.dir_z;
        d.prof_off = poff;
        d.n_prof = 0;
        if (q.kind == MC_SRC_POINT || q.kind == MC_SRC_MAP) {
            if (q.prof_h) {
                const int n = q.n_prof;
                d.n_prof = n;
                for (int k = 0; k <= 2 * n; ++k) {
                    const int order = k <= n ? k : k - n;
                    // adjoint: mirrored profile p(t + pi)
                    const double sg = (adjoint && (order & 1)) ? -1.0 : 1.0;
                    P.prof[poff + k] = (float)(q.prof_h[k] * sg);
                }
                poff += 2 * n + 1;
            } else {
                P.prof[poff++] = 1.f;
            }
        }
        total += q.kind == MC_SRC_MAP ? 2.0 * M_PI * map_abs_sum * A : q.power;
        d.cum = total;
    }
    P.total = total;
    if (n_src == 1 && src[0].kind == MC_SRC_MAP) P.map = src[0].map_d;
}

int occupancy_blocks(TransportFn fn, int block, size_t lds) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void *>(fn), block, lds) != hipSuccess ||
        nb < 1)
        nb = 1;
    return nb;
}

int device_cus() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) return 256;
    return cus;
}

mc_status launch_zero(void *p, size_t bytes, hipStream_t st) {
    const size_t n = bytes / 4;
    if (!n) return MC_OK;
    const unsigned grid = (unsigned)std::min<size_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_fill_zero, dim3(grid), dim3(256), 0, st, (uint32_t *)p, n);
    return hipGetLastError() == hipSuccess ? MC_OK : MC_ERR_DEVICE;
}

mc_status run_mc(const mc_medium *m, const mc_source *src, int n_src, const mc_run *run, double *coeffs,
                 mc_ledger *ledger, void *ws, size_t ws_bytes, void *stream, int adjoint) {
    mc_status st = validate(m, src, n_src, run);
    if (st != MC_OK) return st;
    if (!coeffs) return MC_ERR_INVALID_ARG;
    const Layout L = layout(m, src, run);
    if (!ws || ws_bytes < L.total || (reinterpret_cast<uintptr_t>(ws) & 255)) return MC_ERR_WORKSPACE;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    char *base = static_cast<char *>(ws);
    const int npix = m->nx * m->nz;
    const int N = run->n_harm, K = 2 * N + 1;

    double map_abs_sum = 0;
    const bool is_map = src[0].kind == MC_SRC_MAP;
    Params P;
    fill_params(P, m, src, n_src, run, adjoint, 0.0);
    P.med = reinterpret_cast<const float4 *>(base + L.med);
    P.t64 = reinterpret_cast<double *>(base + L.t64);
    P.t32 = L.lds_mode ? nullptr : reinterpret_cast<float *>(base + L.t32);
    P.led = reinterpret_cast<double *>(base + L.led);
    P.ledc = reinterpret_cast<unsigned long long *>(base + L.ledc);

    // zero the tallies, ledger and packet counters
    if ((st = launch_zero(base + L.t64, L.counters + L.n_chunks * 8 - L.t64, s)) != MC_OK) return st;
    hipLaunchKernelGGL(k_setup_medium, dim3((npix + 255) / 256), dim3(256), 0, s, npix, m->dx, m->mua_d, m->mus_d,
                       reinterpret_cast<float4 *>(base + L.med));
    if (is_map) {
        double *cdf = reinterpret_cast<double *>(base + L.cdf);
        hipLaunchKernelGGL(k_map_cdf, dim3(1), dim3(1024), 0, s, npix, src[0].map_d, cdf);
        // the normalisation needs sum |q|: read the last CDF entry
        if (hipMemcpyAsync(&map_abs_sum, cdf + npix - 1, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return MC_ERR_DEVICE;
        if (!(map_abs_sum > 0)) return MC_ERR_INVALID_ARG;
        fill_params(P, m, src, n_src, run, adjoint, map_abs_sum);
        P.med = reinterpret_cast<const float4 *>(base + L.med);
        P.t64 = reinterpret_cast<double *>(base + L.t64);
        P.t32 = L.lds_mode ? nullptr : reinterpret_cast<float *>(base + L.t32);
        P.led = reinterpret_cast<double *>(base + L.led);
        P.ledc = reinterpret_cast<unsigned long long *>(base + L.ledc);
        P.cdf = cdf;
    }
    if (hipGetLastError() != hipSuccess) return MC_ERR_DEVICE;

    const Kernels &KT = kernels();
    const TransportFn fn = L.lds_mode ? KT.lds[N] : KT.glb[N];
    const size_t lds = L.lds_mode ? (size_t)npix * K * sizeof(float)
                                  : (size_t)kWaves * 64 * K * sizeof(float) + kWaves * 64 * sizeof(int);
    const int block = L.lds_mode ? kBlockLds : kBlock;
    if (L.lds_mode && lds > 64 * 1024 &&
        hipFuncSetAttribute(reinterpret_cast<const void *>(fn), hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) !=
            hipSuccess)
        return MC_ERR_DEVICE;
    const int occ = occupancy_blocks(fn, block, lds);
    const int cus = device_cus();
    for (uint64_t c = 0; c < L.n_chunks; ++c) {
        const uint64_t a = c * kChunk;
        const uint64_t n = std::min<uint64_t>(kChunk, run->n_packets - a);
        P.pid0 = run->first_packet_id + a;
        P.npk = n;
        P.counter = reinterpret_cast<unsigned long long *>(base + L.counters) + c;
        const uint64_t want = (n + block - 1) / block;
        const unsigned grid = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(want, (uint64_t)cus * occ));
        hipEvent_t e0 = nullptr, e1 = nullptr;
        Profile &pr = profile_state();
        bool timed = false;
        {
            std::lock_guard<std::mutex> g(pr.mu);
            timed = pr.on;
        }
        if (timed) {
            if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return MC_ERR_DEVICE;
            if (hipEventRecord(e0, s) != hipSuccess) return MC_ERR_DEVICE;
        }
        hipLaunchKernelGGL(fn, dim3(grid), dim3(block), lds, s, P);
        if (timed) {
            if (hipEventRecord(e1, s) != hipSuccess) return MC_ERR_DEVICE;
            std::lock_guard<std::mutex> g(pr.mu);
            pr.pending.emplace_back(e0, e1);
        }
        if (!L.lds_mode) {
            const size_t tn = (size_t)npix * K;
            hipLaunchKernelGGL(k_fold, dim3((unsigned)std::min<size_t>((tn + 255) / 256, 8192)), dim3(256), 0, s, tn,
                               P.t32, P.t64);
        }
        if (hipGetLastError() != hipSuccess) return MC_ERR_DEVICE;
    }
    const double scale = P.total / ((double)run->n_packets);
    hipLaunchKernelGGL(k_normalise, dim3((npix + 255) / 256), dim3(256), 0, s, npix, N, adjoint,
                       scale / (double)m->dx, P.t64, coeffs);
    if (ledger)
        hipLaunchKernelGGL(k_ledger_out, dim3(1), dim3(1), 0, s, P.led, P.ledc, scale, ledger);
    return hipGetLastError() == hipSuccess ? MC_OK : MC_ERR_DEVICE;
}

}  // namespace

extern "C" {

size_t mc_workspace_bytes(const mc_medium *medium, const mc_source *src, int n_src, const mc_run *run) {
    if (validate(medium, src, n_src, run) != MC_OK) return 0;
    return layout(medium, src, run).total;
}

mc_status mc_forward(const mc_medium *medium, const mc_source *src, int n_src, const mc_run *run, double *coeffs_d,
                     mc_ledger *ledger_d, void *workspace_d, size_t workspace_bytes, void *stream) {
    return run_mc(medium, src, n_src, run, coeffs_d, ledger_d, workspace_d, workspace_bytes, stream, 0);
}

mc_status mc_adjoint(const mc_medium *medium, const mc_source *src, int n_src, const mc_run *run, double *coeffs_d,
                     mc_ledger *ledger_d, void *workspace_d, size_t workspace_bytes, void *stream) {
    return run_mc(medium, src, n_src, run, coeffs_d, ledger_d, workspace_d, workspace_bytes, stream, 1);
}

mc_status mc_residual(const mc_medium *m, const double *coeffs_d, const double *hmeas_d, double *q_star_d,
                      double *eps_d, void *stream) {
    if (!m || m->nx <= 0 || m->nz <= 0 || !(m->dx > 0.f) || !m->mua_d || !coeffs_d || !hmeas_d || !eps_d)
        return MC_ERR_INVALID_ARG;
    const int npix = m->nx * m->nz;
    hipLaunchKernelGGL(k_residual, dim3(1), dim3(1024), 0, reinterpret_cast<hipStream_t>(stream), npix,
                       (double)m->dx * m->dx, m->mua_d, coeffs_d, hmeas_d, q_star_d, eps_d);
    return hipGetLastError() == hipSuccess ? MC_OK : MC_ERR_DEVICE;
}

mc_status mc_gradient(const mc_medium *m, int n_harm, const double *fwd_d, const double *adj_d, const double *hmeas_d,
                      double *dmua_d, double *dmus_d, void *stream) {
    if (!m || m->nx <= 0 || m->nz <= 0 || !(m->dx > 0.f) || !m->mua_d || !m->g_d || !fwd_d || !adj_d || !hmeas_d)
        return MC_ERR_INVALID_ARG;
    if (n_harm < 0 || n_harm > MC_NHARM_MAX) return MC_ERR_INVALID_ARG;
    const int npix = m->nx * m->nz;
    hipLaunchKernelGGL(k_gradient, dim3((npix + 255) / 256), dim3(256), 0, reinterpret_cast<hipStream_t>(stream), npix,
                       n_harm, (double)m->dx * m->dx, m->mua_d, m->g_d, fwd_d, adj_d, hmeas_d, dmua_d, dmus_d);
    return hipGetLastError() == hipSuccess ? MC_OK : MC_ERR_DEVICE;
}

mc_status mc_detect(const mc_medium *m, int n_harm, const double *coeffs_d, const double *det_d, double *out_d,
                    void *stream) {
    if (!m || m->nx <= 0 || m->nz <= 0 || !(m->dx > 0.f) || !coeffs_d || !det_d || !out_d) return MC_ERR_INVALID_ARG;
    if (n_harm < 0 || n_harm > MC_NHARM_MAX) return MC_ERR_INVALID_ARG;
    hipLaunchKernelGGL(k_detect, dim3(1), dim3(1024), 0, reinterpret_cast<hipStream_t>(stream), m->nx * m->nz, n_harm,
                       (double)m->dx * m->dx, coeffs_d, det_d, out_d);
    return hipGetLastError() == hipSuccess ? MC_OK : MC_ERR_DEVICE;
}

mc_status mc_trace(const mc_medium *m, const mc_source *src, int n_src, const mc_run *run, int adjoint,
                   const uint64_t *pids_h, int n_pids, mc_event *events_h, size_t cap, size_t *n_events_h) {
    mc_status st = validate(m, src, n_src, run);
    if (st != MC_OK) return st;
    if (!pids_h || n_pids < 0 || (!events_h && cap) || !n_events_h) return MC_ERR_INVALID_ARG;
    const int npix = m->nx * m->nz;
    const Layout L = layout(m, src, run);
    void *ws = nullptr, *d_pids = nullptr, *d_ev = nullptr, *d_n = nullptr;
    auto cleanup = [&]() {
        if (ws) (void)hipFree(ws);
        if (d_pids) (void)hipFree(d_pids);
        if (d_ev) (void)hipFree(d_ev);
        if (d_n) (void)hipFree(d_n);
    };
    if (hipMalloc(&ws, L.total) != hipSuccess || hipMalloc(&d_pids, sizeof(uint64_t) * std::max(1, n_pids)) != hipSuccess ||
        hipMalloc(&d_ev, sizeof(mc_event) * std::max<size_t>(1, cap)) != hipSuccess ||
        hipMalloc(&d_n, sizeof(unsigned long long)) != hipSuccess) {
        cleanup();
        return MC_ERR_DEVICE;
    }
    char *base = static_cast<char *>(ws);
    Params P;
    double map_abs_sum = 0;
    hipLaunchKernelGGL(k_setup_medium, dim3((npix + 255) / 256), dim3(256), 0, 0, npix, m->dx, m->mua_d, m->mus_d,
                       reinterpret_cast<float4 *>(base + L.med));
    if (src[0].kind == MC_SRC_MAP) {
        double *cdf = reinterpret_cast<double *>(base + L.cdf);
        hipLaunchKernelGGL(k_map_cdf, dim3(1), dim3(1024), 0, 0, npix, src[0].map_d, cdf);
        if (hipMemcpy(&map_abs_sum, cdf + npix - 1, sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) {
            cleanup();
            return MC_ERR_DEVICE;
        }
    }
    fill_params(P, m, src, n_src, run, adjoint, map_abs_sum);
    P.med = reinterpret_cast<const float4 *>(base + L.med);
    P.cdf = reinterpret_cast<const double *>(base + L.cdf);
    if (hipMemcpy(d_pids, pids_h, sizeof(uint64_t) * n_pids, hipMemcpyHostToDevice) != hipSuccess) {
        cleanup();
        return MC_ERR_DEVICE;
    }
    hipLaunchKernelGGL(kernels().tr[run->n_harm], dim3(1), dim3(64), 0, 0, P, (const uint64_t *)d_pids, n_pids,
                       (mc_event *)d_ev, cap, (unsigned long long *)d_n);
    unsigned long long n = 0;
    if (hipGetLastError() != hipSuccess || hipMemcpy(&n, d_n, sizeof(n), hipMemcpyDeviceToHost) != hipSuccess) {
        cleanup();
        return MC_ERR_DEVICE;
    }
    if (cap && hipMemcpy(events_h, d_ev, sizeof(mc_event) * std::min<size_t>(cap, n), hipMemcpyDeviceToHost) != hipSuccess) {
        cleanup();
        return MC_ERR_DEVICE;
    }
    *n_events_h = n;
    cleanup();
    return MC_OK;
}

mc_status mc_philox_fill(uint64_t seed, uint32_t tag, uint64_t pid0, uint64_t n, uint32_t j, uint32_t *out_d,
                         void *stream) {
    if (!out_d || n == 0 || n > (1ull << 32)) return MC_ERR_INVALID_ARG;
    hipLaunchKernelGGL(k_philox_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                       reinterpret_cast<hipStream_t>(stream), seed, tag, pid0, n, j, out_d);
    return hipGetLastError() == hipSuccess ? MC_OK : MC_ERR_DEVICE;
}

const char *mc_status_string(mc_status s) {
    switch (s) {
        case MC_OK: return "ok";
        case MC_ERR_INVALID_ARG: return "invalid argument";
        case MC_ERR_UNSUPPORTED: return "unsupported";
        case MC_ERR_DEVICE: return "device error";
        case MC_ERR_WORKSPACE: return "workspace too small or misaligned";
    }
    return "unknown status";
}

void mc_profile_enable(int on) {
    Profile &pr = profile_state();
    std::lock_guard<std::mutex> g(pr.mu);
    pr.on = on != 0;
}

mc_status mc_profile_read(double *transport_ms, uint64_t *launches, int reset) {
    Profile &pr = profile_state();
    std::lock_guard<std::mutex> g(pr.mu);
    mc_status st = MC_OK;
    for (auto &ev : pr.pending) {
        float ms = 0.f;
        if (hipEventSynchronize(ev.second) != hipSuccess || hipEventElapsedTime(&ms, ev.first, ev.second) != hipSuccess)
            st = MC_ERR_DEVICE;
        pr.ms += ms;
        pr.launches += 1;
        (void)hipEventDestroy(ev.first);
        (void)hipEventDestroy(ev.second);
    }
    pr.pending.clear();
    if (transport_ms) *transport_ms = pr.ms;
    if (launches) *launches = pr.launches;
    if (reset) {
        pr.ms = 0;
        pr.launches = 0;
    }
    return st;
}

const char *mc_build_info(void) {
    return "librmc gfx950: FP32 transport, LDS tally <= 64 KiB else FP32 HBM tally folded to FP64 per 2^22 packets";
}

}  // extern "C"
