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
//  * one lane per packet; every lane of a wave steps and scatters with the
//    same instructions (results committed by select), dead lanes refill
//    between steps;
//  * FP32 transport in pixel-local coordinates (pixel index + offset in
//    [0,1]), so precision does not degrade with the grid size;
//  * the per-visit harmonic sums (K FP32 registers, scaled by a power of two
//    fixed per run) are flushed once per pixel visit as rounded 64-bit
//    integers into LDS tallies (fixed_add):
//      - whole-grid mode (small tallies): the whole grid's tally sits in each
//        workgroup's LDS, added to the FP64 map when the workgroup ends;
//      - tiled mode: square tiles of the grid, packets migrate between tiles
//        in generations (launch and count, sort of record indices by tile,
//        one workgroup job per tile batch, tile tally added to the FP64 map
//        per job); a finisher kernel moves the last packets to their end
//        without migration;
//  * every value a kernel needs that depends on device data (the sum and
//    maximum of a source map, the fixed-point scale, the normalisation) is
//    computed on the device, and the tiled generations are steered by a
//    device control block, so no entry point waits for the device;
//  * each visit adds the same integer multiple of the run's resolution
//    whichever kernel, tile or generation completes it, so the maps depend
//    on the schedule only through FP64 additions, which are exact while a
//    pixel's total is below 2^53 resolution steps;
//  * no MFMA: the transport is not a dense contraction.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <mutex>
#include <new>
#include <vector>

#include "mcrad.h"

namespace {

constexpr int kMaxSrc = 8;
constexpr int kMaxProf = 2 * (2 * MC_NHARM_MAX + 1);  // profile coefficients over all sources
// whole-grid mode: 12 waves share one LDS tally (8 for high orders, whose
// harmonic vectors need more registers)
constexpr int grid_block(int nh) { return nh <= 16 ? 1024 : 512; }
// tiled mode: one workgroup per CU, holding the largest tile tally that
// fits its LDS; 16 waves (4 per SIMD) for orders up to 16, 8 for higher
// orders (whose visit accumulators need twice the registers)
constexpr int tile_block(int nh) { return nh <= 16 ? 1024 : 512; }
constexpr uint64_t kChunk = 1ull << 22;                // whole-grid mode: packets per launch
constexpr size_t kLdsGridMax = 144 * 1024;             // whole-grid mode: tally bytes in LDS
constexpr size_t kLdsTileMax = 150 * 1024;             // tiled mode: tile tally + medium bytes (1 WG/CU)
constexpr uint32_t kInvalidTile = 0xFFFFFFFFu;
constexpr uint32_t kSlice = 256;                       // queue slots a wave reserves at a time (default)
constexpr float kPi = 3.14159265358979323846f;
constexpr uint32_t kMaxInteractions = 1u << 24;         // hard cap per packet (guards invalid media)
// the LDS tallies hold 64-bit fixed-point sums, value * 2^(32 - e) where 2^e
// bounds the magnitude of any packet weight of the run (fixed_add)
constexpr int kFixBits = 32;
constexpr double kFlushTrackMax = 65536.0;             // see mc_tuning::flush_track

enum : int { EV_LAUNCH = 0, EV_CROSS = 1, EV_SCATTER = 2, EV_ESCAPE = 3, EV_KILL = 4, EV_NONE = 5 };

struct SrcDev {
    int kind, lambertian, prof_off, n_prof;
    double x0, z0, x1, z1;      // mm
    float dir_x, dir_z;
    double cum;                 // inclusive prefix of the sampling measure
};

// One problem (a forward or adjoint run) in device memory.  The host fills
// what it knows and hands the struct to k_prob_setup by value; that kernel
// adds what depends on device data (the sum and maximum of a MAP source, the
// fixed-point scale, the normalisation) and stores it.  Every transport
// kernel reads its packets' problem from here.
struct ProbDev {
    int nx, nz, npix, ntx, tile_base, ntiles;   // grid; tiles across; first global tile; tiles
    int nsrc, adjoint;
    float dx;
    uint32_t tag, flags;
    uint64_t seed;
    uint64_t pid0, npk;           // packet range of the run
    uint64_t todo;                // packets to launch (0 for a source of no power)
    float wth, rm, inv_rm;
    float flush_at;               // scaled |a0 accumulator| at which a visit is flushed in parts
    float fx;                     // fixed-point scale of the LDS tallies (a power of two)
    double fx_inv;                // its inverse
    double wbound;                // host part of the bound on |packet weight|
    double flush_track;
    double total;                 // source measure (MAP: 2 pi sum |q| A, set on the device)
    double inv_qbar;              // MAP: npix / sum |q| (equal-count launch)
    double scale;                 // normalisation total / packets (0: no power; NaN: unusable map)
    const float4 *med;            // {mua dx, mus dx, 1/(mus dx), g}
    const double *map;            // MAP source values (sign)
    const double *cdf;            // MAP: inclusive prefix of |map|, then max |map|
    double *t64;                  // FP64 tally [npix][K]
    double *led;                  // 5 doubles
    unsigned long long *ledc;     // [0..3] counts, [4] jobs whose tile tally may have left the fixed-point range
    SrcDev src[kMaxSrc];
    float prof[kMaxProf];
};

// The values a step and a scatter read, uniform over a workgroup's job.
struct Hot {
    int nx, nz;
    uint32_t tag, flags;
    uint64_t seed;
    float wth, rm, inv_rm;
};

__device__ __forceinline__ Hot hot_of(const ProbDev &S) {
    return Hot{S.nx, S.nz, S.tag, S.flags, S.seed, S.wth, S.rm, S.inv_rm};
}

// The device pointers held in device memory (ProbDev's) are generic: an
// access through one compiles to a flat_* instruction, which counts on the
// LDS counter as well as the vector-memory one, so a wait for an LDS read
// also waits for every such load or atomic in flight.  They all point into
// global memory; these two accesses say so (global_* instructions).
typedef float v4f_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float4 load_medium(const float4 *med, int i) {
    const v4f_t v = ((const __attribute__((address_space(1))) v4f_t *)med)[i];
    return make_float4(v.x, v.y, v.z, v.w);
}

// An FP64 add to a tally in global memory whose old value nobody reads.
__device__ __forceinline__ void tally_add(double *p, double v) {
    __hip_atomic_fetch_add((__attribute__((address_space(1))) double *)p, v, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

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
        // one 32x32->64 product each (v_mad_u64_u32) rather than separate low and
        // high multiplies; each three-way XOR is one v_bitop3_b32 (truth table 0x96)
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
        c = make_uint4(__builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c.y, k0, 0x96), (uint32_t)p1,
                       __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c.w, k1, 0x96), (uint32_t)p0);
    }
    return c;
}

template <class PP>
__device__ __forceinline__ uint4 rng_block(const PP &P, uint64_t pid, uint32_t j) {
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

// A packet between two stays in tiles (64 bytes, four 16-byte words).
struct alignas(16) PacketRec {
    float fx, fz, sx, sz;
    float w, w0abs, tau, uh;
    float ur;
    uint32_t k;
    int32_t ix, iz;
    uint64_t pid;
    uint32_t tile;
    uint32_t prob;     // problem of the batch
};
static_assert(sizeof(PacketRec) == 64, "packet record layout");

// State of a lane without a packet.  Free lanes run the same instructions as
// busy ones (their results are discarded), so the state must be harmless: a
// pixel of the grid (or tile) and a finite direction, whose deposits are 0.
__device__ __forceinline__ void idle_packet(Packet &p, int ix, int iz) {
    p.ix = ix;
    p.iz = iz;
    p.fx = p.fz = 0.5f;
    p.sx = 0.f;
    p.sz = 1.f;
    p.isx = INFINITY;
    p.isz = 1.f;
    p.w = p.w0abs = p.tau = p.uh = p.ur = 0.f;
    p.k = 0;
    p.pid = 0;
    p.alive = false;
}

struct LedgerRegs {
    double launched = 0, absorbed = 0, escaped = 0, gain = 0, loss = 0;
    uint32_t packets = 0, segments = 0, visits = 0, scatters = 0;
};

// The tile transport's ledger.  Escape and roulette come about once per
// packet, so a lane meets only a few of them between two flushes (one launch
// or problem): FP32 sums carry them, which keeps the transport loop's
// loop-carried FP64 state to the per-segment absorbed weight.
struct LedgerTile {
    double absorbed = 0;
    float escaped = 0.f, gain = 0.f, loss = 0.f;
    uint32_t segments = 0, visits = 0, scatters = 0;
};

// h = [1, cos t .. cos Nt, sin t .. sin Nt] for the direction (sin t, cos t)
// by the three-term recurrences cos (n+1)t = 2 cos t cos nt - cos (n-1)t and
// sin (n+1)t = 2 cos t sin nt - sin (n-1)t: one FMA per value.  A rounding
// error made at order k reaches order n multiplied by a Chebyshev polynomial
// of the second kind, bounded by n - k + 1, so the error stays below
// n^2/2 ulp (8e-6 at n = 16).
template <int NH>
__device__ __forceinline__ void harmonics(float sx, float sz, float *h) {
    h[0] = 1.f;
    if constexpr (NH >= 1) {
        h[1] = sz;
        h[NH + 1] = sx;
    }
    const float c2 = 2.f * sz;
    if constexpr (NH >= 2) {
        h[2] = fmaf(c2, sz, -1.f);
        h[NH + 2] = c2 * sx;
    }
#pragma unroll
    for (int n = 3; n <= NH; ++n) {
        h[n] = fmaf(c2, h[n - 1], -h[n - 2]);
        h[NH + n] = fmaf(c2, h[NH + n - 1], -h[NH + n - 2]);
    }
}

// Angular profile p(t) = c0/2pi + (1/pi) sum (c_n cos nt + s_n sin nt).
__device__ __forceinline__ float profile(const ProbDev &S, const SrcDev &s, float sx, float sz) {
    const float *c = S.prof + s.prof_off;
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
    // hardware reciprocal (1 ulp): enough for distances to pixel faces
    p.isx = sx != 0.f ? __builtin_amdgcn_rcpf(sx) : INFINITY;
    p.isz = sz != 0.f ? __builtin_amdgcn_rcpf(sz) : INFINITY;
}

// Draw block k: free path (optical depth) and the uniforms used at its end.
// -ln u from the hardware log2 (u >= 2^-24 is never denormal; 1.2e-7
// relative error measured on the generator's grid of u).
template <class PP>
__device__ __forceinline__ void new_leg(const PP &P, Packet &p) {
    const uint4 r = rng_block(P, p.pid, p.k);
    p.tau = __builtin_amdgcn_logf(u01(r.x)) * -0.693147180559945309f;
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
__device__ bool launch_state(const ProbDev &P, uint64_t pid, Packet &p, LedgerRegs &L) {
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
    } else {   // MAP source, uniform position inside the chosen pixel (Sec. 6)
        int lo;
        float wq;
        if (P.flags & MC_FLAG_EQUAL_COUNT) {   // every pixel equally likely, weight q_i / mean |q|
            lo = min((int)((double)u0 * P.npix), P.npix - 1);
            wq = (float)(P.map[lo] * P.inv_qbar);
        } else {   // pixel with probability |q_i| / sum |q|, weight sign(q_i)
            const double t = (double)u0 * P.cdf[P.npix - 1];
            int hi = P.npix - 1;
            lo = 0;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (P.cdf[mid] > t) hi = mid; else lo = mid + 1;
            }
            wq = P.map[lo] < 0.0 ? -1.f : 1.f;
        }
        const int ixs = lo % P.nx, izs = lo / P.nx;
        ax = ixs + (double)u1;
        az = izs + (double)u2;
        sincospif(2.f * u3 - 1.f, &sx, &sz);
        w0 = wq * 2.f * kPi * profile(P, S, sx, sz);
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
    // a packet of zero weight (equal-count launch where q = 0) carries nothing
    // and leaves at once, like one launched outside the grid
    if (p.ix < 0 || p.ix >= P.nx || p.iz < 0 || p.iz >= P.nz || ((P.flags & MC_FLAG_EQUAL_COUNT) && w0 == 0.f)) {
        L.escaped += w0;
        p.alive = false;
        return false;
    }
    p.alive = true;
    new_leg(P, p);
    return true;
}

template <int NH>
__device__ bool launch(const ProbDev &P, uint64_t pid, Packet &p, float *h, LedgerRegs &L) {
    if (!launch_state(P, pid, p, L)) return false;
    harmonics<NH>(p.sx, p.sz, h);
    return true;
}

// f(x) = (1 - e^-x)/x for x >= 0, with f(0) = 1: the fraction of the weight
// absorbed per unit optical depth on a segment.  Below 1/4 its Taylor series
// sum_k (-x)^k/(k+1)! in Horner form, truncated after x^7 (remainder below
// x^8/9! ~ 4e-11 there); above, the library expm1.
__device__ __forceinline__ float absorbed_per_depth(float x) {
    if (x < 0.25f) {
        float t = -1.f / 40320.f;
        t = fmaf(t, x, 1.f / 5040.f);
        t = fmaf(t, x, -1.f / 720.f);
        t = fmaf(t, x, 1.f / 120.f);
        t = fmaf(t, x, -1.f / 24.f);
        t = fmaf(t, x, 1.f / 6.f);
        t = fmaf(t, x, -0.5f);
        return fmaf(t, x, 1.f);
    }
    return -expm1f(-x) * __builtin_amdgcn_rcpf(x);
}

// One segment: run to the next pixel face or to the end of the free path,
// depositing the track length weighted by the decaying weight (Sec. 3).
// Returns EV_CROSS, EV_ESCAPE or EV_SCATTER; T (pixel units) and the pixel
// of the segment are returned through the references.
// Written with selects only: every lane of a wave runs the same instructions.
template <class PP>
__device__ __forceinline__ int step(const PP &P, Packet &p, const float4 m, float &T, float &dw) {
    const bool px = p.sx > 0.f, pz = p.sz > 0.f;
    const float dfx = p.sx != 0.f ? (px ? 1.f - p.fx : p.fx) * fabsf(p.isx) : INFINITY;
    const float dfz = p.sz != 0.f ? (pz ? 1.f - p.fz : p.fz) * fabsf(p.isz) : INFINITY;
    const float d = fminf(dfx, dfz);
    const float od = m.y * d;
    const bool scat = od > p.tau;
    const float l = scat ? p.tau * m.z : d;
    const float x = m.x * l;
    const float wf = p.w * absorbed_per_depth(x);
    dw = wf * x;   // weight absorbed on the segment
    T = wf * l;    // track length weighted by the weight (= dw / mua)
    p.w -= dw;
    const float nfx = fminf(fmaxf(p.fx + l * p.sx, 0.f), 1.f);
    const float nfz = fminf(fmaxf(p.fz + l * p.sz, 0.f), 1.f);
    const bool cx = !scat && dfx <= dfz, cz = !scat && dfz <= dfx;   // faces crossed (both at a corner)
    p.tau = scat ? p.tau : p.tau - od;
    p.ix += cx ? (px ? 1 : -1) : 0;
    p.iz += cz ? (pz ? 1 : -1) : 0;
    p.fx = cx ? (px ? 0.f : 1.f) : nfx;
    p.fz = cz ? (pz ? 0.f : 1.f) : nfz;
    const bool out = (unsigned)p.ix >= (unsigned)P.nx || (unsigned)p.iz >= (unsigned)P.nz;
    return scat ? EV_SCATTER : (out ? EV_ESCAPE : EV_CROSS);
}

// sin(pi x) for |x| <= 1/2: the Taylor series of sin t at t = pi x, with pi
// folded into the coefficients and truncated after t^13 (remainder below
// (pi/2)^15/15! ~ 7e-10).  Both scatter factors use it: the cosine as
// sin(pi min(u, 1 - u)), whose argument is exact and keeps full relative
// accuracy where the cosine goes to zero.
constexpr double kPiD = 3.14159265358979323846;
__device__ __forceinline__ float sinpi_half(float x) {
    constexpr double p2 = kPiD * kPiD;
    constexpr float c1 = (float)kPiD, c3 = (float)(-kPiD * p2 / 6.0), c5 = (float)(kPiD * p2 * p2 / 120.0),
                    c7 = (float)(-kPiD * p2 * p2 * p2 / 5040.0), c9 = (float)(kPiD * p2 * p2 * p2 * p2 / 362880.0),
                    c11 = (float)(-kPiD * p2 * p2 * p2 * p2 * p2 / 39916800.0),
                    c13 = (float)(kPiD * p2 * p2 * p2 * p2 * p2 * p2 / 6227020800.0);
    const float x2 = x * x;
    float q = fmaf(c13, x2, c11);
    q = fmaf(q, x2, c9);
    q = fmaf(q, x2, c7);
    q = fmaf(q, x2, c5);
    q = fmaf(q, x2, c3);
    q = fmaf(q, x2, c1);
    return x * q;
}

// Scatter site, in two parts.  First the termination test on |W| (Sec. 3,
// Sec. 6): Russian roulette below the threshold, or the hard cap on
// interactions; returns true for the lanes whose packet is terminated.
template <class PP, class LG>
__device__ __forceinline__ bool scatter_roulette(const PP &P, Packet &p, const bool at, LG &L) {
    bool kill = false;
    const bool low = at && (p.k >= kMaxInteractions || fabsf(p.w) < P.wth * p.w0abs);
    if (__ballot(low)) {   // rare
        if (low) {
            if (p.k >= kMaxInteractions || (P.flags & MC_FLAG_LITERAL_TRUNCATION) || !(p.ur < P.inv_rm)) {
                kill = true;
                L.loss += p.w;
            } else {
                L.gain += (P.rm - 1.f) * p.w;
                p.w *= P.rm;
            }
        }
    }
    return kill;
}

// Then the 2D HG deflection (eq. scattering_angle) written without atan/tan:
// with a = (1+g) cos(pi(u-1/2)), b = (1-g) sin(pi(u-1/2)), tan(dt/2) = b/a,
// so cos dt = (a^2-b^2)/(a^2+b^2), sin dt = 2ab/(a^2+b^2); and the next
// block of random numbers.  `go` marks the lanes that scatter and survived;
// every lane runs the same instructions and only those lanes commit
// (selects, so the Philox rounds and the deflection form one basic block the
// scheduler can interleave).  `kill` (from the roulette) ends the packet.
template <class PP, class LG>
__device__ __forceinline__ void scatter_deflect(const PP &P, Packet &p, const bool go, const bool kill, const float g,
                                                LG &L) {
    const float y = p.uh - 0.5f;                 // exact
    const float sp = sinpi_half(y);              // sin(pi (u - 1/2))
    const float cp = sinpi_half(0.5f - fabsf(y));  // cos(pi (u - 1/2)); the argument min(u, 1 - u) is exact
    const float a = (1.f + g) * cp, b = (1.f - g) * sp;
    const float inv = __builtin_amdgcn_rcpf(a * a + b * b);
    const float cd = (a * a - b * b) * inv, sd = 2.f * a * b * inv;
    float nx_ = p.sx * cd + p.sz * sd;
    float nz_ = p.sz * cd - p.sx * sd;
    const float rn = __builtin_amdgcn_rsqf(nx_ * nx_ + nz_ * nz_);   // argument ~1
    nx_ *= rn;
    nz_ *= rn;
    const uint4 r = rng_block(P, p.pid, p.k + 1);
    const float tau = __builtin_amdgcn_logf(u01(r.x)) * -0.693147180559945309f;   // see new_leg
    const float isx = nx_ != 0.f ? __builtin_amdgcn_rcpf(nx_) : INFINITY;
    const float isz = nz_ != 0.f ? __builtin_amdgcn_rcpf(nz_) : INFINITY;
    p.sx = go ? nx_ : p.sx;
    p.sz = go ? nz_ : p.sz;
    p.isx = go ? isx : p.isx;
    p.isz = go ? isz : p.isz;
    p.k = go ? p.k + 1 : p.k;
    p.tau = go ? tau : p.tau;
    p.uh = go ? u01(r.y) : p.uh;
    p.ur = go ? u01(r.z) : p.ur;
    p.alive = p.alive && !kill;
    L.scatters += go ? 1u : 0u;
}

// Both parts in order; `at` marks the lanes that scatter.  Returns true for
// the lanes whose packet was terminated.
template <class PP, class LG>
__device__ __forceinline__ bool scatter_masked(const PP &P, Packet &p, const bool at, const float g, LG &L) {
    const bool kill = scatter_roulette(P, p, at, L);
    scatter_deflect(P, p, at && !kill, kill, g, L);
    return kill;
}

template <class PP>
__device__ __forceinline__ bool scatter_dir(const PP &P, Packet &p, const float g, LedgerRegs &L) {
    return !scatter_masked(P, p, true, g, L);
}

template <int NH, class PP>
__device__ __forceinline__ bool scatter(const PP &P, Packet &p, const float g, float *h, LedgerRegs &L) {
    if (!scatter_dir(P, p, g, L)) return false;
    harmonics<NH>(p.sx, p.sz, h);
    return true;
}

// acc = keep * acc + T [1, cos t .. cos Nt, sin t .. sin Nt].  The products
// y_n = T cos nt and T sin nt come straight from the recurrences of
// harmonics() started at y_0 = T (they are linear, so scaling by T commutes
// with them), and one FMA per channel both adds y_n and applies the reset
// after a flush (keep = 0; keep = 1 adds exactly).  Every kernel deposits
// through this function, so a visit's sums are the same bits whichever kernel
// completes it.  The recurrences run for nearly every segment anyway (some
// lane of the wave scatters), so no harmonic vector is stored.
template <int NH>
__device__ __forceinline__ void deposit_harmonics(float T, float sx, float sz, float keep, float *acc) {
    acc[0] = fmaf(acc[0], keep, T);
    if constexpr (NH >= 1) {
        const float c2 = 2.f * sz;
        float cm = T, sm = 0.f, cn = T * sz, sn = T * sx;
        acc[1] = fmaf(acc[1], keep, cn);
        acc[NH + 1] = fmaf(acc[NH + 1], keep, sn);
#pragma unroll
        for (int n = 2; n <= NH; ++n) {
            const float c = fmaf(c2, cn, -cm);
            const float s_ = n == 2 ? c2 * sn : fmaf(c2, sn, -sm);
            cm = cn;
            sm = sn;
            cn = c;
            sn = s_;
            acc[n] = fmaf(acc[n], keep, c);
            acc[NH + n] = fmaf(acc[NH + n], keep, s_);
        }
    }
}

// Ledger of a whole workgroup (every thread calls it): wave sums, then one
// set of device atomics per workgroup.
__device__ __forceinline__ void ledger_flush_block(double *led, unsigned long long *ledc, LedgerRegs &L) {
    __shared__ double s_v[16][5];
    __shared__ unsigned long long s_c[16][4];
    double v[5] = {L.launched, L.absorbed, L.escaped, L.gain, L.loss};
    unsigned long long c[4] = {L.packets, L.segments, L.visits, L.scatters};
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
        for (int i = 0; i < 5; ++i) v[i] += __shfl_xor(v[i], off);
#pragma unroll
        for (int i = 0; i < 4; ++i) c[i] += __shfl_xor(c[i], off);
    }
    const int wave = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    if (__lane_id() == 0) {
        for (int i = 0; i < 5; ++i) s_v[wave][i] = v[i];
        for (int i = 0; i < 4; ++i) s_c[wave][i] = c[i];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < nw; ++w) {
            for (int i = 0; i < 5; ++i) v[i] += s_v[w][i];
            for (int i = 0; i < 4; ++i) c[i] += s_c[w][i];
        }
        for (int i = 0; i < 5; ++i)
            if (v[i] != 0.0) atomicAdd(led + i, v[i]);
        for (int i = 0; i < 4; ++i)
            if (c[i]) atomicAdd(ledc + i, c[i]);
    }
    __syncthreads();   // the staging arrays may be reused by a next call
}

__device__ __forceinline__ void ledger_flush_tile(double *led, unsigned long long *ledc, const LedgerTile &L) {
    LedgerRegs R;
    R.absorbed = L.absorbed;
    R.escaped = L.escaped;
    R.gain = L.gain;
    R.loss = L.loss;
    R.segments = L.segments;
    R.visits = L.visits;
    R.scatters = L.scatters;
    ledger_flush_block(led, ledc, R);
}

// Add v (already scaled by the run's fixed-point factor), rounded to the
// nearest integer, to a 64-bit fixed-point LDS slot.  For |v| < 2^51 the FP64
// sum v + 1.5 2^52 lies in [2^52, 2^53), where the spacing of doubles is 1, so
// its bit pattern minus that of 1.5 2^52 is the rounded integer in two's
// complement.  Integer adds are associative, so the slot holds the same sum in
// any order of arrival, and LDS 64-bit integer atomics outrun FP64 ones on
// this device.
__device__ __forceinline__ void fixed_add(unsigned long long *slot, float v) {
    const double d = (double)v + 0x1.8p52;
    atomicAdd(slot, (unsigned long long)__double_as_longlong(d) - 0x4338000000000000ull);
}

// The same without the subtraction: a slot that received k such adds holds
// k * bits(1.5 2^52) more than the integer sum (mod 2^64), removed once when
// the slot is read (fixed_value) from a count of the adds kept per pixel.
constexpr unsigned long long kFixMagicBits = 0x4338000000000000ull;
__device__ __forceinline__ void fixed_add_raw(unsigned long long *slot, float v) {
    atomicAdd(slot, (unsigned long long)__double_as_longlong((double)v + 0x1.8p52));
}
__device__ __forceinline__ long long fixed_value(unsigned long long raw, uint32_t adds) {
    return (long long)(raw - (unsigned long long)adds * kFixMagicBits);
}

// ------------------------------------------------------------------ whole-grid transport
// Small grids: the whole tally [npix][K] lives in LDS for the workgroup's life
// as 64-bit fixed-point sums (fixed_add), added to the HBM FP64 tally with
// coalesced atomics at the end.  Persistent waves refill dead lanes from a
// global packet counter with one wave-aggregated atomic.
struct GridArgs {
    const ProbDev *pd;
    uint64_t pid0, npk;           // packet range of this launch
    unsigned long long *counter;
};

template <int NH>
__global__ void __launch_bounds__(grid_block(NH)) k_transport_grid(GridArgs A) {
    constexpr int K = 2 * NH + 1;
    extern __shared__ unsigned long long gfx[];   // [npix][K] fixed-point sums (fixed_add)
    __shared__ float s_mag;
    const ProbDev &S = *A.pd;
    if (S.todo == 0) return;   // a source of no power: nothing to transport
    const Hot H = hot_of(S);
    const int npix = S.npix;
    const float4 *med = S.med;
    const int lane = __lane_id();
    for (int i = threadIdx.x; i < npix * K; i += blockDim.x) gfx[i] = 0ull;
    if (threadIdx.x == 0) s_mag = 0.f;
    __syncthreads();
    const float fx = S.fx, flush_at = S.flush_at;

    Packet p;
    idle_packet(p, 0, 0);
    float mag = 0.f;   // sum of the |a0| this lane flushed: bounds every slot's magnitude
    float acc[K], keep = 1.f;   // keep = 0 after a flush: the next deposit restarts the sums
#pragma unroll
    for (int j = 0; j < K; ++j) acc[j] = 0.f;
    LedgerRegs L;
    bool more = true;
    const unsigned long long lt_mask = (1ull << lane) - 1ull;

    for (;;) {
        if (more) {
            const unsigned long long dead = __ballot(!p.alive);
            if (dead) {
                const int ndead = __popcll(dead);
                const int leader = __ffsll((long long)dead) - 1;
                unsigned long long base = 0;
                if (lane == leader) base = atomicAdd(A.counter, (unsigned long long)ndead);
                base = __shfl(base, leader);
                if (base + ndead >= A.npk) more = false;
                if (!p.alive) {
                    const unsigned long long my = base + __popcll(dead & lt_mask);
                    if (my < A.npk) launch_state(S, A.pid0 + my, p, L);
                }
            }
        }
        if (!__ballot(p.alive)) {
            if (!more) break;
        }
        // every lane steps and scatters (no branch); a free lane's results are discarded
        const bool live = p.alive;
        const int pix = live ? p.iz * H.nx + p.ix : 0;
        float T = 0.f, dw = 0.f;
        const float4 mm = load_medium(med, pix);
        int ev = step(H, p, mm, T, dw);
        ev = live ? ev : EV_NONE;
        T = live ? T : 0.f;
        dw = live ? dw : 0.f;
        L.absorbed += (double)dw;
        L.segments += live ? 1u : 0u;
        deposit_harmonics<NH>(T * fx, p.sx, p.sz, keep, acc);   // direction of the segment, before any scatter
        const bool at = ev == EV_SCATTER;
        const bool killed = scatter_masked(H, p, at, mm.w, L);
        const bool vend = killed || (ev != EV_NONE && !at);   // the visit ends
        const bool flush = vend || fabsf(acc[0]) > flush_at;  // a long stay is flushed in parts
        if (ev == EV_ESCAPE) {
            L.escaped += p.w;
            p.alive = false;
        }
        if (flush) {
            unsigned long long *t = gfx + pix * K;
#pragma unroll
            for (int j = 0; j < K; ++j) fixed_add(t + j, acc[j]);
            mag += fabsf(acc[0]);
        }
        L.visits += vend ? 1u : 0u;
        keep = flush ? 0.f : 1.f;
    }
    ledger_flush_block(S.led, S.ledc, L);
    float wm = mag;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) wm += __shfl_xor(wm, o);
    if (lane == 0) atomicAdd(&s_mag, wm);
    __syncthreads();
    if (threadIdx.x == 0 && !(s_mag < 0x1p62f)) atomicAdd(S.ledc + 4, 1ull);   // see k_normalise
    // read once: the atomics below may alias S for all the compiler knows, and
    // a reload per add would make each add wait for the one before it
    double *const t64 = S.t64;
    const double fx_inv = S.fx_inv;
    for (int i = threadIdx.x; i < npix * K; i += blockDim.x) {
        const double v = (double)(long long)gfx[i] * fx_inv;
        if (v != 0.0) tally_add(t64 + i, v);
    }
}

// ------------------------------------------------------------------ tiled transport
// Larger grids: the grid is cut into tw x th tiles whose tallies (64-bit
// fixed-point sums, fixed_add) fit in LDS.  A run -- or a batch of runs
// sharing one packet pool and one global tile index space -- proceeds in
// generations.  Each generation: new packets are launched to keep the pool
// at `live` packets and every record is counted by tile (k_gen_count, whose
// last workgroup scans the counts into a job list); the record indices are
// sorted by tile (k_gen_scatter); a workgroup takes a job (at most job_size
// packets of one tile), keeps that tile's tally and medium in LDS, and moves
// each packet until it leaves the tile, dies, or has made max_visits visits
// there (k_transport_tile).  Records stay where they were written: two pools
// alternate between generations, one read, the other receiving the packets
// that leave.  Every tally update is an LDS atomic; HBM sees one coalesced
// flush of the tile per job.  Once every packet is launched and at most
// finish_at remain, the control block marks the run done: later generations
// do nothing and the finisher (k_finish) moves the rest to their end.

// Device control block of a tiled run (zeroed at set-up).
// The counters that every workgroup or wave of a generation updates with
// device atomics each sit in a 128-byte line of their own: atomics on one
// line are serialised, whichever word they address.
struct GenCtl {
    uint32_t done;                // the finisher threshold was met: later generations do nothing
    uint32_t fin_pool, fin_nc, fin_nl;   // where the finisher finds the records when done
    uint32_t gen_done;            // generations run before the threshold was met
    uint32_t n_rec, n_jobs;
    uint32_t overflow;            // a queue or the job list would have overflowed (output NaN)
    uint32_t new_first_prob;      // first problem with packets left to launch
    uint64_t launched_total, todo_total;
    alignas(128) uint32_t wg_done;      // workgroups of k_gen_count that finished (the last one scans)
    alignas(128) uint32_t job_cursor;   // jobs claimed by the tile kernel's workgroups
    alignas(128) uint32_t nc[2];        // carried-region slots reserved in pool p
    alignas(128) uint32_t nvalid[2];    // valid records among them
    alignas(128) uint32_t nl[2];        // launch-region records of pool p
};

// Batch-wide parameters of the tiled kernels (by value).
// Each tile's sort cursor sits in a 128-byte line of its own: the sort's
// reservations are device atomics, and those on one line are serialised, so
// cursors packed 32 to a line would make the tiles wait for each other.
constexpr uint32_t kCursorStride = 32;

struct Gen {
    int tw, th, ntiles, nprob;
    uint32_t live;                // packets kept alive per generation
    uint32_t cap_c, cap_l;        // slots of a pool's carried and launch regions
    uint32_t job_size, max_visits, tail_visits, finish_at;
    uint32_t job_min;             // smallest job a generation with few packets splits its tiles into
    uint32_t slots;               // workgroups of the tile kernel
    uint32_t quiet_pct;           // a job turns quiet when this percent of its lanes' worth of stays is left
    uint32_t slice;               // slots a wave reserves at a time in a carried region (64 .. 256)
    const ProbDev *probs;
    const uint32_t *tile_prob;    // problem of each global tile
    struct PacketRec *pool[2];    // [cap_c + cap_l] records
    uint32_t *ptile[2];           // tile of each slot (kInvalidTile: empty slot)
    uint32_t *sidx;               // slots of the generation's records sorted by tile [live]
    uint32_t *tile_count;
    uint32_t *tile_cursor;        // [ntiles][kCursorStride]: one 128-byte line per tile's cursor
    uint4 *jobs;                  // (tile, first position in sidx, count, problem)
    uint32_t max_jobs;
    GenCtl *ctl;
    uint64_t *launched;           // packets of each problem launched so far
    unsigned long long *fin_cur;  // finisher work cursors: [0] records, [1 + p] unlaunched packets of problem p
};

// The total of packets to launch: problems whose source has no power (or is
// unusable) launch none, which only the device descriptors know.
__global__ void k_ctl_init(Gen G) {
    uint64_t t = 0;
    for (int p = 0; p < G.nprob; ++p) t += G.probs[p].todo;
    G.ctl->todo_total = t;
}

__device__ __forceinline__ void rec_store(PacketRec *r, const Packet &p, uint32_t tile, uint32_t prob) {
    float4 *q = reinterpret_cast<float4 *>(r);
    q[0] = make_float4(p.fx, p.fz, p.sx, p.sz);
    q[1] = make_float4(p.w, p.w0abs, p.tau, p.uh);
    uint4 *u = reinterpret_cast<uint4 *>(r);
    u[2] = make_uint4(__float_as_uint(p.ur), p.k, (uint32_t)p.ix, (uint32_t)p.iz);
    u[3] = make_uint4((uint32_t)p.pid, (uint32_t)(p.pid >> 32), tile, prob);
}

__device__ __forceinline__ void rec_decode(const uint4 a, const uint4 b, const uint4 c, const uint2 d, Packet &p) {
    p.fx = __uint_as_float(a.x);
    p.fz = __uint_as_float(a.y);
    set_dir(p, __uint_as_float(a.z), __uint_as_float(a.w));
    p.w = __uint_as_float(b.x);
    p.w0abs = __uint_as_float(b.y);
    p.tau = __uint_as_float(b.z);
    p.uh = __uint_as_float(b.w);
    p.ur = __uint_as_float(c.x);
    p.k = c.y;
    p.ix = (int)c.z;
    p.iz = (int)c.w;
    p.pid = (uint64_t)d.x | ((uint64_t)d.y << 32);
    p.alive = true;
}

__device__ __forceinline__ uint32_t rec_load(const PacketRec *r, Packet &p) {
    const float4 *q = reinterpret_cast<const float4 *>(r);
    const float4 a = q[0], b = q[1];
    const uint4 *u = reinterpret_cast<const uint4 *>(r);
    const uint4 c = u[2], d = u[3];
    p.fx = a.x; p.fz = a.y;
    set_dir(p, a.z, a.w);
    p.w = b.x; p.w0abs = b.y; p.tau = b.z; p.uh = b.w;
    p.ur = __uint_as_float(c.x);
    p.k = c.y;
    p.ix = (int)c.z;
    p.iz = (int)c.w;
    p.pid = (uint64_t)d.x | ((uint64_t)d.y << 32);
    p.alive = true;
    return d.w;
}

__device__ __forceinline__ uint32_t tile_in(int tw, int th, int ntx, int ix, int iz) {
    return (uint32_t)((iz / th) * ntx + ix / tw);
}

// Wave-private slices of a pool's carried region: a wave reserves G.slice
// slots with one atomic on the region's counter (shared by every wave of the
// device, so it is touched rarely) and fills them; unused slots are marked
// invalid.
struct QueueSlice {
    uint32_t base = 0, used = 0, nput = 0;
    bool valid = false;
};

__device__ __forceinline__ void slice_close(const Gen &G, int pool, QueueSlice &q) {
    if (!q.valid) return;
    const int lane = __lane_id();
    for (uint32_t i = q.used + lane; i < G.slice; i += 64)
        if (q.base + i < G.cap_c) G.ptile[pool][q.base + i] = kInvalidTile;
}

// Appends the packet of every lane with `put` set to the pool's carried region.
__device__ __forceinline__ void slice_put(const Gen &G, int pool, QueueSlice &q, bool put, const Packet &p,
                                          uint32_t tile, uint32_t prob) {
    const unsigned long long m = __ballot(put);
    if (!m) return;
    const int n = __popcll(m);
    const int lane = __lane_id();
    if (!q.valid || q.used + n > G.slice) {
        slice_close(G, pool, q);
        uint32_t base = 0;
        if (lane == 0) base = atomicAdd(&G.ctl->nc[pool], G.slice);
        q.base = __shfl(base, 0);
        q.used = 0;
        q.valid = true;
    }
    if (put) {
        const uint32_t pos = q.base + q.used + __popcll(m & ((1ull << lane) - 1ull));
        if (pos < G.cap_c) {
            rec_store(G.pool[pool] + pos, p, tile, prob);
            G.ptile[pool][pos] = tile;
        } else {
            atomicOr(&G.ctl->overflow, 1u);   // never written; the run's output becomes NaN
        }
    }
    q.used += n;
    q.nput += n;
}

// End of a wave's appends: pad its last slice and count its records.
__device__ __forceinline__ void slice_finish(const Gen &G, int pool, QueueSlice &q) {
    slice_close(G, pool, q);
    if (q.nput && __lane_id() == 0) atomicAdd(&G.ctl->nvalid[pool], q.nput);
}

// ---- generation step 1: launch and count (the last workgroup scans)
constexpr int kGenBlock = 1024;
constexpr int kHistTiles = 32768;  // tiles histogrammed in LDS (dynamic, 4 bytes each); beyond, wave-aggregated global atomics
constexpr int kMaxAlloc = 256;     // problems that receive new packets in one generation
constexpr int kCountPer = 8;       // carried records per thread and pass of the count

// Counts one record of tile t (LDS histogram, or the global count directly).
__device__ __forceinline__ void count_tile(const Gen &G, uint32_t *hist, bool local, uint32_t t, bool valid) {
    if (local) {
        if (valid) atomicAdd(hist + t, 1u);
        return;
    }
    const int lane = __lane_id();
    bool pend = valid;
    for (;;) {
        const unsigned long long m = __ballot(pend);
        if (!m) break;
        const int leader = __ffsll((long long)m) - 1;
        const uint32_t t0 = __shfl(t, leader);
        const unsigned long long same = __ballot(pend && t == t0);
        if (lane == leader) atomicAdd(G.tile_count + t0, (uint32_t)__popcll(same));
        if (pend && t == t0) pend = false;
    }
}

// The scan of a generation, by the last workgroup of k_gen_count: exclusive
// scan of the tile counts into cursors and a job list; bookkeeping of the
// launches; the finisher decision; reset of the other pool's counters.
// Inclusive scan of one count per thread over the kGenBlock threads of the
// workgroup, and the workgroup's total: within each wave by shuffles, then
// over the waves' totals (two barriers instead of two per doubling step).
// wsum: kGenBlock / 64 words of LDS.
__device__ __forceinline__ uint32_t block_scan(uint32_t v, uint32_t *wsum, uint32_t &total) {
    const int lane = __lane_id(), wave = threadIdx.x >> 6;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t u = __shfl_up(v, off);
        if (lane >= off) v += u;
    }
    if (lane == 63) wsum[wave] = v;
    __syncthreads();
    uint32_t pre = 0, all = 0;
    for (int w = 0; w < kGenBlock / 64; ++w) {
        const uint32_t x = wsum[w];
        pre += w < wave ? x : 0u;
        all += x;
    }
    __syncthreads();   // wsum is free for the next scan
    total = all;
    return v + pre;
}

__device__ void gen_scan(const Gen &G, int g, uint32_t *buf, int np, const uint32_t *a_prob, const uint32_t *a_new) {
    GenCtl *C = G.ctl;
    const int cur = g & 1;
    const int t = threadIdx.x;
    const int per = (G.ntiles + kGenBlock - 1) / kGenBlock;
    const int a = t * per, b = min(G.ntiles, a + per);
    uint32_t nrec = 0;
    for (int i = a; i < b; ++i) nrec += G.tile_count[i];
    uint32_t total = 0;
    const uint32_t rec_incl = block_scan(nrec, buf, total);
    // job size: job_size, or smaller when the generation's records would not
    // give every workgroup two jobs (never below job_min): a generation with
    // few packets then spreads its larger tiles over several workgroups
    const uint32_t want = (uint32_t)(((uint64_t)total + 2ull * G.slots - 1) / (2ull * G.slots));
    const uint32_t js = min(G.job_size, max(G.job_min, want));
    uint32_t njob = 0;
    for (int i = a; i < b; ++i) njob += (G.tile_count[i] + js - 1) / js;
    uint32_t total_jobs = 0;
    const uint32_t job_incl = block_scan(njob, buf, total_jobs);
    const bool fits = total <= G.live && total_jobs <= G.max_jobs;   // hold by construction
    uint32_t roff = rec_incl - nrec, joff = job_incl - njob;
    for (int i = a; i < b; ++i) {
        const uint32_t c = G.tile_count[i];
        G.tile_cursor[(size_t)i * kCursorStride] = roff;
        if (fits)
            for (uint32_t s0 = 0; s0 < c; s0 += js)
                G.jobs[joff++] = make_uint4((uint32_t)i, roff + s0, min(js, c - s0), G.tile_prob[i]);
        roff += c;
        G.tile_count[i] = 0;
    }
    __syncthreads();
    if (t == 0) {
        uint64_t lt = C->launched_total;
        for (int k = 0; k < np; ++k) {
            G.launched[a_prob[k]] += a_new[k];
            lt += a_new[k];
        }
        C->launched_total = lt;
        uint32_t p = C->new_first_prob;
        while (p < (uint32_t)G.nprob && G.launched[p] >= G.probs[p].todo) ++p;
        C->new_first_prob = p;
        C->n_rec = total;
        C->n_jobs = fits ? total_jobs : 0u;
        C->job_cursor = 0;
        if (!fits) C->overflow = 1u;
        // the packets left fit the finisher: this generation moves nothing
        if (lt >= C->todo_total && total <= G.finish_at) {
            C->done = 1u;
            C->fin_pool = (uint32_t)cur;
            C->fin_nc = min(C->nc[cur], G.cap_c);
            C->fin_nl = min(C->nl[cur], G.cap_l);
            C->gen_done = (uint32_t)g;
            C->n_jobs = 0;
        }
        // the other pool receives this generation's leavers, then the next one's launches
        C->nc[cur ^ 1] = 0;
        C->nvalid[cur ^ 1] = 0;
        C->nl[cur ^ 1] = 0;
        C->wg_done = 0;
    }
}

__global__ void __launch_bounds__(kGenBlock) k_gen_count(Gen G, int g) {
    GenCtl *C = G.ctl;
    extern __shared__ uint32_t hist[];   // max(ntiles, 2 kGenBlock) counts (gen_hist_lds), or the scan's buffer
    __shared__ uint32_t a_prob[kMaxAlloc], a_new[kMaxAlloc], a_pre[kMaxAlloc + 1];
    __shared__ uint64_t a_base[kMaxAlloc];
    __shared__ uint32_t w_cnt[kGenBlock / 64];
    __shared__ uint32_t s_base;
    __shared__ int s_np, s_last;
    if (C->done) return;   // uniform: written by an earlier kernel
    const int cur = g & 1;
    const int lane = __lane_id(), wave = threadIdx.x >> 6;
    const bool local = G.ntiles <= kHistTiles;
    if (local)
        for (int i = threadIdx.x; i < G.ntiles; i += kGenBlock) hist[i] = 0u;
    if (threadIdx.x == 0) {
        // new packets fill the pool up to `live`, problem after problem; each
        // problem's share occupies a range of the launch index space rounded
        // up to whole workgroups, so an iteration below serves one problem
        uint64_t room = C->nvalid[cur] < G.live ? G.live - C->nvalid[cur] : 0;
        int m = 0;
        uint32_t pre = 0;
        for (int p = (int)C->new_first_prob; p < G.nprob && room > 0 && m < kMaxAlloc; ++p) {
            const uint64_t left = G.probs[p].todo - G.launched[p];
            if (!left) continue;
            const uint32_t k = (uint32_t)min<uint64_t>(left, room);
            a_prob[m] = (uint32_t)p;
            a_base[m] = G.launched[p];
            a_new[m] = k;
            a_pre[m] = pre;
            pre += (k + kGenBlock - 1) / kGenBlock * kGenBlock;
            room -= k;
            ++m;
        }
        a_pre[m] = pre;
        s_np = m;
    }
    __syncthreads();
    const int np = s_np;
    const uint32_t n_new = a_pre[np];
    LedgerRegs L;
    int lk = -1;   // allocation entry whose problem the ledger L holds (workgroup-uniform)
    for (uint32_t b0 = blockIdx.x * kGenBlock; b0 < n_new; b0 += gridDim.x * kGenBlock) {
        int lo = 0, hi = np - 1;   // the entry whose range holds b0
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (a_pre[mid] <= b0) lo = mid; else hi = mid - 1;
        }
        if (lo != lk) {
            if (lk >= 0) {
                const ProbDev &q = G.probs[a_prob[lk]];
                ledger_flush_block(q.led, q.ledc, L);
                L = LedgerRegs();
            }
            lk = lo;
        }
        const uint32_t prob = a_prob[lo];
        const ProbDev &S = G.probs[prob];
        const uint32_t i = b0 - a_pre[lo] + threadIdx.x;
        Packet p;
        p.alive = false;
        if (i < a_new[lo]) launch_state(S, S.pid0 + a_base[lo] + i, p, L);
        const unsigned long long m = __ballot(p.alive);
        if (lane == 0) w_cnt[wave] = (uint32_t)__popcll(m);
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t tot = 0;
            for (int w = 0; w < kGenBlock / 64; ++w) tot += w_cnt[w];
            s_base = tot ? atomicAdd(&C->nl[cur], tot) : 0u;
        }
        __syncthreads();
        uint32_t tile = kInvalidTile;
        if (p.alive) {
            uint32_t pos = s_base + __popcll(m & ((1ull << lane) - 1ull));
            for (int w = 0; w < wave; ++w) pos += w_cnt[w];
            tile = (uint32_t)S.tile_base + tile_in(G.tw, G.th, S.ntx, p.ix, p.iz);
            if (pos < G.cap_l) {
                rec_store(G.pool[cur] + G.cap_c + pos, p, tile, prob);
                G.ptile[cur][G.cap_c + pos] = tile;
            } else {
                atomicOr(&C->overflow, 1u);
                tile = kInvalidTile;
            }
        }
        count_tile(G, hist, local, tile, tile != kInvalidTile);
        __syncthreads();   // w_cnt and s_base are reused
    }
    if (lk >= 0) {
        const ProbDev &q = G.probs[a_prob[lk]];
        ledger_flush_block(q.led, q.ledc, L);
    }
    // the records carried over from the last generation, kCountPer per
    // thread with every load issued before the first is counted (an index
    // past the records reads the last one, then counts as no record)
    const uint32_t nc = min(C->nc[cur], G.cap_c);
    const uint32_t *ct = G.ptile[cur];
    for (uint32_t b0 = blockIdx.x * kGenBlock * kCountPer; b0 < nc; b0 += gridDim.x * kGenBlock * kCountPer) {
        uint32_t t[kCountPer];
#pragma unroll
        for (int r = 0; r < kCountPer; ++r) t[r] = ct[min(b0 + r * kGenBlock + threadIdx.x, nc - 1u)];
#pragma unroll
        for (int r = 0; r < kCountPer; ++r) {
            const bool in = b0 + r * kGenBlock + threadIdx.x < nc;
            count_tile(G, hist, local, t[r], in && t[r] != kInvalidTile);
        }
    }
    __syncthreads();
    if (local)
        for (int i = threadIdx.x; i < G.ntiles; i += kGenBlock)
            if (hist[i]) atomicAdd(G.tile_count + i, hist[i]);
    // the last workgroup to finish sees every count and scans them
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        s_last = atomicAdd(&C->wg_done, 1u) == gridDim.x - 1;
    }
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    gen_scan(G, g, hist, np, a_prob, a_new);
}

// ---- generation step 2: sort the record indices by tile
// A workgroup takes chunks of kScatterChunk records of the generation (the
// pool's carried region, then its launch region); each record gets its rank
// among the chunk's records of its tile from an LDS atomic on that tile's
// counter, the record of rank 0 reserves the tile's range with one global
// atomic and leaves the range's start in the counter, and every record's
// slot index lands at start + rank; the rank-0 records then clear their
// counters, so a chunk costs in proportion to its records, not to the tiles.
// Beyond kHistTiles tiles, ranks come from wave-aggregated global atomics.
constexpr int kScatterPer = 8;                              // records per thread and chunk
constexpr uint32_t kScatterChunk = 256u * kScatterPer;

__device__ __forceinline__ uint32_t gen_slot(const Gen &G, uint32_t u, uint32_t nc) {
    return u < nc ? u : G.cap_c + (u - nc);
}

__global__ void __launch_bounds__(256) k_gen_scatter(Gen G, int g) {
    extern __shared__ uint32_t cnt[];   // [ntiles] when ntiles <= kHistTiles (gen_hist_lds)
    GenCtl *C = G.ctl;
    if (C->done) return;
    const int cur = g & 1;
    const uint32_t nc = min(C->nc[cur], G.cap_c), nl = min(C->nl[cur], G.cap_l);
    const uint32_t n = nc + nl;
    const uint32_t *pt = G.ptile[cur];
    const int lane = __lane_id();
    if (G.ntiles <= kHistTiles) {
        for (int i = threadIdx.x; i < G.ntiles; i += blockDim.x) cnt[i] = 0u;
        __syncthreads();
        for (uint32_t c0 = blockIdx.x * kScatterChunk; c0 < n; c0 += gridDim.x * kScatterChunk) {
            // the chunk's tiles, every load issued before the first is used
            // (an index past the records reads the last record, then counts
            // as no record)
            uint32_t t[kScatterPer], rank[kScatterPer];
#pragma unroll
            for (int r = 0; r < kScatterPer; ++r) t[r] = pt[gen_slot(G, min(c0 + r * 256u + threadIdx.x, n - 1u), nc)];
#pragma unroll
            for (int r = 0; r < kScatterPer; ++r) {
                if (c0 + r * 256u + threadIdx.x >= n) t[r] = kInvalidTile;
                rank[r] = t[r] != kInvalidTile ? atomicAdd(cnt + t[r], 1u) : 0u;
            }
            __syncthreads();
            // all counts read, then all reservations issued, then all starts
            // written: the compiler cannot tell that a thread's rank-0 records
            // are of different tiles, and interleaved, each LDS write would
            // wait for its atomic's return before the next count is read
            uint32_t cn[kScatterPer], base[kScatterPer];
#pragma unroll
            for (int r = 0; r < kScatterPer; ++r) cn[r] = t[r] != kInvalidTile && rank[r] == 0u ? cnt[t[r]] : 0u;
#pragma unroll
            for (int r = 0; r < kScatterPer; ++r)
                base[r] = cn[r] ? atomicAdd(G.tile_cursor + (size_t)t[r] * kCursorStride, cn[r]) : 0u;
#pragma unroll
            for (int r = 0; r < kScatterPer; ++r)
                if (cn[r]) cnt[t[r]] = base[r];
            __syncthreads();
            // the slot indices: every address formed before the first store
            // (an address register reused from one store to the next would
            // make each store wait for the one before)
            uint32_t *dst[kScatterPer];
            uint32_t val[kScatterPer];
#pragma unroll
            for (int r = 0; r < kScatterPer; ++r) {
                const uint32_t pos = t[r] != kInvalidTile ? cnt[t[r]] + rank[r] : G.live;
                dst[r] = pos < G.live ? G.sidx + pos : nullptr;
                val[r] = gen_slot(G, c0 + r * 256u + threadIdx.x, nc);
            }
#pragma unroll
            for (int r = 0; r < kScatterPer; ++r)
                if (dst[r]) *dst[r] = val[r];
            // keeps every address and value in its own register until all
            // stores are issued (emits no instruction)
#pragma unroll
            for (int r = 0; r < kScatterPer; ++r) asm volatile("" ::"v"(dst[r]), "v"(val[r]));
            __syncthreads();
#pragma unroll
            for (int r = 0; r < kScatterPer; ++r)
                if (cn[r]) cnt[t[r]] = 0u;
            __syncthreads();
        }
        return;
    }
    for (uint32_t b0 = blockIdx.x * blockDim.x; b0 < n; b0 += gridDim.x * blockDim.x) {
        const uint32_t u = b0 + threadIdx.x;
        const uint32_t t = u < n ? pt[gen_slot(G, u, nc)] : kInvalidTile;
        bool pend = t != kInvalidTile;
        for (;;) {
            const unsigned long long m = __ballot(pend);
            if (!m) break;
            const int leader = __ffsll((long long)m) - 1;
            const uint32_t t0 = __shfl(t, leader);
            const unsigned long long same = __ballot(pend && t == t0);
            uint32_t b = 0;
            if (lane == leader) b = atomicAdd(G.tile_cursor + (size_t)t0 * kCursorStride, (uint32_t)__popcll(same));
            b = __shfl(b, leader);
            if (pend && t == t0) {
                const uint32_t pos = b + __popcll(same & ((1ull << lane) - 1ull));
                if (pos < G.live) G.sidx[pos] = gen_slot(G, u, nc);
                pend = false;
            }
        }
    }
}

// ---- generation step 3: move the packets tile by tile
template <int NH>
__global__ void __launch_bounds__(tile_block(NH)) __attribute__((amdgpu_waves_per_eu(NH <= 16 ? 4 : 2)))
k_transport_tile(Gen G, int g) {
    constexpr int K = 2 * NH + 1;
    // [tw*th][K] fixed-point sums: value * fx of the job's problem (fixed_add)
    extern __shared__ unsigned long long fxt[];
    float4 *smed = reinterpret_cast<float4 *>(fxt + (((size_t)G.tw * G.th * K + 1) & ~size_t(1)));
    uint32_t *sadds = reinterpret_cast<uint32_t *>(smed + G.tw * G.th);   // fixed_add_raw adds per pixel
    __shared__ uint32_t s_job[5];
    __shared__ uint32_t s_next;
    __shared__ uint32_t s_left;   // packets of the job whose stay has not ended
    __shared__ float s_mag;
    GenCtl *C = G.ctl;
    if (C->done) return;
    const int cur = g & 1, nxt = cur ^ 1;
    const PacketRec *in = G.pool[cur];
    const int lane = __lane_id();
    const int ntp = G.tw * G.th;
    const unsigned long long lt_mask = (1ull << lane) - 1ull;
    constexpr uint32_t kNone = 0xFFFFFFFFu;
    LedgerTile L;
    QueueSlice q;
    int cur_prob = -1;   // problem whose ledger L holds

    for (;;) {
        if (threadIdx.x == 0) {
            const uint32_t j = atomicAdd(&C->job_cursor, 1u);
            const bool ok = j < C->n_jobs;
            const uint4 jb = ok ? G.jobs[j] : make_uint4(0u, 0u, 0u, 0u);
            s_job[0] = ok ? 1u : 0u;
            s_job[1] = jb.x;
            s_job[2] = jb.y;
            s_job[3] = jb.z;
            s_job[4] = jb.w;
            s_next = 0;
            s_left = jb.z;
            s_mag = 0.f;
        }
        __syncthreads();
        if (!s_job[0]) break;
        const uint32_t tile = s_job[1], first = s_job[2], cnt = s_job[3], prob = s_job[4];
        const ProbDev &pd = G.probs[prob];
        if ((int)prob != cur_prob) {   // the ledger follows the problem (uniform in the workgroup)
            if (cur_prob >= 0) {
                ledger_flush_tile(G.probs[cur_prob].led, G.probs[cur_prob].ledc, L);
                L = LedgerTile();
            }
            cur_prob = (int)prob;
        }
        const Hot H = hot_of(pd);
        const int ntx = pd.ntx, local = (int)tile - pd.tile_base;
        const float4 *gmed = pd.med;
        double *t64 = pd.t64;
        const float fx = pd.fx;   // power of two: the scaled FP32 sums round exactly as unscaled ones
        const float flush_at = pd.flush_at;
        const int tx0 = (local % ntx) * G.tw, tz0 = (local / ntx) * G.th;
        for (int i = threadIdx.x; i < ntp * K; i += blockDim.x) fxt[i] = 0ull;
        for (int i = threadIdx.x; i < ntp; i += blockDim.x) sadds[i] = 0u;
        for (int i = threadIdx.x; i < ntp; i += blockDim.x) {
            const int gx = tx0 + i % G.tw, gz = tz0 + i / G.tw;
            const bool in_grid = gx < H.nx && gz < H.nz;
            smed[i] = in_grid ? load_medium(gmed, gz * H.nx + gx) : make_float4(0.f, 0.f, 0.f, 0.f);
        }
        __syncthreads();

        Packet p;
        idle_packet(p, tx0, tz0);
        uint32_t nvis = 0;
        float mag = 0.f;   // sum of the |a0| this lane flushed in this job: bounds every slot's magnitude
        float acc[K], keep = 1.f;   // keep = 0 after a flush: the next deposit restarts the sums
#pragma unroll
        for (int j = 0; j < K; ++j) acc[j] = 0.f;
        // Each lane holds the record of its next packet in registers, loaded
        // one whole stay ahead, and the pool slot of the packet after it,
        // claimed one more stay ahead, so neither a refill nor the record
        // load waits for memory.
        bool more = true, has_next = false;
        uint32_t nslot = kNone;   // claimed slot whose record is not loaded yet
        // The job turns quiet once the stays not yet ended are at most
        // quiet_pct percent of its lanes' worth (min(cnt, lanes)); from then
        // on a packet pauses after tail_visits more visits, so the workgroup
        // is not held by its longest stays (they resume next generation).
        const uint32_t quiet_at = (uint32_t)(((uint64_t)min(cnt, (uint32_t)tile_block(NH)) * G.quiet_pct) / 100u);
        bool quiet = false;       // wave-uniform
        uint32_t tail_nvis = 0;   // visits of the current stay when the job turned quiet
        // (the last word is the packet id alone: a load whose destination
        // registers are partly dead lets them be reused, and the reuse must then
        // wait for the load)
        uint4 nr0 = make_uint4(0u, 0u, 0u, 0u), nr1 = nr0, nr2 = nr0;
        uint2 nr3 = make_uint2(0u, 0u);
        for (;;) {
            // a free lane takes its prefetched record (the only decode site)
            if (!p.alive && has_next) {
                rec_decode(nr0, nr1, nr2, nr3, p);
                has_next = false;
                nvis = 0;
                tail_nvis = 0;
            }
            // the medium of the pixel of this step, read before the claim below
            // so its LDS latency overlaps with that work
            const bool live = p.alive;
            // 24-bit products (full-rate v_mad_i32_i24): tile sizes and offsets are small
            const int lp = live ? __mul24(p.iz - tz0, G.tw) + (p.ix - tx0) : 0;
            const float4 mm = smed[lp];
            // free record registers take the record of the slot claimed earlier
            // (the slot index is checked here, a stay after its load, not at
            // the claim, where the check would wait for that load)
            if (!has_next && nslot != kNone) {
                if (nslot < G.cap_c + G.cap_l) {   // always true; guards the loads
                    const uint4 *r = reinterpret_cast<const uint4 *>(in + nslot);
                    nr0 = r[0];
                    nr1 = r[1];
                    nr2 = r[2];
                    const uint64_t id = in[nslot].pid;
                    nr3 = make_uint2((uint32_t)id, (uint32_t)(id >> 32));
                    has_next = true;
                }
                nslot = kNone;
            }
            // lanes without a claimed slot claim the next ones of the job
            if (more) {
                const unsigned long long want = __ballot(nslot == kNone);
                if (want) {
                    const int nw = __popcll(want);
                    const int leader = __ffsll((long long)want) - 1;
                    uint32_t base = 0;
                    if (lane == leader) base = atomicAdd(&s_next, (uint32_t)nw);
                    base = __shfl(base, leader);
                    if (base + nw >= cnt) more = false;
                    if (nslot == kNone) {
                        const uint32_t my = base + __popcll(want & lt_mask);
                        if (my < cnt) nslot = G.sidx[first + my];
                    }
                }
            }
            if (!__ballot(p.alive)) {
                if (!more && !__ballot(has_next || nslot != kNone)) break;
            }
            if (!quiet && __hip_atomic_load(&s_left, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) <= quiet_at) {
                quiet = true;
                tail_nvis = nvis;
            }
            // every lane steps (no branch); a free lane's result is discarded
            float T = 0.f, dw = 0.f;
            int ev = step(H, p, mm, T, dw);
            ev = live ? ev : EV_NONE;
            T = live ? T : 0.f;
            dw = live ? dw : 0.f;
            L.absorbed += (double)dw;
            L.segments += live ? 1u : 0u;
            deposit_harmonics<NH>(T * fx, p.sx, p.sz, keep, acc);   // direction of the segment, before any scatter
            const bool at = ev == EV_SCATTER;
            // the roulette decides whether the visit ends here; the deflection
            // and its random numbers come after the flush below, so that their
            // arithmetic overlaps the flush's LDS atomics
            const bool killed = scatter_roulette(H, p, at, L);
            const bool vend = killed || (ev != EV_NONE && !at);   // the visit ends
            // |a_n| <= a0 (one sign per packet): a long stay in one pixel is
            // flushed in parts, so every flush stays inside fixed_add's range
            const bool flush = vend || fabsf(acc[0]) > flush_at;
            if (ev == EV_ESCAPE) {
                L.escaped += p.w;
                p.alive = false;
            }
            bool leave = false;
            uint32_t dest = tile;
            if (flush) {
                unsigned long long *t = fxt + __umul24((uint32_t)lp, (uint32_t)K);
#pragma unroll
                for (int j = 0; j < K; ++j) fixed_add_raw(t + j, acc[j]);
                atomicAdd(sadds + lp, 1u);
                mag += fabsf(acc[0]);
            }
            scatter_deflect(H, p, at && !killed, killed, mm.w, L);
            if (vend) {
                L.visits += 1;
                nvis += 1;
                if (ev == EV_CROSS) {
                    const int ox = p.ix < tx0 ? -1 : (p.ix >= tx0 + G.tw ? 1 : 0);
                    const int oz = p.iz < tz0 ? -1 : (p.iz >= tz0 + G.th ? 1 : 0);
                    const bool out = (ox | oz) != 0;
                    dest = (uint32_t)((int)tile + __mul24(oz, ntx) + ox);   // a crossing moves one pixel: a neighbour tile
                    leave = out || nvis >= (quiet ? min(G.max_visits, tail_nvis + G.tail_visits) : G.max_visits);
                }
            }
            keep = flush ? 0.f : 1.f;
            slice_put(G, nxt, q, leave, p, dest, prob);
            if (leave) {
                p.alive = false;
                nvis = 0;
            }
            const unsigned long long ended = __ballot(live && !p.alive);   // stays that ended here
            if (ended && lane == 0) atomicSub(&s_left, (uint32_t)__popcll(ended));
        }
        // no slot can exceed the sum of the magnitudes flushed into the tile;
        // a job that could have wrapped the 64-bit sums is counted and its
        // run's output becomes NaN (k_normalise)
        float wm = mag;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) wm += __shfl_xor(wm, o);
        if (lane == 0) atomicAdd(&s_mag, wm);
        __syncthreads();
        if (threadIdx.x == 0 && !(s_mag < 0x1p62f)) atomicAdd(pd.ledc + 4, 1ull);
        // fx_inv is read once: the atomics may alias pd for all the compiler
        // knows, and a reload per add would make each add wait for the one before
        const double fx_inv = pd.fx_inv;
        for (int i = threadIdx.x; i < ntp * K; i += blockDim.x) {
            const int lp = i / K, c = i - lp * K;
            const double v = (double)fixed_value(fxt[i], sadds[lp]) * fx_inv;
            const int gx = tx0 + lp % G.tw, gz = tz0 + lp / G.tw;
            if (v != 0.0 && gx < H.nx && gz < H.nz) tally_add(t64 + (size_t)(gz * H.nx + gx) * K + c, v);
        }
        __syncthreads();
    }
    slice_finish(G, nxt, q);
    if (cur_prob >= 0) ledger_flush_tile(G.probs[cur_prob].led, G.probs[cur_prob].ledc, L);   // uniform
}

// ------------------------------------------------------------------ tail finisher
// When few packets remain, the generations would be dominated by the
// longest-lived packets.  The finisher moves each remaining packet to its end
// without migration, whatever problem it belongs to: first the records the
// last generation left (the pool of the generation that found the threshold
// met, or the pool after the last enqueued generation), then -- only if the
// generations ran out before every packet was launched -- the packets of
// each problem not launched yet (one launch per problem, `prob_only`).  A
// wave stages the K-vectors of the visits it completes in LDS and adds them
// to the HBM FP64 tallies as contiguous runs of atomics.
constexpr int kBlockFinish = 256;

// Adds a wave's staged visit sums (n visits of K values) to the HBM tallies:
// consecutive lanes take consecutive values, so each pixel's K channels go
// out as one contiguous run of atomics.  A staged visit carries the address
// of its pixel's K sums and its problem's inverse scale, so the loop reads
// only LDS and its atomics go out back to back.
__device__ __forceinline__ void finish_flush_stage(const float *stage, const unsigned long long *stage_dst,
                                                   const double *stage_scale, int n, int K) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int total = n * K;
    for (int e = __lane_id(); e < total; e += 64) {
        const int v = e / K;
        const float val = stage[e];
        if (val != 0.f)
            tally_add(reinterpret_cast<double *>(stage_dst[v]) + (e - v * K),
                      __builtin_rint((double)val) * stage_scale[v]);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Ledger of lanes that may hold different problems (prob < 0: nothing held):
// the lanes of each problem in turn are summed over the wave and one lane
// adds the sums to that problem's ledger.
__device__ __forceinline__ void ledger_flush_lanes(const Gen &G, int prob, const LedgerRegs &L) {
    const int lane = __lane_id();
    int pend = prob;
    for (;;) {
        const unsigned long long m = __ballot(pend >= 0);
        if (!m) break;
        const int leader = __ffsll((long long)m) - 1;
        const int p0 = __shfl(pend, leader);
        const bool mine = pend == p0;
        double v[5] = {L.launched, L.absorbed, L.escaped, L.gain, L.loss};
        unsigned long long c[4] = {L.packets, L.segments, L.visits, L.scatters};
#pragma unroll
        for (int i = 0; i < 5; ++i) v[i] = mine ? v[i] : 0.0;
#pragma unroll
        for (int i = 0; i < 4; ++i) c[i] = mine ? c[i] : 0ull;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
            for (int i = 0; i < 5; ++i) v[i] += __shfl_xor(v[i], off);
#pragma unroll
            for (int i = 0; i < 4; ++i) c[i] += __shfl_xor(c[i], off);
        }
        if (lane == leader) {
            const ProbDev &S = G.probs[p0];
            for (int i = 0; i < 5; ++i)
                if (v[i] != 0.0) atomicAdd(S.led + i, v[i]);
            for (int i = 0; i < 4; ++i)
                if (c[i]) atomicAdd(S.ledc + i, c[i]);
        }
        if (mine) pend = -1;
    }
}

// Few packets per lane and long histories make this kernel latency-bound, so
// its loop keeps global memory off the dependent chain where it can: the
// medium of the pixel a packet enters is loaded one iteration ahead of its
// use, and a wave gathers the sums of up to 64 completed visits in LDS before
// it adds them to the tally (the wait for those atomics then comes once per
// buffer, not once per visit).  Lanes branch (a lone packet in a wave pays
// only for what it does).
template <int NH>
__global__ void __launch_bounds__(kBlockFinish) k_finish(Gen G, int g_last, int prob_only) {
    constexpr int K = 2 * NH + 1;
    extern __shared__ float stage_all[];
    GenCtl *C = G.ctl;
    const int lane = __lane_id();
    const int wave = threadIdx.x >> 6;
    float *stage = stage_all + wave * 64 * K;
    // after the K-vectors (kBlockFinish * K floats, a multiple of 8 bytes):
    // [wave][64] addresses of the visits' sums, then [wave][64] inverse scales
    unsigned long long *dst_all = reinterpret_cast<unsigned long long *>(stage_all + kBlockFinish * K);
    unsigned long long *stage_dst = dst_all + wave * 64;
    double *stage_scale = reinterpret_cast<double *>(dst_all + kBlockFinish) + wave * 64;
    const unsigned long long lt_mask = (1ull << lane) - 1ull;
    // the work: records of a pool (prob_only < 0) or the unlaunched packets of one problem
    uint32_t pool = 0, nc = 0, nl = 0;
    uint64_t n_work = 0, pid_first = 0;
    unsigned long long *cursor = G.fin_cur + (prob_only < 0 ? 0 : 1 + prob_only);
    if (prob_only < 0) {
        if (C->done) {
            pool = C->fin_pool;
            nc = C->fin_nc;
            nl = C->fin_nl;
        } else {   // the generations ran out: the leavers of the last one
            pool = (uint32_t)(g_last & 1);
            nc = min(C->nc[pool], G.cap_c);
        }
        n_work = (uint64_t)nc + nl;
    } else {
        const ProbDev &S = G.probs[prob_only];
        pid_first = G.launched[prob_only];
        n_work = S.todo > pid_first ? S.todo - pid_first : 0;
        if (!n_work) return;
    }
    LedgerRegs L;
    int lprob = -1;   // problem of the ledger L
    Packet p;
    idle_packet(p, 0, 0);
    Hot H{};
    // a lane's problem: medium (valid from the start, so that an idle lane's
    // prefetch below reads a real pixel), tally, scales
    const float4 *med = G.probs[prob_only < 0 ? 0 : prob_only].med;
    double *t64 = nullptr;
    double fx_inv = 0.0;
    float fx = 0.f, flush_at = 0.f;
    float4 mm = make_float4(0.f, 0.f, 0.f, 0.f);   // medium of the packet's pixel
    float acc[K], keep = 1.f;   // keep = 0 after a flush: the next deposit restarts the sums
#pragma unroll
    for (int j = 0; j < K; ++j) acc[j] = 0.f;
    bool more = true;
    int used = 0;   // visits staged in this wave's buffer (wave-uniform)
    for (;;) {
        if (more) {
            const unsigned long long dead = __ballot(!p.alive);
            if (dead) {
                const int ndead = __popcll(dead);
                const int leader = __ffsll((long long)dead) - 1;
                unsigned long long base = 0;
                if (lane == leader) base = atomicAdd(cursor, (unsigned long long)ndead);
                base = __shfl(base, leader);
                if (base + ndead >= n_work) more = false;
                if (!p.alive) {
                    const uint64_t my = base + __popcll(dead & lt_mask);
                    int np_ = -1;
                    Packet q;
                    q.alive = false;
                    if (my < n_work) {
                        if (prob_only < 0) {
                            const uint32_t slot = my < nc ? (uint32_t)my : G.cap_c + (uint32_t)(my - nc);
                            if (G.ptile[pool][slot] != kInvalidTile) np_ = (int)rec_load(G.pool[pool] + slot, q);
                        } else {
                            np_ = prob_only;
                        }
                    }
                    if (np_ >= 0) {
                        if (np_ != lprob) {   // a lane changes problem: its ledger goes out first (rare)
                            if (lprob >= 0) {
                                const ProbDev &O = G.probs[lprob];
                                double v[5] = {L.launched, L.absorbed, L.escaped, L.gain, L.loss};
                                unsigned long long c[4] = {L.packets, L.segments, L.visits, L.scatters};
                                for (int i = 0; i < 5; ++i)
                                    if (v[i] != 0.0) atomicAdd(O.led + i, v[i]);
                                for (int i = 0; i < 4; ++i)
                                    if (c[i]) atomicAdd(O.ledc + i, c[i]);
                                L = LedgerRegs();
                            }
                            lprob = np_;
                        }
                        const ProbDev &S = G.probs[np_];
                        if (prob_only >= 0) launch_state(S, S.pid0 + pid_first + my, q, L);
                        if (q.alive) {
                            p = q;
                            H = hot_of(S);
                            med = S.med;
                            t64 = S.t64;
                            fx_inv = S.fx_inv;
                            fx = S.fx;
                            flush_at = S.flush_at;
                            mm = load_medium(med, p.iz * H.nx + p.ix);   // a queued or launched packet is inside the grid
                        }
                    }
                }
            }
        }
        if (!__ballot(p.alive)) {
            if (!more) break;
        }
        int ev = EV_NONE, pix = 0;
        float T = 0.f;
        bool vend = false;
        if (p.alive) {
            float dw = 0.f;
            pix = p.iz * H.nx + p.ix;
            ev = step(H, p, mm, T, dw);
            L.absorbed += (double)dw;
            L.segments += 1;
            deposit_harmonics<NH>(T * fx, p.sx, p.sz, keep, acc);   // direction of the segment, before any scatter
            if (ev == EV_SCATTER) {
                if (!scatter_dir(H, p, mm.w, L)) vend = true;   // killed by roulette: the visit ends
            } else {
                vend = true;
                if (ev == EV_ESCAPE) {
                    L.escaped += p.w;
                    p.alive = false;
                }
            }
        }
        // the medium of the pixel the next step starts in (a crossing's new
        // pixel, else the same one; pixel 0 for a lane without a packet),
        // loaded outside any branch so that nothing waits for it before that step
        mm = load_medium(med, p.alive ? p.iz * H.nx + p.ix : 0);
        const bool flush = vend || (ev != EV_NONE && fabsf(acc[0]) > flush_at);
        L.visits += vend ? 1u : 0u;
        const unsigned long long fm = __ballot(flush);
        if (fm) {
            const int nf = __popcll(fm);
            if (used + nf > 64) {   // no room: the staged visits go to the tally first
                finish_flush_stage(stage, stage_dst, stage_scale, used, K);
                used = 0;
            }
            if (flush) {
                const int slot = used + __popcll(fm & lt_mask);
                float *st = stage + slot * K;
#pragma unroll
                for (int j = 0; j < K; ++j) st[j] = acc[j];
                stage_dst[slot] = reinterpret_cast<unsigned long long>(t64 + (size_t)pix * K);
                stage_scale[slot] = fx_inv;
            }
            used += nf;
        }
        if (ev != EV_NONE) keep = flush ? 0.f : 1.f;
    }
    if (used) finish_flush_stage(stage, stage_dst, stage_scale, used, K);
    ledger_flush_lanes(G, lprob, L);
}

// ------------------------------------------------------------------ discrete-ordinates tally
// The comparison tally of mc_run_binned: the same launch, step and scatter as
// the whole-grid transport (persistent lanes refilled from a global packet
// counter), but each segment adds its deposit T to raw[bin][pixel] of its
// direction's angular bin with one FP64 device atomic.
constexpr int kBinnedMax = 4096;

__global__ void __launch_bounds__(256) k_transport_binned(GridArgs A, int n_bins, double *raw) {
    const ProbDev &S = *A.pd;
    if (S.todo == 0) return;
    const Hot H = hot_of(S);
    const int lane = __lane_id();
    Packet p;
    idle_packet(p, 0, 0);
    LedgerRegs L;
    bool more = true;
    const unsigned long long lt_mask = (1ull << lane) - 1ull;
    const double per_rad = (double)n_bins / (2.0 * M_PI);
    for (;;) {
        if (more) {
            const unsigned long long dead = __ballot(!p.alive);
            if (dead) {
                const int ndead = __popcll(dead);
                const int leader = __ffsll((long long)dead) - 1;
                unsigned long long base = 0;
                if (lane == leader) base = atomicAdd(A.counter, (unsigned long long)ndead);
                base = __shfl(base, leader);
                if (base + ndead >= A.npk) more = false;
                if (!p.alive) {
                    const unsigned long long my = base + __popcll(dead & lt_mask);
                    if (my < A.npk) launch_state(S, A.pid0 + my, p, L);
                }
            }
        }
        if (!__ballot(p.alive)) {
            if (!more) break;
        }
        const bool live = p.alive;
        const int pix = live ? p.iz * H.nx + p.ix : 0;
        float T = 0.f, dw = 0.f;
        const float4 mm = S.med[pix];
        int ev = step(H, p, mm, T, dw);
        ev = live ? ev : EV_NONE;
        dw = live ? dw : 0.f;
        L.absorbed += (double)dw;
        L.segments += live ? 1u : 0u;
        if (live && T != 0.f) {   // direction of the segment, before any scatter
            const double th = atan2((double)p.sx, (double)p.sz);
            const int b = min(n_bins - 1, max(0, (int)floor((th + M_PI) * per_rad)));
            unsafeAtomicAdd(raw + (size_t)b * S.npix + pix, (double)T);
        }
        const bool at = ev == EV_SCATTER;
        const bool killed = scatter_masked(H, p, at, mm.w, L);
        if (ev == EV_ESCAPE) {
            L.escaped += p.w;
            p.alive = false;
        }
        L.visits += (killed || (ev != EV_NONE && !at)) ? 1u : 0u;
    }
    ledger_flush_block(S.led, S.ledc, L);
}

// binned[b][i] = raw[b'][i] * scale, b' = b (forward) or b + n_bins/2 (adjoint:
// the mirrored direction); scale = the run's normalisation / (dx w), w the bin width
__global__ void k_binned_normalise(const ProbDev *pd, int n_bins, double bw, const double *raw, double *out) {
    const int npix = pd->npix;
    const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (i >= (size_t)npix * n_bins) return;
    const int b = (int)(i / npix);
    const size_t px = i - (size_t)b * npix;
    const int src = pd->adjoint ? (b + n_bins / 2) % n_bins : b;
    const double scale = pd->scale / ((double)pd->dx * bw);
    out[i] = raw[(size_t)src * npix + px] * scale;
}

// ------------------------------------------------------------------ trace kernel
// Runs the listed packets one after the other through the same device
// functions as the transport kernels and records every event.
template <int NH>
__global__ void k_trace(const ProbDev *pd, const uint64_t *pids, int n_pids, mc_event *ev, size_t cap,
                        unsigned long long *n_ev) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    constexpr int K = 2 * NH + 1;
    const ProbDev &P = *pd;
    const Hot H = hot_of(P);
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
            const int pix = p.iz * P.nx + p.ix;
            const float4 mm = P.med[pix];
            const int e = step(H, p, mm, T, dw);
            if (e == EV_SCATTER) {
                if (scatter<NH>(H, p, mm.w, h, L)) rec(p, EV_SCATTER, k, ix, iz, p.w, T);
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
// Medium table of the transport: {mua dx, mus dx, 1/(mus dx), g} per pixel,
// one 16-byte load per step (the scatter reads g from the same load).
__global__ void k_setup_medium(int npix, float dx, const float *mua, const float *mus, const float *g,
                               float4 *med) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npix) return;
    const float a = mua[i] * dx, s = mus[i] * dx;
    med[i] = make_float4(a, s, s > 0.f ? 1.f / s : 0.f, g[i]);
}

__global__ void k_fill_zero(uint32_t *p, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

// Single-block inclusive scan of |map| in FP64 (fixed order: each thread a
// contiguous run, then a sequential pass over the 1024 run totals); the
// maximum of |map| is stored after the scan.
__global__ void __launch_bounds__(1024) k_map_cdf(int n, const double *map, double *cdf) {
    __shared__ double part[1024], pmax[1024];
    const int t = threadIdx.x;
    const int per = (n + 1023) / 1024;
    const int a = t * per, b = min(n, a + per);
    double s = 0, mx = 0;
    for (int i = a; i < b; ++i) {
        s += fabs(map[i]);
        mx = fmax(mx, fabs(map[i]));
    }
    part[t] = s;
    pmax[t] = mx;
    __syncthreads();
    if (t == 0) {
        double acc = 0;
        for (int i = 0; i < 1024; ++i) {
            const double v = part[i];
            part[i] = acc;
            acc += v;
            mx = fmax(mx, pmax[i]);
        }
        cdf[n] = mx;   // max |q| after the CDF
    }
    __syncthreads();
    s = part[t];
    for (int i = a; i < b; ++i) {
        s += fabs(map[i]);
        cdf[i] = s;
    }
}

// Completes a problem from the host's part (by value) with what depends on
// device data, and stores it.  The MAP source's measure is 2 pi sum |q| A; an
// all-zero map launches nothing and normalises to zero; a NaN anywhere in
// the map, or a weight bound above 2^32 once the equal-count launch's factor
// max |q| / mean |q| is known, launches nothing and normalises to NaN.
// Fixed-point scale fx = 2^(32 - e) with 2^e above the weight bound, so a
// segment adds at most sqrt 2 * 2^32 in scaled units; a visit is flushed in
// parts at flush_track * 2^32 <= 2^48, inside fixed_add's 2^51.  Every thread
// also fills the problem's entries of the tile-to-problem table.
__global__ void k_prob_setup(ProbDev h, ProbDev *out, uint32_t *tile_prob, uint32_t index) {
    for (int k = threadIdx.x; k < h.ntiles; k += blockDim.x)
        if (tile_prob) tile_prob[h.tile_base + k] = index;
    if (threadIdx.x != 0) return;
    bool usable = true;
    double wb = h.wbound;
    if (h.map) {
        const double sum = h.cdf[h.npix - 1], mx = h.cdf[h.npix];
        h.total = 2.0 * M_PI * sum * (double)h.dx * (double)h.dx;
        h.src[0].cum = h.total;
        h.inv_qbar = sum > 0.0 ? (double)h.npix / sum : 0.0;
        if (h.flags & MC_FLAG_EQUAL_COUNT) wb *= mx * h.inv_qbar;
        if (sum == 0.0) h.todo = 0;                    // a source of no power: the field is zero
        else if (!(sum > 0.0) || !(mx < INFINITY)) usable = false;   // NaN or infinity in the map
    }
    if (!(wb <= 0x1p32)) usable = false;
    int e = 0;
    frexp(fmax(wb, 1.0), &e);   // 2^e > wb
    h.fx = (float)ldexp(1.0, kFixBits - e);
    h.fx_inv = ldexp(1.0, e - kFixBits);
    h.flush_at = (float)ldexp(h.flush_track, kFixBits);
    if (!usable) {
        h.todo = 0;
        h.scale = __builtin_nan("");
    } else {
        h.scale = h.todo ? h.total / (double)h.npk : 0.0;
    }
    *out = h;
}

// Normalise (Sec. 6: divide by the packet count; times the source measure and
// the track-length-to-fluence factor 1/(dx Np) in pixel units) and transpose
// [npix][K] -> [K][npix]; the adjoint output reads the mirrored direction,
// (-1)^n on orders n >= 1.  A job whose fixed-point tile tally may have
// wrapped (ledc[4]) or an overflowed queue turns the whole output into NaN.
__global__ void k_normalise(const ProbDev *pd, int N, const GenCtl *ctl, double *out) {
    const int npix = pd->npix;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npix) return;
    const int K = 2 * N + 1;
    const bool bad = pd->ledc[4] != 0 || (ctl && ctl->overflow);
    const double scale = pd->scale / (double)pd->dx;
    const double *t64 = pd->t64;
    for (int c = 0; c < K; ++c) {
        const int n = c <= N ? c : c - N;
        const double f = (pd->adjoint && (n & 1)) ? -scale : scale;
        out[(size_t)c * npix + i] = bad ? __builtin_nan("") : t64[(size_t)i * K + c] * f;
    }
}

__global__ void k_ledger_out(const ProbDev *pd, const GenCtl *ctl, uint32_t generations, mc_ledger *out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double *led = pd->led;
    const unsigned long long *ledc = pd->ledc;
    out->launched = led[0];
    out->absorbed = led[1];
    out->escaped = led[2];
    out->roulette_gain = led[3];
    out->roulette_loss = led[4];
    out->scale = pd->scale;
    out->packets = ledc[0];
    out->segments = ledc[1];
    out->visits = ledc[2];
    out->scatters = ledc[3];
    out->generations = ctl ? (ctl->done ? ctl->gen_done : generations) : 0;
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
// With hmeas the direct term is that of eps, -A a0 (hmeas - mua a0); with an
// upstream gradient gh = dL/dH instead (hmeas == nullptr) it is gh a0, the
// chain rule through H = mua Phi for any loss L(H).
__global__ void k_gradient(int npix, int N, double area, const float *mua, const float *g, const double *fwd,
                           const double *adj, const double *hmeas, const double *gh, double *dmua, double *dmus) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npix) return;
    const double a0 = fwd[i], a0s = adj[i];
    const double direct = hmeas ? -area * a0 * (hmeas[i] - (double)mua[i] * a0) : gh[i] * a0;
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
    if (dmua) dmua[i] = direct + area * (a0 * a0s * (0.5 * ip) + all * ip);
    if (dmus) dmus[i] = area * (wg * ip);
}

// H = mua a0 (Sec. 2, Grueneisen parameter 1).
__global__ void k_absorbed(int npix, const float *mua, const double *a0, double *h) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < npix) h[i] = (double)mua[i] * a0[i];
}

// Adjoint source for an upstream gradient gh = dL/dH: q* = -mua gh / A per
// unit angle (for L = eps, gh = -A (hmeas - H) and q* = mua (hmeas - H)).
__global__ void k_adjoint_source(int npix, double inv_area, const float *mua, const double *gh, double *qs) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < npix) qs[i] = -(double)mua[i] * gh[i] * inv_area;
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
using GridFn = void (*)(GridArgs);
using TileFn = void (*)(Gen, int);
using TraceFn = void (*)(const ProbDev *, const uint64_t *, int, mc_event *, size_t, unsigned long long *);
using FinishFn = void (*)(Gen, int, int);

template <int NH>
struct Table {
    static void fill(GridFn *grid, TileFn *tile, TraceFn *tr, FinishFn *fin) {
        grid[NH] = k_transport_grid<NH>;
        tile[NH] = k_transport_tile<NH>;
        tr[NH] = k_trace<NH>;
        fin[NH] = k_finish<NH>;
        if constexpr (NH > 0) Table<NH - 1>::fill(grid, tile, tr, fin);
    }
};

// Kernel entry points by harmonic order (filled once; never changed after).
struct Kernels {
    GridFn grid[MC_NHARM_MAX + 1];
    TileFn tile[MC_NHARM_MAX + 1];
    TraceFn tr[MC_NHARM_MAX + 1];
    FinishFn fin[MC_NHARM_MAX + 1];
    Kernels() { Table<MC_NHARM_MAX>::fill(grid, tile, tr, fin); }
};

const Kernels &kernels() {
    static const Kernels k;
    return k;
}

// ------------------------------------------------------------------ host helpers
size_t align_up(size_t v) { return (v + 255) & ~size_t(255); }

// Defaults of the tiled transport.  Live packets per generation: on the
// 1e8-packet disc256 gradient 2^25 against 2^24: -1.8% time, 2^26 against
// 2^25: -1.1%.  The finisher threshold, the quiet rule, its tail and the
// smallest job were set together on the 2.83e6-packet disc256 gradient
// (2^16 / 50% / 4 / 512: 206 ms against 234 ms for 2^17 / 100% / 8 / no
// split), which also shortened the 1e8-packet one by 3%.  Once the sort no
// longer serialised on its cursors, generations got cheap enough for a
// shorter tail and larger jobs: tail 1, jobs of 8192, smallest job 1024 run
// forward + adjoint at 2.83e6 packets in 195 ms against 205 ms, and at 1e8
// in 2382 ms against 2484 ms (results bitwise the same).  With one
// 1024-thread workgroup per CU and 23x23 tiles, jobs of 16384: 174 ms and
// 2289 ms.
constexpr uint64_t kLiveMax = 1ull << 26;
constexpr uint64_t kFinishMax = 1ull << 16;   // default finisher threshold: min(this, live / 128)
constexpr uint64_t kGridMaxPackets = 1ull << 21;   // larger runs take the tiled transport
constexpr uint32_t kJobSize = 16384;          // packets per job
constexpr uint64_t kSmallPool = 1ull << 23;   // pools below this many live packets use half-size jobs
constexpr uint32_t kMaxVisitsPerStay = 64;    // a packet pauses after this many visits in one job
// once a job has turned quiet, its packets pause after this many more visits,
// so a wave does not idle behind its longest stay
constexpr uint32_t kTailVisits = 1;
// generations enqueued per call unless the caller says: a base, a share per
// tile along the longest grid side (a packet's life in generations grows with
// the grid measured in tiles) and a share per pool turnover.  Measured with
// 23x23 tiles at 1e8 packets: 36 generations on the 32^2 pencil beam, 130 /
// 189 / 290 / 491 on 128^2 / 192^2 / 256^2 / 512^2 disc phantoms over the
// same 25.6 mm, up to 1.4x that at half the absorption; 434 for the 256^2
// adjoint at 4e8.  A generation that finds the run finished costs ~6 us; one
// too few leaves its packets to the slower finisher.
constexpr uint32_t kGenBase = 100, kGenPerTile = 30, kGenPerPool = 48;
constexpr int kTileWavesMax = 256 * 16;       // bound on resident waves of the tiled kernel
constexpr int kTileSlotsMax = kTileWavesMax / (tile_block(MC_NHARM_MAX) / 64);   // and on its workgroups
constexpr uint32_t kJobMin = 1024;             // smallest job of a generation with few packets (see gen_scan)
constexpr uint32_t kQuietPercent = 50;         // see the quiet rule of k_transport_tile

// The tuning a call runs with: the caller's fields, defaults where zero.
struct TileTuning {
    uint64_t live = kLiveMax;
    uint32_t job = kJobSize, maxvis = kMaxVisitsPerStay, tailvis = kTailVisits;
    uint64_t finish = 0;   // 0: min(2^17, live / 128)
    int tile = 0;          // 0: largest square tile whose tally fits one workgroup's LDS
    uint64_t grid_max = kGridMaxPackets;
    double flush_track = kFlushTrackMax;
    uint32_t max_gen = 0;      // 0: kGenBase + kGenPerPool per pool of live packets the run holds
    uint32_t job_min = kJobMin;
    uint32_t quiet = kQuietPercent;
    uint32_t slice = kSlice;   // not a caller knob: the no-alloc entry point narrows it to save scratch
};

bool tuning_from(const mc_options *o, TileTuning &v) {
    v = TileTuning();
    if (!o || !o->tuning) return true;
    const mc_tuning &t = *o->tuning;
    if (t.live_packets && (t.live_packets < 1024 || t.live_packets > kLiveMax)) return false;
    if (t.job_packets && (t.job_packets < 64 || t.job_packets > (1u << 20))) return false;
    if (t.tile > 256 || t.finish_packets > kLiveMax || t.tail_visits > (1u << 30) || t.max_generations > 65536)
        return false;
    if ((t.min_job_packets && (t.min_job_packets < 64 || t.min_job_packets > (1u << 20))) || t.quiet_percent > 100 ||
        t.reserved)
        return false;
    if (!(t.flush_track >= 0.f && t.flush_track <= (float)kFlushTrackMax)) return false;
    if (t.live_packets) v.live = t.live_packets;
    if (t.job_packets) v.job = t.job_packets;
    if (t.max_visits) v.maxvis = t.max_visits;
    if (t.tile) v.tile = (int)t.tile;
    if (t.finish_packets) v.finish = t.finish_packets;
    if (t.grid_max_packets) v.grid_max = t.grid_max_packets;
    if (t.flush_track > 0.f) v.flush_track = (double)t.flush_track;
    if (t.tail_visits) v.tailvis = t.tail_visits;
    if (t.max_generations) v.max_gen = t.max_generations;
    if (t.min_job_packets) v.job_min = t.min_job_packets;
    if (t.quiet_percent) v.quiet = t.quiet_percent;
    return true;
}

}  // namespace

// Caller-owned timer of transport launches (see mc_timer_create).
struct mc_timer {
    std::mutex mu;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
    double ms = 0;
    uint64_t launches = 0;
};

namespace {

// Records HIP events around a transport launch when the call has a timer.
struct LaunchTimer {
    mc_timer *tm;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    explicit LaunchTimer(mc_timer *t) : tm(t) {}
    mc_status begin(hipStream_t s) {
        if (!tm) return MC_OK;
        if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return MC_ERR_DEVICE;
        return hipEventRecord(e0, s) == hipSuccess ? MC_OK : MC_ERR_DEVICE;
    }
    mc_status end(hipStream_t s) {
        if (!tm) return MC_OK;
        if (hipEventRecord(e1, s) != hipSuccess) return MC_ERR_DEVICE;
        std::lock_guard<std::mutex> g(tm->mu);
        tm->pending.emplace_back(e0, e1);
        return MC_OK;
    }
};

// tile LDS: fixed-point sums [tw*th][K], medium [tw*th], flush counts [tw*th]
size_t tile_lds_bytes(int tw, int th, int K) {
    const size_t tal = ((size_t)tw * th * K * sizeof(double) + 15) & ~size_t(15);
    return tal + (size_t)tw * th * (sizeof(float4) + sizeof(uint32_t));
}

// Tiled transport unless the whole tally (8 bytes per value) fits one
// workgroup's LDS and the run is small (the tiled mode's per-generation
// overhead is ~10 ms; measured on a 32x32 pencil beam, the tiled mode
// overtakes the whole-grid kernel near 2e6 packets and is 5x faster at 1e8).
bool is_tiled(const mc_medium *m, const mc_run *run, const TileTuning &tt) {
    if ((size_t)m->nx * m->nz * (2 * run->n_harm + 1) * sizeof(double) > kLdsGridMax) return true;
    return run->n_packets > tt.grid_max;
}

// Whole-grid mode workspace: problem, medium, CDF, tally, ledger, per-chunk counters.
struct Layout {
    size_t pd, med, cdf, t64, led, ledc, counters, total;
    uint64_t n_chunks;
};

Layout layout(const mc_medium *m, const mc_source *src, const mc_run *run) {
    Layout L{};
    const size_t npix = (size_t)m->nx * m->nz;
    const int K = 2 * run->n_harm + 1;
    size_t off = 0;
    L.pd = off;
    off = align_up(off + sizeof(ProbDev));
    L.med = off;
    off = align_up(off + npix * sizeof(float4));
    L.cdf = off;
    if (src[0].kind == MC_SRC_MAP) off = align_up(off + (npix + 1) * sizeof(double));   // CDF, max |q|
    L.t64 = off;
    off = align_up(off + npix * K * sizeof(double));
    L.led = off;
    off = align_up(off + 8 * sizeof(double));
    L.ledc = off;
    off = align_up(off + 8 * sizeof(unsigned long long));
    L.n_chunks = (run->n_packets + kChunk - 1) / kChunk;
    L.counters = off;
    off = align_up(off + L.n_chunks * sizeof(unsigned long long));
    L.total = off;
    return L;
}

// One problem of a batch, as the caller gave it.
struct BatchProblem {
    const mc_medium *m;
    const mc_source *src;
    int n_src;
    const mc_run *run;
    int adjoint;
    double *coeffs;
    mc_ledger *ledger;
};

// Tiled mode for a batch of problems sharing the harmonic order: per-problem
// descriptor, medium, CDF, tally and ledger; one packet pool (two alternating
// record pools), one set of counters and one global tile index space (problem
// p owns tiles tile_base[p] ..).
struct BatchLayout {
    TileTuning tt;
    int N = 0, K = 0, t = 0, ntiles = 0;
    size_t tile_lds = 0;
    uint64_t live = 0, cap_c = 0, cap_l = 0, max_jobs = 0, total_packets = 0;
    uint32_t job = 0;   // packets per job: the tuning's, halved for small pools
    std::vector<size_t> med, cdf, t64, led, ledc;
    std::vector<int> ntx, ntz, tile_base;
    size_t probs = 0, tile_prob = 0, ctl = 0, launched = 0, fin_cur = 0, tcount = 0, tcursor = 0, jobs = 0,
           sidx = 0, pool[2] = {0, 0}, ptile[2] = {0, 0}, total = 0;
};

BatchLayout batch_layout(const BatchProblem *pb, int n, const TileTuning &tt) {
    BatchLayout B;
    B.tt = tt;
    B.N = pb[0].run->n_harm;
    B.K = 2 * B.N + 1;
    int t = 1;
    while (tile_lds_bytes(t + 1, t + 1, B.K) <= kLdsTileMax) ++t;
    if (B.tt.tile && tile_lds_bytes(B.tt.tile, B.tt.tile, B.K) <= kLdsTileMax) t = B.tt.tile;
    int maxn = 1;
    for (int i = 0; i < n; ++i) maxn = std::max({maxn, pb[i].m->nx, pb[i].m->nz});
    B.t = std::min(t, maxn);
    B.tile_lds = tile_lds_bytes(B.t, B.t, B.K);
    size_t off = 0;
    for (int i = 0; i < n; ++i) {
        const size_t npix = (size_t)pb[i].m->nx * pb[i].m->nz;
        B.med.push_back(off);
        off = align_up(off + npix * sizeof(float4));
        B.cdf.push_back(off);
        if (pb[i].src[0].kind == MC_SRC_MAP) off = align_up(off + (npix + 1) * sizeof(double));   // CDF, max |q|
        B.t64.push_back(off);
        off = align_up(off + npix * B.K * sizeof(double));
        B.led.push_back(off);
        off = align_up(off + 8 * sizeof(double));
        B.ledc.push_back(off);
        off = align_up(off + 8 * sizeof(unsigned long long));
        B.ntx.push_back((pb[i].m->nx + B.t - 1) / B.t);
        B.ntz.push_back((pb[i].m->nz + B.t - 1) / B.t);
        B.tile_base.push_back(B.ntiles);
        B.ntiles += B.ntx.back() * B.ntz.back();
        B.total_packets += pb[i].run->n_packets;
    }
    B.live = std::min<uint64_t>(B.total_packets, B.tt.live);
    // carried region: every packet a generation moves may leave, plus the
    // padding of the wave slices still open when it ends; launch region: at
    // most `live` new packets per generation
    B.cap_c = B.live + (uint64_t)B.tt.slice * kTileWavesMax + 64ull * 64;
    B.cap_l = B.live;
    // a pool below 2^23 live packets spreads over too few jobs of the tuned
    // size to fill the device: half-size jobs (measured on 1e6- and 4e6-packet
    // disc256 gradients: -7%; 4096 stays better for full pools)
    B.job = (B.live < kSmallPool && B.tt.job >= 128) ? B.tt.job / 2 : B.tt.job;
    // jobs of one generation: one per tile plus one per job_size records, or
    // (when job sizes shrink to fill the workgroups) at most two per workgroup
    B.max_jobs = (uint64_t)B.ntiles + std::max<uint64_t>(B.live / B.job, 2ull * kTileSlotsMax) + 2;
    if (!B.tt.max_gen) {
        uint64_t side = 0;   // the longest grid side of any problem, in tiles
        for (int i = 0; i < n; ++i) side = std::max<uint64_t>(side, std::max(B.ntx[i], B.ntz[i]));
        B.tt.max_gen = (uint32_t)std::min<uint64_t>(
            65536, kGenBase + kGenPerTile * side + kGenPerPool * ((B.total_packets + B.live - 1) / B.live));
    }
    B.probs = off;
    off = align_up(off + (size_t)n * sizeof(ProbDev));
    B.tile_prob = off;
    off = align_up(off + (size_t)B.ntiles * sizeof(uint32_t));
    // everything from ctl to the end of the cursors is zeroed at set-up
    B.ctl = off;
    off = align_up(off + sizeof(GenCtl));
    B.launched = off;
    off = align_up(off + (size_t)n * sizeof(uint64_t));
    B.fin_cur = off;
    off = align_up(off + (size_t)(n + 1) * sizeof(unsigned long long));
    B.tcount = off;
    off = align_up(off + (size_t)B.ntiles * sizeof(uint32_t));
    B.tcursor = off;
    off = align_up(off + (size_t)B.ntiles * kCursorStride * sizeof(uint32_t));
    B.jobs = off;
    off = align_up(off + B.max_jobs * sizeof(uint4));
    B.sidx = off;
    off = align_up(off + B.live * sizeof(uint32_t));
    for (int p = 0; p < 2; ++p) {
        B.pool[p] = off;
        off = align_up(off + (B.cap_c + B.cap_l) * sizeof(PacketRec));
        B.ptile[p] = off;
        off = align_up(off + (B.cap_c + B.cap_l) * sizeof(uint32_t));
    }
    B.total = off;
    return B;
}

// Bound on |packet weight|: a launch weight 2 pi p(s) of an angular profile
// p = c0/2pi + (1/pi) sum (c_n cos nt + s_n sin nt) is at most
// |c0| + 2 sum (|c_n| + |s_n|) (1 without a profile, and for pencils and
// lines); a roulette survivor gains at most the factor m W_th.  The
// equal-count map launch multiplies by q_i / mean |q|, bounded on the device
// once max |q| is known (k_prob_setup).
double weight_bound(const mc_source *src, int n_src, const mc_run *run) {
    double wb = 0.0;
    for (int s = 0; s < n_src; ++s) {
        const mc_source &q = src[s];
        double w = 1.0;
        if ((q.kind == MC_SRC_POINT || q.kind == MC_SRC_MAP) && q.prof_h) {
            w = std::fabs(q.prof_h[0]);
            for (int k = 1; k <= 2 * q.n_prof; ++k) w += 2.0 * std::fabs(q.prof_h[k]);
        }
        wb = std::max(wb, w);
    }
    return wb * std::max(1.0, (double)run->roulette_m * (double)run->w_threshold);
}

mc_status validate(const mc_medium *m, const mc_source *src, int n_src, const mc_run *run) {
    if (!m || !src || !run) return MC_ERR_INVALID_ARG;
    if (m->nx <= 0 || m->nz <= 0 || !(m->dx > 0.f) || !m->mua_d || !m->mus_d || !m->g_d) return MC_ERR_INVALID_ARG;
    if ((int64_t)m->nx * m->nz > (1 << 26)) return MC_ERR_UNSUPPORTED;
    if (run->n_harm < 0 || run->n_harm > MC_NHARM_MAX || run->n_packets == 0) return MC_ERR_INVALID_ARG;
    if (!(run->roulette_m > 1.f) || !(run->w_threshold >= 0.f)) return MC_ERR_INVALID_ARG;
    if (run->flags & ~(MC_FLAG_LITERAL_TRUNCATION | MC_FLAG_EQUAL_COUNT)) return MC_ERR_INVALID_ARG;
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
    // the fixed-point tallies resolve weights up to 2^32 (see fixed_add)
    if (!(weight_bound(src, n_src, run) <= 0x1p32)) return MC_ERR_UNSUPPORTED;
    return MC_OK;
}

// The host's part of a problem descriptor (k_prob_setup adds the rest).
void fill_problem(ProbDev &P, const mc_medium *m, const mc_source *src, int n_src, const mc_run *run, int adjoint,
                  double flush_track) {
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
    P.pid0 = run->first_packet_id;
    P.npk = run->n_packets;
    P.todo = run->n_packets;
    P.wth = run->w_threshold;
    P.rm = run->roulette_m;
    P.inv_rm = 1.f / run->roulette_m;
    P.wbound = weight_bound(src, n_src, run);
    P.flush_track = flush_track;
    double total = 0;
    int poff = 0;
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
        if (q.kind != MC_SRC_MAP) total += q.power;   // a MAP source's measure is set on the device
        d.cum = total;
    }
    P.total = total;
    if (n_src == 1 && src[0].kind == MC_SRC_MAP) P.map = src[0].map_d;
}

int occupancy_blocks(const void *fn, int block, size_t lds) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, block, lds) != hipSuccess || nb < 1) nb = 1;
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

mc_status set_lds_limit(const void *fn, size_t lds) {
    if (lds <= 64 * 1024) return MC_OK;
    return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) == hipSuccess ? MC_OK
                                                                                                    : MC_ERR_DEVICE;
}

// Medium table, CDF of a MAP source, then the problem descriptor.
mc_status setup_problem(const ProbDev &host, ProbDev *pd_d, uint32_t *tile_prob, uint32_t index, const float *mua,
                        const float *mus, const float *g, hipStream_t s) {
    hipLaunchKernelGGL(k_setup_medium, dim3((host.npix + 255) / 256), dim3(256), 0, s, host.npix, host.dx, mua, mus, g,
                       const_cast<float4 *>(host.med));
    if (host.map)
        hipLaunchKernelGGL(k_map_cdf, dim3(1), dim3(1024), 0, s, host.npix, host.map, const_cast<double *>(host.cdf));
    hipLaunchKernelGGL(k_prob_setup, dim3(1), dim3(256), 0, s, host, pd_d, tile_prob, index);
    return hipGetLastError() == hipSuccess ? MC_OK : MC_ERR_DEVICE;
}

// Whole-grid mode: persistent launches over chunks of packets.
mc_status run_grid(const ProbDev *pd, const Layout &L, const mc_run *run, mc_timer *timer, char *base,
                   size_t lds, hipStream_t s) {
    const int N = run->n_harm;
    const GridFn fn = kernels().grid[N];
    mc_status st = set_lds_limit(reinterpret_cast<const void *>(fn), lds);
    if (st != MC_OK) return st;
    const int block = grid_block(N);
    const int occ = occupancy_blocks(reinterpret_cast<const void *>(fn), block, lds);
    const int cus = device_cus();
    for (uint64_t c = 0; c < L.n_chunks; ++c) {
        const uint64_t a = c * kChunk;
        const uint64_t n = std::min<uint64_t>(kChunk, run->n_packets - a);
        GridArgs A{pd, run->first_packet_id + a, n, reinterpret_cast<unsigned long long *>(base + L.counters) + c};
        const uint64_t want = (n + block - 1) / block;
        const unsigned grid = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(want, (uint64_t)cus * occ));
        LaunchTimer tm(timer);
        if ((st = tm.begin(s)) != MC_OK) return st;
        hipLaunchKernelGGL(fn, dim3(grid), dim3(block), lds, s, A);
        if ((st = tm.end(s)) != MC_OK) return st;
        if (hipGetLastError() != hipSuccess) return MC_ERR_DEVICE;
    }
    return MC_OK;
}

// Tiled mode: every problem of the batch in one packet pool.  The host
// enqueues the set-up, max_generations generations (each: launch and count,
// sort, transport -- steered by the device control block, see GenCtl), the
// finisher, and the normalisation, and returns without waiting.
mc_status run_batch(const BatchProblem *pb, int n, const TileTuning &tt, mc_timer *timer, void *ws, size_t ws_bytes,
                    hipStream_t s) {
    for (int i = 0; i < n; ++i) {
        mc_status st = validate(pb[i].m, pb[i].src, pb[i].n_src, pb[i].run);
        if (st != MC_OK) return st;
        if (!pb[i].coeffs || pb[i].run->n_harm != pb[0].run->n_harm) return MC_ERR_INVALID_ARG;
    }
    const BatchLayout B = batch_layout(pb, n, tt);
    if (!ws || ws_bytes < B.total || (reinterpret_cast<uintptr_t>(ws) & 255)) return MC_ERR_WORKSPACE;
    if (B.tile_lds > kLdsTileMax || B.cap_c + B.cap_l > 0xFFFFFFF0ull) return MC_ERR_UNSUPPORTED;
    char *base = static_cast<char *>(ws);
    const int N = B.N;
    mc_status st;
    ProbDev *probs_d = reinterpret_cast<ProbDev *>(base + B.probs);
    uint32_t *tile_prob = reinterpret_cast<uint32_t *>(base + B.tile_prob);
    GenCtl *ctl = reinterpret_cast<GenCtl *>(base + B.ctl);
    // counters, cursors and tile counts start at zero; the control block knows the total to launch
    if ((st = launch_zero(base + B.ctl, B.tcursor - B.ctl, s)) != MC_OK) return st;
    for (int i = 0; i < n; ++i) {
        const mc_medium *m = pb[i].m;
        const int npix = m->nx * m->nz;
        if ((st = launch_zero(base + B.t64[i], (size_t)npix * B.K * sizeof(double), s)) != MC_OK) return st;
        if ((st = launch_zero(base + B.led[i], B.ledc[i] + 8 * sizeof(unsigned long long) - B.led[i], s)) != MC_OK)
            return st;
        ProbDev P;
        fill_problem(P, m, pb[i].src, pb[i].n_src, pb[i].run, pb[i].adjoint, tt.flush_track);
        P.ntx = B.ntx[i];
        P.tile_base = B.tile_base[i];
        P.ntiles = B.ntx[i] * B.ntz[i];
        P.med = reinterpret_cast<const float4 *>(base + B.med[i]);
        P.cdf = reinterpret_cast<const double *>(base + B.cdf[i]);
        P.t64 = reinterpret_cast<double *>(base + B.t64[i]);
        P.led = reinterpret_cast<double *>(base + B.led[i]);
        P.ledc = reinterpret_cast<unsigned long long *>(base + B.ledc[i]);
        if ((st = setup_problem(P, probs_d + i, tile_prob, (uint32_t)i, m->mua_d, m->mus_d, m->g_d, s)) != MC_OK)
            return st;
    }
    // total packets to launch (problems whose map has no power launch none:
    // the control block learns this from the descriptors on the device)
    Gen G{};
    G.tw = G.th = B.t;
    G.ntiles = B.ntiles;
    G.nprob = n;
    G.live = (uint32_t)B.live;
    G.cap_c = (uint32_t)B.cap_c;
    G.cap_l = (uint32_t)B.cap_l;
    G.job_size = B.job;
    G.job_min = std::min(B.tt.job_min, B.job);
    G.quiet_pct = B.tt.quiet;
    G.max_visits = B.tt.maxvis;
    G.tail_visits = B.tt.tailvis;
    G.finish_at = (uint32_t)(B.tt.finish ? B.tt.finish : std::min<uint64_t>(kFinishMax, B.tt.live / 128));
    G.slice = B.tt.slice;
    G.probs = probs_d;
    G.tile_prob = tile_prob;
    for (int p = 0; p < 2; ++p) {
        G.pool[p] = reinterpret_cast<PacketRec *>(base + B.pool[p]);
        G.ptile[p] = reinterpret_cast<uint32_t *>(base + B.ptile[p]);
    }
    G.sidx = reinterpret_cast<uint32_t *>(base + B.sidx);
    G.tile_count = reinterpret_cast<uint32_t *>(base + B.tcount);
    G.tile_cursor = reinterpret_cast<uint32_t *>(base + B.tcursor);
    G.jobs = reinterpret_cast<uint4 *>(base + B.jobs);
    G.max_jobs = (uint32_t)B.max_jobs;
    G.ctl = ctl;
    G.launched = reinterpret_cast<uint64_t *>(base + B.launched);
    G.fin_cur = reinterpret_cast<unsigned long long *>(base + B.fin_cur);
    hipLaunchKernelGGL(k_ctl_init, dim3(1), dim3(1), 0, s, G);

    const TileFn fn = kernels().tile[N];
    if ((st = set_lds_limit(reinterpret_cast<const void *>(fn), B.tile_lds)) != MC_OK) return st;
    const int occ = occupancy_blocks(reinterpret_cast<const void *>(fn), tile_block(N), B.tile_lds);
    const int cus = device_cus();
    const unsigned tgrid = (unsigned)std::max(1, std::min(cus * occ, kTileSlotsMax));
    G.slots = tgrid;
    const unsigned cgrid = (unsigned)std::max(1, cus);
    const unsigned sgrid = (unsigned)std::max(1, 4 * cus);
    // the generation kernels' tile histograms (and the scan's buffer) in dynamic LDS
    const bool local_hist = B.ntiles <= kHistTiles;
    const size_t count_lds = sizeof(uint32_t) * std::max<size_t>(local_hist ? B.ntiles : 0, 2 * kGenBlock);
    const size_t scatter_lds = local_hist ? sizeof(uint32_t) * B.ntiles : 0;
    if ((st = set_lds_limit(reinterpret_cast<const void *>(k_gen_count), count_lds)) != MC_OK) return st;
    if ((st = set_lds_limit(reinterpret_cast<const void *>(k_gen_scatter), scatter_lds)) != MC_OK) return st;
    for (uint32_t g = 0; g < B.tt.max_gen; ++g) {
        hipLaunchKernelGGL(k_gen_count, dim3(cgrid), dim3(kGenBlock), count_lds, s, G, (int)g);
        hipLaunchKernelGGL(k_gen_scatter, dim3(sgrid), dim3(256), scatter_lds, s, G, (int)g);
        LaunchTimer tm(timer);
        if ((st = tm.begin(s)) != MC_OK) return st;
        hipLaunchKernelGGL(fn, dim3(tgrid), dim3(tile_block(N)), B.tile_lds, s, G, (int)g);
        if ((st = tm.end(s)) != MC_OK) return st;
        if (hipGetLastError() != hipSuccess) return MC_ERR_DEVICE;
    }
    // the finisher: the records left, then any packets the generations did not launch
    const FinishFn ff = kernels().fin[N];
    const size_t flds = (size_t)kBlockFinish * (2 * N + 1) * sizeof(float) +
                        (size_t)kBlockFinish * (sizeof(unsigned long long) + sizeof(double));
    if ((st = set_lds_limit(reinterpret_cast<const void *>(ff), flds)) != MC_OK) return st;
    const int focc = occupancy_blocks(reinterpret_cast<const void *>(ff), kBlockFinish, flds);
    const unsigned fgrid = (unsigned)std::max<uint64_t>(
        1, std::min<uint64_t>((G.finish_at + kBlockFinish - 1) / kBlockFinish + 1, (uint64_t)cus * focc));
    {
        LaunchTimer tf(timer);
        if ((st = tf.begin(s)) != MC_OK) return st;
        hipLaunchKernelGGL(ff, dim3(fgrid), dim3(kBlockFinish), flds, s, G, (int)B.tt.max_gen, -1);
        if ((st = tf.end(s)) != MC_OK) return st;
    }
    const unsigned fgrid_all = (unsigned)std::max(1, cus * focc);
    for (int i = 0; i < n; ++i)
        hipLaunchKernelGGL(ff, dim3(fgrid_all), dim3(kBlockFinish), flds, s, G, (int)B.tt.max_gen, i);
    // normalisation and ledgers
    for (int i = 0; i < n; ++i) {
        const int npix = pb[i].m->nx * pb[i].m->nz;
        hipLaunchKernelGGL(k_normalise, dim3((npix + 255) / 256), dim3(256), 0, s, probs_d + i, N,
                           (const GenCtl *)ctl, pb[i].coeffs);
        if (pb[i].ledger)
            hipLaunchKernelGGL(k_ledger_out, dim3(1), dim3(1), 0, s, (const ProbDev *)(probs_d + i), (const GenCtl *)ctl,
                               B.tt.max_gen, pb[i].ledger);
    }
    return hipGetLastError() == hipSuccess ? MC_OK : MC_ERR_DEVICE;
}

mc_status run_mc(const mc_medium *m, const mc_source *src, int n_src, const mc_run *run, const TileTuning &tt,
                 mc_timer *timer, double *coeffs, mc_ledger *ledger, void *ws, size_t ws_bytes, hipStream_t s,
                 int adjoint) {
    mc_status st = validate(m, src, n_src, run);
    if (st != MC_OK) return st;
    if (!coeffs) return MC_ERR_INVALID_ARG;
    if (is_tiled(m, run, tt)) {
        const BatchProblem one{m, src, n_src, run, adjoint, coeffs, ledger};
        return run_batch(&one, 1, tt, timer, ws, ws_bytes, s);
    }
    const Layout L = layout(m, src, run);
    if (!ws || ws_bytes < L.total || (reinterpret_cast<uintptr_t>(ws) & 255)) return MC_ERR_WORKSPACE;
    char *base = static_cast<char *>(ws);
    const int npix = m->nx * m->nz;
    const int N = run->n_harm;
    // zero the tally, ledger and chunk counters
    if ((st = launch_zero(base + L.t64, L.counters + L.n_chunks * sizeof(unsigned long long) - L.t64, s)) != MC_OK)
        return st;
    ProbDev P;
    fill_problem(P, m, src, n_src, run, adjoint, tt.flush_track);
    P.med = reinterpret_cast<const float4 *>(base + L.med);
    P.cdf = reinterpret_cast<const double *>(base + L.cdf);
    P.t64 = reinterpret_cast<double *>(base + L.t64);
    P.led = reinterpret_cast<double *>(base + L.led);
    P.ledc = reinterpret_cast<unsigned long long *>(base + L.ledc);
    ProbDev *pd = reinterpret_cast<ProbDev *>(base + L.pd);
    if ((st = setup_problem(P, pd, nullptr, 0, m->mua_d, m->mus_d, m->g_d, s)) != MC_OK) return st;
    const size_t lds = (size_t)npix * (2 * N + 1) * sizeof(double);
    if ((st = run_grid(pd, L, run, timer, base, lds, s)) != MC_OK) return st;
    hipLaunchKernelGGL(k_normalise, dim3((npix + 255) / 256), dim3(256), 0, s, (const ProbDev *)pd, N,
                       (const GenCtl *)nullptr, coeffs);
    if (ledger)
        hipLaunchKernelGGL(k_ledger_out, dim3(1), dim3(1), 0, s, (const ProbDev *)pd, (const GenCtl *)nullptr, 0u, ledger);
    return hipGetLastError() == hipSuccess ? MC_OK : MC_ERR_DEVICE;
}

// Discrete-ordinates runs (mc_run_binned): problem, medium, CDF of a map
// source, raw bins [n_bins][npix], ledger and per-chunk packet counters.
struct BinnedLayout {
    size_t pd, med, cdf, raw, led, ledc, counters, total;
    uint64_t n_chunks;
};

BinnedLayout binned_layout(const mc_medium *m, const mc_source *src, const mc_run *run, int n_bins) {
    BinnedLayout L{};
    const size_t npix = (size_t)m->nx * m->nz;
    size_t off = 0;
    L.pd = off;
    off = align_up(off + sizeof(ProbDev));
    L.med = off;
    off = align_up(off + npix * sizeof(float4));
    L.cdf = off;
    if (src[0].kind == MC_SRC_MAP) off = align_up(off + (npix + 1) * sizeof(double));
    L.raw = off;
    off = align_up(off + npix * (size_t)n_bins * sizeof(double));
    L.led = off;
    off = align_up(off + 8 * sizeof(double));
    L.ledc = off;
    off = align_up(off + 8 * sizeof(unsigned long long));
    L.n_chunks = (run->n_packets + kChunk - 1) / kChunk;
    L.counters = off;
    off = align_up(off + L.n_chunks * sizeof(unsigned long long));
    L.total = off;
    return L;
}

bool binned_args_ok(int n_bins) { return n_bins >= 2 && n_bins <= kBinnedMax && !(n_bins & 1); }

mc_status run_binned(const mc_medium *m, const mc_source *src, int n_src, const mc_run *run, int adjoint, int n_bins,
                     double *out, mc_ledger *ledger, void *ws, size_t ws_bytes, hipStream_t s) {
    mc_status st = validate(m, src, n_src, run);
    if (st != MC_OK) return st;
    if (!out || !binned_args_ok(n_bins) || (adjoint != 0 && adjoint != 1)) return MC_ERR_INVALID_ARG;
    const BinnedLayout L = binned_layout(m, src, run, n_bins);
    if (!ws || ws_bytes < L.total || (reinterpret_cast<uintptr_t>(ws) & 255)) return MC_ERR_WORKSPACE;
    char *base = static_cast<char *>(ws);
    const int npix = m->nx * m->nz;
    const size_t nout = (size_t)npix * n_bins;
    if ((st = launch_zero(base + L.raw, L.total - L.raw, s)) != MC_OK) return st;   // bins, ledger, counters
    ProbDev P;
    fill_problem(P, m, src, n_src, run, adjoint, kFlushTrackMax);
    P.med = reinterpret_cast<const float4 *>(base + L.med);
    P.cdf = reinterpret_cast<const double *>(base + L.cdf);
    P.led = reinterpret_cast<double *>(base + L.led);
    P.ledc = reinterpret_cast<unsigned long long *>(base + L.ledc);
    ProbDev *pd = reinterpret_cast<ProbDev *>(base + L.pd);
    if ((st = setup_problem(P, pd, nullptr, 0, m->mua_d, m->mus_d, m->g_d, s)) != MC_OK) return st;
    double *raw = reinterpret_cast<double *>(base + L.raw);
    const int cus = device_cus();
    const int occ = occupancy_blocks(reinterpret_cast<const void *>(&k_transport_binned), 256, 0);
    for (uint64_t c = 0; c < L.n_chunks; ++c) {
        const uint64_t a = c * kChunk;
        const uint64_t n = std::min<uint64_t>(kChunk, run->n_packets - a);
        GridArgs A{pd, run->first_packet_id + a, n, reinterpret_cast<unsigned long long *>(base + L.counters) + c};
        const unsigned grid = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>((n + 255) / 256, (uint64_t)cus * occ));
        hipLaunchKernelGGL(k_transport_binned, dim3(grid), dim3(256), 0, s, A, n_bins, raw);
        if (hipGetLastError() != hipSuccess) return MC_ERR_DEVICE;
    }
    hipLaunchKernelGGL(k_binned_normalise, dim3((unsigned)((nout + 255) / 256)), dim3(256), 0, s, (const ProbDev *)pd,
                       n_bins, 2.0 * M_PI / n_bins, (const double *)raw, out);
    if (ledger)
        hipLaunchKernelGGL(k_ledger_out, dim3(1), dim3(1), 0, s, (const ProbDev *)pd, (const GenCtl *)nullptr, 0u, ledger);
    return hipGetLastError() == hipSuccess ? MC_OK : MC_ERR_DEVICE;
}

// ------------------------------------------------------------------ no-alloc runs
// mc_run_noalloc takes its workspace from this file-scope device array (each
// GPU the library runs on holds its own copy until the process ends).  In
// host code its name is only a stand-in: its device address comes from
// hipGetSymbolAddress, taken once per device and kept in scratch_table.
constexpr size_t kScratchBytes = MC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
constexpr uint32_t kScratchSlice = 64;   // narrower queue slices: less padding held in the scratch

struct ScratchTable {
    std::mutex mu;
    void *ptr[kMaxDevices] = {};
};
ScratchTable &scratch_table() {
    static ScratchTable t;
    return t;
}

// The device address of the current device's scratch (nullptr on failure).
void *scratch_ptr() {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    ScratchTable &t = scratch_table();
    std::lock_guard<std::mutex> g(t.mu);
    if (!t.ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
        t.ptr[dev] = p;
    }
    return t.ptr[dev];
}

// The tuning of a no-alloc run: the caller's, with narrow slices, and -- unless
// the caller fixed live_packets -- the largest pool whose workspace fits the
// scratch.  Returns false if the run does not fit (host arithmetic only).
bool noalloc_tuning(const mc_medium *m, const mc_source *src, int n_src, const mc_run *run, int adjoint,
                    const mc_options *opts, TileTuning &tt) {
    tt.slice = kScratchSlice;
    if (!is_tiled(m, run, tt)) return layout(m, src, run).total <= kScratchBytes;
    const BatchProblem one{m, src, n_src, run, adjoint, nullptr, nullptr};
    auto fits = [&](uint64_t live) {
        TileTuning t = tt;
        t.live = live;
        return batch_layout(&one, 1, t).total <= kScratchBytes;
    };
    if (opts && opts->tuning && opts->tuning->live_packets) return fits(tt.live);
    if (!fits(1024)) return false;
    uint64_t lo = 1024, hi = tt.live;   // largest live in [1024, tt.live] that fits
    while (lo < hi) {
        const uint64_t mid = lo + (hi - lo + 1) / 2;
        if (fits(mid)) lo = mid; else hi = mid - 1;
    }
    tt.live = lo;
    return true;
}

}  // namespace

extern "C" {

size_t mc_binned_workspace_bytes(const mc_medium *medium, const mc_source *src, int n_src, const mc_run *run,
                                 int n_bins) {
    if (validate(medium, src, n_src, run) != MC_OK || !binned_args_ok(n_bins)) return 0;
    return binned_layout(medium, src, run, n_bins).total;
}

mc_status mc_run_binned(const mc_medium *medium, const mc_source *src, int n_src, const mc_run *run, int adjoint,
                        int n_bins, double *binned_d, mc_ledger *ledger_d, void *workspace_d, size_t workspace_bytes,
                        void *stream) {
    return run_binned(medium, src, n_src, run, adjoint, n_bins, binned_d, ledger_d, workspace_d, workspace_bytes,
                      reinterpret_cast<hipStream_t>(stream));
}

size_t mc_workspace_bytes(const mc_medium *medium, const mc_source *src, int n_src, const mc_run *run,
                          const mc_options *opts) {
    if (validate(medium, src, n_src, run) != MC_OK) return 0;
    TileTuning tt;
    if (!tuning_from(opts, tt)) return 0;
    if (is_tiled(medium, run, tt)) {
        const BatchProblem one{medium, src, n_src, run, 0, nullptr, nullptr};
        return batch_layout(&one, 1, tt).total;
    }
    return layout(medium, src, run).total;
}

size_t mc_batch_workspace_bytes(const mc_problem *probs, int n_probs, const mc_options *opts) {
    if (!probs || n_probs < 1 || n_probs > MC_BATCH_MAX) return 0;
    TileTuning tt;
    if (!tuning_from(opts, tt)) return 0;
    std::vector<BatchProblem> pb(n_probs);
    for (int i = 0; i < n_probs; ++i) {
        const mc_problem &q = probs[i];
        if (validate(&q.medium, q.src, q.n_src, &q.run) != MC_OK || q.run.n_harm != probs[0].run.n_harm) return 0;
        pb[i] = BatchProblem{&q.medium, q.src, q.n_src, &q.run, q.adjoint ? 1 : 0, q.coeffs_d, q.ledger_d};
    }
    return batch_layout(pb.data(), n_probs, tt).total;
}

mc_status mc_run_batch(const mc_problem *probs, int n_probs, const mc_options *opts, void *workspace_d,
                       size_t workspace_bytes, void *stream) {
    if (!probs || n_probs < 1 || n_probs > MC_BATCH_MAX) return MC_ERR_INVALID_ARG;
    std::vector<BatchProblem> pb(n_probs);
    for (int i = 0; i < n_probs; ++i) {
        const mc_problem &q = probs[i];
        pb[i] = BatchProblem{&q.medium, q.src, q.n_src, &q.run, q.adjoint ? 1 : 0, q.coeffs_d, q.ledger_d};
    }
    TileTuning tt;
    if (!tuning_from(opts, tt)) return MC_ERR_INVALID_ARG;
    return run_batch(pb.data(), n_probs, tt, opts ? opts->timer : nullptr, workspace_d, workspace_bytes,
                     reinterpret_cast<hipStream_t>(stream));
}

mc_status mc_forward(const mc_medium *medium, const mc_source *src, int n_src, const mc_run *run,
                     const mc_options *opts, double *coeffs_d, mc_ledger *ledger_d, void *workspace_d,
                     size_t workspace_bytes, void *stream) {
    TileTuning tt;
    if (!tuning_from(opts, tt)) return MC_ERR_INVALID_ARG;
    return run_mc(medium, src, n_src, run, tt, opts ? opts->timer : nullptr, coeffs_d, ledger_d, workspace_d,
                  workspace_bytes, reinterpret_cast<hipStream_t>(stream), 0);
}

mc_status mc_adjoint(const mc_medium *medium, const mc_source *src, int n_src, const mc_run *run,
                     const mc_options *opts, double *coeffs_d, mc_ledger *ledger_d, void *workspace_d,
                     size_t workspace_bytes, void *stream) {
    TileTuning tt;
    if (!tuning_from(opts, tt)) return MC_ERR_INVALID_ARG;
    return run_mc(medium, src, n_src, run, tt, opts ? opts->timer : nullptr, coeffs_d, ledger_d, workspace_d,
                  workspace_bytes, reinterpret_cast<hipStream_t>(stream), 1);
}

mc_status mc_run_noalloc(const mc_medium *medium, const mc_source *src, int n_src, const mc_run *run, int adjoint,
                         const mc_options *opts, double *coeffs_d, mc_ledger *ledger_d, void *stream) {
    mc_status st = validate(medium, src, n_src, run);
    if (st != MC_OK) return st;
    if (!coeffs_d || (adjoint != 0 && adjoint != 1) || (opts && opts->timer)) return MC_ERR_INVALID_ARG;
    TileTuning tt;
    if (!tuning_from(opts, tt)) return MC_ERR_INVALID_ARG;
    if (!noalloc_tuning(medium, src, n_src, run, adjoint, opts, tt)) return MC_ERR_SCRATCH;
    void *ws = scratch_ptr();
    if (!ws) return MC_ERR_DEVICE;
    return run_mc(medium, src, n_src, run, tt, nullptr, coeffs_d, ledger_d, ws, kScratchBytes,
                  reinterpret_cast<hipStream_t>(stream), adjoint);
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
                       n_harm, (double)m->dx * m->dx, m->mua_d, m->g_d, fwd_d, adj_d, hmeas_d, nullptr, dmua_d, dmus_d);
    return hipGetLastError() == hipSuccess ? MC_OK : MC_ERR_DEVICE;
}

mc_status mc_gradient_h(const mc_medium *m, int n_harm, const double *fwd_d, const double *adj_d,
                        const double *grad_h_d, double *dmua_d, double *dmus_d, void *stream) {
    if (!m || m->nx <= 0 || m->nz <= 0 || !(m->dx > 0.f) || !m->mua_d || !m->g_d || !fwd_d || !adj_d || !grad_h_d)
        return MC_ERR_INVALID_ARG;
    if (n_harm < 0 || n_harm > MC_NHARM_MAX) return MC_ERR_INVALID_ARG;
    const int npix = m->nx * m->nz;
    hipLaunchKernelGGL(k_gradient, dim3((npix + 255) / 256), dim3(256), 0, reinterpret_cast<hipStream_t>(stream), npix,
                       n_harm, (double)m->dx * m->dx, m->mua_d, m->g_d, fwd_d, adj_d, nullptr, grad_h_d, dmua_d,
                       dmus_d);
    return hipGetLastError() == hipSuccess ? MC_OK : MC_ERR_DEVICE;
}

mc_status mc_absorbed(const mc_medium *m, const double *coeffs_d, double *h_d, void *stream) {
    if (!m || m->nx <= 0 || m->nz <= 0 || !m->mua_d || !coeffs_d || !h_d) return MC_ERR_INVALID_ARG;
    const int npix = m->nx * m->nz;
    hipLaunchKernelGGL(k_absorbed, dim3((npix + 255) / 256), dim3(256), 0, reinterpret_cast<hipStream_t>(stream), npix,
                       m->mua_d, coeffs_d, h_d);
    return hipGetLastError() == hipSuccess ? MC_OK : MC_ERR_DEVICE;
}

mc_status mc_adjoint_source(const mc_medium *m, const double *grad_h_d, double *q_star_d, void *stream) {
    if (!m || m->nx <= 0 || m->nz <= 0 || !(m->dx > 0.f) || !m->mua_d || !grad_h_d || !q_star_d)
        return MC_ERR_INVALID_ARG;
    const int npix = m->nx * m->nz;
    hipLaunchKernelGGL(k_adjoint_source, dim3((npix + 255) / 256), dim3(256), 0,
                       reinterpret_cast<hipStream_t>(stream), npix, 1.0 / ((double)m->dx * m->dx), m->mua_d, grad_h_d,
                       q_star_d);
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
    ProbDev P;
    fill_problem(P, m, src, n_src, run, adjoint, kFlushTrackMax);
    P.med = reinterpret_cast<const float4 *>(base + L.med);
    P.cdf = reinterpret_cast<const double *>(base + L.cdf);
    ProbDev *pd = reinterpret_cast<ProbDev *>(base + L.pd);
    if (setup_problem(P, pd, nullptr, 0, m->mua_d, m->mus_d, m->g_d, 0) != MC_OK ||
        hipMemcpy(d_pids, pids_h, sizeof(uint64_t) * n_pids, hipMemcpyHostToDevice) != hipSuccess) {
        cleanup();
        return MC_ERR_DEVICE;
    }
    hipLaunchKernelGGL(kernels().tr[run->n_harm], dim3(1), dim3(64), 0, 0, (const ProbDev *)pd,
                       (const uint64_t *)d_pids, n_pids, (mc_event *)d_ev, cap, (unsigned long long *)d_n);
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
        case MC_ERR_SCRATCH: return "the run's workspace exceeds the library's static scratch (MC_SCRATCH_BYTES)";
    }
    return "unknown status";
}

mc_status mc_default_tuning(mc_tuning *t) {
    if (!t) return MC_ERR_INVALID_ARG;
    const TileTuning v;
    t->live_packets = v.live;
    t->job_packets = v.job;
    t->max_visits = v.maxvis;
    t->tile = 0;
    t->finish_packets = std::min<uint64_t>(kFinishMax, v.live / 128);
    t->grid_max_packets = (uint32_t)v.grid_max;
    t->flush_track = (float)v.flush_track;
    t->tail_visits = v.tailvis;
    t->max_generations = 0;   // chosen per run from its packet count and pool
    t->min_job_packets = v.job_min;
    t->quiet_percent = v.quiet;
    return MC_OK;
}

mc_status mc_timer_create(mc_timer **timer) {
    if (!timer) return MC_ERR_INVALID_ARG;
    *timer = new (std::nothrow) mc_timer();
    return *timer ? MC_OK : MC_ERR_DEVICE;
}

mc_status mc_timer_destroy(mc_timer *timer) {
    if (!timer) return MC_ERR_INVALID_ARG;
    for (auto &ev : timer->pending) {
        (void)hipEventSynchronize(ev.second);
        (void)hipEventDestroy(ev.first);
        (void)hipEventDestroy(ev.second);
    }
    delete timer;
    return MC_OK;
}

mc_status mc_timer_read(mc_timer *timer, double *transport_ms, uint64_t *launches, int reset) {
    if (!timer) return MC_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> g(timer->mu);
    mc_status st = MC_OK;
    for (auto &ev : timer->pending) {
        float ms = 0.f;
        if (hipEventSynchronize(ev.second) != hipSuccess || hipEventElapsedTime(&ms, ev.first, ev.second) != hipSuccess)
            st = MC_ERR_DEVICE;
        timer->ms += ms;
        timer->launches += 1;
        (void)hipEventDestroy(ev.first);
        (void)hipEventDestroy(ev.second);
    }
    timer->pending.clear();
    if (transport_ms) *transport_ms = timer->ms;
    if (launches) *launches = timer->launches;
    if (reset) {
        timer->ms = 0;
        timer->launches = 0;
    }
    return st;
}

const char *mc_build_info(void) {
    return "librmc gfx950: FP32 transport; 64-bit fixed-point tally in LDS (whole grid when it fits, else square "
           "tiles with packet migration between tiles, generations steered on the device), added to an FP64 HBM map";
}

}  // extern "C"
