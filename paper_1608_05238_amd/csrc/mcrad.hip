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
//        in generations (launch, counting sort by tile, one workgroup job per
//        tile batch, tile tally added to the FP64 map per job); a finisher
//        kernel moves the last packets to their end without migration;
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
#include <vector>

#include "mcrad.h"

namespace {

constexpr int kMaxSrc = 8;
constexpr int kMaxProf = 2 * (2 * MC_NHARM_MAX + 1);  // profile coefficients over all sources
// whole-grid mode: 12 waves share one LDS tally (8 for high orders, whose
// harmonic vectors need more registers)
constexpr int grid_block(int nh) { return nh <= 16 ? 1024 : 512; }
constexpr int kBlockTile = 512;                        // tiled mode: 8 waves per workgroup, 2 workgroups per CU
constexpr uint64_t kChunk = 1ull << 22;                // whole-grid mode: packets per launch
constexpr size_t kLdsGridMax = 144 * 1024;             // whole-grid mode: tally bytes in LDS
constexpr size_t kLdsTileMax = 72 * 1024;              // tiled mode: tile tally + medium bytes (2 WGs/CU)
constexpr uint32_t kInvalidTile = 0xFFFFFFFFu;
constexpr uint32_t kSlice = 256;                       // queue slots a wave reserves at a time
constexpr float kPi = 3.14159265358979323846f;
constexpr uint32_t kMaxInteractions = 1u << 24;         // hard cap per packet (guards invalid media)
// tiled mode: the LDS tile tally holds 64-bit fixed-point sums, value * 2^(32 - e)
// where 2^e bounds the magnitude of any packet weight of the run (fixed_add)
constexpr int kFixBits = 32;
constexpr double kFlushTrackMax = 65536.0;             // see TileTuning::flush_track

enum : int { EV_LAUNCH = 0, EV_CROSS = 1, EV_SCATTER = 2, EV_ESCAPE = 3, EV_KILL = 4, EV_NONE = 5 };

struct SrcDev {
    int kind, lambertian, prof_off, n_prof;
    double x0, z0, x1, z1;      // mm
    float dir_x, dir_z;
    double cum;                 // inclusive prefix of the sampling measure
};

// Per-problem values the tiled transport needs for a job: one entry per
// problem of a batch (a single run is a batch of one).
struct ProbDev {
    int nx, nz, ntx, tile_base;   // grid, tiles across, first global tile index
    uint32_t tag, flags;
    uint64_t seed;
    float wth, rm, inv_rm;
    float flush_at;               // scaled |a0 accumulator| at which a visit is flushed in parts
    float fx;                     // fixed-point scale of the LDS tile tally (a power of two)
    double fx_inv;                // its inverse
    const float4 *med;
    const float *g;
    double *t64;
    double *led;
    unsigned long long *ledc;     // [4]: jobs whose tile tally may have left the fixed-point range
};

// The values a step and a scatter read, uniform over a workgroup's job.
struct Hot {
    int nx, nz;
    uint32_t tag, flags;
    uint64_t seed;
    float wth, rm, inv_rm;
};

struct Params {
    int nx, nz, npix, nsrc;
    float dx;
    int adjoint;
    uint32_t tag, flags;
    uint64_t seed, pid0, npk;   // packet range of this launch
    float wth, rm, inv_rm;
    double total;
    double inv_qbar;            // MAP: npix / sum |q| (equal-count launch)
    double wbound;              // bound on |packet weight| (launch weight, roulette gain)
    float fx;                   // fixed-point scale of the visit sums (a power of two, fixed_add)
    float flush_at;             // scaled |a0| of a visit at which it is flushed in parts
    double fx_inv;              // 1 / fx
    const float4 *med;          // {mua dx, mus dx, 1/(mua dx), 1/(mus dx)}
    const float *g;
    const double *map;          // MAP source values (sign)
    const double *cdf;          // MAP: inclusive prefix of |map|
    double *t64;                // FP64 tally [npix][K]
    // tiled mode: packets migrate between square tiles whose tallies live in LDS
    int tw, th, ntx, ntiles;
    struct PacketRec *qa;       // unsorted records (appended by launches and leavers)
    uint32_t *qtile;            // tile of each unsorted record (kInvalidTile: empty slot)
    struct PacketRec *qb;       // records sorted by tile
    uint32_t *qcnt;             // [0] raw records in qa, [1] records to scatter, [2] jobs, [3] job cursor,
                                // [4] overflow flag, [5] finisher record cursor, [6] valid records
                                // written by the last transport launch
    uint32_t *tile_count, *tile_cursor;
    uint4 *jobs;                // (tile, first record in qb, count, 0)
    uint32_t cap_a, cap_b, job_size, max_visits, tail_visits;
    const ProbDev *probs;       // batch: problem descriptors
    const uint32_t *tile_prob;  // batch: problem of each global tile
    int tile_base;              // this problem's first global tile
    uint32_t prob;              // this problem's index in the batch
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
__device__ bool launch_state(const Params &P, uint64_t pid, Packet &p, LedgerRegs &L) {
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
__device__ bool launch(const Params &P, uint64_t pid, Packet &p, float *h, LedgerRegs &L) {
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

template <int NH>
__device__ __forceinline__ bool scatter(const Params &P, Packet &p, const float g, float *h, LedgerRegs &L) {
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
template <int NH>
__global__ void __launch_bounds__(grid_block(NH)) k_transport_grid(Params P) {
    constexpr int K = 2 * NH + 1;
    extern __shared__ unsigned long long gfx[];   // [npix][K] fixed-point sums (fixed_add)
    __shared__ float s_mag;
    const int lane = __lane_id();
    for (int i = threadIdx.x; i < P.npix * K; i += blockDim.x) gfx[i] = 0ull;
    if (threadIdx.x == 0) s_mag = 0.f;
    __syncthreads();
    const float fx = P.fx, flush_at = P.flush_at;

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
                if (lane == leader) base = atomicAdd(P.counter, (unsigned long long)ndead);
                base = __shfl(base, leader);
                if (base + ndead >= P.npk) more = false;
                if (!p.alive) {
                    const unsigned long long my = base + __popcll(dead & lt_mask);
                    if (my < P.npk) launch_state(P, P.pid0 + my, p, L);
                }
            }
        }
        if (!__ballot(p.alive)) {
            if (!more) break;
        }
        // every lane steps and scatters (no branch); a free lane's results are discarded
        const bool live = p.alive;
        const int pix = live ? p.iz * P.nx + p.ix : 0;
        float T = 0.f, dw = 0.f;
        const float4 mm = P.med[pix];
        int ev = step(P, p, mm, T, dw);
        ev = live ? ev : EV_NONE;
        T = live ? T : 0.f;
        dw = live ? dw : 0.f;
        L.absorbed += (double)dw;
        L.segments += live ? 1u : 0u;
        deposit_harmonics<NH>(T * fx, p.sx, p.sz, keep, acc);   // direction of the segment, before any scatter
        const bool at = ev == EV_SCATTER;
        const bool killed = scatter_masked(P, p, at, mm.w, L);
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
    ledger_flush_block(P.led, P.ledc, L);
    float wm = mag;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) wm += __shfl_xor(wm, o);
    if (lane == 0) atomicAdd(&s_mag, wm);
    __syncthreads();
    if (threadIdx.x == 0 && !(s_mag < 0x1p62f)) atomicAdd(P.ledc + 4, 1ull);   // see k_normalise
    for (int i = threadIdx.x; i < P.npix * K; i += blockDim.x) {
        const double v = (double)(long long)gfx[i] * P.fx_inv;
        if (v != 0.0) unsafeAtomicAdd(P.t64 + i, v);
    }
}

// ------------------------------------------------------------------ tiled transport
// Larger grids: the grid is cut into tw x th tiles whose tallies (64-bit
// fixed-point sums, fixed_add) fit in LDS.  A run proceeds in generations.  Each generation, the live packets
// (sorted by tile) are split into jobs of at most job_size packets of one
// tile; a workgroup takes a job, keeps that tile's tally and medium in LDS,
// and moves each packet until it leaves the tile, dies, or has made
// max_visits visits there.  Packets that leave (or pause) are written back as
// records and sorted by tile for the next generation; new packets are
// launched to keep the population up.  Every tally update is an LDS atomic;
// HBM sees one coalesced flush of the tile per job.

__device__ __forceinline__ uint32_t tile_of(const Params &P, int ix, int iz) {
    return (uint32_t)((iz / P.th) * P.ntx + ix / P.tw);
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

// Wave-private slices of the unsorted queue: a wave reserves kSlice slots
// with one atomic on the queue counter (shared by every wave of the device,
// so it is touched rarely) and fills them; unused slots are marked invalid.
struct QueueSlice {
    uint32_t base = 0, used = kSlice, nput = 0;
    bool valid = false;
};

__device__ __forceinline__ void slice_close(const Params &P, QueueSlice &q) {
    if (!q.valid) return;
    const int lane = __lane_id();
    for (uint32_t i = q.used + lane; i < kSlice; i += 64)
        if (q.base + i < P.cap_a) P.qtile[q.base + i] = kInvalidTile;
}

// Appends the packet of every lane with `put` set to the unsorted queue.
__device__ __forceinline__ void slice_put(const Params &P, QueueSlice &q, bool put, const Packet &p, uint32_t tile,
                                          uint32_t prob) {
    const unsigned long long m = __ballot(put);
    if (!m) return;
    const int n = __popcll(m);
    const int lane = __lane_id();
    if (q.used + n > kSlice) {
        slice_close(P, q);
        uint32_t base = 0;
        if (lane == 0) base = atomicAdd(P.qcnt, kSlice);
        q.base = __shfl(base, 0);
        q.used = 0;
        q.valid = true;
    }
    if (put) {
        const uint32_t pos = q.base + q.used + __popcll(m & ((1ull << lane) - 1ull));
        if (pos < P.cap_a) {
            rec_store(P.qa + pos, p, tile, prob);
            P.qtile[pos] = tile;
        }
        else atomicOr(P.qcnt + 4, 1u);   // overflow: reported to the host, never written
    }
    q.used += n;
    q.nput += n;
}

// End of a wave's appends: pad its last slice and count its records.
__device__ __forceinline__ void slice_finish(const Params &P, QueueSlice &q) {
    slice_close(P, q);
    if (q.nput && __lane_id() == 0) atomicAdd(P.qcnt + 6, q.nput);
}

// Launch n_new packets (ids pid_base..) and append those inside the grid.
// A grid-stride loop over few workgroups: each iteration reserves queue slots
// with one atomic per workgroup, and the energy ledger is reduced over the
// workgroup before its single set of atomics (the ledger and queue counters
// are single addresses shared by the whole device).
__global__ void __launch_bounds__(256) k_tile_launch(Params P, uint64_t pid_base, uint32_t n_new) {
    __shared__ uint32_t s_cnt[4];
    __shared__ uint32_t s_base;
    const int lane = __lane_id(), wave = threadIdx.x >> 6;
    LedgerRegs L;
    for (uint32_t b0 = blockIdx.x * blockDim.x; b0 < n_new; b0 += gridDim.x * blockDim.x) {
        const uint32_t i = b0 + threadIdx.x;
        Packet p;
        p.alive = false;
        if (i < n_new) launch_state(P, pid_base + i, p, L);
        const unsigned long long m = __ballot(p.alive);
        if (lane == 0) s_cnt[wave] = (uint32_t)__popcll(m);
        __syncthreads();
        if (threadIdx.x == 0) {
            const uint32_t tot = s_cnt[0] + s_cnt[1] + s_cnt[2] + s_cnt[3];
            s_base = tot ? atomicAdd(P.qcnt, tot) : 0u;
        }
        __syncthreads();
        if (p.alive) {
            uint32_t pos = s_base + __popcll(m & ((1ull << lane) - 1ull));
            for (int w = 0; w < wave; ++w) pos += s_cnt[w];
            if (pos < P.cap_a) {
                const uint32_t t = (uint32_t)P.tile_base + tile_of(P, p.ix, p.iz);
                rec_store(P.qa + pos, p, t, P.prob);
                P.qtile[pos] = t;
            } else {
                atomicOr(P.qcnt + 4, 1u);
            }
        }
        __syncthreads();
    }
    ledger_flush_block(P.led, P.ledc, L);
}

// Counting sort of the unsorted queue by tile: counts.  Up to kHistTiles
// tiles a workgroup histograms its share in LDS and adds each non-zero bin
// to the global count once; beyond that, wave-aggregated global atomics.
constexpr int kHistTiles = 4096;

__global__ void __launch_bounds__(256) k_bin_count(Params P) {
    __shared__ uint32_t hist[kHistTiles];
    const uint32_t n = P.qcnt[0] < P.cap_a ? P.qcnt[0] : P.cap_a;
    const int lane = __lane_id();
    const bool local = P.ntiles <= kHistTiles;
    if (local) {
        for (int i = threadIdx.x; i < P.ntiles; i += blockDim.x) hist[i] = 0u;
        __syncthreads();
    }
    for (uint32_t base = blockIdx.x * blockDim.x; base < n; base += gridDim.x * blockDim.x) {
        const uint32_t i = base + threadIdx.x;
        const uint32_t t = i < n ? P.qtile[i] : kInvalidTile;
        if (local) {
            if (t != kInvalidTile) atomicAdd(hist + t, 1u);
            continue;
        }
        bool pend = t != kInvalidTile;
        for (;;) {
            const unsigned long long m = __ballot(pend);
            if (!m) break;
            const int leader = __ffsll((long long)m) - 1;
            const uint32_t t0 = __shfl(t, leader);
            const unsigned long long same = __ballot(pend && t == t0);
            if (lane == leader) atomicAdd(P.tile_count + t0, (uint32_t)__popcll(same));
            if (pend && t == t0) pend = false;
        }
    }
    if (local) {
        __syncthreads();
        for (int i = threadIdx.x; i < P.ntiles; i += blockDim.x)
            if (hist[i]) atomicAdd(P.tile_count + i, hist[i]);
    }
}

// Single block: exclusive scan of the tile counts, job list, counters for the
// next phase.  Tile counts are reset for the next generation.
__global__ void __launch_bounds__(1024) k_bin_scan(Params P) {
    __shared__ uint32_t s_rec[1024], s_job[1024];
    const int t = threadIdx.x;
    const int per = (P.ntiles + 1023) / 1024;
    const int a = t * per, b = min(P.ntiles, a + per);
    uint32_t nrec = 0, njob = 0;
    for (int i = a; i < b; ++i) {
        const uint32_t c = P.tile_count[i];
        nrec += c;
        njob += (c + P.job_size - 1) / P.job_size;
    }
    s_rec[t] = nrec;
    s_job[t] = njob;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {   // inclusive Hillis-Steele scan
        const uint32_t vr = t >= off ? s_rec[t - off] : 0u, vj = t >= off ? s_job[t - off] : 0u;
        __syncthreads();
        s_rec[t] += vr;
        s_job[t] += vj;
        __syncthreads();
    }
    const bool fits = s_rec[1023] <= P.cap_b;   // holds by construction; checked so nothing is written past it
    uint32_t roff = s_rec[t] - nrec, joff = s_job[t] - njob;
    for (int i = a; i < b; ++i) {
        const uint32_t c = P.tile_count[i];
        P.tile_cursor[i] = roff;
        if (fits)
            for (uint32_t s0 = 0; s0 < c; s0 += P.job_size)
                P.jobs[joff++] = make_uint4((uint32_t)i, roff + s0, min(P.job_size, c - s0), P.tile_prob[i]);
        roff += c;
        P.tile_count[i] = 0;
    }
    __syncthreads();
    if (t == 1023) {
        P.qcnt[1] = P.qcnt[0] < P.cap_a ? P.qcnt[0] : P.cap_a;
        P.qcnt[0] = 0;
        P.qcnt[2] = fits ? s_job[1023] : 0u;
        P.qcnt[3] = 0;
        P.qcnt[6] = 0;
        if (!fits) P.qcnt[4] = 1u;
    }
}

// Counting sort: scatter records to their tile's range of the sorted queue.
// A workgroup takes chunks of kScatterChunk records.  Up to kHistTiles tiles,
// each record gets its rank among the chunk's records of its tile from an LDS
// atomic, the workgroup reserves one range per tile it holds with a single
// global atomic, and every record lands at range start + rank; beyond that,
// ranks come from wave-aggregated global atomics.  The 64-byte records are
// moved by four lanes each, so every load and store instruction covers
// sixteen whole records.
constexpr int kScatterPer = 8;                              // records per thread and chunk
constexpr uint32_t kScatterChunk = 256u * kScatterPer;

__device__ __forceinline__ void move_records(const Params &P, uint32_t wave_first, uint32_t pos) {
    const int lane = __lane_id();
    const int part = lane & 3;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int r = q * 16 + (lane >> 2);   // record of the wave this lane helps move
        const uint32_t dst = __shfl(pos, r);
        if (dst < P.cap_b) {
            const uint4 *src = reinterpret_cast<const uint4 *>(P.qa + wave_first + r);
            reinterpret_cast<uint4 *>(P.qb + dst)[part] = src[part];
        }
    }
}

__global__ void __launch_bounds__(256) k_bin_scatter(Params P) {
    __shared__ uint32_t cnt[kHistTiles];
    __shared__ uint32_t start[kHistTiles];
    const uint32_t n = P.qcnt[1];
    const int lane = __lane_id();
    if (P.ntiles <= kHistTiles) {
        for (uint32_t c0 = blockIdx.x * kScatterChunk; c0 < n; c0 += gridDim.x * kScatterChunk) {
            for (int i = threadIdx.x; i < P.ntiles; i += blockDim.x) cnt[i] = 0u;
            __syncthreads();
            uint32_t t[kScatterPer], rank[kScatterPer];
#pragma unroll
            for (int r = 0; r < kScatterPer; ++r) {
                const uint32_t i = c0 + r * 256u + threadIdx.x;
                t[r] = i < n ? P.qtile[i] : kInvalidTile;
                rank[r] = t[r] != kInvalidTile ? atomicAdd(cnt + t[r], 1u) : 0u;
            }
            __syncthreads();
            for (int i = threadIdx.x; i < P.ntiles; i += blockDim.x)
                start[i] = cnt[i] ? atomicAdd(P.tile_cursor + i, cnt[i]) : 0u;
            __syncthreads();
#pragma unroll
            for (int r = 0; r < kScatterPer; ++r) {
                const uint32_t pos = t[r] != kInvalidTile ? start[t[r]] + rank[r] : 0xFFFFFFFFu;
                move_records(P, c0 + r * 256u + threadIdx.x - (uint32_t)lane, pos);
            }
            __syncthreads();
        }
        return;
    }
    for (uint32_t base = blockIdx.x * blockDim.x; base < n; base += gridDim.x * blockDim.x) {
        const uint32_t i = base + threadIdx.x;
        const uint32_t t = i < n ? P.qtile[i] : kInvalidTile;
        bool pend = t != kInvalidTile;
        uint32_t pos = 0xFFFFFFFFu;
        for (;;) {
            const unsigned long long m = __ballot(pend);
            if (!m) break;
            const int leader = __ffsll((long long)m) - 1;
            const uint32_t t0 = __shfl(t, leader);
            const unsigned long long same = __ballot(pend && t == t0);
            uint32_t b0 = 0;
            if (lane == leader) b0 = atomicAdd(P.tile_cursor + t0, (uint32_t)__popcll(same));
            b0 = __shfl(b0, leader);
            if (pend && t == t0) {
                pos = b0 + __popcll(same & ((1ull << lane) - 1ull));
                pend = false;
            }
        }
        move_records(P, i - (uint32_t)lane, pos);
    }
}

template <int NH>
__global__ void __launch_bounds__(kBlockTile) __attribute__((amdgpu_waves_per_eu(NH <= 16 ? 4 : 2))) k_transport_tile(Params P) {
    constexpr int K = 2 * NH + 1;
    // [tw*th][K] fixed-point sums: value * fx of the job's problem (fixed_add)
    extern __shared__ unsigned long long fxt[];
    float4 *smed = reinterpret_cast<float4 *>(fxt + (((size_t)P.tw * P.th * K + 1) & ~size_t(1)));
    uint32_t *sadds = reinterpret_cast<uint32_t *>(smed + P.tw * P.th);   // fixed_add_raw adds per pixel
    __shared__ uint32_t s_job[5];
    __shared__ uint32_t s_next;
    __shared__ float s_mag;
    const int lane = __lane_id();
    const int ntp = P.tw * P.th;
    const unsigned long long lt_mask = (1ull << lane) - 1ull;
    LedgerTile L;
    QueueSlice q;
    int cur = -1;   // problem whose ledger L holds

    for (;;) {
        if (threadIdx.x == 0) {
            const uint32_t j = atomicAdd(P.qcnt + 3, 1u);
            const bool ok = j < P.qcnt[2];
            const uint4 jb = ok ? P.jobs[j] : make_uint4(0u, 0u, 0u, 0u);
            s_job[0] = ok ? 1u : 0u;
            s_job[1] = jb.x;
            s_job[2] = jb.y;
            s_job[3] = jb.z;
            s_job[4] = jb.w;
            s_next = 0;
            s_mag = 0.f;
        }
        __syncthreads();
        if (!s_job[0]) break;
        const uint32_t tile = s_job[1], first = s_job[2], cnt = s_job[3], prob = s_job[4];
        const ProbDev &pd = P.probs[prob];
        if ((int)prob != cur) {   // the ledger follows the problem (uniform in the workgroup)
            if (cur >= 0) {
                ledger_flush_tile(P.probs[cur].led, P.probs[cur].ledc, L);
                L = LedgerTile();
            }
            cur = (int)prob;
        }
        const Hot H{pd.nx, pd.nz, pd.tag, pd.flags, pd.seed, pd.wth, pd.rm, pd.inv_rm};
        const int ntx = pd.ntx, local = (int)tile - pd.tile_base;
        const float4 *gmed = pd.med;
        double *t64 = pd.t64;
        const float fx = pd.fx;   // power of two: the scaled FP32 sums round exactly as unscaled ones
        const float flush_at = pd.flush_at;
        const int tx0 = (local % ntx) * P.tw, tz0 = (local / ntx) * P.th;
        for (int i = threadIdx.x; i < ntp * K; i += blockDim.x) fxt[i] = 0ull;
        for (int i = threadIdx.x; i < ntp; i += blockDim.x) sadds[i] = 0u;
        for (int i = threadIdx.x; i < ntp; i += blockDim.x) {
            const int gx = tx0 + i % P.tw, gz = tz0 + i / P.tw;
            const bool in = gx < H.nx && gz < H.nz;
            smed[i] = in ? gmed[gz * H.nx + gx] : make_float4(0.f, 0.f, 0.f, 0.f);
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
        // one whole stay ahead, so a refill never waits for memory.
        bool more = true, has_next = false;
        uint32_t tail_nvis = 0;   // visits of the current stay when the job ran out of packets
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
            const int lp = live ? __mul24(p.iz - tz0, P.tw) + (p.ix - tx0) : 0;
            const float4 mm = smed[lp];
            // lanes without a prefetched record claim the next ones of the job
            if (more) {
                const unsigned long long want = __ballot(!has_next);
                if (want) {
                    const int nw = __popcll(want);
                    const int leader = __ffsll((long long)want) - 1;
                    uint32_t base = 0;
                    if (lane == leader) base = atomicAdd(&s_next, (uint32_t)nw);
                    base = __shfl(base, leader);
                    if (base + nw >= cnt) {
                        more = false;
                        tail_nvis = nvis;
                    }
                    if (!has_next) {
                        const uint32_t my = base + __popcll(want & lt_mask);
                        if (my < cnt) {
                            const uint4 *r = reinterpret_cast<const uint4 *>(P.qb + first + my);
                            nr0 = r[0];
                            nr1 = r[1];
                            nr2 = r[2];
                            const uint64_t id = P.qb[first + my].pid;
                            nr3 = make_uint2((uint32_t)id, (uint32_t)(id >> 32));
                            has_next = true;
                        }
                    }
                }
            }
            if (!__ballot(p.alive)) {
                if (!more && !__ballot(has_next)) break;
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
                    const int ox = p.ix < tx0 ? -1 : (p.ix >= tx0 + P.tw ? 1 : 0);
                    const int oz = p.iz < tz0 ? -1 : (p.iz >= tz0 + P.th ? 1 : 0);
                    const bool out = (ox | oz) != 0;
                    dest = (uint32_t)((int)tile + __mul24(oz, ntx) + ox);   // a crossing moves one pixel: a neighbour tile
                    // once the job has no packets left to hand out, a packet pauses
                    // after tail_visits more visits so the workgroup is not held by
                    // its longest stay (it resumes next generation)
                    leave = out || nvis >= (more ? P.max_visits : min(P.max_visits, tail_nvis + P.tail_visits));
                }
            }
            keep = flush ? 0.f : 1.f;
            slice_put(P, q, leave, p, dest, prob);
            if (leave) {
                p.alive = false;
                nvis = 0;
            }
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
        for (int i = threadIdx.x; i < ntp * K; i += blockDim.x) {
            const int lp = i / K, c = i - lp * K;
            const double v = (double)fixed_value(fxt[i], sadds[lp]) * pd.fx_inv;
            const int gx = tx0 + lp % P.tw, gz = tz0 + lp / P.tw;
            if (v != 0.0 && gx < H.nx && gz < H.nz) unsafeAtomicAdd(t64 + (size_t)(gz * H.nx + gx) * K + c, v);
        }
        __syncthreads();
    }
    slice_finish(P, q);
    if (cur >= 0) ledger_flush_tile(P.probs[cur].led, P.probs[cur].ledc, L);   // cur is uniform
}

// ------------------------------------------------------------------ tail finisher
// When few packets remain after the last launch, the generations would be
// dominated by the longest-lived packets.  The finisher moves each remaining
// packet to its end without migration; a wave stages the K-vectors of the
// visits it completes in LDS and adds them to the HBM FP64 tally as
// contiguous runs of atomics.
constexpr int kBlockFinish = 256;

// Adds a wave's staged visit sums (n visits of K values) to the HBM tally:
// consecutive lanes take consecutive values, so each pixel's K channels go
// out as one contiguous run of atomics.
__device__ __forceinline__ void finish_flush_stage(const Params &P, const float *stage, const int *stage_pix, int n,
                                                   int K, double fx_inv) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int total = n * K;
    for (int e = __lane_id(); e < total; e += 64) {
        const int v = e / K;
        const float val = stage[e];
        if (val != 0.f)
            unsafeAtomicAdd(P.t64 + (size_t)stage_pix[v] * K + (e - v * K), __builtin_rint((double)val) * fx_inv);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Few packets per lane and long histories make this kernel latency-bound, so
// its loop keeps global memory off the dependent chain where it can: the
// medium of the pixel a packet enters is loaded one iteration ahead of its
// use, and a wave gathers the sums of up to 64 completed visits in LDS before
// it adds them to the tally (the wait for those atomics then comes once per
// buffer, not once per visit).
template <int NH>
__global__ void __launch_bounds__(kBlockFinish) k_finish(Params P, uint32_t n_rec) {
    constexpr int K = 2 * NH + 1;
    extern __shared__ float stage_all[];
    const int lane = __lane_id();
    const int wave = threadIdx.x >> 6;
    float *stage = stage_all + wave * 64 * K;
    int *stage_pix = reinterpret_cast<int *>(stage_all + (kBlockFinish / 64) * 64 * K) + wave * 64;
    const unsigned long long lt_mask = (1ull << lane) - 1ull;
    LedgerRegs L;
    Packet p;
    idle_packet(p, 0, 0);
    float4 mm = make_float4(0.f, 0.f, 0.f, 0.f);   // medium of the packet's pixel
    float acc[K], keep = 1.f;   // keep = 0 after a flush: the next deposit restarts the sums
#pragma unroll
    for (int j = 0; j < K; ++j) acc[j] = 0.f;
    // visit sums are scaled and rounded as in the LDS tallies (fixed_add), so a
    // visit adds the same value whichever kernel completes it
    const float fx = P.fx, flush_at = P.flush_at;
    const double fx_inv = P.fx_inv;
    bool more = true;
    int used = 0;   // visits staged in this wave's buffer (wave-uniform)
    for (;;) {
        if (more) {
            const unsigned long long dead = __ballot(!p.alive);
            if (dead) {
                const int ndead = __popcll(dead);
                const int leader = __ffsll((long long)dead) - 1;
                uint32_t base = 0;
                if (lane == leader) base = atomicAdd(P.qcnt + 5, (uint32_t)ndead);
                base = __shfl(base, leader);
                if (base + ndead >= n_rec) more = false;
                if (!p.alive) {
                    const uint32_t my = base + __popcll(dead & lt_mask);
                    if (my < n_rec && P.qtile[my] != kInvalidTile && P.qa[my].prob == P.prob) {
                        rec_load(P.qa + my, p);   // a queued packet is inside the grid
                        mm = P.med[p.iz * P.nx + p.ix];
                    }
                }
            }
        }
        if (!__ballot(p.alive)) {
            if (!more) break;
        }
        int ev = EV_NONE, pix = 0;
        float T = 0.f, dw = 0.f;
        const float g = mm.w;   // read before mm is reloaded: the scatter need not wait for that load
        if (p.alive) {
            pix = p.iz * P.nx + p.ix;
            ev = step(P, p, mm, T, dw);
            L.absorbed += (double)dw;
            L.segments += 1;
        }
        // the medium of the pixel the next step starts in (a crossing's new
        // pixel, else the same one), loaded by every lane outside any branch so
        // the load lands in mm directly and is waited for only at that step
        mm = P.med[ev == EV_CROSS ? p.iz * P.nx + p.ix : pix];
        deposit_harmonics<NH>(T * fx, p.sx, p.sz, keep, acc);   // direction of the segment, before any scatter
        bool vend = false;
        if (ev == EV_SCATTER) {
            if (!scatter_dir(P, p, g, L)) vend = true;   // the pixel of the step
        } else if (ev != EV_NONE) {
            vend = true;
            if (ev == EV_ESCAPE) {
                L.escaped += p.w;
                p.alive = false;
            }
        }
        const bool flush = vend || fabsf(acc[0]) > flush_at;
        L.visits += vend ? 1u : 0u;
        const unsigned long long fm = __ballot(flush);
        if (fm) {
            const int nf = __popcll(fm);
            if (used + nf > 64) {   // no room: the staged visits go to the tally first
                finish_flush_stage(P, stage, stage_pix, used, K, fx_inv);
                used = 0;
            }
            if (flush) {
                const int slot = used + __popcll(fm & lt_mask);
                float *st = stage + slot * K;
#pragma unroll
                for (int j = 0; j < K; ++j) st[j] = acc[j];
                stage_pix[slot] = pix;
            }
            used += nf;
        }
        keep = flush ? 0.f : 1.f;
    }
    if (used) finish_flush_stage(P, stage, stage_pix, used, K, fx_inv);
    ledger_flush_block(P.led, P.ledc, L);
}

// ------------------------------------------------------------------ discrete-ordinates tally
// The comparison tally of mc_run_binned: the same launch, step and scatter as
// the whole-grid transport (persistent lanes refilled from a global packet
// counter), but each segment adds its deposit T to raw[bin][pixel] of its
// direction's angular bin with one FP64 device atomic.
constexpr int kBinnedMax = 4096;

__global__ void __launch_bounds__(256) k_transport_binned(Params P, int n_bins, double *raw) {
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
                if (lane == leader) base = atomicAdd(P.counter, (unsigned long long)ndead);
                base = __shfl(base, leader);
                if (base + ndead >= P.npk) more = false;
                if (!p.alive) {
                    const unsigned long long my = base + __popcll(dead & lt_mask);
                    if (my < P.npk) launch_state(P, P.pid0 + my, p, L);
                }
            }
        }
        if (!__ballot(p.alive)) {
            if (!more) break;
        }
        const bool live = p.alive;
        const int pix = live ? p.iz * P.nx + p.ix : 0;
        float T = 0.f, dw = 0.f;
        const float4 mm = P.med[pix];
        int ev = step(P, p, mm, T, dw);
        ev = live ? ev : EV_NONE;
        dw = live ? dw : 0.f;
        L.absorbed += (double)dw;
        L.segments += live ? 1u : 0u;
        if (live && T != 0.f) {   // direction of the segment, before any scatter
            const double th = atan2((double)p.sx, (double)p.sz);
            const int b = min(n_bins - 1, max(0, (int)floor((th + M_PI) * per_rad)));
            unsafeAtomicAdd(raw + (size_t)b * P.npix + pix, (double)T);
        }
        const bool at = ev == EV_SCATTER;
        const bool killed = scatter_masked(P, p, at, mm.w, L);
        if (ev == EV_ESCAPE) {
            L.escaped += p.w;
            p.alive = false;
        }
        L.visits += (killed || (ev != EV_NONE && !at)) ? 1u : 0u;
    }
    ledger_flush_block(P.led, P.ledc, L);
}

// binned[b][i] = raw[b'][i] * scale, b' = b (forward) or b + n_bins/2 (adjoint:
// the mirrored direction)
__global__ void k_binned_normalise(int npix, int n_bins, int adjoint, double scale, const double *raw, double *out) {
    const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (i >= (size_t)npix * n_bins) return;
    const int b = (int)(i / npix);
    const size_t px = i - (size_t)b * npix;
    const int src = adjoint ? (b + n_bins / 2) % n_bins : b;
    out[i] = raw[(size_t)src * npix + px] * scale;
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
            const int pix = p.iz * P.nx + p.ix;
            const int e = step(P, p, P.med[pix], T, dw);
            if (e == EV_SCATTER) {
                if (scatter<NH>(P, p, P.g[pix], h, L)) rec(p, EV_SCATTER, k, ix, iz, p.w, T);
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
// contiguous run, then a sequential pass over the 1024 run totals).
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

// Normalise (Sec. 6: divide by the packet count; times the source measure and
// the track-length-to-fluence factor 1/(dx Np) in pixel units) and transpose
// [npix][K] -> [K][npix]; the adjoint output reads the mirrored direction,
// (-1)^n on orders n >= 1.
// A nonzero *range_errors (tiled mode: a job whose fixed-point tile tally may
// have wrapped) turns the whole output into NaN.
__global__ void k_normalise(int npix, int N, int adjoint, double scale, const double *t64,
                            const unsigned long long *range_errors, double *out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npix) return;
    const int K = 2 * N + 1;
    const bool bad = range_errors && *range_errors;
    for (int c = 0; c < K; ++c) {
        const int n = c <= N ? c : c - N;
        const double f = (adjoint && (n & 1)) ? -scale : scale;
        out[(size_t)c * npix + i] = bad ? __builtin_nan("") : t64[(size_t)i * K + c] * f;
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
using TransportFn = void (*)(Params);
using TraceFn = void (*)(Params, const uint64_t *, int, mc_event *, size_t, unsigned long long *);
using FinishFn = void (*)(Params, uint32_t);

template <int NH>
struct Table {
    static void fill(TransportFn *grid, TransportFn *tile, TraceFn *tr, FinishFn *fin) {
        grid[NH] = k_transport_grid<NH>;
        tile[NH] = k_transport_tile<NH>;
        tr[NH] = k_trace<NH>;
        fin[NH] = k_finish<NH>;
        if constexpr (NH > 0) Table<NH - 1>::fill(grid, tile, tr, fin);
    }
};

struct Kernels {
    TransportFn grid[MC_NHARM_MAX + 1], tile[MC_NHARM_MAX + 1];
    TraceFn tr[MC_NHARM_MAX + 1];
    FinishFn fin[MC_NHARM_MAX + 1];
    Kernels() { Table<MC_NHARM_MAX>::fill(grid, tile, tr, fin); }
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

// Tiled-mode sizing.  Tiles are square, as large as lets two workgroups of a
// CU hold their tile's tally, medium and flush counts in LDS.
// live packets per generation (on the 10^8-packet disc256 gradient 2^25
// against 2^24: -1.8% time, 2^26 against 2^25: -1.1%; small runs unchanged
// once the finisher threshold below is kept at 2^17).  The queues then take
// ~13 GB of HBM.
constexpr uint64_t kLiveMax = 1ull << 26;
constexpr uint64_t kFinishMax = 1ull << 17;   // default finisher threshold: min(this, live / 128)
constexpr uint64_t kGridMaxPackets = 1ull << 21;   // larger runs take the tiled transport
constexpr uint32_t kJobSize = 4096;           // packets per job
constexpr uint64_t kSmallPool = 1ull << 23;   // pools below this many live packets use half-size jobs
constexpr uint32_t kMaxVisitsPerStay = 64;    // a packet pauses after this many visits in one job
// once a job has handed out its last packet, its packets pause after this many
// more visits, so a wave does not idle behind its longest stay (measured on
// the 256x256 disc: 8 beats 2, 4, 16 and no limit by 7-9%)
constexpr uint32_t kTailVisits = 8;
constexpr int kTileWavesMax = 256 * 16;       // bound on resident waves of the tiled kernel

// Tuning knobs of the tiled mode.  Process-wide; set through mc_set_tuning()
// (the autotuner) and initialised from the environment (RMC_LIVE, RMC_JOB,
// RMC_MAXVIS, RMC_TAILVIS, RMC_TILE, RMC_FINISH) for measurement sweeps.  A
// run takes one snapshot when its layout is computed.
struct TileTuning {
    uint64_t live = kLiveMax;
    uint32_t job = kJobSize, maxvis = kMaxVisitsPerStay, tailvis = kTailVisits;
    uint64_t finish = 0;   // 0: min(2^17, live / 128)
    int tile = 0;   // 0: largest square tile for two workgroups per CU
    uint64_t grid_max = kGridMaxPackets;   // whole-grid kernel only up to this many packets
    // a visit whose accumulated track length times |weight| reaches flush_track
    // pixels (in units of the run's weight bound) is flushed to the tile tally
    // in parts; at most 2^16, which keeps every flush inside fixed_add's range
    double flush_track = kFlushTrackMax;
};
TileTuning tuning_from_env() {
    TileTuning v;
    auto get = [](const char *n, uint64_t lo, uint64_t hi, uint64_t def) {
        const char *e = std::getenv(n);
        if (!e) return def;
        const unsigned long long x = std::strtoull(e, nullptr, 10);
        return (x >= lo && x <= hi) ? (uint64_t)x : def;
    };
    v.live = get("RMC_LIVE", 1024, 1ull << 26, v.live);
    v.job = (uint32_t)get("RMC_JOB", 64, 1u << 20, v.job);
    v.maxvis = (uint32_t)get("RMC_MAXVIS", 1, 1u << 30, v.maxvis);
    v.tailvis = (uint32_t)get("RMC_TAILVIS", 1, 1u << 30, v.tailvis);
    v.tile = (int)get("RMC_TILE", 1, 256, 0);
    v.finish = get("RMC_FINISH", 1, 1ull << 26, 0);
    return v;
}
struct TuningState {
    std::mutex mu;
    TileTuning t = tuning_from_env();
};
TuningState &tuning_state() {
    static TuningState s;
    return s;
}
TileTuning tuning_snapshot() {
    TuningState &s = tuning_state();
    std::lock_guard<std::mutex> g(s.mu);
    return s.t;
}

struct Layout {
    size_t med, cdf, t64, led, ledc, counters, qa, qtile, qb, tcount, tcursor, jobs, qcnt, total;
    uint64_t n_chunks;
    bool tiled;
    int tw, th, ntx, ntz, ntiles;
    uint64_t live, cap_a, max_jobs;
    size_t tile_lds;
    TileTuning tt;   // the tuning this layout was computed with
};

// tile LDS: fixed-point sums [tw*th][K], medium [tw*th], flush counts [tw*th]
size_t tile_lds_bytes(int tw, int th, int K) {
    const size_t tal = ((size_t)tw * th * K * sizeof(double) + 15) & ~size_t(15);
    return tal + (size_t)tw * th * (sizeof(float4) + sizeof(uint32_t));
}

// Tiled transport unless the whole tally (8 bytes per value) fits one workgroup's LDS and the
// run is small (the tiled mode's per-generation overhead is ~10 ms; measured
// on a 32x32 pencil beam, the tiled mode overtakes the whole-grid kernel near
// 2e6 packets and is 5x faster at 1e8).
bool is_tiled(const mc_medium *m, const mc_run *run, const TileTuning &tt) {
    if ((size_t)m->nx * m->nz * (2 * run->n_harm + 1) * sizeof(double) > kLdsGridMax) return true;
    return run->n_packets > tt.grid_max;
}

// Whole-grid mode: medium, CDF, tally, ledger and per-chunk counters.
Layout layout(const mc_medium *m, const mc_source *src, const mc_run *run) {
    Layout L{};
    const size_t npix = (size_t)m->nx * m->nz;
    const int K = 2 * run->n_harm + 1;
    L.tiled = is_tiled(m, run, tuning_snapshot());
    size_t off = 0;
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
// medium, CDF, tally and ledger; one packet pool, one set of queues and one
// global tile index space (problem p owns tiles tile_base[p] ..).
struct BatchLayout {
    TileTuning tt;
    int N = 0, K = 0, t = 0, ntiles = 0;
    size_t tile_lds = 0;
    uint64_t live = 0, cap_a = 0, max_jobs = 0, total_packets = 0;
    uint32_t job = 0;   // packets per job: the tuning's, halved for small pools
    std::vector<size_t> med, cdf, t64, led, ledc;
    std::vector<int> ntx, ntz, tile_base;
    size_t probs = 0, tile_prob = 0, qcnt = 0, tcount = 0, tcursor = 0, jobs = 0, qa = 0, qtile = 0, qb = 0, total = 0;
};

BatchLayout batch_layout(const BatchProblem *pb, int n) {
    BatchLayout B;
    B.tt = tuning_snapshot();
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
    B.cap_a = 2 * B.live + (uint64_t)kSlice * kTileWavesMax + 64ull * 64;
    // a pool below 2^23 live packets spreads over too few jobs of the tuned
    // size to fill the device: half-size jobs (measured on 1e6- and 4e6-packet
    // disc256 gradients: -7%; 4096 stays better for full pools)
    B.job = (B.live < kSmallPool && B.tt.job >= 128) ? B.tt.job / 2 : B.tt.job;
    B.max_jobs = (uint64_t)B.ntiles + B.live / B.job + 2;
    B.probs = off;
    off = align_up(off + (size_t)n * sizeof(ProbDev));
    B.tile_prob = off;
    off = align_up(off + (size_t)B.ntiles * sizeof(uint32_t));
    B.qcnt = off;
    off = align_up(off + 8 * sizeof(uint32_t));
    B.tcount = off;
    off = align_up(off + (size_t)B.ntiles * sizeof(uint32_t));
    B.tcursor = off;
    off = align_up(off + (size_t)B.ntiles * sizeof(uint32_t));
    B.jobs = off;
    off = align_up(off + B.max_jobs * sizeof(uint4));
    B.qa = off;
    off = align_up(off + B.cap_a * sizeof(PacketRec));
    B.qtile = off;
    off = align_up(off + B.cap_a * sizeof(uint32_t));
    B.qb = off;
    off = align_up(off + B.live * sizeof(PacketRec));
    B.total = off;
    return B;
}

// Bound on |packet weight|: a launch weight 2 pi p(s) of an angular profile
// p = c0/2pi + (1/pi) sum (c_n cos nt + s_n sin nt) is at most
// |c0| + 2 sum (|c_n| + |s_n|) (1 without a profile, and for pencils and
// lines); a roulette survivor gains at most the factor m W_th.  The
// equal-count map launch multiplies by q_i / mean |q|, bounded once max |q|
// is known on the device.
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
    // the fixed-point tile tally resolves weights up to 2^32 (see fixed_add)
    if (!(weight_bound(src, n_src, run) <= 0x1p32)) return MC_ERR_UNSUPPORTED;
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
    P.wbound = weight_bound(src, n_src, run);
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
    if (n_src == 1 && src[0].kind == MC_SRC_MAP) {
        P.map = src[0].map_d;
        P.inv_qbar = map_abs_sum > 0 ? (double)P.npix / map_abs_sum : 0.0;
    }
}

// Fixed-point scale of the visit sums (fixed_add): fx = 2^(32 - e) with 2^e
// above the run's weight bound (times max |q| / mean |q| for the equal-count
// map launch), so a segment adds at most sqrt 2 * 2^32 in scaled units; a
// visit is flushed in parts at flush_track * 2^32 <= 2^48, inside 2^51.
mc_status fixed_point(Params &P, double map_abs_max, double flush_track) {
    double wb = P.wbound;
    if ((P.flags & MC_FLAG_EQUAL_COUNT) && P.map) wb *= map_abs_max * P.inv_qbar;
    if (!(wb <= 0x1p32)) return MC_ERR_UNSUPPORTED;
    int e = 0;
    std::frexp(std::max(wb, 1.0), &e);   // 2^e > wb
    P.fx = (float)std::ldexp(1.0, kFixBits - e);
    P.fx_inv = std::ldexp(1.0, e - kFixBits);
    P.flush_at = (float)std::ldexp(flush_track, kFixBits);
    return MC_OK;
}

int occupancy_blocks(const void *fn, int block, size_t lds) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, block, lds) != hipSuccess ||
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

// Record HIP events around a transport launch when timing is on.
struct LaunchTimer {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    bool on = false;
    mc_status begin(hipStream_t s) {
        Profile &pr = profile_state();
        {
            std::lock_guard<std::mutex> g(pr.mu);
            on = pr.on;
        }
        if (!on) return MC_OK;
        if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return MC_ERR_DEVICE;
        return hipEventRecord(e0, s) == hipSuccess ? MC_OK : MC_ERR_DEVICE;
    }
    mc_status end(hipStream_t s) {
        if (!on) return MC_OK;
        if (hipEventRecord(e1, s) != hipSuccess) return MC_ERR_DEVICE;
        Profile &pr = profile_state();
        std::lock_guard<std::mutex> g(pr.mu);
        pr.pending.emplace_back(e0, e1);
        return MC_OK;
    }
};

mc_status set_lds_limit(const void *fn, size_t lds) {
    if (lds <= 64 * 1024) return MC_OK;
    return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) == hipSuccess ? MC_OK
                                                                                                    : MC_ERR_DEVICE;
}

// Whole-grid mode: persistent launches over chunks of packets.
mc_status run_grid(Params &P, const Layout &L, const mc_run *run, char *base, hipStream_t s) {
    const int N = run->n_harm, K = 2 * N + 1;
    const TransportFn fn = kernels().grid[N];
    const size_t lds = (size_t)P.npix * K * sizeof(double);
    mc_status st = set_lds_limit(reinterpret_cast<const void *>(fn), lds);
    if (st != MC_OK) return st;
    const int block = grid_block(N);
    const int occ = occupancy_blocks(reinterpret_cast<const void *>(fn), block, lds);
    const int cus = device_cus();
    for (uint64_t c = 0; c < L.n_chunks; ++c) {
        const uint64_t a = c * kChunk;
        const uint64_t n = std::min<uint64_t>(kChunk, run->n_packets - a);
        P.pid0 = run->first_packet_id + a;
        P.npk = n;
        P.counter = reinterpret_cast<unsigned long long *>(base + L.counters) + c;
        const uint64_t want = (n + block - 1) / block;
        const unsigned grid = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(want, (uint64_t)cus * occ));
        LaunchTimer tm;
        if ((st = tm.begin(s)) != MC_OK) return st;
        hipLaunchKernelGGL(fn, dim3(grid), dim3(block), lds, s, P);
        if ((st = tm.end(s)) != MC_OK) return st;
        if (hipGetLastError() != hipSuccess) return MC_ERR_DEVICE;
    }
    return MC_OK;
}

// Tiled mode: host-driven generations over one packet pool shared by every
// problem of the batch (launch, sort by tile, transport), one stream
// synchronisation per generation to read the queue length.
mc_status run_batch(const BatchProblem *pb, int n, void *ws, size_t ws_bytes, hipStream_t s) {
    for (int i = 0; i < n; ++i) {
        mc_status st = validate(pb[i].m, pb[i].src, pb[i].n_src, pb[i].run);
        if (st != MC_OK) return st;
        if (!pb[i].coeffs || pb[i].run->n_harm != pb[0].run->n_harm) return MC_ERR_INVALID_ARG;
    }
    const BatchLayout B = batch_layout(pb, n);
    if (!ws || ws_bytes < B.total || (reinterpret_cast<uintptr_t>(ws) & 255)) return MC_ERR_WORKSPACE;
    if (B.tile_lds > kLdsTileMax || B.live > 0xFFFFFFFFull / 4) return MC_ERR_UNSUPPORTED;
    char *base = static_cast<char *>(ws);
    const int N = B.N;
    mc_status st;
    // per problem: zero tally and ledger, medium table, CDF of a map source
    std::vector<Params> PP(n);
    std::vector<ProbDev> PD(n);
    std::vector<uint32_t> tile_prob(B.ntiles);
    std::vector<uint64_t> todo(n), launched(n, 0);
    for (int i = 0; i < n; ++i) {
        const mc_medium *m = pb[i].m;
        const int npix = m->nx * m->nz;
        if ((st = launch_zero(base + B.t64[i], (size_t)npix * B.K * sizeof(double), s)) != MC_OK) return st;
        if ((st = launch_zero(base + B.led[i], B.ledc[i] + 8 * sizeof(unsigned long long) - B.led[i], s)) != MC_OK)
            return st;
        hipLaunchKernelGGL(k_setup_medium, dim3((npix + 255) / 256), dim3(256), 0, s, npix, m->dx, m->mua_d,
                           m->mus_d, m->g_d, reinterpret_cast<float4 *>(base + B.med[i]));
        double map_abs_sum = 0, map_abs_max = 0;
        todo[i] = pb[i].run->n_packets;
        if (pb[i].src[0].kind == MC_SRC_MAP) {
            double *cdf = reinterpret_cast<double *>(base + B.cdf[i]);
            hipLaunchKernelGGL(k_map_cdf, dim3(1), dim3(1024), 0, s, npix, pb[i].src[0].map_d, cdf);
            // the normalisation needs sum |q| (the last CDF entry), the weight bound max |q|
            double h2[2];
            if (hipMemcpyAsync(h2, cdf + npix - 1, 2 * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess)
                return MC_ERR_DEVICE;
            map_abs_sum = h2[0];
            map_abs_max = h2[1];
            if (map_abs_sum == 0.0) todo[i] = 0;   // an all-zero source: the field is zero
            else if (!(map_abs_sum > 0)) return MC_ERR_INVALID_ARG;   // NaN in the map
        }
        Params &P = PP[i];
        fill_params(P, m, pb[i].src, pb[i].n_src, pb[i].run, pb[i].adjoint, map_abs_sum);
        if ((st = fixed_point(P, map_abs_max, B.tt.flush_track)) != MC_OK) return st;
        P.med = reinterpret_cast<const float4 *>(base + B.med[i]);
        P.t64 = reinterpret_cast<double *>(base + B.t64[i]);
        P.led = reinterpret_cast<double *>(base + B.led[i]);
        P.ledc = reinterpret_cast<unsigned long long *>(base + B.ledc[i]);
        P.cdf = reinterpret_cast<const double *>(base + B.cdf[i]);
        P.tw = P.th = B.t;
        P.ntx = B.ntx[i];
        P.ntiles = B.ntiles;
        P.tile_base = B.tile_base[i];
        P.prob = (uint32_t)i;
        P.qa = reinterpret_cast<PacketRec *>(base + B.qa);
        P.qtile = reinterpret_cast<uint32_t *>(base + B.qtile);
        P.qb = reinterpret_cast<PacketRec *>(base + B.qb);
        P.qcnt = reinterpret_cast<uint32_t *>(base + B.qcnt);
        P.tile_count = reinterpret_cast<uint32_t *>(base + B.tcount);
        P.tile_cursor = reinterpret_cast<uint32_t *>(base + B.tcursor);
        P.jobs = reinterpret_cast<uint4 *>(base + B.jobs);
        P.probs = reinterpret_cast<const ProbDev *>(base + B.probs);
        P.tile_prob = reinterpret_cast<const uint32_t *>(base + B.tile_prob);
        P.cap_a = (uint32_t)B.cap_a;
        P.cap_b = (uint32_t)B.live;
        P.job_size = B.job;
        P.max_visits = B.tt.maxvis;
        P.tail_visits = B.tt.tailvis;
        ProbDev &d = PD[i];
        d.nx = m->nx;
        d.nz = m->nz;
        d.ntx = B.ntx[i];
        d.tile_base = B.tile_base[i];
        d.tag = P.tag;
        d.flags = P.flags;
        d.seed = P.seed;
        d.wth = P.wth;
        d.rm = P.rm;
        d.inv_rm = P.inv_rm;
        d.flush_at = P.flush_at;
        d.fx = P.fx;
        d.fx_inv = P.fx_inv;
        d.med = P.med;
        d.g = P.g;
        d.t64 = P.t64;
        d.led = P.led;
        d.ledc = P.ledc;
        for (int k = 0; k < B.ntx[i] * B.ntz[i]; ++k) tile_prob[B.tile_base[i] + k] = (uint32_t)i;
    }
    if ((st = launch_zero(base + B.qcnt, 8 * sizeof(uint32_t), s)) != MC_OK) return st;
    if ((st = launch_zero(base + B.tcount, (size_t)B.ntiles * sizeof(uint32_t), s)) != MC_OK) return st;
    if (hipMemcpyAsync(base + B.probs, PD.data(), (size_t)n * sizeof(ProbDev), hipMemcpyHostToDevice, s) !=
            hipSuccess ||
        hipMemcpyAsync(base + B.tile_prob, tile_prob.data(), (size_t)B.ntiles * sizeof(uint32_t),
                       hipMemcpyHostToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)   // the host arrays go out of scope below
        return MC_ERR_DEVICE;
    if (hipGetLastError() != hipSuccess) return MC_ERR_DEVICE;

    const TransportFn fn = kernels().tile[N];
    if ((st = set_lds_limit(reinterpret_cast<const void *>(fn), B.tile_lds)) != MC_OK) return st;
    const int occ = occupancy_blocks(reinterpret_cast<const void *>(fn), kBlockTile, B.tile_lds);
    const int cus = device_cus();
    const unsigned tgrid = (unsigned)std::max(1, std::min(cus * occ, kTileWavesMax / (kBlockTile / 64)));
    const unsigned bgrid = (unsigned)std::min<uint64_t>((B.cap_a + 255) / 256, 4096);
    const unsigned cgrid = (unsigned)std::min<uint64_t>((B.cap_a + 255) / 256, 4 * (uint64_t)cus);
    const Params &P0 = PP[0];   // the sort and transport kernels read only batch-wide fields
    static thread_local uint32_t *host_cnt = nullptr;   // two slots of the 8 queue counters
    if (!host_cnt && hipHostMalloc(reinterpret_cast<void **>(&host_cnt), 16 * sizeof(uint32_t)) != hipSuccess)
        return MC_ERR_DEVICE;
    struct CountEvents {   // one event per counter slot, on the device of this call
        hipEvent_t e[2] = {nullptr, nullptr};
        ~CountEvents() {
            for (hipEvent_t x : e)
                if (x) (void)hipEventDestroy(x);
        }
    } cev;
    for (hipEvent_t &x : cev.e)
        if (hipEventCreateWithFlags(&x, hipEventDisableTiming) != hipSuccess) return MC_ERR_DEVICE;
    // the tail is handed to the finisher at a fixed count (the tuning's pool
    // size / 128, 131072 by default) whatever the run's size: a small run whose
    // pool is small would otherwise spend hundreds of latency-bound
    // generations on its last few thousand packets (measured: a 1e6-packet
    // disc256 gradient 241 -> 173 ms)
    const uint64_t finish_at = B.tt.finish ? B.tt.finish : std::min<uint64_t>(kFinishMax, B.tt.live / 128);
    uint64_t total_todo = 0, total_launched = 0, carried = 0;
    uint32_t n_rec = 0;   // records in the unsorted queue after the last generation read
    for (int i = 0; i < n; ++i) total_todo += todo[i];
    // one generation: sort the queue by tile, transport, then the queue
    // counters are copied to host slot `slot` and its event recorded
    auto enqueue_gen = [&](int slot) -> mc_status {
        hipLaunchKernelGGL(k_bin_count, dim3(cgrid), dim3(256), 0, s, P0);
        hipLaunchKernelGGL(k_bin_scan, dim3(1), dim3(1024), 0, s, P0);
        hipLaunchKernelGGL(k_bin_scatter, dim3(bgrid), dim3(256), 0, s, P0);
        LaunchTimer tm;
        mc_status r;
        if ((r = tm.begin(s)) != MC_OK) return r;
        hipLaunchKernelGGL(fn, dim3(tgrid), dim3(kBlockTile), B.tile_lds, s, P0);
        if ((r = tm.end(s)) != MC_OK) return r;
        if (hipGetLastError() != hipSuccess) return MC_ERR_DEVICE;
        if (hipMemcpyAsync(host_cnt + 8 * slot, P0.qcnt, 8 * sizeof(uint32_t), hipMemcpyDeviceToHost, s) !=
                hipSuccess ||
            hipEventRecord(cev.e[slot], s) != hipSuccess)
            return MC_ERR_DEVICE;
        return MC_OK;
    };
    auto read_gen = [&](int slot) -> mc_status {
        if (hipEventSynchronize(cev.e[slot]) != hipSuccess) return MC_ERR_DEVICE;
        const uint32_t *c = host_cnt + 8 * slot;
        if (c[4]) return MC_ERR_DEVICE;   // queue overflow (not expected by construction)
        carried = c[6];   // valid records; qa also holds the padding of partly used slices
        n_rec = (uint32_t)std::min<uint64_t>(c[0], B.cap_a);
        return MC_OK;
    };
    // Refill phase: one generation at a time, each refill sized by the count
    // the previous generation left.
    for (uint64_t gen = 0; total_launched < total_todo; ++gen) {
        if (gen > (1ull << 32)) return MC_ERR_DEVICE;
        uint64_t budget = carried < B.live ? B.live - carried : 0;
        for (int i = 0; i < n && budget; ++i) {   // refill the pool, problems in order
            const uint64_t n_new = std::min<uint64_t>(budget, todo[i] - launched[i]);
            if (!n_new) continue;
            const unsigned lgrid = (unsigned)std::min<uint64_t>((n_new + 255) / 256, 8 * (uint64_t)cus);
            hipLaunchKernelGGL(k_tile_launch, dim3(lgrid), dim3(256), 0, s, PP[i],
                               pb[i].run->first_packet_id + launched[i], (uint32_t)n_new);
            launched[i] += n_new;
            total_launched += n_new;
            budget -= n_new;
        }
        if (total_launched == total_todo) break;   // this generation is the drain's first
        if ((st = enqueue_gen(0)) != MC_OK || (st = read_gen(0)) != MC_OK) return st;
    }
    // Drain phase (every packet launched): generations run back to back, the
    // host reading one generation's counters while the next already runs on
    // its output, so the device does not wait for the host in between.  Once
    // at most finish_at packets remain, the generation in flight completes and
    // the finisher takes what it leaves.
    if (total_todo > 0) {
        int inflight = 0, head = 0;   // generations enqueued and not yet read; slot of the oldest
        for (uint64_t gen = 0;; ++gen) {
            if (gen > (1ull << 32)) return MC_ERR_DEVICE;
            while (inflight < 2) {
                if ((st = enqueue_gen((head + inflight) & 1)) != MC_OK) return st;
                ++inflight;
            }
            if ((st = read_gen(head)) != MC_OK) return st;
            head ^= 1;
            --inflight;
            if (carried <= finish_at) {
                if ((st = read_gen(head)) != MC_OK) return st;
                break;
            }
        }
    }
    if (carried > 0) {
        // finish the remaining packets without migration, one launch per
        // problem (each takes only its own records; qcnt[5]: record cursor)
        const FinishFn ff = kernels().fin[N];
        const size_t flds = (size_t)(kBlockFinish / 64) * 64 * (2 * N + 1) * sizeof(float) +
                            (kBlockFinish / 64) * 64 * sizeof(int);
        if ((st = set_lds_limit(reinterpret_cast<const void *>(ff), flds)) != MC_OK) return st;
        const int focc = occupancy_blocks(reinterpret_cast<const void *>(ff), kBlockFinish, flds);
        const unsigned fgrid = (unsigned)std::max<uint64_t>(
            1, std::min<uint64_t>((carried + kBlockFinish - 1) / kBlockFinish, (uint64_t)cus * focc));
        for (int i = 0; i < n; ++i) {
            if (!todo[i]) continue;
            if ((st = launch_zero(PP[i].qcnt + 5, sizeof(uint32_t), s)) != MC_OK) return st;
            LaunchTimer tf;
            if ((st = tf.begin(s)) != MC_OK) return st;
            hipLaunchKernelGGL(ff, dim3(fgrid), dim3(kBlockFinish), flds, s, PP[i], n_rec);
            if ((st = tf.end(s)) != MC_OK) return st;
            if (hipGetLastError() != hipSuccess) return MC_ERR_DEVICE;
        }
    }
    // normalisation and ledgers
    for (int i = 0; i < n; ++i) {
        const mc_medium *m = pb[i].m;
        const int npix = m->nx * m->nz;
        const double scale = PP[i].total / ((double)pb[i].run->n_packets);
        hipLaunchKernelGGL(k_normalise, dim3((npix + 255) / 256), dim3(256), 0, s, npix, N, pb[i].adjoint,
                           todo[i] ? scale / (double)m->dx : 0.0, PP[i].t64, PP[i].ledc + 4, pb[i].coeffs);
        if (pb[i].ledger)
            hipLaunchKernelGGL(k_ledger_out, dim3(1), dim3(1), 0, s, PP[i].led, PP[i].ledc, todo[i] ? scale : 0.0,
                               pb[i].ledger);
    }
    return hipGetLastError() == hipSuccess ? MC_OK : MC_ERR_DEVICE;
}

mc_status run_mc(const mc_medium *m, const mc_source *src, int n_src, const mc_run *run, double *coeffs,
                 mc_ledger *ledger, void *ws, size_t ws_bytes, void *stream, int adjoint) {
    mc_status st = validate(m, src, n_src, run);
    if (st != MC_OK) return st;
    if (!coeffs) return MC_ERR_INVALID_ARG;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (is_tiled(m, run, tuning_snapshot())) {
        const BatchProblem one{m, src, n_src, run, adjoint, coeffs, ledger};
        return run_batch(&one, 1, ws, ws_bytes, s);
    }
    const Layout L = layout(m, src, run);
    if (!ws || ws_bytes < L.total || (reinterpret_cast<uintptr_t>(ws) & 255)) return MC_ERR_WORKSPACE;
    char *base = static_cast<char *>(ws);
    const int npix = m->nx * m->nz;
    const int N = run->n_harm;

    // zero the tally, ledger and chunk counters
    if ((st = launch_zero(base + L.t64, L.counters + L.n_chunks * sizeof(unsigned long long) - L.t64, s)) != MC_OK)
        return st;
    hipLaunchKernelGGL(k_setup_medium, dim3((npix + 255) / 256), dim3(256), 0, s, npix, m->dx, m->mua_d, m->mus_d, m->g_d,
                       reinterpret_cast<float4 *>(base + L.med));
    double map_abs_sum = 0, map_abs_max = 0;
    if (src[0].kind == MC_SRC_MAP) {
        double *cdf = reinterpret_cast<double *>(base + L.cdf);
        hipLaunchKernelGGL(k_map_cdf, dim3(1), dim3(1024), 0, s, npix, src[0].map_d, cdf);
        // the normalisation needs sum |q| (the last CDF entry), the weight bound max |q|
        double h2[2];
        if (hipMemcpyAsync(h2, cdf + npix - 1, 2 * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return MC_ERR_DEVICE;
        map_abs_sum = h2[0];
        map_abs_max = h2[1];
        if (map_abs_sum == 0.0) {   // an all-zero source: the field is zero
            st = launch_zero(coeffs, (size_t)npix * (2 * N + 1) * sizeof(double), s);
            if (st == MC_OK && ledger) st = launch_zero(ledger, sizeof(mc_ledger), s);
            return st;
        }
        if (!(map_abs_sum > 0)) return MC_ERR_INVALID_ARG;   // NaN in the map
    }
    if (hipGetLastError() != hipSuccess) return MC_ERR_DEVICE;
    Params P;
    fill_params(P, m, src, n_src, run, adjoint, map_abs_sum);
    if ((st = fixed_point(P, map_abs_max, tuning_snapshot().flush_track)) != MC_OK) return st;
    P.med = reinterpret_cast<const float4 *>(base + L.med);
    P.t64 = reinterpret_cast<double *>(base + L.t64);
    P.led = reinterpret_cast<double *>(base + L.led);
    P.ledc = reinterpret_cast<unsigned long long *>(base + L.ledc);
    P.cdf = reinterpret_cast<const double *>(base + L.cdf);

    st = run_grid(P, L, run, base, s);
    if (st != MC_OK) return st;
    const double scale = P.total / ((double)run->n_packets);
    hipLaunchKernelGGL(k_normalise, dim3((npix + 255) / 256), dim3(256), 0, s, npix, N, adjoint,
                       scale / (double)m->dx, P.t64, P.ledc + 4, coeffs);
    if (ledger)
        hipLaunchKernelGGL(k_ledger_out, dim3(1), dim3(1), 0, s, P.led, P.ledc, scale, ledger);
    return hipGetLastError() == hipSuccess ? MC_OK : MC_ERR_DEVICE;
}

// Discrete-ordinates runs (mc_run_binned): medium, CDF of a map source, raw
// bins [n_bins][npix], ledger and per-chunk packet counters.
struct BinnedLayout {
    size_t med, cdf, raw, led, ledc, counters, total;
    uint64_t n_chunks;
};

BinnedLayout binned_layout(const mc_medium *m, const mc_source *src, const mc_run *run, int n_bins) {
    BinnedLayout L{};
    const size_t npix = (size_t)m->nx * m->nz;
    size_t off = 0;
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
    hipLaunchKernelGGL(k_setup_medium, dim3((npix + 255) / 256), dim3(256), 0, s, npix, m->dx, m->mua_d, m->mus_d,
                       m->g_d, reinterpret_cast<float4 *>(base + L.med));
    double map_abs_sum = 0;
    if (src[0].kind == MC_SRC_MAP) {
        double *cdf = reinterpret_cast<double *>(base + L.cdf);
        hipLaunchKernelGGL(k_map_cdf, dim3(1), dim3(1024), 0, s, npix, src[0].map_d, cdf);
        if (hipMemcpyAsync(&map_abs_sum, cdf + npix - 1, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return MC_ERR_DEVICE;
        if (map_abs_sum == 0.0) {   // an all-zero source: the field is zero
            st = launch_zero(out, nout * sizeof(double), s);
            if (st == MC_OK && ledger) st = launch_zero(ledger, sizeof(mc_ledger), s);
            return st;
        }
        if (!(map_abs_sum > 0)) return MC_ERR_INVALID_ARG;   // NaN in the map
    }
    Params P;
    fill_params(P, m, src, n_src, run, adjoint, map_abs_sum);
    P.med = reinterpret_cast<const float4 *>(base + L.med);
    P.led = reinterpret_cast<double *>(base + L.led);
    P.ledc = reinterpret_cast<unsigned long long *>(base + L.ledc);
    P.cdf = reinterpret_cast<const double *>(base + L.cdf);
    double *raw = reinterpret_cast<double *>(base + L.raw);
    const int cus = device_cus();
    const int occ = occupancy_blocks(reinterpret_cast<const void *>(&k_transport_binned), 256, 0);
    for (uint64_t c = 0; c < L.n_chunks; ++c) {
        const uint64_t a = c * kChunk;
        const uint64_t n = std::min<uint64_t>(kChunk, run->n_packets - a);
        P.pid0 = run->first_packet_id + a;
        P.npk = n;
        P.counter = reinterpret_cast<unsigned long long *>(base + L.counters) + c;
        const unsigned grid = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>((n + 255) / 256, (uint64_t)cus * occ));
        hipLaunchKernelGGL(k_transport_binned, dim3(grid), dim3(256), 0, s, P, n_bins, raw);
        if (hipGetLastError() != hipSuccess) return MC_ERR_DEVICE;
    }
    // as the coefficients (source measure / packets, track length in pixel
    // units over the pixel area), per unit angle of the bin
    const double scale = P.total / (double)run->n_packets;
    const double bw = 2.0 * M_PI / n_bins;
    hipLaunchKernelGGL(k_binned_normalise, dim3((unsigned)((nout + 255) / 256)), dim3(256), 0, s, npix, n_bins, adjoint,
                       scale / (double)m->dx / bw, raw, out);
    if (ledger) hipLaunchKernelGGL(k_ledger_out, dim3(1), dim3(1), 0, s, P.led, P.ledc, scale, ledger);
    return hipGetLastError() == hipSuccess ? MC_OK : MC_ERR_DEVICE;
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

size_t mc_workspace_bytes(const mc_medium *medium, const mc_source *src, int n_src, const mc_run *run) {
    if (validate(medium, src, n_src, run) != MC_OK) return 0;
    if (is_tiled(medium, run, tuning_snapshot())) {
        const BatchProblem one{medium, src, n_src, run, 0, nullptr, nullptr};
        return batch_layout(&one, 1).total;
    }
    return layout(medium, src, run).total;
}

size_t mc_batch_workspace_bytes(const mc_problem *probs, int n_probs) {
    if (!probs || n_probs < 1 || n_probs > MC_BATCH_MAX) return 0;
    std::vector<BatchProblem> pb(n_probs);
    for (int i = 0; i < n_probs; ++i) {
        const mc_problem &q = probs[i];
        if (validate(&q.medium, q.src, q.n_src, &q.run) != MC_OK || q.run.n_harm != probs[0].run.n_harm) return 0;
        pb[i] = BatchProblem{&q.medium, q.src, q.n_src, &q.run, q.adjoint ? 1 : 0, q.coeffs_d, q.ledger_d};
    }
    return batch_layout(pb.data(), n_probs).total;
}

mc_status mc_run_batch(const mc_problem *probs, int n_probs, void *workspace_d, size_t workspace_bytes,
                       void *stream) {
    if (!probs || n_probs < 1 || n_probs > MC_BATCH_MAX) return MC_ERR_INVALID_ARG;
    std::vector<BatchProblem> pb(n_probs);
    for (int i = 0; i < n_probs; ++i) {
        const mc_problem &q = probs[i];
        pb[i] = BatchProblem{&q.medium, q.src, q.n_src, &q.run, q.adjoint ? 1 : 0, q.coeffs_d, q.ledger_d};
    }
    return run_batch(pb.data(), n_probs, workspace_d, workspace_bytes, reinterpret_cast<hipStream_t>(stream));
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
    hipLaunchKernelGGL(k_setup_medium, dim3((npix + 255) / 256), dim3(256), 0, 0, npix, m->dx, m->mua_d, m->mus_d, m->g_d,
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

mc_status mc_set_tuning(const mc_tuning *t) {
    TileTuning v;   // defaults
    if (t) {
        if (t->live_packets < 1024 || t->live_packets > (1ull << 26) || t->job_packets < 64 ||
            t->job_packets > (1u << 20) || t->max_visits < 1 || t->tile > 256 || t->finish_packets > (1ull << 26) ||
            !(t->flush_track >= 0.f && t->flush_track <= (float)kFlushTrackMax) || t->tail_visits > (1u << 30))
            return MC_ERR_INVALID_ARG;
        v.live = t->live_packets;
        v.grid_max = t->grid_max_packets ? t->grid_max_packets : kGridMaxPackets;
        v.job = t->job_packets;
        v.maxvis = t->max_visits;
        v.tile = (int)t->tile;
        v.finish = t->finish_packets;
        v.flush_track = t->flush_track > 0.f ? (double)t->flush_track : kFlushTrackMax;
        v.tailvis = t->tail_visits ? t->tail_visits : kTailVisits;
    }
    TuningState &s = tuning_state();
    std::lock_guard<std::mutex> g(s.mu);
    s.t = v;
    return MC_OK;
}

mc_status mc_get_tuning(mc_tuning *t) {
    if (!t) return MC_ERR_INVALID_ARG;
    const TileTuning v = tuning_snapshot();
    t->live_packets = v.live;
    t->job_packets = v.job;
    t->max_visits = v.maxvis;
    t->tile = (uint32_t)v.tile;
    t->finish_packets = v.finish;
    t->grid_max_packets = (uint32_t)std::min<uint64_t>(v.grid_max, 0xFFFFFFFFull);
    t->flush_track = (float)v.flush_track;
    t->tail_visits = v.tailvis;
    return MC_OK;
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
    return "librmc gfx950: FP32 transport; 64-bit fixed-point tally in LDS (whole grid when it fits, else square "
           "tiles with packet migration between tiles), added to an FP64 HBM map";
}

}  // extern "C"
