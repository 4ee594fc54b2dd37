/*
 * mcrad.h -- C ABI of librmc.so: forward and adjoint Monte Carlo of radiance
 * in a 2D pixelated medium with a harmonic angular tally, and the functional
 * gradients built from it, on one AMD Instinct MI355X (gfx950).
 *
 * The method is that of Hochuli, Powell, Arridge & Cox, "Quantitative
 * photoacoustic tomography using forward and adjoint Monte Carlo models of
 * radiance" (arXiv:1608.05238).  Each entry point names the section and
 * equation it implements.
 *
 * General rules
 *  - Every array argument whose name ends in _d is a DEVICE pointer owned by
 *    the caller; the library never allocates, frees or keeps it.  Host
 *    pointers end in _h.
 *  - Calls that take a stream only enqueue work on that stream and return:
 *    none of them waits for the device, allocates device memory or keeps
 *    state between calls (mc_trace, which is synchronous, is the one
 *    exception and says so).  Results are valid after the caller
 *    synchronises the stream.  Calls on different streams with different
 *    workspaces may run concurrently.  The library holds no mutable global
 *    state: tuning and timing are passed per call (mc_options).
 *  - Return value: MC_OK, or an error code; no call throws.  Invalid
 *    arguments are detected on the host before anything is enqueued.
 *    MC_ERR_DEVICE reports a failed launch; faults inside a kernel surface at
 *    the caller's next synchronisation.  What only the device can see -- a
 *    NaN in a source map, a weight bound above 2^32 that only the map's
 *    values reveal, a packet queue that overflowed (not reachable by
 *    construction) -- turns the whole output of the run into NaN.
 *  - Maps are row-major [nz][nx]: x (lateral) is the column, z (depth) the
 *    row.  Pixel (ix,iz) covers [ix dx,(ix+1) dx) x [iz dx,(iz+1) dx).
 *  - Harmonic coefficient maps are planar [2N+1][nz][nx] FP64 in the order
 *    a0, a1..aN, b1..bN, with the radiance expansion of Sec. 3.1
 *    (eq. radiance_Fourier): phi = a0/2pi + (1/pi) sum_n (a_n cos n t + b_n sin n t),
 *    t measured from +z towards +x, so a_n = int phi cos(n t) dt.  Each value
 *    is the average over the pixel, per unit source power.
 */
#ifndef MCRAD_H
#define MCRAD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MC_NHARM_MAX 32

typedef enum {
    MC_OK = 0,
    MC_ERR_INVALID_ARG = 1,   /* a size, pointer or parameter is out of range */
    MC_ERR_UNSUPPORTED = 2,   /* a valid request this library does not serve */
    MC_ERR_DEVICE = 3,        /* a HIP call or launch failed */
    MC_ERR_WORKSPACE = 4,     /* workspace missing or smaller than mc_workspace_bytes() */
    MC_ERR_SCRATCH = 5        /* mc_run_noalloc: the run's workspace exceeds MC_SCRATCH_BYTES */
} mc_status;

/* Optical properties (Sec. 2 and 3): device FP32 maps [nz][nx] of the
 * absorption and scattering coefficients (1/mm, >= 0) and the 2D
 * Henyey-Greenstein anisotropy g in (-1, 1].  dx: pixel side in mm. */
typedef struct {
    int32_t nx, nz;
    float dx;
    const float *mua_d, *mus_d, *g_d;
} mc_medium;

typedef enum {
    MC_SRC_PENCIL = 0,   /* collimated beam at (x0,z0) along (dir_x,dir_z) */
    MC_SRC_LINE = 1,     /* segment (x0,z0)-(x1,z1); collimated along dir, or Lambertian about it */
    MC_SRC_POINT = 2,    /* point (x0,z0) with angular profile prof (default isotropic) */
    MC_SRC_MAP = 3       /* volumetric q(x) per unit angle per unit area, angular profile prof */
} mc_source_kind;

/* A light source (Sec. 3, 3.2, 4.1, 6.1) or, for mc_adjoint, an adjoint
 * source (Sec. 4, 6).  Positions in mm, inside [0, nx dx] x [0, nz dx].
 * Several non-MAP sources may be given together: each packet picks one with
 * probability proportional to its power.  A MAP source must be the only one.
 *  prof_h: host array [2 n_prof + 1] = c0, c1..cn, s1..sn giving the angular
 *    profile p(t) = c0/2pi + (1/pi) sum (c_n cos n t + s_n sin n t); NULL
 *    means isotropic (p = 1/2pi).  A POINT source emits power * p(t) per unit
 *    angle; a MAP source emits map(x) * 2pi p(t).  Packets of these two kinds
 *    are launched at a uniform angle with weight 2pi p(t) (times the sign of
 *    the map value), so p may be signed.
 *  map_d: device FP64 [nz][nx] (MAP only), may be signed (adjoint source);
 *    an all-zero map is a source of zero power: the output is zero. */
typedef struct {
    int32_t kind;            /* mc_source_kind */
    float x0, z0, x1, z1;
    float dir_x, dir_z;      /* unit vector */
    int32_t lambertian;      /* LINE: 0 collimated, 1 Lambertian about dir */
    double power;            /* PENCIL/LINE/POINT: > 0 */
    const double *map_d;
    int32_t n_prof;          /* 0..MC_NHARM_MAX */
    const double *prof_h;
} mc_source;

#define MC_FLAG_LITERAL_TRUNCATION 1u  /* stop below the threshold (Sec. 3) instead of roulette */
#define MC_FLAG_EQUAL_COUNT 2u         /* MAP source (Sec. 6 read literally): every pixel equally likely and
                                          the packet weight scaled by q_i / mean |q| (default: pixels drawn
                                          in proportion to |q_i|, weight sign(q_i)); same normalisation.
                                          Packets drawn in a pixel with q = 0 carry nothing and end at once */

/* One Monte Carlo run.  Packet p (first_packet_id <= p < first_packet_id +
 * n_packets) draws its random numbers from Philox4x32-10 with key = seed and
 * counter = (j, stream_tag, p_lo, p_hi): block j = 0 launches it, block k >= 1
 * gives the k-th free path (u0), the scattering angle at its end (u1) and the
 * roulette draw there (u2); u = ((x >> 9) + 0.5) 2^-23.  The result is a
 * pure function of (inputs, seed, stream_tag, packet range). */
typedef struct {
    uint64_t n_packets;        /* >= 1 */
    uint64_t seed;
    uint64_t first_packet_id;
    uint32_t stream_tag;
    int32_t n_harm;            /* N in [0, MC_NHARM_MAX]: K = 2N+1 channels */
    float w_threshold;         /* roulette below w_threshold * |W0| (e.g. 1e-4) */
    float roulette_m;          /* > 1: survive with probability 1/m, weight * m */
    uint32_t flags;            /* MC_FLAG_* */
} mc_run;

/* Energy ledger of one run (device struct written by mc_forward/mc_adjoint).
 * Weight sums are raw packet-weight sums; multiply by `scale` (total source
 * measure / n_packets) for power.  launched + roulette_gain - roulette_loss
 * equals absorbed + escaped up to FP32 rounding.  generations: tiled
 * transport generations the run used before its tail went to the finisher
 * (0 for the whole-grid transport). */
typedef struct {
    double launched, absorbed, escaped, roulette_gain, roulette_loss;
    double scale;
    uint64_t packets, segments, visits, scatters, generations;
} mc_ledger;

/* Tuning of the tiled transport (grids whose tally exceeds one workgroup's
 * LDS).  Results do not depend on these values (bitwise while the FP64 sums
 * are exact, see mc_forward), except flush_track, which moves FP32 partial
 * sums.  A zero field takes its default (mc_default_tuning).
 *  live_packets   packets kept alive per generation, 1024 .. 2^26 (default 2^26)
 *  job_packets    packets of one tile handed to one workgroup, 64 .. 2^20
 *                 (a run or batch whose pool holds fewer than 2^23 live
 *                 packets uses half that, to spread over more workgroups;
 *                 default 16384)
 *  max_visits     visits in one tile before a packet pauses until the next
 *                 generation, >= 1 (default 64)
 *  tile           tile side in pixels, 1 .. 256 (default, or a tile whose
 *                 tally does not fit: the largest square tile whose tally
 *                 fits the LDS of one workgroup per CU, 23 at N = 16)
 *  finish_packets once every packet is launched and at most this many remain
 *                 they finish without migration (default: the smaller of
 *                 2^16 and live_packets / 128)
 *  grid_max_packets  a run whose tally fits one workgroup's LDS uses the
 *                 whole-grid kernel only up to this many packets, larger runs
 *                 the tiled transport (default 2^21)
 *  flush_track    a pixel visit whose accumulated track length, in units of
 *                 the run's weight bound, exceeds this many pixels is added
 *                 to the tile tally in parts, 0 .. 65536 (default 65536)
 *  tail_visits    once a job has turned quiet (quiet_percent), its packets
 *                 pause after this many more visits, 0 .. 2^30 (default 1)
 *  max_generations  tiled generations enqueued per call, 1 .. 65536
 *                 (default 0: 100, plus 30 per tile along the longest
 *                 grid side of any problem, plus 48 per pool of
 *                 live_packets the run's packets fill).  The host enqueues this many without
 *                 waiting; a generation that finds the finisher threshold
 *                 reached does nothing.  Packets still in flight (or not yet
 *                 launched) after the last one are moved to their end by the
 *                 finisher, so the results never depend on it.
 *  min_job_packets  a generation whose records would not give every
 *                 workgroup of the tiled kernel two jobs cuts its tiles into
 *                 smaller jobs, down to this size, 64 .. 2^20 (default 1024)
 *  quiet_percent  a job turns quiet once the packets whose stay in its tile
 *                 has not ended number at most this percent of
 *                 min(job packets, threads of a tile workgroup: 1024 for
 *                 N <= 16, else 512); its packets then pause after
 *                 tail_visits more visits, 1 .. 100 (default 50) */
typedef struct {
    uint64_t live_packets;
    uint32_t job_packets;
    uint32_t max_visits;
    uint32_t tile;
    uint32_t grid_max_packets;
    uint64_t finish_packets;
    float flush_track;
    uint32_t tail_visits;
    uint32_t max_generations;
    uint32_t min_job_packets;
    uint32_t quiet_percent;
    uint32_t reserved;   /* must be 0 */
} mc_tuning;

/* The built-in defaults, every field filled in. */
mc_status mc_default_tuning(mc_tuning *tuning_h);

/* Timing of transport kernel launches, owned by the caller: a run given a
 * timer brackets each of its transport launches with two HIP events recorded
 * on its stream.  mc_timer_read waits for the recorded events, adds their
 * elapsed times to the timer's total and returns the total (ms) and the
 * number of launches since the last reset.  A timer may serve several calls
 * in turn; it is not shared with anything else. */
typedef struct mc_timer mc_timer;
mc_status mc_timer_create(mc_timer **timer_h);
mc_status mc_timer_destroy(mc_timer *timer);
mc_status mc_timer_read(mc_timer *timer, double *transport_ms, uint64_t *launches, int reset);

/* Per-call options: either pointer may be NULL (defaults, no timing); opts
 * itself may be NULL. */
typedef struct {
    const mc_tuning *tuning;
    mc_timer *timer;
} mc_options;

/* Bytes of device workspace a forward/adjoint run needs (tallies, packet
 * queues, source tables).  0 on invalid arguments. */
size_t mc_workspace_bytes(const mc_medium *medium, const mc_source *src, int n_src, const mc_run *run,
                          const mc_options *opts);

/* Forward radiance MC (Sec. 3, 3.1): launch, exponential free paths through
 * the pixels, continuous absorption weighting, roulette, 2D Henyey-Greenstein
 * scattering (eqs. scattering2D, scattering_angle), and the harmonic
 * track-length tally (eq. Fourier_terms) normalised by the packet count
 * (Sec. 6).  coeffs_d: FP64 [2N+1][nz][nx] (overwritten).  ledger_d: device
 * mc_ledger or NULL.  workspace_d: >= mc_workspace_bytes() bytes, 256-byte
 * aligned; its contents are scratch.
 * Tally precision: each pixel visit is summed in FP32 registers; the map is
 * FP64.  The visits are staged in LDS (the whole grid when its tally fits
 * one workgroup, else square tiles) as 64-bit fixed-point sums of
 * value * 2^(32-e), where 2^e bounds the largest packet weight of the run
 * (the source profile bound |c0| + 2 sum |c_n|, times max(1, m W_th) for
 * roulette survivors, times max|q| / mean|q| for the equal-count map
 * launch): every visit is rounded to a multiple of 2^(e-32) before the FP64
 * sum, which is then exact while a pixel's total stays below 2^(21+e), so
 * the output does not depend on the order in which visits are added (it is
 * bitwise reproducible).  A run whose weight bound exceeds 2^32 returns
 * MC_ERR_UNSUPPORTED.  Should a tile's sums ever risk leaving the 64-bit
 * range (not reachable with physical media and the default tuning), the
 * whole output of the run is NaN rather than wrong. */
mc_status mc_forward(const mc_medium *medium, const mc_source *src, int n_src, const mc_run *run,
                     const mc_options *opts, double *coeffs_d, mc_ledger *ledger_d, void *workspace_d,
                     size_t workspace_bytes, void *stream);

/* Adjoint radiance MC (Sec. 4, eq. adjoint_RTE1; Sec. 6): solves the adjoint
 * RTE with source `src` (typically one MAP source q* from mc_residual).  The
 * adjoint field equals the forward field of the direction-mirrored source
 * read at the mirrored direction: source profiles and collimated directions
 * are mirrored on input and the output orders n >= 1 are multiplied by
 * (-1)^n, so coeffs_d holds the adjoint radiance phi*(x, s) itself. */
mc_status mc_adjoint(const mc_medium *medium, const mc_source *src, int n_src, const mc_run *run,
                     const mc_options *opts, double *coeffs_d, mc_ledger *ledger_d, void *workspace_d,
                     size_t workspace_bytes, void *stream);

/* One problem of a batch: a forward (adjoint = 0, as mc_forward) or adjoint
 * (adjoint = 1, as mc_adjoint) run with its own medium, sources, packet
 * range, seed and stream tag.  coeffs_d: FP64 [2N+1][nz][nx] out;
 * ledger_d: device mc_ledger or NULL.  Every problem of a batch has the
 * same n_harm. */
typedef struct {
    mc_medium medium;
    const mc_source *src;
    int32_t n_src;
    mc_run run;
    int32_t adjoint;
    double *coeffs_d;
    mc_ledger *ledger_d;
} mc_problem;

#define MC_BATCH_MAX 4096

/* Workspace bytes of mc_run_batch (0 on invalid arguments). */
size_t mc_batch_workspace_bytes(const mc_problem *probs_h, int n_probs, const mc_options *opts);

/* Many problems (sources, wavelengths, grid sizes) in one packet pool: the
 * tiled transport's generations launch packets of every problem, sort all of
 * them by tile over one tile index space, and each workgroup job moves the
 * packets of one tile of one problem with that problem's medium and tally in
 * LDS.  Every problem's output equals what mc_forward / mc_adjoint gives for
 * it alone (the same packets and visit values; bitwise while the FP64 sums
 * are exact, see mc_forward).  probs_h: host array of n_probs (1 .. MC_BATCH_MAX) problems. */
mc_status mc_run_batch(const mc_problem *probs_h, int n_probs, const mc_options *opts, void *workspace_d,
                       size_t workspace_bytes, void *stream);

/* For callers that cannot allocate device memory -- code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation: a forward
 * (adjoint = 0, as mc_forward) or adjoint (adjoint = 1, as mc_adjoint) run
 * whose workspace is the library's own static device array of
 * MC_SCRATCH_BYTES, which each GPU the library runs on holds until the
 * process ends.  The caller passes inputs and outputs only.  The call
 * allocates nothing (no device, host or pinned memory, no events:
 * opts->timer must be NULL, else MC_ERR_INVALID_ARG) and, like every entry
 * point, does not wait for the device.  Unless opts->tuning sets
 * live_packets, the tiled transport keeps the largest pool of live packets
 * whose queues fit the scratch; the results equal mc_forward's / mc_adjoint's
 * (bitwise while the FP64 sums are exact).  A run whose workspace exceeds
 * MC_SCRATCH_BYTES even with the smallest pool (1024 live packets), or with
 * the caller's live_packets, returns MC_ERR_SCRATCH before anything is
 * enqueued.  Every call on one GPU uses that GPU's one array and overwrites
 * it (the call's own kernels clear what must start at zero): calls that
 * overlap on one GPU -- on different streams, or from different threads --
 * race and give wrong results; serialise them (one stream, or events). */
#define MC_SCRATCH_BYTES (256ull << 20)
mc_status mc_run_noalloc(const mc_medium *medium, const mc_source *src, int n_src, const mc_run *run, int adjoint,
                         const mc_options *opts, double *coeffs_d, mc_ledger *ledger_d, void *stream);

/* Residual (Sec. 2 eq. error_function3, Sec. 6): H = mua a0 (Grueneisen 1),
 * r = hmeas - H, q* = mua r (per unit angle), eps = (dx^2 / 2) sum r^2.
 * coeffs_d: forward FP64 [>=1][nz][nx] (only a0 is read); hmeas_d FP64
 * [nz][nx]; q_star_d FP64 [nz][nx] out (may be NULL); eps_d device double out. */
mc_status mc_residual(const mc_medium *medium, const double *coeffs_d, const double *hmeas_d,
                      double *q_star_d, double *eps_d, void *stream);

/* Gradients (Sec. 5): with a', b' the adjoint coefficients, per pixel dx^2 times
 *   d eps/d mua = -a0 (hmeas - mua a0) + a0 a0' / 2pi + (1/pi) sum_n (a_n a_n' + b_n b_n')
 *                 (eq. grad_2D_abs_integral3)
 *   d eps/d mus = (1/pi) sum_{n>=1} (a_n a_n' + b_n b_n') (1 - g^n)
 *                 (eq. scattering_gradient3)
 * fwd_d, adj_d: FP64 [2N+1][nz][nx] from mc_forward / mc_adjoint.
 * dmua_d, dmus_d: FP64 [nz][nx] out (either may be NULL). */
mc_status mc_gradient(const mc_medium *medium, int n_harm, const double *fwd_d, const double *adj_d,
                      const double *hmeas_d, double *dmua_d, double *dmus_d, void *stream);

/* Absorbed energy density H = mua a0 (Sec. 2, Grueneisen parameter 1).
 * coeffs_d: forward FP64 [>=1][nz][nx] (only a0 is read); h_d: FP64 [nz][nx]
 * out.  Only the medium's mua_d, nx and nz are read. */
mc_status mc_absorbed(const mc_medium *medium, const double *coeffs_d, double *h_d, void *stream);

/* Adjoint source for any loss L(H) (Sec. 5 and 6 by the chain rule): given
 * the upstream gradient grad_h = dL/dH per pixel, q* = -mua grad_h / A per
 * unit angle (A = dx^2).  For L = eps, grad_h = -A (hmeas - H) and q* is the
 * q* = mua (hmeas - H) of mc_residual.  grad_h_d, q_star_d: FP64 [nz][nx]. */
mc_status mc_adjoint_source(const mc_medium *medium, const double *grad_h_d, double *q_star_d, void *stream);

/* Gradients of L(H) with respect to mua and mus (Sec. 5 with the direct term
 * of the chain rule through H = mua Phi), per pixel:
 *   dL/dmua = grad_h a0 + dx^2 [a0 a0'/2pi + (1/pi) sum_n (a_n a_n' + b_n b_n')]
 *   dL/dmus = dx^2 (1/pi) sum_{n>=1} (a_n a_n' + b_n b_n') (1 - g^n)
 * where adj_d is the mc_adjoint field of the source from mc_adjoint_source.
 * With grad_h = -A (hmeas - H) this equals mc_gradient. */
mc_status mc_gradient_h(const mc_medium *medium, int n_harm, const double *fwd_d, const double *adj_d,
                        const double *grad_h_d, double *dmua_d, double *dmus_d, void *stream);

/* Detector readout <phi, b> (Sec. 4.1, eq. adj_definition): the integral over
 * the domain and angle of a radiance times a detector weight function b, both
 * given by harmonic maps with the same convention:
 *   sum_i dx^2 [a0 d0/2pi + (1/pi) sum_n (a_n dc_n + b_n ds_n)].
 * det_d: FP64 [2N+1][nz][nx].  out_d: device double. */
mc_status mc_detect(const mc_medium *medium, int n_harm, const double *coeffs_d, const double *det_d,
                    double *out_d, void *stream);

/* Event record of mc_trace. */
typedef struct {
    uint64_t pid;
    int32_t k;        /* index of the free path the event ends (0: launch) */
    int32_t type;     /* 0 launch, 1 pixel crossing, 2 scatter, 3 escape, 4 roulette kill */
    int32_t ix, iz;   /* pixel of the segment that ends here (launch: start pixel) */
    float x, z;       /* position (mm) */
    float sx, sz;     /* direction after the event */
    float w;          /* weight after the event (escape/kill: the weight lost) */
    float t;          /* track-length deposit of the segment (mm) */
} mc_event;

/* Discrete-ordinates tally, for comparison with the harmonic tally (Sec. 3.1
 * contrasts the harmonic expansion of the radiance with binning it in angle):
 * the radiance averaged over n_bins equal bins of the direction angle
 * theta in [-pi, pi) (bin b covers [-pi + b w, -pi + (b+1) w), w = 2pi/n_bins),
 * per pixel, from the same transport as mc_forward (adjoint = 0) or
 * mc_adjoint (adjoint = 1, read at the mirrored direction: bin b holds what
 * the transport tallied in bin b + n_bins/2).  The same packets, seeds and
 * segment deposits T as those calls; each segment adds its T to its
 * direction's bin with one FP64 device atomic, so this serves comparison
 * runs, not speed.  Normalised as the coefficients and divided by w, so
 * sum_b binned[b] * w equals the a0 map.  binned_d: FP64 [n_bins][nz][nx]
 * (overwritten); n_bins even, 2 .. 4096; ledger_d: device mc_ledger or NULL;
 * workspace_d: >= mc_binned_workspace_bytes() bytes, 256-byte aligned. */
size_t mc_binned_workspace_bytes(const mc_medium *medium, const mc_source *src, int n_src, const mc_run *run,
                                 int n_bins);
mc_status mc_run_binned(const mc_medium *medium, const mc_source *src, int n_src, const mc_run *run, int adjoint,
                        int n_bins, double *binned_d, mc_ledger *ledger_d, void *workspace_d, size_t workspace_bytes,
                        void *stream);

/* Per-event trace of selected packets, run by the same device transport code
 * as mc_forward (adjoint != 0: as mc_adjoint).  Synchronous: allocates its own
 * device buffers, runs on the null stream and copies back.  pids_h: host
 * packet ids; events_h: host buffer of cap events; *n_events_h receives the
 * number of events produced (may exceed cap; only cap are stored). */
mc_status mc_trace(const mc_medium *medium, const mc_source *src, int n_src, const mc_run *run,
                   int adjoint, const uint64_t *pids_h, int n_pids, mc_event *events_h, size_t cap,
                   size_t *n_events_h);

/* Philox4x32-10 blocks (j, tag, pid0 + i) under key seed, i < n, written to
 * out_d[4i..4i+3] (device uint32).  Exposes the generator for checking. */
mc_status mc_philox_fill(uint64_t seed, uint32_t tag, uint64_t pid0, uint64_t n, uint32_t j,
                         uint32_t *out_d, void *stream);

const char *mc_status_string(mc_status s);
/* Library build identifier (architecture and tally configuration). */
const char *mc_build_info(void);

#ifdef __cplusplus
}
#endif
#endif /* MCRAD_H */
