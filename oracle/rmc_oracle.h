/*
 * rmc_oracle.h -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, scalar FP64 CPU implementation of the forward and adjoint
 * radiance Monte Carlo of Hochuli, Powell, Arridge & Cox, "Quantitative
 * photoacoustic tomography using forward and adjoint Monte Carlo models of
 * radiance" (arXiv:1608.05238).  It exists so that tests, the smoke check and
 * the CPU baseline of the benchmark can check the GPU library against an
 * independent implementation.  The product library never links, loads or
 * calls this code, and this code shares nothing (no header, table, helper or
 * generator) with the GPU library.
 *
 * Conventions (the readings of the paper this oracle implements):
 *  - Pixel (ix,iz) covers [ix*dx,(ix+1)*dx) x [iz*dx,(iz+1)*dx); x is lateral,
 *    z is depth.  Arrays are row-major [nz][nx].
 *  - Direction s = (sin t, cos t): the angle t is measured from +z towards +x
 *    (Sec. 3.1, the angle of s relative to the z direction).
 *  - Free path: exponential, tau = -ln U (Sec. 3 prints U/mu_s; the exponential
 *    law is the one that solves the RTE), optical depth consumed pixel by pixel.
 *  - Deposit per segment of length l in pixel i: T = W (1 - exp(-mua l)) / mua
 *    (the track length weighted by the decaying packet weight; W l if mua = 0).
 *    Harmonic tally a0 += T, a_n += T cos(n t), b_n += T sin(n t) (Sec. 3.1,
 *    eq. Fourier_terms).  Normalised output = S_tot / (Np * A) * tally.
 *  - Scatter: 2D Henyey-Greenstein, dt = 2 atan((1-g)/(1+g) tan(pi (U - 1/2)))
 *    (Sec. 3, eq. scattering_angle), t <- t + dt.
 *  - Termination (Sec. 3 and Sec. 6): at each scatter site, if |W| < w_th |W0|
 *    Russian roulette (survive with probability 1/m, W <- m W); a flag selects
 *    the literal "stop below the threshold" rule instead.
 *  - Random numbers: Philox4x32-10 (Salmon et al., SC'11), key = seed,
 *    counter = (j, stream_tag, pid_lo, pid_hi); block j = 0 launches the packet,
 *    block j = k >= 1 serves the k-th free path (u0), the HG angle at its end
 *    (u1) and the roulette draw there (u2).  u = ((x >> 9) + 1/2) 2^-23.
 *  - MAP sources (Sec. 6): a pixel is drawn with probability |q_i|/sum|q| and
 *    the packet carries the sign of q_i; with OR_FLAG_EQUAL_COUNT every pixel
 *    is equally likely and the packet carries q_i / mean|q| (the literal
 *    reading); both are normalised by 2 pi sum|q| A.
 *  - Adjoint (Sec. 4, eq. adjoint_RTE1): the adjoint field is the forward
 *    field of the direction-mirrored source, read at the mirrored direction,
 *    so source profiles are mirrored on input and orders n >= 1 of the output
 *    are multiplied by (-1)^n.
 */
#ifndef RMC_ORACLE_H
#define RMC_ORACLE_H
#include <stdint.h>

#define OR_MAX_HARM 32
#define OR_FLAG_LITERAL_TRUNCATION 1u   /* stop below the threshold instead of roulette (Sec. 3) */
#define OR_FLAG_EQUAL_COUNT 2u          /* MAP source: equal packets per pixel, weight ~ q (Sec. 6 literally) */

typedef struct {
    int nx, nz;
    double dx;                       /* pixel side (mm) */
    const double *mua, *mus, *g;     /* [nz][nx], 1/mm and anisotropy */
} or_medium;

enum { OR_SRC_PENCIL = 0, OR_SRC_LINE = 1, OR_SRC_POINT = 2, OR_SRC_MAP = 3 };

typedef struct {
    int kind;
    double x0, z0, x1, z1;   /* PENCIL/POINT: (x0,z0).  LINE: segment end points */
    double dir_x, dir_z;     /* PENCIL/LINE: unit direction (LINE Lambertian: inward normal) */
    int lambertian;          /* LINE: 0 collimated, 1 Lambertian about dir */
    double power;            /* PENCIL/LINE/POINT: source power */
    const double *map;       /* MAP: q(x) per unit angle per unit area, [nz][nx] (may be signed) */
    int n_prof;              /* POINT/MAP angular profile order; 0 with prof == NULL: isotropic */
    const double *prof;      /* [2 n_prof + 1]: c0, c1..cn, s1..sn; p = c0/2pi + (1/pi) sum(...) */
} or_source;

typedef struct {
    uint64_t n_packets, seed, first_packet_id;
    uint32_t stream_tag;
    int n_harm;                      /* N: orders 1..N, K = 2N+1 channels */
    double w_threshold;              /* roulette threshold relative to |W0| */
    double roulette_m;               /* survival 1/m, weight times m */
    uint32_t flags;                  /* OR_FLAG_* */
    int adjoint;                     /* 1: adjoint run (mirror source, flip output orders) */
} or_run;

typedef struct {
    double launched, absorbed, escaped, roulette_gain, roulette_loss; /* raw packet-weight sums */
    double segments, visits, scatters, packets;                        /* event counts */
    double scale;                    /* S_tot / Np: multiply raw weight sums by this for power */
} or_ledger;

enum { OR_EV_LAUNCH = 0, OR_EV_CROSS = 1, OR_EV_SCATTER = 2, OR_EV_ESCAPE = 3, OR_EV_KILL = 4 };

typedef struct {
    uint64_t pid;
    int32_t k;        /* interaction index of the free path the event ends (0 for launch) */
    int32_t type;     /* OR_EV_* */
    int32_t ix, iz;   /* pixel the segment ran in (launch: start pixel) */
    double x, z;      /* position at the event (mm) */
    double sx, sz;    /* direction after the event */
    double w;         /* weight after the event (escape/kill: weight lost) */
    double t;         /* deposit T of the segment ending here (mm) */
} or_event;

/* Philox4x32-10 block function. */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* Fill out[4*i..4*i+3] with the block (j, tag, pid0+i) under key = seed, i < n. */
void or_philox_fill(uint64_t seed, uint32_t tag, uint64_t pid0, uint64_t n, uint32_t j, uint32_t *out);
double or_u01(uint32_t x);
double or_hg_dtheta(double g, double u);
double or_free_path(double u);

/* Run the MC.  coeffs: [2N+1][nz][nx] normalised (a0, a1..aN, b1..bN).
 * binned (nullable): [n_bins][nz][nx] normalised radiance averaged over each
 * angular bin of width 2pi/n_bins starting at -pi.  Returns 0 or a negative
 * error code. */
int or_mc(const or_medium *m, const or_source *src, int n_src, const or_run *run,
          double *coeffs, or_ledger *led, double *binned, int n_bins, int n_threads);

/* Event trace of the listed packets (same transport, FP64).  Returns 0, or -1
 * on bad input; *n_events counts every event even past cap. */
int or_trace(const or_medium *m, const or_source *src, int n_src, const or_run *run,
             const uint64_t *pids, int n_pids, or_event *ev, int cap, int *n_events);

/* Residual: H = mua a0, r = Hmeas - H, q* = mua r, returns eps = A/2 sum r^2. */
double or_residual(const or_medium *m, const double *coeffs, const double *h_meas, double *q_star);
/* Gradients (per pixel value, i.e. A times the functional gradient). */
void or_gradient(const or_medium *m, int n_harm, const double *fwd, const double *adj,
                 const double *h_meas, double *dmua, double *dmus);
/* Detector readout <phi, b> = sum_i A [a0 d0/2pi + (1/pi) sum_n (a_n dc_n + b_n ds_n)]. */
double or_detect(const or_medium *m, int n_harm, const double *coeffs, const double *det);

#endif
