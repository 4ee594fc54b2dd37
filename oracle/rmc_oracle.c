/*
 * rmc_oracle.c -- TEST INFRASTRUCTURE ONLY (see rmc_oracle.h).
 *
 * Plain scalar FP64 radiance Monte Carlo written from the paper
 * (Hochuli et al., arXiv:1608.05238):
 *   Sec. 3        packet launch, free path, absorption weighting, 2D HG
 *                 scattering (eqs. scattering2D, scattering_angle), threshold
 *   Sec. 3.1      harmonic angular tally (eqs. radiance_Fourier, Fourier_terms)
 *   Sec. 4        adjoint RTE (eq. adjoint_RTE1), volumetric adjoint source
 *   Sec. 5        gradients (eqs. grad_2D_abs_integral3, scattering_gradient3)
 *   Sec. 6        adjoint source q* = mua (Hmeas - H), signed weights,
 *                 |W| termination, normalisation by the packet count
 * Every step is written in the order the paper describes it; nothing is
 * blocked, fused or reordered.  Built without -ffast-math.
 */
#include "rmc_oracle.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_PI 3.14159265358979323846

/* ---------------------------------------------------------------- Philox */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
 * easy as 1, 2, 3", SC'11): ten rounds of two 32x32->64 products with the
 * multipliers below, the Weyl key increments added between rounds. */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static void block_uniforms(uint64_t seed, uint32_t tag, uint64_t pid, uint32_t j, double u[4])
{
    uint32_t ctr[4] = { j, tag, (uint32_t)pid, (uint32_t)(pid >> 32) };
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    uint32_t x[4];
    or_philox4x32_10(ctr, key, x);
    for (int i = 0; i < 4; ++i) u[i] = or_u01(x[i]);
}

void or_philox_fill(uint64_t seed, uint32_t tag, uint64_t pid0, uint64_t n, uint32_t j, uint32_t *out)
{
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    for (uint64_t i = 0; i < n; ++i) {
        uint64_t pid = pid0 + i;
        uint32_t ctr[4] = { j, tag, (uint32_t)pid, (uint32_t)(pid >> 32) };
        or_philox4x32_10(ctr, key, out + 4 * i);
    }
}

/* Uniform on (0,1): the top 23 bits, centred in their cell.  Exact in FP32. */
double or_u01(uint32_t x) { return ((double)(x >> 9) + 0.5) * (1.0 / 8388608.0); }

/* Sec. 3, eq. scattering_angle, with tan(pi U) replaced by the identically
 * distributed tan(pi (U - 1/2)) so the argument never passes pi/2. */
double or_hg_dtheta(double g, double u)
{
    return 2.0 * atan((1.0 - g) / (1.0 + g) * tan(OR_PI * (u - 0.5)));
}

/* Exponential free path in units of 1/mu_s. */
double or_free_path(double u) { return -log(u); }

/* ---------------------------------------------------------------- setup */
typedef struct {
    const or_medium *m;
    const or_source *src;
    int n_src;
    const or_run *run;
    int N, K;
    double meas[64];        /* per-source sampling measure M_s */
    double cum[64];         /* inclusive prefix of meas */
    double total;           /* S_tot */
    double *map_cdf;        /* MAP: inclusive prefix of |map_i| */
    double prof[64][2 * OR_MAX_HARM + 1]; /* per-source angular profile (mirrored if adjoint) */
    int n_prof[64];
} or_ctx;

/* Angular profile p(t) = c0/2pi + (1/pi) sum_n (c_n cos nt + s_n sin nt). */
static double profile_eval(const double *c, int n, double t)
{
    double p = c[0] / (2.0 * OR_PI);
    for (int k = 1; k <= n; ++k)
        p += (c[k] * cos(k * t) + c[n + k] * sin(k * t)) / OR_PI;
    return p;
}

static int ctx_init(or_ctx *c, const or_medium *m, const or_source *src, int n_src, const or_run *run)
{
    memset(c, 0, sizeof(*c));
    if (!m || !src || !run || n_src < 1 || n_src > 64) return -1;
    if (m->nx <= 0 || m->nz <= 0 || !(m->dx > 0) || !m->mua || !m->mus || !m->g) return -1;
    if (run->n_harm < 0 || run->n_harm > OR_MAX_HARM || run->n_packets == 0) return -1;
    if (!(run->roulette_m > 1.0) || !(run->w_threshold >= 0)) return -1;
    int npix = m->nx * m->nz;
    for (int i = 0; i < npix; ++i)
        if (!(m->mua[i] >= 0) || !(m->mus[i] >= 0) || !(m->g[i] > -1.0 && m->g[i] <= 1.0)) return -1;
    c->m = m; c->src = src; c->n_src = n_src; c->run = run;
    c->N = run->n_harm; c->K = 2 * run->n_harm + 1;
    double A = m->dx * m->dx, W = m->nx * m->dx, H = m->nz * m->dx;
    for (int s = 0; s < n_src; ++s) {
        const or_source *q = &src[s];
        if (q->kind == OR_SRC_MAP) {
            if (n_src != 1 || !q->map) return -1;
            c->map_cdf = (double *)malloc(sizeof(double) * npix);
            if (!c->map_cdf) return -1;
            double acc = 0;
            for (int i = 0; i < npix; ++i) { acc += fabs(q->map[i]); c->map_cdf[i] = acc; }
            if (!(acc > 0)) return -1;
            c->meas[s] = 2.0 * OR_PI * acc * A;
        } else {
            if (q->kind < 0 || q->kind > OR_SRC_MAP || !(q->power > 0)) return -1;
            double pts[2][2] = { { q->x0, q->z0 }, { q->x1, q->z1 } };
            int np = q->kind == OR_SRC_LINE ? 2 : 1;
            for (int k = 0; k < np; ++k)
                if (pts[k][0] < 0 || pts[k][0] > W || pts[k][1] < 0 || pts[k][1] > H) return -1;
            if (q->kind != OR_SRC_POINT && fabs(hypot(q->dir_x, q->dir_z) - 1.0) > 1e-6) return -1;
            c->meas[s] = q->power;
        }
        if (q->kind == OR_SRC_POINT || q->kind == OR_SRC_MAP) {
            int n = q->prof ? q->n_prof : 0;
            if (n < 0 || n > OR_MAX_HARM) return -1;
            c->n_prof[s] = n;
            if (q->prof) {
                for (int k = 0; k <= 2 * n; ++k) c->prof[s][k] = q->prof[k];
            } else {
                c->prof[s][0] = 1.0;  /* isotropic: p = 1/2pi */
            }
            if (run->adjoint) {   /* mirror: p(t) -> p(t + pi) */
                for (int k = 1; k <= n; ++k) {
                    double sg = (k & 1) ? -1.0 : 1.0;
                    c->prof[s][k] *= sg;
                    c->prof[s][n + k] *= sg;
                }
            }
        }
        c->total += c->meas[s];
        c->cum[s] = c->total;
    }
    return 0;
}

/* ---------------------------------------------------------------- transport */
typedef struct {
    double *tally;      /* raw [K][npix] */
    double *binned;     /* raw [n_bins][npix] or NULL */
    int n_bins;
    or_ledger led;
    or_event *ev; int cap; int nev;   /* trace sink */
} or_sink;

static void record(or_sink *k, uint64_t pid, int kk, int type, int ix, int iz, double x, double z,
                   double sx, double sz, double w, double t)
{
    if (!k->ev) return;
    if (k->nev < k->cap) {
        or_event *e = &k->ev[k->nev];
        e->pid = pid; e->k = kk; e->type = type; e->ix = ix; e->iz = iz;
        e->x = x; e->z = z; e->sx = sx; e->sz = sz; e->w = w; e->t = t;
    }
    k->nev++;
}

/* Pixel containing (x,z); a point on a face moving towards the lower index
 * belongs to the lower pixel. */
static void locate(const or_medium *m, double x, double z, double sx, double sz, int *ix, int *iz)
{
    double fx = x / m->dx, fz = z / m->dx;
    /* a point given on the outer boundary lies on it, whatever the rounding of x / dx */
    if (fabs(fx) < 1e-9) fx = 0.0;
    if (fabs(fz) < 1e-9) fz = 0.0;
    if (fabs(fx - m->nx) < 1e-9 * m->nx) fx = m->nx;
    if (fabs(fz - m->nz) < 1e-9 * m->nz) fz = m->nz;
    int i = (int)floor(fx), j = (int)floor(fz);
    if (fx == (double)i && sx < 0) i -= 1;
    if (fz == (double)j && sz < 0) j -= 1;
    *ix = i; *iz = j;
}

static double wrap_angle(double t)
{
    return t - 2.0 * OR_PI * floor((t + OR_PI) / (2.0 * OR_PI));
}

static void run_packet(const or_ctx *c, uint64_t pid, or_sink *k)
{
    const or_medium *m = c->m;
    const or_run *run = c->run;
    const int N = c->N, nx = m->nx, nz = m->nz, npix = nx * nz;
    const double dx = m->dx;
    double u[4];

    /* launch (Sec. 3): position, direction and initial weight from block 0 */
    block_uniforms(run->seed, run->stream_tag, pid, 0, u);
    int s = 0;
    if (c->n_src > 1) {
        double t = u[0] * c->total;
        while (s < c->n_src - 1 && !(c->cum[s] > t)) ++s;
    }
    const or_source *q = &c->src[s];
    double x, z, sx, sz, th, W0 = 1.0;
    double flip = run->adjoint ? -1.0 : 1.0;
    if (q->kind == OR_SRC_PENCIL || q->kind == OR_SRC_LINE) {
        double lu = q->kind == OR_SRC_LINE ? u[1] : 0.0;
        x = q->x0 + lu * (q->x1 - q->x0);
        z = q->z0 + lu * (q->z1 - q->z0);
        sx = flip * q->dir_x; sz = flip * q->dir_z;
        th = atan2(sx, sz);
        if (q->kind == OR_SRC_LINE && q->lambertian) {
            double sa = 2.0 * u[2] - 1.0;          /* Lambertian: sin(alpha) uniform */
            th = wrap_angle(th + asin(sa));
            sx = sin(th); sz = cos(th);
        }
    } else if (q->kind == OR_SRC_POINT) {
        x = q->x0; z = q->z0;
        th = OR_PI * (2.0 * u[2] - 1.0);
        sx = sin(th); sz = cos(th);
        W0 = 2.0 * OR_PI * profile_eval(c->prof[s], c->n_prof[s], th);
    } else {  /* MAP source, uniform position inside the chosen pixel */
        int lo;
        double wq;
        if (run->flags & OR_FLAG_EQUAL_COUNT) {
            /* Sec. 6 read literally: pixels drawn with equal probability, the
             * launch weight scaled by the source value (relative to the mean
             * of |q|, so that the normalisation is the same as below) */
            lo = (int)floor(u[0] * npix);
            if (lo > npix - 1) lo = npix - 1;
            wq = q->map[lo] / (c->map_cdf[npix - 1] / npix);
        } else {   /* pixel with probability |q_i| / sum |q|, weight sign(q_i) */
            double t = u[0] * c->map_cdf[npix - 1];
            int hi = npix - 1;
            lo = 0;
            while (lo < hi) {            /* first i with cdf[i] > t */
                int mid = (lo + hi) / 2;
                if (c->map_cdf[mid] > t) hi = mid; else lo = mid + 1;
            }
            wq = q->map[lo] < 0 ? -1.0 : 1.0;
        }
        int ixs = lo % nx, izs = lo / nx;
        x = (ixs + u[1]) * dx;
        z = (izs + u[2]) * dx;
        th = OR_PI * (2.0 * u[3] - 1.0);
        sx = sin(th); sz = cos(th);
        W0 = wq * 2.0 * OR_PI * profile_eval(c->prof[0], c->n_prof[0], th);
    }
    double W = W0, W0abs = fabs(W0);
    k->led.launched += W0;
    k->led.packets += 1;

    int ix, iz;
    locate(m, x, z, sx, sz, &ix, &iz);
    record(k, pid, 0, OR_EV_LAUNCH, ix, iz, x, z, sx, sz, W, 0.0);
    /* a packet of zero weight (equal-count launch in a pixel where q = 0)
     * carries nothing and leaves at once, like one launched outside */
    if (ix < 0 || ix >= nx || iz < 0 || iz >= nz || ((run->flags & OR_FLAG_EQUAL_COUNT) && W0 == 0.0)) {
        k->led.escaped += W;
        record(k, pid, 0, OR_EV_ESCAPE, ix, iz, x, z, sx, sz, W, 0.0);
        return;
    }

    double hc[OR_MAX_HARM + 1], hs[OR_MAX_HARM + 1];
    for (int n = 1; n <= N; ++n) { hc[n] = cos(n * th); hs[n] = sin(n * th); }

    for (uint32_t kk = 1;; ++kk) {
        block_uniforms(run->seed, run->stream_tag, pid, kk, u);
        double tau = or_free_path(u[0]);
        int scatter = 0;
        double T = 0;
        for (;;) {
            int i = iz * nx + ix;
            double mua = m->mua[i], mus = m->mus[i];
            double dfx = INFINITY, dfz = INFINITY;
            if (sx > 0) dfx = ((ix + 1) * dx - x) / sx;
            else if (sx < 0) dfx = (ix * dx - x) / sx;
            if (sz > 0) dfz = ((iz + 1) * dx - z) / sz;
            else if (sz < 0) dfz = (iz * dx - z) / sz;
            if (dfx < 0) dfx = 0;
            if (dfz < 0) dfz = 0;
            double d = dfx < dfz ? dfx : dfz;
            double l;
            if (mus * d > tau) { l = tau / mus; scatter = 1; }
            else { l = d; tau -= mus * d; }
            /* absorption weighting over the segment (Sec. 3) */
            T = mua > 0 ? -W * expm1(-mua * l) / mua : W * l;
            double Wn = W * exp(-mua * l);
            k->led.absorbed += W - Wn;
            W = Wn;
            /* harmonic tally (Sec. 3.1, eq. Fourier_terms) */
            k->tally[i] += T;
            for (int n = 1; n <= N; ++n) {
                k->tally[(size_t)n * npix + i] += T * hc[n];
                k->tally[(size_t)(N + n) * npix + i] += T * hs[n];
            }
            if (k->binned) {
                int b = (int)floor((wrap_angle(th) + OR_PI) / (2.0 * OR_PI) * k->n_bins);
                if (b >= k->n_bins) b = k->n_bins - 1;
                if (b < 0) b = 0;
                k->binned[(size_t)b * npix + i] += T;
            }
            k->led.segments += 1;
            if (scatter) {
                x += l * sx; z += l * sz;
                break;
            }
            /* cross into the neighbouring pixel */
            int oix = ix, oiz = iz;
            if (dfx <= dfz) {
                if (sx > 0) { ix += 1; x = ix * dx; } else { x = ix * dx; ix -= 1; }
            } else {
                x += l * sx;
            }
            if (dfz <= dfx) {
                if (sz > 0) { iz += 1; z = iz * dx; } else { z = iz * dx; iz -= 1; }
            } else {
                z += l * sz;
            }
            k->led.visits += 1;
            if (ix < 0 || ix >= nx || iz < 0 || iz >= nz) {
                k->led.escaped += W;
                record(k, pid, (int)kk, OR_EV_ESCAPE, oix, oiz, x, z, sx, sz, W, T);
                return;
            }
            record(k, pid, (int)kk, OR_EV_CROSS, oix, oiz, x, z, sx, sz, W, T);
        }
        /* scatter site: termination test first (Sec. 3, Sec. 6: on |W|) */
        if (fabs(W) < run->w_threshold * W0abs) {
            if ((run->flags & OR_FLAG_LITERAL_TRUNCATION) || !(u[2] < 1.0 / run->roulette_m)) {
                k->led.roulette_loss += W;
                k->led.visits += 1;
                record(k, pid, (int)kk, OR_EV_KILL, ix, iz, x, z, sx, sz, W, T);
                return;
            }
            k->led.roulette_gain += (run->roulette_m - 1.0) * W;
            W *= run->roulette_m;
        }
        /* 2D Henyey-Greenstein deflection (Sec. 3, eq. scattering_angle) */
        double g = m->g[iz * nx + ix];
        th = wrap_angle(th + or_hg_dtheta(g, u[1]));
        sx = sin(th); sz = cos(th);
        for (int n = 1; n <= N; ++n) { hc[n] = cos(n * th); hs[n] = sin(n * th); }
        k->led.scatters += 1;
        record(k, pid, (int)kk, OR_EV_SCATTER, ix, iz, x, z, sx, sz, W, T);
    }
}

int or_mc(const or_medium *m, const or_source *src, int n_src, const or_run *run,
          double *coeffs, or_ledger *led, double *binned, int n_bins, int n_threads)
{
    or_ctx c;
    if (ctx_init(&c, m, src, n_src, run) != 0) { free(c.map_cdf); return -1; }
    if (!coeffs || (binned && (n_bins <= 0 || (n_bins & 1)))) { free(c.map_cdf); return -1; }
    const int npix = m->nx * m->nz, K = c.K;
    int nt = n_threads > 0 ? n_threads : 1;
    if ((uint64_t)nt > run->n_packets) nt = (int)run->n_packets;
    or_sink *sinks = (or_sink *)calloc(nt, sizeof(or_sink));
    int bad = sinks == NULL;
    for (int t = 0; t < nt && !bad; ++t) {
        sinks[t].tally = (double *)calloc((size_t)K * npix, sizeof(double));
        sinks[t].n_bins = binned ? n_bins : 0;
        sinks[t].binned = binned ? (double *)calloc((size_t)n_bins * npix, sizeof(double)) : NULL;
        if (!sinks[t].tally || (binned && !sinks[t].binned)) bad = 1;
    }
    if (!bad) {
#pragma omp parallel for schedule(static, 1) num_threads(nt)
        for (int t = 0; t < nt; ++t) {
            uint64_t a = run->n_packets * (uint64_t)t / (uint64_t)nt;
            uint64_t b = run->n_packets * (uint64_t)(t + 1) / (uint64_t)nt;
            for (uint64_t p = a; p < b; ++p) run_packet(&c, run->first_packet_id + p, &sinks[t]);
        }
        /* combine per-thread tallies in thread order, then normalise (Sec. 6) */
        double A = m->dx * m->dx;
        double scale = c.total / ((double)run->n_packets * A);
        memset(coeffs, 0, sizeof(double) * (size_t)K * npix);
        if (binned) memset(binned, 0, sizeof(double) * (size_t)n_bins * npix);
        or_ledger L;
        memset(&L, 0, sizeof(L));
        for (int t = 0; t < nt; ++t) {
            for (size_t j = 0; j < (size_t)K * npix; ++j) coeffs[j] += sinks[t].tally[j];
            if (binned)
                for (size_t j = 0; j < (size_t)n_bins * npix; ++j) binned[j] += sinks[t].binned[j];
            L.launched += sinks[t].led.launched; L.absorbed += sinks[t].led.absorbed;
            L.escaped += sinks[t].led.escaped; L.roulette_gain += sinks[t].led.roulette_gain;
            L.roulette_loss += sinks[t].led.roulette_loss; L.segments += sinks[t].led.segments;
            L.visits += sinks[t].led.visits; L.scatters += sinks[t].led.scatters;
            L.packets += sinks[t].led.packets;
        }
        for (int ch = 0; ch < K; ++ch) {
            int n = ch <= c.N ? ch : ch - c.N;
            double f = scale * ((run->adjoint && (n & 1)) ? -1.0 : 1.0);
            for (int i = 0; i < npix; ++i) coeffs[(size_t)ch * npix + i] *= f;
        }
        if (binned) {
            double bw = 2.0 * OR_PI / n_bins;
            for (size_t j = 0; j < (size_t)n_bins * npix; ++j) binned[j] *= scale / bw;
            if (run->adjoint) {   /* read the mirrored direction: bin b <-> b + n_bins/2 */
                double *tmp = (double *)malloc(sizeof(double) * (size_t)n_bins * npix);
                if (tmp) {
                    memcpy(tmp, binned, sizeof(double) * (size_t)n_bins * npix);
                    for (int b = 0; b < n_bins; ++b) {
                        int bb = (b + n_bins / 2) % n_bins;
                        memcpy(binned + (size_t)b * npix, tmp + (size_t)bb * npix, sizeof(double) * npix);
                    }
                    free(tmp);
                } else {
                    bad = 1;
                }
            }
        }
        L.scale = c.total / (double)run->n_packets;
        if (led) *led = L;
    }
    for (int t = 0; t < nt && sinks; ++t) { free(sinks[t].tally); free(sinks[t].binned); }
    free(sinks);
    free(c.map_cdf);
    return bad ? -2 : 0;
}

int or_trace(const or_medium *m, const or_source *src, int n_src, const or_run *run,
             const uint64_t *pids, int n_pids, or_event *ev, int cap, int *n_events)
{
    or_ctx c;
    if (ctx_init(&c, m, src, n_src, run) != 0 || !pids || n_pids < 0 || !ev || !n_events) {
        free(c.map_cdf);
        return -1;
    }
    const int npix = m->nx * m->nz;
    or_sink k;
    memset(&k, 0, sizeof(k));
    k.tally = (double *)calloc((size_t)c.K * npix, sizeof(double));
    if (!k.tally) { free(c.map_cdf); return -2; }
    k.ev = ev; k.cap = cap;
    for (int p = 0; p < n_pids; ++p) run_packet(&c, pids[p], &k);
    *n_events = k.nev;
    free(k.tally);
    free(c.map_cdf);
    return 0;
}

/* ---------------------------------------------------------------- residual / gradient */
/* Sec. 2 eq. error_function3 with H = mua Phi (Grueneisen 1), discretised over
 * pixels; Sec. 6: q* = mua (Hmeas - H), independent of angle. */
double or_residual(const or_medium *m, const double *coeffs, const double *h_meas, double *q_star)
{
    const int npix = m->nx * m->nz;
    const double A = m->dx * m->dx;
    double eps = 0;
    for (int i = 0; i < npix; ++i) {
        double H = m->mua[i] * coeffs[i];
        double r = h_meas[i] - H;
        if (q_star) q_star[i] = m->mua[i] * r;
        eps += 0.5 * A * r * r;
    }
    return eps;
}

/* Sec. 5: eq. grad_2D_abs_integral3 for mua and eq. scattering_gradient3 for
 * mus, times the pixel area (derivative with respect to a pixel value). */
void or_gradient(const or_medium *m, int n_harm, const double *fwd, const double *adj,
                 const double *h_meas, double *dmua, double *dmus)
{
    const int npix = m->nx * m->nz, N = n_harm;
    const double A = m->dx * m->dx;
    for (int i = 0; i < npix; ++i) {
        double a0 = fwd[i], a0s = adj[i];
        double r = h_meas[i] - m->mua[i] * a0;
        double sum_all = 0, sum_g = 0, gn = 1;
        for (int n = 1; n <= N; ++n) {
            gn *= m->g[i];
            double p = fwd[(size_t)n * npix + i] * adj[(size_t)n * npix + i]
                     + fwd[(size_t)(N + n) * npix + i] * adj[(size_t)(N + n) * npix + i];
            sum_all += p;
            sum_g += p * (1.0 - gn);
        }
        dmua[i] = A * (-a0 * r + a0 * a0s / (2.0 * OR_PI) + sum_all / OR_PI);
        dmus[i] = A * (sum_g / OR_PI);
    }
}

/* Inner product of a radiance with a detector weight function, both given by
 * their harmonic coefficients (orthogonality of the basis of eq. radiance_Fourier). */
double or_detect(const or_medium *m, int n_harm, const double *coeffs, const double *det)
{
    const int npix = m->nx * m->nz, N = n_harm;
    const double A = m->dx * m->dx;
    double acc = 0;
    for (int i = 0; i < npix; ++i) {
        double v = coeffs[i] * det[i] / (2.0 * OR_PI);
        for (int n = 1; n <= N; ++n)
            v += (coeffs[(size_t)n * npix + i] * det[(size_t)n * npix + i]
                  + coeffs[(size_t)(N + n) * npix + i] * det[(size_t)(N + n) * npix + i]) / OR_PI;
        acc += A * v;
    }
    return acc;
}
