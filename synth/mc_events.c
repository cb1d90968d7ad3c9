/*
 * Monte-Carlo list-mode SPECT acquisition for seeded synthetic inputs.
 *
 * The paper's evaluation data came from a Monte-Carlo photon simulation that
 * recorded, per detected photon, the position of interaction, the energy and
 * the detector angle (Sec. 3).  That code and its phantom are not available,
 * so this file simulates photon histories in a continuous 2-D object instead:
 *
 *   - emission at a uniformly random point inside a pixel drawn in
 *     proportion to its activity, isotropic in the imaging plane;
 *   - attenuation by midpoint marching through the piecewise-constant
 *     attenuation map (step = pixel/4), with Compton-only energy scaling of
 *     the attenuation coefficient;
 *   - at most one in-plane Compton interaction (the paper keeps only
 *     first-order, in-plane scatter, Sec. 2.2); the in-plane scattering
 *     direction follows the Klein-Nishina shape restricted to the plane;
 *   - an ideal parallel-hole collimator at the camera angles 2*pi*a/N_A,
 *     sampled by forced detection plus rejection so every accepted photon
 *     is an unweighted draw;
 *   - Gaussian blur of the detected position and energy, then the detector
 *     extent and the energy acceptance window.
 *
 * It is input generation only: it never evaluates the reconstruction's path
 * sums, system rows or EM updates, and shares no code with either the
 * reconstruction library or the oracle.
 *
 * Random numbers come from Philox4x32-10 (Salmon, Moraes, Dror, Shaw,
 * "Parallel random numbers: as easy as 1, 2, 3", SC'11), keyed by the seed
 * and counted by candidate index, so the output does not depend on the
 * number of threads.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ME_C2_KEV 510.99895

typedef struct {
    int nx, ny;
    double dx;
    int n_bins;
    double bin_cm;
    int n_angles;
    double angle0;
    double e0, fwhm_e, fwhm_u, win_lo, win_hi;
} mc_geom;

/* ---- Philox4x32-10 ---------------------------------------------------- */
typedef struct { uint32_t v[4]; } u32x4;

static inline void mulhilo(uint32_t a, uint32_t b, uint32_t *hi, uint32_t *lo) {
    uint64_t p = (uint64_t)a * (uint64_t)b;
    *hi = (uint32_t)(p >> 32);
    *lo = (uint32_t)p;
}

static u32x4 philox(u32x4 c, uint32_t k0, uint32_t k1) {
    for (int r = 0; r < 10; ++r) {
        uint32_t hi0, lo0, hi1, lo1;
        mulhilo(0xD2511F53u, c.v[0], &hi0, &lo0);
        mulhilo(0xCD9E8D57u, c.v[2], &hi1, &lo1);
        u32x4 n;
        n.v[0] = hi1 ^ c.v[1] ^ k0;
        n.v[1] = lo1;
        n.v[2] = hi0 ^ c.v[3] ^ k1;
        n.v[3] = lo0;
        c = n;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

/* open interval (0, 1) */
static inline double u01(uint32_t x) { return ((double)(x >> 8) + 0.5) * (1.0 / 16777216.0); }

typedef struct {
    uint32_t k0, k1;
    uint64_t cand;
    uint32_t call;
    u32x4 buf;
    int used;
} rng_t;

static double rnd(rng_t *g) {
    if (g->used == 4) {
        u32x4 c = {{(uint32_t)g->cand, (uint32_t)(g->cand >> 32), g->call++, 0x5eed5eedu}};
        g->buf = philox(c, g->k0, g->k1);
        g->used = 0;
    }
    return u01(g->buf.v[g->used++]);
}

static double normal(rng_t *g) {
    double a = rnd(g), b = rnd(g);
    return sqrt(-2.0 * log(a)) * cos(2.0 * M_PI * b);
}

/* ---- photon physics (own implementation) ------------------------------ */
static double kn_total_over_re2(double e_kev) {
    double x = e_kev / ME_C2_KEV;
    double l = log1p(2.0 * x);
    return 2.0 * M_PI * (((1.0 + x) / (x * x)) * (2.0 * (1.0 + x) / (1.0 + 2.0 * x) - l / x)
                         + l / (2.0 * x) - (1.0 + 3.0 * x) / ((1.0 + 2.0 * x) * (1.0 + 2.0 * x)));
}

/* Klein-Nishina angular shape in units of r_e^2/2 for cos(theta) = c */
static double kn_shape(double e_kev, double c) {
    double p = 1.0 / (1.0 + (e_kev / ME_C2_KEV) * (1.0 - c));
    return p * p * (p + 1.0 / p - (1.0 - c * c));
}

typedef struct {
    const mc_geom *g;
    const float *mu;
    const double *cdf;   /* activity CDF over pixels, cdf[n-1] == 1 */
    int n_pix;
    double box[4];       /* bounding box of mu > 0: xmin xmax ymin ymax */
    double shape_mean;   /* circle-average of kn_shape at e0 */
    double sig_e, sig_u, half_len;
    uint32_t k0, k1;
} mc_ctx;

static inline double mu_at(const mc_ctx *c, double x, double y) {
    const mc_geom *g = c->g;
    double fi = floor(x / g->dx + 0.5 * g->nx), fj = floor(y / g->dx + 0.5 * g->ny);
    if (fi < 0 || fj < 0 || fi >= g->nx || fj >= g->ny) return 0.0;
    return c->mu[(int)fj * g->nx + (int)fi];
}

/* parametric range [t0, t1] of the ray p + t d inside the attenuating box */
static int clip_box(const mc_ctx *c, double px, double py, double ddx, double ddy,
                    double *t0, double *t1) {
    double lo = 0.0, hi = 1e30;
    double p[2] = {px, py}, d[2] = {ddx, ddy};
    for (int k = 0; k < 2; ++k) {
        double bmin = c->box[2 * k], bmax = c->box[2 * k + 1];
        if (fabs(d[k]) < 1e-15) {
            if (p[k] < bmin || p[k] > bmax) return 0;
        } else {
            double ta = (bmin - p[k]) / d[k], tb = (bmax - p[k]) / d[k];
            if (ta > tb) { double t = ta; ta = tb; tb = t; }
            if (ta > lo) lo = ta;
            if (tb < hi) hi = tb;
        }
    }
    if (hi <= lo) return 0;
    *t0 = lo; *t1 = hi;
    return 1;
}

/* optical depth along a ray from (px,py) to infinity, at E0 */
static double march_depth(const mc_ctx *c, double px, double py, double ddx, double ddy) {
    double t0, t1;
    if (!clip_box(c, px, py, ddx, ddy, &t0, &t1)) return 0.0;
    double h = 0.25 * c->g->dx, s = 0.0;
    for (double t = t0; t < t1; t += h) {
        double len = (t + h < t1) ? h : (t1 - t);
        double tm = t + 0.5 * len;
        s += mu_at(c, px + tm * ddx, py + tm * ddy) * len;
    }
    return s;
}

/* distance along the ray at which the optical depth reaches tau; <0 if it escapes */
static double march_to_depth(const mc_ctx *c, double px, double py, double ddx, double ddy,
                             double tau) {
    double t0, t1;
    if (!clip_box(c, px, py, ddx, ddy, &t0, &t1)) return -1.0;
    double h = 0.25 * c->g->dx, s = 0.0;
    for (double t = t0; t < t1; t += h) {
        double len = (t + h < t1) ? h : (t1 - t);
        double tm = t + 0.5 * len;
        double m = mu_at(c, px + tm * ddx, py + tm * ddy);
        if (m > 0.0 && s + m * len >= tau) return t + (tau - s) / m;
        s += m * len;
    }
    return -1.0;
}

typedef struct { int32_t angle; float u_bin; float energy; uint8_t kind; } mc_event;

/* one candidate history; returns 1 and fills *ev if a photon is detected */
static int simulate(const mc_ctx *c, uint64_t cand, mc_event *ev) {
    const mc_geom *g = c->g;
    rng_t r = {c->k0, c->k1, cand, 0, {{0, 0, 0, 0}}, 4};
    /* emission pixel by CDF bisection, then a uniform point inside it */
    double v = rnd(&r);
    int lo = 0, hi = c->n_pix - 1;
    while (lo < hi) { int mid = (lo + hi) / 2; if (c->cdf[mid] < v) lo = mid + 1; else hi = mid; }
    int i = lo % g->nx, j = lo / g->nx;
    double x = (i - 0.5 * (g->nx - 1) + rnd(&r) - 0.5) * g->dx;
    double y = (j - 0.5 * (g->ny - 1) + rnd(&r) - 0.5) * g->dx;
    int scatter = rnd(&r) < 0.5;
    int a = (int)(rnd(&r) * g->n_angles);
    if (a >= g->n_angles) a = g->n_angles - 1;
    double th = g->angle0 + 2.0 * M_PI * a / g->n_angles;
    double nax = cos(th), nay = sin(th), tax = -sin(th), tay = cos(th);
    double bound = 2.0 / c->shape_mean;   /* max over c of kn_shape/shape_mean */
    double u_true, e_true;
    if (!scatter) {
        double depth = march_depth(c, x, y, nax, nay);
        if (rnd(&r) * bound >= exp(-depth)) return 0;
        u_true = x * tax + y * tay;
        e_true = g->e0;
    } else {
        double phi = 2.0 * M_PI * rnd(&r);
        double dpx = cos(phi), dpy = sin(phi);
        double tau = -log(rnd(&r));
        double d = march_to_depth(c, x, y, dpx, dpy, tau);
        if (d < 0.0) return 0;
        double sx = x + d * dpx, sy = y + d * dpy;
        double cs = dpx * nax + dpy * nay;
        double ep = g->e0 / (1.0 + (g->e0 / ME_C2_KEV) * (1.0 - cs));
        double ratio = kn_total_over_re2(ep) / kn_total_over_re2(g->e0);
        double w = kn_shape(g->e0, cs) / c->shape_mean * exp(-ratio * march_depth(c, sx, sy, nax, nay));
        if (rnd(&r) * bound >= w) return 0;
        u_true = sx * tax + sy * tay;
        e_true = ep;
    }
    double u = u_true + c->sig_u * normal(&r);
    double e = e_true + c->sig_e * normal(&r);
    if (u < -c->half_len || u >= c->half_len) return 0;
    if (e < g->win_lo || e > g->win_hi) return 0;
    float ub = (float)(u / g->bin_cm + 0.5 * g->n_bins);
    if (ub >= (float)g->n_bins) ub = nextafterf((float)g->n_bins, 0.0f);
    if (ub < 0.0f) ub = 0.0f;
    ev->angle = a;
    ev->u_bin = ub;
    ev->energy = (float)e;
    ev->kind = (uint8_t)scatter;
    return 1;
}

typedef struct {
    const mc_ctx *c;
    uint64_t first_block;
    int n_blocks, tid, n_threads;
    int block_size;
    mc_event *out;   /* [n_blocks][block_size] */
    int *count;      /* [n_blocks] */
} worker_arg;

static void *worker(void *p) {
    worker_arg *w = (worker_arg *)p;
    for (int b = w->tid; b < w->n_blocks; b += w->n_threads) {
        uint64_t base = (w->first_block + (uint64_t)b) * (uint64_t)w->block_size;
        int n = 0;
        mc_event *dst = w->out + (size_t)b * w->block_size;
        for (int k = 0; k < w->block_size; ++k)
            n += simulate(w->c, base + (uint64_t)k, dst + n);
        w->count[b] = n;
    }
    return NULL;
}

/*
 * Generate exactly n_events detected photons.  Returns the number of
 * candidate histories used, or -1 on bad input / allocation failure.
 */
long long mc_generate(const mc_geom *g, const float *activity, const float *mu,
                      long long n_events, uint64_t seed, int n_threads,
                      int32_t *angle, float *u_bin, float *energy, uint8_t *kind) {
    int n_pix = g->nx * g->ny;
    if (n_events < 0 || n_pix <= 0 || n_threads <= 0) return -1;
    double *cdf = (double *)malloc(sizeof(double) * n_pix);
    if (!cdf) return -1;
    double tot = 0.0;
    for (int p = 0; p < n_pix; ++p) { tot += activity[p] > 0 ? activity[p] : 0.0; cdf[p] = tot; }
    if (tot <= 0.0) { free(cdf); return -1; }
    for (int p = 0; p < n_pix; ++p) cdf[p] /= tot;
    cdf[n_pix - 1] = 1.0;

    mc_ctx c;
    memset(&c, 0, sizeof c);
    c.g = g; c.mu = mu; c.cdf = cdf; c.n_pix = n_pix;
    c.box[0] = c.box[2] = 1e30; c.box[1] = c.box[3] = -1e30;
    for (int j = 0; j < g->ny; ++j)
        for (int i = 0; i < g->nx; ++i)
            if (mu[j * g->nx + i] > 0.0f) {
                double x0 = (i - 0.5 * g->nx) * g->dx, y0 = (j - 0.5 * g->ny) * g->dx;
                if (x0 < c.box[0]) c.box[0] = x0;
                if (x0 + g->dx > c.box[1]) c.box[1] = x0 + g->dx;
                if (y0 < c.box[2]) c.box[2] = y0;
                if (y0 + g->dx > c.box[3]) c.box[3] = y0 + g->dx;
            }
    if (c.box[0] > c.box[1]) { c.box[0] = c.box[1] = c.box[2] = c.box[3] = 0.0; }
    const int M = 4096;
    double sm = 0.0;
    for (int m = 0; m < M; ++m) sm += kn_shape(g->e0, cos(2.0 * M_PI * (m + 0.5) / M));
    c.shape_mean = sm / M;
    c.sig_e = g->fwhm_e / (2.0 * sqrt(2.0 * log(2.0)));
    c.sig_u = g->fwhm_u / (2.0 * sqrt(2.0 * log(2.0)));
    c.half_len = 0.5 * g->n_bins * g->bin_cm;
    c.k0 = (uint32_t)seed;
    c.k1 = (uint32_t)(seed >> 32) ^ 0x2002u;

    const int block = 8192, per_round = 64 * n_threads;
    mc_event *buf = (mc_event *)malloc(sizeof(mc_event) * (size_t)block * per_round);
    int *cnt = (int *)malloc(sizeof(int) * per_round);
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * n_threads);
    worker_arg *wa = (worker_arg *)malloc(sizeof(worker_arg) * n_threads);
    if (!buf || !cnt || !th || !wa) { free(cdf); free(buf); free(cnt); free(th); free(wa); return -1; }

    long long have = 0, tried = 0;
    uint64_t next_block = 0;
    while (have < n_events) {
        /* size the round from the acceptance rate seen so far */
        double rate = tried > 0 && have > 0 ? (double)have / (double)tried : 0.02;
        double want = 1.25 * (double)(n_events - have) / (rate * block) + 1.0;
        int nb = want > per_round ? per_round : (int)want;
        if (nb < 1) nb = 1;
        for (int t = 0; t < n_threads; ++t) {
            wa[t] = (worker_arg){&c, next_block, nb, t, n_threads, block, buf, cnt};
            pthread_create(&th[t], NULL, worker, &wa[t]);
        }
        for (int t = 0; t < n_threads; ++t) pthread_join(th[t], NULL);
        tried += (long long)nb * block;
        for (int b = 0; b < nb && have < n_events; ++b) {
            const mc_event *src = buf + (size_t)b * block;
            for (int k = 0; k < cnt[b] && have < n_events; ++k, ++have) {
                angle[have] = src[k].angle;
                u_bin[have] = src[k].u_bin;
                energy[have] = src[k].energy;
                if (kind) kind[have] = src[k].kind;
            }
        }
        next_block += nb;
        if (next_block > (1ull << 30)) break;   /* an object that detects nothing */
    }
    free(cdf); free(buf); free(cnt); free(th); free(wa);
    return have == n_events ? (long long)(next_block * (uint64_t)block) : -1;
}
