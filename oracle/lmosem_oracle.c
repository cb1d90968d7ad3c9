/*
 * FP64 CPU oracle for list-mode OSEM with attenuation and first-order scatter
 * compensation (Rahman, Laforest, Jha, "A list-mode OSEM-based attenuation
 * and scatter compensation method for SPECT", ISBI 2020).
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code
 * with the GPU library and must never sit on its execution path.
 *
 * Plain, slow and obviously correct: every quantity is evaluated from its
 * definition in double precision, with no lookup tables, no blocking and no
 * reordering.  The only memoisation is of pure functions of the geometry
 * (line integrals), computed once per model.
 *
 * The system model follows Sec. 2.1: an event's density is a mixture over
 * paths (Eq. 2), each path weighted by the activity of its start pixel times
 * an activity-independent path sensitivity s_eff (Eq. 4).  The paper states
 * only what s_eff must model (attenuation, scatter, collimator); the concrete
 * model implemented here is:
 *
 *   grid      N x N pixels of pitch dx; pixel p = (i, j) stored [j][i] with
 *             centre ((i-(N-1)/2) dx, (j-(N-1)/2) dx)
 *   angles    theta_a = angle0 + 2 pi a / N_A; photons travel along
 *             n_a = (cos, sin) to the detector, whose axis is t_a = (-sin, cos);
 *             detector coordinate u = r . t_a over [-N_B w_B / 2, N_B w_B / 2]
 *   primary   path q -> detector: weight exp(-L_a(q)), ends at u_q(a), E0
 *   scatter   path q -> s -> detector (s in the mu > 0 support, s != q; only
 *             first order and in plane, Sec. 2.2):
 *               weight B(q,s) Psi(c)/Psi_bar exp(-rho(E'(c)) L_a(s)),
 *               B(q,s) = mu(s) dx^2 exp(-l(q,s)) / (2 pi |c_s - c_q|),
 *               c = unit(c_s - c_q) . n_a, E'(c) the Compton energy,
 *             ends at u_s(a) with energy E'(c)
 *   response  position: truncated shifted Gaussian K (|d| < 3 sigma_u);
 *             energy: Gaussian G with constant sigma_E
 *   h(q; a,u,E) = sum over paths from q of weight * K(u - u_end) * G(E; E_end)
 *   sens_q   = T sum_{a in subset} sum over paths of weight * D(u_end) * W(E_end)
 *             with D, W the detector and window acceptances of K and G.
 *
 * Pins (tests/test_oracle_*.py): Compton energy by energy-momentum
 * conservation; KN total by quadrature of the differential form and its
 * Thomson / high-energy limits; Psi_bar by its closed form; line integrals by
 * chord lengths, disk chords and brute-force sums; B(q,s) by the interaction
 * probability 1 - exp(-mu R); rows against sensitivities by integration over
 * (u, E); the mu = 0 case against textbook list-mode EM; and the scatter
 * fraction, energy spectrum and position profiles against an independent
 * Monte-Carlo photon simulation.  Fidelity to the authors' own (unpublished)
 * s_eff is parity unpinned: the paper prints no values to compare with.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_ME_C2_KEV 510.99895

typedef struct {
    int n;              /* grid is n x n */
    double dx;          /* pixel pitch, cm */
    int n_bins;
    double bin_cm;
    int n_angles;
    double angle0;
    double e0, fwhm_e, fwhm_u;
    double win_lo, win_hi;
    int n_subsets;
    int scatter;        /* 0: primary paths only, 1: primary + first-order scatter */
    double acq_time;
} orc_config;

typedef struct {
    orc_config c;
    double *mu;         /* [n*n] */
    int n_pix, n_sup;
    int *sup;           /* support pixels (mu > 0), ascending */
    int *sup_index;     /* pixel -> support index or -1 */
    double *L;          /* [n_angles][n_pix] line integral from pixel centre to the detector */
    double *ell;        /* [n_sup][n_sup] line integral between support pixel centres */
    int ell_ready;      /* ell is filled only for scatter models */
    double sigma_e, sigma_u, psi_bar;
    int n_threads;
} orc_model;

/* ------------------------------------------------------------------ */
/* Radiological path (Siddon, Med. Phys. 12(2), 1985): the exact integral
 * of the piecewise-constant map along the segment p0 -> p1.  Crossings of
 * the vertical and horizontal pixel boundaries are generated in increasing
 * order of the segment parameter, merged, and each sub-segment is charged
 * to the pixel containing its midpoint.                                   */
double orc_line_integral(const double *mu, int n, double dx,
                         double x0, double y0, double x1, double y1) {
    double ddx = x1 - x0, ddy = y1 - y0;
    double len = sqrt(ddx * ddx + ddy * ddy);
    if (len == 0.0) return 0.0;
    double half = 0.5 * n * dx;
    /* crossing parameters with x = -half + k dx and y = -half + k dx */
    double ax[n + 1], ay[n + 1];
    int nxs = 0, nys = 0;
    if (ddx != 0.0) {
        for (int k = 0; k <= n; ++k) {
            int kk = ddx > 0 ? k : n - k;          /* increasing parameter order */
            double a = (-half + kk * dx - x0) / ddx;
            if (a > 0.0 && a < 1.0) ax[nxs++] = a;
        }
    }
    if (ddy != 0.0) {
        for (int k = 0; k <= n; ++k) {
            int kk = ddy > 0 ? k : n - k;
            double a = (-half + kk * dx - y0) / ddy;
            if (a > 0.0 && a < 1.0) ay[nys++] = a;
        }
    }
    double sum = 0.0, prev = 0.0;
    int ix = 0, iy = 0;
    for (;;) {
        double next;
        if (ix < nxs && (iy >= nys || ax[ix] <= ay[iy])) next = ax[ix++];
        else if (iy < nys) next = ay[iy++];
        else next = 1.0;
        if (next > prev) {
            double am = 0.5 * (prev + next);
            double xm = x0 + am * ddx, ym = y0 + am * ddy;
            int i = (int)floor(xm / dx + 0.5 * n), j = (int)floor(ym / dx + 0.5 * n);
            if (i >= 0 && i < n && j >= 0 && j < n) sum += mu[j * n + i] * (next - prev) * len;
            prev = next;
        }
        if (next >= 1.0) break;
    }
    return sum;
}

/* ------------------------------------------------------------------ */
/* Photon physics.                                                      */

/* Compton relation: energy after scattering by an angle with cosine c */
double orc_compton_energy(double e, double c) {
    return e / (1.0 + (e / ORC_ME_C2_KEV) * (1.0 - c));
}

/* Klein-Nishina differential cross-section in units of r_e^2 / 2:
 * P^2 (P + 1/P - sin^2), P = E'/E                                      */
double orc_kn_shape(double e, double c) {
    double p = orc_compton_energy(e, c) / e;
    return p * p * (p + 1.0 / p - (1.0 - c * c));
}

/* Klein-Nishina total cross-section in units of r_e^2 (closed form) */
double orc_kn_total(double e) {
    double k = e / ORC_ME_C2_KEV;
    double l = log(1.0 + 2.0 * k);
    double a = (1.0 + k) / (k * k) * (2.0 * (1.0 + k) / (1.0 + 2.0 * k) - l / k);
    double b = l / (2.0 * k);
    double d = (1.0 + 3.0 * k) / ((1.0 + 2.0 * k) * (1.0 + 2.0 * k));
    return 2.0 * M_PI * (a + b - d);
}

/* attenuation scale at energy e relative to e0 (Compton-only) */
double orc_rho(double e, double e0) { return orc_kn_total(e) / orc_kn_total(e0); }

/* periodic trapezoid rule with m nodes over [0, 2 pi), divided by 2 pi */
double orc_circle_mean(double (*f)(double, void *), void *arg, int m) {
    double s = 0.0;
    for (int k = 0; k < m; ++k) s += f(2.0 * M_PI * k / m, arg);
    return s / m;
}

static double psi_of_angle(double phi, void *arg) { return orc_kn_shape(*(double *)arg, cos(phi)); }

/* in-plane normaliser: mean of the KN shape over the circle of directions */
double orc_psi_bar(double e0, int m) { return orc_circle_mean(psi_of_angle, &e0, m); }

/* ------------------------------------------------------------------ */
/* Detector response.                                                   */

static double sigma_of_fwhm(double fwhm) { return fwhm / (2.0 * sqrt(2.0 * log(2.0))); }

/* position response: Gaussian shifted down to zero at |d| = 3 sigma, truncated
 * there, normalised to unit integral                                      */
double orc_K(double d, double s) {
    if (fabs(d) >= 3.0 * s) return 0.0;
    double z = s * sqrt(2.0 * M_PI) * erf(3.0 / sqrt(2.0)) - 6.0 * s * exp(-4.5);
    return (exp(-d * d / (2.0 * s * s)) - exp(-4.5)) / z;
}

/* fraction of K(u - u_p) falling inside [lo, hi] */
static double K_mass(double u_p, double lo, double hi, double s) {
    double a = lo - u_p, b = hi - u_p;
    if (a < -3.0 * s) a = -3.0 * s;
    if (b > 3.0 * s) b = 3.0 * s;
    if (b <= a) return 0.0;
    double z = s * sqrt(2.0 * M_PI) * erf(3.0 / sqrt(2.0)) - 6.0 * s * exp(-4.5);
    double g = s * sqrt(M_PI / 2.0) * (erf(b / (sqrt(2.0) * s)) - erf(a / (sqrt(2.0) * s)));
    return (g - exp(-4.5) * (b - a)) / z;
}

/* fraction of K(u - u_p) falling on the detector [-half, half] */
double orc_D(double u_p, double half, double s) { return K_mass(u_p, -half, half, s); }

/* energy response */
double orc_G(double e, double ep, double s) {
    return exp(-(e - ep) * (e - ep) / (2.0 * s * s)) / (sqrt(2.0 * M_PI) * s);
}

/* fraction of G(.; ep) inside the acceptance window [lo, hi] */
double orc_W(double ep, double lo, double hi, double s) {
    return 0.5 * (erf((hi - ep) / (sqrt(2.0) * s)) - erf((lo - ep) / (sqrt(2.0) * s)));
}

/* ------------------------------------------------------------------ */
/* Model construction.                                                  */

static void centre(const orc_model *m, int p, double *x, double *y) {
    int n = m->c.n;
    *x = ((p % n) - 0.5 * (n - 1)) * m->c.dx;
    *y = ((p / n) - 0.5 * (n - 1)) * m->c.dx;
}

typedef struct {
    orc_model *m;
    int tid, nt;
} build_arg;

static void *build_L(void *p) {
    build_arg *b = (build_arg *)p;
    orc_model *m = b->m;
    int n = m->c.n;
    double far = 4.0 * n * m->c.dx;   /* beyond the grid in every direction */
    for (int idx = b->tid; idx < m->c.n_angles * m->n_pix; idx += b->nt) {
        int a = idx / m->n_pix, pix = idx % m->n_pix;
        double th = m->c.angle0 + 2.0 * M_PI * a / m->c.n_angles;
        double x, y;
        centre(m, pix, &x, &y);
        m->L[idx] = orc_line_integral(m->mu, n, m->c.dx, x, y, x + far * cos(th), y + far * sin(th));
    }
    return NULL;
}

static void *build_ell(void *p) {
    build_arg *b = (build_arg *)p;
    orc_model *m = b->m;
    int ns = m->n_sup;
    for (int qi = b->tid; qi < ns; qi += b->nt) {
        double xq, yq;
        centre(m, m->sup[qi], &xq, &yq);
        for (int si = 0; si < ns; ++si) {
            double xs, ys;
            centre(m, m->sup[si], &xs, &ys);
            m->ell[(size_t)qi * ns + si] =
                qi == si ? 0.0 : orc_line_integral(m->mu, m->c.n, m->c.dx, xq, yq, xs, ys);
        }
    }
    return NULL;
}

static void run_threads(void *(*fn)(void *), orc_model *m) {
    int nt = m->n_threads;
    pthread_t th[256];
    build_arg args[256];
    if (nt > 256) nt = 256;
    for (int t = 0; t < nt; ++t) {
        args[t] = (build_arg){m, t, nt};
        pthread_create(&th[t], NULL, fn, &args[t]);
    }
    for (int t = 0; t < nt; ++t) pthread_join(th[t], NULL);
}

int orc_model_create(const orc_config *cfg, const double *mu, int n_threads, orc_model **out) {
    if (!cfg || !mu || !out || cfg->n <= 0 || cfg->dx <= 0 || cfg->n_angles <= 0 ||
        cfg->n_bins <= 0 || cfg->fwhm_e <= 0 || cfg->fwhm_u <= 0 || cfg->win_lo >= cfg->win_hi ||
        cfg->n_subsets < 1 || cfg->n_subsets > cfg->n_angles)
        return -1;
    orc_model *m = (orc_model *)calloc(1, sizeof(orc_model));
    m->c = *cfg;
    m->n_pix = cfg->n * cfg->n;
    m->n_threads = n_threads > 0 ? n_threads : 1;
    m->mu = (double *)malloc(sizeof(double) * m->n_pix);
    memcpy(m->mu, mu, sizeof(double) * m->n_pix);
    m->sup_index = (int *)malloc(sizeof(int) * m->n_pix);
    m->sup = (int *)malloc(sizeof(int) * m->n_pix);
    for (int p = 0; p < m->n_pix; ++p) {
        if (!(mu[p] >= 0.0) || isinf(mu[p])) { free(m->mu); free(m->sup_index); free(m->sup); free(m); return -1; }
        m->sup_index[p] = -1;
        if (mu[p] > 0.0) { m->sup_index[p] = m->n_sup; m->sup[m->n_sup++] = p; }
    }
    m->sigma_e = sigma_of_fwhm(cfg->fwhm_e);
    m->sigma_u = sigma_of_fwhm(cfg->fwhm_u);
    m->psi_bar = orc_psi_bar(cfg->e0, 512);
    m->L = (double *)malloc(sizeof(double) * (size_t)cfg->n_angles * m->n_pix);
    run_threads(build_L, m);
    m->ell = (double *)malloc(sizeof(double) * (size_t)m->n_sup * (m->n_sup > 0 ? m->n_sup : 1));
    if (cfg->scatter) { run_threads(build_ell, m); m->ell_ready = 1; }
    *out = m;
    return 0;
}

void orc_model_free(orc_model *m) {
    if (!m) return;
    free(m->mu); free(m->sup); free(m->sup_index); free(m->L); free(m->ell); free(m);
}

int orc_n_support(const orc_model *m) { return m->n_sup; }
void orc_support(const orc_model *m, int *out) { memcpy(out, m->sup, sizeof(int) * m->n_sup); }
double orc_psi_bar_of(const orc_model *m) { return m->psi_bar; }
double orc_L(const orc_model *m, int a, int pix) { return m->L[(size_t)a * m->n_pix + pix]; }

/* scatter-point factor B(q,s): probability that a photon emitted at q
 * interacts in pixel s (2-D point-kernel, point pixels)                  */
double orc_B(const orc_model *m, int q, int s) {
    int qi = m->sup_index[q], si = m->sup_index[s];
    if (si < 0 || q == s) return 0.0;
    double xq, yq, xs, ys;
    centre(m, q, &xq, &yq);
    centre(m, s, &xs, &ys);
    double r = hypot(xs - xq, ys - yq);
    double ell = (qi >= 0 && m->ell_ready) ? m->ell[(size_t)qi * m->n_sup + si]
                         : orc_line_integral(m->mu, m->c.n, m->c.dx, xq, yq, xs, ys);
    return m->mu[s] * m->c.dx * m->c.dx * exp(-ell) / (2.0 * M_PI * r);
}

/* ------------------------------------------------------------------ */
/* System row: h(q; a, u, E) = sum_{P in P_q} pr(A|P) s_eff(P)  (Eq. 2/4 with
 * the normaliser of Eq. 4 left out; it cancels in Eq. 8).              */
double orc_h(const orc_model *m, int q, int a, double u, double e) {
    const orc_config *c = &m->c;
    double th = c->angle0 + 2.0 * M_PI * a / c->n_angles;
    double nx = cos(th), ny = sin(th), tx = -sin(th), ty = cos(th);
    double xq, yq;
    centre(m, q, &xq, &yq);
    double uq = xq * tx + yq * ty;
    double h = exp(-orc_L(m, a, q)) * orc_K(u - uq, m->sigma_u) * orc_G(e, c->e0, m->sigma_e);
    if (!c->scatter) return h;
    for (int k = 0; k < m->n_sup; ++k) {
        int s = m->sup[k];
        if (s == q) continue;
        double xs, ys;
        centre(m, s, &xs, &ys);
        double ks = orc_K(u - (xs * tx + ys * ty), m->sigma_u);
        if (ks == 0.0) continue;               /* K vanishes off its support */
        double r = hypot(xs - xq, ys - yq);
        double cs = ((xs - xq) * nx + (ys - yq) * ny) / r;
        double ep = orc_compton_energy(c->e0, cs);
        double w = orc_B(m, q, s) * orc_kn_shape(c->e0, cs) / m->psi_bar
                   * exp(-orc_rho(ep, c->e0) * orc_L(m, a, s));
        h += w * ks * orc_G(e, ep, m->sigma_e);
    }
    return h;
}

/* probability that a photon emitted at q is detected at angle a with position
 * in [ulo, uhi] and energy in [elo, ehi]: the integral of h(q; a, u, E) over
 * that box, i.e. every path weight times the mass of K and G in the box    */
double orc_box_prob(const orc_model *m, int q, int a, double ulo, double uhi,
                    double elo, double ehi) {
    const orc_config *c = &m->c;
    double th = c->angle0 + 2.0 * M_PI * a / c->n_angles;
    double nx = cos(th), ny = sin(th), tx = -sin(th), ty = cos(th);
    double xq, yq;
    centre(m, q, &xq, &yq);
    double s = exp(-orc_L(m, a, q)) * K_mass(xq * tx + yq * ty, ulo, uhi, m->sigma_u)
               * orc_W(c->e0, elo, ehi, m->sigma_e);
    if (!c->scatter) return s;
    for (int k = 0; k < m->n_sup; ++k) {
        int sp = m->sup[k];
        if (sp == q) continue;
        double xs, ys;
        centre(m, sp, &xs, &ys);
        double r = hypot(xs - xq, ys - yq);
        double cs = ((xs - xq) * nx + (ys - yq) * ny) / r;
        double ep = orc_compton_energy(c->e0, cs);
        double w = orc_B(m, q, sp) * orc_kn_shape(c->e0, cs) / m->psi_bar
                   * exp(-orc_rho(ep, c->e0) * orc_L(m, a, sp));
        s += w * K_mass(xs * tx + ys * ty, ulo, uhi, m->sigma_u) * orc_W(ep, elo, ehi, m->sigma_e);
    }
    return s;
}

/* per-angle sensitivity of pixel q: detection anywhere on the detector with
 * an energy inside the acceptance window                                 */
double orc_sens_angle(const orc_model *m, int q, int a) {
    double half = 0.5 * m->c.n_bins * m->c.bin_cm;
    return orc_box_prob(m, q, a, -half, half, m->c.win_lo, m->c.win_hi);
}

/* ------------------------------------------------------------------ */
/* Threaded drivers.                                                    */

typedef struct {
    const orc_model *m;
    const double *box;    /* ulo, uhi, elo, ehi for box sums */
    const int32_t *angle;
    const float *u_bin, *energy;
    long long n_ev;
    const int *qlist;
    int n_q;
    double *out;
    int subset;
    long long lo, hi;
} work_arg;

static double u_cm(const orc_model *m, float u_bin) {
    return ((double)u_bin - 0.5 * m->c.n_bins) * m->c.bin_cm;
}

static void *work_rows(void *p) {
    work_arg *w = (work_arg *)p;
    for (long long j = w->lo; j < w->hi; ++j)
        for (int k = 0; k < w->n_q; ++k)
            w->out[j * w->n_q + k] = orc_h(w->m, w->qlist[k], w->angle[j], u_cm(w->m, w->u_bin[j]),
                                           (double)w->energy[j]);
    return NULL;
}

static void *work_sens(void *p) {
    work_arg *w = (work_arg *)p;
    const orc_config *c = &w->m->c;
    for (long long k = w->lo; k < w->hi; ++k) {
        double s = 0.0;
        for (int a = 0; a < c->n_angles; ++a)
            if (w->subset < 0 || a % c->n_subsets == w->subset)
                s += orc_sens_angle(w->m, w->qlist[k], a);
        w->out[k] = c->acq_time * s;
    }
    return NULL;
}

static void split(void *(*fn)(void *), work_arg proto, long long n, int nt) {
    pthread_t th[256];
    work_arg args[256];
    if (nt > 256) nt = 256;
    if (nt < 1) nt = 1;
    for (int t = 0; t < nt; ++t) {
        args[t] = proto;
        args[t].lo = n * t / nt;
        args[t].hi = n * (t + 1) / nt;
        pthread_create(&th[t], NULL, fn, &args[t]);
    }
    for (int t = 0; t < nt; ++t) pthread_join(th[t], NULL);
}

/* out[j][k] = h(qlist[k]; event j) for every event and listed pixel */
int orc_system_matrix(const orc_model *m, const int32_t *angle, const float *u_bin,
                      const float *energy, long long n_ev, const int *qlist, int n_q, double *out) {
    for (long long j = 0; j < n_ev; ++j)
        if (angle[j] < 0 || angle[j] >= m->c.n_angles) return -2;
    for (int k = 0; k < n_q; ++k)
        if (qlist[k] < 0 || qlist[k] >= m->n_pix) return -2;
    work_arg w = {m, NULL, angle, u_bin, energy, n_ev, qlist, n_q, out, 0, 0, 0};
    split(work_rows, w, n_ev, m->n_threads);
    return 0;
}

/* out[k] = T sum_{a in subset} (per-angle sensitivity of qlist[k]); subset -1 = all angles */
int orc_sensitivity(const orc_model *m, int subset, const int *qlist, int n_q, double *out) {
    if (subset < -1 || subset >= m->c.n_subsets) return -2;
    work_arg w = {m, NULL, NULL, NULL, NULL, 0, qlist, n_q, out, subset, 0, 0};
    split(work_sens, w, n_q, m->n_threads);
    return 0;
}

static void *work_box(void *p) {
    work_arg *w = (work_arg *)p;
    for (long long k = w->lo; k < w->hi; ++k) {
        double s = 0.0;
        for (long long t = 0; t < w->n_ev; ++t)
            s += orc_box_prob(w->m, w->qlist[k], w->angle[t], w->box[0], w->box[1], w->box[2],
                              w->box[3]);
        w->out[k] = s;
    }
    return NULL;
}

/* out[k] = sum over the listed angles of the box probability of pixel qlist[k] */
int orc_box_sums(const orc_model *m, const int32_t *angles, int n_angles, double ulo, double uhi,
                 double elo, double ehi, const int *qlist, int n_q, double *out) {
    for (int t = 0; t < n_angles; ++t)
        if (angles[t] < 0 || angles[t] >= m->c.n_angles) return -2;
    double box[4] = {ulo, uhi, elo, ehi};
    work_arg w = {m, box, angles, NULL, NULL, n_angles, qlist, n_q, out, 0, 0, 0};
    split(work_box, w, n_q, m->n_threads);
    return 0;
}
