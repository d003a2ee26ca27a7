/*
 * epid_oracle.c -- plain, slow, single-threaded FP64 oracle of the EPID transit
 * Monte Carlo hot path.  TEST INFRASTRUCTURE ONLY (see epid_oracle.h).
 *
 * The paper (Sec. 2.1.2) fixes the physics class only: photoelectric, Compton and
 * pair production for photons; Class II condensed history for electrons (discrete
 * hard collisions, continuous slowing down for soft ones); cut-offs 10 keV (photons)
 * and 200 keV (electrons); a voxelised density matrix derived from HU; a multi-layer
 * EPID (Sec. 2.1.3) scored on a 2D pixel grid (Sec. 2.3.3).  Every model detail the
 * paper leaves open is fixed by an explicit reading shared with the engine; this file
 * implements those readings as plainly as possible:
 *   - cross sections are computed from their formulas at every energy (no tables);
 *   - photons are tracked voxel by voxel (Amanatides-Woo), not by delta tracking;
 *   - Klein-Nishina and Moller variates come from numerically inverted closed-form CDFs;
 *   - the restricted range integral and its inverse use Gauss-Legendre quadrature and
 *     Newton iteration in FP64;
 *   - the per-pixel variance is accumulated history by history.
 */
#include "epid_oracle.h"
#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

/* CODATA 2018 */
#define MEC2   0.51099895
#define RE_CM  2.8179403262e-13
#define NAVO   6.02214076e23
#define ALPHA_FS (1.0 / 137.035999084)
#define PI     3.14159265358979323846

/* model constants fixed by the readings of the paper's physics class */
#define C_PE     2.89e-32      /* photoelectric: sigma = C_PE * Z^4 / E^3 (cm^2 MeV^3 per atom) */
#define BREM_K   800.0         /* S_rad / S_col = Z_eff * T / BREM_K (T in MeV) */
#define WCUT     0.200         /* Moller hard-collision threshold (MeV) */
#define KCUT     0.010         /* bremsstrahlung hard-photon threshold (MeV) */
#define NUDGE    1.0e-5        /* cm pushed past a geometric boundary by a boundary-limited step */
#define DE_FRAC  0.9           /* a step may take the energy down to DE_FRAC * T0 at most */
#define MAX_E_STEPS 1000000

enum { R_PHANTOM = 0, R_EPID = 1, R_ESCAPED = 2 };
enum { P_PHOTON = 0, P_ELECTRON = 1, P_POSITRON = 2 };

/* ------------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds of the 4x32      */
/* multiply-xor round with key schedule bumped by the Weyl constants.            */
/* ------------------------------------------------------------------------- */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* The oracle's own stream: one per history, counter = (n_lo, n_hi, history, tag). */
typedef struct {
    uint32_t key[2];
    uint32_t ctr[4];
    uint32_t buf[4];
    int      have;   /* words left in buf */
} orng;

static void orng_init(orng *g, uint64_t seed, uint64_t history)
{
    g->key[0] = (uint32_t)seed;
    g->key[1] = (uint32_t)(seed >> 32);
    g->ctr[0] = 0; g->ctr[1] = 0;
    g->ctr[2] = (uint32_t)history;
    g->ctr[3] = 0x4F52434Cu ^ (uint32_t)(history >> 32);
    g->have = 0;
}

static uint32_t orng_word(orng *g)
{
    if (g->have == 0) {
        orc_philox4x32_10(g->ctr, g->key, g->buf);
        if (++g->ctr[0] == 0) ++g->ctr[1];
        g->have = 4;
    }
    return g->buf[4 - g->have--];
}

/* uniform in the open interval (0,1) with 52 random bits */
static double orng_u(orng *g)
{
    uint32_t a = orng_word(g) >> 6, b = orng_word(g) >> 6;
    return ((double)a * 67108864.0 + (double)b + 0.5) * (1.0 / 4503599627370496.0);
}

/* ------------------------------------------------------------------------- */
/* Material-derived quantities                                                */
/* ------------------------------------------------------------------------- */
static double mat_ne(const orc_material *m)           /* electrons per gram */
{
    double s = 0; for (int i = 0; i < m->n_elem; ++i) s += m->w[i] * m->Z[i] / m->A[i];
    return NAVO * s;
}
static double mat_zeff(const orc_material *m)         /* electron-weighted mean Z */
{
    double a = 0, b = 0;
    for (int i = 0; i < m->n_elem; ++i) { a += m->w[i] * m->Z[i] * (double)m->Z[i] / m->A[i]; b += m->w[i] * m->Z[i] / m->A[i]; }
    return a / b;
}

double orc_x0(const orc_material *m)
{
    /* Dahl's approximation per element, combined as 1/X0 = sum w_i / X0_i (g/cm^2) */
    double inv = 0;
    for (int i = 0; i < m->n_elem; ++i) {
        double Z = m->Z[i];
        double x0 = 716.4 * m->A[i] / (Z * (Z + 1.0) * log(287.0 / sqrt(Z)));
        inv += m->w[i] / x0;
    }
    return 1.0 / inv;
}

/* ------------------------------------------------------------------------- */
/* Photon cross sections                                                      */
/* ------------------------------------------------------------------------- */
double orc_sigma_kn(double E)
{
    /* Klein-Nishina total cross section per free electron (cm^2) */
    double k = E / MEC2;
    double l = log(1.0 + 2.0 * k);
    double t1 = (1.0 + k) / (k * k) * (2.0 * (1.0 + k) / (1.0 + 2.0 * k) - l / k);
    double t2 = l / (2.0 * k);
    double t3 = (1.0 + 3.0 * k) / ((1.0 + 2.0 * k) * (1.0 + 2.0 * k));
    return 2.0 * PI * RE_CM * RE_CM * (t1 + t2 - t3);
}

static double sigma_pe_atom(int Z, double E)
{
    double z2 = (double)Z * Z;
    return C_PE * z2 * z2 / (E * E * E);
}

static double sigma_pair_atom(int Z, double E)
{
    /* zero at and below the 2 m c^2 threshold; Bethe-Heitler-like log growth above */
    if (E <= 2.0 * MEC2) return 0.0;
    double r = 1.0 - 2.0 * MEC2 / E;
    return (28.0 / 9.0) * ALPHA_FS * RE_CM * RE_CM * (double)Z * Z * log(E / (2.0 * MEC2)) * r * r;
}

void orc_photon_mu(const orc_material *m, double E, double out[4])
{
    double c = 0, p = 0, q = 0;
    double skn = orc_sigma_kn(E);
    for (int i = 0; i < m->n_elem; ++i) {
        double nat = NAVO * m->w[i] / m->A[i];          /* atoms per gram of element i */
        c += nat * m->Z[i] * skn;
        p += nat * sigma_pe_atom(m->Z[i], E);
        q += nat * sigma_pair_atom(m->Z[i], E);
    }
    out[1] = c; out[2] = p; out[3] = q;
    out[0] = c + p + q;
}

/* KN density in eps = E'/E (unnormalised): f = 1/eps + eps - sin^2(theta) with
 * 1 - cos(theta) = a (1/eps - 1), a = 1/kappa.  Its antiderivative from eps0 = 1/(1+2 kappa)
 * is written out term by term below. */
static double kn_F(double a, double e0, double e)
{
    double b = (1.0 + a) * (1.0 + a) - 1.0;
    double c = 1.0 - 2.0 * a - 2.0 * a * a;
    return 0.5 * (e * e - e0 * e0) + b * (e - e0) + c * log(e / e0) + a * a * (1.0 / e0 - 1.0 / e);
}
static double kn_f(double a, double e)
{
    double b = (1.0 + a) * (1.0 + a) - 1.0;
    double c = 1.0 - 2.0 * a - 2.0 * a * a;
    return e + b + c / e + a * a / (e * e);
}

double orc_kn_cdf(double E, double eps)
{
    double k = E / MEC2, a = 1.0 / k, e0 = 1.0 / (1.0 + 2.0 * k);
    if (eps <= e0) return 0.0;
    if (eps >= 1.0) return 1.0;
    return kn_F(a, e0, eps) / kn_F(a, e0, 1.0);
}

double orc_kn_sample(double E, double xi)
{
    /* invert the closed-form CDF: safeguarded Newton on [eps0, 1] */
    double k = E / MEC2, a = 1.0 / k, e0 = 1.0 / (1.0 + 2.0 * k);
    double target = xi * kn_F(a, e0, 1.0);
    double lo = e0, hi = 1.0, e = e0 + xi * (1.0 - e0);
    for (int it = 0; it < 200; ++it) {
        double g = kn_F(a, e0, e) - target;
        if (g > 0) hi = e; else lo = e;
        double en = e - g / kn_f(a, e);
        if (!(en > lo && en < hi)) en = 0.5 * (lo + hi);
        if (fabs(en - e) <= 1e-15 * e) { e = en; break; }
        e = en;
        if (hi - lo <= 1e-15) break;
    }
    return e;
}

/* ------------------------------------------------------------------------- */
/* Electron stopping powers and hard-collision cross sections                */
/* ------------------------------------------------------------------------- */
double orc_lcol(const orc_material *m, double T, int restricted, double wcut)
{
    /* Bethe collision stopping power for electrons (ICRU Report 37 form), no density
     * effect; restricted to energy transfers below min(wcut, T/2) when asked. */
    double tau = T / MEC2, g = tau + 1.0;
    double b2 = 1.0 - 1.0 / (g * g);
    double Ir = m->I_eV * 1e-6 / MEC2;
    double D = restricted ? fmin(wcut / MEC2, 0.5 * tau) : 0.5 * tau;
    double F = -1.0 - b2 + log((tau - D) * D) + tau / (tau - D)
             + (0.5 * D * D + (2.0 * tau + 1.0) * log(1.0 - D / tau)) / (g * g);
    double br = log(2.0 * (tau + 2.0) / (Ir * Ir)) + F;
    return 2.0 * PI * RE_CM * RE_CM * MEC2 * mat_ne(m) / b2 * br;
}

double orc_srad(const orc_material *m, double T)
{
    /* radiative stopping power by the textbook ratio S_rad / S_col = Z_eff T / BREM_K */
    return orc_lcol(m, T, 0, 0.0) * mat_zeff(m) * T / BREM_K;
}

double orc_lres(const orc_material *m, double T, double wcut, double kcut)
{
    /* restricted collision loss + soft (k < kcut) part of the 1/k bremsstrahlung spectrum */
    return orc_lcol(m, T, 1, wcut) + orc_srad(m, T) * kcut / T;
}

double orc_sigma_moller(const orc_material *m, double T, double wcut)
{
    if (T <= 2.0 * wcut) return 0.0;
    double g = T / MEC2 + 1.0;
    double b2 = 1.0 - 1.0 / (g * g);
    double ec = wcut / T;
    double c1 = (g - 1.0) * (g - 1.0) / (g * g), c2 = (2.0 * g - 1.0) / (g * g);
    double I = c1 * (0.5 - ec) + 1.0 / ec - 1.0 / (1.0 - ec) - c2 * log((1.0 - ec) / ec);
    return mat_ne(m) * 2.0 * PI * RE_CM * RE_CM * MEC2 / (b2 * T) * I;
}

double orc_sigma_brems(const orc_material *m, double T, double kcut)
{
    if (T <= kcut) return 0.0;
    return orc_srad(m, T) / T * log(T / kcut);
}

double orc_brems_sample(double T, double kcut, double xi)
{
    /* the 1/k spectrum on [kcut, T]: its CDF ln(k/kcut)/ln(T/kcut) inverted */
    return kcut * exp(xi * log(T / kcut));
}

double orc_sigma_hard_max(const orc_material *m, double T0, double wcut, double kcut)
{
    /* the largest hard cross section over the energies a step from T0 can reach, [0.9 T0, T0]:
     * Sigma_Moller + Sigma_brems rises with T on the electron energies in use (a pinned
     * property), so the larger of the two end values bounds it */
    double a = orc_sigma_moller(m, T0, wcut) + orc_sigma_brems(m, T0, kcut);
    double b = orc_sigma_moller(m, DE_FRAC * T0, wcut) + orc_sigma_brems(m, DE_FRAC * T0, kcut);
    return a > b ? a : b;
}

double orc_moller_sample(double T, double wcut, double xi)
{
    /* invert the integrated Moller cross section over eps = W/T in [wcut/T, 1/2] by bisection */
    double g = T / MEC2 + 1.0;
    double ec = wcut / T;
    double c1 = (g - 1.0) * (g - 1.0) / (g * g), c2 = (2.0 * g - 1.0) / (g * g);
#define MOLLER_F(e) (c1 * ((e) - ec) + (1.0 / ec - 1.0 / (e)) + (1.0 / (1.0 - (e)) - 1.0 / (1.0 - ec)) \
                     - c2 * (log((e) / (1.0 - (e))) - log(ec / (1.0 - ec))))
    double tot = MOLLER_F(0.5);
    double lo = ec, hi = 0.5;
    for (int it = 0; it < 200 && hi - lo > 1e-15; ++it) {
        double mid = 0.5 * (lo + hi);
        if (MOLLER_F(mid) < xi * tot) lo = mid; else hi = mid;
    }
#undef MOLLER_F
    return 0.5 * (lo + hi) * T;
}

/* Gauss-Legendre nodes on [-1,1], computed once by Newton iteration on P_n */
#define GL_N 8
static double gl_x[GL_N], gl_w[GL_N];
static pthread_once_t gl_once = PTHREAD_ONCE_INIT;
static void gl_init(void)
{
    for (int i = 0; i < GL_N; ++i) {
        double x = cos(PI * (i + 0.75) / (GL_N + 0.5)), dp = 0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = x;
            for (int k = 2; k <= GL_N; ++k) { double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k; p0 = p1; p1 = p2; }
            dp = GL_N * (x * p1 - p0) / (x * x - 1.0);
            double dx = p1 / dp;
            x -= dx;
            if (fabs(dx) < 1e-16) break;
        }
        gl_x[i] = x;
        gl_w[i] = 2.0 / ((1.0 - x * x) * dp * dp);
    }
}

static double gl_inv_l(const orc_material *m, double a, double b, double wcut, double kcut)
{
    double h = 0.5 * (b - a), c = 0.5 * (a + b), s = 0;
    for (int i = 0; i < GL_N; ++i) s += gl_w[i] / orc_lres(m, c + h * gl_x[i], wcut, kcut);
    return s * h;
}

double orc_range_diff(const orc_material *m, double T_lo, double T_hi, double wcut, double kcut)
{
    /* integral of dT / L_res over [T_lo, T_hi] (g/cm^2); the restricted stopping power has a
     * kink at T = 2 wcut, so the interval is split there, and long intervals are subdivided
     * geometrically so every panel spans at most 5% in energy */
    pthread_once(&gl_once, gl_init);
    if (T_hi <= T_lo) return 0.0;
    double s = 0, a = T_lo;
    double kink = 2.0 * wcut;
    while (a < T_hi) {
        double b = fmin(T_hi, a * 1.05);
        if (a < kink && b > kink) b = kink;
        s += gl_inv_l(m, a, b, wcut, kcut);
        a = b;
    }
    return s;
}

double orc_range_inverse(const orc_material *m, double T0, double dR, double wcut, double kcut)
{
    /* T1 < T0 with range_diff(T1, T0) = dR, by Newton iteration with a bisection safeguard */
    if (dR <= 0) return T0;
    double lo = 1e-3, hi = T0;
    if (orc_range_diff(m, lo, T0, wcut, kcut) <= dR) return lo;
    double T1 = T0 - dR * orc_lres(m, T0, wcut, kcut);
    if (!(T1 > lo && T1 < hi)) T1 = 0.5 * (lo + hi);
    for (int it = 0; it < 100; ++it) {
        double g = orc_range_diff(m, T1, T0, wcut, kcut) - dR;   /* decreasing in T1 */
        if (g > 0) lo = T1; else hi = T1;
        double Tn = T1 + g * orc_lres(m, T1, wcut, kcut);
        if (!(Tn > lo && Tn < hi)) Tn = 0.5 * (lo + hi);
        if (fabs(Tn - T1) <= 1e-14 * T0) { T1 = Tn; break; }
        T1 = Tn;
    }
    return T1;
}

double orc_highland(double T, double x, double X0)
{
    /* Highland-Lynch-Dahl width of the projected angle, unit charge */
    if (x <= 0) return 0.0;
    double E = T + MEC2;
    double pc2 = T * (T + 2.0 * MEC2);
    double bcp = pc2 / E;
    double b2 = pc2 / (E * E);
    double br = 1.0 + 0.038 * log(x / (X0 * b2));
    if (br < 0) br = 0;
    return 13.6 / bcp * sqrt(x / X0) * br;
}

/* ------------------------------------------------------------------------- */
/* Geometry                                                                   */
/* ------------------------------------------------------------------------- */
typedef struct {
    const orc_config *c;
    double bmin[3], bmax[3];               /* phantom box */
    double zl[ORC_MAX_LAYERS + 1];         /* EPID layer planes */
    double hx, hy;                         /* EPID lateral half extents */
    double *mu_cache;                      /* [n_mat][4] at mu_E */
    double mu_E;
    double x0[ORC_MAX_MAT];
} geo_t;

static int in_box(const geo_t *g, const double p[3])
{
    for (int a = 0; a < 3; ++a) if (!(p[a] >= g->bmin[a] && p[a] < g->bmax[a])) return 0;
    return 1;
}

static int epid_layer_of(const geo_t *g, const double p[3])
{
    /* -1 when outside the EPID slab stack (half-open planes and lateral extent) */
    if (!(p[0] >= -g->hx && p[0] < g->hx && p[1] >= -g->hy && p[1] < g->hy)) return -1;
    for (int l = 0; l < g->c->n_layers; ++l) if (p[2] >= g->zl[l] && p[2] < g->zl[l + 1]) return l;
    return -1;
}

static void voxel_of(const geo_t *g, const double p[3], int idx[3])
{
    const int n[3] = { g->c->nx, g->c->ny, g->c->nz };
    for (int a = 0; a < 3; ++a) {
        int i = (int)floor((p[a] - g->bmin[a]) / g->c->spacing[a]);
        if (i < 0) i = 0;
        if (i >= n[a]) i = n[a] - 1;
        idx[a] = i;
    }
}

/* Particle outside every region moves on a straight line: first the phantom box (if its
 * ray enters it), else the EPID front face within its lateral extent, else it escapes.
 * Particles that leave the EPID never come back. */
static int vacuum_move(const geo_t *g, double p[3], const double d[3], int prev_region)
{
    if (prev_region == R_EPID) return R_ESCAPED;
    double tin = -INFINITY, tout = INFINITY;
    int hit_box = 1;
    for (int a = 0; a < 3; ++a) {
        if (d[a] != 0) {
            double t1 = (g->bmin[a] - p[a]) / d[a], t2 = (g->bmax[a] - p[a]) / d[a];
            if (t1 > t2) { double t = t1; t1 = t2; t2 = t; }
            if (t1 > tin) tin = t1;
            if (t2 < tout) tout = t2;
        } else if (!(p[a] >= g->bmin[a] && p[a] < g->bmax[a])) hit_box = 0;
    }
    double tb = (hit_box && tin > 0 && tin < tout) ? tin : INFINITY;
    double te = INFINITY;
    if (d[2] > 0 && p[2] <= g->zl[0]) {
        double t = (g->zl[0] - p[2]) / d[2];
        double x = p[0] + t * d[0], y = p[1] + t * d[1];
        if (x >= -g->hx && x < g->hx && y >= -g->hy && y < g->hy) te = t;
    }
    if (tb == INFINITY && te == INFINITY) return R_ESCAPED;
    if (tb <= te) {
        for (int a = 0; a < 3; ++a) p[a] += tb * d[a];
        return R_PHANTOM;
    }
    p[0] += te * d[0]; p[1] += te * d[1]; p[2] = g->zl[0];
    return R_EPID;
}

/* where a particle at p (moving along d) belongs after it was last in region r */
static int classify(const geo_t *g, double p[3], const double d[3], int r)
{
    if (r == R_PHANTOM) return in_box(g, p) ? R_PHANTOM : vacuum_move(g, p, d, R_PHANTOM);
    if (r == R_EPID) return epid_layer_of(g, p) >= 0 ? R_EPID : R_ESCAPED;
    if (in_box(g, p)) return R_PHANTOM;
    return vacuum_move(g, p, d, -1);
}

/* rotate unit vector d by polar angle (cos_t, sin_t) and azimuth phi, using an explicit
 * orthonormal frame built around d */
static void rotate(double d[3], double ct, double st, double phi)
{
    double ax[3] = { 0, 0, 0 };
    double a0 = fabs(d[0]), a1 = fabs(d[1]), a2 = fabs(d[2]);
    if (a0 <= a1 && a0 <= a2) ax[0] = 1; else if (a1 <= a2) ax[1] = 1; else ax[2] = 1;
    double e1[3] = { d[1] * ax[2] - d[2] * ax[1], d[2] * ax[0] - d[0] * ax[2], d[0] * ax[1] - d[1] * ax[0] };
    double n = sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
    e1[0] /= n; e1[1] /= n; e1[2] /= n;
    double e2[3] = { d[1] * e1[2] - d[2] * e1[1], d[2] * e1[0] - d[0] * e1[2], d[0] * e1[1] - d[1] * e1[0] };
    double cp = cos(phi), sp = sin(phi), r[3];
    for (int a = 0; a < 3; ++a) r[a] = ct * d[a] + st * (cp * e1[a] + sp * e2[a]);
    n = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    for (int a = 0; a < 3; ++a) d[a] = r[a] / n;
}

static void isotropic(orng *rng, double d[3])
{
    double ct = 2.0 * orng_u(rng) - 1.0, phi = 2.0 * PI * orng_u(rng);
    double st = sqrt(fmax(0.0, 1.0 - ct * ct));
    d[0] = st * cos(phi); d[1] = st * sin(phi); d[2] = ct;
}

/* ------------------------------------------------------------------------- */
/* Transport                                                                   */
/* ------------------------------------------------------------------------- */
typedef struct {
    double p[3], d[3], E;
    int    type, region, unscat;
} part_t;

#define STACK_MAX 4096
typedef struct {
    geo_t     *g;
    orng       rng;
    part_t     st[STACK_MAX];
    int        n;
    /* history accumulators */
    double    *hacc;           /* per pixel, this history */
    int       *touched;
    int        ntouched;
    double     dep, esc, rest;  /* ledger of this history */
    orc_counters *cnt;
    int        err;
    uint64_t   hist;           /* history being transported */
    orc_event *ev;             /* optional event trace */
    uint64_t   ev_cap, ev_n;
} ctx_t;

/* the next trace record (zeroed), or NULL when tracing is off or the buffer is full */
static orc_event *ev_new(ctx_t *c, int kind, const double p[3])
{
    if (!c->ev) return NULL;
    uint64_t i = c->ev_n++;
    if (i >= c->ev_cap) return NULL;
    orc_event *e = &c->ev[i];
    memset(e, 0, sizeof *e);
    e->hist = c->hist;
    e->kind = kind;
    e->region = -1;
    e->layer = -1;
    e->pixel = -1;
    for (int a = 0; a < 3; ++a) e->pos[a] = p[a];
    return e;
}

static void vcopy(double d[3], const double s[3]) { d[0] = s[0]; d[1] = s[1]; d[2] = s[2]; }

static void push(ctx_t *c, const double p[3], const double d[3], double E, int type, int region, int unscat)
{
    if (c->n >= STACK_MAX) { c->err = ORC_E_LOOP; return; }
    part_t *q = &c->st[c->n++];
    memcpy(q->p, p, sizeof q->p); memcpy(q->d, d, sizeof q->d);
    q->E = E; q->type = type; q->region = region; q->unscat = unscat;
}

/* energy deposit: always in the ledger; tallied when it lies in the scoring layer and the image */
static void deposit(ctx_t *c, int region, int layer, const double p[3], double E)
{
    const orc_config *cf = c->g->c;
    orc_event *ev = ev_new(c, ORC_EV_DEPOSIT, p);
    if (ev) { ev->region = (region == R_PHANTOM || region == R_EPID) ? region : -1; ev->layer = layer; ev->E0 = E; }
    c->dep += E;
    if (region == R_PHANTOM) { c->cnt->e_dep_phantom += E; return; }
    if (region != R_EPID) { c->cnt->e_dep_other += E; return; }
    c->cnt->e_dep_epid += E;
    if (layer != cf->scoring_layer || E == 0.0) return;
    double fu = floor((p[0] + c->g->hx) / cf->pitch_u), fv = floor((p[1] + c->g->hy) / cf->pitch_v);
    if (!(fu >= 0 && fu < cf->npx_u && fv >= 0 && fv < cf->npx_v)) return;
    int pix = (int)fv * cf->npx_u + (int)fu;
    if (ev) ev->pixel = pix;
    if (c->hacc[pix] == 0.0) c->touched[c->ntouched++] = pix;
    c->hacc[pix] += E;
    c->cnt->n_tally_deposits++;
}

/* point deposit located by position: the phantom box, or the EPID layer containing p */
static void deposit_at(ctx_t *c, int r, const double p[3], double E)
{
    int l = -1;
    if (r == R_PHANTOM) { if (!in_box(c->g, p)) r = -1; }
    else if (r == R_EPID) { l = epid_layer_of(c->g, p); if (l < 0) r = -1; }
    deposit(c, r, l, p, E);
}

static void escape(ctx_t *c, double E) { c->esc += E; c->cnt->e_escaped += E; }

static void spawn(ctx_t *c, const double p[3], const double d[3], double E, int type, int r);

/* a positron at rest at p (region r) annihilates into two photons of m c^2, back to back
 * along an isotropic direction (reading R4) */
static void annihilate(ctx_t *c, const double p[3], int r)
{
    double da[3], db[3];
    isotropic(&c->rng, da);
    db[0] = -da[0]; db[1] = -da[1]; db[2] = -da[2];
    c->cnt->n_annih++;
    c->rest -= 2.0 * MEC2;
    orc_event *ev = ev_new(c, ORC_EV_ANNIH, p);
    if (ev) { ev->Ec[0] = MEC2; ev->Ec[1] = MEC2; vcopy(ev->dc[0], da); vcopy(ev->dc[1], db); }
    spawn(c, p, da, MEC2, P_PHOTON, r);
    spawn(c, p, db, MEC2, P_PHOTON, r);
}

/* a newly created particle of kinetic energy E at p in region r (the parent's region) */
static void spawn(ctx_t *c, const double p[3], const double d[3], double E, int type, int r)
{
    const orc_config *cf = c->g->c;
    if (type == P_PHOTON) {
        if (E < cf->pcut) { deposit_at(c, r, p, E); return; }
    } else {
        if (!cf->coupled || E < cf->ecut) {
            deposit_at(c, r, p, E);
            if (type == P_POSITRON) annihilate(c, p, r);
            return;
        }
    }
    double q[3] = { p[0], p[1], p[2] };
    int nr = classify(c->g, q, d, r);
    if (nr == R_ESCAPED) { escape(c, E); return; }
    push(c, q, d, E, type, nr, 0);
}

static const double *mu_at(geo_t *g, double E)
{
    if (E != g->mu_E) {
        uint32_t pm = g->c->proc_mask;
        for (int m = 0; m < g->c->n_mat; ++m) {
            double *o = g->mu_cache + 4 * m;
            orc_photon_mu(&g->c->mat[m], E, o);
            /* only the enabled processes attenuate the photon */
            o[0] = ((pm & 1) ? o[1] : 0.0) + ((pm & 2) ? o[2] : 0.0) + ((pm & 4) ? o[3] : 0.0);
        }
        g->mu_E = E;
    }
    return g->mu_cache;
}

/* photon interaction in material m at point p (region r, EPID layer for the tally) */
static void photon_interact(ctx_t *c, part_t *ph, int m, int *alive)
{
    const orc_config *cf = c->g->c;
    const double *mu = mu_at(c->g, ph->E) + 4 * m;
    double muc = (cf->proc_mask & 1) ? mu[1] : 0, mup = (cf->proc_mask & 2) ? mu[2] : 0,
           mur = (cf->proc_mask & 4) ? mu[3] : 0;
    double x = orng_u(&c->rng) * (muc + mup + mur);
    int first = ph->unscat && ph->region == R_EPID && epid_layer_of(c->g, ph->p) == cf->scoring_layer;
    ph->unscat = 0;
    if (x < muc) {
        c->cnt->n_compton++;
        double E = ph->E;
        double eps = orc_kn_sample(E, orng_u(&c->rng));
        double k = E / MEC2;
        double ct = 1.0 - (1.0 / eps - 1.0) / k;
        if (ct < -1) ct = -1;
        if (ct > 1) ct = 1;
        double st = sqrt(fmax(0.0, 1.0 - ct * ct));
        double phi = 2.0 * PI * orng_u(&c->rng);
        double d0[3] = { ph->d[0], ph->d[1], ph->d[2] };
        rotate(ph->d, ct, st, phi);
        double Ep = eps * E, T = E - Ep;
        /* electron direction from momentum conservation: p_e = E d0 - E' d1 */
        double pe[3] = { E * d0[0] - Ep * ph->d[0], E * d0[1] - Ep * ph->d[1], E * d0[2] - Ep * ph->d[2] };
        double n = sqrt(pe[0] * pe[0] + pe[1] * pe[1] + pe[2] * pe[2]);
        if (n > 0) { pe[0] /= n; pe[1] /= n; pe[2] /= n; } else { pe[0] = d0[0]; pe[1] = d0[1]; pe[2] = d0[2]; }
        ph->E = Ep;
        if (first) { c->cnt->n_first_collision++; c->cnt->e_first_collision += T; }
        orc_event *ev = ev_new(c, ORC_EV_COMPTON, ph->p);
        if (ev) { ev->E0 = E; ev->E1 = Ep; vcopy(ev->d0, d0); vcopy(ev->d1, ph->d); ev->Ec[0] = T; vcopy(ev->dc[0], pe); }
        spawn(c, ph->p, pe, T, P_ELECTRON, ph->region);
        if (Ep < cf->pcut) { deposit_at(c, ph->region, ph->p, Ep); *alive = 0; }
    } else if (x < muc + mup) {
        c->cnt->n_photo++;
        if (first) { c->cnt->n_first_collision++; c->cnt->e_first_collision += ph->E; }
        orc_event *ev = ev_new(c, ORC_EV_PHOTO, ph->p);
        if (ev) { ev->E0 = ph->E; vcopy(ev->d0, ph->d); ev->Ec[0] = ph->E; vcopy(ev->dc[0], ph->d); }
        spawn(c, ph->p, ph->d, ph->E, P_ELECTRON, ph->region);
        *alive = 0;
    } else {
        c->cnt->n_pair++;
        double T = ph->E - 2.0 * MEC2;
        double tm = orng_u(&c->rng) * T, tp = T - tm;
        c->rest += 2.0 * MEC2;
        if (first) { c->cnt->n_first_collision++; c->cnt->e_first_collision += T; }
        orc_event *ev = ev_new(c, ORC_EV_PAIR, ph->p);
        if (ev) {
            ev->E0 = ph->E; vcopy(ev->d0, ph->d);
            ev->Ec[0] = tm; vcopy(ev->dc[0], ph->d); ev->Ec[1] = tp; vcopy(ev->dc[1], ph->d);
        }
        spawn(c, ph->p, ph->d, tm, P_ELECTRON, ph->region);
        spawn(c, ph->p, ph->d, tp, P_POSITRON, ph->region);
        *alive = 0;
    }
}

static void transport_photon(ctx_t *c, part_t ph)
{
    geo_t *g = c->g;
    const orc_config *cf = g->c;
    int alive = 1;
    while (alive) {
        if (ph.region == R_PHANTOM) {
            /* regular voxel-by-voxel tracking with an optical depth drawn once per flight */
            double tau = -log(orng_u(&c->rng));
            int idx[3]; voxel_of(g, ph.p, idx);
            const int n[3] = { cf->nx, cf->ny, cf->nz };
            double t = 0;
            int interacted = 0;
            for (;;) {
                c->cnt->voxel_visits++;
                long v = ((long)idx[2] * cf->ny + idx[1]) * cf->nx + idx[0];
                int m = cf->vox_mat[v];
                double mu = cf->vox_rho[v] * mu_at(g, ph.E)[4 * m];
                double tn = INFINITY; int ax = -1;
                for (int a = 0; a < 3; ++a) {
                    if (ph.d[a] > 0) { double tt = (g->bmin[a] + (idx[a] + 1) * cf->spacing[a] - ph.p[a]) / ph.d[a]; if (tt < tn) { tn = tt; ax = a; } }
                    else if (ph.d[a] < 0) { double tt = (g->bmin[a] + idx[a] * cf->spacing[a] - ph.p[a]) / ph.d[a]; if (tt < tn) { tn = tt; ax = a; } }
                }
                if (tn < t) tn = t;
                double seg = tn - t;
                if (mu * seg > tau) {
                    t += tau / mu;
                    for (int a = 0; a < 3; ++a) ph.p[a] += t * ph.d[a];
                    photon_interact(c, &ph, m, &alive);
                    interacted = 1;
                    break;
                }
                tau -= mu * seg;
                t = tn;
                idx[ax] += ph.d[ax] > 0 ? 1 : -1;
                if (idx[ax] < 0 || idx[ax] >= n[ax]) break;
            }
            if (!interacted) {
                for (int a = 0; a < 3; ++a) ph.p[a] += t * ph.d[a];
                int nr = vacuum_move(g, ph.p, ph.d, R_PHANTOM);
                if (nr == R_ESCAPED) { escape(c, ph.E); return; }
                ph.region = nr;
                if (nr == R_EPID) {
                    c->cnt->photon_epid_entries++;
                    if (ph.unscat) c->cnt->unscattered_at_epid++;
                }
            }
        } else {
            /* EPID: exact slab tracking, optical depth carried across layer planes */
            int layer = epid_layer_of(g, ph.p);
            if (layer < 0) layer = 0;
            double tau = -log(orng_u(&c->rng));
            for (;;) {
                int m = cf->layer_mat[layer];
                double mu = cf->layer_rho[layer] * mu_at(g, ph.E)[4 * m];
                double tz = INFINITY; int dz = 0;
                if (ph.d[2] > 0) { tz = (g->zl[layer + 1] - ph.p[2]) / ph.d[2]; dz = 1; }
                else if (ph.d[2] < 0) { tz = (g->zl[layer] - ph.p[2]) / ph.d[2]; dz = -1; }
                double tl = INFINITY;
                if (ph.d[0] > 0) tl = fmin(tl, (g->hx - ph.p[0]) / ph.d[0]);
                else if (ph.d[0] < 0) tl = fmin(tl, (-g->hx - ph.p[0]) / ph.d[0]);
                if (ph.d[1] > 0) tl = fmin(tl, (g->hy - ph.p[1]) / ph.d[1]);
                else if (ph.d[1] < 0) tl = fmin(tl, (-g->hy - ph.p[1]) / ph.d[1]);
                if (tz < 0) tz = 0;
                if (tl < 0) tl = 0;
                double tb = fmin(tz, tl);
                if (mu * tb > tau) {
                    double t = tau / mu;
                    for (int a = 0; a < 3; ++a) ph.p[a] += t * ph.d[a];
                    photon_interact(c, &ph, m, &alive);
                    break;
                }
                tau -= mu * tb;
                for (int a = 0; a < 3; ++a) ph.p[a] += tb * ph.d[a];
                if (tl <= tz) { escape(c, ph.E); return; }
                ph.p[2] = dz > 0 ? g->zl[layer + 1] : g->zl[layer];
                layer += dz;
                if (layer < 0 || layer >= cf->n_layers) { escape(c, ph.E); return; }
            }
        }
    }
}

/* distance from p along d to the boundary of the current cell (voxel, or layer slab within
 * the EPID lateral extent) */
static double cell_distance(const geo_t *g, int region, const double p[3], const double d[3], int *layer_out,
                            int *m_out, double *rho_out, double *smin)
{
    const orc_config *cf = g->c;
    double lo[3], hi[3];
    if (region == R_PHANTOM) {
        int idx[3]; voxel_of(g, p, idx);
        long v = ((long)idx[2] * cf->ny + idx[1]) * cf->nx + idx[0];
        *m_out = cf->vox_mat[v]; *rho_out = cf->vox_rho[v]; *layer_out = -1;
        *smin = cf->step_floor * fmin(cf->spacing[0], fmin(cf->spacing[1], cf->spacing[2]));
        for (int a = 0; a < 3; ++a) { lo[a] = g->bmin[a] + idx[a] * cf->spacing[a]; hi[a] = lo[a] + cf->spacing[a]; }
    } else {
        int l = epid_layer_of(g, p);
        if (l < 0) l = (p[2] < g->zl[0]) ? 0 : cf->n_layers - 1;   /* on the entry plane */
        *layer_out = l; *m_out = cf->layer_mat[l]; *rho_out = cf->layer_rho[l];
        *smin = cf->step_floor * cf->layer_t[l];
        lo[0] = -g->hx; hi[0] = g->hx; lo[1] = -g->hy; hi[1] = g->hy; lo[2] = g->zl[l]; hi[2] = g->zl[l + 1];
    }
    double t = INFINITY;
    for (int a = 0; a < 3; ++a) {
        if (d[a] > 0) t = fmin(t, (hi[a] - p[a]) / d[a]);
        else if (d[a] < 0) t = fmin(t, (lo[a] - p[a]) / d[a]);
    }
    return t < 0 ? 0 : t;
}

static void transport_electron(ctx_t *c, part_t e)
{
    geo_t *g = c->g;
    const orc_config *cf = g->c;
    double T = e.E;
    for (long step = 0;; ++step) {
        if (step > MAX_E_STEPS) { c->err = ORC_E_LOOP; return; }
        int layer, m; double rho, smin;
        const double dist = cell_distance(g, e.region, e.p, e.d, &layer, &m, &rho, &smin);
        double sg = fmax(dist + NUDGE, smin);
        const orc_material *mat = &cf->mat[m];
        c->cnt->e_steps++;
        if (rho <= 0) {
            c->cnt->e_track += sg;
            for (int a = 0; a < 3; ++a) e.p[a] += sg * e.d[a];
        } else {
            /* the distance to a hard event is drawn against the largest hard cross section
             * the step can meet (its energy falls by at most 10%); at the end of such a step
             * the event is real with probability Sigma_hard(T1) / that maximum */
            double smax = (cf->proc_mask & 8) ? 0.0 : orc_sigma_hard_max(mat, T, WCUT, KCUT);
            double xi1 = orng_u(&c->rng), xi2 = orng_u(&c->rng), xi3 = orng_u(&c->rng), xi4 = orng_u(&c->rng);
            double s_hard = smax > 0 ? -log(xi1) / (rho * smax) : INFINITY;
            double s_de = orc_range_diff(mat, DE_FRAC * T, T, WCUT, KCUT) / rho;
            double s_pix = (e.region == R_EPID && layer == cf->scoring_layer) ? 0.5 * fmin(cf->pitch_u, cf->pitch_v) : INFINITY;
            double s = fmin(fmin(s_hard, s_de), fmin(sg, s_pix));
            int hard = s_hard <= fmin(s_de, fmin(sg, s_pix));
            double T1 = (s == s_de) ? DE_FRAC * T : orc_range_inverse(mat, T, rho * s, WCUT, KCUT);
            double h[3], p0[3], d0[3];
            vcopy(p0, e.p); vcopy(d0, e.d);
            c->cnt->e_track += s;
            for (int a = 0; a < 3; ++a) h[a] = e.p[a] + xi2 * s * e.d[a];
            /* the continuous loss is left at the hinge point, in the cell that holds it */
            deposit_at(c, e.region, h, T - T1);
            double th = (cf->proc_mask & 16) ? 0.0 : orc_highland(T, rho * s, g->x0[m]) * sqrt(-2.0 * log(xi3));
            rotate(e.d, cos(th), sin(th), 2.0 * PI * xi4);
            for (int a = 0; a < 3; ++a) e.p[a] = h[a] + (1.0 - xi2) * s * e.d[a];
            orc_event *ev = ev_new(c, ORC_EV_ESTEP, p0);
            if (ev) {
                ev->region = e.region; ev->layer = layer; ev->E0 = T; ev->E1 = T1;
                vcopy(ev->d0, d0); vcopy(ev->d1, e.d); vcopy(ev->dc[0], h);
                ev->aux[0] = s; ev->aux[1] = rho * s; ev->Ec[0] = g->x0[m];
            }
            T = T1;
            if (hard) {
                double sm = orc_sigma_moller(mat, T, WCUT), sb = orc_sigma_brems(mat, T, KCUT);
                double u = orng_u(&c->rng) * smax;
                double dd0[3];
                vcopy(dd0, e.d);
                if (u < sm) {
                    c->cnt->n_moller++;
                    double W = orc_moller_sample(T, WCUT, orng_u(&c->rng));
                    double Tp = T - W;
                    double cd = sqrt(W * (T + 2.0 * MEC2) / (T * (W + 2.0 * MEC2)));
                    double cp = sqrt(Tp * (T + 2.0 * MEC2) / (T * (Tp + 2.0 * MEC2)));
                    double phi = 2.0 * PI * orng_u(&c->rng);
                    double dd[3] = { e.d[0], e.d[1], e.d[2] };
                    rotate(dd, fmin(cd, 1.0), sqrt(fmax(0.0, 1.0 - cd * cd)), phi);
                    rotate(e.d, fmin(cp, 1.0), sqrt(fmax(0.0, 1.0 - cp * cp)), phi + PI);
                    orc_event *em = ev_new(c, ORC_EV_MOLLER, e.p);
                    if (em) { em->E0 = T; em->E1 = Tp; vcopy(em->d0, dd0); vcopy(em->d1, e.d); em->Ec[0] = W; vcopy(em->dc[0], dd); }
                    T = Tp;
                    spawn(c, e.p, dd, W, P_ELECTRON, e.region);
                } else if (u < sm + sb) {
                    c->cnt->n_brems++;
                    double k = orc_brems_sample(T, KCUT, orng_u(&c->rng));
                    orc_event *eb = ev_new(c, ORC_EV_BREMS, e.p);
                    if (eb) { eb->E0 = T; eb->E1 = T - k; vcopy(eb->d0, dd0); vcopy(eb->d1, e.d); eb->Ec[0] = k; vcopy(eb->dc[0], e.d); }
                    T -= k;
                    spawn(c, e.p, e.d, k, P_PHOTON, e.region);
                } else {
                    orc_event *en = ev_new(c, ORC_EV_NULL, e.p);
                    if (en) { en->E0 = T; vcopy(en->d0, e.d); }
                }
            }
        }
        if (T < cf->ecut) {
            /* below the cut-off: deposit at the end point and, for a positron, annihilate there */
            deposit_at(c, e.region, e.p, T);
            if (e.type == P_POSITRON) annihilate(c, e.p, e.region);
            return;
        }
        int nr = classify(g, e.p, e.d, e.region);
        if (nr == R_ESCAPED) { escape(c, T); return; }
        e.region = nr;
    }
}

static void sample_source(ctx_t *c, uint64_t h, part_t *out)
{
    const orc_config *cf = c->g->c;
    orng *r = &c->rng;
    memset(out, 0, sizeof *out);
    out->unscat = 1;
    if (cf->n_phsp > 0) {
        const double *q = cf->phsp + 8 * (h % cf->n_phsp);
        for (int a = 0; a < 3; ++a) { out->p[a] = q[a]; out->d[a] = q[3 + a]; }
        out->E = q[6]; out->type = (int)q[7];
        return;
    }
    /* energy: inverse CDF over bin weights (linear search of the cumulative sum), then uniform in the bin */
    double tot = 0; for (int i = 0; i < cf->nbins; ++i) tot += cf->weights[i];
    double x = orng_u(r) * tot, acc = 0; int bin = cf->nbins - 1;
    for (int i = 0; i < cf->nbins; ++i) { acc += cf->weights[i]; if (x < acc && cf->weights[i] > 0) { bin = i; break; } }
    out->E = cf->edges[bin] + orng_u(r) * (cf->edges[bin + 1] - cf->edges[bin]);
    /* segment of this history */
    int s = 0;
    if (cf->n_seg > 1) { uint64_t cum = 0; for (s = 0; s < cf->n_seg - 1; ++s) { cum += cf->seg_hist[s]; if (h < cum) break; } }
    const double *a = cf->a + (size_t)s * cf->n_pairs, *b = cf->b + (size_t)s * cf->n_pairs;
    /* leaf pair with probability proportional to its open width, then uniform inside it */
    double wt = 0; for (int k = 0; k < cf->n_pairs; ++k) wt += b[k] - a[k];
    x = orng_u(r) * wt; acc = 0; int kp = cf->n_pairs - 1;
    for (int k = 0; k < cf->n_pairs; ++k) { acc += b[k] - a[k]; if (x < acc && b[k] > a[k]) { kp = k; break; } }
    double px = a[kp] + orng_u(r) * (b[kp] - a[kp]);
    double py = cf->y0 + (kp + orng_u(r)) * cf->leaf_w;
    out->type = P_PHOTON;
    if (cf->beam_kind == 0) {
        out->p[0] = px; out->p[1] = py; out->p[2] = cf->src[2];
        out->d[0] = 0; out->d[1] = 0; out->d[2] = 1;
    } else {
        double v[3] = { px - cf->src[0], py - cf->src[1], cf->iso_z - cf->src[2] };
        double n = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        for (int k = 0; k < 3; ++k) { out->p[k] = cf->src[k]; out->d[k] = v[k] / n; }
    }
}

int orc_source(const orc_config *cf, uint64_t h, double out[8])
{
    geo_t g;
    memset(&g, 0, sizeof g);
    g.c = cf;
    ctx_t *c = (ctx_t *)calloc(1, sizeof(ctx_t));
    c->g = &g;
    orng_init(&c->rng, cf->seed, h);
    part_t p;
    sample_source(c, h, &p);
    for (int a = 0; a < 3; ++a) { out[a] = p.p[a]; out[3 + a] = p.d[a]; }
    out[6] = p.E; out[7] = p.type;
    free(c);
    return ORC_OK;
}

int orc_map_hu(const int16_t *hu, uint64_t n, int n_pts, const double *ch, const double *cr,
               int n_ranges, const double *hu_upper, const int *mat_of, uint8_t *om, double *orho)
{
    if (n_pts < 1 || n_ranges < 1) return ORC_E_ARG;
    for (uint64_t i = 0; i < n; ++i) {
        double x = hu[i], rho;
        if (x <= ch[0]) rho = cr[0];
        else if (x >= ch[n_pts - 1]) rho = cr[n_pts - 1];
        else {
            int k = 0; while (!(x >= ch[k] && x < ch[k + 1])) ++k;
            rho = cr[k] + (cr[k + 1] - cr[k]) * (x - ch[k]) / (ch[k + 1] - ch[k]);
        }
        int r = n_ranges - 1;
        for (int k = 0; k < n_ranges - 1; ++k) if (x < hu_upper[k]) { r = k; break; }
        om[i] = (uint8_t)mat_of[r];
        orho[i] = rho;
    }
    return ORC_OK;
}

int orc_run(const orc_config *cf, uint64_t first, uint64_t count, double *sum, double *sum2, orc_counters *cnt)
{
    return orc_run_traced(cf, first, count, sum, sum2, cnt, NULL, 0, NULL);
}

int orc_run_traced(const orc_config *cf, uint64_t first, uint64_t count, double *sum, double *sum2, orc_counters *cnt,
                   orc_event *ev, uint64_t cap, uint64_t *n_ev)
{
    if (!cf || !sum || !sum2 || !cnt || cf->n_layers < 1 || cf->n_layers > ORC_MAX_LAYERS || cf->n_mat < 1) return ORC_E_ARG;
    pthread_once(&gl_once, gl_init);
    geo_t g;
    memset(&g, 0, sizeof g);
    g.c = cf;
    const int n[3] = { cf->nx, cf->ny, cf->nz };
    for (int a = 0; a < 3; ++a) { g.bmin[a] = cf->origin[a]; g.bmax[a] = cf->origin[a] + n[a] * cf->spacing[a]; }
    g.zl[0] = cf->front_z;
    for (int l = 0; l < cf->n_layers; ++l) g.zl[l + 1] = g.zl[l] + cf->layer_t[l];
    g.hx = 0.5 * cf->npx_u * cf->pitch_u;
    g.hy = 0.5 * cf->npx_v * cf->pitch_v;
    g.mu_cache = (double *)calloc(4 * cf->n_mat, sizeof(double));
    g.mu_E = -1;
    for (int m = 0; m < cf->n_mat; ++m) g.x0[m] = orc_x0(&cf->mat[m]);
    int npix = cf->npx_u * cf->npx_v;
    ctx_t *c = (ctx_t *)calloc(1, sizeof(ctx_t));
    c->g = &g;
    c->hacc = (double *)calloc(npix, sizeof(double));
    c->touched = (int *)malloc(sizeof(int) * (size_t)npix);
    c->cnt = cnt;
    c->ev = ev;
    c->ev_cap = ev ? cap : 0;
    c->ev_n = 0;
    for (uint64_t h = first; h < first + count && !c->err; ++h) {
        c->hist = h;
        orng_init(&c->rng, cf->seed, h);
        c->n = 0; c->ntouched = 0; c->dep = 0; c->esc = 0; c->rest = 0;
        part_t src;
        sample_source(c, h, &src);
        double ein = src.E;
        cnt->e_in += ein;
        cnt->n_hist++;
        int r = classify(&g, src.p, src.d, -1);
        if (r == R_ESCAPED) escape(c, src.E);
        else {
            src.region = r;
            if (r == R_EPID && src.type == P_PHOTON) { cnt->photon_epid_entries++; cnt->unscattered_at_epid++; }
            push(c, src.p, src.d, src.E, src.type, r, src.unscat);
        }
        while (c->n > 0 && !c->err) {
            part_t q = c->st[--c->n];
            if (q.type == P_PHOTON) transport_photon(c, q); else transport_electron(c, q);
        }
        /* per-history ledger: incident = deposited + escaped + rest energy created by pairs
         * and not returned by annihilation */
        double resid = fabs(ein - (c->dep + c->esc + c->rest)) / ein;
        if (resid > cnt->max_ledger_resid) cnt->max_ledger_resid = resid;
        cnt->e_rest_balance += c->rest;
        for (int i = 0; i < c->ntouched; ++i) {
            int p = c->touched[i];
            double e = c->hacc[p];
            sum[p] += e; sum2[p] += e * e;
            c->hacc[p] = 0.0;
        }
    }
    int err = c->err;
    if (n_ev) *n_ev = c->ev_n;
    free(c->hacc); free(c->touched); free(c); free(g.mu_cache);
    return err;
}

/* ------------------------------------------------------------------------------------ */
/* dose-response correction inputs (Sec. 2.2, Sec. 3.1)                                 */
/* ------------------------------------------------------------------------------------ */
static int cmp_double(const void *x, const void *y)
{
    const double a = *(const double *)x, b = *(const double *)y;
    return (a > b) - (a < b);
}

/* line integral of the density along the segment S -> T (g/cm^2) */
static double ray_density_integral(const orc_config *cf, const double S[3], const double T[3], double *buf)
{
    const int n[3] = { cf->nx, cf->ny, cf->nz };
    double d[3], lo[3], hi[3];
    double amin = 0.0, amax = 1.0;
    for (int a = 0; a < 3; ++a) {
        d[a] = T[a] - S[a];
        lo[a] = cf->origin[a];
        hi[a] = cf->origin[a] + n[a] * cf->spacing[a];
        if (d[a] == 0.0) {
            if (S[a] < lo[a] || S[a] >= hi[a]) return 0.0;   /* parallel to the slab and outside it */
        } else {
            double a1 = (lo[a] - S[a]) / d[a], a2 = (hi[a] - S[a]) / d[a];
            if (a1 > a2) { double t = a1; a1 = a2; a2 = t; }
            if (a1 > amin) amin = a1;
            if (a2 < amax) amax = a2;
        }
    }
    if (!(amax > amin)) return 0.0;
    /* the crossings: the entry and exit parameters and every voxel plane strictly between */
    int m = 0;
    buf[m++] = amin;
    buf[m++] = amax;
    for (int a = 0; a < 3; ++a) {
        if (d[a] == 0.0) continue;
        for (int i = 0; i <= n[a]; ++i) {
            const double al = (lo[a] + i * cf->spacing[a] - S[a]) / d[a];
            if (al > amin && al < amax) buf[m++] = al;
        }
    }
    qsort(buf, (size_t)m, sizeof(double), cmp_double);
    const double len = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    double sum = 0.0;
    for (int k = 0; k + 1 < m; ++k) {
        const double a0 = buf[k], a1 = buf[k + 1];
        if (!(a1 > a0)) continue;
        const double mid = 0.5 * (a0 + a1);
        int idx[3];
        for (int a = 0; a < 3; ++a) {
            int i = (int)floor((S[a] + mid * d[a] - lo[a]) / cf->spacing[a]);
            idx[a] = i < 0 ? 0 : (i >= n[a] ? n[a] - 1 : i);
        }
        sum += cf->vox_rho[((size_t)idx[2] * cf->ny + idx[1]) * cf->nx + idx[0]] * (a1 - a0) * len;
    }
    return sum;
}

int orc_radiological_thickness(const orc_config *cf, double *out)
{
    if (!cf || !out || cf->scoring_layer < 0 || cf->scoring_layer >= cf->n_layers) return ORC_E_ARG;
    double zmid = cf->front_z;
    for (int l = 0; l < cf->scoring_layer; ++l) zmid += cf->layer_t[l];
    zmid += 0.5 * cf->layer_t[cf->scoring_layer];
    const double hx = 0.5 * cf->npx_u * cf->pitch_u, hy = 0.5 * cf->npx_v * cf->pitch_v;
    const double zlo = cf->origin[2], zhi = cf->origin[2] + cf->nz * cf->spacing[2];
    double *buf = (double *)malloc(sizeof(double) * (size_t)(cf->nx + cf->ny + cf->nz + 8));
    if (!buf) return ORC_E_ARG;
    for (int v = 0; v < cf->npx_v; ++v)
        for (int u = 0; u < cf->npx_u; ++u) {
            const double x = -hx + (u + 0.5) * cf->pitch_u, y = -hy + (v + 0.5) * cf->pitch_v;
            double S[3], T[3];
            if (cf->beam_kind == 1) {
                S[0] = cf->src[0]; S[1] = cf->src[1]; S[2] = cf->src[2];
                T[0] = x; T[1] = y; T[2] = zmid;
            } else {   /* parallel beam: a line along +z through the pixel centre, past the box */
                S[0] = x; S[1] = y; S[2] = zlo - 1.0;
                T[0] = x; T[1] = y; T[2] = zhi + 1.0;
            }
            out[(size_t)v * cf->npx_u + u] = ray_density_integral(cf, S, T, buf);   /* g/cm^2 over 1 g/cm^3 */
        }
    free(buf);
    return ORC_OK;
}

double orc_equivalent_square(const orc_config *cf)
{
    double xmin = INFINITY, xmax = -INFINITY;
    int kmin = -1, kmax = -1;
    for (int s = 0; s < cf->n_seg; ++s)
        for (int k = 0; k < cf->n_pairs; ++k) {
            const double a = cf->a[(size_t)s * cf->n_pairs + k], b = cf->b[(size_t)s * cf->n_pairs + k];
            if (!(b > a)) continue;   /* closed pair */
            if (a < xmin) xmin = a;
            if (b > xmax) xmax = b;
            if (kmin < 0 || k < kmin) kmin = k;
            if (k > kmax) kmax = k;
        }
    if (kmin < 0) return 0.0;
    const double A = xmax - xmin, B = (kmax + 1 - kmin) * cf->leaf_w;
    return 2.0 * A * B / (A + B);
}

/* the interval [x_i, x_{i+1}] of an ascending node list holding x (clamped), and the weight of x_{i+1} */
static void bracket(const double *x, int n, double v, int *i_out, double *f_out)
{
    if (n == 1 || v <= x[0]) { *i_out = 0; *f_out = 0.0; return; }
    if (v >= x[n - 1]) { *i_out = n - 2; *f_out = 1.0; return; }
    int i = 0;
    while (i + 1 < n - 1 && v >= x[i + 1]) ++i;
    *i_out = i;
    *f_out = (v - x[i]) / (x[i + 1] - x[i]);
}

double orc_response_factor(const double *tn, int nt, const double *sn, int ns, const double *k, double t, double s)
{
    int i, j;
    double ft, fs;
    bracket(tn, nt, t, &i, &ft);
    bracket(sn, ns, s, &j, &fs);
    const int i1 = nt > 1 ? i + 1 : i, j1 = ns > 1 ? j + 1 : j;
    const double k00 = k[j * nt + i], k01 = k[j * nt + i1], k10 = k[j1 * nt + i], k11 = k[j1 * nt + i1];
    return (1.0 - fs) * ((1.0 - ft) * k00 + ft * k01) + fs * ((1.0 - ft) * k10 + ft * k11);
}

