/*
 * peo.c -- plain FP64 CPU oracle (TEST INFRASTRUCTURE ONLY; see peo.h).
 *
 * Nitz, "Robust, Rapid, and Simple Gravitational-wave Parameter Estimation",
 * arXiv:2410.05190. Each function names the passage of the paper it follows,
 * or the published source of the model piece the paper leaves open.
 * Built with gcc -O2 (no fast-math); OpenMP only splits independent draws.
 */
#include "peo.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

static const double PI = 3.14159265358979323846;
static const double EULER_GAMMA = 0.5772156649015329;

/* Physical constants (the paper fixes none): IAU nominal GM_sun, exact c,
 * the IAU parsec, and a spherical Earth of the mean radius. */
static const double GM_SUN = 1.32712440018e20; /* m^3 s^-2 */
static const double C_SI = 299792458.0;         /* m/s */
static const double MPC_M = 3.0856775814913673e22;
static const double R_EARTH = 6.371e6;

double peo_t_sun(void) { return GM_SUN / (C_SI * C_SI * C_SI); }
double peo_mpc_m(void) { return MPC_M; }
double peo_c_si(void) { return C_SI; }
double peo_r_earth(void) { return R_EARTH; }

int peo_dim(int params) { return params == PEO_PARAMS_4D ? 4 : 11; }

/* Neumaier compensated summation. */
typedef struct {
    double s, c;
} nsum;
static void nadd(nsum *a, double x)
{
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x))
        a->c += (a->s - t) + x;
    else
        a->c += (x - t) + a->s;
    a->s = t;
}
static double nval(const nsum *a) { return a->s + a->c; }

/*
 * TaylorF2 phase coefficients (stationary-phase approximation of the
 * inspiral). Non-spinning terms to 3.5PN: Buonanno, Iyer, Ochsner, Pan,
 * Sathyaprakash, PRD 80, 084043 (2009), TaylorF2 phase. Aligned-spin terms:
 * spin-orbit at 1.5, 2.5, 3 and 3.5PN and spin-spin at 2PN (black-hole
 * quadrupole), as compiled by Mishra, Kela, Arun, Faye, PRD 93, 084054 (2016);
 * here written per body, with S = x1^2 chi1 + x2^2 chi2 and
 * Sig = x2 chi2 - x1 chi1 (x_i = m_i / M).
 * The 5th-order term carries (1 + 3 ln v) with the reference velocity 1: the
 * constant belongs to the coalescence phase.
 */
void peo_pn_coeffs(double eta, double delta, double chi1, double chi2, double phi[8], double phil[8])
{
    const double x1 = 0.5 * (1.0 + delta), x2 = 0.5 * (1.0 - delta);
    const double S = x1 * x1 * chi1 + x2 * x2 * chi2;
    const double Sig = x2 * chi2 - x1 * chi1;
    const double eta2 = eta * eta, eta3 = eta2 * eta;
    const double pi2 = PI * PI;
    int j;
    for (j = 0; j < 8; j++) {
        phi[j] = 0.0;
        phil[j] = 0.0;
    }
    phi[0] = 1.0;
    phi[1] = 0.0;
    phi[2] = 3715.0 / 756.0 + 55.0 / 9.0 * eta;
    /* 1.5PN: tail + spin-orbit */
    phi[3] = -16.0 * PI + 188.0 / 3.0 * S + 25.0 * delta * Sig;
    /* 2PN: point mass + spin-spin sigma */
    {
        double sigma = 79.0 / 8.0 * eta * chi1 * chi2 + 81.0 / 16.0 * (x1 * x1 * chi1 * chi1 + x2 * x2 * chi2 * chi2);
        phi[4] = 15293365.0 / 508032.0 + 27145.0 / 504.0 * eta + 3085.0 / 72.0 * eta2 - 10.0 * sigma;
    }
    /* 2.5PN: point mass + spin-orbit gamma; log term 3x */
    {
        double gam = (554345.0 / 1134.0 + 110.0 / 9.0 * eta) * S + (13915.0 / 84.0 - 10.0 / 3.0 * eta) * delta * Sig;
        phi[5] = PI * (38645.0 / 756.0 - 65.0 / 9.0 * eta) - gam;
        phil[5] = 3.0 * phi[5];
    }
    /* 3PN: point mass (with ln(4v) split into ln 4 + ln v) + spin-orbit tail */
    phi[6] = 11583231236531.0 / 4694215680.0 - 640.0 / 3.0 * pi2 - 6848.0 / 21.0 * EULER_GAMMA -
             6848.0 / 21.0 * log(4.0) + (-15737765635.0 / 3048192.0 + 2255.0 / 12.0 * pi2) * eta +
             76055.0 / 1728.0 * eta2 - 127825.0 / 1296.0 * eta3 + PI * (3760.0 * S + 1490.0 * delta * Sig) / 3.0;
    phil[6] = -6848.0 / 21.0;
    /* 3.5PN: point mass + spin-orbit */
    phi[7] = PI * (77096675.0 / 254016.0 + 378515.0 / 1512.0 * eta - 74045.0 / 756.0 * eta2) +
             (-8980424995.0 / 762048.0 + 6586595.0 / 756.0 * eta - 305.0 / 36.0 * eta2) * S -
             (170978035.0 / 48384.0 - 2876425.0 / 672.0 * eta - 4735.0 / 144.0 * eta2) * delta * Sig;
}

/* Psi(f) = 2 pi f tc - phic - pi/4 + 3/(128 eta v^5) sum_j (phi_j + phil_j ln v) v^j,
 * v = (pi M f)^(1/3), M in seconds. */
double peo_psi(const peo_source *s, double f)
{
    const double v = cbrt(PI * s->M * peo_t_sun() * f);
    const double lnv = log(v);
    double sum = 0.0, vk = 1.0;
    int j;
    for (j = 0; j < 8; j++) {
        sum += (s->phi[j] + s->phil[j] * lnv) * vk;
        vk *= v;
    }
    return 2.0 * PI * f * s->tc - s->phic - PI / 4.0 + 3.0 / (128.0 * s->eta * pow(v, 5.0)) * sum;
}

/* Test-mass ISCO of the total mass: f = 1/(6^(3/2) pi M). */
double peo_f_isco(double M) { return 1.0 / (pow(6.0, 1.5) * PI * M * peo_t_sun()); }

/* Number of bins with f_k < f_isco (brute force). */
long peo_kcut(const peo_event *ev, double fisco)
{
    long k = 0;
    while (k < ev->n_bins && ev->f_lo + (double)k * ev->df < fisco)
        k++;
    return k;
}

/* Long-wavelength response of an L-shaped detector on a spherical Earth.
 * Detector tensor D = (x x^T - y y^T)/2 with the y arm 90 degrees east of x;
 * polarisation tensors from the sky basis rotated by psi. */
void peo_antenna(const double geom[3], double ra, double dec, double psi, double gmst, double *fplus,
                 double *fcross, double *dt)
{
    const double lat = geom[0], lon = geom[1], az = geom[2];
    double up[3], east[3], north[3], xa[3], ya[3], Dt[3][3];
    double n[3], u[3], w[3], X[3], Y[3];
    double lam = ra - gmst;
    double fp = 0.0, fc = 0.0, rn = 0.0;
    int i, j;
    up[0] = cos(lat) * cos(lon);
    up[1] = cos(lat) * sin(lon);
    up[2] = sin(lat);
    east[0] = -sin(lon);
    east[1] = cos(lon);
    east[2] = 0.0;
    north[0] = -sin(lat) * cos(lon);
    north[1] = -sin(lat) * sin(lon);
    north[2] = cos(lat);
    for (i = 0; i < 3; i++) {
        xa[i] = cos(az) * north[i] + sin(az) * east[i];
        ya[i] = -sin(az) * north[i] + cos(az) * east[i];
    }
    for (i = 0; i < 3; i++)
        for (j = 0; j < 3; j++)
            Dt[i][j] = 0.5 * (xa[i] * xa[j] - ya[i] * ya[j]);
    n[0] = cos(dec) * cos(lam);
    n[1] = cos(dec) * sin(lam);
    n[2] = sin(dec);
    u[0] = -sin(lam);
    u[1] = cos(lam);
    u[2] = 0.0;
    w[0] = -sin(dec) * cos(lam);
    w[1] = -sin(dec) * sin(lam);
    w[2] = cos(dec);
    for (i = 0; i < 3; i++) {
        X[i] = cos(psi) * u[i] + sin(psi) * w[i];
        Y[i] = -sin(psi) * u[i] + cos(psi) * w[i];
    }
    for (i = 0; i < 3; i++)
        for (j = 0; j < 3; j++) {
            fp += Dt[i][j] * (X[i] * X[j] - Y[i] * Y[j]);
            fc += Dt[i][j] * (X[i] * Y[j] + Y[i] * X[j]);
        }
    for (i = 0; i < 3; i++)
        rn += up[i] * n[i];
    *fplus = fp;
    *fcross = fc;
    *dt = -R_EARTH * rn / C_SI;
}

int peo_source_from_theta(const peo_event *ev, const double *th, peo_source *s)
{
    int d, ok;
    memset(s, 0, sizeof(*s));
    if (ev->params == PEO_PARAMS_4D) {
        double mc = th[0], eta = th[1], chi = th[2];
        s->mc = mc;
        s->eta = eta;
        s->M = mc * pow(eta, -0.6);
        s->delta = sqrt(fmax(0.0, 1.0 - 4.0 * eta));
        s->chi1 = chi;
        s->chi2 = chi;
        s->tc = th[3];
        s->phic = 0.0;
        for (d = 0; d < ev->n_det; d++) {
            s->rre[d] = ev->amp0 * ev->strain_scale;
            s->rim[d] = 0.0;
            s->dt[d] = 0.0;
        }
        ok = (mc > 0.0) && (eta > 0.0) && (eta <= 0.25) && (fabs(chi) <= ev->chi_max);
    } else {
        double mc = th[0], q = th[1], ra = th[4], dec = th[5], iota = th[6], psi = th[7], dl = th[8];
        double amp, ci = cos(iota);
        s->mc = mc;
        s->eta = q / ((1.0 + q) * (1.0 + q));
        s->M = mc * pow(1.0 + q, 1.2) * pow(q, -0.6);
        s->delta = (1.0 - q) / (1.0 + q);
        s->chi1 = th[2];
        s->chi2 = th[3];
        s->tc = th[9];
        s->phic = (ev->phase == PEO_PHASE_EXPLICIT) ? th[10] : 0.0;
        /* Newtonian SPA amplitude: sqrt(5/24) pi^(-2/3) Mc^(5/6) / dL (G = c = 1) */
        amp = sqrt(5.0 / 24.0) * pow(PI, -2.0 / 3.0) * pow(mc * peo_t_sun(), 5.0 / 6.0) / (dl * MPC_M / C_SI);
        amp *= ev->strain_scale;
        for (d = 0; d < ev->n_det; d++) {
            double fp, fc, dt;
            peo_antenna(ev->det_geom[d], ra, dec, psi, ev->gmst, &fp, &fc, &dt);
            /* h_d = F+ h+ + Fx hx, h+ = A (1+cos^2 i)/2 e^{-i Phi}, hx = -i A cos i e^{-i Phi} */
            s->rre[d] = amp * fp * 0.5 * (1.0 + ci * ci);
            s->rim[d] = -amp * fc * ci;
            s->dt[d] = dt;
        }
        ok = (mc > 0.0) && (q > 0.0) && (q <= 1.0) && (fabs(th[2]) <= ev->chi_max) &&
             (fabs(th[3]) <= ev->chi_max) && (fabs(dec) <= 0.5 * PI) && (iota >= 0.0) && (iota <= PI) &&
             (ev->distance == PEO_DIST_MARG || ((dl > 0.0) && (dl <= ev->dl_max)));
    }
    peo_pn_coeffs(s->eta, s->delta, s->chi1, s->chi2, s->phi, s->phil);
    s->fisco = peo_f_isco(s->M);
    s->kcut = -1; /* filled by the callers that need the cut */
    s->in_support = ok;
    return ok;
}

/* Model waveform of detector d at bin k: R_d f^-7/6 exp(-i [Psi(f) + 2 pi f dt_d]). */
static void wf_bin(const peo_event *ev, const peo_source *s, int d, long k, double *hr, double *hi)
{
    const double f = ev->f_lo + (double)k * ev->df;
    const double ph = peo_psi(s, f) + 2.0 * PI * f * s->dt[d];
    const double a = pow(f, -7.0 / 6.0);
    const double c = cos(ph), sn = sin(ph);
    /* (rre + i rim)(c - i sn) */
    *hr = a * (s->rre[d] * c + s->rim[d] * sn);
    *hi = a * (s->rim[d] * c - s->rre[d] * sn);
}

void peo_waveform(const peo_event *ev, const double *theta, long kcut_override, double *h)
{
    peo_source s;
    long k, kc;
    int d;
    peo_source_from_theta(ev, theta, &s);
    kc = kcut_override >= 0 ? kcut_override : peo_kcut(ev, s.fisco);
    if (kc > ev->n_bins)
        kc = ev->n_bins;
    for (d = 0; d < ev->n_det; d++)
        for (k = 0; k < ev->n_bins; k++) {
            double *o = h + 2 * ((long)d * ev->n_bins + k);
            if (k < kc)
                wf_bin(ev, &s, d, k, &o[0], &o[1]);
            else
                o[0] = o[1] = 0.0;
        }
}

/* Eq. 1 discretised: (a|b) = 4 df Re sum_k conj(a_k) b_k / S_k. */
double peo_inner(const peo_event *ev, int d, const double *a, const double *b)
{
    nsum acc = {0.0, 0.0};
    long k;
    const double *S = ev->psd + (long)d * ev->n_bins;
    const double *ad = a + 2 * (long)d * ev->n_bins, *bd = b + 2 * (long)d * ev->n_bins;
    for (k = 0; k < ev->n_bins; k++)
        nadd(&acc, 4.0 * ev->df * (ad[2 * k] * bd[2 * k] + ad[2 * k + 1] * bd[2 * k + 1]) / S[k]);
    return nval(&acc);
}

/* ln I0(x) from the integral representation I0(x) = (1/pi) int_0^pi exp(x cos t) dt
 * (DLMF 10.32.1), trapezoid rule: exponentially convergent for this periodic
 * analytic integrand. exp(x (cos t - 1)) is written as exp(-2 x sin^2(t/2)); the
 * range is cut where that factor falls below e^-750 (it is even about t = 0, so the
 * truncated rule keeps its exponential convergence). */
double peo_log_i0(double x)
{
    const long m = 4096;
    long i;
    double tmax = PI, s;
    nsum acc = {0.0, 0.0};
    x = fabs(x);
    if (x == 0.0)
        return 0.0;
    s = sqrt(375.0 / x);
    if (s < 1.0)
        tmax = 2.0 * asin(s);
    for (i = 0; i <= m; i++) {
        double t = tmax * (double)i / (double)m;
        double sh = sin(0.5 * t);
        double wgt = (i == 0 || i == m) ? 0.5 : 1.0;
        nadd(&acc, wgt * exp(-2.0 * x * sh * sh));
    }
    return x + log(nval(&acc) * tmax / (PI * (double)m));
}

/* ln I0(x) by the same integral representation as peo_log_i0 with 128 nodes:
 * the trapezoid rule on the periodic integrand converges geometrically, and 128
 * nodes over the truncated range keep its error below 1e-30 for every x (the
 * distance integral evaluates it many times per draw). */
static double log_i0_quick(double x)
{
    const long m = 128;
    long i;
    double tmax = PI, s, acc = 0.0;
    x = fabs(x);
    if (x == 0.0)
        return 0.0;
    s = sqrt(375.0 / x);
    if (s < 1.0)
        tmax = 2.0 * asin(s);
    for (i = 0; i <= m; i++) {
        double t = tmax * (double)i / (double)m;
        double sh = sin(0.5 * t);
        acc += ((i == 0 || i == m) ? 0.5 : 1.0) * exp(-2.0 * x * sh * sh);
    }
    return x + log(acc * tmax / (PI * (double)m));
}

/* Log of the distance integrand in u = ln(dl_max / dL) = ln x, u >= 0:
 * 3 x^-4 exp(phi(x) - b x^2) dx = 3 exp(-3u + phi(e^u) - b e^{2u}) du. */
static double dm_logf(double u, double a, double b, int ex)
{
    const double x = exp(u);
    return log(3.0) - 3.0 * u + (ex ? a * x : log_i0_quick(a * x)) - b * x * x;
}

typedef struct {
    double a, b, G;
    int ex;
} dm_arg;

static double dm_f(const dm_arg *q, double u) { return exp(dm_logf(u, q->a, q->b, q->ex) - q->G); }

/* Adaptive Simpson on [lo, hi] (Richardson-corrected once converged); the
 * tolerance halves with each split, down to the rounding level of the integrand. */
static double dm_simpson(const dm_arg *q, double lo, double hi, double flo, double fm, double fhi, double whole,
                         double tol, int depth)
{
    const double m = 0.5 * (lo + hi), lm = 0.5 * (lo + m), rm = 0.5 * (m + hi);
    const double flm = dm_f(q, lm), frm = dm_f(q, rm);
    const double left = (m - lo) / 6.0 * (flo + 4.0 * flm + fm), right = (hi - m) / 6.0 * (fm + 4.0 * frm + fhi);
    const double d = left + right - whole;
    /* converged, or at the level of the integrand's own rounding: its logarithm
     * is a difference of terms up to ~1e4, so its values carry ~1e-13 relative error */
    if (depth >= 24 || fabs(d) <= 15.0 * fmax(tol, 1e-13 * fabs(left + right)))
        return left + right + d / 15.0;
    return dm_simpson(q, lo, m, flo, flm, fm, left, 0.5 * tol, depth + 1) +
           dm_simpson(q, m, hi, fm, frm, fhi, right, 0.5 * tol, depth + 1);
}

/* The integral over u in [0, 40] (x up to e^40; beyond, the integrand is below
 * e^-120 of its prior weight alone) on 16384 panels, each refined adaptively to
 * 1e-16 of the coarse total, in units of exp(G), G the largest coarse sample.
 * The integrand's peak has width ~1/rho in u, rho the matched-filter SNR at the
 * best distance; the coarse samples (every 1.2e-3) resolve it for rho up to ~800. */
double peo_log_dist_marg(double a, double b, int explicit_phase)
{
    const int N = 16384;
    const double U = 40.0, h = U / N;
    double *f = (double *)malloc(sizeof(double) * (2 * N + 1));
    dm_arg q;
    double coarse = 0.0, tot = 0.0, G = -INFINITY;
    int j;
    q.a = a;
    q.b = b;
    q.ex = explicit_phase;
    for (j = 0; j <= 2 * N; j++) {
        f[j] = dm_logf(0.5 * h * j, a, b, explicit_phase);
        if (f[j] > G)
            G = f[j];
    }
    q.G = G;
    for (j = 0; j <= 2 * N; j++)
        f[j] = exp(f[j] - G);
    for (j = 0; j < N; j++)
        coarse += h / 6.0 * (f[2 * j] + 4.0 * f[2 * j + 1] + f[2 * j + 2]);
    for (j = 0; j < N; j++) {
        const double whole = h / 6.0 * (f[2 * j] + 4.0 * f[2 * j + 1] + f[2 * j + 2]);
        tot += dm_simpson(&q, j * h, (j + 1) * h, f[2 * j], f[2 * j + 1], f[2 * j + 2], whole, 1e-16 * coarse, 0);
    }
    free(f);
    return G + log(tot);
}

/* ln L from Z and H (Eq. 3): explicit phase Re Z - H/2; marginalised over a
 * uniform coalescence phase ln I0(|Z|) - H/2; distance-marginalised events take
 * Z and H at the reference distance dl_max and integrate over dL. */
static double loglike_from_zh(const peo_event *ev, double Zr, double Zi, double H)
{
    const int ex = (ev->phase == PEO_PHASE_EXPLICIT);
    if (ev->distance == PEO_DIST_MARG)
        return peo_log_dist_marg(ex ? Zr : hypot(Zr, Zi), 0.5 * H, ex);
    return ex ? Zr - 0.5 * H : peo_log_i0(hypot(Zr, Zi)) - 0.5 * H;
}

/* The parameters the likelihood's waveform is evaluated at: theta itself, or
 * theta with dL at the reference distance dl_max for distance-marginalised events. */
static void likelihood_theta(const peo_event *ev, const double *th, double *out)
{
    memcpy(out, th, sizeof(double) * peo_dim(ev->params));
    if (ev->params == PEO_PARAMS_11D && ev->distance == PEO_DIST_MARG)
        out[8] = ev->dl_max;
}

static double loglike_time_marg(const peo_event *ev, const peo_source *s, const double *X, double H);
static double fmax_d(double a, double b) { return a > b ? a : b; }

/* Eq. 3 with Eq. 1: Z = sum_d (d_d|h_d) as a complex overlap, H = sum_d (h_d|h_d).
 * Explicit phase: ln L = Re Z - H/2. Marginalised over a uniform coalescence
 * phase: ln L = ln I0(|Z|) - H/2. Time-marginalised events integrate the
 * likelihood over tc (see loglike_time_marg). */
static double loglike_one(const peo_event *ev, const double *th_in, double *zh)
{
    peo_source s;
    nsum zr = {0, 0}, zi = {0, 0}, hh = {0, 0};
    int d;
    long k;
    double Zr, Zi, H, th[PEO_MAX_DIM];
    likelihood_theta(ev, th_in, th);
    if (!peo_source_from_theta(ev, th, &s)) {
        if (zh)
            zh[0] = zh[1] = zh[2] = 0.0;
        return -INFINITY;
    }
    s.kcut = peo_kcut(ev, s.fisco);
    double *X = NULL; /* time-marginalised events: the detector-summed integrand per bin */
    if (ev->time_marg && s.kcut > 0)
        X = (double *)calloc(2 * (size_t)s.kcut, sizeof(double));
    for (d = 0; d < ev->n_det; d++) {
        const double *S = ev->psd + (long)d * ev->n_bins;
        const double *dd = ev->data + 2 * (long)d * ev->n_bins;
        for (k = 0; k < s.kcut; k++) {
            double hr, hi, w;
            wf_bin(ev, &s, d, k, &hr, &hi);
            w = 4.0 * ev->df / S[k];
            /* conj(d) h */
            nadd(&zr, w * (dd[2 * k] * hr + dd[2 * k + 1] * hi));
            nadd(&zi, w * (dd[2 * k] * hi - dd[2 * k + 1] * hr));
            nadd(&hh, w * (hr * hr + hi * hi));
            if (X) {
                X[2 * k] += w * (dd[2 * k] * hr + dd[2 * k + 1] * hi);
                X[2 * k + 1] += w * (dd[2 * k] * hi - dd[2 * k + 1] * hr);
            }
        }
    }
    if (ev->time_marg) {
        const double lt = loglike_time_marg(ev, &s, X, nval(&hh));
        free(X);
        if (zh) {
            zh[0] = nval(&zr);
            zh[1] = nval(&zi);
            zh[2] = nval(&hh);
        }
        return lt;
    }
    Zr = nval(&zr);
    Zi = nval(&zi);
    H = nval(&hh);
    if (zh) {
        zh[0] = Zr;
        zh[1] = Zi;
        zh[2] = H;
    }
    return loglike_from_zh(ev, Zr, Zi, H);
}

/* Time-marginalised likelihood (the paper marginalises extrinsic parameters,
 * Sec. III): with a flat prior on tc over [tc_lo, tc_hi] of width T,
 *   L_t = (1/T) int_{tc_lo}^{tc_hi} L(theta with tc = t) dt.
 * Shifting tc by u multiplies the model at f_k by exp(-2 pi i f_k u), so with
 * X_k the detector-summed conj(d) h / S integrand at the draw's own tc (s->tc),
 * Z(t) = sum_k X_k exp(-2 pi i f_k (t - s->tc)) and H does not change; each
 * node's ln L follows from Z(t), H as in loglike_from_zh. The integral is
 * Simpson's rule over the whole window: a scan at spacing 1/(8 f_max) finds
 * the largest |Z(t)|; the likelihood's peak in t is no narrower than
 * 1/(2 pi f_max sqrt(|Z|max)) (the curvature of Re Z(t) is at most
 * (2 pi f_max)^2 |Z|), and the nodes are spaced at a quarter of that and at
 * most T/4000, so that both the peak and a window edge that cuts it are
 * resolved. */
static void z_at(const peo_event *ev, const peo_source *s, const double *X, double t, double *zr, double *zi)
{
    nsum a = {0, 0}, b = {0, 0};
    long k;
    const double u = t - s->tc;
    for (k = 0; k < s->kcut; k++) {
        const double f = ev->f_lo + (double)k * ev->df;
        const double ph = -2.0 * PI * f * u, c = cos(ph), sn = sin(ph);
        nadd(&a, X[2 * k] * c - X[2 * k + 1] * sn);
        nadd(&b, X[2 * k] * sn + X[2 * k + 1] * c);
    }
    *zr = nval(&a);
    *zi = nval(&b);
}

static double loglike_time_marg(const peo_event *ev, const peo_source *s, const double *X, double H)
{
    const double T = ev->tc_hi - ev->tc_lo;
    double zmax = 0.0, zr, zi, h, lmax = -INFINITY, acc = 0.0;
    long j, nc, nf;
    double *lv;
    if (s->kcut <= 0)
        return loglike_from_zh(ev, 0.0, 0.0, H);
    {
        const double fmax = ev->f_lo + (double)s->kcut * ev->df;
        nc = (long)ceil(T * 8.0 * fmax) + 1;
        for (j = 0; j < nc; j++) {
            z_at(ev, s, X, ev->tc_lo + T * (double)j / (double)(nc - 1), &zr, &zi);
            if (hypot(zr, zi) > zmax)
                zmax = hypot(zr, zi);
        }
        h = 0.25 / (2.0 * PI * fmax * sqrt(fmax_d(zmax, 1.0)));
    }
    nf = (long)ceil(T / h);
    if (nf < 4000)
        nf = 4000;
    nf += (nf & 1) + 1; /* an even number of intervals */
    lv = (double *)malloc(sizeof(double) * (size_t)nf);
    for (j = 0; j < nf; j++) {
        z_at(ev, s, X, ev->tc_lo + T * (double)j / (double)(nf - 1), &zr, &zi);
        lv[j] = loglike_from_zh(ev, zr, zi, H);
        if (lv[j] > lmax)
            lmax = lv[j];
    }
    if (lmax == -INFINITY) {
        free(lv);
        return -INFINITY;
    }
    for (j = 0; j < nf; j++)
        acc += ((j == 0 || j == nf - 1) ? 1.0 : (j & 1) ? 4.0 : 2.0) * exp(lv[j] - lmax);
    free(lv);
    /* (1/T) * (T/(nf-1))/3 * sum */
    return lmax + log(acc / 3.0) - log((double)(nf - 1));
}

#ifdef _OPENMP
#include <omp.h>
#endif

void peo_loglike(const peo_event *ev, const double *theta, long n, double *loglike, double *zh, int n_threads)
{
    const int D = peo_dim(ev->params);
    long i;
#ifdef _OPENMP
    if (n_threads > 0)
        omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (i = 0; i < n; i++) {
        double th[PEO_MAX_DIM];
        int j;
        for (j = 0; j < D; j++)
            th[j] = theta[(long)j * n + i];
        loglike[i] = loglike_one(ev, th, zh ? zh + 3 * i : NULL);
    }
    (void)n_threads;
}

/* Finite-difference steps (a reading of the method; the paper fixes none):
 * each step moves the waveform phase by about 1e-3 rad at the band edge that
 * is most sensitive to it, from the Newtonian phase Phi_N(f) = 3/128 (pi Mc f)^(-5/3);
 * amplitude-only angles use 1e-4 rad and the distance 1e-4 dL. */
void peo_default_steps(const peo_event *ev, const double *th, double *st)
{
    peo_source s;
    double fhi = ev->f_lo + (double)ev->n_bins * ev->df;
    double ftop, phin, mc = th[0];
    peo_source_from_theta(ev, th, &s);
    ftop = s.fisco < fhi ? s.fisco : fhi;
    phin = 3.0 / 128.0 * pow(PI * mc * peo_t_sun() * ev->f_lo, -5.0 / 3.0);
    if (ev->params == PEO_PARAMS_4D) {
        st[0] = 1e-3 * mc / (5.0 / 3.0 * phin);
        st[1] = 1e-3 / phin;
        st[2] = 1e-3 / phin;
        st[3] = 1e-3 / (2.0 * PI * ftop);
    } else {
        double sky = 1e-3 / (2.0 * PI * ftop * R_EARTH / C_SI);
        st[0] = 1e-3 * mc / (5.0 / 3.0 * phin);
        st[1] = 1e-3 / phin;
        st[2] = 1e-3 / phin;
        st[3] = 1e-3 / phin;
        st[4] = sky;
        st[5] = sky;
        st[6] = 1e-4;
        st[7] = 1e-4;
        st[8] = 1e-4 * th[8];
        st[9] = 1e-3 / (2.0 * PI * ftop);
        st[10] = 0.0; /* coalescence phase: analytic column */
    }
}

/* Prior regularisation 12/range^2 (the precision of a uniform distribution
 * over the prior range) for bounded and periodic coordinates. */
static void prior_reg(const peo_event *ev, double *reg)
{
    if (ev->params == PEO_PARAMS_4D) {
        reg[0] = 0.0;
        reg[1] = 12.0 / (0.25 * 0.25);
        reg[2] = 12.0 / (4.0 * ev->chi_max * ev->chi_max);
        reg[3] = 0.0;
    } else {
        reg[0] = 0.0;
        reg[1] = 12.0;
        reg[2] = reg[3] = 12.0 / (4.0 * ev->chi_max * ev->chi_max);
        reg[4] = 12.0 / (4.0 * PI * PI);
        reg[5] = 12.0 / (PI * PI);
        reg[6] = 12.0 / (PI * PI);
        reg[7] = 12.0 / (PI * PI);
        reg[8] = 12.0 / (ev->dl_max * ev->dl_max);
        reg[9] = 0.0;
        reg[10] = 12.0 / (4.0 * PI * PI);
    }
}

/*
 * Fisher metric of the network waveform, g_ij = sum_d (d_i h_d | d_j h_d)
 * (the metric induced by the inner product, Sec. II.A), with the cut frozen at
 * theta0, central differences for every sampled coordinate except the
 * coalescence phase, whose derivative is exactly i h. For the marginalised
 * likelihood the phase direction is projected out (Schur complement).
 */
int peo_metric_fd(const peo_event *ev, const double *th0, const double *steps, int flags, double *g)
{
    const int D = peo_dim(ev->params);
    const int is4 = (ev->params == PEO_PARAMS_4D);
    const int Dp = is4 ? D + 1 : D;  /* with the phase column */
    const int iphi = is4 ? D : 10;   /* index of the phase coordinate */
    peo_source s0, sp[PEO_MAX_DIM], sm[PEO_MAX_DIM];
    double den[PEO_MAX_DIM];
    int fd[PEO_MAX_DIM + 1];
    nsum G[PEO_MAX_DIM + 1][PEO_MAX_DIM + 1];
    double Gd[PEO_MAX_DIM + 1][PEO_MAX_DIM + 1];
    double reg[PEO_MAX_DIM];
    int a, b, d;
    long k;
    peo_source_from_theta(ev, th0, &s0);
    /* frozen cut */
    s0.kcut = peo_kcut(ev, s0.fisco);
    memset(G, 0, sizeof(G));
    for (a = 0; a < Dp; a++)
        fd[a] = (a != iphi);
    for (a = 0; a < D; a++) {
        double tp[PEO_MAX_DIM], tm[PEO_MAX_DIM];
        if (!fd[a])
            continue;
        memcpy(tp, th0, sizeof(double) * D);
        memcpy(tm, th0, sizeof(double) * D);
        tp[a] = th0[a] + steps[a];
        tm[a] = th0[a] - steps[a];
        den[a] = (tp[a] - th0[a]) + (th0[a] - tm[a]);
        peo_source_from_theta(ev, tp, &sp[a]);
        peo_source_from_theta(ev, tm, &sm[a]);
    }
    for (d = 0; d < ev->n_det; d++) {
        const double *S = ev->psd + (long)d * ev->n_bins;
        for (k = 0; k < s0.kcut; k++) {
            double dr[PEO_MAX_DIM + 1], di[PEO_MAX_DIM + 1];
            double w = 4.0 * ev->df / S[k];
            for (a = 0; a < Dp; a++) {
                if (fd[a]) {
                    double pr, pi_, mr, mi;
                    wf_bin(ev, &sp[a], d, k, &pr, &pi_);
                    wf_bin(ev, &sm[a], d, k, &mr, &mi);
                    dr[a] = (pr - mr) / den[a];
                    di[a] = (pi_ - mi) / den[a];
                } else {
                    double hr, hi;
                    wf_bin(ev, &s0, d, k, &hr, &hi);
                    /* d h / d phic = i h */
                    dr[a] = -hi;
                    di[a] = hr;
                }
            }
            for (a = 0; a < Dp; a++)
                for (b = a; b < Dp; b++)
                    nadd(&G[a][b], w * (dr[a] * dr[b] + di[a] * di[b]));
        }
    }
    for (a = 0; a < Dp; a++)
        for (b = a; b < Dp; b++)
            Gd[a][b] = Gd[b][a] = nval(&G[a][b]);

    if (flags & 2) {
        for (a = 0; a < Dp; a++)
            for (b = 0; b < Dp; b++)
                g[a * Dp + b] = Gd[a][b];
        return 0;
    }
    /* project out the phase for the marginalised likelihood */
    if (ev->phase == PEO_PHASE_MARG) {
        double gpp = Gd[iphi][iphi];
        double P[PEO_MAX_DIM + 1][PEO_MAX_DIM + 1];
        for (a = 0; a < Dp; a++)
            for (b = 0; b < Dp; b++)
                P[a][b] = (a == iphi || b == iphi) ? 0.0 : Gd[a][b] - Gd[a][iphi] * Gd[iphi][b] / gpp;
        memcpy(Gd, P, sizeof(P));
    }
    /* distance-marginalised likelihood: project out dL the same way */
    if (!is4 && ev->distance == PEO_DIST_MARG) {
        const int il = 8;
        double gll = Gd[il][il];
        double P[PEO_MAX_DIM + 1][PEO_MAX_DIM + 1];
        for (a = 0; a < Dp; a++)
            for (b = 0; b < Dp; b++)
                P[a][b] = (a == il || b == il) ? 0.0 : Gd[a][b] - Gd[a][il] * Gd[il][b] / gll;
        memcpy(Gd, P, sizeof(P));
    }
    for (a = 0; a < D; a++)
        for (b = 0; b < D; b++)
            g[a * D + b] = Gd[a][b];
    if (!(flags & 1)) {
        prior_reg(ev, reg);
        for (a = 0; a < D; a++)
            g[a * D + a] += reg[a];
    }
    return 0;
}

/* ---------------- draws (proposal N(theta0, g^-1)) ---------------- */

static uint32_t mulhilo32(uint32_t a, uint32_t b, uint32_t *hi)
{
    uint64_t p = (uint64_t)a * (uint64_t)b;
    *hi = (uint32_t)(p >> 32);
    return (uint32_t)p;
}

/* Philox4x32 with 10 rounds, as defined by Salmon et al. (SC'11): two 32x32->64
 * multiplies per round, Weyl-sequence key schedule. */
void peo_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    int r;
    for (r = 0; r < 10; r++) {
        uint32_t hi0, hi1;
        uint32_t lo0 = mulhilo32(0xD2511F53u, x0, &hi0);
        uint32_t lo1 = mulhilo32(0xCD9E8D57u, x2, &hi1);
        uint32_t y0 = hi1 ^ x1 ^ k0, y2 = hi0 ^ x3 ^ k1;
        x0 = y0;
        x1 = lo1;
        x2 = y2;
        x3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = x0;
    out[1] = x1;
    out[2] = x2;
    out[3] = x3;
}

/* 53-bit uniform on (0, 1] from two words: 27 high bits of a, 26 of b. */
static double u53(uint32_t a, uint32_t b)
{
    return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6) + 1.0) * (1.0 / 9007199254740992.0);
}

/* Block (i, j): counter (i lo, i hi, j, stream), key (seed lo, seed hi). */
static void block_uniforms(uint64_t seed, uint32_t stream, uint64_t i, uint32_t j, double *ua, double *ub)
{
    uint32_t ctr[4], key[2], o[4];
    ctr[0] = (uint32_t)i;
    ctr[1] = (uint32_t)(i >> 32);
    ctr[2] = j;
    ctr[3] = stream;
    key[0] = (uint32_t)seed;
    key[1] = (uint32_t)(seed >> 32);
    peo_philox4x32_10(ctr, key, o);
    *ua = u53(o[0], o[1]);
    *ub = u53(o[2], o[3]);
}

void peo_uniforms(uint64_t seed, uint32_t stream, long n, int npairs, double *u)
{
    long i;
    int j;
    for (i = 0; i < n; i++)
        for (j = 0; j < npairs; j++)
            block_uniforms(seed, stream, (uint64_t)i, (uint32_t)j, &u[i * 2 * npairs + 2 * j],
                           &u[i * 2 * npairs + 2 * j + 1]);
}

/* Cholesky g = L L^T (row-major lower L). Returns 0, or 3 if not positive definite. */
static int cholesky(const double *g, int D, double *L)
{
    int i, j, k;
    memset(L, 0, sizeof(double) * D * D);
    for (i = 0; i < D; i++)
        for (j = 0; j <= i; j++) {
            double s = g[i * D + j];
            for (k = 0; k < j; k++)
                s -= L[i * D + k] * L[j * D + k];
            if (i == j) {
                if (!(s > 0.0))
                    return 3;
                L[i * D + i] = sqrt(s);
            } else
                L[i * D + j] = s / L[j * D + j];
        }
    return 0;
}

static int periodic_dims(const peo_event *ev, int *idx, double *per)
{
    if (ev->params == PEO_PARAMS_4D)
        return 0;
    idx[0] = 4;
    per[0] = 2.0 * PI; /* ra */
    idx[1] = 7;
    per[1] = PI; /* psi */
    idx[2] = 10;
    per[2] = 2.0 * PI; /* phic */
    return 3;
}

/* Prior (App. A.3 weights need log pi; the paper's priors are "natural"):
 * flat in Mc, eta or q, spins, tc, ra, psi, phic; cos(dec); sin(iota); dL^2.
 * Normalisations are dropped. */
double peo_logprior(const peo_event *ev, const double *th)
{
    peo_source s;
    if (!peo_source_from_theta(ev, th, &s))
        return -INFINITY;
    if (ev->params == PEO_PARAMS_4D)
        return 0.0;
    if (ev->distance == PEO_DIST_MARG) /* the dL prior is inside the marginalised likelihood */
        return log(cos(th[5])) + log(sin(th[6]));
    return log(cos(th[5])) + log(sin(th[6])) + 2.0 * log(th[8]);
}

/* Density of the wrapped Gaussian at theta: log sum over images k in {-2,...,2}^p of
 * N(theta + k P; theta0, g^-1), with the quadratic form evaluated as |L^T x|^2.
 * theta and theta0 both lie in [0, P) on the periodic coordinates, so every
 * omitted image is at least 2P from theta0: its term is below e^-24 of the
 * largest while the proposal's width stays within P / sqrt(12) (the prior
 * precision 12/P^2 of the metric bounds it there). */
static double logq_one(int D, const double *L, const double *th0, const double *th, int np, const int *pidx,
                       const double *per)
{
    int nimg = 1, m, a, r, c;
    double lq[125], mx = -INFINITY, acc = 0.0, logdet = 0.0;
    for (a = 0; a < np; a++)
        nimg *= 5;
    for (m = 0; m < nimg; m++) {
        double x[PEO_MAX_DIM], q = 0.0;
        int code = m;
        for (a = 0; a < D; a++)
            x[a] = th[a] - th0[a];
        for (a = 0; a < np; a++) {
            int kk = code % 5 - 2;
            code /= 5;
            x[pidx[a]] += kk * per[a];
        }
        for (r = 0; r < D; r++) {
            double y = 0.0;
            for (c = r; c < D; c++)
                y += L[c * D + r] * x[c];
            q += y * y;
        }
        lq[m] = -0.5 * q;
        if (lq[m] > mx)
            mx = lq[m];
    }
    for (m = 0; m < nimg; m++)
        acc += exp(lq[m] - mx);
    for (r = 0; r < D; r++)
        logdet += log(L[r * D + r]);
    return mx + log(acc) + logdet - 0.5 * D * log(2.0 * PI);
}

/* Inverse of a symmetric positive-definite matrix: L L^T X = I solved column by
 * column. Returns 0, or 3 if the matrix is not positive definite. */
static int spd_inverse(const double *g, int D, double *inv)
{
    double L[PEO_MAX_DIM * PEO_MAX_DIM], y[PEO_MAX_DIM];
    int i, j, k, rc = cholesky(g, D, L);
    if (rc)
        return rc;
    for (j = 0; j < D; j++) {
        for (i = 0; i < D; i++) { /* L y = e_j */
            double t = (i == j) ? 1.0 : 0.0;
            for (k = 0; k < i; k++)
                t -= L[i * D + k] * y[k];
            y[i] = t / L[i * D + i];
        }
        for (i = D - 1; i >= 0; i--) { /* L^T x = y */
            double t = y[i];
            for (k = i + 1; k < D; k++)
                t -= L[k * D + i] * inv[k * D + j];
            inv[i * D + j] = t / L[i * D + i];
        }
    }
    return 0;
}

/* Marginalised coordinates: dL (index 8) of distance-marginalised events and
 * phic (index 10) of 11-D phase-marginalised events are never used by the
 * likelihood, so the proposal density the weights need is that of the other
 * coordinates. dec_g: g with each marginalised row and column decoupled by the
 * Schur complement (its diagonal entry kept), the metric the draws are taken
 * with. Lm: Cholesky factor of the marginal precision of the Dm kept
 * coordinates, the inverse of the sub-block of the covariance g^-1; keep: their
 * indices; pidx_m: the periodic ones among them (np_m of them). */
typedef struct {
    double dec_g[PEO_MAX_DIM * PEO_MAX_DIM];
    double Lm[PEO_MAX_DIM * PEO_MAX_DIM];
    int keep[PEO_MAX_DIM];
    int Dm, np_m;
    int pidx_m[3];
    double per_m[3];
} marg_prop;

static int marg_dims(const peo_event *ev, int *marg)
{
    int n = 0;
    if (ev->params != PEO_PARAMS_11D)
        return 0;
    if (ev->distance == PEO_DIST_MARG)
        marg[n++] = 8;
    if (ev->time_marg)
        marg[n++] = 9;
    if (ev->phase == PEO_PHASE_MARG)
        marg[n++] = 10;
    return n;
}

static int marg_proposal(const double *g, int D, int nm, const int *marg, int np, const int *pidx,
                         const double *per, marg_prop *mp)
{
    double C[PEO_MAX_DIM * PEO_MAX_DIM], Cm[PEO_MAX_DIM * PEO_MAX_DIM], gm[PEO_MAX_DIM * PEO_MAX_DIM];
    double t[PEO_MAX_DIM * PEO_MAX_DIM];
    int a, b, i, rc, is_m[PEO_MAX_DIM] = {0};
    memcpy(mp->dec_g, g, sizeof(double) * D * D);
    for (i = 0; i < nm; i++) {
        const int il = marg[i];
        is_m[il] = 1;
        memcpy(t, mp->dec_g, sizeof(double) * D * D);
        for (a = 0; a < D; a++)
            for (b = 0; b < D; b++)
                mp->dec_g[a * D + b] = (a == il || b == il) ? ((a == b) ? t[il * D + il] : 0.0)
                                                             : t[a * D + b] - t[a * D + il] * t[il * D + b] / t[il * D + il];
    }
    rc = spd_inverse(g, D, C);
    if (rc)
        return rc;
    mp->Dm = 0;
    for (a = 0; a < D; a++)
        if (!is_m[a])
            mp->keep[mp->Dm++] = a;
    for (a = 0; a < mp->Dm; a++)
        for (b = 0; b < mp->Dm; b++)
            Cm[a * mp->Dm + b] = C[mp->keep[a] * D + mp->keep[b]];
    rc = spd_inverse(Cm, mp->Dm, gm);
    if (rc)
        return rc;
    rc = cholesky(gm, mp->Dm, mp->Lm);
    if (rc)
        return rc;
    mp->np_m = 0;
    for (i = 0; i < np; i++)
        for (a = 0; a < mp->Dm; a++)
            if (mp->keep[a] == pidx[i]) {
                mp->pidx_m[mp->np_m] = a;
                mp->per_m[mp->np_m++] = per[i];
            }
    return 0;
}

static double logq_marg(const marg_prop *mp, const double *th0, const double *th)
{
    double t0[PEO_MAX_DIM], t[PEO_MAX_DIM];
    int a;
    for (a = 0; a < mp->Dm; a++) {
        t0[a] = th0[mp->keep[a]];
        t[a] = th[mp->keep[a]];
    }
    return logq_one(mp->Dm, mp->Lm, t0, t, mp->np_m, mp->pidx_m, mp->per_m);
}

/* theta0 with its periodic coordinates wrapped into [0, P) (the centre of the
 * images of log q; the draws themselves do not depend on it). */
static void wrap_centre(const peo_event *ev, const double *th0, double *out)
{
    int pidx[3], np, a, D = peo_dim(ev->params);
    double per[3];
    np = periodic_dims(ev, pidx, per);
    for (a = 0; a < D; a++)
        out[a] = th0[a];
    for (a = 0; a < np; a++)
        out[pidx[a]] = th0[pidx[a]] - per[a] * floor(th0[pidx[a]] / per[a]);
}

int peo_draw(const peo_event *ev, const double *th0, const double *g, uint64_t seed, uint32_t stream, long n,
             double *theta, double *logq, double *logprior)
{
    const int D = peo_dim(ev->params);
    double L[PEO_MAX_DIM * PEO_MAX_DIM], c0[PEO_MAX_DIM];
    marg_prop mp;
    int pidx[3], marg[3], np, nm, rc;
    double per[3];
    long i;
    np = periodic_dims(ev, pidx, per);
    nm = marg_dims(ev, marg);
    wrap_centre(ev, th0, c0);
    rc = nm ? marg_proposal(g, D, nm, marg, np, pidx, per, &mp) : 0;
    if (!rc)
        rc = cholesky(nm ? mp.dec_g : g, D, L);
    if (rc) {
        for (i = 0; i < n; i++) {
            int a;
            for (a = 0; a < D; a++)
                theta[(long)a * n + i] = th0[a];
            logq[i] = 0.0;
            logprior[i] = -INFINITY;
        }
        return rc;
    }
    for (i = 0; i < n; i++) {
        double z[PEO_MAX_DIM + 1], y[PEO_MAX_DIM], th[PEO_MAX_DIM];
        int j, r, c, a;
        for (j = 0; 2 * j < D; j++) {
            double ua, ub, rad;
            block_uniforms(seed, stream, (uint64_t)i, (uint32_t)j, &ua, &ub);
            /* Box-Muller */
            rad = sqrt(-2.0 * log(ua));
            z[2 * j] = rad * cos(2.0 * PI * ub);
            z[2 * j + 1] = rad * sin(2.0 * PI * ub);
        }
        /* theta = theta0 + L^-T z: back substitution with L^T */
        for (r = D - 1; r >= 0; r--) {
            double s = z[r];
            for (c = r + 1; c < D; c++)
                s -= L[c * D + r] * y[c];
            y[r] = s / L[r * D + r];
        }
        for (a = 0; a < D; a++)
            th[a] = th0[a] + y[a];
        for (a = 0; a < np; a++) {
            double P = per[a], v = th[pidx[a]];
            th[pidx[a]] = v - P * floor(v / P);
        }
        if (D == 11 && ev->time_marg) {
            /* tc: its mean under the proposal given the other coordinates (the
               centre the likelihood's integral over tc is taken about), from
               their offsets to the centre, periodic ones to the nearest image */
            double m = c0[9], dlt[PEO_MAX_DIM];
            for (a = 0; a < D; a++)
                dlt[a] = th[a] - c0[a];
            for (a = 0; a < np; a++) {
                const double P = per[a];
                dlt[pidx[a]] -= P * floor(dlt[pidx[a]] / P + 0.5);
            }
            for (a = 0; a < D; a++)
                if (a != 9)
                    m -= g[9 * D + a] / g[9 * D + 9] * dlt[a];
            th[9] = m;
        }
        for (a = 0; a < D; a++)
            theta[(long)a * n + i] = th[a];
        logq[i] = nm ? logq_marg(&mp, c0, th) : logq_one(D, L, c0, th, np, pidx, per);
        logprior[i] = peo_logprior(ev, th);
    }
    return 0;
}

/* Extrinsic coordinates of tile draws: the coordinates outside sub_mask drawn
 * from the proposal's marginal over them (declaration in peo.h). */
/* The conditional form: the kept coordinates E (outside sub_mask and the
 * marginalised ones M) given the tiled ones I, from N(theta0, g^-1) with M
 * integrated out. Over A = I + E the covariance is the block C_AA of C = g^-1;
 * E given I has mean theta0_E + C_EI C_II^-1 (theta_I - theta0_I) and covariance
 * S = C_EE - C_EI C_II^-1 C_IE. Draws: y_E = Lp^-T z_E with Lp the Cholesky
 * factor of S^-1 over E in index order and z the normals of peo_draw at the
 * coordinates of E. */
static int tile_extrinsic_cond(const peo_event *ev, const double *th0, const double *g, const int *is_m,
                               unsigned sub_mask, uint64_t seed, uint32_t stream, long n, double *theta, double *logq,
                               double *logprior)
{
    const int D = peo_dim(ev->params);
    double C[PEO_MAX_DIM * PEO_MAX_DIM], CII[PEO_MAX_DIM * PEO_MAX_DIM] = {0}, CIIi[PEO_MAX_DIM * PEO_MAX_DIM];
    double B[PEO_MAX_DIM * PEO_MAX_DIM], S[PEO_MAX_DIM * PEO_MAX_DIM], P[PEO_MAX_DIM * PEO_MAX_DIM];
    double Lp[PEO_MAX_DIM * PEO_MAX_DIM], c0[PEO_MAX_DIM], per[3], per_e[3];
    int I[PEO_MAX_DIM], E[PEO_MAX_DIM], pidx[3], pidx_e[3], nI = 0, nE = 0, np, np_e = 0, a, b, k, rc;
    long i;
    np = periodic_dims(ev, pidx, per);
    for (a = 0; a < D; a++) {
        if (sub_mask >> a & 1u)
            I[nI++] = a;
        else if (!is_m[a])
            E[nE++] = a;
    }
    rc = spd_inverse(g, D, C);
    if (rc)
        return rc;
    for (a = 0; a < nI; a++)
        for (b = 0; b < nI; b++)
            CII[a * nI + b] = C[I[a] * D + I[b]];
    rc = spd_inverse(CII, nI, CIIi);
    if (rc)
        return rc;
    /* B = C_EI C_II^-1, S = C_EE - B C_IE */
    for (a = 0; a < nE; a++)
        for (b = 0; b < nI; b++) {
            double t = 0.0;
            for (k = 0; k < nI; k++)
                t += C[E[a] * D + I[k]] * CIIi[k * nI + b];
            B[a * nI + b] = t;
        }
    for (a = 0; a < nE; a++)
        for (b = 0; b < nE; b++) {
            double t = C[E[a] * D + E[b]];
            for (k = 0; k < nI; k++)
                t -= B[a * nI + k] * C[I[k] * D + E[b]];
            S[a * nE + b] = t;
        }
    for (a = 0; a < nE; a++)
        for (b = 0; b < a; b++)
            S[a * nE + b] = S[b * nE + a] = 0.5 * (S[a * nE + b] + S[b * nE + a]);
    rc = spd_inverse(S, nE, P);
    if (!rc)
        rc = cholesky(P, nE, Lp);
    if (rc)
        return rc;
    for (k = 0; k < np; k++)
        for (a = 0; a < nE; a++)
            if (E[a] == pidx[k]) {
                pidx_e[np_e] = a;
                per_e[np_e++] = per[k];
            }
    wrap_centre(ev, th0, c0);
    for (i = 0; i < n; i++) {
        double z[PEO_MAX_DIM + 1], y[PEO_MAX_DIM], th[PEO_MAX_DIM], m[PEO_MAX_DIM], tE[PEO_MAX_DIM];
        int j, r, c;
        for (j = 0; 2 * j < D; j++) {
            double ua, ub, rad;
            block_uniforms(seed, stream, (uint64_t)i, (uint32_t)j, &ua, &ub);
            rad = sqrt(-2.0 * log(ua));
            z[2 * j] = rad * cos(2.0 * PI * ub);
            z[2 * j + 1] = rad * sin(2.0 * PI * ub);
        }
        for (a = 0; a < D; a++)
            th[a] = theta[(long)a * n + i];
        /* conditional mean, then y = Lp^-T z_E */
        for (a = 0; a < nE; a++) {
            double t = th0[E[a]];
            for (k = 0; k < nI; k++)
                t += B[a * nI + k] * (th[I[k]] - th0[I[k]]);
            m[a] = t;
        }
        for (r = nE - 1; r >= 0; r--) {
            double s = z[E[r]];
            for (c = r + 1; c < nE; c++)
                s -= Lp[c * nE + r] * y[c];
            y[r] = s / Lp[r * nE + r];
        }
        for (a = 0; a < nE; a++)
            th[E[a]] = m[a] + y[a];
        for (a = 0; a < D; a++)
            if (is_m[a])
                th[a] = th0[a];
        for (a = 0; a < np; a++) {
            double Pp = per[a], v = th[pidx[a]];
            th[pidx[a]] = v - Pp * floor(v / Pp);
        }
        for (a = 0; a < np_e; a++) {
            const double Pp = per_e[a];
            m[pidx_e[a]] -= Pp * floor(m[pidx_e[a]] / Pp);
        }
        if (D == 11 && ev->time_marg) {
            double mt = c0[9], dlt[PEO_MAX_DIM];
            for (a = 0; a < D; a++)
                dlt[a] = th[a] - c0[a];
            for (a = 0; a < np; a++) {
                const double Pp = per[a];
                dlt[pidx[a]] -= Pp * floor(dlt[pidx[a]] / Pp + 0.5);
            }
            for (a = 0; a < D; a++)
                if (a != 9)
                    mt -= g[9 * D + a] / g[9 * D + 9] * dlt[a];
            th[9] = mt;
        }
        for (a = 0; a < D; a++)
            theta[(long)a * n + i] = th[a];
        for (a = 0; a < nE; a++)
            tE[a] = th[E[a]];
        logq[i] += logq_one(nE, Lp, m, tE, np_e, pidx_e, per_e);
        if (logprior[i] != -INFINITY)
            logprior[i] = peo_logprior(ev, th);
    }
    return 0;
}

int peo_tile_extrinsic(const peo_event *ev, const double *th0, const double *g, unsigned sub_mask, int conditional,
                       uint64_t seed, uint32_t stream, long n, double *theta, double *logq, double *logprior)
{
    const int D = peo_dim(ev->params);
    double L[PEO_MAX_DIM * PEO_MAX_DIM], c0[PEO_MAX_DIM], per[3];
    marg_prop mp;
    int pidx[3], mm[3], marg[PEO_MAX_DIM], is_m[PEO_MAX_DIM] = {0}, np, nm = 0, k, a, rc;
    long i;
    np = periodic_dims(ev, pidx, per);
    if (sub_mask == 0 || (sub_mask >> D) != 0)
        return 1;
    for (a = 0; a < np; a++)
        if (sub_mask >> pidx[a] & 1u)
            return 1;
    /* decoupled: the tiled coordinates and the likelihood's marginalised ones */
    k = marg_dims(ev, mm);
    for (a = 0; a < k; a++)
        is_m[mm[a]] = 1;
    for (a = 0; a < D; a++)
        if (sub_mask >> a & 1u)
            is_m[a] = 1;
    if (conditional) {
        int ism[PEO_MAX_DIM] = {0};
        for (a = 0; a < k; a++)
            ism[mm[a]] = 1;
        for (a = 0; a < D; a++)
            if ((sub_mask >> a & 1u) && ism[a])
                return 1;
        return tile_extrinsic_cond(ev, th0, g, ism, sub_mask, seed, stream, n, theta, logq, logprior);
    }
    for (a = 0; a < D; a++)
        if (is_m[a])
            marg[nm++] = a;
    wrap_centre(ev, th0, c0);
    rc = marg_proposal(g, D, nm, marg, np, pidx, per, &mp);
    if (!rc)
        rc = cholesky(mp.dec_g, D, L);
    if (rc)
        return rc;
    for (i = 0; i < n; i++) {
        double z[PEO_MAX_DIM + 1], y[PEO_MAX_DIM], th[PEO_MAX_DIM];
        int j, r, c;
        for (j = 0; 2 * j < D; j++) {
            double ua, ub, rad;
            block_uniforms(seed, stream, (uint64_t)i, (uint32_t)j, &ua, &ub);
            rad = sqrt(-2.0 * log(ua));
            z[2 * j] = rad * cos(2.0 * PI * ub);
            z[2 * j + 1] = rad * sin(2.0 * PI * ub);
        }
        for (r = D - 1; r >= 0; r--) {
            double s = z[r];
            for (c = r + 1; c < D; c++)
                s -= L[c * D + r] * y[c];
            y[r] = s / L[r * D + r];
        }
        for (a = 0; a < D; a++)
            th[a] = (sub_mask >> a & 1u) ? theta[(long)a * n + i] : th0[a] + y[a];
        for (a = 0; a < np; a++) {
            double P = per[a], v = th[pidx[a]];
            th[pidx[a]] = v - P * floor(v / P);
        }
        if (D == 11 && ev->time_marg) {
            /* tc: its mean under the proposal given the other coordinates of the
               composed draw, as peo_draw sets it */
            double m = c0[9], dlt[PEO_MAX_DIM];
            for (a = 0; a < D; a++)
                dlt[a] = th[a] - c0[a];
            for (a = 0; a < np; a++) {
                const double P = per[a];
                dlt[pidx[a]] -= P * floor(dlt[pidx[a]] / P + 0.5);
            }
            for (a = 0; a < D; a++)
                if (a != 9)
                    m -= g[9 * D + a] / g[9 * D + 9] * dlt[a];
            th[9] = m;
        }
        for (a = 0; a < D; a++)
            theta[(long)a * n + i] = th[a];
        logq[i] += logq_marg(&mp, c0, th);
        if (logprior[i] != -INFINITY)
            logprior[i] = peo_logprior(ev, th);
    }
    return 0;
}

int peo_logq_theta(const peo_event *ev, const double *th0, const double *g, const double *theta, long n,
                   double *logq)
{
    const int D = peo_dim(ev->params);
    double L[PEO_MAX_DIM * PEO_MAX_DIM], per[3], c0[PEO_MAX_DIM];
    marg_prop mp;
    int pidx[3], marg[3], np, nm, rc;
    long i;
    np = periodic_dims(ev, pidx, per);
    nm = marg_dims(ev, marg);
    wrap_centre(ev, th0, c0);
    rc = nm ? marg_proposal(g, D, nm, marg, np, pidx, per, &mp) : cholesky(g, D, L);
    if (rc)
        return rc;
    for (i = 0; i < n; i++) {
        double th[PEO_MAX_DIM];
        int a;
        for (a = 0; a < D; a++)
            th[a] = theta[(long)a * n + i];
        logq[i] = nm ? logq_marg(&mp, c0, th) : logq_one(D, L, c0, th, np, pidx, per);
    }
    return 0;
}

/* Log-density of a mixture of the wrapped metric Gaussians of peo_draw (the
 * paper's proposal is itself a mixture of local proposals, weighted by their
 * share of the posterior, Sec. II.A; here the components are Gaussians in the
 * local metric, e.g. the proposals of successive refinement rounds, Sec. III.A):
 *   ln q(theta) = ln sum_m pi_m q_m(theta),  pi_m = weights_m / sum_k weights_k,
 * with q_m the density peo_logq_theta gives for (theta0 + m D, g + m D D).
 * Weights must be finite and >= 0 with a positive sum. Returns 0, -1 for bad
 * weights, or a component's nonzero code (metric not positive definite). */
int peo_mixture_logq(const peo_event *ev, int m, const double *weights, const double *theta0, const double *g,
                     const double *theta, long n, double *logq)
{
    const int D = peo_dim(ev->params);
    double wsum = 0.0;
    double *lqm;
    long i;
    int k, rc = 0;
    if (m < 1)
        return -1;
    for (k = 0; k < m; k++) {
        if (!(weights[k] >= 0.0) || !isfinite(weights[k]))
            return -1;
        wsum += weights[k];
    }
    if (!(wsum > 0.0))
        return -1;
    lqm = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1) * (size_t)m);
    if (!lqm)
        return -1;
    for (k = 0; k < m && !rc; k++)
        rc = peo_logq_theta(ev, theta0 + (long)k * D, g + (long)k * D * D, theta, n, lqm + (long)k * n);
    if (!rc) {
        for (i = 0; i < n; i++) {
            /* log-sum-exp over the components with positive weight */
            double mx = -INFINITY;
            nsum acc = {0, 0};
            for (k = 0; k < m; k++) {
                if (weights[k] > 0.0) {
                    const double t = log(weights[k] / wsum) + lqm[(long)k * n + i];
                    if (t > mx)
                        mx = t;
                }
            }
            if (mx == -INFINITY) {
                logq[i] = -INFINITY;
                continue;
            }
            for (k = 0; k < m; k++)
                if (weights[k] > 0.0)
                    nadd(&acc, exp(log(weights[k] / wsum) + lqm[(long)k * n + i] - mx));
            logq[i] = mx + log(acc.s + acc.c);
        }
    }
    free(lqm);
    return rc;
}

/* Eq. 5: w_i = L_i pi_i / g_i, in logs; Eq. 6: ESS = (sum w)^2 / sum w^2.
 * Weights are normalised; lnZ = ln mean(w). Draws with -inf log weight count in N. */
void peo_weights_ess(const double *ll, const double *lp, const double *lq, long n, double *w, double *stats)
{
    long i, nin = 0;
    double m = -INFINITY;
    nsum s1 = {0, 0}, s2 = {0, 0};
    long bad = 0;
    for (i = 0; i < n; i++) {
        double l = ll[i] + lp[i] - lq[i];
        if (isfinite(l)) {
            nin++;
            if (l > m)
                m = l;
        } else if (!(l == -INFINITY)) {
            bad++; /* NaN or +inf: no weight is defined */
        }
    }
    if (bad > 0) {
        /* an undefined log-weight leaves the normalisation undefined: every
           estimate is NaN (only -inf, a draw outside the support, has weight 0) */
        if (w)
            for (i = 0; i < n; i++)
                w[i] = NAN;
        stats[0] = NAN;
        stats[1] = NAN;
        stats[2] = NAN;
        stats[3] = (double)nin;
        return;
    }
    if (nin == 0) {
        if (w)
            for (i = 0; i < n; i++)
                w[i] = 0.0;
        stats[0] = 0.0;
        stats[1] = -INFINITY;
        stats[2] = -INFINITY;
        stats[3] = 0.0;
        return;
    }
    for (i = 0; i < n; i++) {
        double l = ll[i] + lp[i] - lq[i];
        if (isfinite(l)) {
            double e = exp(l - m);
            nadd(&s1, e);
            nadd(&s2, e * e);
        }
    }
    if (w)
        for (i = 0; i < n; i++) {
            double l = ll[i] + lp[i] - lq[i];
            w[i] = isfinite(l) ? exp(l - m) / nval(&s1) : 0.0;
        }
    stats[0] = nval(&s1) * nval(&s1) / nval(&s2);
    stats[1] = m + log(nval(&s1)) - log((double)n);
    stats[2] = m;
    stats[3] = (double)nin;
}

/*
 * Proposal update between rounds of importance sampling (Sec. III.A, end of
 * the efficiency discussion: the proposal can be refined iteratively from the
 * local metric around the sampled points). The new centre is the
 * importance-weighted mean of the draws; the proposal around it is the metric
 * there (peo_metric_fd at the new centre, by the caller).
 * Offsets from the current centre, each periodic coordinate taken to its
 * image nearest theta0: d_i = theta_i - theta0, d -> d - P floor(d/P + 1/2).
 *   m      = sum_i w_i d_i / sum_i w_i
 *   theta0' = theta0 + m, periodic coordinates wrapped into [0, P)
 *   C      = sum_i w_i d_i d_i^T / sum_i w_i - m m^T   (D x D, row-major)
 * Draws with w_i = 0 are skipped (their parameters may lie outside the
 * support). With no positive weight theta0' = theta0 and C = 0. Weights need
 * not be normalised. Returns the number of draws with w_i > 0.
 */
long peo_proposal_update(const peo_event *ev, const double *th0, const double *theta, long n, const double *w,
                         double *th0_out, double *cov)
{
    const int D = peo_dim(ev->params);
    int pidx[3], np, a, b;
    double per[PEO_MAX_DIM];
    nsum sw = {0, 0}, s1[PEO_MAX_DIM], s2[PEO_MAX_DIM * PEO_MAX_DIM];
    long i, cnt = 0;
    double pp[3];
    np = periodic_dims(ev, pidx, pp);
    for (a = 0; a < D; a++)
        per[a] = 0.0;
    for (a = 0; a < np; a++)
        per[pidx[a]] = pp[a];
    for (a = 0; a < D; a++)
        s1[a].s = s1[a].c = 0.0;
    for (a = 0; a < D * D; a++)
        s2[a].s = s2[a].c = 0.0;
    for (i = 0; i < n; i++) {
        double d[PEO_MAX_DIM];
        if (!(w[i] > 0.0))
            continue;
        cnt++;
        for (a = 0; a < D; a++) {
            double v = theta[(long)a * n + i] - th0[a];
            if (per[a] > 0.0)
                v -= per[a] * floor(v / per[a] + 0.5);
            d[a] = v;
        }
        nadd(&sw, w[i]);
        for (a = 0; a < D; a++) {
            nadd(&s1[a], w[i] * d[a]);
            for (b = 0; b < D; b++)
                nadd(&s2[a * D + b], w[i] * d[a] * d[b]);
        }
    }
    if (cnt == 0) {
        for (a = 0; a < D; a++)
            th0_out[a] = th0[a];
        if (cov)
            for (a = 0; a < D * D; a++)
                cov[a] = 0.0;
        return 0;
    }
    {
        const double W = nval(&sw);
        double m[PEO_MAX_DIM];
        for (a = 0; a < D; a++) {
            m[a] = nval(&s1[a]) / W;
            th0_out[a] = th0[a] + m[a];
            if (per[a] > 0.0)
                th0_out[a] -= per[a] * floor(th0_out[a] / per[a]);
        }
        if (cov)
            for (a = 0; a < D; a++)
                for (b = 0; b < D; b++)
                    cov[a * D + b] = nval(&s2[a * D + b]) / W - m[a] * m[b];
    }
    return cnt;
}

/*
 * Tile-mixture proposal (Sec. II.A: tile the metric space, give each tile the
 * prior volume closest to its template, and propose from the tiles in
 * proportion to that volume times the posterior at the template; App. A:
 * template bank, tiling of the prior volume, proposal), on the slice of the
 * prior a detection points to: the ball of radius R in whitened coordinates
 * y = L^T (theta - c) of a metric G = L L^T around a centre c.
 */

/* Squared Euclidean distance of whitened points, summed in index order. */
static double wdist2(int D, const double *a, long sa, const double *b, long sb)
{
    double s = 0.0;
    int k;
    for (k = 0; k < D; k++) {
        double d = a[(long)k * sa] - b[(long)k * sb];
        s += d * d;
    }
    return s;
}

int peo_slice_dims(const peo_event *ev, const peo_slice *sl, int *idx)
{
    const int D = peo_dim(ev->params);
    int a, S = 0;
    for (a = 0; a < D; a++)
        if (sl->sub_mask == 0 || (sl->sub_mask >> a & 1u))
            idx[S++] = a;
    return S;
}

/* Candidate i of the slice: y_a = R (2 u_a - 1) (a < S) with u_a the
 * (a mod 2)-th uniform of Philox block (seed, stream, i, a / 2); kept if
 * |y|^2 <= R^2 and theta (the centre, plus L^-T y on the sliced coordinates)
 * lies in the prior's support. Returns 1 if kept. */
int peo_slice_candidate(const peo_event *ev, const peo_slice *sl, uint64_t seed, uint32_t stream, uint64_t i,
                        double *y, double *theta)
{
    const int D = peo_dim(ev->params);
    double u[PEO_MAX_DIM + 1], x[PEO_MAX_DIM], r2 = 0.0;
    peo_source src;
    int a, r, c, idx[PEO_MAX_DIM];
    const int S = peo_slice_dims(ev, sl, idx);
    for (a = 0; 2 * a < S; a++)
        block_uniforms(seed, stream, i, (uint32_t)a, &u[2 * a], &u[2 * a + 1]);
    for (a = 0; a < S; a++) {
        y[a] = sl->radius * (2.0 * u[a] - 1.0);
        r2 += y[a] * y[a];
    }
    /* theta_S - c_S = L^-T y: back substitution with L^T */
    for (r = S - 1; r >= 0; r--) {
        double t = y[r];
        for (c = r + 1; c < S; c++)
            t -= sl->chol[c * S + r] * x[c];
        x[r] = t / sl->chol[r * S + r];
    }
    for (a = 0; a < D; a++)
        theta[a] = sl->centre[a];
    for (a = 0; a < S; a++)
        theta[idx[a]] = sl->centre[idx[a]] + x[a];
    if (!(r2 <= sl->radius * sl->radius))
        return 0;
    return peo_source_from_theta(ev, theta, &src) ? 1 : 0;
}

/* The kept candidates among first .. first + n - 1, in order: y [S][n],
 * theta [D][n] (row stride n), logprior [n]. Returns how many were kept. */
long peo_slice_sample(const peo_event *ev, const peo_slice *sl, uint64_t seed, uint32_t stream, long first, long n,
                      double *y, double *theta, double *logprior)
{
    const int D = peo_dim(ev->params);
    long i, k = 0;
    int a, idx[PEO_MAX_DIM];
    const int S = peo_slice_dims(ev, sl, idx);
    for (i = 0; i < n; i++) {
        double yy[PEO_MAX_DIM], th[PEO_MAX_DIM];
        if (!peo_slice_candidate(ev, sl, seed, stream, (uint64_t)(first + i), yy, th))
            continue;
        for (a = 0; a < S; a++)
            y[(long)a * n + k] = yy[a];
        for (a = 0; a < D; a++)
            theta[(long)a * n + k] = th[a];
        logprior[k] = peo_logprior(ev, th);
        k++;
    }
    return k;
}

/* Stochastic template bank in the slice (App. A, template bank generation;
 * the stochastic placement the paper uses, in its plain form): candidates in
 * order (consecutive counters from 0, batches of `batch`), a kept candidate
 * becomes a template when its whitened squared distance to every template so
 * far is at least min_dist^2. Stops after the first batch that adds fewer
 * than stop_fraction * (kept candidates of the batch), when max_tiles
 * templates exist, or after max_batches batches. Templates: y [S][max_tiles],
 * theta [D][max_tiles] (row stride max_tiles). Returns the number of templates;
 * *consumed = candidates drawn. */
long peo_tile_bank(const peo_event *ev, const peo_slice *sl, double min_dist, uint64_t seed, uint32_t stream,
                   long batch, long max_tiles, double stop_fraction, long max_batches, double *ty, double *tth,
                   long *consumed)
{
    const int D = peo_dim(ev->params);
    const double r2 = min_dist * min_dist;
    long m = 0, b, i;
    int a, idx[PEO_MAX_DIM];
    const int S = peo_slice_dims(ev, sl, idx);
    *consumed = 0;
    for (b = 0; b < max_batches && m < max_tiles; b++) {
        long kept = 0, added = 0;
        for (i = 0; i < batch && m < max_tiles; i++) {
            double yy[PEO_MAX_DIM], th[PEO_MAX_DIM];
            long j, ok = 1;
            const uint64_t ci = (uint64_t)(b * batch + i);
            *consumed = (long)ci + 1;
            if (!peo_slice_candidate(ev, sl, seed, stream, ci, yy, th))
                continue;
            kept++;
            for (j = 0; j < m; j++)
                if (wdist2(S, yy, 1, ty + j, max_tiles) < r2) {
                    ok = 0;
                    break;
                }
            if (!ok)
                continue;
            for (a = 0; a < S; a++)
                ty[(long)a * max_tiles + m] = yy[a];
            for (a = 0; a < D; a++)
                tth[(long)a * max_tiles + m] = th[a];
            m++;
            added++;
        }
        if (m >= max_tiles || (double)added < stop_fraction * (double)kept)
            break;
    }
    return m;
}

/* Tile of each sample: the template nearest in whitened coordinates, the
 * lowest index among equals. tiles [D][ld_t], samples [D][ld_s]. */
void peo_tile_assign(int D, long n_tiles, const double *ty, long ld_t, long n, const double *y, long ld_s,
                     int *tile_of)
{
    long s, j;
    for (s = 0; s < n; s++) {
        long best = 0;
        double bd = wdist2(D, y + s, ld_s, ty, ld_t);
        for (j = 1; j < n_tiles; j++) {
            double d = wdist2(D, y + s, ld_s, ty + j, ld_t);
            if (d < bd) {
                bd = d;
                best = j;
            }
        }
        tile_of[s] = (int)best;
    }
}

/* Proposal draws: sample s carries mass m_s = exp(ll_{t(s)} - max ll + lp_s -
 * max lp) (its tile's likelihood times its prior density; 0 if either is
 * -inf); draw i takes the first uniform u of Philox block (seed, stream, i, 0)
 * and the smallest s with u C_P <= C_s, C_s = m_0 + ... + m_s (compensated).
 * theta_i = sample s, logprior_i = lp_s, logq_i = ln m_s - ln(C_P / P): the
 * proposal density relative to the flat measure the samples were drawn from
 * (each sample 1/P there, m_s / C_P here). index_i = s. With no positive mass: logprior -inf, logq 0,
 * index -1, theta = sample 0; returns 5. Else returns 0. */
int peo_tile_draw(long n_tiles, const double *tile_ll, long P, const int *tile_of, const double *lp, int D,
                  const double *samples, long ld, uint64_t seed, uint32_t stream, long n, double *theta,
                  double *logq, double *logprior, long *index)
{
    double lmax = -INFINITY, pmax = -INFINITY, tot;
    double *C;
    nsum acc = {0, 0};
    long s, i, j;
    int a;
    for (j = 0; j < n_tiles; j++)
        if (isfinite(tile_ll[j]) && tile_ll[j] > lmax)
            lmax = tile_ll[j];
    for (s = 0; s < P; s++)
        if (isfinite(lp[s]) && lp[s] > pmax)
            pmax = lp[s];
    C = (double *)malloc(sizeof(double) * (P > 0 ? P : 1));
    for (s = 0; s < P; s++) {
        const double l = tile_ll[tile_of[s]];
        const double m = (isfinite(l) && isfinite(lp[s])) ? exp((l - lmax) + (lp[s] - pmax)) : 0.0;
        nadd(&acc, m);
        C[s] = nval(&acc);
    }
    tot = P > 0 ? C[P - 1] : 0.0;
    for (i = 0; i < n; i++) {
        double u, u2;
        block_uniforms(seed, stream, (uint64_t)i, 0, &u, &u2);
        if (!(tot > 0.0)) {
            for (a = 0; a < D; a++)
                theta[(long)a * n + i] = P > 0 ? samples[(long)a * ld] : 0.0;
            logq[i] = 0.0;
            logprior[i] = -INFINITY;
            index[i] = -1;
            continue;
        }
        {
            const double target = u * tot;
            long lo = 0, hi = P - 1;
            while (lo < hi) { /* smallest s with target <= C_s */
                long mid = lo + (hi - lo) / 2;
                if (target <= C[mid])
                    hi = mid;
                else
                    lo = mid + 1;
            }
            s = lo;
        }
        for (a = 0; a < D; a++)
            theta[(long)a * n + i] = samples[(long)a * ld + s];
        logprior[i] = lp[s];
        logq[i] = ((tile_ll[tile_of[s]] - lmax) + (lp[s] - pmax)) - log(tot / (double)P);
        index[i] = s;
    }
    free(C);
    return tot > 0.0 ? 0 : 5;
}

/*
 * Tile weights for the next round (the iterative update of the proposal the
 * paper suggests at the end of Sec. III.A, applied to the tile mixture): the
 * posterior mass of tile j estimated by importance sampling from the previous
 * round, P_j = sum of the normalised weights w_i of the draws from tile j,
 * mixed with the previous round's tile probabilities p_j (defensive share
 * alpha):  pi_j = (1 - alpha) P_j / sum P + alpha p_j,
 * p_j = exp(l_j - max l) V_j / sum_k exp(l_k - max l) V_k, with V_j = sum over
 * the tile's samples of exp(lp_s - max lp) (its prior volume). The result
 * l'_j = ln pi_j - ln V_j (-inf where pi_j or V_j is 0) fed to peo_tile_draw
 * gives sample s the mass pi_j exp(lp_s) / V_j. index: the previous draws'
 * sample indices (negative ones are skipped).
 */
void peo_tile_reweight(long n_tiles, const double *tile_ll, long P, const int *tile_of, const double *lp, long n,
                       const long *index, const double *w, double alpha, double *out)
{
    double lmax = -INFINITY, pmax = -INFINITY, ptot, wtot;
    nsum *V = (nsum *)calloc((size_t)(n_tiles > 0 ? n_tiles : 1), sizeof(nsum));
    nsum *Ph = (nsum *)calloc((size_t)(n_tiles > 0 ? n_tiles : 1), sizeof(nsum));
    nsum pt = {0, 0}, wt = {0, 0};
    long s, j, i;
    for (j = 0; j < n_tiles; j++)
        if (isfinite(tile_ll[j]) && tile_ll[j] > lmax)
            lmax = tile_ll[j];
    for (s = 0; s < P; s++)
        if (isfinite(lp[s]) && lp[s] > pmax)
            pmax = lp[s];
    for (s = 0; s < P; s++)
        if (isfinite(lp[s]))
            nadd(&V[tile_of[s]], exp(lp[s] - pmax));
    for (i = 0; i < n; i++)
        if (index[i] >= 0 && w[i] > 0.0) {
            nadd(&Ph[tile_of[index[i]]], w[i]);
            nadd(&wt, w[i]);
        }
    for (j = 0; j < n_tiles; j++)
        if (isfinite(tile_ll[j]))
            nadd(&pt, exp(tile_ll[j] - lmax) * nval(&V[j]));
    ptot = nval(&pt);
    wtot = nval(&wt);
    for (j = 0; j < n_tiles; j++) {
        const double v = nval(&V[j]);
        const double pj = (ptot > 0.0 && isfinite(tile_ll[j])) ? exp(tile_ll[j] - lmax) * v / ptot : 0.0;
        const double hj = wtot > 0.0 ? nval(&Ph[j]) / wtot : 0.0;
        const double pi = (1.0 - alpha) * hj + alpha * pj;
        out[j] = (pi > 0.0 && v > 0.0) ? log(pi) - log(v) : -INFINITY;
    }
    free(V);
    free(Ph);
}

/*
 * Relative binning (Zackay, Dai & Venumadhav 2018, arXiv:1806.08792; the paper
 * lists such reduced representations among the ways to speed the likelihood
 * up, Sec. I). Around a fiducial waveform h0 close to the peak, the ratio
 * h/h0 of any nearby waveform is smooth in frequency and is replaced, bin by
 * bin, by its linear interpolation between the bin edges; the data then enter
 * only through per-bin sums.
 *
 * Edges: grid indices 0 = k_0 < k_1 < ... < k_B = K. The next edge is the
 * first k at which the phase envelope
 *   E(f) = 2 pi sum_a sgn(a) (f / f_a)^a,  a in {-5/3, -2/3, 1, 5/3, 7/3},
 *   f_a = f_lo for a < 0 and f_hi = f_lo + K df for a > 0,
 * has grown by at least eps since the last edge. Returns the number of edges,
 * or -1 if more than max_edges would be needed.
 */
static double rb_envelope(double f, double f_lo, double f_hi)
{
    static const double a[5] = {-5.0 / 3.0, -2.0 / 3.0, 1.0, 5.0 / 3.0, 7.0 / 3.0};
    double e = 0.0;
    int i;
    for (i = 0; i < 5; i++)
        e += (a[i] < 0.0 ? -1.0 : 1.0) * pow(f / (a[i] < 0.0 ? f_lo : f_hi), a[i]);
    return 2.0 * PI * e;
}

long peo_relbin_edges(const peo_event *ev, double eps, long max_edges, long *edges)
{
    const long K = ev->n_bins;
    const double f_hi = ev->f_lo + (double)K * ev->df;
    long k, b = 0;
    double eb;
    if (max_edges < 2 || K < 1)
        return -1;
    edges[0] = 0;
    eb = rb_envelope(ev->f_lo, ev->f_lo, f_hi);
    for (k = 1; k < K; k++) {
        const double e = rb_envelope(ev->f_lo + (double)k * ev->df, ev->f_lo, f_hi);
        if (e - eb >= eps) {
            if (b + 2 >= max_edges)
                return -1;
            edges[++b] = k;
            eb = e;
        }
    }
    edges[++b] = K;
    return b + 1;
}

/* Phase of detector d's model at f (radians): Psi(f) + 2 pi f dt_d. */
static double rb_phase(const peo_source *s, int d, double f)
{
    return peo_psi(s, f) + 2.0 * PI * f * s->dt[d];
}

/*
 * Relative-binning log-likelihoods of n draws about the fiducial theta_f.
 * Per detector, c_k = 4 df conj(d_k) h0_k / S_k with the unit-response
 * fiducial h0_k = f_k^-7/6 exp(-i Phi0_d(f_k)) (no cut). For a draw with
 * response R_d, phase Phi_d and cut kc, rho(f) = exp(-i (Phi_d - Phi0_d)(f))
 * is interpolated linearly between the edges of each bin:
 *   Z_d = R_d sum_b sum_{k in b, k < kc} c_k (rho_b + (rho_{b+1} - rho_b)
 *         (f_k - f_b) / (f_{b+1} - f_b)),
 * Z = sum_d Z_d; H = sum_d |R_d|^2 sum_{k < kc} 4 df f_k^-7/3 / S_k exactly;
 * ln L from Z and H as in peo_loglike. zh: Re Z, Im Z, H (may be NULL).
 */
void peo_relbin_loglike(const peo_event *ev, const double *theta_f, long n_edges, const long *edges,
                        const double *theta, long n, double *loglike, double *zh)
{
    const int D = peo_dim(ev->params);
    const long K = ev->n_bins;
    peo_source s0;
    double *c = (double *)malloc(sizeof(double) * 2 * (size_t)ev->n_det * (size_t)K);
    long i, k, b;
    int d;
    peo_source_from_theta(ev, theta_f, &s0);
    for (d = 0; d < ev->n_det; d++) {
        const double *S = ev->psd + (long)d * K;
        const double *dd = ev->data + 2 * (long)d * K;
        for (k = 0; k < K; k++) {
            const double f = ev->f_lo + (double)k * ev->df;
            const double ph = rb_phase(&s0, d, f), a = pow(f, -7.0 / 6.0), w = 4.0 * ev->df / S[k];
            const double hr = a * cos(ph), hi = -a * sin(ph);
            /* conj(d) h0 */
            c[2 * ((long)d * K + k)] = w * (dd[2 * k] * hr + dd[2 * k + 1] * hi);
            c[2 * ((long)d * K + k) + 1] = w * (dd[2 * k] * hi - dd[2 * k + 1] * hr);
        }
    }
    for (i = 0; i < n; i++) {
        double th_in[PEO_MAX_DIM], th[PEO_MAX_DIM];
        peo_source s;
        nsum zr = {0, 0}, zi = {0, 0}, hh = {0, 0};
        double Zr, Zi, H;
        int a;
        for (a = 0; a < D; a++)
            th_in[a] = theta[(long)a * n + i];
        likelihood_theta(ev, th_in, th);
        if (!peo_source_from_theta(ev, th, &s)) {
            loglike[i] = -INFINITY;
            if (zh)
                zh[3 * i] = zh[3 * i + 1] = zh[3 * i + 2] = 0.0;
            continue;
        }
        s.kcut = peo_kcut(ev, s.fisco);
        for (d = 0; d < ev->n_det; d++) {
            const double *S = ev->psd + (long)d * K;
            nsum ur = {0, 0}, ui = {0, 0};
            for (b = 0; b + 1 < n_edges && edges[b] < s.kcut; b++) {
                const long k0 = edges[b], k1 = edges[b + 1];
                const double f0 = ev->f_lo + (double)k0 * ev->df, f1 = ev->f_lo + (double)k1 * ev->df;
                const double p0 = rb_phase(&s, d, f0) - rb_phase(&s0, d, f0);
                const double p1 = rb_phase(&s, d, f1) - rb_phase(&s0, d, f1);
                const double r0r = cos(p0), r0i = -sin(p0), r1r = cos(p1), r1i = -sin(p1);
                const double sr = (r1r - r0r) / (f1 - f0), si = (r1i - r0i) / (f1 - f0);
                for (k = k0; k < k1 && k < s.kcut; k++) {
                    const double t = ev->f_lo + (double)k * ev->df - f0;
                    const double qr = r0r + sr * t, qi = r0i + si * t;
                    const double cr = c[2 * ((long)d * K + k)], ci = c[2 * ((long)d * K + k) + 1];
                    nadd(&ur, cr * qr - ci * qi);
                    nadd(&ui, cr * qi + ci * qr);
                }
            }
            /* times R_d */
            nadd(&zr, s.rre[d] * nval(&ur) - s.rim[d] * nval(&ui));
            nadd(&zi, s.rre[d] * nval(&ui) + s.rim[d] * nval(&ur));
            for (k = 0; k < s.kcut; k++) {
                const double f = ev->f_lo + (double)k * ev->df;
                nadd(&hh, (s.rre[d] * s.rre[d] + s.rim[d] * s.rim[d]) * 4.0 * ev->df * pow(f, -7.0 / 3.0) / S[k]);
            }
        }
        Zr = nval(&zr);
        Zi = nval(&zi);
        H = nval(&hh);
        if (zh) {
            zh[3 * i] = Zr;
            zh[3 * i + 1] = Zi;
            zh[3 * i + 2] = H;
        }
        loglike[i] = loglike_from_zh(ev, Zr, Zi, H);
    }
    free(c);
}

/* Waveform similarity (App. A maps the prior volume to tiles by it; Sec. III
 * uses the plain overlap for aligned spins): the match of a and b is their
 * complex overlap <h_a, h_b> = 4 df sum_d sum_k conj(h_a) h_b / S, maximised
 * over a constant phase (its modulus), divided by the norms,
 *   m(a, b) = |<h_a, h_b>| / sqrt((h_a|h_a)(h_b|h_b)),
 * each waveform zero above its own ISCO bin. 0 when either norm is 0. The
 * waveforms of a pair are made bin by bin (the same as in loglike_one). */
static double match_pair(const peo_event *ev, const peo_source *sa, const peo_source *sb)
{
    nsum re = {0, 0}, im = {0, 0}, na = {0, 0}, nb = {0, 0};
    int d;
    long k;
    for (d = 0; d < ev->n_det; d++) {
        const double *S = ev->psd + (long)d * ev->n_bins;
        for (k = 0; k < ev->n_bins && (k < sa->kcut || k < sb->kcut); k++) {
            double ar = 0.0, ai = 0.0, br = 0.0, bi = 0.0;
            const double w = 4.0 * ev->df / S[k];
            if (k < sa->kcut)
                wf_bin(ev, sa, d, k, &ar, &ai);
            if (k < sb->kcut)
                wf_bin(ev, sb, d, k, &br, &bi);
            nadd(&re, w * (ar * br + ai * bi));
            nadd(&im, w * (ar * bi - ai * br));
            nadd(&na, w * (ar * ar + ai * ai));
            nadd(&nb, w * (br * br + bi * bi));
        }
    }
    if (!(nval(&na) > 0.0) || !(nval(&nb) > 0.0))
        return 0.0;
    return hypot(nval(&re), nval(&im)) / sqrt(nval(&na) * nval(&nb));
}

/* The match maximised over a grid of time shifts as well (App. A maps the prior
 * volume to templates by their overlap maximised over the extrinsic time and
 * phase): max over tau_j = j dt, |j| <= n_shift, of
 *   |sum_d sum_k w_k conj(a_dk) b_dk exp(-2 pi i f_k tau_j)| / sqrt(<a,a> <b,b>),
 * b shifted in time by tau_j (its tc moved by tau_j), each bin's rotation from
 * the sine and cosine of the full angle. */
static double match_pair_shift(const peo_event *ev, const peo_source *sa, const peo_source *sb, double dt,
                               int n_shift)
{
    const int nj = 2 * n_shift + 1;
    nsum na = {0, 0}, nb = {0, 0};
    nsum *re = (nsum *)calloc((size_t)nj, sizeof(nsum)), *im = (nsum *)calloc((size_t)nj, sizeof(nsum));
    double best = 0.0;
    int d, j;
    long k;
    if (!re || !im) {
        free(re);
        free(im);
        return -1.0;
    }
    for (d = 0; d < ev->n_det; d++) {
        const double *S = ev->psd + (long)d * ev->n_bins;
        for (k = 0; k < ev->n_bins && (k < sa->kcut || k < sb->kcut); k++) {
            double ar = 0.0, ai = 0.0, br = 0.0, bi = 0.0, cr, ci;
            const double w = 4.0 * ev->df / S[k];
            const double f = ev->f_lo + (double)k * ev->df;
            if (k < sa->kcut)
                wf_bin(ev, sa, d, k, &ar, &ai);
            if (k < sb->kcut)
                wf_bin(ev, sb, d, k, &br, &bi);
            nadd(&na, w * (ar * ar + ai * ai));
            nadd(&nb, w * (br * br + bi * bi));
            cr = w * (ar * br + ai * bi); /* w conj(a) b */
            ci = w * (ar * bi - ai * br);
            for (j = 0; j < nj; j++) {
                const double ang = -2.0 * PI * f * ((double)(j - n_shift) * dt);
                const double c = cos(ang), sn = sin(ang);
                nadd(&re[j], cr * c - ci * sn);
                nadd(&im[j], cr * sn + ci * c);
            }
        }
    }
    if (nval(&na) > 0.0 && nval(&nb) > 0.0)
        for (j = 0; j < nj; j++) {
            const double m = hypot(nval(&re[j]), nval(&im[j])) / sqrt(nval(&na) * nval(&nb));
            if (m > best)
                best = m;
        }
    free(re);
    free(im);
    return best;
}

double peo_match_shift(const peo_event *ev, const double *theta_a, const double *theta_b, double dt, int n_shift)
{
    peo_source sa, sb;
    double ta[PEO_MAX_DIM], tb[PEO_MAX_DIM];
    likelihood_theta(ev, theta_a, ta);
    likelihood_theta(ev, theta_b, tb);
    if (!peo_source_from_theta(ev, ta, &sa) || !peo_source_from_theta(ev, tb, &sb))
        return -1.0;
    sa.kcut = peo_kcut(ev, sa.fisco);
    sb.kcut = peo_kcut(ev, sb.fisco);
    return match_pair_shift(ev, &sa, &sb, dt, n_shift);
}

/* Tile of each sample by the time-shift-maximised match (brute force over the
 * templates and the shifts); as peo_tile_assign_match otherwise. */
void peo_tile_assign_match_shift(const peo_event *ev, long n_tiles, const double *tth, long ld_t, long n,
                                 const double *th, long ld_s, double dt, int n_shift, int *tile_of, double *match)
{
    const int D = ev->params == PEO_PARAMS_4D ? 4 : 11;
    peo_source *st = (peo_source *)malloc(sizeof(peo_source) * (size_t)(n_tiles > 0 ? n_tiles : 1));
    long j, s;
    for (j = 0; j < n_tiles; j++) {
        double t[PEO_MAX_DIM], tl[PEO_MAX_DIM];
        int a;
        for (a = 0; a < D; a++)
            t[a] = tth[(long)a * ld_t + j];
        likelihood_theta(ev, t, tl);
        peo_source_from_theta(ev, tl, &st[j]);
        st[j].kcut = peo_kcut(ev, st[j].fisco);
    }
#pragma omp parallel for schedule(dynamic, 1)
    for (s = 0; s < n; s++) {
        double t[PEO_MAX_DIM], tl[PEO_MAX_DIM], bm = -1.0;
        peo_source ss;
        long best = 0, jj;
        int a;
        for (a = 0; a < D; a++)
            t[a] = th[(long)a * ld_s + s];
        likelihood_theta(ev, t, tl);
        peo_source_from_theta(ev, tl, &ss);
        ss.kcut = peo_kcut(ev, ss.fisco);
        for (jj = 0; jj < n_tiles; jj++) {
            const double m = match_pair_shift(ev, &ss, &st[jj], dt, n_shift);
            if (m > bm) {
                bm = m;
                best = jj;
            }
        }
        tile_of[s] = (int)best;
        match[s] = bm;
    }
    free(st);
}

/* Match of two parameter points (see match_pair); -1 if either is outside the
 * support. */
double peo_match(const peo_event *ev, const double *theta_a, const double *theta_b)
{
    peo_source sa, sb;
    double ta[PEO_MAX_DIM], tb[PEO_MAX_DIM];
    likelihood_theta(ev, theta_a, ta);
    likelihood_theta(ev, theta_b, tb);
    if (!peo_source_from_theta(ev, ta, &sa) || !peo_source_from_theta(ev, tb, &sb))
        return -1.0;
    sa.kcut = peo_kcut(ev, sa.fisco);
    sb.kcut = peo_kcut(ev, sb.fisco);
    return match_pair(ev, &sa, &sb);
}

/* Tile of each sample by waveform similarity (App. A): the template of
 * largest match with the sample, the lowest index among equals, by brute force
 * over every template. tth [D][ld_t] (n_tiles used), th [D][ld_s] (n used);
 * tile_of [n], match [n] (the largest match). */
void peo_tile_assign_match(const peo_event *ev, long n_tiles, const double *tth, long ld_t, long n,
                           const double *th, long ld_s, int *tile_of, double *match)
{
    const int D = ev->params == PEO_PARAMS_4D ? 4 : 11;
    peo_source *st = (peo_source *)malloc(sizeof(peo_source) * (size_t)(n_tiles > 0 ? n_tiles : 1));
    long j, s;
    for (j = 0; j < n_tiles; j++) {
        double t[PEO_MAX_DIM], tl[PEO_MAX_DIM];
        int a;
        for (a = 0; a < D; a++)
            t[a] = tth[(long)a * ld_t + j];
        likelihood_theta(ev, t, tl);
        peo_source_from_theta(ev, tl, &st[j]);
        st[j].kcut = peo_kcut(ev, st[j].fisco);
    }
#pragma omp parallel for schedule(dynamic, 1)
    for (s = 0; s < n; s++) {
        double t[PEO_MAX_DIM], tl[PEO_MAX_DIM], bm = -1.0;
        peo_source ss;
        long best = 0, jj;
        int a;
        for (a = 0; a < D; a++)
            t[a] = th[(long)a * ld_s + s];
        likelihood_theta(ev, t, tl);
        peo_source_from_theta(ev, tl, &ss);
        ss.kcut = peo_kcut(ev, ss.fisco);
        for (jj = 0; jj < n_tiles; jj++) {
            const double m = match_pair(ev, &ss, &st[jj]);
            if (m > bm) {
                bm = m;
                best = jj;
            }
        }
        tile_of[s] = (int)best;
        match[s] = bm;
    }
    free(st);
}
