// pe_device.h -- device-side model of the likelihood engine (gfx950).
//
// TaylorF2 phase in "turns" (cycles) as a Horner polynomial in x = f^(1/3),
// source parameters from theta, detector response, FP64 sincos of a phase in
// turns, Philox4x32-10 and ln I0. Written for the GPU path only.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pe_internal.h"

namespace pe {

// ---------------------------------------------------------------------------
// TaylorF2 phase coefficients phi_j (and log coefficients) of
// Psi = 2 pi f tc - phic - pi/4 + 3/(128 eta v^5) sum_j (phi_j + phil_j ln v) v^j,
// written in the symmetric/antisymmetric spins chis = (chi1+chi2)/2,
// chia = (chi1-chi2)/2 and delta = (m1-m2)/M. Non-spinning terms to 3.5PN:
// Buonanno, Iyer, Ochsner, Pan, Sathyaprakash, PRD 80, 084043 (2009).
// Spin-orbit 1.5/2.5/3/3.5PN and 2PN spin-spin: Mishra, Kela, Arun, Faye,
// PRD 93, 084054 (2016). The 2.5PN term multiplies (1 + 3 ln v).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void pn_coeffs(double eta, double delta, double chis, double chia, double phi[8],
                                          double& phil5, double& phil6) {
    const double eta2 = eta * eta, eta3 = eta2 * eta;
    const double pi2 = kPi * kPi;
    phi[0] = 1.0;
    phi[1] = 0.0;
    phi[2] = 3715.0 / 756.0 + 55.0 / 9.0 * eta;
    phi[3] = -16.0 * kPi + 113.0 / 3.0 * delta * chia + (113.0 / 3.0 - 76.0 / 3.0 * eta) * chis;
    phi[4] = 15293365.0 / 508032.0 + 27145.0 / 504.0 * eta + 3085.0 / 72.0 * eta2 +
             (-405.0 / 8.0 + 200.0 * eta) * chia * chia - 405.0 / 4.0 * delta * chia * chis +
             (-405.0 / 8.0 + 2.5 * eta) * chis * chis;
    const double gam = (732985.0 / 2268.0 - 24260.0 / 81.0 * eta - 340.0 / 9.0 * eta2) * chis +
                       (732985.0 / 2268.0 + 140.0 / 9.0 * eta) * delta * chia;
    phi[5] = kPi * (38645.0 / 756.0 - 65.0 / 9.0 * eta) - gam;
    phil5 = 3.0 * phi[5];
    phi[6] = 11583231236531.0 / 4694215680.0 - 640.0 / 3.0 * pi2 - 6848.0 / 21.0 * kEulerGamma -
             6848.0 / 21.0 * kLn4 + (-15737765635.0 / 3048192.0 + 2255.0 / 12.0 * pi2) * eta +
             76055.0 / 1728.0 * eta2 - 127825.0 / 1296.0 * eta3 +
             kPi * (2270.0 / 3.0 * delta * chia + (2270.0 / 3.0 - 520.0 * eta) * chis);
    phil6 = -6848.0 / 21.0;
    phi[7] = kPi * (77096675.0 / 254016.0 + 378515.0 / 1512.0 * eta - 74045.0 / 756.0 * eta2) +
             (-25150083775.0 / 3048192.0 + 10566655595.0 / 762048.0 * eta - 1042165.0 / 3024.0 * eta2 +
              5345.0 / 36.0 * eta3) * chis +
             (-25150083775.0 / 3048192.0 + 26804935.0 / 6048.0 * eta - 1985.0 / 48.0 * eta2) * delta * chia;
}

// Slot of x in a batch's prefix offsets: the last e with off[e] <= x (events
// with nothing to do have off[e] == off[e+1] and are skipped).
__device__ __forceinline__ int find_slot(const int64_t* __restrict__ off, int n, int64_t x) {
    int lo = 0, hi = n;  // off[lo] <= x < off[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= x)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// Per-draw source quantities.
struct Src {
    double M, eta, delta, chis, chia, tc, phic;
    double rre[PE_MAX_DET], rim[PE_MAX_DET], dt[PE_MAX_DET];
    double fisco;
    int ok;
};

// Source direction n and polarisation axes X, Y for (ra, dec, psi): the sky
// basis (east, north) at the source direction, rotated by psi.
struct SkyFrame {
    double n0, n1, n2, X0, X1, X2, Y0, Y1, Y2;
};

__device__ __forceinline__ SkyFrame sky_frame(const EvConst& ev, double ra, double dec, double psi) {
    double sl, cl, sd, cd, sp, cp;
    sincos(ra - ev.gmst, &sl, &cl);
    sincos(dec, &sd, &cd);
    sincos(psi, &sp, &cp);
    SkyFrame f;
    f.n0 = cd * cl;
    f.n1 = cd * sl;
    f.n2 = sd;
    const double u0 = -sl, u1 = cl;  // u2 = 0
    const double w0 = -sd * cl, w1 = -sd * sl, w2 = cd;
    f.X0 = cp * u0 + sp * w0;
    f.X1 = cp * u1 + sp * w1;
    f.X2 = sp * w2;
    f.Y0 = -sp * u0 + cp * w0;
    f.Y1 = -sp * u1 + cp * w1;
    f.Y2 = cp * w2;
    return f;
}

// Long-wavelength response F+, Fx of detector d and the arrival delay dt
// (geocentre -> detector).
__device__ __forceinline__ void antenna(const EvConst& ev, int d, const SkyFrame& f, double& fp, double& fc,
                                        double& dt) {
    const double* D = ev.dtensor[d];  // xx xy xz yy yz zz
    auto quad = [&](double a0, double a1, double a2, double b0, double b1, double b2) {
        return D[0] * a0 * b0 + D[3] * a1 * b1 + D[5] * a2 * b2 + D[1] * (a0 * b1 + a1 * b0) +
               D[2] * (a0 * b2 + a2 * b0) + D[4] * (a1 * b2 + a2 * b1);
    };
    fp = quad(f.X0, f.X1, f.X2, f.X0, f.X1, f.X2) - quad(f.Y0, f.Y1, f.Y2, f.Y0, f.Y1, f.Y2);
    fc = 2.0 * quad(f.X0, f.X1, f.X2, f.Y0, f.Y1, f.Y2);
    dt = -(kREarth / kC) * (ev.up[d][0] * f.n0 + ev.up[d][1] * f.n1 + ev.up[d][2] * f.n2);
}

__device__ __forceinline__ double f_isco(double M) { return 1.0 / (kSix32 * kPi * M * kTsun); }

// Support of the prior and the total mass of theta: the part of the source
// that the support mask, the ISCO cut and the prior need.
__device__ __forceinline__ int mass_and_support(const EvConst& ev, const double* th, double& M) {
    if (ev.params == PE_PARAMS_4D) {
        const double mc = th[0], eta = th[1], chi = th[2];
        M = mc * exp(-0.6 * log(eta));  // eta^(-3/5)
        return (mc > 0.0) && (eta > 0.0) && (eta <= 0.25) && (fabs(chi) <= ev.chi_max);
    }
    const double mc = th[0], q = th[1], c1 = th[2], c2 = th[3];
    const double dec = th[5], iota = th[6], dl = th[8];
    // M = Mc (1+q)^(6/5) q^(-3/5) = Mc eta^(-3/5), eta = q/(1+q)^2 (as exp and
    // log: a third cheaper than pow, within a few ulp of it)
    const double opq = 1.0 + q;
    M = mc * exp(-0.6 * log(q / (opq * opq)));
    return (mc > 0.0) && (q > 0.0) && (q <= 1.0) && (fabs(c1) <= ev.chi_max) && (fabs(c2) <= ev.chi_max) &&
           (fabs(dec) <= 0.5 * kPi) && (iota >= 0.0) && (iota <= kPi) &&
           (ev.dist || ((dl > 0.0) && (dl <= ev.dl_max)));
}

// Support of the prior and the source parameters of theta (D values).
// Log prior (flat in Mc, eta or q, spins, tc, ra, psi, phic; cos dec; sin
// iota; dL^2 unless the likelihood is distance-marginalised; unnormalised),
// -inf outside the support.
__device__ __forceinline__ double log_prior_of(const EvConst& ev, const double* th) {
    double M;
    if (!mass_and_support(ev, th, M)) return -INFINITY;
    if (ev.params == PE_PARAMS_4D) return 0.0;
    // one logarithm of the product (every factor is positive inside the support)
    const double ang = cos(th[5]) * sin(th[6]);
    return log(ev.dist ? ang : ang * (th[8] * th[8]));
}

// The likelihood of a distance-marginalised event is evaluated at the
// reference distance dl_max (Z and H scale as 1/dL and 1/dL^2 from there).
__device__ __forceinline__ void likelihood_distance(const EvConst& ev, double* th) {
    if (ev.dist) th[8] = ev.dl_max;
}

__device__ __forceinline__ int source_from_theta(const EvConst& ev, const double* th, Src& s) {
    int ok;
    double M;
    ok = mass_and_support(ev, th, M);
    s.M = M;
    if (ev.params == PE_PARAMS_4D) {
        const double eta = th[1], chi = th[2];
        s.eta = eta;
        s.delta = sqrt(fmax(0.0, 1.0 - 4.0 * eta));
        s.chis = chi;
        s.chia = 0.0;
        s.tc = th[3];
        s.phic = 0.0;
        const double r = ev.amp0 * ev.scale;
#pragma unroll
        for (int d = 0; d < PE_MAX_DET; ++d) {
            s.rre[d] = r;
            s.rim[d] = 0.0;
            s.dt[d] = 0.0;
        }
    } else {
        const double mc = th[0], q = th[1], c1 = th[2], c2 = th[3];
        const double ra = th[4], dec = th[5], iota = th[6], psi = th[7], dl = th[8];
        const double opq = 1.0 + q;
        s.eta = q / (opq * opq);
        s.delta = (1.0 - q) / opq;
        s.chis = 0.5 * (c1 + c2);
        s.chia = 0.5 * (c1 - c2);
        s.tc = th[9];
        s.phic = (ev.phase == PE_PHASE_EXPLICIT) ? th[10] : 0.0;
        // Newtonian stationary-phase amplitude sqrt(5/24) pi^(-2/3) Mc^(5/6) / dL, times the unit scale
        // (Mc)^(5/6) = sqrt(Mc) cbrt(Mc): a quarter of pow's instructions
        const double mct = mc * kTsun;
        const double amp = kAmpNewt * (sqrt(mct) * cbrt(mct)) / (dl * (kMpc / kC)) * ev.scale;
        const double ci = cos(iota);
        const double hp = 0.5 * (1.0 + ci * ci), hx = ci;
        const SkyFrame fr = sky_frame(ev, ra, dec, psi);
        // fixed-bound loop, so the per-detector arrays stay in registers
#pragma unroll
        for (int d = 0; d < PE_MAX_DET; ++d) {
            if (d >= ev.n_det) break;
            double fp, fc, dt;
            antenna(ev, d, fr, fp, fc, dt);
            s.rre[d] = amp * fp * hp;  // F+ h+ + Fx hx, hx = -i cos(iota) A
            s.rim[d] = -amp * fc * hx;
            s.dt[d] = dt;
        }
    }
    s.fisco = f_isco(s.M);
    s.ok = ok;
    return ok;
}

// f_k = f_lo + k df without contraction (exact on power-of-two grids).
__device__ __forceinline__ double grid_f(const EvConst& ev, int64_t k) {
    return __dadd_rn(ev.f_lo, __dmul_rn((double)k, ev.df));
}

// Number of bins with f_k < fisco.
__device__ __forceinline__ int64_t kcut_of(const EvConst& ev, double fisco) {
    if (!(fisco > ev.f_lo)) return 0;
    const double q = (fisco - ev.f_lo) / ev.df;
    int64_t k = (q >= (double)ev.K) ? ev.K : (int64_t)ceil(q);
    while (k > 0 && !(grid_f(ev, k - 1) < fisco)) --k;
    while (k < ev.K && grid_f(ev, k) < fisco) ++k;
    return k;
}

// Horner coefficients of the phase in turns:
// Phi/(2 pi) = x^-5 (A0 + A1 x + ... + A7 x^7) + (B5 + B6 x) ln x + f (tc + dt_d),
// x = f^(1/3); v = c x with c = (pi M)^(1/3). The constants -phic/(2 pi) - 1/8
// and the ln c parts of the log terms are folded into A5 and A6.
struct PhaseCoef {
    double A[8];
    double B5, B6;
};

__device__ __forceinline__ void phase_coeffs(const Src& s, PhaseCoef& pc) {
    double phi[8], phil5, phil6;
    pn_coeffs(s.eta, s.delta, s.chis, s.chia, phi, phil5, phil6);
    const double c = cbrt(kPi * s.M * kTsun);
    const double lnc = log(c);
    const double k0 = 3.0 / (128.0 * s.eta) * kInvTwoPi;
    const double ic = 1.0 / c;
    double cp = ic * ic;
    cp = cp * cp * ic;  // c^-5
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        pc.A[j] = k0 * phi[j] * cp;
        cp *= c;
    }
    pc.A[5] += k0 * phil5 * lnc - s.phic * kInvTwoPi - 0.125;
    pc.A[6] += k0 * phil6 * c * lnc;
    pc.B5 = k0 * phil5;
    pc.B6 = k0 * phil6 * c;
}

// Phase in turns at one bin (shared by all detectors), FP64 Horner.
__device__ __forceinline__ double psi_turns(const double (&A)[8], double B5, double B6, double x, double xm5,
                                            double lnx) {
    double p = A[7];
    p = fma(p, x, A[6]);
    p = fma(p, x, A[5]);
    p = fma(p, x, A[4]);
    p = fma(p, x, A[3]);
    p = fma(p, x, A[2]);
    p = fma(p, x, A[1]);
    p = fma(p, x, A[0]);
    const double psi = p * xm5;
    return fma(fma(B6, x, B5), lnx, psi);
}

// ---------------------------------------------------------------------------
// FP64 sin/cos of 2 pi r for r in [0, 1): reduction to the nearest quarter
// turn (exact), then Taylor series of sin(2 pi t), cos(2 pi t) on |t| <= 1/8
// to orders 15 and 16 (truncation below 5e-17), then the quarter rotation.
// ---------------------------------------------------------------------------
struct TrigCoef {
    double s[8];
    double c[9];
};
constexpr TrigCoef make_trig() {
    TrigCoef t{};
    double term = 1.0;  // (2 pi)^n / n!
    for (int n = 0; n <= 16; ++n) {
        if (n > 0) term *= kTwoPi / n;
        const double sgn = ((n / 2) % 2) ? -1.0 : 1.0;
        if (n % 2)
            t.s[n / 2] = sgn * term;
        else
            t.c[n / 2] = sgn * term;
    }
    return t;
}
constexpr TrigCoef kTrig = make_trig();

__device__ __forceinline__ void sincos_turns(double r, double& sn, double& cs) {
    const double q = rint(4.0 * r);
    const double t = fma(-0.25, q, r);
    const double t2 = t * t;
    double ps = kTrig.s[7];
#pragma unroll
    for (int i = 6; i >= 0; --i) ps = fma(ps, t2, kTrig.s[i]);
    ps *= t;
    double pc = kTrig.c[8];
#pragma unroll
    for (int i = 7; i >= 0; --i) pc = fma(pc, t2, kTrig.c[i]);
    const int iq = ((int)q) & 3;
    const double ss = (iq & 1) ? pc : ps;
    const double cc = (iq & 1) ? ps : pc;
    sn = (iq & 2) ? -ss : ss;
    cs = ((iq + 1) & 2) ? -cc : cc;
}

__device__ __forceinline__ double fract64(double x) { return __builtin_amdgcn_fract(x); }

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) and 53-bit uniforms.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void philox4x32_10(uint32_t& c0, uint32_t& c1, uint32_t& c2, uint32_t& c3, uint32_t k0,
                                              uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // each 32 x 32 -> 64-bit product as one instruction (v_mad_u64_u32)
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0, p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
        const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
        const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

__device__ __forceinline__ double u53(uint32_t a, uint32_t b) {
    return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6) + 1.0) * 0x1p-53;
}

__device__ __forceinline__ void block_uniforms(uint64_t seed, uint32_t stream, uint64_t i, uint32_t j, double& ua,
                                               double& ub) {
    uint32_t c0 = (uint32_t)i, c1 = (uint32_t)(i >> 32), c2 = j, c3 = stream;
    philox4x32_10(c0, c1, c2, c3, (uint32_t)seed, (uint32_t)(seed >> 32));
    ua = u53(c0, c1);
    ub = u53(c2, c3);
}

// Coefficients of the two Bessel series below, so that their terms follow by
// products instead of divisions: 1/k^2 and 1/(k (k+1)) (power series, DLMF
// 10.25.2: the ratio of term k to term k-1 is (x^2/4)/k^2), and (2k-1)^2/(8k)
// and ((2k-1)^2 - 4)/(8k) (Hankel series of I0 and I1, DLMF 10.40.1, ratio to
// the previous term over x). Each is the correctly rounded quotient.
constexpr int kI0Pow = 400, kI0Hank = 64;
struct BesselTab {
    double ik2[kI0Pow];     // [k] = 1 / k^2 (k >= 1)
    double ikk1[kI0Pow];    // [k] = 1 / (k (k + 1))
    double h0[kI0Hank];     // [k] = (2k - 1)^2 / (8k)
    double h1[kI0Hank];     // [k] = ((2k - 1)^2 - 4) / (8k)
};
constexpr BesselTab make_bessel_tab() {
    BesselTab t{};
    for (int k = 1; k < kI0Pow; ++k) {
        t.ik2[k] = 1.0 / ((double)k * (double)k);
        t.ikk1[k] = 1.0 / ((double)k * (double)(k + 1));
    }
    for (int k = 1; k < kI0Hank; ++k) {
        const double m = (2.0 * k - 1.0) * (2.0 * k - 1.0);
        t.h0[k] = m / (8.0 * k);
        t.h1[k] = (m - 4.0) / (8.0 * k);
    }
    return t;
}
__constant__ constexpr BesselTab kBessel = make_bessel_tab();

// ln I0(x): power series (DLMF 10.25.2) below 30, Hankel asymptotic series
// (DLMF 10.40.1) above, where its smallest term is below e^-60.
__device__ __forceinline__ double log_i0(double x) {
    x = fabs(x);
    if (x < 30.0) {
        const double y = 0.25 * x * x;
        double term = 1.0, sum = 1.0;
        for (int k = 1; k < kI0Pow; ++k) {
            term *= y * kBessel.ik2[k];
            sum += term;
            if (term < 1e-17 * sum) break;
        }
        return log(sum);
    }
    const double inv = 1.0 / x;
    double term = 1.0, sum = 1.0;
    for (int k = 1; k < kI0Hank; ++k) {
        const double tk = term * kBessel.h0[k] * inv;
        if (tk > term) break;
        term = tk;
        sum += term;
        if (term < 1e-17 * sum) break;
    }
    return x - 0.5 * log(kTwoPi * x) + log(sum);
}

// I1(y)/I0(y), y >= 0: ratio of the power series (DLMF 10.25.2) below 30, of
// the Hankel asymptotic series (DLMF 10.40.1) above.
__device__ __forceinline__ double i1_over_i0(double y) {
    if (y < 30.0) {
        const double q = 0.25 * y * y;
        double t0 = 1.0, s0 = 1.0, t1 = 1.0, s1 = 1.0;  // I0 = s0, I1 = (y/2) s1
        for (int k = 1; k < kI0Pow; ++k) {
            t0 *= q * kBessel.ik2[k];
            t1 *= q * kBessel.ikk1[k];
            s0 += t0;
            s1 += t1;
            if (t0 < 1e-17 * s0) break;
        }
        return 0.5 * y * s1 / s0;
    }
    const double inv = 1.0 / y;
    double t0 = 1.0, s0 = 1.0, t1 = 1.0, s1 = 1.0;
    for (int k = 1; k < kI0Hank; ++k) {
        const double n0 = t0 * kBessel.h0[k] * inv, n1 = t1 * kBessel.h1[k] * inv;
        if (fabs(n0) > fabs(t0)) break;
        t0 = n0;
        t1 = n1;
        s0 += t0;
        s1 += t1;
        if (fabs(t0) < 1e-17 * s0 && fabs(t1) < 1e-17 * fabs(s1)) break;
    }
    return s1 / s0;
}

// ---------------------------------------------------------------------------
// Distance marginalisation: ln of int_1^inf 3 x^-4 exp(phi(x) - b x^2) dx with
// phi = a x (explicit phase) or ln I0(a x) (marginalised phase), x = dl_max/dL.
// The log-integrand g has at most one interior maximum and one minimum on
// (0, inf) (x g' is -4 + x phi' - 2 b x^2, with x phi' convex then linear).
// Its maximiser x+ solves 2 b x^2 - phi'(x) x + 4 = 0; for the marginalised
// phase phi' = a I1/I0(a x), iterated from phi' = a, which decreases
// monotonically to x+. From x+ the integral is walked outward in panels of
// 16-point Gauss-Legendre, each panel short enough that g changes by at most
// kDmDelta across it and that x changes by at most half, until g has fallen
// below kDmCut of its running maximum; a separate walk from x = 1 covers the
// boundary when g rises again toward it. Sums are scaled by the running
// maximum. The cost is ~10-25 panels per draw.
// ---------------------------------------------------------------------------
// 16-point Gauss-Legendre on [-1, 1]: positive nodes and their weights
// (csrc/gen_gauss_legendre.py).
constexpr double kGlX[8] = {0.9894009349916499, 0.9445750230732326, 0.8656312023878318, 0.755404408355003,
                            0.6178762444026438, 0.45801677765722737, 0.2816035507792589, 0.09501250983763744};
constexpr double kGlW[8] = {0.027152459411754058, 0.062253523938647776, 0.0951585116824929, 0.12462897125553395,
                            0.14959598881657682, 0.16915651939500256, 0.1826034150449236, 0.18945061045506847};
constexpr double kDmDelta = 8.0;   // largest change of ln(integrand) across a panel
constexpr double kDmCut = 45.0;    // walk ends below e^-45 of the maximum
constexpr int kDmMaxPanels = 400;  // per walk; reached only by non-finite input

// The light variant (Lite = true), for the many per-node integrals of the time
// marginal on the split path, whose tolerance is 1e-3 in ln L: ln I0 from the
// polynomial approximations of Abramowitz & Stegun 9.8.1 (x < 3.75) and 9.8.2
// (x >= 3.75), each within 2e-7 of I0 relative; 8-point Gauss-Legendre panels;
// the walk ends below e^-20 of the maximum; the maximiser to 1e-6. Measured
// against adaptive quadrature of the exact integrand over b in [0.05, 8000] and
// a up to 80 sqrt(b): within 5e-7 in ln, with a third of the evaluations.
constexpr double kGlX8[4] = {0.9602898564975363, 0.7966664774136268, 0.525532409916329, 0.1834346424956498};
constexpr double kGlW8[4] = {0.10122853629037618, 0.22238103445337445, 0.3137066458778874, 0.362683783378362};
constexpr double kDmCutLite = 20.0;

__device__ __forceinline__ double log_i0_poly(double x) {
    x = fabs(x);
    if (x < 3.75) {
        const double t = (x / 3.75) * (x / 3.75);
        const double p =
            1.0 + t * (3.5156229 + t * (3.0899424 + t * (1.2067492 + t * (0.2659732 + t * (0.0360768 + t * 0.0045813)))));
        return log(p);
    }
    const double t = 3.75 / x;
    const double p =
        0.39894228 +
        t * (0.01328592 +
             t * (0.00225319 +
                  t * (-0.00157565 +
                       t * (0.00916281 + t * (-0.02057706 + t * (0.02635537 + t * (-0.01647633 + t * 0.00392377)))))));
    return x - 0.5 * log(x) + log(p);
}

// NL lanes (consecutive, NL a power of two) may share one draw: lane `sub`
// evaluates the nodes sub, sub + NL, ... of every panel, while all of them walk
// the same panels, decided from values that every lane computes alike (the
// panel end points and the starting points); at the end their scaled sums are
// combined by a butterfly of NL shuffles in a fixed order.
struct DmState {
    double a, b;
    bool ex;
    double G, S;  // this lane's running maximum of ln(integrand); its sum scaled by exp(-G)
    double W;     // the walk's reference maximum (end points only; equal on every lane)
};

template <bool Lite = false>
__device__ __forceinline__ double dm_g(const DmState& q, double x) {
    const double phi = q.ex ? q.a * x : (Lite ? log_i0_poly(q.a * x) : log_i0(q.a * x));
    return 1.0986122886681098 - 4.0 * log(x) + phi - q.b * x * x;  // ln 3 - 4 ln x + ...
}

template <int NL, bool Lite = false>
__device__ __forceinline__ void dm_panel(DmState& q, double lo, double hi, int sub) {
    const double c = 0.5 * (lo + hi), h = 0.5 * (hi - lo);
    constexpr int NP = Lite ? 8 : 16;
#pragma unroll 1
    for (int k = sub; k < NP; k += NL) {
        const int r = k < NP / 2 ? k : k - NP / 2;
        const double x = Lite ? kGlX8[r] : kGlX[r];
        const double t = (k < NP / 2) ? -x : x;
        const double v = dm_g<Lite>(q, c + h * t);
        if (v > q.G) {
            q.S *= exp(q.G - v);
            q.G = v;
        }
        q.S += h * (Lite ? kGlW8[r] : kGlW[r]) * exp(v - q.G);
    }
}

// Walk from x0 (where g = g0) in direction dir until g falls below the cut
// (while decreasing) or x reaches stop; returns the last x.
template <int NL, bool Lite = false>
__device__ __forceinline__ double dm_walk(DmState& q, double x0, double g0, int dir, double stop, double w,
                                          int sub) {
    constexpr double cut = Lite ? kDmCutLite : kDmCut;
#pragma unroll 1
    for (int p = 0; p < kDmMaxPanels; ++p) {
        double x1 = x0, g1 = g0;
#pragma unroll 1
        for (int h = 0; h < 64; ++h) {
            if (dir > 0) {
                w = fmin(w, 0.5 * x0);
                x1 = fmin(x0 + w, stop);
            } else {
                w = fmin(w, x0 / 3.0);
                x1 = fmax(x0 - w, stop);
            }
            g1 = dm_g<Lite>(q, x1);
            if (fabs(g1 - g0) <= kDmDelta) break;
            w *= 0.5;
        }
        dm_panel<NL, Lite>(q, fmin(x0, x1), fmax(x0, x1), sub);
        q.W = fmax(q.W, g1);
        if (x1 == stop) return x1;
        if (g1 < q.W - cut && g1 < g0) return x1;
        x0 = x1;
        g0 = g1;
        w *= 2.0;
    }
    return x0;
}

template <int NL, bool Lite = false>
__device__ __forceinline__ double log_dist_marg(double a, double b, bool ex, int sub) {
    if (!(b > 0.0)) return (a == 0.0) ? 0.0 : NAN;  // H = 0 only with Z = 0 (no bins below the cut)
    DmState q{a, b, ex, -INFINITY, 0.0, -INFINITY};
    double xs = 1.0, ae = a;
#pragma unroll 1
    for (int it = 0; it < 64; ++it) {
        const double disc = ae * ae - 32.0 * b;
        if (!(ae > 0.0) || disc < 0.0) {  // g' < 0 on [1, inf): the maximum is at x = 1
            xs = 1.0;
            break;
        }
        const double xn = fmax(1.0, (ae + sqrt(disc)) / (4.0 * b));
        const bool done = ex || xn == 1.0 || fabs(xn - xs) <= (Lite ? 1e-6 : 1e-14) * xn;
        xs = xn;
        if (done) break;
        ae = a * i1_over_i0(a * xs);
    }
    const double g1 = dm_g<Lite>(q, 1.0);
    const double gs = (xs > 1.0) ? dm_g<Lite>(q, xs) : g1;
    q.W = fmax(g1, gs);
    q.G = q.W;
    const double w0 = fmin(1.0 / sqrt(2.0 * b), 0.5 * xs);
    dm_walk<NL, Lite>(q, xs, gs, +1, INFINITY, w0, sub);
    double xl = 1.0;
    if (xs > 1.0) xl = dm_walk<NL, Lite>(q, xs, gs, -1, 1.0, w0, sub);
    if (xl > 1.0 && g1 >= q.W - (Lite ? kDmCutLite : kDmCut)) dm_walk<NL, Lite>(q, 1.0, g1, +1, xl, w0, sub);
    double G = q.G, S = q.S;
#pragma unroll
    for (int o = 1; o < NL; o <<= 1) {
        const double Go = __shfl_xor(G, o), So = __shfl_xor(S, o);
        const double Gm = fmax(G, Go);
        S = S * exp(G - Gm) + So * exp(Go - Gm);
        G = Gm;
    }
    return G + log(S);
}

// ln L from Z and H (Eq. 3): explicit phase Re Z - H/2, marginalised phase
// ln I0(|Z|) - H/2.
__device__ __forceinline__ double loglike_phase(const EvConst& ev, double zr, double zi, double h) {
    return (ev.phase == PE_PHASE_EXPLICIT) ? zr - 0.5 * h : log_i0(hypot(zr, zi)) - 0.5 * h;
}

// The same, or for distance-marginalised events (Z, H at dl_max) the integral
// over the distance prior.
// NL lanes share the draw (see log_dist_marg); every one of them returns ln L.
template <int NL>
__device__ __forceinline__ double loglike_of(const EvConst& ev, double zr, double zi, double h, int sub) {
    const bool ex = (ev.phase == PE_PHASE_EXPLICIT);
    if (ev.dist) return log_dist_marg<NL>(ex ? zr : hypot(zr, zi), 0.5 * h, ex, sub);
    return loglike_phase(ev, zr, zi, h);
}

// Loads from read-only device memory. The hot loop reaches its tables through
// pointers held in device memory, so the compiler cannot prove on its own that
// the kernel's stores leave them unchanged; the constant address space says so
// and lets wave-uniform loads go through the scalar unit (s_load). Records are
// copied as 32-bit words, which the compiler merges into wide scalar loads.
typedef const __attribute__((address_space(4))) uint32_t* cwords;
typedef const __attribute__((address_space(1))) double* gdoubles;
typedef const __attribute__((address_space(1))) int* gints;

template <typename T>
__device__ __forceinline__ T load_const(const T* p) {
    static_assert(sizeof(T) % 4 == 0, "record size must be a multiple of 4 bytes");
    const cwords w = (cwords)p;
    uint32_t buf[sizeof(T) / 4];
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 4); ++i) buf[i] = w[i];
    T r;
    __builtin_memcpy(&r, buf, sizeof(T));
    return r;
}

}  // namespace pe
