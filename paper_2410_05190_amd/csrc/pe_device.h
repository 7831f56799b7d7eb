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
        M = mc * pow(eta, -0.6);
        return (mc > 0.0) && (eta > 0.0) && (eta <= 0.25) && (fabs(chi) <= ev.chi_max);
    }
    const double mc = th[0], q = th[1], c1 = th[2], c2 = th[3];
    const double dec = th[5], iota = th[6], dl = th[8];
    const double opq = 1.0 + q;
    M = mc * pow(opq, 1.2) * pow(q, -0.6);
    return (mc > 0.0) && (q > 0.0) && (q <= 1.0) && (fabs(c1) <= ev.chi_max) && (fabs(c2) <= ev.chi_max) &&
           (fabs(dec) <= 0.5 * kPi) && (iota >= 0.0) && (iota <= kPi) && (dl > 0.0) && (dl <= ev.dl_max);
}

// Support of the prior and the source parameters of theta (D values).
// Log prior (flat in Mc, eta or q, spins, tc, ra, psi, phic; cos dec; sin
// iota; dL^2; unnormalised), -inf outside the support.
__device__ __forceinline__ double log_prior_of(const EvConst& ev, const double* th) {
    double M;
    if (!mass_and_support(ev, th, M)) return -INFINITY;
    return (ev.params == PE_PARAMS_4D) ? 0.0 : log(cos(th[5])) + log(sin(th[6])) + 2.0 * log(th[8]);
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
        const double amp =
            kAmpNewt * pow(mc * kTsun, 5.0 / 6.0) / (dl * (kMpc / kC)) * ev.scale;
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
        const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
        const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
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

// ln I0(x): power series (DLMF 10.25.2) below 30, Hankel asymptotic series
// (DLMF 10.40.1) above, where its smallest term is below e^-60.
__device__ __forceinline__ double log_i0(double x) {
    x = fabs(x);
    if (x < 30.0) {
        const double y = 0.25 * x * x;
        double term = 1.0, sum = 1.0;
        for (int k = 1; k < 400; ++k) {
            term *= y / ((double)k * (double)k);
            sum += term;
            if (term < 1e-17 * sum) break;
        }
        return log(sum);
    }
    const double inv = 1.0 / x;
    double term = 1.0, sum = 1.0;
    for (int k = 1; k < 64; ++k) {
        const double tk = term * (2.0 * k - 1.0) * (2.0 * k - 1.0) / (8.0 * k) * inv;
        if (tk > term) break;
        term = tk;
        sum += term;
        if (term < 1e-17 * sum) break;
    }
    return x - 0.5 * log(kTwoPi * x) + log(sum);
}

}  // namespace pe
