"""Pins of the oracle's inner product (Sec. II.A, Eq. 1), log-likelihood (Eq. 2-3),
ISCO cut and noise model against closed forms, quadrature and statistics."""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle
from events import build_event
from paper_2410_05190_amd import synth

mpmath = pytest.importorskip("mpmath")


def _ev4(K, f_lo, df, S, amp0=1.0):
    psd = np.full((1, K), S) if np.isscalar(S) else np.asarray(S).reshape(1, K)
    return oracle.Event(1, K, f_lo, df, data=None, psd=psd, strain_scale=1.0, params=oracle.PARAMS_4D,
                        phase=oracle.PHASE_MARG, amp0=amp0, chi_max=0.4)


@pytest.mark.parametrize("K,mc,eta", [(4000, 1.2, 0.24), (30000, 1.3, 0.2), (3000, 8.0, 0.2)])
def test_hh_constant_psd_is_hurwitz_zeta(K, mc, eta):
    """(h|h) with S = S0 and |h| = A f^-7/6 on f_k = df (a + k), k < kcut:
    4 df A^2 / S0 sum_k f_k^-7/3 = 4 A^2 df^(-4/3) / S0 [zeta(7/3, a) - zeta(7/3, a + kcut)]."""
    f_lo, df, S0, A = 20.0, 1.0 / 16.0, 3e-48, 2e-22
    ev = _ev4(K, f_lo, df, S0, amp0=A)
    th = np.array([mc, eta, 0.0, 0.0])
    h = ev.waveform(th)
    ok, src = ev.source(th)
    kc = ev.kcut(src.fisco)
    hh = ev.inner(0, h, h)
    a = mpmath.mpf(f_lo) / mpmath.mpf(df)
    want = 4 * mpmath.mpf(A) ** 2 * mpmath.mpf(df) ** (-mpmath.mpf(4) / 3) / mpmath.mpf(S0) * (
        mpmath.zeta(mpmath.mpf(7) / 3, a) - mpmath.zeta(mpmath.mpf(7) / 3, a + kc))
    assert hh == pytest.approx(float(want), rel=1e-12)


def test_hh_config_psd_matches_snr_integral():
    """Left-point sum vs the continuous SNR integral with the Euler-Maclaurin corrections
    sum_{k<n} h g(a + k h) = int_a^b g - h/2 (g(b) - g(a)) + h^2/12 (g'(b) - g'(a)) + O(h^4)."""
    f_lo, df, K = 40.0, 1.0 / 32.0, 31488
    f = synth.frequencies(f_lo, df, K)
    S = synth.psd_analytic(f)
    A = 3e-22
    ev = _ev4(K, f_lo, df, S, amp0=A)
    th = np.array([1.25, 0.245, 0.0, 0.0])
    h = ev.waveform(th)
    hh = ev.inner(0, h, h)
    ok, src = ev.source(th)
    b = f_lo + ev.kcut(src.fisco) * df

    def g(x):
        return 4.0 * A * A * x ** (-7.0 / 3.0) / synth.psd_analytic(x)

    def gp(x, e=1e-4):
        return (g(x + e) - g(x - e)) / (2 * e)

    edges = np.geomspace(f_lo, b, 40)
    integral = sum(integrate.quad(g, lo, hi, epsabs=0, epsrel=1e-13, limit=200)[0]
                   for lo, hi in zip(edges[:-1], edges[1:]))
    em = integral - df / 2 * (g(b) - g(f_lo)) + df * df / 12 * (gp(b) - gp(f_lo))
    assert hh == pytest.approx(em, rel=1e-10)
    # without the correction terms the sum is off by far more than the tolerance
    assert abs(hh - integral) / hh > 1e-6


def test_fisco_is_kepler_frequency_at_6M():
    """GW frequency = 2 x orbital frequency; Schwarzschild ISCO at r = 6 G M / c^2, Kepler's law."""
    GM = 1.32712440018e20
    c = oracle.c_si()
    for M in (1.0, 2.8, 20.0, 80.0):
        r = 6 * GM * M / c ** 2
        f_orb = math.sqrt(GM * M / r ** 3) / (2 * math.pi)
        assert oracle.f_isco(M) == pytest.approx(2 * f_orb, rel=1e-13)


def test_kcut_brute_force():
    f_lo, df, K = 20.0, 1.0 / 256.0, 519168
    ev = oracle.Event(1, K, f_lo, df)
    rng = np.random.default_rng(1)
    for fisco in list(rng.uniform(10, 2100, 40)) + [20.0, 20.0 + df, 1000.0, 2048.0, 2048.0 - df, 5.0]:
        want = int(np.count_nonzero(f_lo + np.arange(K) * df < fisco))
        assert ev.kcut(fisco) == want


def test_zero_noise_explicit_loglike_is_half_snr_squared():
    """d = h(theta_inj): ln L/L_n = (s|h) - (h|h)/2 = rho^2/2 at the injection (Eq. 3)."""
    b = build_event(1, 0, n_bins=40000, zero_noise=True, storage="f64")
    ll, zh = b.ev.loglike(b.theta_inj[:, None], return_zh=True)
    assert zh[0, 2] == pytest.approx(b.snr ** 2, rel=1e-12)
    assert ll[0] == pytest.approx(b.snr ** 2 / 2, rel=1e-12)
    assert zh[0, 0] == pytest.approx(b.snr ** 2, rel=1e-12)
    assert abs(zh[0, 1]) < 1e-9 * b.snr ** 2


def test_zero_noise_marginalised_loglike():
    b = build_event(0, 0, n_bins=8000, zero_noise=True)
    ll, zh = b.ev.loglike(b.theta_inj[:, None], return_zh=True)
    rho2 = b.snr ** 2
    assert zh[0, 2] == pytest.approx(rho2, rel=1e-12)
    assert math.hypot(zh[0, 0], zh[0, 1]) == pytest.approx(rho2, rel=1e-12)
    want = float(mpmath.log(mpmath.besseli(0, rho2))) - rho2 / 2
    assert ll[0] == pytest.approx(want, rel=1e-12)


def test_marginalisation_is_phase_average():
    """ln L_marg(theta) = ln (1/2pi) int exp(ln L_explicit(theta, phic)) dphic, by brute-force
    trapezoid over phic with the explicit-phase oracle (exponentially convergent)."""
    b = build_event(1, 1, n_bins=3000)
    d = b.desc()
    d.pop("phase")
    ev_m = oracle.Event(data=b.data, psd=b.psd, phase=oracle.PHASE_MARG, **d)
    M = 1024
    th = np.repeat(b.theta_inj[:, None], M, axis=1)
    th[0] *= 1.0 + 2e-5  # off the peak
    th[10] = 2 * np.pi * np.arange(M) / M
    lle = b.ev.loglike(th)
    mx = lle.max()
    brute = mx + math.log(np.mean(np.exp(lle - mx)))
    llm = ev_m.loglike(th[:, :1])[0]
    assert llm == pytest.approx(brute, abs=1e-10 * max(1.0, abs(brute)))


@pytest.mark.parametrize("x", [1e-8, 1e-3, 0.5, 2.0, 10.0, 29.9, 30.1, 100.0, 700.0, 1e3, 1e4, 1e5])
def test_log_i0_against_scipy(x):
    from scipy.special import i0e
    want = math.log(i0e(x)) + x
    assert oracle.log_i0(x) == pytest.approx(want, rel=1e-14, abs=1e-15)


def test_noise_statistics():
    """Across noise realisations (n|h) ~ N(0, rho^2) and (n|n) -> 2 per bin (Eq. 2 noise model)."""
    cfg = 0
    f_lo, df, _ = synth.grid(cfg)
    K = 2048
    f = synth.frequencies(f_lo, df, K)
    S = synth.psd_analytic(f)[None, :]
    ev = _ev4(K, f_lo, df, S[0], amp0=3e-22)
    h = ev.waveform(np.array([1.2, 0.24, 0.0, 0.0]))
    rho2 = ev.inner(0, h, h)
    nh, nn = [], []
    for e in range(400):
        n = synth.noise(cfg, 1000 + e, S, df)
        nh.append(ev.inner(0, n, h))
        nn.append(ev.inner(0, n, n) / K)
    nh = np.array(nh)
    nn = np.array(nn)
    N = len(nh)
    assert abs(nh.mean()) < 5 * math.sqrt(rho2 / N)
    assert abs(nh.var() / rho2 - 1) < 5 * math.sqrt(2.0 / N)
    assert abs(nn.mean() - 2.0) < 5 * 2.0 / math.sqrt(N * K)
