"""Pins of the oracle's waveform metric (the Fisher form of the metric induced by the inner
product, Sec. II.A) against closed-form columns and against the Hessian of the zero-noise
log-likelihood (Eq. 3): at d = h(theta0), -d2 ln L / dtheta_i dtheta_j = g_ij exactly."""
import math

import numpy as np
import pytest

import oracle
from events import build_event
from paper_2410_05190_amd import synth


def _sums(b, h):
    f = synth.frequencies(b.f_lo, b.df, b.n_bins)
    S = b.psd.astype(np.float64)
    a2 = (np.abs(h) ** 2) / S * 4 * b.df
    return a2.sum(), (a2 * f).sum(), (a2 * f * f).sum()


@pytest.mark.parametrize("event", [0, 2])
def test_metric_closed_form_columns_11d(event):
    b = build_event(1, event, n_bins=20000)
    g = b.ev.metric(b.theta_inj, flags=3)
    h = b.ev.waveform(b.theta_inj)
    s0, s1, s2 = _sums(b, h)
    assert np.allclose(g, g.T, rtol=0, atol=1e-12 * np.abs(g).max())
    assert g[10, 10] == pytest.approx(s0, rel=1e-12)                       # phic: rho^2
    assert g[9, 9] == pytest.approx((2 * math.pi) ** 2 * s2, rel=1e-6)     # tc
    assert g[9, 10] == pytest.approx(-2 * math.pi * s1, rel=1e-6)         # tc-phic
    assert g[8, 8] == pytest.approx(s0 / b.theta_inj[8] ** 2, rel=1e-6)   # dL: amplitude 1/dL
    assert g[8, 10] == pytest.approx(0.0, abs=1e-9 * math.sqrt(g[8, 8] * g[10, 10]))
    assert np.all(np.linalg.eigvalsh(g / np.sqrt(np.outer(np.diag(g), np.diag(g)))) > -1e-9)


def test_metric_closed_form_4d_raw():
    b = build_event(0, 0, n_bins=12000)
    g = b.ev.metric(b.theta_inj, flags=2)
    assert g.shape == (5, 5)
    h = b.ev.waveform(b.theta_inj)
    s0, s1, s2 = _sums(b, h)
    assert g[4, 4] == pytest.approx(s0, rel=1e-12)
    assert g[3, 3] == pytest.approx((2 * math.pi) ** 2 * s2, rel=1e-6)
    assert g[3, 4] == pytest.approx(-2 * math.pi * s1, rel=1e-6)


def _hessian(fun, x0, steps):
    D = len(x0)
    pts = [x0.copy()]
    index = {}

    def add(key, x):
        index[key] = len(pts)
        pts.append(x)

    for i in range(D):
        for si in (1, -1):
            x = x0.copy()
            x[i] += si * steps[i]
            add((i, si), x)
        for j in range(i + 1, D):
            for si in (1, -1):
                for sj in (1, -1):
                    x = x0.copy()
                    x[i] += si * steps[i]
                    x[j] += sj * steps[j]
                    add((i, si, j, sj), x)
    vals = fun(np.array(pts).T)
    f0 = vals[0]
    H = np.zeros((D, D))
    for i in range(D):
        H[i, i] = (vals[index[(i, 1)]] - 2 * f0 + vals[index[(i, -1)]]) / steps[i] ** 2
        for j in range(i + 1, D):
            H[i, j] = H[j, i] = (vals[index[(i, 1, j, 1)]] - vals[index[(i, 1, j, -1)]]
                                 - vals[index[(i, -1, j, 1)]] + vals[index[(i, -1, j, -1)]]) / (4 * steps[i] * steps[j])
    return H


def _band_limited_event(params, phase, n_det, snr=20.0):
    """Zero-noise event whose band (20-320 Hz) lies below the ISCO of every nearby draw, so the
    cut does not move under the finite differences."""
    cfg = 1 if params == oracle.PARAMS_11D else 0
    f_lo, df, K = 20.0, 0.125, 2400
    f = synth.frequencies(f_lo, df, K)
    S = np.tile(synth.psd_analytic(f), (n_det, 1))
    geom = synth.detectors(1, n_det)
    inj = synth.injection(cfg, 3)
    th = inj["theta"].copy()
    common = dict(params=params, phase=phase, chi_max=0.4, dl_max=1e4, det_geom=geom)
    ref = oracle.Event(n_det, K, f_lo, df, psd=S, amp0=1.0, **common)
    h1 = ref.waveform(th)
    rho1 = math.sqrt(sum(ref.inner(d, h1, h1) for d in range(n_det)))
    amp0 = 0.0
    if params == oracle.PARAMS_4D:
        amp0 = snr / rho1
    else:
        th[8] = rho1 / snr
    tmp = oracle.Event(n_det, K, f_lo, df, psd=S, amp0=amp0, **common)
    h = tmp.waveform(th)
    ev = oracle.Event(n_det, K, f_lo, df, data=h, psd=S, amp0=amp0, **common)
    return ev, th


def test_metric_equals_loglike_hessian_11d():
    ev, th = _band_limited_event(oracle.PARAMS_11D, oracle.PHASE_EXPLICIT, 3)
    g = ev.metric(th, flags=3)
    steps = 0.03 / np.sqrt(np.diag(g))
    H = _hessian(ev.loglike, th, steps)
    norm = np.sqrt(np.outer(np.diag(g), np.diag(g)))
    assert np.max(np.abs(-H - g) / norm) < 1e-4


def test_projected_metric_equals_profile_hessian_4d():
    """Marginalised form: the phase-projected metric is the Hessian of the phase-maximised
    zero-noise log-likelihood |Z| - H/2 (a profile likelihood)."""
    ev, th = _band_limited_event(oracle.PARAMS_4D, oracle.PHASE_MARG, 1)
    g = ev.metric(th, flags=1)

    def prof(theta):
        _, zh = ev.loglike(theta, return_zh=True)
        return np.hypot(zh[:, 0], zh[:, 1]) - 0.5 * zh[:, 2]

    steps = 0.03 / np.sqrt(np.diag(g))
    H = _hessian(prof, th, steps)
    norm = np.sqrt(np.outer(np.diag(g), np.diag(g)))
    assert np.max(np.abs(-H - g) / norm) < 1e-4


def test_regularisation_is_prior_precision():
    b = build_event(1, 0, n_bins=4000)
    g0 = b.ev.metric(b.theta_inj, flags=1)
    g1 = b.ev.metric(b.theta_inj, flags=0)
    reg = np.diag(g1 - g0)
    pi = math.pi
    want = [0, 12, 12 / (4 * 0.16), 12 / (4 * 0.16), 12 / (4 * pi * pi), 12 / pi ** 2, 12 / pi ** 2,
            12 / pi ** 2, 12 / b.dl_max ** 2, 0, 12 / (4 * pi * pi)]
    np.testing.assert_allclose(reg, want, rtol=1e-9, atol=1e-12 * np.abs(np.diag(g0)).max())
    assert np.allclose(g1 - np.diag(np.diag(g1)), g0 - np.diag(np.diag(g0)), rtol=0, atol=0)


def test_fd_step_convergence():
    """Central differences converge as O(eps^2): halving the default steps changes g by far less
    than the metric's tolerance elsewhere (1e-6 relative)."""
    b = build_event(1, 1, n_bins=20000)
    st = b.ev.default_steps(b.theta_inj)
    g1 = b.ev.metric(b.theta_inj, steps=st, flags=3)
    g2 = b.ev.metric(b.theta_inj, steps=st / 2, flags=3)
    norm = np.sqrt(np.outer(np.diag(g1), np.diag(g1)))
    assert np.max(np.abs(g1 - g2) / norm) < 1e-6
