"""Pins of the oracle's distance-marginalised likelihood and of the proposal and prior that go with
it. The paper marginalises the extrinsic parameters with analytic or numerical formulas (Sec. III);
for the distance that is the integral of the likelihood over the dL^2 prior (Singer & Price 2016).

    L_D = int_0^dmax (3 dL^2 / dmax^3) L(dL) ddL = int_1^inf 3 x^-4 exp(phi(x) - b x^2) dx,

x = dmax/dL, phi = a x with a = Re Z (explicit phase) or ln I0(a x) with a = |Z| (marginalised
phase), Z and H taken at the reference distance dmax, b = H/2. Pinned against: the closed form
without signal (a = 0), mpmath quadrature, a brute-force integral of the oracle's own likelihood
re-evaluated at every distance, the textbook marginal of a Gaussian for the metric and the draws'
log q, and the prior with its distance factor removed."""
import math

import mpmath
import numpy as np
import pytest
from scipy import special

import oracle
from events import build_event


def _no_signal(b):
    """3 int_1^inf x^-4 e^{-b x^2} dx by the recurrence I_n = (e^{-b} - 2b I_{n-2}) / (n - 1) from
    integrating d/dx[x^{1-n} e^{-b x^2}] over [1, inf), with I_0 = sqrt(pi/b)/2 erfc(sqrt b)."""
    i0 = 0.5 * math.sqrt(math.pi / b) * special.erfc(math.sqrt(b))
    i2 = math.exp(-b) - 2 * b * i0
    i4 = (math.exp(-b) - 2 * b * i2) / 3
    return math.log(3 * i4)


@pytest.mark.parametrize("b", [0.05, 0.5, 2.0, 6.0])
@pytest.mark.parametrize("explicit", [True, False])
def test_closed_form_without_signal(b, explicit):
    assert oracle.log_dist_marg(0.0, b, explicit) == pytest.approx(_no_signal(b), abs=1e-12)


def test_no_data_no_template_is_the_prior_mass():
    # Z = H = 0 (a draw with no bin below its cut): L = 1 at every distance, L_D = 1
    assert abs(oracle.log_dist_marg(0.0, 0.0, True)) < 1e-13
    assert abs(oracle.log_dist_marg(0.0, 0.0, False)) < 1e-13


def _mp_reference(a, b, explicit):
    mpmath.mp.dps = 30
    a_, b_ = mpmath.mpf(a), mpmath.mpf(b)
    if explicit:
        phi = lambda x: a_ * x
        xs = float(a / (2 * b)) if a > 0 else 1.0
    else:
        phi = lambda x: mpmath.log(mpmath.besseli(0, a_ * x))
        xs = float(a / (2 * b))
    f = lambda x: 3 * x ** -4 * mpmath.exp(phi(x) - b_ * x * x)
    # breakpoints around the peak (width ~ 1/sqrt(2b) in x) so that the quadrature sees it
    w = 1.0 / math.sqrt(2 * b)
    pts = sorted({1.0} | {xs + k * w for k in range(-12, 13) if xs + k * w > 1.0})
    v = mpmath.quad(f, pts + [mpmath.inf])
    return float(mpmath.log(v))


@pytest.mark.parametrize("a,b,explicit", [
    (0.5, 0.02, True), (0.5, 0.02, False),      # weak: prior-dominated, heavy tail in x
    (-4.0, 3.0, True),                          # anti-correlated template
    (12.0, 8.0, True), (12.0, 8.0, False),      # peak near the upper distance bound
    (187.5, 28.1, True), (187.5, 28.1, False),  # network SNR ~25 at dL = 0.3 dmax
    (2.0e3, 1.0e3, False),                      # peak at x ~ 1: the boundary dL = dmax
    (9.0e4, 4.5e4, True),                       # matched-filter SNR 300
])
def test_against_mpmath(a, b, explicit):
    want = _mp_reference(a, b, explicit)
    got = oracle.log_dist_marg(a, b, explicit)
    assert got == pytest.approx(want, abs=1e-11 * max(1.0, abs(want)))


@pytest.mark.parametrize("cfg,explicit", [(1, True), (2, False)])
def test_brute_force_over_distance(cfg, explicit):
    """ln L_D of a draw equals ln of the prior-weighted integral, over dL, of the sampled-distance
    oracle's likelihood re-evaluated (waveform and all) at each distance: composite Simpson in
    u = ln(dmax/dL) on [0, 9], 9001 nodes. The dist-marginalised event ignores the draw's dL."""
    b = build_event(cfg, 1, n_bins=2500 if cfg == 1 else None)
    d = b.desc()
    d.pop("distance")
    ev_dm = oracle.Event(data=b.data, psd=b.psd, distance=oracle.DIST_MARG, **d)
    th = b.theta_inj.copy()
    th[0] *= 1.0 + 3e-5  # off the peak
    u = np.linspace(0.0, 9.0, 9001)
    thu = np.repeat(th[:, None], len(u), axis=1)
    thu[8] = b.dl_max * np.exp(-u)
    ll = b.ev.loglike(thu, n_threads=8)
    lf = math.log(3.0) - 3.0 * u + ll
    m = lf.max()
    h = u[1] - u[0]
    wts = np.ones(len(u))
    wts[1:-1:2] = 4.0
    wts[2:-1:2] = 2.0
    brute = m + math.log(h / 3.0 * np.sum(wts * np.exp(lf - m)))
    th_any = th.copy()
    th_any[8] = -7.0  # not a distance at all: unused by the marginalised likelihood
    got = ev_dm.loglike(np.stack([th, th_any], 1))
    assert got[0] == got[1]
    assert got[0] == pytest.approx(brute, abs=1e-8 * max(1.0, abs(brute)))
    assert explicit == (b.phase == oracle.PHASE_EXPLICIT)


def _gauss_marginal(g, keep):
    """Precision of the marginal of N(., g^-1) over the coordinates `keep` (textbook: invert the
    covariance's sub-block), in 50-digit arithmetic: the unregularised 11-D Fisher matrix has a
    condition number near 1e18."""
    mpmath.mp.dps = 50
    C = mpmath.inverse(mpmath.matrix(g.tolist()))
    sub = mpmath.matrix([[C[i, j] for j in keep] for i in keep])
    P = mpmath.inverse(sub)
    return np.array([[float(P[i, j]) for j in range(len(keep))] for i in range(len(keep))])


@pytest.mark.parametrize("cfg", [1, 2])
def test_metric_projects_out_distance(cfg):
    b = build_event(cfg, 2, n_bins=4000 if cfg == 1 else None)
    d = b.desc()
    d.pop("distance")
    ev_dm = oracle.Event(data=b.data, psd=b.psd, distance=oracle.DIST_MARG, **d)
    gs = b.ev.metric(b.theta_inj, flags=1)
    gd = ev_dm.metric(b.theta_inj, flags=1)
    phase_out = b.phase == oracle.PHASE_MARG
    keep = [i for i in range(11) if i != 8 and not (phase_out and i == 10)]
    np.testing.assert_allclose(gd[np.ix_(keep, keep)], _gauss_marginal(gs[np.ix_(keep + [8], keep + [8])],
                                                                         list(range(len(keep)))),
                               rtol=1e-8, atol=1e-10 * np.abs(gd).max())
    assert np.all(gd[8] == 0.0) and np.all(gd[:, 8] == 0.0)
    # regularised: only the prior precision 12/dmax^2 remains in the distance row
    gr = ev_dm.metric(b.theta_inj)
    assert gr[8, 8] == pytest.approx(12.0 / b.dl_max ** 2, rel=1e-15)
    assert np.count_nonzero(gr[8]) == 1


def test_draws_have_the_marginal_proposal_density():
    """log q of a draw of a distance-marginalised event is the log of the proposal's marginal
    density over the other ten coordinates: brute force, the sampled event's 11-D wrapped density
    integrated over dL (trapezoid over +-14 sigma), for a metric with distance cross terms."""
    b = build_event(1, 3, n_bins=4000)
    d = b.desc()
    d.pop("distance")
    ev_dm = oracle.Event(data=b.data, psd=b.psd, distance=oracle.DIST_MARG, **d)
    g = b.ev.metric(b.theta_inj)  # full metric: dL correlated with iota and the masses
    assert abs(g[8, 6]) > 0
    rc, th, lq, lp = ev_dm.draw(b.theta_inj, g, 11, 0, 6)
    assert rc == 0
    sig = 1.0 / math.sqrt(np.linalg.inv(np.linalg.inv(g)[8:9, 8:9])[0, 0])  # marginal sd of dL
    for i in range(th.shape[1]):
        t = np.linspace(-14 * sig, 14 * sig, 4001)
        tt = np.repeat(th[:, i:i + 1], len(t), axis=1)
        tt[8] = b.theta_inj[8] + t
        lfull = b.ev.logq_theta(b.theta_inj, g, tt)[1]
        m = lfull.max()
        brute = m + math.log(np.trapezoid(np.exp(lfull - m), t))
        assert lq[i] == pytest.approx(brute, abs=1e-9)
    np.testing.assert_allclose(ev_dm.logq_theta(b.theta_inj, g, th)[1], lq, rtol=0, atol=1e-12)


def test_decoupled_metric_leaves_the_other_coordinates_unchanged():
    """With the event's own (dL-decoupled) metric, a distance-marginalised draw and a sampled-
    distance draw from the same generator agree in every coordinate but none differ at all."""
    b = build_event(1, 4, n_bins=4000)
    d = b.desc()
    d.pop("distance")
    ev_dm = oracle.Event(data=b.data, psd=b.psd, distance=oracle.DIST_MARG, **d)
    g = ev_dm.metric(b.theta_inj)
    rc1, th1, lq1, lp1 = ev_dm.draw(b.theta_inj, g, 5, 2, 50)
    rc2, th2, lq2, lp2 = b.ev.draw(b.theta_inj, g, 5, 2, 50)
    np.testing.assert_array_equal(th1, th2)
    # the sampled event's log q carries the dL factor N(dL; dL0, 1/g_88) on top of the marginal
    ldl = -0.5 * g[8, 8] * (th2[8] - b.theta_inj[8]) ** 2 + 0.5 * math.log(g[8, 8] / (2 * math.pi))
    # (the marginal's route inverts the metric twice: rounding ~1e-11 relative at its conditioning)
    np.testing.assert_allclose(lq2 - ldl, lq1, rtol=0, atol=2e-9)


def test_prior_drops_the_distance_factor():
    b = build_event(1, 0, n_bins=2000)
    d = b.desc()
    d.pop("distance")
    ev_dm = oracle.Event(data=b.data, psd=b.psd, distance=oracle.DIST_MARG, **d)
    th = b.theta_inj.copy()
    assert ev_dm.logprior(th) == pytest.approx(b.ev.logprior(th) - 2 * math.log(th[8]), abs=1e-14)
    for dl in (-3.0, 0.0, 2.0 * b.dl_max):
        th[8] = dl
        assert b.ev.logprior(th) == -math.inf
        assert math.isfinite(ev_dm.logprior(th))


def test_relbin_with_one_bin_per_point_is_exact():
    b = build_event(1, 2, n_bins=3000)
    d = b.desc()
    d.pop("distance")
    ev_dm = oracle.Event(data=b.data, psd=b.psd, distance=oracle.DIST_MARG, **d)
    e = ev_dm.relbin_edges(0.0)
    g = ev_dm.metric(b.theta_inj)
    rc, th, lq, lp = ev_dm.draw(b.theta_inj, g, 4, 0, 20)
    rb = ev_dm.relbin_loglike(b.theta_inj, e, th)
    ex = ev_dm.loglike(th)
    f = np.isfinite(ex)
    np.testing.assert_allclose(rb[f], ex[f], rtol=0, atol=1e-8 * np.abs(ex[f]).max())
