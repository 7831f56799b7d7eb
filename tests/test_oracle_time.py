"""Pins of the oracle's time-marginalised likelihood and its proposal.

The paper marginalises the extrinsic parameters (Sec. III). For the coalescence time with a flat prior
on [tc_lo, tc_hi], L_t = (1/T) int L(theta with tc = t) dt. The oracle evaluates Z(t) by shifting the
draw's integrand in time and integrates with Simpson's rule over the whole window. It is pinned by:
  - re-evaluating the sampled-tc likelihood with the waveform recomputed at every tc (a different code
    path) and integrating that with scipy's Simpson rule on a fine grid;
  - the narrow-window limit, which equals the sampled-tc likelihood at the window's centre;
  - data carrying nothing, where every node gives -H/2 and L_t = exp(-H/2) exactly;
  - the draws: tc is its conditional mean under the proposal given the other coordinates, and log q
    is the proposal's marginal over tc (the 11-D density integrated over tc by brute force).
"""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle
from events import build_event


def _tm_event(b, tc_lo, tc_hi, phase=None, data=True):
    kw = b.desc()
    if phase is not None:
        kw["phase"] = phase
    for k in ("n_det", "n_bins", "time_marg", "tc_lo", "tc_hi"):
        kw.pop(k)
    return oracle.Event(b.n_det, b.n_bins, data=b.data if data else np.zeros_like(b.data), psd=b.psd,
                        time_marg=1, tc_lo=tc_lo, tc_hi=tc_hi, **kw)


def _sampled_event(b, phase=None):
    kw = b.desc()
    if phase is not None:
        kw["phase"] = phase
    for k in ("n_det", "n_bins", "time_marg", "tc_lo", "tc_hi"):
        kw.pop(k)
    return oracle.Event(b.n_det, b.n_bins, data=b.data, psd=b.psd, **kw)


@pytest.mark.parametrize("phase", [oracle.PHASE_EXPLICIT, oracle.PHASE_MARG])
def test_time_integral_against_recomputed_waveforms(phase):
    """(1/T) int L dt from the oracle against Simpson's rule over 6001 sampled-tc likelihoods whose
    waveforms are recomputed at each tc."""
    b = build_event(1, 0, n_bins=3000)
    tinj = b.theta_inj[9]
    lo, hi = tinj - 1.5e-3, tinj + 1.5e-3
    ev_t = _tm_event(b, lo, hi, phase)
    ev_s = _sampled_event(b, phase)
    rng = np.random.default_rng(4)
    ths = np.repeat(b.theta_inj[:, None], 3, axis=1)
    ths[9] += rng.uniform(-3e-4, 3e-4, 3)  # centres off the peak: the integral does not depend on them
    ths[0] *= 1 + rng.normal(0, 2e-6, 3)
    got = ev_t.loglike(ths)
    ts = np.linspace(lo, hi, 6001)
    for i in range(3):
        grid = np.repeat(ths[:, i:i + 1], ts.size, axis=1)
        grid[9] = ts
        ll = ev_s.loglike(grid)
        m = ll.max()
        want = m + math.log(integrate.simpson(np.exp(ll - m), x=ts) / (hi - lo))
        assert got[i] == pytest.approx(want, abs=1e-8)


def test_narrow_window_is_the_sampled_likelihood():
    """A window of 1e-9 s about the draw's tc: L_t equals the sampled-tc likelihood there."""
    b = build_event(1, 1, n_bins=3000)
    th = b.theta_inj[:, None].copy()
    ev_s = _sampled_event(b)
    ev_t = _tm_event(b, th[9, 0] - 5e-10, th[9, 0] + 5e-10)
    assert ev_t.loglike(th)[0] == pytest.approx(ev_s.loglike(th)[0], abs=1e-8)


@pytest.mark.parametrize("phase", [oracle.PHASE_EXPLICIT, oracle.PHASE_MARG])
def test_no_data_gives_exp_minus_half_h(phase):
    """Data carrying nothing: Z(t) = 0 at every node, ln L_t = -H/2 exactly (ln I0(0) = 0)."""
    b = build_event(1, 2, n_bins=3000)
    ev_t = _tm_event(b, -0.002, 0.002, phase, data=False)
    th = b.theta_inj[:, None].copy()
    ll, zh = ev_t.loglike(th, return_zh=True)
    assert zh[0, 2] > 0
    assert ll[0] == pytest.approx(-0.5 * zh[0, 2], rel=1e-13)


def test_draws_centre_tc_and_marginal_logq():
    """Draws of a time-marginalised event: tc = theta0_tc - sum_j (g_tj / g_tt)(theta_j - theta0_j),
    and log q equals the 11-D proposal density integrated over tc (trapezoid over +-12 sd)."""
    b = build_event(1, 1, n_bins=3000)
    ev_t = _tm_event(b, -0.01, 0.01)
    ev_s = _sampled_event(b)
    g = ev_s.metric(b.theta_inj)
    th0 = b.theta_inj
    rc, th, lq, lp = ev_t.draw(th0, g, 17, 0, 40)
    assert rc == 0
    per = {4: 2 * math.pi, 7: math.pi, 10: 2 * math.pi}
    d = th - th0[:, None]
    for i, P in per.items():  # periodic offsets taken to the image nearest the centre
        d[i] = (d[i] + P / 2) % P - P / 2
    others = [a for a in range(11) if a != 9]
    want_tc = th0[9] - (g[9, others][:, None] * d[others]).sum(0) / g[9, 9]
    np.testing.assert_allclose(th[9], want_tc, rtol=0, atol=1e-12)
    sd = 1.0 / math.sqrt(np.linalg.inv(np.linalg.inv(g)[np.ix_([9], [9])])[0, 0])
    sd_t = math.sqrt(np.linalg.inv(g)[9, 9])
    nodes = np.linspace(-12 * sd_t, 12 * sd_t, 2401)
    vals = []
    for u in nodes:
        t = th.copy()
        t[9] = th0[9] + u
        rc, lf = ev_s.logq_theta(th0, g, t)
        vals.append(lf)
    vals = np.array(vals)
    m = vals.max(axis=0)
    want = m + np.log(np.trapezoid(np.exp(vals - m), x=nodes, axis=0))
    assert sd > 0
    np.testing.assert_allclose(lq, want, rtol=0, atol=1e-8)
