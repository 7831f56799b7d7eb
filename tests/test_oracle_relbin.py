"""Pins of the oracle's relative-binning likelihood (Zackay, Dai & Venumadhav 2018; the paper
lists such reduced representations among the ways to speed the likelihood up, Sec. I): the bin
edges against the envelope rule, limits where the linear model of h/h0 is exact (the fiducial
itself, a constant phase offset, one bin per grid point), the interpolation bound for a pure time
shift, and the accuracy on draws from the proposal."""
import math

import numpy as np
import pytest

import oracle
from events import build_event


def _envelope(f, f_lo, f_hi):
    e = 0.0
    for a in (-5 / 3, -2 / 3, 1.0, 5 / 3, 7 / 3):
        e += (-1.0 if a < 0 else 1.0) * (f / (f_lo if a < 0 else f_hi)) ** a
    return 2 * math.pi * e


def test_edges_follow_the_envelope_rule():
    b = build_event(0, 0)
    ev = b.ev
    eps = 0.05
    e = ev.relbin_edges(eps)
    K = b.n_bins
    assert e[0] == 0 and e[-1] == K and np.all(np.diff(e) > 0)
    f_hi = b.f_lo + K * b.df
    E = np.array([_envelope(b.f_lo + k * b.df, b.f_lo, f_hi) for k in range(K)])
    inner = e[1:-1]
    prev = e[:-2]
    # each inner edge is the first grid point where the envelope has grown by eps since the previous
    assert np.all(E[inner] - E[prev] >= eps * (1 - 1e-12))
    assert np.all(E[inner - 1] - E[prev] < eps * (1 + 1e-12))
    with pytest.raises(ValueError):
        ev.relbin_edges(eps, max_edges=10)


@pytest.mark.parametrize("cfg", [0, 1])
def test_fiducial_point_is_exact(cfg):
    b = build_event(cfg, 1, n_bins=20000)
    ev = b.ev
    e = ev.relbin_edges(0.05)
    ll, zh = ev.relbin_loglike(b.theta_inj, e, b.theta_inj[:, None], return_zh=True)
    lo, zo = ev.loglike(b.theta_inj[:, None], return_zh=True)
    np.testing.assert_allclose(zh, zo, rtol=1e-11, atol=1e-9)


def test_one_bin_per_grid_point_is_exact_for_any_draw():
    b = build_event(1, 2, n_bins=6000)
    ev = b.ev
    e = ev.relbin_edges(0.0)
    assert len(e) == b.n_bins + 1
    g = ev.metric(b.theta_inj)
    rc, th, lq, lp = ev.draw(b.theta_inj, g, 4, 0, 40)
    ll, zh = ev.relbin_loglike(b.theta_inj, e, th, return_zh=True)
    lo, zo = ev.loglike(th, return_zh=True)
    f = np.isfinite(lo)
    assert np.array_equal(np.isfinite(ll), f)
    np.testing.assert_allclose(zh[f], zo[f], rtol=1e-10, atol=1e-8)


def test_constant_phase_offset_is_exact():
    # explicit-phase 11-D event: a draw that differs from the fiducial only in phic has h/h0 constant
    b = build_event(1, 3, n_bins=20000)
    ev = b.ev
    e = ev.relbin_edges(0.3)
    th = np.repeat(b.theta_inj[:, None], 3, axis=1)
    th[10] = [0.3, 2.0, 5.5]
    ll, zh = ev.relbin_loglike(b.theta_inj, e, th, return_zh=True)
    lo, zo = ev.loglike(th, return_zh=True)
    np.testing.assert_allclose(zh, zo, rtol=1e-11, atol=1e-8)


def test_time_shift_within_the_interpolation_bound():
    # h/h0 = exp(-2 pi i f dt): linear interpolation over a bin of width B errs by at most
    # B^2/8 (2 pi dt)^2 in modulus, so |Z_rb - Z| <= |R| sum_b B_b^2/8 (2 pi dt)^2 sum_{k in b} |c_k|
    b = build_event(0, 0)
    ev = b.ev
    e = ev.relbin_edges(0.1)
    f = b.f_lo + np.arange(b.n_bins) * b.df
    d = b.data[0].astype(np.complex128)
    S = b.psd[0].astype(np.float64)
    absc = 4 * b.df * np.abs(d) * f ** (-7 / 6) / S
    R = b.amp0 * b.strain_scale
    for dt in (2e-5, 1e-4, 4e-4):
        th = b.theta_inj.copy()
        th[3] += dt
        ll, zh = ev.relbin_loglike(b.theta_inj, e, th[:, None], return_zh=True)
        lo, zo = ev.loglike(th[:, None], return_zh=True)
        bound = 0.0
        for j in range(len(e) - 1):
            k0, k1 = e[j], e[j + 1]
            B = (k1 - k0) * b.df
            bound += B * B / 8 * (2 * math.pi * dt) ** 2 * absc[k0:k1].sum()
        err = abs(complex(*zh[0, :2]) - complex(*zo[0, :2]))
        assert err <= abs(R) * bound * (1 + 1e-9) + 1e-9
        assert err > 0.0


def test_accuracy_on_proposal_draws():
    for cfg, nb, tol in ((0, None, 2e-2), (1, 60000, 1e-1)):
        b = build_event(cfg, 0, n_bins=nb)
        ev = b.ev
        e = ev.relbin_edges(0.03)
        g = ev.metric(b.theta_inj)
        rc, th, lq, lp = ev.draw(b.theta_inj, g, 3, 0, 200)
        ll = ev.relbin_loglike(b.theta_inj, e, th)
        lo = ev.loglike(th, n_threads=8)
        f = np.isfinite(lo)
        assert np.array_equal(np.isfinite(ll), f)
        assert np.abs(ll[f] - lo[f]).max() < tol
