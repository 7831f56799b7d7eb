"""Pins of the oracle's tile-mixture proposal (Sec. II.A; App. A: template bank, tiling of the
prior volume, proposal): the slice sampler against its own geometry (whitening identity, ball
volume, uniform-ball moments), the stochastic bank against its packing and covering properties,
the tile assignment against brute force, the proposal draws against closed forms, sampling
frequencies and the importance-sampling identity, and the whole chain's efficiency."""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
from events import build_event


def _slice(b, radius, centre=None):
    g = b.ev.metric(b.theta_inj)
    L = np.linalg.cholesky(g)
    c = b.theta_inj if centre is None else centre
    return oracle.make_slice(c, L, radius), L, c


def _support4(th, chi_max):
    return (th[0] > 0) & (th[1] > 0) & (th[1] <= 0.25) & (np.abs(th[2]) <= chi_max)


def test_slice_candidates_follow_their_definition():
    b = build_event(0, 0)
    sl, L, c = _slice(b, 6.0)
    u = oracle.uniforms(9, 3, 200, 2).reshape(200, 4)  # two Philox blocks per candidate (D = 4)
    for i in range(200):
        ok, y, th = b.ev.slice_candidate(sl, 9, 3, i)
        assert np.array_equal(y, 6.0 * (2.0 * u[i, :4] - 1.0))
        np.testing.assert_allclose(L.T @ (th - c), y, rtol=0, atol=1e-9 * 6.0)
        assert ok == bool((y @ y <= 36.0) and _support4(th[:, None], b.chi_max)[0])


def test_slice_samples_are_uniform_in_the_ball():
    # a slice far from every support edge: all of the ball is kept, so the kept fraction is the
    # ball-to-cube volume ratio pi^2/32 (D = 4) and E|y|^2 = D R^2 / (D + 2)
    b = build_event(0, 0)
    centre = np.array([1.2, 0.2, 0.0, 0.0])
    sl, L, c = _slice(b, 0.5, centre)
    n = 400000
    y, th, lp = b.ev.slice_sample(sl, 21, 0, 0, n)
    k = y.shape[1]
    p = math.pi ** 2 / 32
    assert abs(k / n - p) < 5 * math.sqrt(p * (1 - p) / n)
    r2 = (y * y).sum(0)
    assert r2.max() <= 0.25
    assert abs(r2.mean() - 4 * 0.25 / 6) < 5 * r2.std() / math.sqrt(k)
    assert np.all(np.abs(y.mean(1)) < 5 * y.std(1) / math.sqrt(k))
    assert np.all(lp == 0.0)  # flat prior of the 4-D set inside the support
    # the samples are the kept candidates, in order
    y2, th2, _ = b.ev.slice_sample(sl, 21, 0, 0, 100)
    kept = [b.ev.slice_candidate(sl, 21, 0, i) for i in range(100)]
    ys = np.array([t[1] for t in kept if t[0]]).T
    assert np.array_equal(y2, ys)


def test_support_edges_cut_the_slice():
    b = build_event(0, 0)
    sl, L, c = _slice(b, 6.0)  # the injection's eta is close to 0.25: the ball crosses the edge
    y, th, lp = b.ev.slice_sample(sl, 4, 0, 0, 200000)
    assert np.all(_support4(th, b.chi_max))
    assert np.all((y * y).sum(0) <= 36.0)
    assert y.shape[1] < 0.97 * math.pi ** 2 / 32 * 200000


def test_bank_packing_and_covering():
    b = build_event(0, 0)
    sl, L, c = _slice(b, 4.0)
    r = 1.0
    ty, tth, used = b.ev.tile_bank(sl, r, 5, 1, 2048, 5000, 0.002, 500)
    m = ty.shape[1]
    assert 20 < m < 5000
    d2 = ((ty[:, :, None] - ty[:, None, :]) ** 2).sum(0)
    np.fill_diagonal(d2, np.inf)
    assert d2.min() >= r * r * (1 - 1e-12)
    # templates are kept candidates of the slice, their theta the slice's map of their y
    np.testing.assert_allclose(L.T @ (tth - c[:, None]), ty, rtol=0, atol=1e-9)
    # covering: every kept candidate consumed lies within r of some template
    y, th, _ = b.ev.slice_sample(sl, 5, 1, 0, used)
    dmin = np.sqrt(((y[:, :, None] - ty[:, None, :]) ** 2).sum(0).min(1))
    assert dmin.max() < r
    # and fresh samples of the slice are almost all covered (the bank stopped at 0.2% new)
    y2, _, _ = b.ev.slice_sample(sl, 5, 2, 0, 50000)
    dmin2 = np.sqrt(((y2[:, :, None] - ty[:, None, :]) ** 2).sum(0).min(1))
    assert (dmin2 >= r).mean() < 0.01
    # deterministic
    ty2, _, used2 = b.ev.tile_bank(sl, r, 5, 1, 2048, 5000, 0.002, 500)
    assert np.array_equal(ty, ty2) and used == used2


def test_assignment_is_the_nearest_template():
    rng = np.random.default_rng(7)
    ty = rng.normal(0, 2, (4, 300))
    y = rng.normal(0, 2, (4, 20000))
    got = oracle.tile_assign(ty, y)
    d2 = ((y[:, :, None] - ty[:, None, :]) ** 2).sum(0)
    want = d2.argmin(1)
    diff = np.flatnonzero(got != want)
    # different summation order may only flip exact or near ties
    for s in diff:
        assert abs(d2[s, got[s]] - d2[s, want[s]]) <= 1e-12 * d2[s, want[s]]
    assert len(diff) <= 2
    # exact ties go to the lowest index
    t2 = np.array([[0.0, 2.0, -2.0], [0.0, 0.0, 0.0], [0.0, 0.0, 0.0], [0.0, 0.0, 0.0]])
    s2 = np.array([[1.0, -1.0, 3.0], [0.0, 0.0, 0.0], [0.0, 0.0, 0.0], [0.0, 0.0, 0.0]])
    assert list(oracle.tile_assign(t2, s2)) == [0, 0, 1]


def test_draws_with_equal_masses_follow_the_closed_form():
    P, n = 1000, 5000
    to = np.arange(P, dtype=np.int32) % 7
    samples = np.vstack([np.arange(P, dtype=float)] * 4)
    rc, th, lq, lp, idx = oracle.tile_draw(np.full(7, -3.0), to, np.zeros(P), samples, 11, 2, n)
    u = oracle.uniforms(11, 2, n, 1)[:, 0, 0]
    assert rc == 0
    assert np.array_equal(idx, np.ceil(u * P).astype(np.int64) - 1)
    assert np.array_equal(th[0], idx.astype(float))
    np.testing.assert_allclose(lq, 0.0, atol=1e-12)  # proposal = the samples' own measure


def test_draw_frequencies_follow_tile_likelihood_and_prior():
    rng = np.random.default_rng(8)
    P, n = 3000, 200000
    to = rng.integers(0, 5, P).astype(np.int32)
    tl = np.array([0.0, math.log(3.0), -math.inf, -1.0, 0.5])
    lp = rng.normal(0, 0.3, P)
    rc, th, lq, lpo, idx = oracle.tile_draw(tl, to, lp, np.zeros((4, P)), 12, 0, n)
    assert rc == 0 and np.all(idx >= 0)
    mass = np.exp(tl[to] + lp)
    mass[~np.isfinite(tl[to])] = 0.0
    tile_mass = np.bincount(to, weights=mass, minlength=5)
    counts = np.bincount(to[idx], minlength=5)
    assert counts[2] == 0  # a tile with zero likelihood is never drawn
    keep = tile_mass > 0
    exp = n * tile_mass[keep] / tile_mass.sum()
    chi2 = ((counts[keep] - exp) ** 2 / exp).sum()
    assert stats.chi2.sf(chi2, keep.sum() - 1) > 1e-4
    assert np.array_equal(lpo, lp[idx])
    # importance-sampling identity: E_q[exp(-logq)] = (samples with positive mass) / P
    assert abs(np.exp(-lq).mean() - (mass > 0).mean()) < 5 * np.exp(-lq).std() / math.sqrt(n)


def test_draws_with_no_positive_mass():
    rc, th, lq, lp, idx = oracle.tile_draw(np.full(3, -np.inf), np.zeros(10, np.int32), np.zeros(10),
                                          np.ones((4, 10)), 1, 0, 5)
    assert rc == 5 and np.all(idx == -1) and np.all(lp == -np.inf) and np.all(lq == 0)


def test_tile_mixture_chain_is_efficient():
    """Config-0 event: slice of radius 6 around the trigger, bank at whitened spacing 1, 10^6
    candidates of prior samples, likelihood at the templates, 4096 proposal draws. The paper's
    BNS efficiencies are tens of percent; the injection-centred Gaussian gets < 0.1% here."""
    b = build_event(0, 0)
    ev = b.ev
    sl, L, c = _slice(b, 6.0)
    ty, tth, _ = ev.tile_bank(sl, 1.0, 5, 1, 4096, 20000, 0.002, 400)
    y, th, lp = ev.slice_sample(sl, 5, 2, 0, 1000000)
    to = oracle.tile_assign(ty, y)
    llt = ev.loglike(tth, n_threads=8)
    rc, thd, lq, lpd, idx = oracle.tile_draw(llt, to, lp, th, 7, 0, 4096)
    ll = ev.loglike(thd, n_threads=8)
    w, st = oracle.weights_ess(ll, lpd, lq)
    assert st[0] / 4096 > 0.10


def test_reweight_with_full_defensive_share_keeps_the_previous_masses():
    rng = np.random.default_rng(13)
    P, M, n = 4000, 50, 3000
    to = rng.integers(0, M, P).astype(np.int32)
    tl = rng.normal(0, 2, M)
    lp = rng.normal(0, 0.4, P)
    idx = rng.integers(0, P, n)
    w = rng.random(n)
    w /= w.sum()
    out = oracle.tile_reweight(tl, to, lp, idx, w, 1.0)
    # sample masses exp(out_t + lp) must be proportional to exp(tl_t + lp): out - tl is constant
    d = out - tl
    np.testing.assert_allclose(d, d[0], rtol=0, atol=1e-12)


def test_reweight_puts_the_mass_where_the_weights_are():
    P, M = 600, 6
    to = (np.arange(P) % M).astype(np.int32)
    lp = np.zeros(P)
    tl = np.zeros(M)
    idx = np.array([0, 6, 1, 2, -1])  # tiles 0, 0, 1, 2 and a draw without a sample
    w = np.array([0.5, 0.3, 0.2, 0.0, 0.7])
    out = oracle.tile_reweight(tl, to, lp, idx, w, 0.0)
    # pi = (0.8, 0.2, 0, 0, 0, 0) over tiles of 100 samples each
    np.testing.assert_allclose(out[:2], np.log([0.8, 0.2]) - math.log(100.0), rtol=0, atol=1e-14)
    assert np.all(out[2:] == -np.inf)
    mix = oracle.tile_reweight(tl, to, lp, idx, w, 0.25)
    np.testing.assert_allclose(np.exp(mix) * 100, 0.75 * np.array([0.8, 0.2, 0, 0, 0, 0]) + 0.25 / 6, rtol=1e-13)


def test_reweight_estimates_tile_posterior_masses():
    # tiles with known target masses; draws from uniform tile probabilities, weights = target/proposal
    rng = np.random.default_rng(14)
    M, per = 20, 50
    P = M * per
    to = np.repeat(np.arange(M), per).astype(np.int32)
    true = rng.random(M) ** 3
    true /= true.sum()
    n = 400000
    idx = rng.integers(0, P, n)
    w = true[to[idx]] * M
    w /= w.sum()
    out = oracle.tile_reweight(np.zeros(M), to, np.zeros(P), idx, w, 0.0)
    est = np.exp(out) * per
    np.testing.assert_allclose(est, true, rtol=0, atol=5 * math.sqrt(true.max() / n) + 1e-12)


def test_reweighted_round_raises_the_efficiency():
    """The config-0 chain of test_tile_mixture_chain_is_efficient, then one reweighted round."""
    b = build_event(0, 0)
    ev = b.ev
    sl, L, c = _slice(b, 6.0)
    ty, tth, _ = ev.tile_bank(sl, 1.0, 5, 1, 4096, 20000, 0.002, 400)
    y, th, lp = ev.slice_sample(sl, 5, 2, 0, 4000000)
    to = oracle.tile_assign(ty, y)
    llt = ev.loglike(tth, n_threads=8)
    eff = []
    ell = llt
    for rnd in range(2):
        rc, thd, lq, lpd, idx = oracle.tile_draw(ell, to, lp, th, 7, rnd, 4096)
        ll = ev.loglike(thd, n_threads=8)
        w, st = oracle.weights_ess(ll, lpd, lq)
        eff.append(st[0] / 4096)
        ell = oracle.tile_reweight(ell, to, lp, idx, w, 0.1)
    assert eff[1] > 0.2 and eff[1] > 3 * eff[0]


def _overlap(b, ta, tb):
    """Complex overlap 4 df sum conj(h_a) h_b / S and the two norms, in numpy from the oracle's
    waveforms (each zero above its own cut)."""
    ha = b.ev.waveform(ta)
    hb = b.ev.waveform(tb)
    w = 4.0 * b.df / b.psd.astype(np.float64)
    o = (w * np.conj(ha) * hb).sum()
    return o, float((w * np.abs(ha) ** 2).sum()), float((w * np.abs(hb) ** 2).sum())


def test_match_is_the_phase_maximised_overlap():
    """The oracle's match (App. A's waveform similarity) against numpy: |<h_a, h_b>| over the norms,
    and the largest normalised real overlap over a grid of constant phase shifts (to the grid's
    resolution); 1 for a point with itself, symmetric, at most 1."""
    b = build_event(0, 0, n_bins=4000)
    rng = np.random.default_rng(3)
    g = b.ev.metric(b.theta_inj)
    cov = np.linalg.inv(g)
    assert b.ev.match(b.theta_inj, b.theta_inj) == pytest.approx(1.0, abs=1e-13)
    pts = []
    while len(pts) < 8:  # points inside the support
        t = b.theta_inj + rng.multivariate_normal(np.zeros(4), cov * 4.0)
        if np.isfinite(b.ev.logprior(t)):
            pts.append(t)
    for ta, tb in zip(pts[::2], pts[1::2]):
        m = b.ev.match(ta, tb)
        o, na, nb = _overlap(b, ta, tb)
        assert m == pytest.approx(abs(o) / math.sqrt(na * nb), rel=1e-12)
        phis = np.linspace(0.0, 2 * math.pi, 20001)
        best = np.max(np.real(np.exp(1j * phis) * o)) / math.sqrt(na * nb)
        assert m == pytest.approx(best, abs=1e-7)
        assert b.ev.match(tb, ta) == pytest.approx(m, rel=1e-13)
        assert 0.0 <= m <= 1.0


def test_mismatch_follows_the_metric():
    """1 - m(theta, theta + d) = d^T g d / (2 (h|h)) + O(|d|^3) with g the phase-projected metric of
    the 4-D set (the metric is the second-order expansion of the mismatch, Sec. II.A): at metric
    lengths 1e-3 .. 1e-4 in random directions the two agree to 1e-3 relative."""
    b = build_event(0, 0, n_bins=4000)
    th = b.theta_inj
    g = b.ev.metric(th)
    h = b.ev.waveform(th)
    hh = b.ev.inner(0, h, h)
    rng = np.random.default_rng(11)
    for eps in (1e-3, 3e-4, 1e-4):
        for _ in range(3):
            d = rng.standard_normal(4)
            d /= math.sqrt(d @ g @ d)
            mm = 1.0 - b.ev.match(th, th + eps * d)
            assert mm == pytest.approx(0.5 * eps * eps / hh, rel=1e-3)


def test_match_assignment_is_the_largest_match():
    """Tile by match against brute force in numpy over every template (from the oracle's waveforms):
    the template of largest match, and that match."""
    b = build_event(0, 1, n_bins=3000)
    sl, L, c = _slice(b, 4.0)
    ty, tth, used = b.ev.tile_bank(sl, 1.0, 7, 1, 512, 40, 0.0, 20)
    y, th, lp = b.ev.slice_sample(sl, 7, 2, 0, 400)
    th = th[:, :30]
    to, mv = b.ev.tile_assign_match(tth, th)
    for s in range(th.shape[1]):
        ms = []
        for j in range(tth.shape[1]):
            o, na, nb = _overlap(b, th[:, s], tth[:, j])
            ms.append(abs(o) / math.sqrt(na * nb))
        ms = np.array(ms)
        assert mv[s] == pytest.approx(ms.max(), rel=1e-12)
        assert ms[to[s]] == pytest.approx(ms.max(), rel=1e-12)
