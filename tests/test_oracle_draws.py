"""Pins of the oracle's proposal (Gaussian in the metric around theta0), its counter-based
generator (Philox4x32-10) and its log-density, and of the prior."""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
from events import build_event


def test_philox_is_a_bijection_with_avalanche():
    """Flipping one input bit changes about half of the 128 output bits (a 10-round Philox
    property); distinct counters never collide over a small sample."""
    rng = np.random.default_rng(3)
    flips = []
    seen = set()
    for _ in range(300):
        ctr = [int(x) for x in rng.integers(0, 2 ** 32, 4)]
        key = [int(x) for x in rng.integers(0, 2 ** 32, 2)]
        a = oracle.philox4x32_10(ctr, key)
        seen.add(tuple(a))
        bit = int(rng.integers(0, 128))
        c2 = list(ctr)
        c2[bit // 32] ^= 1 << (bit % 32)
        b = oracle.philox4x32_10(c2, key)
        flips.append(sum(bin(x ^ y).count("1") for x, y in zip(a, b)))
    assert len(seen) == 300
    assert abs(np.mean(flips) - 64) < 2.0


def test_uniforms_range_and_distribution():
    u = oracle.uniforms(12345, 7, 50000, 2).ravel()
    assert np.all(u > 0) and np.all(u <= 1)
    assert abs(u.mean() - 0.5) < 5 * math.sqrt(1 / 12 / u.size)
    counts, _ = np.histogram(u, bins=100, range=(0, 1))
    chi2 = ((counts - u.size / 100) ** 2 / (u.size / 100)).sum()
    assert stats.chi2.sf(chi2, 99) > 1e-4
    assert abs(np.corrcoef(u[:-1], u[1:])[0, 1]) < 5 / math.sqrt(u.size)
    # exactly representable 53-bit grid
    assert np.all(np.round(u * 2.0 ** 53) == u * 2.0 ** 53)
    # different streams and seeds give different sequences
    assert not np.array_equal(oracle.uniforms(12345, 8, 10, 1), oracle.uniforms(12345, 7, 10, 1))
    assert not np.array_equal(oracle.uniforms(12346, 7, 10, 1), oracle.uniforms(12345, 7, 10, 1))


def _spd(D, rng, scale):
    A = rng.standard_normal((D, D))
    C = A @ A.T + D * np.eye(D)
    s = np.asarray(scale)
    return C / np.outer(s, s)


def test_draw_moments_4d():
    b = build_event(0, 0, n_bins=4000)
    rng = np.random.default_rng(5)
    th0 = b.theta_inj
    g = _spd(4, rng, [1e-3, 1e-2, 1e-1, 1e-3])
    n = 40000
    rc, th, lq, lp = b.ev.draw(th0, g, 99, 1, n)
    assert rc == 0
    cov = np.linalg.inv(g)
    sd = np.sqrt(np.diag(cov))
    assert np.all(np.abs(th.mean(1) - th0) < 5 * sd / math.sqrt(n))
    emp = np.cov(th)
    corr_err = np.abs(emp - cov) / np.outer(sd, sd)
    assert corr_err.max() < 5 * math.sqrt(2.0 / n)
    # standardised draws are N(0, 1): KS on the first coordinate
    z = (th[0] - th0[0]) / sd[0]
    assert stats.kstest(z, "norm").pvalue > 1e-4


def test_draw_wraps_periodic_and_moments_11d():
    b = build_event(1, 0, n_bins=4000)
    th0 = b.theta_inj.copy()
    rng = np.random.default_rng(6)
    scale = [1e-3, 0.1, 0.1, 0.1, 0.5, 0.3, 0.3, 0.6, 20.0, 1e-3, 1.0]
    g = _spd(11, rng, scale)
    n = 30000
    rc, th, lq, lp = b.ev.draw(th0, g, 2024, 3, n)
    assert rc == 0
    for i, P in ((4, 2 * math.pi), (7, math.pi), (10, 2 * math.pi)):
        assert np.all(th[i] >= 0) and np.all(th[i] < P)
    cov = np.linalg.inv(g)
    sd = np.sqrt(np.diag(cov))
    for i in (0, 1, 2, 3, 5, 6, 8, 9):
        assert abs(th[i].mean() - th0[i]) < 5 * sd[i] / math.sqrt(n)
    # wrapped coordinate: circular mean of the angle tracks theta0 for the wrapped normal
    for i, P in ((4, 2 * math.pi), (7, math.pi), (10, 2 * math.pi)):
        ang = 2 * math.pi * th[i] / P
        want = math.exp(-0.5 * (2 * math.pi * sd[i] / P) ** 2)
        m = np.mean(np.exp(1j * ang))
        assert abs(abs(m) - want) < 5 / math.sqrt(n)
        assert abs(np.angle(m * np.exp(-2j * math.pi * th0[i] / P))) < 5 / math.sqrt(n) / max(want, 1e-3)


def test_logq_two_routes():
    """z-form (whitened normals from the uniforms, image shifts mapped through L^T) against the
    oracle's theta-form (the wrapped-Gaussian density evaluated from theta alone)."""
    b = build_event(1, 1, n_bins=4000)
    th0 = b.theta_inj.copy()
    rng = np.random.default_rng(8)
    scale = [1e-3, 0.1, 0.1, 0.1, 0.8, 0.3, 0.3, 0.5, 20.0, 1e-3, 1.5]
    g = _spd(11, rng, scale)
    n = 500
    seed, stream = 77, 2
    rc, th, lq, lp = b.ev.draw(th0, g, seed, stream, n)
    u = oracle.uniforms(seed, stream, n, 6)
    r = np.sqrt(-2 * np.log(u[:, :, 0]))
    z = np.empty((n, 12))
    z[:, 0::2] = r * np.cos(2 * np.pi * u[:, :, 1])
    z[:, 1::2] = r * np.sin(2 * np.pi * u[:, :, 1])
    z = z[:, :11]
    L = np.linalg.cholesky(g)
    x_unwrapped = th0[:, None] + np.linalg.solve(L.T, z.T)
    per = {4: 2 * math.pi, 7: math.pi, 10: 2 * math.pi}
    k0 = np.zeros((11, n))
    for i, P in per.items():
        k0[i] = np.round((x_unwrapped[i] - th[i]) / P)
    np.testing.assert_allclose(th, x_unwrapped - k0 * np.array([per.get(i, 0) for i in range(11)])[:, None],
                               rtol=0, atol=1e-9)
    logdet = np.log(np.diag(L)).sum()
    lz = np.empty(n)
    import itertools
    for m in range(n):
        terms = []
        for ks in itertools.product((-2, -1, 0, 1, 2), repeat=3):
            shift = np.zeros(11)
            for (i, P), kk in zip(per.items(), ks):
                shift[i] = (kk - k0[i, m]) * P
            y = z[m] + L.T @ shift
            terms.append(-0.5 * y @ y)
        terms = np.array(terms)
        mx = terms.max()
        lz[m] = mx + np.log(np.exp(terms - mx).sum()) + logdet - 5.5 * math.log(2 * math.pi)
    np.testing.assert_allclose(lq, lz, rtol=0, atol=1e-8)
    rc2, lq2 = b.ev.logq_theta(th0, g, th)
    assert rc2 == 0
    np.testing.assert_array_equal(lq, lq2)


def _broad_periodic_metric(rng):
    """11-D precision whose periodic coordinates (ra, psi, phic) sit at the prior-limited width
    P / sqrt(12), coupled to each other and to the rest."""
    scale = [1e-3, 0.1, 0.1, 0.1, 1.0, 0.3, 0.3, 1.0, 20.0, 1e-3, 1.0]
    g = _spd(11, rng, scale) * 0.05
    per = {4: 2 * math.pi, 7: math.pi, 10: 2 * math.pi}
    C = np.linalg.inv(g)
    for i, P in per.items():  # covariance of each periodic coordinate = (P / sqrt(12))^2
        f = (P / math.sqrt(12.0)) / math.sqrt(C[i, i])
        C[i, :] *= f
        C[:, i] *= f
    return np.linalg.inv(C), per


def _wrapped_logpdf(th, th0, C, per, kmax):
    """log sum over images k in [-kmax, kmax]^3 of N(theta + k P; theta0, C) (scipy)."""
    import itertools
    mvn = stats.multivariate_normal(th0, C)
    terms = []
    for ks in itertools.product(range(-kmax, kmax + 1), repeat=3):
        shift = np.zeros(11)
        for (i, P), kk in zip(per.items(), ks):
            shift[i] = kk * P
        terms.append(mvn.logpdf((th + shift[:, None]).T))
    terms = np.array(terms)
    mx = terms.max(axis=0)
    return mx + np.log(np.exp(terms - mx).sum(axis=0))


def test_logq_broad_periodic_coordinates_against_many_images():
    """Periodic coordinates as broad as the prior precision allows (sd P / sqrt(12)) and a centre
    outside [0, P): the oracle's images -2..2 about the wrapped centre against scipy's Gaussian summed
    over images -6..6 about the raw centre (exact to e^-(6P)^2/(2 sd^2)), within 1e-9."""
    b = build_event(1, 1, n_bins=4000)
    rng = np.random.default_rng(21)
    g, per = _broad_periodic_metric(rng)
    th0 = b.theta_inj.copy()
    th0[4] += 2 * math.pi * 3 + 0.3   # ra: three periods up
    th0[7] -= math.pi * 2 + 0.2       # psi: two periods down
    th0[10] += 2 * math.pi            # phic: one period up
    rc, th, lq, lp = b.ev.draw(th0, g, 31, 0, 300)
    assert rc == 0
    for i, P in per.items():
        assert np.all((th[i] >= 0) & (th[i] < P))
    want = _wrapped_logpdf(th, th0, np.linalg.inv(g), per, 6)
    np.testing.assert_allclose(lq, want, rtol=0, atol=1e-9)


def test_phase_marginal_logq_is_the_integral_over_phic():
    """11-D phase-marginalised events leave phic out of the proposal density: log q equals the log of
    the full 11-D wrapped density integrated over phic (periodic trapezoid rule, 128 nodes), for a
    metric that couples phic to the other coordinates."""
    b = build_event(2, 0, n_bins=2000)
    assert b.phase == oracle.PHASE_MARG
    full = oracle.Event(b.n_det, b.n_bins, b.f_lo, b.df, data=b.data, psd=b.psd, strain_scale=b.strain_scale,
                        params=b.params, phase=oracle.PHASE_EXPLICIT, amp0=b.amp0, gmst=b.gmst,
                        chi_max=b.chi_max, dl_max=b.dl_max, det_geom=b.det_geom)
    rng = np.random.default_rng(22)
    g, per = _broad_periodic_metric(rng)
    th0 = b.theta_inj.copy()
    rc, th, lq, lp = b.ev.draw(th0, g, 41, 0, 60)
    assert rc == 0
    nodes = 2 * math.pi * np.arange(128) / 128
    vals = []
    for phi in nodes:
        t = th.copy()
        t[10] = phi
        rc, lf = full.logq_theta(th0, g, t)
        vals.append(lf)
    vals = np.array(vals)
    mx = vals.max(axis=0)
    want = mx + np.log(np.exp(vals - mx).mean(axis=0) * 2 * math.pi)
    np.testing.assert_allclose(lq, want, rtol=0, atol=1e-9)
    # the drawn phic is not used: moving it leaves log q unchanged
    t = th.copy()
    t[10] = (t[10] + 1.234) % (2 * math.pi)
    rc, lq2 = b.ev.logq_theta(th0, g, t)
    np.testing.assert_allclose(lq2, lq, rtol=0, atol=1e-12)


def test_logq_unwrapped_is_gaussian_density():
    """4-D (no periodic coordinate): log q equals scipy's multivariate normal logpdf."""
    b = build_event(0, 0, n_bins=4000)
    rng = np.random.default_rng(9)
    g = _spd(4, rng, [1e-3, 1e-2, 1e-1, 1e-3])
    rc, th, lq, lp = b.ev.draw(b.theta_inj, g, 5, 0, 200)
    want = stats.multivariate_normal(b.theta_inj, np.linalg.inv(g)).logpdf(th.T)
    np.testing.assert_allclose(lq, want, rtol=1e-10, atol=1e-8)


def test_logprior_and_support():
    b = build_event(1, 0, n_bins=4000)
    th = b.theta_inj.copy()
    want = math.log(math.cos(th[5])) + math.log(math.sin(th[6])) + 2 * math.log(th[8])
    assert b.ev.logprior(th) == pytest.approx(want, rel=1e-14)
    for i, bad in ((1, 1.0001), (1, -0.1), (2, 0.41), (3, -0.41), (5, 1.6), (6, -0.01), (6, 3.2),
                   (8, -1.0), (8, b.dl_max * 1.01), (0, -1.0)):
        t = th.copy()
        t[i] = bad
        assert b.ev.logprior(t) == -math.inf
    b4 = build_event(0, 0, n_bins=4000)
    t = b4.theta_inj.copy()
    assert b4.ev.logprior(t) == 0.0
    t[1] = 0.2501
    assert b4.ev.logprior(t) == -math.inf


def test_singular_metric_marks_every_draw_out_of_support():
    b = build_event(0, 0, n_bins=4000)
    g = np.diag([1.0, 1.0, -1.0, 1.0])
    rc, th, lq, lp = b.ev.draw(b.theta_inj, g, 1, 0, 10)
    assert rc == 3
    assert np.all(lp == -math.inf)
    assert np.all(th == b.theta_inj[:, None])
