"""Pins of the oracle's tile mixture over the intrinsic coordinates of the 11-D set (Sec. III: the
prior volume is tiled over the intrinsic parameters, which partially decouple from the extrinsic
ones; App. A: bank, tiling of the prior volume, proposal): the sub-slice sampler against its own
geometry, and the extrinsic completion of the tile draws against the Gaussian marginal written from
its definition (covariance block, explicit image sum), its moments, and its independence from the
tiled coordinates."""
import math

import numpy as np
from scipy import optimize, stats
from scipy.special import logsumexp

import oracle
from events import build_event

INTRINSIC = 0xF  # Mc, q, chi1z, chi2z
PERIODS = {4: 2 * math.pi, 7: math.pi, 10: 2 * math.pi}


def _intrinsic_slice(b, radius, g=None):
    g = b.ev.metric(b.theta_inj) if g is None else g
    C = np.linalg.inv(g)
    GI = np.linalg.inv(C[:4, :4])  # the proposal's marginal precision over the intrinsic coordinates
    L = np.linalg.cholesky(GI)
    return oracle.make_slice(b.theta_inj, L, radius, INTRINSIC), L, g


def _wrapped_centre(th0):
    c0 = np.array(th0, dtype=np.float64)
    for k, P in PERIODS.items():
        c0[k] = th0[k] - P * math.floor(th0[k] / P)
    return c0


def _marginal_logpdf(x, th0, g, keep):
    """Log density of the marginal of N(th0, g^-1) over `keep`, wrapped: the covariance block and an
    explicit sum over the images -2..2 of every periodic coordinate kept."""
    C = np.linalg.inv(g)
    Ck = C[np.ix_(keep, keep)]
    c0 = _wrapped_centre(th0)[keep]
    pk = [(j, PERIODS[k]) for j, k in enumerate(keep) if k in PERIODS]
    terms = []
    for img in np.ndindex(*([5] * len(pk))):
        s = np.array(x, dtype=np.float64)[keep]
        for (j, P), t in zip(pk, img):
            s[j] += (t - 2) * P
        terms.append(stats.multivariate_normal.logpdf(s, c0, Ck))
    return logsumexp(terms)


def test_sub_slice_candidates_follow_their_definition():
    b = build_event(1, 0, n_bins=4000)
    sl, L, g = _intrinsic_slice(b, 3.0)
    assert b.ev.slice_dims(sl) == 4
    u = oracle.uniforms(9, 3, 100, 2).reshape(100, 4)  # two Philox blocks per candidate (S = 4)
    kept = 0
    for i in range(100):
        ok, y, th = b.ev.slice_candidate(sl, 9, 3, i)
        assert np.array_equal(y, 3.0 * (2.0 * u[i] - 1.0))
        assert np.array_equal(th[4:], b.theta_inj[4:])  # extrinsic coordinates stay at the centre
        np.testing.assert_allclose(L.T @ (th[:4] - b.theta_inj[:4]), y, rtol=0, atol=1e-9 * 3.0)
        src_ok = th[0] > 0 and 0 < th[1] <= 1 and abs(th[2]) <= b.chi_max and abs(th[3]) <= b.chi_max
        assert ok == bool(y @ y <= 9.0 and src_ok)
        kept += ok
    assert kept > 20
    # samples: the kept candidates in order, y with S rows, theta with all D
    y, th, lp = b.ev.slice_sample(sl, 9, 3, 0, 100)
    assert y.shape == (4, kept) and th.shape == (11, kept)
    assert np.all(lp == b.ev.logprior(th[:, 0]))  # flat in the intrinsic coordinates


def test_sub_slice_bank_packs_in_the_intrinsic_coordinates():
    b = build_event(1, 0, n_bins=4000)
    sl, L, g = _intrinsic_slice(b, 3.0)
    ty, tth, used = b.ev.tile_bank(sl, 1.0, 5, 1, 2048, 5000, 0.002, 50)
    m = ty.shape[1]
    assert ty.shape[0] == 4 and tth.shape == (11, m) and 20 < m < 5000
    d2 = ((ty[:, :, None] - ty[:, None, :]) ** 2).sum(0)
    np.fill_diagonal(d2, np.inf)
    assert d2.min() >= 1.0 - 1e-12
    np.testing.assert_allclose(L.T @ (tth[:4] - b.theta_inj[:4, None]), ty, rtol=0, atol=1e-9 * 3.0)
    assert np.all(tth[4:] == b.theta_inj[4:, None])


def _intrinsic_inputs(th0, n, seed=1):
    rng = np.random.default_rng(seed)
    th = np.tile(np.asarray(th0, dtype=np.float64)[:, None], (1, n))
    th[:4] += rng.normal(size=(4, n)) * np.array([1e-4, 0.05, 0.03, 0.03])[:, None]
    return th


def test_extrinsic_density_is_the_wrapped_marginal():
    b = build_event(1, 0, n_bins=4000)  # explicit phase, distance and tc sampled: all 7 extrinsic drawn
    th0 = b.theta_inj
    g = b.ev.metric(th0)
    n = 400
    th = _intrinsic_inputs(th0, n)
    lq_in = np.linspace(-3.0, 2.0, n)
    lp_in = np.zeros(n)
    lp_in[5] = -np.inf  # a draw without a sample keeps its -inf
    rc, t2, lq, lp = b.ev.tile_extrinsic(th0, g, INTRINSIC, 7, 3, th, lq_in, lp_in)
    assert rc == 0
    assert np.array_equal(t2[:4], th[:4])
    keep = list(range(4, 11))
    ref = np.array([_marginal_logpdf(t2[:, i], th0, g, keep) for i in range(40)])
    np.testing.assert_allclose(lq[:40] - lq_in[:40], ref, rtol=0, atol=1e-9)
    assert lp[5] == -np.inf
    lp_ref = np.array([b.ev.logprior(t2[:, i]) for i in range(n)])
    ok = np.arange(n) != 5
    np.testing.assert_array_equal(lp[ok], lp_ref[ok])
    for k, P in PERIODS.items():
        assert np.all((t2[k] >= 0) & (t2[k] < P))


def test_extrinsic_draws_follow_the_marginal_and_ignore_the_tiled_coordinates():
    # a narrow proposal (100 g): wrapping leaves the offsets Gaussian, so their whitened
    # covariance under the marginal's precision is the identity
    b = build_event(1, 0, n_bins=4000)
    th0 = b.theta_inj
    g = 100.0 * b.ev.metric(th0)
    n = 20000
    th = _intrinsic_inputs(th0, n)
    rc, t2, lq, lp = b.ev.tile_extrinsic(th0, g, INTRINSIC, 11, 0, th, np.zeros(n), np.zeros(n))
    assert rc == 0
    keep = list(range(4, 11))
    c0 = _wrapped_centre(th0)
    off = t2[keep] - c0[keep, None]
    for j, k in enumerate(keep):
        if k in PERIODS:
            P = PERIODS[k]
            off[j] -= P * np.floor(off[j] / P + 0.5)
    Ck = np.linalg.inv(g)[np.ix_(keep, keep)]
    W = np.linalg.cholesky(np.linalg.inv(Ck))
    w = W.T @ off
    assert np.all(np.abs(w.mean(1)) < 5.0 / math.sqrt(n))
    assert np.abs(np.cov(w) - np.eye(len(keep))).max() < 6.0 * math.sqrt(2.0 / n)
    # the conditional covariance (the tiled coordinates held fixed) is narrower: a draw that used it
    # would fail the check above; the extrinsic values do not depend on the tiled ones
    th_b = th.copy()
    th_b[:4] += 0.01
    _, t3, lq3, _ = b.ev.tile_extrinsic(th0, g, INTRINSIC, 11, 0, th_b, np.zeros(n), np.zeros(n))
    assert np.array_equal(t3[4:], t2[4:]) and np.array_equal(lq3, lq)


def test_extrinsic_with_the_likelihood_marginals():
    # time-, phase- and distance-marginalised event: only ra, dec, iota, psi enter log q; tc is the
    # proposal's conditional mean given the composed draw
    b = build_event(1, 0, n_bins=4000, phase=oracle.PHASE_MARG, distance=1,
                    time_marg={"tc_lo": -0.02, "tc_hi": 0.02, "tm_points": 64})
    th0 = b.theta_inj
    g = b.ev.metric(th0)
    n = 60
    th = _intrinsic_inputs(th0, n)
    rc, t2, lq, lp = b.ev.tile_extrinsic(th0, g, INTRINSIC, 3, 1, th, np.zeros(n), np.zeros(n))
    assert rc == 0
    keep = [4, 5, 6, 7]
    ref = np.array([_marginal_logpdf(t2[:, i], th0, g, keep) for i in range(n)])
    np.testing.assert_allclose(lq, ref, rtol=0, atol=1e-9)
    c0 = _wrapped_centre(th0)
    for i in range(0, n, 12):
        x = t2[:, i].copy()
        d = x - c0
        for k, P in PERIODS.items():
            d[k] -= P * math.floor(d[k] / P + 0.5)

        def quad(t):
            e = d.copy()
            e[9] = t - c0[9]
            return e @ g @ e

        r = optimize.minimize_scalar(quad, bracket=(c0[9] - 1e-3, c0[9] + 1e-3), tol=1e-14)
        assert abs(x[9] - r.x) < 1e-9


def test_extrinsic_rejects_periodic_or_empty_masks():
    b = build_event(1, 0, n_bins=2000)
    th0 = b.theta_inj
    g = b.ev.metric(th0)
    th = _intrinsic_inputs(th0, 4)
    for mask in (0, 0xF | (1 << 4), 1 << 7, 1 << 11):
        rc, *_ = b.ev.tile_extrinsic(th0, g, mask, 1, 0, th, np.zeros(4), np.zeros(4))
        assert rc != 0


def _conditional(th0, g, thI, I, E):
    """Mean and covariance of the coordinates E given those of I = thI under N(th0, g^-1), the other
    coordinates integrated out: the covariance blocks of g^-1 (the definition)."""
    C = np.linalg.inv(g)
    B = C[np.ix_(E, I)] @ np.linalg.inv(C[np.ix_(I, I)])
    m = th0[E] + B @ (thI - th0[I])
    S = C[np.ix_(E, E)] - B @ C[np.ix_(I, E)]
    return m, S


def _wrapped_logpdf(x, m, S, E):
    pk = [(j, PERIODS[k]) for j, k in enumerate(E) if k in PERIODS]
    mw = np.array(m, dtype=np.float64)
    for j, P in pk:
        mw[j] -= P * math.floor(mw[j] / P)
    terms = []
    for img in np.ndindex(*([5] * len(pk))):
        s = np.array(x, dtype=np.float64)
        for (j, P), t in zip(pk, img):
            s[j] += (t - 2) * P
        terms.append(stats.multivariate_normal.logpdf(s, mw, S))
    return logsumexp(terms)


def test_conditional_extrinsic_density_is_the_wrapped_conditional():
    b = build_event(1, 0, n_bins=4000)
    th0 = b.theta_inj
    g = b.ev.metric(th0)
    n = 60
    th = _intrinsic_inputs(th0, n, seed=4)
    rc, t2, lq, lp = b.ev.tile_extrinsic(th0, g, INTRINSIC, 7, 3, th, np.zeros(n), np.zeros(n), conditional=True)
    assert rc == 0
    assert np.array_equal(t2[:4], th[:4])
    I, E = [0, 1, 2, 3], list(range(4, 11))
    for i in range(n):
        m, S = _conditional(th0, g, th[:4, i], I, E)
        # 1e-8: both sides invert blocks of g^-1, whose condition number here is ~1e9 (tc)
        assert abs(lq[i] - _wrapped_logpdf(t2[E, i], m, S, E)) < 1e-8
    for k, P in PERIODS.items():
        assert np.all((t2[k] >= 0) & (t2[k] < P))


def test_conditional_extrinsic_moments_follow_the_tiled_draw():
    # every draw with the same intrinsic point, a narrow proposal: the extrinsic offsets from the
    # conditional mean have the conditional covariance, narrower than the marginal's
    b = build_event(1, 0, n_bins=4000)
    th0 = b.theta_inj
    g = 100.0 * b.ev.metric(th0)
    n = 20000
    thI = th0[:4] + np.array([2e-5, 0.01, -0.01, 0.005])
    th = np.tile(th0[:, None], (1, n))
    th[:4] = thI[:, None]
    rc, t2, lq, lp = b.ev.tile_extrinsic(th0, g, INTRINSIC, 13, 0, th, np.zeros(n), np.zeros(n), conditional=True)
    assert rc == 0
    I, E = [0, 1, 2, 3], list(range(4, 11))
    m, S = _conditional(th0, g, thI, I, E)
    off = t2[E] - m[:, None]
    for j, k in enumerate(E):
        if k in PERIODS:
            P = PERIODS[k]
            off[j] -= P * np.floor(off[j] / P + 0.5)
    W = np.linalg.cholesky(np.linalg.inv(S))
    w = W.T @ off
    assert np.all(np.abs(w.mean(1)) < 5.0 / math.sqrt(n))
    assert np.abs(np.cov(w) - np.eye(len(E))).max() < 6.0 * math.sqrt(2.0 / n)
    Cm = np.linalg.inv(g)[np.ix_(E, E)]
    assert np.all(np.diag(S) <= np.diag(Cm) * (1 + 1e-12))
    assert np.linalg.det(S) < 0.9 * np.linalg.det(Cm)


def test_conditional_extrinsic_with_the_likelihood_marginals():
    # time-, phase- and distance-marginalised: ra, dec, iota, psi given the intrinsic point, with tc,
    # phic and dL integrated out
    b = build_event(1, 0, n_bins=4000, phase=oracle.PHASE_MARG, distance=1,
                    time_marg={"tc_lo": -0.02, "tc_hi": 0.02, "tm_points": 64})
    th0 = b.theta_inj
    g = b.ev.metric(th0)
    n = 40
    th = _intrinsic_inputs(th0, n, seed=6)
    rc, t2, lq, lp = b.ev.tile_extrinsic(th0, g, INTRINSIC, 3, 1, th, np.zeros(n), np.zeros(n), conditional=True)
    assert rc == 0
    I, E = [0, 1, 2, 3], [4, 5, 6, 7]
    for i in range(n):
        m, S = _conditional(th0, g, th[:4, i], I, E)
        assert abs(lq[i] - _wrapped_logpdf(t2[E, i], m, S, E)) < 1e-9
    # the draw with the intrinsic point at the centre has the conditional mean at the centre
    th[:4, 0] = th0[:4]
    rc, t3, lq3, _ = b.ev.tile_extrinsic(th0, g, INTRINSIC, 3, 1, th[:, :1], np.zeros(1), np.zeros(1),
                                         conditional=True)
    m, S = _conditional(th0, g, th0[:4], I, E)
    np.testing.assert_allclose(m, th0[E], rtol=0, atol=1e-12)


def test_network_match_at_shared_extrinsics_is_the_intrinsic_match():
    """The match of two 11-D points that share their extrinsic coordinates (as a slice over the
    intrinsic ones makes them): with equal PSDs the detectors' common responses and delays factor
    out, so the three-detector network match equals the one-detector match of the same points, does
    not move when the shared extrinsic values change, and is 1 for a point with itself."""
    b3 = build_event(1, 0, n_bins=3000)
    b1 = build_event(1, 0, n_bins=3000, n_det=1)
    a = b3.theta_inj.copy()
    rng = np.random.default_rng(4)
    for _ in range(5):
        bpt = a.copy()
        bpt[0] *= 1.0 + 2e-4 * rng.standard_normal()
        bpt[1] = min(1.0, bpt[1] * (1.0 + 0.02 * rng.standard_normal()))
        bpt[2] += 0.02 * rng.standard_normal()
        bpt[3] += 0.02 * rng.standard_normal()
        m3 = b3.ev.match(a, bpt)
        m1 = b1.ev.match(a, bpt)
        assert 0.0 < m3 < 1.0
        assert abs(m3 - m1) <= 1e-12, (m3, m1)
        a2, b2 = a.copy(), bpt.copy()
        for k, v in ((4, 1.3), (5, -0.4), (6, 2.1), (7, 0.3), (8, 0.7 * a[8]), (9, a[9] + 1e-3), (10, 4.0)):
            a2[k] = b2[k] = v
        assert abs(b3.ev.match(a2, b2) - m3) <= 1e-12
    assert abs(b3.ev.match(a, a) - 1.0) <= 1e-14


def test_shift_maximised_match_pins():
    """The match maximised over time shifts j dt (|j| <= J) as well: no shifts is the plain match;
    a copy of a point moved in tc by an exact grid shift (any other coordinate shared) matches it to
    1; the maximum over the grid is at least the unshifted match and grows with the grid; and the
    maximum over a fine grid agrees with a scalar maximisation of the closed-form shifted overlap
    (numpy, from the oracle's waveforms: |sum_k w conj(a_k) b_k e^(-2 pi i f_k t)|)."""
    from scipy.optimize import minimize_scalar

    b = build_event(1, 0, n_bins=3000)
    a = b.theta_inj.copy()
    rng = np.random.default_rng(6)
    dt = 2e-4
    for _ in range(3):
        bpt = a.copy()
        bpt[0] *= 1.0 + 3e-4 * rng.standard_normal()
        bpt[2] += 0.02 * rng.standard_normal()
        m0 = b.ev.match(a, bpt)
        assert abs(b.ev.match_shift(a, bpt, dt, 0) - m0) <= 1e-13
        m4 = b.ev.match_shift(a, bpt, dt, 4)
        m16 = b.ev.match_shift(a, bpt, dt, 16)
        assert m0 <= m4 + 1e-15 <= m16 + 2e-15
        # the same point moved by +3 dt in tc: the shifts -3 dt bring it back
        c = a.copy()
        c[9] += 3 * dt
        assert abs(b.ev.match_shift(a, c, dt, 4) - 1.0) <= 1e-11
        assert b.ev.match_shift(a, c, dt, 2) < 1.0 - 1e-6
    # the closed form of the shifted overlap (numpy on the oracle's waveforms) on the same grid, and
    # a continuous maximisation about its best grid point
    bpt = a.copy()
    bpt[0] *= 1.0 + 2e-5
    bpt[9] += 3.3e-4
    f = b.f_lo + b.df * np.arange(b.n_bins)
    ha = b.ev.waveform(a)
    hb = b.ev.waveform(bpt)
    w = 4 * b.df / b.psd.astype(np.float64)
    c = (w * np.conj(ha) * hb).sum(axis=0)
    na = float((w * np.abs(ha) ** 2).sum())
    nb = float((w * np.abs(hb) ** 2).sum())

    def ov(t):
        return abs((c * np.exp(-2j * np.pi * f * t)).sum()) / math.sqrt(na * nb)

    dt, J = 2e-5, 250
    grid = np.array([ov(j * dt) for j in range(-J, J + 1)])
    got = b.ev.match_shift(a, bpt, dt, J)
    assert abs(got - grid.max()) <= 1e-12
    jb = int(np.argmax(grid))
    assert 0 < jb < 2 * J  # an interior maximum (the chirp mass's shift is absorbed by tc)
    t0 = (jb - J) * dt
    r = minimize_scalar(lambda t: -ov(t), bounds=(t0 - dt, t0 + dt), method="bounded", options={"xatol": 1e-10})
    assert got <= -r.fun + 1e-12 and got >= -r.fun - 1e-3
