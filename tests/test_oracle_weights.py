"""Pins of the oracle's importance weights (App. A.3, Eq. 5) and effective sample size (Eq. 6),
and of the whole CPU chain (metric -> draws -> likelihood -> weights) against brute-force
quadrature of the evidence on a tiny frequency grid."""
import math

import numpy as np
import pytest
from scipy import optimize, special

import oracle
from paper_2410_05190_amd import synth


def _ws(ll, lp=None, lq=None):
    ll = np.asarray(ll, dtype=np.float64)
    lp = np.zeros_like(ll) if lp is None else lp
    lq = np.zeros_like(ll) if lq is None else lq
    return oracle.weights_ess(ll, lp, lq)


def test_equal_weights_give_ess_n_exactly():
    for n in (1, 7, 4096, 100003):
        w, st = _ws(np.full(n, -3.7))
        assert st[0] == n
        assert st[3] == n
        assert np.all(w == 1.0 / n)


def test_single_finite_weight_gives_ess_one():
    ll = np.full(1000, -np.inf)
    ll[123] = 5.0
    w, st = _ws(ll)
    assert st[0] == 1.0 and st[3] == 1 and w[123] == 1.0 and w.sum() == 1.0
    assert st[1] == pytest.approx(5.0 - math.log(1000))


def test_two_levels_closed_form():
    n1, n2, a, b = 300, 700, 0.0, -1.3
    ll = np.concatenate([np.full(n1, a), np.full(n2, b)])
    w, st = _ws(ll)
    ea, eb = math.exp(a), math.exp(b)
    assert st[0] == pytest.approx((n1 * ea + n2 * eb) ** 2 / (n1 * ea * ea + n2 * eb * eb), rel=1e-14)


def test_shift_invariance_and_log_evidence():
    rng = np.random.default_rng(1)
    ll = rng.normal(0, 3, 5000)
    lp = rng.normal(0, 1, 5000)
    lq = rng.normal(0, 1, 5000)
    w1, s1 = _ws(ll, lp, lq)
    w2, s2 = _ws(ll + 1234.5, lp, lq)
    np.testing.assert_allclose(w1, w2, rtol=1e-10)
    assert s1[0] == pytest.approx(s2[0], rel=1e-10)
    assert s2[1] - s1[1] == pytest.approx(1234.5, rel=1e-12)
    lw = ll + lp - lq
    assert s1[1] == pytest.approx(special.logsumexp(lw) - math.log(lw.size), rel=1e-13)
    assert w1.sum() == pytest.approx(1.0, rel=1e-14)
    assert s1[2] == lw.max()


def test_lognormal_weights_efficiency():
    """ln w ~ N(0, s^2): ESS/N -> E[w]^2 / E[w^2] = exp(-s^2)."""
    rng = np.random.default_rng(2)
    s = 0.5
    w, st = _ws(rng.normal(0, s, 2_000_000))
    assert st[0] / 2_000_000 == pytest.approx(math.exp(-s * s), rel=5e-3)


def test_all_out_of_support():
    w, st = _ws(np.full(10, -np.inf))
    assert st[0] == 0 and st[3] == 0 and st[1] == -math.inf and np.all(w == 0)


def test_proposal_equal_to_target_gives_ess_n():
    """If L pi is proportional to g (Eq. 5 with the proposal equal to the posterior) every weight is
    equal and ESS = N (the paper's statement about Eq. 6)."""
    rng = np.random.default_rng(4)
    lq = rng.normal(0, 5, 1000)
    lp = rng.normal(0, 1, 1000)
    ll = lq - lp + 2.5
    w, st = _ws(ll, lp, lq)
    assert st[0] == pytest.approx(1000, rel=1e-12)
    assert st[1] == pytest.approx(2.5, rel=1e-12)


def _tiny_event(snr=3000.0, eta=0.15, K=128, df=8.0, f_lo=40.0, seed_event=5):
    f = synth.frequencies(f_lo, df, K)
    S = synth.psd_analytic(f)[None, :]
    th = np.array([1.2, eta, 0.0, 0.0])
    ref = oracle.Event(1, K, f_lo, df, psd=S, params=oracle.PARAMS_4D, phase=oracle.PHASE_MARG, amp0=1.0,
                       chi_max=0.9)
    h1 = ref.waveform(th)
    A = snr / math.sqrt(ref.inner(0, h1, h1))
    sig = oracle.Event(1, K, f_lo, df, psd=S, params=oracle.PARAMS_4D, phase=oracle.PHASE_MARG, amp0=A,
                       chi_max=0.9)
    d = sig.waveform(th) + synth.noise(0, seed_event, S, df)
    return oracle.Event(1, K, f_lo, df, data=d, psd=S, params=oracle.PARAMS_4D, phase=oracle.PHASE_MARG, amp0=A,
                        chi_max=0.9), th


@pytest.mark.slow
def test_whole_chain_evidence_and_means_against_grid_quadrature():
    """Tiny grid (128 bins, high SNR so the posterior is near-Gaussian): ln Z and posterior means from the importance-sampling chain agree with
    a trapezoid quadrature of L pi within Monte-Carlo error. The quadrature grid lies on the principal
    axes of the Laplace approximation at the peak (finite-difference Hessian of ln L), so it is
    independent of the proposal the chain uses."""
    ev, th_inj = _tiny_event()
    sd = np.sqrt(np.diag(np.linalg.inv(ev.metric(th_inj))))
    res = optimize.minimize(lambda x: -ev.loglike((th_inj + x * sd)[:, None])[0], np.zeros(4),
                            method="Nelder-Mead", options=dict(xatol=1e-6, fatol=1e-9, maxiter=8000))
    th0 = th_inj + res.x * sd
    g = ev.metric(th0)
    N = 40000
    rc, T, lq, lp = ev.draw(th0, g, 31, 0, N)
    assert rc == 0
    ll = ev.loglike(T)
    w, st = oracle.weights_ess(ll, lp, lq)
    ess = st[0]
    assert ess > 0.005 * N
    lnz_is = st[1]
    mean_is = T @ w

    # Laplace covariance from a central-difference Hessian of ln L at the peak
    hs = 0.05 * sd
    D = 4
    f0 = ev.loglike(th0[:, None])[0]
    Hm = np.zeros((D, D))
    for i in range(D):
        for j in range(i, D):
            pts = []
            for si, sj in ((1, 1), (1, -1), (-1, 1), (-1, -1)):
                x = th0.copy()
                x[i] += si * hs[i]
                x[j] += sj * hs[j]
                pts.append(x)
            v = ev.loglike(np.array(pts).T)
            Hm[i, j] = Hm[j, i] = (v[0] - v[1] - v[2] + v[3]) / (4 * hs[i] * hs[j])
    lam, V = np.linalg.eigh(np.linalg.inv(-Hm))
    assert np.all(lam > 0)
    B = V * np.sqrt(lam)
    n1, lim = 21, 7.0
    u1 = np.linspace(-lim, lim, n1)
    h = u1[1] - u1[0]
    U = np.stack(np.meshgrid(u1, u1, u1, u1, indexing="ij"), 0).reshape(4, -1)
    TH = th0[:, None] + B @ U
    llg = ev.loglike(TH)
    lpg = np.array([ev.logprior(TH[:, j]) for j in range(TH.shape[1])])
    lw = llg + lpg
    m = lw[np.isfinite(lw)].max()
    wg = np.where(np.isfinite(lw), np.exp(lw - m), 0.0)
    # the grid's outer shell carries no mass: the box holds the whole posterior
    edge = np.any(np.abs(U) > lim - 1.5 * h, axis=0)
    assert wg[edge].sum() < 1e-4 * wg.sum()
    vol = h ** 4 * abs(np.linalg.det(B))
    lnz_grid = m + math.log(wg.sum() * vol)
    mean_grid = TH @ wg / wg.sum()
    post_sd = np.sqrt(((TH - mean_grid[:, None]) ** 2) @ wg / wg.sum())
    # IS estimate of ln Z has relative error ~ 1/sqrt(ESS)
    assert abs(lnz_is - lnz_grid) < 5.0 / math.sqrt(ess)
    assert np.all(np.abs(mean_is - mean_grid) < 5 * post_sd / math.sqrt(ess))


def test_undefined_log_weight_makes_every_estimate_nan():
    """A NaN or +inf log-weight has no weight (Eq. 5 needs a finite likelihood ratio or an
    excluded draw): ESS, ln Z, max ln w and every weight are NaN, the finite count stays;
    -inf alone is a draw outside the support, weight 0."""
    rng = np.random.default_rng(5)
    for bad in (np.nan, np.inf):
        ll = rng.normal(size=500)
        ll[[3, 77]] = [-np.inf, bad]
        w, st = _ws(ll)
        assert np.all(np.isnan(w)) and np.all(np.isnan(st[:3])) and st[3] == 498
    ll = rng.normal(size=500)
    ll[3] = -np.inf
    w, st = _ws(ll)
    assert np.isfinite(st).all() and w[3] == 0 and st[3] == 499
