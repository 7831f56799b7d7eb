"""Proposal update between importance-sampling rounds (Sec. III.A, end of the efficiency
discussion) on the GPU, through the C ABI: parity of pe_proposal_update with the oracle on the
same seeded draws and weights, edge cases, and pe_refine (the rounds of metric, draws,
likelihood, weights and update enqueued by the library) against the same calls made one by one."""
import math

import numpy as np
import pytest

import oracle
from events import build_event
from gpu_util import dev, host, note, torch_cuda, upload_event
from paper_2410_05190_amd import binding

pytestmark = pytest.mark.gpu

PERIODIC = {4: 2 * math.pi, 7: math.pi, 10: 2 * math.pi}


def _draws11(rng, n, th0):
    """Seeded parameter sets around th0, wide enough that the periodic coordinates wrap."""
    sd = np.array([1e-3, 0.05, 0.05, 0.05, 0.8, 0.2, 0.3, 0.9, 20.0, 1e-3, 1.5])
    th = th0[:, None] + sd[:, None] * rng.standard_normal((11, n))
    for a, P in PERIODIC.items():
        th[a] = np.mod(th[a], P)
    return th


def _weights(rng, n, zero_frac=0.4):
    w = np.exp(rng.normal(0.0, 3.0, n))
    w[rng.random(n) < zero_frac] = 0.0
    return w


def _check(ev_o, th0, th, w, got_c, got_cov):
    out_o, cov_o, _ = ev_o.proposal_update(th0, th, w)
    scale = np.abs(th - th0[:, None]).max(axis=1) + 1e-300
    err_c = np.abs(got_c - out_o)
    # a periodic centre near 0 or P may land on either side of the wrap
    for a, P in PERIODIC.items():
        if a < len(th0):
            err_c[a] = min(err_c[a], abs(err_c[a] - P))
    assert np.all(err_c <= 1e-12 * scale), (err_c / scale).max()
    # the covariance is a difference of raw second moments: its rounding scales with them
    d = th - th0[:, None]
    for a, P in PERIODIC.items():
        if a < len(th0):
            d[a] -= P * np.floor(d[a] / P + 0.5)
    pos = w > 0
    m2 = (d[:, pos] ** 2 * w[pos]).sum(axis=1) / w[pos].sum()
    cs = np.sqrt(np.outer(m2, m2)) + 1e-300
    assert np.all(np.abs(got_cov - cov_o) <= 1e-10 * cs), (np.abs(got_cov - cov_o) / cs).max()


def test_update_parity_11d_and_4d():
    torch = torch_cuda()
    rng = np.random.default_rng(31)
    for cfg, n in ((1, 70001), (1, 1), (1, 4096), (0, 12345), (0, 4096 * 3)):
        b = build_event(cfg, 0, n_bins=4096)
        ev, data, psd = upload_event(b)
        th0 = b.theta_inj.copy()
        if b.params == oracle.PARAMS_11D:
            th0[4], th0[7], th0[10] = 0.02, math.pi - 0.01, 6.25  # centres next to the wrap points
            th = _draws11(rng, n, th0)
        else:
            th = th0[:, None] + np.array([1e-3, 5e-3, 0.05, 1e-4])[:, None] * rng.standard_normal((4, n))
        w = _weights(rng, n)
        if n == 1:
            w[0] = 2.5
        note(f"update parity: config {cfg}, n {n}")
        c, cov = ev.proposal_update(dev(th), dev(w), dev(th0), cov=True)
        ev.status()
        _check(b.ev, th0, th, w, host(c), host(cov))
        # bitwise reproducible, and in place
        t0 = dev(th0)
        c2 = ev.proposal_update(dev(th), dev(w), t0)
        binding.pe_proposal_update(ev.handle, dev(th), dev(w), n, t0, t0)
        torch.cuda.synchronize()
        assert np.array_equal(host(c2), host(c)) and np.array_equal(host(t0), host(c))
        ev.close()


def test_update_edge_cases():
    torch = torch_cuda()
    b = build_event(1, 0, n_bins=4096)
    ev, data, psd = upload_event(b)
    th0 = b.theta_inj.copy()
    rng = np.random.default_rng(32)
    th = _draws11(rng, 5000, th0)
    # no positive weight: centre unchanged, covariance zero
    c, cov = ev.proposal_update(dev(th), dev(np.zeros(5000)), dev(th0), cov=True)
    assert np.array_equal(host(c), th0) and not host(cov).any()
    # zero-weight draws are never read: NaN parameters there change nothing
    w = _weights(rng, 5000, 0.5)
    th_nan = th.copy()
    th_nan[:, w == 0] = np.nan
    a = host(ev.proposal_update(dev(th), dev(w), dev(th0)))
    bb = host(ev.proposal_update(dev(th_nan), dev(w), dev(th0)))
    assert np.array_equal(a, bb)
    # n = 0
    t = torch.empty((11, 0), dtype=torch.float64, device="cuda")
    c = ev.proposal_update(t, torch.empty(0, dtype=torch.float64, device="cuda"), dev(th0))
    assert np.array_equal(host(c), th0)
    ev.close()


def test_refine_equals_the_calls_one_by_one_and_raises_ess():
    """pe_refine from a centre displaced by one proposal width (zero-noise 4-D event) equals the
    explicit sequence of single calls bit for bit, and the ESS rises from round to round."""
    torch = torch_cuda()
    b = build_event(0, 0, zero_noise=True)
    inj = b.theta_inj
    sd = np.sqrt(np.diag(np.linalg.inv(b.ev.metric(inj))))
    th0 = inj.copy()
    th0[0] += sd[0]
    th0[3] += sd[3]
    ev, data, psd = upload_event(b)
    n, rounds, seed = 8192, 3, 777
    c_r, g_r, st_r = ev.refine(dev(th0), rounds, n, seed)
    t0 = dev(th0)
    stats = []
    for r in range(rounds):
        g = ev.metric(t0)
        th, lq, lp = ev.draw(t0, g, seed, r, n)
        ll = ev.loglike(th)
        w, st = binding.weights_ess(ll, lp, lq)
        stats.append(host(st))
        t0 = ev.proposal_update(th, w, t0)
    g = ev.metric(t0)
    ev.status()
    assert np.array_equal(host(c_r), host(t0))
    assert np.array_equal(host(g_r), host(g))
    assert np.array_equal(host(st_r), np.array(stats))
    ess = host(st_r)[:, 0]
    note(f"refine ESS per round: {ess}")
    assert ess[1] > 3 * ess[0] and ess[2] > ess[0]
    ev.close()


def test_refine_argument_errors():
    torch = torch_cuda()
    b = build_event(0, 0, n_bins=1024)
    ev, data, psd = upload_event(b)
    with pytest.raises(binding.PeError):
        ev.refine(dev(b.theta_inj), 0, 16, 1)
    with pytest.raises(binding.PeError):
        ev.refine(dev(b.theta_inj), 65, 16, 1)
    ev.close()
