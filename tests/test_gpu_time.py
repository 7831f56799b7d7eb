"""GPU parity of the time-marginalised likelihood and its proposal against the oracle.

The oracle integrates the likelihood over the whole tc window with Simpson's rule at a spacing far
below the likelihood's width in tc. The library evaluates each draw at tm_points nodes spread over the
window and takes the end-corrected trapezoid rule. Here the nodes are half the narrowest width in tc
apart (1/sqrt(g_tc,tc) of the explicit-phase metric at the injection, where |Z| is largest). For a draw
whose likelihood peak lies well inside the window, that rule's error is far below the split path's
1e-3 and FP64's 1e-6. Draws whose peak a window edge cuts are integrated to O(h^4). For a Gaussian peak
cut anywhere, with the nodes half its width apart, that error is at most 0.03 in ln L_t (computed for
the rule's weights), so those draws are held to 0.05. Draws: tc at its conditional mean, and log q the
marginal over tc, against the oracle within 1e-9 proposal standard deviations and 1e-8.
"""
import math

import numpy as np
import pytest

from events import build_event
from gpu_util import dev, host, note, torch_cuda, upload_event
from paper_2410_05190_amd import binding
from tm_cases import edge_fraction, tm_event

pytestmark = pytest.mark.gpu


def test_time_marg_draw_parity():
    torch_cuda()
    b, _, g, sig_t = tm_event(1, 2, 20000)
    n = 2001
    rc, th_o, lq_o, lp_o = b.ev.draw(b.theta_inj, g, 4242, 1, n)
    assert rc == 0
    ev, data, psd = upload_event(b)
    th, lq, lp = ev.draw(dev(b.theta_inj), dev(g), 4242, 1, n)
    ev.status()
    th, lq, lp = host(th), host(lq), host(lp)
    dth = th - th_o
    for i, P in ((4, 2 * math.pi), (7, math.pi), (10, 2 * math.pi)):
        dth[i] = (dth[i] + P / 2) % P - P / 2
    sd = np.sqrt(np.diag(np.linalg.inv(g)))
    err = np.max(np.abs(dth) / sd[:, None])
    note(f"time-marginalised draws: max |dtheta|/sd {err:.2e} (tc sd {sd[9]:.2e} s), "
         f"logq {np.abs(lq - lq_o).max():.2e}")
    assert err < 1e-9
    np.testing.assert_allclose(lq, lq_o, rtol=0, atol=1e-8)
    fin = np.isfinite(lp_o)
    assert np.array_equal(fin, np.isfinite(lp))
    ev.close()


@pytest.mark.parametrize("cfg,n_bins,phase,distance,n,half_window,own",
                         [(1, 12000, None, 0, 24, 0.05, False), (2, None, None, 0, 24, 0.2, False),
                          (1, 12000, 0, 0, 24, 0.05, False), (1, 12000, 0, 0, 24, 0.05, True),
                          (2, None, None, 0, 24, 0.2, True), (2, None, None, 0, 12, 0.004, False)])
def test_time_marg_loglike_parity(cfg, n_bins, phase, distance, n, half_window, own):
    """ln L_t of proposal draws (split and FP64) against the oracle's whole-window integral. Config 1
    shape with explicit and marginalised phase; config 2 (phase marginalised, two detectors), also
    with a window of +-4 ms that cuts most draws' peaks. own: phase-marginalised events with the nodes
    half the envelope's width apart (the phase-projected metric's 1/sqrt(g_tc,tc), about four times
    the explicit-phase width), the narrowest scale of ln I0(|Z(t)|)."""
    torch_cuda()
    b, b0, g, sig_t = tm_event(cfg, 1, n_bins, phase=phase, distance=distance, half_window=half_window,
                               own_width=own)
    rc, th, lq, lp = b.ev.draw(b.theta_inj, g, 777, 0, 400)
    live = np.flatnonzero(np.isfinite(lp))[:n]
    th = np.ascontiguousarray(th[:, live])
    note(f"oracle time-marginalised loglike cfg {cfg} K {b.n_bins} ({n} draws, {b.tm_points} nodes, "
         f"tc width {sig_t:.2e} s)")
    ll_o = b.ev.loglike(th)
    edge = edge_fraction(b, b0, th, sig_t, ll_o)
    inner = edge < 1e-10
    ev, data, psd = upload_event(b)
    ll = host(ev.loglike(dev(th), precision=binding.PE_PREC_SPLIT))
    ll64 = host(ev.loglike(dev(th), precision=binding.PE_PREC_FP64))
    ev.status()
    d = np.abs(ll - ll_o)
    d64 = np.abs(ll64 - ll_o)
    note(f"  {inner.sum()} of {n} draws with their peak inside: split max |dlnL| "
         f"{d[inner].max() if inner.any() else 0:.2e}, fp64 {d64[inner].max() if inner.any() else 0:.2e}; "
         f"cut by an edge: fp64 {d64[~inner].max() if (~inner).any() else 0:.2e}; "
         f"lnL_t {ll_o.min():.1f} .. {ll_o.max():.1f}")
    assert np.all(np.isfinite(ll_o))
    if half_window >= 0.05:
        assert inner.sum() >= n * 3 // 4
    assert np.all(d[inner] <= 1e-3)
    assert np.all(d64[inner] <= 1e-6)
    assert np.all(d64[~inner] <= 5e-2) and np.all(d[~inner] <= 5e-2)
    ev.close()


def _rule(ll_nodes):
    """The library's stated rule on node values [M, n]: ln sum_m c_m L_m - ln(M - 1), with the
    end-corrected trapezoid weights 17/48, 59/48, 43/48, 49/48 at each end and 1 inside."""
    M = ll_nodes.shape[0]
    c = np.ones(M)
    for e, v in enumerate((17 / 48, 59 / 48, 43 / 48, 49 / 48)):
        c[e] = c[M - 1 - e] = v
    x = ll_nodes + np.log(c)[:, None]
    m = x.max(axis=0)
    return m + np.log(np.exp(x - m).sum(axis=0)) - math.log(M - 1)


@pytest.mark.parametrize("distance,phase", [(1, None), (0, 1)])
def test_time_marg_nodes_against_oracle_node_likelihoods(distance, phase):
    """The nodes and the rule, apart from its quadrature error: ln L_t from the library against the
    stated rule applied to the oracle's sampled-tc likelihoods at the same nodes (tc_lo + m T/(M-1)).
    With the distance marginalised too (config 2 event, +-4 ms window, 46 nodes), where the oracle's
    own window integral would take its distance integral at thousands of times per draw; and with
    the explicit phase. The whole-window integral itself is pinned by the tests above."""
    torch_cuda()
    b, b0, g, sig_t = tm_event(2, 1, None, phase=phase, distance=distance, half_window=0.004)
    rc, th, lq, lp = b.ev.draw(b.theta_inj, g, 778, 0, 64)
    live = np.flatnonzero(np.isfinite(lp))[:4]
    th = np.ascontiguousarray(th[:, live])
    M, n = b.tm_points, th.shape[1]
    nodes = b.tc_lo + (b.tc_hi - b.tc_lo) * np.arange(M) / (M - 1)
    nodes[-1] = b.tc_hi
    grid = np.repeat(th, M, axis=1)  # draw i, node m at i M + m
    grid[9] = np.tile(nodes, n)
    note(f"oracle sampled-tc likelihoods at {M} nodes x {n} draws (distance {distance}, phase {phase})")
    ll_o = _rule(b0.ev.loglike(grid).reshape(n, M).T)
    ev, data, psd = upload_event(b)
    ll = host(ev.loglike(dev(th), precision=binding.PE_PREC_SPLIT))
    ll64 = host(ev.loglike(dev(th), precision=binding.PE_PREC_FP64))
    ev.status()
    note(f"  split {np.abs(ll - ll_o).max():.2e}, fp64 {np.abs(ll64 - ll_o).max():.2e}; "
         f"lnL_t {ll_o.min():.2f} .. {ll_o.max():.2f}")
    assert np.all(np.isfinite(ll_o))
    assert np.abs(ll - ll_o).max() <= 1e-3
    assert np.abs(ll64 - ll_o).max() <= 1e-6
    ev.close()


def test_time_marg_in_a_multi_event_batch():
    """A time-marginalised event next to a plain one in one batch: both equal their single calls bit for bit."""
    torch_cuda()
    b, _, g, sig_t = tm_event(2, 3, None)
    c = build_event(2, 4)
    rc, th_b, _, _ = b.ev.draw(b.theta_inj, g, 5, 0, 700)
    rc, th_c, _, _ = c.ev.draw(c.theta_inj, c.ev.metric(c.theta_inj), 6, 0, 900)
    eb, d1, p1 = upload_event(b)
    ec, d2, p2 = upload_event(c)
    tb, tc_ = dev(th_b), dev(th_c)
    one_b = host(eb.loglike(tb))
    one_c = host(ec.loglike(tc_))
    mb, mc = (host(x) for x in binding.loglike_multi([eb, ec], [tb, tc_]))
    assert np.array_equal(one_b, mb, equal_nan=True) and np.array_equal(one_c, mc, equal_nan=True)
    with pytest.raises(binding.PeError):
        eb.loglike(tb, aux=True)
    eb.close()
    ec.close()
