"""Distance marginalisation on the GPU, through the C ABI, against the oracle: the metric with dL
projected out, draws with dL decoupled and the marginal log q, the distance-marginalised
log-likelihood on the FP64, split and relative-binning paths, and a whole chain to ESS.

Tolerances as for the sampled-distance parity tests: the metric 1e-6 of sqrt(g_ii g_jj); draws
1e-9 proposal standard deviations, log q 1e-8 (the oracle takes the marginal by inverting the
metric twice, the GPU by dropping the decoupled normal); FP64 log-likelihoods within the phase-
rounding bound of gpu_util.fp64_tol plus 1e-9 relative for the two quadratures (each ~1e-13); the
split path within 1e-3; relative binning against the oracle's relative binning to 1e-8 of |Z|."""
import math

import numpy as np
import pytest

import oracle
from events import build_event
from gpu_util import dev, fp64_tol, host, note, torch_cuda, upload_event
from paper_2410_05190_amd import binding, synth

pytestmark = pytest.mark.gpu


def _events(cfg, event, n_bins):
    b = build_event(cfg, event, n_bins=n_bins, distance=oracle.DIST_MARG)
    bs = build_event(cfg, event, n_bins=n_bins)  # the same data with dL sampled
    return b, bs


@pytest.mark.parametrize("cfg,K", [(1, 60000), (2, None)])
def test_metric_projects_out_distance(cfg, K):
    torch_cuda()
    b, _ = _events(cfg, 1, K)
    ev, data, psd = upload_event(b)
    st = b.ev.default_steps(b.theta_inj)
    for flags in (0, 1):
        go = b.ev.metric(b.theta_inj, steps=st, flags=flags)
        gg = host(ev.metric(dev(b.theta_inj), fd_step=dev(st), flags=flags))
        norm = np.sqrt(np.outer(np.abs(np.diag(go)), np.abs(np.diag(go))))
        norm[norm == 0] = 1.0
        err = np.max(np.abs(gg - go) / norm)
        note(f"distance-marginalised metric cfg={cfg} flags={flags}: {err:.2e}")
        assert err < 1e-6
        assert np.count_nonzero(gg[8]) == (1 if flags == 0 else 0)
    ev.close()


def test_draws_decouple_distance_and_report_the_marginal():
    torch_cuda()
    b, bs = _events(1, 2, 20000)
    ev, data, psd = upload_event(b)
    # a metric with distance cross terms (the sampled event's) and the event's own (decoupled)
    for g in (bs.ev.metric(b.theta_inj), b.ev.metric(b.theta_inj)):
        n = 3001
        rc, th_o, lq_o, lp_o = b.ev.draw(b.theta_inj, g, 77, 5, n)
        assert rc == 0
        th, lq, lp = ev.draw(dev(b.theta_inj), dev(g), 77, 5, n)
        ev.status()
        th, lq, lp = host(th), host(lq), host(lp)
        dth = th - th_o
        for i, P in ((4, 2 * math.pi), (7, math.pi), (10, 2 * math.pi)):
            dth[i] = (dth[i] + P / 2) % P - P / 2
        sd = np.sqrt(np.diag(np.linalg.inv(g)))
        err = np.max(np.abs(dth) / sd[:, None])
        note(f"distance-marginalised draws: max |dtheta|/sd {err:.2e}, logq {np.abs(lq - lq_o).max():.2e}")
        assert err < 1e-9
        np.testing.assert_allclose(lq, lq_o, rtol=0, atol=1e-8)
        fin = np.isfinite(lp_o)
        assert np.array_equal(fin, np.isfinite(lp))
        np.testing.assert_allclose(lp[fin], lp_o[fin], rtol=0, atol=1e-9)
    ev.close()


@pytest.mark.parametrize("cfg,K,n", [(1, 60000, 300), (2, None, 400)])
def test_loglike_parity(cfg, K, n):
    torch_cuda()
    b, _ = _events(cfg, 3, K)
    ev, data, psd = upload_event(b)
    g = b.ev.metric(b.theta_inj)
    rc, th, lq, lp = b.ev.draw(b.theta_inj, g, 31, 0, n)
    th[8, ::3] = -5.0  # the drawn distance is never used
    ll_o, zh_o = b.ev.loglike(th, n_threads=8, return_zh=True)
    f = np.isfinite(ll_o)
    note(f"distance-marginalised loglike cfg={cfg}: {f.sum()} of {n} in support, "
         f"ln L in [{ll_o[f].min():.1f}, {ll_o[f].max():.1f}]")
    tol64 = fp64_tol(b)
    ll, ax = ev.loglike(dev(th), precision=binding.PE_PREC_FP64, aux=True)
    ll, ax = host(ll), host(ax)
    assert np.array_equal(np.isfinite(ll), f)
    np.testing.assert_allclose(ax[f], zh_o[f], rtol=1e-10, atol=1e-10 * np.abs(zh_o[f]).max())
    d64 = np.abs(ll[f] - ll_o[f])
    assert np.all(d64 <= tol64 + 1e-9 * np.maximum(1.0, np.abs(ll_o[f])))
    ls = host(ev.loglike(dev(th), precision=binding.PE_PREC_SPLIT))
    ds = np.abs(ls[f] - ll_o[f])
    note(f"  FP64 max |dlnL| {d64.max():.2e} (bound {tol64:.1e}), split {ds.max():.2e}")
    assert ds.max() <= 1e-3
    # relative binning about the injection, against the oracle's relative binning
    ev.relbin_setup(dev(b.theta_inj), 0.03)
    e = ev.relbin_edges()
    lr, ar = ev.loglike(dev(th), precision=binding.PE_PREC_RELBIN, aux=True)
    lr, ar = host(lr), host(ar)
    lr_o, zr_o = b.ev.relbin_loglike(b.theta_inj, e, th, return_zh=True)
    scale = np.abs(zr_o[f]).max()
    np.testing.assert_allclose(ar[f], zr_o[f], rtol=0, atol=1e-11 * scale)
    np.testing.assert_allclose(lr[f], lr_o[f], rtol=0, atol=1e-8 * scale)
    ev.status()
    ev.close()


def test_batch_mixes_marginalised_and_sampled_distance():
    """One pe_loglike_multi call over a distance-marginalised event and a sampled-distance event
    gives each the results of its own single-event call, bit for bit."""
    torch_cuda()
    b, bs = _events(1, 4, 30000)
    evd, dd, pd = upload_event(b)
    evs, ds, ps = upload_event(bs)
    g = bs.ev.metric(bs.theta_inj)
    rc, th, lq, lp = bs.ev.draw(bs.theta_inj, g, 9, 0, 500)
    t = dev(th)
    for prec in (binding.PE_PREC_SPLIT, binding.PE_PREC_FP64):
        lls = binding.loglike_multi([evd, evs], [t, t], precision=prec)
        assert np.array_equal(host(lls[0]), host(evd.loglike(t, precision=prec)))
        assert np.array_equal(host(lls[1]), host(evs.loglike(t, precision=prec)))
        assert not np.array_equal(host(lls[0]), host(lls[1]))
    evd.close()
    evs.close()


def test_loglike_split_parity_c1_full_size_sampled():
    """Config 1 at full size in the benchmark's launch shape (65 536 draws, 519 168 bins, split
    precision) with the distance marginalised: every draw through the GPU, sampled draws (the
    lowest and highest cuts and 40 at random) through the oracle."""
    torch_cuda()
    b = build_event(1, 0, distance=oracle.DIST_MARG)
    N = 65536
    g = b.ev.metric(b.theta_inj)
    rc, th, lq, lp = b.ev.draw(b.theta_inj, g, synth.draw_seed(1, 0), 0, N)
    assert rc == 0
    ev, data, psd = upload_event(b)
    ev.reserve(N)
    note("gpu split distance-marginalised loglike c1 full size")
    ll_s = host(ev.loglike(dev(th), precision=binding.PE_PREC_SPLIT))
    ev.status()
    rng = np.random.default_rng(5)
    live = np.flatnonzero(np.isfinite(ll_s))
    pick = np.sort(np.concatenate([rng.choice(live, 40, replace=False), live[:4], live[-4:]]))
    note(f"oracle loglike on {pick.size} sampled draws")
    ll_o = b.ev.loglike(th[:, pick], n_threads=8)
    d = np.abs(ll_s[pick] - ll_o)
    note(f"  c1 full distance-marginalised split max |dlnL| = {d.max():.3e}")
    assert d.max() <= 1e-3
    assert np.array_equal(np.isfinite(lp), np.isfinite(ll_s))
    ev.close()


def test_chain_to_ess_within_tolerance():
    """Metric, draws, split log-likelihoods and weights of a distance-marginalised event: ESS and
    the normalised weights agree with the oracle's chain within 1e-3 relative."""
    torch_cuda()
    b, _ = _events(1, 5, 60000)
    ev, data, psd = upload_event(b)
    go = b.ev.metric(b.theta_inj)
    n = 2000
    rc, th_o, lq_o, lp_o = b.ev.draw(b.theta_inj, go, 5150, 2, n)
    ll_o = b.ev.loglike(th_o, n_threads=8)
    w_o, st_o = oracle.weights_ess(ll_o, lp_o, lq_o)
    th, lq, lp = ev.draw(dev(b.theta_inj), dev(go), 5150, 2, n)
    ll = ev.loglike(th, precision=binding.PE_PREC_SPLIT)
    w, st = binding.weights_ess(ll, lp, lq)
    ev.status()
    w, st = host(w), host(st)
    note(f"distance-marginalised chain: ESS gpu {st[0]:.4f} oracle {st_o[0]:.4f}")
    assert st[0] == pytest.approx(st_o[0], rel=1e-3)
    big = w_o > 1e-6 * w_o.max()
    np.testing.assert_allclose(w[big], w_o[big], rtol=1e-3)
    ev.close()


def test_descriptor_checks():
    torch = torch_cuda()
    b = build_event(0, 0, n_bins=2048)
    data = torch.from_numpy(np.ascontiguousarray(b.data)).cuda()
    psd = torch.from_numpy(np.ascontiguousarray(b.psd)).cuda()
    from gpu_util import desc_kwargs
    kw = desc_kwargs(b)
    kw["distance"] = binding.PE_DIST_MARG  # 4-D has no distance
    with pytest.raises(binding.PeError):
        binding.Event(data, psd, **kw)
    kw["distance"] = 7
    with pytest.raises(binding.PeError):
        binding.Event(data, psd, **kw)


@pytest.mark.parametrize("snr,zero_noise", [(60.0, True), (8.0, False)])
def test_loud_and_quiet_events_and_a_draw_without_bins(snr, zero_noise):
    """The integral's regimes: a loud noise-free event (narrow peak in distance) and a quiet one
    (prior-dominated, heavy tail), FP64 path against the oracle; a draw whose ISCO cut lies below the
    band has Z = H = 0, so its likelihood is 1 at every distance and ln L_D = 0."""
    torch_cuda()
    b = build_event(1, 6, n_bins=40000, zero_noise=zero_noise, snr=snr, distance=oracle.DIST_MARG)
    ev, data, psd = upload_event(b)
    g = b.ev.metric(b.theta_inj)
    rc, th, lq, lp = b.ev.draw(b.theta_inj, g, 3, 1, 120)
    th[:, 0] = b.theta_inj
    th[:, 1] = b.theta_inj
    th[0, 1] = 400.0  # ISCO below the band's 20 Hz: no bin below the cut
    ll_o = b.ev.loglike(th, n_threads=8)
    ll = host(ev.loglike(dev(th), precision=binding.PE_PREC_FP64))
    f = np.isfinite(ll_o)
    assert np.array_equal(np.isfinite(ll), f)
    assert ll[1] == 0.0 and abs(ll_o[1]) < 1e-13
    tol = fp64_tol(b) + 1e-9 * np.maximum(1.0, np.abs(ll_o[f]))
    d = np.abs(ll[f] - ll_o[f])
    note(f"distance-marginalised SNR {snr}: ln L_D at the injection {ll_o[0]:.3f}, max |dlnL| {d.max():.2e}")
    assert np.all(d <= tol)
    ev.close()


@pytest.mark.parametrize("n", [1, 63, 65, 257])
def test_ragged_batches(n):
    """Batches that end inside a workgroup of the distance kernel (64 draws per block, four lanes
    each) and of the relative-binning kernel (64 draws per block): every path against the oracle."""
    torch_cuda()
    b, _ = _events(1, 7, 20000)
    ev, data, psd = upload_event(b)
    g = b.ev.metric(b.theta_inj)
    rc, th, lq, lp = b.ev.draw(b.theta_inj, g, 77, 3, n)
    ll_o = b.ev.loglike(th, n_threads=8)
    f = np.isfinite(ll_o)
    ll64 = host(ev.loglike(dev(th), precision=binding.PE_PREC_FP64))
    ls = host(ev.loglike(dev(th), precision=binding.PE_PREC_SPLIT))
    assert np.array_equal(np.isfinite(ll64), f) and np.array_equal(np.isfinite(ls), f)
    tol = fp64_tol(b) + 1e-9 * np.maximum(1.0, np.abs(ll_o[f]))
    assert np.all(np.abs(ll64[f] - ll_o[f]) <= tol)
    assert np.all(np.abs(ls[f] - ll_o[f]) <= 1e-3)
    ev.relbin_setup(dev(b.theta_inj), 0.03)
    e = ev.relbin_edges()
    lr = host(ev.loglike(dev(th), precision=binding.PE_PREC_RELBIN))
    lr_o, zr_o = b.ev.relbin_loglike(b.theta_inj, e, th, return_zh=True)
    assert np.array_equal(np.isfinite(lr), f)
    if f.any():
        np.testing.assert_allclose(lr[f], lr_o[f], rtol=0, atol=1e-8 * np.abs(zr_o[f]).max())
    ev.close()
