"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle on the same
seeded inputs (element by element), plus edge cases and error paths.

Tolerances:
  - FP64 path: per draw |d ln L| and |d Z| within the rounding model
    16 u (|sum_k t_k M_k| + 6 sqrt(sum_k |t_k|^2 M_k^2)) and the worst case 32 u sum_k |t_k| M_k
    (gpu_util.fp64_draw_bounds: both sides round bin k's phase differently by at most ~16 u M_k,
    M_k the magnitude of the phase's terms there); H within 1e-12 relative (a sum of positive
    terms); where the per-draw sums are too slow to form, the band-edge bound
    32 u Phi_N(f_lo) sum_k |t_k| of gpu_util.fp64_tol;
  - split path: |d ln L| <= 1e-3 absolute (the stated bound); the internal target is 2.5e-4,
    which keeps ESS and the weights within 1e-3 relative;
  - metric: 1e-6 of sqrt(g_ii g_jj) (finite differences of phases computed in two different
    algebraic forms);
  - draws: uniforms bit-exact; theta within 1e-9 proposal standard deviations (and in the
    whitened coordinates L^T dtheta); log q 1e-8; weights/ESS 1e-12 relative on identical inputs.
"""
import math

import numpy as np
import pytest

import oracle
from events import build_event
from gpu_util import desc_kwargs, dev, fp64_draw_bounds, fp64_tol, host, note, torch_cuda, upload_event
from paper_2410_05190_amd import binding
from paper_2410_05190_amd import synth

pytestmark = pytest.mark.gpu


def _wave_extremes(b, th, live, n):
    """n of the live draws: the draws ordered by cut as the hot loop's plan orders them (by the
    bin count below f_isco), cut into waves of 64, and the lowest- and highest-cut draw of n/2
    waves spread evenly over them: the waves whose lanes stop at different bins, so that the
    masked tail of every kind of wave is checked."""
    fis = np.array([b.ev.source(th[:, i])[1].fisco for i in live])
    kc = np.clip(np.ceil((fis - b.f_lo) / b.df), 0, b.n_bins)
    order = live[np.argsort(kc, kind="stable")]
    waves = [order[s:s + 64] for s in range(0, order.size, 64)]
    sel = np.linspace(0, len(waves) - 1, min(n // 2, len(waves))).round().astype(int)
    pick = np.unique(np.concatenate([[waves[w][0], waves[w][-1]] for w in np.unique(sel)]))
    return np.sort(pick)


def _oracle_draws(b, n, seed=11, stream=0, g=None):
    g = b.ev.metric(b.theta_inj) if g is None else g
    rc, th, lq, lp = b.ev.draw(b.theta_inj, g, seed, stream, n)
    assert rc == 0
    return g, th, lq, lp


def test_library_loads_on_gpu():
    torch = torch_cuda()
    binding.load()
    assert binding.pe_dim(binding.PE_PARAMS_11D) == 11
    assert torch.cuda.device_count() >= 1


def test_uniforms_bit_exact():
    torch = torch_cuda()
    for seed, stream, n, npairs in ((1, 0, 1000, 6), (2 ** 63 + 12345, 77, 257, 2), (0, 2 ** 32 - 1, 3, 1)):
        u = torch.empty((n, npairs, 2), dtype=torch.float64, device="cuda")
        binding.pe_rng_uniforms(seed, stream, n, npairs, u)
        want = oracle.uniforms(seed, stream, n, npairs)
        np.testing.assert_array_equal(host(u), want)


@pytest.mark.parametrize("cfg,K", [(0, 31488), (1, 30000), (1, 519168), (2, 8032)])
def test_waveform_parity(cfg, K):
    torch = torch_cuda()
    note(f"waveform cfg={cfg} K={K}")
    b = build_event(cfg, 0, n_bins=K)
    d = binding.make_desc(b.n_det, b.n_bins, data_dtype=binding.PE_C128,
                          psd_dtype=binding.PE_F64 if b.psd.dtype == np.float64 else binding.PE_F32,
                          **desc_kwargs(b))
    h = torch.empty((b.n_det, b.n_bins, 2), dtype=torch.float64, device="cuda")
    snr2 = torch.zeros(1, dtype=torch.float64, device="cuda")
    psd = torch.from_numpy(b.psd).cuda()
    binding.pe_waveform(d, dev(b.theta_inj), psd, h, snr2)
    hg = host(h)
    hg = hg[..., 0] + 1j * hg[..., 1]
    ho = b.ev.waveform(b.theta_inj)
    scale = np.abs(ho).max()
    err = np.abs(hg - ho).max() / scale
    note(f"  max |dh|/max|h| = {err:.3e}")
    assert err < 1e-9
    want = sum(b.ev.inner(i, ho, ho) for i in range(b.n_det))
    assert host(snr2)[0] == pytest.approx(want, rel=1e-10)


def test_loglike_fp64_parity_c0_full():
    """Config 0 at full size: 4096 draws, 31488 bins, FP64 path."""
    torch_cuda()
    b = build_event(0, 0)
    g, th, lq, lp = _oracle_draws(b, 4096)
    note("oracle loglike c0 (4096 draws x 31488 bins)")
    ll_o, zh_o = b.ev.loglike(th, return_zh=True)
    ev, data, psd = upload_event(b)
    ll, aux = ev.loglike(dev(th), precision=binding.PE_PREC_FP64, aux=True)
    ev.status()
    ll = host(ll)
    aux = host(aux)
    fin = np.isfinite(ll_o)
    assert np.array_equal(fin, np.isfinite(ll))
    assert fin.sum() > 100 and (~fin).sum() > 100  # both live and out-of-support draws present
    d = np.abs(ll[fin] - ll_o[fin])
    bw, bm = fp64_draw_bounds(b, th[:, fin])
    dz = np.hypot(aux[fin, 0] - zh_o[fin, 0], aux[fin, 1] - zh_o[fin, 1])
    e = np.maximum(d, dz)
    note(f"  c0 fp64 max |dlnL| = {d.max():.3e}, max |dZ| = {dz.max():.3e}; largest error / model bound "
         f"{np.max(e / bm):.3f}, / worst case {np.max(e / bw):.4f} (model {bm.min():.2e} .. {bm.max():.2e}; "
         f"band-edge {fp64_tol(b):.2e}; live {fin.sum()})")
    assert np.all(e <= bm) and np.all(e <= bw)
    np.testing.assert_allclose(aux[fin, 2], zh_o[fin, 2], rtol=1e-12, atol=0)


@pytest.mark.parametrize("K,n,event", [(40000, 1500, 0), (100003, 777, 1)])
def test_loglike_split_and_fp64_parity_c1_small(K, n, event):
    """Config-1 shape (3 detectors, 11-D, complex64/FP32 storage) on a truncated grid, ragged sizes."""
    torch_cuda()
    b = build_event(1, event, n_bins=K)
    g, th, lq, lp = _oracle_draws(b, n, seed=5 + event)
    note(f"oracle loglike c1 K={K} n={n}")
    ll_o, zh_o = b.ev.loglike(th, return_zh=True)
    ev, data, psd = upload_event(b)
    ths = dev(th)
    ll_s = host(ev.loglike(ths, precision=binding.PE_PREC_SPLIT))
    ll_d = host(ev.loglike(ths, precision=binding.PE_PREC_FP64))
    ev.status()
    fin = np.isfinite(ll_o)
    assert np.array_equal(fin, np.isfinite(ll_s)) and np.array_equal(fin, np.isfinite(ll_d))
    ds = np.abs(ll_s[fin] - ll_o[fin]).max()
    d64 = np.abs(ll_d[fin] - ll_o[fin])
    bw, bm = fp64_draw_bounds(b, th[:, fin])
    note(f"  split max |dlnL| = {ds:.3e}; fp64 max |dlnL| = {d64.max():.3e}, largest error / model bound "
         f"{np.max(d64 / bm):.3f}, / worst case {np.max(d64 / bw):.4f} (model {bm.min():.2e} .. {bm.max():.2e}; "
         f"band-edge {fp64_tol(b):.2e}); live {fin.sum()}/{n}")
    assert np.all(d64 <= bm) and np.all(d64 <= bw)
    assert ds <= 1e-3


def test_loglike_split_parity_c1_full_size_sampled():
    """Config 1 at full size in the benchmark's launch shape (65536 draws, 519168 bins), checked
    on draws sampled for the oracle."""
    torch_cuda()
    b = build_event(1, 0)
    N = 65536
    g, th, lq, lp = _oracle_draws(b, N, seed=synth.draw_seed(1, 0))
    ev, data, psd = upload_event(b)
    ev.reserve(N)
    note("gpu split loglike c1 full size")
    ll_s = host(ev.loglike(dev(th), precision=binding.PE_PREC_SPLIT))
    ev.status()
    live = np.flatnonzero(np.isfinite(ll_s))
    pick = _wave_extremes(b, th, live, 1024)
    note(f"oracle loglike on {pick.size} sampled draws (the lowest and highest cut of 512 waves)")
    ll_o = b.ev.loglike(th[:, pick])
    d = np.abs(ll_s[pick] - ll_o)
    note(f"  c1 full split max |dlnL| = {d.max():.3e}")
    assert d.max() <= 1e-3
    # support decisions are exact for every draw (the oracle's prior is finite exactly on the support)
    assert np.array_equal(np.isfinite(lp), np.isfinite(ll_s))


def test_metric_parity():
    torch = torch_cuda()
    for cfg, K in ((0, 31488), (1, 60000), (2, 8032)):
        b = build_event(cfg, 1, n_bins=K)
        ev, data, psd = upload_event(b)
        st = b.ev.default_steps(b.theta_inj)
        for flags in (0, 1):
            go = b.ev.metric(b.theta_inj, steps=st, flags=flags)
            gg = host(ev.metric(dev(b.theta_inj), fd_step=dev(st), flags=flags))
            gd = host(ev.metric(dev(b.theta_inj), fd_step=None, flags=flags))
            norm = np.sqrt(np.outer(np.abs(np.diag(go)), np.abs(np.diag(go))))
            norm[norm == 0] = 1.0
            e1 = np.max(np.abs(gg - go) / norm)
            e2 = np.max(np.abs(gd - go) / norm)
            note(f"metric cfg={cfg} flags={flags}: explicit steps {e1:.2e}, default steps {e2:.2e}")
            assert e1 < 1e-6 and e2 < 1e-6
        ev.status()


def test_draw_parity():
    torch = torch_cuda()
    for cfg in (0, 1):
        b = build_event(cfg, 2, n_bins=20000)
        g = b.ev.metric(b.theta_inj)
        n = 3001
        rc, th_o, lq_o, lp_o = b.ev.draw(b.theta_inj, g, 987654321, 3, n)
        ev, data, psd = upload_event(b)
        th, lq, lp = ev.draw(dev(b.theta_inj), dev(g), 987654321, 3, n)
        ev.status()
        th, lq, lp = host(th), host(lq), host(lp)
        dth = th - th_o
        if cfg == 1:  # periodic coordinates compared on the circle
            for i, P in ((4, 2 * math.pi), (7, math.pi), (10, 2 * math.pi)):
                dth[i] = (dth[i] + P / 2) % P - P / 2
        sd = np.sqrt(np.diag(np.linalg.inv(g)))
        err = np.max(np.abs(dth) / sd[:, None])
        white = np.max(np.abs(np.linalg.cholesky(g).T @ dth))
        note(f"draws cfg={cfg}: max |dtheta|/sd {err:.2e}, whitened {white:.2e}, logq {np.abs(lq - lq_o).max():.2e}")
        assert err < 1e-9 and white < 1e-9
        np.testing.assert_allclose(lq, lq_o, rtol=0, atol=1e-8)
        fin = np.isfinite(lp_o)
        assert np.array_equal(fin, np.isfinite(lp))
        # theta agrees to ~1e-11 sd, so ln dL, ln cos(dec), ln sin(iota) agree to ~1e-11
        np.testing.assert_allclose(lp[fin], lp_o[fin], rtol=0, atol=1e-9)


@pytest.mark.parametrize("cfg,couple,shift", [(1, "none", False), (1, "weak", False), (1, "weak", True),
                                              (2, "weak", True), (1, "strong", True)])
def test_draw_parity_image_sum(cfg, couple, shift):
    """Broad periodic coordinates (ra, psi, phic with unit precision, so that neighbouring images
    carry weight), with and without couplings between them, and with the centre several periods
    outside [0, P) (the images are taken about the wrapped centre). Weak couplings keep every pair
    term |g_pq P_p P_q| within 50, where the draw kernel sums the 125 images as products of
    per-coordinate and pair factors; strong ones take the image-by-image sum. Config 2's events are
    phase-marginalised: phic is left out of log q. log q and theta against the oracle."""
    torch_cuda()
    b = build_event(cfg, 2, n_bins=20000 if cfg == 1 else None)
    g = np.diag(np.diag(b.ev.metric(b.theta_inj)))
    pidx = [4, 7, 10]
    c = {"none": (0.0, 0.0), "weak": (0.3, 0.5), "strong": (0.9, 0.0)}[couple]
    block = np.array([[1.0, c[0], 0.0], [c[0], 1.0, c[1]], [0.0, c[1], 1.0]])
    if couple == "strong":
        block = block * 10.0
    g[np.ix_(pidx, pidx)] = block
    per = np.array([2 * math.pi, math.pi, 2 * math.pi])
    gam = np.abs(block * np.outer(per, per) - np.diag(np.diag(block * np.outer(per, per))))
    assert (gam.max() <= 50.0) == (couple != "strong")
    th0 = b.theta_inj.copy()
    if shift:
        th0[4] += 3 * per[0]
        th0[7] -= 2 * per[1]
        th0[10] += per[2]
    n = 4001
    rc, th_o, lq_o, lp_o = b.ev.draw(th0, g, 31337, 2, n)
    assert rc == 0
    ev, data, psd = upload_event(b)
    th, lq, lp = ev.draw(dev(th0), dev(g), 31337, 2, n)
    ev.status()
    th, lq, lp = host(th), host(lq), host(lp)
    dth = th - th_o
    for i, P in zip(pidx, per):
        dth[i] = (dth[i] + P / 2) % P - P / 2
    sd = np.sqrt(np.diag(np.linalg.inv(g)))
    err = np.max(np.abs(dth) / sd[:, None])
    note(f"image sum cfg {cfg} couplings {couple} shifted {shift}: max |dtheta|/sd {err:.2e}, "
         f"logq {np.abs(lq - lq_o).max():.2e}")
    assert err < 1e-9
    np.testing.assert_allclose(lq, lq_o, rtol=0, atol=1e-8)
    fin = np.isfinite(lp_o)
    assert np.array_equal(fin, np.isfinite(lp))
    np.testing.assert_allclose(lp[fin], lp_o[fin], rtol=0, atol=1e-9)


def test_weights_parity_and_identities():
    torch = torch_cuda()
    rng = np.random.default_rng(9)
    for n in (1, 1000, 65536, 262144 + 3):
        ll = rng.normal(0, 4, n)
        ll[rng.random(n) < 0.3] = -np.inf
        lp = rng.normal(0, 1, n)
        lq = rng.normal(0, 1, n)
        w, st = binding.weights_ess(dev(ll), dev(lp), dev(lq))
        w_o, st_o = oracle.weights_ess(ll, lp, lq)
        np.testing.assert_allclose(host(w), w_o, rtol=1e-12, atol=1e-300)
        np.testing.assert_allclose(host(st), st_o, rtol=1e-12)
    # equal weights: ESS = N exactly; all -inf: ESS = 0
    w, st = binding.weights_ess(dev(np.full(4096, -2.0)), dev(np.zeros(4096)), dev(np.zeros(4096)))
    assert host(st)[0] == 4096.0
    w, st = binding.weights_ess(dev(np.full(10, -np.inf)), dev(np.zeros(10)), dev(np.zeros(10)))
    s = host(st)
    assert s[0] == 0 and s[3] == 0 and s[1] == -np.inf and np.all(host(w) == 0)
    # a NaN or +inf log-weight: every estimate NaN, the finite count kept (as the oracle); the bad
    # entry sits in the second of three weight blocks
    rng = np.random.default_rng(12)
    for bad in (np.nan, np.inf):
        ll = rng.normal(size=9000)
        ll[[5, 6000]] = [-np.inf, bad]
        w, st = binding.weights_ess(dev(ll), dev(np.zeros(9000)), dev(np.zeros(9000)))
        w_o, st_o = oracle.weights_ess(ll, np.zeros(9000), np.zeros(9000))
        s = host(st)
        assert np.all(np.isnan(host(w))) and np.all(np.isnan(s[:3])) and s[3] == st_o[3] == 8998


def test_split_weights_and_ess_within_tolerance():
    """Whole chain at config-1 shape: ESS and normalised weights from the split path agree with the
    oracle's within 1e-3 relative (on weights above 1e-6 of the largest)."""
    torch = torch_cuda()
    b = build_event(1, 3, n_bins=60000)
    g = b.ev.metric(b.theta_inj)
    n = 2000
    seed = 424242
    rc, th_o, lq_o, lp_o = b.ev.draw(b.theta_inj, g, seed, 1, n)
    ll_o = b.ev.loglike(th_o)
    w_o, st_o = oracle.weights_ess(ll_o, lp_o, lq_o)
    ev, data, psd = upload_event(b)
    th, lq, lp = ev.draw(dev(b.theta_inj), dev(g), seed, 1, n)
    ll = ev.loglike(dev(th_o), precision=binding.PE_PREC_SPLIT)
    w, st = binding.weights_ess(ll, lp, lq)
    ev.status()
    w, st = host(w), host(st)
    note(f"ESS gpu {st[0]:.6f} oracle {st_o[0]:.6f}")
    assert st[0] == pytest.approx(st_o[0], rel=1e-3)
    big = w_o > 1e-6 * w_o.max()
    np.testing.assert_allclose(w[big], w_o[big], rtol=1e-3)


def test_edge_cases_and_determinism():
    torch = torch_cuda()
    b = build_event(1, 0, n_bins=5000)
    ev, data, psd = upload_event(b)
    # n = 0 is a no-op
    e = torch.empty((11, 0), dtype=torch.float64, device="cuda")
    binding.pe_loglike_batch(ev.handle, e, 0, binding.PE_PREC_SPLIT, torch.empty(0, dtype=torch.float64,
                                                                                  device="cuda"))
    # single draw at the injection
    th1 = b.theta_inj[:, None].copy()
    tol64 = fp64_tol(b)
    for prec in (binding.PE_PREC_SPLIT, binding.PE_PREC_FP64):
        ll = host(ev.loglike(dev(th1), precision=prec))
        assert abs(ll[0] - b.ev.loglike(th1)[0]) < (1e-3 if prec == binding.PE_PREC_SPLIT else tol64)
    # every draw out of support
    bad = np.repeat(b.theta_inj[:, None], 300, axis=1)
    bad[1] = 1.5
    ll = host(ev.loglike(dev(bad)))
    assert np.all(ll == -np.inf)
    # bitwise reproducible
    g = b.ev.metric(b.theta_inj)
    rc, th, lq, lp = b.ev.draw(b.theta_inj, g, 5, 0, 1000)
    a1 = host(ev.loglike(dev(th)))
    a2 = host(ev.loglike(dev(th)))
    assert np.array_equal(a1, a2, equal_nan=True)
    ev.status()


@pytest.mark.parametrize("cfg,n_det,K", [(1, 4, 20000), (1, 3, 17), (1, 2, 1), (0, None, 6000), (2, 1, None)])
def test_edge_shapes_parity(cfg, n_det, K):
    """Shapes at the edges of the kernels' assumptions: four detectors (the maximum), a band shorter
    than one FP32 block, a single bin, the 4-D parameter set through the split path, one detector.
    Split within 1e-3 and FP64 within its derived bound of the oracle, on every draw."""
    torch_cuda()
    b = build_event(cfg, 0, n_det=n_det, n_bins=K)
    # a diagonal proposal (the metric of a one-bin band is singular): 1% of each coordinate
    scale = 0.01 * np.maximum(np.abs(b.theta_inj), 0.05)
    rc, th, lq, lp = b.ev.draw(b.theta_inj, np.diag(1.0 / scale ** 2), 77, 0, 600)
    assert rc == 0
    ev, data, psd = upload_event(b)
    ll_o = np.full(th.shape[1], -np.inf)
    live = np.flatnonzero(np.isfinite(lp))
    ll_o[live] = b.ev.loglike(th[:, live])
    tol = fp64_tol(b)
    for prec, bound in ((binding.PE_PREC_SPLIT, 1e-3), (binding.PE_PREC_FP64, max(tol, 1e-12))):
        ll = host(ev.loglike(dev(th), precision=prec))
        assert np.array_equal(np.isfinite(ll), np.isfinite(ll_o))
        d = np.abs(ll[live] - ll_o[live]) if live.size else np.zeros(1)
        note(f"edge cfg {cfg} n_det {b.n_det} K {b.n_bins} prec {prec}: max |dlnL| {d.max():.2e} (bound {bound:.1e})")
        assert d.max() <= bound
    ev.status()


def test_event_input_errors():
    torch = torch_cuda()
    b = build_event(1, 0, n_bins=2000)
    psd = b.psd.copy()
    psd[0, 17] = 0.0
    data = torch.from_numpy(b.data).cuda()
    with pytest.raises(binding.PeError) as ei:
        binding.Event(data, torch.from_numpy(psd).cuda(), **desc_kwargs(b))
    assert ei.value.status == 1
    dat = b.data.copy()
    dat[2, 5] = np.nan
    with pytest.raises(binding.PeError) as ei:
        binding.Event(torch.from_numpy(dat).cuda(), torch.from_numpy(b.psd).cuda(),
                      **desc_kwargs(b))
    assert ei.value.status == 5
    ev, d_, p_ = upload_event(b)
    gbad = np.eye(11)
    gbad[3, 3] = -1.0
    th, lq, lp = ev.draw(dev(b.theta_inj), dev(gbad), 1, 0, 100)
    with pytest.raises(binding.PeError) as ei:
        ev.status()
    assert ei.value.status == 4
    assert np.all(host(lp) == -np.inf)
    ev.status()  # cleared


def test_result_is_the_same_alone_and_in_the_mix():
    """A draw's log-likelihood does not depend on the order of the draws of its batch (which
    changes the cut buckets, the waves and their masked tails, and the work items): bitwise
    identical, in both precisions. Nor on the other events of a multi-event batch. The frequency
    decomposition follows the event's own live draws (their number and largest cut), so a subset
    of them agrees within the rounding of the FP32 (split) or FP64 sums, not bit for bit."""
    torch = torch_cuda()
    b = build_event(1, 1, n_bins=60000)
    g = b.ev.metric(b.theta_inj)
    rc, th, lq, lp = b.ev.draw(b.theta_inj, g, 99, 0, 5000)
    ev, data, psd = upload_event(b)
    other = build_event(1, 2, n_bins=45000)
    rc, th_o, _, _ = other.ev.draw(other.theta_inj, other.ev.metric(other.theta_inj), 7, 0, 3000)
    ev_o, data_o, psd_o = upload_event(other)
    pick = [3, 17, 256, 4095, 4999]
    perm = np.random.default_rng(1).permutation(th.shape[1])
    tol64 = fp64_tol(b)
    for prec in (binding.PE_PREC_SPLIT, binding.PE_PREC_FP64):
        full = host(ev.loglike(dev(th), precision=prec))
        rev = host(ev.loglike(dev(th[:, ::-1].copy()), precision=prec))[::-1]
        shuf = np.empty_like(full)
        shuf[perm] = host(ev.loglike(dev(th[:, perm].copy()), precision=prec))
        assert np.array_equal(full, rev) and np.array_equal(full, shuf)
        alone_o = host(ev_o.loglike(dev(th_o), precision=prec))
        mix, mix_o = binding.loglike_multi([ev, ev_o], [dev(th), dev(th_o)], precision=prec)
        assert np.array_equal(full, host(mix)) and np.array_equal(alone_o, host(mix_o))
        few = host(ev.loglike(dev(th[:, pick].copy()), precision=prec))
        ones = np.array([host(ev.loglike(dev(th[:, i:i + 1].copy()), precision=prec))[0] for i in pick])
        fin = np.isfinite(full[pick])
        d_few = np.max(np.abs(few - full[pick])[fin], initial=0.0)
        d_one = np.max(np.abs(ones - full[pick])[fin], initial=0.0)
        note(f"subset prec={prec}: max |d lnL| few {d_few:.1e} alone {d_one:.1e}")
        bound = 2.5e-4 if prec == binding.PE_PREC_SPLIT else 2 * tol64
        assert d_few <= bound and d_one <= bound
        assert np.array_equal(np.isfinite(few), np.isfinite(full[pick]))
    ev.status()
    ev_o.status()


def test_multi_event_batch_config2():
    """Config 2 (BBH, 2 detectors, K = 8032): events of uneven draw counts (0, 1, a few, thousands,
    one with every draw out of support) plus a 3-detector event in one pe_loglike_multi call:
    every event's results equal its own pe_loglike_batch bit for bit, and the oracle within the
    bounds of each precision."""
    torch = torch_cuda()
    counts = [0, 1, 300, 5000, 17, 2000, 64]
    built, evs, keep, thetas = [], [], [], []
    for e, n in enumerate(counts):
        b = build_event(2, e, n_det=3 if e == 6 else None)
        g = b.ev.metric(b.theta_inj)
        rc, th, lq, lp = b.ev.draw(b.theta_inj, g, synth.draw_seed(2, e), 0, max(n, 1))
        th = th[:, :n].copy()
        if e == 4:
            th[1] = 1.5  # q > 1: outside the support
        ev, data, psd = upload_event(b)
        built.append(b)
        evs.append(ev)
        keep.append((data, psd))
        thetas.append(th)
    rng = np.random.default_rng(2)
    for prec in (binding.PE_PREC_SPLIT, binding.PE_PREC_FP64):
        lls, axs = binding.loglike_multi(evs, [dev(t) for t in thetas], precision=prec, aux=True)
        for e, (b, ev, th) in enumerate(zip(built, evs, thetas)):
            ll = host(lls[e])
            if th.shape[1] == 0:
                assert ll.size == 0
                continue
            one, ax1 = ev.loglike(dev(th), precision=prec, aux=True)
            assert np.array_equal(ll, host(one)) and np.array_equal(host(axs[e]), host(ax1))
            if e == 4:
                assert np.all(ll == -np.inf) and np.all(host(axs[e]) == 0.0)
                continue
            live = np.flatnonzero(np.isfinite(ll))
            if live.size == 0:
                continue
            pick = live if live.size <= 64 else np.sort(rng.choice(live, 64, replace=False))
            ll_o = b.ev.loglike(th[:, pick])
            d = np.abs(ll[pick] - ll_o)
            bound = 1e-3 if prec == binding.PE_PREC_SPLIT else fp64_tol(b)
            note(f"c2 multi event {e} n={th.shape[1]} prec={prec}: max |d lnL| {d.max():.2e} (bound {bound:.1e})")
            assert d.max() <= bound
    for ev in evs:
        ev.status()
    with pytest.raises(binding.PeError):
        binding.loglike_multi([evs[2], evs[2]], [dev(thetas[2]), dev(thetas[2])])


def test_batch_run_whole_path_equals_single_event_calls():
    """pe_batch_run over events of different shapes (1, 2 and 3 detectors; 4-D and 11-D; sizes
    from 0 to thousands of draws) runs prep, metric, draws, log-likelihoods and weights as one
    set of launches per stage; every output equals the single-event calls bit for bit."""
    torch = torch_cuda()
    f64 = dict(dtype=torch.float64, device="cuda")
    shapes = [(2, 0, None, 900), (2, 1, 1, 0), (2, 2, 3, 2500), (0, 0, None, 700), (1, 3, None, 1200),
              (2, 4, None, 1)]
    evs, items, single = [], [], []
    for cfg, e, nd, n in shapes:
        b = build_event(cfg, e, n_det=nd, n_bins=6000 if cfg == 1 else None)
        ev, data, psd = upload_event(b)
        D = ev.dim
        th0 = dev(b.theta_inj)
        bufs = {k: torch.full(shape, float("nan"), **f64) for k, shape in
                [("g", (D, D)), ("theta", (D, max(n, 1))), ("logq", (max(n, 1),)), ("logprior", (max(n, 1),)),
                 ("loglike", (max(n, 1),)), ("aux", (max(n, 1), 3)), ("w", (max(n, 1),)), ("stats", (4,))]}
        seed = 1234 + 10 * cfg + e
        items.append(binding.make_item(ev, n=n, data=data, psd=psd, theta0=th0, seed=seed, stream_id=7, **bufs))
        evs.append((b, ev, data, psd, th0, n, bufs, seed))
    for prec in (binding.PE_PREC_SPLIT, binding.PE_PREC_FP64):
        binding.pe_batch_run(items, binding.PE_STAGE_ALL, prec)
        torch.cuda.synchronize()
        for b, ev, data, psd, th0, n, bufs, seed in evs:
            ev.status()
            D = ev.dim
            ev.update(data, psd)
            g = ev.metric(th0)
            assert torch.equal(g, bufs["g"])
            if n == 0:
                continue
            th, lq, lp = ev.draw(th0, g, seed, 7, n)
            assert torch.equal(th, bufs["theta"][:, :n]) and torch.equal(lq, bufs["logq"][:n])
            assert torch.equal(lp, bufs["logprior"][:n])
            ll, ax = ev.loglike(th, precision=prec, aux=True)
            assert np.array_equal(host(ll), host(bufs["loglike"][:n]))
            live = torch.isfinite(ll)
            assert torch.equal(ax[live], bufs["aux"][:n][live])
            w, st = binding.weights_ess(ll, lp, lq)
            assert torch.equal(w, bufs["w"][:n]) and torch.equal(st, bufs["stats"])
            note(f"batch_run cfg {b.config} n_det {b.n_det} n={n} prec={prec}: ESS {float(st[0]):.3f} of {n}")
    for b, ev, *_ in evs:
        ev.close()


def test_batch_config2_full_size_sampled():
    """Config 2 at full size in the benchmark's launch configuration: 64 BBH events with their
    2^14..2^18 draws each (6.5 M draws, drawn by the oracle) through one pe_batch_run (metric,
    log-likelihoods, weights as one launch set per stage, autotuned plan); the metric of every event
    and ln L on 3 sampled draws per event against the oracle."""
    from concurrent.futures import ThreadPoolExecutor
    torch = torch_cuda()
    f64 = dict(dtype=torch.float64, device="cuda")
    Ns = synth.n_draws_batch(2, 64)
    bs = [build_event(2, e) for e in range(64)]
    gs = [b.ev.metric(b.theta_inj) for b in bs]
    with ThreadPoolExecutor(8) as pool:  # the oracle's draws release the GIL
        draws = list(pool.map(lambda e: bs[e].ev.draw(bs[e].theta_inj, gs[e], synth.draw_seed(2, e), 0, Ns[e]),
                              range(64)))
    note(f"c2 full: {sum(Ns)} oracle draws")
    evs, items, outs = [], [], []
    for e, b in enumerate(bs):
        ev, data, psd = upload_event(b)
        rc, th, lq, lp = draws[e]
        o = dict(th0=dev(b.theta_inj), g=torch.empty((11, 11), **f64), theta=dev(th), logq=dev(lq), logprior=dev(lp),
                 ll=torch.empty(Ns[e], **f64), w=torch.empty(Ns[e], **f64), st=torch.empty(4, **f64), keep=(data, psd))
        evs.append(ev)
        outs.append(o)
        items.append(binding.make_item(ev, n=Ns[e], theta0=o["th0"], g=o["g"], theta=o["theta"], logq=o["logq"],
                                       logprior=o["logprior"], loglike=o["ll"], w=o["w"], stats=o["st"]))
    before = binding.pe_get_plan()
    it, mb, ms = binding.pe_autotune_plan(evs, [o["theta"] for o in outs], Ns, binding.PE_PREC_SPLIT, reps=1)
    try:
        binding.pe_set_plan(it, mb)
        binding.pe_batch_run(items, binding.PE_STAGE_METRIC | binding.PE_STAGE_LOGLIKE | binding.PE_STAGE_WEIGHTS,
                             binding.PE_PREC_SPLIT)
        torch.cuda.synchronize()
    finally:
        binding.pe_set_plan(*before)
    rng = np.random.default_rng(22)
    worst_g, worst_l = 0.0, 0.0
    for e, (b, o) in enumerate(zip(bs, outs)):
        evs[e].status()
        g = host(o["g"])
        s = np.sqrt(np.outer(np.diag(gs[e]), np.diag(gs[e])))
        worst_g = max(worst_g, float(np.max(np.abs(g - gs[e]) / s)))
        ll = host(o["ll"])
        rc, th, lq, lp = draws[e]
        assert np.array_equal(np.isfinite(ll), np.isfinite(lp))
        live = np.flatnonzero(np.isfinite(ll))
        pick = rng.choice(live, 3, replace=False)
        worst_l = max(worst_l, float(np.max(np.abs(ll[pick] - b.ev.loglike(th[:, pick])))))
        st = host(o["st"])
        assert st[3] == live.size and 1.0 <= st[0] <= live.size
    note(f"c2 full: plan ({it}, {mb}); max metric error {worst_g:.2e} of sqrt(g_ii g_jj); "
         f"max |dlnL| {worst_l:.2e} on 192 sampled draws")
    assert worst_g <= 1e-6
    assert worst_l <= 1e-3
    for ev in evs:
        ev.close()


@pytest.mark.parametrize("cfg,event", [(2, 7), (1, 3)])
def test_split_large_amplitude_draws_within_bound(cfg, event):
    """Draws far louder than the data (distance shrunk up to 40-100x, so |Z| passes 1e4): the split
    path's hardware sine/cosine error grows with the size of the coherent sum, so such draws are
    re-evaluated in FP64 and every draw stays within the 1e-3 bound of the oracle."""
    torch_cuda()
    b = build_event(cfg, event, n_bins=None if cfg == 2 else 60000)
    g = b.ev.metric(b.theta_inj)
    rc, th, lq, lp = b.ev.draw(b.theta_inj, g, 5, 0, 400)
    th = th.copy()
    th[8] = b.theta_inj[8] / np.geomspace(1.0, 40.0 if cfg == 2 else 100.0, th.shape[1])
    ev, data, psd = upload_event(b)
    ll, ax = ev.loglike(dev(th), precision=binding.PE_PREC_SPLIT, aux=True)
    ll, ax = host(ll), host(ax)
    ev.status()
    live = np.flatnonzero(np.isfinite(ll))
    ll_o, zh = b.ev.loglike(th[:, live], return_zh=True)
    d = np.abs(ll[live] - ll_o)
    zmax = float(np.max(np.hypot(zh[:, 0], zh[:, 1])))
    note(f"large-amplitude draws cfg {cfg}: |Z| up to {zmax:.3g}, max |dlnL| {d.max():.2e} over {live.size} draws")
    assert zmax > 1e4
    assert d.max() <= 1e-3


def test_autotuned_plan_is_reproducible_and_within_tolerance():
    """The autotuner returns a plan from its grid; under that plan the results are reproducible bit
    for bit and agree with the oracle within the split bound; the library's plan is untouched by
    the tuning itself."""
    torch_cuda()
    bs = [build_event(2, e) for e in range(3)]
    evs, ths, keep = [], [], []
    for i, b in enumerate(bs):
        rc, th, lq, lp = b.ev.draw(b.theta_inj, b.ev.metric(b.theta_inj), 40 + i, 0, 3000 + 1000 * i)
        ev, data, psd = upload_event(b)
        evs.append(ev)
        ths.append(th)
        keep.append((data, psd))
    dth = [dev(t) for t in ths]
    before = binding.pe_get_plan()
    it, mb, ms = binding.pe_autotune_plan(evs, dth, [t.shape[1] for t in ths], binding.PE_PREC_SPLIT, reps=1)
    assert binding.pe_get_plan() == before
    assert it in (4096, 8192, 16384, 32768, 65536) and mb in (256, 512, 1024, 2048, 4096) and ms > 0
    note(f"autotuned plan: items_target {it}, min_group_bins {mb}, {ms:.3f} ms per batch")
    try:
        binding.pe_set_plan(it, mb)
        a = [host(x) for x in binding.loglike_multi(evs, dth)]
        c = [host(x) for x in binding.loglike_multi(evs, dth)]
    finally:
        binding.pe_set_plan(*before)
    for b, t, x, y in zip(bs, ths, a, c):
        assert np.array_equal(x, y)
        live = np.flatnonzero(np.isfinite(x))[:40]
        assert np.max(np.abs(x[live] - b.ev.loglike(t[:, live]))) <= 1e-3
    for ev in evs:
        ev.close()


def test_long_signal_config4_full_size_sampled():
    """Config 4 at full size (3 detectors, K = 2 086 912, 262 144 draws; event 0, SNR 43; the SNR-95
    event of the configuration's upper range is in test_gpu_guard.py): the FP64
    phase over ~1e5 rad and the split path's compensated FP32 sums against the oracle on sampled
    draws; the FP64 path within its derived bound."""
    torch_cuda()
    b = build_event(4, 0)
    note(f"c4 snr {b.snr:.1f} K {b.n_bins}")
    # proposal covariance from a shorter band (the metric is data-independent); parity needs only
    # draws near the injection
    bs = build_event(4, 0, n_bins=150000)
    g = bs.ev.metric(b.theta_inj)
    N = 262144
    rc, th, lq, lp = b.ev.draw(b.theta_inj, g, synth.draw_seed(4, 0), 0, N)
    ev, data, psd = upload_event(b)
    ev.reserve(N)
    tht = dev(th)
    note("gpu split + fp64 loglike c4 full size")
    ll_s = host(ev.loglike(tht, precision=binding.PE_PREC_SPLIT))
    ll_d = host(ev.loglike(tht, precision=binding.PE_PREC_FP64))
    ev.status()
    assert np.array_equal(np.isfinite(lp), np.isfinite(ll_s)) and np.array_equal(np.isfinite(lp), np.isfinite(ll_d))
    live = np.flatnonzero(np.isfinite(ll_s))
    pick = _wave_extremes(b, th, live, 1024)
    note(f"oracle loglike on {pick.size} sampled draws (the lowest and highest cut of 512 waves, K = {b.n_bins})")
    ll_o = b.ev.loglike(th[:, pick])
    ds = np.abs(ll_s[pick] - ll_o)
    dd = np.abs(ll_d[pick] - ll_o)
    sub64 = pick[:: max(1, pick.size // 32)]
    bw, bm = fp64_draw_bounds(b, th[:, sub64])
    dsub = np.abs(ll_d[sub64] - ll_o[np.searchsorted(pick, sub64)])
    note(f"  c4 split max |dlnL| = {ds.max():.3e}; fp64 max |dlnL| = {dd.max():.3e} (band-edge bound "
         f"{fp64_tol(b):.2e}; on {sub64.size} of them the largest error / model bound {np.max(dsub / bm):.3f}, "
         f"/ worst case {np.max(dsub / bw):.4f}); |lnL| up to {np.abs(ll_o).max():.3e}")
    assert ds.max() <= 1e-3
    assert dd.max() <= fp64_tol(b)
    assert np.all(dsub <= bm) and np.all(dsub <= bw)
