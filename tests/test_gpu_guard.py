"""GPU tests of the split path's error bound and its FP64 re-evaluation.

Each split-path draw gets a bound on its |d ln L|. The bound comes from the measured error spectrum of
the hardware sine/cosine and the data's noise statistics. Draws above the budget of pe_set_split_guard
are re-evaluated in FP64, on the hot loop's own layout, within the same call. The tests check:
  - budget 0: every live draw is re-evaluated, and the split call then equals the FP64 path to FP64
    rounding (the re-evaluation may split the band into more groups than the FP64 path; 1e-12 relative,
    1e-9 absolute), for single events and a multi-event batch;
  - noise-free data: the worst-case regime lists the loud draws, and every draw stays within 1e-3 of the
    oracle;
  - a config-4-shaped event at SNR 95 (the top of that configuration's range), full size: sampled draws
    (the loudest included) are within 1e-3 of the oracle. Draws the default budget leaves on the split
    path are within that budget even with re-evaluation switched off.
"""
import numpy as np
import pytest

from events import build_event
from gpu_util import dev, host, note, torch_cuda, upload_event
from paper_2410_05190_amd import binding
from paper_2410_05190_amd import synth

pytestmark = pytest.mark.gpu


class _budget:
    def __init__(self, b):
        self.b = b

    def __enter__(self):
        self.keep = binding.pe_get_split_guard()
        binding.pe_set_split_guard(self.b)

    def __exit__(self, *exc):
        binding.pe_set_split_guard(self.keep)


def _draws(b, n, seed, metric_event=None):
    g = (metric_event or b).ev.metric(b.theta_inj)
    rc, th, lq, lp = b.ev.draw(b.theta_inj, g, seed, 0, n)
    assert rc == 0
    return th


@pytest.mark.parametrize("cfg,K,n", [(1, 40000, 1500), (0, 31488, 700), (2, 8032, 3000)])
def test_zero_budget_equals_fp64_path(cfg, K, n):
    """Budget 0 sends every live draw through the FP64 re-evaluation, so split == FP64 to rounding."""
    torch_cuda()
    b = build_event(cfg, 1, n_bins=K)
    th = dev(_draws(b, n, 21))
    ev, data, psd = upload_event(b)
    ll_d = host(ev.loglike(th, precision=binding.PE_PREC_FP64))
    live_d, redo_d = binding.pe_loglike_counts(ev)
    assert redo_d == 0
    with _budget(0.0):
        ll_s, ax_s = ev.loglike(th, precision=binding.PE_PREC_SPLIT, aux=True)
        ll_s, ax_s = host(ll_s), host(ax_s)
        live, redo = binding.pe_loglike_counts(ev)
    ev.status()
    note(f"cfg {cfg}: live {live}, re-evaluated {redo}")
    assert live == live_d and redo == live and live > 0
    fin = np.isfinite(ll_d)
    assert np.array_equal(fin, np.isfinite(ll_s))
    np.testing.assert_allclose(ll_s[fin], ll_d[fin], rtol=1e-12, atol=1e-9)
    ll_d2, ax_d = ev.loglike(th, precision=binding.PE_PREC_FP64, aux=True)
    np.testing.assert_allclose(ax_s, host(ax_d), rtol=1e-12, atol=1e-9)
    ev.close()


def test_zero_budget_multi_event_batch_equals_fp64():
    """The same in one multi-event batch (config 2 events of uneven draw counts), every event re-evaluated."""
    torch_cuda()
    bs = [build_event(2, e) for e in range(4)]
    evs, ths, keep = [], [], []
    for i, b in enumerate(bs):
        th = _draws(b, 500 + 700 * i, 30 + i)
        ev, data, psd = upload_event(b)
        evs.append(ev)
        ths.append(dev(th))
        keep.append((data, psd))
    want = [host(x) for x in binding.loglike_multi(evs, ths, precision=binding.PE_PREC_FP64)]
    with _budget(0.0):
        got = [host(x) for x in binding.loglike_multi(evs, ths, precision=binding.PE_PREC_SPLIT)]
        counts = [binding.pe_loglike_counts(ev) for ev in evs]
    for w, g, (live, redo) in zip(want, got, counts):
        assert redo == live and live > 0
        fin = np.isfinite(w)
        assert np.array_equal(fin, np.isfinite(g))
        np.testing.assert_allclose(g[fin], w[fin], rtol=1e-12, atol=1e-9)
    for ev in evs:
        ev.close()


def test_noise_free_loud_event_worst_case_regime():
    """Noise-free data: the phases of a matched sum do not scatter, so the bound is the worst case
    (max |eps| times sum |w|); at SNR 120 the draws near the peak are listed, and every draw is within
    1e-3 of the oracle."""
    torch_cuda()
    b = build_event(1, 2, n_bins=60000, zero_noise=True, snr=120.0)
    th = _draws(b, 1200, 41)
    ev, data, psd = upload_event(b)
    ll = host(ev.loglike(dev(th), precision=binding.PE_PREC_SPLIT))
    live, redo = binding.pe_loglike_counts(ev)
    ev.status()
    fin = np.flatnonzero(np.isfinite(ll))
    ll_o = b.ev.loglike(th[:, fin])
    d = np.abs(ll[fin] - ll_o)
    note(f"noise-free SNR 120: live {live}, re-evaluated {redo}, max |dlnL| {d.max():.2e}")
    assert redo > 0
    assert d.max() <= 1e-3
    ev.close()


def _sample_by_cut(b, th, live, n_pick, rng):
    """n_pick live draws: the highest- and lowest-cut ones (the ends of the cut ordering, where waves
    mix cuts and the masked tail runs) and a random rest."""
    f_lo, df, K = b.f_lo, b.df, b.n_bins
    tsun = 1.32712440018e20 / 299792458.0 ** 3
    q = th[1, live]
    M = th[0, live] * (1 + q) ** 1.2 * q ** -0.6
    kc = np.clip(np.ceil((1.0 / (6.0 ** 1.5 * np.pi * M * tsun) - f_lo) / df), 0, K)
    order = live[np.argsort(-kc, kind="stable")]
    ends = np.concatenate([order[:64], order[-64:]])
    rest = rng.choice(np.setdiff1d(live, ends), n_pick - ends.size, replace=False)
    return np.sort(np.concatenate([ends, rest]))


@pytest.mark.timeout(600)
def test_loud_config4_event_full_size_sampled():
    """Config-4 shape at SNR 95 (3 detectors, K = 2 086 912, 262 144 draws): 1024 sampled draws against
    the oracle within 1e-3, with the loudest draws among them; the draws that the default budget keeps
    on the split path stay within that budget also when no draw is re-evaluated."""
    torch_cuda()
    b = build_event(4, 1, snr=95.0)
    note(f"c4 snr {b.snr:.1f} K {b.n_bins}")
    bs = build_event(4, 1, n_bins=150000, snr=95.0)
    N = 262144
    th = _draws(b, N, synth.draw_seed(4, 1), metric_event=bs)
    ev, data, psd = upload_event(b)
    ev.reserve(N)
    tht = dev(th)
    note("gpu split loglike c4 SNR 95, default budget")
    ll, ax = ev.loglike(tht, precision=binding.PE_PREC_SPLIT, aux=True)
    ll, ax = host(ll), host(ax)
    live_n, redo_n = binding.pe_loglike_counts(ev)
    with _budget(float("inf")):
        ll_free = host(ev.loglike(tht, precision=binding.PE_PREC_SPLIT))
        assert binding.pe_loglike_counts(ev)[1] == 0
    ev.status()
    live = np.flatnonzero(np.isfinite(ll))
    zmag = np.hypot(ax[live, 0], ax[live, 1])
    rng = np.random.default_rng(9)
    pick = _sample_by_cut(b, th, live, 1024 - 32, rng)
    loud = live[np.argsort(-zmag)[:32]]
    pick = np.unique(np.concatenate([pick, loud]))
    note(f"  live {live_n}, re-evaluated {redo_n}; |Z| up to {zmag.max():.3g}; oracle on {pick.size} draws")
    ll_o = b.ev.loglike(th[:, pick])
    d = np.abs(ll[pick] - ll_o)
    kept = ll_free[pick] == ll[pick]  # draws the default budget left on the split path
    d_free = np.abs(ll_free[pick] - ll_o)
    note(f"  c4 SNR 95 max |dlnL| {d.max():.2e}; split-only draws {kept.sum()} max {d_free[kept].max():.2e}; "
         f"no re-evaluation max {d_free.max():.2e}")
    assert d.max() <= 1e-3
    assert d_free[kept].max() <= binding.pe_get_split_guard()
    assert redo_n < 0.1 * live_n  # the loud event stays on the split path
    ev.close()
