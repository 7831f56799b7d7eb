"""GPU: the serving loop (pe_server_*) through the C ABI. Requests of different shapes arrive while
others are on the GPU, share hot-loop slices (continuous batching, graph replay or direct
launches) and must return exactly what the single-event calls return for the same inputs: every
ln L, weight and ESS bit for bit, alone or in the mix. Sampled served draws are also checked
against the oracle (split: 1e-3; FP64: the per-draw rounding model of gpu_util.fp64_draw_bounds).
The per-bucket plans of pe_server_tune: served results equal the single-event calls under the
bucket's plan."""
import time

import numpy as np
import pytest

from events import build_event
from gpu_util import desc_kwargs, dev, fp64_draw_bounds, host, note, torch_cuda, upload_event
from paper_2410_05190_amd import binding

pytestmark = pytest.mark.gpu

SHAPES = [  # (config, event, n_det, n_bins, draws, host data, distance-marginalised)
    (1, 0, 3, 40000, 3000, False, 0),
    (2, 1, 2, None, 20000, True, 0),
    (1, 2, 1, 30000, 700, True, 0),
    (0, 0, None, None, 2500, False, 0),
    (2, 3, 3, None, 5000, False, 0),
    (1, 4, 2, 25000, 1, True, 0),
    (1, 5, 3, None, 16384, False, 0),  # full config-1 band (519 168 bins)
    (1, 6, 3, 30000, 2000, False, 1),
    (2, 7, 2, None, 3000, True, 1),
]


def _single(b, ev, theta0, n, seed, stream_id, prec):
    """The same request through the single-event calls."""
    g = ev.metric(dev(theta0))
    th, lq, lp = ev.draw(dev(theta0), g, seed, stream_id, n)
    ll = ev.loglike(th, precision=prec)
    w, st = binding.weights_ess(ll, lp, lq)
    return host(th), host(ll), host(w), host(st)


def _run(prec, use_graph, slice_ms, budget=1 << 32, max_active=64):
    torch = torch_cuda()
    built = []
    for cfg, e, nd, K, n, on_host, dist in SHAPES:
        b = build_event(cfg, e, n_det=nd, n_bins=K, distance=dist)
        built.append((b, n, on_host))
    srv = binding.Server(budget, precision=prec, max_active=max_active, slice_ms=slice_ms, use_graph=use_graph)
    tickets, outs, keep = [], [], []
    for i, (b, n, on_host) in enumerate(built):
        kw = desc_kwargs(b)
        dd, pd = (binding.PE_C64 if b.data.dtype == np.complex64 else binding.PE_C128,
                  binding.PE_F32 if b.psd.dtype == np.float32 else binding.PE_F64)
        desc = binding.make_desc(b.n_det, b.n_bins, data_dtype=dd, psd_dtype=pd, **kw)
        if on_host:
            data, psd = b.data, b.psd
        else:
            data = torch.from_numpy(np.ascontiguousarray(b.data)).cuda()
            psd = torch.from_numpy(np.ascontiguousarray(b.psd)).cuda()
            torch.cuda.synchronize()
        keep.append((data, psd))
        D = 4 if b.params == binding.PE_PARAMS_4D else 11
        ll = np.full(n, np.nan)
        w = np.full(n, np.nan)
        th = np.full((D, n), np.nan)
        outs.append((ll, w, th))
        tickets.append(srv.submit(desc, data, psd, b.theta_inj, n, seed=100 + i, stream_id=3, loglike_out=ll,
                                  w_out=w, theta_out=th))
        if i == 2:
            time.sleep(0.05)  # the rest arrive while the first ones are on the GPU
    results = [srv.wait(t, timeout=120.0) for t in tickets]
    counters = srv.counters()
    srv.close()
    note(f"server prec={prec} graph={use_graph} slice={slice_ms} ms: {counters}")
    for i, ((b, n, _), res, (ll, w, th)) in enumerate(zip(built, results, outs)):
        assert res.status == 0, (i, res.status)
        ev, d_, p_ = upload_event(b)
        th1, ll1, w1, st1 = _single(b, ev, b.theta_inj, n, 100 + i, 3, prec)
        ev.close()
        note(f"  request {i}: n={n} ESS {res.stats[0]:.3f} admitted with {res.n_active} active, "
             f"latency {1e3 * (res.t_done - res.t_submit):.1f} ms")
        assert np.array_equal(th, th1)
        assert np.array_equal(ll, ll1)
        assert np.array_equal(w, w1)
        assert np.array_equal(np.array(res.stats[:]), st1)
        _oracle_check(b, th, ll, prec, i)
    return results, counters


def _oracle_check(b, th, ll, prec, i, n=6):
    """A few served draws (the live ones, spread over the request) against the oracle."""
    live = np.flatnonzero(np.isfinite(ll))
    if live.size == 0:
        return
    pick = live[np.linspace(0, live.size - 1, min(n, live.size)).round().astype(int)]
    pick = np.unique(pick)
    ll_o = b.ev.loglike(np.ascontiguousarray(th[:, pick]))
    d = np.abs(ll[pick] - ll_o)
    if prec == binding.PE_PREC_SPLIT:
        tol = np.full(pick.size, 1e-3)
    else:
        tol = fp64_draw_bounds(b, np.ascontiguousarray(th[:, pick]))[1]
        if b.distance:  # the two distance quadratures, each ~1e-13 relative
            tol = tol + 1e-9 * np.maximum(1.0, np.abs(ll_o))
    note(f"  request {i}: {pick.size} served draws against the oracle, max |dlnL| {d.max():.2e}")
    assert np.all(d <= tol)


def test_server_mixed_requests_equal_single_event_calls_graph():
    results, c = _run(binding.PE_PREC_SPLIT, True, 0.02)  # tiny slices: each request spans several
    assert c["completed"] == len(SHAPES)
    assert c["graph_replays"] == c["slices"] and c["slices"] > len(SHAPES)
    assert max(r.n_active for r in results) > 0  # requests were on the device together


def test_server_direct_launches_fp64():
    results, c = _run(binding.PE_PREC_FP64, False, 1.0)
    assert c["graph_replays"] == 0 and c["completed"] == len(SHAPES)


def test_server_admission_by_memory_budget():
    """A budget that holds about one request at a time: requests wait for memory, complete in
    order, and one larger than the whole budget is refused with PE_ERR_BUDGET."""
    torch_cuda()
    b = build_event(2, 5)
    kw = desc_kwargs(b)
    desc = binding.make_desc(b.n_det, b.n_bins, data_dtype=binding.PE_C64, psd_dtype=binding.PE_F32, **kw)
    srv = binding.Server(80 << 20, max_active=8, slice_ms=2.0)
    ts = [srv.submit(desc, b.data, b.psd, b.theta_inj, 100000, seed=i) for i in range(4)]
    big = srv.submit(desc, b.data, b.psd, b.theta_inj, 4000000, seed=9)
    res = [srv.wait(t, timeout=120.0) for t in ts]
    rb = srv.wait(big, timeout=10.0)
    c = srv.counters()
    srv.close()
    note(f"budget test: {c}")
    assert all(r.status == 0 for r in res)
    assert rb.status == binding.PE_ERR_BUDGET
    assert c["admission_waits"] > 0 and c["peak_slab_bytes"] <= 80 << 20
    assert all(res[i].t_done <= res[i + 1].t_done for i in range(3))


def test_server_tuned_plans_per_bucket():
    """pe_server_tune on two shape buckets (config-1 shape, 3 detectors, 2^16 bins; config 2, 2
    detectors, 2^13 bins): one plan per bucket, and requests of those shapes served with them equal
    the single-event calls run under pe_set_plan with their bucket's plan, bit for bit."""
    torch = torch_cuda()
    shapes = [(1, 8, 3, 60000, 6000), (2, 9, 2, None, 20000)]
    built, evs, ths, ns = [], [], [], []
    for cfg, e, nd, K, n in shapes:
        b = build_event(cfg, e, n_det=nd, n_bins=K)
        ev, d_, p_ = upload_event(b)
        g = ev.metric(dev(b.theta_inj))
        th, lq, lp = ev.draw(dev(b.theta_inj), g, 7, 1, n)
        built.append((b, n, ev, d_, p_))
        evs.append(ev)
        ths.append(th)
        ns.append(n)
    srv = binding.Server(1 << 32, max_active=16, slice_ms=0.05)
    srv.tune(evs, ths, ns, reps=1)
    plans = srv.plans()
    note(f"tuned plans (n_det, log2 K, items_target, min_group_bins, ms): {plans}")
    assert sorted((p[0], p[1]) for p in plans) == [(2, 13), (3, 16)]
    tickets, outs = [], []
    for i, (b, n, ev, d_, p_) in enumerate(built):
        desc = binding.make_desc(b.n_det, b.n_bins, data_dtype=binding.PE_C64, psd_dtype=binding.PE_F32,
                                 **desc_kwargs(b))
        ll = np.full(n, np.nan)
        w = np.full(n, np.nan)
        tickets.append(srv.submit(desc, b.data, b.psd, b.theta_inj, n, seed=50 + i, stream_id=2, loglike_out=ll,
                                  w_out=w))
        outs.append((ll, w))
    results = [srv.wait(t, timeout=120.0) for t in tickets]
    srv.close()
    keep = binding.pe_get_plan()
    try:
        for i, ((b, n, ev, d_, p_), res, (ll, w)) in enumerate(zip(built, results, outs)):
            assert res.status == 0
            plan = [p for p in plans if p[0] == b.n_det][0]
            binding.pe_set_plan(plan[2], plan[3])
            th1, ll1, w1, st1 = _single(b, ev, b.theta_inj, n, 50 + i, 2, binding.PE_PREC_SPLIT)
            assert np.array_equal(ll, ll1)
            assert np.array_equal(w, w1)
    finally:
        binding.pe_set_plan(*keep)
    for x in built:
        x[2].close()
