"""bench.py's command-line contract, checked without a GPU: more than one GPU is refused with a
message, and every leg the default run calls is defined."""
import ast
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_default_legs_are_defined():
    tree = ast.parse(open(os.path.join(ROOT, "bench.py")).read())
    defined = {n.name for n in tree.body if isinstance(n, ast.FunctionDef)}
    called = {n.func.id for n in ast.walk(tree) if isinstance(n, ast.Call) and isinstance(n.func, ast.Name)}
    for name in ("main", "make_data", "make_event", "serve_bench", "cpu_baseline", "host_terms", "percentiles"):
        assert name in defined
    local = {c for c in called if c in defined or c.startswith(("make_", "serve_", "cpu_"))}
    assert local <= defined, local - defined


def test_config2_cpu_baseline_runs_on_host_data():
    """The config-2 leg of the oracle timing, on two small host-built events of that shape (noise
    plus the oracle's own injection): it returns positive rates and counts only in-support draws."""
    import numpy as np

    sys.path.insert(0, ROOT)
    import bench
    import oracle
    from paper_2410_05190_amd import binding, synth

    c = 2
    cfg = synth.CONFIGS[c]
    f_lo, df, K = synth.grid(c)
    nd = cfg["n_det"]
    S = np.tile(synth.psd_analytic(synth.frequencies(f_lo, df, K)), (nd, 1))
    geom = synth.detectors(c, nd)
    inputs = []
    for e in range(2):
        th0 = synth.injection(c, e)["theta"].copy()
        common = dict(f_lo=f_lo, df=df, strain_scale=1.0, params=binding.PE_PARAMS_11D,
                      phase=binding.PE_PHASE_MARG, gmst=0.0, chi_max=cfg["chi_max"], dl_max=cfg["dl_max"] or 1e4,
                      det_geom=geom)
        ref = oracle.Event(nd, K, f_lo, df, data=None, psd=S, strain_scale=1.0, params=common["params"],
                           phase=common["phase"], amp0=0.0, gmst=0.0, chi_max=common["chi_max"],
                           dl_max=common["dl_max"], det_geom=geom)
        data = np.ascontiguousarray(ref.waveform(th0) + synth.noise(c, e, S, df), dtype=np.complex128)
        inputs.append(dict(data=data, psd=S, theta_inj=th0, amp0=0.0, common=common, N=256))
    r = bench.cpu_config2(inputs)
    assert r["kind"] == "oracle" and r["value"] > 0 and r["terms_per_s"] > 0 and r["cores"] >= 1
    n_live = int(r["sample"].split(" in-support")[0].split()[-1])
    assert 0 < n_live <= 512
