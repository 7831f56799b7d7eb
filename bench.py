#!/usr/bin/env python3
"""Benchmark of the metric-importance-sampling likelihood path on one MI355X.

One step = the whole hot path for the events of the benchmark workload (default: one
event of the 3-detector BNS shape, 11-D, 519168 bins per detector, complex64 data and
FP32 PSD, 65536 proposal draws, split precision; --config 2: 64 BBH events of uneven
draw counts whose log-likelihoods share one multi-event batch):
  event-table preparation -> metric at the proposal centre -> Gaussian draws ->
  log-likelihoods -> importance weights and ESS,
with every input already resident in HBM. Prints one JSON line.

Synthetic data: the seeded coloured-noise workload of paper_2410_05190_amd.synth with a
TaylorF2 injection made by the library's own waveform call.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# VALU issue model of the hot-loop kernels, in issue slots (lane-cycles) of the
# minimal instruction sequence: the phase polynomial (10 FP64 ops) is shared by
# the detectors of a bin; each term (draw, detector, bin) of the split kernel
# costs FP64 FMA + fract, FP64->FP32 convert, FP32 add, two FP32 FMAs and
# v_sin_f32 + v_cos_f32, one slot each. The transcendentals hold their unit one
# cycle longer (SQ_ACTIVE_INST_VALU - SQ_INSTS_VALU = SQ_INSTS_VALU_TRANS_F32),
# but that cycle overlaps the instructions that follow: the kernel issues more
# than one slot per cycle per CU if it is charged two. The FP64 kernel's term:
# FMA + fract, the 26-op FP64 sincos, four FMAs.
PSI_OPS_PER_DRAW_BIN = 10
SPLIT_OPS_PER_TERM = 6 + 2
FP64_OPS_PER_TERM = 2 + 26 + 4
# HBM bytes per launch of the split kernel at the benchmark shape (config 1, automatic
# groups), from rocprofv3 FETCH_SIZE x 1.9999 + WRITE_SIZE x 1.0 (KiB per dispatch), the
# factors read off a 1 GiB device-to-device copy in the same runs (profiles/
# loglike_split_config1.md); None when the kernel has changed since the counters were taken.
SPLIT_TRAFFIC_BYTES = 537122371
VALU_PEAK = 256 * 64 * 2.4e9  # lane-ops/s: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz
# Algorithmic floating-point work per term (draw, detector, bin) of the split path: the FP64
# phase polynomial (about 24 flops with its log term and scaling) shared by the detectors plus
# the FP64 time-shift FMA and fract (3); the FP32 complex multiply-accumulate (8; the sine/cosine
# pair is not counted as flops). Vector peaks: FP64 78.6 TFLOP/s, FP32 157.3 TFLOP/s.
PSI_FLOP64_PER_DRAW_BIN = 24.0
FLOP64_PER_TERM = 3.0
FLOP32_PER_TERM = 8.0
FP64_PEAK = 78.6e12
FP32_PEAK = 157.3e12
SPLIT_TRAFFIC_SOURCE = "rocprofv3 FETCH_SIZE x 1.9999 + WRITE_SIZE x 1.0 per launch (profiles/loglike_split_config1.md)"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", type=int, default=1)
    ap.add_argument("--precision", choices=["split", "fp64"], default="split")
    ap.add_argument("--chunks", type=int, default=0)
    ap.add_argument("--autotune", choices=["auto", "on", "off"], default="auto",
                    help="pick the hot loop's plan with the library's autotuner before timing (auto: batches and "
                         "small events)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=1024,
                    help="cpu_baseline: in-support draws of the benchmark event timed on the oracle")
    ap.add_argument("--serve-events", type=int, default=120,
                    help="requests of the serving load (Poisson arrivals); 0 skips the serving leg")
    ap.add_argument("--serve-rate", type=float, default=5.0, help="arrival rate of the serving load (1/s)")
    ap.add_argument("--serve-slice-ms", type=float, default=8.0)
    ap.add_argument("--serve-budget-gib", type=float, default=32.0)
    ap.add_argument("--serve-no-graph", action="store_true")
    ap.add_argument("--serve-no-baseline", action="store_true")
    ap.add_argument("--serve-no-tune", action="store_true",
                    help="serving leg: skip the server's per-bucket plan autotuner (library's default plan)")
    ap.add_argument("--drift-sample", type=int, default=-1,
                    help="draws of the last step compared with the oracle (FP64-phase drift); -1: 1024 for config 4, "
                         "else 0")
    ap.add_argument("--refine-rounds", type=int, default=3,
                    help="rounds of proposal refinement before the refined-proposal leg (0 skips the leg)")
    ap.add_argument("--refine-draws", type=int, default=16384, help="draws per refinement round")
    ap.add_argument("--mixture-k", type=int, default=6,
                    help="mixture leg: components at the pilot round's k heaviest draws (0 skips the leg)")
    ap.add_argument("--relbin-eps", type=float, default=0.02,
                    help="relative-binning leg: envelope step between bin edges (0 skips the leg)")
    ap.add_argument("--tile-radius", type=float, default=6.0, help="tile-mixture leg: slice radius (whitened)")
    ap.add_argument("--tile-spacing", type=float, default=1.0, help="tile-mixture leg: template spacing (whitened)")
    ap.add_argument("--tile-candidates", type=int, default=4000000,
                    help="tile-mixture leg: slice candidates for the prior samples (0 skips the leg; 4-D only)")
    ap.add_argument("--itile-radius", type=float, default=4.0,
                    help="intrinsic tile leg (11-D): slice radius in the intrinsic marginal metric (whitened)")
    ap.add_argument("--itile-spacing", type=float, default=1.0, help="intrinsic tile leg: template spacing")
    ap.add_argument("--itile-rounds", type=int, default=4,
                    help="intrinsic tile leg: rounds per step (each later round reweights the tiles and takes the "
                         "other coordinates from the previous round's weighted moments)")
    ap.add_argument("--imatch-samples", type=int, default=262144,
                    help="intrinsic match-tile leg: prior samples assigned by waveform match (0 skips the leg)")
    ap.add_argument("--imatch-dt", type=float, default=5e-5, help="intrinsic match-tile leg: time-shift step (s)")
    ap.add_argument("--itile-time", type=int, default=1,
                    help="intrinsic tile leg: 1 marginalises tc as well (as the time legs) and runs a second leg "
                         "with tc sampled; 0 runs only the leg with tc sampled")
    ap.add_argument("--itile-candidates", type=int, default=4000000,
                    help="intrinsic tile leg: slice candidates for the prior samples (0 skips the leg)")
    ap.add_argument("--no-distance-leg", action="store_true",
                    help="skip the distance-marginalised leg (11-D configurations)")
    ap.add_argument("--time-leg", type=int, default=1,
                    help="1: the leg with time, phase and distance marginalised (11-D configurations); 0 skips it")
    ap.add_argument("--time-leg-draws", type=int, default=65536,
                    help="time-marginalised leg: proposal draws per step (each evaluated at every tc node)")
    ap.add_argument("--no-batch-leg", action="store_true",
                    help="skip the config-2 leg (64 BBH events per step through pe_batch_run) of the default run")
    ap.add_argument("--long-steps", type=int, default=3,
                    help="config-4 leg: timed steps per event (SNR 43 and SNR 95); 0 skips the leg")
    ap.add_argument("--long-loud-snr", type=float, default=95.0, help="config-4 leg: SNR of the loud event")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run one plain device-to-device copy of this size first (HBM counter calibration)")
    return ap.parse_args()


def host_terms(theta, cfg, f_lo, df, K, n_det):
    """Algorithmic term count: sum over in-support draws of n_det x #{k : f_k < f_isco(M)}."""
    import numpy as np
    tsun = 1.32712440018e20 / 299792458.0 ** 3
    mc = theta[0]
    with np.errstate(all="ignore"):
        if cfg["params"] == "4d":
            M = mc * theta[1] ** -0.6
        else:
            q = theta[1]
            M = mc * (1 + q) ** 1.2 * q ** -0.6
        fisco = 1.0 / (6.0 ** 1.5 * math.pi * M * tsun)
        kc = np.clip(np.ceil((fisco - f_lo) / df), 0, K)
    return np.nan_to_num(kc)


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "bench.py measures one GPU only: run it with --gpus 1 "
                                   "(the library runs on one GPU; how it would shard is described, not implemented)"}), flush=True)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2410_05190_amd import binding, synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_calibration_mib:
        nbytes = args.copy_calibration_mib << 20
        src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"copy calibration: {nbytes} bytes read, {nbytes} bytes written", file=sys.stderr, flush=True)
        del src, dst
    c = args.config
    cfg = synth.CONFIGS[c]
    f_lo, df, K = synth.grid(c)
    nd = cfg["n_det"]
    n_events = cfg.get("batch", 1)
    Ns = synth.n_draws_batch(c, n_events) if cfg["n_draws"] is None else [cfg["n_draws"]] * n_events
    prec = binding.PE_PREC_SPLIT if args.precision == "split" else binding.PE_PREC_FP64
    kname = "loglike_split" if prec == binding.PE_PREC_SPLIT else "loglike_fp64"
    if args.chunks:
        binding.pe_set_chunks(args.chunks)
    evs = [make_event(c, e, N) for e, N in enumerate(Ns)]
    D = evs[0]["ev"].dim
    stats = torch.zeros((max(args.steps, 1), n_events, 4), dtype=torch.float64, device="cuda")

    def step(i, st_rows):
        if n_events == 1:
            # the single-event calls of the path
            x = evs[0]
            h_ = x["ev"].handle
            binding.pe_event_update(h_, x["data"], x["psd"])
            binding.pe_metric(h_, x["theta0"], None, 0, x["g"])
            binding.pe_draw(h_, x["theta0"], x["g"], x["seed"], i, x["N"], x["theta"], x["lq"], x["lp"])
            binding.pe_loglike_batch(h_, x["theta"], x["N"], prec, x["ll"], None)
            binding.pe_weights_ess(x["ll"], x["lp"], x["lq"], x["N"], x["w"], st_rows[0])
        else:
            # every stage as one set of launches over the batch of events
            items = [binding.make_item(x["ev"], n=x["N"], data=x["data"], psd=x["psd"], theta0=x["theta0"],
                                       seed=x["seed"], stream_id=i, g=x["g"], theta=x["theta"], logq=x["lq"],
                                       logprior=x["lp"], loglike=x["ll"], w=x["w"], stats=st_rows[e])
                     for e, x in enumerate(evs)]
            binding.pe_batch_run(items, binding.PE_STAGE_ALL, prec)

    for i in range(args.warmup):
        step(1000 + i, stats[0])
    torch.cuda.synchronize()
    for x in evs:
        x["ev"].status()
    plan = {"tuned": False}
    small = sum(Ns) * K < 10 ** 9  # launch-latency-bound shapes: the default plan leaves CUs idle
    if args.autotune == "on" or (args.autotune == "auto" and (n_events > 1 or small)):
        if args.warmup == 0:
            step(999, stats[0])
        t_tune = time.perf_counter()
        it, mb, best_ms = binding.pe_autotune_plan([x["ev"] for x in evs], [x["theta"] for x in evs],
                                                   [x["N"] for x in evs], prec, reps=2)
        binding.pe_set_plan(it, mb)
        plan = {"tuned": True, "tune_s": time.perf_counter() - t_tune, "best_loglike_ms": best_ms}
        step(998, stats[0])
        torch.cuda.synchronize()
    plan["items_target"], plan["min_group_bins"] = binding.pe_get_plan()

    binding.pe_profile_enable(True)
    binding.pe_profile_read(kname)
    ev_a = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ev_b = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ev_a[i].record()
        step(i, stats[i])
        ev_b[i].record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    binding.pe_profile_enable(False)
    k_ms, k_n = binding.pe_profile_read(kname)
    for x in evs:
        x["ev"].status()
    lat = sorted(a.elapsed_time(b) for a, b in zip(ev_a, ev_b))
    wall = t1 - t0
    st = stats.cpu().numpy()[: args.steps]
    n_live = st[:, :, 3].sum()
    ess = st[:, :, 0].sum()
    n_draws = sum(Ns) * args.steps
    # terms of the last step (its draws are still in `theta`)
    terms_last = 0.0
    for x in evs:
        kc = host_terms(x["theta"].cpu().numpy(), cfg, f_lo, df, K, nd)
        live_last = np.isfinite(x["ll"].cpu().numpy())
        terms_last += float(nd * kc[live_last].sum())
    db_last = terms_last / nd
    ops_per_term = SPLIT_OPS_PER_TERM if prec == binding.PE_PREC_SPLIT else FP64_OPS_PER_TERM
    # one hot-loop launch per step: its average duration
    k_avg_s = k_ms / max(k_n, 1) / 1e3
    ops_last = db_last * PSI_OPS_PER_DRAW_BIN + terms_last * ops_per_term
    achieved = ops_last / k_avg_s if k_avg_s > 0 else float("nan")
    traffic = SPLIT_TRAFFIC_BYTES if (prec == binding.PE_PREC_SPLIT and c == 1 and not args.chunks) else None
    fvec = vector_fraction(db_last, terms_last, nd, k_avg_s) if prec == binding.PE_PREC_SPLIT else None
    redo_last = [binding.pe_loglike_counts(x["ev"]) for x in evs]

    out = {
        "metric": "likelihood evals/s and ESS/s per event; p50/p99 event latency under load",
        "value": n_live / wall,
        "unit": "likelihood evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 phase + f32" if prec == binding.PE_PREC_SPLIT else "f64",
        "data": "synthetic (seeded coloured Gaussian noise + TaylorF2 injection)",
        "config": {"workload": cfg["name"], "n_det": nd, "n_bins": K, "events_per_step": n_events,
                   "draws_per_event": Ns[0] if n_events == 1 else Ns, "dim": D,
                   "precision": args.precision, "chunks": args.chunks or "auto", "plan": plan},
        "draws_per_s": n_draws / wall,
        "in_support_fraction": n_live / n_draws,
        "ess_per_s": ess / wall,
        "ess_per_event_mean": ess / (args.steps * n_events),
        "terms_per_s_hot_kernel": terms_last / k_avg_s if k_avg_s > 0 else None,
        "event_latency_ms": {"p50": lat[len(lat) // 2], "p99": lat[min(len(lat) - 1, int(0.99 * len(lat)))],
                             "kind": "isolated events, one at a time" if n_events == 1 else
                             f"one batch of {n_events} events, one batch at a time"},
        "roofline": {"bound": "alu", "kernel": kname, "achieved": achieved / 1e12, "peak": VALU_PEAK / 1e12,
                     "unit": "Tlane-op/s", "frac": achieved / VALU_PEAK, "traffic": traffic,
                     "traffic_source": SPLIT_TRAFFIC_SOURCE if traffic else None,
                     "kernel_ms_avg": k_avg_s * 1e3, "kernel_launches": k_n, "ops_per_launch": ops_last,
                     "frac_vector": fvec},
        "split_reevaluated_fp64": {"draws_last_step": int(sum(r[1] for r in redo_last)),
                                   "live_last_step": int(sum(r[0] for r in redo_last))},
    }
    first = evs[0]
    # the drift check reads the last timed step's draws and log-likelihoods: before the other legs
    # reuse those buffers
    n_drift = args.drift_sample if args.drift_sample >= 0 else (1024 if c == 4 else 0)
    if n_drift > 0:
        out["drift"] = drift_leg(first, n_drift, prec)
    if n_events == 1 and args.refine_rounds > 0:
        out["refined"] = refine_leg(first, args.refine_rounds, args.refine_draws, max(args.steps, 1), prec)
    if n_events == 1 and args.mixture_k > 0:
        start = first["theta0"]
        if "refined" in out:
            start = torch.tensor(out["refined"]["centre"], dtype=torch.float64, device="cuda")
        out["mixture"] = mixture_leg(first, start, args.mixture_k, max(args.steps, 1), prec)
    if n_events == 1 and args.relbin_eps > 0:
        out["relbin"] = relbin_leg(first, args.relbin_eps, max(args.steps, 1), prec)
    if n_events == 1 and D == 11 and not args.no_distance_leg:
        centres = {"injection": first["theta0"]}
        if "refined" in out:
            centres["refined"] = torch.tensor(out["refined"]["centre"], dtype=torch.float64, device="cuda")
        out["distance_marginalised"] = distance_leg(first, centres, max(args.steps, 1), prec)
        out["phase_and_distance_marginalised"] = distance_leg(first, centres, max(args.steps, 1), prec,
                                                              phase=binding.PE_PHASE_MARG)
        out["phase_and_distance_marginalised"]["kind"] = (
            "likelihood marginalised over the coalescence phase (ln I0 form) and the luminosity distance "
            "(dL^2 prior); both left out of the proposal density")
        if args.time_leg:
            # nodes half the phase-marginalised integrand's width in tc apart over the window: that
            # integrand follows the envelope |Z(t)|, whose curvature is g_tc,tc with the phase
            # projected out (the Schur complement of the explicit-phase metric's phic row)
            gh = first["g"].cpu().numpy()
            g_tt = gh[9, 9] - gh[9, 10] ** 2 / gh[10, 10]
            lo, hi = first["theta_inj"][9] - 0.01, first["theta_inj"][9] + 0.01
            pts = int(math.ceil((hi - lo) / (0.5 / math.sqrt(g_tt)))) + 1
            tm = {"tc_lo": float(lo), "tc_hi": float(hi), "tm_points": pts}
            how = ("block moments of each draw's integrand (one likelihood-like pass, then every node from the "
                   "moments)" if prec == binding.PE_PREC_SPLIT else "every node a likelihood evaluation")
            leg = distance_leg(first, centres, max(args.steps // 4, 2), prec, phase=binding.PE_PHASE_MARG,
                               time_marg=tm, n_draws=args.time_leg_draws)
            leg["kind"] = (f"likelihood marginalised over the coalescence time (flat over 20 ms about the injected "
                           f"tc; end-corrected trapezoid rule on {pts} nodes over the window, from {how}), the "
                           f"phase and the distance; all three left out of the proposal density")
            leg["time_nodes"] = tm
            out["time_phase_and_distance_marginalised"] = leg
            leg = distance_leg(first, centres, max(args.steps // 4, 2), prec, phase=binding.PE_PHASE_MARG,
                               time_marg=tm, n_draws=args.time_leg_draws, distance=False)
            leg["kind"] = (f"likelihood marginalised over the coalescence time (as the leg above) and the phase; "
                           f"the distance sampled")
            out["time_and_phase_marginalised"] = leg
    if n_events == 1 and D == 4 and args.tile_candidates > 0:
        out["tiles"] = tile_leg(first, args, max(args.steps, 1), prec)
    if n_events == 1 and D == 11 and args.itile_candidates > 0:
        # tc marginalised as in the time legs (nodes half the envelope's width apart over 20 ms), or sampled
        gh = first["g"].cpu().numpy()
        g_tt = gh[9, 9] - gh[9, 10] ** 2 / gh[10, 10]
        lo, hi = first["theta_inj"][9] - 0.01, first["theta_inj"][9] + 0.01
        tm = {"tc_lo": float(lo), "tc_hi": float(hi),
              "tm_points": int(math.ceil((hi - lo) / (0.5 / math.sqrt(g_tt)))) + 1}
        out["intrinsic_tiles"] = intrinsic_tile_leg(first, args, max(args.steps // 4, 2), prec,
                                                    time_marg=tm if args.itile_time else None)
        if args.itile_time:
            # the same chain with tc drawn with the extrinsic coordinates (no time marginal)
            out["intrinsic_tiles_tc_sampled"] = intrinsic_tile_leg(first, args, max(args.steps // 4, 2), prec)
    if n_events == 1 and D == 11 and args.imatch_samples > 0:
        out["intrinsic_match_tiles"] = intrinsic_match_leg(first, args, max(args.steps // 4, 2), prec)
    for x in evs:
        x["ev"].close()

    # the proposal with the highest ESS per second on this event (whole chains for the tile legs)
    cands = {"gaussian_at_injection": out["ess_per_s"]}
    for k in ("distance_marginalised", "phase_and_distance_marginalised", "time_phase_and_distance_marginalised",
              "time_and_phase_marginalised"):
        for cn, v in out.get(k, {}).items():
            if isinstance(v, dict) and "ess_per_s" in v:
                cands[f"{k}/{cn}"] = v["ess_per_s"]
    if "refined" in out and "ess_per_s" in out["refined"]:
        cands["refined"] = out["refined"]["ess_per_s"]
    if "tiles" in out:
        cands["tiles"] = out["tiles"]["ess_per_s"]
    for k in ("intrinsic_tiles", "intrinsic_tiles_tc_sampled"):
        if k in out:
            cands[k] = out[k]["ess_per_s_chain"]
    best = max(cands, key=lambda k: cands[k])
    out["ess_per_s_best"] = {"value": cands[best], "leg": best}
    c2_inputs = None
    if c == 1 and not args.no_batch_leg:
        out["config2"] = batch_leg(2, max(args.steps, 1), prec)
        c2_inputs = out["config2"].pop("_cpu_inputs")
    if c == 1 and args.long_steps > 0:
        out["config4"] = long_leg(args.long_steps, args.long_loud_snr, prec)
    if args.serve_events > 0:
        out["serving"] = serve_bench(args)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(c, args.cpu_sample, first["data"], first["psd"], first["theta_inj"],
                                           first["amp0"], first["common"])
        if c == 1:
            out["cpu_baseline"]["config0_full"] = cpu_config0()
            if "config4" in out:
                out["cpu_baseline"]["config4_sample"] = out["config4"]["snr_43"]["drift"]["oracle_rate"]
            if c2_inputs:
                out["cpu_baseline"]["config2_sample"] = cpu_config2(c2_inputs)
    print(json.dumps(out), flush=True)


def vector_fraction(draw_bins, terms, n_det, t_s):
    """Vector-ALU fraction of the split hot kernel by algorithmic FLOPs: FP64 (phase polynomial per
    (draw, bin), time shift and fract per term) against 78.6 TFLOP/s plus FP32 (complex MAC per term)
    against 157.3 TFLOP/s, over the kernel's average launch time."""
    if not t_s > 0:
        return None
    f64 = draw_bins * PSI_FLOP64_PER_DRAW_BIN + terms * FLOP64_PER_TERM
    f32 = terms * FLOP32_PER_TERM
    return {"frac": f64 / (FP64_PEAK * t_s) + f32 / (FP32_PEAK * t_s), "flop64_per_launch": f64,
            "flop32_per_launch": f32, "fp64_tflops": f64 / t_s / 1e12, "fp32_tflops": f32 / t_s / 1e12,
            "counts": "per term: FP64 24/n_det + 3, FP32 8 (sine/cosine not counted)"}


def batch_leg(c, steps, prec):
    """Config 2: 64 BBH-mass events of 2^14..2^18 draws, every stage one set of launches over the batch
    (pe_batch_run), the hot loop's plan from the autotuner. Evals/s, ESS/s, the batch's latency and the
    hot kernel's share."""
    import numpy as np
    import torch

    from paper_2410_05190_amd import binding, synth

    cfg = synth.CONFIGS[c]
    n_ev = cfg.get("batch", 64)
    Ns = synth.n_draws_batch(c, n_ev)
    evs = [make_event(c, e, N) for e, N in enumerate(Ns)]
    st = torch.zeros((steps, n_ev, 4), dtype=torch.float64, device="cuda")
    kname = "loglike_split" if prec == binding.PE_PREC_SPLIT else "loglike_fp64"

    def step(i, rows):
        items = [binding.make_item(x["ev"], n=x["N"], data=x["data"], psd=x["psd"], theta0=x["theta0"],
                                   seed=x["seed"], stream_id=i, g=x["g"], theta=x["theta"], logq=x["lq"],
                                   logprior=x["lp"], loglike=x["ll"], w=x["w"], stats=rows[e])
                 for e, x in enumerate(evs)]
        binding.pe_batch_run(items, binding.PE_STAGE_ALL, prec)

    keep = binding.pe_get_plan()
    for i in range(3):
        step(900 + i, st[0])
    torch.cuda.synchronize()
    it, mb, best = binding.pe_autotune_plan([x["ev"] for x in evs], [x["theta"] for x in evs],
                                            [x["N"] for x in evs], prec, reps=2)
    binding.pe_set_plan(it, mb)
    for i in range(10):  # warm-up at the tuned plan (first-use costs of the plan's shapes)
        step(950 + i, st[0])
    binding.pe_profile_enable(True)
    binding.pe_profile_read(kname)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        step(i, st[i])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    binding.pe_profile_enable(False)
    k_ms, k_n = binding.pe_profile_read(kname)
    binding.pe_set_plan(*keep)
    for x in evs:
        x["ev"].status()
    s = st.cpu().numpy()
    wall = t1 - t0
    redo = [binding.pe_loglike_counts(x["ev"]) for x in evs]
    # the first four events' data and draw counts, for the oracle's timing of the same events
    cpu_inputs = [dict(data=x["data"].cpu().numpy(), psd=x["psd"].cpu().numpy(), theta_inj=x["theta_inj"],
                       amp0=x["amp0"], common=x["common"], N=x["N"]) for x in evs[:4]]
    for x in evs:
        x["ev"].close()
    return {"_cpu_inputs": cpu_inputs,
            "workload": cfg["name"], "events_per_step": n_ev, "draws_per_step": int(sum(Ns)),
            "n_bins": synth.grid(c)[2], "n_det": cfg["n_det"], "steps": steps, "ms_per_step": 1e3 * wall / steps,
            "evals_per_s": float(s[:, :, 3].sum()) / wall, "ess_per_s": float(s[:, :, 0].sum()) / wall,
            "ess_per_event_mean": float(s[:, :, 0].mean()), "hot_kernel_ms_avg": k_ms / max(k_n, 1),
            "plan": {"items_target": it, "min_group_bins": mb, "autotune_best_loglike_ms": best},
            "split_reevaluated_fp64": int(sum(r[1] for r in redo)),
            "kind": "every stage one set of launches over the 64 events (pe_batch_run)"}


def long_leg(steps, loud_snr, prec):
    """Config 4 (3 detectors, K = 2 086 912, 262 144 draws): the benchmark step on event 0 (SNR 43) and
    on event 1 at SNR `loud_snr` (the top of the configuration's range), each after one untimed step.
    Step time, hot-kernel time, the draws the split path re-evaluated in FP64, and the FP64-phase drift
    against the oracle (1024 draws of SNR 43, 256 of the loud event)."""
    import torch

    from paper_2410_05190_amd import binding, synth

    kname = "loglike_split" if prec == binding.PE_PREC_SPLIT else "loglike_fp64"
    N = synth.CONFIGS[4]["n_draws"]
    res = {"workload": synth.CONFIGS[4]["name"], "n_bins": synth.grid(4)[2], "draws_per_event": N}
    for key, e, snr, n_drift in (("snr_43", 0, None, 1024), ("snr_loud", 1, loud_snr, 256)):
        x = make_event(4, e, N, snr=snr)
        h_ = x["ev"].handle
        st = torch.zeros((steps, 4), dtype=torch.float64, device="cuda")
        binding.pe_profile_enable(True)
        for i in range(-1, steps):
            if i == 0:
                torch.cuda.synchronize()
                binding.pe_profile_read(kname)
                binding.pe_profile_read("loglike_redo")
                t0 = time.perf_counter()
            binding.pe_event_update(h_, x["data"], x["psd"])
            binding.pe_metric(h_, x["theta0"], None, 0, x["g"])
            binding.pe_draw(h_, x["theta0"], x["g"], x["seed"], max(i, 0), N, x["theta"], x["lq"], x["lp"])
            binding.pe_loglike_batch(h_, x["theta"], N, prec, x["ll"], None)
            binding.pe_weights_ess(x["ll"], x["lp"], x["lq"], N, x["w"], st[max(i, 0)])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        binding.pe_profile_enable(False)
        k_ms, k_n = binding.pe_profile_read(kname)
        r_ms, r_n = binding.pe_profile_read("loglike_redo")
        live, redo = binding.pe_loglike_counts(x["ev"])
        x["ev"].status()
        s = st.cpu().numpy()
        res[key] = {"snr": float(snr) if snr else float(synth.injection(4, e)["snr"]), "steps": steps,
                    "ms_per_step": 1e3 * (t1 - t0) / steps, "evals_per_s": float(s[:, 3].sum()) / (t1 - t0),
                    "ess_per_event_mean": float(s[:, 0].mean()), "hot_kernel_ms_avg": k_ms / max(k_n, 1),
                    "reevaluation_ms_avg": r_ms / max(r_n, 1), "live_last_step": live,
                    "reevaluated_fp64_last_step": redo,
                    "drift": drift_leg(x, n_drift, prec)}
        x["ev"].close()
        del x
    res["loud_over_quiet_step_time"] = res["snr_loud"]["ms_per_step"] / res["snr_43"]["ms_per_step"]
    return res


def refine_leg(x, rounds, n_round, steps, prec):
    """Proposal refinement (pe_refine: `rounds` rounds of metric, draws, likelihood, weights and
    weighted-centre update from the injection-centred start), then `steps` full steps (event
    update, metric, N draws, likelihood, weights) at the refined centre. ESS per event and ESS/s
    of the refined proposal, with and without the refinement's own cost."""
    import torch

    from paper_2410_05190_amd import binding
    h_ = x["ev"].handle
    N = x["N"]
    dev = x["theta0"].device
    t0 = x["theta0"].clone()
    g = torch.empty_like(x["g"])
    st_r = torch.empty((rounds, 4), dtype=torch.float64, device=dev)
    st_f = torch.empty((steps, 4), dtype=torch.float64, device=dev)
    bufs = [torch.empty((x["ev"].dim, n_round), dtype=torch.float64, device=dev)] + \
           [torch.empty(n_round, dtype=torch.float64, device=dev) for _ in range(4)]
    x["ev"].reserve(max(N, n_round))
    # one untimed refinement from a different seed first (first-use costs of the round size)
    binding.pe_refine(h_, t0.clone(), g, rounds, n_round, x["seed"] + 5, prec, *bufs, st_r)
    torch.cuda.synchronize()
    ta = time.perf_counter()
    binding.pe_refine(h_, t0, g, rounds, n_round, x["seed"] + 7, prec, *bufs, st_r)
    torch.cuda.synchronize()
    tb = time.perf_counter()
    for i in range(steps):
        binding.pe_event_update(h_, x["data"], x["psd"])
        binding.pe_metric(h_, t0, None, 0, g)
        binding.pe_draw(h_, t0, g, x["seed"] + 11, i, N, x["theta"], x["lq"], x["lp"])
        binding.pe_loglike_batch(h_, x["theta"], N, prec, x["ll"], None)
        binding.pe_weights_ess(x["ll"], x["lp"], x["lq"], N, x["w"], st_f[i])
    torch.cuda.synchronize()
    tc = time.perf_counter()
    x["ev"].status()
    sr = st_r.cpu().numpy()
    sf = st_f.cpu().numpy()
    ess_f = float(sf[:, 0].mean())
    t_ref, t_step = tb - ta, (tc - tb) / steps
    return {
        "kind": "proposal recentred on the weighted mean of the draws, metric at the new centre (pe_refine)",
        "rounds": rounds, "draws_per_round": n_round, "ess_per_round": [float(v) for v in sr[:, 0]],
        "refine_ms": 1e3 * t_ref, "steps": steps, "draws_per_step": N, "ms_per_step": 1e3 * t_step,
        "ess_per_event_mean": ess_f, "efficiency": ess_f / N,
        "ess_per_s": ess_f / t_step,
        "ess_per_s_with_refine": ess_f / (t_ref + t_step),
        "evals_per_s": float(sf[:, 3].sum()) / (tc - tb),
        "centre": [float(v) for v in t0.cpu().numpy()],
    }


def mixture_leg(x, centre, k, steps, prec, n_pilot=16384):
    """A small mixture of metric Gaussians (pe_mixture_logq). A pilot round of the single Gaussian
    at `centre` (metric there, n_pilot draws, likelihoods, weights) picks its k heaviest draws; each
    becomes a component centred there with the metric at that point and a share of 3/4 in
    proportion to its weight; the single Gaussian keeps 1/4, so the mixture still covers what the
    pilot covered. Each step: the event's N draws stratified over the components (pe_draw per
    component; N pi_m each), the mixture's log q at all of them (pe_mixture_logq), likelihoods and
    weights. ESS per event and ESS/s, with and without the pilot and metrics, beside the pilot's."""
    import numpy as np
    import torch

    from paper_2410_05190_amd import binding
    h_ = x["ev"].handle
    N, D = x["N"], x["ev"].dim
    dev = centre.device
    f64 = dict(dtype=torch.float64, device=dev)
    x["ev"].reserve(max(N, n_pilot))
    tp = [torch.empty((D, n_pilot), **f64)] + [torch.empty(n_pilot, **f64) for _ in range(4)]
    st_p = torch.empty(4, **f64)

    def setup(seed):
        g0 = torch.empty((D, D), **f64)
        binding.pe_event_update(h_, x["data"], x["psd"])
        binding.pe_metric(h_, centre, None, 0, g0)
        binding.pe_draw(h_, centre, g0, seed, 0, n_pilot, tp[0], tp[1], tp[2])
        binding.pe_loglike_batch(h_, tp[0], n_pilot, prec, tp[3], None)
        binding.pe_weights_ess(tp[3], tp[2], tp[1], n_pilot, tp[4], st_p)
        top = torch.topk(tp[4], k)
        cens = torch.cat([centre[None, :], tp[0][:, top.indices].T]).contiguous()
        gs = torch.empty((k + 1, D, D), **f64)
        gs[0].copy_(g0)
        for m in range(1, k + 1):
            binding.pe_metric(h_, cens[m].contiguous(), None, 0, gs[m])
        wt = top.values.cpu().numpy()
        share = wt / wt.sum() if wt.sum() > 0 else np.full(k, 1.0 / k)
        return cens, gs, np.concatenate([[0.25], 0.75 * share])

    setup(x["seed"] + 21)  # untimed: first-use costs
    torch.cuda.synchronize()
    ta = time.perf_counter()
    cens, gs, pis = setup(x["seed"] + 23)
    torch.cuda.synchronize()
    tb = time.perf_counter()
    counts = np.floor(N * pis).astype(int)
    counts[int(np.argmax(pis))] += N - int(counts.sum())
    offs = np.concatenate([[0], np.cumsum(counts)])
    part = [(torch.empty((D, max(int(c), 1)), **f64), torch.empty(max(int(c), 1), **f64),
             torch.empty(max(int(c), 1), **f64)) for c in counts]
    st_f = torch.empty((steps, 4), **f64)

    def step(i, row):
        for m, c in enumerate(counts):
            if c == 0:
                continue
            th_m, lq_m, lp_m = part[m]
            binding.pe_draw(h_, cens[m], gs[m], x["seed"] + 29, 16 * i + m, int(c), th_m, lq_m, lp_m)
            x["theta"][:, offs[m]:offs[m + 1]].copy_(th_m[:, :c])
            x["lp"][offs[m]:offs[m + 1]].copy_(lp_m[:c])
        binding.pe_mixture_logq(h_, pis, cens, gs, x["theta"], N, x["lq"])
        binding.pe_loglike_batch(h_, x["theta"], N, prec, x["ll"], None)
        binding.pe_weights_ess(x["ll"], x["lp"], x["lq"], N, x["w"], row)

    step(1000, st_f[0])  # untimed
    torch.cuda.synchronize()
    tc = time.perf_counter()
    for i in range(steps):
        step(i, st_f[i])
    torch.cuda.synchronize()
    td = time.perf_counter()
    x["ev"].status()
    sf = st_f.cpu().numpy()
    ess_f = float(sf[:, 0].mean())
    t_setup, t_step = tb - ta, (td - tc) / steps
    return {
        "kind": "mixture of metric Gaussians at the pilot round's heaviest draws plus the pilot's own "
                "(pe_mixture_logq; draws stratified over the components)",
        "components": int(k + 1), "weights": [float(v) for v in pis], "pilot_draws": n_pilot,
        "pilot_ess": float(st_p[0].item()), "setup_ms": 1e3 * t_setup, "steps": steps, "draws_per_step": N,
        "ms_per_step": 1e3 * t_step, "ess_per_event_mean": ess_f, "efficiency": ess_f / N,
        "ess_per_s": ess_f / t_step, "ess_per_s_with_setup": ess_f / (t_setup + t_step),
        "evals_per_s": float(sf[:, 3].sum()) / (td - tc),
    }


def relbin_leg(x, eps, steps, prec):
    """Relative binning about the injection (the trigger point): the same step as the main leg
    (event update, metric, N draws, likelihoods, weights) with relative-binning likelihoods, and
    the binning error against the main leg's precision on the last step's draws."""
    import numpy as np
    import torch

    from paper_2410_05190_amd import binding
    ev = x["ev"]
    h_ = ev.handle
    N = x["N"]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev.relbin_setup(x["theta0"], eps)
    t1 = time.perf_counter()
    n_edges = len(ev.relbin_edges())
    st = torch.empty((steps, 4), dtype=torch.float64, device="cuda")
    for i in range(-1, steps):  # step -1: untimed warm-up
        if i == 0:
            torch.cuda.synchronize()
            t2 = time.perf_counter()
        binding.pe_event_update(h_, x["data"], x["psd"])
        binding.pe_metric(h_, x["theta0"], None, 0, x["g"])
        binding.pe_draw(h_, x["theta0"], x["g"], x["seed"], max(i, 0), N, x["theta"], x["lq"], x["lp"])
        binding.pe_loglike_batch(h_, x["theta"], N, binding.PE_PREC_RELBIN, x["ll"], None)
        binding.pe_weights_ess(x["ll"], x["lp"], x["lq"], N, x["w"], st[max(i, 0)])
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    ll_rb = x["ll"].clone()
    binding.pe_loglike_batch(h_, x["theta"], N, prec, x["ll"], None)
    torch.cuda.synchronize()
    ev.status()
    a, b = ll_rb.cpu().numpy(), x["ll"].cpu().numpy()
    f = np.isfinite(b)
    err = np.abs(a[f] - b[f])
    # where the weights are: ln L within 20 of the largest (the far tails carry no weight)
    core = b[f] > b[f].max() - 20.0 if err.size else np.zeros(0, dtype=bool)
    s = st.cpu().numpy()
    t_step = (t3 - t2) / steps
    return {
        "kind": "relative binning about the trigger point (per-bin sums of the fiducial-phased data)",
        "eps": eps, "edges": n_edges, "setup_ms": 1e3 * (t1 - t0), "steps": steps, "draws_per_step": N,
        "ms_per_step": 1e3 * t_step, "evals_per_s": float(s[:, 3].sum()) / (t3 - t2),
        "ess_per_event_mean": float(s[:, 0].mean()), "ess_per_s": float(s[:, 0].mean()) / t_step,
        "abs_dlnL_vs_main_precision": {"max": float(err.max()) if err.size else None,
                                       "median": float(np.median(err)) if err.size else None,
                                       "draws": int(err.size),
                                       "max_within_20_of_peak": float(err[core].max()) if core.any() else None,
                                       "draws_within_20_of_peak": int(core.sum())},
    }


def distance_leg(x, centres, steps, prec, phase=None, time_marg=None, n_draws=None, distance=True):
    """Distance-marginalised likelihood (PE_DIST_MARG: the likelihood integrated over the dL^2
    prior per draw; the metric, draws and prior without dL): the same step as the main leg on a
    second event over the same data, at each proposal centre (the injection, and the refined
    centre of the refinement leg when it ran). ESS per event and ESS/s. phase=PE_PHASE_MARG also
    marginalises the coalescence phase (ln I0 form; phic left out of the proposal density);
    time_marg = {tc_lo, tc_hi, tm_points} also the coalescence time (the likelihood integrated over
    tm_points nodes spanning the window, tc left out of the proposal density); distance=False keeps
    the distance sampled."""
    import torch

    from paper_2410_05190_amd import binding
    common = dict(x["common"])
    if phase is not None:
        common["phase"] = phase
    if time_marg:
        common.update(time_marg=1, **time_marg)
    ev = binding.Event(x["data"], x["psd"], amp0=x["amp0"],
                       distance=binding.PE_DIST_MARG if distance else binding.PE_DIST_SAMPLED, **common)
    N = n_draws or x["N"]
    ev.reserve(N)
    h_ = ev.handle
    g = torch.empty_like(x["g"])
    res = {"kind": "likelihood marginalised over the luminosity distance (dL^2 prior), per draw in FP64"}
    for name, t0 in centres.items():
        st = torch.empty((steps, 4), dtype=torch.float64, device="cuda")
        for i in range(-1, steps):  # step -1: untimed warm-up
            if i == 0:
                torch.cuda.synchronize()
                ta = time.perf_counter()
            binding.pe_event_update(h_, x["data"], x["psd"])
            binding.pe_metric(h_, t0, None, 0, g)
            binding.pe_draw(h_, t0, g, x["seed"] + 13, max(i, 0), N, x["theta"], x["lq"], x["lp"])
            binding.pe_loglike_batch(h_, x["theta"], N, prec, x["ll"], None)
            binding.pe_weights_ess(x["ll"], x["lp"], x["lq"], N, x["w"], st[max(i, 0)])
        torch.cuda.synchronize()
        tb = time.perf_counter()
        ev.status()
        s = st.cpu().numpy()
        ess = float(s[:, 0].mean())
        t_step = (tb - ta) / steps
        res[name] = {"steps": steps, "draws_per_step": N, "ms_per_step": 1e3 * t_step,
                     "evals_per_s": float(s[:, 3].sum()) / (tb - ta), "ess_per_event_mean": ess,
                     "efficiency": ess / N, "ess_per_s": ess / t_step}
    ev.close()
    return res


def tile_leg(x, args, steps, prec):
    """Tile-mixture proposal: the precompute (stochastic bank and prior samples in the slice around
    the trigger, nearest-template assignment), then `steps` online steps (likelihood at every
    template, N proposal draws, their likelihoods, weights). ESS per event and ESS/s."""
    import numpy as np
    import torch

    from paper_2410_05190_amd import binding
    ev = x["ev"]
    h_ = ev.handle
    N = x["N"]
    binding.pe_metric(h_, x["theta0"], None, 0, x["g"])
    L = np.linalg.cholesky(x["g"].cpu().numpy())
    sl = binding.make_slice(x["theta_inj"], L, args.tile_radius)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ty, tth, used = ev.tile_bank(sl, args.tile_spacing, x["seed"], 1, 4096, 200000, 0.002, 2000)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    y, th, lp = ev.slice_sample(sl, x["seed"], 2, 0, args.tile_candidates)
    to = binding.tile_assign(ty, y)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    tth = tth.contiguous()
    M = tth.shape[1]
    llt = torch.empty(M, dtype=torch.float64, device="cuda")
    st = torch.empty((steps, 4), dtype=torch.float64, device="cuda")
    ev.reserve(max(M, N))
    st2 = torch.empty((steps, 4), dtype=torch.float64, device="cuda")
    for i in range(-1, steps):  # step -1: untimed warm-up (first-use costs)
        if i == 0:
            torch.cuda.synchronize()
            t_on = time.perf_counter()
        binding.pe_loglike_batch(h_, tth, M, prec, llt, None)
        thd, lq, lpd, idx = binding.tile_draw(llt, to, lp, th, x["seed"] + 3, max(i, 0), N)
        binding.pe_loglike_batch(h_, thd, N, prec, x["ll"], None)
        binding.pe_weights_ess(x["ll"], lpd, lq, N, x["w"], st[max(i, 0)])
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    # two rounds per step: the second draws from the tiles reweighted by the first round's weights
    for i in range(-1, steps):
        if i == 0:
            torch.cuda.synchronize()
            t4 = time.perf_counter()
        binding.pe_loglike_batch(h_, tth, M, prec, llt, None)
        thd, lq, lpd, idx = binding.tile_draw(llt, to, lp, th, x["seed"] + 5, 2 * max(i, 0), N)
        binding.pe_loglike_batch(h_, thd, N, prec, x["ll"], None)
        binding.pe_weights_ess(x["ll"], lpd, lq, N, x["w"], st[max(i, 0)])
        ell = binding.tile_reweight(llt, to, lp, idx, x["w"], 0.1)
        thd, lq, lpd, idx = binding.tile_draw(ell, to, lp, th, x["seed"] + 5, 2 * max(i, 0) + 1, N)
        binding.pe_loglike_batch(h_, thd, N, prec, x["ll"], None)
        binding.pe_weights_ess(x["ll"], lpd, lq, N, x["w"], st2[max(i, 0)])
    torch.cuda.synchronize()
    t5 = time.perf_counter()
    # the same online step with the samples tiled by waveform match (App. A) among their 8 nearest
    # templates instead of by whitened distance
    torch.cuda.synchronize()
    t6 = time.perf_counter()
    tom, mv = binding.tile_assign_match(ev, ty, tth, y, th, n_cand=8)
    torch.cuda.synchronize()
    t7 = time.perf_counter()
    st3 = torch.empty((steps, 4), dtype=torch.float64, device="cuda")
    for i in range(-1, steps):
        binding.pe_loglike_batch(h_, tth, M, prec, llt, None)
        thd, lq, lpd, idx = binding.tile_draw(llt, tom, lp, th, x["seed"] + 3, max(i, 0), N)
        binding.pe_loglike_batch(h_, thd, N, prec, x["ll"], None)
        binding.pe_weights_ess(x["ll"], lpd, lq, N, x["w"], st3[max(i, 0)])
    torch.cuda.synchronize()
    moved = float((tom != to).double().mean())
    ev.status()
    s = st.cpu().numpy()
    s2 = st2.cpu().numpy()
    s3 = st3.cpu().numpy()
    ess = float(s[:, 0].mean())
    ess2 = float(s2[:, 0].mean())
    t_step = (t3 - t_on) / steps
    t_step2 = (t5 - t4) / steps
    return {
        "kind": "tile mixture: templates in the whitened slice, prior samples weighted by their tile's likelihood",
        "slice_radius": args.tile_radius, "spacing": args.tile_spacing, "templates": M,
        "bank_candidates": used, "prior_samples": int(y.shape[1]), "bank_ms": 1e3 * (t1 - t0),
        "samples_and_assign_ms": 1e3 * (t2 - t1), "steps": steps, "draws_per_step": N,
        "ms_per_step": 1e3 * t_step, "ess_per_event_mean": ess, "efficiency": ess / N,
        "ess_per_event_min": float(s[:, 0].min()), "ess_per_event_max": float(s[:, 0].max()),
        "ess_per_s": ess / t_step, "evals_per_s": (M + N) / t_step,
        "reweighted": {"kind": "second round from the tiles reweighted by the first round's weights "
                               "(defensive share 0.1); ESS of the second round",
                       "ms_per_step": 1e3 * t_step2, "ess_per_event_mean": ess2, "efficiency": ess2 / N,
                       "ess_per_event_min": float(s2[:, 0].min()), "ess_per_event_max": float(s2[:, 0].max()),
                       "ess_per_s": ess2 / t_step2},
        "match_tiles": {"kind": "samples tiled by waveform match (overlap maximised over a constant phase) "
                                "among their 8 nearest templates; the first-round step as above",
                        "assign_ms": 1e3 * (t7 - t6), "share_reassigned": moved,
                        "mean_match": float(mv.mean()), "ess_per_event_mean": float(s3[:, 0].mean()),
                        "ess_per_event_min": float(s3[:, 0].min()), "ess_per_event_max": float(s3[:, 0].max())},
    }


def intrinsic_tile_leg(x, args, steps, prec, time_marg=None):
    """Tile mixture over the intrinsic coordinates of the 11-D set (Sec. III: the intrinsic parameters
    are tiled, the extrinsic ones partially decouple), iterated (the proposal update the paper suggests
    at the end of Sec. III.A): the likelihood marginalised over the phase and the distance (and the
    coalescence time with time_marg); a bank and prior samples in the ball of the proposal's marginal
    metric over (Mc, q, chi1z, chi2z) about the injection, nearest-template tiles. One step is a chain
    of R rounds of N draws: round 1 weights the tiles by their template's likelihood (extrinsic
    coordinates at the injection) and draws the other coordinates from the metric proposal's marginal;
    each later round reweights the tiles by the previous round's weights and draws the other
    coordinates from a Gaussian with the previous round's weighted centre and covariance over them.
    The injection-centred Gaussian on the same event is timed beside it."""
    import numpy as np
    import torch

    from paper_2410_05190_amd import binding
    common = dict(x["common"])
    common["phase"] = binding.PE_PHASE_MARG
    if time_marg:
        common.update(time_marg=1, **time_marg)
    ev = binding.Event(x["data"], x["psd"], amp0=x["amp0"], distance=binding.PE_DIST_MARG, **common)
    N = x["N"]
    R = max(1, args.itile_rounds)
    h_ = ev.handle
    th0 = x["theta0"]
    g = ev.metric(th0)
    gh = g.cpu().numpy()
    GI = np.linalg.inv(np.linalg.inv(gh)[:4, :4])
    sl = binding.make_slice(x["theta_inj"], np.linalg.cholesky(GI), args.itile_radius, 0xF)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ty, tth, used = ev.tile_bank(sl, args.itile_spacing, x["seed"], 1, 4096, 200000, 0.002, 2000)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    y, th, lp = ev.slice_sample(sl, x["seed"], 2, 0, args.itile_candidates)
    to = binding.tile_assign(ty, y)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    tth = tth.contiguous()
    M = tth.shape[1]
    ev.reserve(max(M, N))
    f64 = dict(dtype=torch.float64, device="cuda")
    llt = torch.empty(M, **f64)
    ll = torch.empty(N, **f64)
    w = torch.empty(N, **f64)
    st = torch.empty((steps, R, 4), **f64)
    c2 = torch.empty(11, **f64)
    cov = torch.empty((11, 11), **f64)
    ext = [4, 5, 6, 7] + ([] if time_marg else [9])  # the coordinates drawn besides the tiles
    print(f"intrinsic tiles: {M} templates, {y.shape[1]} samples, {R} rounds", file=sys.stderr, flush=True)
    t_rounds = np.zeros(R)
    modes = ["marginal"] * R  # of the extrinsic completion, by round (last step)
    for i in range(-1, steps):  # step -1: untimed warm-up
        if i == 0:
            torch.cuda.synchronize()
            ta = time.perf_counter()
        s = max(i, 0)
        binding.pe_loglike_batch(h_, tth, M, prec, llt, None)
        vals, c, gg, flags = llt, th0, g, 0
        for r in range(R):
            tr = time.perf_counter()
            thd, lq, lpd, idx = binding.tile_draw(vals, to, lp, th, x["seed"] + 7, R * s + r, N)
            binding.pe_tile_extrinsic(h_, c, gg, 0xF, flags, x["seed"] + 8, R * s + r, N, thd, lq, lpd)
            binding.pe_loglike_batch(h_, thd, N, prec, ll, None)
            binding.pe_weights_ess(ll, lpd, lq, N, w, st[s, r])
            if r + 1 < R:
                # the next round: the tiles reweighted; the other coordinates from the weighted Gaussian of
                # this round, given each draw's intrinsic point once the round has the effective samples
                # to estimate that regression (20 per coordinate), else from its marginal
                vals = binding.tile_reweight(vals, to, lp, idx, w, 0.1)
                binding.pe_proposal_update(h_, thd, w, N, c, c2, cov)
                keep = [0, 1, 2, 3] + ext
                cond = float(st[s, r, 0]) >= 20 * len(keep)
                sel = keep if cond else ext
                gm = np.eye(11)
                gm[np.ix_(sel, sel)] = np.linalg.inv(cov.cpu().numpy()[np.ix_(sel, sel)])
                c, gg, flags = c2.clone(), torch.from_numpy(gm).cuda(), binding.PE_TILE_CONDITIONAL if cond else 0
                modes[r + 1] = "conditional" if cond else "marginal"
            if i >= 0:
                torch.cuda.synchronize()
                t_rounds[r] += time.perf_counter() - tr
    torch.cuda.synchronize()
    tb = time.perf_counter()
    # the injection-centred Gaussian on the same event
    stg = torch.empty((steps, 4), **f64)
    for i in range(-1, steps):
        if i == 0:
            torch.cuda.synchronize()
            tc = time.perf_counter()
        binding.pe_draw(h_, th0, g, x["seed"] + 9, max(i, 0), N, x["theta"], x["lq"], x["lp"])
        binding.pe_loglike_batch(h_, x["theta"], N, prec, ll, None)
        binding.pe_weights_ess(ll, x["lp"], x["lq"], N, w, stg[max(i, 0)])
    torch.cuda.synchronize()
    td = time.perf_counter()
    ev.status()
    ev.close()
    s_, sg = st.cpu().numpy(), stg.cpu().numpy()
    t_step = (tb - ta) / steps
    t_g = (td - tc) / steps
    ess = s_[:, :, 0].mean(0)
    eg = float(sg[:, 0].mean())
    t_last = t_rounds[-1] / steps
    return {
        "kind": ("tile mixture over (Mc, q, chi1z, chi2z), the other coordinates drawn apart; likelihood "
                 "marginalised over phase and distance" + (" and tc" if time_marg else "") + f"; {R} rounds per "
                 "step, each later round from the tiles reweighted by the previous one and the other coordinates "
                 "from the previous round's weighted Gaussian, given each draw's intrinsic point once that round "
                 "has 20 effective samples per coordinate"),
        "slice_radius": args.itile_radius, "spacing": args.itile_spacing, "templates": M, "bank_candidates": used,
        "prior_samples": int(y.shape[1]), "bank_ms": 1e3 * (t1 - t0), "samples_and_assign_ms": 1e3 * (t2 - t1),
        "steps": steps, "rounds": R, "draws_per_round": N, "ms_per_step": 1e3 * t_step,
        "ms_per_round": [float(1e3 * t / steps) for t in t_rounds],
        "ess_per_event_by_round": [float(e) for e in ess], "extrinsic_by_round": modes,
        "efficiency_last_round": float(ess[-1]) / N,
        "ess_last_round_min": float(s_[:, -1, 0].min()), "ess_last_round_max": float(s_[:, -1, 0].max()),
        "ess_per_s_last_round": float(ess[-1]) / t_last, "ess_per_s_chain": float(ess[-1]) / t_step,
        "gaussian_same_event": {"ms_per_step": 1e3 * t_g, "ess_per_event_mean": eg, "efficiency": eg / N,
                                "ess_per_s": eg / t_g},
    }


def intrinsic_match_leg(x, args, steps, prec):
    """The first round of the intrinsic tile chain (phase and distance marginalised, tc drawn) on
    tiles assigned two ways over the same bank and prior samples: the whitened-nearest template
    (pe_tile_assign) and the largest network match, maximised over the phase and a grid of time
    shifts, among the 8 nearest (pe_tile_assign_match_shift, App. A). ESS per event of the round for each, the share of samples whose tile changes, the mean
    match of each sample to its nearest and to its chosen template, and the assignment's time."""
    import numpy as np
    import torch

    from paper_2410_05190_amd import binding
    common = dict(x["common"])
    common["phase"] = binding.PE_PHASE_MARG
    ev = binding.Event(x["data"], x["psd"], amp0=x["amp0"], distance=binding.PE_DIST_MARG, **common)
    N = x["N"]
    h_ = ev.handle
    th0 = x["theta0"]
    g = ev.metric(th0)
    gh = g.cpu().numpy()
    GI = np.linalg.inv(np.linalg.inv(gh)[:4, :4])
    sl = binding.make_slice(x["theta_inj"], np.linalg.cholesky(GI), args.itile_radius, 0xF)
    ty, tth, used = ev.tile_bank(sl, args.itile_spacing, x["seed"], 1, 4096, 200000, 0.002, 2000)
    y, th, lp = ev.slice_sample(sl, x["seed"], 2, 0, args.imatch_samples)
    tth = tth.contiguous()
    M = tth.shape[1]
    ev.reserve(max(M, N))
    to_near = binding.tile_assign(ty, y)
    # the match maximised over the template's time shift too (+-16 steps of dt): the slice's whitening
    # comes from the proposal's marginal over the intrinsic coordinates, in which tc is free
    dt, J = args.imatch_dt, 16
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    to_match, mv = binding.tile_assign_match_shift(ev, ty, tth, y, th, dt, J, n_cand=8)
    torch.cuda.synchronize()
    t_match = time.perf_counter() - t0
    _, mv_near = binding.tile_assign_match_shift(ev, ty, tth, y, th, dt, J, n_cand=1)
    _, mv_fixed = binding.tile_assign_match(ev, ty, tth, y, th, n_cand=1)
    f64 = dict(dtype=torch.float64, device="cuda")
    llt = torch.empty(M, **f64)
    binding.pe_loglike_batch(h_, tth, M, prec, llt, None)
    ll = torch.empty(N, **f64)
    w = torch.empty(N, **f64)
    ess = {}
    for name, to in (("nearest", to_near), ("match", to_match)):
        st = torch.empty((steps, 4), **f64)
        for i in range(steps):
            thd, lq, lpd, idx = binding.tile_draw(llt, to, lp, th, x["seed"] + 7, i, N)
            binding.pe_tile_extrinsic(h_, th0, g, 0xF, 0, x["seed"] + 8, i, N, thd, lq, lpd)
            binding.pe_loglike_batch(h_, thd, N, prec, ll, None)
            binding.pe_weights_ess(ll, lpd, lq, N, w, st[i])
        ess[name] = [float(v) for v in st[:, 0].cpu().numpy()]
    ev.status()
    ev.close()
    changed = float((to_near != to_match).float().mean().item())
    return {
        "kind": "first round of the intrinsic tile chain (phase and distance marginalised, tc drawn) on nearest "
                "and on match tiles (largest network match, maximised over phase and time shift, among the 8 "
                "whitened-nearest templates)",
        "templates": M, "prior_samples": int(y.shape[1]), "shift_step_s": dt, "shifts": 2 * J + 1,
        "assign_match_ms": 1e3 * t_match, "tile_changed_fraction": changed,
        "mean_match_nearest_shared_tc": float(mv_fixed.mean().item()),
        "mean_match_nearest": float(mv_near.mean().item()), "mean_match_chosen": float(mv.mean().item()), "steps": steps, "draws_per_round": N,
        "ess_per_event_nearest": float(np.mean(ess["nearest"])), "ess_per_event_match": float(np.mean(ess["match"])),
        "ess_by_step": ess,
    }


def make_data(c, e, nd=None, snr=None):
    """Synthetic event e of configuration c (nd detectors: the first nd of the configuration's network)
    on the device: the injection is made by the library's own waveform (amplitude or distance set to the
    target SNR; `snr` overrides the configuration's draw), plus seeded noise. Returns the description and
    device data."""
    import numpy as np
    import torch

    from paper_2410_05190_amd import binding, synth

    cfg = synth.CONFIGS[c]
    f_lo, df, K = synth.grid(c)
    nd = nd or cfg["n_det"]
    four_d = cfg["params"] == "4d"
    params = binding.PE_PARAMS_4D if four_d else binding.PE_PARAMS_11D
    phase = binding.PE_PHASE_MARG if cfg["phase"] == "marg" else binding.PE_PHASE_EXPLICIT
    f = synth.frequencies(f_lo, df, K)
    S = np.tile(synth.psd_analytic(f), (nd, 1))
    geom = synth.detectors(c, nd)
    inj = synth.injection(c, e)
    f32 = cfg["storage"] == "f32"
    s = synth.F32_STRAIN_SCALE if f32 else 1.0
    psd_t = torch.from_numpy((S * s * s).astype(np.float32 if f32 else np.float64)).cuda()
    dl_max = cfg["dl_max"] or 1e4
    common = dict(f_lo=f_lo, df=df, strain_scale=s, params=params, phase=phase, gmst=0.0,
                  chi_max=cfg["chi_max"], dl_max=dl_max, det_geom=geom)
    pdt = binding.PE_F32 if f32 else binding.PE_F64
    ddt = binding.PE_C64 if f32 else binding.PE_C128
    theta_inj = inj["theta"].copy()
    h = torch.empty((nd, K, 2), dtype=torch.float64, device="cuda")
    snr2 = torch.zeros(1, dtype=torch.float64, device="cuda")
    desc1 = binding.make_desc(nd, K, data_dtype=ddt, psd_dtype=pdt, amp0=1.0, **common)
    binding.pe_waveform(desc1, torch.from_numpy(theta_inj).cuda(), psd_t, h, snr2)
    rho1 = math.sqrt(float(snr2.item()))
    amp0 = 0.0
    target = float(snr) if snr else inj["snr"]
    if four_d:
        amp0 = target / rho1
    else:
        theta_inj[8] = rho1 / target
    desc = binding.make_desc(nd, K, data_dtype=ddt, psd_dtype=pdt, amp0=amp0, **common)
    binding.pe_waveform(desc, torch.from_numpy(theta_inj).cuda(), psd_t, h, snr2)
    noise = torch.from_numpy(synth.noise(c, e, S, df) * s).cuda()
    data = torch.view_as_complex(h) + noise
    data = data.to(torch.complex64 if f32 else torch.complex128).contiguous()
    del noise, h
    return {"desc": desc, "data": data, "psd": psd_t, "theta_inj": theta_inj, "amp0": amp0, "common": common}


def make_event(c, e, N, nd=None, snr=None):
    """make_data plus an event with its device buffers for N draws."""
    import torch

    from paper_2410_05190_amd import binding, synth

    x = make_data(c, e, nd, snr)
    ev = binding.Event(x["data"], x["psd"], amp0=x["amp0"], **x["common"])
    ev.reserve(N)
    D = ev.dim
    f64 = dict(dtype=torch.float64, device="cuda")
    x.update({"ev": ev, "N": N, "theta0": torch.from_numpy(x["theta_inj"]).cuda(),
              "g": torch.empty((D, D), **f64), "theta": torch.empty((D, N), **f64), "lq": torch.empty(N, **f64),
              "lp": torch.empty(N, **f64), "ll": torch.empty(N, **f64), "w": torch.empty(N, **f64),
              "seed": synth.draw_seed(c, e)})
    return x


def percentiles(lat_ms):
    import numpy as np
    a = np.sort(np.asarray(lat_ms))
    return {"p50": float(np.percentile(a, 50)), "p99": float(np.percentile(a, 99)), "max": float(a[-1])}


def serve_bench(args):
    """The serving load: requests shaped like configs 1 and 2 (70/30), 1..3 detectors, 2^14..2^18 draws,
    Poisson arrivals at --serve-rate, through the serving loop (continuous batching, graph-replayed hot
    slices); then the same trace served one request at a time with the plain FP64 path (single-event
    calls, no graphs, no batching) as the baseline. Latency = completion - arrival."""
    import numpy as np
    import torch

    from paper_2410_05190_amd import binding, synth

    # a long-lived server starts from a clean device: the earlier legs' cached blocks go back first
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    tr = synth.serving_trace(args.serve_events, args.serve_rate)
    n = args.serve_events
    keys = sorted({(int(tr["shape"][i]), int(tr["n_det"][i]), int(tr["pool"][i])) for i in range(n)})
    pool = {k: make_data(k[0], synth.SERVE["pool_base"] + k[2], k[1]) for k in keys}
    torch.cuda.synchronize()
    print(f"serving: {n} requests over {tr['t'][-1]:.1f} s, pool of {len(pool)} events", file=sys.stderr, flush=True)

    def request(i):
        k = (int(tr["shape"][i]), int(tr["n_det"][i]), int(tr["pool"][i]))
        return pool[k], int(tr["n_draws"][i]), synth.draw_seed(3, i)

    srv = binding.Server(int(args.serve_budget_gib * (1 << 30)), precision=binding.PE_PREC_SPLIT, max_active=256,
                         slice_ms=args.serve_slice_ms, use_graph=not args.serve_no_graph)
    tuned = None
    if not args.serve_no_tune:
        # the server's autotuner: one plan per shape bucket from the pool events, 2^14 draws each
        f64 = dict(dtype=torch.float64, device="cuda")
        tev, tth = [], []
        for k, x in pool.items():
            ev = binding.Event(x["data"], x["psd"], amp0=x["amp0"], **x["common"])
            th0 = torch.from_numpy(x["theta_inj"]).cuda()
            g = ev.metric(th0)
            th, lq, lp = ev.draw(th0, g, 77, 1, 1 << 14)
            tev.append(ev)
            tth.append(th)
        torch.cuda.synchronize()
        ta = time.perf_counter()
        srv.tune(tev, tth, [1 << 14] * len(tev), reps=1)
        tuned = {"seconds": time.perf_counter() - ta, "events": len(tev), "draws_per_event": 1 << 14,
                 "plans": [{"n_det": p[0], "log2_bins": p[1], "items_target": p[2], "min_group_bins": p[3],
                            "ms_per_batch": p[4]} for p in srv.plans()]}
        for ev in tev:
            ev.close()
        print(f"serving: tuned {len(tuned['plans'])} shape buckets in {tuned['seconds']:.1f} s", file=sys.stderr,
              flush=True)
    # warm-up (kernel loading, graph capture): two requests, not timed
    for i in range(2):
        x, N, seed = request(i)
        srv.wait(srv.submit(x["desc"], x["data"], x["psd"], x["theta_inj"], N, seed=seed, stream_id=999))
    busy0 = srv.busy_ms()
    t0 = srv.now()
    tickets = []
    for i in range(n):
        while srv.now() - t0 < tr["t"][i]:
            time.sleep(min(0.002, max(0.0, tr["t"][i] - (srv.now() - t0))))
        x, N, seed = request(i)
        tickets.append(srv.submit(x["desc"], x["data"], x["psd"], x["theta_inj"], N, seed=seed, stream_id=i))
        if (i + 1) % 250 == 0:
            print(f"serving: {i + 1} of {n} requests submitted at {srv.now() - t0:.1f} s", file=sys.stderr,
                  flush=True)
    res = [srv.wait(t) for t in tickets]
    busy1 = srv.busy_ms()
    counters = srv.counters()
    srv.close()
    bad = [r.status for r in res if r.status not in (0, 4)]
    lat = [1e3 * (r.t_done - r.t_submit) for r in res]
    t_end = max(r.t_done for r in res) - t0
    live = sum(r.stats[3] for r in res)
    ess = sum(r.stats[0] for r in res)
    out = {"requests": n, "arrival_rate_hz": args.serve_rate, "window_s": t_end,
           "latency_ms": percentiles(lat), "evals_per_s": live / t_end, "ess_per_s": ess / t_end,
           "draws": int(sum(int(tr["n_draws"][i]) for i in range(n))), "failed": len(bad),
           "slice_ms": args.serve_slice_ms, "graph": not args.serve_no_graph, "counters": counters,
           "gpu_busy": {"slices_ms": busy1["slices"] - busy0["slices"],
                        "admission_ms": busy1["admission"] - busy0["admission"],
                        "fraction": (busy1["slices"] - busy0["slices"] + busy1["admission"] - busy0["admission"])
                        / (1e3 * t_end)},
           "tuned": tuned,
           "kind": "continuous batching, split precision, admission by HBM budget"}
    print(f"serving: p50 {out['latency_ms']['p50']:.1f} ms p99 {out['latency_ms']['p99']:.1f} ms, GPU busy "
          f"{out['gpu_busy']['fraction']:.3f}", file=sys.stderr, flush=True)

    if not args.serve_no_baseline:
        # serial plain-FP64 baseline on the same trace
        f64 = dict(dtype=torch.float64, device="cuda")
        evs = {}
        for k, x in pool.items():
            nmax = max(int(tr["n_draws"][i]) for i in range(n)
                       if (int(tr["shape"][i]), int(tr["n_det"][i]), int(tr["pool"][i])) == k)
            ev = binding.Event(x["data"], x["psd"], amp0=x["amp0"], **x["common"])
            ev.reserve(nmax)
            D = ev.dim
            evs[k] = (ev, torch.from_numpy(x["theta_inj"]).cuda(), torch.empty((D, D), **f64),
                      torch.empty((D, nmax), **f64), torch.empty(nmax, **f64), torch.empty(nmax, **f64),
                      torch.empty(nmax, **f64), torch.empty(nmax, **f64), torch.empty(4, **f64))
        torch.cuda.synchronize()
        lat0, live0, ess0 = [], 0.0, 0.0
        t0 = time.perf_counter()
        for i in range(n):
            while time.perf_counter() - t0 < tr["t"][i]:
                time.sleep(min(0.002, max(0.0, tr["t"][i] - (time.perf_counter() - t0))))
            k = (int(tr["shape"][i]), int(tr["n_det"][i]), int(tr["pool"][i]))
            x = pool[k]
            ev, th0, g, th, lq, lp, ll, w, st = evs[k]
            N = int(tr["n_draws"][i])
            h_ = ev.handle
            binding.pe_event_update(h_, x["data"], x["psd"])
            binding.pe_metric(h_, th0, None, 0, g)
            binding.pe_draw(h_, th0, g, synth.draw_seed(3, i), i, N, th, lq, lp)
            binding.pe_loglike_batch(h_, th, N, binding.PE_PREC_FP64, ll, None)
            binding.pe_weights_ess(ll, lp, lq, N, w, st)
            sv = st.cpu().numpy()
            lat0.append(1e3 * (time.perf_counter() - t0 - tr["t"][i]))
            live0 += sv[3]
            ess0 += sv[0]
        t_end0 = time.perf_counter() - t0
        for v in evs.values():
            v[0].close()
        out["baseline"] = {"kind": "same trace, one request at a time, plain FP64 path, no graphs or batching",
                           "latency_ms": percentiles(lat0), "evals_per_s": live0 / t_end0,
                           "ess_per_s": ess0 / t_end0, "window_s": t_end0}
        print(f"serving baseline: p50 {out['baseline']['latency_ms']['p50']:.1f} ms "
              f"p99 {out['baseline']['latency_ms']['p99']:.1f} ms", file=sys.stderr, flush=True)
    return out


def drift_leg(x, n_sample, prec):
    """FP64-phase drift at this shape: on the first n_sample in-support draws of the last step, ln L
    of the timed path and of the plain FP64 GPU path against the FP64 oracle (host threads), with the
    phase-rounding bound of the FP64 comparison (2 x 16 u Phi_N sum_k |t_k| at the injection)."""
    import numpy as np
    import torch

    import oracle
    from paper_2410_05190_amd import binding

    th_all = x["theta"].cpu().numpy()
    ll_all = x["ll"].cpu().numpy()
    live = np.flatnonzero(np.isfinite(ll_all))[:n_sample]
    th = np.ascontiguousarray(th_all[:, live])
    ll_fast = ll_all[live]
    ll64 = torch.empty(live.size, dtype=torch.float64, device="cuda")
    binding.pe_loglike_batch(x["ev"].handle, torch.from_numpy(th).cuda(), live.size, binding.PE_PREC_FP64, ll64)
    ll64 = ll64.cpu().numpy()
    d_h = x["data"].cpu().numpy()
    p_h = x["psd"].cpu().numpy()
    cm = x["common"]
    ev = oracle.Event(d_h.shape[0], d_h.shape[1], cm["f_lo"], cm["df"], data=d_h, psd=p_h,
                      strain_scale=cm["strain_scale"], params=cm["params"], phase=cm["phase"], amp0=x["amp0"],
                      gmst=cm["gmst"], chi_max=cm["chi_max"], dl_max=cm["dl_max"], det_geom=cm["det_geom"])
    t0 = time.perf_counter()
    ll_o = ev.loglike(th, n_threads=os.cpu_count() or 1)
    t1 = time.perf_counter()
    h = ev.waveform(x["theta_inj"])
    d = d_h.astype(np.complex128)
    S = p_h.astype(np.float64)
    sabs = float((4 * cm["df"] * np.abs(d) * np.abs(h) / S).sum())
    phin = 3.0 / 128.0 * (math.pi * x["theta_inj"][0] * oracle.t_sun() * cm["f_lo"]) ** (-5.0 / 3.0)
    bound = 2 * 16 * np.finfo(np.float64).eps * phin * sabs
    df_ = np.abs(ll_fast - ll_o)
    d64 = np.abs(ll64 - ll_o)
    threads = os.cpu_count() or 1
    terms = float(d_h.shape[0] * host_cut(th, cm, d_h.shape[1]).sum())
    rate = {"value": live.size / (t1 - t0), "unit": "likelihood evals/s", "cores": threads,
            "per_core": live.size / (t1 - t0) / threads, "terms_per_s": terms / (t1 - t0), "kind": "oracle",
            "sample": f"{live.size} in-support draws of the timed step, K = {d_h.shape[1]}"}
    return {"draws": int(live.size), "oracle_s": t1 - t0, "oracle_rate": rate,
            "phase_newtonian_rad_at_f_lo": 2 * math.pi * phin,
            "timed_path": {"precision": "split" if prec == binding.PE_PREC_SPLIT else "fp64",
                           "max_abs_dlnL": float(df_.max()), "median_abs_dlnL": float(np.median(df_)),
                           "bound": 1e-3 if prec == binding.PE_PREC_SPLIT else bound},
            "fp64_path": {"max_abs_dlnL": float(d64.max()), "median_abs_dlnL": float(np.median(d64)), "bound": bound},
            "max_abs_lnL": float(np.abs(ll_o).max())}


def cpu_baseline(c, n_sample, data, psd_t, theta_inj, amp0, common):
    """The FP64 oracle as it stands, on the host cores: its own metric and draws for the same
    event, then the log-likelihood of n_sample draws (timed) and the weights."""
    import numpy as np

    import oracle

    threads = os.cpu_count() or 1
    d_h = data.cpu().numpy()
    p_h = psd_t.cpu().numpy()
    ev = oracle.Event(d_h.shape[0], d_h.shape[1], common["f_lo"], common["df"], data=d_h, psd=p_h,
                      strain_scale=common["strain_scale"], params=common["params"], phase=common["phase"],
                      amp0=amp0, gmst=common["gmst"], chi_max=common["chi_max"], dl_max=common["dl_max"],
                      det_geom=common["det_geom"])
    t0 = time.perf_counter()
    g = ev.metric(theta_inj)
    t1 = time.perf_counter()
    rc, th, lq, lp = ev.draw(theta_inj, g, 12345, 0, 4 * n_sample)
    live = np.flatnonzero(np.isfinite(lp))[:n_sample]
    th = np.ascontiguousarray(th[:, live])
    t2 = time.perf_counter()
    ll = ev.loglike(th, n_threads=threads)
    t3 = time.perf_counter()
    oracle.weights_ess(ll, lp[live], lq[live])
    terms = float(d_h.shape[0] * host_cut(th, common, d_h.shape[1]).sum())
    return {"value": live.size / (t3 - t2), "unit": "likelihood evals/s", "cores": threads, "kind": "oracle",
            "per_core": live.size / (t3 - t2) / threads, "terms_per_s": terms / (t3 - t2),
            "terms_per_s_per_core": terms / (t3 - t2) / threads,
            "sample": f"{live.size} in-support draws of the benchmark event (oracle's own metric and draws); "
                      f"oracle metric {t1 - t0:.1f} s single-threaded, not in value"}


def cpu_config2(inputs):
    """The oracle on four events of config 2 (the batch leg's first four: same data, each event's own
    draw count), its own metric and draws per event; every in-support draw's log-likelihood timed
    on all host threads."""
    import numpy as np

    import oracle

    threads = os.cpu_count() or 1
    n_live, terms, t_ll = 0, 0.0, 0.0
    for x in inputs:
        d_h, p_h, cm = x["data"], x["psd"], x["common"]
        ev = oracle.Event(d_h.shape[0], d_h.shape[1], cm["f_lo"], cm["df"], data=d_h, psd=p_h,
                          strain_scale=cm["strain_scale"], params=cm["params"], phase=cm["phase"], amp0=x["amp0"],
                          gmst=cm["gmst"], chi_max=cm["chi_max"], dl_max=cm["dl_max"], det_geom=cm["det_geom"])
        g = ev.metric(x["theta_inj"])
        rc, th, lq, lp = ev.draw(x["theta_inj"], g, 12345, 0, x["N"])
        th = np.ascontiguousarray(th[:, np.isfinite(lp)])
        t0 = time.perf_counter()
        ev.loglike(th, n_threads=threads)
        t_ll += time.perf_counter() - t0
        n_live += th.shape[1]
        terms += float(d_h.shape[0] * host_cut(th, cm, d_h.shape[1]).sum())
    return {"value": n_live / t_ll, "unit": "likelihood evals/s", "cores": threads, "kind": "oracle",
            "per_core": n_live / t_ll / threads, "terms_per_s": terms / t_ll,
            "terms_per_s_per_core": terms / t_ll / threads,
            "sample": f"4 events of config 2 (the batch's first four, their own metric and "
                      f"{sum(x['N'] for x in inputs)} draws), {n_live} in-support draws timed"}


def cpu_config0():
    """The oracle on config 0 at full size: the 4096 draws of the event (its own metric and draws),
    all host threads."""
    import numpy as np

    import oracle
    from paper_2410_05190_amd import synth

    c = 0
    cfg = synth.CONFIGS[c]
    f_lo, df, K = synth.grid(c)
    f = synth.frequencies(f_lo, df, K)
    S = synth.psd_analytic(f)[None, :]
    geom = synth.detectors(c, 1)
    inj = synth.injection(c, 0)
    th0 = inj["theta"].copy()
    common = dict(params=oracle.PARAMS_4D, phase=oracle.PHASE_MARG, gmst=0.0, chi_max=cfg["chi_max"],
                  dl_max=cfg["dl_max"] or 1e4, det_geom=geom)
    ref = oracle.Event(1, K, f_lo, df, data=None, psd=S, strain_scale=1.0, amp0=1.0, **common)
    h1 = ref.waveform(th0)
    amp0 = inj["snr"] / math.sqrt(ref.inner(0, h1, h1))
    inj_ev = oracle.Event(1, K, f_lo, df, data=None, psd=S, strain_scale=1.0, amp0=amp0, **common)
    data = np.ascontiguousarray(inj_ev.waveform(th0) + synth.noise(c, 0, S, df), dtype=np.complex128)
    ev = oracle.Event(1, K, f_lo, df, data=data, psd=np.ascontiguousarray(S), strain_scale=1.0, amp0=amp0, **common)
    threads = os.cpu_count() or 1
    g = ev.metric(th0)
    rc, th, lq, lp = ev.draw(th0, g, 12345, 0, cfg["n_draws"])
    t0 = time.perf_counter()
    ll = ev.loglike(th, n_threads=threads)
    t1 = time.perf_counter()
    live = int(np.isfinite(ll).sum())
    terms = float(host_cut(th[:, np.isfinite(ll)], dict(f_lo=f_lo, df=df, params=oracle.PARAMS_4D), K).sum())
    return {"value": th.shape[1] / (t1 - t0), "unit": "draws/s (all 4096, in and out of support)",
            "live_evals_per_s": live / (t1 - t0), "cores": threads, "per_core": th.shape[1] / (t1 - t0) / threads,
            "terms_per_s": terms / (t1 - t0), "sample": f"config 0 at full size: {th.shape[1]} draws, K = {K}"}


def host_cut(theta, common, K):
    """ISCO cut (bins below f_isco) of each draw on the host, from the masses alone."""
    import numpy as np

    from paper_2410_05190_amd import binding
    tsun = 1.32712440018e20 / 299792458.0 ** 3
    with np.errstate(all="ignore"):
        if common["params"] == binding.PE_PARAMS_4D:
            M = theta[0] * theta[1] ** -0.6
        else:
            q = theta[1]
            M = theta[0] * (1 + q) ** 1.2 * q ** -0.6
        fisco = 1.0 / (6.0 ** 1.5 * math.pi * M * tsun)
        kc = np.clip(np.ceil((fisco - common["f_lo"]) / common["df"]), 0, K)
    return np.nan_to_num(kc)



if __name__ == "__main__":
    main()
