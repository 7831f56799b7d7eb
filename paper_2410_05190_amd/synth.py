"""Seeded synthetic workloads: PSD, coloured Gaussian noise, detector sites and
injection parameters for the five benchmark configurations.

This module holds the workload definition only. It computes no waveform, no
inner product and no likelihood: whoever builds an event adds the injected
signal with its own waveform code. Both the GPU library's users (the
benchmark) and the CPU oracle's tests draw their inputs from here.

Streams are numpy PCG64(SeedSequence([BASE_SEED, config, event, stream])).
"""
import math

import numpy as np

BASE_SEED = 241005190

# stream identifiers inside an event's seed sequence
ST_INJECTION = 1
ST_NOISE = 2
ST_DETECTORS = 3
ST_DRAW_SEED = 4
ST_SERVE = 5

F32_STRAIN_SCALE = 1e21  # stored = physical * scale, stored PSD = physical * scale^2

CONFIGS = {
    0: dict(name="fp64-1det-4d", f_lo=40.0, f_hi=1024.0, df=1.0 / 32.0, n_det=1, params="4d", phase="marg",
            n_draws=4096, storage="f64", mc=(1.1, 1.4), q=(0.7, 1.0), chi=(-0.05, 0.05), snr=(15.0, 15.0),
            chi_max=0.4, dl_max=None),
    1: dict(name="split-3det-bns-11d", f_lo=20.0, f_hi=2048.0, df=1.0 / 256.0, n_det=3, params="11d",
            phase="explicit", n_draws=65536, storage="f32", mc=(1.1, 1.4), q=(0.7, 1.0), chi=(-0.05, 0.05),
            snr=(12.0, 25.0), chi_max=0.4, dl_max=2000.0),
    2: dict(name="split-2det-bbh-batch", f_lo=20.0, f_hi=1024.0, df=1.0 / 8.0, n_det=2, params="11d",
            phase="marg", n_draws=None, storage="f32", mtot=(20.0, 80.0), q=(0.25, 1.0), chi=(-0.8, 0.8),
            snr=(10.0, 30.0), chi_max=0.85, dl_max=20000.0, batch=64),
    4: dict(name="split-3det-long", f_lo=10.0, f_hi=2048.0, df=1.0 / 1024.0, n_det=3, params="11d",
            phase="explicit", n_draws=262144, storage="f32", mc=(1.1, 1.4), q=(0.7, 1.0), chi=(-0.05, 0.05),
            snr=(30.0, 100.0), chi_max=0.4, dl_max=2000.0),
}


def rng(config, event, stream):
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([BASE_SEED, int(config), int(event),
                                                                       int(stream)])))


def grid(config):
    c = CONFIGS[config]
    n_bins = int(round((c["f_hi"] - c["f_lo"]) / c["df"]))
    return c["f_lo"], c["df"], n_bins


def frequencies(f_lo, df, n_bins):
    return f_lo + np.arange(n_bins, dtype=np.float64) * df


def psd_analytic(f):
    """S_n(f) = 1e-49 [x^-4.14 - 5 x^-2 + 111 (1 - x^2 + x^4/2) / (1 + x^2/2)], x = f / 215 Hz."""
    x = np.asarray(f, dtype=np.float64) / 215.0
    return 1e-49 * (x ** -4.14 - 5.0 * x ** -2 + 111.0 * (1.0 - x * x + 0.5 * x ** 4) / (1.0 + 0.5 * x * x))


def detectors(config, n_det):
    """n_det L-shaped detectors: latitude asin U[-1,1], longitude U[0,2pi), x-arm azimuth U[0,2pi)
    (from north toward east). One network per configuration."""
    g = rng(config, 0, ST_DETECTORS)
    out = np.zeros((n_det, 3))
    for i in range(n_det):
        out[i, 0] = math.asin(g.uniform(-1.0, 1.0))
        out[i, 1] = g.uniform(0.0, 2.0 * math.pi)
        out[i, 2] = g.uniform(0.0, 2.0 * math.pi)
    return out


def noise(config, event, psd, df):
    """Stationary coloured Gaussian noise: Re and Im independent N(0, S/(4 df)) per bin."""
    g = rng(config, event, ST_NOISE)
    sig = np.sqrt(np.asarray(psd) / (4.0 * df))
    return sig * g.standard_normal(sig.shape) + 1j * sig * g.standard_normal(sig.shape)


def injection(config, event):
    """Injection parameters and target network SNR. Returns dict with the physical parameters and
    'theta' in the sampled parameterisation (4-D: Mc, eta, chi_eff, tc; 11-D: Mc, q, chi1, chi2, ra, dec,
    iota, psi, dL, tc, phic). In 11-D the distance is a placeholder of 1 Mpc: the event builder rescales it
    to reach 'snr'. In 4-D the amplitude is set the same way."""
    c = CONFIGS[config]
    g = rng(config, event, ST_INJECTION)
    if "mtot" in c:
        mtot = g.uniform(*c["mtot"])
        q = g.uniform(*c["q"])
        eta = q / (1.0 + q) ** 2
        mc = mtot * eta ** 0.6
    else:
        mc = g.uniform(*c["mc"])
        q = g.uniform(*c["q"])
        eta = q / (1.0 + q) ** 2
    chi1 = g.uniform(*c["chi"])
    chi2 = g.uniform(*c["chi"])
    tc = g.uniform(-0.01, 0.01)
    snr = g.uniform(*c["snr"]) if c["snr"][0] != c["snr"][1] else c["snr"][0]
    ra = g.uniform(0.0, 2.0 * math.pi)
    dec = math.asin(g.uniform(-1.0, 1.0))
    iota = math.acos(g.uniform(-1.0, 1.0))
    psi = g.uniform(0.0, math.pi)
    phic = g.uniform(0.0, 2.0 * math.pi)
    out = dict(mc=mc, q=q, eta=eta, chi1=chi1, chi2=chi2, tc=tc, snr=snr, ra=ra, dec=dec, iota=iota, psi=psi,
               phic=phic)
    if c["params"] == "4d":
        chi_eff = (chi1 + q * chi2) / (1.0 + q)
        out["theta"] = np.array([mc, eta, chi_eff, tc])
    else:
        out["theta"] = np.array([mc, q, chi1, chi2, ra, dec, iota, psi, 1.0, tc, phic])
    return out


# Serving load: Poisson arrivals of requests shaped like config 1 (BNS) or
# config 2 (BBH), each with 1..3 detectors (the first n_det of that
# configuration's network) and 2^14..2^18 draws; the event data of a request
# is one of POOL pool events per (shape, n_det).
SERVE = dict(name="serving-bns-bbh-mix", n_events=2000, rate_hz=5.0, bns_fraction=0.7, pool=4, pool_base=100)


def serving_trace(n_events, rate_hz=SERVE["rate_hz"]):
    """Arrival times (s, first at 0), shape config (1 or 2), n_det, draw count and pool index of each
    request, seeded."""
    g = rng(3, 0, ST_SERVE)
    gaps = g.exponential(1.0 / rate_hz, n_events)
    t = np.concatenate([[0.0], np.cumsum(gaps[1:])])
    shape = np.where(g.uniform(size=n_events) < SERVE["bns_fraction"], 1, 2)
    n_det = g.integers(1, 4, size=n_events)
    n_draws = 2 ** g.integers(14, 19, size=n_events)
    pool = g.integers(0, SERVE["pool"], size=n_events)
    return dict(t=t, shape=shape, n_det=n_det, n_draws=n_draws, pool=pool)


def draw_seed(config, event):
    """64-bit key of the proposal's counter-based generator for this event."""
    return int(rng(config, event, ST_DRAW_SEED).integers(0, 2 ** 63 - 1))


def n_draws_batch(config, n_events):
    """Draw counts for a batch: uniformly one of 2^14 .. 2^18."""
    g = rng(config, 0, ST_SERVE)
    return [int(2 ** g.integers(14, 19)) for _ in range(n_events)]


def to_storage(config, data, psd):
    """Storage form of an event: complex128/f64 physical (fp64 config) or scaled complex64/f32."""
    c = CONFIGS[config]
    if c["storage"] == "f64":
        return np.ascontiguousarray(data, dtype=np.complex128), np.ascontiguousarray(psd, dtype=np.float64), 1.0
    s = F32_STRAIN_SCALE
    return (np.ascontiguousarray(data * s, dtype=np.complex64), np.ascontiguousarray(psd * s * s, dtype=np.float32),
            s)
