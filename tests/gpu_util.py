"""Helpers of the GPU tests: upload an event built by tests/events.py and run the
library through the C ABI. Every input here comes from the synthetic workload and
the CPU oracle; nothing the GPU computes is fed back to the oracle."""
import sys

import numpy as np

from paper_2410_05190_amd import binding


def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def desc_kwargs(b):
    return dict(f_lo=b.f_lo, df=b.df, strain_scale=b.strain_scale, params=b.params, phase=b.phase, amp0=b.amp0,
                gmst=b.gmst, chi_max=b.chi_max, dl_max=b.dl_max, det_geom=b.det_geom, distance=b.distance,
                time_marg=b.time_marg, tm_points=b.tm_points, tc_lo=b.tc_lo, tc_hi=b.tc_hi)


def upload_event(b):
    torch = torch_cuda()
    data = torch.from_numpy(np.ascontiguousarray(b.data)).cuda()
    psd = torch.from_numpy(np.ascontiguousarray(b.psd)).cuda()
    ev = binding.Event(data, psd, **desc_kwargs(b))
    return ev, data, psd


def dev(x):
    torch = torch_cuda()
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def fp64_tol(b):
    """Bound on |d ln L| between the FP64 path and the oracle: both evaluate the phase in FP64 by
    different algebraic routes, so each bin's phase differs by at most ~16 u |Phi|, with |Phi|
    bounded by the Newtonian phase at the band's low edge, Phi_N = 3/128 (pi Mc f_lo)^(-5/3); a
    phase error dPhi moves a term t_k by |t_k| dPhi, so |d ln L| <= 16 u Phi_N sum_k |t_k|, with
    sum_k |t_k| = sum_d sum_k 4 df |d_k| |h_k| / S_k taken at the injection; doubled for margin."""
    import math

    import oracle
    h = b.ev.waveform(b.theta_inj)
    d = b.data.astype(np.complex128)
    S = b.psd.astype(np.float64)
    sabs = float((4 * b.df * np.abs(d) * np.abs(h) / S).sum())
    phin = 3.0 / 128.0 * (math.pi * b.theta_inj[0] * oracle.t_sun() * b.f_lo) ** (-5.0 / 3.0)
    return 2 * 16 * np.finfo(np.float64).eps * phin * sabs


def fp64_draw_bounds(b, th):
    """Per-draw bounds on |d Z| (and so on |d ln L|) between the FP64 path and the oracle, for the
    draws th [D, n]: (worst, model). Each side rounds bin k's phase by at most ~16 u M_k, with M_k
    the sum of the magnitudes of the phase's terms at f_k (the PN series term by term,
    2 pi f_k (|tc| + |delay_d|), |phic| + pi/4); a phase error d_k moves the term
    t_k = 4 df conj(d_k) h_k / S_k by -i t_k d_k.
      worst = 32 u sum_k |t_k| M_k: every bin's error at its largest and aligned.
      model = 16 u (|sum_k t_k M_k| + 6 sqrt(sum_k |t_k|^2 M_k^2)): the rounding model of the two
        routes, a part proportional to M_k across the band (the rounding of the per-draw
        coefficients, which follows the terms' phases) plus per-bin roundings that are
        independent from bin to bin, whose sum is a random walk (6 standard deviations of the
        largest per-bin error); a statistical bound, within ~10x of the measured errors.
    The band-edge form of fp64_tol bounds every M_k by the Newtonian phase at f_lo and takes the
    sums at the injection. Out-of-support draws get NaN."""
    import math

    import oracle
    K = b.n_bins
    f = b.f_lo + b.df * np.arange(K)
    d = b.data.astype(np.complex128)
    S = b.psd.astype(np.float64)
    tsun = oracle.t_sun()
    u = np.finfo(np.float64).eps
    out = np.full(th.shape[1], np.nan)
    mod = np.full(th.shape[1], np.nan)
    for i in range(th.shape[1]):
        ok, src = b.ev.source(th[:, i])
        if not ok:
            continue
        h = b.ev.waveform(th[:, i])
        v = np.cbrt(math.pi * src.M * tsun * f)
        lnv = np.log(v)
        acc = np.zeros(K)
        vk = np.ones(K)
        for j in range(8):
            acc += np.abs(src.phi[j] + src.phil[j] * lnv) * vk
            vk *= v
        mpn = 3.0 / (128.0 * src.eta * v ** 5) * acc + abs(src.phic) + math.pi / 4.0
        s1 = s2 = 0.0
        s3 = 0j
        for q in range(b.n_det):
            mk = mpn + 2.0 * math.pi * f * (abs(src.tc) + abs(src.dt[q]))
            tm = 4.0 * b.df * np.conj(d[q]) * h[q] / S[q] * mk
            a = np.abs(tm)
            s1 += float(a.sum())
            s2 += float((a * a).sum())
            s3 += complex(tm.sum())
        out[i] = 32.0 * u * s1
        mod[i] = 16.0 * u * (abs(s3) + 6.0 * math.sqrt(s2))
    return out, mod
