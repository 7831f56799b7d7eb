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
