"""Time-marginalised test events: a window about the injected tc with nodes half the narrowest
likelihood width in tc apart (1/sqrt(g_tc,tc) of the explicit-phase metric at the injection, where
|Z| is largest), and the share of the likelihood mass at the window's edges."""
import math

import numpy as np

import oracle
from events import build_event


def tm_event(cfg, event, n_bins, phase=None, distance=0, half_window=0.05, own_width=False):
    """(time-marginalised event, the same event with tc sampled, sampled-tc metric at the injection,
    the narrowest tc width). own_width: the width from the event's own metric (for a phase-marginalised
    event the envelope's width, the phase projected out) instead of the explicit-phase one."""
    b0 = build_event(cfg, event, n_bins=n_bins, phase=phase, distance=distance)
    g = b0.ev.metric(b0.theta_inj)
    if own_width:
        sig_t = 1.0 / math.sqrt(g[9, 9])
    else:
        b1 = build_event(cfg, event, n_bins=n_bins, phase=oracle.PHASE_EXPLICIT)
        sig_t = 1.0 / math.sqrt(b1.ev.metric(b1.theta_inj)[9, 9])
    tinj = b0.theta_inj[9]
    pts = int(math.ceil(2 * half_window / (0.5 * sig_t))) + 1
    tm = {"tc_lo": tinj - half_window, "tc_hi": tinj + half_window, "tm_points": pts}
    b = build_event(cfg, event, n_bins=n_bins, phase=phase, distance=distance, time_marg=tm)
    return b, b0, g, sig_t


def edge_fraction(b, b0, th, sig_t, ll_t):
    """(L(tc_lo) + L(tc_hi)) sig_t / (T L_t) per draw, from the sampled-tc oracle: the likelihood mass
    within a width of the window's edges relative to the integral."""
    T = b.tc_hi - b.tc_lo
    out = np.zeros(th.shape[1])
    for t in (b.tc_lo, b.tc_hi):
        e = th.copy()
        e[9] = t
        out += np.exp(b0.ev.loglike(e) - ll_t) * sig_t / T
    return out

