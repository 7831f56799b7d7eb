"""FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY.

ctypes wrapper around liboracle.so (built from peo.c by oracle/build.py).
Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package; the GPU library never does. All arrays are float64 numpy
arrays; FP32/complex64 event inputs are promoted exactly before the call.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_lib = None

PARAMS_4D = 0
PARAMS_11D = 1
PHASE_MARG = 0
PHASE_EXPLICIT = 1
DIST_SAMPLED = 0
DIST_MARG = 1
MAX_DET = 4

_dp = ctypes.POINTER(ctypes.c_double)


class _Event(ctypes.Structure):
    _fields_ = [("n_det", ctypes.c_int), ("n_bins", ctypes.c_long), ("f_lo", ctypes.c_double),
                ("df", ctypes.c_double), ("data", _dp), ("psd", _dp), ("strain_scale", ctypes.c_double),
                ("params", ctypes.c_int), ("phase", ctypes.c_int), ("amp0", ctypes.c_double),
                ("gmst", ctypes.c_double), ("chi_max", ctypes.c_double), ("dl_max", ctypes.c_double),
                ("det_geom", (ctypes.c_double * 3) * MAX_DET), ("distance", ctypes.c_int),
                ("time_marg", ctypes.c_int), ("tc_lo", ctypes.c_double), ("tc_hi", ctypes.c_double)]


class _Slice(ctypes.Structure):
    _fields_ = [("centre", ctypes.c_double * 11), ("chol", ctypes.c_double * 121), ("radius", ctypes.c_double),
                ("sub_mask", ctypes.c_uint)]


class _Source(ctypes.Structure):
    _fields_ = [("in_support", ctypes.c_int), ("mc", ctypes.c_double), ("M", ctypes.c_double),
                ("eta", ctypes.c_double), ("delta", ctypes.c_double), ("chi1", ctypes.c_double),
                ("chi2", ctypes.c_double), ("tc", ctypes.c_double), ("phic", ctypes.c_double),
                ("rre", ctypes.c_double * MAX_DET), ("rim", ctypes.c_double * MAX_DET),
                ("dt", ctypes.c_double * MAX_DET), ("fisco", ctypes.c_double), ("kcut", ctypes.c_long),
                ("phi", ctypes.c_double * 8), ("phil", ctypes.c_double * 8)]


def lib():
    global _lib
    if _lib is None:
        path = os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path):
            _build.build()
        L = ctypes.CDLL(path)
        L.peo_t_sun.restype = ctypes.c_double
        L.peo_mpc_m.restype = ctypes.c_double
        L.peo_c_si.restype = ctypes.c_double
        L.peo_r_earth.restype = ctypes.c_double
        L.peo_psi.restype = ctypes.c_double
        L.peo_psi.argtypes = [ctypes.POINTER(_Source), ctypes.c_double]
        L.peo_f_isco.restype = ctypes.c_double
        L.peo_f_isco.argtypes = [ctypes.c_double]
        L.peo_kcut.restype = ctypes.c_long
        L.peo_kcut.argtypes = [ctypes.POINTER(_Event), ctypes.c_double]
        L.peo_pn_coeffs.argtypes = [ctypes.c_double] * 4 + [_dp, _dp]
        L.peo_antenna.argtypes = [_dp, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                  _dp, _dp, _dp]
        L.peo_source_from_theta.restype = ctypes.c_int
        L.peo_source_from_theta.argtypes = [ctypes.POINTER(_Event), _dp, ctypes.POINTER(_Source)]
        L.peo_waveform.argtypes = [ctypes.POINTER(_Event), _dp, ctypes.c_long, _dp]
        L.peo_inner.restype = ctypes.c_double
        L.peo_inner.argtypes = [ctypes.POINTER(_Event), ctypes.c_int, _dp, _dp]
        L.peo_log_i0.restype = ctypes.c_double
        L.peo_log_i0.argtypes = [ctypes.c_double]
        L.peo_log_dist_marg.restype = ctypes.c_double
        L.peo_log_dist_marg.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int]
        L.peo_loglike.argtypes = [ctypes.POINTER(_Event), _dp, ctypes.c_long, _dp, _dp, ctypes.c_int]
        L.peo_default_steps.argtypes = [ctypes.POINTER(_Event), _dp, _dp]
        L.peo_metric_fd.restype = ctypes.c_int
        L.peo_metric_fd.argtypes = [ctypes.POINTER(_Event), _dp, _dp, ctypes.c_int, _dp]
        L.peo_philox4x32_10.argtypes = [ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_uint32),
                                        ctypes.POINTER(ctypes.c_uint32)]
        L.peo_uniforms.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_long, ctypes.c_int, _dp]
        L.peo_draw.restype = ctypes.c_int
        L.peo_draw.argtypes = [ctypes.POINTER(_Event), _dp, _dp, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_long,
                               _dp, _dp, _dp]
        L.peo_logq_theta.restype = ctypes.c_int
        L.peo_logq_theta.argtypes = [ctypes.POINTER(_Event), _dp, _dp, _dp, ctypes.c_long, _dp]
        L.peo_mixture_logq.restype = ctypes.c_int
        L.peo_mixture_logq.argtypes = [ctypes.POINTER(_Event), ctypes.c_int, _dp, _dp, _dp, _dp, ctypes.c_long, _dp]
        L.peo_logprior.restype = ctypes.c_double
        L.peo_logprior.argtypes = [ctypes.POINTER(_Event), _dp]
        L.peo_weights_ess.argtypes = [_dp, _dp, _dp, ctypes.c_long, _dp, _dp]
        _sp = ctypes.POINTER(_Slice)
        _ip = ctypes.POINTER(ctypes.c_int)
        _lp = ctypes.POINTER(ctypes.c_long)
        L.peo_slice_candidate.restype = ctypes.c_int
        L.peo_slice_candidate.argtypes = [ctypes.POINTER(_Event), _sp, ctypes.c_uint64, ctypes.c_uint32,
                                          ctypes.c_uint64, _dp, _dp]
        L.peo_slice_sample.restype = ctypes.c_long
        L.peo_slice_sample.argtypes = [ctypes.POINTER(_Event), _sp, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_long,
                                       ctypes.c_long, _dp, _dp, _dp]
        L.peo_slice_dims.restype = ctypes.c_int
        L.peo_slice_dims.argtypes = [ctypes.POINTER(_Event), _sp, _ip]
        L.peo_tile_extrinsic.restype = ctypes.c_int
        L.peo_tile_extrinsic.argtypes = [ctypes.POINTER(_Event), _dp, _dp, ctypes.c_uint, ctypes.c_int, ctypes.c_uint64,
                                         ctypes.c_uint32, ctypes.c_long, _dp, _dp, _dp]
        L.peo_tile_bank.restype = ctypes.c_long
        L.peo_tile_bank.argtypes = [ctypes.POINTER(_Event), _sp, ctypes.c_double, ctypes.c_uint64, ctypes.c_uint32,
                                    ctypes.c_long, ctypes.c_long, ctypes.c_double, ctypes.c_long, _dp, _dp, _lp]
        L.peo_tile_assign.argtypes = [ctypes.c_int, ctypes.c_long, _dp, ctypes.c_long, ctypes.c_long, _dp,
                                      ctypes.c_long, _ip]
        L.peo_match.restype = ctypes.c_double
        L.peo_match.argtypes = [ctypes.POINTER(_Event), _dp, _dp]
        L.peo_tile_assign_match.argtypes = [ctypes.POINTER(_Event), ctypes.c_long, _dp, ctypes.c_long,
                                            ctypes.c_long, _dp, ctypes.c_long, _ip, _dp]
        L.peo_match_shift.restype = ctypes.c_double
        L.peo_match_shift.argtypes = [ctypes.POINTER(_Event), _dp, _dp, ctypes.c_double, ctypes.c_int]
        L.peo_tile_assign_match_shift.argtypes = [ctypes.POINTER(_Event), ctypes.c_long, _dp, ctypes.c_long,
                                                  ctypes.c_long, _dp, ctypes.c_long, ctypes.c_double, ctypes.c_int,
                                                  _ip, _dp]
        L.peo_tile_draw.restype = ctypes.c_int
        L.peo_tile_draw.argtypes = [ctypes.c_long, _dp, ctypes.c_long, _ip, _dp, ctypes.c_int, _dp, ctypes.c_long,
                                    ctypes.c_uint64, ctypes.c_uint32, ctypes.c_long, _dp, _dp, _dp, _lp]
        L.peo_tile_reweight.argtypes = [ctypes.c_long, _dp, ctypes.c_long, _ip, _dp, ctypes.c_long, _lp, _dp,
                                        ctypes.c_double, _dp]
        L.peo_relbin_edges.restype = ctypes.c_long
        L.peo_relbin_edges.argtypes = [ctypes.POINTER(_Event), ctypes.c_double, ctypes.c_long, _lp]
        L.peo_relbin_loglike.argtypes = [ctypes.POINTER(_Event), _dp, ctypes.c_long, _lp, _dp, ctypes.c_long, _dp, _dp]
        L.peo_proposal_update.restype = ctypes.c_long
        L.peo_proposal_update.argtypes = [ctypes.POINTER(_Event), _dp, _dp, ctypes.c_long, _dp, _dp, _dp]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(_dp)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def t_sun():
    return lib().peo_t_sun()


def mpc_m():
    return lib().peo_mpc_m()


def c_si():
    return lib().peo_c_si()


def r_earth():
    return lib().peo_r_earth()


class Event:
    """An event for the oracle. data: complex [n_det, K] (any complex dtype, promoted exactly),
    psd: real [n_det, K]. data/psd may be None for template-only use (psd needed for inner products)."""

    def __init__(self, n_det, n_bins, f_lo, df, data=None, psd=None, strain_scale=1.0, params=PARAMS_11D,
                 phase=PHASE_EXPLICIT, amp0=0.0, gmst=0.0, chi_max=0.4, dl_max=1e4, det_geom=None,
                 distance=DIST_SAMPLED, time_marg=0, tc_lo=0.0, tc_hi=0.0):
        self.n_det = int(n_det)
        self.n_bins = int(n_bins)
        self.f_lo = float(f_lo)
        self.df = float(df)
        self.params = int(params)
        self.phase = int(phase)
        self.dim = 4 if self.params == PARAMS_4D else 11
        if data is not None:
            d = np.asarray(data)
            assert d.shape == (self.n_det, self.n_bins)
            self._data = np.ascontiguousarray(np.stack([d.real.astype(np.float64), d.imag.astype(np.float64)], -1))
        else:
            self._data = None
        self._psd = _f64(psd) if psd is not None else None
        if self._psd is not None:
            assert self._psd.shape == (self.n_det, self.n_bins)
        s = _Event()
        s.n_det = self.n_det
        s.n_bins = self.n_bins
        s.f_lo = self.f_lo
        s.df = self.df
        s.data = _p(self._data) if self._data is not None else _dp()
        s.psd = _p(self._psd) if self._psd is not None else _dp()
        s.strain_scale = float(strain_scale)
        s.params = self.params
        s.phase = self.phase
        s.amp0 = float(amp0)
        s.gmst = float(gmst)
        s.chi_max = float(chi_max)
        s.dl_max = float(dl_max)
        self.distance = int(distance)
        s.distance = self.distance
        self.time_marg = int(time_marg)
        s.time_marg = self.time_marg
        s.tc_lo = float(tc_lo)
        s.tc_hi = float(tc_hi)
        if det_geom is not None:
            g = np.asarray(det_geom, dtype=np.float64).reshape(-1, 3)
            for i in range(g.shape[0]):
                for j in range(3):
                    s.det_geom[i][j] = g[i, j]
        self._s = s

    @property
    def ref(self):
        return ctypes.byref(self._s)

    # ---- model pieces ----
    def source(self, theta):
        th = _f64(theta)
        src = _Source()
        ok = lib().peo_source_from_theta(self.ref, _p(th), ctypes.byref(src))
        return bool(ok), src

    def psi(self, theta, f):
        _, src = self.source(theta)
        return np.array([lib().peo_psi(ctypes.byref(src), float(x)) for x in np.atleast_1d(f)])

    def kcut(self, fisco):
        return lib().peo_kcut(self.ref, float(fisco))

    def waveform(self, theta, kcut_override=-1):
        th = _f64(theta)
        h = np.zeros((self.n_det, self.n_bins, 2))
        lib().peo_waveform(self.ref, _p(th), int(kcut_override), _p(h))
        return h[..., 0] + 1j * h[..., 1]

    def inner(self, d, a, b):
        """(a|b) for detector d; a, b complex [n_det, K]."""
        A = np.ascontiguousarray(np.stack([a.real, a.imag], -1).astype(np.float64))
        B = np.ascontiguousarray(np.stack([b.real, b.imag], -1).astype(np.float64))
        return lib().peo_inner(self.ref, int(d), _p(A), _p(B))

    # ---- likelihood ----
    def loglike(self, theta, n_threads=0, return_zh=False):
        th = _f64(theta)
        D, n = th.shape
        assert D == self.dim
        ll = np.empty(n)
        zh = np.empty((n, 3))
        lib().peo_loglike(self.ref, _p(th), n, _p(ll), _p(zh), int(n_threads))
        return (ll, zh) if return_zh else ll

    def default_steps(self, theta0):
        th = _f64(theta0)
        st = np.zeros(self.dim)
        lib().peo_default_steps(self.ref, _p(th), _p(st))
        return st

    def metric(self, theta0, steps=None, flags=0):
        th = _f64(theta0)
        st = self.default_steps(th) if steps is None else _f64(steps)
        n = self.dim + (1 if (flags & 2) and self.params == PARAMS_4D else 0)
        g = np.zeros((n, n))
        lib().peo_metric_fd(self.ref, _p(th), _p(st), int(flags), _p(g))
        return g

    def draw(self, theta0, g, seed, stream, n):
        th0 = _f64(theta0)
        gg = _f64(g)
        theta = np.zeros((self.dim, n))
        lq = np.zeros(n)
        lp = np.zeros(n)
        rc = lib().peo_draw(self.ref, _p(th0), _p(gg), int(seed), int(stream), int(n), _p(theta), _p(lq), _p(lp))
        return rc, theta, lq, lp

    def logq_theta(self, theta0, g, theta):
        th0 = _f64(theta0)
        gg = _f64(g)
        th = _f64(theta)
        n = th.shape[1]
        lq = np.zeros(n)
        rc = lib().peo_logq_theta(self.ref, _p(th0), _p(gg), _p(th), n, _p(lq))
        return rc, lq

    def mixture_logq(self, weights, theta0s, gs, theta):
        """ln of the mixture sum_m pi_m q_m(theta), pi = weights / sum(weights), q_m the wrapped
        metric Gaussian of (theta0s[m], gs[m]) (peo_mixture_logq): returns (rc, logq [n])."""
        ww = _f64(weights)
        m = ww.shape[0]
        th0 = _f64(theta0s).reshape(m, self.dim)
        gg = _f64(gs).reshape(m, self.dim, self.dim)
        th = _f64(theta)
        n = th.shape[1]
        lq = np.zeros(n)
        rc = lib().peo_mixture_logq(self.ref, m, _p(ww), _p(th0), _p(gg), _p(th), n, _p(lq))
        return rc, lq

    def proposal_update(self, theta0, theta, w):
        """Weighted centre and covariance of the draws about theta0 (peo_proposal_update):
        returns (theta0_new [D], cov [D, D], number of positive weights)."""
        th0 = _f64(theta0)
        th = _f64(theta)
        ww = _f64(w)
        n = ww.shape[0]
        assert th.shape == (self.dim, n)
        out = np.zeros(self.dim)
        cov = np.zeros((self.dim, self.dim))
        cnt = lib().peo_proposal_update(self.ref, _p(th0), _p(th), n, _p(ww), _p(out), _p(cov))
        return out, cov, int(cnt)

    # ---- tile-mixture proposal ----
    def slice_dims(self, sl):
        """Number of sliced coordinates (all of them when the slice's sub_mask is 0)."""
        idx = (ctypes.c_int * 11)()
        return int(lib().peo_slice_dims(self.ref, ctypes.byref(sl), idx))

    def slice_candidate(self, sl, seed, stream, i):
        y = np.zeros(self.slice_dims(sl))
        th = np.zeros(self.dim)
        ok = lib().peo_slice_candidate(self.ref, ctypes.byref(sl), int(seed), int(stream), int(i), _p(y), _p(th))
        return bool(ok), y, th

    def slice_sample(self, sl, seed, stream, first, n):
        """Kept candidates first..first+n-1 of the slice: (y [S, k], theta [D, k], logprior [k])."""
        y = np.zeros((self.slice_dims(sl), n))
        th = np.zeros((self.dim, n))
        lp = np.zeros(n)
        k = lib().peo_slice_sample(self.ref, ctypes.byref(sl), int(seed), int(stream), int(first), int(n), _p(y),
                                   _p(th), _p(lp))
        return y[:, :k].copy(), th[:, :k].copy(), lp[:k].copy()

    def tile_bank(self, sl, min_dist, seed, stream, batch, max_tiles, stop_fraction, max_batches):
        """Stochastic bank: (templates y [S, m], theta [D, m], candidates consumed)."""
        ty = np.zeros((self.slice_dims(sl), max_tiles))
        tth = np.zeros((self.dim, max_tiles))
        used = ctypes.c_long(0)
        m = lib().peo_tile_bank(self.ref, ctypes.byref(sl), float(min_dist), int(seed), int(stream), int(batch),
                                int(max_tiles), float(stop_fraction), int(max_batches), _p(ty), _p(tth),
                                ctypes.byref(used))
        return ty[:, :m].copy(), tth[:, :m].copy(), int(used.value)

    def tile_extrinsic(self, theta0, g, sub_mask, seed, stream, theta, logq, logprior, conditional=False):
        """Tile draws completed by the proposal's marginal over the coordinates outside sub_mask, or by
        their conditional given the draw's sub_mask coordinates (peo_tile_extrinsic):
        (rc, theta [D, n], logq [n], logprior [n]), new arrays."""
        th0 = _f64(theta0)
        gg = _f64(g)
        th = np.array(theta, dtype=np.float64, order="C", copy=True)
        lq = np.array(logq, dtype=np.float64, copy=True)
        lp = np.array(logprior, dtype=np.float64, copy=True)
        n = th.shape[1]
        assert th.shape == (self.dim, n) and lq.shape == (n,) and lp.shape == (n,)
        rc = lib().peo_tile_extrinsic(self.ref, _p(th0), _p(gg), ctypes.c_uint(int(sub_mask)), int(bool(conditional)),
                                      int(seed), int(stream), int(n), _p(th), _p(lq), _p(lp))
        return rc, th, lq, lp

    # ---- relative binning ----
    def relbin_edges(self, eps, max_edges=1 << 20):
        e = np.zeros(max_edges, dtype=np.int64)
        m = lib().peo_relbin_edges(self.ref, float(eps), int(max_edges), e.ctypes.data_as(ctypes.POINTER(ctypes.c_long)))
        if m < 0:
            raise ValueError("too many relative-binning edges")
        return e[:m].copy()

    def relbin_loglike(self, theta_f, edges, theta, return_zh=False):
        tf = _f64(theta_f)
        ed = np.ascontiguousarray(edges, dtype=np.int64)
        th = _f64(theta)
        n = th.shape[1]
        ll = np.zeros(n)
        zh = np.zeros((n, 3))
        lib().peo_relbin_loglike(self.ref, _p(tf), ed.shape[0], ed.ctypes.data_as(ctypes.POINTER(ctypes.c_long)),
                                 _p(th), n, _p(ll), _p(zh))
        return (ll, zh) if return_zh else ll

    def logprior(self, theta):
        th = _f64(theta)
        return lib().peo_logprior(self.ref, _p(th))

    def match(self, theta_a, theta_b):
        """Waveform match of two points (overlap maximised over a constant phase, normalised)."""
        return lib().peo_match(self.ref, _p(_f64(theta_a)), _p(_f64(theta_b)))

    def match_shift(self, theta_a, theta_b, dt, n_shift):
        """The match maximised over the time shifts j dt, |j| <= n_shift, too (peo_match_shift)."""
        return lib().peo_match_shift(self.ref, _p(_f64(theta_a)), _p(_f64(theta_b)), float(dt), int(n_shift))

    def tile_assign_match_shift(self, tiles_theta, theta, dt, n_shift):
        """Template of largest shift-maximised match of every sample (brute force): (tile_of, match)."""
        tt = _f64(tiles_theta)
        th = _f64(theta)
        m = tt.shape[1]
        n = th.shape[1]
        out = np.zeros(n, dtype=np.int32)
        mv = np.zeros(n)
        lib().peo_tile_assign_match_shift(self.ref, m, _p(tt), m, n, _p(th), n, float(dt), int(n_shift),
                                          out.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _p(mv))
        return out, mv

    def tile_assign_match(self, tiles_theta, theta):
        """Template of largest match of every sample (brute force): (tile_of, match)."""
        tt = _f64(tiles_theta)
        th = _f64(theta)
        m = tt.shape[1]
        n = th.shape[1]
        out = np.zeros(n, dtype=np.int32)
        mv = np.zeros(n)
        lib().peo_tile_assign_match(self.ref, m, _p(tt), m, n, _p(th), n,
                                    out.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _p(mv))
        return out, mv


def pn_coeffs(eta, delta, chi1, chi2):
    phi = np.zeros(8)
    phil = np.zeros(8)
    lib().peo_pn_coeffs(float(eta), float(delta), float(chi1), float(chi2), _p(phi), _p(phil))
    return phi, phil


def f_isco(M):
    return lib().peo_f_isco(float(M))


def antenna(geom, ra, dec, psi, gmst=0.0):
    g = _f64(geom)
    fp = np.zeros(1)
    fc = np.zeros(1)
    dt = np.zeros(1)
    lib().peo_antenna(_p(g), float(ra), float(dec), float(psi), float(gmst), _p(fp), _p(fc), _p(dt))
    return fp[0], fc[0], dt[0]


def log_i0(x):
    return lib().peo_log_i0(float(x))


def philox4x32_10(ctr, key):
    c = (ctypes.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (ctypes.c_uint32 * 4)()
    lib().peo_philox4x32_10(c, k, o)
    return [int(o[i]) for i in range(4)]


def uniforms(seed, stream, n, npairs):
    u = np.zeros((n, npairs, 2))
    lib().peo_uniforms(int(seed), int(stream), int(n), int(npairs), _p(u))
    return u


def make_slice(centre, chol, radius, sub_mask=0):
    """Slice of the prior: ball of `radius` in y = L^T (theta_S - centre_S), chol = lower L (S x S)
    over the coordinates in sub_mask (all when 0; the others stay at the centre)."""
    sl = _Slice()
    c = np.asarray(centre, dtype=np.float64)
    Lm = np.asarray(chol, dtype=np.float64)
    S = Lm.shape[0]
    for a in range(c.shape[0]):
        sl.centre[a] = float(c[a])
    for a in range(S):
        for b in range(S):
            sl.chol[a * S + b] = float(Lm[a, b])
    sl.radius = float(radius)
    sl.sub_mask = int(sub_mask)
    return sl


def tile_assign(tiles_y, y):
    """Nearest template (whitened distance, lowest index among equals) of every sample."""
    ty = _f64(tiles_y)
    yy = _f64(y)
    D, m = ty.shape
    n = yy.shape[1]
    out = np.zeros(n, dtype=np.int32)
    lib().peo_tile_assign(D, m, _p(ty), m, n, _p(yy), n, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
    return out


def tile_draw(tile_ll, tile_of, logprior, samples, seed, stream, n):
    """Tile-mixture proposal draws: (rc, theta [D, n], logq, logprior, index)."""
    tl = _f64(tile_ll)
    to = np.ascontiguousarray(tile_of, dtype=np.int32)
    lp = _f64(logprior)
    sm = _f64(samples)
    D, P = sm.shape
    theta = np.zeros((D, n))
    lq = np.zeros(n)
    lpo = np.zeros(n)
    idx = np.zeros(n, dtype=np.int64)
    rc = lib().peo_tile_draw(tl.shape[0], _p(tl), P, to.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _p(lp), D,
                             _p(sm), P, int(seed), int(stream), int(n), _p(theta), _p(lq), _p(lpo),
                             idx.ctypes.data_as(ctypes.POINTER(ctypes.c_long)))
    return rc, theta, lq, lpo, idx


def tile_reweight(tile_ll, tile_of, logprior, index, w, alpha):
    """Per-tile values for the next round's tile_draw (peo_tile_reweight)."""
    tl = _f64(tile_ll)
    to = np.ascontiguousarray(tile_of, dtype=np.int32)
    lp = _f64(logprior)
    ix = np.ascontiguousarray(index, dtype=np.int64)
    ww = _f64(w)
    out = np.zeros(tl.shape[0])
    lib().peo_tile_reweight(tl.shape[0], _p(tl), lp.shape[0], to.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                            _p(lp), ix.shape[0], ix.ctypes.data_as(ctypes.POINTER(ctypes.c_long)), _p(ww),
                            float(alpha), _p(out))
    return out


def weights_ess(loglike, logprior, logq):
    ll = _f64(loglike)
    lp = _f64(logprior)
    lq = _f64(logq)
    n = ll.shape[0]
    w = np.zeros(n)
    st = np.zeros(4)
    lib().peo_weights_ess(_p(ll), _p(lp), _p(lq), n, _p(w), _p(st))
    return w, st


def log_dist_marg(a, b, explicit_phase):
    """ln of int_1^inf 3 x^-4 exp(phi(x) - b x^2) dx, phi = a x (explicit phase) or ln I0(a x)."""
    return lib().peo_log_dist_marg(float(a), float(b), int(bool(explicit_phase)))
