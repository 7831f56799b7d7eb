"""Thin ctypes binding of libpe.so (include/pe.h), same names as the C ABI.

Argument marshalling only: torch tensors supply device memory (data_ptr) and
the current HIP stream; every computation runs in the library's kernels.
There is no CPU fallback: if libpe.so is missing or no GPU is visible the
calls raise.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpe.so")

PE_OK = 0
STATUS_NAMES = {0: "PE_OK", 1: "PE_ERR_ARG", 2: "PE_ERR_OOM", 3: "PE_ERR_HIP", 4: "PE_ERR_SINGULAR",
                5: "PE_ERR_NONFINITE", 6: "PE_ERR_BUDGET", 7: "PE_ERR_TIMEOUT"}
PE_ERR_BUDGET = 6
PE_PREC_FP64 = 0
PE_PREC_SPLIT = 1
PE_PREC_RELBIN = 2
PE_PHASE_MARG = 0
PE_PHASE_EXPLICIT = 1
PE_DIST_SAMPLED = 0
PE_DIST_MARG = 1
PE_PARAMS_4D = 0
PE_PARAMS_11D = 1
PE_C128 = 0
PE_C64 = 1
PE_F64 = 0
PE_F32 = 1
MAX_DET = 4

EXPORTS = ["pe_dim", "pe_event_create", "pe_event_update", "pe_event_status", "pe_event_reserve",
           "pe_event_destroy", "pe_metric", "pe_draw", "pe_mixture_logq", "pe_loglike_batch", "pe_loglike_multi", "pe_batch_run", "pe_weights_ess", "pe_weights_ess_noalloc", "pe_proposal_update", "pe_refine", "pe_slice_sample", "pe_tile_bank",
           "pe_tile_assign", "pe_tile_assign_match", "pe_tile_assign_match_shift", "pe_tile_draw", "pe_tile_extrinsic", "pe_tile_reweight", "pe_relbin_setup", "pe_relbin_edges",
           "pe_waveform",
           "pe_rng_uniforms", "pe_profile_enable", "pe_profile_read", "pe_set_chunks", "pe_set_plan", "pe_get_plan",
           "pe_autotune_plan", "pe_set_split_guard", "pe_get_split_guard", "pe_loglike_counts", "pe_last_error",
           "pe_server_create", "pe_server_submit", "pe_server_wait", "pe_server_now", "pe_server_counters",
           "pe_server_busy", "pe_server_tune", "pe_server_plans", "pe_server_destroy"]


class PeError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class EventDesc(ctypes.Structure):
    _fields_ = [("n_det", ctypes.c_int32), ("n_bins", ctypes.c_int64), ("f_lo", ctypes.c_double),
                ("df", ctypes.c_double), ("data_dtype", ctypes.c_int32), ("psd_dtype", ctypes.c_int32),
                ("strain_scale", ctypes.c_double), ("params", ctypes.c_int32), ("phase", ctypes.c_int32),
                ("amp0", ctypes.c_double), ("gmst", ctypes.c_double), ("chi_max", ctypes.c_double),
                ("dl_max", ctypes.c_double), ("det_geom", (ctypes.c_double * 3) * MAX_DET),
                ("distance", ctypes.c_int32), ("time_marg", ctypes.c_int32), ("tm_points", ctypes.c_int32),
                ("tc_lo", ctypes.c_double), ("tc_hi", ctypes.c_double)]


class Slice(ctypes.Structure):
    """pe_slice_t: ball of `radius` in y = L^T (theta_S - centre_S) over the coordinates of sub_mask
    (all of them when 0)."""
    _fields_ = [("centre", ctypes.c_double * 11), ("chol", ctypes.c_double * 121), ("radius", ctypes.c_double),
                ("sub_mask", ctypes.c_uint32)]


def make_slice(centre, chol, radius, sub_mask=0):
    """chol: lower factor L (S x S) of the metric over the sliced coordinates."""
    import numpy as np
    sl = Slice()
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


def slice_dims(dim, slice_):
    """Number of sliced coordinates of a slice on an event of `dim` coordinates."""
    return dim if slice_.sub_mask == 0 else bin(int(slice_.sub_mask)).count("1")


_lib = None


PE_STAGE_PREP, PE_STAGE_METRIC, PE_STAGE_DRAW, PE_STAGE_LOGLIKE, PE_STAGE_WEIGHTS = 1, 2, 4, 8, 16
PE_STAGE_ALL = 31


class BatchItem(ctypes.Structure):
    """pe_batch_item_t."""
    _fields_ = [("ev", ctypes.c_void_p), ("data", ctypes.c_void_p), ("psd", ctypes.c_void_p),
                ("theta0", ctypes.c_void_p), ("fd_step", ctypes.c_void_p), ("metric_flags", ctypes.c_int32),
                ("stream_id", ctypes.c_uint32), ("seed", ctypes.c_uint64), ("g", ctypes.c_void_p),
                ("n", ctypes.c_int64), ("theta", ctypes.c_void_p), ("logq", ctypes.c_void_p),
                ("logprior", ctypes.c_void_p), ("loglike", ctypes.c_void_p), ("aux", ctypes.c_void_p),
                ("w", ctypes.c_void_p), ("stats", ctypes.c_void_p)]


PE_ERR_TIMEOUT = 7


class ServerConfig(ctypes.Structure):
    """pe_server_config_t."""
    _fields_ = [("hbm_budget", ctypes.c_int64), ("precision", ctypes.c_int32), ("max_active", ctypes.c_int32),
                ("slice_ms", ctypes.c_double), ("use_graph", ctypes.c_int32), ("max_groups", ctypes.c_int32),
                ("items_target", ctypes.c_int32), ("min_group_bins", ctypes.c_int32)]


class Request(ctypes.Structure):
    """pe_request_t."""
    _fields_ = [("desc", EventDesc), ("data", ctypes.c_void_p), ("psd", ctypes.c_void_p),
                ("data_on_host", ctypes.c_int32), ("metric_flags", ctypes.c_int32), ("theta0", ctypes.c_void_p),
                ("seed", ctypes.c_uint64), ("stream_id", ctypes.c_uint32), ("pad", ctypes.c_int32),
                ("n_draws", ctypes.c_int64), ("loglike_out", ctypes.c_void_p), ("w_out", ctypes.c_void_p),
                ("theta_out", ctypes.c_void_p)]


class Result(ctypes.Structure):
    """pe_result_t."""
    _fields_ = [("ticket", ctypes.c_int64), ("status", ctypes.c_int32), ("n_active", ctypes.c_int32),
                ("stats", ctypes.c_double * 4), ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_done", ctypes.c_double)]


def load(path=LIB_PATH):
    """Load libpe.so and declare the signatures (no GPU call is made)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run paper_2410_05190_amd/build.py (no CPU fallback exists)")
    L = ctypes.CDLL(path)
    vp, i32, i64, u64, u32, dp = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint32,
                                  ctypes.c_void_p)
    sig = {
        "pe_dim": (i32, [i32]),
        "pe_event_create": (i32, [ctypes.POINTER(EventDesc), vp, vp, vp, ctypes.POINTER(vp)]),
        "pe_event_update": (i32, [vp, vp, vp, vp]),
        "pe_event_status": (i32, [vp, vp]),
        "pe_event_reserve": (i32, [vp, i64]),
        "pe_event_destroy": (i32, [vp]),
        "pe_metric": (i32, [vp, dp, dp, i32, dp, vp]),
        "pe_draw": (i32, [vp, dp, dp, u64, u32, i64, dp, dp, dp, vp]),
        "pe_tile_extrinsic": (i32, [vp, dp, dp, u32, i32, u64, u32, i64, dp, dp, dp, vp]),
        "pe_mixture_logq": (i32, [vp, i32, dp, dp, dp, dp, i64, dp, vp]),
        "pe_loglike_batch": (i32, [vp, dp, i64, i32, dp, dp, vp]),
        "pe_loglike_multi": (i32, [i32, vp, vp, vp, i32, vp, vp, vp]),
        "pe_batch_run": (i32, [i32, vp, i32, i32, vp]),
        "pe_weights_ess": (i32, [dp, dp, dp, i64, dp, dp, vp]),
        "pe_weights_ess_noalloc": (i32, [dp, dp, dp, i64, dp, dp, vp]),
        "pe_proposal_update": (i32, [vp, dp, dp, i64, dp, dp, dp, vp]),
        "pe_slice_sample": (i32, [vp, ctypes.POINTER(Slice), u64, u32, i64, i64, dp, dp, dp, vp, vp]),
        "pe_tile_bank": (i32, [vp, ctypes.POINTER(Slice), ctypes.c_double, u64, u32, i32, i32, ctypes.c_double, i32,
                               dp, dp, ctypes.POINTER(i32), ctypes.POINTER(i64), vp]),
        "pe_tile_assign": (i32, [i32, i32, dp, i64, i64, dp, i64, vp, vp]),
        "pe_tile_draw": (i32, [i32, dp, i64, vp, dp, i32, dp, i64, u64, u32, i64, dp, dp, dp, vp, vp]),
        "pe_tile_assign_match": (i32, [vp, i32, dp, dp, i64, i64, dp, dp, i64, i32, vp, dp, vp]),
        "pe_tile_assign_match_shift": (i32, [vp, i32, dp, dp, i64, i64, dp, dp, i64, i32, ctypes.c_double, i32, vp,
                                              dp, vp]),
        "pe_tile_reweight": (i32, [i32, dp, i64, vp, dp, i64, vp, dp, ctypes.c_double, dp, vp]),
        "pe_relbin_setup": (i32, [vp, dp, ctypes.c_double, i32, vp]),
        "pe_relbin_edges": (i32, [vp, vp, i32, ctypes.POINTER(i32)]),
        "pe_refine": (i32, [vp, dp, dp, i32, i64, u64, i32, dp, dp, dp, dp, dp, dp, vp]),
        "pe_waveform": (i32, [ctypes.POINTER(EventDesc), dp, vp, dp, dp, vp]),
        "pe_rng_uniforms": (i32, [u64, u32, i64, i32, dp, vp]),
        "pe_profile_enable": (i32, [i32]),
        "pe_profile_read": (i32, [ctypes.c_char_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64)]),
        "pe_set_chunks": (i32, [i32]),
        "pe_set_split_guard": (i32, [ctypes.c_double]),
        "pe_get_split_guard": (i32, [ctypes.POINTER(ctypes.c_double)]),
        "pe_loglike_counts": (i32, [vp, ctypes.POINTER(i64), vp]),
        "pe_set_plan": (i32, [i32, i32]),
        "pe_get_plan": (i32, [ctypes.POINTER(i32), ctypes.POINTER(i32)]),
        "pe_autotune_plan": (i32, [i32, vp, vp, vp, i32, i32, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                   ctypes.POINTER(ctypes.c_double), vp]),
        "pe_server_create": (i32, [ctypes.POINTER(ServerConfig), ctypes.POINTER(vp)]),
        "pe_server_submit": (i32, [vp, ctypes.POINTER(Request), ctypes.POINTER(i64)]),
        "pe_server_wait": (i32, [vp, i64, ctypes.c_double, ctypes.POINTER(Result)]),
        "pe_server_now": (ctypes.c_double, [vp]),
        "pe_server_counters": (i32, [vp, ctypes.POINTER(i64)]),
        "pe_server_busy": (i32, [vp, ctypes.POINTER(ctypes.c_double)]),
        "pe_server_tune": (i32, [vp, i32, vp, vp, vp, i32]),
        "pe_server_plans": (i32, [vp, i32, ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i32)]),
        "pe_server_destroy": (i32, [vp]),
        "pe_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(status):
    if status != PE_OK:
        raise PeError(status, _lib.pe_last_error().decode())


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t, dtype=None, name="tensor", allow_none=False):
    if t is None:
        if allow_none:
            return None
        raise ValueError(f"{name} is required")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def make_desc(n_det, n_bins, f_lo, df, data_dtype=PE_C128, psd_dtype=PE_F64, strain_scale=1.0,
              params=PE_PARAMS_11D, phase=PE_PHASE_EXPLICIT, amp0=0.0, gmst=0.0, chi_max=0.4, dl_max=1e4,
              det_geom=None, distance=PE_DIST_SAMPLED, time_marg=0, tm_points=0, tc_lo=0.0, tc_hi=0.0):
    d = EventDesc()
    d.n_det = int(n_det)
    d.n_bins = int(n_bins)
    d.f_lo = float(f_lo)
    d.df = float(df)
    d.data_dtype = int(data_dtype)
    d.psd_dtype = int(psd_dtype)
    d.strain_scale = float(strain_scale)
    d.params = int(params)
    d.phase = int(phase)
    d.amp0 = float(amp0)
    d.gmst = float(gmst)
    d.chi_max = float(chi_max)
    d.dl_max = float(dl_max)
    d.distance = int(distance)
    d.time_marg = int(time_marg)
    d.tm_points = int(tm_points)
    d.tc_lo = float(tc_lo)
    d.tc_hi = float(tc_hi)
    if det_geom is not None:
        g = np.asarray(det_geom, dtype=np.float64).reshape(-1, 3)
        for i in range(g.shape[0]):
            for j in range(3):
                d.det_geom[i][j] = g[i, j]
    return d


def dtypes_of(data, psd):
    import torch
    dd = {torch.complex128: PE_C128, torch.complex64: PE_C64}[data.dtype]
    pd = {torch.float64: PE_F64, torch.float32: PE_F32}[psd.dtype]
    return dd, pd


# ---------------------------------------------------------------- C-ABI mirror
def pe_dim(params):
    return load().pe_dim(int(params))


def pe_event_create(desc, data, psd, stream=None):
    load()
    h = ctypes.c_void_p()
    _check(_lib.pe_event_create(ctypes.byref(desc), _ptr(data, name="data"), _ptr(psd, name="psd"), _stream(stream),
                                ctypes.byref(h)))
    return h


def pe_event_update(ev, data, psd, stream=None):
    _check(_lib.pe_event_update(ev, _ptr(data, name="data"), _ptr(psd, name="psd"), _stream(stream)))


def pe_event_status(ev, stream=None):
    _check(load().pe_event_status(ev, _stream(stream)))


def pe_event_reserve(ev, max_draws):
    _check(load().pe_event_reserve(ev, int(max_draws)))


def pe_event_destroy(ev):
    _check(load().pe_event_destroy(ev))


def pe_metric(ev, theta0, fd_step, flags, g, stream=None):
    import torch
    _check(_lib.pe_metric(ev, _ptr(theta0, torch.float64, "theta0"),
                          _ptr(fd_step, torch.float64, "fd_step", allow_none=True), int(flags),
                          _ptr(g, torch.float64, "g"), _stream(stream)))


def pe_draw(ev, theta0, g, seed, stream_id, n, theta, logq, logprior, stream=None):
    import torch
    f64 = torch.float64
    _check(_lib.pe_draw(ev, _ptr(theta0, f64, "theta0"), _ptr(g, f64, "g"), int(seed) & 0xFFFFFFFFFFFFFFFF,
                        int(stream_id) & 0xFFFFFFFF, int(n), _ptr(theta, f64, "theta"), _ptr(logq, f64, "logq"),
                        _ptr(logprior, f64, "logprior"), _stream(stream)))


PE_MIX_MAX = 16


def pe_mixture_logq(ev, weights, theta0s, gs, theta, n, logq, stream=None):
    """weights: m floats (host); theta0s [m, D], gs [m, D, D], theta [D, n], logq [n] (device, float64)."""
    import torch
    f64 = torch.float64
    w = [float(x) for x in weights]
    arr = (ctypes.c_double * max(len(w), 1))(*w)
    _check(load().pe_mixture_logq(ev, len(w), ctypes.cast(arr, ctypes.POINTER(ctypes.c_double)),
                                  _ptr(theta0s, f64, "theta0s"), _ptr(gs, f64, "gs"), _ptr(theta, f64, "theta"),
                                  int(n), _ptr(logq, f64, "logq"), _stream(stream)))


PE_TILE_CONDITIONAL = 1


def pe_tile_extrinsic(ev, theta0, g, sub_mask, flags, seed, stream_id, n, theta, logq, logprior, stream=None):
    import torch
    f64 = torch.float64
    _check(load().pe_tile_extrinsic(ev, _ptr(theta0, f64, "theta0"), _ptr(g, f64, "g"), int(sub_mask) & 0xFFFFFFFF,
                                    int(flags), int(seed) & 0xFFFFFFFFFFFFFFFF, int(stream_id) & 0xFFFFFFFF, int(n),
                                    _ptr(theta, f64, "theta"), _ptr(logq, f64, "logq"),
                                    _ptr(logprior, f64, "logprior"), _stream(stream)))


def pe_loglike_batch(ev, theta, n, precision, loglike, aux=None, stream=None):
    import torch
    f64 = torch.float64
    _check(_lib.pe_loglike_batch(ev, _ptr(theta, f64, "theta"), int(n), int(precision), _ptr(loglike, f64, "loglike"),
                                 _ptr(aux, f64, "aux", allow_none=True), _stream(stream)))


def pe_loglike_multi(events, thetas, ns, precision, loglikes, auxs=None, stream=None):
    """One batch over several events: events[e] evaluates ns[e] draws thetas[e] into loglikes[e]."""
    import torch
    f64 = torch.float64
    ne = len(events)
    if not (len(thetas) == len(ns) == len(loglikes) == ne) or (auxs is not None and len(auxs) != ne):
        raise ValueError("events, thetas, ns, loglikes (and auxs) must have one entry per event")
    ev_a = (ctypes.c_void_p * max(ne, 1))(*[e.handle if isinstance(e, Event) else e for e in events])
    th_a = (ctypes.c_void_p * max(ne, 1))(*[_ptr(t, f64, "theta") for t in thetas])
    n_a = (ctypes.c_int64 * max(ne, 1))(*[int(n) for n in ns])
    ll_a = (ctypes.c_void_p * max(ne, 1))(*[_ptr(t, f64, "loglike") for t in loglikes])
    ax_a = None
    if auxs is not None:
        ax_a = (ctypes.c_void_p * max(ne, 1))(*[_ptr(t, f64, "aux", allow_none=True) for t in auxs])
    _check(load().pe_loglike_multi(ne, ev_a, th_a, n_a, int(precision), ll_a, ax_a, _stream(stream)))


def make_item(ev, n=0, data=None, psd=None, theta0=None, fd_step=None, metric_flags=0, seed=0, stream_id=0, g=None,
              theta=None, logq=None, logprior=None, loglike=None, aux=None, w=None, stats=None):
    """A pe_batch_item_t from device tensors (None = NULL)."""
    def p(t):
        return None if t is None else t.data_ptr()
    it = BatchItem()
    it.ev = ev.handle.value if isinstance(ev, Event) else (ev.value if isinstance(ev, ctypes.c_void_p) else ev)
    it.data, it.psd, it.theta0, it.fd_step = p(data), p(psd), p(theta0), p(fd_step)
    it.metric_flags = int(metric_flags)
    it.stream_id = int(stream_id) & 0xFFFFFFFF
    it.seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    it.g, it.n = p(g), int(n)
    it.theta, it.logq, it.logprior, it.loglike = p(theta), p(logq), p(logprior), p(loglike)
    it.aux, it.w, it.stats = p(aux), p(w), p(stats)
    return it


def pe_batch_run(items, stages, precision, stream=None):
    arr = (BatchItem * max(len(items), 1))(*items)
    _check(load().pe_batch_run(len(items), ctypes.cast(arr, ctypes.c_void_p), int(stages), int(precision),
                               _stream(stream)))


def pe_weights_ess(loglike, logprior, logq, n, w, stats, stream=None):
    import torch
    f64 = torch.float64
    _check(load().pe_weights_ess(_ptr(loglike, f64, "loglike"), _ptr(logprior, f64, "logprior"),
                                 _ptr(logq, f64, "logq"), int(n), _ptr(w, f64, "w", allow_none=True),
                                 _ptr(stats, f64, "stats"), _stream(stream)))


def pe_weights_ess_noalloc(loglike, logprior, logq, n, w, stats, stream=None):
    import torch
    f64 = torch.float64
    _check(load().pe_weights_ess_noalloc(_ptr(loglike, f64, "loglike"), _ptr(logprior, f64, "logprior"),
                                 _ptr(logq, f64, "logq"), int(n), _ptr(w, f64, "w", allow_none=True),
                                 _ptr(stats, f64, "stats"), _stream(stream)))


def pe_proposal_update(ev, theta, w, n, theta0, theta0_out, cov=None, stream=None):
    import torch
    f64 = torch.float64
    _check(load().pe_proposal_update(ev, _ptr(theta, f64, "theta"), _ptr(w, f64, "w"), int(n),
                                     _ptr(theta0, f64, "theta0"), _ptr(theta0_out, f64, "theta0_out"),
                                     _ptr(cov, f64, "cov", allow_none=True), _stream(stream)))


def pe_refine(ev, theta0, g, rounds, n, seed, precision, theta, logq, logprior, loglike, w, stats, stream=None):
    import torch
    f64 = torch.float64
    _check(load().pe_refine(ev, _ptr(theta0, f64, "theta0"), _ptr(g, f64, "g"), int(rounds), int(n),
                            int(seed) & 0xFFFFFFFFFFFFFFFF, int(precision), _ptr(theta, f64, "theta"),
                            _ptr(logq, f64, "logq"), _ptr(logprior, f64, "logprior"), _ptr(loglike, f64, "loglike"),
                            _ptr(w, f64, "w"), _ptr(stats, f64, "stats"), _stream(stream)))


def pe_slice_sample(ev, slice_, seed, stream_id, first, n, y, theta, logprior, count, stream=None):
    import torch
    f64 = torch.float64
    _check(load().pe_slice_sample(ev, ctypes.byref(slice_), int(seed) & 0xFFFFFFFFFFFFFFFF, int(stream_id) & 0xFFFFFFFF,
                                  int(first), int(n), _ptr(y, f64, "y"), _ptr(theta, f64, "theta"),
                                  _ptr(logprior, f64, "logprior"), _ptr(count, torch.int64, "count"), _stream(stream)))


def pe_tile_bank(ev, slice_, min_dist, seed, stream_id, batch, max_tiles, stop_fraction, max_batches, tiles_y,
                 tiles_theta, stream=None):
    """Returns (n_tiles, candidates consumed)."""
    import torch
    f64 = torch.float64
    m = ctypes.c_int32(0)
    used = ctypes.c_int64(0)
    _check(load().pe_tile_bank(ev, ctypes.byref(slice_), float(min_dist), int(seed) & 0xFFFFFFFFFFFFFFFF,
                               int(stream_id) & 0xFFFFFFFF, int(batch), int(max_tiles), float(stop_fraction),
                               int(max_batches), _ptr(tiles_y, f64, "tiles_y"), _ptr(tiles_theta, f64, "tiles_theta"),
                               ctypes.byref(m), ctypes.byref(used), _stream(stream)))
    return m.value, used.value


def pe_tile_assign(dim, n_tiles, tiles_y, ld_tiles, n, y, ld_y, tile_of, stream=None):
    import torch
    f64 = torch.float64
    _check(load().pe_tile_assign(int(dim), int(n_tiles), _ptr(tiles_y, f64, "tiles_y"), int(ld_tiles), int(n),
                                 _ptr(y, f64, "y"), int(ld_y), _ptr(tile_of, torch.int32, "tile_of"), _stream(stream)))


def pe_tile_draw(n_tiles, tile_loglike, n_samples, tile_of, sample_logprior, dim, samples_theta, ld, seed, stream_id, n,
                 theta, logq, logprior, index=None, stream=None):
    import torch
    f64 = torch.float64
    _check(load().pe_tile_draw(int(n_tiles), _ptr(tile_loglike, f64, "tile_loglike"), int(n_samples),
                               _ptr(tile_of, torch.int32, "tile_of"), _ptr(sample_logprior, f64, "sample_logprior"),
                               int(dim), _ptr(samples_theta, f64, "samples_theta"), int(ld),
                               int(seed) & 0xFFFFFFFFFFFFFFFF, int(stream_id) & 0xFFFFFFFF, int(n),
                               _ptr(theta, f64, "theta"), _ptr(logq, f64, "logq"), _ptr(logprior, f64, "logprior"),
                               _ptr(index, torch.int64, "index", allow_none=True), _stream(stream)))


def pe_waveform(desc, theta, psd, h, snr2=None, stream=None):
    import torch
    f64 = torch.float64
    _check(load().pe_waveform(ctypes.byref(desc), _ptr(theta, f64, "theta"), _ptr(psd, name="psd", allow_none=True),
                              _ptr(h, None, "h"), _ptr(snr2, f64, "snr2", allow_none=True), _stream(stream)))


def pe_rng_uniforms(seed, stream_id, n, npairs, u, stream=None):
    import torch
    _check(load().pe_rng_uniforms(int(seed) & 0xFFFFFFFFFFFFFFFF, int(stream_id) & 0xFFFFFFFF, int(n), int(npairs),
                                  _ptr(u, torch.float64, "u"), _stream(stream)))


def pe_profile_enable(enable):
    _check(load().pe_profile_enable(1 if enable else 0))


def pe_profile_read(kernel):
    ms = ctypes.c_double()
    cnt = ctypes.c_int64()
    _check(load().pe_profile_read(kernel.encode(), ctypes.byref(ms), ctypes.byref(cnt)))
    return ms.value, cnt.value


def pe_set_chunks(n_chunks):
    _check(load().pe_set_chunks(int(n_chunks)))


def pe_set_split_guard(budget):
    _check(load().pe_set_split_guard(float(budget)))


def pe_get_split_guard():
    b = ctypes.c_double()
    _check(load().pe_get_split_guard(ctypes.byref(b)))
    return b.value


def pe_loglike_counts(ev, stream=None):
    """(in-support draws, draws re-evaluated in FP64) of the event's last log-likelihood batch."""
    out = (ctypes.c_int64 * 2)()
    _check(load().pe_loglike_counts(ev.handle if isinstance(ev, Event) else ev, out, _stream(stream)))
    return int(out[0]), int(out[1])


def pe_set_plan(items_target, min_group_bins):
    _check(load().pe_set_plan(int(items_target), int(min_group_bins)))


def pe_get_plan():
    a, b = ctypes.c_int32(), ctypes.c_int32()
    _check(load().pe_get_plan(ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def pe_autotune_plan(events, thetas, ns, precision, reps=2, stream=None):
    """Fastest (items_target, min_group_bins) for this workload and its time per batch (ms)."""
    import torch
    ne = len(events)
    ev_a = (ctypes.c_void_p * max(ne, 1))(*[e.handle if isinstance(e, Event) else e for e in events])
    th_a = (ctypes.c_void_p * max(ne, 1))(*[_ptr(t, torch.float64, "theta") for t in thetas])
    n_a = (ctypes.c_int64 * max(ne, 1))(*[int(n) for n in ns])
    a, b, ms = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
    _check(load().pe_autotune_plan(ne, ev_a, th_a, n_a, int(precision), int(reps), ctypes.byref(a), ctypes.byref(b),
                                   ctypes.byref(ms), _stream(stream)))
    return a.value, b.value, ms.value


def pe_last_error():
    return load().pe_last_error().decode()


# ---------------------------------------------------------------- convenience
class Event:
    """Owns a pe_event_t. data: complex128/complex64 [n_det, K] device tensor; psd: float64/float32."""

    def __init__(self, data, psd, stream=None, **desc_kw):
        dd, pd = dtypes_of(data, psd)
        n_det, K = psd.shape
        self.desc = make_desc(n_det, K, data_dtype=dd, psd_dtype=pd, **desc_kw)
        self.dim = pe_dim(self.desc.params)
        self.handle = pe_event_create(self.desc, data, psd, stream)

    def close(self):
        if self.handle is not None:
            pe_event_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def update(self, data, psd, stream=None):
        pe_event_update(self.handle, data, psd, stream)

    def status(self, stream=None):
        pe_event_status(self.handle, stream)

    def reserve(self, n):
        pe_event_reserve(self.handle, n)

    def metric(self, theta0, fd_step=None, flags=0, stream=None):
        import torch
        g = torch.empty((self.dim, self.dim), dtype=torch.float64, device=theta0.device)
        pe_metric(self.handle, theta0, fd_step, flags, g, stream)
        return g

    def draw(self, theta0, g, seed, stream_id, n, stream=None):
        import torch
        dev = theta0.device
        theta = torch.empty((self.dim, n), dtype=torch.float64, device=dev)
        lq = torch.empty(n, dtype=torch.float64, device=dev)
        lp = torch.empty(n, dtype=torch.float64, device=dev)
        pe_draw(self.handle, theta0, g, seed, stream_id, n, theta, lq, lp, stream)
        return theta, lq, lp

    def mixture_logq(self, weights, theta0s, gs, theta, stream=None):
        import torch
        n = theta.shape[1]
        lq = torch.empty(n, dtype=torch.float64, device=theta.device)
        pe_mixture_logq(self.handle, weights, theta0s, gs, theta, n, lq, stream)
        return lq

    def proposal_update(self, theta, w, theta0, cov=False, stream=None):
        """pe_proposal_update: returns the new centre (and the weighted covariance if cov)."""
        import torch
        out = torch.empty(self.dim, dtype=torch.float64, device=theta0.device)
        c = torch.empty((self.dim, self.dim), dtype=torch.float64, device=theta0.device) if cov else None
        pe_proposal_update(self.handle, theta, w, theta.shape[1], theta0, out, c, stream)
        return (out, c) if cov else out

    def refine(self, theta0, rounds, n, seed, precision=PE_PREC_SPLIT, stream=None):
        """pe_refine: returns (refined centre, metric there, per-round stats [rounds, 4])."""
        import torch
        dev = theta0.device
        t0 = theta0.clone()
        g = torch.empty((self.dim, self.dim), dtype=torch.float64, device=dev)
        bufs = [torch.empty((self.dim, n), dtype=torch.float64, device=dev)] + \
               [torch.empty(n, dtype=torch.float64, device=dev) for _ in range(4)]
        st = torch.empty((rounds, 4), dtype=torch.float64, device=dev)
        pe_refine(self.handle, t0, g, rounds, n, seed, precision, *bufs, st, stream)
        return t0, g, st

    def slice_sample(self, slice_, seed, stream_id, first, n, stream=None):
        """pe_slice_sample: (y [S, k], theta [D, k], logprior [k]) of the kept candidates (synchronises)."""
        import torch
        f64 = dict(dtype=torch.float64, device="cuda")
        y = torch.empty((slice_dims(self.dim, slice_), n), **f64)
        th = torch.empty((self.dim, n), **f64)
        lp = torch.empty(n, **f64)
        cnt = torch.empty(1, dtype=torch.int64, device="cuda")
        pe_slice_sample(self.handle, slice_, seed, stream_id, first, n, y, th, lp, cnt, stream)
        k = int(cnt.item())
        return y[:, :k], th[:, :k], lp[:k]

    def tile_bank(self, slice_, min_dist, seed, stream_id, batch, max_tiles, stop_fraction, max_batches, stream=None):
        """pe_tile_bank: (templates y [S, m], theta [D, m], candidates consumed)."""
        import torch
        f64 = dict(dtype=torch.float64, device="cuda")
        ty = torch.empty((slice_dims(self.dim, slice_), max_tiles), **f64)
        tth = torch.empty((self.dim, max_tiles), **f64)
        m, used = pe_tile_bank(self.handle, slice_, min_dist, seed, stream_id, batch, max_tiles, stop_fraction,
                               max_batches, ty, tth, stream)
        return ty[:, :m], tth[:, :m], used

    def relbin_setup(self, theta_f, eps, max_edges=1 << 20, stream=None):
        """pe_relbin_setup: relative binning about theta_f (device tensor [D]); then
        loglike(..., precision=PE_PREC_RELBIN)."""
        import torch
        _check(load().pe_relbin_setup(self.handle, _ptr(theta_f, torch.float64, "theta_f"), float(eps),
                                      int(max_edges), _stream(stream)))

    def relbin_edges(self):
        import numpy as np
        n = ctypes.c_int32(0)
        _check(load().pe_relbin_edges(self.handle, None, 0, ctypes.byref(n)))
        out = np.zeros(max(n.value, 1), dtype=np.int64)
        if n.value:
            _check(load().pe_relbin_edges(self.handle, out.ctypes.data_as(ctypes.c_void_p), n.value, ctypes.byref(n)))
        return out[: n.value]

    def loglike(self, theta, precision=PE_PREC_SPLIT, aux=False, stream=None):
        import torch
        n = theta.shape[1]
        ll = torch.empty(n, dtype=torch.float64, device=theta.device)
        ax = torch.empty((n, 3), dtype=torch.float64, device=theta.device) if aux else None
        pe_loglike_batch(self.handle, theta, n, precision, ll, ax, stream)
        return (ll, ax) if aux else ll


def weights_ess(loglike, logprior, logq, want_w=True, stream=None):
    import torch
    n = loglike.shape[0]
    w = torch.empty(n, dtype=torch.float64, device=loglike.device) if want_w else None
    st = torch.empty(4, dtype=torch.float64, device=loglike.device)
    pe_weights_ess(loglike, logprior, logq, n, w, st, stream)
    return w, st


def tile_assign(tiles_y, y, stream=None):
    """pe_tile_assign over [D, m] and [D, n] tensors (any row stride): int32 tile of every sample."""
    import torch
    D, m = tiles_y.shape
    n = y.shape[1]
    ty = tiles_y if tiles_y.stride(1) == 1 else tiles_y.contiguous()
    yy = y if y.stride(1) == 1 else y.contiguous()
    out = torch.empty(n, dtype=torch.int32, device=y.device)
    _check(load().pe_tile_assign(int(D), int(m), ctypes.c_void_p(ty.data_ptr()), int(ty.stride(0)), int(n),
                                 ctypes.c_void_p(yy.data_ptr()), int(yy.stride(0)), ctypes.c_void_p(out.data_ptr()),
                                 _stream(stream)))
    return out


def tile_assign_match_shift(ev, tiles_y, tiles_theta, y, theta, dt, n_shift, n_cand=8, stream=None):
    """pe_tile_assign_match_shift: as tile_assign_match, the match maximised over the time shifts
    j dt (|j| <= n_shift) as well."""
    import torch
    m = tiles_y.shape[1]
    n = y.shape[1]
    ty = tiles_y.contiguous()
    tt = tiles_theta.contiguous()
    yy = y.contiguous()
    th = theta.contiguous()
    out = torch.empty(n, dtype=torch.int32, device=y.device)
    mv = torch.empty(n, dtype=torch.float64, device=y.device)
    h = ev.handle if isinstance(ev, Event) else ev
    _check(load().pe_tile_assign_match_shift(h, int(m), ctypes.c_void_p(ty.data_ptr()),
                                             ctypes.c_void_p(tt.data_ptr()), int(m), int(n),
                                             ctypes.c_void_p(yy.data_ptr()), ctypes.c_void_p(th.data_ptr()), int(n),
                                             int(n_cand), float(dt), int(n_shift), ctypes.c_void_p(out.data_ptr()),
                                             ctypes.c_void_p(mv.data_ptr()), _stream(stream)))
    return out, mv


def tile_assign_match(ev, tiles_y, tiles_theta, y, theta, n_cand=8, stream=None):
    """pe_tile_assign_match: (int32 tile, match) of every sample; templates [4, m] and samples [4, n]
    as y and theta tensors of one row stride each."""
    import torch
    m = tiles_y.shape[1]
    n = y.shape[1]
    ty = tiles_y.contiguous()
    tt = tiles_theta.contiguous()
    yy = y.contiguous()
    th = theta.contiguous()
    out = torch.empty(n, dtype=torch.int32, device=y.device)
    mv = torch.empty(n, dtype=torch.float64, device=y.device)
    h = ev.handle if isinstance(ev, Event) else ev
    _check(load().pe_tile_assign_match(h, int(m), ctypes.c_void_p(ty.data_ptr()), ctypes.c_void_p(tt.data_ptr()),
                                       int(m), int(n), ctypes.c_void_p(yy.data_ptr()),
                                       ctypes.c_void_p(th.data_ptr()), int(n), int(n_cand),
                                       ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(mv.data_ptr()),
                                       _stream(stream)))
    return out, mv


def tile_draw(tile_loglike, tile_of, sample_logprior, samples_theta, seed, stream_id, n, stream=None):
    """pe_tile_draw: (theta [D, n], logq, logprior, index)."""
    import torch
    D, P = samples_theta.shape
    sm = samples_theta if samples_theta.stride(1) == 1 else samples_theta.contiguous()
    f64 = dict(dtype=torch.float64, device=sm.device)
    th = torch.empty((D, n), **f64)
    lq = torch.empty(n, **f64)
    lp = torch.empty(n, **f64)
    idx = torch.empty(n, dtype=torch.int64, device=sm.device)
    _check(load().pe_tile_draw(int(tile_loglike.shape[0]), _ptr(tile_loglike, torch.float64, "tile_loglike"), int(P),
                               _ptr(tile_of, torch.int32, "tile_of"),
                               _ptr(sample_logprior, torch.float64, "sample_logprior"), int(D),
                               ctypes.c_void_p(sm.data_ptr()), int(sm.stride(0)), int(seed) & 0xFFFFFFFFFFFFFFFF,
                               int(stream_id) & 0xFFFFFFFF, int(n), _ptr(th, torch.float64, "theta"),
                               _ptr(lq, torch.float64, "logq"), _ptr(lp, torch.float64, "logprior"),
                               _ptr(idx, torch.int64, "index"), _stream(stream)))
    return th, lq, lp, idx


def tile_extrinsic(ev, theta0, g, sub_mask, theta, logq, logprior, seed, stream_id, conditional=False, stream=None):
    """pe_tile_extrinsic on copies: (theta [D, n], logq, logprior) of the composed draws (the
    coordinates outside sub_mask drawn from the proposal's marginal over them, or from their
    conditional given each draw's sub_mask coordinates)."""
    th = theta.contiguous().clone()
    lq = logq.clone()
    lp = logprior.clone()
    n = th.shape[1]
    pe_tile_extrinsic(ev.handle, theta0, g, sub_mask, PE_TILE_CONDITIONAL if conditional else 0, seed, stream_id, n,
                      th, lq, lp, stream)
    return th, lq, lp


def tile_reweight(tile_loglike, tile_of, sample_logprior, index, w, alpha, stream=None):
    """pe_tile_reweight: per-tile values for the next round's tile_draw."""
    import torch
    out = torch.empty_like(tile_loglike)
    _check(load().pe_tile_reweight(int(tile_loglike.shape[0]), _ptr(tile_loglike, torch.float64, "tile_loglike"),
                                   int(tile_of.shape[0]), _ptr(tile_of, torch.int32, "tile_of"),
                                   _ptr(sample_logprior, torch.float64, "sample_logprior"), int(index.shape[0]),
                                   _ptr(index, torch.int64, "index"), _ptr(w, torch.float64, "w"), float(alpha),
                                   _ptr(out, torch.float64, "out"), _stream(stream)))
    return out


def loglike_multi(events, thetas, precision=PE_PREC_SPLIT, aux=False, stream=None):
    """pe_loglike_multi over Event objects; returns a list of loglike tensors (and aux tensors)."""
    import torch
    ns = [t.shape[1] for t in thetas]
    lls = [torch.empty(n, dtype=torch.float64, device=t.device) for n, t in zip(ns, thetas)]
    axs = [torch.empty((n, 3), dtype=torch.float64, device=t.device) for n, t in zip(ns, thetas)] if aux else None
    pe_loglike_multi(events, thetas, ns, precision, lls, axs, stream)
    return (lls, axs) if aux else lls


class Server:
    """Owns a pe_server_t. submit() takes numpy host arrays or device tensors for data/psd, a host
    theta0, the draw seed and count, and optional host output arrays (kept alive until the result
    is collected by wait())."""

    def __init__(self, hbm_budget, precision=PE_PREC_SPLIT, max_active=256, slice_ms=8.0, use_graph=True,
                 max_groups=0, items_target=0, min_group_bins=0):
        L = load()
        cfg = ServerConfig(int(hbm_budget), int(precision), int(max_active), float(slice_ms), int(bool(use_graph)),
                           int(max_groups), int(items_target), int(min_group_bins))
        h = ctypes.c_void_p()
        _check(L.pe_server_create(ctypes.byref(cfg), ctypes.byref(h)))
        self.handle = h
        self._keep = {}

    def now(self):
        return load().pe_server_now(self.handle)

    def submit(self, desc, data, psd, theta0, n_draws, seed, stream_id=0, metric_flags=0, loglike_out=None,
               w_out=None, theta_out=None):
        import numpy as np
        r = Request()
        r.desc = desc
        on_host = isinstance(data, np.ndarray)
        if on_host:
            data = np.ascontiguousarray(data)
            psd = np.ascontiguousarray(psd)
            r.data, r.psd = data.ctypes.data, psd.ctypes.data
        else:
            r.data, r.psd = data.data_ptr(), psd.data_ptr()
        r.data_on_host = int(on_host)
        r.metric_flags = int(metric_flags)
        th0 = np.ascontiguousarray(theta0, dtype=np.float64)
        r.theta0 = th0.ctypes.data
        r.seed = int(seed) & 0xFFFFFFFFFFFFFFFF
        r.stream_id = int(stream_id) & 0xFFFFFFFF
        r.n_draws = int(n_draws)
        outs = []
        for name, arr in (("loglike_out", loglike_out), ("w_out", w_out), ("theta_out", theta_out)):
            if arr is not None:
                assert arr.dtype == np.float64 and arr.flags["C_CONTIGUOUS"]
                setattr(r, name, arr.ctypes.data)
                outs.append(arr)
        t = ctypes.c_int64()
        _check(load().pe_server_submit(self.handle, ctypes.byref(r), ctypes.byref(t)))
        self._keep[t.value] = (data, psd, th0, outs)
        return t.value

    def wait(self, ticket, timeout=-1.0):
        res = Result()
        _check(load().pe_server_wait(self.handle, int(ticket), float(timeout), ctypes.byref(res)))
        self._keep.pop(int(ticket), None)
        return res

    def counters(self):
        out = (ctypes.c_int64 * 6)()
        _check(load().pe_server_counters(self.handle, out))
        keys = ("completed", "slices", "items", "graph_replays", "peak_slab_bytes", "admission_waits")
        return dict(zip(keys, list(out)))

    def busy_ms(self):
        """Device milliseconds so far: {"slices", "admission"} (pe_server_busy)."""
        out = (ctypes.c_double * 2)()
        _check(load().pe_server_busy(self.handle, out))
        return {"slices": out[0], "admission": out[1]}

    def tune(self, events, thetas, ns, reps=2):
        """Per-bucket plans from these events and device draws (pe_server_tune)."""
        import torch
        ne = len(events)
        ev_a = (ctypes.c_void_p * ne)(*[e.handle if isinstance(e, Event) else e for e in events])
        th_a = (ctypes.c_void_p * ne)(*[_ptr(t, torch.float64, "theta") for t in thetas])
        n_a = (ctypes.c_int64 * ne)(*[int(n) for n in ns])
        _check(load().pe_server_tune(self.handle, ne, ev_a, th_a, n_a, int(reps)))

    def plans(self):
        """[(n_det, log2 of the bin bound, items_target, min_group_bins, ms)] (pe_server_plans)."""
        c = ctypes.c_int32()
        _check(load().pe_server_plans(self.handle, 0, None, None, ctypes.byref(c)))
        n = max(c.value, 1)
        out = (ctypes.c_int32 * (4 * n))()
        ms = (ctypes.c_double * n)()
        _check(load().pe_server_plans(self.handle, n, out, ms, ctypes.byref(c)))
        return [(out[4 * i], out[4 * i + 1], out[4 * i + 2], out[4 * i + 3], ms[i]) for i in range(c.value)]

    def close(self):
        if self.handle is not None:
            h, self.handle = self.handle, None
            _check(load().pe_server_destroy(h))
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
