// pe_api.hip -- host runtime of the likelihood engine: the C ABI of include/pe.h,
// argument validation, device tables and workspace, stream ordering, profiling.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "pe_internal.h"

namespace {

thread_local std::string g_err;

pe_status_t fail(pe_status_t s, const std::string& msg) {
    g_err = msg;
    return s;
}

#define PE_HIP(call)                                                                                  \
    do {                                                                                              \
        hipError_t _e = (call);                                                                       \
        if (_e != hipSuccess) return fail(PE_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(_e)); \
    } while (0)

int g_chunks = 0;  // cap on the hot loop's groups of chunks per event; 0 = automatic (64)

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

pe_status_t validate_desc(const pe_event_desc_t* d) {
    if (!d) return fail(PE_ERR_ARG, "desc is NULL");
    if (d->n_det < 1 || d->n_det > PE_MAX_DET) return fail(PE_ERR_ARG, "n_det must be in 1..4");
    if (d->n_bins < 1 || d->n_bins > (int64_t)1 << 30) return fail(PE_ERR_ARG, "n_bins must be in 1..2^30");
    if (!(d->f_lo > 0.0) || !std::isfinite(d->f_lo)) return fail(PE_ERR_ARG, "f_lo must be > 0");
    if (!(d->df > 0.0) || !std::isfinite(d->df)) return fail(PE_ERR_ARG, "df must be > 0");
    if (d->data_dtype != PE_C128 && d->data_dtype != PE_C64) return fail(PE_ERR_ARG, "bad data_dtype");
    if (d->psd_dtype != PE_F64 && d->psd_dtype != PE_F32) return fail(PE_ERR_ARG, "bad psd_dtype");
    if (!(d->strain_scale > 0.0) || !std::isfinite(d->strain_scale)) return fail(PE_ERR_ARG, "strain_scale must be > 0");
    if (d->params != PE_PARAMS_4D && d->params != PE_PARAMS_11D) return fail(PE_ERR_ARG, "bad params");
    if (d->phase != PE_PHASE_MARG && d->phase != PE_PHASE_EXPLICIT) return fail(PE_ERR_ARG, "bad phase");
    if (d->params == PE_PARAMS_4D && d->phase != PE_PHASE_MARG)
        return fail(PE_ERR_ARG, "the 4-D parameter set is always phase-marginalised");
    if (d->params == PE_PARAMS_4D && !(d->amp0 > 0.0)) return fail(PE_ERR_ARG, "4-D needs amp0 > 0");
    if (!(d->chi_max >= 0.0)) return fail(PE_ERR_ARG, "chi_max must be >= 0");
    if (d->params == PE_PARAMS_11D && !(d->dl_max > 0.0)) return fail(PE_ERR_ARG, "11-D needs dl_max > 0");
    return PE_OK;
}

// Detector tensor D = (x x^T - y y^T)/2 from latitude, longitude and the
// x-arm azimuth (north toward east); y arm 90 degrees east of x.
void build_const(const pe_event_desc_t& d, pe::EvConst& ec) {
    std::memset(&ec, 0, sizeof(ec));
    ec.n_det = d.n_det;
    ec.params = d.params;
    ec.phase = d.phase;
    ec.dim = pe_dim(d.params);
    ec.K = d.n_bins;
    ec.f_lo = d.f_lo;
    ec.df = d.df;
    ec.scale = d.strain_scale;
    ec.amp0 = d.amp0;
    ec.gmst = d.gmst;
    ec.chi_max = d.chi_max;
    ec.dl_max = d.dl_max;
    for (int i = 0; i < d.n_det; ++i) {
        const double lat = d.det_geom[i][0], lon = d.det_geom[i][1], az = d.det_geom[i][2];
        const double up[3] = {std::cos(lat) * std::cos(lon), std::cos(lat) * std::sin(lon), std::sin(lat)};
        const double east[3] = {-std::sin(lon), std::cos(lon), 0.0};
        const double north[3] = {-std::sin(lat) * std::cos(lon), -std::sin(lat) * std::sin(lon), std::cos(lat)};
        double x[3], y[3];
        for (int a = 0; a < 3; ++a) {
            x[a] = std::cos(az) * north[a] + std::sin(az) * east[a];
            y[a] = -std::sin(az) * north[a] + std::cos(az) * east[a];
        }
        auto T = [&](int a, int b) { return 0.5 * (x[a] * x[b] - y[a] * y[b]); };
        ec.dtensor[i][0] = T(0, 0);
        ec.dtensor[i][1] = T(0, 1);
        ec.dtensor[i][2] = T(0, 2);
        ec.dtensor[i][3] = T(1, 1);
        ec.dtensor[i][4] = T(1, 2);
        ec.dtensor[i][5] = T(2, 2);
        for (int a = 0; a < 3; ++a) ec.up[i][a] = up[a];
    }
}

template <typename T>
pe_status_t dalloc(T** p, size_t count) {
    *p = nullptr;
    if (count == 0) count = 1;
    hipError_t e = hipMalloc((void**)p, count * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(PE_ERR_OOM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
    }
    return PE_OK;
}

template <typename T>
void dfree(T*& p) {
    if (p) (void)hipFree(p);
    p = nullptr;
}

void free_batch(pe::BatchDev& b) {
    dfree(b.evs);
    dfree(b.doff);
    dfree(b.ioff);
    dfree(b.hdr);
    b.cap = 0;
}

pe_status_t ensure_batch(pe::BatchDev& b, int n_events) {
    if (n_events <= b.cap) return PE_OK;
    if (b.cap > 0) PE_HIP(hipDeviceSynchronize());  // earlier batches may still read the old buffers
    free_batch(b);
    pe_status_t s;
    if ((s = dalloc(&b.evs, (size_t)n_events)) != PE_OK) return s;
    if ((s = dalloc(&b.doff, (size_t)n_events + 1)) != PE_OK) return s;
    if ((s = dalloc(&b.ioff, (size_t)n_events + 1)) != PE_OK) return s;
    if ((s = dalloc(&b.hdr, 4)) != PE_OK) return s;
    b.cap = n_events;
    return PE_OK;
}

void free_draw_ws(pe_event_s* ev) {
    dfree(ev->kc_all);
    dfree(ev->hist);
    dfree(ev->plan);
    dfree(ev->idx);
    dfree(ev->coef);
    dfree(ev->kcut);
    dfree(ev->resp);
    dfree(ev->hh);
    dfree(ev->partial);
    ev->npad = 0;
    ev->partial_cap = 0;
}

void free_event(pe_event_s* ev) {
    if (!ev) return;
    free_draw_ws(ev);
    free_batch(ev->self);
    dfree(ev->rec32);
    dfree(ev->rec64);
    dfree(ev->pw);
    dfree(ev->pfx);
    dfree(ev->status);
    dfree(ev->mws);
    delete ev;
}

// Per-draw workspace for batches of up to n draws. The hot loop keeps up to 64
// groups of partials per draw and detector; min(64 npad, 2^22) slots per
// detector bound the groups of large batches (16 at 2^18 draws), where the plan
// asks for few groups anyway (it aims at ~16k work items per event).
pe_status_t ensure_ws(pe_event_s* ev, int64_t n) {
    const int64_t npad = ((n + pe::kTile - 1) / pe::kTile) * pe::kTile;
    if (npad <= ev->npad && ev->partial) return PE_OK;
    PE_HIP(hipDeviceSynchronize());
    const int64_t np = npad > ev->npad ? npad : ev->npad;
    free_draw_ws(ev);
    const int nd = ev->desc.n_det;
    const int64_t cap = std::min<int64_t>(64 * np, (int64_t)1 << 22);
    pe_status_t s;
    if ((s = dalloc(&ev->kc_all, (size_t)np)) != PE_OK) return s;
    if ((s = dalloc(&ev->hist, (size_t)pe::kBuckets)) != PE_OK) return s;
    if ((s = dalloc(&ev->plan, 1)) != PE_OK) return s;
    if ((s = dalloc(&ev->idx, (size_t)np)) != PE_OK) return s;
    if ((s = dalloc(&ev->coef, (size_t)pe::kNCoef * np)) != PE_OK) return s;
    if ((s = dalloc(&ev->kcut, (size_t)np)) != PE_OK) return s;
    if ((s = dalloc(&ev->resp, (size_t)2 * nd * np)) != PE_OK) return s;
    if ((s = dalloc(&ev->hh, (size_t)np)) != PE_OK) return s;
    if ((s = dalloc(&ev->partial, (size_t)nd * cap)) != PE_OK) return s;
    ev->npad = np;
    ev->partial_cap = cap;
    return PE_OK;
}

pe::EvDev make_evdev(const pe_event_s* ev, const double* theta, int64_t n, double* loglike, double* aux) {
    pe::EvDev d;
    std::memset(&d, 0, sizeof(d));
    d.ec = ev->ec;
    d.rec32 = ev->rec32;
    d.rec64 = ev->rec64;
    d.pfx = ev->pfx;
    d.kc_all = ev->kc_all;
    d.hist = ev->hist;
    d.idx = ev->idx;
    d.kcut = ev->kcut;
    d.coef = ev->coef;
    d.resp = ev->resp;
    d.hh = ev->hh;
    d.partial = ev->partial;
    d.plan = ev->plan;
    d.npad = ev->npad;
    int64_t mg = ev->partial_cap / (ev->npad > 0 ? ev->npad : 1);
    if (mg > 64) mg = 64;
    if (g_chunks > 0 && mg > g_chunks) mg = g_chunks;
    d.max_groups = (int)(mg < 1 ? 1 : mg);
    d.theta = theta;
    d.n = n;
    d.loglike = loglike;
    d.aux = aux;
    return d;
}

// Upload the descriptors of ne events (same n_det) and launch the batch.
pe_status_t run_batch(pe::BatchDev& b, const std::vector<pe::EvDev>& evs, int n_det, int precision,
                      hipStream_t st) {
    const int ne = (int)evs.size();
    pe_status_t s = ensure_batch(b, ne);
    if (s != PE_OK) return s;
    std::vector<int64_t> off(ne + 1, 0);
    for (int e = 0; e < ne; ++e) off[e + 1] = off[e] + evs[e].n;
    PE_HIP(hipMemcpyAsync(b.evs, evs.data(), sizeof(pe::EvDev) * ne, hipMemcpyHostToDevice, st));
    PE_HIP(hipMemcpyAsync(b.doff, off.data(), sizeof(int64_t) * (ne + 1), hipMemcpyHostToDevice, st));
    PE_HIP(pe::launch_batch(b, ne, n_det, off[ne], precision, st));
    return PE_OK;
}

// ------------------------------------------------------------------ profiling
std::mutex g_prof_mu;
bool g_prof_on = false;
std::map<std::string, std::vector<std::pair<hipEvent_t, hipEvent_t>>> g_prof;
std::map<std::string, hipEvent_t> g_prof_open;

}  // namespace

namespace pe {

void prof_begin(const char* name, hipStream_t st) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (!g_prof_on) return;
    hipEvent_t a;
    if (hipEventCreate(&a) != hipSuccess) return;
    (void)hipEventRecord(a, st);
    g_prof_open[name] = a;
}

void prof_end(const char* name, hipStream_t st) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (!g_prof_on) return;
    auto it = g_prof_open.find(name);
    if (it == g_prof_open.end()) return;
    hipEvent_t b;
    if (hipEventCreate(&b) != hipSuccess) return;
    (void)hipEventRecord(b, st);
    g_prof[name].push_back({it->second, b});
    g_prof_open.erase(it);
}

}  // namespace pe

extern "C" {

int32_t pe_dim(int32_t params) {
    return params == PE_PARAMS_4D ? 4 : (params == PE_PARAMS_11D ? 11 : 0);
}

const char* pe_last_error(void) { return g_err.c_str(); }

pe_status_t pe_event_create(const pe_event_desc_t* desc, const void* data_dev, const void* psd_dev, void* stream,
                            pe_event_t* out) {
    if (!out) return fail(PE_ERR_ARG, "out is NULL");
    *out = nullptr;
    pe_status_t s = validate_desc(desc);
    if (s != PE_OK) return s;
    if (!data_dev || !psd_dev) return fail(PE_ERR_ARG, "data and psd must be device pointers");
    pe_event_s* ev = new (std::nothrow) pe_event_s();
    if (!ev) return fail(PE_ERR_OOM, "host allocation failed");
    ev->desc = *desc;
    build_const(*desc, ev->ec);
    const int64_t K = desc->n_bins;
    const int nd = desc->n_det;
    if ((s = dalloc(&ev->rec32, (size_t)(K + pe::kTabPad))) != PE_OK ||
        (s = dalloc(&ev->rec64, (size_t)(K + pe::kTabPad))) != PE_OK ||
        (s = dalloc(&ev->pw, (size_t)nd * K)) != PE_OK || (s = dalloc(&ev->pfx, (size_t)nd * (K + 1))) != PE_OK ||
        (s = dalloc(&ev->status, 1)) != PE_OK || (s = dalloc(&ev->mws, (size_t)pe::kMwsTotal)) != PE_OK) {
        free_event(ev);
        return s;
    }
    hipStream_t st = as_stream(stream);
    hipError_t e = hipMemsetAsync(ev->status, 0, sizeof(int), st);
    if (e == hipSuccess) e = hipMemsetAsync(ev->rec32 + K, 0, sizeof(pe::Rec32) * pe::kTabPad, st);
    if (e == hipSuccess) e = hipMemsetAsync(ev->rec64 + K, 0, sizeof(pe::Rec64) * pe::kTabPad, st);
    if (e == hipSuccess) e = hipMemsetAsync(ev->mws, 0, sizeof(double) * pe::kMwsTotal, st);
    if (e == hipSuccess) e = pe::launch_prep(ev, data_dev, psd_dev, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        free_event(ev);
        return fail(PE_ERR_HIP, std::string("event preparation: ") + hipGetErrorString(e));
    }
    s = pe_event_status(ev, stream);
    if (s != PE_OK) {
        std::string msg = g_err;
        free_event(ev);
        return fail(s, msg);
    }
    *out = ev;
    return PE_OK;
}

pe_status_t pe_event_update(pe_event_t ev, const void* data_dev, const void* psd_dev, void* stream) {
    if (!ev) return fail(PE_ERR_ARG, "event is NULL");
    if (!data_dev || !psd_dev) return fail(PE_ERR_ARG, "data and psd must be device pointers");
    PE_HIP(pe::launch_prep(ev, data_dev, psd_dev, as_stream(stream)));
    return PE_OK;
}

pe_status_t pe_event_status(pe_event_t ev, void* stream) {
    if (!ev) return fail(PE_ERR_ARG, "event is NULL");
    hipStream_t st = as_stream(stream);
    PE_HIP(hipStreamSynchronize(st));
    int flags = 0;
    PE_HIP(hipMemcpy(&flags, ev->status, sizeof(int), hipMemcpyDeviceToHost));
    if (flags) PE_HIP(hipMemset(ev->status, 0, sizeof(int)));
    if (flags & pe::kStBadPsd) return fail(PE_ERR_ARG, "PSD values must be positive and finite");
    if (flags & pe::kStNonfinite) return fail(PE_ERR_NONFINITE, "data contains inf or nan");
    if (flags & pe::kStSingular) return fail(PE_ERR_SINGULAR, "metric is not positive definite");
    return PE_OK;
}

pe_status_t pe_event_reserve(pe_event_t ev, int64_t max_draws) {
    if (!ev) return fail(PE_ERR_ARG, "event is NULL");
    if (max_draws < 0 || max_draws > ((int64_t)1 << 30)) return fail(PE_ERR_ARG, "max_draws must be in 0..2^30");
    return ensure_ws(ev, max_draws);
}

pe_status_t pe_event_destroy(pe_event_t ev) {
    if (!ev) return fail(PE_ERR_ARG, "event is NULL");
    (void)hipDeviceSynchronize();
    free_event(ev);
    return PE_OK;
}

pe_status_t pe_metric(pe_event_t ev, const double* theta0_dev, const double* fd_step_dev, int32_t flags,
                      double* g_dev, void* stream) {
    if (!ev) return fail(PE_ERR_ARG, "event is NULL");
    if (!theta0_dev || !g_dev) return fail(PE_ERR_ARG, "theta0 and g must be device pointers");
    if (flags & ~1) return fail(PE_ERR_ARG, "unknown metric flags");
    PE_HIP(pe::launch_metric(ev, theta0_dev, fd_step_dev, flags, g_dev, as_stream(stream)));
    return PE_OK;
}

pe_status_t pe_draw(pe_event_t ev, const double* theta0_dev, const double* g_dev, uint64_t seed, uint32_t stream_id,
                    int64_t n, double* theta_dev, double* logq_dev, double* logprior_dev, void* stream) {
    if (!ev) return fail(PE_ERR_ARG, "event is NULL");
    if (n < 0 || n > ((int64_t)1 << 30)) return fail(PE_ERR_ARG, "n must be in 0..2^30");
    if (!theta0_dev || !g_dev) return fail(PE_ERR_ARG, "theta0 and g must be device pointers");
    if (n > 0 && (!theta_dev || !logq_dev || !logprior_dev)) return fail(PE_ERR_ARG, "output pointers are NULL");
    PE_HIP(pe::launch_draw(ev, theta0_dev, g_dev, seed, stream_id, n, theta_dev, logq_dev, logprior_dev,
                           as_stream(stream)));
    return PE_OK;
}

pe_status_t pe_loglike_batch(pe_event_t ev, const double* theta_dev, int64_t n, int32_t precision,
                             double* loglike_dev, double* aux_dev, void* stream) {
    if (!ev) return fail(PE_ERR_ARG, "event is NULL");
    if (n < 0 || n > ((int64_t)1 << 30)) return fail(PE_ERR_ARG, "n must be in 0..2^30");
    if (precision != PE_PREC_FP64 && precision != PE_PREC_SPLIT) return fail(PE_ERR_ARG, "bad precision");
    if (n == 0) return PE_OK;
    if (!theta_dev || !loglike_dev) return fail(PE_ERR_ARG, "theta and loglike must be device pointers");
    pe_status_t s = ensure_ws(ev, n);
    if (s != PE_OK) return s;
    std::vector<pe::EvDev> one(1, make_evdev(ev, theta_dev, n, loglike_dev, aux_dev));
    return run_batch(ev->self, one, ev->desc.n_det, precision, as_stream(stream));
}

pe_status_t pe_loglike_multi(int32_t n_events, const pe_event_t* events, const double* const* theta_dev,
                             const int64_t* n, int32_t precision, double* const* loglike_dev,
                             double* const* aux_dev, void* stream) {
    if (n_events < 0 || n_events > 65535 || (n_events > 0 && (!events || !theta_dev || !n || !loglike_dev)))
        return fail(PE_ERR_ARG, "bad batch arrays (n_events must be in 0..65535)");
    if (precision != PE_PREC_FP64 && precision != PE_PREC_SPLIT) return fail(PE_ERR_ARG, "bad precision");
    // One batch per detector count; its descriptor buffers are those of its
    // first event, so two calls race only where they share an event.
    std::vector<pe::EvDev> cls[PE_MAX_DET + 1];
    pe_event_s* owner[PE_MAX_DET + 1] = {};
    for (int e = 0; e < n_events; ++e) {
        pe_event_s* ev = events[e];
        if (!ev) return fail(PE_ERR_ARG, "event is NULL");
        for (int f = 0; f < e; ++f)
            if (events[f] == ev) return fail(PE_ERR_ARG, "an event appears twice in the batch");
        if (n[e] < 0 || n[e] > ((int64_t)1 << 30)) return fail(PE_ERR_ARG, "n must be in 0..2^30");
        if (n[e] == 0) continue;
        if (!theta_dev[e] || !loglike_dev[e]) return fail(PE_ERR_ARG, "theta and loglike must be device pointers");
        pe_status_t s = ensure_ws(ev, n[e]);
        if (s != PE_OK) return s;
        const int nd = ev->desc.n_det;
        if (!owner[nd]) owner[nd] = ev;
        cls[nd].push_back(make_evdev(ev, theta_dev[e], n[e], loglike_dev[e], aux_dev ? aux_dev[e] : nullptr));
    }
    for (int nd = 1; nd <= PE_MAX_DET; ++nd) {
        if (cls[nd].empty()) continue;
        pe_status_t s = run_batch(owner[nd]->self, cls[nd], nd, precision, as_stream(stream));
        if (s != PE_OK) return s;
    }
    return PE_OK;
}

pe_status_t pe_weights_ess(const double* loglike_dev, const double* logprior_dev, const double* logq_dev, int64_t n,
                           double* w_dev, double* stats_dev, void* stream) {
    if (n < 0) return fail(PE_ERR_ARG, "n must be >= 0");
    if (!stats_dev) return fail(PE_ERR_ARG, "stats must be a device pointer");
    if (n > 0 && (!loglike_dev || !logprior_dev || !logq_dev)) return fail(PE_ERR_ARG, "inputs are NULL");
    PE_HIP(pe::launch_weights(loglike_dev, logprior_dev, logq_dev, n, w_dev, stats_dev, as_stream(stream)));
    return PE_OK;
}

pe_status_t pe_waveform(const pe_event_desc_t* desc, const double* theta_dev, const void* psd_dev, double* h_dev,
                        double* snr2_dev, void* stream) {
    pe_event_desc_t d2;
    if (!desc) return fail(PE_ERR_ARG, "desc is NULL");
    d2 = *desc;
    if (d2.params == PE_PARAMS_4D && !(d2.amp0 > 0.0)) d2.amp0 = 1.0;
    pe_status_t s = validate_desc(&d2);
    if (s != PE_OK) return s;
    if (!theta_dev || !h_dev) return fail(PE_ERR_ARG, "theta and h must be device pointers");
    if (snr2_dev && !psd_dev) return fail(PE_ERR_ARG, "snr2 needs the PSD");
    pe::EvConst ec;
    build_const(*desc, ec);
    const int64_t nb = (ec.K + 255) / 256;
    double* scratch = nullptr;
    if ((s = dalloc(&scratch, (size_t)(32 + nb))) != PE_OK) return s;
    hipStream_t st = as_stream(stream);
    hipError_t e = pe::launch_waveform(ec, desc->psd_dtype, theta_dev, psd_dev, h_dev, snr2_dev, scratch, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    dfree(scratch);
    if (e != hipSuccess) return fail(PE_ERR_HIP, std::string("waveform: ") + hipGetErrorString(e));
    return PE_OK;
}

pe_status_t pe_rng_uniforms(uint64_t seed, uint32_t stream_id, int64_t n, int32_t npairs, double* u_dev,
                            void* stream) {
    if (n < 0 || npairs < 0 || npairs > 64) return fail(PE_ERR_ARG, "bad n or npairs");
    if (n * npairs > 0 && !u_dev) return fail(PE_ERR_ARG, "u must be a device pointer");
    PE_HIP(pe::launch_uniforms(seed, stream_id, n, npairs, u_dev, as_stream(stream)));
    return PE_OK;
}

pe_status_t pe_profile_enable(int32_t enable) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_on = enable != 0;
    return PE_OK;
}

pe_status_t pe_profile_read(const char* kernel, double* total_ms, int64_t* launches) {
    if (!kernel || !total_ms || !launches) return fail(PE_ERR_ARG, "NULL argument");
    std::vector<std::pair<hipEvent_t, hipEvent_t>> v;
    {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        auto it = g_prof.find(kernel);
        if (it != g_prof.end()) {
            v.swap(it->second);
            g_prof.erase(it);
        }
    }
    double tot = 0.0;
    pe_status_t s = PE_OK;
    for (auto& p : v) {
        float ms = 0.0f;
        if (hipEventSynchronize(p.second) != hipSuccess || hipEventElapsedTime(&ms, p.first, p.second) != hipSuccess)
            s = fail(PE_ERR_HIP, "profiling event failed");
        tot += ms;
        (void)hipEventDestroy(p.first);
        (void)hipEventDestroy(p.second);
    }
    *total_ms = tot;
    *launches = (int64_t)v.size();
    return s;
}

pe_status_t pe_set_chunks(int32_t n_chunks) {
    if (n_chunks < 0 || n_chunks > 64) return fail(PE_ERR_ARG, "n_chunks must be in 0..64");
    g_chunks = n_chunks;
    return PE_OK;
}

}  // extern "C"
