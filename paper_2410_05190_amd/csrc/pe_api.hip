// pe_api.hip -- host runtime of the likelihood engine: the C ABI of include/pe.h,
// argument validation, event memory, batch areas, stream ordering, profiling.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "pe_host.h"

namespace {

thread_local std::string g_err;
int g_chunks = 0;             // cap on the hot loop's groups of chunks per event; 0 = automatic (64)
int g_items_target = 16384;   // plan: work items per event
int g_min_group_bins = 1024;  // plan: bins per group at least
double g_redo_budget = pe::kRedoBudget;  // split path: FP64 re-evaluation above this |d ln L| estimate

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

}  // namespace

namespace pe {

pe_status_t fail(pe_status_t s, const std::string& msg) {
    g_err = msg;
    return s;
}

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
    if (d->distance != PE_DIST_SAMPLED && d->distance != PE_DIST_MARG) return fail(PE_ERR_ARG, "bad distance");
    if (d->distance == PE_DIST_MARG && d->params != PE_PARAMS_11D)
        return fail(PE_ERR_ARG, "distance marginalisation needs the 11-D parameter set");
    if (d->time_marg != 0 && d->time_marg != 1) return fail(PE_ERR_ARG, "time_marg must be 0 or 1");
    if (d->time_marg) {
        if (d->params != PE_PARAMS_11D) return fail(PE_ERR_ARG, "time marginalisation needs the 11-D parameter set");
        if (d->tm_points < 8 || d->tm_points > PE_MAX_TM_POINTS)
            return fail(PE_ERR_ARG, "tm_points must be in 8..PE_MAX_TM_POINTS");
        if (!(d->tc_lo < d->tc_hi) || !std::isfinite(d->tc_lo) || !std::isfinite(d->tc_hi))
            return fail(PE_ERR_ARG, "the tc window needs tc_lo < tc_hi");
    }
    return PE_OK;
}

// Whether a time-marginalised event's batch takes the block-moment path: split
// precision and a window that the moments cover (ec.tm_P > 0).
bool tm_moments(const pe_event_s* ev, int precision) {
    return ev->desc.time_marg && precision == PE_PREC_SPLIT && ev->ec.tm_P > 0;
}

// Draws the workspace must hold for a batch of n: a time-marginalised event
// off the moment path evaluates every draw at each of its tc nodes.
int64_t ws_draws(const pe_event_s* ev, int64_t n, int precision) {
    return (ev->desc.time_marg && !tm_moments(ev, precision)) ? n * ev->desc.tm_points : n;
}

// The block moments of a batch of n draws (own allocation, grown on demand).
pe_status_t ensure_moments(pe_event_s* ev, int64_t n) {
    const int64_t cols = std::max<int64_t>(npad_for(n), kTile);
    if (cols <= ev->tm_mom_cols && ev->tm_mem) return PE_OK;
    const int64_t blocks = ev->desc.n_bins / ev->ec.tm_fine + 2;
    PE_HIP(hipDeviceSynchronize());
    dfree_bytes(ev->tm_mem);
    ev->tm_mem = nullptr;
    ev->tm_mom_cols = 0;
    pe_status_t s = dalloc_bytes(&ev->tm_mem, sizeof(double2) * (size_t)blocks * ev->ec.tm_P * (size_t)cols);
    if (s != PE_OK) return s;
    ev->tm_mom_cols = cols;
    if (!ev->tm_pow && ev->ec.tm_fine <= kTmPowMaxBins) {
        // the block's power table, once per event (the device is idle here)
        s = dalloc_bytes(&ev->tm_pow, sizeof(float) * (size_t)ev->ec.tm_fine * ev->ec.tm_P);
        if (s != PE_OK) return s;
        PE_HIP(launch_tm_powers((float*)ev->tm_pow, ev->ec.tm_fine, ev->ec.tm_P, nullptr));
        PE_HIP(hipDeviceSynchronize());
    }
    return PE_OK;
}

// Detector tensor D = (x x^T - y y^T)/2 from latitude, longitude and the
// x-arm azimuth (north toward east); y arm 90 degrees east of x.
void build_const(const pe_event_desc_t& d, EvConst& ec) {
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
    ec.dist = (d.distance == PE_DIST_MARG) ? 1 : 0;
    ec.tm = d.time_marg ? 1 : 0;
    ec.tm_points = d.time_marg ? d.tm_points : 0;
    if (d.time_marg) {
        // block width of the moment path: the widest multiple of kBlk bins with
        // pi (width) |u| <= kTmAlpha over the window, with 8 moments, else 16
        const double U = 0.5 * (d.tc_hi - d.tc_lo);
        const double alpha[2] = {kTmAlpha8, kTmAlpha16};
        const int P[2] = {8, 16};
        for (int i = 0; i < 2 && ec.tm_P == 0; ++i) {
            const double bins = alpha[i] / (kPi * d.df * U);
            const int64_t f = bins >= (double)(1 << 24) ? (1 << 24) : ((int64_t)bins / kBlk) * kBlk;
            if (f >= kBlk) {
                ec.tm_P = P[i];
                ec.tm_fine = (int32_t)f;
            }
        }
        ec.tm_tmid = 0.5 * (d.tc_lo + d.tc_hi);
        ec.tm_a = kPi * ec.tm_fine * d.df;
    }
    ec.tc_lo = d.tc_lo;
    ec.tc_hi = d.tc_hi;
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

pe_status_t dalloc_bytes(char** p, size_t bytes) {
    *p = nullptr;
    hipError_t e = hipMalloc((void**)p, bytes ? bytes : 1);
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(PE_ERR_OOM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
    }
    return PE_OK;
}

void dfree_bytes(char*& p) {
    if (p) (void)hipFree(p);
    p = nullptr;
}

// ------------------------------------------------------------- event memory
// Tables: rec32/rec64 (K + kTabPad records), pw, pfx, status word, metric and
// draw workspace. Workspace for npad draws: cuts, bucket counts, plan, order,
// coefficient rows, responses, (h|h) and the hot loop's partials.
int64_t npad_for(int64_t n) { return ((n + kTile - 1) / kTile) * kTile; }

// Groups of frequency chunks a batch of np draws may use on an event of K
// bins: at most 64, at most one per 1024 bins (the plan never asks for more),
// and at most 2^22 / np so that the partials stay bounded.
int64_t groups_cap(int64_t np, int64_t K) {
    int64_t g = std::min<int64_t>(64, std::max<int64_t>(1, K / 1024));
    g = std::min<int64_t>(g, ((int64_t)1 << 22) / std::max<int64_t>(np, 1));
    return std::max<int64_t>(g, 1);
}

// Partial slots per detector of a workspace for up to npad draws: enough for
// any batch of np <= npad draws (np * groups_cap(np, K) never exceeds it), and
// for the prologue's parameter records (kRecStride doubles per draw), which
// use the same memory before the hot loop runs.
int64_t partial_cap_for(int64_t npad, int64_t K, int n_det) {
    const int64_t groups = std::min<int64_t>(npad * std::min<int64_t>(64, std::max<int64_t>(1, K / 1024)),
                                             std::max<int64_t>((int64_t)1 << 22, npad));
    const int64_t recs = (kRecStride * npad + 2 * n_det - 1) / (2 * n_det);
    return std::max(groups, recs);
}

size_t layout_tables(pe_event_s* ev, char* base) {
    Carver c(base);
    const int64_t K = ev->desc.n_bins;
    const int nd = ev->desc.n_det;
    ev->rec32 = c.take<Rec32>((size_t)(K + kTabPad));
    ev->rec64 = c.take<Rec64>((size_t)(K + kTabPad));
    ev->pw = c.take<double>((size_t)nd * K);
    ev->pfx = c.take<double>((size_t)nd * (K + 1));
    ev->pl1 = c.take<double>((size_t)nd * (K + 1));
    ev->pw2 = c.take<double>((size_t)nd * (K + 1));
    ev->ppw = c.take<double>((size_t)nd * (K + 1));
    ev->guard = c.take<double>((size_t)kGuardLen);
    ev->status = c.take<int>(1);
    ev->mws = c.take<double>((size_t)kMwsTotal);
    ev->mix_chol = c.take<double>((size_t)PE_MIX_MAX * kCholLen);
    return c.size();
}

size_t layout_ws(pe_event_s* ev, int64_t npad, char* base) {
    Carver c(base);
    const int nd = ev->desc.n_det;
    const int64_t cap = partial_cap_for(npad, ev->desc.n_bins, nd);
    ev->kc_all = c.take<int>((size_t)npad);
    ev->hist = c.take<int>((size_t)kBuckets);
    ev->plan = c.take<EvPlan>(2);
    ev->idx = c.take<int>((size_t)npad);
    ev->rflag = c.take<int>((size_t)npad);
    ev->rcnt = c.take<int>((size_t)(npad / kTile + 1));
    ev->rpos = c.take<int>((size_t)npad);
    ev->zd = c.take<double2>((size_t)npad);
    if (ev->desc.time_marg) {
        ev->tm_theta = c.take<double>((size_t)PE_MAX_DIM * npad);
        ev->tm_ll = c.take<double>((size_t)npad);
    }
    ev->coef = c.take<double>((size_t)kNCoef * npad);
    ev->kcut = c.take<int>((size_t)npad);
    ev->resp = c.take<double>((size_t)2 * nd * npad);
    ev->hh = c.take<double>((size_t)npad);
    ev->partial = c.take<double2>((size_t)nd * cap);
    if (base) {
        ev->npad = npad;
        ev->partial_cap = cap;
    }
    return c.size();
}

size_t tables_bytes(const pe_event_desc_t& d) {
    pe_event_s tmp;
    tmp.desc = d;
    return layout_tables(&tmp, nullptr);
}

size_t ws_bytes(const pe_event_desc_t& d, int64_t npad) {
    pe_event_s tmp;
    tmp.desc = d;
    return layout_ws(&tmp, npad, nullptr);
}

size_t event_footprint(const pe_event_desc_t& d, int64_t max_draws) {
    return align_up(tables_bytes(d), 256) + ws_bytes(d, npad_for(max_draws));
}

// Grow the workspace to hold batches of n draws (own memory only).
pe_status_t ensure_ws(pe_event_s* ev, int64_t n) {
    const int64_t npad = npad_for(n);
    if (npad <= ev->npad && ev->partial) return PE_OK;
    if (!ev->own_mem) return fail(PE_ERR_ARG, "the event was sized for fewer draws");
    PE_HIP(hipDeviceSynchronize());
    dfree_bytes(ev->ws_mem);
    ev->npad = 0;
    ev->partial = nullptr;
    pe_status_t s = dalloc_bytes(&ev->ws_mem, ws_bytes(ev->desc, npad));
    if (s != PE_OK) return s;
    layout_ws(ev, npad, ev->ws_mem);
    return PE_OK;
}

void free_event(pe_event_s* ev) {
    if (!ev) return;
    if (ev->own_mem) {
        dfree_bytes(ev->tab_mem);
        dfree_bytes(ev->ws_mem);
    }
    dfree_bytes(ev->rb_mem);
    dfree_bytes(ev->tm_mem);
    dfree_bytes(ev->tm_pow);
    delete ev;
}

// Event object with its pointers laid out in `mem` (tables, then workspace for
// max_draws), or in its own allocations when mem is NULL.
pe_status_t new_event(const pe_event_desc_t* desc, char* mem, int64_t max_draws, pe_event_s** out) {
    *out = nullptr;
    pe_status_t s = validate_desc(desc);
    if (s != PE_OK) return s;
    pe_event_s* ev = new (std::nothrow) pe_event_s();
    if (!ev) return fail(PE_ERR_OOM, "host allocation failed");
    ev->desc = *desc;
    build_const(*desc, ev->ec);
    if (mem) {
        ev->own_mem = false;
        const size_t tb = align_up(tables_bytes(*desc), 256);
        ev->tab_mem = mem;
        ev->ws_mem = mem + tb;
        layout_tables(ev, ev->tab_mem);
        layout_ws(ev, npad_for(max_draws), ev->ws_mem);
    } else {
        if ((s = dalloc_bytes(&ev->tab_mem, tables_bytes(*desc))) != PE_OK) {
            free_event(ev);
            return s;
        }
        layout_tables(ev, ev->tab_mem);
        if (max_draws > 0 && (s = ensure_ws(ev, max_draws)) != PE_OK) {
            free_event(ev);
            return s;
        }
    }
    *out = ev;
    return PE_OK;
}

// --------------------------------------------------------------- batch areas
// One device buffer per (stream, kind): header, argument records, offsets
// (uploaded with one copy, skipped when identical to the last upload), then
// scratch. Batches on one stream are ordered, so the buffer is reused safely;
// the area's lock is held from the upload until the launches are queued.
std::mutex g_areas_mu;
std::map<std::pair<void*, int>, std::unique_ptr<Area>> g_areas;

Area& area_for(hipStream_t st, int kind) {
    std::lock_guard<std::mutex> lk(g_areas_mu);
    auto& p = g_areas[{(void*)st, kind}];
    if (!p) p.reset(new Area());
    return *p;
}

size_t area_bytes(int ne, size_t arg_bytes, size_t scratch_bytes) {
    const size_t o_args = 256;
    const size_t o_off = align_up(o_args + arg_bytes, 256);
    const size_t o_off2 = align_up(o_off + sizeof(int64_t) * (ne + 1), 256);
    const size_t o_scr = align_up(o_off2 + sizeof(int64_t) * (ne + 1), 256);
    return o_scr + std::max<size_t>(scratch_bytes, 256);
}

pe_status_t reserve_area(Area& A, size_t bytes) {
    if (bytes <= A.cap) return PE_OK;
    PE_HIP(hipDeviceSynchronize());  // earlier batches may still read the old buffer
    dfree_bytes(A.dev);
    A.cap = 0;
    A.shadow.clear();
    pe_status_t s = dalloc_bytes(&A.dev, bytes);
    if (s != PE_OK) return s;
    A.cap = bytes;
    return PE_OK;
}

void release_area(Area& A) {
    dfree_bytes(A.dev);
    A.cap = 0;
    A.shadow.clear();
    for (int k = 0; k < 2; ++k) {
        if (A.done[k]) {
            (void)hipEventSynchronize(A.done[k]);
            (void)hipEventDestroy(A.done[k]);
            A.done[k] = nullptr;
        }
        if (A.host[k]) (void)hipHostFree(A.host[k]);
        A.host[k] = A.host_dev[k] = nullptr;
        A.host_cap[k] = 0;
    }
}

// Copies an argument image from pinned host memory into the area on the
// stream: 16-byte words, grid-strided. A kernel keeps the upload on the
// compute queue, ordered with the launches around it, and leaves the host free:
// the runtime's small host-to-device copies have stalled the host for
// milliseconds behind the stream's earlier work.
__global__ __launch_bounds__(256) void k_upload(uint4* __restrict__ dst, const uint4* __restrict__ src, int64_t n16) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n16; i += (int64_t)gridDim.x * 256) dst[i] = src[i];
}

hipError_t upload_bytes(char* dst, const char* src, size_t bytes, hipStream_t st) {
    const int64_t n16 = (int64_t)((bytes + 15) / 16);
    if (n16 == 0) return hipSuccess;
    const unsigned grid = (unsigned)std::min<int64_t>((n16 + 1023) / 1024, 64);
    k_upload<<<grid, 256, 0, st>>>((uint4*)dst, (const uint4*)src, n16);
    return hipGetLastError();
}

// The next pinned staging buffer of the area, at least `bytes` long (rounded
// up to 16-byte words), once the upload last made from it has completed.
pe_status_t staging_buffer(Area& A, size_t bytes, int& k) {
    k = A.next;
    A.next ^= 1;
    if (A.done[k]) PE_HIP(hipEventSynchronize(A.done[k]));
    else PE_HIP(hipEventCreateWithFlags(&A.done[k], hipEventDisableTiming));
    if (A.host_cap[k] < bytes + 16) {
        if (A.host[k]) PE_HIP(hipHostFree(A.host[k]));
        A.host[k] = nullptr;
        A.host_cap[k] = 0;
        const size_t cap = align_up(std::max<size_t>(bytes + bytes / 2, 1 << 14), 256);
        PE_HIP(hipHostMalloc((void**)&A.host[k], cap, hipHostMallocDefault));
        A.host_cap[k] = cap;
        PE_HIP(hipHostGetDevicePointer((void**)&A.host_dev[k], A.host[k], 0));
    }
    return PE_OK;
}

size_t loglike_scratch_bytes(int ne) { return sizeof(int64_t) * kQueues * (ne + 1); }

double redo_budget_setting() { return g_redo_budget; }

pe_status_t upload_area(Area& A, int ne, int64_t total, int64_t total2, const void* args, size_t arg_bytes,
                        const std::vector<int64_t>& off, const std::vector<int64_t>* off2, size_t scratch_bytes,
                        hipStream_t st, BatchPtrs& out) {
    // a fixed area keeps one layout (sized for layout_ne records of
    // layout_rec bytes) so that its pointers never move
    const int lne = A.fixed ? A.layout_ne : ne;
    const size_t lab = A.fixed ? A.layout_rec * (size_t)A.layout_ne : arg_bytes;
    if (A.fixed && (ne > A.layout_ne || arg_bytes > lab))
        return fail(PE_ERR_BUDGET, "batch exceeds the area's fixed capacity");
    const size_t o_args = 256;
    const size_t o_off = align_up(o_args + lab, 256);
    const size_t o_off2 = align_up(o_off + sizeof(int64_t) * (lne + 1), 256);
    const size_t o_scr = align_up(o_off2 + sizeof(int64_t) * (lne + 1), 256);
    const size_t need = o_scr + std::max<size_t>(scratch_bytes, 256);
    if (need > A.cap) {
        if (A.fixed) return fail(PE_ERR_BUDGET, "batch exceeds the area's fixed capacity");
        PE_HIP(hipDeviceSynchronize());  // earlier batches may still read the old buffer
        dfree_bytes(A.dev);
        A.cap = 0;
        A.shadow.clear();
        const size_t cap = std::max<size_t>(need + need / 2, 1 << 16);
        pe_status_t s = dalloc_bytes(&A.dev, cap);
        if (s != PE_OK) return s;
        A.cap = cap;
    }
    std::vector<char> img(o_scr, 0);
    BatchHdr h = {};
    h.ne = ne;
    h.total = total;
    h.redo_budget = g_redo_budget;
    h.total2 = total2;
    std::memcpy(img.data(), &h, sizeof(h));
    if (arg_bytes) std::memcpy(img.data() + o_args, args, arg_bytes);
    std::memcpy(img.data() + o_off, off.data(), sizeof(int64_t) * (ne + 1));
    if (off2) std::memcpy(img.data() + o_off2, off2->data(), sizeof(int64_t) * (ne + 1));
    if (A.fixed || img != A.shadow) {
        int k;
        pe_status_t s = staging_buffer(A, img.size(), k);
        if (s != PE_OK) return s;
        std::memcpy(A.host[k], img.data(), img.size());
        const char* src = A.host_dev[k];
        // the image's parts start on 256-byte offsets; whole 16-byte words are
        // copied (the staging buffer and the area extend past each part)
        if (A.fixed) {
            // only the used parts
            PE_HIP(upload_bytes(A.dev, src, o_args + arg_bytes, st));
            PE_HIP(upload_bytes(A.dev + o_off, src + o_off, sizeof(int64_t) * (ne + 1), st));
            if (off2) PE_HIP(upload_bytes(A.dev + o_off2, src + o_off2, sizeof(int64_t) * (ne + 1), st));
        } else {
            PE_HIP(upload_bytes(A.dev, src, img.size(), st));
            A.shadow.swap(img);
        }
        PE_HIP(hipEventRecord(A.done[k], st));
    }
    out.hdr = (BatchHdr*)A.dev;
    out.args = A.dev + o_args;
    out.off = (int64_t*)(A.dev + o_off);
    out.off2 = (int64_t*)(A.dev + o_off2);
    out.scratch = (double*)(A.dev + o_scr);
    return PE_OK;
}

// Bytes of a fixed area for ne records of rec bytes and the given scratch.
size_t fixed_area_bytes(int ne, size_t rec, size_t scratch_bytes) { return area_bytes(ne, rec * (size_t)ne, scratch_bytes); }

// ------------------------------------------------------------ stage runners
PrepArg prep_arg(const pe_event_s* ev, const void* data, const void* psd) {
    PrepArg a;
    std::memset(&a, 0, sizeof(a));
    a.ec = ev->ec;
    a.data = data;
    a.psd = psd;
    a.data_f32 = ev->desc.data_dtype == PE_C64;
    a.psd_f32 = ev->desc.psd_dtype == PE_F32;
    a.rec32 = ev->rec32;
    a.rec64 = ev->rec64;
    a.pw = ev->pw;
    a.pfx = ev->pfx;
    a.pl1 = ev->pl1;
    a.pw2 = ev->pw2;
    a.ppw = ev->ppw;
    a.seg = ev->mws + kMwsScan;
    a.guard = ev->guard;
    a.status = ev->status;
    return a;
}

pe_status_t run_prep(const std::vector<PrepArg>& all, hipStream_t st) {
    for (int cls = 0; cls < 4; ++cls) {
        std::vector<PrepArg> v;
        for (const PrepArg& a : all)
            if (a.data_f32 * 2 + a.psd_f32 == cls) v.push_back(a);
        if (v.empty()) continue;
        const int ne = (int)v.size();
        std::vector<int64_t> off(ne + 1, 0);
        int max_seg = 1, max_det = 1;  // the scan grid: the batch's most segments and detectors
        for (int e = 0; e < ne; ++e) {
            off[e + 1] = off[e] + blocks256(v[e].ec.K + kTabPad);
            const int64_t K = v[e].ec.K;
            const int64_t seg = std::max<int64_t>(1024, (K + kScanSeg - 1) / kScanSeg);
            max_seg = std::max(max_seg, (int)((K + seg - 1) / seg));
            max_det = std::max(max_det, (int)v[e].ec.n_det);
        }
        Area& A = area_for(st, kAreaPrep);
        std::lock_guard<std::mutex> lk(A.mu);
        BatchPtrs b;
        pe_status_t s = upload_area(A, ne, off[ne], 0, v.data(), sizeof(PrepArg) * ne, off, nullptr, 0, st, b);
        if (s != PE_OK) return s;
        PE_HIP(launch_prep_batch(b, ne, off[ne], cls >> 1, cls & 1, max_seg, max_det, st));
    }
    return PE_OK;
}

MetricArg metric_arg(const pe_event_s* ev, const double* theta0, const double* steps, int flags, double* g) {
    MetricArg a;
    std::memset(&a, 0, sizeof(a));
    a.ec = ev->ec;
    a.tab = ev->rec64;
    a.pw = ev->pw;
    a.mws = ev->mws;
    a.theta0 = theta0;
    a.steps = steps;
    a.g = g;
    a.flags = flags;
    return a;
}

pe_status_t run_metric(const std::vector<MetricArg>& v, hipStream_t st) {
    const int ne = (int)v.size();
    if (ne == 0) return PE_OK;
    std::vector<int64_t> off(ne + 1, 0);
    for (int e = 0; e < ne; ++e) off[e + 1] = off[e] + metric_blocks(v[e].ec.K);
    Area& A = area_for(st, kAreaMetric);
    std::lock_guard<std::mutex> lk(A.mu);
    BatchPtrs b;
    pe_status_t s = upload_area(A, ne, off[ne], 0, v.data(), sizeof(MetricArg) * ne, off, nullptr, 0, st, b);
    if (s != PE_OK) return s;
    PE_HIP(launch_metric_batch(b, ne, off[ne], st));
    return PE_OK;
}

DrawArg draw_arg(const pe_event_s* ev, const double* theta0, const double* g, uint64_t seed, uint32_t stream_id,
                 int64_t n, double* theta, double* logq, double* logprior) {
    DrawArg a;
    std::memset(&a, 0, sizeof(a));
    a.ec = ev->ec;
    a.theta0 = theta0;
    a.g = g;
    a.chol = ev->mws + kMwsChol;
    a.status = ev->status;
    a.seed = seed;
    a.stream_id = stream_id;
    a.n = n;
    a.theta = theta;
    a.logq = logq;
    a.logprior = logprior;
    return a;
}

pe_status_t run_draw(const std::vector<DrawArg>& v, hipStream_t st, bool ext) {
    const int ne = (int)v.size();
    if (ne == 0) return PE_OK;
    std::vector<int64_t> off(ne + 1, 0);
    for (int e = 0; e < ne; ++e) off[e + 1] = off[e] + blocks256(v[e].n);
    Area& A = area_for(st, kAreaDraw);
    std::lock_guard<std::mutex> lk(A.mu);
    BatchPtrs b;
    pe_status_t s = upload_area(A, ne, off[ne], 0, v.data(), sizeof(DrawArg) * ne, off, nullptr, 0, st, b);
    if (s != PE_OK) return s;
    PE_HIP(launch_draw_batch(b, ne, off[ne], st, ext));
    return PE_OK;
}

EvDev loglike_arg(const pe_event_s* ev, const double* theta, int64_t n, double* loglike, double* aux) {
    EvDev d;
    std::memset(&d, 0, sizeof(d));
    d.ec = ev->ec;
    d.rec32 = ev->rec32;
    d.rec64 = ev->rec64;
    d.pfx = ev->pfx;
    d.pl1 = ev->pl1;
    d.pw2 = ev->pw2;
    d.ppw = ev->ppw;
    d.guard = ev->guard;
    d.kc_all = ev->kc_all;
    d.hist = ev->hist;
    d.idx = ev->idx;
    d.kcut = ev->kcut;
    d.coef = ev->coef;
    d.resp = ev->resp;
    d.hh = ev->hh;
    d.partial = ev->partial;
    d.plan = ev->plan;
    d.rflag = ev->rflag;
    d.rcnt = ev->rcnt;
    d.rpos = ev->rpos;
    d.zd = ev->zd;
    d.status = ev->status;
    // Row stride and group cap follow from n alone (the workspace holds at
    // least this much), so a batch's plan does not depend on how large the
    // event's workspace happens to be.
    const int64_t np = std::max<int64_t>(npad_for(n), kTile);
    d.npad = np;
    int64_t mg = groups_cap(np, ev->desc.n_bins);
    if (g_chunks > 0 && mg > g_chunks) mg = g_chunks;
    d.max_groups = (int)mg;
    d.items_target = g_items_target;
    d.min_group_bins = g_min_group_bins;
    d.tile_lo = 0;
    d.tile_hi = INT_MAX;
    d.flags = kLlPrologue | kLlFinalize;
    d.theta = theta;
    d.n = n;
    d.loglike = loglike;
    d.aux = aux;
    return d;
}

pe_status_t run_loglike(const std::vector<EvDev>& v, int precision, hipStream_t st) {
    const int ne = (int)v.size();
    if (ne == 0) return PE_OK;
    std::vector<int64_t> poff(ne + 1, 0), foff(ne + 1, 0);
    bool any_dist = false;
    int max_det = 0;
    for (int e = 0; e < ne; ++e) {
        poff[e + 1] = poff[e] + ((v[e].flags & kLlPrologue) ? blocks256(v[e].n) : 0);
        foff[e + 1] = foff[e] + ((v[e].flags & kLlFinalize) ? blocks256(v[e].n) : 0);
        any_dist = any_dist || v[e].ec.dist;
        max_det = std::max(max_det, v[e].ec.n_det);
    }
    Area& A = area_for(st, kAreaLoglike);
    std::lock_guard<std::mutex> lk(A.mu);
    BatchPtrs b;
    pe_status_t s = upload_area(A, ne, poff[ne], foff[ne], v.data(), sizeof(EvDev) * ne, poff, &foff,
                                loglike_scratch_bytes(ne), st, b);
    if (s != PE_OK) return s;
    PE_HIP(launch_loglike_batch(b, ne, poff[ne], foff[ne], precision, true, any_dist, max_det, st));
    return PE_OK;
}

// A moment-path batch (events of one moment count P): prologue, the hot loop
// writing block moments, and the tc nodes from the moments.
pe_status_t run_loglike_moments(const std::vector<EvDev>& v, int P, hipStream_t st) {
    const int ne = (int)v.size();
    if (ne == 0) return PE_OK;
    std::vector<int64_t> poff(ne + 1, 0), foff(ne + 1, 0);
    for (int e = 0; e < ne; ++e) {
        poff[e + 1] = poff[e] + blocks256(v[e].n);
        foff[e + 1] = foff[e] + blocks256(v[e].n);
    }
    Area& A = area_for(st, kAreaLoglike);
    std::lock_guard<std::mutex> lk(A.mu);
    BatchPtrs b;
    pe_status_t s = upload_area(A, ne, poff[ne], foff[ne], v.data(), sizeof(EvDev) * ne, poff, &foff,
                                loglike_scratch_bytes(ne), st, b);
    if (s != PE_OK) return s;
    PE_HIP(launch_loglike_moments(b, ne, poff[ne], foff[ne], P, st));
    return PE_OK;
}

// The log-likelihood batch entry of an event's n draws (its workspace grown
// as needed). A time-marginalised event on the block-moment path evaluates its
// draws once, at the window's centre, in the moment batch; off it, every tc
// node is a draw (expanded into the workspace by run_jobs), evaluated in the
// main batch and summed by the node reduction.
pe_status_t loglike_entry(pe_event_s* ev, const double* theta, int64_t n, double* loglike, double* aux,
                          int precision, LlJobs& jobs) {
    pe_status_t s = ensure_ws(ev, ws_draws(ev, n, precision));
    if (s != PE_OK) return s;
    if (!ev->desc.time_marg) {
        jobs.main.push_back(loglike_arg(ev, theta, n, loglike, aux));
        return PE_OK;
    }
    if (tm_moments(ev, precision)) {
        if ((s = ensure_moments(ev, n)) != PE_OK) return s;
        jobs.tm.push_back(TmJob{ev, theta, n, loglike, true});
        EvDev d = loglike_arg(ev, ev->tm_theta, n, loglike, nullptr);
        d.flags |= kLlMoments;
        d.tm_mom = (double2*)ev->tm_mem;
        d.tm_pow = (const float*)ev->tm_pow;
        jobs.mom.push_back(d);
        return PE_OK;
    }
    jobs.tm.push_back(TmJob{ev, theta, n, loglike, false});
    jobs.main.push_back(loglike_arg(ev, ev->tm_theta, n * ev->desc.tm_points, ev->tm_ll, nullptr));
    return PE_OK;
}

pe_status_t run_jobs(const LlJobs& jobs, int precision, hipStream_t st) {
    for (const TmJob& j : jobs.tm) {
        if (j.moments)
            PE_HIP(launch_tm_centre(j.theta, j.n, j.ev->ec, j.ev->tm_theta, st));
        else
            PE_HIP(launch_tm_expand(j.theta, j.n, j.ev->ec, j.ev->tm_theta, st));
    }
    pe_status_t s = run_loglike(jobs.main, precision, st);
    for (int P : {8, 16}) {
        std::vector<EvDev> vp;
        for (const EvDev& d : jobs.mom)
            if (d.ec.tm_P == P) vp.push_back(d);
        if (s == PE_OK) s = run_loglike_moments(vp, P, st);
    }
    if (s != PE_OK) return s;
    for (const TmJob& j : jobs.tm)
        if (!j.moments) PE_HIP(launch_tm_reduce(j.ev->tm_ll, j.n, j.ev->ec, j.loglike, st));
    return PE_OK;
}

pe_status_t run_weights(const std::vector<WeightArg>& v, hipStream_t st) {
    const int ne = (int)v.size();
    if (ne == 0) return PE_OK;
    std::vector<int64_t> boff(ne + 1, 0), doff(ne + 1, 0);
    for (int e = 0; e < ne; ++e) {
        boff[e + 1] = boff[e] + (v[e].n + kWBlock - 1) / kWBlock;
        doff[e + 1] = doff[e] + blocks256(v[e].n);
    }
    Area& A = area_for(st, kAreaWeights);
    std::lock_guard<std::mutex> lk(A.mu);
    BatchPtrs b;
    const size_t scratch = sizeof(double4) * std::max<int64_t>(boff[ne], 1) + sizeof(double2) * ne;
    pe_status_t s =
        upload_area(A, ne, boff[ne], doff[ne], v.data(), sizeof(WeightArg) * ne, boff, &doff, scratch, st, b);
    if (s != PE_OK) return s;
    PE_HIP(launch_weights_batch(b, ne, boff[ne], doff[ne], st));
    return PE_OK;
}

pe_status_t run_update(const std::vector<UpdateArg>& v, hipStream_t st) {
    const int ne = (int)v.size();
    if (ne == 0) return PE_OK;
    std::vector<int64_t> boff(ne + 1, 0);
    for (int e = 0; e < ne; ++e) boff[e + 1] = boff[e] + (v[e].n + kWBlock - 1) / kWBlock;
    Area& A = area_for(st, kAreaUpdate);
    std::lock_guard<std::mutex> lk(A.mu);
    BatchPtrs b;
    const size_t scratch = sizeof(double) * kUpdNQ * std::max<int64_t>(boff[ne], 1);
    pe_status_t s = upload_area(A, ne, boff[ne], 0, v.data(), sizeof(UpdateArg) * ne, boff, nullptr, scratch, st, b);
    if (s != PE_OK) return s;
    PE_HIP(launch_update_batch(b, ne, boff[ne], st));
    return PE_OK;
}

int chunks_setting() { return g_chunks; }

// ------------------------------------------------------------------ profiling
std::mutex g_prof_mu;
bool g_prof_on = false;
std::map<std::string, std::vector<std::pair<hipEvent_t, hipEvent_t>>> g_prof;
std::map<std::string, hipEvent_t> g_prof_open;

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

// ------------------------------------------------ allocation-free weights
// pe_weights_ess_noalloc keeps its batch header, argument record, offsets and
// per-block partial sums in the file-scope device array `scratch` (one copy
// per GPU, held until the process ends). Host code never hands the array's
// name to a kernel or a copy: it uses the device address that
// hipGetSymbolAddress returns, taken once per device (with that device
// current) on the entry point's first call there.
constexpr int64_t kNoAllocMaxDraws = (int64_t)1 << 24;
constexpr size_t kNoAllocArgs = 256, kNoAllocOff = 512, kNoAllocOff2 = 768, kNoAllocPart = 1024;
constexpr size_t kNoAllocBytes =
    kNoAllocPart + sizeof(double4) * (size_t)(kNoAllocMaxDraws / kWBlock) + sizeof(double2) + 256;
static_assert(sizeof(BatchHdr) <= kNoAllocArgs, "batch header fits its slot");
static_assert(kNoAllocArgs + sizeof(WeightArg) <= kNoAllocOff, "argument record fits its slot");

static __device__ __align__(256) char scratch[kNoAllocBytes];

constexpr int kNoAllocDevices = 64;
std::mutex g_noalloc_mu;
char* g_noalloc_ptr[kNoAllocDevices] = {};

// The current device's address of `scratch`.
pe_status_t noalloc_scratch(char** out) {
    int dev = 0;
    PE_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kNoAllocDevices) return fail(PE_ERR_ARG, "device index beyond the supported 64");
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (!g_noalloc_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(PE_ERR_HIP, std::string("address of the allocation-free scratch: ") + hipGetErrorString(e));
        g_noalloc_ptr[dev] = (char*)p;
    }
    *out = g_noalloc_ptr[dev];
    return PE_OK;
}

// Writes the one-event batch of the weights stage into the scratch: header,
// argument record (passed by value) and the two offset arrays.
__global__ void k_noalloc_weights_area(char* __restrict__ base, WeightArg a, int64_t nb, int64_t nd) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    BatchHdr h = {};
    h.ne = 1;
    h.total = nb;
    h.total2 = nd;
    *(BatchHdr*)base = h;
    *(WeightArg*)(base + kNoAllocArgs) = a;
    int64_t* o = (int64_t*)(base + kNoAllocOff);
    o[0] = 0;
    o[1] = nb;
    int64_t* o2 = (int64_t*)(base + kNoAllocOff2);
    o2[0] = 0;
    o2[1] = nd;
}

pe_status_t check_n(int64_t n) {
    if (n < 0 || n > ((int64_t)1 << 30)) return fail(PE_ERR_ARG, "n must be in 0..2^30");
    return PE_OK;
}

pe_status_t check_precision(int32_t precision) {
    if (precision != PE_PREC_FP64 && precision != PE_PREC_SPLIT) return fail(PE_ERR_ARG, "bad precision");
    return PE_OK;
}

}  // namespace pe

using namespace pe;

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
    pe_event_s* ev = nullptr;
    if ((s = new_event(desc, nullptr, 0, &ev)) != PE_OK) return s;
    hipStream_t st = as_stream(stream);
    hipError_t e = hipMemsetAsync(ev->tab_mem, 0, tables_bytes(*desc), st);
    if (e != hipSuccess) {
        free_event(ev);
        return fail(PE_ERR_HIP, std::string("event preparation: ") + hipGetErrorString(e));
    }
    s = run_prep(std::vector<PrepArg>(1, prep_arg(ev, data_dev, psd_dev)), st);
    if (s == PE_OK) s = pe_event_status(ev, stream);
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
    return run_prep(std::vector<PrepArg>(1, prep_arg(ev, data_dev, psd_dev)), as_stream(stream));
}

pe_status_t pe_event_status(pe_event_t ev, void* stream) {
    if (!ev) return fail(PE_ERR_ARG, "event is NULL");
    hipStream_t st = as_stream(stream);
    PE_HIP(hipStreamSynchronize(st));
    int flags = 0;
    PE_HIP(hipMemcpy(&flags, ev->status, sizeof(int), hipMemcpyDeviceToHost));
    if (flags) PE_HIP(hipMemset(ev->status, 0, sizeof(int)));
    if (flags & kStBadPsd) return fail(PE_ERR_ARG, "PSD values must be positive and finite");
    if (flags & kStNonfinite) return fail(PE_ERR_NONFINITE, "data contains inf or nan");
    if (flags & kStSingular) return fail(PE_ERR_SINGULAR, "metric is not positive definite");
    return PE_OK;
}

pe_status_t pe_event_reserve(pe_event_t ev, int64_t max_draws) {
    if (!ev) return fail(PE_ERR_ARG, "event is NULL");
    if (max_draws < 0 || max_draws > ((int64_t)1 << 30)) return fail(PE_ERR_ARG, "max_draws must be in 0..2^30");
    pe_status_t s = ensure_ws(ev, ws_draws(ev, max_draws, PE_PREC_SPLIT));
    if (s == PE_OK && tm_moments(ev, PE_PREC_SPLIT) && max_draws > 0) s = ensure_moments(ev, max_draws);
    return s;
}

pe_status_t pe_event_destroy(pe_event_t ev) {
    if (!ev) return fail(PE_ERR_ARG, "event is NULL");
    if (!ev->own_mem) return fail(PE_ERR_ARG, "the event belongs to a server");
    (void)hipDeviceSynchronize();
    free_event(ev);
    return PE_OK;
}

pe_status_t pe_metric(pe_event_t ev, const double* theta0_dev, const double* fd_step_dev, int32_t flags,
                      double* g_dev, void* stream) {
    if (!ev) return fail(PE_ERR_ARG, "event is NULL");
    if (!theta0_dev || !g_dev) return fail(PE_ERR_ARG, "theta0 and g must be device pointers");
    if (flags & ~1) return fail(PE_ERR_ARG, "unknown metric flags");
    return run_metric(std::vector<MetricArg>(1, metric_arg(ev, theta0_dev, fd_step_dev, flags, g_dev)),
                      as_stream(stream));
}

pe_status_t pe_draw(pe_event_t ev, const double* theta0_dev, const double* g_dev, uint64_t seed, uint32_t stream_id,
                    int64_t n, double* theta_dev, double* logq_dev, double* logprior_dev, void* stream) {
    if (!ev) return fail(PE_ERR_ARG, "event is NULL");
    pe_status_t s = check_n(n);
    if (s != PE_OK) return s;
    if (!theta0_dev || !g_dev) return fail(PE_ERR_ARG, "theta0 and g must be device pointers");
    if (n > 0 && (!theta_dev || !logq_dev || !logprior_dev)) return fail(PE_ERR_ARG, "output pointers are NULL");
    return run_draw(std::vector<DrawArg>(1, draw_arg(ev, theta0_dev, g_dev, seed, stream_id, n, theta_dev, logq_dev,
                                                     logprior_dev)),
                    as_stream(stream));
}

pe_status_t pe_mixture_logq(pe_event_t ev, int32_t m, const double* weights, const double* theta0_dev,
                            const double* g_dev, const double* theta_dev, int64_t n, double* logq_dev, void* stream) {
    if (!ev) return fail(PE_ERR_ARG, "event is NULL");
    if (m < 1 || m > PE_MIX_MAX) return fail(PE_ERR_ARG, "m must be in 1..PE_MIX_MAX");
    if (!weights) return fail(PE_ERR_ARG, "weights is NULL (a host array of m values)");
    double wsum = 0.0;
    for (int k = 0; k < m; ++k) {
        if (!std::isfinite(weights[k]) || weights[k] < 0.0) return fail(PE_ERR_ARG, "weights must be finite and >= 0");
        wsum += weights[k];
    }
    if (!(wsum > 0.0) || !std::isfinite(wsum)) return fail(PE_ERR_ARG, "weights must have a positive finite sum");
    pe_status_t s = check_n(n);
    if (s != PE_OK) return s;
    if (!theta0_dev || !g_dev) return fail(PE_ERR_ARG, "theta0 and g must be device pointers");
    if (n > 0 && (!theta_dev || !logq_dev)) return fail(PE_ERR_ARG, "theta and logq are NULL");
    if (n == 0) return PE_OK;
    hipStream_t st = as_stream(stream);
    const int D = ev->ec.dim;
    // the components' factors: k_cholesky's records, as pe_draw makes them
    std::vector<DrawArg> v;
    for (int k = 0; k < m; ++k) {
        DrawArg a = draw_arg(ev, theta0_dev + (int64_t)k * D, g_dev + (int64_t)k * D * D, 0, 0, 0, nullptr, nullptr,
                             nullptr);
        a.chol = ev->mix_chol + (int64_t)k * kCholLen;
        v.push_back(a);
    }
    if ((s = run_draw(v, st)) != PE_OK) return s;
    MixArg a;
    std::memset(&a, 0, sizeof(a));
    a.ec = ev->ec;
    a.chol = ev->mix_chol;
    a.theta0 = theta0_dev;
    a.theta = theta_dev;
    a.logq = logq_dev;
    a.status = ev->status;
    a.n = n;
    a.m = m;
    for (int k = 0; k < m; ++k) a.lpi[k] = weights[k] > 0.0 ? std::log(weights[k] / wsum) : -INFINITY;
    PE_HIP(launch_mix_logq(a, st));
    return PE_OK;
}

pe_status_t pe_tile_extrinsic(pe_event_t ev, const double* theta0_dev, const double* g_dev, uint32_t sub_mask,
                              int32_t flags, uint64_t seed, uint32_t stream_id, int64_t n, double* theta_dev,
                              double* logq_dev, double* logprior_dev, void* stream) {
    if (!ev) return fail(PE_ERR_ARG, "event is NULL");
    if (ev->ec.dim != 11) return fail(PE_ERR_ARG, "the extrinsic completion takes an 11-D event");
    constexpr uint32_t periodic = (1u << 4) | (1u << 7) | (1u << 10);
    if (sub_mask == 0 || (sub_mask >> 11) != 0 || (sub_mask & periodic) != 0)
        return fail(PE_ERR_ARG, "sub_mask must be nonzero, below bit 11 and without ra, psi, phic");
    if (flags & ~PE_TILE_CONDITIONAL) return fail(PE_ERR_ARG, "unknown flags");
    const bool cond = (flags & PE_TILE_CONDITIONAL) != 0;
    const uint32_t marg = (ev->ec.dist ? 1u << 8 : 0u) | (ev->ec.tm ? 1u << 9 : 0u);
    if (cond && (sub_mask & marg) != 0)
        return fail(PE_ERR_ARG, "a conditional completion cannot condition on a marginalised coordinate");
    pe_status_t s = check_n(n);
    if (s != PE_OK) return s;
    if (!theta0_dev || !g_dev) return fail(PE_ERR_ARG, "theta0 and g must be device pointers");
    if (n > 0 && (!theta_dev || !logq_dev || !logprior_dev)) return fail(PE_ERR_ARG, "draw arrays are NULL");
    if (n == 0) return PE_OK;
    DrawArg a = draw_arg(ev, theta0_dev, g_dev, seed, stream_id, n, theta_dev, logq_dev, logprior_dev);
    a.dmask = sub_mask | (cond ? kDrawCond : 0u);
    return run_draw(std::vector<DrawArg>(1, a), as_stream(stream), true);
}

pe_status_t pe_loglike_batch(pe_event_t ev, const double* theta_dev, int64_t n, int32_t precision,
                             double* loglike_dev, double* aux_dev, void* stream) {
    if (!ev) return fail(PE_ERR_ARG, "event is NULL");
    if (precision == PE_PREC_RELBIN) {
        pe_status_t s = check_n(n);
        if (s != PE_OK) return s;
        if (n == 0) return PE_OK;
        if (!theta_dev || !loglike_dev) return fail(PE_ERR_ARG, "theta and loglike must be device pointers");
        if (ev->desc.time_marg) return fail(PE_ERR_ARG, "relative binning does not take a time-marginalised event");
        return run_relbin(ev, theta_dev, n, loglike_dev, aux_dev, as_stream(stream));
    }
    pe_status_t s = check_n(n);
    if (s == PE_OK) s = check_precision(precision);
    if (s != PE_OK) return s;
    if (n == 0) return PE_OK;
    if (!theta_dev || !loglike_dev) return fail(PE_ERR_ARG, "theta and loglike must be device pointers");
    if (ev->desc.time_marg && aux_dev) return fail(PE_ERR_ARG, "aux is not available for a time-marginalised event");
    LlJobs jobs;
    if ((s = loglike_entry(ev, theta_dev, n, loglike_dev, aux_dev, precision, jobs)) != PE_OK) return s;
    return run_jobs(jobs, precision, as_stream(stream));
}

pe_status_t pe_loglike_multi(int32_t n_events, const pe_event_t* events, const double* const* theta_dev,
                             const int64_t* n, int32_t precision, double* const* loglike_dev,
                             double* const* aux_dev, void* stream) {
    if (n_events < 0 || n_events > 65535 || (n_events > 0 && (!events || !theta_dev || !n || !loglike_dev)))
        return fail(PE_ERR_ARG, "bad batch arrays (n_events must be in 0..65535)");
    pe_status_t s = check_precision(precision);
    if (s != PE_OK) return s;
    LlJobs jobs;
    for (int e = 0; e < n_events; ++e) {
        pe_event_s* ev = events[e];
        if (!ev) return fail(PE_ERR_ARG, "event is NULL");
        for (int f = 0; f < e; ++f)
            if (events[f] == ev) return fail(PE_ERR_ARG, "an event appears twice in the batch");
        if ((s = check_n(n[e])) != PE_OK) return s;
        if (n[e] == 0) continue;
        if (!theta_dev[e] || !loglike_dev[e]) return fail(PE_ERR_ARG, "theta and loglike must be device pointers");
        if (ev->desc.time_marg && aux_dev && aux_dev[e])
            return fail(PE_ERR_ARG, "aux is not available for a time-marginalised event");
        if ((s = loglike_entry(ev, theta_dev[e], n[e], loglike_dev[e], aux_dev ? aux_dev[e] : nullptr, precision,
                               jobs)) != PE_OK)
            return s;
    }
    return run_jobs(jobs, precision, as_stream(stream));
}

pe_status_t pe_batch_run(int32_t n_items, const pe_batch_item_t* items, int32_t stages, int32_t precision,
                         void* stream) {
    if (n_items < 0 || n_items > 65535 || (n_items > 0 && !items))
        return fail(PE_ERR_ARG, "bad items (n_items must be in 0..65535)");
    if (stages & ~PE_STAGE_ALL) return fail(PE_ERR_ARG, "unknown stages");
    pe_status_t s = check_precision(precision);
    if (s != PE_OK) return s;
    std::vector<PrepArg> vp;
    std::vector<MetricArg> vm;
    std::vector<DrawArg> vd;
    LlJobs jobs;
    std::vector<WeightArg> vw;
    for (int e = 0; e < n_items; ++e) {
        const pe_batch_item_t& it = items[e];
        pe_event_s* ev = it.ev;
        if (!ev) return fail(PE_ERR_ARG, "item " + std::to_string(e) + ": event is NULL");
        for (int f = 0; f < e; ++f)
            if (items[f].ev == ev) return fail(PE_ERR_ARG, "an event appears twice in the batch");
        if ((s = check_n(it.n)) != PE_OK) return s;
        if (stages & PE_STAGE_PREP) {
            if (!it.data || !it.psd) return fail(PE_ERR_ARG, "item " + std::to_string(e) + ": data and psd needed");
            vp.push_back(prep_arg(ev, it.data, it.psd));
        }
        if (stages & PE_STAGE_METRIC) {
            if (!it.theta0 || !it.g) return fail(PE_ERR_ARG, "item " + std::to_string(e) + ": theta0 and g needed");
            if (it.metric_flags & ~1) return fail(PE_ERR_ARG, "unknown metric flags");
            vm.push_back(metric_arg(ev, it.theta0, it.fd_step, it.metric_flags, it.g));
        }
        if (stages & PE_STAGE_DRAW) {
            if (!it.theta0 || !it.g || (it.n > 0 && (!it.theta || !it.logq || !it.logprior)))
                return fail(PE_ERR_ARG, "item " + std::to_string(e) + ": draw pointers needed");
            vd.push_back(draw_arg(ev, it.theta0, it.g, it.seed, it.stream_id, it.n, it.theta, it.logq, it.logprior));
        }
        if ((stages & PE_STAGE_LOGLIKE) && it.n > 0) {
            if (!it.theta || !it.loglike)
                return fail(PE_ERR_ARG, "item " + std::to_string(e) + ": theta and loglike needed");
            if (ev->desc.time_marg && it.aux)
                return fail(PE_ERR_ARG, "item " + std::to_string(e) + ": no aux for a time-marginalised event");
            if ((s = loglike_entry(ev, it.theta, it.n, it.loglike, it.aux, precision, jobs)) != PE_OK) return s;
        }
        if (stages & PE_STAGE_WEIGHTS) {
            if (!it.stats || (it.n > 0 && (!it.loglike || !it.logprior || !it.logq)))
                return fail(PE_ERR_ARG, "item " + std::to_string(e) + ": weight pointers needed");
            WeightArg w = {it.loglike, it.logprior, it.logq, it.n, it.w, it.stats};
            vw.push_back(w);
        }
    }
    hipStream_t st = as_stream(stream);
    if ((s = run_prep(vp, st)) != PE_OK) return s;
    if ((s = run_metric(vm, st)) != PE_OK) return s;
    if ((s = run_draw(vd, st)) != PE_OK) return s;
    if ((s = run_jobs(jobs, precision, st)) != PE_OK) return s;
    return run_weights(vw, st);
}

pe_status_t pe_weights_ess(const double* loglike_dev, const double* logprior_dev, const double* logq_dev, int64_t n,
                           double* w_dev, double* stats_dev, void* stream) {
    if (n < 0) return fail(PE_ERR_ARG, "n must be >= 0");
    if (!stats_dev) return fail(PE_ERR_ARG, "stats must be a device pointer");
    if (n > 0 && (!loglike_dev || !logprior_dev || !logq_dev)) return fail(PE_ERR_ARG, "inputs are NULL");
    WeightArg w = {loglike_dev, logprior_dev, logq_dev, n, w_dev, stats_dev};
    return run_weights(std::vector<WeightArg>(1, w), as_stream(stream));
}

pe_status_t pe_weights_ess_noalloc(const double* loglike_dev, const double* logprior_dev, const double* logq_dev,
                                   int64_t n, double* w_dev, double* stats_dev, void* stream) {
    if (n < 0) return fail(PE_ERR_ARG, "n must be >= 0");
    if (n > kNoAllocMaxDraws) return fail(PE_ERR_ARG, "n exceeds 2^24, the limit of the allocation-free scratch");
    if (!stats_dev) return fail(PE_ERR_ARG, "stats must be a device pointer");
    if (n > 0 && (!loglike_dev || !logprior_dev || !logq_dev)) return fail(PE_ERR_ARG, "inputs are NULL");
    char* base = nullptr;
    pe_status_t s = noalloc_scratch(&base);
    if (s != PE_OK) return s;
    const WeightArg a = {loglike_dev, logprior_dev, logq_dev, n, w_dev, stats_dev};
    const int64_t nb = (n + kWBlock - 1) / kWBlock, nd = blocks256(n);
    hipStream_t st = as_stream(stream);
    k_noalloc_weights_area<<<1, 64, 0, st>>>(base, a, nb, nd);
    PE_HIP(hipGetLastError());
    BatchPtrs b;
    b.hdr = (BatchHdr*)base;
    b.args = base + kNoAllocArgs;
    b.off = (int64_t*)(base + kNoAllocOff);
    b.off2 = (int64_t*)(base + kNoAllocOff2);
    b.scratch = (double*)(base + kNoAllocPart);
    PE_HIP(launch_weights_batch(b, 1, nb, nd, st));
    return PE_OK;
}

pe_status_t pe_proposal_update(pe_event_t ev, const double* theta_dev, const double* w_dev, int64_t n,
                               const double* theta0_dev, double* theta0_out_dev, double* cov_dev, void* stream) {
    if (!ev) return fail(PE_ERR_ARG, "event is NULL");
    pe_status_t s = check_n(n);
    if (s != PE_OK) return s;
    if (!theta0_dev || !theta0_out_dev) return fail(PE_ERR_ARG, "theta0 and theta0_out must be device pointers");
    if (n > 0 && (!theta_dev || !w_dev)) return fail(PE_ERR_ARG, "theta and w must be device pointers");
    UpdateArg a = {theta_dev, w_dev, n, theta0_dev, theta0_out_dev, cov_dev, ev->ec.dim, ev->ec.params};
    return run_update(std::vector<UpdateArg>(1, a), as_stream(stream));
}

pe_status_t pe_refine(pe_event_t ev, double* theta0_dev, double* g_dev, int32_t rounds, int64_t n, uint64_t seed,
                      int32_t precision, double* theta_dev, double* logq_dev, double* logprior_dev,
                      double* loglike_dev, double* w_dev, double* stats_dev, void* stream) {
    if (!ev) return fail(PE_ERR_ARG, "event is NULL");
    if (rounds < 1 || rounds > 64) return fail(PE_ERR_ARG, "rounds must be in 1..64");
    pe_status_t s = check_n(n);
    if (s == PE_OK) s = check_precision(precision);
    if (s != PE_OK) return s;
    if (n < 1) return fail(PE_ERR_ARG, "n must be >= 1");
    if (!theta0_dev || !g_dev || !theta_dev || !logq_dev || !logprior_dev || !loglike_dev || !w_dev || !stats_dev)
        return fail(PE_ERR_ARG, "every buffer must be a device pointer");
    for (int r = 0; r < rounds; ++r) {
        if ((s = pe_metric(ev, theta0_dev, nullptr, 0, g_dev, stream)) != PE_OK) return s;
        if ((s = pe_draw(ev, theta0_dev, g_dev, seed, (uint32_t)r, n, theta_dev, logq_dev, logprior_dev, stream)) !=
            PE_OK)
            return s;
        if ((s = pe_loglike_batch(ev, theta_dev, n, precision, loglike_dev, nullptr, stream)) != PE_OK) return s;
        if ((s = pe_weights_ess(loglike_dev, logprior_dev, logq_dev, n, w_dev, stats_dev + 4 * r, stream)) != PE_OK)
            return s;
        if ((s = pe_proposal_update(ev, theta_dev, w_dev, n, theta0_dev, theta0_dev, nullptr, stream)) != PE_OK)
            return s;
    }
    return pe_metric(ev, theta0_dev, nullptr, 0, g_dev, stream);
}

pe_status_t pe_waveform(const pe_event_desc_t* desc, const double* theta_dev, const void* psd_dev, double* h_dev,
                        double* snr2_dev, void* stream) {
    if (!desc) return fail(PE_ERR_ARG, "desc is NULL");
    pe_event_desc_t d2 = *desc;
    if (d2.params == PE_PARAMS_4D && !(d2.amp0 > 0.0)) d2.amp0 = 1.0;
    pe_status_t s = validate_desc(&d2);
    if (s != PE_OK) return s;
    if (!theta_dev || !h_dev) return fail(PE_ERR_ARG, "theta and h must be device pointers");
    if (snr2_dev && !psd_dev) return fail(PE_ERR_ARG, "snr2 needs the PSD");
    EvConst ec;
    build_const(*desc, ec);
    const int64_t nb = (ec.K + 255) / 256;
    char* scratch = nullptr;
    if ((s = dalloc_bytes(&scratch, sizeof(double) * (size_t)(32 + nb))) != PE_OK) return s;
    hipStream_t st = as_stream(stream);
    hipError_t e = launch_waveform(ec, desc->psd_dtype, theta_dev, psd_dev, h_dev, snr2_dev, (double*)scratch, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    dfree_bytes(scratch);
    if (e != hipSuccess) return fail(PE_ERR_HIP, std::string("waveform: ") + hipGetErrorString(e));
    return PE_OK;
}

pe_status_t pe_rng_uniforms(uint64_t seed, uint32_t stream_id, int64_t n, int32_t npairs, double* u_dev,
                            void* stream) {
    if (n < 0 || npairs < 0 || npairs > 64) return fail(PE_ERR_ARG, "bad n or npairs");
    if (n * npairs > 0 && !u_dev) return fail(PE_ERR_ARG, "u must be a device pointer");
    PE_HIP(launch_uniforms(seed, stream_id, n, npairs, u_dev, as_stream(stream)));
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

pe_status_t pe_set_plan(int32_t items_target, int32_t min_group_bins) {
    if (items_target < 256 || items_target > (1 << 20)) return fail(PE_ERR_ARG, "items_target must be in 256..2^20");
    if (min_group_bins < 32 || min_group_bins > (1 << 20)) return fail(PE_ERR_ARG, "min_group_bins must be in 32..2^20");
    g_items_target = items_target;
    g_min_group_bins = min_group_bins;
    return PE_OK;
}

pe_status_t pe_get_plan(int32_t* items_target, int32_t* min_group_bins) {
    if (!items_target || !min_group_bins) return fail(PE_ERR_ARG, "NULL argument");
    *items_target = g_items_target;
    *min_group_bins = g_min_group_bins;
    return PE_OK;
}

pe_status_t pe_autotune_plan(int32_t n_events, const pe_event_t* events, const double* const* theta_dev,
                             const int64_t* n, int32_t precision, int32_t reps, int32_t* best_items_target,
                             int32_t* best_min_group_bins, double* best_ms, void* stream) {
    if (!best_items_target || !best_min_group_bins || !best_ms) return fail(PE_ERR_ARG, "NULL output");
    if (reps < 1 || reps > 100) return fail(PE_ERR_ARG, "reps must be in 1..100");
    std::vector<double*> ll;
    std::vector<const double*> th;
    std::vector<pe_event_t> evv;
    std::vector<int64_t> nn;
    pe_status_t s = PE_OK;
    for (int e = 0; e < n_events && events && n; ++e) {
        if (n[e] <= 0) continue;
        char* p = nullptr;
        if ((s = dalloc_bytes(&p, sizeof(double) * (size_t)n[e])) != PE_OK) break;
        ll.push_back((double*)p);
        th.push_back(theta_dev[e]);
        evv.push_back(events[e]);
        nn.push_back(n[e]);
    }
    const int32_t keep_items = g_items_target, keep_bins = g_min_group_bins;
    hipStream_t st = as_stream(stream);
    hipEvent_t a = nullptr, b = nullptr;
    double best = 1e300;
    int32_t bi = keep_items, bb = keep_bins;
    if (s == PE_OK && (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess))
        s = fail(PE_ERR_HIP, "autotune events");
    const int32_t items[] = {4096, 8192, 16384, 32768, 65536};
    const int32_t bins[] = {256, 512, 1024, 2048, 4096};
    for (int32_t it : items) {
        for (int32_t bn : bins) {
            if (s != PE_OK) break;
            g_items_target = it;
            g_min_group_bins = bn;
            // one untimed run, then reps timed ones
            s = pe_loglike_multi((int32_t)evv.size(), evv.data(), th.data(), nn.data(), precision, ll.data(),
                                 nullptr, stream);
            if (s != PE_OK) break;
            if (hipEventRecord(a, st) != hipSuccess) s = fail(PE_ERR_HIP, "autotune record");
            for (int r = 0; r < reps && s == PE_OK; ++r)
                s = pe_loglike_multi((int32_t)evv.size(), evv.data(), th.data(), nn.data(), precision, ll.data(),
                                     nullptr, stream);
            float ms = 0.0f;
            if (s == PE_OK && (hipEventRecord(b, st) != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
                               hipEventElapsedTime(&ms, a, b) != hipSuccess))
                s = fail(PE_ERR_HIP, "autotune timing");
            if (s == PE_OK && ms / reps < best) {
                best = ms / reps;
                bi = it;
                bb = bn;
            }
        }
    }
    g_items_target = keep_items;
    g_min_group_bins = keep_bins;
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    (void)hipStreamSynchronize(st);
    for (double* p : ll) {
        char* c = (char*)p;
        dfree_bytes(c);
    }
    if (s != PE_OK) return s;
    *best_items_target = bi;
    *best_min_group_bins = bb;
    *best_ms = best;
    return PE_OK;
}

pe_status_t pe_set_split_guard(double budget) {
    if (!(budget >= 0.0)) return fail(PE_ERR_ARG, "budget must be >= 0 (inf: never re-evaluate)");
    g_redo_budget = budget;
    return PE_OK;
}

pe_status_t pe_get_split_guard(double* budget) {
    if (!budget) return fail(PE_ERR_ARG, "NULL argument");
    *budget = g_redo_budget;
    return PE_OK;
}

pe_status_t pe_loglike_counts(pe_event_t ev, int64_t out[2], void* stream) {
    if (!ev || !out) return fail(PE_ERR_ARG, "NULL argument");
    if (!ev->plan) {
        out[0] = out[1] = 0;
        return PE_OK;
    }
    EvPlan p[2];
    PE_HIP(hipStreamSynchronize(as_stream(stream)));
    PE_HIP(hipMemcpy(p, ev->plan, sizeof(p), hipMemcpyDeviceToHost));
    out[0] = p[0].n_active;
    out[1] = p[1].n_active;
    return PE_OK;
}

pe_status_t pe_set_chunks(int32_t n_chunks) {
    if (n_chunks < 0 || n_chunks > 64) return fail(PE_ERR_ARG, "n_chunks must be in 0..64");
    g_chunks = n_chunks;
    return PE_OK;
}

}  // extern "C"
