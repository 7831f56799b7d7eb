// pe_server.hip -- serving loop of the likelihood engine: requests admitted by
// device-memory budget into one slab, batched admission stages, hot-loop
// slices over one work queue shared by every active request (continuous
// batching), optional hipGraph replay of the slice.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <climits>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "pe_host.h"

namespace pe {
namespace {

constexpr int64_t kMaxServerDraws = (int64_t)1 << 22;

// First-fit allocator over one device slab in 256-byte granules; frees
// coalesce with their neighbours.
class Slab {
  public:
    pe_status_t init(size_t bytes) {
        cap_ = (bytes / 256) * 256;
        pe_status_t s = dalloc_bytes(&base_, cap_);
        if (s != PE_OK) return s;
        free_.clear();
        free_[0] = cap_;
        used_ = peak_ = 0;
        return PE_OK;
    }
    void release() {
        dfree_bytes(base_);
        free_.clear();
        cap_ = used_ = 0;
    }
    bool alloc(size_t bytes, size_t* off) {
        bytes = (bytes + 255) / 256 * 256;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const size_t rest = it->second - bytes;
            const size_t at = it->first + bytes;
            free_.erase(it);
            if (rest) free_[at] = rest;
            used_ += bytes;
            peak_ = std::max(peak_, used_);
            return true;
        }
        return false;
    }
    void free(size_t off, size_t bytes) {
        bytes = (bytes + 255) / 256 * 256;
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    char* base() const { return base_; }
    size_t capacity() const { return cap_; }
    size_t peak() const { return peak_; }

  private:
    char* base_ = nullptr;
    size_t cap_ = 0, used_ = 0, peak_ = 0;
    std::map<size_t, size_t> free_;
};

struct Req {
    int64_t ticket = 0;
    pe_request_t r;
    std::vector<double> theta0;
    int D = 0;
    size_t bytes = 0, off = 0;
    pe_event_s* ev = nullptr;
    double *d_theta0 = nullptr, *d_g = nullptr, *d_theta = nullptr, *d_logq = nullptr, *d_logprior = nullptr;
    double *d_loglike = nullptr, *d_w = nullptr, *d_stats = nullptr;
    void *d_data = nullptr, *d_psd = nullptr;
    EvPlan plan = {};
    int tiles_done = 0;
    double tile_ops = 0.0;  // lane-operations of one tile (cost model)
    pe_result_t res = {};
};

size_t elem_data(const pe_event_desc_t& d) { return d.data_dtype == PE_C64 ? 8 : 16; }
size_t elem_psd(const pe_event_desc_t& d) { return d.psd_dtype == PE_F32 ? 4 : 8; }

// Per-request buffers after the event's own range.
size_t request_buffers(Req* q, char* base) {
    Carver c(base);
    const int64_t n = q->r.n_draws;
    const int D = q->D;
    const pe_event_desc_t& d = q->r.desc;
    q->d_theta0 = c.take<double>(D);
    q->d_g = c.take<double>((size_t)D * D);
    q->d_theta = c.take<double>((size_t)D * n);
    q->d_logq = c.take<double>(n);
    q->d_logprior = c.take<double>(n);
    q->d_loglike = c.take<double>(n);
    q->d_w = c.take<double>(n);
    q->d_stats = c.take<double>(4);
    if (q->r.data_on_host) {
        q->d_data = c.take<char>((size_t)d.n_det * d.n_bins * elem_data(d));
        q->d_psd = c.take<char>((size_t)d.n_det * d.n_bins * elem_psd(d));
    }
    return c.size();
}

// Shape bucket of a request for the plan table: detector count and the
// number of bins rounded up to a power of two.
struct Bucket {
    int n_det, log2k;
    bool operator<(const Bucket& o) const { return n_det != o.n_det ? n_det < o.n_det : log2k < o.log2k; }
};

Bucket bucket_of(const pe_event_desc_t& d) {
    int l = 0;
    while (l < 40 && ((int64_t)1 << l) < d.n_bins) ++l;
    return Bucket{d.n_det, l};
}

struct BucketPlan {
    int32_t items_target, min_group_bins;
    double ms;  // the tuning batch's time per log-likelihood batch
};

double now_s() {
    using namespace std::chrono;
    return duration_cast<duration<double>>(steady_clock::now().time_since_epoch()).count();
}

}  // namespace
}  // namespace pe

using namespace pe;

struct pe_server_s {
    pe_server_config_t cfg;
    int device = 0;
    hipStream_t st = nullptr;
    Slab slab;
    Area a_ll, a_w;  // fixed areas of the slice
    int cap_ne = 0;
    int64_t cap_wblocks = 0, cap_fblocks = 0, cap_dblocks = 0;
    hipGraphExec_t graph = nullptr;
    hipEvent_t ev_a = nullptr, ev_b = nullptr, ev_c = nullptr, ev_d = nullptr;
    std::map<Bucket, BucketPlan> plans;  // tuned plans per shape bucket (pe_server_tune)
    double busy_slice_ms = 0.0, busy_admit_ms = 0.0;  // device time of the slices and admission stages
    double* h_stage = nullptr;  // pinned: stats, plans, status words
    double rate = 0.0;          // lane-operations per ms of the hot loop (running estimate)
    double t0 = 0.0;

    std::mutex mu;
    std::condition_variable cv, cv_done;
    std::deque<Req*> pending;
    std::vector<Req*> active;
    std::unordered_map<int64_t, Req*> all;
    int64_t next_ticket = 1;
    bool stop = false;
    pe_status_t fatal = PE_OK;
    std::thread worker;
    int64_t n_done = 0, n_slices = 0, n_items = 0, n_replays = 0, n_waits = 0;

    void run();
    void admit();
    pe_status_t slice();
    void finish(Req* q, int status);
    pe_status_t capture(const BatchPtrs& bll, const BatchPtrs& bw);
};

void pe_server_s::finish(Req* q, int status) {
    if (q->ev) {
        free_event(q->ev);
        q->ev = nullptr;
    }
    if (q->bytes) slab.free(q->off, q->bytes);
    q->bytes = 0;
    const double t = now_s() - t0;
    std::lock_guard<std::mutex> lk(mu);
    q->res.status = status;
    q->res.t_done = t;
    ++n_done;
    cv_done.notify_all();
}

// Admit queued requests in arrival order while memory and slots allow, then
// run their admission stages as one batch per stage and read back their plans.
void pe_server_s::admit() {
    std::vector<Req*> fresh;
    for (;;) {
        Req* q;
        {
            std::lock_guard<std::mutex> lk(mu);
            if (pending.empty()) break;
            q = pending.front();
        }
        if ((int)(active.size() + fresh.size()) >= cap_ne) {
            ++n_waits;
            break;
        }
        size_t off = 0;
        if (!slab.alloc(q->bytes, &off)) {
            ++n_waits;
            break;
        }
        {
            std::lock_guard<std::mutex> lk(mu);
            pending.pop_front();
        }
        q->off = off;
        char* base = slab.base() + off;
        const size_t evb = event_footprint(q->r.desc, q->r.n_draws);
        pe_event_s* ev = nullptr;
        if (new_event(&q->r.desc, base, q->r.n_draws, &ev) != PE_OK) {
            finish(q, PE_ERR_ARG);
            continue;
        }
        q->ev = ev;
        request_buffers(q, base + evb);
        q->res.t_admit = now_s() - t0;
        q->res.n_active = (int)(active.size() + fresh.size());
        fresh.push_back(q);
    }
    if (fresh.empty()) return;
    std::vector<PrepArg> vp;
    std::vector<MetricArg> vm;
    std::vector<DrawArg> vd;
    std::vector<EvDev> vl;
    pe_status_t s = PE_OK;
    for (Req* q : fresh) {
        const pe_event_desc_t& d = q->r.desc;
        hipError_t e = hipMemsetAsync(q->ev->status, 0, sizeof(int), st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(q->d_theta0, q->theta0.data(), sizeof(double) * q->D, hipMemcpyHostToDevice, st);
        const void* data = q->r.data;
        const void* psd = q->r.psd;
        if (e == hipSuccess && q->r.data_on_host) {
            e = hipMemcpyAsync(q->d_data, data, (size_t)d.n_det * d.n_bins * elem_data(d), hipMemcpyHostToDevice, st);
            if (e == hipSuccess)
                e = hipMemcpyAsync(q->d_psd, psd, (size_t)d.n_det * d.n_bins * elem_psd(d), hipMemcpyHostToDevice,
                                   st);
            data = q->d_data;
            psd = q->d_psd;
        }
        if (e != hipSuccess) s = PE_ERR_HIP;
        vp.push_back(prep_arg(q->ev, data, psd));
        vm.push_back(metric_arg(q->ev, q->d_theta0, nullptr, q->r.metric_flags, q->d_g));
        vd.push_back(draw_arg(q->ev, q->d_theta0, q->d_g, q->r.seed, q->r.stream_id, q->r.n_draws, q->d_theta,
                              q->d_logq, q->d_logprior));
        EvDev l = loglike_arg(q->ev, q->d_theta, q->r.n_draws, q->d_loglike, nullptr);
        if (cfg.items_target > 0) l.items_target = cfg.items_target;
        if (cfg.min_group_bins > 0) l.min_group_bins = cfg.min_group_bins;
        {
            std::lock_guard<std::mutex> lk(mu);
            const auto it = plans.find(bucket_of(d));
            if (it != plans.end()) {
                l.items_target = it->second.items_target;
                l.min_group_bins = it->second.min_group_bins;
            }
        }
        l.flags = kLlPrologue;
        l.tile_lo = l.tile_hi = 0;
        if (cfg.max_groups > 0 && l.max_groups > cfg.max_groups) l.max_groups = cfg.max_groups;
        vl.push_back(l);
    }
    if (s == PE_OK && hipEventRecord(ev_c, st) != hipSuccess) s = PE_ERR_HIP;
    if (s == PE_OK) s = run_prep(vp, st);
    if (s == PE_OK) s = run_metric(vm, st);
    if (s == PE_OK) s = run_draw(vd, st);
    if (s == PE_OK) s = run_loglike(vl, cfg.precision, st);
    if (s == PE_OK && hipEventRecord(ev_d, st) != hipSuccess) s = PE_ERR_HIP;
    // plans and status words to the pinned stage (8 doubles per request)
    for (size_t i = 0; i < fresh.size() && s == PE_OK; ++i) {
        if (hipMemcpyAsync(h_stage + 8 * i, fresh[i]->ev->plan, sizeof(EvPlan), hipMemcpyDeviceToHost, st) !=
                hipSuccess ||
            hipMemcpyAsync(h_stage + 8 * i + 4, fresh[i]->ev->status, sizeof(int), hipMemcpyDeviceToHost, st) !=
                hipSuccess)
            s = PE_ERR_HIP;
    }
    if (s == PE_OK && hipStreamSynchronize(st) != hipSuccess) s = PE_ERR_HIP;
    float ams = 0.0f;
    if (s == PE_OK && hipEventElapsedTime(&ams, ev_c, ev_d) == hipSuccess) busy_admit_ms += ams;
    if (s != PE_OK) {
        fatal = s;
        for (Req* q : fresh) finish(q, s);
        return;
    }
    for (size_t i = 0; i < fresh.size(); ++i) {
        Req* q = fresh[i];
        std::memcpy(&q->plan, h_stage + 8 * i, sizeof(EvPlan));
        int flags = 0;
        std::memcpy(&flags, h_stage + 8 * i + 4, sizeof(int));
        if (flags & kStBadPsd) {
            finish(q, PE_ERR_ARG);
            continue;
        }
        if (flags & kStNonfinite) {
            finish(q, PE_ERR_NONFINITE);
            continue;
        }
        // singular metric: the draws sit at theta0 with prior -inf, as for
        // pe_draw; the request still completes (ESS 0) and reports it
        if (flags & kStSingular) q->res.status = PE_ERR_SINGULAR;
        q->tile_ops = 256.0 * q->plan.kmax * (10.0 + (cfg.precision == PE_PREC_SPLIT ? 10.0 : 32.0) * q->r.desc.n_det);
        active.push_back(q);
    }
}

pe_status_t pe_server_s::capture(const BatchPtrs& bll, const BatchPtrs& bw) {
    hipGraph_t g = nullptr;
    PE_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    // the captured slice serves every later mix of requests: it keeps the distance pass
    hipError_t e = launch_loglike_batch(bll, cap_ne, 0, cap_fblocks, cfg.precision, false, true, PE_MAX_DET, st);
    if (e == hipSuccess) e = launch_weights_batch(bw, cap_ne, cap_wblocks, cap_dblocks, st);
    hipError_t e2 = hipStreamEndCapture(st, &g);
    if (e != hipSuccess) return fail(PE_ERR_HIP, std::string("slice capture: ") + hipGetErrorString(e));
    if (e2 != hipSuccess) return fail(PE_ERR_HIP, std::string("slice capture: ") + hipGetErrorString(e2));
    e = hipGraphInstantiate(&graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        graph = nullptr;
        return fail(PE_ERR_HIP, std::string("slice instantiate: ") + hipGetErrorString(e));
    }
    return PE_OK;
}

// One slice of the hot loop: tiles of the active requests, shortest remaining
// work first, up to about slice_ms of estimated work (at least one tile);
// requests whose last tile is in the slice are finalised and weighted in it.
pe_status_t pe_server_s::slice() {
    std::vector<Req*> order(active);
    std::stable_sort(order.begin(), order.end(), [](const Req* a, const Req* b) {
        return (a->plan.tiles - a->tiles_done) * a->tile_ops < (b->plan.tiles - b->tiles_done) * b->tile_ops;
    });
    double budget = cfg.slice_ms * rate;
    std::vector<EvDev> vl;
    std::vector<WeightArg> vw;
    std::vector<Req*> sel, fin;
    std::vector<int> take;
    for (Req* q : order) {
        const int rem = q->plan.tiles - q->tiles_done;
        int t = rem;
        if (rem > 0 && rem * q->tile_ops > budget) {
            t = (int)(budget / q->tile_ops);
            if (t < 1 && sel.empty()) t = 1;
            if (t < 1) break;
        }
        EvDev l = loglike_arg(q->ev, q->d_theta, q->r.n_draws, q->d_loglike, nullptr);
        if (cfg.max_groups > 0 && l.max_groups > cfg.max_groups) l.max_groups = cfg.max_groups;
        l.tile_lo = q->tiles_done;
        l.tile_hi = q->tiles_done + t;
        l.flags = (t == rem) ? kLlFinalize : 0;
        vl.push_back(l);
        sel.push_back(q);
        take.push_back(t);
        budget -= t * q->tile_ops;
        if (t == rem) {
            WeightArg w = {q->d_loglike, q->d_logprior, q->d_logq, q->r.n_draws, q->d_w, q->d_stats};
            vw.push_back(w);
            fin.push_back(q);
        }
        if (budget <= 0.0) break;
    }
    const int ne = (int)vl.size();
    std::vector<int64_t> poff(ne + 1, 0), foff(ne + 1, 0);
    for (int e = 0; e < ne; ++e) foff[e + 1] = foff[e] + ((vl[e].flags & kLlFinalize) ? blocks256(vl[e].n) : 0);
    const int nw = (int)vw.size();
    std::vector<int64_t> boff(nw + 1, 0), doff(nw + 1, 0);
    for (int e = 0; e < nw; ++e) {
        boff[e + 1] = boff[e] + (vw[e].n + kWBlock - 1) / kWBlock;
        doff[e + 1] = doff[e] + blocks256(vw[e].n);
    }
    BatchPtrs bll, bw;
    pe_status_t s = upload_area(a_ll, ne, poff[ne], foff[ne], vl.data(), sizeof(EvDev) * ne, poff, &foff,
                                loglike_scratch_bytes(cap_ne), st, bll);
    if (s == PE_OK)
        s = upload_area(a_w, nw, boff[nw], doff[nw], vw.data(), sizeof(WeightArg) * nw, boff, &doff,
                        sizeof(double4) * cap_wblocks + sizeof(double2) * cap_ne, st, bw);
    if (s != PE_OK) return s;
    PE_HIP(hipEventRecord(ev_a, st));
    if (cfg.use_graph) {
        if (!graph && (s = capture(bll, bw)) != PE_OK) return s;
        PE_HIP(hipGraphLaunch(graph, st));
        ++n_replays;
    } else {
        PE_HIP(launch_loglike_batch(bll, ne, 0, foff[ne], cfg.precision, false, true, PE_MAX_DET, st));
        PE_HIP(launch_weights_batch(bw, nw, boff[nw], doff[nw], st));
    }
    PE_HIP(hipEventRecord(ev_b, st));
    for (int i = 0; i < nw; ++i) {
        Req* q = fin[i];
        const int64_t n = q->r.n_draws;
        PE_HIP(hipMemcpyAsync(h_stage + 8 * i, q->d_stats, 4 * sizeof(double), hipMemcpyDeviceToHost, st));
        PE_HIP(hipMemcpyAsync(h_stage + 8 * i + 4, q->ev->status, sizeof(int), hipMemcpyDeviceToHost, st));
        if (q->r.loglike_out)
            PE_HIP(hipMemcpyAsync(q->r.loglike_out, q->d_loglike, n * sizeof(double), hipMemcpyDeviceToHost, st));
        if (q->r.w_out) PE_HIP(hipMemcpyAsync(q->r.w_out, q->d_w, n * sizeof(double), hipMemcpyDeviceToHost, st));
        if (q->r.theta_out)
            PE_HIP(hipMemcpyAsync(q->r.theta_out, q->d_theta, (size_t)q->D * n * sizeof(double),
                                  hipMemcpyDeviceToHost, st));
    }
    PE_HIP(hipStreamSynchronize(st));
    // running estimate of the hot loop's rate from this slice's duration
    double done_ops = 0.0;
    int64_t items = 0;
    for (int e = 0; e < ne; ++e) {
        done_ops += take[e] * sel[e]->tile_ops;
        items += (int64_t)take[e] * sel[e]->plan.n_groups;
        sel[e]->tiles_done += take[e];
    }
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, ev_a, ev_b) == hipSuccess) {
        busy_slice_ms += ms;
        if (ms > 0.5f && done_ops > 0.0) rate = 0.8 * rate + 0.2 * (done_ops / ms);
    }
    ++n_slices;
    n_items += items;
    for (int i = 0; i < nw; ++i) {
        Req* q = fin[i];
        std::memcpy(q->res.stats, h_stage + 8 * i, 4 * sizeof(double));
        int flags = 0;
        std::memcpy(&flags, h_stage + 8 * i + 4, sizeof(int));
        // a NaN ESS: some log-weight was NaN or +inf (no weight defined)
        if (((flags & kStNonfinite) || std::isnan(q->res.stats[0])) && q->res.status == PE_OK)
            q->res.status = PE_ERR_NONFINITE;
        active.erase(std::find(active.begin(), active.end(), q));
        finish(q, q->res.status);
    }
    return PE_OK;
}

void pe_server_s::run() {
    (void)hipSetDevice(device);
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(mu);
            cv.wait(lk, [&] { return stop || !pending.empty() || !active.empty(); });
            if (stop && pending.empty() && active.empty()) return;
        }
        if (fatal == PE_OK) admit();
        if (fatal == PE_OK && !active.empty()) {
            pe_status_t s = slice();
            if (s != PE_OK) fatal = s;
        }
        if (fatal != PE_OK) {
            // fail everything still queued or active
            std::vector<Req*> left(active);
            active.clear();
            {
                std::lock_guard<std::mutex> lk(mu);
                left.insert(left.end(), pending.begin(), pending.end());
                pending.clear();
            }
            for (Req* q : left) finish(q, fatal);
        }
    }
}

extern "C" {

pe_status_t pe_server_create(const pe_server_config_t* cfg, pe_server_t* out) {
    if (!out) return fail(PE_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (!cfg) return fail(PE_ERR_ARG, "cfg is NULL");
    if (cfg->hbm_budget < ((int64_t)1 << 20)) return fail(PE_ERR_ARG, "hbm_budget must be at least 1 MiB");
    if (cfg->precision != PE_PREC_FP64 && cfg->precision != PE_PREC_SPLIT) return fail(PE_ERR_ARG, "bad precision");
    if (cfg->max_active < 1 || cfg->max_active > 4096) return fail(PE_ERR_ARG, "max_active must be in 1..4096");
    if (!(cfg->slice_ms > 0.0)) return fail(PE_ERR_ARG, "slice_ms must be > 0");
    if (cfg->max_groups < 0 || cfg->max_groups > 64) return fail(PE_ERR_ARG, "max_groups must be in 0..64");
    if (cfg->items_target != 0 && (cfg->items_target < 256 || cfg->items_target > (1 << 20)))
        return fail(PE_ERR_ARG, "items_target must be 0 or in 256..2^20");
    if (cfg->min_group_bins != 0 && (cfg->min_group_bins < 32 || cfg->min_group_bins > (1 << 20)))
        return fail(PE_ERR_ARG, "min_group_bins must be 0 or in 32..2^20");
    pe_server_s* s = new (std::nothrow) pe_server_s();
    if (!s) return fail(PE_ERR_OOM, "host allocation failed");
    s->cfg = *cfg;
    s->cap_ne = cfg->max_active;
    s->cap_wblocks = (int64_t)cfg->max_active * (kMaxServerDraws / kWBlock);
    s->cap_dblocks = (int64_t)cfg->max_active * (kMaxServerDraws / 256);
    s->cap_fblocks = s->cap_dblocks;
    s->rate = (cfg->precision == PE_PREC_SPLIT ? 3.0e13 : 1.0e13) / 1e3;
    s->t0 = now_s();
    pe_status_t st = PE_OK;
    auto bail = [&](pe_status_t e) {
        if (s->h_stage) (void)hipHostFree(s->h_stage);
        if (s->ev_a) (void)hipEventDestroy(s->ev_a);
        if (s->ev_b) (void)hipEventDestroy(s->ev_b);
        if (s->ev_c) (void)hipEventDestroy(s->ev_c);
        if (s->ev_d) (void)hipEventDestroy(s->ev_d);
        release_area(s->a_ll);
        release_area(s->a_w);
        s->slab.release();
        if (s->st) (void)hipStreamDestroy(s->st);
        delete s;
        return e;
    };
    if (hipGetDevice(&s->device) != hipSuccess || hipStreamCreateWithFlags(&s->st, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreate(&s->ev_a) != hipSuccess || hipEventCreate(&s->ev_b) != hipSuccess ||
        hipEventCreate(&s->ev_c) != hipSuccess || hipEventCreate(&s->ev_d) != hipSuccess ||
        hipHostMalloc((void**)&s->h_stage, sizeof(double) * 8 * (size_t)cfg->max_active, hipHostMallocDefault) !=
            hipSuccess)
        return bail(fail(PE_ERR_HIP, "server stream, events or pinned stage"));
    s->a_ll.fixed = s->a_w.fixed = true;
    s->a_ll.layout_ne = s->a_w.layout_ne = s->cap_ne;
    s->a_ll.layout_rec = sizeof(EvDev);
    s->a_w.layout_rec = sizeof(WeightArg);
    const size_t ll_bytes = fixed_area_bytes(s->cap_ne, sizeof(EvDev), loglike_scratch_bytes(s->cap_ne));
    const size_t w_bytes = fixed_area_bytes(s->cap_ne, sizeof(WeightArg),
                                            sizeof(double4) * s->cap_wblocks + sizeof(double2) * s->cap_ne);
    if ((st = dalloc_bytes(&s->a_ll.dev, ll_bytes)) != PE_OK) return bail(st);
    s->a_ll.cap = ll_bytes;
    if ((st = dalloc_bytes(&s->a_w.dev, w_bytes)) != PE_OK) return bail(st);
    s->a_w.cap = w_bytes;
    if ((st = s->slab.init((size_t)cfg->hbm_budget)) != PE_OK) return bail(st);
    prime_hot_grids();
    s->worker = std::thread([s] { s->run(); });
    *out = s;
    return PE_OK;
}

pe_status_t pe_server_submit(pe_server_t srv, const pe_request_t* req, int64_t* ticket) {
    if (!srv || !req || !ticket) return fail(PE_ERR_ARG, "NULL argument");
    pe_status_t s = validate_desc(&req->desc);
    if (s != PE_OK) return s;
    if (req->n_draws < 1 || req->n_draws > kMaxServerDraws) return fail(PE_ERR_ARG, "n_draws must be in 1..2^22");
    if (!req->data || !req->psd || !req->theta0) return fail(PE_ERR_ARG, "data, psd and theta0 are required");
    if (req->metric_flags & ~1) return fail(PE_ERR_ARG, "unknown metric flags");
    if (req->desc.time_marg) return fail(PE_ERR_ARG, "the server does not take time-marginalised events");
    Req* q = new (std::nothrow) Req();
    if (!q) return fail(PE_ERR_OOM, "host allocation failed");
    q->r = *req;
    q->D = pe_dim(req->desc.params);
    q->theta0.assign(req->theta0, req->theta0 + q->D);
    q->bytes = event_footprint(req->desc, req->n_draws) + request_buffers(q, nullptr);
    q->res.t_submit = pe_server_now(srv);
    std::lock_guard<std::mutex> lk(srv->mu);
    q->ticket = q->res.ticket = srv->next_ticket++;
    srv->all[q->ticket] = q;
    *ticket = q->ticket;
    if (q->bytes > srv->slab.capacity()) {
        q->res.status = PE_ERR_BUDGET;
        q->res.t_admit = q->res.t_done = q->res.t_submit;
        ++srv->n_done;
        srv->cv_done.notify_all();
        return PE_OK;
    }
    srv->pending.push_back(q);
    srv->cv.notify_all();
    return PE_OK;
}

pe_status_t pe_server_wait(pe_server_t srv, int64_t ticket, double timeout_s, pe_result_t* out) {
    if (!srv || !out) return fail(PE_ERR_ARG, "NULL argument");
    std::unique_lock<std::mutex> lk(srv->mu);
    auto it = srv->all.find(ticket);
    if (it == srv->all.end()) return fail(PE_ERR_ARG, "unknown ticket");
    Req* q = it->second;
    auto ready = [&] { return q->res.t_done > 0.0; };
    if (timeout_s < 0.0)
        srv->cv_done.wait(lk, ready);
    else if (!srv->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), ready))
        return fail(PE_ERR_TIMEOUT, "request not complete");
    *out = q->res;
    srv->all.erase(it);
    delete q;
    return PE_OK;
}

double pe_server_now(pe_server_t srv) { return srv ? now_s() - srv->t0 : 0.0; }

pe_status_t pe_server_counters(pe_server_t srv, int64_t out[6]) {
    if (!srv || !out) return fail(PE_ERR_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(srv->mu);
    out[0] = srv->n_done;
    out[1] = srv->n_slices;
    out[2] = srv->n_items;
    out[3] = srv->n_replays;
    out[4] = (int64_t)srv->slab.peak();
    out[5] = srv->n_waits;
    return PE_OK;
}

pe_status_t pe_server_busy(pe_server_t srv, double out[2]) {
    if (!srv || !out) return fail(PE_ERR_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(srv->mu);
    out[0] = srv->busy_slice_ms;
    out[1] = srv->busy_admit_ms;
    return PE_OK;
}

pe_status_t pe_server_tune(pe_server_t srv, int32_t n, const pe_event_t* events, const double* const* theta_dev,
                           const int64_t* n_draws, int32_t reps) {
    if (!srv || !events || !theta_dev || !n_draws) return fail(PE_ERR_ARG, "NULL argument");
    if (n < 1 || n > 4096) return fail(PE_ERR_ARG, "n must be in 1..4096");
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        if (!srv->pending.empty() || !srv->active.empty()) return fail(PE_ERR_ARG, "tune an idle server");
    }
    std::map<Bucket, std::vector<int>> groups;
    for (int i = 0; i < n; ++i) {
        if (!events[i] || !theta_dev[i]) return fail(PE_ERR_ARG, "NULL event or draws");
        groups[bucket_of(events[i]->desc)].push_back(i);
    }
    for (const auto& kv : groups) {
        std::vector<pe_event_t> ev;
        std::vector<const double*> th;
        std::vector<int64_t> nn;
        for (int i : kv.second) {
            ev.push_back(events[i]);
            th.push_back(theta_dev[i]);
            nn.push_back(n_draws[i]);
        }
        int32_t it = 0, mb = 0;
        double ms = 0.0;
        const pe_status_t s = pe_autotune_plan((int32_t)ev.size(), ev.data(), th.data(), nn.data(),
                                               srv->cfg.precision, reps, &it, &mb, &ms, srv->st);
        if (s != PE_OK) return s;
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->plans[kv.first] = BucketPlan{it, mb, ms};
    }
    return PE_OK;
}

pe_status_t pe_server_plans(pe_server_t srv, int32_t max, int32_t* out, double* ms, int32_t* count) {
    if (!srv || !count || (max > 0 && !out)) return fail(PE_ERR_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(srv->mu);
    int32_t c = 0;
    for (const auto& kv : srv->plans) {
        if (c < max) {
            out[4 * c] = kv.first.n_det;
            out[4 * c + 1] = kv.first.log2k;
            out[4 * c + 2] = kv.second.items_target;
            out[4 * c + 3] = kv.second.min_group_bins;
            if (ms) ms[c] = kv.second.ms;
        }
        ++c;
    }
    *count = c;
    return PE_OK;
}

pe_status_t pe_server_destroy(pe_server_t srv) {
    if (!srv) return fail(PE_ERR_ARG, "server is NULL");
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
        srv->cv.notify_all();
    }
    srv->worker.join();
    (void)hipStreamSynchronize(srv->st);
    if (srv->graph) (void)hipGraphExecDestroy(srv->graph);
    for (auto& kv : srv->all) delete kv.second;
    (void)hipHostFree(srv->h_stage);
    (void)hipEventDestroy(srv->ev_a);
    (void)hipEventDestroy(srv->ev_b);
    (void)hipEventDestroy(srv->ev_c);
    (void)hipEventDestroy(srv->ev_d);
    release_area(srv->a_ll);
    release_area(srv->a_w);
    srv->slab.release();
    (void)hipStreamDestroy(srv->st);
    pe_status_t f = srv->fatal;
    delete srv;
    return f == PE_OK ? PE_OK : fail(f, "the server stopped on an error");
}

}  // extern "C"
