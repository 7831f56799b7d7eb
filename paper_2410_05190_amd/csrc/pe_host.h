// pe_host.h -- host-side runtime shared by the C ABI (pe_api.hip) and the
// serving loop (pe_server.hip): errors, event memory, batch stage runners.
#pragma once

#include <mutex>
#include <string>
#include <vector>

#include "pe_internal.h"

namespace pe {

// Records msg as the calling thread's last error and returns s.
pe_status_t fail(pe_status_t s, const std::string& msg);

#define PE_HIP(call)                                                                                      \
    do {                                                                                                  \
        hipError_t _e = (call);                                                                           \
        if (_e != hipSuccess) return ::pe::fail(PE_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(_e)); \
    } while (0)

// Sequential carving of one device range into 256-byte aligned buffers; with a
// NULL base it only measures.
struct Carver {
    char* base;
    size_t off = 0;
    explicit Carver(char* b) : base(b) {}
    template <typename T>
    T* take(size_t count) {
        off = (off + 255) / 256 * 256;
        T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
        off += (count ? count : 1) * sizeof(T);
        return p;
    }
    size_t size() const { return (off + 255) / 256 * 256; }
};

pe_status_t validate_desc(const pe_event_desc_t* d);
void build_const(const pe_event_desc_t& d, EvConst& ec);
pe_status_t dalloc_bytes(char** p, size_t bytes);
void dfree_bytes(char*& p);

// Event memory: bytes of the tables and of the workspace for npad draws, and
// the footprint of an event sized for max_draws (one range).
size_t tables_bytes(const pe_event_desc_t& d);
size_t ws_bytes(const pe_event_desc_t& d, int64_t npad);
size_t event_footprint(const pe_event_desc_t& d, int64_t max_draws);
int64_t npad_for(int64_t n);
int64_t partial_cap_for(int64_t npad, int64_t K, int n_det);
int64_t groups_cap(int64_t np, int64_t K);

// New event laid out in `mem` (a range of event_footprint bytes, not owned)
// or in its own allocations (mem NULL). Does not prepare the tables.
pe_status_t new_event(const pe_event_desc_t* desc, char* mem, int64_t max_draws, pe_event_s** out);
void free_event(pe_event_s* ev);
pe_status_t ensure_ws(pe_event_s* ev, int64_t n);

// A batch area: one device buffer holding the header, the argument records,
// the offsets (uploaded with one copy, skipped when identical to the last
// upload) and kind-specific scratch. Batches on one stream are ordered, so the
// buffer is reused safely; `mu` is held from the upload until the launches are
// queued. A fixed area never reallocates (its pointers may be captured in a
// graph); a batch that does not fit is an error.
struct Area {
    std::mutex mu;
    char* dev = nullptr;
    size_t cap = 0;
    bool fixed = false;
    int layout_ne = 0;      // fixed layout: records
    size_t layout_rec = 0;  // fixed layout: bytes per record
    std::vector<char> shadow;
    // pinned staging of the uploads, two buffers used in turn; done[k] is
    // recorded after the copy from buffer k, so the host refills a buffer only
    // once its previous copy has left it
    char* host[2] = {nullptr, nullptr};
    char* host_dev[2] = {nullptr, nullptr};  // the same buffers' device-side addresses
    size_t host_cap[2] = {0, 0};
    hipEvent_t done[2] = {nullptr, nullptr};
    int next = 0;
};

size_t area_bytes(int ne, size_t arg_bytes, size_t scratch_bytes);
size_t fixed_area_bytes(int ne, size_t rec, size_t scratch_bytes);
pe_status_t reserve_area(Area& A, size_t bytes);
void release_area(Area& A);
pe_status_t upload_area(Area& A, int ne, int64_t total, int64_t total2, const void* args, size_t arg_bytes,
                        const std::vector<int64_t>& off, const std::vector<int64_t>* off2, size_t scratch_bytes,
                        hipStream_t st, BatchPtrs& out);

// Scratch of a log-likelihood batch: the queue offsets for ne events.
size_t loglike_scratch_bytes(int ne);

// Budget of the split path's error estimate above which a draw is
// re-evaluated in FP64 (global setting, written into each batch header).
double redo_budget_setting();

// Argument records of the batched stages.
PrepArg prep_arg(const pe_event_s* ev, const void* data, const void* psd);
MetricArg metric_arg(const pe_event_s* ev, const double* theta0, const double* steps, int flags, double* g);
DrawArg draw_arg(const pe_event_s* ev, const double* theta0, const double* g, uint64_t seed, uint32_t stream_id,
                 int64_t n, double* theta, double* logq, double* logprior);
EvDev loglike_arg(const pe_event_s* ev, const double* theta, int64_t n, double* loglike, double* aux);

// Time-marginalised events in a log-likelihood batch (see loglike_entry).
struct TmJob {
    pe_event_s* ev;
    const double* theta;
    int64_t n;
    double* loglike;
    bool moments;  // block-moment path (else every tc node evaluated as a draw)
};
// The log-likelihood batches of one call: the plain events (and time-marginalised
// events on the node path, as their node draws) in one batch, the events on
// the block-moment path in another.
struct LlJobs {
    std::vector<EvDev> main, mom;
    std::vector<TmJob> tm;
};
pe_status_t loglike_entry(pe_event_s* ev, const double* theta, int64_t n, double* loglike, double* aux,
                          int precision, LlJobs& jobs);
pe_status_t run_jobs(const LlJobs& jobs, int precision, hipStream_t st);
bool tm_moments(const pe_event_s* ev, int precision);
int64_t ws_draws(const pe_event_s* ev, int64_t n, int precision);
pe_status_t ensure_moments(pe_event_s* ev, int64_t n);

// Stage runners: upload the records to the stream's area and queue the launches.
pe_status_t run_prep(const std::vector<PrepArg>& v, hipStream_t st);
pe_status_t run_metric(const std::vector<MetricArg>& v, hipStream_t st);
pe_status_t run_draw(const std::vector<DrawArg>& v, hipStream_t st, bool ext = false);
pe_status_t run_loglike(const std::vector<EvDev>& v, int precision, hipStream_t st);
pe_status_t run_weights(const std::vector<WeightArg>& v, hipStream_t st);
pe_status_t run_update(const std::vector<UpdateArg>& v, hipStream_t st);
// Relative-binning log-likelihoods (pe_relbin.hip); needs pe_relbin_setup.
pe_status_t run_relbin(pe_event_s* ev, const double* theta, int64_t n, double* loglike, double* aux, hipStream_t st);

}  // namespace pe
