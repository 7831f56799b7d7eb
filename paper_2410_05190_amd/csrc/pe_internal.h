// pe_internal.h -- shared declarations of the library's host runtime and kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pe.h"

namespace pe {

// Physical constants (the paper fixes none): IAU nominal GM_sun, exact c,
// IAU parsec, mean Earth radius (spherical Earth).
constexpr double kPi = 3.141592653589793238462643383279502884;
constexpr double kTwoPi = 6.283185307179586476925286766559005768;
constexpr double kInvTwoPi = 0.159154943091895335768883763372514362;
constexpr double kLn4 = 1.386294361119890618834464242916353136;
constexpr double kEulerGamma = 0.577215664901532860606512090082402431;
constexpr double kGMsun = 1.32712440018e20;
constexpr double kC = 299792458.0;
constexpr double kTsun = kGMsun / (kC * kC * kC);
constexpr double kMpc = 3.0856775814913673e22;
constexpr double kREarth = 6.371e6;
constexpr double kSix32 = 14.69693845669906858918;    // 6^(3/2)
constexpr double kAmpNewt = 0.21278751013966339916;   // sqrt(5/24) pi^(-2/3)

// Per-event constants, passed to kernels by value.
struct EvConst {
    int32_t n_det, params, phase, dim;
    int32_t dist, pad_;  // dist: 1 for a distance-marginalised likelihood (11-D)
    int64_t K;
    double f_lo, df, scale, amp0, gmst, chi_max, dl_max;
    double dtensor[PE_MAX_DET][6];  // detector tensor (x x^T - y y^T)/2: xx xy xz yy yz zz
    double up[PE_MAX_DET][3];       // unit vector to the detector from the geocentre
};

// Per-bin table records, one 64-byte (split) or 96-byte (FP64) record per bin
// so that a wave reads a bin with one scalar load.
struct alignas(64) Rec32 {
    double f, x, xm5, lnx;  // f, f^(1/3), f^(-5/3), ln(f)/3
    float2 w[PE_MAX_DET];   // |w|, arg(w)/(2 pi) in [0, 1)
};
struct alignas(32) Rec64 {
    double f, x, xm5, lnx;
    double2 w[PE_MAX_DET];  // w = 4 df f^(-7/6) d / S
};
static_assert(sizeof(Rec32) == 64, "Rec32 must be one 64-byte scalar load");
static_assert(sizeof(Rec64) == 96, "Rec64 must be 96 bytes");

// Per-draw coefficient rows (structure of arrays, row stride = npad).
constexpr int kCoefA = 0;     // A0..A7
constexpr int kCoefB5 = 8;
constexpr int kCoefB6 = 9;
constexpr int kCoefTau = 10;  // tau_d = tc + dt_d, PE_MAX_DET rows
constexpr int kNCoef = 14;
// Parameter records of the live draws in position order (doubles per draw),
// written by the scatter into the partial buffer and read by the coefficients.
constexpr int kRecStride = 12;
static_assert(kRecStride >= PE_MAX_DIM, "a record holds one draw's parameters");
static_assert(kRecStride % 2 == 0, "records are written as 16-byte pairs");

constexpr int kTile = 256;    // draws per workgroup of the hot loop
constexpr int kBlk = 16;      // bins per FP32 block sum before its fold into FP64
constexpr int kBuckets = 4096;  // ISCO-cut buckets of the draw ordering
constexpr int kTabPad = 8;      // zeroed records past the last bin

// Device status bits (event status word).
constexpr int kStBadPsd = 1;
constexpr int kStNonfinite = 2;
constexpr int kStSingular = 4;
constexpr int kStRedoFull = 8;  // the split path's FP64 re-evaluation list overflowed

// Workspace of the metric: per FD source, coefficients, response and delays.
constexpr int kMetricSrcStride = 32;  // doubles: A[8], B5, B6, rre[4], rim[4], tau[4], pad
constexpr int kMetricMaxDp = PE_MAX_DIM + 1;
constexpr int kMetricNG = kMetricMaxDp * (kMetricMaxDp + 1) / 2;  // 78 >= 66
constexpr int kMetricBlocks = 512;

// Blocks of the metric reduction for an event of K bins: one per 256 bins, at
// most kMetricBlocks (a function of the event only).
__host__ __device__ inline int metric_blocks(int64_t K) {
    const int64_t b = (K + 255) / 256;
    return (int)(b < kMetricBlocks ? b : kMetricBlocks);
}

// Blocks of 256 in n items.
__host__ __device__ inline int64_t blocks256(int64_t n) { return (n + 255) / 256; }

// Device-side plan of one event in a log-likelihood batch.
struct EvPlan {
    int n_active;  // live draws
    int kmax;      // bound on their cuts: upper edge of the highest non-empty cut bucket
    int fine;      // bins per chunk (a multiple of kBlk)
    int n_fine;    // chunks over [0, kmax)
    int n_groups;  // groups of chunks = partials per draw and detector
    int tiles;     // tiles of kTile live draws
};

// ---------------------------------------------------------------------------
// Batched launches. Every stage of the path runs as one set of launches over a
// list of events: a header {ne, ...} and per-event argument records in device
// memory, plus prefix offsets of the flattened index space (draws, bins or
// blocks). Kernels read the counts from device memory and walk the flattened
// space with grid-stride loops, so one launch shape serves any batch (and a
// captured graph can be replayed on new contents).
// ---------------------------------------------------------------------------
struct PrepArg {
    EvConst ec;
    const void *data, *psd;
    int data_f32, psd_f32;
    Rec32 *rec32;
    Rec64 *rec64;
    double *pw, *pfx, *seg;
    int *status;
};

struct MetricArg {
    EvConst ec;
    const Rec64 *tab;
    const double *pw;
    double *mws;
    const double *theta0, *steps;
    double *g;
    int flags, pad;
};

struct DrawArg {
    EvConst ec;
    const double *theta0, *g;
    double *chol;
    int *status;
    uint64_t seed;
    uint32_t stream_id, pad;
    int64_t n;
    double *theta, *logq, *logprior;
};

// One event of a log-likelihood batch. flags select the stages it takes part
// in: kLlPrologue (support, cut buckets, plan, per-draw coefficients) and
// kLlFinalize (combine the partials, ln L); the hot loop evaluates the draw
// tiles [tile_lo, tile_hi) of its plan (the whole event: 0, INT_MAX).
struct EvDev {
    EvConst ec;
    const Rec32 *rec32;
    const Rec64 *rec64;
    const double *pfx;
    int *kc_all, *hist, *idx, *kcut;
    double *coef, *resp, *hh;
    double2 *partial;
    EvPlan *plan;
    int *status;
    int64_t npad;
    int max_groups;      // cap on the groups of chunks (partial capacity / npad)
    int items_target;    // plan: work items the event's tiles x groups aim at
    int min_group_bins;  // plan: bins per group at least
    int tile_lo, tile_hi;
    int flags;
    int pad2;
    const double *theta;
    int64_t n;
    double *loglike, *aux;
};

constexpr int kLlPrologue = 1;
constexpr int kLlFinalize = 2;

struct WeightArg {
    const double *ll, *lp, *lq;
    int64_t n;
    double *w, *stats;
};

// Proposal update: sums of w, w d, w d d^T (upper triangle) per block of
// kWBlock draws, then per event in a fixed order.
constexpr int kUpdNQ = 1 + PE_MAX_DIM + PE_MAX_DIM * (PE_MAX_DIM + 1) / 2;  // 78
struct UpdateArg {
    const double *theta, *w;
    int64_t n;
    const double *th0;
    double *th0_out, *cov;
    int32_t dim, params;
};

// Hot-loop work queues: one per XCD (workgroup b of a launch runs on XCD
// b mod kQueues).
constexpr int kQueues = 8;

// Header of a batch in device memory.
struct BatchHdr {
    int ne;                // events
    int redo_cap;          // log-likelihood batches: capacity of the FP64 re-evaluation list
    int64_t total;         // flattened size (blocks)
    int64_t total2;        // second flattened size (blocks)
    int qitems[kQueues];   // hot-loop items per queue (written by k_b_items)
    int qnext[kQueues];    // queue counters
    int redo_count;        // entries appended to the re-evaluation list (reset by k_b_items)
    int pad;
};

// Split precision and the hardware sine/cosine of gfx950 (v_sin_f32 and
// v_cos_f32 of a turn-based argument), measured over 2^24 arguments in
// [-2, 2): at most 1.25e-7 off, and on average too small in magnitude by
// 3.23e-8 (phase bias below 1e-10). The mean magnitude bias adds coherently
// over a matched sum, so the split path scales its sums by kTrigGain; the rest
// can still add coherently when the terms' phases align, by at most ~1e-7 of
// sum_d |R_d| |Z_d|, so a draw whose sum exceeds kRedoMagnitude is re-evaluated
// in FP64, which keeps |d ln L| below 1e-3 for every draw.
constexpr double kTrigGain = 1.0 + 3.23e-8;
constexpr double kRedoMagnitude = 6000.0;
// Entries of the re-evaluation list in a batch's scratch, at most.
constexpr int kRedoCapMax = 1 << 20;

constexpr int kWBlock = 4096;  // draws per block of the weights reduction (256 threads x 16)

}  // namespace pe

struct pe_event_s {
    pe_event_desc_t desc;
    pe::EvConst ec;
    // tables
    pe::Rec32 *rec32 = nullptr;
    pe::Rec64 *rec64 = nullptr;
    double *pw = nullptr;   // [n_det][K] 4 df f^(-7/3) / S
    double *pfx = nullptr;  // [n_det][K+1] exclusive prefix of pw
    int *status = nullptr;  // device status word
    double *mws = nullptr;  // metric + draw workspace
    // per-draw workspace
    int64_t npad = 0;
    int *kc_all = nullptr;  // [npad] cut per draw, -1 out of support
    int *hist = nullptr;    // [kBuckets] bucket counts, then offsets
    int *idx = nullptr;
    pe::EvPlan *plan = nullptr;
    int64_t partial_cap = 0;  // double2 entries per detector
    double *coef = nullptr;   // [kNCoef][npad]
    int *kcut = nullptr;      // [npad]
    double *resp = nullptr;   // [2*n_det][npad] Re/Im R_d
    double *hh = nullptr;     // [npad] (h|h)
    double2 *partial = nullptr;
    // memory: the tables and the workspace each in one range; owned by the
    // event (hipMalloc) unless a server placed the event in its slab
    char *tab_mem = nullptr;
    char *ws_mem = nullptr;
    bool own_mem = true;
    // relative binning about a fiducial point (pe_relbin_setup); own memory
    int32_t rb_n = 0;            // bin edges (bins = rb_n - 1)
    char *rb_mem = nullptr;
    int64_t *rb_k = nullptr;     // [rb_n] grid index of each edge
    double *rb_erec = nullptr;   // [rb_n][4] f, f^(1/3), f^(-5/3), ln(f)/3 at the edges
    double *rb_phi0 = nullptr;   // [n_det][rb_n] fiducial phase at the edges, turns
    double2 *rb_A = nullptr;     // [n_det][rb_n - 1][2] per-bin sums A0, A1
    double2 *rb_P = nullptr;     // [n_det][K + 1][2] prefix sums P0, P1 (partial bins)
    double *rb_fid = nullptr;    // [PE_MAX_DIM] fiducial point
};

namespace pe {

// Kinds of batch areas.
enum AreaKind {
    kAreaPrep = 0,
    kAreaMetric = 1,
    kAreaDraw = 2,
    kAreaLoglike = 3,
    kAreaWeights = 4,
    kAreaUpdate = 5,
    kAreaKinds = 6
};

// Device pointers into an uploaded batch area.
struct BatchPtrs {
    BatchHdr *hdr;
    void *args;       // argument records
    int64_t *off;     // [ne + 1] prefix offsets of the flattened space
    int64_t *off2;    // [ne + 1] second offsets (weights: draws; loglike: finalize draws)
    double *scratch;  // kind-specific scratch
};

// kernel launchers (pe_kernels.hip, pe_loglike.hip). Each takes the batch's
// device pointers, the number of events, the flattened size(s) known on the
// host (for the grid) and the stream.
// Offsets are in blocks that each belong to one event: 256 bins (prep: K +
// kTabPad bins per event), metric_blocks(K) (metric), 256 draws (draws,
// log-likelihood prologue and finalize, weight normalisation) or kWBlock
// draws (weight reduction).
hipError_t launch_prep_batch(const BatchPtrs &b, int ne, int64_t total_blocks, int data_f32, int psd_f32,
                             hipStream_t st);
hipError_t launch_metric_batch(const BatchPtrs &b, int ne, int64_t total_blocks, hipStream_t st);
hipError_t launch_draw_batch(const BatchPtrs &b, int ne, int64_t total_blocks, hipStream_t st);
// any_dist: some event of the batch is distance-marginalised (adds k_b_dist).
hipError_t launch_loglike_batch(const BatchPtrs &b, int ne, int64_t prologue_blocks, int64_t finalize_blocks,
                                int precision, bool profile, bool any_dist, hipStream_t st);
hipError_t launch_weights_batch(const BatchPtrs &b, int ne, int64_t total_blocks, int64_t total_draw_blocks,
                                hipStream_t st);
hipError_t launch_update_batch(const BatchPtrs &b, int ne, int64_t total_blocks, hipStream_t st);
void prime_hot_grids();
hipError_t launch_waveform(const EvConst &ec, int data_psd_dtype, const double *theta, const void *psd, double *h,
                           double *snr2, double *scratch, hipStream_t st);
hipError_t launch_uniforms(uint64_t seed, uint32_t stream_id, int64_t n, int npairs, double *u, hipStream_t st);

// metric workspace layout (doubles)
constexpr int64_t kMwsSteps = 0;                                     // D steps
constexpr int64_t kMwsDen = 16;                                      // D step sums
constexpr int64_t kMwsSrc = 32;                                      // (2D+1) sources
constexpr int64_t kMwsPart = kMwsSrc + (2 * PE_MAX_DIM + 1) * kMetricSrcStride;
constexpr int64_t kMwsChol = kMwsPart + (int64_t)kMetricBlocks * kMetricNG;  // L (D*D) + logdet + flag
constexpr int kScanSeg = 256;                                        // segments of the prefix scan
// the Cholesky record: L (row-major D*D), log det, success flag, the periodic
// block of L L^T (G00 G01 G02 G11 G12 G22), the reciprocals 1/L_rr
constexpr int kCholLogdet = PE_MAX_DIM * PE_MAX_DIM;
constexpr int kCholOk = kCholLogdet + 1;
constexpr int kCholG = kCholLogdet + 2;
constexpr int kCholRdiag = kCholLogdet + 8;
constexpr int kCholLen = kCholRdiag + PE_MAX_DIM;
constexpr int64_t kMwsScan = kMwsChol + kCholLen;  // segment sums [n_det][kScanSeg]
constexpr int64_t kMwsTotal = kMwsScan + (int64_t)PE_MAX_DET * kScanSeg;
constexpr int64_t kMwsKcut = kMwsSrc - 4;  // frozen cut of the metric (stored as double)

// profiling hooks (pe_api.hip)
void prof_begin(const char *name, hipStream_t st);
void prof_end(const char *name, hipStream_t st);

}  // namespace pe
