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
    int32_t tm, tm_points;  // tm: 1 for a time-marginalised likelihood (11-D), its tc nodes
    double tc_lo, tc_hi;
    // time marginal from block moments (split precision): tm_P moments per
    // block of tm_fine bins (0: not available for this window, see kTmAlpha),
    // evaluated about tm_tmid; tm_a = pi tm_fine df
    int32_t tm_P, tm_fine;
    double tm_tmid, tm_a;
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
constexpr int kRedoTile = 64; // draws per workgroup (one wave) of the FP64 re-evaluation
constexpr int kBlk = 16;      // bins per FP32 block sum before its fold into FP64
constexpr int kBuckets = 4096;  // ISCO-cut buckets of the draw ordering
constexpr int kTabPad = 8;      // zeroed records past the last bin

// Device status bits (event status word).
constexpr int kStBadPsd = 1;
constexpr int kStNonfinite = 2;
constexpr int kStSingular = 4;

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
    int tiles;     // tiles of kTile live draws (plan of the re-evaluation: of kRedoTile listed draws)
    int stride;    // column stride of the partials (the re-evaluation's; the main plan uses npad)
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
    double *pl1, *pw2, *ppw;  // [n_det][K+1] exclusive prefixes of |w|, |w|^2 and the whitened power |w|^2/pw
                              // (split-path error estimate)
    double *guard;  // [PE_MAX_DET][kGuardStride] noise statistics of the data (split-path error estimate)
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

// dmask: coordinates decoupled besides the likelihood's marginalised ones
// (the tiled coordinates of an extrinsic completion; 0 for plain draws). With
// kDrawCond set in it, the other coordinates are drawn given the tiled ones
// instead (their rows conditioned on, not integrated out).
constexpr uint32_t kDrawCond = 1u << 31;
struct DrawArg {
    EvConst ec;
    const double *theta0, *g;
    double *chol;
    int *status;
    uint64_t seed;
    uint32_t stream_id, dmask;
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
    const double *pl1, *pw2, *ppw;  // [n_det][K+1] exclusive prefixes of |w|, |w|^2, |w|^2/pw
    const double *guard;  // noise statistics of the event's data (see kGuardStride)
    int *kc_all, *hist, *idx, *kcut;
    double *coef, *resp, *hh;
    double2 *partial;
    EvPlan *plan;    // [2]: the batch's plan, then the plan of the FP64 re-evaluation
    int *rflag;      // [npad] split finalize: rank of a re-evaluated draw in its block of 256, else -1
    int *rcnt;       // [npad / 256] re-evaluated draws per block, then their offsets
    int *rpos;       // [npad] positions of the re-evaluated draws, ascending
    double2 *zd;     // [npad] Z of distance-marginalised events (read by k_b_dist)
    double2 *tm_mom; // time marginal from block moments: [n_fine][tm_P][npad] moments of each draw's integrand
    const float *tm_pow;  // [tm_fine][tm_P] x^p of each bin's offset in its block (NULL: formed per bin)
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
constexpr int kLlMoments = 4;  // time-marginalised event on the block-moment path (plan chunks of ec.tm_fine bins)

// Block moments of the time marginal. Within a block of bins with centre f_c
// and half-width D/2, exp(-2 pi i f u) = exp(-2 pi i f_c u) sum_p (-i a u)^p x^p / p!
// with x = (f - f_c) / (D/2) in [-1, 1] and a = pi D; the series is cut after
// P terms, which leaves at most |a u|^P / P! / (1 - |a u| / (P + 1)) of the
// block's sum of |terms|. The block width is chosen so that |a u| <= kTmAlpha[P]
// over the window (u = t - tm_tmid, |u| <= T / 2): 3.9e-10 and 3.5e-11 of the
// sum of |terms| for P = 8 and 16.
constexpr int kTmMoments = 16;  // the most moments a block carries
constexpr double kTmAlpha8 = 0.25, kTmAlpha16 = 1.5;

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
    int pad0;
    int64_t total;         // flattened size (blocks)
    int64_t total2;        // second flattened size (blocks)
    int qitems[kQueues];   // hot-loop items per queue (written by k_items<false>, then k_items<true>)
    int qnext[kQueues];    // queue counters
    double redo_budget;    // split path: |d ln L| estimate above which a draw is re-evaluated in FP64
};

// ---------------------------------------------------------------------------
// Error of the split path and when a draw is re-evaluated in FP64.
//
// The hardware sine/cosine of gfx950 (v_sin_f32, v_cos_f32 of a turn-based
// argument t) returns exp(-2 pi i t) (1 + eps(t)) with, measured over every
// FP32 argument in [2^-30, 2): |eps| at most 1.277e-7 once the mean magnitude
// bias (-3.23e-8) is removed by kTrigGain, RMS 3.67e-8, and Fourier
// coefficients c_m of eps(t) (t in [0, 1)) of at most 1e-8 for |m| <= 8 (the
// low ones 5e-10 .. 1.1e-9). The error of a detector's sum
// Z_d = sum_k |w_k| exp(-2 pi i t_k) is then
//   sum_m c_m Z_d^(1-m),  Z_d^(j) = sum_k |w_k| exp(-2 pi i j t_k):
// j = 0 is L1 = sum |w_k| (term c_1 L1), j = 1 is Z_d itself, and |j| >= 2
// add coherently only as far as the data's phases follow the template's. For
// data with Gaussian noise at the PSD's level, the phase of bin k scatters
// about the signal's with a Rice distribution; its harmonic j keeps the factor
// e_j(a) <= (0.7 a)^(j-1) of the signal's coherent sum (a = signal / noise
// amplitude in the bin; e_j from the Bessel-function form of the Rice moments),
// so only the lowest c_m matter when a is small (configs 0, 1, 4: a < 0.4).
// Around these expectations the sum scatters with RMS (per-term error) x
// sqrt(sum |w_k|^2); the per-term RMS adds to the trigonometric one the FP32
// rounding of the turn-based argument (two roundings, <= 3.9e-8 turns RMS).
// Per draw the finalize bounds |d ln L| per detector by the smaller of
//   eps_coh(a) C_d + kEpsL1 |R_d| L1_d   and the worst case   kEpsMax |R_d| L1_d
// (L1_d = sum |w_k| and W2_d = sum |w_k|^2 below the draw's cut; C_d the
// larger of |R_d Z_d| and the matched magnitude sqrt(H_d rho2_d), rho2_d a
// bound on the detector's signal power below the cut from the data's whitened
// power there in excess of the noise's) plus the scatter kEpsInc sqrt(sum_d |R_d|^2 W2_d),
// which adds in quadrature over the detectors. Where the data carry less than
// the PSD's noise (e.g. noise-free injections) only the worst case applies.
// Draws whose bound exceeds the batch's redo budget are re-evaluated in FP64
// on the hot loop's own layout.
constexpr double kTrigGain = 1.0 + 3.23e-8;
constexpr double kEpsMax = 1.4e-7;       // max |eps| (1.277e-7 measured)
constexpr double kEpsL1 = 7.0e-10;       // |c_1| (5.6e-10 measured)
constexpr double kEpsRms = 4.4e-8;       // RMS of eps (3.67e-8 measured), tail of the harmonic sum
constexpr double kEpsInc = 1.5e-6;       // 6 x per-term RMS 2.5e-7 (argument roundings ~2e-7 rad, trig
                                         // 3.7e-8, FP32 weights and block sums)
// |c_{1-j}| + |c_{1+j}| for j = 1..7 (measured, x1.5)
constexpr double kEpsHarm[7] = {1.5e-9, 2.2e-9, 6.3e-9, 3.0e-9, 8.0e-9, 7.6e-10, 1.5e-8};
constexpr double kRedoBudget = 5e-4;     // default: half of the split path's stated 1e-3
// Noise statistics per detector (event tables): the bound rho2 on the signal
// power (< 0: the data carry less than the noise the PSD implies), the largest
// 4 df f^-7/3 / S of the band, and over the whole band L1 = sum |w_k| and
// sqrt(sum |w_k|^2) (diagnostics; the finalize uses the prefixes pl1, pw2).
constexpr int kGuardStride = 4;
constexpr int kGuardRho2 = 0, kGuardPwMax = 1, kGuardL1 = 2, kGuardW2 = 3;
constexpr int kGuardLen = kGuardStride * PE_MAX_DET;

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
    double *pl1 = nullptr;  // [n_det][K+1] exclusive prefix of |w|
    double *pw2 = nullptr;  // [n_det][K+1] exclusive prefix of |w|^2
    double *ppw = nullptr;  // [n_det][K+1] exclusive prefix of the whitened data power |w|^2 / pw
    double *guard = nullptr;  // [kGuardLen] noise statistics of the data
    int *status = nullptr;  // device status word
    double *mws = nullptr;  // metric + draw workspace
    double *mix_chol = nullptr;  // [PE_MIX_MAX][kCholLen] factors of a mixture's component metrics
    // per-draw workspace
    int64_t npad = 0;
    int *kc_all = nullptr;  // [npad] cut per draw, -1 out of support
    int *hist = nullptr;    // [kBuckets] bucket counts, then offsets
    int *idx = nullptr;
    pe::EvPlan *plan = nullptr;  // [2]: batch plan, FP64 re-evaluation plan
    int *rflag = nullptr;        // [npad]
    int *rcnt = nullptr;         // [npad / 256]
    int *rpos = nullptr;         // [npad]
    double2 *zd = nullptr;       // [npad]
    // time-marginalised events: the draws at every trapezoid node and their ln L
    // (the workspace's npad counts these node draws)
    double *tm_theta = nullptr;  // [PE_MAX_DIM][npad]
    double *tm_ll = nullptr;     // [npad]
    char *tm_mem = nullptr;      // block moments of the time marginal (own allocation, grown on demand)
    char *tm_pow = nullptr;      // [tm_fine][tm_P] floats: the moment powers of a bin's offset (own allocation)
    int64_t tm_mom_cols = 0;     // draw columns tm_mem holds
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
                             int max_seg, int max_det, hipStream_t st);
hipError_t launch_metric_batch(const BatchPtrs &b, int ne, int64_t total_blocks, hipStream_t st);
hipError_t launch_draw_batch(const BatchPtrs &b, int ne, int64_t total_blocks, hipStream_t st, bool ext = false);
// Mixture log-density (pe_mixture_logq): the components' factors are in chol
// (k_cholesky's records, one per component).
struct MixArg {
    EvConst ec;
    const double *chol;    // [m][kCholLen]
    const double *theta0;  // [m][D] component centres
    const double *theta;   // [D][n]
    double *logq;          // [n]
    int *status;
    int64_t n;
    int m;
    double lpi[PE_MIX_MAX];  // ln of each component's normalised weight (-inf: weight 0)
};
hipError_t launch_mix_logq(const MixArg &a, hipStream_t st);
// any_dist: some event of the batch is distance-marginalised (adds k_b_dist);
// max_det: no event of the batch has more detectors (at most 2: the FP64
// re-evaluation's two-detector kernel).
hipError_t launch_loglike_batch(const BatchPtrs &b, int ne, int64_t prologue_blocks, int64_t finalize_blocks,
                                int precision, bool profile, bool any_dist, int max_det, hipStream_t st);
hipError_t launch_weights_batch(const BatchPtrs &b, int ne, int64_t total_blocks, int64_t total_draw_blocks,
                                hipStream_t st);
hipError_t launch_update_batch(const BatchPtrs &b, int ne, int64_t total_blocks, hipStream_t st);
void prime_hot_grids();
// Time-marginalised events: node draws [D][n M] from theta [D][n]; ln L of each
// draw from the node log-likelihoods (theta: the draws, for their tc).
hipError_t launch_tm_expand(const double* theta, int64_t n, const EvConst& ec, double* out, hipStream_t st);
hipError_t launch_tm_reduce(const double* ll, int64_t n, const EvConst& ec, double* out, hipStream_t st);
hipError_t launch_tm_centre(const double* theta, int64_t n, const EvConst& ec, double* out, hipStream_t st);
// The moment powers x^p (p < tm_P) of every offset i < tm_fine in a block of the
// block-moment path, as the moment hot loop forms them per bin.
hipError_t launch_tm_powers(float* out, int fine, int P, hipStream_t st);
constexpr int kTmPowMaxBins = 1 << 16;  // wider blocks form the powers per bin
hipError_t launch_loglike_moments(const BatchPtrs& b, int ne, int64_t prologue_blocks, int64_t node_blocks, int P,
                                  hipStream_t st);
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
// time-marginalised events: g_{tc,j} / g_{tc,tc} of the metric as given (the
// conditional mean of tc given the other coordinates)
constexpr int kCholTm = kCholRdiag + PE_MAX_DIM;
// conditional extrinsic completion: the metric's coupling of the kept to the
// tiled coordinates (after the marginalised ones are decoupled), D x D row-major
constexpr int kCholCond = kCholTm + PE_MAX_DIM;
constexpr int kCholLen = kCholCond + PE_MAX_DIM * PE_MAX_DIM;
constexpr int64_t kMwsScan = kMwsChol + kCholLen;  // segment sums [kSegSums][n_det][kScanSeg]
// per segment: pw (prefix scan), whitened data power, L1 and L2 of w, max pw
constexpr int kSegSums = 5;
constexpr int64_t kMwsTotal = kMwsScan + (int64_t)kSegSums * PE_MAX_DET * kScanSeg;
constexpr int64_t kMwsKcut = kMwsSrc - 4;  // frozen cut of the metric (stored as double)

// profiling hooks (pe_api.hip)
void prof_begin(const char *name, hipStream_t st);
void prof_end(const char *name, hipStream_t st);

}  // namespace pe
