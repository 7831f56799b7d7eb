// pe_kernels.hip -- HIP kernels of the likelihood engine for gfx950 (MI355X).
//
// Every stage runs as one set of launches over a batch of events (argument
// records and offsets in device memory; grid-stride loops over the flattened
// bins, draws or blocks):
//   k_prep, k_seg_*        event tables and the (h|h) prefix sums
//   k_metric_*             finite-difference Fisher matrix at the proposal centre
//   k_cholesky, k_draw     the Gaussian proposal's draws, log q and log prior
//   (pe_loglike.hip)       per-draw scalars, the hot loop and ln L
//   k_w_*                  log-sum-exp weights and ESS (Eqs. 5-6)
// plus the waveform of one point (injections) and the proposal's uniforms.
#include <math.h>

#include "pe_device.h"

namespace pe {

// Grid of a grid-stride launch over `total` items of `per` threads each.
static unsigned stride_grid(int64_t total, int per = 256, unsigned cap = 16384) {
    int64_t g = (total + per - 1) / per;
    if (g < 1) g = 1;
    return (unsigned)(g < (int64_t)cap ? g : cap);
}
static unsigned event_grid(int ne, unsigned cap = 4096) {
    return (unsigned)(ne < 1 ? 1 : (ne < (int)cap ? ne : cap));
}

// ===========================================================================
// event preparation
// ===========================================================================
template <typename DT, typename ST>
__device__ __forceinline__ void prep_bin(const PrepArg& A, int64_t k) {
    const EvConst& ev = A.ec;
    const DT* __restrict__ data = (const DT*)A.data;
    const ST* __restrict__ psd = (const ST*)A.psd;
    const double f = grid_f(ev, k);
    const double x = cbrt(f);
    const double x2 = x * x;
    Rec32 r32;
    Rec64 r64;
    r32.f = r64.f = f;
    r32.x = r64.x = x;
    r32.xm5 = r64.xm5 = 1.0 / (x2 * x2 * x);
    r32.lnx = r64.lnx = log(f) * (1.0 / 3.0);
    const double f76 = f * sqrt(x);  // f^(7/6)
    int bad = 0;
#pragma unroll
    for (int d = 0; d < PE_MAX_DET; ++d) {
        if (d < ev.n_det) {
            const int64_t o = (int64_t)d * ev.K + k;
            const double S = (double)psd[o];
            const double dr = (double)data[2 * o], di = (double)data[2 * o + 1];
            if (!(S > 0.0) || !isfinite(S)) bad |= kStBadPsd;
            if (!isfinite(dr) || !isfinite(di)) bad |= kStNonfinite;
            const double a = 4.0 * ev.df / (S * f76);
            const double wr = a * dr, wi = a * di;
            r64.w[d] = make_double2(wr, wi);
            double al = atan2(wi, wr) * kInvTwoPi;
            if (al < 0.0) al += 1.0;
            r32.w[d] = make_float2((float)hypot(wr, wi), (float)al);
            A.pw[o] = 4.0 * ev.df / (S * f76 * f76);
        } else {
            r64.w[d] = make_double2(0.0, 0.0);
            r32.w[d] = make_float2(0.0f, 0.0f);
        }
    }
    A.rec32[k] = r32;
    A.rec64[k] = r64;
    if (bad) atomicOr(A.status, bad);
}

// Bins of every event of the batch (one storage class per launch), in blocks
// of 256 bins that each belong to one event (koff: block offsets); the
// kTabPad records past each table's end are zeroed here too.
template <typename DT, typename ST>
__global__ __launch_bounds__(256) void k_prep(const BatchHdr* __restrict__ hdr, const PrepArg* __restrict__ args,
                                              const int64_t* __restrict__ koff) {
    const int ne = hdr->ne;
    const int64_t nblk = koff[ne];
    for (int64_t b = blockIdx.x; b < nblk; b += gridDim.x) {
        const int e = find_slot(koff, ne, b);
        const PrepArg& A = args[e];
        const int64_t k = (b - koff[e]) * 256 + threadIdx.x;
        if (k < A.ec.K) {
            prep_bin<DT, ST>(A, k);
        } else if (k < A.ec.K + kTabPad) {
            Rec32 z32 = {};
            Rec64 z64 = {};
            A.rec32[k] = z32;
            A.rec64[k] = z64;
        }
    }
}

// Exclusive prefix C_k = sum_{j<k} pw_j (k = 0..K) per event and detector, in
// two passes over contiguous segments: segment sums, then each segment adds
// the sums before it (fixed order) and scans its bins in coalesced 256-wide
// tiles (wave shuffle scan + LDS across the four waves).
// Grid: (the batch's most segments, its most detectors, events); blocks past
// the event's segment or detector count return at once.
// Segments of the scan: at least 1024 bins each, at most kScanSeg of them.
__device__ __forceinline__ void scan_layout(int64_t K, int64_t& seg, int& nseg) {
    seg = max((int64_t)1024, (K + kScanSeg - 1) / kScanSeg);
    nseg = (int)((K + seg - 1) / seg);
}

__device__ __forceinline__ double block_sum4(double s, double* sh) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    const double r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
    __syncthreads();
    return r;
}

__device__ __forceinline__ double block_max4(double s, double* sh) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s = fmax(s, __shfl_xor(s, o));
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    const double r = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
    __syncthreads();
    return r;
}

// Per segment and detector: the sum of pw (for the prefix scan) and the noise
// statistics of the data behind the split path's error estimate: whitened
// power 4 df |d|^2 / S = |w|^2 / pw, L1 and L2 of the folded weights w, the
// largest pw. Slices of A.seg: [kSegSums][PE_MAX_DET][kScanSeg].
__global__ __launch_bounds__(256) void k_seg_sums(const BatchHdr* __restrict__ hdr,
                                                  const PrepArg* __restrict__ args) {
    __shared__ double sh[4];
    const int ne = hdr->ne;
    const int d = blockIdx.y, b = blockIdx.x;
    for (int e = blockIdx.z; e < ne; e += gridDim.z) {
        const PrepArg& A = args[e];
        const int64_t K = A.ec.K;
        int64_t seg;
        int nseg;
        scan_layout(K, seg, nseg);
        if (d >= A.ec.n_det || b >= nseg) continue;
        const double* a = A.pw + (int64_t)d * K;
        const int64_t k0 = (int64_t)b * seg;
        const int64_t k1 = min(k0 + seg, K);
        double s = 0.0, pwr = 0.0, l1 = 0.0, l2 = 0.0, mx = 0.0;
        for (int64_t k = k0 + threadIdx.x; k < k1; k += 256) {
            const double pw = a[k];
            const double2 w = A.rec64[k].w[d];
            const double w2 = w.x * w.x + w.y * w.y;
            s += pw;
            if (pw > 0.0) pwr += w2 / pw;
            l1 += sqrt(w2);
            l2 += w2;
            mx = fmax(mx, pw);
        }
        s = block_sum4(s, sh);
        pwr = block_sum4(pwr, sh);
        l1 = block_sum4(l1, sh);
        l2 = block_sum4(l2, sh);
        mx = block_max4(mx, sh);
        if (threadIdx.x == 0) {
            const int64_t o = (int64_t)d * kScanSeg + b, slice = (int64_t)PE_MAX_DET * kScanSeg;
            A.seg[o] = s;
            A.seg[slice + o] = pwr;
            A.seg[2 * slice + o] = l1;
            A.seg[3 * slice + o] = l2;
            A.seg[4 * slice + o] = mx;
        }
    }
}

// Each segment: its carries (the sums of the segment sums before it, one block
// reduction each), then block-wide inclusive scans per 256 bins of pw (into
// pfx), |w| (into pl1), |w|^2 (into pw2) and the whitened power |w|^2 / pw (into
// ppw).
// Exclusive scans of NV values per thread over the block at once (one pair of
// barriers for all of them); tile[i]: the block's total of value i. Each value
// sees exactly the arithmetic of a scan of its own.
template <int NV>
__device__ __forceinline__ void block_scan_excl(const double (&v)[NV], double (*sh)[NV], double (&x)[NV],
                                                double (&tile)[NV]) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    double inc[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) inc[i] = v[i];
#pragma unroll
    for (int off = 1; off < 64; off <<= 1)
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            const double u = __shfl_up(inc[i], off);
            if (lane >= off) inc[i] += u;
        }
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        double exc = __shfl_up(inc[i], 1);
        if (lane == 0) exc = 0.0;
        x[i] = exc;
        if (lane == 63) sh[w][i] = inc[i];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        double woff = 0.0;
        for (int q = 0; q < w; ++q) woff += sh[q][i];
        tile[i] = (sh[0][i] + sh[1][i]) + (sh[2][i] + sh[3][i]);
        x[i] += woff;
    }
    __syncthreads();
}

// Sums of NV values over the block at once (the arithmetic of block_sum4 per value).
template <int NV>
__device__ __forceinline__ void block_sums(double (&s)[NV], double (*sh)[NV]) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
#pragma unroll
        for (int i = 0; i < NV; ++i) s[i] += __shfl_xor(s[i], o);
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int i = 0; i < NV; ++i) sh[threadIdx.x >> 6][i] = s[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NV; ++i) s[i] = (sh[0][i] + sh[1][i]) + (sh[2][i] + sh[3][i]);
    __syncthreads();
}

__global__ __launch_bounds__(256) void k_seg_scan(const BatchHdr* __restrict__ hdr,
                                                  const PrepArg* __restrict__ args) {
    __shared__ double sh[4];
    __shared__ double sh4[4][4];
    const int ne = hdr->ne;
    const int d = blockIdx.y, b = blockIdx.x;
    for (int e = blockIdx.z; e < ne; e += gridDim.z) {
        const PrepArg& A = args[e];
        const int64_t K = A.ec.K;
        int64_t seg;
        int nseg;
        scan_layout(K, seg, nseg);
        if (d >= A.ec.n_det || b >= nseg) continue;
        const double* a = A.pw + (int64_t)d * K;
        const int64_t po = (int64_t)d * (K + 1);
        double* o = A.pfx + po;
        double* o1 = A.pl1 + po;
        double* o2 = A.pw2 + po;
        double* o3 = A.ppw + po;
        const int64_t slice = (int64_t)PE_MAX_DET * kScanSeg;
        const double* sg = A.seg + (int64_t)d * kScanSeg + threadIdx.x;
        const bool before = (int)threadIdx.x < b;
        double cr[4] = {before ? sg[0] : 0.0, before ? sg[2 * slice] : 0.0, before ? sg[3 * slice] : 0.0,
                        before ? sg[slice] : 0.0};
        block_sums<4>(cr, sh4);
        double carry = cr[0], carry1 = cr[1], carry2 = cr[2], carry3 = cr[3];
        const int64_t k0 = (int64_t)b * seg;
        const int64_t k1 = min(k0 + seg, K);
        for (int64_t base = k0; base < k1; base += 256) {
            const int64_t k = base + threadIdx.x;
            double v = 0.0, v1 = 0.0, v2 = 0.0, v3 = 0.0;
            if (k < k1) {
                v = a[k];
                const double2 w = A.rec64[k].w[d];
                v2 = w.x * w.x + w.y * w.y;
                v1 = sqrt(v2);
                if (v > 0.0) v3 = v2 / v;
            }
            const double vv[4] = {v, v1, v2, v3};
            double xx[4], tt[4];
            block_scan_excl<4>(vv, sh4, xx, tt);
            if (k < k1) {
                o[k] = carry + xx[0];
                o1[k] = carry1 + xx[1];
                o2[k] = carry2 + xx[2];
                o3[k] = carry3 + xx[3];
            }
            carry += tt[0];
            carry1 += tt[1];
            carry2 += tt[2];
            carry3 += tt[3];
        }
        if (b == nseg - 1 && threadIdx.x == 0) {
            o[K] = carry;
            o1[K] = carry1;
            o2[K] = carry2;
            o3[K] = carry3;
        }
        if (b == 0) {
            // the detector's noise statistics: segments combined in a fixed order
            const int t = threadIdx.x;
            const bool in = t < nseg;
            const double pwr = block_sum4(in ? sg[slice] : 0.0, sh);
            const double l1 = block_sum4(in ? sg[2 * slice] : 0.0, sh);
            const double l2 = block_sum4(in ? sg[3 * slice] : 0.0, sh);
            const double mx = block_max4(in ? sg[4 * slice] : 0.0, sh);
            if (t == 0) {
                // Gaussian noise at the PSD's level gives each bin whitened power 2 on
                // average (sd 2 sqrt(K) over the band); the excess bounds the signal's
                // power rho^2 (6 sd of margin). Data with less than the noise's power
                // less 6 sd get -1: the noise-based error estimate does not apply.
                const double Kd = (double)K, slack = 12.0 * sqrt(Kd), excess = pwr - 2.0 * Kd;
                double* G = A.guard + d * kGuardStride;
                G[kGuardRho2] = excess < -slack ? -1.0 : excess + slack;
                G[kGuardPwMax] = mx;
                G[kGuardL1] = l1;
                G[kGuardW2] = sqrt(l2);
            }
        }
    }
}

hipError_t launch_prep_batch(const BatchPtrs& b, int ne, int64_t total_blocks, int data_f32, int psd_f32,
                             int max_seg, int max_det, hipStream_t st) {
    if (ne <= 0) return hipSuccess;
    const PrepArg* args = (const PrepArg*)b.args;
    const unsigned nb = stride_grid(total_blocks, 1);
    if (data_f32 && psd_f32)
        k_prep<float, float><<<nb, 256, 0, st>>>(b.hdr, args, b.off);
    else if (data_f32)
        k_prep<float, double><<<nb, 256, 0, st>>>(b.hdr, args, b.off);
    else if (psd_f32)
        k_prep<double, float><<<nb, 256, 0, st>>>(b.hdr, args, b.off);
    else
        k_prep<double, double><<<nb, 256, 0, st>>>(b.hdr, args, b.off);
    // blocks past an event's segments or detectors return at once; the grid spans the batch's largest
    const dim3 g((unsigned)std::min(max_seg, kScanSeg), (unsigned)std::min(max_det, PE_MAX_DET), event_grid(ne, 64));
    k_seg_sums<<<g, 256, 0, st>>>(b.hdr, args);
    k_seg_scan<<<g, 256, 0, st>>>(b.hdr, args);
    return hipGetLastError();
}

// ===========================================================================
// metric (finite-difference Fisher matrix on the same model code)
// ===========================================================================
__device__ __forceinline__ void default_steps(const EvConst& ev, const double* th, double* st) {
    Src s;
    source_from_theta(ev, th, s);
    const double fhi = ev.f_lo + (double)ev.K * ev.df;
    const double ftop = fmin(s.fisco, fhi);
    const double mc = th[0];
    const double phin = 3.0 / 128.0 * pow(kPi * mc * kTsun * ev.f_lo, -5.0 / 3.0);
    const double dmc = 1e-3 * mc / (5.0 / 3.0 * phin);
    const double dtc = 1e-3 / (kTwoPi * ftop);
    if (ev.params == PE_PARAMS_4D) {
        st[0] = dmc;
        st[1] = 1e-3 / phin;
        st[2] = 1e-3 / phin;
        st[3] = dtc;
    } else {
        const double sky = 1e-3 / (kTwoPi * ftop * kREarth / kC);
        st[0] = dmc;
        st[1] = st[2] = st[3] = 1e-3 / phin;
        st[4] = st[5] = sky;
        st[6] = st[7] = 1e-4;
        st[8] = 1e-4 * th[8];
        st[9] = dtc;
        st[10] = 0.0;
    }
}

// Sources of the stencil: index 0 = theta0, 2a+1 / 2a+2 = theta0 +/- step_a.
// One workgroup per event.
__global__ __launch_bounds__(32) void k_metric_setup(const BatchHdr* __restrict__ hdr,
                                                     const MetricArg* __restrict__ args) {
    const int ne = hdr->ne;
    const int t = threadIdx.x;
    __shared__ double st[PE_MAX_DIM];
    for (int e = blockIdx.x; e < ne; e += gridDim.x) {
        const MetricArg& A = args[e];
        const EvConst& ev = A.ec;
        const int D = ev.dim;
        double* mws = A.mws;
        double th0[PE_MAX_DIM];
#pragma unroll
        for (int a = 0; a < PE_MAX_DIM; ++a) th0[a] = (a < D) ? A.theta0[a] : 0.0;
        if (t == 0) {
            double s[PE_MAX_DIM];
            if (A.steps)
                for (int a = 0; a < D; ++a) s[a] = A.steps[a];
            else
                default_steps(ev, th0, s);
            for (int a = 0; a < D; ++a) {
                st[a] = s[a];
                mws[kMwsSteps + a] = s[a];
                const double tp = th0[a] + s[a], tm = th0[a] - s[a];
                mws[kMwsDen + a] = (tp - th0[a]) + (th0[a] - tm);
            }
            Src s0;
            source_from_theta(ev, th0, s0);
            mws[kMwsKcut] = (double)kcut_of(ev, s0.fisco);
        }
        __syncthreads();
        if (t < 2 * D + 1) {
            double th[PE_MAX_DIM];
#pragma unroll
            for (int a = 0; a < PE_MAX_DIM; ++a) th[a] = th0[a];
            if (t > 0) {
                const int a = (t - 1) / 2;
                th[a] = ((t - 1) % 2 == 0) ? th0[a] + st[a] : th0[a] - st[a];
            }
            Src s;
            source_from_theta(ev, th, s);
            PhaseCoef pc;
            phase_coeffs(s, pc);
            double* o = mws + kMwsSrc + (int64_t)t * kMetricSrcStride;
            for (int a = 0; a < 8; ++a) o[a] = pc.A[a];
            o[8] = pc.B5;
            o[9] = pc.B6;
            for (int d = 0; d < PE_MAX_DET; ++d) {
                o[10 + d] = s.rre[d];
                o[14 + d] = s.rim[d];
                o[18 + d] = s.tc + s.dt[d];
            }
        }
        __syncthreads();
    }
}

__device__ __forceinline__ void model_unit(const double* __restrict__ src, int d, const Rec64& r, double& hr,
                                           double& hi) {
    double A[8];
#pragma unroll
    for (int a = 0; a < 8; ++a) A[a] = src[a];
    const double ph = fma(r.f, src[18 + d], psi_turns(A, src[8], src[9], r.x, r.xm5, r.lnx));
    double sn, cs;
    sincos_turns(fract64(ph), sn, cs);
    const double rr = src[10 + d], ri = src[14 + d];
    // R (cos - i sin)
    hr = rr * cs + ri * sn;
    hi = ri * cs - rr * sn;
}

// Columns: coordinates 0..D-1 by central differences, except the phase column
// (index DP-1 in 4-D, 10 in 11-D), which is i h(theta0). Block lb of the
// event's nb blocks takes the tiles of kMetricTile bins lb, lb + nb, ... below
// the frozen cut, in two steps with the whole workgroup on each:
//   1. the derivative columns at every (bin, detector) of the tile, into LDS:
//      task (column, bin, detector) with the bins fastest, so that a wave reads
//      consecutive bin records and one source record;
//   2. the products: thread (q, part) owns matrix entry q of the packed upper
//      triangle and sums its weighted products over the bins part, part + NR, ...
// The NR partial sums of each entry are added in a fixed order at the end, so
// the block's partial does not depend on scheduling.
constexpr int kMetricTile = 32;

// Shared memory of the metric partial (one set for both parameter sets).
struct MetricLds {
    double ssrc[(2 * PE_MAX_DIM + 1) * kMetricSrcStride];  // the sources' records
    double2 us[kMetricTile * PE_MAX_DET * kMetricMaxDp];  // derivative columns
    double ps[kMetricTile * PE_MAX_DET];                  // 4 df / S
    double red[256];
};

template <int D, int DP>
__device__ __forceinline__ void metric_partial(const MetricArg& A, int lb, int nb, MetricLds& L) {
    constexpr int NG = DP * (DP + 1) / 2;
    constexpr int PH = (DP == D) ? D - 1 : D;  // phase column
    constexpr int NS = 2 * (DP - 1) + 1;       // sources 0 .. NS-1 (the phase column uses source 0)
    constexpr int NR = 256 / NG;               // threads per matrix entry
    const int t = threadIdx.x;
    const double* mws = A.mws;
    const int64_t kc = (int64_t)mws[kMwsKcut];
    const int64_t K = A.ec.K;
    const int nd = A.ec.n_det;
    for (int w = t; w < NS * kMetricSrcStride; w += 256) L.ssrc[w] = mws[kMwsSrc + w];
    // this thread's matrix entry (a, b), b >= a, and its share of the bins
    const int q = t % NG, part = t / NG;
    int qa = 0, qb = 0;
    {
        int r = q;
#pragma unroll
        for (int a = 0; a < DP; ++a) {
            const int len = DP - a;
            if (r >= 0 && r < len) {
                qa = a;
                qb = a + r;
            }
            r -= len;
        }
    }
    double acc = 0.0;
    __syncthreads();
    const int nbd = nd * kMetricTile;  // (bin, detector) pairs of a tile, detector-major
    for (int64_t k0 = (int64_t)lb * kMetricTile; k0 < kc; k0 += (int64_t)nb * kMetricTile) {
        // 1. derivative columns
#pragma unroll 1
        for (int w = t; w < nbd * DP; w += 256) {
            const int c = w / nbd, jd = w - c * nbd;
            const int j = jd % kMetricTile, d = jd / kMetricTile;
            const int64_t k = k0 + j;
            double2 u = make_double2(0.0, 0.0);
            if (k < kc) {
                const Rec64 r = A.tab[k];
                if (c == PH) {
                    double hr, hi;
                    model_unit(L.ssrc, d, r, hr, hi);
                    u = make_double2(-hi, hr);  // i h(theta0)
                } else {
                    double pr, pi_, mr, mi;
                    model_unit(L.ssrc + (2 * c + 1) * kMetricSrcStride, d, r, pr, pi_);
                    model_unit(L.ssrc + (2 * c + 2) * kMetricSrcStride, d, r, mr, mi);
                    const double den = mws[kMwsDen + c];
                    u = make_double2((pr - mr) / den, (pi_ - mi) / den);
                }
            }
            L.us[jd * DP + c] = u;
        }
        for (int w = t; w < nbd; w += 256) {
            const int j = w % kMetricTile, d = w / kMetricTile;
            const int64_t k = k0 + j;
            L.ps[w] = (k < kc) ? A.pw[(int64_t)d * K + k] : 0.0;
        }
        __syncthreads();
        // 2. products of this thread's entry over its bins
        if (part < NR) {
            for (int jd = part; jd < nbd; jd += NR) {
                const double2 ua = L.us[jd * DP + qa], ub = L.us[jd * DP + qb];
                acc = fma(L.ps[jd], ua.x * ub.x + ua.y * ub.y, acc);
            }
        }
        __syncthreads();
    }
    L.red[t] = acc;
    __syncthreads();
    if (t < NG) {
        double v = 0.0;
        for (int r = 0; r < NR; ++r) v += L.red[t + r * NG];
        A.mws[kMwsPart + (int64_t)lb * kMetricNG + t] = v;
    }
    __syncthreads();
}

// Blocks of every event (moff: block offsets); each dispatches on its
// event's parameter set (uniform across the workgroup).
__global__ __launch_bounds__(256) void k_metric_partial(const BatchHdr* __restrict__ hdr,
                                                        const MetricArg* __restrict__ args,
                                                        const int64_t* __restrict__ moff) {
    __shared__ MetricLds lds;
    const int ne = hdr->ne;
    const int64_t nblk = moff[ne];
    for (int64_t b = blockIdx.x; b < nblk; b += gridDim.x) {
        const int e = find_slot(moff, ne, b);
        const MetricArg& A = args[e];
        const int lb = (int)(b - moff[e]);
        const int nb = (int)(moff[e + 1] - moff[e]);
        if (A.ec.params == PE_PARAMS_4D)
            metric_partial<4, 5>(A, lb, nb, lds);
        else
            metric_partial<11, 11>(A, lb, nb, lds);
    }
}

// Fixed-order sum of the block partials (16 lanes per entry, each summing every
// 16th block, then a butterfly over the 16), phase projection (marginalised
// likelihood) and prior regularisation; one workgroup of 1024 per event.
__global__ __launch_bounds__(1024) void k_metric_final(const BatchHdr* __restrict__ hdr,
                                                       const MetricArg* __restrict__ args) {
    __shared__ double Gs[kMetricNG];
    const int ne = hdr->ne;
    const int t = threadIdx.x;
    const int sub = t & 15;
    for (int e = blockIdx.x; e < ne; e += gridDim.x) {
        const MetricArg& A = args[e];
        const EvConst& ev = A.ec;
        const int D = ev.dim;
        const int DP = (ev.params == PE_PARAMS_4D) ? 5 : 11;
        const int NG = DP * (DP + 1) / 2;
        const int nb = metric_blocks(ev.K);
        for (int q0 = 0; q0 < NG; q0 += 64) {
            const int q = q0 + (t >> 4);
            double acc = 0.0;
            if (q < NG)
                for (int b = sub; b < nb; b += 16) acc += A.mws[kMwsPart + (int64_t)b * kMetricNG + q];
#pragma unroll
            for (int o = 8; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 16);
            if (q < NG && sub == 0) Gs[q] = acc;
        }
        __syncthreads();
        // g_ab: one entry per thread, from the packed upper triangle (row a holds
        // b = a .. DP-1); marginalised phase: the Schur complement of the phase
        // coordinate PH; then the prior precision on the diagonal.
        const int PH = (DP == D) ? D - 1 : D;
        constexpr int DL = 8;  // distance coordinate (11-D)
        auto at = [&](int a, int b) {
            const int lo = min(a, b), hi = max(a, b);
            return Gs[lo * DP - lo * (lo - 1) / 2 + (hi - lo)];
        };
        const bool sp = (ev.phase == PE_PHASE_MARG);
        const bool sd = (ev.params == PE_PARAMS_11D) && ev.dist;
        if (t < D * D) {
            const int a = t / D, b = t - (t / D) * D;
            double m = at(a, b);
            // Schur complement of the projected coordinates: the phase for the
            // marginalised phase, dL for the marginalised distance, or both
            if ((sp && (a == PH || b == PH)) || (sd && (a == DL || b == DL))) {
                m = 0.0;
            } else if (sp && sd) {
                const double pp = at(PH, PH), pl = at(PH, DL), ll = at(DL, DL);
                const double det = pp * ll - pl * pl;
                m -= (at(a, DL) * (pp * at(DL, b) - pl * at(PH, b)) + at(a, PH) * (ll * at(PH, b) - pl * at(DL, b))) / det;
            } else if (sp) {
                m -= at(a, PH) * at(PH, b) / at(PH, PH);
            } else if (sd) {
                m -= at(a, DL) * at(DL, b) / at(DL, DL);
            }
            double reg = 0.0;
            if (a == b && !(A.flags & 1)) {
                if (ev.params == PE_PARAMS_4D) {
                    reg = (a == 1) ? 12.0 / 0.0625 : (a == 2) ? 3.0 / (ev.chi_max * ev.chi_max) : 0.0;
                } else {
                    const double p2 = 3.0 / (kPi * kPi);  // 12 / (2 pi)^2
                    const double p1 = 12.0 / (kPi * kPi);
                    switch (a) {
                        case 1: reg = 12.0; break;
                        case 2:
                        case 3: reg = 3.0 / (ev.chi_max * ev.chi_max); break;
                        case 4:
                        case 10: reg = p2; break;
                        case 5:
                        case 6:
                        case 7: reg = p1; break;
                        case 8: reg = 12.0 / (ev.dl_max * ev.dl_max); break;
                        default: reg = 0.0;
                    }
                }
            }
            A.g[a * D + b] = m + reg;
        }
        __syncthreads();
    }
}

hipError_t launch_metric_batch(const BatchPtrs& b, int ne, int64_t total_blocks, hipStream_t st) {
    if (ne <= 0) return hipSuccess;
    const MetricArg* args = (const MetricArg*)b.args;
    k_metric_setup<<<event_grid(ne), 32, 0, st>>>(b.hdr, args);
    k_metric_partial<<<stride_grid(total_blocks, 1, 8192), 256, 0, st>>>(b.hdr, args, b.off);
    k_metric_final<<<event_grid(ne), 1024, 0, st>>>(b.hdr, args);
    return hipGetLastError();
}

// ===========================================================================
// draws
// ===========================================================================
// Cholesky factor g = L L^T of one event's metric (row-major L), log det L and
// a success flag, in registers (D is a template constant).
template <int D>
__device__ __forceinline__ void cholesky_one(const DrawArg& A) {
    double g[D][D];
    double L[D][D];
    int ok = 1;
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) {
            L[i][j] = 0.0;
            g[i][j] = A.g[i * D + j];
        }
    // coordinates the likelihood does not use: dL (index 8) of a
    // distance-marginalised likelihood, phic (index 10) of an 11-D
    // phase-marginalised one; and those of dmask (tiled coordinates whose
    // values come from elsewhere). Each is decoupled by the Schur complement of
    // its row and column (its diagonal kept), in index order; the other
    // coordinates' distribution is unchanged and the drawn value is never used
    const bool dist = (D == 11) && A.ec.dist;
    const bool pmarg = (D == 11) && A.ec.phase == PE_PHASE_MARG;
    const bool tmarg = (D == 11) && A.ec.tm;
    const uint32_t dmask = (D == 11) ? (A.dmask & ~kDrawCond) : 0u;
    const bool cond = (D == 11) && (A.dmask & kDrawCond);
    if constexpr (D == 11) {
        // time-marginalised likelihood: tc is not drawn but set to its mean
        // given the other coordinates, from g_{tc,j} / g_{tc,tc} of g as given
#pragma unroll
        for (int j = 0; j < D; ++j) A.chol[kCholTm + j] = (tmarg && j != 9 && g[9][9] > 0.0) ? g[9][j] / g[9][9] : 0.0;
#pragma unroll
        for (int il = 0; il < D; ++il) {
            const bool dec = (((dmask >> il) & 1u) && !cond) || (il == 8 && dist) || (il == 9 && tmarg) ||
                             (il == 10 && pmarg);
            if (!dec) continue;
            const double gll = g[il][il];
            ok = ok && gll > 0.0;
            double cl[D];
#pragma unroll
            for (int i = 0; i < D; ++i) cl[i] = g[i][il];
#pragma unroll
            for (int i = 0; i < D; ++i)
#pragma unroll
                for (int j = 0; j < D; ++j)
                    g[i][j] = (i == il || j == il) ? ((i == j) ? gll : 0.0) : (ok ? g[i][j] - cl[i] * cl[j] / gll : g[i][j]);
        }
        if (cond) {
            // conditioning on the tiled coordinates: their coupling to the others
            // kept for the draws' mean shift, then their rows and columns cleared
#pragma unroll
            for (int i = 0; i < D; ++i)
#pragma unroll
                for (int j = 0; j < D; ++j) {
                    const bool ti = (dmask >> i) & 1u, tj = (dmask >> j) & 1u;
                    A.chol[kCholCond + i * D + j] = (!ti && tj) ? g[i][j] : 0.0;
                    if ((ti || tj) && i != j) g[i][j] = 0.0;
                }
        }
    }
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j <= i; ++j) {
            double s = g[i][j];
#pragma unroll
            for (int k = 0; k < j; ++k) s -= L[i][k] * L[j][k];
            if (i == j) {
                ok = ok && (s > 0.0);
                L[i][i] = ok ? sqrt(s) : 1.0;
            } else {
                L[i][j] = s / L[j][j];
            }
        }
    double logdet = 0.0;
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) A.chol[i * D + j] = ok ? L[i][j] : 0.0;
    // log det of the factor of the density log q reports: without the decoupled
    // coordinates' L_ii (the marginal over them)
    if (ok)
#pragma unroll
        for (int a = 0; a < D; ++a)
            if (!(dist && a == 8) && !(tmarg && a == 9) && !(pmarg && a == 10) && !((dmask >> a) & 1u))
                logdet += log(L[a][a]);
    A.chol[kCholLogdet] = logdet;
    A.chol[kCholOk] = ok ? 1.0 : 0.0;
#pragma unroll
    for (int a = 0; a < D; ++a) A.chol[kCholRdiag + a] = ok ? 1.0 / L[a][a] : 0.0;
    // (L L^T) at the periodic coordinates (11-D: ra, psi, phic), for the image sum of log q
    if constexpr (D == 11) {
        constexpr int pidx[3] = {4, 7, 10};
        int w = 0;
#pragma unroll
        for (int p = 0; p < 3; ++p)
#pragma unroll
            for (int q = p; q < 3; ++q) {
                double gpq = 0.0;
#pragma unroll
                for (int r = 0; r < D; ++r) gpq += L[pidx[p]][r] * L[pidx[q]][r];
                A.chol[kCholG + w++] = ok ? gpq : 0.0;
            }
    }
    if (!ok) atomicOr(A.status, kStSingular);
}

// One thread per event.
__global__ __launch_bounds__(64) void k_cholesky(const BatchHdr* __restrict__ hdr, const DrawArg* __restrict__ args) {
    const int ne = hdr->ne;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < ne; e += gridDim.x * blockDim.x) {
        const DrawArg& A = args[e];
        if (A.ec.dim == 4)
            cholesky_one<4>(A);
        else
            cholesky_one<11>(A);
    }
}

// ln of the proposal's wrapped Gaussian density (images -2..2 of each periodic
// coordinate about the wrapped centre, summed with a running maximum) for a
// point whose whitened offset from the centre is z = L^T (theta - theta0) (D
// entries) and which lies k0_p whole periods from the wrapped centre's cell at
// the periodic coordinates. L (row-major), log det, G and the success flag are
// in lc. The decoupled coordinates (marginalised by the likelihood, or in dmask)
// are left out: the density is the marginal over the others.
template <int D>
__device__ __forceinline__ double wrapped_logq(const EvConst& ev, const double* lc, const double* z, double (&k0)[3],
                                               uint32_t dmask) {
    constexpr int NP = (D == 4) ? 0 : 3;
    constexpr int pidx[3] = {4, 7, 10};
    const double per[3] = {kTwoPi, kPi, kTwoPi};
    const bool tmarg = (D == 11) && ev.tm;
    // whitened offset of image m: L^T (x - c) = z + L^T s with c the wrapped
    // centre and s = (k - k0) P on the periodic rows, so its squared norm is
    // |z|^2 + 2 s.a + s^T G s with a_p = (L^T row pidx_p) . z and G = L L^T there.
    // Decoupled coordinates (dL of a distance-marginalised likelihood, phic of an
    // 11-D phase-marginalised one): their normals move them alone and log q is
    // the marginal over them (their z and, for phic, its images left out).
    const bool dist = (D == 11) && ev.dist;
    const bool pmarg = (D == 11) && ev.phase == PE_PHASE_MARG;
    double zz = 0.0;
#pragma unroll
    for (int r = 0; r < D; ++r)
        if (!(dist && r == 8) && !(tmarg && r == 9) && !(pmarg && r == 10) && !((dmask >> r) & 1u))
            zz = fma(z[r], z[r], zz);
    double a[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int r = 0; r <= pidx[p]; ++r) a[p] = fma(lc[pidx[p] * D + r], z[r], a[p]);
    const double* G = lc + kCholG;  // G00 G01 G02 G11 G12 G22
    // images of phic: all five, or only k = k0 (no shift) when it is marginalised
    const int t2lo = pmarg ? 2 : 0, t2hi = pmarg ? 2 : 4;
    if (pmarg) k0[2] = 0.0;
    double mx = -INFINITY, acc = 0.0;
    if constexpr (NP == 3) {
        // Factorised image sum. With image k = (t_0, t_1, t_2), t in {-2..2}
        // and o_p = -k0_p P_p, the shift is s_p = P_p t_p + o_p and
        //   -qf/2 = -C/2 + sum_p v_p(t_p) - sum_{p<q} gam_pq t_p t_q,
        //   C = |z|^2 + 2 o.a + o^T G o,  v_p(t) = -P_p t b_p - G_pp P_p^2 t^2 / 2,
        //   b = a + G o,  gam_pq = G_pq P_p P_q,
        // so each of the 125 terms is a product of three per-coordinate factors
        // exp(v_p - V_p) <= 1 (V_p their largest exponent) and three pair
        // factors exp(-gam t_p t_q), t_p t_q in -4..4: 15 + 6 exponentials instead
        // of 125. Taken when every |gam| <= 50, so that the pair factors stay
        // within e^+-200 (a condition on the event's metric, uniform over the
        // workgroup).
        const double g00 = G[0], g01 = G[1], g02 = G[2], g11 = G[3], g12 = G[4], g22 = G[5];
        const double gam01 = g01 * per[0] * per[1], gam02 = g02 * per[0] * per[2], gam12 = g12 * per[1] * per[2];
        if (fabs(gam01) <= 50.0 && fabs(gam02) <= 50.0 && fabs(gam12) <= 50.0) {
            const double o0 = -k0[0] * per[0], o1 = -k0[1] * per[1], o2 = -k0[2] * per[2];
            const double go0 = g00 * o0 + g01 * o1 + g02 * o2;
            const double go1 = g01 * o0 + g11 * o1 + g12 * o2;
            const double go2 = g02 * o0 + g12 * o1 + g22 * o2;
            const double C = zz + 2.0 * (o0 * a[0] + o1 * a[1] + o2 * a[2]) + (o0 * go0 + o1 * go1 + o2 * go2);
            const double b[3] = {a[0] + go0, a[1] + go1, a[2] + go2};
            const double gpp[3] = {g00, g11, g22};
            // phic marginalised: its only image is t_2 = 0 (index 2), whose
            // factor is exp(0) = 1 and whose pair factors are exp(0) = 1
            const int np = pmarg ? 2 : 3;
            double f[3][5], V = 0.0;
#pragma unroll
            for (int p = 0; p < 3; ++p) {
                if (p >= np) break;
                const double h = -0.5 * gpp[p] * per[p] * per[p];
                double v[5], Vp = -INFINITY;
#pragma unroll
                for (int t = 0; t < 5; ++t) {
                    const double tt = (double)(t - 2);
                    v[t] = -per[p] * tt * b[p] + h * tt * tt;
                    Vp = fmax(Vp, v[t]);
                }
#pragma unroll
                for (int t = 0; t < 5; ++t) f[p][t] = exp(v[t] - Vp);
                V += Vp;
            }
            // x_pq[j] = exp(-gam_pq (j - 4)), j - 4 = t_p t_q in -4..4
            double x01[9];
            const double e01 = exp(-gam01), i01 = 1.0 / e01;
            x01[4] = 1.0;
#pragma unroll
            for (int j = 1; j <= 4; ++j) x01[4 + j] = x01[3 + j] * e01;
#pragma unroll
            for (int j = 1; j <= 4; ++j) x01[4 - j] = x01[5 - j] * i01;
            if (pmarg) {
                // sum over t_0, t_1 of f_0 f_1 x01, nested over t_1
#pragma unroll
                for (int t0 = 0; t0 < 5; ++t0) {
                    double s1 = 0.0;
#pragma unroll
                    for (int t1 = 0; t1 < 5; ++t1) s1 = fma(f[1][t1], x01[4 + (t0 - 2) * (t1 - 2)], s1);
                    acc = fma(f[0][t0], s1, acc);
                }
            } else {
                double x02[9], x12[9];
                const double e02 = exp(-gam02), e12 = exp(-gam12);
                x02[4] = x12[4] = 1.0;
#pragma unroll
                for (int j = 1; j <= 4; ++j) {
                    x02[4 + j] = x02[3 + j] * e02;
                    x12[4 + j] = x12[3 + j] * e12;
                }
                const double i02 = 1.0 / e02, i12 = 1.0 / e12;
#pragma unroll
                for (int j = 1; j <= 4; ++j) {
                    x02[4 - j] = x02[5 - j] * i02;
                    x12[4 - j] = x12[5 - j] * i12;
                }
                // nested: for each t_0, y(t_2) = f_2 x02; for each t_1 the sum over
                // t_2 of y x12, weighted by f_1 x01; then by f_0
#pragma unroll
                for (int t0 = 0; t0 < 5; ++t0) {
                    double y[5];
#pragma unroll
                    for (int t2 = 0; t2 < 5; ++t2) y[t2] = f[2][t2] * x02[4 + (t0 - 2) * (t2 - 2)];
                    double s1 = 0.0;
#pragma unroll
                    for (int t1 = 0; t1 < 5; ++t1) {
                        double s2 = 0.0;
#pragma unroll
                        for (int t2 = 0; t2 < 5; ++t2) s2 = fma(y[t2], x12[4 + (t1 - 2) * (t2 - 2)], s2);
                        s1 = fma(f[1][t1] * x01[4 + (t0 - 2) * (t1 - 2)], s2, s1);
                    }
                    acc = fma(f[0][t0], s1, acc);
                }
            }
            mx = -0.5 * C + V;
        }
    }
    const int nimg = (NP == 0) ? 1 : 25 * (t2hi - t2lo + 1);
#pragma unroll 1
    for (int m = (acc > 0.0) ? nimg : 0; m < nimg; ++m) {
        double qf = zz;
        if (NP == 3) {
            const int t0 = m % 5, t1 = (m / 5) % 5, t2 = t2lo + m / 25;
            const double s0 = ((double)(t0 - 2) - k0[0]) * per[0];
            const double s1 = ((double)(t1 - 2) - k0[1]) * per[1];
            const double s2 = ((double)(t2 - 2) - k0[2]) * per[2];
            const double lin = s0 * a[0] + s1 * a[1] + s2 * a[2];
            const double quad = s0 * (s0 * G[0] + 2.0 * (s1 * G[1] + s2 * G[2])) +
                                s1 * (s1 * G[3] + 2.0 * s2 * G[4]) + s2 * s2 * G[5];
            qf = zz + 2.0 * lin + quad;
        }
        // exp of anything below -800 is exactly zero in FP64: skip those terms
        const double l = -0.5 * qf;
        if (l > mx) {
            const double dl = mx - l;
            acc = (dl < -800.0) ? 1.0 : acc * exp(dl) + 1.0;
            mx = l;
        } else if (l - mx >= -800.0) {
            acc += exp(l - mx);
        }
    }
    const uint32_t margm = (dist ? 1u << 8 : 0u) | (tmarg ? 1u << 9 : 0u) | (pmarg ? 1u << 10 : 0u);
    const int dkeep = D - __builtin_popcount(margm | dmask);
    return mx + log(acc) + lc[kCholLogdet] - 0.5 * dkeep * log(kTwoPi);
}

// Draw i of an event: normals, theta = theta0 + L^-T z (wrapped), log q of the
// wrapped Gaussian (images -2..2 of each periodic coordinate about theta0
// wrapped into [0, P), summed with a running maximum), log prior. L
// (row-major), its log det and the success flag are in LDS (lc).
//
// Ext (extrinsic completion of tile draws): the coordinates of A.dmask keep the
// values theta holds on entry, log q is added to the entry's value, and the log
// prior stays -inf where it was.
//
// Ext with kDrawCond: the other coordinates given the tiled ones. With L the
// factor of the metric conditioned on them (their rows cleared after the
// marginalised coordinates are decoupled), the draw's mean moves by
// delta = -(L L^T)^-1 r, r = (coupling) (theta_tiled - theta0_tiled): u = -L^-1 r,
// delta = L^-T u; theta = theta0 + delta + L^-T z, and log q is the wrapped
// density about theta0 + delta (the whitened offset is z again).
template <int D, bool Ext = false>
__device__ __forceinline__ void draw_one(const DrawArg& A, const double* lc, int64_t i) {
    const EvConst& ev = A.ec;
    const int64_t n = A.n;
    const uint32_t dmask = Ext ? (A.dmask & ~kDrawCond) : 0u;
    const bool cond = Ext && (A.dmask & kDrawCond);
    double th0[D];
#pragma unroll
    for (int a = 0; a < D; ++a) th0[a] = A.theta0[a];
    if (lc[kCholOk] == 0.0) {
        if (!Ext) {
#pragma unroll
            for (int a = 0; a < D; ++a) A.theta[(int64_t)a * n + i] = th0[a];
            A.logq[i] = 0.0;
        }
        A.logprior[i] = -INFINITY;
        return;
    }
    double z[D + 1];
#pragma unroll
    for (int j = 0; 2 * j < D; ++j) {
        double ua, ub, sn, cs;
        block_uniforms(A.seed, A.stream_id, (uint64_t)i, (uint32_t)j, ua, ub);
        const double rad = sqrt(-2.0 * log(ua));
        sincos_turns(ub >= 1.0 ? 0.0 : ub, sn, cs);  // 2 pi ub
        z[2 * j] = rad * cs;
        z[2 * j + 1] = rad * sn;
    }
    // theta = theta0 + L^-T z (back substitution with L^T)
    double y[D];
#pragma unroll
    for (int r = D - 1; r >= 0; --r) {
        double s = z[r];
#pragma unroll
        for (int c = r + 1; c < D; ++c) s -= lc[c * D + r] * y[c];
        y[r] = s * lc[kCholRdiag + r];
    }
    const bool distm = (D == 11) && ev.dist, pmargm = (D == 11) && ev.phase == PE_PHASE_MARG;
    double yu[D];  // the conditional mean's shift (0 unless cond)
#pragma unroll
    for (int a = 0; a < D; ++a) yu[a] = 0.0;
    if (cond) {
        double u[D];
#pragma unroll
        for (int r = 0; r < D; ++r) {
            double t = 0.0;
#pragma unroll
            for (int j = 0; j < D; ++j)
                if ((dmask >> j) & 1u) t = fma(lc[kCholCond + r * D + j], A.theta[(int64_t)j * n + i] - th0[j], t);
            double sr = -t;
#pragma unroll
            for (int k = 0; k < r; ++k) sr -= lc[r * D + k] * u[k];
            u[r] = sr * lc[kCholRdiag + r];
        }
#pragma unroll
        for (int r = D - 1; r >= 0; --r) {
            double sr = u[r];
#pragma unroll
            for (int c = r + 1; c < D; ++c) sr -= lc[c * D + r] * yu[c];
            yu[r] = sr * lc[kCholRdiag + r];
        }
    }
    double th[D];
#pragma unroll
    for (int a = 0; a < D; ++a) {
        const bool margd = (a == 8 && distm) || (a == 10 && pmargm);  // unused by the likelihood
        th[a] = ((dmask >> a) & 1u) ? A.theta[(int64_t)a * n + i]
                                    : ((cond && margd) ? th0[a] : th0[a] + yu[a] + y[a]);
    }
    constexpr int NP = (D == 4) ? 0 : 3;
    constexpr int pidx[3] = {4, 7, 10};
    const double per[3] = {kTwoPi, kPi, kTwoPi};
    // k0_p: periods between the wrapped draw and the wrapped centre
    double k0[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        const double v = th[pidx[p]];
        const double kw = floor(v / per[p]);
        th[pidx[p]] = v - per[p] * kw;
        k0[p] = kw - floor((th0[pidx[p]] + yu[pidx[p]]) / per[p]);
    }
    const bool tmarg = (D == 11) && ev.tm;
    if (tmarg) {
        // tc: its mean under the proposal given the other coordinates, from
        // their offsets to the wrapped centre (periodic ones to the nearest image)
        double dlt[D];
#pragma unroll
        for (int a = 0; a < D; ++a) dlt[a] = th[a] - th0[a];
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            const double c0 = th0[pidx[p]] - per[p] * floor(th0[pidx[p]] / per[p]);
            const double d = th[pidx[p]] - c0;
            dlt[pidx[p]] = d - per[p] * floor(d / per[p] + 0.5);
        }
        double m = th0[9 % D];
#pragma unroll
        for (int a = 0; a < D; ++a)
            if (a != 9) m -= lc[kCholTm + a] * dlt[a];
        th[9 % D] = m;
    }
#pragma unroll
    for (int a = 0; a < D; ++a) A.theta[(int64_t)a * n + i] = th[a];
    const double lq = wrapped_logq<D>(ev, lc, z, k0, dmask);
    if (Ext) {
        A.logq[i] += lq;
        if (A.logprior[i] != -INFINITY) A.logprior[i] = log_prior_of(ev, th);
    } else {
        A.logq[i] = lq;
        A.logprior[i] = log_prior_of(ev, th);
    }
}

// Blocks of 256 draws that each belong to one event (doff: block offsets).
// At least 3 workgroups per CU: the register budget of 3 waves per SIMD (a few
// registers spill; without the bound the compiler takes 211 and runs 2 waves).
__global__ __launch_bounds__(256, 3) void k_draw(const BatchHdr* __restrict__ hdr, const DrawArg* __restrict__ args,
                                              const int64_t* __restrict__ doff) {
    __shared__ double lc[kCholLen];
    const int ne = hdr->ne;
    const int64_t nblk = doff[ne];
    for (int64_t b = blockIdx.x; b < nblk; b += gridDim.x) {
        const int e = find_slot(doff, ne, b);
        const DrawArg& A = args[e];
        __syncthreads();  // the previous block's readers are done with lc
        for (int q = threadIdx.x; q < kCholLen; q += 256) lc[q] = A.chol[q];
        __syncthreads();
        const int64_t i = (b - doff[e]) * 256 + threadIdx.x;
        if (i < A.n) {
            if (A.ec.dim == 4)
                draw_one<4>(A, lc, i);
            else
                draw_one<11>(A, lc, i);
        }
    }
}

// The extrinsic completion of tile draws (11-D events, draw_one<11, true>).
__global__ __launch_bounds__(256, 3) void k_draw_ext(const BatchHdr* __restrict__ hdr,
                                                  const DrawArg* __restrict__ args, const int64_t* __restrict__ doff) {
    __shared__ double lc[kCholLen];
    const int ne = hdr->ne;
    const int64_t nblk = doff[ne];
    for (int64_t b = blockIdx.x; b < nblk; b += gridDim.x) {
        const int e = find_slot(doff, ne, b);
        const DrawArg& A = args[e];
        __syncthreads();
        for (int q = threadIdx.x; q < kCholLen; q += 256) lc[q] = A.chol[q];
        __syncthreads();
        const int64_t i = (b - doff[e]) * 256 + threadIdx.x;
        if (i < A.n && A.ec.dim == 11) draw_one<11, true>(A, lc, i);
    }
}

hipError_t launch_draw_batch(const BatchPtrs& b, int ne, int64_t total_blocks, hipStream_t st, bool ext) {
    if (ne <= 0) return hipSuccess;
    const DrawArg* args = (const DrawArg*)b.args;
    k_cholesky<<<stride_grid(ne, 64), 64, 0, st>>>(b.hdr, args);
    if (ext)
        k_draw_ext<<<stride_grid(total_blocks, 1), 256, 0, st>>>(b.hdr, args, b.off);
    else
        k_draw<<<stride_grid(total_blocks, 1), 256, 0, st>>>(b.hdr, args, b.off);
    return hipGetLastError();
}

// ===========================================================================
// Mixture log-density: ln sum_k pi_k q_k(theta) at given points, q_k the
// wrapped density of component k (its factor from k_cholesky, as for pe_draw).
// For point theta and centre c_k wrapped into [0, P): z = L_k^T (theta - c_k)
// and k0 = 0 (the images are taken about the wrapped centre), then q_k as
// draw_one evaluates it (wrapped_logq); components in order, running maximum.
// ===========================================================================
constexpr int kMixRec = kCholRdiag;  // the part of a component's record the density reads

template <int D>
__device__ __forceinline__ void mix_one(const MixArg& A, const double* lc_all, const double* cen_all, int64_t i) {
    const int64_t n = A.n;
    double th[D];
#pragma unroll
    for (int a = 0; a < D; ++a) th[a] = A.theta[(int64_t)a * n + i];
    double mx = -INFINITY, acc = 0.0;
    bool bad = false;
    for (int k = 0; k < A.m; ++k) {
        const double lpi = A.lpi[k];
        if (lpi == -INFINITY) continue;
        const double* lc = lc_all + k * kMixRec;
        if (lc[kCholOk] == 0.0) {
            bad = true;
            continue;
        }
        const double* c = cen_all + k * PE_MAX_DIM;
        double dl[D], z[D];
#pragma unroll
        for (int a = 0; a < D; ++a) dl[a] = th[a] - c[a];
#pragma unroll
        for (int r = 0; r < D; ++r) {
            double t = 0.0;
#pragma unroll
            for (int a = r; a < D; ++a) t = fma(lc[a * D + r], dl[a], t);
            z[r] = t;
        }
        double k0[3] = {0.0, 0.0, 0.0};
        const double l = lpi + wrapped_logq<D>(A.ec, lc, z, k0, 0u);
        if (l > mx) {
            acc = (mx == -INFINITY) ? 1.0 : acc * exp(mx - l) + 1.0;
            mx = l;
        } else if (l > -INFINITY) {
            acc += exp(l - mx);
        }
    }
    A.logq[i] = bad ? NAN : ((mx == -INFINITY) ? -INFINITY : mx + log(acc));
}

// Blocks of 256 points; every block stages the components' records and wrapped
// centres in LDS.
template <int D>
__global__ __launch_bounds__(256) void k_mix_logq(MixArg A) {
    __shared__ double lc[PE_MIX_MAX * kMixRec];
    __shared__ double cen[PE_MIX_MAX * PE_MAX_DIM];
    for (int q = threadIdx.x; q < A.m * kMixRec; q += 256) {
        const int k = q / kMixRec, r = q - k * kMixRec;
        lc[q] = A.chol[(int64_t)k * kCholLen + r];
    }
    for (int q = threadIdx.x; q < A.m * PE_MAX_DIM; q += 256) {
        const int k = q / PE_MAX_DIM, a = q - k * PE_MAX_DIM;
        double v = (a < D) ? A.theta0[k * D + a] : 0.0;
        if (D == 11 && (a == 4 || a == 7 || a == 10)) {
            const double P = (a == 7) ? kPi : kTwoPi;
            v -= P * floor(v / P);
        }
        cen[q] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        for (int k = 0; k < A.m; ++k)
            if (A.lpi[k] != -INFINITY && lc[k * kMixRec + kCholOk] == 0.0) {
                atomicOr(A.status, kStSingular);
                break;
            }
    }
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < A.n; i += (int64_t)gridDim.x * 256)
        mix_one<D>(A, lc, cen, i);
}

hipError_t launch_mix_logq(const MixArg& a, hipStream_t st) {
    if (a.n <= 0) return hipSuccess;
    const unsigned grid = stride_grid((a.n + 255) / 256, 1);
    if (a.ec.dim == 4)
        k_mix_logq<4><<<grid, 256, 0, st>>>(a);
    else
        k_mix_logq<11><<<grid, 256, 0, st>>>(a);
    return hipGetLastError();
}

// ===========================================================================
// weights and ESS: ln w = ln L + ln prior - ln q; per block of kWBlock draws
// its max and the sums of exp(ln w - max) and exp(2 (ln w - max)); per event
// the blocks combined in a fixed order; then the normalised weights.
// ===========================================================================
__device__ __forceinline__ void neumaier(double& s, double& c, double x) {
    const double t = s + x;
    if (fabs(s) >= fabs(x))
        c += (s - t) + x;
    else
        c += (x - t) + s;
    s = t;
}

__device__ __forceinline__ double block_max256(double v, double* sh) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    const double r = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
    __syncthreads();
    return r;
}

__device__ __forceinline__ double block_sum256(double v, double* sh) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    const double r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
    __syncthreads();
    return r;
}

// part[b] = {max, sum exp(l - max), sum exp(2 (l - max)), finite count}; a
// block holding a NaN or +inf log-weight (no weight defined) gets max = NaN.
__global__ __launch_bounds__(256) void k_w_part(const BatchHdr* __restrict__ hdr, const WeightArg* __restrict__ args,
                                                const int64_t* __restrict__ boff, double4* __restrict__ part) {
    __shared__ double sh[4];
    const int ne = hdr->ne;
    const int64_t nblk = boff[ne];
    for (int64_t b = blockIdx.x; b < nblk; b += gridDim.x) {
        const int e = find_slot(boff, ne, b);
        const WeightArg& A = args[e];
        const int64_t i0 = (b - boff[e]) * kWBlock;
        double l[kWBlock / 256];
        double m = -INFINITY, cnt = 0.0, bad = 0.0;
#pragma unroll
        for (int j = 0; j < kWBlock / 256; ++j) {
            const int64_t i = i0 + threadIdx.x + 256 * j;
            double v = -INFINITY;
            if (i < A.n) v = A.ll[i] + A.lp[i] - A.lq[i];
            if (!isfinite(v)) {
                if (!(v == -INFINITY)) bad += 1.0;
                v = -INFINITY;
            }
            l[j] = v;
            if (v > -INFINITY) {
                m = fmax(m, v);
                cnt += 1.0;
            }
        }
        const double M = block_sum256(bad, sh) > 0.0 ? NAN : block_max256(m, sh);
        double s1 = 0.0, s2 = 0.0;
        if (M > -INFINITY) {  // false for NaN
#pragma unroll
            for (int j = 0; j < kWBlock / 256; ++j) {
                if (l[j] > -INFINITY) {
                    const double x = exp(l[j] - M);
                    s1 += x;
                    s2 += x * x;
                }
            }
        }
        const double S1 = block_sum256(s1, sh);
        const double S2 = block_sum256(s2, sh);
        const double C = block_sum256(cnt, sh);
        if (threadIdx.x == 0) part[b] = make_double4(M, S1, S2, C);
    }
}

// Per event: combine its blocks in index order; stats and {max, 1/S1} for the
// normalisation.
__global__ __launch_bounds__(256) void k_w_final(const BatchHdr* __restrict__ hdr, const WeightArg* __restrict__ args,
                                                 const int64_t* __restrict__ boff, const double4* __restrict__ part,
                                                 double2* __restrict__ fin) {
    __shared__ double sh[4];
    const int ne = hdr->ne;
    for (int e = blockIdx.x; e < ne; e += gridDim.x) {
        const WeightArg& A = args[e];
        const int64_t b0 = boff[e], b1 = boff[e + 1];
        double m = -INFINITY, bad = 0.0, cnt = 0.0;
        for (int64_t b = b0 + threadIdx.x; b < b1; b += 256) {
            const double4 p = part[b];
            cnt += p.w;
            if (isnan(p.x)) bad += 1.0;
            else m = fmax(m, p.x);
        }
        const double nbad = block_sum256(bad, sh);
        const double M = nbad > 0.0 ? -INFINITY : block_max256(m, sh);
        double a = 0.0, ac = 0.0, q = 0.0, qc = 0.0;
        if (M > -INFINITY) {
            for (int64_t b = b0 + threadIdx.x; b < b1; b += 256) {
                const double4 p = part[b];
                if (p.x > -INFINITY) {
                    const double r = exp(p.x - M);
                    neumaier(a, ac, p.y * r);
                    neumaier(q, qc, p.z * (r * r));
                }
            }
        }
        const double S1 = block_sum256(a + ac, sh);
        const double S2 = block_sum256(q + qc, sh);
        const double nin = block_sum256(cnt, sh);
        if (threadIdx.x == 0) {
            if (nbad > 0.0) {  // an undefined log-weight: every estimate is NaN
                A.stats[0] = NAN;
                A.stats[1] = NAN;
                A.stats[2] = NAN;
                A.stats[3] = nin;
                fin[e] = make_double2(NAN, NAN);
            } else if (nin == 0.0) {
                A.stats[0] = 0.0;
                A.stats[1] = -INFINITY;
                A.stats[2] = -INFINITY;
                A.stats[3] = 0.0;
                fin[e] = make_double2(0.0, 0.0);
            } else {
                A.stats[0] = S1 * S1 / S2;
                A.stats[1] = M + log(S1) - log((double)A.n);
                A.stats[2] = M;
                A.stats[3] = nin;
                fin[e] = make_double2(M, 1.0 / S1);
            }
        }
    }
}

// Blocks of 256 draws that each belong to one event (doff: block offsets).
__global__ __launch_bounds__(256) void k_w_norm(const BatchHdr* __restrict__ hdr, const WeightArg* __restrict__ args,
                                                const int64_t* __restrict__ doff, const double2* __restrict__ fin) {
    const int ne = hdr->ne;
    const int64_t nblk = doff[ne];
    for (int64_t b = blockIdx.x; b < nblk; b += gridDim.x) {
        const int e = find_slot(doff, ne, b);
        const WeightArg& A = args[e];
        const int64_t i = (b - doff[e]) * 256 + threadIdx.x;
        if (!A.w || i >= A.n) continue;
        const double l = A.ll[i] + A.lp[i] - A.lq[i];
        const double2 f = fin[e];
        A.w[i] = isnan(f.x) ? NAN : (isfinite(l) && f.y > 0.0) ? exp(l - f.x) * f.y : 0.0;
    }
}

hipError_t launch_weights_batch(const BatchPtrs& b, int ne, int64_t total_blocks, int64_t total_draw_blocks,
                                hipStream_t st) {
    if (ne <= 0) return hipSuccess;
    const WeightArg* args = (const WeightArg*)b.args;
    double4* part = (double4*)b.scratch;
    double2* fin = (double2*)(part + (total_blocks > 0 ? total_blocks : 1));
    k_w_part<<<stride_grid(total_blocks, 1, 8192), 256, 0, st>>>(b.hdr, args, b.off, part);
    k_w_final<<<event_grid(ne), 256, 0, st>>>(b.hdr, args, b.off, part, fin);
    k_w_norm<<<stride_grid(total_draw_blocks, 1), 256, 0, st>>>(b.hdr, args, b.off2, fin);
    return hipGetLastError();
}

// ===========================================================================
// proposal update: weighted centre and covariance of the draws about theta0,
// periodic offsets taken to the nearest image. Per block of kWBlock draws of
// one event: sums of w, w d_a, w d_a d_b (a <= b), each thread over its draws
// in order, then a wave shuffle tree and the four waves in a fixed order; per
// event the blocks are combined in order.
// ===========================================================================
__device__ __forceinline__ double update_period(int params, int a) {
    if (params == PE_PARAMS_4D) return 0.0;
    return (a == 4 || a == 10) ? kTwoPi : (a == 7) ? kPi : 0.0;
}

template <int D>
__device__ __forceinline__ void update_part(const UpdateArg& A, int64_t i0, int64_t i1, double* sh,
                                            double* __restrict__ out) {
    constexpr int NQ = 1 + D + D * (D + 1) / 2;
    double acc[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
    double th0[D], per[D];
#pragma unroll
    for (int a = 0; a < D; ++a) {
        th0[a] = A.th0[a];
        per[a] = update_period(A.params, a);
    }
    for (int64_t i = i0 + threadIdx.x; i < i1; i += 256) {
        const double w = A.w[i];
        if (!(w > 0.0)) continue;
        double d[D];
#pragma unroll
        for (int a = 0; a < D; ++a) {
            double v = A.theta[(int64_t)a * A.n + i] - th0[a];
            if (per[a] > 0.0) v -= per[a] * floor(v / per[a] + 0.5);
            d[a] = v;
        }
        acc[0] += w;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            const double wd = w * d[a];
            acc[1 + a] += wd;
#pragma unroll
            for (int b = a; b < D; ++b) acc[1 + D + a * D - a * (a - 1) / 2 + (b - a)] += wd * d[b];
        }
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        double v = acc[q];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
        if (lane == 0) sh[wv * kUpdNQ + q] = v;
    }
    __syncthreads();
    for (int q = threadIdx.x; q < NQ; q += 256)
        out[q] = (sh[q] + sh[kUpdNQ + q]) + (sh[2 * kUpdNQ + q] + sh[3 * kUpdNQ + q]);
    __syncthreads();
}

__global__ __launch_bounds__(256) void k_u_part(const BatchHdr* __restrict__ hdr, const UpdateArg* __restrict__ args,
                                                const int64_t* __restrict__ boff, double* __restrict__ part) {
    __shared__ double sh[4 * kUpdNQ];
    const int ne = hdr->ne;
    const int64_t nblk = boff[ne];
    for (int64_t b = blockIdx.x; b < nblk; b += gridDim.x) {
        const int e = find_slot(boff, ne, b);
        const UpdateArg& A = args[e];
        const int64_t i0 = (b - boff[e]) * kWBlock;
        const int64_t i1 = min(i0 + kWBlock, A.n);
        if (A.dim == 4)
            update_part<4>(A, i0, i1, sh, part + b * kUpdNQ);
        else
            update_part<11>(A, i0, i1, sh, part + b * kUpdNQ);
    }
}

// One workgroup per event: block sums in order, then centre and covariance.
// theta0 is read into shared memory before anything is written, so the
// output may overwrite it.
__global__ __launch_bounds__(256) void k_u_final(const BatchHdr* __restrict__ hdr, const UpdateArg* __restrict__ args,
                                                 const int64_t* __restrict__ boff, const double* __restrict__ part) {
    __shared__ double S[kUpdNQ];
    __shared__ double c0[PE_MAX_DIM], m[PE_MAX_DIM];
    const int ne = hdr->ne;
    const int t = threadIdx.x;
    for (int e = blockIdx.x; e < ne; e += gridDim.x) {
        const UpdateArg& A = args[e];
        const int D = A.dim;
        const int NQ = 1 + D + D * (D + 1) / 2;
        if (t < NQ) {
            double acc = 0.0;
            for (int64_t b = boff[e]; b < boff[e + 1]; ++b) acc += part[b * kUpdNQ + t];
            S[t] = acc;
        }
        if (t < D) c0[t] = A.th0[t];
        __syncthreads();
        const double W = S[0];
        if (t < D) {
            const double mt = (W > 0.0) ? S[1 + t] / W : 0.0;
            m[t] = mt;
            double c = c0[t] + mt;
            const double P = update_period(A.params, t);
            if (W > 0.0 && P > 0.0) c -= P * floor(c / P);
            A.th0_out[t] = (W > 0.0) ? c : c0[t];
        }
        __syncthreads();
        if (A.cov && t < D * D) {
            const int a = t / D, b = t - (t / D) * D;
            const int lo = min(a, b), hi = max(a, b);
            const double s2 = S[1 + D + lo * D - lo * (lo - 1) / 2 + (hi - lo)];
            A.cov[t] = (W > 0.0) ? s2 / W - m[a] * m[b] : 0.0;
        }
        __syncthreads();
    }
}

hipError_t launch_update_batch(const BatchPtrs& b, int ne, int64_t total_blocks, hipStream_t st) {
    if (ne <= 0) return hipSuccess;
    const UpdateArg* args = (const UpdateArg*)b.args;
    k_u_part<<<stride_grid(total_blocks, 1, 8192), 256, 0, st>>>(b.hdr, args, b.off, b.scratch);
    k_u_final<<<event_grid(ne), 256, 0, st>>>(b.hdr, args, b.off, b.scratch);
    return hipGetLastError();
}

// ===========================================================================
// waveform of one point (injections), and the proposal's uniforms
// ===========================================================================
__global__ void k_wave_setup(EvConst ev, const double* __restrict__ theta, double* __restrict__ scratch) {
    if (threadIdx.x != 0) return;
    double th[PE_MAX_DIM];
    for (int a = 0; a < ev.dim; ++a) th[a] = theta[a];
    Src s;
    source_from_theta(ev, th, s);
    PhaseCoef pc;
    phase_coeffs(s, pc);
    for (int a = 0; a < 8; ++a) scratch[a] = pc.A[a];
    scratch[8] = pc.B5;
    scratch[9] = pc.B6;
    for (int d = 0; d < PE_MAX_DET; ++d) {
        scratch[10 + d] = s.rre[d];
        scratch[14 + d] = s.rim[d];
        scratch[18 + d] = s.tc + s.dt[d];
    }
    scratch[24] = (double)kcut_of(ev, s.fisco);
}

template <typename ST>
__global__ __launch_bounds__(256) void k_wave(EvConst ev, const double* __restrict__ scratch,
                                              const ST* __restrict__ psd, double* __restrict__ h,
                                              double* __restrict__ part) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double acc = 0.0;
    if (k < ev.K) {
        const int64_t kc = (int64_t)scratch[24];
        Rec64 r;
        r.f = grid_f(ev, k);
        r.x = cbrt(r.f);
        r.xm5 = 1.0 / (r.x * r.x * r.x * r.x * r.x);
        r.lnx = log(r.f) * (1.0 / 3.0);
        const double amp = 1.0 / (r.f * sqrt(r.x));  // f^(-7/6)
        for (int d = 0; d < ev.n_det; ++d) {
            double hr = 0.0, hi = 0.0;
            if (k < kc) {
                model_unit(scratch, d, r, hr, hi);
                hr *= amp;
                hi *= amp;
            }
            const int64_t o = (int64_t)d * ev.K + k;
            h[2 * o] = hr;
            h[2 * o + 1] = hi;
            if (psd) acc += 4.0 * ev.df * (hr * hr + hi * hi) / (double)psd[o];
        }
    }
    if (part) {
        __shared__ double sh[256];
        sh[threadIdx.x] = acc;
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
            __syncthreads();
        }
        if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
    }
}

__global__ __launch_bounds__(256) void k_sum_parts(const double* __restrict__ part, int64_t np,
                                                   double* __restrict__ out) {
    __shared__ double sh[256];
    double a = 0.0;
    for (int64_t i = threadIdx.x; i < np; i += 256) a += part[i];
    sh[threadIdx.x] = a;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sh[0];
}

hipError_t launch_waveform(const EvConst& ec, int psd_dtype, const double* theta, const void* psd, double* h,
                           double* snr2, double* scratch, hipStream_t st) {
    const int64_t nb = (ec.K + 255) / 256;
    double* part = (psd && snr2) ? scratch + 32 : nullptr;
    k_wave_setup<<<1, 64, 0, st>>>(ec, theta, scratch);
    if (psd_dtype == PE_F32)
        k_wave<float><<<(unsigned)nb, 256, 0, st>>>(ec, scratch, (const float*)psd, h, part);
    else
        k_wave<double><<<(unsigned)nb, 256, 0, st>>>(ec, scratch, (const double*)psd, h, part);
    if (part) k_sum_parts<<<1, 256, 0, st>>>(part, nb, snr2);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_uniforms(uint64_t seed, uint32_t stream_id, int64_t n, int npairs,
                                                  double* __restrict__ u) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * npairs) return;
    const int64_t i = t / npairs;
    const int j = (int)(t % npairs);
    double ua, ub;
    block_uniforms(seed, stream_id, (uint64_t)i, (uint32_t)j, ua, ub);
    u[2 * t] = ua;
    u[2 * t + 1] = ub;
}

hipError_t launch_uniforms(uint64_t seed, uint32_t stream_id, int64_t n, int npairs, double* u, hipStream_t st) {
    const int64_t tot = n * npairs;
    if (tot == 0) return hipSuccess;
    k_uniforms<<<(unsigned)((tot + 255) / 256), 256, 0, st>>>(seed, stream_id, n, npairs, u);
    return hipGetLastError();
}

}  // namespace pe
