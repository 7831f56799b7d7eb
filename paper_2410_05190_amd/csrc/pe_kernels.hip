// pe_kernels.hip -- HIP kernels of the likelihood engine for gfx950 (MI355X).
//
// Hot path, per event and batch of draws:
//   k_prep, k_seg_*        event tables and the (h|h) prefix sums (once per event)
//   (pe_loglike.hip)       per-draw scalars, the hot loop and ln L for batches of
//                          draws of one or many events
//   k_weights              log-sum-exp weights and ESS (Eqs. 5-6)
// plus the metric (finite-difference Fisher matrix) and the Gaussian draws.
#include <math.h>

#include "pe_device.h"

namespace pe {

// ===========================================================================
// event preparation
// ===========================================================================
template <typename DT, typename ST>
__global__ __launch_bounds__(256) void k_prep(EvConst ev, const DT* __restrict__ data, const ST* __restrict__ psd,
                                              Rec32* __restrict__ rec32, Rec64* __restrict__ rec64,
                                              double* __restrict__ pw, int* __restrict__ status) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= ev.K) return;
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
            pw[o] = 4.0 * ev.df / (S * f76 * f76);
        } else {
            r64.w[d] = make_double2(0.0, 0.0);
            r32.w[d] = make_float2(0.0f, 0.0f);
        }
    }
    rec32[k] = r32;
    rec64[k] = r64;
    if (bad) atomicOr(status, bad);
}

// Exclusive prefix C_k = sum_{j<k} pw_j (k = 0..K) per detector, in two passes
// over kScanSeg contiguous segments: segment sums, then each segment adds the
// sums before it (fixed order) and scans its bins in coalesced 256-wide tiles
// (wave shuffle scan + LDS across the four waves).
__global__ __launch_bounds__(256) void k_seg_sums(const double* __restrict__ pw, int64_t K, int64_t seg,
                                                  double* __restrict__ tot) {
    __shared__ double sh[4];
    const int d = blockIdx.y, b = blockIdx.x;
    const double* a = pw + (int64_t)d * K;
    const int64_t k0 = (int64_t)b * seg;
    const int64_t k1 = min(k0 + seg, K);
    double s = 0.0;
    for (int64_t k = k0 + threadIdx.x; k < k1; k += 256) s += a[k];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) tot[d * kScanSeg + b] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

__global__ __launch_bounds__(256) void k_seg_scan(const double* __restrict__ pw, int64_t K, int64_t seg,
                                                  const double* __restrict__ tot, double* __restrict__ pfx) {
    __shared__ double sh[4];
    const int d = blockIdx.y, b = blockIdx.x;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const double* a = pw + (int64_t)d * K;
    double* o = pfx + (int64_t)d * (K + 1);
    double carry = 0.0;
    for (int i = 0; i < b; ++i) carry += tot[d * kScanSeg + i];
    const int64_t k0 = (int64_t)b * seg;
    const int64_t k1 = min(k0 + seg, K);
    for (int64_t base = k0; base < k1; base += 256) {
        const int64_t k = base + threadIdx.x;
        const double v = (k < k1) ? a[k] : 0.0;
        double inc = v;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const double u = __shfl_up(inc, off);
            if (lane >= off) inc += u;
        }
        double exc = __shfl_up(inc, 1);
        if (lane == 0) exc = 0.0;
        if (lane == 63) sh[w] = inc;
        __syncthreads();
        double woff = 0.0;
        for (int i = 0; i < w; ++i) woff += sh[i];
        const double tile = (sh[0] + sh[1]) + (sh[2] + sh[3]);
        __syncthreads();
        if (k < k1) o[k] = carry + (woff + exc);
        carry += tile;
    }
    if (b == gridDim.x - 1 && threadIdx.x == 0) o[K] = carry;
}

hipError_t launch_prep(const pe_event_s* ev, const void* data, const void* psd, hipStream_t st) {
    const EvConst& ec = ev->ec;
    const unsigned nb = (unsigned)((ec.K + 255) / 256);
    const bool c64 = ev->desc.data_dtype == PE_C64, f32 = ev->desc.psd_dtype == PE_F32;
    if (c64 && f32)
        k_prep<float, float><<<nb, 256, 0, st>>>(ec, (const float*)data, (const float*)psd, ev->rec32, ev->rec64,
                                                  ev->pw, ev->status);
    else if (c64)
        k_prep<float, double><<<nb, 256, 0, st>>>(ec, (const float*)data, (const double*)psd, ev->rec32, ev->rec64,
                                                   ev->pw, ev->status);
    else if (f32)
        k_prep<double, float><<<nb, 256, 0, st>>>(ec, (const double*)data, (const float*)psd, ev->rec32, ev->rec64,
                                                   ev->pw, ev->status);
    else
        k_prep<double, double><<<nb, 256, 0, st>>>(ec, (const double*)data, (const double*)psd, ev->rec32,
                                                    ev->rec64, ev->pw, ev->status);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t seg = (ec.K + kScanSeg - 1) / kScanSeg;
    double* tot = ev->mws + kMwsScan;
    k_seg_sums<<<dim3(kScanSeg, ec.n_det), 256, 0, st>>>(ev->pw, ec.K, seg, tot);
    k_seg_scan<<<dim3(kScanSeg, ec.n_det), 256, 0, st>>>(ev->pw, ec.K, seg, tot, ev->pfx);
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
__global__ void k_metric_setup(EvConst ev, const double* __restrict__ theta0, const double* __restrict__ steps_in,
                               double* __restrict__ mws) {
    const int t = threadIdx.x;
    const int D = ev.dim;
    __shared__ double st[PE_MAX_DIM];
    double th0[PE_MAX_DIM];
#pragma unroll
    for (int a = 0; a < PE_MAX_DIM; ++a) th0[a] = (a < D) ? theta0[a] : 0.0;
    if (t == 0) {
        double s[PE_MAX_DIM];
        if (steps_in)
            for (int a = 0; a < D; ++a) s[a] = steps_in[a];
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
    if (t >= 2 * D + 1) return;
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
// (index DP-1 in 4-D, 10 in 11-D), which is i h(theta0).
template <int NDET, int D, int DP>
__global__ __launch_bounds__(256) void k_metric_partial(EvConst ev, const Rec64* __restrict__ tab,
                                                        const double* __restrict__ pw, double* __restrict__ mws) {
    constexpr int NG = DP * (DP + 1) / 2;
    constexpr int PH = (DP == D) ? D - 1 : D;  // phase column
    const int64_t kc = (int64_t)mws[kMwsKcut];
    const double* src = mws + kMwsSrc;
    double den[D];
#pragma unroll
    for (int a = 0; a < D; ++a) den[a] = mws[kMwsDen + a];
    double G[NG];
#pragma unroll
    for (int q = 0; q < NG; ++q) G[q] = 0.0;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < kc; k += (int64_t)gridDim.x * blockDim.x) {
        const Rec64 r = tab[k];
#pragma unroll
        for (int d = 0; d < NDET; ++d) {
            const double p = pw[(int64_t)d * ev.K + k];
            double ur[DP], ui[DP];
#pragma unroll
            for (int a = 0; a < DP; ++a) {
                if (a == PH) {
                    double hr, hi;
                    model_unit(src, d, r, hr, hi);
                    ur[a] = -hi;  // i h
                    ui[a] = hr;
                } else {
                    double pr, pi_, mr, mi;
                    model_unit(src + (2 * a + 1) * kMetricSrcStride, d, r, pr, pi_);
                    model_unit(src + (2 * a + 2) * kMetricSrcStride, d, r, mr, mi);
                    ur[a] = (pr - mr) / den[a];
                    ui[a] = (pi_ - mi) / den[a];
                }
            }
            int q = 0;
#pragma unroll
            for (int a = 0; a < DP; ++a)
#pragma unroll
                for (int b = a; b < DP; ++b) {
                    G[q] = fma(p, ur[a] * ur[b] + ui[a] * ui[b], G[q]);
                    ++q;
                }
        }
    }
    // wave butterfly, then the four waves through LDS
    __shared__ double sh[4][NG];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NG; ++q) {
        double v = G[q];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
        if (lane == 0) sh[wv][q] = v;
    }
    __syncthreads();
    for (int q = threadIdx.x; q < NG; q += blockDim.x)
        mws[kMwsPart + (int64_t)blockIdx.x * kMetricNG + q] = (sh[0][q] + sh[1][q]) + (sh[2][q] + sh[3][q]);
}

__global__ __launch_bounds__(128) void k_metric_final(EvConst ev, int DP, int flags, const double* __restrict__ mws,
                                                      double* __restrict__ g) {
    __shared__ double Gs[kMetricNG];
    const int NG = DP * (DP + 1) / 2;
    const int t = threadIdx.x;
    if (t < NG) {
        double acc[8];
        for (int q = 0; q < 8; ++q) acc[q] = 0.0;
        for (int b = 0; b < kMetricBlocks; ++b) acc[b & 7] += mws[kMwsPart + (int64_t)b * kMetricNG + t];
        for (int w = 4; w > 0; w >>= 1)
            for (int q = 0; q < w; ++q) acc[q] += acc[q + w];
        Gs[t] = acc[0];
    }
    __syncthreads();
    if (t != 0) return;
    const int D = ev.dim;
    const int PH = (DP == D) ? D - 1 : D;
    double M[kMetricMaxDp][kMetricMaxDp];
    int q = 0;
    for (int a = 0; a < DP; ++a)
        for (int b = a; b < DP; ++b) {
            M[a][b] = M[b][a] = Gs[q];
            ++q;
        }
    if (ev.phase == PE_PHASE_MARG) {
        const double gpp = M[PH][PH];
        double P[kMetricMaxDp][kMetricMaxDp];
        for (int a = 0; a < DP; ++a)
            for (int b = 0; b < DP; ++b)
                P[a][b] = (a == PH || b == PH) ? 0.0 : M[a][b] - M[a][PH] * M[PH][b] / gpp;
        for (int a = 0; a < DP; ++a)
            for (int b = 0; b < DP; ++b) M[a][b] = P[a][b];
    }
    double reg[PE_MAX_DIM];
    if (ev.params == PE_PARAMS_4D) {
        reg[0] = 0.0;
        reg[1] = 12.0 / 0.0625;
        reg[2] = 3.0 / (ev.chi_max * ev.chi_max);
        reg[3] = 0.0;
    } else {
        const double p2 = 3.0 / (kPi * kPi);  // 12 / (2 pi)^2
        const double p1 = 12.0 / (kPi * kPi);
        reg[0] = 0.0;
        reg[1] = 12.0;
        reg[2] = reg[3] = 3.0 / (ev.chi_max * ev.chi_max);
        reg[4] = p2;
        reg[5] = reg[6] = reg[7] = p1;
        reg[8] = 12.0 / (ev.dl_max * ev.dl_max);
        reg[9] = 0.0;
        reg[10] = p2;
    }
    for (int a = 0; a < D; ++a)
        for (int b = 0; b < D; ++b) g[a * D + b] = M[a][b] + ((a == b && !(flags & 1)) ? reg[a] : 0.0);
}

template <int NDET>
static hipError_t launch_metric_nd(const pe_event_s* ev, double* mws, hipStream_t st) {
    if (ev->ec.params == PE_PARAMS_4D)
        k_metric_partial<NDET, 4, 5><<<kMetricBlocks, 256, 0, st>>>(ev->ec, ev->rec64, ev->pw, mws);
    else
        k_metric_partial<NDET, 11, 11><<<kMetricBlocks, 256, 0, st>>>(ev->ec, ev->rec64, ev->pw, mws);
    return hipGetLastError();
}

hipError_t launch_metric(const pe_event_s* ev, const double* theta0, const double* steps, int flags, double* g,
                         hipStream_t st) {
    const EvConst& ec = ev->ec;
    k_metric_setup<<<1, 32, 0, st>>>(ec, theta0, steps, ev->mws);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    switch (ec.n_det) {
        case 1: e = launch_metric_nd<1>(ev, ev->mws, st); break;
        case 2: e = launch_metric_nd<2>(ev, ev->mws, st); break;
        case 3: e = launch_metric_nd<3>(ev, ev->mws, st); break;
        default: e = launch_metric_nd<4>(ev, ev->mws, st); break;
    }
    if (e != hipSuccess) return e;
    const int DP = (ec.params == PE_PARAMS_4D) ? 5 : 11;
    k_metric_final<<<1, 128, 0, st>>>(ec, DP, flags, ev->mws, g);
    return hipGetLastError();
}

// ===========================================================================
// draws
// ===========================================================================
__global__ void k_cholesky(int D, const double* __restrict__ g, double* __restrict__ chol, int* __restrict__ status) {
    if (threadIdx.x != 0) return;
    double L[PE_MAX_DIM * PE_MAX_DIM];
    int ok = 1;
    for (int a = 0; a < D * D; ++a) L[a] = 0.0;
    for (int i = 0; i < D && ok; ++i)
        for (int j = 0; j <= i; ++j) {
            double s = g[i * D + j];
            for (int k = 0; k < j; ++k) s -= L[i * D + k] * L[j * D + k];
            if (i == j) {
                if (!(s > 0.0)) {
                    ok = 0;
                    break;
                }
                L[i * D + i] = sqrt(s);
            } else {
                L[i * D + j] = s / L[j * D + j];
            }
        }
    double logdet = 0.0;
    for (int a = 0; a < D * D; ++a) chol[a] = L[a];
    if (ok)
        for (int a = 0; a < D; ++a) logdet += log(L[a * D + a]);
    chol[PE_MAX_DIM * PE_MAX_DIM] = logdet;
    chol[PE_MAX_DIM * PE_MAX_DIM + 1] = ok ? 1.0 : 0.0;
    if (!ok) atomicOr(status, kStSingular);
}

__global__ __launch_bounds__(256) void k_draw(EvConst ev, const double* __restrict__ theta0,
                                              const double* __restrict__ chol, uint64_t seed, uint32_t stream_id,
                                              int64_t n, double* __restrict__ theta, double* __restrict__ logq,
                                              double* __restrict__ logprior) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int D = ev.dim;
    double th0[PE_MAX_DIM];
    for (int a = 0; a < D; ++a) th0[a] = theta0[a];
    if (chol[PE_MAX_DIM * PE_MAX_DIM + 1] == 0.0) {
        for (int a = 0; a < D; ++a) theta[(int64_t)a * n + i] = th0[a];
        logq[i] = 0.0;
        logprior[i] = -INFINITY;
        return;
    }
    double z[PE_MAX_DIM + 1];
    for (int j = 0; 2 * j < D; ++j) {
        double ua, ub, sn, cs;
        block_uniforms(seed, stream_id, (uint64_t)i, (uint32_t)j, ua, ub);
        const double rad = sqrt(-2.0 * log(ua));
        sincos_turns(ub >= 1.0 ? 0.0 : ub, sn, cs);  // 2 pi ub
        z[2 * j] = rad * cs;
        z[2 * j + 1] = rad * sn;
    }
    // theta = theta0 + L^-T z (back substitution with L^T)
    double y[PE_MAX_DIM];
    for (int r = D - 1; r >= 0; --r) {
        double s = z[r];
        for (int c = r + 1; c < D; ++c) s -= chol[c * D + r] * y[c];
        y[r] = s / chol[r * D + r];
    }
    double th[PE_MAX_DIM];
    for (int a = 0; a < D; ++a) th[a] = th0[a] + y[a];
    const int np = (ev.params == PE_PARAMS_4D) ? 0 : 3;
    const int pidx[3] = {4, 7, 10};
    const double per[3] = {kTwoPi, kPi, kTwoPi};
    double k0[3] = {0.0, 0.0, 0.0};
    for (int p = 0; p < np; ++p) {
        const double v = th[pidx[p]];
        k0[p] = floor(v / per[p]);
        th[pidx[p]] = v - per[p] * k0[p];
    }
    for (int a = 0; a < D; ++a) theta[(int64_t)a * n + i] = th[a];
    // log-density of the wrapped Gaussian: images k in {-1,0,1}^p, whitened
    // offset L^T (x - theta0) = z + L^T s with s = (k - k0) P on the periodic rows
    const int nimg = (np == 0) ? 1 : 27;
    double lq[27];
    double mx = -INFINITY;
    for (int m = 0; m < nimg; ++m) {
        double s[3];
        int code = m;
        for (int p = 0; p < np; ++p) {
            s[p] = ((double)(code % 3 - 1) - k0[p]) * per[p];
            code /= 3;
        }
        double qf = 0.0;
        for (int r = 0; r < D; ++r) {
            double v = z[r];
            for (int p = 0; p < np; ++p)
                if (pidx[p] >= r) v += chol[pidx[p] * D + r] * s[p];
            qf += v * v;
        }
        lq[m] = -0.5 * qf;
        mx = fmax(mx, lq[m]);
    }
    double acc = 0.0;
    for (int m = 0; m < nimg; ++m) acc += exp(lq[m] - mx);
    logq[i] = mx + log(acc) + chol[PE_MAX_DIM * PE_MAX_DIM] - 0.5 * D * log(kTwoPi);
    Src src;
    const int ok = source_from_theta(ev, th, src);
    double lp = -INFINITY;
    if (ok) lp = (ev.params == PE_PARAMS_4D) ? 0.0 : log(cos(th[5])) + log(sin(th[6])) + 2.0 * log(th[8]);
    logprior[i] = lp;
}

hipError_t launch_draw(const pe_event_s* ev, const double* theta0, const double* g, uint64_t seed, uint32_t stream_id,
                       int64_t n, double* theta, double* logq, double* logprior, hipStream_t st) {
    double* chol = ev->mws + kMwsChol;
    k_cholesky<<<1, 64, 0, st>>>(ev->ec.dim, g, chol, ev->status);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || n == 0) return e;
    k_draw<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(ev->ec, theta0, chol, seed, stream_id, n, theta, logq,
                                                        logprior);
    return hipGetLastError();
}

// ===========================================================================
// weights and ESS (one workgroup; fixed-order reductions)
// ===========================================================================
__device__ __forceinline__ void neumaier(double& s, double& c, double x) {
    const double t = s + x;
    if (fabs(s) >= fabs(x))
        c += (s - t) + x;
    else
        c += (x - t) + s;
    s = t;
}

__global__ __launch_bounds__(1024) void k_weights(const double* __restrict__ ll, const double* __restrict__ lp,
                                                  const double* __restrict__ lq, int64_t n, double* __restrict__ w,
                                                  double* __restrict__ stats) {
    __shared__ double s1[1024], s2[1024];
    __shared__ long long sc[1024];
    const int t = threadIdx.x;
    double m = -INFINITY;
    long long cnt = 0;
    for (int64_t i = t; i < n; i += 1024) {
        const double l = ll[i] + lp[i] - lq[i];
        if (isfinite(l)) {
            ++cnt;
            m = fmax(m, l);
        }
    }
    s1[t] = m;
    sc[t] = cnt;
    __syncthreads();
    for (int o = 512; o > 0; o >>= 1) {
        if (t < o) {
            s1[t] = fmax(s1[t], s1[t + o]);
            sc[t] += sc[t + o];
        }
        __syncthreads();
    }
    const double mx = s1[0];
    const long long nin = sc[0];
    __syncthreads();
    if (nin == 0) {
        if (w)
            for (int64_t i = t; i < n; i += 1024) w[i] = 0.0;
        if (t == 0) {
            stats[0] = 0.0;
            stats[1] = -INFINITY;
            stats[2] = -INFINITY;
            stats[3] = 0.0;
        }
        return;
    }
    double a = 0.0, ac = 0.0, b = 0.0, bc = 0.0;
    for (int64_t i = t; i < n; i += 1024) {
        const double l = ll[i] + lp[i] - lq[i];
        if (isfinite(l)) {
            const double e = exp(l - mx);
            neumaier(a, ac, e);
            neumaier(b, bc, e * e);
        }
    }
    s1[t] = a + ac;
    s2[t] = b + bc;
    __syncthreads();
    for (int o = 512; o > 0; o >>= 1) {
        if (t < o) {
            s1[t] += s1[t + o];
            s2[t] += s2[t + o];
        }
        __syncthreads();
    }
    const double S1 = s1[0], S2 = s2[0];
    if (w) {
        const double inv = 1.0 / S1;
        for (int64_t i = t; i < n; i += 1024) {
            const double l = ll[i] + lp[i] - lq[i];
            w[i] = isfinite(l) ? exp(l - mx) * inv : 0.0;
        }
    }
    if (t == 0) {
        stats[0] = S1 * S1 / S2;
        stats[1] = mx + log(S1) - log((double)n);
        stats[2] = mx;
        stats[3] = (double)nin;
    }
}

hipError_t launch_weights(const double* ll, const double* lp, const double* lq, int64_t n, double* w, double* stats,
                          hipStream_t st) {
    k_weights<<<1, 1024, 0, st>>>(ll, lp, lq, n, w, stats);
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
