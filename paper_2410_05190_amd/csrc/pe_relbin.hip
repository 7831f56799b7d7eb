// pe_relbin.hip -- relative binning (Zackay, Dai & Venumadhav 2018) about a
// fiducial point: per-bin sums of the fiducial-phased data once per setup,
// then O(bins) work per draw.
//
//   k_rb_erec     edge records f, f^(1/3), f^(-5/3), ln(f)/3 (as the bin tables)
//   k_rb_fid      the fiducial's phase polynomial and delays
//   k_rb_phi0     fiducial phase at every edge (turns)
//   k_rb_terms    a_k = conj(w_k) e^{-i Phi0(f_k)} and a_k (f_k - f_b), shifted by one
//   k_rb_scan_*   prefix sums of those four components per detector
//   k_rb_bins     per-bin sums A0, A1 from the prefix sums
//   k_rb_ll       per draw: support, cut, (h|h) from the prefix table, Z from the
//                 bins below the cut (the bin holding the cut from the prefix
//                 sums), ln L of Eq. 3
#include <hip/hip_runtime.h>
#include <math.h>

#include <cmath>
#include <vector>

#include "pe_device.h"
#include "pe_host.h"

namespace pe {
namespace {

double rb_envelope(double f, double f_lo, double f_hi) {
    static const double a[5] = {-5.0 / 3.0, -2.0 / 3.0, 1.0, 5.0 / 3.0, 7.0 / 3.0};
    double e = 0.0;
    for (int i = 0; i < 5; ++i) e += (a[i] < 0.0 ? -1.0 : 1.0) * pow(f / (a[i] < 0.0 ? f_lo : f_hi), a[i]);
    return 2.0 * kPi * e;
}

// Fiducial coefficients: A[8], B5, B6, tau[PE_MAX_DET].
constexpr int kRbFid = 10 + PE_MAX_DET;

__global__ void k_rb_erec(EvConst ev, const int64_t* __restrict__ kk, int n, double* __restrict__ erec) {
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= n) return;
    const double f = grid_f(ev, kk[e]);
    const double x = cbrt(f);
    const double x2 = x * x;
    erec[4 * e] = f;
    erec[4 * e + 1] = x;
    erec[4 * e + 2] = 1.0 / (x2 * x2 * x);
    erec[4 * e + 3] = log(f) * (1.0 / 3.0);
}

__global__ void k_rb_fid(EvConst ev, const double* __restrict__ th, double* __restrict__ fid) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double t[PE_MAX_DIM];
    for (int a = 0; a < PE_MAX_DIM; ++a) t[a] = (a < ev.dim) ? th[a] : 0.0;
    Src s;
    source_from_theta(ev, t, s);
    PhaseCoef pc;
    phase_coeffs(s, pc);
    for (int a = 0; a < 8; ++a) fid[a] = pc.A[a];
    fid[8] = pc.B5;
    fid[9] = pc.B6;
    for (int d = 0; d < PE_MAX_DET; ++d) fid[10 + d] = (d < ev.n_det) ? s.tc + s.dt[d] : 0.0;
}

__device__ __forceinline__ double fid_phase(const double* fid, int d, double f, double x, double xm5, double lnx) {
    double A[8];
#pragma unroll
    for (int a = 0; a < 8; ++a) A[a] = fid[a];
    return fma(f, fid[10 + d], psi_turns(A, fid[8], fid[9], x, xm5, lnx));
}

__global__ void k_rb_phi0(int n_det, int n, const double* __restrict__ erec, const double* __restrict__ fid,
                          double* __restrict__ phi0) {
    const int e = blockIdx.x * 256 + threadIdx.x;
    const int d = blockIdx.y;
    if (e >= n || d >= n_det) return;
    phi0[(int64_t)d * n + e] = fid_phase(fid, d, erec[4 * e], erec[4 * e + 1], erec[4 * e + 2], erec[4 * e + 3]);
}

// P[d][k + 1] = {a_k, a_k (f_k - f_b)} (two double2), P[d][0] = 0; b = the bin of k.
__global__ __launch_bounds__(256) void k_rb_terms(EvConst ev, const Rec64* __restrict__ rec,
                                                  const int64_t* __restrict__ kk, int n,
                                                  const double* __restrict__ erec, const double* __restrict__ fid,
                                                  double2* __restrict__ P) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int d = blockIdx.y;
    const int64_t K = ev.K;
    if (d >= ev.n_det || k > K) return;
    double2* Pd = P + (int64_t)d * (K + 1) * 2;
    if (k == K) {
        Pd[0] = make_double2(0.0, 0.0);
        Pd[1] = make_double2(0.0, 0.0);
        return;
    }
    // bin of k: the last edge <= k
    int lo = 0, hi = n - 2;
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (kk[mid] <= k)
            lo = mid;
        else
            hi = mid - 1;
    }
    const Rec64& r = rec[k];
    double sn, cs;
    sincos_turns(fract64(fid_phase(fid, d, r.f, r.x, r.xm5, r.lnx)), sn, cs);
    const double2 wv = r.w[d];
    const double wr = wv.x, wi = wv.y;
    // conj(w) (cs - i sn)
    const double ar = wr * cs - wi * sn;
    const double ai = -(wr * sn + wi * cs);
    const double t = r.f - erec[4 * lo];
    Pd[2 * (k + 1)] = make_double2(ar, ai);
    Pd[2 * (k + 1) + 1] = make_double2(ar * t, ai * t);
}

// Inclusive prefix sums over entries 0..K of each of the 4 doubles per entry,
// per detector: segment sums, then per segment its carry (one block
// reduction) and a block-wide scan 256 entries at a time.
__device__ __forceinline__ double rb_block_sum(double s, double* sh) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    const double r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(256) void k_rb_scan_sums(double* __restrict__ P, int64_t K1, int64_t seg,
                                                      double* __restrict__ ssum, int nseg) {
    __shared__ double sh[4];
    const int sgi = blockIdx.x, c = blockIdx.y, d = blockIdx.z;
    const double* x = P + (int64_t)d * K1 * 4 + c;
    const int64_t k0 = (int64_t)sgi * seg, k1 = min(K1, k0 + seg);
    double s = 0.0;
    for (int64_t k = k0 + threadIdx.x; k < k1; k += 256) s += x[4 * k];
    s = rb_block_sum(s, sh);
    if (threadIdx.x == 0) ssum[((int64_t)d * 4 + c) * nseg + sgi] = s;
}

__global__ __launch_bounds__(256) void k_rb_scan_write(double* __restrict__ P, int64_t K1, int64_t seg,
                                                       const double* __restrict__ ssum, int nseg) {
    __shared__ double sh[4];
    const int sgi = blockIdx.x, c = blockIdx.y, d = blockIdx.z;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    double* x = P + (int64_t)d * K1 * 4 + c;
    const double* ss = ssum + ((int64_t)d * 4 + c) * nseg;
    double carry = 0.0;
    for (int q = threadIdx.x; q < sgi; q += 256) carry += ss[q];
    carry = rb_block_sum(carry, sh);
    const int64_t k0 = (int64_t)sgi * seg, k1 = min(K1, k0 + seg);
    for (int64_t base = k0; base < k1; base += 256) {
        const int64_t k = base + threadIdx.x;
        double inc = (k < k1) ? x[4 * k] : 0.0;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const double u = __shfl_up(inc, off);
            if (lane >= off) inc += u;
        }
        if (lane == 63) sh[w] = inc;
        __syncthreads();
        double woff = 0.0;
        for (int q = 0; q < w; ++q) woff += sh[q];
        const double tile = (sh[0] + sh[1]) + (sh[2] + sh[3]);
        __syncthreads();
        if (k < k1) x[4 * k] = carry + (woff + inc);
        carry += tile;
    }
}

__global__ void k_rb_bins(int n_det, int64_t K, const int64_t* __restrict__ kk, int n, const double2* __restrict__ P,
                          double2* __restrict__ A) {
    const int b = blockIdx.x * 256 + threadIdx.x;
    const int d = blockIdx.y;
    if (b >= n - 1 || d >= n_det) return;
    const double2* Pd = P + (int64_t)d * (K + 1) * 2;
    const double2 a0 = Pd[2 * kk[b + 1]], a1 = Pd[2 * kk[b]];
    const double2 c0 = Pd[2 * kk[b + 1] + 1], c1 = Pd[2 * kk[b] + 1];
    double2* Ad = A + ((int64_t)d * (n - 1) + b) * 2;
    Ad[0] = make_double2(a0.x - a1.x, a0.y - a1.y);
    Ad[1] = make_double2(c0.x - c1.x, c0.y - c1.y);
}

struct RbArg {
    EvConst ec;
    const double* theta;
    int64_t n;
    double* loglike;
    double* aux;
    const double* pfx;
    const int64_t* kk;
    const double* erec;
    const double* phi0;
    const double2* A;
    const double2* P;
    int n_edges;
};

// A workgroup holds 64 draws (one per lane) in each of its kRbSeg waves; wave
// sg sums its draws over the sg-th contiguous share of the bins, so the bin
// index is uniform across the wave and every per-bin table entry (edge record,
// fiducial phase, bin coefficients) arrives through scalar loads. The draw's
// phase polynomial at an edge is evaluated once for all detectors. The waves'
// partial sums are combined through shared memory in a fixed order.
constexpr int kRbSeg = 4;

template <int ND>
__device__ __forceinline__ void rb_segment(const RbArg& a, const Src& s, const PhaseCoef& pc, int64_t kc, int kcmax,
                                           int b0, int b1, double& zr, double& zi) {
    const int64_t K = a.ec.K;
    const int nb = a.n_edges - 1;
    double tau[ND], ur[ND], ui[ND], r0r[ND], r0i[ND];
    {
        const double* er = a.erec + 4 * b0;
        const double psi = psi_turns(pc.A, pc.B5, pc.B6, er[1], er[2], er[3]);
#pragma unroll
        for (int d = 0; d < ND; ++d) {
            tau[d] = s.tc + s.dt[d];
            ur[d] = ui[d] = 0.0;
            double sn, cs;
            sincos_turns(fract64(fma(er[0], tau[d], psi) - a.phi0[(int64_t)d * a.n_edges + b0]), sn, cs);
            r0r[d] = cs;
            r0i[d] = -sn;
        }
    }
    // the wave walks its bins up to the largest cut among its draws; a lane
    // adds bin b only while b starts below its own cut
    for (int b = b0; b < b1 && a.kk[b] < kcmax; ++b) {
        const bool live = a.kk[b] < kc;
        const double* er = a.erec + 4 * (b + 1);
        const double psi = psi_turns(pc.A, pc.B5, pc.B6, er[1], er[2], er[3]);
        const double inv = 1.0 / (er[0] - a.erec[4 * b]);
        const bool full = a.kk[b + 1] <= kc;
#pragma unroll
        for (int d = 0; d < ND; ++d) {
            double sn, cs;
            sincos_turns(fract64(fma(er[0], tau[d], psi) - a.phi0[(int64_t)d * a.n_edges + b + 1]), sn, cs);
            const double r1r = cs, r1i = -sn;
            const double sr = (r1r - r0r[d]) * inv, si = (r1i - r0i[d]) * inv;
            const double2* Ad = a.A + ((int64_t)d * nb + b) * 2;
            double2 A0 = Ad[0], A1 = Ad[1];
            if (!full && live) {
                const double2* Pd = a.P + (int64_t)d * (K + 1) * 2;
                const double2 p0 = Pd[2 * kc], q0 = Pd[2 * a.kk[b]];
                const double2 p1 = Pd[2 * kc + 1], q1 = Pd[2 * a.kk[b] + 1];
                A0 = make_double2(p0.x - q0.x, p0.y - q0.y);
                A1 = make_double2(p1.x - q1.x, p1.y - q1.y);
            }
            if (live) {
                ur[d] += r0r[d] * A0.x - r0i[d] * A0.y + sr * A1.x - si * A1.y;
                ui[d] += r0r[d] * A0.y + r0i[d] * A0.x + sr * A1.y + si * A1.x;
            }
            r0r[d] = r1r;
            r0i[d] = r1i;
        }
    }
#pragma unroll
    for (int d = 0; d < ND; ++d) {
        zr += s.rre[d] * ur[d] - s.rim[d] * ui[d];
        zi += s.rre[d] * ui[d] + s.rim[d] * ur[d];
    }
}

__device__ __forceinline__ int wave_max_i(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
    return v;
}

// Four workgroups per CU: the register budget of four waves per SIMD (a few
// values spill; the kernel waits on FP64 chains and gains more from the waves).
__global__ __launch_bounds__(256, 4) void k_rb_ll(RbArg a) {
    __shared__ double sz[kRbSeg][64][2];
    const int lane = threadIdx.x & 63;
    const int sg = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // the wave's share of the bins
    const int64_t i = (int64_t)blockIdx.x * 64 + lane;
    const EvConst& ev = a.ec;
    double zr = 0.0, zi = 0.0, h = 0.0;
    int ok = 0;
    int64_t kc = 0;
    Src s = {};
    PhaseCoef pc = {};
    if (i < a.n) {
        double th[PE_MAX_DIM];
#pragma unroll
        for (int q = 0; q < PE_MAX_DIM; ++q) th[q] = (q < ev.dim) ? a.theta[(int64_t)q * a.n + i] : 0.0;
        likelihood_distance(ev, th);
        ok = source_from_theta(ev, th, s);
        if (ok) {
            phase_coeffs(s, pc);
            kc = kcut_of(ev, s.fisco);
        }
    }
    const int kcmax = wave_max_i(ok ? (int)kc : 0);
    const int nb = a.n_edges - 1;
    const int b0 = (int)((int64_t)sg * nb / kRbSeg), b1 = (int)((int64_t)(sg + 1) * nb / kRbSeg);
    if (kcmax > 0 && b0 < b1 && a.kk[b0] < kcmax) {
        // lanes without a draw (or out of support) follow with kc = 0: they add nothing
        switch (ev.n_det) {
            case 1: rb_segment<1>(a, s, pc, kc, kcmax, b0, b1, zr, zi); break;
            case 2: rb_segment<2>(a, s, pc, kc, kcmax, b0, b1, zr, zi); break;
            case 3: rb_segment<3>(a, s, pc, kc, kcmax, b0, b1, zr, zi); break;
            default: rb_segment<4>(a, s, pc, kc, kcmax, b0, b1, zr, zi); break;
        }
    }
    sz[sg][lane][0] = zr;
    sz[sg][lane][1] = zi;
    __syncthreads();
    if (sg != 0 || i >= a.n) return;
    if (!ok) {
        a.loglike[i] = -INFINITY;
        if (a.aux) {
            a.aux[3 * i] = 0.0;
            a.aux[3 * i + 1] = 0.0;
            a.aux[3 * i + 2] = 0.0;
        }
        return;
    }
    zr = (sz[0][lane][0] + sz[1][lane][0]) + (sz[2][lane][0] + sz[3][lane][0]);
    zi = (sz[0][lane][1] + sz[1][lane][1]) + (sz[2][lane][1] + sz[3][lane][1]);
    const int64_t K = ev.K;
#pragma unroll
    for (int d = 0; d < PE_MAX_DET; ++d) {  // fixed bound: the per-detector arrays stay in registers
        if (d >= ev.n_det) break;
        h += (s.rre[d] * s.rre[d] + s.rim[d] * s.rim[d]) * a.pfx[(int64_t)d * (K + 1) + kc];
    }
    const double ll = loglike_of<1>(ev, zr, zi, h, 0);
    a.loglike[i] = ll;
    if (a.aux) {
        a.aux[3 * i] = zr;
        a.aux[3 * i + 1] = zi;
        a.aux[3 * i + 2] = h;
    }
}

unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

pe_status_t run_relbin(pe_event_s* ev, const double* theta, int64_t n, double* loglike, double* aux, hipStream_t st) {
    if (ev->rb_n < 2) return fail(PE_ERR_ARG, "relative binning needs pe_relbin_setup on the event first");
    RbArg a;
    a.ec = ev->ec;
    a.theta = theta;
    a.n = n;
    a.loglike = loglike;
    a.aux = aux;
    a.pfx = ev->pfx;
    a.kk = ev->rb_k;
    a.erec = ev->rb_erec;
    a.phi0 = ev->rb_phi0;
    a.A = ev->rb_A;
    a.P = ev->rb_P;
    a.n_edges = ev->rb_n;
    k_rb_ll<<<(unsigned)((n + 63) / 64), 64 * kRbSeg, 0, st>>>(a);
    PE_HIP(hipGetLastError());
    return PE_OK;
}

}  // namespace pe

using namespace pe;

extern "C" pe_status_t pe_relbin_setup(pe_event_t ev, const double* theta_f_dev, double eps, int32_t max_edges,
                                       void* stream) {
    if (!ev) return fail(PE_ERR_ARG, "event is NULL");
    if (!theta_f_dev) return fail(PE_ERR_ARG, "theta_f must be a device pointer");
    if (!(eps >= 0.0) || !std::isfinite(eps)) return fail(PE_ERR_ARG, "eps must be >= 0");
    if (max_edges < 2) return fail(PE_ERR_ARG, "max_edges must be >= 2");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const EvConst& ec = ev->ec;
    const int64_t K = ec.K;
    const double f_hi = ec.f_lo + (double)K * ec.df;
    // edges on the host
    std::vector<int64_t> kk;
    kk.push_back(0);
    double eb = rb_envelope(ec.f_lo, ec.f_lo, f_hi);
    for (int64_t k = 1; k < K; ++k) {
        const double e = rb_envelope(ec.f_lo + (double)k * ec.df, ec.f_lo, f_hi);
        if (e - eb >= eps) {
            if ((int64_t)kk.size() + 1 >= max_edges) return fail(PE_ERR_BUDGET, "more relative-binning edges than max_edges");
            kk.push_back(k);
            eb = e;
        }
    }
    kk.push_back(K);
    const int n = (int)kk.size();
    const int nd = ec.n_det;
    // memory: edges, edge records, fiducial, phases, bins, prefix sums, scan scratch
    const int64_t seg = std::max<int64_t>(1024, (K + 1 + 1023) / 1024);
    const int nseg = (int)((K + 1 + seg - 1) / seg);
    Carver c(nullptr);
    c.take<int64_t>(n);
    c.take<double>(4 * (size_t)n);
    c.take<double>(kRbFid);
    c.take<double>((size_t)nd * n);
    c.take<double2>((size_t)nd * (n - 1) * 2);
    c.take<double2>((size_t)nd * (K + 1) * 2);
    c.take<double>((size_t)nd * 4 * nseg);
    c.take<double>(PE_MAX_DIM);
    PE_HIP(hipStreamSynchronize(st));  // a previous setup's buffers may still be read
    dfree_bytes(ev->rb_mem);
    ev->rb_n = 0;
    pe_status_t s = dalloc_bytes(&ev->rb_mem, c.size());
    if (s != PE_OK) return s;
    Carver m(ev->rb_mem);
    ev->rb_k = m.take<int64_t>(n);
    ev->rb_erec = m.take<double>(4 * (size_t)n);
    double* fid = m.take<double>(kRbFid);
    ev->rb_phi0 = m.take<double>((size_t)nd * n);
    ev->rb_A = m.take<double2>((size_t)nd * (n - 1) * 2);
    ev->rb_P = m.take<double2>((size_t)nd * (K + 1) * 2);
    double* ssum = m.take<double>((size_t)nd * 4 * nseg);
    ev->rb_fid = m.take<double>(PE_MAX_DIM);
    PE_HIP(hipMemcpyAsync(ev->rb_k, kk.data(), sizeof(int64_t) * n, hipMemcpyHostToDevice, st));
    PE_HIP(hipMemcpyAsync(ev->rb_fid, theta_f_dev, sizeof(double) * ec.dim, hipMemcpyDeviceToDevice, st));
    k_rb_erec<<<nblk(n), 256, 0, st>>>(ec, ev->rb_k, n, ev->rb_erec);
    k_rb_fid<<<1, 64, 0, st>>>(ec, ev->rb_fid, fid);
    k_rb_phi0<<<dim3(nblk(n), nd), 256, 0, st>>>(nd, n, ev->rb_erec, fid, ev->rb_phi0);
    k_rb_terms<<<dim3(nblk(K + 1), nd), 256, 0, st>>>(ec, ev->rec64, ev->rb_k, n, ev->rb_erec, fid, ev->rb_P);
    k_rb_scan_sums<<<dim3(nseg, 4, nd), 256, 0, st>>>((double*)ev->rb_P, K + 1, seg, ssum, nseg);
    k_rb_scan_write<<<dim3(nseg, 4, nd), 256, 0, st>>>((double*)ev->rb_P, K + 1, seg, ssum, nseg);
    k_rb_bins<<<dim3(nblk(n), nd), 256, 0, st>>>(nd, K, ev->rb_k, n, ev->rb_P, ev->rb_A);
    PE_HIP(hipGetLastError());
    PE_HIP(hipStreamSynchronize(st));
    ev->rb_n = n;
    return PE_OK;
}

extern "C" pe_status_t pe_relbin_edges(pe_event_t ev, int64_t* edges, int32_t cap, int32_t* n) {
    if (!ev || !n) return fail(PE_ERR_ARG, "event and n must not be NULL");
    *n = ev->rb_n;
    if (ev->rb_n == 0 || !edges) return PE_OK;  // NULL edges: the count only
    if (cap < ev->rb_n) return fail(PE_ERR_ARG, "edges array too small");
    PE_HIP(hipMemcpy(edges, ev->rb_k, sizeof(int64_t) * ev->rb_n, hipMemcpyDeviceToHost));
    return PE_OK;
}
