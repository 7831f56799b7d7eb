// pe_tiles.hip -- the tile-mixture proposal (Sec. II.A; App. A: template bank,
// tiling of the prior volume, proposal) on a slice of the prior: the ball
// |y| <= R in whitened coordinates y = L^T (theta - c) of a metric G = L L^T.
//
//   k_slice_count / k_slice_scan / k_slice_write
//                  slice samples: candidates from Philox, kept ones compacted
//                  in candidate order (count, block offsets, write)
//   k_bank_cand    one batch of bank candidates and whether each is at least
//                  min_dist from every template so far (the host then takes
//                  the batch in order against the batch's own new templates)
//   k_tile_assign  nearest template of every sample, templates staged in LDS
//   k_match_rows, k_tile_topc, k_tile_match
//                  tiles by waveform match: phase coefficients of templates and
//                  samples, each sample's nearest templates, their matches
//   k_tile_max, k_tile_mass, k_scan_sums, k_scan_write, k_tile_pick
//                  proposal draws: per-sample masses, FP64 prefix sums,
//                  inverse-CDF pick by binary search
//
// Candidate coordinates, whitened distances and the acceptance tests are
// evaluated without contractions, so their decisions are the same bit for bit
// on every run (and in any other IEEE FP64 evaluation in the same order).
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <vector>

#include "pe_device.h"
#include "pe_host.h"

namespace pe {
namespace {

// idx: the S sliced coordinates in index order (all D without a sub_mask);
// L is S x S.
struct Slice {
    double c[PE_MAX_DIM];
    double L[PE_MAX_DIM * PE_MAX_DIM];
    double R;
    int idx[PE_MAX_DIM];
};

// |a - b|^2 summed in index order, no contractions (host and device).
template <int D>
__host__ __device__ __forceinline__ double wdist2(const double* a, int64_t sa, const double* b, int64_t sb) {
#pragma clang fp contract(off)
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const double d = a[k * sa] - b[k * sb];
        s += d * d;
    }
    return s;
}

__host__ double wdist2_rt(int D, const double* a, int64_t sa, const double* b, int64_t sb) {
    return D == 4 ? wdist2<4>(a, sa, b, sb) : wdist2<11>(a, sa, b, sb);
}

// Candidate i of the slice: y (S sliced coordinates), theta (all D); 1 if kept.
template <int S, int D>
__device__ __forceinline__ int slice_candidate(const EvConst& ev, const Slice& sl, uint64_t seed, uint32_t st,
                                               uint64_t i, double (&y)[S], double (&th)[D]) {
#pragma clang fp contract(off)
    double u[S + 1];
#pragma unroll
    for (int a = 0; 2 * a < S; ++a) block_uniforms(seed, st, i, (uint32_t)a, u[2 * a], u[2 * a + 1]);
    double r2 = 0.0;
#pragma unroll
    for (int a = 0; a < S; ++a) {
        y[a] = sl.R * (2.0 * u[a] - 1.0);
        r2 += y[a] * y[a];
    }
    double x[S];
#pragma unroll
    for (int r = S - 1; r >= 0; --r) {
        double t = y[r];
#pragma unroll
        for (int c = r + 1; c < S; ++c) t -= sl.L[c * S + r] * x[c];
        x[r] = t / sl.L[r * S + r];
    }
#pragma unroll
    for (int a = 0; a < D; ++a) th[a] = sl.c[a];
    if constexpr (S == D) {
#pragma unroll
        for (int a = 0; a < D; ++a) th[a] = sl.c[a] + x[a];
    } else {
        // sliced coordinates by index (a short unrolled search keeps th in registers)
#pragma unroll
        for (int a = 0; a < S; ++a)
#pragma unroll
            for (int b = 0; b < D; ++b)
                if (sl.idx[a] == b) th[b] = sl.c[b] + x[a];
    }
    if (!(r2 <= sl.R * sl.R)) return 0;
    double M;
    return mass_and_support(ev, th, M);
}

// --------------------------------------------------------------- slice samples
template <int S, int D>
__global__ __launch_bounds__(256) void k_slice_count(EvConst ev, Slice sl, uint64_t seed, uint32_t st, int64_t first,
                                                     int64_t n, int64_t* __restrict__ bcount) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    int keep = 0;
    if (k < n) {
        double y[S], th[D];
        keep = slice_candidate<S, D>(ev, sl, seed, st, (uint64_t)(first + k), y, th);
    }
    const int c = __syncthreads_count(keep);
    if (threadIdx.x == 0) bcount[blockIdx.x] = c;
}

// Exclusive scan of the nb block counts in place (one workgroup, in order);
// the total into total[0].
__global__ __launch_bounds__(1024) void k_slice_scan(int64_t* __restrict__ bcount, int64_t nb,
                                                     int64_t* __restrict__ total) {
    __shared__ int64_t sh[1024];
    const int t = threadIdx.x;
    const int64_t per = (nb + 1023) / 1024;
    const int64_t b0 = t * per, b1 = min(nb, b0 + per);
    int64_t s = 0;
    for (int64_t b = b0; b < b1; ++b) s += bcount[b];
    sh[t] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int64_t v = (t >= off) ? sh[t - off] : 0;
        __syncthreads();
        sh[t] += v;
        __syncthreads();
    }
    int64_t run = sh[t] - s;
    for (int64_t b = b0; b < b1; ++b) {
        const int64_t c = bcount[b];
        bcount[b] = run;
        run += c;
    }
    if (t == 1023) total[0] = sh[1023];
}

template <int S, int D>
__global__ __launch_bounds__(256) void k_slice_write(EvConst ev, Slice sl, uint64_t seed, uint32_t st, int64_t first,
                                                     int64_t n, const int64_t* __restrict__ boff,
                                                     double* __restrict__ yo, double* __restrict__ tho,
                                                     double* __restrict__ lpo) {
    __shared__ int wcount[4];
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    int keep = 0;
    double y[S], th[D];
    if (k < n) keep = slice_candidate<S, D>(ev, sl, seed, st, (uint64_t)(first + k), y, th);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint64_t mask = __ballot(keep);
    if (lane == 0) wcount[w] = __popcll(mask);
    __syncthreads();
    int woff = 0;
    for (int q = 0; q < w; ++q) woff += wcount[q];
    if (keep) {
        const int64_t pos = boff[blockIdx.x] + woff + __popcll(mask & ((1ull << lane) - 1));
#pragma unroll
        for (int a = 0; a < S; ++a) yo[a * n + pos] = y[a];
#pragma unroll
        for (int a = 0; a < D; ++a) tho[a * n + pos] = th[a];
        lpo[pos] = log_prior_of(ev, th);
    }
}

__global__ void k_set_count(int64_t* c) { c[0] = 0; }

// ----------------------------------------------------------------------- bank
// Candidates b0 .. b0 + nb - 1: y [S][nb], theta [D][nb], flag = 0 (not kept),
// 1 (kept, within min_dist of a template), 2 (kept, at least min_dist from all m).
template <int S, int D>
__global__ __launch_bounds__(256) void k_bank_cand(EvConst ev, Slice sl, uint64_t seed, uint32_t st, int64_t b0,
                                                   int nb, const double* __restrict__ ty, int64_t ldt, int m,
                                                   double r2, double* __restrict__ cy, double* __restrict__ cth,
                                                   int* __restrict__ flag) {
    __shared__ double tl[256 * S];
    const int k = blockIdx.x * 256 + threadIdx.x;
    double y[S], th[D];
    int keep = 0;
    if (k < nb) keep = slice_candidate<S, D>(ev, sl, seed, st, (uint64_t)(b0 + k), y, th);
    bool far = keep != 0;
    for (int j0 = 0; j0 < m; j0 += 256) {
        const int cnt = min(256, m - j0);
        __syncthreads();
        for (int q = threadIdx.x; q < cnt * S; q += 256) {
            const int a = q / cnt, j = q - a * cnt;
            tl[a * 256 + j] = ty[a * ldt + j0 + j];
        }
        __syncthreads();
        if (far)
            for (int j = 0; j < cnt; ++j)
                if (wdist2<S>(y, 1, tl + j, 256) < r2) {
                    far = false;
                    break;
                }
    }
    if (k < nb) {
#pragma unroll
        for (int a = 0; a < S; ++a) cy[a * nb + k] = y[a];
#pragma unroll
        for (int a = 0; a < D; ++a) cth[a * nb + k] = th[a];
        flag[k] = keep ? (far ? 2 : 1) : 0;
    }
}

// ------------------------------------------------------------------ assignment
template <int D>
__global__ __launch_bounds__(256) void k_tile_assign(int m, const double* __restrict__ ty, int64_t ldt, int64_t n,
                                                     const double* __restrict__ ys, int64_t lds,
                                                     int* __restrict__ tile_of) {
    __shared__ double tl[256 * D];
    const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double y[D];
#pragma unroll
    for (int a = 0; a < D; ++a) y[a] = (s < n) ? ys[a * lds + s] : 0.0;
    double bd = INFINITY;
    int best = 0;
    for (int j0 = 0; j0 < m; j0 += 256) {
        const int cnt = min(256, m - j0);
        __syncthreads();
        for (int q = threadIdx.x; q < cnt * D; q += 256) {
            const int a = q / cnt, j = q - a * cnt;
            tl[a * 256 + j] = ty[a * ldt + j0 + j];
        }
        __syncthreads();
        for (int j = 0; j < cnt; ++j) {
            const double d = wdist2<D>(y, 1, tl + j, 256);
            if (d < bd || j0 + j == 0) {
                bd = d;
                best = j0 + j;
            }
        }
    }
    if (s < n) tile_of[s] = best;
}

// ------------------------------------------------------ assignment by match
// Tiles by waveform similarity (App. A), for the 4-D set (one detector, a
// common amplitude f^-7/6): the match of a sample s and a template t is
//   |sum_k pw_k exp(2 pi i (Psi_s(f_k) - Psi_t(f_k)))| / sqrt(P_s P_t),
// over the bins below both cuts, pw = 4 df f^-7/3 / S, P the prefix of pw at a
// point's cut (its norm), Psi in turns with the 2 pi f tc term. Each sample's
// candidates are its n_cand nearest templates in whitened coordinates; the
// match picks among them (the lowest template index among equal matches).

// Coefficient rows of points: A0..A7, B5, B6, tc, and the detector weights
// |R_d|^2 / sum_e |R_e|^2 ([kMatchRow][n]); cut; norm sum_d w_d P_d(cut).
constexpr int kMatchW = 11;
constexpr int kMatchRow = kMatchW + PE_MAX_DET;

__global__ __launch_bounds__(256) void k_match_rows(EvConst ec, const double* __restrict__ th, int64_t ld, int64_t n,
                                                    const double* __restrict__ pfx, double* __restrict__ rows,
                                                    int* __restrict__ kc, double* __restrict__ nrm) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        double t[PE_MAX_DIM];
#pragma unroll
        for (int a = 0; a < PE_MAX_DIM; ++a) t[a] = a < ec.dim ? th[a * ld + i] : 0.0;
        Src s;
        const int ok = source_from_theta(ec, t, s);
        PhaseCoef pc;
        phase_coeffs(s, pc);
#pragma unroll
        for (int a = 0; a < 8; ++a) rows[a * n + i] = pc.A[a];
        rows[8 * n + i] = pc.B5;
        rows[9 * n + i] = pc.B6;
        rows[10 * n + i] = s.tc + s.dt[0];
        const int k = ok ? (int)kcut_of(ec, s.fisco) : 0;
        // detector weights: each detector's share of the point's response power
        // (one detector: exactly 1)
        double r2[PE_MAX_DET], tot = 0.0;
#pragma unroll
        for (int d = 0; d < PE_MAX_DET; ++d) {
            r2[d] = (d < ec.n_det) ? s.rre[d] * s.rre[d] + s.rim[d] * s.rim[d] : 0.0;
            tot += r2[d];
        }
        double nm = 0.0;
#pragma unroll
        for (int d = 0; d < PE_MAX_DET; ++d) {
            const double w = (d >= ec.n_det) ? 0.0 : (tot > 0.0 ? r2[d] / tot : 1.0 / ec.n_det);
            rows[(kMatchW + d) * n + i] = w;
            if (d < ec.n_det) nm += w * pfx[(int64_t)d * (ec.K + 1) + k];
        }
        kc[i] = k;
        nrm[i] = nm;
    }
}

// The n_cand nearest templates of each sample, nearest first (ties: lower index).
template <int C>
__global__ __launch_bounds__(256) void k_tile_topc(int m, const double* __restrict__ ty, int64_t ldt, int64_t n,
                                                   const double* __restrict__ ys, int64_t lds,
                                                   int* __restrict__ cand) {
    __shared__ double tl[256 * 4];
    const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double y[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) y[a] = (s < n) ? ys[a * lds + s] : 0.0;
    double bd[C];
    int bi[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        bd[c] = INFINITY;
        bi[c] = 0;
    }
    for (int j0 = 0; j0 < m; j0 += 256) {
        const int cnt = min(256, m - j0);
        __syncthreads();
        for (int q = threadIdx.x; q < cnt * 4; q += 256) {
            const int a = q / cnt, j = q - a * cnt;
            tl[a * 256 + j] = ty[a * ldt + j0 + j];
        }
        __syncthreads();
        for (int j = 0; j < cnt; ++j) {
            double d = wdist2<4>(y, 1, tl + j, 256);
            int id = j0 + j;
            // insertion into the sorted list (strictly smaller distance moves ahead)
#pragma unroll
            for (int c = 0; c < C; ++c) {
                if (d < bd[c]) {
                    const double td = bd[c];
                    const int ti = bi[c];
                    bd[c] = d;
                    bi[c] = id;
                    d = td;
                    id = ti;
                }
            }
        }
    }
    if (s < n)
#pragma unroll
        for (int c = 0; c < C; ++c) cand[(int64_t)c * n + s] = (c < m) ? bi[c] : bi[0];
}

// MERGE: keep the better of this launch's choice and the one already in
// tile_of/match (earlier launches took lower template indices).
template <int C, bool MERGE = false>
__global__ __launch_bounds__(256) void k_tile_match(const Rec64* __restrict__ tab, const double* __restrict__ pw,
                                                    int n_det, int64_t K, int64_t n, const double* __restrict__ srow,
                                                    const int* __restrict__ skc, const double* __restrict__ snrm,
                                                    int64_t m, const double* __restrict__ trow,
                                                    const int* __restrict__ tkc, const double* __restrict__ tnrm,
                                                    const int* __restrict__ cand, int* __restrict__ tile_of,
                                                    double* __restrict__ match) {
    const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const bool valid = s < n;
    const int64_t sl = valid ? s : n - 1;
    double As[8], Ts[C][8], B5s, B6s, tcs, B5t[C], B6t[C], tct[C];
#pragma unroll
    for (int a = 0; a < 8; ++a) As[a] = srow[a * n + sl];
    B5s = srow[8 * n + sl];
    B6s = srow[9 * n + sl];
    tcs = srow[10 * n + sl];
    double wd[PE_MAX_DET];
#pragma unroll
    for (int d = 0; d < PE_MAX_DET; ++d) wd[d] = srow[(kMatchW + d) * n + sl];
    const int kcs = skc[sl];
    int ti[C], kl[C], kmax = 0;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        ti[c] = cand[(int64_t)c * n + sl];
#pragma unroll
        for (int a = 0; a < 8; ++a) Ts[c][a] = trow[a * m + ti[c]];
        B5t[c] = trow[8 * m + ti[c]];
        B6t[c] = trow[9 * m + ti[c]];
        tct[c] = trow[10 * m + ti[c]];
        kl[c] = min(kcs, tkc[ti[c]]);
        kmax = max(kmax, kl[c]);
    }
    // the wave walks to its largest cut; lanes mask the bins past theirs
    int wk = kmax;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) wk = max(wk, __shfl_xor(wk, o));
    wk = __builtin_amdgcn_readfirstlane(wk);
    double ar[C], ai[C];
#pragma unroll
    for (int c = 0; c < C; ++c) ar[c] = ai[c] = 0.0;
    for (int k = 0; k < wk; ++k) {
        const Rec64 r = load_const(tab + k);
        // the bin's weight over the detectors (the points share their responses)
        double w = wd[0] * load_const(pw + k);
        for (int d = 1; d < n_det; ++d) w = fma(wd[d], load_const(pw + (int64_t)d * K + k), w);
        const double ps = fma(r.f, tcs, psi_turns(As, B5s, B6s, r.x, r.xm5, r.lnx));
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const double pt = fma(r.f, tct[c], psi_turns(Ts[c], B5t[c], B6t[c], r.x, r.xm5, r.lnx));
            double sn, cs;
            sincos_turns(fract64(ps - pt), sn, cs);
            const double wm = (k < kl[c]) ? w : 0.0;
            ar[c] = fma(wm, cs, ar[c]);
            ai[c] = fma(wm, sn, ai[c]);
        }
    }
    if (!valid) return;
    double bm = -1.0;
    int best = ti[0];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const double den = snrm[s] * tnrm[ti[c]];
        const double mc = den > 0.0 ? hypot(ar[c], ai[c]) / sqrt(den) : 0.0;
        if (mc > bm || (mc == bm && ti[c] < best)) {
            bm = mc;
            best = ti[c];
        }
    }
    if (MERGE && !(bm > match[s])) return;  // ties keep the lower index found before
    tile_of[s] = best;
    if (match) match[s] = bm;
}

// The match maximised over the time shifts tau_j = j dt (|j| <= n_shift) too,
// one lane per (candidate c, sample s) pair p = c n + s: per block of 8 shifts,
// a walk over the bins accumulates O_j = sum_k W_k exp(2 pi i (Psi_s - Psi_t -
// f_k tau_j)), the block's first rotation from its angle, the next ones by the
// bin's step exp(-2 pi i f_k dt); out[p] = max_j |O_j| / sqrt(P_s P_t).
// k_pick_shift then takes each sample's best candidate.
constexpr int kShiftBlock = 8;

__global__ __launch_bounds__(256) void k_tile_match_shift(const Rec64* __restrict__ tab, const double* __restrict__ pw,
                                                          int n_det, int64_t K, int64_t n,
                                                          const double* __restrict__ srow, const int* __restrict__ skc,
                                                          const double* __restrict__ snrm, int64_t m,
                                                          const double* __restrict__ trow, const int* __restrict__ tkc,
                                                          const double* __restrict__ tnrm, const int* __restrict__ cand,
                                                          int n_cand, double dt, int n_shift,
                                                          const double2* __restrict__ step, double* __restrict__ out) {
    const int64_t np = (int64_t)n_cand * n;
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const bool valid = p < np;
    const int64_t pl = valid ? p : np - 1;
    const int64_t sl = pl % n;
    double As[8], B5s, B6s, tcs;
#pragma unroll
    for (int a = 0; a < 8; ++a) As[a] = srow[a * n + sl];
    B5s = srow[8 * n + sl];
    B6s = srow[9 * n + sl];
    tcs = srow[10 * n + sl];
    double wd[PE_MAX_DET];
#pragma unroll
    for (int d = 0; d < PE_MAX_DET; ++d) wd[d] = srow[(kMatchW + d) * n + sl];
    const int ti = cand[pl];
    double At[8];
#pragma unroll
    for (int a = 0; a < 8; ++a) At[a] = trow[a * m + ti];
    const double B5t = trow[8 * m + ti], B6t = trow[9 * m + ti], tct = trow[10 * m + ti];
    const int kl = min(skc[sl], tkc[ti]);
    int wk = kl;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) wk = max(wk, __shfl_xor(wk, o));
    wk = __builtin_amdgcn_readfirstlane(wk);
    const int nj = 2 * n_shift + 1;
    double mc = 0.0;
    for (int j0 = 0; j0 < nj; j0 += kShiftBlock) {
        const double tau0 = (double)(j0 - n_shift) * dt;
        double orr[kShiftBlock], oi[kShiftBlock];
#pragma unroll
        for (int q = 0; q < kShiftBlock; ++q) orr[q] = oi[q] = 0.0;
        for (int k = 0; k < wk; ++k) {
            const Rec64 r = load_const(tab + k);
            double w = wd[0] * load_const(pw + k);
            for (int d = 1; d < n_det; ++d) w = fma(wd[d], load_const(pw + (int64_t)d * K + k), w);
            const double ps = fma(r.f, tcs, psi_turns(As, B5s, B6s, r.x, r.xm5, r.lnx));
            const double pt = fma(r.f, tct, psi_turns(At, B5t, B6t, r.x, r.xm5, r.lnx));
            double sn, cs;
            sincos_turns(fract64(ps - pt - r.f * tau0), sn, cs);
            const double2 rot = load_const(step + k);  // (cos, sin) of -2 pi f_k dt
            const double rc = rot.x, rs = rot.y;
            const double wm = (k < kl) ? w : 0.0;
            double zr = wm * cs, zi = wm * sn;
#pragma unroll
            for (int q = 0; q < kShiftBlock; ++q) {
                orr[q] += zr;
                oi[q] += zi;
                const double nr = zr * rc - zi * rs;
                zi = zr * rs + zi * rc;
                zr = nr;
            }
        }
#pragma unroll
        for (int q = 0; q < kShiftBlock; ++q)
            if (j0 + q < nj) mc = fmax(mc, hypot(orr[q], oi[q]));
    }
    if (!valid) return;
    const double den = snrm[sl] * tnrm[ti];
    out[p] = den > 0.0 ? mc / sqrt(den) : 0.0;
}

// The shift step of every bin: (cos, sin) of -2 pi f_k dt, as the walk would
// form it per bin (the same function of the same argument).
__global__ __launch_bounds__(256) void k_shift_step(const Rec64* __restrict__ tab, int64_t K, double dt,
                                                    double2* __restrict__ step) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= K) return;
    double rs, rc;
    sincos_turns(fract64(-tab[k].f * dt), rs, rc);
    step[k] = make_double2(rc, rs);
}

// Each sample's best of its n_cand candidates (ties: the lower index); MERGE
// keeps the better of that and the choice already in tile_of/match.
template <bool MERGE>
__global__ __launch_bounds__(256) void k_pick_shift(int64_t n, int n_cand, const int* __restrict__ cand,
                                                    const double* __restrict__ mcs, int* __restrict__ tile_of,
                                                    double* __restrict__ match) {
    const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (s >= n) return;
    double bm = -1.0;
    int best = cand[s];
    for (int c = 0; c < n_cand; ++c) {
        const int ti = cand[(int64_t)c * n + s];
        const double mc = mcs[(int64_t)c * n + s];
        if (mc > bm || (mc == bm && ti < best)) {
            bm = mc;
            best = ti;
        }
    }
    if (MERGE && !(bm > match[s])) return;
    tile_of[s] = best;
    match[s] = bm;
}

// Candidates t0 .. t0 + 7 for every sample (the last template repeated past m).
__global__ __launch_bounds__(256) void k_fill_cand(int* __restrict__ cand, int64_t n, int t0, int m) {
    const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (s >= n) return;
#pragma unroll
    for (int c = 0; c < 8; ++c) cand[(int64_t)c * n + s] = min(t0 + c, m - 1);
}

// ---------------------------------------------------------------------- draws
// part[2 b] = max finite tile log-likelihood seen by block b, part[2 b + 1] =
// max finite sample log prior (order-free, so deterministic).
__global__ __launch_bounds__(256) void k_tile_max(int m, const double* __restrict__ tll, int64_t P,
                                                  const double* __restrict__ lp, double* __restrict__ part) {
    __shared__ double sh[8];
    double a = -INFINITY, b = -INFINITY;
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < m; j += stride)
        if (isfinite(tll[j])) a = fmax(a, tll[j]);
    for (int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x; s < P; s += stride)
        if (isfinite(lp[s])) b = fmax(b, lp[s]);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        a = fmax(a, __shfl_xor(a, o));
        b = fmax(b, __shfl_xor(b, o));
    }
    if ((threadIdx.x & 63) == 0) {
        sh[threadIdx.x >> 6] = a;
        sh[4 + (threadIdx.x >> 6)] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
        part[2 * blockIdx.x + 1] = fmax(fmax(sh[4], sh[5]), fmax(sh[6], sh[7]));
    }
}

// mass[s] = exp((ll_t(s) - lmax) + (lp_s - pmax)), the maxima folded from the
// nb block parts first (every thread folds them: nb is small).
__global__ __launch_bounds__(256) void k_tile_mass(const double* __restrict__ part, int nb,
                                                   const double* __restrict__ tll, const int* __restrict__ tile_of,
                                                   const double* __restrict__ lp, int64_t P, double* __restrict__ mass,
                                                   double* __restrict__ mx) {
    double lmax = -INFINITY, pmax = -INFINITY;
    for (int b = 0; b < nb; ++b) {
        lmax = fmax(lmax, part[2 * b]);
        pmax = fmax(pmax, part[2 * b + 1]);
    }
    const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (s == 0) {
        mx[0] = lmax;
        mx[1] = pmax;
    }
    if (s >= P) return;
    const double l = tll[tile_of[s]], p = lp[s];
    mass[s] = (isfinite(l) && isfinite(p)) ? exp((l - lmax) + (p - pmax)) : 0.0;
}

// Inclusive prefix sums of x[0..P) in place, in two passes over nseg
// contiguous segments: segment sums, then each segment adds the sums before
// it (one block reduction) and scans its elements 256 at a time.
__device__ __forceinline__ double block_sum(double s, double* sh) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    const double r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(256) void k_scan_sums(const double* __restrict__ x, int64_t P, int64_t seg,
                                                   double* __restrict__ ssum) {
    __shared__ double sh[4];
    const int64_t k0 = (int64_t)blockIdx.x * seg, k1 = min(P, k0 + seg);
    double s = 0.0;
    for (int64_t k = k0 + threadIdx.x; k < k1; k += 256) s += x[k];
    s = block_sum(s, sh);
    if (threadIdx.x == 0) ssum[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_scan_write(double* __restrict__ x, int64_t P, int64_t seg,
                                                    const double* __restrict__ ssum) {
    __shared__ double sh[4];
    const int b = blockIdx.x;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    double carry = 0.0;
    for (int q = threadIdx.x; q < b; q += 256) carry += ssum[q];
    carry = block_sum(carry, sh);
    const int64_t k0 = (int64_t)b * seg, k1 = min(P, k0 + seg);
    for (int64_t base = k0; base < k1; base += 256) {
        const int64_t k = base + threadIdx.x;
        double inc = (k < k1) ? x[k] : 0.0;
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
        if (k < k1) x[k] = carry + (woff + inc);
        carry += tile;
    }
}

template <int D>
__global__ __launch_bounds__(256) void k_tile_pick(const double* __restrict__ C, int64_t P,
                                                   const double* __restrict__ mx, const double* __restrict__ tll,
                                                   const int* __restrict__ tile_of, const double* __restrict__ lp,
                                                   const double* __restrict__ smp, int64_t ld, uint64_t seed,
                                                   uint32_t st, int64_t n, double* __restrict__ theta,
                                                   double* __restrict__ logq, double* __restrict__ logprior,
                                                   int64_t* __restrict__ index) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const double tot = P > 0 ? C[P - 1] : 0.0;
    if (!(tot > 0.0)) {
#pragma unroll
        for (int a = 0; a < D; ++a) theta[a * n + i] = P > 0 ? smp[a * ld] : 0.0;
        logq[i] = 0.0;
        logprior[i] = -INFINITY;
        if (index) index[i] = -1;
        return;
    }
    double u, u2;
    block_uniforms(seed, st, (uint64_t)i, 0u, u, u2);
    const double target = u * tot;
    int64_t lo = 0, hi = P - 1;
    while (lo < hi) {  // smallest s with target <= C_s
        const int64_t mid = lo + (hi - lo) / 2;
        if (target <= C[mid])
            hi = mid;
        else
            lo = mid + 1;
    }
    const int64_t s = lo;
#pragma unroll
    for (int a = 0; a < D; ++a) theta[a * n + i] = smp[a * ld + s];
    logprior[i] = lp[s];
    logq[i] = ((tll[tile_of[s]] - mx[0]) + (lp[s] - mx[1])) - log(tot / (double)P);
    if (index) index[i] = s;
}

// --------------------------------------------------------------- reweighting
// Per-tile sums in 64-bit fixed point (order-free, so deterministic): prior
// volume in units of 2^-32 of the largest sample's, weights in units of 2^-52.
constexpr double kVolScale = 4294967296.0;         // 2^32
constexpr double kWScale = 4503599627370496.0;     // 2^52

__global__ void k_rw_zero(int m, unsigned long long* __restrict__ a, unsigned long long* __restrict__ b) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j < m) {
        a[j] = 0ull;
        b[j] = 0ull;
    }
}

__global__ __launch_bounds__(256) void k_rw_prior(const double* __restrict__ part, int nb, int64_t P,
                                                  const int* __restrict__ tile_of, const double* __restrict__ lp,
                                                  unsigned long long* __restrict__ vfx) {
    double pmax = -INFINITY;
    for (int b = 0; b < nb; ++b) pmax = fmax(pmax, part[2 * b + 1]);
    const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (s >= P || !isfinite(lp[s])) return;
    atomicAdd(&vfx[tile_of[s]], (unsigned long long)rint(exp(lp[s] - pmax) * kVolScale));
}

__global__ __launch_bounds__(256) void k_rw_post(int64_t n, const int64_t* __restrict__ index,
                                                 const double* __restrict__ w, const int* __restrict__ tile_of,
                                                 unsigned long long* __restrict__ pfx) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n || index[i] < 0 || !(w[i] > 0.0)) return;
    atomicAdd(&pfx[tile_of[index[i]]], (unsigned long long)rint(fmin(w[i], 1.0) * kWScale));
}

// One workgroup: sum_j exp(l_j - lmax) V_j (fixed order) and sum_j P_j, then
// out_j = ln((1 - alpha) P_j / sum P + alpha p_j) - ln V_j.
__global__ __launch_bounds__(1024) void k_rw_final(int m, const double* __restrict__ tll,
                                                   const double* __restrict__ part, int nb,
                                                   const unsigned long long* __restrict__ vfx,
                                                   const unsigned long long* __restrict__ pfx, double alpha,
                                                   double* __restrict__ out) {
    __shared__ double shp[16];
    __shared__ unsigned long long shw[16];
    double lmax = -INFINITY;
    for (int b = 0; b < nb; ++b) lmax = fmax(lmax, part[2 * b]);
    double ps = 0.0;
    unsigned long long ws = 0ull;
    for (int j = threadIdx.x; j < m; j += 1024) {
        if (isfinite(tll[j])) ps += exp(tll[j] - lmax) * ((double)vfx[j] / kVolScale);
        ws += pfx[j];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        ps += __shfl_xor(ps, o);
        ws += __shfl_xor(ws, o);
    }
    if ((threadIdx.x & 63) == 0) {
        shp[threadIdx.x >> 6] = ps;
        shw[threadIdx.x >> 6] = ws;
    }
    __syncthreads();
    double ptot = 0.0;
    unsigned long long wtot = 0ull;
    for (int q = 0; q < 16; ++q) {
        ptot += shp[q];
        wtot += shw[q];
    }
    for (int j = threadIdx.x; j < m; j += 1024) {
        const double v = (double)vfx[j] / kVolScale;
        const double pj = (ptot > 0.0 && isfinite(tll[j])) ? exp(tll[j] - lmax) * v / ptot : 0.0;
        const double hj = wtot > 0ull ? (double)pfx[j] / (double)wtot : 0.0;
        const double pi = (1.0 - alpha) * hj + alpha * pj;
        out[j] = (pi > 0.0 && v > 0.0) ? log(pi) - log(v) : -INFINITY;
    }
}

// ------------------------------------------------------------------- scratch
// One growing device buffer per stream; work on a stream is ordered, so it is
// reused safely, and the stream is drained before a buffer is replaced.
std::mutex g_scr_mu;
std::map<hipStream_t, std::pair<char*, size_t>> g_scr;

pe_status_t scratch_for(hipStream_t st, size_t bytes, char** out) {
    std::lock_guard<std::mutex> lk(g_scr_mu);
    auto& e = g_scr[st];
    if (e.second < bytes) {
        PE_HIP(hipStreamSynchronize(st));
        dfree_bytes(e.first);
        e.second = 0;
        pe_status_t s = dalloc_bytes(&e.first, bytes);
        if (s != PE_OK) return s;
        e.second = bytes;
    }
    *out = e.first;
    return PE_OK;
}

// Number of sliced coordinates (the event's D without a sub_mask).
int slice_dims(const pe_event_s* ev, const pe_slice_t& s) {
    return s.sub_mask == 0 ? ev->ec.dim : __builtin_popcount(s.sub_mask);
}

Slice to_slice(const pe_event_s* ev, const pe_slice_t& s) {
    Slice o;
    for (int a = 0; a < PE_MAX_DIM; ++a) o.c[a] = s.centre[a];
    for (int a = 0; a < PE_MAX_DIM * PE_MAX_DIM; ++a) o.L[a] = s.chol[a];
    o.R = s.radius;
    int S = 0;
    for (int a = 0; a < PE_MAX_DIM; ++a) o.idx[a] = 0;
    for (int a = 0; a < ev->ec.dim; ++a)
        if (s.sub_mask == 0 || (s.sub_mask >> a & 1u)) o.idx[S++] = a;
    return o;
}

pe_status_t check_slice(const pe_event_s* ev, const pe_slice_t* s) {
    if (!ev) return fail(PE_ERR_ARG, "event is NULL");
    if (!s) return fail(PE_ERR_ARG, "slice is NULL");
    const int D = ev->ec.dim;
    if (s->sub_mask != 0 && (D != 11 || (s->sub_mask >> 11) != 0 || __builtin_popcount(s->sub_mask) != 4))
        return fail(PE_ERR_ARG, "sub_mask must be 0 or name 4 of the 11 coordinates of an 11-D event");
    const int S = slice_dims(ev, *s);
    if (!(s->radius > 0.0) || !std::isfinite(s->radius)) return fail(PE_ERR_ARG, "slice radius must be > 0");
    for (int r = 0; r < D; ++r)
        if (!std::isfinite(s->centre[r])) return fail(PE_ERR_ARG, "slice centre must be finite");
    for (int r = 0; r < S; ++r) {
        if (!(s->chol[r * S + r] > 0.0)) return fail(PE_ERR_ARG, "slice factor needs a positive diagonal");
        for (int c = 0; c <= r; ++c)
            if (!std::isfinite(s->chol[r * S + c])) return fail(PE_ERR_ARG, "slice factor must be finite");
    }
    return PE_OK;
}

unsigned nblocks(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace
}  // namespace pe

using namespace pe;

extern "C" pe_status_t pe_slice_sample(pe_event_t ev, const pe_slice_t* slice, uint64_t seed, uint32_t stream_id,
                                       int64_t first, int64_t n, double* y_dev, double* theta_dev,
                                       double* logprior_dev, int64_t* count_dev, void* stream) {
    pe_status_t s = check_slice(ev, slice);
    if (s != PE_OK) return s;
    if (n < 0 || n > ((int64_t)1 << 30) || first < 0) return fail(PE_ERR_ARG, "n must be in 0..2^30, first >= 0");
    if (!count_dev || (n > 0 && (!y_dev || !theta_dev || !logprior_dev)))
        return fail(PE_ERR_ARG, "output pointers are NULL");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const int64_t nb = std::max<int64_t>(1, (n + 255) / 256);
    char* scr = nullptr;
    if ((s = scratch_for(st, sizeof(int64_t) * nb, &scr)) != PE_OK) return s;
    int64_t* bc = reinterpret_cast<int64_t*>(scr);
    const Slice sl = to_slice(ev, *slice);
    const EvConst& ec = ev->ec;
    if (n == 0) {
        k_set_count<<<1, 1, 0, st>>>(count_dev);
        PE_HIP(hipGetLastError());
        return PE_OK;
    }
    const int S = slice_dims(ev, *slice);
    if (ec.dim == 4) {
        k_slice_count<4, 4><<<nblocks(n), 256, 0, st>>>(ec, sl, seed, stream_id, first, n, bc);
        k_slice_scan<<<1, 1024, 0, st>>>(bc, nb, count_dev);
        k_slice_write<4, 4><<<nblocks(n), 256, 0, st>>>(ec, sl, seed, stream_id, first, n, bc, y_dev, theta_dev,
                                                         logprior_dev);
    } else if (S == 11) {
        k_slice_count<11, 11><<<nblocks(n), 256, 0, st>>>(ec, sl, seed, stream_id, first, n, bc);
        k_slice_scan<<<1, 1024, 0, st>>>(bc, nb, count_dev);
        k_slice_write<11, 11><<<nblocks(n), 256, 0, st>>>(ec, sl, seed, stream_id, first, n, bc, y_dev, theta_dev,
                                                           logprior_dev);
    } else {
        k_slice_count<4, 11><<<nblocks(n), 256, 0, st>>>(ec, sl, seed, stream_id, first, n, bc);
        k_slice_scan<<<1, 1024, 0, st>>>(bc, nb, count_dev);
        k_slice_write<4, 11><<<nblocks(n), 256, 0, st>>>(ec, sl, seed, stream_id, first, n, bc, y_dev, theta_dev,
                                                          logprior_dev);
    }
    PE_HIP(hipGetLastError());
    return PE_OK;
}

extern "C" pe_status_t pe_tile_bank(pe_event_t ev, const pe_slice_t* slice, double min_dist, uint64_t seed,
                                    uint32_t stream_id, int32_t batch, int32_t max_tiles, double stop_fraction,
                                    int32_t max_batches, double* tiles_y_dev, double* tiles_theta_dev,
                                    int32_t* n_tiles, int64_t* consumed, void* stream) {
    pe_status_t s = check_slice(ev, slice);
    if (s != PE_OK) return s;
    if (!(min_dist > 0.0) || batch < 1 || batch > (1 << 20) || max_tiles < 1 || max_tiles > (1 << 24) ||
        max_batches < 1 || !(stop_fraction >= 0.0))
        return fail(PE_ERR_ARG, "bad bank parameters");
    if (!tiles_y_dev || !tiles_theta_dev || !n_tiles || !consumed) return fail(PE_ERR_ARG, "NULL output");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const int D = ev->ec.dim;
    const int S = slice_dims(ev, *slice);
    const Slice sl = to_slice(ev, *slice);
    const double r2 = min_dist * min_dist;
    char* scr = nullptr;
    const size_t cand_bytes = sizeof(double) * (S + D) * (size_t)batch;
    if ((s = scratch_for(st, cand_bytes + sizeof(int) * (size_t)batch, &scr)) != PE_OK) return s;
    double* cy = reinterpret_cast<double*>(scr);
    double* cth = cy + (size_t)S * batch;
    int* flag = reinterpret_cast<int*>(scr + cand_bytes);
    std::vector<double> hy((size_t)S * batch), hth((size_t)D * batch);
    std::vector<int> hf(batch);
    std::vector<double> ny, nth;  // this batch's new templates, [k][S] and [k][D]
    int m = 0;
    int64_t used = 0;
    for (int b = 0; b < max_batches && m < max_tiles; ++b) {
        const int64_t b0 = (int64_t)b * batch;
        if (D == 4)
            k_bank_cand<4, 4><<<nblocks(batch), 256, 0, st>>>(ev->ec, sl, seed, stream_id, b0, batch, tiles_y_dev,
                                                               max_tiles, m, r2, cy, cth, flag);
        else if (S == 11)
            k_bank_cand<11, 11><<<nblocks(batch), 256, 0, st>>>(ev->ec, sl, seed, stream_id, b0, batch,
                                                                 tiles_y_dev, max_tiles, m, r2, cy, cth, flag);
        else
            k_bank_cand<4, 11><<<nblocks(batch), 256, 0, st>>>(ev->ec, sl, seed, stream_id, b0, batch, tiles_y_dev,
                                                                max_tiles, m, r2, cy, cth, flag);
        PE_HIP(hipGetLastError());
        PE_HIP(hipMemcpyAsync(hy.data(), cy, sizeof(double) * S * batch, hipMemcpyDeviceToHost, st));
        PE_HIP(hipMemcpyAsync(hth.data(), cth, sizeof(double) * D * batch, hipMemcpyDeviceToHost, st));
        PE_HIP(hipMemcpyAsync(hf.data(), flag, sizeof(int) * batch, hipMemcpyDeviceToHost, st));
        PE_HIP(hipStreamSynchronize(st));
        const int m0 = m;
        int64_t kept = 0, added = 0;
        ny.clear();
        nth.clear();
        for (int i = 0; i < batch && m < max_tiles; ++i) {
            used = b0 + i + 1;
            if (hf[i] == 0) continue;
            ++kept;
            if (hf[i] != 2) continue;
            bool ok = true;
            for (int j = 0; j < m - m0 && ok; ++j)
                if (wdist2_rt(S, hy.data() + i, batch, ny.data() + (size_t)j * S, 1) < r2) ok = false;
            if (!ok) continue;
            for (int a = 0; a < S; ++a) ny.push_back(hy[(size_t)a * batch + i]);
            for (int a = 0; a < D; ++a) nth.push_back(hth[(size_t)a * batch + i]);
            ++m;
            ++added;
        }
        // append the new templates, one row segment per coordinate
        if (added > 0) {
            std::vector<double> rowy(added), rowt(added);
            for (int a = 0; a < D; ++a) {
                for (int64_t j = 0; j < added; ++j) {
                    if (a < S) rowy[j] = ny[(size_t)j * S + a];
                    rowt[j] = nth[(size_t)j * D + a];
                }
                if (a < S)
                    PE_HIP(hipMemcpyAsync(tiles_y_dev + (size_t)a * max_tiles + m0, rowy.data(),
                                          sizeof(double) * added, hipMemcpyHostToDevice, st));
                PE_HIP(hipMemcpyAsync(tiles_theta_dev + (size_t)a * max_tiles + m0, rowt.data(),
                                      sizeof(double) * added, hipMemcpyHostToDevice, st));
                // the copies read rowy and rowt: drain before the next row overwrites them
                PE_HIP(hipStreamSynchronize(st));
            }
        }
        if (m >= max_tiles || (double)added < stop_fraction * (double)kept) break;
    }
    *n_tiles = m;
    *consumed = used;
    return PE_OK;
}

extern "C" pe_status_t pe_tile_assign(int32_t dim, int32_t n_tiles, const double* tiles_y_dev, int64_t ld_tiles,
                                      int64_t n, const double* y_dev, int64_t ld_y, int32_t* tile_of_dev,
                                      void* stream) {
    if (dim != 4 && dim != 11) return fail(PE_ERR_ARG, "dim must be 4 or 11");
    if (n_tiles < 1 || n_tiles > (1 << 24) || ld_tiles < n_tiles) return fail(PE_ERR_ARG, "bad n_tiles or ld_tiles");
    if (n < 0 || n > ((int64_t)1 << 30) || ld_y < n) return fail(PE_ERR_ARG, "bad n or ld_y");
    if (!tiles_y_dev || (n > 0 && (!y_dev || !tile_of_dev))) return fail(PE_ERR_ARG, "NULL pointer");
    if (n == 0) return PE_OK;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (dim == 4)
        k_tile_assign<4><<<nblocks(n), 256, 0, st>>>(n_tiles, tiles_y_dev, ld_tiles, n, y_dev, ld_y, tile_of_dev);
    else
        k_tile_assign<11><<<nblocks(n), 256, 0, st>>>(n_tiles, tiles_y_dev, ld_tiles, n, y_dev, ld_y, tile_of_dev);
    PE_HIP(hipGetLastError());
    return PE_OK;
}

// pe_tile_assign_match (n_shift 0) and pe_tile_assign_match_shift.
static pe_status_t assign_match(pe_event_t ev, int32_t n_tiles, const double* tiles_y_dev,
                                const double* tiles_theta_dev, int64_t ld_tiles, int64_t n, const double* y_dev,
                                const double* theta_dev, int64_t ld, int32_t n_cand, double dt, int32_t n_shift,
                                int32_t* tile_of_dev, double* match_dev, void* stream) {
    if (!ev) return fail(PE_ERR_ARG, "event is NULL");
    if (n_shift < 0 || n_shift > 4096) return fail(PE_ERR_ARG, "n_shift must be in 0..4096");
    if (n_shift > 0 && !(dt > 0.0 && std::isfinite(dt))) return fail(PE_ERR_ARG, "dt must be positive and finite");
    if (n_shift > 0 && match_dev == nullptr) return fail(PE_ERR_ARG, "the shift search needs match_dev");
    if (ev->desc.params == PE_PARAMS_4D && ev->desc.n_det != 1)
        return fail(PE_ERR_ARG, "match-based tiles of the 4-D parameter set take one detector");
    if (n_cand != 0 && n_cand != 1 && n_cand != 2 && n_cand != 4 && n_cand != 8)
        return fail(PE_ERR_ARG, "n_cand must be 0 (every template), 1, 2, 4 or 8");
    if (n_tiles < 1 || n_tiles > (1 << 24) || ld_tiles < n_tiles) return fail(PE_ERR_ARG, "bad n_tiles or ld_tiles");
    if (n < 0 || n > ((int64_t)1 << 30) || ld < n) return fail(PE_ERR_ARG, "bad n or ld");
    if (!tiles_y_dev || !tiles_theta_dev || (n > 0 && (!y_dev || !theta_dev || !tile_of_dev)))
        return fail(PE_ERR_ARG, "NULL pointer");
    if (n == 0) return PE_OK;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    // scratch: rows, cuts and norms of the templates and samples, the pairs'
    // matches and the bins' shift steps (shift search), the candidates; sized by
    // a measuring pass of the same carving (each buffer 256-byte aligned)
    const int64_t m = n_tiles;
    double *trow, *tnrm, *srow, *snrm, *pmc = nullptr;
    double2* step = nullptr;
    int *tkc, *skc, *cand;
    auto carve = [&](Carver& c) {
        trow = c.take<double>((size_t)kMatchRow * m);
        tnrm = c.take<double>((size_t)m);
        srow = c.take<double>((size_t)kMatchRow * n);
        snrm = c.take<double>((size_t)n);
        tkc = c.take<int>((size_t)m);
        skc = c.take<int>((size_t)n);
        if (n_shift > 0) {
            pmc = c.take<double>((size_t)8 * n);
            step = c.take<double2>((size_t)ev->ec.K);
        }
        cand = c.take<int>((size_t)(n_cand ? n_cand : 8) * n);
    };
    Carver meas(nullptr);
    carve(meas);
    char* mem = nullptr;
    pe_status_t s = dalloc_bytes(&mem, meas.size());
    if (s != PE_OK) return s;
    Carver c(mem);
    carve(c);
    k_match_rows<<<nblocks(m), 256, 0, st>>>(ev->ec, tiles_theta_dev, ld_tiles, m, ev->pfx, trow, tkc, tnrm);
    k_match_rows<<<nblocks(n), 256, 0, st>>>(ev->ec, theta_dev, ld, n, ev->pfx, srow, skc, snrm);
    if (n_shift > 0) {
        k_shift_step<<<nblocks(ev->ec.K), 256, 0, st>>>(ev->rec64, ev->ec.K, dt, step);
        // candidates: the n_cand nearest, or every template eight per launch
        if (n_cand > 0) {
            switch (n_cand) {
                case 1: k_tile_topc<1><<<nblocks(n), 256, 0, st>>>(n_tiles, tiles_y_dev, ld_tiles, n, y_dev, ld, cand); break;
                case 2: k_tile_topc<2><<<nblocks(n), 256, 0, st>>>(n_tiles, tiles_y_dev, ld_tiles, n, y_dev, ld, cand); break;
                case 4: k_tile_topc<4><<<nblocks(n), 256, 0, st>>>(n_tiles, tiles_y_dev, ld_tiles, n, y_dev, ld, cand); break;
                default: k_tile_topc<8><<<nblocks(n), 256, 0, st>>>(n_tiles, tiles_y_dev, ld_tiles, n, y_dev, ld, cand); break;
            }
            k_tile_match_shift<<<nblocks((int64_t)n_cand * n), 256, 0, st>>>(
                ev->rec64, ev->pw, ev->ec.n_det, ev->ec.K, n, srow, skc, snrm, m, trow, tkc, tnrm, cand, n_cand, dt,
                n_shift, step, pmc);
            k_pick_shift<false><<<nblocks(n), 256, 0, st>>>(n, n_cand, cand, pmc, tile_of_dev, match_dev);
        } else {
            for (int t0 = 0; t0 < n_tiles; t0 += 8) {
                const int nc = std::min(8, n_tiles - t0);
                k_fill_cand<<<nblocks(n), 256, 0, st>>>(cand, n, t0, n_tiles);
                k_tile_match_shift<<<nblocks((int64_t)nc * n), 256, 0, st>>>(
                    ev->rec64, ev->pw, ev->ec.n_det, ev->ec.K, n, srow, skc, snrm, m, trow, tkc, tnrm, cand, nc, dt,
                    n_shift, step, pmc);
                if (t0 == 0)
                    k_pick_shift<false><<<nblocks(n), 256, 0, st>>>(n, nc, cand, pmc, tile_of_dev, match_dev);
                else
                    k_pick_shift<true><<<nblocks(n), 256, 0, st>>>(n, nc, cand, pmc, tile_of_dev, match_dev);
            }
        }
    } else switch (n_cand) {
        case 0:
            // every template, eight per launch, the best kept across launches
            if (match_dev == nullptr) {
                dfree_bytes(mem);
                return fail(PE_ERR_ARG, "n_cand 0 needs match_dev");
            }
            for (int t0 = 0; t0 < n_tiles; t0 += 8) {
                k_fill_cand<<<nblocks(n), 256, 0, st>>>(cand, n, t0, n_tiles);
                if (t0 == 0)
                    k_tile_match<8><<<nblocks(n), 256, 0, st>>>(ev->rec64, ev->pw, ev->ec.n_det, ev->ec.K, n, srow,
                                                                skc, snrm, m, trow, tkc, tnrm, cand, tile_of_dev,
                                                                match_dev);
                else
                    k_tile_match<8, true><<<nblocks(n), 256, 0, st>>>(ev->rec64, ev->pw, ev->ec.n_det, ev->ec.K, n,
                                                                      srow, skc, snrm, m, trow, tkc, tnrm, cand,
                                                                      tile_of_dev, match_dev);
            }
            break;
        case 1:
            k_tile_topc<1><<<nblocks(n), 256, 0, st>>>(n_tiles, tiles_y_dev, ld_tiles, n, y_dev, ld, cand);
            k_tile_match<1><<<nblocks(n), 256, 0, st>>>(ev->rec64, ev->pw, ev->ec.n_det, ev->ec.K, n, srow, skc, snrm, m, trow, tkc, tnrm,
                                                        cand, tile_of_dev, match_dev);
            break;
        case 2:
            k_tile_topc<2><<<nblocks(n), 256, 0, st>>>(n_tiles, tiles_y_dev, ld_tiles, n, y_dev, ld, cand);
            k_tile_match<2><<<nblocks(n), 256, 0, st>>>(ev->rec64, ev->pw, ev->ec.n_det, ev->ec.K, n, srow, skc, snrm, m, trow, tkc, tnrm,
                                                        cand, tile_of_dev, match_dev);
            break;
        case 4:
            k_tile_topc<4><<<nblocks(n), 256, 0, st>>>(n_tiles, tiles_y_dev, ld_tiles, n, y_dev, ld, cand);
            k_tile_match<4><<<nblocks(n), 256, 0, st>>>(ev->rec64, ev->pw, ev->ec.n_det, ev->ec.K, n, srow, skc, snrm, m, trow, tkc, tnrm,
                                                        cand, tile_of_dev, match_dev);
            break;
        default:
            k_tile_topc<8><<<nblocks(n), 256, 0, st>>>(n_tiles, tiles_y_dev, ld_tiles, n, y_dev, ld, cand);
            k_tile_match<8><<<nblocks(n), 256, 0, st>>>(ev->rec64, ev->pw, ev->ec.n_det, ev->ec.K, n, srow, skc, snrm, m, trow, tkc, tnrm,
                                                        cand, tile_of_dev, match_dev);
            break;
    }
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    dfree_bytes(mem);
    if (e != hipSuccess) return fail(PE_ERR_HIP, hipGetErrorString(e));
    return PE_OK;
}

extern "C" pe_status_t pe_tile_assign_match(pe_event_t ev, int32_t n_tiles, const double* tiles_y_dev,
                                            const double* tiles_theta_dev, int64_t ld_tiles, int64_t n,
                                            const double* y_dev, const double* theta_dev, int64_t ld, int32_t n_cand,
                                            int32_t* tile_of_dev, double* match_dev, void* stream) {
    return assign_match(ev, n_tiles, tiles_y_dev, tiles_theta_dev, ld_tiles, n, y_dev, theta_dev, ld, n_cand, 0.0, 0,
                        tile_of_dev, match_dev, stream);
}

extern "C" pe_status_t pe_tile_assign_match_shift(pe_event_t ev, int32_t n_tiles, const double* tiles_y_dev,
                                                  const double* tiles_theta_dev, int64_t ld_tiles, int64_t n,
                                                  const double* y_dev, const double* theta_dev, int64_t ld,
                                                  int32_t n_cand, double dt, int32_t n_shift, int32_t* tile_of_dev,
                                                  double* match_dev, void* stream) {
    if (n_shift < 1) return fail(PE_ERR_ARG, "n_shift must be at least 1");
    return assign_match(ev, n_tiles, tiles_y_dev, tiles_theta_dev, ld_tiles, n, y_dev, theta_dev, ld, n_cand, dt,
                        n_shift, tile_of_dev, match_dev, stream);
}

extern "C" pe_status_t pe_tile_draw(int32_t n_tiles, const double* tile_loglike_dev, int64_t n_samples,
                                    const int32_t* tile_of_dev, const double* sample_logprior_dev, int32_t dim,
                                    const double* samples_theta_dev, int64_t ld, uint64_t seed, uint32_t stream_id,
                                    int64_t n, double* theta_dev, double* logq_dev, double* logprior_dev,
                                    int64_t* index_dev, void* stream) {
    if (dim != 4 && dim != 11) return fail(PE_ERR_ARG, "dim must be 4 or 11");
    if (n_tiles < 1 || n_tiles > (1 << 24)) return fail(PE_ERR_ARG, "bad n_tiles");
    if (n_samples < 1 || n_samples > ((int64_t)1 << 30) || ld < n_samples) return fail(PE_ERR_ARG, "bad n_samples or ld");
    if (n < 0 || n > ((int64_t)1 << 30)) return fail(PE_ERR_ARG, "n must be in 0..2^30");
    if (!tile_loglike_dev || !tile_of_dev || !sample_logprior_dev || !samples_theta_dev)
        return fail(PE_ERR_ARG, "NULL input");
    if (n > 0 && (!theta_dev || !logq_dev || !logprior_dev)) return fail(PE_ERR_ARG, "NULL output");
    if (n == 0) return PE_OK;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const int nbm = 64;
    const int64_t seg = std::max<int64_t>(1024, (n_samples + 1023) / 1024);
    const int nseg = (int)((n_samples + seg - 1) / seg);
    const size_t bytes = sizeof(double) * ((size_t)n_samples + 2 * nbm + 2 + nseg);
    char* scr = nullptr;
    pe_status_t s = scratch_for(st, bytes, &scr);
    if (s != PE_OK) return s;
    double* C = reinterpret_cast<double*>(scr);
    double* part = C + n_samples;
    double* mx = part + 2 * nbm;
    double* ssum = mx + 2;
    k_tile_max<<<nbm, 256, 0, st>>>(n_tiles, tile_loglike_dev, n_samples, sample_logprior_dev, part);
    k_tile_mass<<<nblocks(n_samples), 256, 0, st>>>(part, nbm, tile_loglike_dev, tile_of_dev, sample_logprior_dev,
                                                     n_samples, C, mx);
    k_scan_sums<<<nseg, 256, 0, st>>>(C, n_samples, seg, ssum);
    k_scan_write<<<nseg, 256, 0, st>>>(C, n_samples, seg, ssum);
    if (dim == 4)
        k_tile_pick<4><<<nblocks(n), 256, 0, st>>>(C, n_samples, mx, tile_loglike_dev, tile_of_dev, sample_logprior_dev,
                                                    samples_theta_dev, ld, seed, stream_id, n, theta_dev, logq_dev,
                                                    logprior_dev, index_dev);
    else
        k_tile_pick<11><<<nblocks(n), 256, 0, st>>>(C, n_samples, mx, tile_loglike_dev, tile_of_dev,
                                                     sample_logprior_dev, samples_theta_dev, ld, seed, stream_id, n,
                                                     theta_dev, logq_dev, logprior_dev, index_dev);
    PE_HIP(hipGetLastError());
    return PE_OK;
}

extern "C" pe_status_t pe_tile_reweight(int32_t n_tiles, const double* tile_loglike_dev, int64_t n_samples,
                                        const int32_t* tile_of_dev, const double* sample_logprior_dev, int64_t n,
                                        const int64_t* index_dev, const double* w_dev, double alpha, double* out_dev,
                                        void* stream) {
    if (n_tiles < 1 || n_tiles > (1 << 24)) return fail(PE_ERR_ARG, "bad n_tiles");
    if (n_samples < 1 || n_samples > ((int64_t)1 << 31)) return fail(PE_ERR_ARG, "n_samples must be in 1..2^31");
    if (n < 0 || n > ((int64_t)1 << 30)) return fail(PE_ERR_ARG, "n must be in 0..2^30");
    if (!(alpha >= 0.0 && alpha <= 1.0)) return fail(PE_ERR_ARG, "alpha must be in [0, 1]");
    if (!tile_loglike_dev || !tile_of_dev || !sample_logprior_dev || !out_dev || (n > 0 && (!index_dev || !w_dev)))
        return fail(PE_ERR_ARG, "NULL pointer");
    if (out_dev == tile_loglike_dev) return fail(PE_ERR_ARG, "out may not alias tile_loglike");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const int nbm = 64;
    const size_t bytes = sizeof(double) * 2 * nbm + sizeof(unsigned long long) * 2 * (size_t)n_tiles;
    char* scr = nullptr;
    pe_status_t s = scratch_for(st, bytes, &scr);
    if (s != PE_OK) return s;
    double* part = reinterpret_cast<double*>(scr);
    unsigned long long* vfx = reinterpret_cast<unsigned long long*>(part + 2 * nbm);
    unsigned long long* pfx = vfx + n_tiles;
    k_rw_zero<<<nblocks(n_tiles), 256, 0, st>>>(n_tiles, vfx, pfx);
    k_tile_max<<<nbm, 256, 0, st>>>(n_tiles, tile_loglike_dev, n_samples, sample_logprior_dev, part);
    k_rw_prior<<<nblocks(n_samples), 256, 0, st>>>(part, nbm, n_samples, tile_of_dev, sample_logprior_dev, vfx);
    if (n > 0) k_rw_post<<<nblocks(n), 256, 0, st>>>(n, index_dev, w_dev, tile_of_dev, pfx);
    k_rw_final<<<1, 1024, 0, st>>>(n_tiles, tile_loglike_dev, part, nbm, vfx, pfx, alpha, out_dev);
    PE_HIP(hipGetLastError());
    return PE_OK;
}
