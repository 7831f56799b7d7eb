// pe_loglike.hip -- log-likelihoods of batches of draws of one or many events
// (Eq. 3), one set of launches per batch whatever the number of events.
//
//   k_b_reset     clear the cut histograms and plans of the events starting here
//   k_b_support   support mask, ISCO cut and cut bucket of every draw
//   k_b_plan      per event: bucket offsets, live count, frequency decomposition
//   k_items       offsets of every event's work items in the batch's queues
//                 (<false>: the hot loop's; <true>: the re-evaluation's)
//   k_b_scatter   live draws into their cut buckets
//   k_b_coeffs    per live draw: phase polynomial, delays, responses, (h|h)
//   k_b_split / k_b_f64   hot loop: persistent workgroups take (event, tile of
//                 256 draws, group of frequency chunks) items off one queue;
//                 lanes = draws; the bin records are staged in LDS (split) or
//                 read through scalar loads (FP64), and each is reused by the
//                 64 draws of a wave and the 256 of a workgroup
//   k_b_finalize  fixed-order combine of the group partials, ln L; split path:
//                 the draw's error estimate, and the draws to re-evaluate
//   k_r_plan, k_r_scatter, k_items<true>, k_r_f64, k_r_finalize
//                 split path: FP64 re-evaluation of the listed draws on the hot
//                 loop's own layout (tiles of 256 listed draws x groups of chunks)
//   k_b_dist      distance-marginalised events: ln L integrated over dL
//
// An event's decomposition (chunk length, groups) is planned on the device from
// its own live draws only (their largest cut bucket and their number), so its
// results do not depend on the other events of the batch, nor on how its tiles
// are spread over launches. Events of any detector count share one queue: each
// item dispatches on its event's count (uniform across the workgroup).
#include <math.h>

#include "pe_device.h"

namespace pe {


__device__ __forceinline__ int bucket_shift(int64_t K) {
    int s = 0;
    while ((K >> s) >= kBuckets) ++s;
    return s;
}

__global__ __launch_bounds__(256) void k_b_reset(const BatchHdr* __restrict__ hdr, const EvDev* __restrict__ evs) {
    const int ne = hdr->ne;
    for (int e = blockIdx.y; e < ne; e += gridDim.y) {
        const EvDev& E = evs[e];
        if (!(E.flags & kLlPrologue)) continue;
        E.hist[blockIdx.x * 256 + threadIdx.x] = 0;
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            EvPlan z = {};
            E.plan[0] = z;
            E.plan[1] = z;
        }
    }
}

__device__ __forceinline__ void gather_theta(const EvDev& E, int64_t i, double th[PE_MAX_DIM]) {
#pragma unroll
    for (int j = 0; j < PE_MAX_DIM; ++j) th[j] = (j < E.ec.dim) ? E.theta[(int64_t)j * E.n + i] : 0.0;
}

// Smallest and largest bucket of a block's live draws (bk < 0: none), for
// every thread of the block. sh: 8 ints of shared memory.
__device__ __forceinline__ void block_bucket_range(int bk, int* sh, int& lo, int& hi) {
    int a = bk >= 0 ? bk : kBuckets, z = bk;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        a = min(a, __shfl_xor(a, o));
        z = max(z, __shfl_xor(z, o));
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sh[w] = a;
        sh[4 + w] = z;
    }
    __syncthreads();
    lo = min(min(sh[0], sh[1]), min(sh[2], sh[3]));
    hi = max(max(sh[4], sh[5]), max(sh[6], sh[7]));
    __syncthreads();
}

// Support mask, ISCO cut and cut bucket. Buckets run from the longest cut down,
// so a wave of the hot loop holds draws whose cuts differ by less than one bucket.
// Blocks of 256 draws that each belong to one event (poff: block offsets of
// the events in their prologue). The draws of an event crowd into few buckets,
// so each block counts its own in shared memory over its bucket range and adds
// the counts to the event's histogram once per bucket.
// (at least five workgroups per CU: five waves per SIMD)
__global__ __launch_bounds__(256, 5) void k_b_support(const BatchHdr* __restrict__ hdr, const EvDev* __restrict__ evs,
                                                   const int64_t* __restrict__ poff) {
    __shared__ int lh[kBuckets];
    __shared__ int sh[8];
    const int ne = hdr->ne;
    const int64_t nblk = poff[ne];
    for (int64_t b = blockIdx.x; b < nblk; b += gridDim.x) {
        const int e = find_slot(poff, ne, b);
        const EvDev& E = evs[e];
        const int64_t i = (b - poff[e]) * 256 + threadIdx.x;
        int bk = -1;
        if (i < E.n) {
            double th[PE_MAX_DIM];
            gather_theta(E, i, th);
            double M;
            if (!mass_and_support(E.ec, th, M)) {
                E.kc_all[i] = -1;
                E.loglike[i] = -INFINITY;
                if (E.aux) {
                    E.aux[3 * i] = 0.0;
                    E.aux[3 * i + 1] = 0.0;
                    E.aux[3 * i + 2] = 0.0;
                }
            } else {
                const int kc = (int)kcut_of(E.ec, f_isco(M));
                E.kc_all[i] = kc;
                bk = (kBuckets - 1) - (kc >> bucket_shift(E.ec.K));
            }
        }
        int lo, hi;
        block_bucket_range(bk, sh, lo, hi);
        if (hi < 0) continue;  // uniform: no live draw in the block
        for (int q = lo + (int)threadIdx.x; q <= hi; q += 256) lh[q] = 0;
        __syncthreads();
        if (bk >= 0) atomicAdd(&lh[bk], 1);
        __syncthreads();
        for (int q = lo + (int)threadIdx.x; q <= hi; q += 256) {
            const int c = lh[q];
            if (c) atomicAdd(&E.hist[q], c);
        }
        __syncthreads();
    }
}

// One workgroup per event: exclusive scan of the bucket counts in place (4 per
// thread), the live count, and the frequency decomposition of the hot loop:
// about items_target work items for the event alone (groups a power of two up
// to 64 and up to the cap), at least min_group_bins bins per group, 8 chunks
// per group spread over [0, kmax), chunk length a multiple of kBlk. kmax is the upper edge of the highest non-empty cut bucket:
// a bound on every live cut that follows from the event's own draws.
__global__ __launch_bounds__(1024) void k_b_plan(const BatchHdr* __restrict__ hdr, const EvDev* __restrict__ evs) {
    __shared__ int sh[1024];
    __shared__ int first;
    const int ne = hdr->ne;
    const int t = threadIdx.x;
    for (int e = blockIdx.x; e < ne; e += gridDim.x) {
        const EvDev& E = evs[e];
        if (!(E.flags & kLlPrologue)) continue;
        int* hist = E.hist;
        if (t == 0) first = kBuckets;
        const int a0 = hist[4 * t], a1 = hist[4 * t + 1], a2 = hist[4 * t + 2], a3 = hist[4 * t + 3];
        const int c = a0 + a1 + a2 + a3;
        sh[t] = c;
        __syncthreads();
        if (c > 0) atomicMin(&first, 4 * t + (a0 > 0 ? 0 : a1 > 0 ? 1 : a2 > 0 ? 2 : 3));
        for (int off = 1; off < 1024; off <<= 1) {
            const int v = (t >= off) ? sh[t - off] : 0;
            __syncthreads();
            sh[t] += v;
            __syncthreads();
        }
        const int ex = sh[t] - c;
        hist[4 * t] = ex;
        hist[4 * t + 1] = ex + a0;
        hist[4 * t + 2] = ex + a0 + a1;
        hist[4 * t + 3] = ex + a0 + a1 + a2;
        if (t == 1023) {
            EvPlan p = {};
            p.n_active = sh[1023];
            p.tiles = (p.n_active + kTile - 1) / kTile;
            if (p.n_active > 0) {
                const int sh_b = bucket_shift(E.ec.K);
                const int64_t top = ((int64_t)(kBuckets - first) << sh_b);  // one past the top bucket's last cut
                p.kmax = (int)(top < E.ec.K ? top : E.ec.K);
                const int want = (E.items_target + p.tiles - 1) / p.tiles;
                int G = 1;
                while (G < want && G < 64) G <<= 1;
                const int by_bins = max(1, p.kmax / E.min_group_bins);
                G = min(G, min(by_bins, E.max_groups));
                while (G & (G - 1)) G &= G - 1;  // a power of two
                const int target = 8 * G;
                int fine = ((p.kmax + target - 1) / target + kBlk - 1) / kBlk * kBlk;
                fine = max(fine, kBlk);
                if (E.flags & kLlMoments) fine = E.ec.tm_fine;  // the moment blocks
                p.n_groups = G;
                p.fine = fine;
                p.n_fine = (p.kmax + fine - 1) / fine;
            } else {
                p.fine = kBlk;
            }
            *E.plan = p;
        }
        __syncthreads();
    }
}

// Items of an event in queue x: with G >= 8 groups (a multiple of 8), the
// groups g = x (mod 8) of every tile, so an XCD reads only its eighth of the
// frequency chunks through its L2; with G < 8, every eighth item of the
// event's (tile, group) sequence.
__device__ __forceinline__ int64_t queue_items(int64_t ntiles, int G, int x) {
    if (G >= kQueues) return ntiles * (G / kQueues);
    const int64_t T = ntiles * G;
    return T > x ? (T - x + kQueues - 1) / kQueues : 0;
}

// Per queue: offsets of every event's items (ioff[x][ne + 1]), the item
// total, and the counter reset. One workgroup of kItemThreads: its threads
// first write every event's item count per queue (events spread over the
// threads, their plans read in parallel), then wave x scans queue x's counts
// in place, 64 events per step (shuffle scan, running carry).
constexpr int kItemThreads = 64 * kQueues;

template <bool Redo>
__device__ __forceinline__ void items_of(const EvDev& E, int64_t (&c)[kQueues]) {
#pragma unroll
    for (int x = 0; x < kQueues; ++x) c[x] = 0;
    if (Redo) {
        if (!(E.flags & kLlFinalize)) return;
        const EvPlan r = E.plan[1];
        if (r.tiles > 0 && r.n_groups > 0)
#pragma unroll
            for (int x = 0; x < kQueues; ++x) c[x] = queue_items(r.tiles, r.n_groups, x);
    } else {
        const EvPlan p = *E.plan;
        const int lo = max(0, E.tile_lo), hi = min(p.tiles, E.tile_hi);
        if (hi > lo && p.n_groups > 0)
#pragma unroll
            for (int x = 0; x < kQueues; ++x) c[x] = queue_items(hi - lo, p.n_groups, x);
    }
}

template <bool Redo>
__global__ __launch_bounds__(kItemThreads) void k_items(BatchHdr* __restrict__ hdr, const EvDev* __restrict__ evs,
                                                      int64_t* __restrict__ ioff) {
    const int ne = hdr->ne, t = threadIdx.x;
    for (int e = t; e < ne; e += kItemThreads) {
        int64_t c[kQueues];
        items_of<Redo>(evs[e], c);
#pragma unroll
        for (int x = 0; x < kQueues; ++x) ioff[(int64_t)x * (ne + 1) + e] = c[x];
    }
    __syncthreads();
    const int x = t >> 6, lane = t & 63;
    int64_t* o = ioff + (int64_t)x * (ne + 1);
    int64_t carry = 0;
    for (int e0 = 0; e0 < ne; e0 += 64) {
        const int e = e0 + lane;
        const int64_t v = (e < ne) ? o[e] : 0;
        int64_t inc = v;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int64_t u = __shfl_up(inc, off);
            if (lane >= off) inc += u;
        }
        if (e < ne) o[e] = carry + inc - v;
        carry += __shfl(inc, 63);
    }
    if (lane == 0) {
        o[ne] = carry;
        hdr->qitems[x] = (int)carry;
        hdr->qnext[x] = 0;
    }
}

// Live draws into their buckets; the order inside a bucket is immaterial. A
// block ranks its draws per bucket in shared memory and claims one run of
// positions per bucket, so a block's draws of one bucket sit side by side.
// Each live draw then writes its index, its cut and its parameters (one record
// of kRecStride doubles, as 16-byte stores) at its position in the record
// buffer (the event's partial buffer, idle until the hot loop); the lanes of a
// bucket's run write one contiguous span, which the L2 merges before HBM.
// k_b_coeffs reads the records in position order.
__global__ __launch_bounds__(256) void k_b_scatter(const BatchHdr* __restrict__ hdr, const EvDev* __restrict__ evs,
                                                   const int64_t* __restrict__ poff) {
    __shared__ int lh[kBuckets];
    __shared__ int sh[8];
    const int ne = hdr->ne;
    const int t = threadIdx.x;
    const int64_t nblk = poff[ne];
    for (int64_t b = blockIdx.x; b < nblk; b += gridDim.x) {
        const int e = find_slot(poff, ne, b);
        const EvDev& E = evs[e];
        const int64_t i = (b - poff[e]) * 256 + t;
        int bk = -1, kc = -1;
        if (i < E.n) {
            kc = E.kc_all[i];
            if (kc >= 0) bk = (kBuckets - 1) - (kc >> bucket_shift(E.ec.K));
        }
        int lo, hi;
        block_bucket_range(bk, sh, lo, hi);
        if (hi < 0) continue;  // uniform: no live draw in the block
        for (int q = lo + t; q <= hi; q += 256) lh[q] = 0;
        __syncthreads();
        const int rank = bk >= 0 ? atomicAdd(&lh[bk], 1) : 0;
        __syncthreads();
        for (int q = lo + t; q <= hi; q += 256) {
            const int c = lh[q];
            if (c) lh[q] = atomicAdd(&E.hist[q], c);
        }
        __syncthreads();
        if (bk >= 0) {
            const int64_t pos = (int64_t)lh[bk] + rank;
            E.idx[pos] = (int)i;
            E.kcut[pos] = kc;
            double th[kRecStride];
#pragma unroll
            for (int a = 0; a < kRecStride; ++a) th[a] = (a < E.ec.dim) ? E.theta[(int64_t)a * E.n + i] : 0.0;
            double2* rec = (double2*)((double*)E.partial + pos * kRecStride);
#pragma unroll
            for (int a = 0; a < kRecStride / 2; ++a) rec[a] = make_double2(th[2 * a], th[2 * a + 1]);
        }
        __syncthreads();  // lh is reused by the block's next iteration
    }
}

__global__ __launch_bounds__(256) void k_b_coeffs(const BatchHdr* __restrict__ hdr, const EvDev* __restrict__ evs,
                                                  const int64_t* __restrict__ poff) {
    const int ne = hdr->ne;
    const int64_t nblk = poff[ne];
    for (int64_t b = blockIdx.x; b < nblk; b += gridDim.x) {
        const int e = find_slot(poff, ne, b);
        const EvDev& E = evs[e];
        const int64_t j = (b - poff[e]) * 256 + threadIdx.x;
        if (j >= E.plan->n_active) continue;
        const int64_t np = E.npad;
        double th[PE_MAX_DIM];
#pragma unroll
        for (int a = 0; a < PE_MAX_DIM; ++a) th[a] = (a < E.ec.dim) ? ((const double*)E.partial)[j * kRecStride + a] : 0.0;
        likelihood_distance(E.ec, th);
        Src s;
        source_from_theta(E.ec, th, s);
        PhaseCoef pc;
        phase_coeffs(s, pc);
#pragma unroll
        for (int a = 0; a < 8; ++a) E.coef[(kCoefA + a) * np + j] = pc.A[a];
        E.coef[kCoefB5 * np + j] = pc.B5;
        E.coef[kCoefB6 * np + j] = pc.B6;
        const int64_t kc = E.kcut[j];
        double h = 0.0;
#pragma unroll
        for (int d = 0; d < PE_MAX_DET; ++d) {
            if (d >= E.ec.n_det) break;
            E.coef[(kCoefTau + d) * np + j] = s.tc + s.dt[d];
            E.resp[(2 * d) * np + j] = s.rre[d];
            E.resp[(2 * d + 1) * np + j] = s.rim[d];
            h += (s.rre[d] * s.rre[d] + s.rim[d] * s.rim[d]) * E.pfx[(int64_t)d * (E.ec.K + 1) + kc];
        }
        E.hh[j] = h;
    }
}

// ---------------------------------------------------------------------------
// hot loop
// ---------------------------------------------------------------------------
__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
    return __builtin_amdgcn_readfirstlane(v);
}
__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
    return __builtin_amdgcn_readfirstlane(v);
}

struct DrawRow {
    double A[8];
    double B5, B6;
};

// Split precision: FP64 phase in turns and its fract in FP64; from the reduced
// phase on FP32: sin/cos of 2 pi (r + alpha) by the hardware's turn-based
// v_sin_f32/v_cos_f32, |w|-weighted products summed over kBlk bins in FP32.
template <int NDET, bool MASK>
__device__ __forceinline__ void bin_split(const Rec32& r, const DrawRow& row, const double (&tau)[NDET], bool live,
                                          float (&br)[NDET], float (&bi)[NDET]) {
    const double psi = psi_turns(row.A, row.B5, row.B6, r.x, r.xm5, r.lnx);
#pragma unroll
    for (int d = 0; d < NDET; ++d) {
        const double ph = fma(r.f, tau[d], psi);
        const float t = (float)fract64(ph) + r.w[d].y;
        const float sn = __builtin_amdgcn_sinf(t);
        const float cs = __builtin_amdgcn_cosf(t);
        const float m = MASK ? (live ? r.w[d].x : 0.0f) : r.w[d].x;
        br[d] = fmaf(m, cs, br[d]);
        bi[d] = fmaf(-m, sn, bi[d]);
    }
}

// Plain FP64: complex128 weights and the FP64 sincos of the reduced phase.
template <int NDET, bool MASK>
__device__ __forceinline__ void bin_f64(const Rec64& r, const DrawRow& row, const double (&tau)[NDET], bool live,
                                        double (&zr)[NDET], double (&zi)[NDET]) {
    const double psi = psi_turns(row.A, row.B5, row.B6, r.x, r.xm5, r.lnx);
#pragma unroll
    for (int d = 0; d < NDET; ++d) {
        const double ph = fma(r.f, tau[d], psi);
        double sn, cs;
        sincos_turns(fract64(ph), sn, cs);
        const double wr = MASK ? (live ? r.w[d].x : 0.0) : r.w[d].x;
        const double wi = MASK ? (live ? r.w[d].y : 0.0) : r.w[d].y;
        // conj(w) (cos - i sin)
        zr[d] = fma(wr, cs, zr[d]);
        zr[d] = fma(-wi, sn, zr[d]);
        zi[d] = fma(-wr, sn, zi[d]);
        zi[d] = fma(-wi, cs, zi[d]);
    }
}

struct Item {
    int e, tile, g;
};

// Work tickets. A workgroup on XCD x0 takes items from queue x0 (for short
// items it claims the next ticket while it works on the current one), and only
// once queue x0 has run dry does it wait on the other queues in turn. q < 0:
// every queue is empty (every workgroup reaches that exit).
struct Ticket {
    int q, v;
};

// A queue whose counter has passed its item count stays empty (counters only
// grow), so a plain load settles it without an atomic.
__device__ __forceinline__ bool queue_open(BatchHdr* __restrict__ hdr, int q) {
    return __hip_atomic_load(&hdr->qnext[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < hdr->qitems[q];
}

__device__ __forceinline__ Ticket steal_ticket(BatchHdr* __restrict__ hdr, int x0) {
    for (int k = 1; k < kQueues; ++k) {
        const int qq = (x0 + k) & (kQueues - 1);
        if (!queue_open(hdr, qq)) continue;
        const int v = atomicAdd(&hdr->qnext[qq], 1);
        if (v < hdr->qitems[qq]) return Ticket{qq, v};
    }
    return Ticket{-1, 0};
}

// Checks a ticket claimed from queue x0 (thread 0 only).
__device__ __forceinline__ Ticket own_or_steal(BatchHdr* __restrict__ hdr, int x0, int v) {
    return (v < hdr->qitems[x0]) ? Ticket{x0, v} : steal_ticket(hdr, x0);
}

// The next ticket of queue x0, or another queue's (thread 0 only).
__device__ __forceinline__ Ticket next_ticket(BatchHdr* __restrict__ hdr, int x0) {
    return queue_open(hdr, x0) ? own_or_steal(hdr, x0, atomicAdd(&hdr->qnext[x0], 1)) : steal_ticket(hdr, x0);
}

// Item of ticket (q, x); REDO: items of the FP64 re-evaluation (plan[1], tiles from 0).
template <bool REDO>
__device__ __forceinline__ void decode_item(const int64_t* __restrict__ ioff, int ne, const EvDev* __restrict__ evs,
                                            int q, int x, Item& it) {
    const int64_t* o = ioff + (int64_t)q * (ne + 1);
    int lo = 0, hi = ne;  // o[lo] <= x < o[hi]; offsets through the scalar cache
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (load_const(o + mid) <= (int64_t)x)
            lo = mid;
        else
            hi = mid;
    }
    it.e = lo;
    const int l = x - (int)load_const(o + it.e);
    const int G = load_const(evs[it.e].plan + (REDO ? 1 : 0)).n_groups;
    const int tlo = REDO ? 0 : max(0, evs[it.e].tile_lo);
    if (G >= kQueues) {
        const int gq = G / kQueues;
        it.tile = tlo + l / gq;
        it.g = q + kQueues * (l - (l / gq) * gq);
    } else {
        const int f = q + kQueues * l;
        it.tile = tlo + f / G;
        it.g = f - (f / G) * G;
    }
}

// The persistent loop of the hot kernels: process(it) for every item this
// workgroup draws.
template <bool REDO, typename F>
__device__ __forceinline__ void item_loop(BatchHdr* __restrict__ hdr, const int64_t* __restrict__ ioff,
                                          const EvDev* __restrict__ evs, F process) {
    // two ticket slots used in turn: a slot is rewritten only after the barrier
    // that follows every wave's read of it
    __shared__ int s_q[2], s_v[2];
    const int ne = hdr->ne;
    const int x0 = blockIdx.x & (kQueues - 1);
    if (threadIdx.x == 0) {
        const Ticket t = next_ticket(hdr, x0);
        s_q[0] = t.q;
        s_v[0] = t.v;
    }
    __syncthreads();
    int slot = 0;
    int q = __builtin_amdgcn_readfirstlane(s_q[0]);
    int v = __builtin_amdgcn_readfirstlane(s_v[0]);
    while (q >= 0) {
        Item it;
        decode_item<REDO>(ioff, ne, evs, q, v, it);
        // Short items (under ~4k bins) claim the next ticket before they run, so
        // the atomic's latency hides behind them; long ones claim it when done,
        // which keeps the last items spread evenly over the workgroups.
        const EvPlan pl = load_const(evs[it.e].plan);
        const bool early = pl.kmax < 4096 * pl.n_groups;
        int nv = 0;
        if (early && threadIdx.x == 0) nv = queue_open(hdr, x0) ? atomicAdd(&hdr->qnext[x0], 1) : INT_MAX;
        process(it);
        slot ^= 1;
        if (threadIdx.x == 0) {
            const Ticket t = early ? own_or_steal(hdr, x0, nv) : next_ticket(hdr, x0);
            s_q[slot] = t.q;
            s_v[slot] = t.v;
        }
        __syncthreads();
        q = __builtin_amdgcn_readfirstlane(s_q[slot]);
        v = __builtin_amdgcn_readfirstlane(s_v[slot]);
    }
}

// The row and delays of the draw at position jl, its cut, and the wave's range
// of cuts over its valid lanes.
template <int NDET>
__device__ __forceinline__ void load_row(const EvDev& E, int64_t jl, bool valid, DrawRow& row, double (&tau)[NDET],
                                         int& kc, int& wmin, int& wmax) {
    const int64_t np = E.npad;
    const gdoubles coef = (gdoubles)E.coef;
#pragma unroll
    for (int a = 0; a < 8; ++a) row.A[a] = coef[(kCoefA + a) * np + jl];
    row.B5 = coef[kCoefB5 * np + jl];
    row.B6 = coef[kCoefB6 * np + jl];
#pragma unroll
    for (int d = 0; d < NDET; ++d) tau[d] = coef[(kCoefTau + d) * np + jl];
    kc = ((gints)E.kcut)[jl];
    wmin = wave_min(valid ? kc : 0x7fffffff);
    wmax = wave_max(valid ? kc : 0);
}

// The lane's draw (position tile * 256 + lane), its row and delays, its cut,
// and the wave's range of cuts.
template <int NDET>
__device__ __forceinline__ void item_setup(const EvDev& E, int nact, int tile, int& j, bool& valid, DrawRow& row,
                                           double (&tau)[NDET], int& kc, int& wmin, int& wmax) {
    j = tile * kTile + (int)threadIdx.x;
    valid = j < nact;
    load_row<NDET>(E, valid ? j : nact - 1, valid, row, tau, kc, wmin, wmax);
}

// One item of the split hot loop. The workgroup stages the bin records of its
// chunks in LDS (pieces of kStage bins, 16-byte coalesced loads by all 256
// threads), and each wave reads them back with broadcast LDS loads: every lane
// of a wave needs the same record at the same time. Sums: FP32 over blocks of
// kBlk bins, folded into FP64 accumulators (an FP64 add costs one issue slot,
// as an FP32 one does without packed math). Blocks sit on multiples of kBlk
// (chunks start on one), and a lane folds a block only if the block starts
// below its own cut, so a draw's operations do not depend on the draws sharing
// its wave. The workgroup walks each chunk up to the largest cut among its
// four waves; a wave computes only below its own largest cut.
constexpr int kStage = 256;

template <int NDET>
__device__ __forceinline__ void split_item(const EvDev& E, const EvPlan& p, int tile, int g, Rec32* srec,
                                           int* sred) {
    int j, kc, wmin, wmax;
    bool valid;
    DrawRow row;
    double tau[NDET];
    item_setup<NDET>(E, p.n_active, tile, j, valid, row, tau, kc, wmin, wmax);
    const Rec32* tab = E.rec32;
    const int K = (int)E.ec.K;
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) sred[wv] = wmax;
    __syncthreads();
    const int gmax = max(max(sred[0], sred[1]), max(sred[2], sred[3]));
    double sr[NDET], si[NDET];
#pragma unroll
    for (int d = 0; d < NDET; ++d) sr[d] = si[d] = 0.0;
    // bins [ks, ke) of a chunk whose records sit at sp[0 ..): full blocks below kA,
    // then the masked blocks up to kB
    auto piece = [&](const Rec32* sp, int ks, int ke, int kA, int kB) {
        for (int kb = ks; kb < min(ke, kA); kb += kBlk) {
            float br[NDET], bi[NDET];
#pragma unroll
            for (int d = 0; d < NDET; ++d) br[d] = bi[d] = 0.0f;
#pragma unroll 4
            for (int q = 0; q < kBlk; ++q) {
                const Rec32 r = sp[kb - ks + q];
                bin_split<NDET, false>(r, row, tau, true, br, bi);
            }
#pragma unroll
            for (int d = 0; d < NDET; ++d) {
                sr[d] += (double)br[d];
                si[d] += (double)bi[d];
            }
        }
        for (int kb = max(ks, kA); kb < min(ke, kB); kb += kBlk) {
            const int kq = min(kb + kBlk, kB);
            float br[NDET], bi[NDET];
#pragma unroll
            for (int d = 0; d < NDET; ++d) br[d] = bi[d] = 0.0f;
            for (int k = kb; k < kq; ++k) {
                const Rec32 r = sp[k - ks];
                bin_split<NDET, true>(r, row, tau, k < kc, br, bi);
            }
            if (kb < kc) {
#pragma unroll
                for (int d = 0; d < NDET; ++d) {
                    sr[d] += (double)br[d];
                    si[d] += (double)bi[d];
                }
            }
        }
    };
    // the wave's full and masked ranges of a chunk starting at k0
    auto ranges = [&](int k0, int k1, int& kA, int& kB) {
        const bool on = k0 < wmax;  // this wave has cuts above the chunk's start
        kA = on ? k0 + (max(0, min(wmin, k1) - k0) / kBlk) * kBlk : k0;
        kB = on ? max(kA, min(k1, wmax)) : k0;
    };
    int nci = 0;  // the item's chunks below the workgroup's largest cut
    for (int c = g; c < p.n_fine && c * p.fine < gmax; c += p.n_groups) ++nci;
    if (nci > 0 && nci * p.fine <= kStage) {
        // short chunks (short bands, many groups): all of the item's chunks staged at
        // once, chunk i at record i * fine, one pair of barriers for the item; the
        // bins and their order per lane are those of the piecewise walk below
        constexpr int kParts = (int)(sizeof(Rec32) / 16);
        const int per = p.fine * kParts;
        __syncthreads();  // the previous item's records have been read
        for (int q = threadIdx.x; q < nci * per; q += 256) {
            const int i = q / per, r = q - i * per;
            const int k0 = (g + i * p.n_groups) * p.fine;
            const int k = k0 + r / kParts;
            if (k < min(min(k0 + p.fine, K), gmax)) ((uint4*)srec)[q] = ((const uint4*)(tab + k))[r % kParts];
        }
        __syncthreads();
        for (int i = 0; i < nci; ++i) {
            const int k0 = (g + i * p.n_groups) * p.fine;
            const int k1 = min(k0 + p.fine, K);
            int kA, kB;
            ranges(k0, k1, kA, kB);
            piece(srec + i * p.fine, k0, min(k1, gmax), kA, kB);
        }
    } else if (p.n_groups == 1) {
        // one group: the item's chunks tile [0, gmax) end to end, so it is staged
        // in full pieces across the chunk boundaries (the same 16-bin blocks, in
        // the same order, as the walk chunk by chunk; fewer barrier pairs)
        int kA, kB;
        ranges(0, K, kA, kB);
        for (int ks = 0; ks < gmax; ks += kStage) {
            const int ke = min(ks + kStage, gmax);
            __syncthreads();  // the previous piece has been read
            const uint4* src = (const uint4*)(tab + ks);
            uint4* dst = (uint4*)srec;
            for (int q = threadIdx.x; q < (ke - ks) * (int)(sizeof(Rec32) / 16); q += 256) dst[q] = src[q];
            __syncthreads();
            piece(srec, ks, ke, kA, kB);
        }
    } else {
        for (int c = g; c < p.n_fine; c += p.n_groups) {
            const int k0 = c * p.fine;
            if (k0 >= gmax) break;  // uniform over the workgroup
            const int k1 = min(k0 + p.fine, K);
            int kA, kB;
            ranges(k0, k1, kA, kB);
            const int kl = min(k1, gmax);
            for (int ks = k0; ks < kl; ks += kStage) {
                const int ke = min(ks + kStage, kl);
                __syncthreads();  // the previous piece has been read
                const uint4* src = (const uint4*)(tab + ks);
                uint4* dst = (uint4*)srec;
                for (int q = threadIdx.x; q < (ke - ks) * (int)(sizeof(Rec32) / 16); q += 256) dst[q] = src[q];
                __syncthreads();
                piece(srec, ks, ke, kA, kB);
            }
        }
    }
    __syncthreads();  // sred and srec are reused by the next item
    if (valid) {
#pragma unroll
        for (int d = 0; d < NDET; ++d) E.partial[((int64_t)g * NDET + d) * E.npad + j] = make_double2(sr[d], si[d]);
    }
}

// FP64 walk of one item's chunks (group g of the plan) for the lane's draw.
template <int NDET>
__device__ __forceinline__ void f64_walk(const EvDev& E, const EvPlan& p, int g, const DrawRow& row,
                                         const double (&tau)[NDET], int kc, int wmin, int wmax, double (&zr)[NDET],
                                         double (&zi)[NDET]) {
    const Rec64* tab = E.rec64;
    const int K = (int)E.ec.K;
#pragma unroll
    for (int d = 0; d < NDET; ++d) zr[d] = zi[d] = 0.0;
    for (int c = g; c < p.n_fine; c += p.n_groups) {
        const int k0 = c * p.fine;
        if (k0 >= wmax) break;
        const int k1 = min(k0 + p.fine, K);
        const int kA = max(k0, min(k1, wmin));
        const int kB = max(kA, min(k1, wmax));
        int k = k0;
#pragma unroll 2
        for (; k < kA; ++k) {
            const Rec64 r = load_const(tab + k);
            bin_f64<NDET, false>(r, row, tau, true, zr, zi);
        }
        for (; k < kB; ++k) {
            const Rec64 r = load_const(tab + k);
            bin_f64<NDET, true>(r, row, tau, k < kc, zr, zi);
        }
    }
}

template <int NDET>
__device__ __forceinline__ void f64_item(const EvDev& E, const EvPlan& p, int tile, int g) {
    int j, kc, wmin, wmax;
    bool valid;
    DrawRow row;
    double tau[NDET];
    item_setup<NDET>(E, p.n_active, tile, j, valid, row, tau, kc, wmin, wmax);
    double zr[NDET], zi[NDET];
    f64_walk<NDET>(E, p, g, row, tau, kc, wmin, wmax, zr, zi);
    if (valid) {
#pragma unroll
        for (int d = 0; d < NDET; ++d) E.partial[((int64_t)g * NDET + d) * E.npad + j] = make_double2(zr[d], zi[d]);
    }
}

// One item of the FP64 re-evaluation: lane r of the tile takes the r-th listed
// draw (position rpos[r]); its partials go to column r. The walk is the FP64
// kernel's, under the same plan, so each listed draw gets the FP64 path's value.
// Tiles of the re-evaluation are one wave (kRedoTile draws): the listed draws
// are few, and one-wave workgroups give the persistent grid enough waves per
// SIMD to hide the latency of the FP64 sine/cosine chains (a draw's arithmetic
// does not depend on the tile size).
// The walk stages the records of each piece of kRedoTile bins in LDS (one
// record per lane, 16-byte vector loads) and every lane reads them back by
// broadcast: the few tiles of listed draws reuse a record too little for the
// scalar loads of the FP64 kernel to find it in L2, and a lone wave would wait
// on each of them. The bins and their order are f64_walk's.
template <int NDET>
__device__ __forceinline__ void redo_walk(const EvDev& E, const EvPlan& p, int g, const DrawRow& row,
                                          const double (&tau)[NDET], int kc, int wmin, int wmax,
                                          double (&zr)[NDET], double (&zi)[NDET], Rec64* srec) {
    const Rec64* tab = E.rec64;
    const int K = (int)E.ec.K;
#pragma unroll
    for (int d = 0; d < NDET; ++d) zr[d] = zi[d] = 0.0;
    for (int c = g; c < p.n_fine; c += p.n_groups) {
        const int k0 = c * p.fine;
        if (k0 >= wmax) break;
        const int k1 = min(k0 + p.fine, K);
        const int kA = max(k0, min(k1, wmin));
        const int kB = max(kA, min(k1, wmax));
        for (int ks = k0; ks < kB; ks += kRedoTile) {
            const int ke = min(ks + kRedoTile, kB);
            __syncthreads();  // the previous piece has been read
            if (ks + (int)threadIdx.x < ke) {
                const uint4* src = (const uint4*)(tab + ks + threadIdx.x);
                uint4* dst = (uint4*)(srec + threadIdx.x);
#pragma unroll
                for (int q = 0; q < (int)(sizeof(Rec64) / 16); ++q) dst[q] = src[q];
            }
            __syncthreads();
            const int ka = min(ke, kA);
            for (int k = ks; k < ka; ++k) bin_f64<NDET, false>(srec[k - ks], row, tau, true, zr, zi);
            for (int k = max(ks, kA); k < ke; ++k) bin_f64<NDET, true>(srec[k - ks], row, tau, k < kc, zr, zi);
        }
    }
}

template <int NDET>
__device__ __forceinline__ void redo_item(const EvDev& E, const EvPlan& rp, int tile, int g, Rec64* srec) {
    const int r = tile * kRedoTile + (int)threadIdx.x;
    const bool valid = r < rp.n_active;
    const int jl = ((gints)E.rpos)[valid ? r : rp.n_active - 1];
    int kc, wmin, wmax;
    DrawRow row;
    double tau[NDET];
    load_row<NDET>(E, jl, valid, row, tau, kc, wmin, wmax);
    double zr[NDET], zi[NDET];
    redo_walk<NDET>(E, rp, g, row, tau, kc, wmin, wmax, zr, zi, srec);
    if (valid) {
#pragma unroll
        for (int d = 0; d < NDET; ++d) E.partial[((int64_t)g * NDET + d) * rp.stride + r] = make_double2(zr[d], zi[d]);
    }
}

__global__ __launch_bounds__(256) void k_b_split(BatchHdr* __restrict__ hdr, const EvDev* __restrict__ evs,
                                                 const int64_t* __restrict__ ioff) {
    __shared__ Rec32 srec[kStage];
    __shared__ int sred[4];
    item_loop<false>(hdr, ioff, evs, [&](const Item& it) {
        const EvDev& E = evs[it.e];
        const EvPlan p = load_const(E.plan);
        switch (E.ec.n_det) {
            case 1: split_item<1>(E, p, it.tile, it.g, srec, sred); break;
            case 2: split_item<2>(E, p, it.tile, it.g, srec, sred); break;
            case 3: split_item<3>(E, p, it.tile, it.g, srec, sred); break;
            default: split_item<4>(E, p, it.tile, it.g, srec, sred); break;
        }
    });
}

__global__ __launch_bounds__(256) void k_b_f64(BatchHdr* __restrict__ hdr, const EvDev* __restrict__ evs,
                                               const int64_t* __restrict__ ioff) {
    item_loop<false>(hdr, ioff, evs, [&](const Item& it) {
        const EvDev& E = evs[it.e];
        const EvPlan p = load_const(E.plan);
        switch (E.ec.n_det) {
            case 1: f64_item<1>(E, p, it.tile, it.g); break;
            case 2: f64_item<2>(E, p, it.tile, it.g); break;
            case 3: f64_item<3>(E, p, it.tile, it.g); break;
            default: f64_item<4>(E, p, it.tile, it.g); break;
        }
    });
}

// Fixed-order combine of a draw's group partials for one detector (8
// interleaved accumulators, then a pairwise tree); col: the draw's column.
__device__ __forceinline__ void combine_groups(const EvDev& E, int d, int nd, int G, int64_t col, int64_t np,
                                               double& ar, double& ai) {
    double xr[8], xi[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) xr[q] = xi[q] = 0.0;
    for (int c = 0; c < G; ++c) {
        const double2 v = E.partial[((int64_t)c * nd + d) * np + col];
        xr[c & 7] += v.x;
        xi[c & 7] += v.y;
    }
#pragma unroll
    for (int w = 4; w > 0; w >>= 1)
#pragma unroll
        for (int q = 0; q < w; ++q) {
            xr[q] += xr[q + w];
            xi[q] += xi[q + w];
        }
    ar = xr[0];
    ai = xi[0];
}

// Coherent part of the split path's error per unit of coherent magnitude, for
// data whose per-bin signal-to-noise amplitude is at most sqrt(a2): harmonic j
// of the hardware error keeps the factor (0.7 a)^(j-1) of the coherent sum;
// harmonics 8 and up are bounded together (Cauchy-Schwarz over their RMS).
__device__ __forceinline__ double eps_coherent(double a2) {
    const double g = 0.7 * sqrt(a2);
    if (!(g < 0.9)) return kEpsMax;
    double s = 0.0, gp = 1.0;
#pragma unroll
    for (int j = 0; j < 7; ++j) {
        s += kEpsHarm[j] * gp;
        gp *= g;
    }
    s += kEpsRms * 1.4142135623730951 * gp / sqrt(1.0 - g * g);
    return fmin(s, kEpsMax);
}

// Bound on |d ln L| of the split path for one detector of a draw (see
// kEpsHarm): guard G, |R_d|, the detector's FP32-path sum (ar, ai), and below
// the draw's cut kc: C = sum pw, l1 = sum |w|, w2 = sum |w|^2 and pp = sum of the
// whitened data power. lin gains the part that adds linearly over detectors,
// var the variance of the scatter (in units of kEpsInc^2).
// The signal power below the cut is bounded like the band's (see kGuardRho2):
// noise gives each bin whitened power 2 on average, sd 2 sqrt(kc) over the kc
// bins, so rho2 = pp - 2 kc + 12 sqrt(kc) bounds it with 6 sd of margin; data
// with less power than the noise less 6 sd there take the worst case only.
__device__ __forceinline__ void split_error(const double* __restrict__ G, double rm, double ar, double ai, double c,
                                            double l1, double w2, double pp, int kc, double& lin, double& var) {
    if (rm == 0.0 || c == 0.0) return;
    var += rm * rm * w2;
    const double worst = kEpsMax * rm * l1;  // every term's error at its largest
    const double slack = 12.0 * sqrt((double)kc), excess = pp - 2.0 * (double)kc;
    if (G[kGuardRho2] < 0.0 || excess < -slack) {  // no noise to scatter the phases: the worst case only
        lin += worst;
        return;
    }
    const double rho2 = excess + slack;
    const double coh = fmax(rm * hypot(ar, ai), sqrt(rm * rm * c * rho2));
    lin += fmin(worst, eps_coherent(rho2 * G[kGuardPwMax] / c) * coh + kEpsL1 * rm * l1);
}

// Fixed-order combine of the group partials, then ln L of Eq. 3. The split
// path also bounds each draw's error and marks the draws above the batch's
// redo budget: rflag[j] = the draw's rank among the marked draws of its block
// of 256 positions (-1: not marked), rcnt[block] = their count.
template <bool SPLIT>
__global__ __launch_bounds__(256) void k_b_finalize(BatchHdr* __restrict__ hdr, const EvDev* __restrict__ evs,
                                                    const int64_t* __restrict__ foff) {
    __shared__ int swc[4];
    const int ne = hdr->ne;
    const double budget = hdr->redo_budget;
    const int64_t nblk = foff[ne];
    for (int64_t b = blockIdx.x; b < nblk; b += gridDim.x) {
        const int e = find_slot(foff, ne, b);
        const EvDev& E = evs[e];
        const int64_t blk = b - foff[e];
        const int64_t j = blk * 256 + threadIdx.x;
        const EvPlan p = *E.plan;
        bool redo = false;
        if (j < p.n_active) {
            const int64_t np = E.npad;
            const int nd = E.ec.n_det;
            const int kc = E.kcut[j];
            double zr = 0.0, zi = 0.0, lin = 0.0, var = 0.0;
            for (int d = 0; d < nd; ++d) {
                double ar, ai;
                combine_groups(E, d, nd, p.n_groups, j, E.npad, ar, ai);
                if (SPLIT) {
                    ar *= kTrigGain;
                    ai *= kTrigGain;
                }
                const double rr = E.resp[(2 * d) * np + j], ri = E.resp[(2 * d + 1) * np + j];
                zr += rr * ar - ri * ai;
                zi += rr * ai + ri * ar;
                if (SPLIT) {
                    const int64_t o = (int64_t)d * (E.ec.K + 1) + kc;
                    split_error(E.guard + d * kGuardStride, hypot(rr, ri), ar, ai, E.pfx[o], E.pl1[o], E.pw2[o],
                                E.ppw[o], kc, lin, var);
                }
            }
            if (SPLIT) {
                const double err = lin + kEpsInc * sqrt(var);
                redo = !(err <= budget) || budget <= 0.0;
            }
            const double h = E.hh[j];
            const int64_t i = E.idx[j];
            if (E.ec.dist)  // k_b_dist integrates over the distance
                E.zd[j] = make_double2(zr, zi);
            else
                E.loglike[i] = loglike_phase(E.ec, zr, zi, h);
            if (E.aux) {
                E.aux[3 * i] = zr;
                E.aux[3 * i + 1] = zi;
                E.aux[3 * i + 2] = h;
            }
        }
        if (SPLIT) {
            const uint64_t bal = __ballot(redo);
            const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
            if (lane == 0) swc[wv] = __popcll(bal);
            __syncthreads();
            int before = 0;
            for (int w = 0; w < wv; ++w) before += swc[w];
            E.rflag[j] = redo ? before + __popcll(bal & ((1ull << lane) - 1ull)) : -1;
            if (threadIdx.x == 0) E.rcnt[blk] = (swc[0] + swc[1]) + (swc[2] + swc[3]);
            __syncthreads();  // swc is reused by the next block
        }
    }
}

// Per event that finalises: exclusive scan of the marked counts of its blocks
// (in place: rcnt becomes each block's offset) and the plan of the FP64
// re-evaluation: the event's chunks for the marked draws, in as many groups as
// their partials allow, up to every chunk its own group (8G groups, those past
// n_fine empty): the marked draws are usually few, and short items keep any
// single wave's walk from setting the kernel's length. The grouping differs from
// the FP64 path's, so a re-evaluated draw equals that path's value to rounding.
__global__ __launch_bounds__(1024) void k_r_plan(const BatchHdr* __restrict__ hdr, const EvDev* __restrict__ evs) {
    __shared__ int sh[1024];
    const int ne = hdr->ne;
    const int t = threadIdx.x;
    for (int e = blockIdx.x; e < ne; e += gridDim.x) {
        const EvDev& E = evs[e];
        if (!(E.flags & kLlFinalize)) continue;
        const EvPlan p = E.plan[0];
        const int nb = (p.n_active + 255) / 256;
        int carry = 0;
        for (int base = 0; base < nb; base += 4096) {
            int v[4], c = 0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int i = base + 4 * t + q;
                v[q] = i < nb ? E.rcnt[i] : 0;
                c += v[q];
            }
            sh[t] = c;
            __syncthreads();
            for (int off = 1; off < 1024; off <<= 1) {
                const int u = t >= off ? sh[t - off] : 0;
                __syncthreads();
                sh[t] += u;
                __syncthreads();
            }
            int run = carry + sh[t] - c;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int i = base + 4 * t + q;
                if (i < nb) E.rcnt[i] = run;
                run += v[q];
            }
            carry += sh[1023];
            __syncthreads();
        }
        if (t == 0) {
            EvPlan r = p;
            r.n_active = carry;
            r.tiles = (carry + kRedoTile - 1) / kRedoTile;
            const int64_t cols = (int64_t)r.tiles * kRedoTile;
            const int64_t cap = (int64_t)E.max_groups * E.npad;  // partial columns the workspace holds
            r.stride = (int)cols;
            while (carry > 0 && r.n_groups < 8 * p.n_groups && 2 * (int64_t)r.n_groups * cols <= cap)
                r.n_groups *= 2;
            E.plan[1] = r;
        }
        __syncthreads();
    }
}

// Marked draws into the re-evaluation list, in position order.
__global__ __launch_bounds__(256) void k_r_scatter(const BatchHdr* __restrict__ hdr, const EvDev* __restrict__ evs,
                                                   const int64_t* __restrict__ foff) {
    const int ne = hdr->ne;
    const int64_t nblk = foff[ne];
    for (int64_t b = blockIdx.x; b < nblk; b += gridDim.x) {
        const int e = find_slot(foff, ne, b);
        const EvDev& E = evs[e];
        if (E.plan[1].n_active == 0) continue;  // uniform over the block
        const int64_t blk = b - foff[e];
        const int64_t j = blk * 256 + threadIdx.x;
        if (j >= E.plan[0].n_active) continue;
        const int r = E.rflag[j];
        if (r >= 0) E.rpos[E.rcnt[blk] + r] = (int)j;
    }
}

// The re-evaluation's persistent walk over the listed draws' items, for events of
// up to MAXD detectors.
template <int MAXD>
__device__ __forceinline__ void redo_items(BatchHdr* __restrict__ hdr, const EvDev* __restrict__ evs,
                                           const int64_t* __restrict__ ioff, Rec64* srec) {
    int items = 0;
#pragma unroll
    for (int q = 0; q < kQueues; ++q) items += hdr->qitems[q];
    if (items == 0) return;  // nothing listed (uniform over the grid)
    item_loop<true>(hdr, ioff, evs, [&](const Item& it) {
        const EvDev& E = evs[it.e];
        const EvPlan rp = load_const(E.plan + 1);
        switch (E.ec.n_det) {
            case 1: redo_item<1>(E, rp, it.tile, it.g, srec); break;
            case 2: redo_item<2>(E, rp, it.tile, it.g, srec); break;
            case 3: if (MAXD >= 3) redo_item<3>(E, rp, it.tile, it.g, srec); break;
            default: if (MAXD >= 4) redo_item<4>(E, rp, it.tile, it.g, srec); break;
        }
    });
}

__global__ __launch_bounds__(kRedoTile) void k_r_f64(BatchHdr* __restrict__ hdr, const EvDev* __restrict__ evs,
                                               const int64_t* __restrict__ ioff) {
    __shared__ Rec64 srec[kRedoTile];
    redo_items<PE_MAX_DET>(hdr, evs, ioff, srec);
}

// Batches whose events have at most two detectors: without the three- and
// four-detector bodies the walk fits 128 registers, four waves per SIMD instead
// of three (the walk's FP64 sine/cosine chains are latency-bound). Same
// arithmetic per draw as k_r_f64.
__global__ __launch_bounds__(kRedoTile) __attribute__((amdgpu_waves_per_eu(4))) void k_r_f64_2det(
    BatchHdr* __restrict__ hdr, const EvDev* __restrict__ evs, const int64_t* __restrict__ ioff) {
    __shared__ Rec64 srec[kRedoTile];
    redo_items<2>(hdr, evs, ioff, srec);
}

// ln L of the re-evaluated draws from their FP64 partials, combined exactly as
// the FP64 path's finalize combines them.
__global__ __launch_bounds__(256) void k_r_finalize(const BatchHdr* __restrict__ hdr, const EvDev* __restrict__ evs,
                                                    const int64_t* __restrict__ foff) {
    const int ne = hdr->ne;
    const int64_t nblk = foff[ne];
    for (int64_t b = blockIdx.x; b < nblk; b += gridDim.x) {
        const int e = find_slot(foff, ne, b);
        const EvDev& E = evs[e];
        const EvPlan rp = E.plan[1];
        const int64_t r = (b - foff[e]) * 256 + threadIdx.x;
        if (r >= rp.n_active) continue;
        const int64_t j = E.rpos[r];
        const int64_t np = E.npad;
        const int nd = E.ec.n_det;
        double zr = 0.0, zi = 0.0;
        for (int d = 0; d < nd; ++d) {
            double ar, ai;
            combine_groups(E, d, nd, rp.n_groups, r, rp.stride, ar, ai);
            const double rr = E.resp[(2 * d) * np + j], ri = E.resp[(2 * d + 1) * np + j];
            zr += rr * ar - ri * ai;
            zi += rr * ai + ri * ar;
        }
        const double h = E.hh[j];
        const int64_t i = E.idx[j];
        if (E.ec.dist)
            E.zd[j] = make_double2(zr, zi);
        else
            E.loglike[i] = loglike_phase(E.ec, zr, zi, h);
        if (E.aux) {
            E.aux[3 * i] = zr;
            E.aux[3 * i + 1] = zi;
            E.aux[3 * i + 2] = h;
        }
    }
}

// Distance-marginalised events: ln L of each live draw from the Z that the
// finalize (or the FP64 re-evaluation) left in zd at its position and H, integrated over the distance prior by kDistLanes lanes per
// draw (a block covers a quarter of a finalize block's 256 positions). Kept out
// of the finalize so that the finalize's register budget (and occupancy) stays
// that of the plain likelihood; blocks of other events return at once.
constexpr int kDistLanes = 4;

__global__ __launch_bounds__(256) void k_b_dist(const BatchHdr* __restrict__ hdr, const EvDev* __restrict__ evs,
                                                const int64_t* __restrict__ foff) {
    const int ne = hdr->ne;
    const int64_t nblk = foff[ne] * kDistLanes;
    const int sub = threadIdx.x % kDistLanes;
    for (int64_t b = blockIdx.x; b < nblk; b += gridDim.x) {
        const int64_t fb = b / kDistLanes;
        const int e = find_slot(foff, ne, fb);
        const EvDev& E = evs[e];
        if (!E.ec.dist) continue;
        const int64_t j = (fb - foff[e]) * 256 + (b - fb * kDistLanes) * (256 / kDistLanes) + threadIdx.x / kDistLanes;
        if (j >= E.plan->n_active) continue;  // the same for the draw's lanes
        const double2 z = E.zd[j];
        const double ll = loglike_of<kDistLanes>(E.ec, z.x, z.y, E.hh[j], sub);
        if (sub == 0) E.loglike[E.idx[j]] = ll;
    }
}

// Time-marginalised events. Every draw is evaluated at M nodes spread evenly
// over the whole tc window, t_m = tc_lo + m h with h = T / (M - 1), whatever
// the draw's own tc: the draws at the nodes (draw i, node m at position
// i M + m; layout [D][n M]) go through the likelihood like any other draws.
// The integral over the window is the extended trapezoid rule with fourth-order
// end corrections (Gregory's form: weights 17/48, 59/48, 43/48, 49/48 on the
// four nodes at each end and 1 inside, exact for cubics; M >= 8), so
//   ln L_t = ln sum_m c_m L_m - ln (M - 1).
// Inside the window the rule converges like the plain trapezoid rule on a
// smooth peak (error ~ exp(-2 pi^2 s^2 / h^2) for a peak of width s); a peak
// that the window cuts leaves an O(h^4) error from the end corrections.
__device__ __forceinline__ double tm_node(const EvConst& ec, int m) {
    const int M = ec.tm_points;
    return (m == M - 1) ? ec.tc_hi : ec.tc_lo + (ec.tc_hi - ec.tc_lo) * ((double)m / (double)(M - 1));
}

__device__ __forceinline__ double tm_weight(int m, int M) {
    const int e = (m < M - 1 - m) ? m : M - 1 - m;  // distance from the nearer end
    return e == 0 ? 17.0 / 48.0 : e == 1 ? 59.0 / 48.0 : e == 2 ? 43.0 / 48.0 : e == 3 ? 49.0 / 48.0 : 1.0;
}

__global__ __launch_bounds__(256) void k_tm_expand(const double* __restrict__ theta, int64_t n, EvConst ec,
                                                   double* __restrict__ out) {
    const int M = ec.tm_points;
    const int64_t nout = n * M;
    for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < nout; q += (int64_t)gridDim.x * 256) {
        const int64_t i = q / M;
        const int m = (int)(q - i * M);
        for (int a = 0; a < ec.dim; ++a)
            out[(int64_t)a * nout + q] = (a == 9) ? tm_node(ec, m) : theta[(int64_t)a * n + i];
    }
}

// One wave per draw: lane l takes the nodes l, l + 64, ... (coalesced reads),
// keeping its largest ln L_m and the weighted sum of exp(ln L_m - max) with a
// running maximum; a butterfly then merges the lanes' (max, sum) pairs. Both
// partners of an exchange form the same commutative sum, so every lane ends
// with the same value, and the order of the merge is fixed.
__global__ __launch_bounds__(256) void k_tm_reduce(const double* __restrict__ ll, int64_t n, EvConst ec,
                                                   double* __restrict__ out) {
    const int M = ec.tm_points;
    const double lnorm = -log((double)(M - 1));
    const int lane = threadIdx.x & 63;
    const int64_t waves = ((int64_t)gridDim.x * 256) >> 6;
    for (int64_t i = ((int64_t)blockIdx.x * 256 + threadIdx.x) >> 6; i < n; i += waves) {
        double mx = -INFINITY, acc = 0.0;
        int bad = 0;
        for (int m = lane; m < M; m += 64) {
            const double v = ll[i * M + m];
            if (isnan(v) || v == INFINITY) bad = 1;
            if (!(v > -INFINITY)) continue;
            const double c = tm_weight(m, M);
            if (v > mx) {
                acc = acc * exp(mx - v) + c;
                mx = v;
            } else {
                acc += c * exp(v - mx);
            }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const double mo = __shfl_xor(mx, o), ao = __shfl_xor(acc, o);
            bad |= __shfl_xor(bad, o);
            const double mm = fmax(mx, mo);
            if (mm > -INFINITY)
                acc = (mx > -INFINITY ? acc * exp(mx - mm) : 0.0) + (mo > -INFINITY ? ao * exp(mo - mm) : 0.0);
            mx = mm;
        }
        if (lane == 0) out[i] = bad ? NAN : (mx > -INFINITY ? mx + log(acc) + lnorm : -INFINITY);
    }
}

static unsigned tm_grid(int64_t blocks) { return (unsigned)(blocks < 1 ? 1 : (blocks < 16384 ? blocks : 16384)); }

hipError_t launch_tm_expand(const double* theta, int64_t n, const EvConst& ec, double* out, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    k_tm_expand<<<tm_grid(blocks256(n * ec.tm_points)), 256, 0, st>>>(theta, n, ec, out);
    return hipGetLastError();
}

hipError_t launch_tm_reduce(const double* ll, int64_t n, const EvConst& ec, double* out, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    k_tm_reduce<<<tm_grid(blocks256(n * 64)), 256, 0, st>>>(ll, n, ec, out);
    return hipGetLastError();
}

// The draws of a moment-path batch: theta with tc at the window's centre.
__global__ __launch_bounds__(256) void k_tm_centre(const double* __restrict__ theta, int64_t n, EvConst ec,
                                                   double* __restrict__ out) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        for (int a = 0; a < ec.dim; ++a) out[(int64_t)a * n + i] = (a == 9) ? ec.tm_tmid : theta[(int64_t)a * n + i];
}

// x^p of offset i in a block of `fine` bins: x = (i - (fine - 1) / 2) (2 / fine)
// in FP32 and its powers by repeated products, exactly as the moment hot loop
// forms them per bin (there (float)k - kmid is the same exact half-integer).
__global__ __launch_bounds__(256) void k_tm_powers(float* __restrict__ out, int fine, int P) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= fine) return;
    const float kmid = 0.5f * (float)(fine - 1);
    const float inv_half = 2.0f / (float)fine;
    const float x = ((float)i - kmid) * inv_half;
    float xp = 1.0f;
    for (int q = 0; q < P; ++q) {
        out[(int64_t)i * P + q] = xp;
        xp *= x;
    }
}

hipError_t launch_tm_powers(float* out, int fine, int P, hipStream_t st) {
    if (fine <= 0) return hipSuccess;
    k_tm_powers<<<(fine + 255) / 256, 256, 0, st>>>(out, fine, P);
    return hipGetLastError();
}

hipError_t launch_tm_centre(const double* theta, int64_t n, const EvConst& ec, double* out, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    k_tm_centre<<<tm_grid(blocks256(n)), 256, 0, st>>>(theta, n, ec, out);
    return hipGetLastError();
}

// Workgroups that fit on the GPU at once for a hot-loop kernel.
template <typename Kern>
static unsigned resident_grid(Kern kernel, int block = kTile) {
    int per_cu = 0, dev = 0, n_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 2048;
    if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 2048;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, 0) != hipSuccess || per_cu < 1)
        per_cu = 1;
    return (unsigned)(per_cu * n_cu);
}

static unsigned grid_for(int64_t blocks, unsigned cap = 16384) {
    if (blocks < 1) blocks = 1;
    return (unsigned)(blocks < (int64_t)cap ? blocks : cap);
}

static unsigned split_grid() {
    static const unsigned grid = resident_grid(k_b_split);
    return grid;
}
static unsigned f64_grid() {
    static const unsigned grid = resident_grid(k_b_f64);
    return grid;
}
static unsigned redo_grid() {
    static const unsigned grid = resident_grid(k_r_f64, kRedoTile);
    return grid;
}
static unsigned redo_grid_2det() {
    static const unsigned grid = resident_grid(k_r_f64_2det, kRedoTile);
    return grid;
}

// Evaluates the hot loop's resident grids (device queries) ahead of any graph
// capture.
void prime_hot_grids() {
    (void)split_grid();
    (void)f64_grid();
    (void)redo_grid();
    (void)redo_grid_2det();
}

hipError_t launch_loglike_batch(const BatchPtrs& b, int ne, int64_t prologue_blocks, int64_t finalize_blocks,
                                int precision, bool profile, bool any_dist, int max_det, hipStream_t st) {
    if (ne <= 0) return hipSuccess;
    const EvDev* evs = (const EvDev*)b.args;
    int64_t* ioff = (int64_t*)b.scratch;
    const unsigned eg = (unsigned)min(ne, 1024);
    if (prologue_blocks > 0) {
        const unsigned nb = grid_for(prologue_blocks);
        k_b_reset<<<dim3(kBuckets / 256, eg), 256, 0, st>>>(b.hdr, evs);
        k_b_support<<<nb, 256, 0, st>>>(b.hdr, evs, b.off);
        k_b_plan<<<eg, 1024, 0, st>>>(b.hdr, evs);
        k_b_scatter<<<nb, 256, 0, st>>>(b.hdr, evs, b.off);
    }
    k_items<false><<<1, kItemThreads, 0, st>>>(b.hdr, evs, ioff);
    if (prologue_blocks > 0) k_b_coeffs<<<grid_for(prologue_blocks), 256, 0, st>>>(b.hdr, evs, b.off);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (precision == PE_PREC_SPLIT) {
        const unsigned grid = split_grid();
        if (profile) prof_begin("loglike_split", st);
        k_b_split<<<grid, kTile, 0, st>>>(b.hdr, evs, ioff);
        if (profile) prof_end("loglike_split", st);
    } else {
        const unsigned grid = f64_grid();
        if (profile) prof_begin("loglike_fp64", st);
        k_b_f64<<<grid, kTile, 0, st>>>(b.hdr, evs, ioff);
        if (profile) prof_end("loglike_fp64", st);
    }
    if (finalize_blocks > 0) {
        const unsigned fg = grid_for(finalize_blocks);
        if (precision == PE_PREC_SPLIT) {
            k_b_finalize<true><<<fg, 256, 0, st>>>(b.hdr, evs, b.off2);
            // FP64 re-evaluation of the draws whose error estimate exceeds the budget
            k_r_plan<<<eg, 1024, 0, st>>>(b.hdr, evs);
            k_r_scatter<<<fg, 256, 0, st>>>(b.hdr, evs, b.off2);
            k_items<true><<<1, kItemThreads, 0, st>>>(b.hdr, evs, ioff);
            if (profile) prof_begin("loglike_redo", st);
            if (max_det <= 2)
                k_r_f64_2det<<<redo_grid_2det(), kRedoTile, 0, st>>>(b.hdr, evs, ioff);
            else
                k_r_f64<<<redo_grid(), kRedoTile, 0, st>>>(b.hdr, evs, ioff);
            if (profile) prof_end("loglike_redo", st);
            k_r_finalize<<<fg, 256, 0, st>>>(b.hdr, evs, b.off2);
        } else {
            k_b_finalize<false><<<fg, 256, 0, st>>>(b.hdr, evs, b.off2);
        }
        if (any_dist) k_b_dist<<<grid_for(finalize_blocks * kDistLanes), 256, 0, st>>>(b.hdr, evs, b.off2);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Time marginal on the block-moment path (split precision). The draws are
// evaluated once, with tc at the window's centre t_mid. Shifting tc by u
// multiplies a detector term at f by exp(-2 pi i f u), so with y_k the
// detector-summed term sum_d R_d z_dk of bin k,
//   Z(u) = sum_k y_k exp(-2 pi i f_k u)
//        = sum_c exp(-2 pi i f_c u) sum_p mu_cp (-i a u)^p / p!,
//   mu_cp = sum_{k in block c} y_k x_k^p,  x_k = (f_k - f_c) / (D / 2),
// over blocks c of D = ec.tm_fine bins' width with centres f_c and a = pi D
// (the plan's chunks are these blocks). The hot loop writes the moments; the
// node kernel forms Z at every tc node from them.
// ---------------------------------------------------------------------------

// One item of the moment hot loop: split_item's walk (records staged in LDS,
// FP32 sums over kBlk bins folded into FP64, the same masking of bins past a
// lane's cut), with the detector terms combined with the draw's responses and
// summed into the P moments of each chunk, written to tm_mom[(c P + p) npad + j].
template <int P>
struct PowRow {
    float v[P];
};

template <int NDET, int P, bool TAB>
__device__ __forceinline__ void split_tm_item(const EvDev& E, const EvPlan& p, int tile, int g, Rec32* srec,
                                              int* sred) {
    int j, kc, wmin, wmax;
    bool valid;
    DrawRow row;
    double tau[NDET];
    item_setup<NDET>(E, p.n_active, tile, j, valid, row, tau, kc, wmin, wmax);
    const Rec32* tab = E.rec32;
    const int K = (int)E.ec.K;
    const int64_t np = E.npad;
    const int jl = valid ? j : p.n_active - 1;
    float rr[NDET], ri[NDET];
#pragma unroll
    for (int d = 0; d < NDET; ++d) {
        rr[d] = (float)((const double*)E.resp)[(2 * d) * np + jl];
        ri[d] = (float)((const double*)E.resp)[(2 * d + 1) * np + jl];
    }
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) sred[wv] = wmax;
    __syncthreads();
    const int gmax = max(max(sred[0], sred[1]), max(sred[2], sred[3]));
    const float inv_half = 2.0f / (float)p.fine;
    for (int c = g; c < p.n_fine; c += p.n_groups) {
        const int k0 = c * p.fine;
        if (k0 >= gmax) break;  // uniform over the workgroup
        const int k1 = min(k0 + p.fine, K);
        const bool on = k0 < wmax;
        const int kA = on ? k0 + (max(0, min(wmin, k1) - k0) / kBlk) * kBlk : k0;
        const int kB = on ? max(kA, min(k1, wmax)) : k0;
        const int kl = min(k1, gmax);
        const float kmid = (float)k0 + 0.5f * (float)(p.fine - 1);
        double mr[P], mi[P];
#pragma unroll
        for (int q = 0; q < P; ++q) mr[q] = mi[q] = 0.0;
        for (int ks = k0; ks < kl; ks += kStage) {
            const int ke = min(ks + kStage, kl);
            __syncthreads();  // the previous piece has been read
            const uint4* src = (const uint4*)(tab + ks);
            uint4* dst = (uint4*)srec;
            for (int q = threadIdx.x; q < (ke - ks) * (int)(sizeof(Rec32) / 16); q += 256) dst[q] = src[q];
            __syncthreads();
            for (int kb = ks; kb < min(ke, kB); kb += kBlk) {
                const int kq = min(kb + kBlk, kB);
                float br[P], bi[P];
#pragma unroll
                for (int q = 0; q < P; ++q) br[q] = bi[q] = 0.0f;
                for (int k = kb; k < kq; ++k) {
                    const Rec32 r = srec[k - ks];
                    const double psi = psi_turns(row.A, row.B5, row.B6, r.x, r.xm5, r.lnx);
                    const bool live = (k < kA) || (k < kc);
                    float yr = 0.0f, yi = 0.0f;
#pragma unroll
                    for (int d = 0; d < NDET; ++d) {
                        const double ph = fma(r.f, tau[d], psi);
                        const float t = (float)fract64(ph) + r.w[d].y;
                        const float sn = __builtin_amdgcn_sinf(t);
                        const float cs = __builtin_amdgcn_cosf(t);
                        const float m = live ? r.w[d].x : 0.0f;
                        const float tr = m * cs, ti = -m * sn;
                        yr = fmaf(rr[d], tr, fmaf(-ri[d], ti, yr));
                        yi = fmaf(rr[d], ti, fmaf(ri[d], tr, yi));
                    }
                    if constexpr (TAB) {
                        // the same powers from the event's table (scalar loads: k is uniform)
                        const PowRow<P> pw = load_const((const PowRow<P>*)(E.tm_pow + (int64_t)(k - k0) * P));
#pragma unroll
                        for (int q = 0; q < P; ++q) {
                            br[q] = fmaf(yr, pw.v[q], br[q]);
                            bi[q] = fmaf(yi, pw.v[q], bi[q]);
                        }
                    } else {
                        const float x = ((float)k - kmid) * inv_half;
                        float xp = 1.0f;
#pragma unroll
                        for (int q = 0; q < P; ++q) {
                            br[q] = fmaf(yr, xp, br[q]);
                            bi[q] = fmaf(yi, xp, bi[q]);
                            xp *= x;
                        }
                    }
                }
                if (kb < kA || kb < kc) {
#pragma unroll
                    for (int q = 0; q < P; ++q) {
                        mr[q] += (double)br[q];
                        mi[q] += (double)bi[q];
                    }
                }
            }
        }
        if (valid && on) {
#pragma unroll
            for (int q = 0; q < P; ++q) E.tm_mom[((int64_t)c * P + q) * np + j] = make_double2(mr[q], mi[q]);
        }
    }
    __syncthreads();  // sred and srec are reused by the next item
}

template <int P>
__global__ __launch_bounds__(256) void k_b_split_tm(BatchHdr* __restrict__ hdr, const EvDev* __restrict__ evs,
                                                    const int64_t* __restrict__ ioff) {
    __shared__ Rec32 srec[kStage];
    __shared__ int sred[4];
    item_loop<false>(hdr, ioff, evs, [&](const Item& it) {
        const EvDev& E = evs[it.e];
        const EvPlan p = load_const(E.plan);
        if (E.tm_pow) {
            switch (E.ec.n_det) {
                case 1: split_tm_item<1, P, true>(E, p, it.tile, it.g, srec, sred); break;
                case 2: split_tm_item<2, P, true>(E, p, it.tile, it.g, srec, sred); break;
                case 3: split_tm_item<3, P, true>(E, p, it.tile, it.g, srec, sred); break;
                default: split_tm_item<4, P, true>(E, p, it.tile, it.g, srec, sred); break;
            }
        } else {
            switch (E.ec.n_det) {
                case 1: split_tm_item<1, P, false>(E, p, it.tile, it.g, srec, sred); break;
                case 2: split_tm_item<2, P, false>(E, p, it.tile, it.g, srec, sred); break;
                case 3: split_tm_item<3, P, false>(E, p, it.tile, it.g, srec, sred); break;
                default: split_tm_item<4, P, false>(E, p, it.tile, it.g, srec, sred); break;
            }
        }
    });
}

// One workgroup per live draw position. In passes of 256 tc nodes (one per
// thread), the draw's moments are staged in LDS in pieces of kTmPiece chunks;
// each thread carries its node's Z(u) and the chunk phasor exp(-2 pi i f_c u)
// (advanced chunk to chunk by exp(-2 pi i D u)) over the chunks below the
// draw's cut, then takes the node's ln L from Z and H (the phase and distance
// marginals as the event has them) into a running weighted log-sum-exp with
// the end-corrected trapezoid weights of k_tm_reduce. The threads' (max, sum)
// pairs merge by a wave butterfly and then over the four waves in order.
// Distance-marginalised events take two passes: the distance integral at a
// node, ln L_D = ln int 3 x^-4 exp(phi(x) - b x^2) dx over x >= 1, is at most
// max_x (a x - b x^2) (phi <= a x for both phase forms, and 3 x^-4 integrates
// to 1): a^2 / (4 b) when a >= 2 b, else a - b. The first pass finds the node
// with the largest such bound and integrates there (L*); the second integrates
// only the nodes whose bound reaches L* - kTmSkip, the others adding less than
// e^-kTmSkip of the largest term each (with at most 16384 nodes, below 7e-7 of
// the sum together).
constexpr int kTmPiece = 128;

// ln L at a node: the phase marginal exactly, the distance integral in its
// light form (within 5e-7 in ln; see log_dist_marg).
__device__ __forceinline__ double node_loglike(const EvConst& ec, double zr, double zi, double h) {
    if (!ec.dist) return loglike_phase(ec, zr, zi, h);
    const bool ex = (ec.phase == PE_PHASE_EXPLICIT);
    return log_dist_marg<1, true>(ex ? zr : hypot(zr, zi), 0.5 * h, ex, 0);
}
constexpr double kTmSkip = 24.0;
constexpr int kTmCached = 4;  // nodes per thread whose Z stays in registers (M <= 1024)

__device__ __forceinline__ double dist_bound(const EvConst& ec, double zr, double zi, double h) {
    const double a = (ec.phase == PE_PHASE_EXPLICIT) ? zr : hypot(zr, zi), b = 0.5 * h;
    if (!(b > 0.0)) return (a == 0.0) ? 0.0 : INFINITY;
    return (a >= 2.0 * b) ? a * a / (4.0 * b) : a - b;
}

// Z(u) of node m of draw j (act: m < M; threads past M follow the staging
// barriers and return 0).
template <int P>
__device__ __forceinline__ void tm_node_z(const EvDev& E, const EvPlan& p, int64_t j, int nch, int m, bool act,
                                          double2* smom, double& zr, double& zi) {
    const EvConst& ec = E.ec;
    const int M = ec.tm_points;
    const double T = ec.tc_hi - ec.tc_lo;
    const double Df = (double)p.fine * ec.df;  // block width (Hz)
    const double fc0 = ec.f_lo + 0.5 * (double)(p.fine - 1) * ec.df;
    const int64_t np = E.npad;
    const double t = (m == M - 1) ? ec.tc_hi : ec.tc_lo + T * ((double)m / (double)(M - 1));
    const double u = act ? t - ec.tm_tmid : 0.0;
    // (-i a u)^k / k!
    double bre[P], bim[P];
    bre[0] = 1.0;
    bim[0] = 0.0;
#pragma unroll
    for (int k = 1; k < P; ++k) {
        const double s = ec.tm_a * u / (double)k;  // multiply by -i s
        bre[k] = bim[k - 1] * s;
        bim[k] = -bre[k - 1] * s;
    }
    double pr, pi_, sr, si;
    sincos_turns(-fract64(fc0 * u), pi_, pr);  // exp(-2 pi i f_c0 u)
    sincos_turns(-fract64(Df * u), si, sr);    // step to the next chunk
    // S_k = sum_c mu_ck exp(-2 pi i f_c u): P independent sums over the chunks,
    // then Z = sum_k S_k (-i a u)^k / k!
    double ar[P], ai[P];
#pragma unroll
    for (int k = 0; k < P; ++k) ar[k] = ai[k] = 0.0;
    zr = zi = 0.0;
    for (int c0 = 0; c0 < nch; c0 += kTmPiece) {
        const int nc = min(kTmPiece, nch - c0);
        __syncthreads();  // the previous piece has been read
        for (int w = threadIdx.x; w < nc * P; w += 256)
            smom[w] = E.tm_mom[((int64_t)(c0 + w / P) * P + (w % P)) * np + j];
        __syncthreads();
        for (int c = 0; c < nc; ++c) {
#pragma unroll
            for (int k = 0; k < P; ++k) {
                const double2 v = smom[c * P + k];
                ar[k] = fma(v.x, pr, fma(-v.y, pi_, ar[k]));
                ai[k] = fma(v.x, pi_, fma(v.y, pr, ai[k]));
            }
            const double nr = pr * sr - pi_ * si;
            pi_ = pr * si + pi_ * sr;
            pr = nr;
        }
    }
#pragma unroll
    for (int k = 0; k < P; ++k) {
        zr = fma(ar[k], bre[k], fma(-ai[k], bim[k], zr));
        zi = fma(ar[k], bim[k], fma(ai[k], bre[k], zi));
    }
}

template <int P>
__global__ __launch_bounds__(256) void k_tm_nodes(const BatchHdr* __restrict__ hdr, const EvDev* __restrict__ evs,
                                                  const int64_t* __restrict__ foff) {
    __shared__ double2 smom[kTmPiece * P];
    __shared__ double sg[4], ss[4];
    __shared__ int sb[4], sm[4];
    __shared__ double sL;
    const int ne = hdr->ne;
    const int64_t npos = foff[ne] * 256;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int64_t q = blockIdx.x; q < npos; q += gridDim.x) {
        const int e = find_slot(foff, ne, q >> 8);
        const EvDev& E = evs[e];
        const EvConst& ec = E.ec;
        const EvPlan p = *E.plan;
        const int64_t j = q - foff[e] * 256;
        if (j >= p.n_active) continue;  // uniform over the workgroup
        const int kc = E.kcut[j];
        const int nch = (kc + p.fine - 1) / p.fine;
        const double h = E.hh[j];
        const int M = ec.tm_points;
        double mx = -INFINITY, acc = 0.0;
        int bad = 0;
        // the node's ln L into the running weighted log-sum-exp
        auto take = [&](int m, double zr, double zi, double lstar) {
            double v;
            if (ec.dist && dist_bound(ec, zr, zi, h) < lstar - kTmSkip)
                v = -INFINITY;  // below e^-kTmSkip of the largest node
            else
                v = node_loglike(ec, zr, zi, h);
            if (isnan(v) || v == INFINITY) bad = 1;
            if (v > -INFINITY) {
                const double cw = tm_weight(m, M);
                if (v > mx) {
                    acc = acc * exp(mx - v) + cw;
                    mx = v;
                } else {
                    acc += cw * exp(v - mx);
                }
            }
        };
        // distance-marginalised events: the node of the largest bound (the
        // smallest such m on ties) over the workgroup, from each thread's (ub, um)
        auto best_node = [&](double ub, int um, int& bm) {
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                const double uo = __shfl_xor(ub, o);
                const int mo = __shfl_xor(um, o);
                if (uo > ub || (uo == ub && mo < um)) {
                    ub = uo;
                    um = mo;
                }
            }
            if (lane == 0) {
                sg[wv] = ub;
                sm[wv] = um;
            }
            __syncthreads();
            double bu = sg[0];
            bm = sm[0];
            for (int w = 1; w < 4; ++w)
                if (sg[w] > bu || (sg[w] == bu && sm[w] < bm)) {
                    bu = sg[w];
                    bm = sm[w];
                }
        };
        if (M <= kTmCached * 256) {
            // each thread's nodes' Z kept in registers: one pass over the moments
            double cr[kTmCached], ci[kTmCached];
#pragma unroll
            for (int i = 0; i < kTmCached; ++i) {
                cr[i] = ci[i] = 0.0;
                if (i * 256 < M) {  // uniform
                    const int m = i * 256 + (int)threadIdx.x;
                    tm_node_z<P>(E, p, j, nch, m, m < M, smom, cr[i], ci[i]);
                }
            }
            double lstar = -INFINITY;
            if (ec.dist) {
                double ub = -INFINITY;
                int um = 0;
#pragma unroll
                for (int i = 0; i < kTmCached; ++i) {
                    const int m = i * 256 + (int)threadIdx.x;
                    const double bnd = dist_bound(ec, cr[i], ci[i], h);
                    if (m < M && bnd > ub) {
                        ub = bnd;
                        um = m;
                    }
                }
                int bm;
                best_node(ub, um, bm);
                // the owner of that node integrates there
#pragma unroll
                for (int i = 0; i < kTmCached; ++i)
                    if (i * 256 + (int)threadIdx.x == bm) sL = node_loglike(ec, cr[i], ci[i], h);
                __syncthreads();
                lstar = sL;
            }
#pragma unroll
            for (int i = 0; i < kTmCached; ++i) {
                const int m = i * 256 + (int)threadIdx.x;
                if (m < M) take(m, cr[i], ci[i], lstar);
            }
        } else {
            // more nodes: Z recomputed per pass
            double lstar = -INFINITY;
            if (ec.dist) {
                double ub = -INFINITY;
                int um = 0;
                for (int m0 = 0; m0 < M; m0 += 256) {
                    const int m = m0 + (int)threadIdx.x;
                    double zr, zi;
                    tm_node_z<P>(E, p, j, nch, m, m < M, smom, zr, zi);
                    const double bnd = dist_bound(ec, zr, zi, h);
                    if (m < M && bnd > ub) {
                        ub = bnd;
                        um = m;
                    }
                }
                int bm;
                best_node(ub, um, bm);
                double zr, zi;
                tm_node_z<P>(E, p, j, nch, bm, true, smom, zr, zi);  // collective staging
                if (threadIdx.x == 0) sL = node_loglike(ec, zr, zi, h);
                __syncthreads();
                lstar = sL;
            }
            for (int m0 = 0; m0 < M; m0 += 256) {
                const int m = m0 + (int)threadIdx.x;
                double zr, zi;
                tm_node_z<P>(E, p, j, nch, m, m < M, smom, zr, zi);
                if (m < M) take(m, zr, zi, lstar);
            }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const double mo = __shfl_xor(mx, o), ao = __shfl_xor(acc, o);
            bad |= __shfl_xor(bad, o);
            const double mm = fmax(mx, mo);
            if (mm > -INFINITY)
                acc = (mx > -INFINITY ? acc * exp(mx - mm) : 0.0) + (mo > -INFINITY ? ao * exp(mo - mm) : 0.0);
            mx = mm;
        }
        __syncthreads();  // sg is free again
        if (lane == 0) {
            sg[wv] = mx;
            ss[wv] = acc;
            sb[wv] = bad;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double G = -INFINITY, S = 0.0;
            int b = 0;
            for (int w = 0; w < 4; ++w) {
                b |= sb[w];
                if (!(sg[w] > -INFINITY)) continue;
                if (sg[w] > G) {
                    S = S * exp(G - sg[w]) + ss[w];
                    G = sg[w];
                } else {
                    S += ss[w] * exp(sg[w] - G);
                }
            }
            E.loglike[E.idx[j]] = b ? NAN : (G > -INFINITY ? G + log(S) - log((double)(M - 1)) : -INFINITY);
        }
        __syncthreads();  // sg, ss, sb, sL are reused by the next draw
    }
}

template <int P>
static void launch_moments_p(const BatchPtrs& b, const EvDev* evs, int64_t* ioff, unsigned grid, unsigned ng,
                             hipStream_t st) {
    k_b_split_tm<P><<<grid, kTile, 0, st>>>(b.hdr, evs, ioff);
    k_tm_nodes<P><<<ng, 256, 0, st>>>(b.hdr, evs, b.off2);
}

static unsigned split_tm_grid(int P) {
    static const unsigned g8 = resident_grid(k_b_split_tm<8>);
    static const unsigned g16 = resident_grid(k_b_split_tm<16>);
    return P == 8 ? g8 : g16;
}

hipError_t launch_loglike_moments(const BatchPtrs& b, int ne, int64_t prologue_blocks, int64_t node_blocks, int P,
                                  hipStream_t st) {
    if (ne <= 0) return hipSuccess;
    if (P != 8 && P != 16) return hipErrorInvalidValue;
    const EvDev* evs = (const EvDev*)b.args;
    int64_t* ioff = (int64_t*)b.scratch;
    const unsigned eg = (unsigned)min(ne, 1024);
    const unsigned nb = grid_for(prologue_blocks);
    k_b_reset<<<dim3(kBuckets / 256, eg), 256, 0, st>>>(b.hdr, evs);
    k_b_support<<<nb, 256, 0, st>>>(b.hdr, evs, b.off);
    k_b_plan<<<eg, 1024, 0, st>>>(b.hdr, evs);
    k_b_scatter<<<nb, 256, 0, st>>>(b.hdr, evs, b.off);
    k_items<false><<<1, kItemThreads, 0, st>>>(b.hdr, evs, ioff);
    k_b_coeffs<<<nb, 256, 0, st>>>(b.hdr, evs, b.off);
    const unsigned ng = grid_for(node_blocks * 256);
    if (P == 8)
        launch_moments_p<8>(b, evs, ioff, split_tm_grid(8), ng, st);
    else
        launch_moments_p<16>(b, evs, ioff, split_tm_grid(16), ng, st);
    return hipGetLastError();
}

}  // namespace pe
