// kernels.hip -- HIP kernels of the betweenness library (gfx950).
//
// Batched form: a persistent launch of B workgroups, one state slab each;
// every workgroup takes sources from a device counter and runs the whole
// per-source pipeline with workgroup barriers only (one block per root
// vertex with the block's threads sharing that source, Sec. 3.1).
//
// Plain form: one source at a time on the whole GPU; a one-thread control
// kernel advances a phase machine held in device memory and a grid-wide step
// kernel executes the current phase, so the host only launches pairs of
// kernels and polls for completion now and then.
#include <algorithm>

#include "kernels.h"
#include "dev_common.h"
#include "passes.h"

#define WG_SCOPE __HIP_MEMORY_SCOPE_WORKGROUP
#define AG_SCOPE __HIP_MEMORY_SCOPE_AGENT

// ---------------------------------------------------------------------------
// Batched form
// ---------------------------------------------------------------------------
// Far values this many band widths or more beyond the threshold wait in the
// outer pile, which is scanned only when the threshold passes its bound.
#ifndef OUTER_BANDS
#define OUTER_BANDS 16
#endif

__device__ __forceinline__ uint32_t sat_add_u32(uint32_t x, uint64_t y)
{
    const uint64_t t = (uint64_t)x + y;
    return t > BC_INF ? BC_INF : (uint32_t)t;
}

struct WgCtl {
    int near_len, next_cnt, order_cnt, far_cnt, kept_cnt, pend_cnt;
    int outer_cnt, okept_cnt, resplit;
    int huge_cnt;
    int32_t huge_q[EXPAND_WG_CAP]; // hubs of the current pass, expanded by the workgroup
    int cur, fcur, ocur;
    int32_t gen, band_gen;
    uint32_t thr, thr_old, far_min, bound, outer_min;
    int band_start, nbands;
    int abort;
    int32_t prev_s; // this slab's previous source whose dependencies are not in bcp yet
    long long src_idx;
    unsigned long long iters;
    unsigned int bands, srounds, drounds;
    unsigned long long ticks[5]; // per-phase device time of this workgroup
    // far-bucket ring: entries per slot, the bucket of the current band, the
    // next non-empty one (offset from bcur, 0 = none), outer pile must be scanned
    int bcnt[BC_BUCKETS_MAX];
    int32_t bcur;
    int bnext, forced;
};

// Phase timing of one workgroup: thread 0 reads the constant-rate device
// clock at phase boundaries (phases: 0 init, 1 expansion, 2 counts,
// 3 dependencies, 4 far split).
__device__ __forceinline__ void phase_mark(WgCtl &C, long long &t0, int phase)
{
    if (threadIdx.x == 0) {
        const long long t = wall_clock64();
        C.ticks[phase] += (unsigned long long)(t - t0);
        t0 = t;
    }
}

// Far-bucket ring: after band C.bcur closed, the next band is the least
// non-empty bucket, over the ring and a lower bound of the outer pile (values
// beyond the ring, or pushes a full bucket could not take).  When the outer
// pile may hold values of the new ring window, or a bucket overflowed, it is
// scanned: entries of the new band's bucket join the band at once, entries of
// later buckets in the window move into the ring (or stay, if theirs is
// full), settled entries are dropped.  Then the ring bucket's entries move into
// the near queue as the band [b delta, (b + 1) delta); entries whose vertex
// was put in a lower bucket since, or settled in an earlier band, and repeats
// are skipped.  Returns false once no vertex is left, or when the band bound
// trips.
template <int NT>
__device__ __forceinline__ bool bucket_next_band(const Slab &S, WgCtl &C, const BatchArgs &a,
                                                 unsigned long long iter_cap)
{
    const int tid = threadIdx.x;
    const int lane = lane_id();
    const int nbk = a.nbk;
    const uint32_t D = a.delta;
    // the least non-empty ring bucket in (bcur, bcur + nbk), as an offset
    if (tid < WAVE) {
        int found = 0;
        for (int j0 = 1; j0 < nbk && !found; j0 += WAVE) {
            const int j = j0 + lane;
            const bool ne = j < nbk && C.bcnt[(int)(((uint32_t)C.bcur + j) % (uint32_t)nbk)] > 0;
            const uint64_t m = __ballot(ne);
            if (m)
                found = j0 + __ffsll((unsigned long long)m) - 1;
        }
        if (lane == 0)
            C.bnext = found;
    }
    __syncthreads();
    if (tid == 0) {
        uint64_t b = UINT64_MAX;
        if (C.bnext > 0)
            b = (uint64_t)C.bcur + (uint64_t)C.bnext;
        if (C.outer_cnt > 0) {
            // outer_min is at most the distance of every unsettled outer entry
            uint64_t bo = C.outer_min / D;
            if (bo < (uint64_t)C.bcur + 1)
                bo = (uint64_t)C.bcur + 1;
            if (bo < b)
                b = bo;
        }
        C.bnext = b == UINT64_MAX ? -1 : 0;
        if (b != UINT64_MAX) {
            C.bcur = (int32_t)b;
            C.thr_old = C.thr;
            C.thr = sat_add_u32(0u, (b + 1) * D);
            C.bound = sat_add_u32(0u, (b + (uint64_t)nbk) * D);
            C.gen += 1;
            C.band_gen = C.gen;
            C.near_len = 0;
            C.resplit = C.outer_cnt > 0 &&
                        (C.forced || (uint64_t)(C.outer_min / D) < b + (uint64_t)nbk);
            if (C.resplit) {
                C.forced = 0;
                C.outer_min = BC_INF;
                C.okept_cnt = 0;
            }
            if (++C.iters > iter_cap)
                C.abort = 1;
        }
    }
    __syncthreads();
    if (C.bnext < 0 || C.abort)
        return false;
    const uint32_t bcur = (uint32_t)C.bcur;
    int32_t *nq = C.cur ? S.qb : S.qa;
    if (C.resplit) {
        const int32_t *in = C.ocur ? S.ob : S.oa;
        int32_t *out = C.ocur ? S.oa : S.ob;
        const int len = C.outer_cnt;
        uint32_t kmin = BC_INF;
        for (int base = (tid / WAVE) * WAVE; base < len; base += NT) {
            const int i = base + lane;
            bool keep = false, mv = false;
            int32_t v = 0;
            uint32_t dv = 0;
            if (i < len) {
                v = in[i];
                dv = dist_get(S, v);
                const uint32_t b = dv / D;
                if (b == bcur) {
                    mv = atomic_xchg_i32<WG_SCOPE>(&S.stamp[v], C.gen) != C.gen;
                } else if (b > bcur) {
                    keep = true;
                    if ((uint64_t)b < (uint64_t)bcur + nbk) {
                        const int slot = (int)(b % (uint32_t)nbk);
                        const int k = atomicAdd(&C.bcnt[slot], 1);
                        if (k < a.bcap) {
                            S.fa[(size_t)slot * (size_t)a.bcap + (size_t)k] = v;
                            // the entry is current for bucket b (its key at most b's
                            // already when the pile took it from a full bucket)
                            __hip_atomic_fetch_min(&S.pred1[v], BUCKET_KEY(b), __ATOMIC_RELAXED,
                                                   WG_SCOPE);
                            keep = false;
                        } else {
                            C.forced = 1;
                        }
                    }
                }
                // An entry leaving the pile clears its pile flag: unlike in the
                // two-tier pile, a vertex can need the pile again (when a lower
                // bucket it drops into is full).  Each vertex has at most one
                // entry in the pile at a time.
                if (b >= bcur && !keep)
                    __hip_atomic_fetch_and(&S.infar[v], ~2, __ATOMIC_RELAXED, WG_SCOPE);
            }
            if (keep)
                kmin = dv < kmin ? dv : kmin;
            int k = wave_alloc(&C.okept_cnt, keep);
            if (keep)
                out[k] = v;
            k = wave_alloc(&C.near_len, mv);
            if (mv)
                nq[k] = v;
            k = wave_alloc(&C.order_cnt, mv);
            if (mv)
                S.order[k] = v;
        }
        kmin = wave_min_u32(kmin);
        if (lane == 0 && kmin != BC_INF)
            atomicMin(&C.outer_min, kmin);
        __syncthreads();
        if (tid == 0) {
            C.ocur ^= 1;
            C.outer_cnt = C.okept_cnt;
        }
    }
    const int slot = (int)(bcur % (uint32_t)nbk);
    const int len = C.bcnt[slot] < a.bcap ? C.bcnt[slot] : a.bcap;
    const int32_t *in = S.fa + (size_t)slot * (size_t)a.bcap;
    for (int base = (tid / WAVE) * WAVE; base < len; base += NT) {
        const int i = base + lane;
        bool mv = false;
        int32_t v = 0;
        if (i < len) {
            v = in[i];
            // current exactly when the vertex's least bucket is still this one:
            // a later push to a lower bucket lowers the key, and the count pass
            // of the band a vertex settles in overwrites it (no distance read)
            if (S.pred1[v] == BUCKET_KEY(bcur))
                mv = atomic_xchg_i32<WG_SCOPE>(&S.stamp[v], C.gen) != C.gen;
        }
        int k = wave_alloc(&C.near_len, mv);
        if (mv)
            nq[k] = v;
        k = wave_alloc(&C.order_cnt, mv);
        if (mv)
            S.order[k] = v;
    }
    __syncthreads();
    if (tid == 0)
        C.bcnt[slot] = 0;
    __syncthreads();
    return true;
}

// Runs the count (or dependency) rounds over the members order[b0, b1) of
// one band inside a workgroup.  Returns false if the round bound tripped.
template <bool PACKED, int NT, bool SIGMA, bool ATOMIC_BC, bool RECORD>
__device__ __forceinline__ bool wg_band_rounds(const DevGraph &g, const Slab &S, WgCtl &C, const BatchArgs &a,
                               int32_t s, long long idx, int b0, int b1, double *bc,
                               uint64_t &st_arcs, uint64_t &st_dag)
{
    const int tid = threadIdx.x;
    const int32_t *items = S.order + b0;
    int len = b1 - b0;
    int which = 0;
    const int cap = len + 2;
    for (int round = 0;; ++round) {
        if (tid == 0)
            C.pend_cnt = 0;
        __syncthreads();
        RoundCtx rc;
        rc.items = items;
        rc.len = len;
        rc.worker = tid / WAVE;
        rc.nworkers = NT / WAVE;
        rc.lane_max = a.lane_max;
        rc.s = s;
        rc.src_idx = idx;
        rc.first_round = round == 0;
        rc.pend_q = which ? S.qb : S.qa;
        rc.pend_cnt = &C.pend_cnt;
        rc.err = a.err;
        rc.item_err = a.item_err;
        rc.perm = ATOMIC_BC ? a.perm : nullptr;
        rc.keys = a.ebc == nullptr;
        rc.band_gen = C.band_gen;
        rc.wave_deg = a.wave_deg;
        rc.count_arcs = 0; // counted in the streaming pass of the next initialisation
        if (SIGMA)
            sigma_round<PACKED, WG_SCOPE, RECORD>(g, S, rc, st_arcs, st_dag);
        else
            delta_round<PACKED, WG_SCOPE, ATOMIC_BC>(g, S, rc, bc);
        __syncthreads();
        const int nl = C.pend_cnt;
        __syncthreads(); // everyone has read pend_cnt before it is touched again
        if (tid == 0) {
            if (SIGMA)
                C.srounds++;
            else
                C.drounds++;
        }
        if (nl == 0)
            return true;
        if (round + 1 >= cap)
            return false;
        items = which ? S.qb : S.qa;
        which ^= 1;
        len = nl;
    }
}

// Re-bases the 8-bit LDS distances to nb (see LDS8_WIN): entries below nb are
// settled, their distances go to d[] and they become 0; the others are
// shifted (an entry kept in d[] comes back into the window when it fits).
// No other access to the entries may run meanwhile.
__device__ __forceinline__ void lds8_rebase(const Slab &S, uint32_t nb, int tid, int nthreads)
{
    const uint32_t ob = S.base8;
    const int words = (S.H + 3) >> 2;
    for (int wi = tid; wi < words; wi += nthreads) {
        const uint32_t w = lds_ptr(S.ld)[wi];
        uint32_t out = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t u = (uint32_t)wi * 4u + (uint32_t)j;
            const uint32_t h = (w >> (8 * j)) & 0xffu;
            uint32_t e = h;
            if ((int32_t)u < S.H) {
                if (h - 1u < LDS8_WIN) {
                    const uint32_t dv = ob + h - 1u;
                    if (dv < nb) {
                        S.d[u] = dv;
                        e = 0u;
                    } else {
                        e = dv - nb + 1u; // at most h, as nb >= ob
                    }
                } else if (h == LDS8_FAR) {
                    const uint32_t dv = S.d[u];
                    if (dv < nb)
                        e = 0u;
                    else if (dv - nb + 1u <= LDS8_WIN)
                        e = dv - nb + 1u;
                }
            }
            out |= e << (8 * j);
        }
        lds_ptr(S.ld)[wi] = out;
    }
}

template <bool PACKED, int NT, bool ATOMIC_BC, int LB, bool BKT>
__global__ __launch_bounds__(NT) void k_batched(BatchArgs a)
{
    __shared__ WgCtl C;
    extern __shared__ uint32_t lds_dist[];
    const int tid = threadIdx.x;
    const int lane = lane_id();
    const DevGraph &g = a.g;
    const int n = g.n;
    Slab S = slab_at(a.slab_base, a.L, blockIdx.x);
    S.ld = lds_dist;
    S.H = a.H;
    // compile-time constants: each instantiation keeps one distance path
    S.w16 = LB == 16;
    S.w8 = LB == 8;
    if (!ATOMIC_BC)
        for (int v = tid; v < n; v += NT)
            S.bcp[v] = 0.0;
    uint64_t st_arcs = 0, st_dag = 0, st_imp = 0;
    if (tid == 0) {
        C.gen = (int32_t)S.hdr[0];
        C.prev_s = -1;
        C.iters = 0;
        C.bands = C.srounds = C.drounds = 0;
        for (int i = 0; i < 5; ++i)
            C.ticks[i] = 0;
    }
    long long tmark = tid == 0 ? wall_clock64() : 0;
    __syncthreads();
    const unsigned long long iter_cap = 8ull * (unsigned long long)n + 1024ull;

    for (;;) {
        if (tid == 0)
            C.src_idx = (long long)atomicAdd(a.next_src, 1ull);
        __syncthreads();
        const long long idx = C.src_idx;
        if (idx >= a.k)
            break;
        const int32_t s_in = a.sources[idx];
        if (s_in < 0 || s_in >= n) {
            // a device-side source list is checked here: report and skip
            if (tid == 0)
                atomicOr(&a.err[0], (unsigned long long)BC_ERRBIT_SOURCE);
            __syncthreads();
            continue;
        }
        const int32_t s = a.iperm ? a.iperm[s_in] : s_in;
        // With per-slab partial sums the dependencies are added to bcp while
        // the next source's initialisation streams over the vertices (below),
        // instead of one random access per vertex in the dependency pass.
        double *bc = ATOMIC_BC ? (a.item_out ? a.item_out[idx] : a.bc_out) : nullptr;

        // Queue tags only grow; restart them long before they could wrap.
        if (C.gen > (1 << 30)) {
            for (int v = tid; v < n; v += NT)
                S.stamp[v] = 0;
            __syncthreads();
            if (tid == 0)
                C.gen = 0;
        }
        // Initialisation (Alg. 1): d = inf and sigma = 0 everywhere.
        S.base8 = 0;
        if (LB < 32) {
            constexpr int per = 32 / LB;
            for (int v = tid; v < (S.H + per - 1) / per; v += NT)
                lds_ptr(S.ld)[v] = 0xffffffffu; // every entry LDS16_INF / LDS8_INF
        } else {
            for (int v = tid; v < S.H; v += NT)
                S.ld[v] = BC_INF;
        }
        {
            // d[] of this slab is complete here (the previous source wrote its
            // LDS part back), so the previous source's reached vertices are
            // those with a finite distance: their dependencies go into the
            // partial sums and their out-degrees into the arc statistic, in
            // one coalesced pass.  After a completed source the vertices
            // without in-arcs (from g.n_act on) are untouched but for that
            // source itself, so only [0, n_act) and the source are visited;
            // the launch's first source, and one after an abort, visit all.
            const int32_t ps = C.prev_s;
            auto reset = [&](int v) {
                if (ps >= 0 && S.d[v] != BC_INF) {
                    st_arcs += g.row[v + 1] - g.row[v];
                    if (!ATOMIC_BC && v != ps)
                        S.bcp[v] += S.delta[v];
                }
                if (LB < 32 || v >= S.H)
                    S.d[v] = BC_INF;
                S.sigma[v] = 0;
                if (a.kahn)
                    S.scnt[v] = 0;
                S.infar[v] = 0; // far-pile flags and tie count start clear
                if (a.ebc == nullptr)
                    *key_ptr(S, v) = KEY_NONE; // no predecessor key yet
                if (BKT)
                    S.pred1[v] = INT32_MAX; // in no far bucket yet
            };
            const int lim = ps >= 0 ? g.n_act : n;
            for (int v = tid; v < lim; v += NT)
                reset(v);
            if (ps >= lim && tid == 0)
                reset(ps);
            for (int j = tid; j < a.nbk; j += NT)
                C.bcnt[j] = 0;
        }
        __syncthreads();
        if (tid == 0) {
            dist_set(S, s, 0);
            S.sigma[s] = 1;
            C.gen += 1;
            S.stamp[s] = C.gen;
            S.qa[0] = s;
            S.order[0] = s;
            S.band_off[0] = 0;
            C.cur = 0;
            C.fcur = 0;
            C.near_len = 1;
            C.next_cnt = 0;
            C.order_cnt = 1;
            C.far_cnt = 0;
            C.outer_cnt = 0;
            C.ocur = 0;
            C.huge_cnt = 0;
            C.band_gen = C.gen;
            C.thr = a.delta;
            C.far_min = BC_INF;
            C.outer_min = BC_INF;
            C.bound = BKT ? sat_add_u32(0u, (uint64_t)a.nbk * a.delta)
                                : sat_add_u32(a.delta, (uint64_t)OUTER_BANDS * a.delta);
            C.bcur = 0;
            C.forced = 0;
            C.band_start = 0;
            C.nbands = 0;
            C.abort = 0;
            C.iters = 0;
        }
        __syncthreads();
        phase_mark(C, tmark, 0);

        // Forward pass: near-far bands of width delta.
        for (;;) {
            while (C.near_len > 0) {
                ExpandCtx ec;
                ec.items = C.cur ? S.qb : S.qa;
                ec.len = C.near_len;
                ec.all_vertices = a.node_parallel;
                ec.cur_tag = C.gen;
                ec.vw = a.vw;
                ec.worker = tid / WAVE;
                ec.nworkers = NT / WAVE;
                ec.thr = C.thr;
                ec.tag_next = C.gen + 1;
                ec.band_gen = C.band_gen;
                ec.lane_max = a.lane_max;
                ec.next_q = C.cur ? S.qa : S.qb;
                ec.next_cnt = &C.next_cnt;
                ec.order = S.order;
                ec.order_cnt = &C.order_cnt;
                ec.far_q = C.fcur ? S.fb : S.fa;
                ec.far_cnt = &C.far_cnt;
                ec.bound = C.bound;
                ec.outer_q = C.ocur ? S.ob : S.oa;
                ec.outer_cnt = &C.outer_cnt;
                const bool hubs = a.hubs && !a.vw;
                ec.huge_q = hubs ? C.huge_q : nullptr;
                ec.huge_cnt = &C.huge_cnt;
                ec.keys = a.ebc == nullptr;
                ec.trow = g.trow;
                ec.lane_deg = a.lane_deg;
                ec.wave_deg = a.wave_deg;
                ec.wg_deg = a.wg_deg;
                ec.bk = S.fa;
                ec.bcnt = C.bcnt;
                ec.bdelta = a.delta;
                ec.nbk = a.nbk;
                ec.bcap = a.bcap;
                ec.forced = &C.forced;
                uint32_t fmin = BC_INF, omin = BC_INF;
                expand_pass<PACKED, WG_SCOPE, BKT>(g, S, ec, fmin, omin, st_imp);
                if (hubs) {
                    __syncthreads();
                    // the listed hubs, each by the whole workgroup
                    const int nh = C.huge_cnt < EXPAND_WG_CAP ? C.huge_cnt : EXPAND_WG_CAP;
                    for (int h = 0; h < nh; ++h) {
                        const int32_t v = C.huge_q[h];
                        const uint32_t hb = g.row[v], he = g.row[v + 1];
                        const uint32_t hd = dist_get(S, v);
                        for (uint32_t e = hb + tid; e < he; e += NT) {
                            uint32_t u, w;
                            arc_at<PACKED>(g.arc, g.wt, e, g.wshift, g.wmask, u, w);
                            relax<WG_SCOPE, BKT>(S, ec, u, hd + w, dist_peek(S, u), (uint32_t)v, fmin,
                                            omin, st_imp);
                        }
                    }
                }
                fmin = wave_min_u32(fmin);
                omin = wave_min_u32(omin);
                if (lane == 0 && fmin != BC_INF)
                    atomicMin(&C.far_min, fmin);
                if (lane == 0 && omin != BC_INF)
                    atomicMin(&C.outer_min, omin);
                __syncthreads();
                if (tid == 0) {
                    C.cur ^= 1;
                    C.near_len = C.next_cnt;
                    C.next_cnt = 0;
                    C.huge_cnt = 0;
                    C.gen += 1;
                    if (++C.iters > iter_cap) {
                        C.abort = 1;
                        C.near_len = 0;
                    }
                }
                __syncthreads();
            }
            phase_mark(C, tmark, 1);
            if (C.abort)
                break;
            // The band is closed: its members order[b0, b1) have final distances.
            const int b0 = C.band_start, b1 = C.order_cnt;
            if (b1 > b0) {
                const bool ok =
                    a.kahn ? wg_band_rounds<PACKED, NT, true, ATOMIC_BC, true>(
                                 g, S, C, a, s, idx, b0, b1, bc, st_arcs, st_dag)
                           : wg_band_rounds<PACKED, NT, true, ATOMIC_BC, false>(
                                 g, S, C, a, s, idx, b0, b1, bc, st_arcs, st_dag);
                if (!ok) {
                    if (tid == 0)
                        C.abort = 1;
                    __syncthreads();
                    break;
                }
            }
            phase_mark(C, tmark, 2);
            if (tid == 0) {
                if (b1 > b0) {
                    C.nbands += 1;
                    S.band_off[C.nbands] = b1;
                }
                C.band_start = b1;
            }
            __syncthreads();
            if constexpr (LB == 8) {
                // every vertex below the closed band's threshold is settled and
                // every later offered value lies above it
                if (C.thr - S.base8 > LDS8_REBASE) {
                    const uint32_t nb = C.thr;
                    lds8_rebase(S, nb, tid, NT);
                    __syncthreads();
                    S.base8 = nb;
                }
            }
            if constexpr (BKT) {
                const bool more = bucket_next_band<NT>(S, C, a, iter_cap);
                phase_mark(C, tmark, 4);
                if (!more)
                    break;
                continue;
            }
            if (C.far_cnt == 0 && C.outer_cnt == 0)
                break;
            // Next band: threshold from the least far distance seen.
            if (tid == 0) {
                C.thr_old = C.thr;
                const uint32_t fm = C.far_min < C.outer_min ? C.far_min : C.outer_min;
                const uint32_t lo = fm > C.thr ? fm : C.thr;
                C.thr = sat_add_u32(lo, (uint64_t)a.delta);
                C.far_min = BC_INF;
                C.gen += 1;
                C.band_gen = C.gen;
                C.near_len = 0;
                C.kept_cnt = 0;
                C.okept_cnt = 0;
                C.resplit = C.thr > C.bound && C.outer_cnt > 0;
                if (C.thr > C.bound) {
                    C.bound = sat_add_u32(C.thr, (uint64_t)OUTER_BANDS * a.delta);
                    if (C.resplit)
                        C.outer_min = BC_INF;
                }
                if (++C.iters > iter_cap)
                    C.abort = 1;
            }
            __syncthreads();
            if (C.abort)
                break;
            if (C.resplit) {
                // the threshold passed the bound: bring the outer pile's entries
                // below the new bound into the inner pile
                OuterSplitCtx op;
                op.outer_in = C.ocur ? S.ob : S.oa;
                op.len = C.outer_cnt;
                op.worker = tid / WAVE;
                op.nworkers = NT / WAVE;
                op.thr_old = C.thr_old;
                op.bound = C.bound;
                op.inner_q = C.fcur ? S.fb : S.fa;
                op.inner_cnt = &C.far_cnt;
                op.outer_out = C.ocur ? S.oa : S.ob;
                op.kept_cnt = &C.okept_cnt;
                uint32_t kmin = BC_INF;
                outer_split_pass(S, op, kmin);
                kmin = wave_min_u32(kmin);
                if (lane == 0 && kmin != BC_INF)
                    atomicMin(&C.outer_min, kmin);
                __syncthreads();
                if (tid == 0) {
                    C.ocur ^= 1;
                    C.outer_cnt = C.okept_cnt;
                }
                __syncthreads();
            }
            {
                SplitCtx sp;
                sp.far_in = C.fcur ? S.fb : S.fa;
                sp.len = C.far_cnt;
                sp.worker = tid / WAVE;
                sp.nworkers = NT / WAVE;
                sp.thr_old = C.thr_old;
                sp.thr = C.thr;
                sp.tag = C.gen;
                sp.near_q = C.cur ? S.qb : S.qa;
                sp.near_cnt = &C.near_len;
                sp.order = S.order;
                sp.order_cnt = &C.order_cnt;
                sp.far_out = C.fcur ? S.fa : S.fb;
                sp.kept_cnt = &C.kept_cnt;
                sp.clear_flags = 0;
                uint32_t kmin = BC_INF;
                split_pass(S, sp, kmin);
                kmin = wave_min_u32(kmin);
                if (lane == 0 && kmin != BC_INF)
                    atomicMin(&C.far_min, kmin);
            }
            __syncthreads();
            if (tid == 0) {
                C.fcur ^= 1;
                C.far_cnt = C.kept_cnt;
            }
            __syncthreads();
            phase_mark(C, tmark, 4);
        }

        // Backward pass (Alg. 3), either band by band in reverse with pulls over
        // out-arcs, or in Kahn's order over the recorded shortest-path DAG,
        // from the vertices without successors towards the source.
        if (!C.abort && !a.kahn) {
            const int nb = C.nbands;
            for (int b = nb - 1; b >= 0; --b) {
                const int b0 = S.band_off[b], b1 = S.band_off[b + 1];
                if (!wg_band_rounds<PACKED, NT, false, ATOMIC_BC, false>(
                        g, S, C, a, s, idx, b0, b1, bc, st_arcs, st_dag)) {
                    if (tid == 0)
                        C.abort = 1;
                    break;
                }
            }
        }
        // Kahn's order band by band, last band first: successor counts cover
        // only arcs inside a band, and a vertex's successors in later bands
        // are all done before its own band starts.
        if (!C.abort && a.kahn) {
            const int cap = C.order_cnt + 2;
            int steps = 0;
            for (int b = C.nbands - 1; b >= 0 && !C.abort; --b) {
                const int b0 = S.band_off[b], b1 = S.band_off[b + 1];
                if (tid == 0)
                    C.pend_cnt = 0;
                __syncthreads();
                kahn_leaves(S, S.order + b0, b1 - b0, tid / WAVE, NT / WAVE, S.qa, &C.pend_cnt);
                __syncthreads();
                int len = C.pend_cnt;
                __syncthreads();
                const int32_t *items = S.qa;
                int which = 0;
                while (len > 0) {
                    if (++steps > cap) {
                        if (tid == 0)
                            C.abort = 1;
                        __syncthreads();
                        break;
                    }
                    if (tid == 0)
                        C.pend_cnt = 0;
                    __syncthreads();
                    KahnCtx kc;
                    kc.items = items;
                    kc.len = len;
                    kc.worker = tid / WAVE;
                    kc.nworkers = NT / WAVE;
                    kc.lane_max = a.lane_max;
                    kc.s = s;
                    kc.next_q = which ? S.qa : S.qb;
                    kc.next_cnt = &C.pend_cnt;
                    kc.perm = ATOMIC_BC ? a.perm : nullptr;
                    kc.ebc = a.ebc;
                    kc.emap = a.emap;
                    kahn_step<PACKED, WG_SCOPE, ATOMIC_BC>(g, S, kc, bc);
                    __syncthreads();
                    len = C.pend_cnt;
                    __syncthreads();
                    items = which ? S.qa : S.qb;
                    which ^= 1;
                    if (tid == 0)
                        C.drounds++;
                }
            }
        }
        phase_mark(C, tmark, 3);
        // The LDS-resident distances go back to the slab so that the slab
        // holds the complete per-source state.
        if (S.w8) {
            for (int v = tid; v < S.H; v += NT) {
                const uint32_t e = lds8_ptr(S.ld)[v];
                if (e - 1u < LDS8_WIN)
                    S.d[v] = S.base8 + e - 1u; // else d[v] already holds it (or BC_INF)
            }
        } else if (S.w16) {
            for (int v = tid; v < S.H; v += NT) {
                const uint32_t x = lds16_ptr(S.ld)[v];
                if (x < LDS16_FAR)
                    S.d[v] = x; // else d[v] already holds it (or BC_INF)
            }
        } else {
            for (int v = tid; v < S.H; v += NT)
                S.d[v] = S.ld[v];
        }
        __syncthreads();
        if (C.abort) {
            // Leave the slab reusable and report; the result is not valid.
            for (int v = tid; v < n; v += NT)
                S.infar[v] = 0;
            if (tid == 0)
                atomicOr(&a.err[0], (unsigned long long)BC_ERRBIT_INTERNAL);
        }
        if (tid == 0) {
            atomicAdd(&a.stats->reached, (unsigned long long)C.order_cnt);
            atomicAdd(&a.stats->bands, (unsigned long long)C.nbands);
            atomicAdd(&a.stats->iterations, C.iters);
            C.prev_s = C.abort ? -1 : s;
        }
        __syncthreads();
    }
    // the last source's dependencies and arc statistic (it reached no vertex
    // without in-arcs but itself)
    if (C.prev_s >= 0) {
        const int32_t ps = C.prev_s;
        for (int v = tid; v < g.n_act; v += NT)
            if (S.d[v] != BC_INF) {
                st_arcs += g.row[v + 1] - g.row[v];
                if (!ATOMIC_BC && v != ps)
                    S.bcp[v] += S.delta[v];
            }
        if (ps >= g.n_act && tid == 0)
            st_arcs += g.row[ps + 1] - g.row[ps];
    }

    // Flush per-lane statistics: one atomic per wave.
    {
        unsigned long long x;
        x = st_arcs;
        for (int o = 32; o > 0; o >>= 1)
            x += __shfl_xor(x, o);
        if (lane == 0)
            atomicAdd(&a.stats->arcs, x);
        x = st_dag;
        for (int o = 32; o > 0; o >>= 1)
            x += __shfl_xor(x, o);
        if (lane == 0)
            atomicAdd(&a.stats->dag, x);
        x = st_imp;
        for (int o = 32; o > 0; o >>= 1)
            x += __shfl_xor(x, o);
        if (lane == 0)
            atomicAdd(&a.stats->improvements, x);
    }
    if (tid == 0) {
        S.hdr[0] = C.gen;
        atomicAdd(&a.stats->sigma_rounds, (unsigned long long)C.srounds);
        atomicAdd(&a.stats->delta_rounds, (unsigned long long)C.drounds);
        for (int i = 0; i < 5; ++i)
            atomicAdd(&a.stats->ticks[i], C.ticks[i]);
    }
}

// Sum of the per-slab partial centralities, slab after slab.
// Sums the slabs' partial centralities into out.  Blocks along y take slab
// groups of per_group slabs each (so that a small graph with many slabs still
// fills the GPU); with more than one group they add into out, which the
// launcher has zeroed, else each vertex's sum is stored.
__global__ void k_reduce_partials(char *slab_base, SlabLayout L, int nslabs, int n, double *out,
                                  const int32_t *perm, int per_group)
{
    const int b0 = (int)blockIdx.y * per_group;
    const int b1 = b0 + per_group < nslabs ? b0 + per_group : nslabs;
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        double acc = 0.0;
        for (int b = b0; b < b1; ++b)
            acc += ((const double *)(slab_base + (size_t)b * L.stride + L.bcp))[v];
        const int o = perm ? perm[v] : v;
        if (gridDim.y == 1)
            out[o] = acc;
        else
            unsafeAtomicAdd(&out[o], acc);
    }
}

// ---------------------------------------------------------------------------
// Plain form
// ---------------------------------------------------------------------------
enum { PH_EXPAND = 0, PH_SIGMA = 1, PH_SPLIT = 2, PH_DELTA = 3, PH_DONE = 4 };

__device__ void plain_start_delta(PlainCtl *c, const Slab &S)
{
    c->dband = c->nbands - 1;
    if (c->dband < 0) {
        c->phase = PH_DONE;
        return;
    }
    c->b0 = S.band_off[c->dband];
    c->b1 = S.band_off[c->dband + 1];
    c->round = 0;
    c->pend_cnt = 0;
    c->phase = PH_DELTA;
}

// A band is finished (its counts are final): record it, then either start
// the backward pass or open the next band by splitting the far pile.
__device__ void plain_end_band(PlainCtl *c, const Slab &S, uint32_t delta)
{
    if (c->b1 > c->b0) {
        c->nbands += 1;
        S.band_off[c->nbands] = c->b1;
    }
    c->band_start = c->b1;
    if (c->far_cnt == 0) {
        plain_start_delta(c, S);
        return;
    }
    c->thr_old = c->thr;
    const uint32_t lo = c->far_min > c->thr ? c->far_min : c->thr;
    const uint64_t t = (uint64_t)lo + delta;
    c->thr = t > BC_INF ? BC_INF : (uint32_t)t;
    c->far_min = BC_INF;
    c->gen += 1;
    c->band_gen = c->gen;
    c->near_len = 0;
    c->kept_cnt = 0;
    c->iters += 1;
    c->phase = PH_SPLIT;
}

__global__ void k_plain_init(PlainArgs a)
{
    Slab S = slab_at(a.slab_base, a.L, 0);
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < a.g.n; v += gridDim.x * blockDim.x) {
        S.d[v] = BC_INF;
        S.sigma[v] = 0;
    }
}

__global__ void k_plain_setup(PlainArgs a, int32_t s, long long idx, double *bc_out)
{
    Slab S = slab_at(a.slab_base, a.L, 0);
    PlainCtl *c = a.ctl;
    S.d[s] = 0;
    S.sigma[s] = 1;
    c->gen += 1;
    S.stamp[s] = c->gen;
    S.qa[0] = s;
    S.order[0] = s;
    S.band_off[0] = 0;
    c->s = s;
    c->src_idx = idx;
    c->bc_out = bc_out;
    c->cur = 0;
    c->fcur = 0;
    c->pcur = 0;
    c->near_len = 1;
    c->next_cnt = 0;
    c->order_cnt = 1;
    c->far_cnt = 0;
    c->kept_cnt = 0;
    c->pend_cnt = 0;
    c->pend_len = 0;
    c->band_gen = c->gen;
    c->thr = a.delta;
    c->thr_old = 0;
    c->far_min = BC_INF;
    c->band_start = 0;
    c->nbands = 0;
    c->round = 0;
    c->b0 = c->b1 = 0;
    c->iters = 0;
    c->abort = 0;
    c->finished = 0;
    c->srounds = 0;
    c->drounds = 0;
    c->phase = PH_EXPAND;
}

// Restarts the queue tags (they only grow) long before they could wrap.
__global__ void k_plain_clear_stamps(PlainArgs a)
{
    Slab S = slab_at(a.slab_base, a.L, 0);
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < a.g.n; v += gridDim.x * blockDim.x)
        S.stamp[v] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0)
        a.ctl->gen = 0;
}

template <bool PACKED>
__global__ __launch_bounds__(256) void k_plain_step(PlainArgs a)
{
    PlainCtl *c = a.ctl;
    const int phase = c->phase;
    if (phase == PH_DONE)
        return;
    const DevGraph &g = a.g;
    Slab S = slab_at(a.slab_base, a.L, 0);
    const int worker = (int)((blockIdx.x * blockDim.x + threadIdx.x) / WAVE);
    const int nworkers = (int)(gridDim.x * blockDim.x / WAVE);
    const int lane = lane_id();
    if (phase == PH_EXPAND) {
        ExpandCtx ec;
        ec.items = c->cur ? S.qb : S.qa;
        ec.len = c->near_len;
        ec.all_vertices = 0;
        ec.cur_tag = c->gen;
        ec.vw = a.vw;
        ec.worker = worker;
        ec.nworkers = nworkers;
        ec.thr = c->thr;
        ec.tag_next = c->gen + 1;
        ec.band_gen = c->band_gen;
        ec.lane_max = a.lane_max;
        ec.next_q = c->cur ? S.qa : S.qb;
        ec.next_cnt = &c->next_cnt;
        ec.order = S.order;
        ec.order_cnt = &c->order_cnt;
        ec.far_q = c->fcur ? S.fb : S.fa;
        ec.far_cnt = &c->far_cnt;
        ec.bound = BC_INF; // one far pile: the whole grid scans it per band
        ec.bk = nullptr;
        ec.outer_q = nullptr;
        ec.outer_cnt = nullptr;
        ec.huge_q = nullptr; // a hub is one wave's work here (the grid is the team)
        ec.huge_cnt = nullptr;
        ec.keys = 0;
        ec.trow = nullptr;
        ec.lane_deg = a.lane_deg;
        ec.wave_deg = a.wave_deg;
        ec.wg_deg = BC_INF;
        uint32_t fmin = BC_INF, omin = BC_INF;
        uint64_t imp = 0;
        expand_pass<PACKED, AG_SCOPE>(g, S, ec, fmin, omin, imp);
        fmin = wave_min_u32(fmin);
        unsigned long long x = imp;
        for (int o = 32; o > 0; o >>= 1)
            x += __shfl_xor(x, o);
        if (lane == 0) {
            if (fmin != BC_INF)
                atomicMin(&c->far_min, fmin);
            if (x)
                atomicAdd(&a.stats->improvements, x);
        }
    } else if (phase == PH_SPLIT) {
        SplitCtx sp;
        sp.far_in = c->fcur ? S.fb : S.fa;
        sp.len = c->far_cnt;
        sp.worker = worker;
        sp.nworkers = nworkers;
        sp.thr_old = c->thr_old;
        sp.thr = c->thr;
        sp.tag = c->gen;
        sp.near_q = c->cur ? S.qb : S.qa;
        sp.near_cnt = &c->near_len;
        sp.order = S.order;
        sp.order_cnt = &c->order_cnt;
        sp.far_out = c->fcur ? S.fa : S.fb;
        sp.kept_cnt = &c->kept_cnt;
        sp.clear_flags = 1;
        uint32_t kmin = BC_INF;
        split_pass(S, sp, kmin);
        kmin = wave_min_u32(kmin);
        if (lane == 0 && kmin != BC_INF)
            atomicMin(&c->far_min, kmin);
    } else {
        RoundCtx rc;
        const bool first = c->round == 0;
        rc.items = first ? S.order + c->b0 : (c->pcur ? S.qb : S.qa);
        rc.len = first ? c->b1 - c->b0 : c->pend_len;
        rc.worker = worker;
        rc.nworkers = nworkers;
        rc.lane_max = a.lane_max;
        rc.s = c->s;
        rc.src_idx = c->src_idx;
        rc.first_round = first;
        rc.pend_q = first ? S.qa : (c->pcur ? S.qa : S.qb);
        rc.pend_cnt = &c->pend_cnt;
        rc.err = a.err;
        rc.item_err = nullptr;
        rc.perm = a.perm;
        rc.keys = 0; // the plain form records no predecessor keys
        rc.count_arcs = 1;
        rc.band_gen = 0;
        rc.wave_deg = a.wave_deg;
        if (phase == PH_SIGMA) {
            uint64_t arcs = 0, dag = 0;
            sigma_round<PACKED, AG_SCOPE, false>(g, S, rc, arcs, dag);
            unsigned long long x = arcs, y = dag;
            for (int o = 32; o > 0; o >>= 1) {
                x += __shfl_xor(x, o);
                y += __shfl_xor(y, o);
            }
            if (lane == 0) {
                if (x)
                    atomicAdd(&a.stats->arcs, x);
                if (y)
                    atomicAdd(&a.stats->dag, y);
            }
        } else {
            delta_round<PACKED, AG_SCOPE, false>(g, S, rc, c->bc_out);
        }
    }
}

__global__ void k_plain_control(PlainArgs a)
{
    PlainCtl *c = a.ctl;
    Slab S = slab_at(a.slab_base, a.L, 0);
    switch (c->phase) {
    case PH_EXPAND:
        c->cur ^= 1;
        c->near_len = c->next_cnt;
        c->next_cnt = 0;
        c->gen += 1;
        c->iters += 1;
        if (c->near_len == 0) {
            c->b0 = c->band_start;
            c->b1 = c->order_cnt;
            c->round = 0;
            c->pend_cnt = 0;
            if (c->b1 > c->b0)
                c->phase = PH_SIGMA;
            else
                plain_end_band(c, S, a.delta);
        }
        break;
    case PH_SIGMA:
        c->srounds += 1;
        if (c->pend_cnt > 0) {
            c->pcur = c->round == 0 ? 0 : c->pcur ^ 1;
            c->pend_len = c->pend_cnt;
            c->pend_cnt = 0;
            c->round += 1;
            if (c->round > c->b1 - c->b0 + 2)
                c->abort = 1;
        } else {
            plain_end_band(c, S, a.delta);
        }
        break;
    case PH_SPLIT:
        c->fcur ^= 1;
        c->far_cnt = c->kept_cnt;
        c->kept_cnt = 0;
        if (c->near_len > 0) {
            c->phase = PH_EXPAND;
        } else {
            c->b0 = c->b1 = c->band_start;
            plain_end_band(c, S, a.delta);
        }
        break;
    case PH_DELTA:
        c->drounds += 1;
        if (c->pend_cnt > 0) {
            c->pcur = c->round == 0 ? 0 : c->pcur ^ 1;
            c->pend_len = c->pend_cnt;
            c->pend_cnt = 0;
            c->round += 1;
            if (c->round > c->b1 - c->b0 + 2)
                c->abort = 1;
        } else {
            c->dband -= 1;
            if (c->dband < 0) {
                c->phase = PH_DONE;
            } else {
                c->b0 = S.band_off[c->dband];
                c->b1 = S.band_off[c->dband + 1];
                c->round = 0;
                c->pend_cnt = 0;
            }
        }
        break;
    default:
        break;
    }
    if (c->phase != PH_DONE && (c->abort || c->iters > c->iter_cap)) {
        c->abort = 1;
        c->phase = PH_DONE;
    }
    if (c->phase == PH_DONE && !c->finished) {
        c->finished = 1;
        if (c->abort) {
            atomicOr(&a.err[0], (unsigned long long)BC_ERRBIT_INTERNAL);
        }
        a.stats->reached += (unsigned long long)c->order_cnt;
        a.stats->bands += (unsigned long long)c->nbands;
        a.stats->iterations += c->iters;
        a.stats->sigma_rounds += c->srounds;
        a.stats->delta_rounds += c->drounds;
    }
}

__global__ void k_plain_clear_infar(PlainArgs a)
{
    Slab S = slab_at(a.slab_base, a.L, 0);
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < a.g.n; v += gridDim.x * blockDim.x)
        S.infar[v] = 0;
}

// ---------------------------------------------------------------------------
// Utilities
// ---------------------------------------------------------------------------
__global__ void k_fill_u32(uint32_t *p, size_t count, uint32_t value)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = value;
}

// One past the last vertex with an in-arc (0 if none): *out starts at 0.
__global__ void k_inarc_bound(const uint32_t *trow, int32_t n, int *out)
{
    int last = 0;
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x)
        if (trow[v + 1] > trow[v])
            last = v + 1;
    for (int o = 32; o > 0; o >>= 1) {
        const int y = __shfl_xor(last, o);
        last = y > last ? y : last;
    }
    if (lane_id() == 0 && last > 0)
        atomicMax(out, last);
}

__global__ void k_fill_u64(unsigned long long *p, size_t count, unsigned long long value)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = value;
}

// Clears the persistent parts of every slab (queue tags, far flags, header).
__global__ void k_slab_reset(char *slab_base, SlabLayout L, int nslabs, int n)
{
    const int slot = blockIdx.y;
    if (slot >= nslabs)
        return;
    Slab S = slab_at(slab_base, L, slot);
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        S.stamp[v] = 0;
        S.infar[v] = 0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0)
        S.hdr[0] = 0;
}

// Copies one slab's per-source state out, with unreached vertices shown as
// (INT32_MAX, 0, 0).
__global__ void k_export_state(char *slab_base, SlabLayout L, int slot, int n, int32_t *d,
                               uint64_t *sigma, double *delta, const int32_t *perm)
{
    Slab S = slab_at(slab_base, L, slot);
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        const uint32_t dv = S.d[v];
        const bool r = dv != BC_INF;
        const int32_t o = perm ? perm[v] : v;
        d[o] = (int32_t)dv;
        if (sigma)
            sigma[o] = r ? S.sigma[v] : 0ull;
        if (delta)
            delta[o] = r ? S.delta[v] : 0.0;
    }
}

// Dynamic update of one arc tail -> head, weight w_old -> w_new (0: absent).
// With a = dist(s, tail) and b = dist(s, head) before the change, the arc is
// in the shortest-path DAG of s before iff a + w_old = b, and it lies on, or
// shortens, a shortest path after iff a + w_new <= b.  When neither holds the
// old distances stay exact after the change and the set of tight arcs (the
// DAG, hence the counts and dependencies of s) is the same.
__device__ __forceinline__ bool arc_changes_dag(uint32_t a, uint32_t b, int32_t w_old,
                                                int32_t w_new)
{
    if (a == BC_INF)
        return false; // the tail is not reached from s
    const uint64_t ta = a;
    if (w_old > 0 && b != BC_INF && ta + (uint32_t)w_old == b)
        return true;
    return w_new > 0 && (b == BC_INF || ta + (uint32_t)w_new <= b);
}

// Sources whose DAG the change alters; dt[s] = dist(s, tail), dh[s] =
// dist(s, head) in the caller's numbering (INT32_MAX: unreachable).  `both`:
// the reverse arc head -> tail changes too (undirected graphs).
__global__ void k_dynamic_affected(const int32_t *dt, const int32_t *dh, int n, int32_t w_old,
                                   int32_t w_new, int both, int32_t *list, int *cnt)
{
    const long long stride = (long long)gridDim.x * blockDim.x;
    // every lane of a wave runs the same number of iterations (wave_alloc is a
    // wave-wide operation)
    const long long span = ((long long)n + stride - 1) / stride * stride;
    for (long long s = blockIdx.x * blockDim.x + threadIdx.x; s < span; s += stride) {
        bool hit = false;
        if (s < n) {
            const uint32_t a = (uint32_t)dt[s], b = (uint32_t)dh[s];
            hit = arc_changes_dag(a, b, w_old, w_new) ||
                  (both && arc_changes_dag(b, a, w_old, w_new));
        }
        const int k = wave_alloc(cnt, hit);
        if (hit)
            list[k] = (int32_t)s;
    }
}

// list[i] = i (every vertex as a source)
__global__ void k_iota(int32_t *list, int n)
{
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x)
        list[v] = v;
}

// bc += after - before, the affected sources' dependencies on the new graph
// replacing those on the old one.
__global__ void k_dynamic_apply(double *bc, const double *before, const double *after, int n)
{
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x)
        bc[v] += after[v] - before[v];
}

// ---------------------------------------------------------------------------
// Host-side launchers
// ---------------------------------------------------------------------------
size_t batched_lds_bytes(int H, int lb)
{
    const int per = 32 / lb;
    return (size_t)((H + per - 1) / per) * 4;
}

template <bool PACKED, int NT, bool ATOMIC, int LB, bool BKT>
static void launch_batched_t(const BatchArgs &a, int nslabs, hipStream_t st)
{
    const size_t lds = batched_lds_bytes(a.H, LB);
    if (lds > 48 * 1024)
        (void)hipFuncSetAttribute((const void *)k_batched<PACKED, NT, ATOMIC, LB, BKT>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL((k_batched<PACKED, NT, ATOMIC, LB, BKT>), dim3(nslabs), dim3(NT), lds, st,
                       a);
}

// Every instantiation of the batched kernel: (packed arcs, threads, atomic
// output, LDS distance width, far-bucket ring).  The ring and the 8-bit
// distances are built for packed-arc graphs only; the others keep the
// two-tier far pile and 16- or 32-bit distances.
#define BC_FOR_EACH_BATCHED(X)                                                                  \
    X(true, 256, false, 32, false) X(true, 256, true, 32, false)                               \
    X(true, 512, false, 32, false) X(true, 512, true, 32, false)                               \
    X(true, 1024, false, 32, false) X(true, 1024, true, 32, false)                             \
    X(false, 256, false, 32, false) X(false, 256, true, 32, false)                             \
    X(false, 512, false, 32, false) X(false, 512, true, 32, false)                             \
    X(false, 1024, false, 32, false) X(false, 1024, true, 32, false)                           \
    X(true, 256, false, 16, false) X(true, 256, true, 16, false)                               \
    X(true, 512, false, 16, false) X(true, 512, true, 16, false)                               \
    X(true, 1024, false, 16, false) X(true, 1024, true, 16, false)                             \
    X(false, 256, false, 16, false) X(false, 256, true, 16, false)                             \
    X(false, 512, false, 16, false) X(false, 512, true, 16, false)                             \
    X(false, 1024, false, 16, false) X(false, 1024, true, 16, false)                           \
    X(true, 256, false, 8, false) X(true, 256, true, 8, false)                                 \
    X(true, 512, false, 8, false) X(true, 512, true, 8, false)                                 \
    X(true, 1024, false, 8, false) X(true, 1024, true, 8, false)                               \
    X(true, 256, false, 32, true) X(true, 256, true, 32, true)                                 \
    X(true, 256, false, 16, true) X(true, 256, true, 16, true)                                 \
    X(true, 256, false, 8, true) X(true, 256, true, 8, true)                                   \
    X(true, 512, false, 32, true) X(true, 512, true, 32, true)                                 \
    X(true, 512, false, 16, true) X(true, 512, true, 16, true)                                 \
    X(true, 512, false, 8, true) X(true, 512, true, 8, true)                                   \
    X(true, 1024, false, 32, true) X(true, 1024, true, 32, true)                               \
    X(true, 1024, false, 16, true) X(true, 1024, true, 16, true)                               \
    X(true, 1024, false, 8, true) X(true, 1024, true, 8, true)

hipError_t launch_batched(const BatchArgs &a, bool packed, int nt, bool atomic_bc, int nslabs,
                          hipStream_t st)
{
    const int lb = a.lds_bits;
    const bool bkt = a.buckets != 0;
#define BC_CASE(P, T, A, W, B)                                                                  \
    if (packed == P && nt == T && atomic_bc == A && lb == W && bkt == B) {                      \
        launch_batched_t<P, T, A, W, B>(a, nslabs, st);                                         \
        return hipGetLastError();                                                               \
    }
    BC_FOR_EACH_BATCHED(BC_CASE)
#undef BC_CASE
    return hipErrorInvalidValue;
}

int batched_blocks_per_cu(bool packed, int nt, bool atomic_bc, int lb)
{
    return batched_blocks_per_cu_lds(packed, nt, atomic_bc, lb, 0);
}

int batched_blocks_per_cu_lds(bool packed, int nt, bool atomic_bc, int lb, size_t lds_bytes)
{
    int blocks = 0;
    hipError_t e = hipErrorInvalidValue;
#define BC_OCC(P, T, A, W, B)                                                                   \
    if (packed == P && nt == T && atomic_bc == A && lb == W && !B) {                            \
        if (lds_bytes > 48 * 1024)                                                              \
            (void)hipFuncSetAttribute((const void *)k_batched<P, T, A, W, B>,                   \
                                      hipFuncAttributeMaxDynamicSharedMemorySize,               \
                                      (int)lds_bytes);                                          \
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_batched<P, T, A, W, B>, T,  \
                                                         lds_bytes);                            \
    }
    BC_FOR_EACH_BATCHED(BC_OCC)
#undef BC_OCC
    if (e != hipSuccess || blocks < 1) {
        (void)hipGetLastError();
        return 1;
    }
    return blocks;
}

hipError_t launch_reduce_partials(char *slab_base, const SlabLayout &L, int nslabs, int n,
                                  double *out, const int32_t *perm, hipStream_t st)
{
    int blocks = (n + 255) / 256;
    if (blocks > 4096)
        blocks = 4096;
    if (blocks < 1)
        blocks = 1;
    // about 1024 blocks in all: slab groups when the vertices alone give fewer
    int groups = 1;
    if (blocks < 1024 && nslabs > 1)
        groups = std::min(nslabs, (1024 + blocks - 1) / blocks);
    const int per_group = (nslabs + groups - 1) / std::max(groups, 1);
    groups = per_group > 0 ? (nslabs + per_group - 1) / per_group : 1;
    if (groups > 1) {
        const hipError_t e = launch_fill_u64((unsigned long long *)out, (size_t)n, 0ull, st);
        if (e != hipSuccess)
            return e;
    }
    hipLaunchKernelGGL(k_reduce_partials, dim3(blocks, std::max(groups, 1)), dim3(256), 0, st,
                       slab_base, L, nslabs, n, out, perm, std::max(per_group, 1));
    return hipGetLastError();
}

hipError_t launch_plain_source(const PlainArgs &a, bool packed, int grid, int32_t s,
                               long long idx, bool clear_stamps, double *bc_out, hipStream_t st)
{
    int fb = (a.g.n + 255) / 256;
    if (fb > 2048)
        fb = 2048;
    if (fb < 1)
        fb = 1;
    if (clear_stamps)
        hipLaunchKernelGGL(k_plain_clear_stamps, dim3(fb), dim3(256), 0, st, a);
    hipLaunchKernelGGL(k_plain_init, dim3(fb), dim3(256), 0, st, a);
    hipLaunchKernelGGL(k_plain_setup, dim3(1), dim3(1), 0, st, a, s, idx, bc_out);
    (void)packed;
    (void)grid;
    return hipGetLastError();
}

hipError_t launch_plain_steps(const PlainArgs &a, bool packed, int grid, int pairs,
                              hipStream_t st)
{
    for (int i = 0; i < pairs; ++i) {
        if (packed)
            hipLaunchKernelGGL(k_plain_step<true>, dim3(grid), dim3(256), 0, st, a);
        else
            hipLaunchKernelGGL(k_plain_step<false>, dim3(grid), dim3(256), 0, st, a);
        hipLaunchKernelGGL(k_plain_control, dim3(1), dim3(1), 0, st, a);
    }
    return hipGetLastError();
}

hipError_t launch_plain_clear_infar(const PlainArgs &a, hipStream_t st)
{
    int fb = (a.g.n + 255) / 256;
    if (fb > 2048)
        fb = 2048;
    if (fb < 1)
        fb = 1;
    hipLaunchKernelGGL(k_plain_clear_infar, dim3(fb), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *p, size_t count, uint32_t value, hipStream_t st)
{
    if (count == 0)
        return hipSuccess;
    size_t blocks = (count + 255) / 256;
    if (blocks > 4096)
        blocks = 4096;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, st, p, count, value);
    return hipGetLastError();
}

hipError_t launch_inarc_bound(const uint32_t *trow, int32_t n, int *out, hipStream_t st)
{
    hipError_t e = launch_fill_u32((uint32_t *)out, 1, 0u, st);
    if (e != hipSuccess || n <= 0)
        return e;
    int blocks = (n + 255) / 256;
    if (blocks > 4096)
        blocks = 4096;
    hipLaunchKernelGGL(k_inarc_bound, dim3(blocks), dim3(256), 0, st, trow, n, out);
    return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long *p, size_t count, unsigned long long value,
                           hipStream_t st)
{
    if (count == 0)
        return hipSuccess;
    size_t blocks = (count + 255) / 256;
    if (blocks > 4096)
        blocks = 4096;
    hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)blocks), dim3(256), 0, st, p, count, value);
    return hipGetLastError();
}

hipError_t launch_slab_reset(char *slab_base, const SlabLayout &L, int nslabs, int n,
                             hipStream_t st)
{
    int bx = (n + 255) / 256;
    if (bx > 256)
        bx = 256;
    if (bx < 1)
        bx = 1;
    hipLaunchKernelGGL(k_slab_reset, dim3(bx, nslabs), dim3(256), 0, st, slab_base, L, nslabs, n);
    return hipGetLastError();
}

hipError_t launch_export_state(char *slab_base, const SlabLayout &L, int slot, int n, int32_t *d,
                               uint64_t *sigma, double *delta, const int32_t *perm,
                               hipStream_t st)
{
    int blocks = (n + 255) / 256;
    if (blocks > 4096)
        blocks = 4096;
    if (blocks < 1)
        blocks = 1;
    hipLaunchKernelGGL(k_export_state, dim3(blocks), dim3(256), 0, st, slab_base, L, slot, n, d,
                       sigma, delta, perm);
    return hipGetLastError();
}

static int flat_blocks(int n)
{
    int blocks = (n + 255) / 256;
    return blocks > 4096 ? 4096 : blocks < 1 ? 1 : blocks;
}

hipError_t launch_dynamic_affected(const int32_t *dt, const int32_t *dh, int n, int32_t w_old,
                                   int32_t w_new, int both, int32_t *list, int *cnt,
                                   hipStream_t st)
{
    hipLaunchKernelGGL(k_dynamic_affected, dim3(flat_blocks(n)), dim3(256), 0, st, dt, dh, n,
                       w_old, w_new, both, list, cnt);
    return hipGetLastError();
}

hipError_t launch_dynamic_apply(double *bc, const double *before, const double *after, int n,
                                hipStream_t st)
{
    hipLaunchKernelGGL(k_dynamic_apply, dim3(flat_blocks(n)), dim3(256), 0, st, bc, before,
                       after, n);
    return hipGetLastError();
}

hipError_t launch_iota(int32_t *list, int n, hipStream_t st)
{
    hipLaunchKernelGGL(k_iota, dim3(flat_blocks(n)), dim3(256), 0, st, list, n);
    return hipGetLastError();
}
