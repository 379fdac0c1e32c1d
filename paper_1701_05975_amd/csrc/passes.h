// passes.h -- the per-source steps of weighted Brandes, written as wave-level
// routines over a list of vertices.  The batched form calls them with the
// waves of one workgroup and counters in LDS; the plain form with every wave
// of the grid and counters in global memory.
//
// Mapping of vertices to lanes (the warp-centric idea of Sec. 3.4 recast for
// 64-lane wavefronts), by degree: a low-degree vertex is handled by one lane,
// which walks its arcs in order; a medium one by a group of EXPAND_GROUP
// lanes; a large one by the whole wave, the 64 lanes striding over its arcs
// together (and in the batched expansion a hub by the whole workgroup).  Only
// queued vertices get lanes (the work-efficient queue of Sec. 3.3); a fixed
// group width and a scan over every vertex (node-parallel) are selectable for
// comparison.
#pragma once

#include "dev_common.h"

template <int SCOPE>
__device__ __forceinline__ uint32_t atomic_min_u32(uint32_t *p, uint32_t v)
{
    return __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, SCOPE);
}

template <int SCOPE>
__device__ __forceinline__ uint32_t dist_min(const Slab &S, uint32_t u, uint32_t v)
{
    if ((int32_t)u < S.H) {
        if (S.w8) {
            // 8-bit entry (see LDS8_WIN): compare-and-swap its word.  v lies
            // above the base (it is offered from the band being expanded), so
            // an entry of 0 (settled below the base) is already smaller.
            // Entries only move down (unreached, then kept in d[] or a value
            // in the window, then smaller values), so the loop ends.
            lds_u32 *wp = lds_ptr(S.ld) + (u >> 2);
            const uint32_t sh = (u & 3u) * 8u;
            const uint32_t fit = v - S.base8 + 1u; // window code of v, if at most LDS8_WIN
            uint32_t cur = *wp;
            for (;;) {
                const uint32_t h = (cur >> sh) & 0xffu;
                if (h - 1u < LDS8_WIN && S.base8 + h - 1u <= v)
                    return S.base8 + h - 1u; // already at most v
                if (h == 0u)
                    return 0u;
                if (fit > LDS8_WIN && h == LDS8_FAR) // kept in d[]
                    return atomic_min_u32<SCOPE>(&S.d[u], v);
                // h is unreached, kept in d[] while v fits, or a larger value
                const uint32_t e = fit <= LDS8_WIN ? fit : LDS8_FAR;
                const uint32_t nw = (cur & ~(0xffu << sh)) | (e << sh);
                uint32_t expect = cur;
                if (__hip_atomic_compare_exchange_strong(wp, &expect, nw, __ATOMIC_RELAXED,
                                                         __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_WORKGROUP)) {
                    if (e == LDS8_FAR) // first value that does not fit (h was unreached)
                        return atomic_min_u32<SCOPE>(&S.d[u], v);
                    return h - 1u < LDS8_WIN ? S.base8 + h - 1u : BC_INF; // d[u] was larger
                }
                cur = expect;
            }
        }
        if (!S.w16)
            return __hip_atomic_fetch_min(lds_ptr(S.ld) + u, v, __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_WORKGROUP);
        // 16-bit entry: LDS has no 16-bit minimum, so compare-and-swap the
        // 32-bit word holding it.  Entries only move down (unreached, then
        // kept in d[], then a value below LDS16_FAR, then smaller values), and
        // each failed swap saw another lane move one of the word's two
        // entries, so the loop ends.
        lds_u32 *wp = lds_ptr(S.ld) + (u >> 1);
        const uint32_t sh = (u & 1u) * 16u;
        uint32_t cur = *wp;
        for (;;) {
            const uint32_t h = (cur >> sh) & 0xffffu;
            if (h < LDS16_FAR && h <= v)
                return h; // already at most v
            if (v >= LDS16_FAR && h == LDS16_FAR) // kept in d[]
                return atomic_min_u32<SCOPE>(&S.d[u], v);
            // h is unreached, or kept in d[] while v fits, or a larger value
            const uint32_t e = v < LDS16_FAR ? v : LDS16_FAR;
            const uint32_t nw = (cur & ~(0xffffu << sh)) | (e << sh);
            uint32_t expect = cur;
            if (__hip_atomic_compare_exchange_strong(wp, &expect, nw, __ATOMIC_RELAXED,
                                                     __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_WORKGROUP)) {
                if (e == LDS16_FAR) // first value that does not fit (h was unreached)
                    return atomic_min_u32<SCOPE>(&S.d[u], v);
                return h < LDS16_FAR ? h : BC_INF; // d[u] held at least LDS16_FAR
            }
            cur = expect;
        }
    }
    return atomic_min_u32<SCOPE>(&S.d[u], v);
}

template <int SCOPE>
__device__ __forceinline__ int atomic_xchg_i32(int32_t *p, int32_t v)
{
    return __hip_atomic_exchange(p, v, __ATOMIC_RELAXED, SCOPE);
}

template <int SCOPE>
__device__ __forceinline__ int atomic_or_i32(int32_t *p, int32_t v)
{
    return __hip_atomic_fetch_or(p, v, __ATOMIC_RELAXED, SCOPE);
}

template <int SCOPE>
__device__ __forceinline__ uint64_t load_u64(const uint64_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, SCOPE);
}

template <int SCOPE>
__device__ __forceinline__ void store_u64(uint64_t *p, uint64_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, SCOPE);
}

template <int SCOPE>
__device__ __forceinline__ double load_f64(const double *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, SCOPE);
}

template <int SCOPE>
__device__ __forceinline__ void store_f64(double *p, double v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, SCOPE);
}

// ---------------------------------------------------------------------------
// Forward pass, frontier expansion (Alg. 2 relaxation step over the queue of
// Alg. 5; near-far banding instead of the Eq. 4 settle rule).
//
// Every arc (v, u, w) of a queued vertex v proposes d[v] + w for u; atomicMin
// keeps the least.  A lane that lowered d[u] below the band threshold puts u
// in the next near queue (once per queue, by tag) and, the first time in this
// band, in the band's member list; a lower value at or above the threshold
// sends u to the far pile (once, by flag): the inner pile below the pile
// bound, else the outer pile, which is only scanned when the threshold
// passes the bound.
// ---------------------------------------------------------------------------
struct ExpandCtx {
    const int32_t *items;
    int len;
    int all_vertices;     // node-parallel: scan every vertex, expand those queued now
    int32_t cur_tag;      // tag of the queue being expanded (node-parallel filter)
    int vw;               // 0: lane or wave by degree; else a fixed group of vw lanes
    int worker, nworkers; // wave index and wave count over the item list
    uint32_t thr;         // band threshold: d < thr is near
    int32_t tag_next;     // tag of the queue being filled
    int32_t band_gen;     // tag of the band's first queue
    int lane_max;
    int32_t *next_q;
    int *next_cnt;
    int32_t *order;
    int *order_cnt;
    int32_t *far_q;
    int *far_cnt;
    uint32_t bound;       // far values at or above go to the outer pile (BC_INF: none)
    int32_t *outer_q;
    int *outer_cnt;
    int32_t *huge_q;      // optional: vertices with more than EXPAND_WG_DEG arcs are listed
    int *huge_cnt;        // here for the whole workgroup to expand after the pass
    int keys;             // record each vertex's (distance, predecessor) key and ties
    const uint32_t *trow; // with keys: in-row offsets, whose slices hold the tie entries
    uint32_t lane_deg;    // adaptive mapping: at most this many arcs -> one lane,
    uint32_t wave_deg;    // at most this many -> a group of EXPAND_GROUP lanes, more -> a wave,
    uint32_t wg_deg;      // more than this (batched, huge_q set) -> the whole workgroup
    // Far-bucket ring (batched form, relax<.., true>; else the two-tier pile above).  A far
    // value below `bound` goes to bucket value / bdelta, slot bucket % nbk,
    // when that bucket is lower than any the vertex was put in before (its
    // record's pred1 word holds the least so far); a full bucket sends the
    // vertex to the outer pile and sets *forced, so that the pile is scanned
    // at the next band change.
    int32_t *bk;
    int *bcnt;
    uint32_t bdelta;
    int nbk, bcap;
    int *forced;
};

// Predecessor keys (batched form).  While distances are being found, the
// dependency field of a vertex (unused until its count is taken) holds the
// least (distance << 32 | tail) over the improvements it received, and the
// bits from TIE_SHIFT up in its far-flags word count the relaxations that
// matched its distance at the time (ties).  A relaxation that offers v its
// final distance comes from a tight arc whose tail is at its own final
// distance (one from a larger tail distance offers more), and it always
// leaves an event: exactly one of them lowers d[v] to that value, and is the
// key, each other one is a tie.  Ties at a larger distance belong to values
// that were improved on later.  So the key's tail and the tails of the ties
// at the key's distance name every shortest-path predecessor, each once per
// tight arc and per expansion of its tail at that distance: a tail improved
// while it is being expanded can be expanded again at the same distance.
//
// The first TIE_MAX ties of a vertex are kept as (distance, tail) pairs in
// its own slice of preds[] (two words each, as far as the slice holds them),
// which the count pass reads until it writes the vertex's DAG list there.  A
// vertex whose ties were all kept and whose predecessor tails are all
// distinct takes its count and its DAG list from the key and those pairs
// without reading its in-arcs; the list then names tails rather than in-row
// positions, and VFLAG_TLIST in the far-flags word says so.  A vertex with
// more ties, or with a tail seen twice (a second expansion, or parallel tight
// arcs: the pairs cannot tell these apart), scans its in-arcs.
#define VFLAG_TLIST 4
#define VFLAG_SCAN 8 // the count pass found a repeated tail: v scans in every round
#define TIE_SHIFT 4
#define TIE_MAX 7
#define KEY_NONE (~0ull)

__device__ __forceinline__ uint64_t *key_ptr(const Slab &S, int32_t v)
{
    return reinterpret_cast<uint64_t *>(&S.delta[v]);
}

// Arcs handled per step by a lane that walks its own row: their heads and
// the heads' distances are loaded together, so several independent loads per
// lane are in flight instead of one dependent chain per arc.
#ifndef LANE_UNROLL
#define LANE_UNROLL 2
#endif

// Adaptive expansion (Sec. 3.4's degree-aware mapping, three tiers): a vertex
// with at most lane_deg arcs is walked by one lane, one with at most wave_deg
// by a group of EXPAND_GROUP lanes, a larger one by the wave.  The thresholds
// are run-time values (BC_DEF_LANE_DEG and BC_DEF_WAVE_DEG by default); the
// group width is fixed.
#ifndef EXPAND_GROUP
#define EXPAND_GROUP 16
#endif
// Fourth tier (batched form): a vertex with more than wg_deg arcs (default
// BC_HUB_DEG) is expanded by every thread of the workgroup after the pass, so
// that one hub does not keep one wave busy while the others wait at the
// barrier.  The list holds EXPAND_WG_CAP vertices; further ones take the wave
// path.
#define EXPAND_WG_CAP 256

template <int SCOPE, bool BKT = false>
__device__ __forceinline__ void relax(const Slab &S, const ExpandCtx &c, uint32_t u, uint32_t nd,
                                      uint32_t du, uint32_t tail, uint32_t &far_min,
                                      uint32_t &outer_min, uint64_t &nimp)
{
    bool imp = false, tie = nd == du;
    if (nd < du) {
        uint32_t old = dist_min<SCOPE>(S, u, nd);
        imp = nd < old;
        tie = nd == old;
    }
    if (c.keys) {
        if (imp)
            __hip_atomic_fetch_min(key_ptr(S, (int32_t)u), (uint64_t)nd << 32 | tail,
                                   __ATOMIC_RELAXED, SCOPE);
        // counting stops past TIE_MAX (beyond it a vertex scans anyway), so
        // the count stays below TIE_MAX + 2 + the threads of the workgroup
        if (tie && ((uint32_t)__hip_atomic_load(&S.infar[u], __ATOMIC_RELAXED, SCOPE) >>
                    TIE_SHIFT) <= TIE_MAX) {
            const uint32_t t = (uint32_t)__hip_atomic_fetch_add(&S.infar[u], 1 << TIE_SHIFT,
                                                                __ATOMIC_RELAXED, SCOPE) >>
                               TIE_SHIFT;
            if (t < TIE_MAX) {
                const uint32_t tb = c.trow[u], te = c.trow[u + 1];
                if (tb + 2 * (t + 1) <= te) {
                    S.preds[tb + 2 * t] = (int32_t)nd;
                    S.preds[tb + 2 * t + 1] = (int32_t)tail;
                }
            }
        }
    }
    bool pn = false, pm = false, pf = false, po = false;
    int bslot = -1; // far-bucket ring: the slot u goes to
    if (imp) {
        ++nimp;
        if (nd < c.thr) {
            int32_t ot = atomic_xchg_i32<SCOPE>(&S.stamp[u], c.tag_next);
            pn = ot != c.tag_next;
            pm = ot < c.band_gen;
        } else if (nd < c.bound) {
            if (BKT) {
                const uint32_t b = nd / c.bdelta;
                if (BUCKET_KEY(b) <
                    __hip_atomic_fetch_min(&S.pred1[u], BUCKET_KEY(b), __ATOMIC_RELAXED, SCOPE))
                    bslot = (int)(b % (uint32_t)c.nbk);
            } else {
                far_min = nd < far_min ? nd : far_min;
                pf = (atomic_or_i32<SCOPE>(&S.infar[u], 1) & 1) == 0;
            }
        } else {
            outer_min = nd < outer_min ? nd : outer_min;
            po = (atomic_or_i32<SCOPE>(&S.infar[u], 2) & 2) == 0;
        }
    }
    if (BKT && __ballot(bslot >= 0)) {
        if (bslot >= 0) {
            const int k = atomicAdd(&c.bcnt[bslot], 1);
            if (k < c.bcap) {
                c.bk[(size_t)bslot * (size_t)c.bcap + (size_t)k] = (int32_t)u;
            } else { // a full bucket: the outer pile keeps u until the next band change
                *c.forced = 1;
                outer_min = nd < outer_min ? nd : outer_min;
                po = (atomic_or_i32<SCOPE>(&S.infar[u], 2) & 2) == 0;
            }
        }
    }
    if (__ballot(imp)) {
        int k = wave_alloc(c.next_cnt, pn);
        if (pn)
            c.next_q[k] = (int32_t)u;
        k = wave_alloc(c.order_cnt, pm);
        if (pm)
            c.order[k] = (int32_t)u;
        k = wave_alloc(c.far_cnt, pf);
        if (pf)
            c.far_q[k] = (int32_t)u;
        if (__ballot(po)) {
            k = wave_alloc(c.outer_cnt, po);
            if (po)
                c.outer_q[k] = (int32_t)u;
        }
    }
}

// Fixed virtual-warp mapping (Sec. 3.4): a group of vw lanes per vertex,
// striding over its arcs; vw = 1 is one thread per vertex, vw = 64 one wave.
template <bool PACKED, int SCOPE, bool BKT = false>
__device__ __forceinline__ void expand_pass_vw(const DevGraph &g, const Slab &S, const ExpandCtx &c,
                               uint32_t &far_min, uint32_t &outer_min, uint64_t &nimp)
{
    const int W = c.vw;
    const int groups = WAVE / W;
    const int lane = lane_id(), grp = lane / W, sub = lane % W;
    const int len = c.all_vertices ? g.n : c.len;
    for (int base = c.worker * groups; base < len; base += c.nworkers * groups) {
        const int i = base + grp;
        bool valid = i < len;
        int v = 0;
        if (valid) {
            v = c.all_vertices ? i : c.items[i];
            if (c.all_vertices)
                valid = S.stamp[v] == c.cur_tag;
        }
        uint32_t beg = 0, end = 0, dv = BC_INF;
        if (valid) {
            beg = g.row[v];
            end = g.row[v + 1];
            dv = dist_get(S, v);
        }
        for (uint32_t e = beg + sub; e < end; e += W) {
            uint32_t u, w;
            arc_at<PACKED>(g.arc, g.wt, e, g.wshift, g.wmask, u, w);
            relax<SCOPE, BKT>(S, c, u, dv + w, dist_peek(S, u), (uint32_t)v, far_min, outer_min, nimp);
        }
    }
}

template <bool PACKED, int SCOPE, bool BKT = false>
__device__ __forceinline__ void expand_pass(const DevGraph &g, const Slab &S, const ExpandCtx &c,
                            uint32_t &far_min, uint32_t &outer_min, uint64_t &nimp)
{
    if (c.vw > 0) {
        expand_pass_vw<PACKED, SCOPE, BKT>(g, S, c, far_min, outer_min, nimp);
        return;
    }
    const int lane = lane_id();
    const int len = c.all_vertices ? g.n : c.len;
    for (int base = c.worker * WAVE; base < len; base += c.nworkers * WAVE) {
        const int i = base + lane;
        bool valid = i < len;
        uint32_t beg = 0, end = 0, dv = BC_INF;
        int v = 0;
        if (valid) {
            v = c.all_vertices ? i : c.items[i];
            if (c.all_vertices)
                valid = S.stamp[v] == c.cur_tag;
            if (valid) {
                beg = g.row[v];
                end = g.row[v + 1];
                dv = dist_get(S, v);
            }
        }
        const uint32_t deg = end - beg;
        const bool light = valid && deg <= c.lane_deg;
        const bool mid = valid && deg > c.lane_deg && deg <= c.wave_deg;
        bool heavy = valid && deg > c.wave_deg;
        if (c.huge_q) {
            const bool huge = heavy && deg > c.wg_deg;
            const int k = wave_alloc(c.huge_cnt, huge);
            if (huge && k < EXPAND_WG_CAP) {
                c.huge_q[k] = v;
                heavy = false;
            }
        }
        if (light) {
            for (uint32_t e0 = beg; e0 < end; e0 += LANE_UNROLL) {
                uint32_t u[LANE_UNROLL], w[LANE_UNROLL], du[LANE_UNROLL];
#pragma unroll
                for (int j = 0; j < LANE_UNROLL; ++j) {
                    u[j] = 0;
                    w[j] = 0;
                    if (e0 + j < end)
                        arc_at<PACKED>(g.arc, g.wt, e0 + j, g.wshift, g.wmask, u[j], w[j]);
                }
#pragma unroll
                for (int j = 0; j < LANE_UNROLL; ++j)
                    du[j] = e0 + j < end ? dist_peek(S, u[j]) : 0u;
#pragma unroll
                for (int j = 0; j < LANE_UNROLL; ++j)
                    if (e0 + j < end)
                        relax<SCOPE, BKT>(S, c, u[j], dv + w[j], du[j], (uint32_t)v, far_min, outer_min,
                                     nimp);
            }
        }
        // Medium degree: up to WAVE / EXPAND_GROUP vertices at a time, one per
        // group of lanes.  The shuffles run on every lane: a lane whose group
        // has no vertex may be the source another group reads from.
        uint64_t mm = __ballot(mid);
        const int grp = lane / EXPAND_GROUP, sub = lane % EXPAND_GROUP;
        while (mm) {
            uint64_t t = mm;
            for (int k = 0; k < grp; ++k)
                t &= t - 1;
            const bool have = t != 0;
            const int l = have ? __ffsll((unsigned long long)t) - 1 : 0;
            for (int k = 0; k < WAVE / EXPAND_GROUP; ++k)
                mm &= mm - 1;
            const uint32_t mb = (uint32_t)__shfl((int)beg, l);
            const uint32_t me0 = (uint32_t)__shfl((int)end, l);
            const uint32_t md = (uint32_t)__shfl((int)dv, l);
            const uint32_t mv = (uint32_t)__shfl(v, l);
            const uint32_t me = have ? me0 : mb;
            constexpr int G = EXPAND_GROUP;
            for (uint32_t e0 = mb + sub; e0 < me; e0 += G * 2) {
                uint32_t u[2], w[2], du[2];
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    u[j] = 0;
                    w[j] = 0;
                    if (e0 + G * j < me)
                        arc_at<PACKED>(g.arc, g.wt, e0 + G * j, g.wshift, g.wmask, u[j], w[j]);
                }
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    du[j] = e0 + G * j < me ? dist_peek(S, u[j]) : 0u;
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    if (e0 + G * j < me)
                        relax<SCOPE, BKT>(S, c, u[j], md + w[j], du[j], mv, far_min, outer_min, nimp);
            }
        }
        uint64_t hm = __ballot(heavy);
        while (hm) {
            const int l = __ffsll((unsigned long long)hm) - 1;
            hm &= hm - 1;
            const uint32_t hb = (uint32_t)__shfl((int)beg, l);
            const uint32_t he = (uint32_t)__shfl((int)end, l);
            const uint32_t hd = (uint32_t)__shfl((int)dv, l);
            const uint32_t hv = (uint32_t)__shfl(v, l);
            for (uint32_t e = hb + lane; e < he; e += WAVE) {
                uint32_t u, w;
                arc_at<PACKED>(g.arc, g.wt, e, g.wshift, g.wmask, u, w);
                relax<SCOPE, BKT>(S, c, u, hd + w, dist_peek(S, u), hv, far_min, outer_min, nimp);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Far pile split at a band change.  Entries whose distance dropped below the
// previous threshold were settled through the near queue already (dropped);
// entries below the new threshold move to the near queue and become members
// of the new band; the rest stay in the far pile.
// ---------------------------------------------------------------------------
struct SplitCtx {
    const int32_t *far_in;
    int len;
    int worker, nworkers;
    uint32_t thr_old, thr;
    int32_t tag;
    int32_t *near_q;
    int *near_cnt;
    int32_t *order;
    int *order_cnt;
    int32_t *far_out;
    int *kept_cnt;
    int clear_flags; // clear the pile flag of entries leaving the pile (else the
                     // caller clears every flag before the next source: a vertex
                     // that left the pile never returns to it, as its distance
                     // is now below the threshold and only decreases)
};

__device__ __forceinline__ void split_pass(const Slab &S, const SplitCtx &c, uint32_t &kept_min)
{
    const int lane = lane_id();
    for (int base = c.worker * WAVE; base < c.len; base += c.nworkers * WAVE) {
        const int i = base + lane;
        const bool valid = i < c.len;
        int32_t v = 0;
        uint32_t dv = 0;
        if (valid) {
            v = c.far_in[i];
            dv = dist_get(S, v);
        }
        const bool drop = valid && dv < c.thr_old;
        const bool move = valid && !drop && dv < c.thr;
        const bool keep = valid && !drop && !move;
        if (c.clear_flags && (drop || move))
            S.infar[v] &= ~1; // each vertex sits at most once in a pile
        if (move)
            S.stamp[v] = c.tag;
        if (keep)
            kept_min = dv < kept_min ? dv : kept_min;
        int k = wave_alloc(c.near_cnt, move);
        if (move)
            c.near_q[k] = v;
        k = wave_alloc(c.order_cnt, move);
        if (move)
            c.order[k] = v;
        k = wave_alloc(c.kept_cnt, keep);
        if (keep)
            c.far_out[k] = v;
    }
}

// Outer pile pass, when the band threshold has passed the pile bound: entries
// already settled are dropped, entries below the new bound join the inner
// pile (unless already there), the rest stay in the outer pile.  Flags of
// entries leaving the outer pile are left set (they never return to it; the
// caller clears every flag before the next source).
struct OuterSplitCtx {
    const int32_t *outer_in;
    int len;
    int worker, nworkers;
    uint32_t thr_old, bound;
    int32_t *inner_q;
    int *inner_cnt;
    int32_t *outer_out;
    int *kept_cnt;
};

__device__ __forceinline__ void outer_split_pass(const Slab &S, const OuterSplitCtx &c,
                                                 uint32_t &kept_min)
{
    const int lane = lane_id();
    for (int base = c.worker * WAVE; base < c.len; base += c.nworkers * WAVE) {
        const int i = base + lane;
        const bool valid = i < c.len;
        int32_t v = 0;
        uint32_t dv = 0;
        int32_t f = 0;
        if (valid) {
            v = c.outer_in[i];
            dv = dist_get(S, v);
            f = S.infar[v];
        }
        const bool drop = valid && dv < c.thr_old;
        const bool move = valid && !drop && dv < c.bound;
        const bool keep = valid && !drop && !move;
        const bool join = move && !(f & 1);
        if (join)
            S.infar[v] = f | 1;
        if (keep)
            kept_min = dv < kept_min ? dv : kept_min;
        int k = wave_alloc(c.inner_cnt, join);
        if (join)
            c.inner_q[k] = v;
        k = wave_alloc(c.kept_cnt, keep);
        if (keep)
            c.outer_out[k] = v;
    }
}

// ---------------------------------------------------------------------------
// Rounds over the members of one band, for the path counts and for the
// dependencies.  A member whose inputs are not all final yet is put on the
// pending list for the next round; the member of least distance among the
// pending ones always has final inputs, so every round makes progress.
// ---------------------------------------------------------------------------
struct RoundCtx {
    const int32_t *items;
    int len;
    int worker, nworkers;
    int lane_max;
    int32_t s;          // the source
    long long src_idx;  // its index in the source list (error reports)
    bool first_round;
    int32_t *pend_q;
    int *pend_cnt;
    unsigned long long *err; // [0] error bits, [1] first overflowing source index
    unsigned int *item_err;  // optional per-source-entry overflow flags
    const int32_t *perm;     // optional: caller's vertex id of each internal vertex, used
                             // when adding into a caller-indexed output
    int keys;                // predecessor keys were recorded (count pass shortcut)
    int32_t band_gen;        // queue tag of the band's first pass: a vertex with a tag at
                             // least this is a member of the band being counted
    uint32_t wave_deg;       // more in-arcs than this: the whole wave (else a group of
                             // EXPAND_GROUP lanes above lane_max, one lane below)
    int count_arcs;          // add each member's out-degree to `arcs` in the first round
                             // (the batched form counts them in its streaming pass instead)
};

__device__ __forceinline__ void report_sigma_overflow(const RoundCtx &c)
{
    atomicOr(&c.err[0], (unsigned long long)BC_ERRBIT_SIGMA);
    atomicMin((long long *)&c.err[1], c.src_idx);
    if (c.item_err)
        c.item_err[c.src_idx] = 1u;
}

// Path counts (the counting rule of Alg. 2, evaluated by pulling): sigma[v]
// is the sum of sigma[u] over arcs (u, v, w) with d[u] + w == d[v].  With
// weights >= 1 every such u has d[u] < d[v], so it belongs to this band or
// an earlier one.
//
// With RECORD, the in-row positions of the tight in-arcs of v are also
// written to preds[trow[v] ..] (the slice of v's own in-row, so no allocation
// is needed), ended by -1 when there are fewer than the in-degree; a vertex
// with a single predecessor keeps it in its record instead.  Successor
// counts scnt are kept only for DAG arcs inside the band (a predecessor in
// the same band is stored as -(x + 2)): the dependency pass runs band by band
// in reverse, so a vertex's successors in later bands are always done before
// its own band starts.
// A recorded DAG arc (in-row position at preds[slot]) whose tail lies in the
// band being counted: count it as a successor of the tail, and mark the entry.
template <bool PACKED, int SCOPE>
__device__ __forceinline__ void count_if_same_band(const DevGraph &g, const Slab &S,
                                                   const RoundCtx &c, uint32_t slot)
{
    const int32_t pos = S.preds[slot];
    uint32_t u, w;
    arc_at<PACKED>(g.tarc, g.twt, (uint32_t)pos, g.wshift, g.wmask, u, w);
    if (S.stamp[u] >= c.band_gen) {
        S.preds[slot] = -(pos + 2);
        __hip_atomic_fetch_add(&S.scnt[u], 1, __ATOMIC_RELAXED, SCOPE);
    }
}

// A DAG list entry for tail t (tails, not in-row positions: VFLAG_TLIST):
// a tail in the band being counted is stored as -(t + 2) and gains a
// pending successor.
template <int SCOPE>
__device__ __forceinline__ int32_t tail_entry(const Slab &S, const RoundCtx &c, int32_t t)
{
    if (S.stamp[t] < c.band_gen)
        return t;
    __hip_atomic_fetch_add(&S.scnt[t], 1, __ATOMIC_RELAXED, SCOPE);
    return -(t + 2);
}

// The count of v from its key and kept ties (see key_ptr), without reading
// its in-arcs.  Returns false when v has to scan them (a tie was not kept,
// or a tail is seen twice);
// sets pend when a predecessor is not counted yet.  The key's distance is v's
// final distance: every decrease of d[v] is an improvement and the key keeps
// the least of them.
template <int SCOPE, bool RECORD>
__device__ __forceinline__ bool keyed_count(const DevGraph &g, const Slab &S, const RoundCtx &c,
                                            int32_t v, bool &pend, uint64_t &dag)
{
    const uint64_t key = load_u64<SCOPE>(key_ptr(S, v));
    const int32_t fl = S.infar[v];
    const uint32_t nt = (uint32_t)fl >> TIE_SHIFT;
    if (key == KEY_NONE || nt > TIE_MAX || (fl & VFLAG_SCAN))
        return false;
    uint32_t tb = 0, te = 0;
    if (nt > 0) {
        tb = g.trow[v];
        te = g.trow[v + 1];
        if (tb + 2 * nt > te)
            return false;
    }
    const uint32_t dk = (uint32_t)(key >> 32);
    const int32_t u0 = (int32_t)(uint32_t)key;
    // A tail seen twice: scan, in this round and in any later one (a scan
    // that has to wait for a predecessor has already written over the pairs).
    bool twice = false;
    for (uint32_t i = 0; i < nt && !twice; ++i) {
        if ((uint32_t)S.preds[tb + 2 * i] != dk)
            continue;
        const int32_t t = S.preds[tb + 2 * i + 1];
        twice = t == u0;
        for (uint32_t j = 0; j < i && !twice; ++j)
            twice = (uint32_t)S.preds[tb + 2 * j] == dk && S.preds[tb + 2 * j + 1] == t;
    }
    if (twice) {
        S.infar[v] = fl | VFLAG_SCAN;
        return false;
    }
    uint64_t acc = load_u64<SCOPE>(&S.sigma[u0]);
    bool ready = acc != 0, ovf = false;
    uint32_t m = 0; // ties at the final distance
    for (uint32_t i = 0; i < nt && ready; ++i) {
        if ((uint32_t)S.preds[tb + 2 * i] != dk)
            continue;
        const uint64_t su = load_u64<SCOPE>(&S.sigma[S.preds[tb + 2 * i + 1]]);
        if (su == 0) {
            ready = false;
        } else {
            const uint64_t x = acc + su;
            ovf |= x < acc;
            acc = x;
            ++m;
        }
    }
    if (!ready) {
        pend = true; // the pairs stay for the next round
        return true;
    }
    if (ovf) {
        report_sigma_overflow(c);
        acc = ~0ull;
    }
    store_u64<SCOPE>(&S.sigma[v], acc);
    store_f64<SCOPE>(&S.delta[v], RECORD ? 0.0 : -1.0);
    dag += 1 + m;
    if (RECORD) {
        if (m == 0) { // one predecessor: in the record, no DAG list
            const int32_t e = tail_entry<SCOPE>(S, c, u0);
            S.pred1[v] = e;
        } else {
            // The list overwrites the pairs from the front: the j-th tail goes
            // to slot j <= i + 1 after pair i (slots 2i, 2i + 1) has been read,
            // so no pair is overwritten before it is read.
            uint32_t j = 1;
            for (uint32_t i = 0; i < nt; ++i) {
                const uint32_t di = (uint32_t)S.preds[tb + 2 * i];
                const int32_t t = S.preds[tb + 2 * i + 1];
                if (di == dk)
                    S.preds[tb + j++] = tail_entry<SCOPE>(S, c, t);
            }
            S.preds[tb] = tail_entry<SCOPE>(S, c, u0);
            if (tb + j < te)
                S.preds[tb + j] = -1;
            S.pred1[v] = -1;
            S.infar[v] = fl | VFLAG_TLIST;
        }
    } else {
        S.pred1[v] = -1; // a counted vertex's far-bucket value is gone (see VREC_PRED1)
    }
    return true;
}

template <bool PACKED, int SCOPE, bool RECORD>
__device__ __forceinline__ void sigma_round(const DevGraph &g, const Slab &S, const RoundCtx &c, uint64_t &arcs,
                            uint64_t &dag)
{
    const int lane = lane_id();
    for (int base = c.worker * WAVE; base < c.len; base += c.nworkers * WAVE) {
        const int i = base + lane;
        const bool valid = i < c.len;
        int32_t v = 0;
        uint32_t beg = 0, end = 0;
        if (valid) {
            v = c.items[i];
            if (c.first_round && c.count_arcs)
                arcs += g.row[v + 1] - g.row[v];
        }
        const bool is_src = valid && v == c.s;
        bool pend = false;
        // A vertex whose predecessors are known from its key and kept ties
        // takes its count from them (see key_ptr) without reading its
        // in-arcs; the others scan their in-arcs below.
        bool keyed = false;
        if (c.keys && valid && !is_src)
            keyed = keyed_count<SCOPE, RECORD>(g, S, c, v, pend, dag);
        if (valid && !keyed) {
            beg = g.trow[v];
            end = g.trow[v + 1];
        }
        if (is_src) {
            // sigma[s] = 1 was set at initialisation; s has no DAG predecessors
            store_f64<SCOPE>(&S.delta[v], RECORD ? 0.0 : -1.0);
            S.pred1[v] = -1;
            if (RECORD && end > beg)
                S.preds[beg] = -1;
        }
        const uint32_t deg = end - beg;
        const bool heavy = valid && !is_src && !keyed && deg > c.wave_deg;
        const bool mid = valid && !is_src && !keyed && !heavy && deg > (uint32_t)c.lane_max;
        if (valid && !is_src && !keyed && !heavy && !mid) {
            const uint32_t dv = dist_get(S, v);
            uint64_t acc = 0;
            bool ready = true, ovf = false;
            uint32_t tight = 0;
            for (uint32_t e0 = beg; e0 < end && ready; e0 += LANE_UNROLL) {
                uint32_t u[LANE_UNROLL], w[LANE_UNROLL], du[LANE_UNROLL];
#pragma unroll
                for (int j = 0; j < LANE_UNROLL; ++j) {
                    u[j] = 0;
                    w[j] = 0;
                    if (e0 + j < end)
                        arc_at<PACKED>(g.tarc, g.twt, e0 + j, g.wshift, g.wmask, u[j], w[j]);
                }
#pragma unroll
                for (int j = 0; j < LANE_UNROLL; ++j)
                    du[j] = e0 + j < end ? dist_get(S, u[j]) : BC_INF;
#pragma unroll
                for (int j = 0; j < LANE_UNROLL; ++j) {
                    if (ready && e0 + j < end && du[j] + w[j] == dv) {
                        const uint64_t su = load_u64<SCOPE>(&S.sigma[u[j]]);
                        if (su == 0) {
                            ready = false;
                        } else {
                            const uint64_t t = acc + su;
                            ovf |= t < acc;
                            acc = t;
                            if (RECORD) // the in-row position identifies the DAG arc
                                S.preds[beg + tight] = (int32_t)(e0 + j);
                            ++tight;
                        }
                    }
                }
            }
            if (ready) {
                if (ovf) {
                    report_sigma_overflow(c);
                    acc = ~0ull; // stays non-zero so dependants do not wait forever
                }
                store_u64<SCOPE>(&S.sigma[v], acc);
                store_f64<SCOPE>(&S.delta[v], RECORD ? 0.0 : -1.0);
                dag += tight;
                S.pred1[v] = -1;
                if (RECORD) {
                    if (beg + tight < end)
                        S.preds[beg + tight] = -1;
                    for (uint32_t j = 0; j < tight; ++j)
                        count_if_same_band<PACKED, SCOPE>(g, S, c, beg + j);
                }
            }
            pend = !ready;
        }
        {
            const int k = wave_alloc(c.pend_cnt, pend);
            if (pend)
                c.pend_q[k] = v;
        }
        // Medium in-degree: a group of EXPAND_GROUP lanes per vertex, up to
        // WAVE / EXPAND_GROUP vertices at a time.  Shuffles and ballots run on
        // every lane; each group reads only its own bits.
        uint64_t mm = __ballot(mid);
        const int grp = lane / EXPAND_GROUP, sub = lane % EXPAND_GROUP;
        const int gshift = grp * EXPAND_GROUP;
        const uint64_t gbits = (1ull << EXPAND_GROUP) - 1;
        while (mm) {
            uint64_t t = mm;
            for (int k = 0; k < grp; ++k)
                t &= t - 1;
            const bool have = t != 0;
            const int l = have ? __ffsll((unsigned long long)t) - 1 : 0;
            for (int k = 0; k < WAVE / EXPAND_GROUP; ++k)
                mm &= mm - 1;
            const int32_t mv = __shfl(v, l);
            const uint32_t mb = (uint32_t)__shfl((int)beg, l);
            const uint32_t me0 = (uint32_t)__shfl((int)end, l);
            const uint32_t me = have ? me0 : mb;
            const uint32_t mdv = have ? dist_get(S, mv) : 0u;
            uint64_t acc = 0;
            bool ready = true, ovf = false;
            uint32_t rec = 0; // tight arcs of the group so far (uniform in the group)
            for (uint32_t e0 = mb; e0 < me; e0 += EXPAND_GROUP) {
                const uint32_t e = e0 + sub;
                bool tt = false;
                if (e < me) {
                    uint32_t u, w;
                    arc_at<PACKED>(g.tarc, g.twt, e, g.wshift, g.wmask, u, w);
                    if (dist_get(S, u) + w == mdv) {
                        const uint64_t su = load_u64<SCOPE>(&S.sigma[u]);
                        if (su == 0) {
                            ready = false;
                        } else {
                            const uint64_t x = acc + su;
                            ovf |= x < acc;
                            acc = x;
                            tt = true;
                        }
                    }
                }
                const uint64_t gm = (__ballot(tt) >> gshift) & gbits;
                if (RECORD && tt)
                    S.preds[mb + rec + __popcll(gm & ((1ull << sub) - 1))] = (int32_t)e;
                rec += (uint32_t)__popcll(gm);
                if ((__ballot(!ready) >> gshift) & gbits)
                    break;
            }
            bool gready = ready;
            for (int o = 1; o < EXPAND_GROUP; o <<= 1) {
                const uint64_t y = __shfl_xor(acc, o);
                const int oy = __shfl_xor((int)ovf, o);
                const int ry = __shfl_xor((int)gready, o);
                const uint64_t z = acc + y;
                ovf = ovf || oy || z < acc;
                acc = z;
                gready = gready && ry;
            }
            if (have && gready && sub == 0) {
                if (ovf) {
                    report_sigma_overflow(c);
                    acc = ~0ull;
                }
                store_u64<SCOPE>(&S.sigma[mv], acc);
                store_f64<SCOPE>(&S.delta[mv], RECORD ? 0.0 : -1.0);
                dag += rec;
                S.pred1[mv] = -1;
                if (RECORD && mb + rec < me)
                    S.preds[mb + rec] = -1;
            }
            if (RECORD && have && gready)
                for (uint32_t j = sub; j < rec; j += EXPAND_GROUP)
                    count_if_same_band<PACKED, SCOPE>(g, S, c, mb + j);
            const bool p = have && !gready && sub == 0;
            const int k = wave_alloc(c.pend_cnt, p);
            if (p)
                c.pend_q[k] = mv;
        }
        uint64_t hm = __ballot(heavy);
        while (hm) {
            const int l = __ffsll((unsigned long long)hm) - 1;
            hm &= hm - 1;
            const int32_t hv = __shfl(v, l);
            const uint32_t hb = (uint32_t)__shfl((int)beg, l);
            const uint32_t he = (uint32_t)__shfl((int)end, l);
            const uint32_t dv = dist_get(S, hv);
            uint64_t acc = 0;
            bool ready = true, ovf = false;
            uint32_t tight = 0;      // this lane's tight arcs
            uint32_t recorded = 0;   // tight arcs of the wave so far (uniform)
            for (uint32_t e0 = hb; e0 < he; e0 += WAVE) {
                const uint32_t e = e0 + lane;
                bool t = false;
                if (e < he) {
                    uint32_t u, w;
                    arc_at<PACKED>(g.tarc, g.twt, e, g.wshift, g.wmask, u, w);
                    if (dist_get(S, u) + w == dv) {
                        const uint64_t su = load_u64<SCOPE>(&S.sigma[u]);
                        if (su == 0) {
                            ready = false;
                        } else {
                            const uint64_t x = acc + su;
                            ovf |= x < acc;
                            acc = x;
                            ++tight;
                            t = true;
                            if (RECORD) {
                                const uint64_t tm = __ballot(true);
                                S.preds[hb + recorded + lanes_below(tm)] = (int32_t)e;
                            }
                        }
                    }
                }
                recorded += (uint32_t)__popcll(__ballot(t));
                if (__ballot(!ready))
                    break;
            }
            const bool all_ready = __ballot(!ready) == 0;
            acc = wave_sum_u64_checked(acc, ovf);
            tight = wave_sum_u32(tight);
            if (all_ready && lane == 0) {
                if (ovf) {
                    report_sigma_overflow(c);
                    acc = ~0ull;
                }
                store_u64<SCOPE>(&S.sigma[hv], acc);
                store_f64<SCOPE>(&S.delta[hv], RECORD ? 0.0 : -1.0);
                dag += tight;
                S.pred1[hv] = -1;
                if (RECORD && hb + tight < he)
                    S.preds[hb + tight] = -1;
            }
            if (RECORD && all_ready)
                for (uint32_t j = lane; j < tight; j += WAVE)
                    count_if_same_band<PACKED, SCOPE>(g, S, c, hb + j);
            const bool p = !all_ready && lane == 0;
            const int k = wave_alloc(c.pend_cnt, p);
            if (p)
                c.pend_q[k] = hv;
        }
    }
}

// Dependencies (Sec. 2.1 recursion, Alg. 3): delta[v] is the sum over arcs
// (v, u, w) with d[u] == d[v] + w of sigma[v] / sigma[u] * (1 + delta[u]);
// every such u lies in this band or a later one.  A vertex other than the
// source adds its dependency to the centrality: plainly into `bc` when the
// caller owns it for this source (ATOMIC_BC false), with an FP64 atomic add
// otherwise; not at all when `bc` is null (the caller adds the dependencies
// later, in one streaming pass).
template <bool PACKED, int SCOPE, bool ATOMIC_BC>
__device__ __forceinline__ void delta_round(const DevGraph &g, const Slab &S, const RoundCtx &c, double *bc)
{
#pragma clang fp contract(off)
    const int lane = lane_id();
    for (int base = c.worker * WAVE; base < c.len; base += c.nworkers * WAVE) {
        const int i = base + lane;
        const bool valid = i < c.len;
        int32_t v = 0;
        uint32_t beg = 0, end = 0;
        if (valid) {
            v = c.items[i];
            beg = g.row[v];
            end = g.row[v + 1];
        }
        const bool heavy = valid && (end - beg) > (uint32_t)c.lane_max;
        bool pend = false;
        if (valid && !heavy) {
            const uint32_t dv = dist_get(S, v);
            const double sv = (double)S.sigma[v];
            double acc = 0.0;
            bool ready = true;
            for (uint32_t e0 = beg; e0 < end && ready; e0 += LANE_UNROLL) {
                uint32_t u[LANE_UNROLL], w[LANE_UNROLL], du[LANE_UNROLL];
#pragma unroll
                for (int j = 0; j < LANE_UNROLL; ++j) {
                    u[j] = 0;
                    w[j] = 0;
                    if (e0 + j < end)
                        arc_at<PACKED>(g.arc, g.wt, e0 + j, g.wshift, g.wmask, u[j], w[j]);
                }
#pragma unroll
                for (int j = 0; j < LANE_UNROLL; ++j)
                    du[j] = e0 + j < end ? dist_get(S, u[j]) : BC_INF;
#pragma unroll
                for (int j = 0; j < LANE_UNROLL; ++j) {
                    if (ready && du[j] != BC_INF && du[j] == dv + w[j]) {
                        const double dl = load_f64<SCOPE>(&S.delta[u[j]]);
                        if (dl < 0.0)
                            ready = false;
                        else
                            acc += sv / (double)S.sigma[u[j]] * (1.0 + dl);
                    }
                }
            }
            if (ready) {
                store_f64<SCOPE>(&S.delta[v], acc);
                if (bc && v != c.s) {
                    const int32_t o = c.perm ? c.perm[v] : v;
                    if (ATOMIC_BC)
                        unsafeAtomicAdd(&bc[o], acc);
                    else
                        bc[o] += acc;
                }
            }
            pend = !ready;
        }
        {
            const int k = wave_alloc(c.pend_cnt, pend);
            if (pend)
                c.pend_q[k] = v;
        }
        uint64_t hm = __ballot(heavy);
        while (hm) {
            const int l = __ffsll((unsigned long long)hm) - 1;
            hm &= hm - 1;
            const int32_t hv = __shfl(v, l);
            const uint32_t hb = (uint32_t)__shfl((int)beg, l);
            const uint32_t he = (uint32_t)__shfl((int)end, l);
            const uint32_t dv = dist_get(S, hv);
            const double sv = (double)S.sigma[hv];
            double acc = 0.0;
            bool ready = true;
            for (uint32_t e = hb + lane; e < he; e += WAVE) {
                uint32_t u, w;
                arc_at<PACKED>(g.arc, g.wt, e, g.wshift, g.wmask, u, w);
                const uint32_t du = dist_get(S, u);
                if (du != BC_INF && du == dv + w) {
                    const double dl = load_f64<SCOPE>(&S.delta[u]);
                    if (dl < 0.0) {
                        ready = false;
                        break;
                    }
                    acc += sv / (double)S.sigma[u] * (1.0 + dl);
                }
            }
            const bool all_ready = __ballot(!ready) == 0;
            acc = wave_sum_f64(acc);
            if (all_ready && lane == 0) {
                store_f64<SCOPE>(&S.delta[hv], acc);
                if (bc && hv != c.s) {
                    const int32_t o = c.perm ? c.perm[hv] : hv;
                    if (ATOMIC_BC)
                        unsafeAtomicAdd(&bc[o], acc);
                    else
                        bc[o] += acc;
                }
            }
            const bool p = !all_ready && lane == 0;
            const int k = wave_alloc(c.pend_cnt, p);
            if (p)
                c.pend_q[k] = hv;
        }
    }
}

// ---------------------------------------------------------------------------
// Dependencies by pushing along the recorded shortest-path DAG (Sec. 2.1
// recursion, Alg. 3 evaluated in reverse topological order): a vertex whose
// successors have all added their terms is final; it adds its dependency to
// the centrality and pushes sigma[u] / sigma[w] * (1 + delta[w]) into every
// recorded predecessor u, whose successor count drops by one.  A predecessor
// whose count reaches zero joins the next frontier.
// ---------------------------------------------------------------------------
struct KahnCtx {
    const int32_t *items;
    int len;
    int worker, nworkers;
    int lane_max;
    int32_t s;
    int32_t *next_q;
    int *next_cnt;
    const int32_t *perm; // optional caller-indexed output
    double *ebc;         // optional edge betweenness (caller arc order)
    const uint32_t *emap; // in-row position -> caller arc index
};

template <int SCOPE>
__device__ __forceinline__ bool push_dependency(const Slab &S, int32_t u, double c)
{
    __hip_atomic_fetch_add(&S.delta[u], c, __ATOMIC_RELAXED, SCOPE);
    return __hip_atomic_fetch_sub(&S.scnt[u], 1, __ATOMIC_RELAXED, SCOPE) == 1;
}

// Adds a dependency term into u.  A predecessor in the same band also has
// its count of pending successors lowered (true when that reaches zero); one
// in an earlier band only receives the term, with nothing to wait for.
template <int SCOPE>
__device__ __forceinline__ bool push_to(const Slab &S, int32_t u, double c, bool same)
{
    if (same)
        return push_dependency<SCOPE>(S, u, c);
    __hip_atomic_fetch_add(&S.delta[u], c, __ATOMIC_RELAXED, SCOPE);
    return false;
}

// A recorded predecessor: the tail of the in-arc at in-row position pos.
template <bool PACKED>
__device__ __forceinline__ int32_t pred_vertex(const DevGraph &g, int32_t pos)
{
    uint32_t u, w;
    arc_at<PACKED>(g.tarc, g.twt, (uint32_t)pos, g.wshift, g.wmask, u, w);
    return (int32_t)u;
}

template <bool PACKED, int SCOPE, bool ATOMIC_BC>
__device__ __forceinline__ void kahn_step(const DevGraph &g, const Slab &S, const KahnCtx &c, double *bc)
{
#pragma clang fp contract(off)
    const int lane = lane_id();
    for (int base = c.worker * WAVE; base < c.len; base += c.nworkers * WAVE) {
        const int i = base + lane;
        const bool valid = i < c.len;
        int32_t w = 0, p1 = -1;
        uint32_t pb = 0, pe = 0;
        double dw = 0.0, sw = 1.0;
        if (valid) {
            w = c.items[i];
            p1 = S.pred1[w];
            dw = load_f64<SCOPE>(&S.delta[w]);
            if (bc && w != c.s) {
                const int32_t o = c.perm ? c.perm[w] : w;
                if (ATOMIC_BC)
                    unsafeAtomicAdd(&bc[o], dw);
                else
                    bc[o] += dw;
            }
        }
        // A lane walks up to lane_max recorded predecessors; the rest of a
        // longer list is finished by the whole wave.
        bool more = false;
        if (valid && p1 != -1) { // the only predecessor, kept in the record
            // sigma[w] was copied from sigma[u], so their ratio is exactly 1
            const double term = 1.0 + dw;
            const int32_t u = p1 < 0 ? -(p1 + 2) : p1;
            const bool fin = push_to<SCOPE>(S, u, term, p1 < 0);
            const int k = wave_alloc(c.next_cnt, fin);
            if (fin)
                c.next_q[k] = u;
        } else if (valid) { // the list in preds[], at w's in-row
            pb = g.trow[w];
            pe = g.trow[w + 1];
            sw = (double)S.sigma[w];
            // a list of tails (at most TIE_MAX + 1) is walked by the lane whole
            const bool tails = (S.infar[w] & VFLAG_TLIST) != 0;
            const uint32_t lim = !tails && pe - pb > (uint32_t)c.lane_max ? pb + c.lane_max : pe;
            uint32_t j = pb;
            for (; j < lim; ++j) {
                const int32_t raw = S.preds[j];
                if (raw == -1)
                    break;
                const int32_t pos = raw < 0 ? -(raw + 2) : raw;
                const int32_t u = tails ? pos : pred_vertex<PACKED>(g, pos);
                const double term = (double)S.sigma[u] / sw * (1.0 + dw);
                if (c.ebc) // the term is the source's dependency on the arc u -> w
                    unsafeAtomicAdd(&c.ebc[c.emap[pos]], term);
                const bool fin = push_to<SCOPE>(S, u, term, raw < 0);
                const int k = wave_alloc(c.next_cnt, fin);
                if (fin)
                    c.next_q[k] = u;
            }
            more = j == lim && lim < pe;
            pb = lim;
        }
        uint64_t hm = __ballot(more);
        while (hm) {
            const int l = __ffsll((unsigned long long)hm) - 1;
            hm &= hm - 1;
            const uint32_t hb = (uint32_t)__shfl((int)pb, l);
            const uint32_t he = (uint32_t)__shfl((int)pe, l);
            const double hd = __shfl(dw, l);
            const double hs = __shfl(sw, l);
            for (uint32_t e0 = hb; e0 < he; e0 += WAVE) {
                const uint32_t e = e0 + lane;
                const int32_t raw = e < he ? S.preds[e] : -1;
                const uint64_t endm = __ballot(raw == -1);
                const int stop = endm ? __ffsll((unsigned long long)endm) - 1 : WAVE;
                bool fin = false;
                int32_t u = 0;
                if (lane < stop) {
                    const int32_t pos = raw < 0 ? -(raw + 2) : raw;
                    u = pred_vertex<PACKED>(g, pos);
                    const double term = (double)S.sigma[u] / hs * (1.0 + hd);
                    if (c.ebc)
                        unsafeAtomicAdd(&c.ebc[c.emap[pos]], term);
                    fin = push_to<SCOPE>(S, u, term, raw < 0);
                }
                const int k = wave_alloc(c.next_cnt, fin);
                if (fin)
                    c.next_q[k] = u;
                if (endm)
                    break;
            }
        }
    }
}

// Members with no DAG successor left in their band start the band's dependency pass.
__device__ __forceinline__ void kahn_leaves(const Slab &S, const int32_t *order, int n_r, int worker,
                                            int nworkers, int32_t *q, int *cnt)
{
    const int lane = lane_id();
    for (int base = worker * WAVE; base < n_r; base += nworkers * WAVE) {
        const int i = base + lane;
        int32_t v = 0;
        bool leaf = false;
        if (i < n_r) {
            v = order[i];
            leaf = S.scnt[v] == 0;
        }
        const int k = wave_alloc(cnt, leaf);
        if (leaf)
            q[k] = v;
    }
}
