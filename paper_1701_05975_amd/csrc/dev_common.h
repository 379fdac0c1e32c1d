// dev_common.h -- device-side building blocks shared by the batched and the
// plain forms of the betweenness kernels (gfx950, 64-lane wavefronts).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "shared_types.h"

template <bool PACKED>
__device__ __forceinline__ void arc_at(const uint32_t *arc, const int32_t *wt, uint32_t e,
                                       uint32_t wshift, uint32_t wmask, uint32_t &head,
                                       uint32_t &w)
{
    uint32_t a = arc[e];
    if constexpr (PACKED) {
        head = a >> wshift;
        w = (a & wmask) + 1u;
    } else {
        head = a;
        w = (uint32_t)wt[e];
    }
}

// One field of the per-vertex records, indexed like an array.
template <typename T, int OFF>
struct VField {
    char *rec;
    __device__ __forceinline__ T &operator[](int64_t v) const
    {
        return *reinterpret_cast<T *>(rec + v * VREC_BYTES + OFF);
    }
};

struct Slab {
    uint32_t *d;       // tentative / final distance, BC_INF = unreached
    VField<int32_t, VREC_STAMP> stamp;
    VField<int32_t, VREC_INFAR> infar;
    VField<int32_t, VREC_SCNT> scnt;
    VField<int32_t, VREC_PRED1> pred1;
    VField<uint64_t, VREC_SIGMA> sigma;
    VField<double, VREC_DELTA> delta;
    double *bcp;       // per-slab partial centrality (batched form)
    int32_t *order;    // members of each band, band after band
    int32_t *qa, *qb;  // near queues / pending lists
    int32_t *fa, *fb;  // inner far piles (distance below the pile bound)
    int32_t *oa, *ob;  // outer far piles (distance at or above the pile bound)
    int32_t *band_off; // band b = order[band_off[b] .. band_off[b+1])
    int64_t *hdr;      // [0] = last queue tag used by this slab
    uint32_t *ld;      // distances of vertices 0 .. H-1 kept in LDS (batched form)
    int32_t H;         // number of LDS-resident distances (0 = none)
    int32_t w16;       // LDS entries are 16-bit; LDS16_FAR = look in d[]
    int32_t w8;        // LDS entries are 8-bit, relative to base8 (see LDS8_WIN)
    uint32_t base8;    // 8-bit entries: the window's base (a band threshold)
    int32_t *preds;    // in-row positions of v's DAG in-arcs, at preds[trow[v] ...],
                       // ended by -1 when fewer than the in-degree
};

__device__ __forceinline__ Slab slab_at(char *base, const SlabLayout &L, int slot)
{
    char *p = base + (size_t)slot * L.stride;
    Slab s;
    s.d = (uint32_t *)(p + L.d);
    s.stamp.rec = s.infar.rec = s.scnt.rec = s.pred1.rec = s.sigma.rec = s.delta.rec = p + L.rec;
    s.bcp = (double *)(p + L.bcp);
    s.order = (int32_t *)(p + L.order);
    s.qa = (int32_t *)(p + L.qa);
    s.qb = (int32_t *)(p + L.qb);
    s.fa = (int32_t *)(p + L.fa);
    s.fb = (int32_t *)(p + L.fb);
    s.oa = (int32_t *)(p + L.oa);
    s.ob = (int32_t *)(p + L.ob);
    s.band_off = (int32_t *)(p + L.band_off);
    s.hdr = (int64_t *)(p + L.hdr);
    s.ld = nullptr;
    s.H = 0;
    s.w16 = 0;
    s.w8 = 0;
    s.base8 = 0;
    s.preds = (int32_t *)(p + L.preds);
    return s;
}

// Distances: vertices below S.H (the highest in-degree ones after relabelling)
// live in LDS, the rest in the slab in HBM.  The LDS side goes through an
// explicit local-address-space pointer so that it compiles to ds_* accesses.
typedef __attribute__((address_space(3))) uint32_t lds_u32;

__device__ __forceinline__ lds_u32 *lds_ptr(uint32_t *p) { return (lds_u32 *)p; }

// With 16-bit entries LDS16_INF marks an unreached resident vertex, and a
// resident vertex whose distance does not fit below LDS16_FAR holds
// LDS16_FAR in LDS and its distance in d[]; d[] of a resident vertex only
// ever holds such values (or BC_INF).
#define LDS16_INF 0xffffu
#define LDS16_FAR 0xfffeu
typedef __attribute__((address_space(3))) uint16_t lds_u16;

__device__ __forceinline__ lds_u16 *lds16_ptr(uint32_t *p) { return (lds_u16 *)p; }

// With 8-bit entries (four per word) a resident vertex's entry is relative
// to base8, which follows the bands: e in [1, LDS8_WIN] is the distance
// base8 + e - 1; 0 is a vertex settled below base8, whose distance is in d[];
// LDS8_FAR is a distance that did not fit the window when it was set, kept in
// d[]; LDS8_INF is unreached.  base8 only moves between bands, to a closed
// band's threshold (every value offered later lies above it): entries below
// the new base are written to d[] and become 0, the others are re-based.
#define LDS8_INF 0xffu
#define LDS8_FAR 0xfeu
#define LDS8_WIN 253u
#define LDS8_REBASE 64u // re-base once the band threshold is this far above base8
typedef __attribute__((address_space(3))) uint8_t lds_u8;

__device__ __forceinline__ lds_u8 *lds8_ptr(uint32_t *p) { return (lds_u8 *)p; }

__device__ __forceinline__ uint32_t dist_get(const Slab &S, uint32_t u)
{
    uint32_t r;
    if ((int32_t)u < S.H) {
        if (S.w8) {
            const uint32_t e = lds8_ptr(S.ld)[u];
            if (e - 1u < LDS8_WIN)
                r = S.base8 + e - 1u;
            else if (e == LDS8_INF)
                r = BC_INF;
            else
                r = S.d[u]; // settled below the base, or kept in d[]
        } else if (S.w16) {
            r = lds16_ptr(S.ld)[u];
            if (r == LDS16_INF)
                r = BC_INF;
            else if (r == LDS16_FAR)
                r = S.d[u];
        } else {
            r = lds_ptr(S.ld)[u];
        }
    } else {
        r = S.d[u];
    }
    return r;
}

// dist_get for the pre-check of a relaxation: a vertex settled below the
// 8-bit base can take no offered value (each lies above the base), so 0
// stands in for its distance there without a read of d[].
__device__ __forceinline__ uint32_t dist_peek(const Slab &S, uint32_t u)
{
    if (S.w8 && (int32_t)u < S.H) {
        const uint32_t e = lds8_ptr(S.ld)[u];
        if (e - 1u < LDS8_WIN)
            return S.base8 + e - 1u;
        if (e == 0u)
            return 0u;
        return e == LDS8_INF ? BC_INF : S.d[u];
    }
    return dist_get(S, u);
}

// Single-thread store of a distance (no concurrent access to the entry's word).
__device__ __forceinline__ void dist_set(const Slab &S, uint32_t u, uint32_t v)
{
    if ((int32_t)u < S.H) {
        if (S.w8) {
            uint32_t e;
            if (v == BC_INF) {
                e = LDS8_INF;
            } else if (v < S.base8) {
                e = 0u;
                S.d[u] = v;
            } else if (v - S.base8 + 1u <= LDS8_WIN) {
                e = v - S.base8 + 1u;
            } else {
                e = LDS8_FAR;
                S.d[u] = v;
            }
            lds8_ptr(S.ld)[u] = (uint8_t)e;
        } else if (S.w16) {
            lds16_ptr(S.ld)[u] =
                (uint16_t)(v < LDS16_FAR ? v : v == BC_INF ? LDS16_INF : LDS16_FAR);
            if (v >= LDS16_FAR)
                S.d[u] = v;
        } else {
            lds_ptr(S.ld)[u] = v;
        }
    } else {
        S.d[u] = v;
    }
}

// ---------------------------------------------------------------------------
// Wave helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

__device__ __forceinline__ uint32_t lanes_below(uint64_t mask)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Wave-aggregated slot allocation on a counter (LDS or global): every active
// lane with `pred` gets a distinct index; one atomic per wave.
__device__ __forceinline__ int wave_alloc(int *counter, bool pred)
{
    uint64_t mask = __ballot(pred);
    if (mask == 0)
        return -1;
    int leader = __ffsll((unsigned long long)mask) - 1;
    int base = 0;
    if (lane_id() == leader)
        base = atomicAdd(counter, __popcll(mask));
    base = __shfl(base, leader);
    return pred ? base + (int)lanes_below(mask) : -1;
}

__device__ __forceinline__ uint32_t wave_min_u32(uint32_t x)
{
    for (int o = 32; o > 0; o >>= 1) {
        uint32_t y = __shfl_xor(x, o);
        x = y < x ? y : x;
    }
    return x;
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t x)
{
    for (int o = 32; o > 0; o >>= 1)
        x += __shfl_xor(x, o);
    return x;
}

// Sum of unsigned 64-bit values across the wave with wrap detection.
__device__ __forceinline__ uint64_t wave_sum_u64_checked(uint64_t x, bool &ovf)
{
    bool o = ovf;
    for (int k = 32; k > 0; k >>= 1) {
        uint64_t y = __shfl_xor(x, k);
        uint64_t t = x + y;
        o |= t < x;
        x = t;
    }
    ovf = __ballot(o) != 0;
    return x;
}

__device__ __forceinline__ double wave_sum_f64(double x)
{
    for (int k = 32; k > 0; k >>= 1)
        x += __shfl_xor(x, k);
    return x;
}

