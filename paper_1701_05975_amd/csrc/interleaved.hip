// interleaved.hip -- source-interleaved multi-source form of Brandes' method.
//
// A group of 64 sources shares one wavefront, one lane per source.  The state
// of a group is laid out vertex-major with the 64 sources of a vertex side by
// side ([group][vertex][lane]): when a wave walks the arcs of a vertex, every
// arc is read once for all 64 sources, and the distance, count and dependency
// accesses of the wave at the arc's head are one contiguous row (256 bytes of
// distances, 512 of counts or dependencies) instead of 64 scattered lines.
//
// Per group the passes are those of the other forms (Sec. 2.1, Algs. 1-3):
//   forward  -- near-far bands of width Delta shared by the 64 sources
//               (Sec. 3.2): a vertex is queued once per round with the mask of
//               the sources whose distance at it improved below the band
//               threshold; improvements beyond it go to a far list with a
//               per-vertex mask and return when the threshold passes them;
//   counts   -- sigma in topological order of each source's shortest-path
//               DAG: every vertex counts its tight in-arcs per source, the
//               sources start, and a vertex whose count reaches zero for a
//               source has its final sigma and pushes it along its tight
//               out-arcs (Alg. 2's counting rule, in Kahn's order);
//   deps     -- the same in reverse: the count pass leaves each vertex's number
//               of tight out-arcs, the DAG's leaves start, and a final vertex
//               pushes sigma_u/sigma_w (1 + delta_w) into its tight
//               predecessors (Alg. 3);
//   BC       -- each vertex adds its dependencies over the lanes whose source
//               is another vertex (Alg. 3), in a fixed order.
// Every round is one launch over a queue of (group, vertex) entries; the host
// reads the queue lengths between launches.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "dev_common.h"
#include "interleaved.h"

namespace {

__device__ __forceinline__ unsigned long long first_lane_u64(unsigned long long x)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(x >> 32));
    return (unsigned long long)hi << 32 | lo;
}

__device__ __forceinline__ size_t cell(uint32_t e, int lane)
{
    return (size_t)e * WAVE + (size_t)lane;
}

// Appends entry e to a queue unless this round already queued it.
__device__ __forceinline__ void queue_once(const IlArgs &a, uint32_t e, uint32_t round,
                                           uint32_t *qout, unsigned int *qlen)
{
    if (atomicExch(&a.stamp[e], round) != round)
        qout[atomicAdd(qlen, 1u)] = e;
}

// Appends of one wave to a queue, staged in registers (lane k holds slot k):
// one atomic on the queue's length per 64 entries instead of one per entry,
// as every wave of the grid appends to the same queue.  Every lane of the
// wave calls push and flush with the same arguments.
struct WaveQueue {
    uint32_t *out;
    unsigned int *len;
    uint32_t slot;
    int n;
    __device__ __forceinline__ WaveQueue(uint32_t *o, unsigned int *l) : out(o), len(l), slot(0), n(0) {}
    __device__ __forceinline__ void flush(int lane)
    {
        if (n == 0)
            return;
        uint32_t base = 0;
        if (lane == 0)
            base = atomicAdd(len, (unsigned int)n);
        base = __builtin_amdgcn_readfirstlane(base);
        if (lane < n)
            out[base + lane] = slot;
        n = 0;
    }
    __device__ __forceinline__ void push(uint32_t e, int lane)
    {
        if (lane == n)
            slot = e;
        if (++n == WAVE)
            flush(lane);
    }
};

// Queues entry e (through the wave's stager) unless this round already
// queued it; lane 0 takes the stamp.
__device__ __forceinline__ void queue_once_w(const IlArgs &a, uint32_t e, uint32_t round,
                                             WaveQueue &wq, int lane)
{
    uint32_t fresh = 0;
    if (lane == 0)
        fresh = atomicExch(&a.stamp[e], round) != round ? 1u : 0u;
    if (__builtin_amdgcn_readfirstlane(fresh))
        wq.push(e, lane);
}

__device__ __forceinline__ double wave_sum_f64(double x)
{
    for (int o = 32; o > 0; o >>= 1)
        x += __shfl_xor(x, o);
    return x;
}

__device__ __forceinline__ uint32_t wave_min_u32_il(uint32_t x)
{
    for (int o = 32; o > 0; o >>= 1) {
        const uint32_t y = __shfl_xor(x, o);
        x = y < x ? y : x;
    }
    return x;
}

__global__ void k_il_init(IlArgs a)
{
    const size_t cells = (size_t)a.groups * (size_t)a.n * WAVE;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < cells; i += stride) {
        a.d[i] = BC_INF;
        a.sigma[i] = 0ull;
        a.delta[i] = 0.0;
        a.cnt[i] = 0;
    }
    const size_t entries = (size_t)a.groups * (size_t)a.n;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < entries; i += stride) {
        a.act[i] = 0ull;
        a.far[i] = 0ull;
        a.stamp[i] = 0u;
    }
}

// Lane j of the sweep takes source-list entry j (none past k): distance 0,
// one path, queued with its lane bit.
__global__ void k_il_seed(IlArgs a, const int32_t *sources, long long k, const int32_t *iperm,
                          uint32_t *qout, uint32_t round)
{
    const int lanes = a.groups * WAVE;
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < lanes; j += gridDim.x * blockDim.x) {
        int32_t s = -1;
        if (j < k) {
            const int32_t s_in = sources[j];
            if (s_in < 0 || s_in >= a.n)
                atomicOr(&a.err[0], (unsigned long long)BC_ERRBIT_SOURCE);
            else
                s = iperm ? iperm[s_in] : s_in;
        }
        a.lane_src[j] = s;
        if (s < 0)
            continue;
        const uint32_t e = (uint32_t)(j / WAVE) * (uint32_t)a.n + (uint32_t)s;
        const int lane = j % WAVE;
        a.d[cell(e, lane)] = 0u;
        a.sigma[cell(e, lane)] = 1ull;
        atomicOr(&a.act[e], 1ull << lane);
        queue_once(a, e, round, qout, &a.ctl->qlen);
    }
}

// Start of a round: each queued entry takes its lane mask (later improvements
// queue it again) and is split into work items of at most IL_CHUNK arcs, so
// that the arcs of a high-degree vertex are walked by many waves at once.
__global__ void k_il_take(IlArgs a, const uint32_t *q, uint32_t qlen, int in_arcs)
{
    const int lane = lane_id();
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    // every lane of a wave runs the same iterations (wave-wide scan below)
    const size_t span = ((size_t)qlen + stride - 1) / stride * stride;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < span; i += stride) {
        uint32_t chunks = 0;
        if (i < qlen) {
            const uint32_t e = q[i];
            const unsigned long long m = atomicExch(&a.act[e], 0ull);
            a.qm[i] = m;
            if (m) {
                const uint32_t v = e % (uint32_t)a.n;
                const uint32_t deg = in_arcs ? a.g.trow[v + 1] - a.g.trow[v]
                                             : a.g.row[v + 1] - a.g.row[v];
                chunks = (deg + IL_CHUNK - 1) / IL_CHUNK;
            }
        }
        uint32_t incl = chunks;
        for (int o = 1; o < WAVE; o <<= 1) {
            const uint32_t t = __shfl_up(incl, o);
            if (lane >= o)
                incl += t;
        }
        const uint32_t total = __shfl(incl, WAVE - 1);
        uint32_t base = 0;
        if (lane == WAVE - 1 && total)
            base = atomicAdd(&a.ctl->ilen, total);
        base = __shfl(base, WAVE - 1);
        const uint32_t first = base + incl - chunks;
        for (uint32_t c = 0; c < chunks; ++c)
            a.items[first + c] = (unsigned long long)i << 32 | c;
    }
}

// A work item: queue slot i, arcs [c * IL_CHUNK, (c + 1) * IL_CHUNK) of the row.
struct IlItem {
    uint32_t e, grp, v, base, beg, end;
    unsigned long long m;
};

__device__ __forceinline__ IlItem il_item(const IlArgs &a, const uint32_t *q,
                                          const uint32_t *rows, uint32_t t)
{
    const unsigned long long it = a.items[t];
    const uint32_t i = (uint32_t)(it >> 32), c = (uint32_t)it;
    IlItem r;
    r.e = q[i];
    r.m = a.qm[i];
    r.grp = r.e / (uint32_t)a.n;
    r.v = r.e - r.grp * (uint32_t)a.n;
    r.base = r.grp * (uint32_t)a.n;
    const uint32_t b = rows[r.v], e = rows[r.v + 1];
    r.beg = b + c * IL_CHUNK;
    r.end = e - r.beg > IL_CHUNK ? r.beg + IL_CHUNK : e;
    return r;
}

// Arcs handled together by a wave: their atomics are issued before any
// result is used, so that their round trips overlap.
#define IL_UNROLL 4

// One forward round over the work items: the lanes of the item's mask whose
// distance lies below the band threshold relax the item's arcs.
template <bool PACKED>
__global__ void k_il_relax(IlArgs a, const uint32_t *q, uint32_t *qout, uint32_t *fout,
                           uint32_t thr, uint32_t round)
{
    const int lane = lane_id();
    const uint32_t wid = (blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
    const uint32_t nw = gridDim.x * blockDim.x / WAVE;
    const DevGraph &g = a.g;
    const uint32_t ilen = a.ctl->ilen;
    WaveQueue qq(qout, &a.ctl->qlen), fq(fout, &a.ctl->flen);
    for (uint32_t t = wid; t < ilen; t += nw) {
        const IlItem it = il_item(a, q, g.row, t);
        const bool on = (it.m >> lane) & 1ull;
        const uint32_t dv = on ? a.d[cell(it.e, lane)] : BC_INF;
        const bool live = on && dv < thr;
        for (uint32_t j = it.beg; j < it.end; j += IL_UNROLL) {
            uint32_t u[IL_UNROLL], nd[IL_UNROLL], old[IL_UNROLL];
#pragma unroll
            for (int k = 0; k < IL_UNROLL; ++k) {
                uint32_t w = 0;
                u[k] = 0;
                if (j + k < it.end)
                    arc_at<PACKED>(g.arc, g.wt, j + k, g.wshift, g.wmask, u[k], w);
                nd[k] = dv + w;
                old[k] = 0;
            }
#pragma unroll
            for (int k = 0; k < IL_UNROLL; ++k)
                if (live && j + k < it.end)
                    old[k] = atomicMin(&a.d[cell(it.base + u[k], lane)], nd[k]);
#pragma unroll
            for (int k = 0; k < IL_UNROLL; ++k) {
                if (j + k >= it.end)
                    break;
                const bool imp = live && nd[k] < old[k];
                const unsigned long long bn = __ballot(imp && nd[k] < thr);
                const unsigned long long bf = __ballot(imp && nd[k] >= thr);
                const uint32_t eu = it.base + u[k];
                if (bn) {
                    if (lane == 0)
                        atomicOr(&a.act[eu], bn);
                    queue_once_w(a, eu, round, qq, lane);
                }
                if (bf) {
                    uint32_t first = 0;
                    if (lane == 0)
                        first = atomicOr(&a.far[eu], bf) == 0ull ? 1u : 0u;
                    if (__builtin_amdgcn_readfirstlane(first))
                        fq.push(eu, lane);
                }
            }
        }
    }
    qq.flush(lane);
    fq.flush(lane);
}

// Far-list pass when the band threshold moves from thr_old to thr_new: lanes
// already below thr_old are settled (dropped), lanes below thr_new join the
// next band, the others stay (with their least distance reported).
__global__ void k_il_far(IlArgs a, const uint32_t *fin, uint32_t flen, uint32_t *qout,
                         uint32_t *fout, uint32_t thr_old, uint32_t thr_new, uint32_t round)
{
    const int lane = lane_id();
    const uint32_t wid = (blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
    const uint32_t nw = gridDim.x * blockDim.x / WAVE;
    WaveQueue qq(qout, &a.ctl->qlen), fq(fout, &a.ctl->flen);
    uint32_t wmin = BC_INF;
    for (uint32_t i = wid; i < flen; i += nw) {
        const uint32_t e = fin[i];
        const unsigned long long fm = first_lane_u64(lane == 0 ? a.far[e] : 0ull);
        const bool on = (fm >> lane) & 1ull;
        const uint32_t dv = on ? a.d[cell(e, lane)] : BC_INF;
        const bool drop = on && dv < thr_old;
        const bool move = on && !drop && dv < thr_new;
        const bool keep = on && !drop && !move;
        const unsigned long long km = __ballot(keep), mv = __ballot(move);
        const uint32_t kmin = wave_min_u32_il(keep ? dv : BC_INF);
        wmin = kmin < wmin ? kmin : wmin;
        if (lane == 0)
            a.far[e] = km;
        if (mv) {
            if (lane == 0)
                atomicOr(&a.act[e], mv);
            queue_once_w(a, e, round, qq, lane);
        }
        if (km)
            fq.push(e, lane);
    }
    qq.flush(lane);
    fq.flush(lane);
    if (lane == 0 && wmin != BC_INF)
        atomicMin(&a.ctl->minkept, wmin);
}

// Tight in-arcs per (vertex, source): the number of DAG predecessors whose
// counts must arrive before the vertex's count is final.  The sources (the
// only reached vertices without one) are queued.
template <bool PACKED>
__global__ void k_il_count_in(IlArgs a, uint32_t *qout, uint32_t round)
{
    const int lane = lane_id();
    const uint32_t entries = (uint32_t)a.groups * (uint32_t)a.n;
    const uint32_t wid = (blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
    const uint32_t nw = gridDim.x * blockDim.x / WAVE;
    const DevGraph &g = a.g;
    WaveQueue qq(qout, &a.ctl->qlen);
    unsigned long long nreached = 0;
    for (uint32_t e = wid; e < entries; e += nw) {
        const uint32_t grp = e / (uint32_t)a.n, v = e - grp * (uint32_t)a.n;
        const uint32_t dv = a.d[cell(e, lane)];
        const bool reached = dv != BC_INF;
        if (__ballot(reached) == 0ull)
            continue;
        const uint32_t base = grp * (uint32_t)a.n;
        int32_t c = 0;
        const uint32_t tb = g.trow[v], te = g.trow[v + 1];
        for (uint32_t j = tb; j < te; j += IL_UNROLL) {
            uint32_t p[IL_UNROLL], w[IL_UNROLL], dp[IL_UNROLL];
#pragma unroll
            for (int k = 0; k < IL_UNROLL; ++k) {
                p[k] = 0;
                w[k] = 0;
                if (j + k < te)
                    arc_at<PACKED>(g.tarc, g.twt, j + k, g.wshift, g.wmask, p[k], w[k]);
            }
#pragma unroll
            for (int k = 0; k < IL_UNROLL; ++k)
                dp[k] = reached && j + k < te ? a.d[cell(base + p[k], lane)] : BC_INF;
#pragma unroll
            for (int k = 0; k < IL_UNROLL; ++k)
                c += (dp[k] != BC_INF && (uint64_t)dp[k] + w[k] == dv) ? 1 : 0;
        }
        a.cnt[cell(e, lane)] = c;
        const unsigned long long ready = __ballot(reached && c == 0);
        nreached += (unsigned long long)__popcll(__ballot(reached));
        if (ready) {
            if (lane == 0)
                a.act[e] = ready;
            queue_once_w(a, e, round, qq, lane);
        }
    }
    qq.flush(lane);
    if (lane == 0 && nreached)
        atomicAdd(&a.ctl->reached, nreached);
}

// One count round over the work items: vertices whose count is final for the
// lanes in their mask add it into their tight out-neighbours; a neighbour
// whose last pending predecessor this was becomes final for that lane and is
// queued.
template <bool PACKED>
__global__ void k_il_sigma(IlArgs a, const uint32_t *q, uint32_t *qout, uint32_t round)
{
    const int lane = lane_id();
    const uint32_t wid = (blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
    const uint32_t nw = gridDim.x * blockDim.x / WAVE;
    const DevGraph &g = a.g;
    const uint32_t ilen = a.ctl->ilen;
    WaveQueue qq(qout, &a.ctl->qlen);
    for (uint32_t t = wid; t < ilen; t += nw) {
        const IlItem it = il_item(a, q, g.row, t);
        const bool on = (it.m >> lane) & 1ull;
        const uint32_t dv = on ? a.d[cell(it.e, lane)] : BC_INF;
        const unsigned long long sv = on ? a.sigma[cell(it.e, lane)] : 0ull;
        bool ovf = false;
        int32_t ntight = 0;
        for (uint32_t j = it.beg; j < it.end; j += IL_UNROLL) {
            uint32_t u[IL_UNROLL], du[IL_UNROLL], w[IL_UNROLL];
            unsigned long long old[IL_UNROLL];
            int32_t left[IL_UNROLL];
            bool tight[IL_UNROLL];
#pragma unroll
            for (int k = 0; k < IL_UNROLL; ++k) {
                u[k] = 0;
                w[k] = 0;
                if (j + k < it.end)
                    arc_at<PACKED>(g.arc, g.wt, j + k, g.wshift, g.wmask, u[k], w[k]);
            }
#pragma unroll
            for (int k = 0; k < IL_UNROLL; ++k)
                du[k] = on && j + k < it.end ? a.d[cell(it.base + u[k], lane)] : BC_INF;
#pragma unroll
            for (int k = 0; k < IL_UNROLL; ++k) {
                tight[k] = du[k] != BC_INF && du[k] == (uint64_t)dv + w[k];
                ntight += tight[k] ? 1 : 0;
                old[k] = 0;
                left[k] = 0;
                if (tight[k]) {
                    old[k] = atomicAdd(&a.sigma[cell(it.base + u[k], lane)], sv);
                    left[k] = atomicSub(&a.cnt[cell(it.base + u[k], lane)], 1);
                }
            }
#pragma unroll
            for (int k = 0; k < IL_UNROLL; ++k) {
                if (j + k >= it.end)
                    break;
                ovf |= tight[k] && old[k] + sv < old[k];
                const unsigned long long br = __ballot(tight[k] && left[k] == 1);
                if (br) {
                    const uint32_t eu = it.base + u[k];
                    if (lane == 0)
                        atomicOr(&a.act[eu], br);
                    queue_once_w(a, eu, round, qq, lane);
                }
            }
        }
        // the vertex's pending count is zero now (its count is final): it
        // becomes the number of its DAG successors, for the dependency pass
        if (ntight)
            atomicAdd(&a.cnt[cell(it.e, lane)], ntight);
        if (ovf) {
            atomicOr(&a.err[0], (unsigned long long)BC_ERRBIT_SIGMA);
            atomicMin(&a.err[1],
                      (unsigned long long)(a.src_base + (long long)it.grp * WAVE + lane));
        }
    }
    qq.flush(lane);
}

// Start of the dependency pass: the count pass left, per reached (vertex,
// source), the number of its DAG successors; the reached ones without any
// (the DAG's leaves) are queued.
__global__ void k_il_leaves(IlArgs a, uint32_t *qout, uint32_t round)
{
    const int lane = lane_id();
    const uint32_t entries = (uint32_t)a.groups * (uint32_t)a.n;
    const uint32_t wid = (blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
    const uint32_t nw = gridDim.x * blockDim.x / WAVE;
    WaveQueue qq(qout, &a.ctl->qlen);
    for (uint32_t e = wid; e < entries; e += nw) {
        const bool reached = a.d[cell(e, lane)] != BC_INF;
        const unsigned long long leaves = __ballot(reached && a.cnt[cell(e, lane)] == 0);
        if (leaves) {
            if (lane == 0)
                a.act[e] = leaves;
            queue_once_w(a, e, round, qq, lane);
        }
    }
    qq.flush(lane);
}

// One dependency round over the work items (in-arcs): vertices whose
// dependency is final for the lanes in their mask push sigma_p / sigma_v
// (1 + delta_v) into each tight predecessor p; a predecessor whose last
// pending successor this was is queued.
template <bool PACKED>
__global__ void k_il_delta(IlArgs a, const uint32_t *q, uint32_t *qout, uint32_t round)
{
    const int lane = lane_id();
    const uint32_t wid = (blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
    const uint32_t nw = gridDim.x * blockDim.x / WAVE;
    const DevGraph &g = a.g;
    const uint32_t ilen = a.ctl->ilen;
    WaveQueue qq(qout, &a.ctl->qlen);
    for (uint32_t t = wid; t < ilen; t += nw) {
        const IlItem it = il_item(a, q, g.trow, t);
        const bool on = (it.m >> lane) & 1ull;
        const uint32_t dv = on ? a.d[cell(it.e, lane)] : BC_INF;
        const double sv = on ? (double)a.sigma[cell(it.e, lane)] : 1.0;
        const double f = on ? 1.0 + a.delta[cell(it.e, lane)] : 0.0;
        for (uint32_t j = it.beg; j < it.end; j += IL_UNROLL) {
            uint32_t p[IL_UNROLL], dp[IL_UNROLL], w[IL_UNROLL];
            int32_t left[IL_UNROLL];
            bool tight[IL_UNROLL];
#pragma unroll
            for (int k = 0; k < IL_UNROLL; ++k) {
                p[k] = 0;
                w[k] = 0;
                if (j + k < it.end)
                    arc_at<PACKED>(g.tarc, g.twt, j + k, g.wshift, g.wmask, p[k], w[k]);
            }
#pragma unroll
            for (int k = 0; k < IL_UNROLL; ++k)
                dp[k] = on && j + k < it.end ? a.d[cell(it.base + p[k], lane)] : BC_INF;
#pragma unroll
            for (int k = 0; k < IL_UNROLL; ++k) {
                tight[k] = dp[k] != BC_INF && (uint64_t)dp[k] + w[k] == dv;
                left[k] = 0;
                if (tight[k]) {
                    const size_t c = cell(it.base + p[k], lane);
                    const double sp = (double)a.sigma[c];
                    atomicAdd(&a.delta[c], sp / sv * f);
                    left[k] = atomicSub(&a.cnt[c], 1);
                }
            }
#pragma unroll
            for (int k = 0; k < IL_UNROLL; ++k) {
                if (j + k >= it.end)
                    break;
                const unsigned long long br = __ballot(tight[k] && left[k] == 1);
                if (br) {
                    const uint32_t ep = it.base + p[k];
                    if (lane == 0)
                        atomicOr(&a.act[ep], br);
                    queue_once_w(a, ep, round, qq, lane);
                }
            }
        }
    }
    qq.flush(lane);
}

// bc[v] += the dependencies of v over every lane of every group whose source
// is another vertex; one wave per vertex, groups in order, lanes summed by a
// fixed tree.
__global__ void k_il_bc(IlArgs a, double *bc, const int32_t *perm)
{
    const int lane = lane_id();
    const uint32_t wid = (blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
    const uint32_t nw = gridDim.x * blockDim.x / WAVE;
    for (uint32_t v = wid; v < (uint32_t)a.n; v += nw) {
        double acc = 0.0;
        for (int grp = 0; grp < a.groups; ++grp) {
            const int32_t s = a.lane_src[grp * WAVE + lane];
            const uint32_t e = (uint32_t)grp * (uint32_t)a.n + v;
            if (s >= 0 && (uint32_t)s != v)
                acc += a.delta[cell(e, lane)];
        }
        acc = wave_sum_f64(acc);
        if (lane == 0)
            bc[perm ? perm[v] : (int32_t)v] += acc;
    }
}

int wave_blocks(size_t waves)
{
    // 256-thread blocks (4 waves each)
    size_t b = (waves + 3) / 4;
    if (b > 16384)
        b = 16384;
    return b < 1 ? 1 : (int)b;
}

} // namespace

hipError_t launch_il_init(const IlArgs &a, const int32_t *sources, long long k,
                          const int32_t *iperm, uint32_t *qout, uint32_t round, hipStream_t st)
{
    hipLaunchKernelGGL(k_il_init, dim3(8192), dim3(256), 0, st, a);
    const int lanes = a.groups * WAVE;
    hipLaunchKernelGGL(k_il_seed, dim3((lanes + 255) / 256), dim3(256), 0, st, a, sources, k,
                       iperm, qout, round);
    return hipGetLastError();
}

static int item_blocks(uint32_t qlen)
{
    // at least 2048 blocks, so that the chunks of high-degree vertices spread
    return std::max(wave_blocks(qlen), 2048);
}

hipError_t launch_il_relax(const IlArgs &a, bool packed, const uint32_t *q, uint32_t qlen,
                           uint32_t *qout, uint32_t *fout, uint32_t thr, uint32_t round,
                           hipStream_t st)
{
    hipLaunchKernelGGL(k_il_take, dim3((qlen + 255) / 256), dim3(256), 0, st, a, q, qlen, 0);
    const dim3 grid(item_blocks(qlen)), block(256);
    if (packed)
        hipLaunchKernelGGL(k_il_relax<true>, grid, block, 0, st, a, q, qout, fout, thr, round);
    else
        hipLaunchKernelGGL(k_il_relax<false>, grid, block, 0, st, a, q, qout, fout, thr, round);
    return hipGetLastError();
}

hipError_t launch_il_far(const IlArgs &a, const uint32_t *fin, uint32_t flen, uint32_t *qout,
                         uint32_t *fout, uint32_t thr_old, uint32_t thr_new, uint32_t round,
                         hipStream_t st)
{
    hipLaunchKernelGGL(k_il_far, dim3(wave_blocks(flen)), dim3(256), 0, st, a, fin, flen, qout,
                       fout, thr_old, thr_new, round);
    return hipGetLastError();
}

hipError_t launch_il_count(const IlArgs &a, bool packed, bool in_arcs, uint32_t *qout,
                           uint32_t round, hipStream_t st)
{
    const dim3 grid(wave_blocks((size_t)a.groups * (size_t)a.n)), block(256);
    if (in_arcs) {
        if (packed)
            hipLaunchKernelGGL(k_il_count_in<true>, grid, block, 0, st, a, qout, round);
        else
            hipLaunchKernelGGL(k_il_count_in<false>, grid, block, 0, st, a, qout, round);
    } else {
        hipLaunchKernelGGL(k_il_leaves, grid, block, 0, st, a, qout, round);
    }
    return hipGetLastError();
}

hipError_t launch_il_round(const IlArgs &a, bool packed, bool deps, const uint32_t *q,
                           uint32_t qlen, uint32_t *qout, uint32_t round, hipStream_t st)
{
    hipLaunchKernelGGL(k_il_take, dim3((qlen + 255) / 256), dim3(256), 0, st, a, q, qlen,
                       deps ? 1 : 0);
    const dim3 grid(item_blocks(qlen)), block(256);
    if (deps) {
        if (packed)
            hipLaunchKernelGGL(k_il_delta<true>, grid, block, 0, st, a, q, qout, round);
        else
            hipLaunchKernelGGL(k_il_delta<false>, grid, block, 0, st, a, q, qout, round);
    } else {
        if (packed)
            hipLaunchKernelGGL(k_il_sigma<true>, grid, block, 0, st, a, q, qout, round);
        else
            hipLaunchKernelGGL(k_il_sigma<false>, grid, block, 0, st, a, q, qout, round);
    }
    return hipGetLastError();
}

hipError_t launch_il_bc(const IlArgs &a, double *bc, const int32_t *perm, hipStream_t st)
{
    hipLaunchKernelGGL(k_il_bc, dim3(wave_blocks((size_t)a.n)), dim3(256), 0, st, a, bc, perm);
    return hipGetLastError();
}
