// ingest.hip -- graph ingest from device arrays (bc_create_graph_device).
//
// The caller's CSR (row offsets int64[n+1], heads int32[nnz], weights
// int32[nnz], Sec. 3.1) is validated, renumbered, packed and transposed on
// the device, and the result has the same device layout as the host ingest
// of bc_create_graph builds from the same arrays: the same renumbering by
// decreasing in-degree (ties by id), the same arc order in every row of the
// transpose (by arc index), the same pairing of reverse arcs.  The building
// blocks are a stable least-significant-digit radix sort of (64-bit key,
// 32-bit value) pairs and an exclusive scan, both written for 64-lane waves.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <memory>
#include <vector>

#include "bc_internal.h"
#include "dev_common.h"
#include "kernels.h"

namespace {

constexpr int SCAN_NT = 1024;        // threads of a scan block
constexpr int SCAN_PER = 4;          // items per thread
constexpr int SCAN_TILE = SCAN_NT * SCAN_PER;
constexpr int RADIX_BITS = 8;
constexpr int RADIX = 1 << RADIX_BITS;
constexpr int RADIX_CHUNKS = 16;     // 64-element chunks per wave tile
constexpr int RADIX_TILE = WAVE * RADIX_CHUNKS;
constexpr int RADIX_WAVES = 4;       // waves (tiles) per workgroup

int blocks_for(size_t items, int per_block, int cap = 1 << 20)
{
    size_t b = (items + (size_t)per_block - 1) / (size_t)per_block;
    return (int)std::max<size_t>(1, std::min<size_t>(b, (size_t)cap));
}

// ---------------------------------------------------------------------------
// Exclusive scan of uint32 (totals below 2^32)
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t wave_incl_scan_u32(uint32_t x)
{
    const int lane = lane_id();
    for (int o = 1; o < WAVE; o <<= 1) {
        const uint32_t y = __shfl_up(x, o);
        if (lane >= o)
            x += y;
    }
    return x;
}

// Scans one tile of SCAN_TILE items per block; the block's total goes to
// sums[blockIdx.x].
__global__ __launch_bounds__(SCAN_NT) void k_scan_tiles(const uint32_t *in, uint32_t *out,
                                                       size_t count, uint32_t *sums)
{
    __shared__ uint32_t wsum[SCAN_NT / WAVE];
    const size_t base = (size_t)blockIdx.x * SCAN_TILE + (size_t)threadIdx.x * SCAN_PER;
    uint32_t v[SCAN_PER];
    uint32_t t = 0;
#pragma unroll
    for (int j = 0; j < SCAN_PER; ++j) {
        v[j] = base + j < count ? in[base + j] : 0u;
        t += v[j];
    }
    const int w = threadIdx.x / WAVE;
    const uint32_t incl = wave_incl_scan_u32(t);
    if (lane_id() == WAVE - 1)
        wsum[w] = incl;
    __syncthreads();
    if (w == 0) {
        const uint32_t x = lane_id() < SCAN_NT / WAVE ? wsum[lane_id()] : 0u;
        const uint32_t xi = wave_incl_scan_u32(x);
        if (lane_id() < SCAN_NT / WAVE)
            wsum[lane_id()] = xi - x; // exclusive prefix of each wave
        if (lane_id() == SCAN_NT / WAVE - 1)
            sums[blockIdx.x] = xi;
    }
    __syncthreads();
    uint32_t run = wsum[w] + incl - t;
#pragma unroll
    for (int j = 0; j < SCAN_PER; ++j) {
        if (base + j < count)
            out[base + j] = run;
        run += v[j];
    }
}

__global__ void k_scan_add(uint32_t *out, size_t count, const uint32_t *offs)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count)
        out[i] += offs[i / SCAN_TILE];
}

// out[i] = sum of in[0 .. i-1]; in and out may be the same array.  *total
// (device, may be null) receives the sum of all items.
void scan_exclusive(const uint32_t *in, uint32_t *out, size_t count, uint32_t *total,
                    hipStream_t st)
{
    const size_t tiles = (count + SCAN_TILE - 1) / SCAN_TILE;
    DevBuf sums;
    sums.alloc(std::max<size_t>(tiles, 1) * 4 + 4);
    uint32_t *s = (uint32_t *)sums.p;
    hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)std::max<size_t>(tiles, 1)), dim3(SCAN_NT),
                       0, st, in, out, count, s);
    hip_check(hipGetLastError(), "scan");
    if (tiles > 1) {
        scan_exclusive(s, s, tiles, total, st);
        hipLaunchKernelGGL(k_scan_add, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st,
                           out, count, s);
        hip_check(hipGetLastError(), "scan add");
    } else if (total) {
        hip_check(hipMemcpyAsync(total, s, 4, hipMemcpyDeviceToDevice, st), "scan total");
    }
    hip_check(hipStreamSynchronize(st), "scan"); // the tile sums are released here
}

// ---------------------------------------------------------------------------
// Stable LSD radix sort of (key u64, value u32) pairs, 8 bits per pass.
//
// Each wave owns a tile of RADIX_TILE consecutive items, read in 64-item
// chunks in order; the digit histograms are stored digit-major over the
// tiles, so one exclusive scan gives every (digit, tile) its first output
// position, and inside a tile an item's rank among the equal digits before
// it comes from ballots.  Equal digits keep their input order: the sort is
// stable, so a sort by a secondary key followed by one by the primary key
// orders by both.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(WAVE * RADIX_WAVES) void k_radix_hist(const uint64_t *keys,
                                                                  uint32_t count, int shift,
                                                                  uint32_t ntiles, uint32_t *hist)
{
    __shared__ uint32_t h[RADIX_WAVES][RADIX];
    const int w = threadIdx.x / WAVE, lane = lane_id();
    const uint32_t tile = blockIdx.x * RADIX_WAVES + w;
    for (int d = lane; d < RADIX; d += WAVE)
        h[w][d] = 0;
    __syncthreads();
    if (tile < ntiles) {
        const uint32_t base = tile * RADIX_TILE;
        for (int c = 0; c < RADIX_CHUNKS; ++c) {
            const uint32_t i = base + c * WAVE + lane;
            if (i < count)
                atomicAdd(&h[w][(keys[i] >> shift) & (RADIX - 1)], 1u);
        }
    }
    __syncthreads();
    if (tile < ntiles)
        for (int d = lane; d < RADIX; d += WAVE)
            hist[(size_t)d * ntiles + tile] = h[w][d];
}

__global__ __launch_bounds__(WAVE * RADIX_WAVES) void k_radix_scatter(
    const uint64_t *keys, const uint32_t *vals, uint64_t *okeys, uint32_t *ovals, uint32_t count,
    int shift, uint32_t ntiles, const uint32_t *offs)
{
    __shared__ uint32_t pos[RADIX_WAVES][RADIX];
    const int w = threadIdx.x / WAVE, lane = lane_id();
    const uint32_t tile = blockIdx.x * RADIX_WAVES + w;
    if (tile >= ntiles)
        return; // whole wave: the tile index is uniform in the wave
    for (int d = lane; d < RADIX; d += WAVE)
        pos[w][d] = offs[(size_t)d * ntiles + tile];
    const uint32_t base = tile * RADIX_TILE;
    for (int c = 0; c < RADIX_CHUNKS; ++c) {
        const uint32_t i = base + c * WAVE + lane;
        const bool valid = i < count;
        uint64_t k = 0;
        uint32_t v = 0, d = 0;
        if (valid) {
            k = keys[i];
            v = vals[i];
            d = (uint32_t)(k >> shift) & (RADIX - 1);
        }
        // lanes holding the same digit
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < RADIX_BITS; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        const uint32_t rank = lanes_below(peers);
        const uint32_t at = valid ? pos[w][d] + rank : 0u;
        // the last of the peers advances the digit's position for the next chunk
        const bool last = valid && (peers >> lane) == 1ull;
        __builtin_amdgcn_wave_barrier();
        if (last)
            pos[w][d] = at + 1u;
        __builtin_amdgcn_wave_barrier();
        if (valid) {
            okeys[at] = k;
            ovals[at] = v;
        }
    }
}

int bit_width_u64(uint64_t x)
{
    int b = 0;
    while (x) {
        ++b;
        x >>= 1;
    }
    return b;
}

// Sorts (keys, vals) by the key bits [0, bits) in place (the buffers are
// swapped with the scratch pair as needed so that the result ends in keys,
// vals).
struct SortBufs {
    DevBuf k2, v2, hist;
};

void radix_sort(uint64_t *keys, uint32_t *vals, uint32_t count, int bits, SortBufs &tmp,
                hipStream_t st)
{
    if (count < 2 || bits <= 0)
        return;
    const uint32_t ntiles = (count + RADIX_TILE - 1) / RADIX_TILE;
    if (tmp.k2.bytes < (size_t)count * 8)
        tmp.k2.alloc((size_t)count * 8);
    if (tmp.v2.bytes < (size_t)count * 4)
        tmp.v2.alloc((size_t)count * 4);
    if (tmp.hist.bytes < (size_t)ntiles * RADIX * 4)
        tmp.hist.alloc((size_t)ntiles * RADIX * 4);
    uint64_t *ka = keys, *kb = (uint64_t *)tmp.k2.p;
    uint32_t *va = vals, *vb = (uint32_t *)tmp.v2.p;
    uint32_t *hist = (uint32_t *)tmp.hist.p;
    const unsigned blocks = (ntiles + RADIX_WAVES - 1) / RADIX_WAVES;
    int passes = 0;
    for (int shift = 0; shift < bits; shift += RADIX_BITS, ++passes) {
        hipLaunchKernelGGL(k_radix_hist, dim3(blocks), dim3(WAVE * RADIX_WAVES), 0, st, ka, count,
                           shift, ntiles, hist);
        hip_check(hipGetLastError(), "radix histogram");
        scan_exclusive(hist, hist, (size_t)ntiles * RADIX, nullptr, st);
        hipLaunchKernelGGL(k_radix_scatter, dim3(blocks), dim3(WAVE * RADIX_WAVES), 0, st, ka, va,
                           kb, vb, count, shift, ntiles, hist);
        hip_check(hipGetLastError(), "radix scatter");
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    if (passes & 1) {
        hip_check(hipMemcpyAsync(keys, ka, (size_t)count * 8, hipMemcpyDeviceToDevice, st),
                  "sort copy");
        hip_check(hipMemcpyAsync(vals, va, (size_t)count * 4, hipMemcpyDeviceToDevice, st),
                  "sort copy");
    }
}

// ---------------------------------------------------------------------------
// Ingest kernels
// ---------------------------------------------------------------------------
struct IngestSummary {
    unsigned long long bad_row;  // smallest row whose offsets decrease (ULLONG_MAX: none)
    unsigned long long bad_col;  // smallest arc whose head is out of range
    unsigned long long bad_w;    // smallest arc whose weight is below 1
    unsigned long long wsum;     // sum of the weights
    unsigned int maxdeg, wmax, nz_rows, max_indeg;
    int32_t bad_w_value, bad_col_value;
    long long row0, rown;        // row_ptr[0], row_ptr[n]
};

// Validation (the checks of the host ingest) and the per-vertex in-degrees.
__global__ void k_ingest_check(int32_t n, uint32_t nnz, const int64_t *row_ptr,
                               const int32_t *col, const int32_t *w, uint32_t *indeg,
                               IngestSummary *sum)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    const size_t span = std::max<size_t>((size_t)n, (size_t)nnz);
    const size_t tid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid == 0) {
        sum->row0 = row_ptr[0];
        sum->rown = row_ptr[n];
    }
    // every lane of a wave runs the same number of iterations (wave reductions)
    const size_t iters = (span + stride - 1) / stride;
    uint32_t maxdeg = 0, wmax = 0, nz = 0;
    unsigned long long wsum = 0;
    for (size_t it = 0; it < iters; ++it) {
        const size_t i = tid + it * stride;
        if (i < (size_t)n) {
            const long long d = row_ptr[i + 1] - row_ptr[i];
            if (d < 0)
                atomicMin(&sum->bad_row, (unsigned long long)i);
            else if (d > 0) {
                nz += 1;
                const uint32_t dd = d > 0xffffffffll ? 0xffffffffu : (uint32_t)d;
                maxdeg = dd > maxdeg ? dd : maxdeg;
            }
        }
        if (i < (size_t)nnz) {
            const int32_t c = col[i];
            const int32_t x = w[i];
            if (c < 0 || c >= n)
                atomicMin(&sum->bad_col, (unsigned long long)i);
            else
                atomicAdd(&indeg[c], 1u);
            if (x < 1)
                atomicMin(&sum->bad_w, (unsigned long long)i);
            else {
                wmax = (uint32_t)x > wmax ? (uint32_t)x : wmax;
                wsum += (unsigned long long)x;
            }
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        const uint32_t a = __shfl_xor(maxdeg, o), b = __shfl_xor(wmax, o);
        maxdeg = a > maxdeg ? a : maxdeg;
        wmax = b > wmax ? b : wmax;
        nz += __shfl_xor(nz, o);
        wsum += __shfl_xor(wsum, o);
    }
    if (lane_id() == 0) {
        atomicMax(&sum->maxdeg, maxdeg);
        atomicMax(&sum->wmax, wmax);
        atomicAdd(&sum->nz_rows, nz);
        atomicAdd(&sum->wsum, wsum);
    }
}

__global__ void k_ingest_bad_values(const int32_t *col, const int32_t *w, IngestSummary *sum)
{
    if (sum->bad_col != ~0ull)
        sum->bad_col_value = col[sum->bad_col];
    if (sum->bad_w != ~0ull)
        sum->bad_w_value = w[sum->bad_w];
}

__global__ void k_max_indeg(const uint32_t *indeg, int32_t n, IngestSummary *sum)
{
    uint32_t m = 0;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < (size_t)n; i += stride)
        m = indeg[i] > m ? indeg[i] : m;
    for (int o = 32; o > 0; o >>= 1) {
        const uint32_t y = __shfl_xor(m, o);
        m = y > m ? y : m;
    }
    if (lane_id() == 0)
        atomicMax(&sum->max_indeg, m);
}

// Sort keys of the renumbering: decreasing in-degree; the stable sort keeps
// equal in-degrees in id order, as the host's stable sort does.
__global__ void k_renumber_keys(const uint32_t *indeg, int32_t n, uint32_t maxin, uint64_t *keys,
                                uint32_t *vals)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t v = (size_t)blockIdx.x * blockDim.x + threadIdx.x; v < (size_t)n; v += stride) {
        keys[v] = maxin - indeg[v];
        vals[v] = (uint32_t)v;
    }
}

// Sum of the in-degrees of the first `top` vertices of the order.
__global__ void k_top_sum(const uint32_t *indeg, const uint32_t *order, int32_t top,
                          unsigned long long *out)
{
    unsigned long long s = 0;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < (size_t)top; i += stride)
        s += indeg[order[i]];
    for (int o = 32; o > 0; o >>= 1)
        s += __shfl_xor(s, o);
    if (lane_id() == 0 && s)
        atomicAdd(out, s);
}

// perm[i] = order[i] (internal -> caller), iperm[order[i]] = i, and the
// internal out-degrees (deg[i] = out-degree of order[i]) and in-degrees.
__global__ void k_apply_order(const uint32_t *order, int32_t n, const int64_t *row_ptr,
                              const uint32_t *indeg, int32_t *perm, int32_t *iperm, uint32_t *deg,
                              uint32_t *tdeg)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < (size_t)n; i += stride) {
        const uint32_t o = order[i];
        perm[i] = (int32_t)o;
        iperm[o] = (int32_t)i;
        deg[i] = (uint32_t)(row_ptr[o + 1] - row_ptr[o]);
        tdeg[i] = indeg[o];
    }
}

__global__ void k_row_u32(const int64_t *row_ptr, int32_t n, uint32_t *row)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i <= (size_t)n; i += stride)
        row[i] = (uint32_t)row_ptr[i];
}

// The row holding arc position p: the last v with row[v] <= p.
__device__ __forceinline__ uint32_t row_of(const uint32_t *row, int32_t n, uint32_t p)
{
    uint32_t lo = 0, hi = (uint32_t)n; // row[lo] <= p < row[hi]
    while (hi - lo > 1) {
        const uint32_t mid = lo + (hi - lo) / 2;
        if (row[mid] <= p)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// Internal arcs: arc position p of internal row i comes from caller arc
// src = row_ptr[perm[i]] + (p - row[i]) (src = p without renumbering); its
// head is renumbered.  Writes the head (tail[] gets the internal tail), the
// weight, and the caller arc index (edge betweenness).
__global__ void k_internal_arcs(int32_t n, uint32_t nnz, const uint32_t *row,
                                const int64_t *row_ptr, const int32_t *col, const int32_t *w,
                                const int32_t *perm, const int32_t *iperm, uint32_t *head,
                                uint32_t *tail, int32_t *wt, uint32_t *ce)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x; p < (size_t)nnz; p += stride) {
        const uint32_t i = row_of(row, n, (uint32_t)p);
        const size_t src = perm ? (size_t)row_ptr[perm[i]] + (p - row[i]) : p;
        const int32_t c = col[src];
        head[p] = (uint32_t)(iperm ? iperm[c] : c);
        tail[p] = i;
        wt[p] = w[src];
        if (ce)
            ce[p] = (uint32_t)src;
    }
}

__global__ void k_pack_arcs(uint32_t nnz, const uint32_t *head, const int32_t *wt, int packed,
                            uint32_t wshift, uint32_t wmask, uint32_t *arc)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x; p < (size_t)nnz; p += stride)
        arc[p] = packed ? (head[p] << wshift) | ((uint32_t)(wt[p] - 1) & wmask) : head[p];
}

// Keys (primary << shift | secondary) over the arcs, values = arc positions.
__global__ void k_pair_keys(uint32_t nnz, const uint32_t *a, const uint32_t *b, int shift,
                            uint64_t *keys, uint32_t *vals, const uint32_t *order)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < (size_t)nnz; i += stride) {
        const uint32_t p = order ? order[i] : (uint32_t)i;
        keys[i] = b ? ((uint64_t)a[p] << shift) | b[p] : (uint64_t)a[p];
        vals[i] = p;
    }
}

__global__ void k_weight_keys(uint32_t nnz, const int32_t *wt, uint64_t *keys, uint32_t *vals)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < (size_t)nnz; i += stride) {
        keys[i] = (uint64_t)(uint32_t)wt[i];
        vals[i] = (uint32_t)i;
    }
}

// Transpose entries: in-row position q holds the arc sorted[q] (tail, weight).
__global__ void k_transpose_arcs(uint32_t nnz, const uint32_t *sorted, const uint32_t *tail,
                                 const int32_t *wt, int packed, uint32_t wshift, uint32_t wmask,
                                 uint32_t *tarc, int32_t *twt)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < (size_t)nnz; q += stride) {
        const uint32_t p = sorted[q];
        const uint32_t t = tail[p];
        const int32_t x = wt[p];
        tarc[q] = packed ? (t << wshift) | ((uint32_t)(x - 1) & wmask) : t;
        if (twt)
            twt[q] = x;
    }
}

// Undirected check and reverse-arc pairing: fwd lists the arcs sorted by
// (tail, head, weight, position), bwd by (head, tail, weight, position).  The
// graph is symmetric iff the i-th entries agree as (tail, head, weight) vs
// (head, tail, weight) for every i; then rev[fwd[i]] = bwd[i].
__global__ void k_pair_reverse(uint32_t nnz, const uint32_t *fwd, const uint32_t *bwd,
                               const uint32_t *head, const uint32_t *tail, const int32_t *wt,
                               uint32_t *rev, unsigned int *mismatch)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    bool bad = false;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < (size_t)nnz; i += stride) {
        const uint32_t f = fwd[i], b = bwd[i];
        bad |= tail[f] != head[b] || head[f] != tail[b] || wt[f] != wt[b];
        if (rev)
            rev[f] = b;
    }
    if (__ballot(bad) && lane_id() == 0)
        atomicOr(mismatch, 1u);
}

__global__ void k_emap(uint32_t nnz, const uint32_t *through, const uint32_t *ce, uint32_t *emap)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x; p < (size_t)nnz; p += stride) {
        const uint32_t a = through[p];
        emap[p] = ce ? ce[a] : a;
    }
}

#define GRID(items) dim3((unsigned)blocks_for((size_t)(items), 256, 8192)), dim3(256), 0

// Sorts the arc positions stably by (a << shift | b) after a stable sort by
// the weight (when by_weight): the result lists the arcs ordered by
// (a, b, weight, position).
void sort_arcs(uint32_t nnz, const uint32_t *a, const uint32_t *b, int shift, int key_bits,
               const int32_t *wt, int wbits, uint64_t *keys, uint32_t *vals, SortBufs &tmp,
               hipStream_t st)
{
    const uint32_t *order = nullptr;
    DevBuf by_w;
    if (wt && wbits > 0) {
        hipLaunchKernelGGL(k_weight_keys, GRID(nnz), st, nnz, wt, keys, vals);
        radix_sort(keys, vals, nnz, wbits, tmp, st);
        by_w.alloc((size_t)nnz * 4);
        hip_check(hipMemcpyAsync(by_w.p, vals, (size_t)nnz * 4, hipMemcpyDeviceToDevice, st),
                  "copy");
        order = (const uint32_t *)by_w.p;
    }
    hipLaunchKernelGGL(k_pair_keys, GRID(nnz), st, nnz, a, b, shift, keys, vals, order);
    radix_sort(keys, vals, nnz, key_bits, tmp, st);
    hip_check(hipStreamSynchronize(st), "sort arcs");
}

} // namespace

// Builds graph g (fields already zeroed) from the caller's device CSR.
void create_graph_device(int32_t n, int64_t nnz64, const int64_t *row_ptr, const int32_t *col,
                         const int32_t *w, uint32_t flags, hipStream_t st, bc_graph *g)
{
    const uint32_t nnz = (uint32_t)nnz64;
    const bool directed = (flags & BC_DIRECTED) != 0;
    const bool want_edges = (flags & BC_EDGE_BC) != 0;

    // 1. validation and in-degrees
    DevBuf sumb, indegb;
    sumb.alloc(sizeof(IngestSummary));
    indegb.alloc((size_t)n * 4);
    {
        IngestSummary init;
        memset(&init, 0, sizeof init);
        init.bad_row = init.bad_col = init.bad_w = ~0ull;
        hip_check(hipMemcpyAsync(sumb.p, &init, sizeof init, hipMemcpyHostToDevice, st), "init");
    }
    hip_check(launch_fill_u32((uint32_t *)indegb.p, (size_t)n, 0u, st), "clear");
    IngestSummary *dsum = (IngestSummary *)sumb.p;
    uint32_t *indeg = (uint32_t *)indegb.p;
    hipLaunchKernelGGL(k_ingest_check, GRID(std::max<size_t>((size_t)n, nnz)), st, n, nnz, row_ptr,
                       col, w, indeg, dsum);
    hipLaunchKernelGGL(k_ingest_bad_values, dim3(1), dim3(1), 0, st, col, w, dsum);
    hipLaunchKernelGGL(k_max_indeg, GRID(n), st, indeg, n, dsum);
    hip_check(hipGetLastError(), "ingest check");
    IngestSummary S;
    hip_check(hipMemcpyAsync(&S, dsum, sizeof S, hipMemcpyDeviceToHost, st), "summary");
    hip_check(hipStreamSynchronize(st), "ingest check");
    if (S.row0 != 0 || S.rown != nnz64)
        throw bc_error(BC_E_GRAPH, "row_ptr[0] must be 0 and row_ptr[n] must equal nnz");
    if (S.bad_row != ~0ull)
        throw bc_error(BC_E_GRAPH, "row_ptr decreases at row %lld", (long long)S.bad_row);
    if (S.bad_col != ~0ull && S.bad_col <= S.bad_w)
        throw bc_error(BC_E_GRAPH, "col[%lld] = %d out of range", (long long)S.bad_col,
                       S.bad_col_value);
    if (S.bad_w != ~0ull)
        throw bc_error(BC_E_WEIGHT, "w[%lld] = %d is below 1", (long long)S.bad_w, S.bad_w_value);
    const int32_t wmax = nnz ? (int32_t)S.wmax : 1;
    if ((int64_t)(n - 1) * (int64_t)wmax > (int64_t)INT32_MAX - 1)
        throw bc_error(BC_E_DIST_OVERFLOW, "(n-1)*max weight = %lld does not fit in int32",
                       (long long)(n - 1) * wmax);

    g->n = n;
    g->nnz = nnz64;
    g->directed = directed;
    g->wmax = wmax;
    g->maxdeg = (int32_t)std::min<uint32_t>(S.maxdeg, INT32_MAX);
    const int colbits = bit_width_u64((uint64_t)(n - 1));
    const int wbits = bit_width_u64((uint64_t)(wmax - 1));
    g->packed = colbits + wbits <= 32 && wbits < 32;
    g->wshift = g->packed ? (uint32_t)wbits : 0u;
    g->wmask = g->packed ? (wbits == 0 ? 0u : (uint32_t)((1ull << wbits) - 1)) : 0u;
    g->wbytes = wmax <= 255 ? 1 : (wmax <= 65535 ? 2 : 4);
    g->avg_deg = S.nz_rows ? (double)nnz64 / (double)S.nz_rows : 0.0;
    g->wmean = nnz ? (double)S.wsum / (double)nnz64 : 1.0;

    SortBufs tmp;
    // 2. renumbering by decreasing in-degree when the in-degrees are skewed
    DevBuf keysb, valsb;
    const size_t sort_n = std::max<size_t>((size_t)n, (size_t)nnz);
    keysb.alloc(std::max<size_t>(sort_n, 1) * 8);
    valsb.alloc(std::max<size_t>(sort_n, 1) * 4);
    uint64_t *keys = (uint64_t *)keysb.p;
    uint32_t *vals = (uint32_t *)valsb.p;
    bool renumber = false;
    if (!(flags & BC_KEEP_ORDER) && n > 1 && nnz > 0) {
        hipLaunchKernelGGL(k_renumber_keys, GRID(n), st, indeg, n, S.max_indeg, keys, vals);
        radix_sort(keys, vals, (uint32_t)n, bit_width_u64(S.max_indeg), tmp, st);
        DevBuf topb;
        topb.alloc(8);
        hip_check(launch_fill_u64((unsigned long long *)topb.p, 1, 0ull, st), "clear");
        const int32_t top = std::max<int32_t>(1, n / 100);
        hipLaunchKernelGGL(k_top_sum, GRID(top), st, indeg, vals, top,
                           (unsigned long long *)topb.p);
        unsigned long long top_arcs = 0;
        hip_check(hipMemcpyAsync(&top_arcs, topb.p, 8, hipMemcpyDeviceToHost, st), "top");
        hip_check(hipStreamSynchronize(st), "renumbering");
        renumber = (double)top_arcs > 0.05 * (double)nnz64;
    }
    DevBuf degb, tdegb;
    degb.alloc(((size_t)n + 1) * 4);
    tdegb.alloc(((size_t)n + 1) * 4);
    g->row.alloc(((size_t)n + 1) * 4);
    uint32_t *row = (uint32_t *)g->row.p;
    if (renumber) {
        g->renumbered = true;
        g->perm.alloc((size_t)n * 4);
        g->iperm.alloc((size_t)n * 4);
        hipLaunchKernelGGL(k_apply_order, GRID(n), st, vals, n, row_ptr, indeg,
                           (int32_t *)g->perm.p, (int32_t *)g->iperm.p, (uint32_t *)degb.p,
                           (uint32_t *)tdegb.p);
        hip_check(hipGetLastError(), "renumber");
        hip_check(launch_fill_u32((uint32_t *)degb.p + n, 1, 0u, st), "clear");
        scan_exclusive((const uint32_t *)degb.p, row, (size_t)n + 1, nullptr, st);
        g->host_iperm.resize((size_t)n);
        hip_check(hipMemcpyAsync(g->host_iperm.data(), g->iperm.p, (size_t)n * 4,
                                 hipMemcpyDeviceToHost, st),
                  "numbering");
    } else {
        hipLaunchKernelGGL(k_row_u32, GRID((size_t)n + 1), st, row_ptr, n, row);
        hip_check(hipGetLastError(), "rows");
    }

    // 3. internal arcs (heads renumbered), packed
    DevBuf headb, tailb, wtb, ceb;
    headb.alloc(std::max<size_t>(nnz, 1) * 4);
    tailb.alloc(std::max<size_t>(nnz, 1) * 4);
    wtb.alloc(std::max<size_t>(nnz, 1) * 4);
    if (want_edges && renumber)
        ceb.alloc(std::max<size_t>(nnz, 1) * 4);
    uint32_t *head = (uint32_t *)headb.p, *tail = (uint32_t *)tailb.p;
    int32_t *wt = (int32_t *)wtb.p;
    uint32_t *ce = (uint32_t *)ceb.p;
    if (nnz > 0) {
        hipLaunchKernelGGL(k_internal_arcs, GRID(nnz), st, n, nnz, row, row_ptr, col, w,
                           renumber ? (const int32_t *)g->perm.p : nullptr,
                           renumber ? (const int32_t *)g->iperm.p : nullptr, head, tail, wt, ce);
        g->arc.alloc((size_t)nnz * 4);
        hipLaunchKernelGGL(k_pack_arcs, GRID(nnz), st, nnz, head, wt, (int)g->packed, g->wshift,
                           g->wmask, (uint32_t *)g->arc.p);
        if (!g->packed) {
            g->wt.alloc((size_t)nnz * 4);
            hip_check(hipMemcpyAsync(g->wt.p, wt, (size_t)nnz * 4, hipMemcpyDeviceToDevice, st),
                      "weights");
        }
        hip_check(hipGetLastError(), "arcs");
    }

    // 4. transpose (directed) or symmetry check and reverse arcs (undirected)
    DevBuf through; // per in-row position: the arc it stands for (edge map)
    if (directed) {
        g->trow.alloc(((size_t)n + 1) * 4);
        uint32_t *tdeg = renumber ? (uint32_t *)tdegb.p : indeg;
        if (!renumber) {
            hip_check(hipMemcpyAsync(tdegb.p, indeg, (size_t)n * 4, hipMemcpyDeviceToDevice, st),
                      "in-degrees");
            tdeg = (uint32_t *)tdegb.p;
        }
        hip_check(launch_fill_u32(tdeg + n, 1, 0u, st), "clear");
        scan_exclusive(tdeg, (uint32_t *)g->trow.p, (size_t)n + 1, nullptr, st);
        if (nnz > 0) {
            // arcs stably by head: every in-row lists its arcs by arc position
            sort_arcs(nnz, head, nullptr, 0, colbits, nullptr, 0, keys, vals, tmp, st);
            g->tarc.alloc((size_t)nnz * 4);
            if (!g->packed)
                g->twt.alloc((size_t)nnz * 4);
            hipLaunchKernelGGL(k_transpose_arcs, GRID(nnz), st, nnz, vals, tail, wt,
                               (int)g->packed, g->wshift, g->wmask, (uint32_t *)g->tarc.p,
                               g->packed ? nullptr : (int32_t *)g->twt.p);
            hip_check(hipGetLastError(), "transpose");
            if (want_edges) {
                through.alloc((size_t)nnz * 4);
                hip_check(hipMemcpyAsync(through.p, vals, (size_t)nnz * 4,
                                         hipMemcpyDeviceToDevice, st),
                          "copy");
            }
        }
    } else if (nnz > 0) {
        const int wb = bit_width_u64((uint64_t)wmax);
        DevBuf fwd;
        fwd.alloc((size_t)nnz * 4);
        sort_arcs(nnz, tail, head, colbits, 2 * colbits, wt, wb, keys, vals, tmp, st);
        hip_check(hipMemcpyAsync(fwd.p, vals, (size_t)nnz * 4, hipMemcpyDeviceToDevice, st),
                  "copy");
        sort_arcs(nnz, head, tail, colbits, 2 * colbits, wt, wb, keys, vals, tmp, st);
        DevBuf mis;
        mis.alloc(4);
        hip_check(launch_fill_u32((uint32_t *)mis.p, 1, 0u, st), "clear");
        if (want_edges)
            through.alloc((size_t)nnz * 4);
        hipLaunchKernelGGL(k_pair_reverse, GRID(nnz), st, nnz, (const uint32_t *)fwd.p, vals, head,
                           tail, wt, want_edges ? (uint32_t *)through.p : nullptr,
                           (unsigned int *)mis.p);
        hip_check(hipGetLastError(), "symmetry");
        unsigned int bad = 0;
        hip_check(hipMemcpyAsync(&bad, mis.p, 4, hipMemcpyDeviceToHost, st), "symmetry");
        hip_check(hipStreamSynchronize(st), "symmetry");
        if (bad)
            throw bc_error(BC_E_GRAPH,
                           "undirected graph is not symmetric (every arc needs a reverse arc of "
                           "equal weight); pass BC_DIRECTED for one-way arcs");
    }

    // 5. edge map: in-row position -> caller arc index
    if (want_edges && nnz > 0) {
        g->emap.alloc((size_t)nnz * 4);
        hipLaunchKernelGGL(k_emap, GRID(nnz), st, nnz, (const uint32_t *)through.p,
                           renumber ? ce : nullptr, (uint32_t *)g->emap.p);
        hip_check(hipGetLastError(), "edge map");
    }
    g->edges_ready = want_edges;
    set_inarc_bound(g, st);
}
