// kernels.h -- argument blocks and launchers shared by the host runtime and
// the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "shared_types.h"

struct BatchArgs {
    DevGraph g;
    char *slab_base;
    SlabLayout L;
    const int32_t *sources;
    long long k;
    unsigned long long *next_src; // device counter handing out sources
    double *bc_out;               // output (atomic accumulation mode)
    double *const *item_out;      // optional: output of each source-list entry (serving)
    unsigned int *item_err;       // optional: set to 1 for each entry whose counts overflowed
    const int32_t *iperm;         // caller id -> internal id (null: identity)
    const int32_t *perm;          // internal id -> caller id (null: identity)
    int32_t H;                    // distances of internal vertices 0..H-1 kept in LDS
    int32_t lds_bits;             // width of the LDS distance entries: 32, 16 or 8 (8: packed arcs)
    int32_t hubs;                 // the graph has vertices of more than wg_deg arcs
    int32_t kahn;                 // 1: dependencies along the recorded DAG; 0: band pulls
    int32_t vw;                   // expansion: 0 adaptive lane/wave, else lanes per vertex
    int32_t node_parallel;        // expansion scans every vertex instead of the queue
    double *ebc;                  // optional edge betweenness output (caller arc order)
    const uint32_t *emap;         // in-row position -> caller arc index
    uint32_t delta;               // band width
    int lane_max;                 // count/dependency passes: lane up to this many arcs
    uint32_t lane_deg, wave_deg;  // expansion tiers: lane / group of lanes / wave by degree
    uint32_t wg_deg;              // expansion: more arcs than this -> the whole workgroup
    DevStats *stats;
    unsigned long long *err;      // [0] error bits, [1] first overflowing source index
    // Far-bucket ring (0: the two-tier far pile): nbk buckets of width delta, each
    // holding up to bcap vertices in the slab's far-pile memory (fa onwards).
    int32_t buckets = 0, nbk = 0, bcap = 0;
};

// Phase machine of the plain form (device memory, one per graph).
struct PlainCtl {
    int phase;
    int32_t s;
    long long src_idx;
    int near_len, next_cnt, order_cnt, far_cnt, kept_cnt, pend_len, pend_cnt;
    int cur, fcur, pcur;
    int32_t gen, band_gen;
    uint32_t thr, thr_old, far_min;
    int band_start, nbands, dband, round, b0, b1;
    unsigned long long iters, iter_cap;
    int abort, finished;
    unsigned long long srounds, drounds;
    double *bc_out; // caller-indexed output of the current computation
};

struct PlainArgs {
    DevGraph g;
    int32_t vw;                   // expansion mapping, as in BatchArgs
    const int32_t *perm;          // internal id -> caller id (null: identity)
    char *slab_base;
    SlabLayout L;
    PlainCtl *ctl;
    double *bc_out;
    uint32_t delta;
    int lane_max;
    uint32_t lane_deg, wave_deg;  // expansion tiers, as in BatchArgs
    DevStats *stats;
    unsigned long long *err;
};

hipError_t launch_batched(const BatchArgs &a, bool packed, int nt, bool atomic_bc, int nslabs,
                          hipStream_t st);
int batched_blocks_per_cu_lds(bool packed, int nt, bool atomic_bc, int lds_bits, size_t lds_bytes);
int batched_blocks_per_cu(bool packed, int nt, bool atomic_bc, int lds_bits);
// dynamic LDS of a batched launch: H resident distances of lds_bits each
size_t batched_lds_bytes(int H, int lds_bits);
hipError_t launch_reduce_partials(char *slab_base, const SlabLayout &L, int nslabs, int n,
                                  double *out, const int32_t *perm, hipStream_t st);
hipError_t launch_plain_source(const PlainArgs &a, bool packed, int grid, int32_t s,
                               long long idx, bool clear_stamps, double *bc_out, hipStream_t st);
hipError_t launch_plain_steps(const PlainArgs &a, bool packed, int grid, int pairs,
                              hipStream_t st);
hipError_t launch_plain_clear_infar(const PlainArgs &a, hipStream_t st);
hipError_t launch_fill_u32(uint32_t *p, size_t count, uint32_t value, hipStream_t st);
// *out = one past the last vertex v with trow[v + 1] > trow[v] (0 if none)
hipError_t launch_inarc_bound(const uint32_t *trow, int32_t n, int *out, hipStream_t st);
hipError_t launch_fill_u64(unsigned long long *p, size_t count, unsigned long long value,
                           hipStream_t st);
hipError_t launch_slab_reset(char *slab_base, const SlabLayout &L, int nslabs, int n,
                             hipStream_t st);
hipError_t launch_export_state(char *slab_base, const SlabLayout &L, int slot, int n, int32_t *d,
                               uint64_t *sigma, double *delta, const int32_t *perm,
                               hipStream_t st);
hipError_t launch_dynamic_affected(const int32_t *dt, const int32_t *dh, int n, int32_t w_old,
                                   int32_t w_new, int both, int32_t *list, int *cnt,
                                   hipStream_t st);
hipError_t launch_iota(int32_t *list, int n, hipStream_t st);
hipError_t launch_dynamic_apply(double *bc, const double *before, const double *after, int n,
                                hipStream_t st);
