// shared_types.h -- plain data layouts shared by host code and kernels.
#pragma once

#include <stddef.h>
#include <stdint.h>

#define BC_INF 0x7fffffffu
#define WAVE 64

// ---------------------------------------------------------------------------
// Graph as seen by the kernels.
//
// The arcs leaving v are row[v] .. row[v+1]-1 (CSR, Sec. 3.1).  When the
// head index and the weight fit together in 32 bits the arc is one word,
// head << wshift | (weight - 1); otherwise `arc` holds the heads and `wt`
// the weights.  trow/tarc/twt are the arcs entering each vertex (the same
// arrays as row/arc/wt for an undirected graph).
// ---------------------------------------------------------------------------
struct DevGraph {
    const uint32_t *row;
    const uint32_t *arc;
    const int32_t *wt;
    const uint32_t *trow;
    const uint32_t *tarc;
    const int32_t *twt;
    int32_t n;
    uint32_t wshift;
    uint32_t wmask;
};

// ---------------------------------------------------------------------------
// Per-source state ("slab").  One slab per source in flight.
// ---------------------------------------------------------------------------
struct Slab {
    uint32_t *d;       // tentative / final distance, BC_INF = unreached
    uint64_t *sigma;   // shortest-path count (0 = not yet final in the count pass)
    double *delta;     // dependency (negative = not yet final in the dependency pass)
    double *bcp;       // per-slab partial centrality (batched form)
    int32_t *stamp;    // tag of the latest near queue the vertex entered
    int32_t *infar;    // 1 while the vertex sits in the far pile
    int32_t *order;    // members of each band, band after band
    int32_t *qa, *qb;  // near queues / pending lists
    int32_t *fa, *fb;  // far piles
    int32_t *band_off; // band b = order[band_off[b] .. band_off[b+1])
    int64_t *hdr;      // [0] = last queue tag used by this slab
    uint32_t *ld;      // distances of vertices 0 .. H-1 kept in LDS (batched form)
    int32_t H;         // number of LDS-resident distances (0 = none)
    int32_t *scnt;     // shortest-path-DAG successors not yet accumulated (batched form)
    int32_t *pcnt;     // number of recorded DAG predecessors of each vertex
    int32_t *preds;    // in-row positions of v's DAG in-arcs, at preds[trow[v] ...]
};

// Byte offsets of the slab arrays inside one slot (all 256-byte aligned).
struct SlabLayout {
    size_t d, sigma, delta, bcp, stamp, infar, order, qa, qb, fa, fb, band_off, hdr, scnt, pcnt,
        preds, stride;
};

// ---------------------------------------------------------------------------
// Error reporting shared by all kernels: err[0] is a bit set, err[1] the
// smallest source-list index whose path counts overflowed.
// ---------------------------------------------------------------------------
#define BC_ERRBIT_SIGMA 1
#define BC_ERRBIT_INTERNAL 2
#define BC_ERRBIT_SOURCE 4

struct DevStats {
    unsigned long long reached, arcs, dag, improvements, bands, iterations, sigma_rounds,
        delta_rounds;
    // device wall-clock ticks summed over workgroups: initialisation, frontier
    // expansion, count rounds, dependency rounds, far-pile splits
    unsigned long long ticks[5];
};
