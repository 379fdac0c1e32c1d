// shared_types.h -- plain data layouts shared by host code and kernels.
#pragma once

#include <stddef.h>
#include <stdint.h>

#define BC_INF 0x7fffffffu
#define WAVE 64
// Default degree thresholds of the adaptive mapping: at most BC_DEF_LANE_DEG
// arcs -> one lane, at most BC_DEF_WAVE_DEG -> a group of lanes, more -> a
// wave; in the batched expansion more than BC_HUB_DEG -> the whole workgroup
// (only graphs that have such a vertex pay for the step).
#define BC_DEF_LANE_DEG 8
#define BC_DEF_WAVE_DEG 64
#define BC_HUB_DEG 512
// Most buckets of the far-bucket ring (batched form).
#define BC_BUCKETS_MAX 128

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
    int32_t n_act; // vertices from n_act on have no in-arcs: no source reaches them
                   // (each is reached only as a source itself)
    uint32_t wshift;
    uint32_t wmask;
};

// ---------------------------------------------------------------------------
// Per-source state ("slab").  One slab per source in flight.
//
// Distances, the most often read field (every arc relaxation and every
// tightness test reads one at a random vertex), stay a dense array so that
// a cache line holds as many of them as possible.  The other per-vertex
// fields, which the count, dependency and split passes touch together,
// share one 32-byte record, so that such a visit of a random vertex fetches
// one line instead of one line per field.  Record layout:
// ---------------------------------------------------------------------------
#define VREC_BYTES 32
#define VREC_STAMP 0  // i32 tag of the latest near queue the vertex entered
#define VREC_INFAR 4  // i32 bit 0: in the inner far pile; bit 1: in the outer far pile
#define VREC_SCNT 8   // i32 shortest-path-DAG successors not yet accumulated
#define VREC_PRED1 12 // i32 the only DAG predecessor, or -1: the list in preds[]; before the
                      // vertex is counted (bucket ring), BUCKET_KEY of the least far bucket
                      // it was put in: below every value the count pass writes, so a ring
                      // entry is current exactly when its bucket's key is there
// Ring bucket b as kept in the record: below every predecessor encoding while
// buckets and vertex ids stay below 2^30 (the ring is only planned then).
#define BUCKET_KEY(b) ((int32_t)((uint32_t)INT32_MIN + (uint32_t)(b)))
#define VREC_SIGMA 16 // u64 shortest-path count (0 = not yet final in the count pass)
#define VREC_DELTA 24 // f64 dependency (negative = not yet final in the pull pass)

// Byte offsets of the slab arrays inside one slot (all 256-byte aligned).
struct SlabLayout {
    size_t d, rec, bcp, order, qa, qb, fa, fb, bx, oa, ob, band_off, hdr, preds, stride;
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
