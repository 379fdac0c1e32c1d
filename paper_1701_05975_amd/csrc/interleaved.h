// interleaved.h -- argument block and launchers of the source-interleaved
// form, shared by its host driver and its HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "shared_types.h"

// Source-interleaved form: the state of `groups` groups of 64 sources; entry
// e = group * n + vertex, and each state array holds one 64-lane row per entry
// (lane b = the group's b-th source).
// Arcs per work item of a round (a vertex with more arcs is split).
#define IL_CHUNK 256u

struct IlCtl {
    unsigned int qlen;     // entries appended to the output queue this launch
    unsigned int flen;     // entries in the far list being built
    unsigned int minkept;  // least distance kept in the far list by a far pass
    unsigned int ilen;     // work items of the current round
    unsigned long long reached;
};

struct IlArgs {
    DevGraph g;
    int n, groups;
    uint32_t *d;                // [entries][64] distances, BC_INF = unreached
    unsigned long long *sigma;  // [entries][64] shortest-path counts
    double *delta;              // [entries][64] dependencies
    int32_t *cnt;               // [entries][64] pending DAG neighbours
    unsigned long long *act;    // [entries] lanes to process when the entry is dequeued
    unsigned long long *far;    // [entries] lanes with a distance beyond the band
    uint32_t *stamp;            // [entries] last round that queued the entry
    int32_t *lane_src;          // [groups * 64] internal source id, -1 = empty lane
    unsigned long long *qm;     // [entries] lane mask taken by each queue slot this round
    unsigned long long *items;  // work items (queue slot << 32 | arc chunk) of the round
    IlCtl *ctl;
    unsigned long long *err;    // [0] error bits, [1] first overflowing source-list index
    long long src_base;         // source-list index of the sweep's first lane
};

hipError_t launch_il_init(const IlArgs &a, const int32_t *sources, long long k,
                          const int32_t *iperm, uint32_t *qout, uint32_t round, hipStream_t st);
hipError_t launch_il_relax(const IlArgs &a, bool packed, const uint32_t *q, uint32_t qlen,
                           uint32_t *qout, uint32_t *fout, uint32_t thr, uint32_t round,
                           hipStream_t st);
hipError_t launch_il_far(const IlArgs &a, const uint32_t *fin, uint32_t flen, uint32_t *qout,
                         uint32_t *fout, uint32_t thr_old, uint32_t thr_new, uint32_t round,
                         hipStream_t st);
hipError_t launch_il_count(const IlArgs &a, bool packed, bool in_arcs, uint32_t *qout,
                           uint32_t round, hipStream_t st);
hipError_t launch_il_round(const IlArgs &a, bool packed, bool deps, const uint32_t *q,
                           uint32_t qlen, uint32_t *qout, uint32_t round, hipStream_t st);
hipError_t launch_il_bc(const IlArgs &a, double *bc, const int32_t *perm, hipStream_t st);
