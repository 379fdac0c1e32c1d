// bc_internal.h -- host-side objects behind the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <new>
#include <stdexcept>
#include <string>

#include "../../include/bc.h"
#include "kernels.h"
#include "interleaved.h"

struct bc_error {
    bc_status status;
    std::string msg;
    bc_error(bc_status s, const char *fmt, ...) __attribute__((format(printf, 3, 4)));
};

void hip_check(hipError_t e, const char *what);
void bc_set_last_error(const std::string &msg);
// Sets the thread's last-error message from e and returns its status.
bc_status bc_fail(const bc_error &e);

// Runs f, turning any exception into a status (no exception crosses the C ABI).
template <class F> bc_status bc_guarded(F &&f)
{
    try {
        bc_set_last_error(std::string());
        f();
        return BC_OK;
    } catch (const bc_error &e) {
        return bc_fail(e);
    } catch (const std::bad_alloc &) {
        bc_set_last_error("host allocation failed");
        return BC_E_NOMEM;
    } catch (const std::exception &e) {
        bc_set_last_error(e.what());
        return BC_E_INTERNAL;
    } catch (...) {
        bc_set_last_error("unknown failure");
        return BC_E_INTERNAL;
    }
}

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() { release(); }
    void alloc(size_t n);
    void release();
};

// Device counters of one computation (one block per graph).
struct DevCounters {
    unsigned long long next_src;
    unsigned long long err[2];
    unsigned long long pad;
    DevStats stats;
};

struct Workspace {
    DevBuf base;
    SlabLayout L{};
    int nslabs = 0;
};

struct ResolvedOptions {
    int mode = BC_MODE_BATCHED;
    int batch = 1;
    int delta = 1;
    int lane_max = 32;
    int wg_threads = 256;
    int accumulate = 1;
    int autotune = 0;
    int lds_vertices = 0; // H: distances kept in LDS per source
    int lds_bits = 32;    // width of an LDS distance entry (8, 16 or 32)
    int dep_mode = 1;     // 1 recorded DAG (Kahn), 2 band pulls
    int vw = 0;           // expansion lanes per vertex (0 adaptive)
    int lane_deg = BC_DEF_LANE_DEG; // adaptive expansion: one lane up to this many arcs,
    int wave_deg = BC_DEF_WAVE_DEG; // a group of lanes up to this many, a wave above,
    int wg_deg = BC_HUB_DEG;        // the whole workgroup above this (batched form)
    int node_parallel = 0;
    int far_buckets = 0;  // batched: 0 auto, 1 far-bucket ring, 2 two-tier pile
    int il_groups = 0;    // interleaved form: groups of 64 sources per sweep (0 = by memory)
    hipStream_t stream = nullptr;
};

struct TunedOptions {
    bool valid = false;
    int delta = 0, lane_max = 0, wg_threads = 0, dep_mode = 0;
    int lane_deg = 0, wave_deg = 0, wg_deg = 0;
    int batch = 0; // sources in flight (0 = the full occupancy of wg_threads)
    int lds_bits = 0;
    double best_ms_per_source = 0.0;
};

struct bc_graph {
    int32_t n = 0;
    int64_t nnz = 0;
    bool directed = false;
    int32_t wmax = 1;
    int32_t maxdeg = 0;
    int32_t n_act = 0; // vertices from here on have no in-arcs (see DevGraph)
    int wbytes = 1;
    double avg_deg = 0.0, wmean = 1.0;
    bool packed = false;
    bool renumbered = false; // device ids are by decreasing in-degree
    uint32_t wshift = 0, wmask = 0;
    int device = 0;
    int num_cus = 1;
    hipStream_t stream = nullptr;
    hipEvent_t ev_k0 = nullptr, ev_k1 = nullptr; // around the main kernel launch

    DevBuf row, arc, wt;    // out-arcs
    DevBuf trow, tarc, twt; // in-arcs (directed graphs only)
    DevBuf perm, iperm;     // internal -> caller id, caller -> internal id (when renumbered)
    DevBuf emap;            // in-row position -> caller arc index (edge betweenness)
    bool edges_ready = false;
    std::vector<int32_t> host_iperm;
    DevBuf ctl;             // DevCounters
    DevBuf plain_ctl;       // PlainCtl
    DevBuf src_buf;         // uploaded source lists
    DevCounters *host_counters = nullptr;
    PlainCtl *host_plain = nullptr;
    bool plain_ctl_ready = false;
    long long plain_gen_hint = 0;
    // captured sweep of the plain form: PLAIN_GRAPH_PAIRS (step, control) pairs
    hipGraphExec_t plain_exec = nullptr;
    uint32_t plain_exec_delta = 0;
    int plain_exec_lane_max = 0;
    int plain_exec_vw = 0;
    uint64_t plain_exec_tiers = 0;
    const void *plain_exec_slab = nullptr;

    Workspace batched, plain;
    TunedOptions tuned;
    int64_t tune_trials = 0; // timed autotuner candidates so far
    std::atomic<int> server_refs{0}; // live servers that hold this graph
    bool last_stats_valid = false;
    bc_stats last_stats{};

    DevGraph view() const;
    const int32_t *perm_dev() const { return renumbered ? (const int32_t *)perm.p : nullptr; }
    const int32_t *iperm_dev() const { return renumbered ? (const int32_t *)iperm.p : nullptr; }
    int32_t internal_id(int32_t v) const { return renumbered ? host_iperm[(size_t)v] : v; }
    ~bc_graph();
};

struct bc_result {
    int32_t n = 0;
    DevBuf bc;
    bc_stats stats{};
};

SlabLayout slab_layout(int32_t n, int64_t pred_slots);
int default_delta(const bc_graph *g);
// Width of the LDS distance entries for a requested width (0 = by graph).
int lds_bits_for(const bc_graph *g, int requested);
// LDS-resident distances per source and the matching workgroups per CU.
// want_slabs > 0: the caller fixed the sources in flight, so no more workgroups
// than those need share a CU's LDS.
void batched_lds_plan(const bc_graph *g, int nt, bool atomic_bc, int requested, int bits,
                      int &H, int &per_cu, int64_t want_slabs = 0);
ResolvedOptions resolve_options(bc_graph *g, const bc_options *opt, int64_t k);
// Most state slabs a batched launch may use (60% of the free device memory,
// at most 65535).
int64_t batch_cap(bc_graph *g);
void compute_device(bc_graph *g, const int32_t *src_dev, const int32_t *src_host, int64_t k,
                    const bc_options *opt, double *bc_dev, bc_stats *stats,
                    double *ebc_dev = nullptr);
void autotune(bc_graph *g, ResolvedOptions &r, const bc_options *opt, const int32_t *src_dev,
              int64_t k);
void reset_device_counters(bc_graph *g, hipStream_t st);
// Device-side ingest behind bc_create_graph_device: validates the caller's
// device CSR and builds g's device layout on stream st (g's runtime fields,
// stream and counters already set up).
void create_graph_device(int32_t n, int64_t nnz, const int64_t *row_ptr, const int32_t *col,
                         const int32_t *w, uint32_t flags, hipStream_t st, bc_graph *g);
// Sets g->n_act from g's device in-row offsets (the last step of both
// ingest paths; waits for stream st).
void set_inarc_bound(bc_graph *g, hipStream_t st);
// Far-bucket ring of a batched launch with band width r.delta: whether it is
// used, and its number of buckets.
void bucket_plan(const bc_graph *g, const ResolvedOptions &r, int &buckets, int &nbk);
// Degree-tier fields of the batched kernel's arguments.
void set_tier_args(const bc_graph *g, int lane_deg, int wave_deg, int wg_deg, BatchArgs &a);
void read_device_counters(bc_graph *g, hipStream_t st, DevCounters &out);
// Status of a finished computation from its device counters (throws on an
// out-of-range source, a tripped iteration bound or a count overflow).
void check_device_errors(const DevCounters &c);
// Statistics of a finished computation (st may be NULL).
void fill_stats(bc_graph *g, const ResolvedOptions &r, const DevCounters &c, int64_t k,
                double ms, double kernel_ms, int64_t launches, bc_stats *st);
// Source-interleaved form: groups of 64 sources per sweep for n vertices, nnz
// arcs, k sources and the given free device bytes (0: not even one fits).
int interleaved_groups_per_sweep(int32_t n, int64_t nnz, int64_t k, size_t free_bytes);
void run_interleaved(bc_graph *g, const ResolvedOptions &r, const int32_t *src_dev, int64_t k,
                     double *bc_dev, DevCounters &cnt, float &ms);
// One launch of the batched kernel over nslabs slabs at slab_base (reset,
// layout L) plus the reduction of their partial sums, with g->ev_k0/ev_k1
// recorded around the kernel; counters reset and outputs cleared by the caller.
void launch_batched_pass(bc_graph *g, const ResolvedOptions &r, const int32_t *src_dev,
                         int64_t k, double *bc_dev, char *slab_base, const SlabLayout &L,
                         int nslabs, double *ebc_dev, hipStream_t st);
void run_batched(bc_graph *g, const ResolvedOptions &r, const int32_t *src_dev, int64_t k,
                 double *bc_dev, DevCounters &cnt, float &ms, float *kernel_ms,
                 double *ebc_dev = nullptr);
