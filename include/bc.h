/*
 * bc.h -- C ABI of the MI355X betweenness-centrality library.
 *
 * The library computes betweenness centrality on weighted graphs with
 * Brandes' method as laid out by Fan, Xu & Zhao ("A GPU-Based Solution to
 * Fast Calculation of Betweenness Centrality on Large Weighted Networks"):
 * per source s, a weighted single-source shortest-path pass that records
 * distances d(s,.) and shortest-path counts sigma_s(.) (Sec. 2.2, Sec. 3.1,
 * Alg. 2), then a dependency pass in reverse distance order (Sec. 2.1 recursion,
 * Alg. 3) whose values are added to the centrality of every vertex other
 * than s.
 *
 *   BC_S(v) = sum over s in S, s != v, of delta_s(v)
 *           = sum over s in S and t != s, v, of sigma_st(v) / sigma_st
 *
 * (Sec. 2.1, Eq. 1, restricted to a source multiset S; ordered pairs, no
 * normalisation).  With S = all vertices this is Eq. 1 exactly.
 *
 * Conventions shared by every entry point
 *   - Every call returns a bc_status; no C++ exception crosses the ABI.  On
 *     failure bc_last_error() describes the cause (thread-local string, valid
 *     until the next call on the same thread).
 *   - Out-parameters are written only when the call returns BC_OK.
 *   - Host pointers are read during the call only and stay owned by the
 *     caller.  Device pointers must point to memory of the current HIP
 *     device, allocated by the caller, and stay owned by the caller.
 *   - Handles (bc_graph, bc_result) are owned by the library and released
 *     only by the matching destroy call.  A graph handle must not be used by
 *     two threads at once.
 *   - Numeric types: distances int32 (INT32_MAX marks "unreachable"),
 *     path counts uint64 (an overflow is an error, never a wrap),
 *     dependencies and centralities IEEE double.
 */
#ifndef BC_H
#define BC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    BC_OK = 0,
    BC_E_INVAL = 1,          /* bad argument: null pointer, negative size, source out of range */
    BC_E_GRAPH = 2,          /* malformed CSR, or an undirected graph whose arcs are not symmetric */
    BC_E_WEIGHT = 3,         /* an arc weight below 1 */
    BC_E_DIST_OVERFLOW = 4,  /* (n-1) * max weight does not fit below INT32_MAX */
    BC_E_SIGMA_OVERFLOW = 5, /* a shortest-path count exceeded 2^64 - 1 */
    BC_E_NOMEM = 6,          /* device or host allocation failed */
    BC_E_DEVICE = 7,         /* HIP runtime error, or no usable GPU */
    BC_E_BUSY = 8,           /* request refused (server queue full / not admissible) */
    BC_E_TIMEOUT = 9,        /* wait deadline passed */
    BC_E_INTERNAL = 10       /* an internal safety bound tripped; results are not valid */
} bc_status;

/* bc_create_graph flags */
#define BC_DIRECTED 1u   /* arcs are one-way; without it every arc must have a reverse arc
                            of equal weight (checked) */
#define BC_KEEP_ORDER 2u /* keep the caller's vertex numbering on the device; by default a
                            graph whose in-degrees are skewed is renumbered internally by
                            decreasing in-degree (results are always in the caller's ids) */
#define BC_EDGE_BC 4u    /* prepare edge betweenness (bc_compute_edges*): a 4-byte map per
                            arc is kept on the device */

typedef struct bc_graph bc_graph;
typedef struct bc_result bc_result;

/*
 * bc_create_graph -- copy a weighted graph to the device.
 *
 * The graph is given in CSR form plus a parallel weight array (Sec. 3.1):
 * row_ptr[n+1] (int64, row_ptr[0] = 0, non-decreasing, row_ptr[n] = nnz),
 * col[nnz] (arc heads, 0 <= col < n) and w[nnz] (integer weights >= 1).
 * Row v lists the arcs leaving v.  Without BC_DIRECTED the graph is
 * undirected (Sec. 2.1): every arc (u, v, w) must have the reverse arc
 * (v, u, w), which is verified.  Parallel arcs are distinct paths; self-loops
 * are allowed and never lie on a shortest path.
 *
 * Errors: BC_E_INVAL (n < 1, nnz < 0, null pointer, nnz >= 2^32 - 1),
 * BC_E_GRAPH, BC_E_WEIGHT, BC_E_DIST_OVERFLOW, BC_E_NOMEM, BC_E_DEVICE.
 * The host arrays are copied; *out receives a new handle.
 */
bc_status bc_create_graph(int32_t n, int64_t nnz, const int64_t *row_ptr, const int32_t *col,
                          const int32_t *w, uint32_t flags, bc_graph **out);

/*
 * bc_create_graph_device -- bc_create_graph for a CSR already in device memory
 * (for example the data pointers of torch tensors).
 *
 * row_ptr_dev[n+1] (int64), col_dev[nnz] and w_dev[nnz] (int32) are device
 * arrays of the current device with the meaning and rules of bc_create_graph
 * (CSR plus a parallel weight array, Sec. 3.1; undirected graphs must be
 * symmetric, Sec. 2.1).  Validation, renumbering, packing, the transpose of a
 * directed graph and the symmetry check of an undirected one all run on the
 * device, on `stream` (a hipStream_t; NULL = the new graph's own stream), so
 * the work is ordered after whatever the caller queued there before.  The
 * resulting graph has the same device layout as bc_create_graph builds from
 * the same arrays.  The arrays are only read, stay owned by the caller and may
 * be reused once the call returns (it waits for its device work).
 *
 * Errors: as bc_create_graph (BC_E_GRAPH, BC_E_WEIGHT and BC_E_DIST_OVERFLOW
 * come from the device checks, with the first offending row or arc named in
 * bc_last_error).  Temporary device memory of about 40 bytes per arc is used
 * during the call.
 */
bc_status bc_create_graph_device(int32_t n, int64_t nnz, const int64_t *row_ptr_dev,
                                 const int32_t *col_dev, const int32_t *w_dev, uint32_t flags,
                                 void *stream, bc_graph **out);

/* Release a graph and every device buffer cached on it.  NULL is accepted.
   BC_E_BUSY (nothing released) while a live server holds the graph: a server
   holds every graph submitted to it until bc_server_destroy. */
bc_status bc_destroy_graph(bc_graph *g);

typedef struct {
    int32_t n;
    int64_t nnz;
    int32_t directed;
    int32_t w_max;
    int32_t max_out_degree;
    int32_t packed_arcs; /* 1 when arc head and weight share one 32-bit word on the device */
    int32_t renumbered;  /* 1 when the device numbering is by decreasing in-degree */
    int64_t device_bytes; /* graph bytes resident on the device */
    /* the autotuner's cached choice (bc_options.autotune); 0 fields before it ran */
    int32_t tuned;        /* 1 once a call with autotune set has tuned this graph */
    int32_t tuned_delta, tuned_wg_threads, tuned_lane_max_deg, tuned_dep_mode;
    int32_t tuned_expand_lane_deg, tuned_wave_max_deg, tuned_wg_min_deg;
    int32_t tuned_batch;  /* sources in flight; 0 = the full occupancy of the workgroup size */
    int32_t tuned_lds_bits; /* width of the LDS distance entries */
    int64_t tuning_trials; /* candidate settings timed on this graph so far */
} bc_graph_info;

bc_status bc_get_graph_info(const bc_graph *g, bc_graph_info *info);

/* Execution forms. */
typedef enum {
    BC_MODE_AUTO = 0,    /* batched */
    BC_MODE_BATCHED = 1, /* many sources in flight, one workgroup and one state slab per source,
                            one persistent launch (coarse-grained source parallelism, Sec. 3.1) */
    BC_MODE_PLAIN = 2,   /* one source at a time on the whole GPU, phase by phase */
    BC_MODE_INTERLEAVED = 3 /* sources in groups of 64 sharing one wavefront, one lane per
                               source, the state of a group laid out [vertex][source] so that
                               an arc read serves all 64 sources; rounds over queues of
                               (group, vertex) entries, as many groups per sweep as 60% of the
                               free device memory (at most 160 GiB) holds, or batch
                               sources (rounded up to a multiple of 64) when batch > 0;
                               lane and workgroup options do not apply; edge
                               betweenness and bc_source_state need the other forms
                               (BC_E_INVAL) */
} bc_mode;

/*
 * Options.  A zero field selects the default (or the autotuned value when
 * autotune is set).  The result never depends on the options beyond
 * floating-point summation order.
 */
typedef struct {
    int32_t mode;         /* bc_mode */
    int32_t batch;        /* batched: sources in flight (state slabs); 0 = fill the GPU;
                             interleaved: at most this many sources per sweep */
    int32_t delta;        /* near-far band width in weight units (>= 1); 0 = heuristic (the
                             interleaved form: at least 4 times the maximum weight) */
    int32_t lane_max_deg; /* count and dependency passes: vertices with at most this many
                             in-arcs (recorded predecessors) are handled by one lane, larger
                             ones by a whole 64-lane wave */
    int32_t wg_threads;   /* batched: threads per workgroup (256, 512 or 1024); with batch
                             set, a CU's LDS is shared only by the workgroups those
                             sources need */
    int32_t autotune;     /* 1 = time candidate settings once per graph and keep the best:
                             band width, workgroup size, dependency method, lane_max_deg,
                             the expansion degree tiers and the sources in flight, each
                             unless set here, on a prefix of the source list (batched
                             form); later calls reuse the choice (bc_get_graph_info) */
    int32_t accumulate;   /* 0 = default, 1 = per-slot partial sums + reduction,
                             2 = device-wide FP64 atomic adds into the output */
    int32_t lds_vertices; /* batched: distances of this many highest in-degree vertices are
                             kept in LDS per source; 0 = as many as fit, -1 = none */
    int32_t dep_mode;     /* batched dependency pass: 0 = default (1), 1 = push along the
                             shortest-path DAG recorded by the count pass, band by band in
                             reverse and in Kahn's order inside a band, 2 = pull over
                             out-arcs band by band in reverse */
    int32_t virtual_warp; /* frontier expansion: 0 = by degree, one lane per vertex up to 8
                             arcs, a group of 16 lanes up to 64, a whole wave above (and in
                             the batched form the whole workgroup above 512);
                             1, 2, 4, ..., 64 = a fixed group of that many lanes per vertex
                             (the warp-centric mapping of Sec. 3.4) */
    int32_t node_parallel;/* batched frontier expansion: 0 = over the queue (work-efficient,
                             Sec. 3.3); 1 = over every vertex, expanding those queued
                             (node-parallel, Alg. 2) -- for comparison only */
    int32_t lds_bits;     /* batched: width of the LDS distance entries: 0 = auto (16 for
                             graphs renumbered by in-degree, else 32), 8, 16 or 32.  With 16 the
                             cache holds twice the vertices; distances of 65535 and more of
                             those vertices are kept in device memory instead.  With 8 (packed
                             arcs; else 16 is used) it holds four times the vertices, each as
                             an offset into a 253-wide window that follows the bands: settled
                             vertices below the window and values beyond it are kept in
                             device memory.  Suits graphs whose arc weights are about the
                             window's width or less */
    /* Degree tiers of the adaptive frontier expansion (virtual_warp = 0; the
       degree-aware thread mapping of Sec. 3.4 on 64-lane wavefronts).  A queued
       vertex with d out-arcs is expanded by one lane if d <= expand_lane_deg, by a
       group of 16 lanes if d <= wave_max_deg, else by one whole wave; in the
       batched form a vertex with d > wg_min_deg is expanded by the whole
       workgroup after the pass.  The count pass hands vertices with more than
       wave_max_deg in-arcs to a whole wave.  0 = default (8, 64, 512); a
       threshold below the one before it is raised to it.  The plain form has no
       workgroup tier; the interleaved form uses none of them. */
    int32_t expand_lane_deg;
    int32_t wave_max_deg;
    int32_t wg_min_deg;
    int32_t far_buckets;  /* batched: how far values wait for their band (the near-far
                             split of Sec. 3.2's phases).  1 = a ring of buckets of width
                             delta, one per future band up to the maximum weight (at most
                             128), each vertex entering a bucket only when its tentative
                             distance drops into a lower one, so a band takes just its own
                             bucket; bands are then aligned to multiples of delta.
                             2 = a two-tier pile (values within 16 band widths, then the
                             rest), rescanned at every band change.  0 = the ring when the
                             maximum weight spans at least 16 band widths, else the pile.
                             The ring needs head and weight packed in one arc word
                             (bc_graph_info.packed_arcs), fewer than 2^30 vertices and
                             fewer than 2^30 bands up to (n - 1) times the maximum
                             weight; other graphs keep the pile */
    void *stream;         /* hipStream_t to run on; NULL = the graph's own stream */
} bc_options;

typedef struct {
    double ms;                /* device time of the computation (HIP events) */
    int64_t sources;          /* k */
    int64_t reached;          /* sum over sources of reached vertices (n_R) */
    int64_t arcs_out_reached; /* sum over sources of arcs leaving reached vertices (A_R) */
    int64_t dag_arcs;         /* sum over sources of shortest-path DAG arcs (E_D) */
    int64_t improvements;     /* successful distance decreases (relaxation work) */
    int64_t bands;            /* near-far bands (distance buckets) */
    int64_t iterations;       /* frontier expansion steps */
    int64_t sigma_rounds;     /* path-count rounds over band members */
    int64_t delta_rounds;     /* dependency rounds over band members */
    int64_t first_bad_source; /* smallest source-list index whose counts overflowed, else -1 */
    double algo_bytes;        /* algorithmic bytes of the work (see bc_algo_bytes) */
    double kernel_ms;         /* device time of the main kernel launches alone (HIP events) */
    int64_t kernel_launches;  /* number of main kernel launches timed in kernel_ms */
    int64_t phase_ticks[5];   /* batched form: device clock ticks summed over workgroups spent
                                 in initialisation, frontier expansion, count rounds,
                                 dependency rounds and far-pile splits */
    /* the settings the computation ran with (defaults and autotuned values filled in) */
    int32_t mode, batch, delta, lane_max_deg, wg_threads, accumulate, lds_vertices, dep_mode,
        virtual_warp, node_parallel, lds_bits, expand_lane_deg, wave_max_deg, wg_min_deg,
        far_buckets; /* far_buckets: 1 ring, 2 pile (batched form), 0 other forms */
} bc_stats;

/*
 * bc_compute -- betweenness over a multiset of sources.
 *
 * sources[k] (host, int32) lists the sources; NULL with k = n means all
 * vertices 0..n-1 (exact Eq. 1).  Repeated sources count once per
 * occurrence; k = 0 gives an all-zero result.  The result is the unscaled
 * sum of the listed sources' dependencies.  Runs on opt->stream (or the
 * graph's stream) and returns after the result is complete.
 *
 * Errors: BC_E_INVAL (source out of range, k < 0), BC_E_SIGMA_OVERFLOW (the
 * result handle is still not produced; bc_last_error names the first
 * failing source index), BC_E_NOMEM, BC_E_DEVICE, BC_E_INTERNAL.
 */
bc_status bc_compute(bc_graph *g, const int32_t *sources, int64_t k, const bc_options *opt,
                     bc_result **out);

/*
 * bc_compute_device -- as bc_compute, for data already on the device.
 *
 * sources_dev[k] is a device int32 array; bc_dev[n] is a device double array
 * that receives the result (overwritten).  Sources are range-checked on the
 * device; an out-of-range entry yields BC_E_INVAL (bc_dev is then not valid).  The call enqueues the work on
 * opt->stream (or the graph's stream) and waits for it; stats may be NULL.
 * No host<->device transfer of inputs or outputs takes place.
 */
bc_status bc_compute_device(bc_graph *g, const int32_t *sources_dev, int64_t k,
                            const bc_options *opt, double *bc_dev, bc_stats *stats);

/*
 * bc_compute_device_noalloc -- as bc_compute_device in the batched form, for
 * callers that cannot allocate device memory during the call (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc).  It
 * calls no hipMalloc, hipFree or other allocating routine: the per-source
 * state slabs live in a fixed device array of BC_NOALLOC_SCRATCH_BYTES that
 * each GPU holds from the library's load until the process ends.  The
 * caller still provides sources_dev[k] and bc_dev[n] (device memory).
 *
 * Sources in flight are capped by how many state slabs fit in the array; a
 * graph whose single slab (about 84 bytes per vertex plus 4 per arc) does not
 * fit gives BC_E_NOMEM and leaves bc_dev untouched.  Only the batched form
 * runs here: opt->mode other than BC_MODE_AUTO / BC_MODE_BATCHED, or
 * opt->autotune set, gives BC_E_INVAL.  Every call on one GPU shares that
 * GPU's array and resets the slabs it uses; calls that overlap on one GPU (from
 * any thread or stream) race and must be serialised by the caller.  Other
 * errors as bc_compute_device.
 */
#define BC_NOALLOC_SCRATCH_BYTES (64ull << 20)
bc_status bc_compute_device_noalloc(bc_graph *g, const int32_t *sources_dev, int64_t k,
                                    const bc_options *opt, double *bc_dev, bc_stats *stats);

/*
 * Edge betweenness (the paper's tool reports node and edge BC, Sec. 1): for
 * every arc e = (v, u) of the caller's CSR, ebc[e] = sum over the listed
 * sources s and all targets t of sigma_st(e) / sigma_st, where sigma_st(e)
 * counts the shortest s-t paths that use the arc; equivalently the sum over s
 * of sigma_sv / sigma_su * (1 + delta_s(u)) when e lies on a shortest path
 * from s.  For an undirected graph the two arcs of an edge are reported
 * separately (their sum is the edge's value).  Node centralities are returned
 * as well.  The graph must have been created with BC_EDGE_BC; the batched form
 * is used (BC_E_INVAL for BC_MODE_PLAIN), with the recorded-DAG dependency pass.
 *
 * bc_compute_edges: host source list (NULL with k = n for all vertices), host
 * outputs bc_host[n] (may be NULL) and ebc_host[nnz].
 * bc_compute_edges_device: device source list and device outputs bc_dev[n],
 * ebc_dev[nnz]; stats may be NULL.
 */
bc_status bc_compute_edges(bc_graph *g, const int32_t *sources, int64_t k, const bc_options *opt,
                           double *bc_host, double *ebc_host);
bc_status bc_compute_edges_device(bc_graph *g, const int32_t *sources_dev, int64_t k,
                                  const bc_options *opt, double *bc_dev, double *ebc_dev,
                                  bc_stats *stats);

/* Copy a result's centralities to host memory bc_host[n]. */
bc_status bc_result_bc(const bc_result *r, double *bc_host);
/* Device pointer to a result's centralities (double[n], owned by the result). */
bc_status bc_result_device_ptr(const bc_result *r, const double **bc_dev);
bc_status bc_result_stats(const bc_result *r, bc_stats *stats);
bc_status bc_destroy_result(bc_result *r);

/*
 * bc_source_state -- full per-vertex state of one source, for checking.
 *
 * Runs source s alone with the given options (batched or plain form; batch
 * and autotune are ignored) and copies to host arrays of n elements, in the
 * caller's vertex ids:
 *   d[v]     -- the shortest distance d(s, v) of the forward pass (Sec. 2.2;
 *               Alg. 1 initialises it, Alg. 2 relaxes it), INT32_MAX when v
 *               is unreachable;
 *   sigma[v] -- the number of shortest s-v paths, counted by Alg. 2's rule
 *               (a strictly shorter distance replaces the count, an equal one
 *               adds to it), 0 when unreachable;
 *   delta[v] -- the dependency delta_s(v) of the Sec. 2.1 recursion as Alg. 3
 *               accumulates it, 0 when unreachable; delta_s(s) equals the
 *               number of reached vertices minus one.
 * Any output pointer may be NULL.  Errors: BC_E_INVAL (null graph, s out of
 * range, BC_MODE_INTERLEAVED), BC_E_SIGMA_OVERFLOW, BC_E_NOMEM, BC_E_DEVICE;
 * the outputs are then not written.
 */
bc_status bc_source_state(bc_graph *g, int32_t s, const bc_options *opt, int32_t *d,
                          uint64_t *sigma, double *delta);

/*
 * bc_update_arc_device -- centralities after one arc changes (dynamic BC, the
 * extension Sec. 5 leaves to future work).
 *
 * The change: the arc tail -> head had weight w_old (0: absent) and has
 * weight w_new (0: removed); w_old != w_new, both >= 0.  For an undirected
 * graph the edge {tail, head} changes, i.e. both of its arcs.  g_old and
 * g_new are the graph before and after (caller-created, same n and
 * directedness, differing in that arc only: checked through n, directedness
 * and nnz, otherwise the caller's responsibility).  g_rev is g_old with every
 * arc reversed, for a directed graph; it must be NULL for an undirected one.
 *
 * bc_dev[n] (device) holds the centralities of g_old over all sources (as
 * bc_compute_device with every vertex as a source) and receives those of
 * g_new.  Only the affected sources are run again, once on each graph: a
 * source s is affected when, with the distances before the change, the arc
 * was on a shortest path from s (dist(s,tail) + w_old = dist(s,head)) or lies
 * on or shortens one after it (dist(s,tail) + w_new <= dist(s,head)), for
 * either arc of an undirected edge.  Every other source keeps its distances
 * and shortest-path DAG, hence its dependencies.  dist(s, tail) and
 * dist(s, head) come from two single-source passes on the reversed graph
 * (g_rev, or g_old when undirected); a self-loop change affects no source.
 * When more than half of the sources are affected, every source of g_new is
 * run instead (n source passes rather than 2 x affected) and bc_dev is
 * overwritten with that result.
 *
 * affected_dev (device int32[n], may be NULL) receives the affected sources
 * in no particular order; *affected (may be NULL) their number.  Rounding:
 * otherwise bc_dev[v] gains (sum after - sum before) over the affected
 * sources, so its error is relative to the larger of the old and new
 * centrality.  Runs on
 * opt->stream (or the graphs' streams) and returns when bc_dev is complete.
 *
 * Errors: BC_E_INVAL (null graph or output, graphs that do not match, arc out
 * of range, no change in weight, missing or superfluous g_rev), otherwise as
 * bc_compute_device (bc_dev is then not valid).
 */
bc_status bc_update_arc_device(bc_graph *g_old, bc_graph *g_new, bc_graph *g_rev,
                               int32_t tail, int32_t head, int32_t w_old, int32_t w_new,
                               const bc_options *opt, double *bc_dev, int32_t *affected_dev,
                               int64_t *affected);

/*
 * bc_algo_bytes -- the algorithmic HBM bytes of one source's Brandes pass:
 *   arcs * (16 + 2 * weight_bytes) + 72 * reached + 24 * dag_arcs + 20 * n
 * (two passes over the arcs of reached vertices with a 4-byte distance gather
 * each, per-vertex state reads and writes, the count and dependency gathers
 * along shortest-path DAG arcs, and the per-source initialisation).
 */
double bc_algo_bytes(int32_t n, int32_t weight_bytes, int64_t arcs, int64_t reached,
                     int64_t dag_arcs);

/* ------------------------------------------------------------------------
 * Serving: a request loop with continuous batching.
 *
 * The server owns one scheduler thread and all device work of its requests.
 * Graphs are caller-owned bc_graph handles that stay resident; per graph the
 * server keeps a few sweep contexts (state slabs, a stream).  A sweep is one
 * bounded launch of the batched form over sources taken from the admitted
 * requests of that graph, oldest request first, each source adding its
 * dependencies into its own request's result (FP64 atomics).  A request that
 * arrives while others run is admitted, first come first served, as soon as
 * the free device memory and the server's result budget allow its result
 * buffer (8 n bytes), and its sources join the next sweep of its graph.
 * Results equal bc_compute over the same sources up to floating-point
 * summation order.  A failing source (path-count overflow) fails only its own
 * request.
 * ------------------------------------------------------------------------ */
typedef struct bc_server bc_server;

typedef struct {
    int64_t result_budget_bytes;  /* device bytes that admitted, unretrieved results may hold;
                                     0 = a quarter of the free memory at creation */
    int64_t slab_bytes_per_sweep; /* state-slab memory of one sweep context; 0 = 1/16 of the
                                     free memory at creation */
    int32_t max_active;           /* admitted, unfinished requests; 0 = 64 */
    int32_t sweeps_per_graph;     /* concurrent sweeps per graph; 0 = 4 (with the default
                                     slots, one graph can then fill the GPU when alone) */
    int32_t slots_per_sweep;      /* sources in flight per sweep; 0 = a quarter of the GPU's
                                     resident workgroups, within the slab memory */
    int32_t items_per_sweep;      /* sources per sweep; 0 = the slots (each workgroup takes one
                                     source, so a sweep ends after about one source's time
                                     and frees its compute units for other sweeps) */
    bc_options compute;           /* delta, lane_max_deg and wg_threads of the sweeps; 0 fields
                                     take the graph's autotuned (else default) values; mode,
                                     batch, accumulate and stream are ignored */
    int32_t order;                /* which admitted request of a graph a free sweep serves
                                     first: 0 = the oldest; 1 = the one with the fewest
                                     sources left (short requests overtake long ones) */
    int32_t graph_order;          /* which graph's sweep starts first when several wait:
                                     0 = the graph of the oldest admitted request; 1 = the
                                     graph whose best request has the least work left
                                     (sources left x (n + arcs)) */
    double gpu_share;             /* share of the GPU's resident workgroups that the sweeps in
                                     flight may hold together (a sweep holds its slots); a
                                     sweep beyond it waits for one to end instead of queueing
                                     on the device behind running workgroups; 0 = 1.0,
                                     negative = no bound */
    double starve_after_s;        /* a request waiting this many seconds since its arrival is
                                     served before all younger ones (oldest first), in both
                                     orders above; bounds how long short requests can hold a
                                     long one back; 0 = never */
} bc_server_opts;

typedef struct {
    int64_t submitted, completed, failed, waiting, active;
    double p50_ms, p99_ms, mean_ms, max_ms; /* arrival -> completion of completed requests */
    double queue_ms_sum;                    /* total arrival -> admission time */
    double gteps;          /* sum of k*m over retrieved requests / (last completion - first
                              arrival) */
    int64_t sweeps;        /* sweep launches so far */
    int64_t device_bytes_in_use; /* result bytes held by admitted, unretrieved requests */
} bc_server_stats;

/* Start a server on the current device (opts may be NULL for defaults). */
bc_status bc_server_create(const bc_server_opts *opts, bc_server **out);
/*
 * Queue a request: betweenness of graph g over sources[k] (host array, copied;
 * k = 0 allowed).  Returns at once with a ticket.  BC_E_BUSY if the result can
 * never fit the server's budget; BC_E_INVAL for out-of-range sources.  From
 * its first request on, the server holds g (bc_destroy_graph returns BC_E_BUSY)
 * until bc_server_destroy.  If the device memory for g's sweep state cannot be
 * found, the requests of g waiting for a sweep fail with BC_E_NOMEM (returned
 * by bc_server_wait) and the server goes on with the other graphs.
 */
bc_status bc_server_submit(bc_server *sv, bc_graph *g, const int32_t *sources, int64_t k,
                           uint64_t *ticket);
/*
 * Wait for a request (timeout_us < 0 waits forever) and take its result; the
 * result handle owns the device buffer (release with bc_destroy_result) and its
 * stats report ms = arrival-to-completion latency.  BC_E_TIMEOUT leaves the
 * request queued; a failed request returns its error and is discarded.
 */
bc_status bc_server_wait(bc_server *sv, uint64_t ticket, int64_t timeout_us, bc_result **out);
bc_status bc_server_get_stats(bc_server *sv, bc_server_stats *stats);
/* Stop the scheduler after the sweeps in flight, free every unretrieved result. */
bc_status bc_server_destroy(bc_server *sv);

const char *bc_last_error(void);

/* Library version string. */
const char *bc_version(void);

#ifdef __cplusplus
}
#endif

#endif /* BC_H */
