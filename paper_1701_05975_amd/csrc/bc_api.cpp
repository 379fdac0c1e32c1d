// bc_api.cpp -- host runtime behind the C ABI declared in include/bc.h.
//
// Graph ingest (CSR validation, symmetric check, transpose for directed
// graphs, arc packing, upload), per-graph workspaces (state slabs, counters),
// the batched and plain drivers, results and error reporting.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/bc.h"
#include "bc_internal.h"
#include "kernels.h"

// ---------------------------------------------------------------------------
// Errors
// ---------------------------------------------------------------------------
static thread_local std::string g_last_error;

bc_error::bc_error(bc_status s, const char *fmt, ...) : status(s)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    msg = buf;
}

void hip_check(hipError_t e, const char *what)
{
    if (e == hipSuccess)
        return;
    bc_status s = (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) ? BC_E_NOMEM
                                                                               : BC_E_DEVICE;
    (void)hipGetLastError(); // clear the non-sticky error state
    throw bc_error(s, "%s: %s", what, hipGetErrorString(e));
}

void bc_set_last_error(const std::string &msg) { g_last_error = msg; }

bc_status bc_fail(const bc_error &e)
{
    g_last_error = e.msg;
    return e.status;
}

template <class F> static bc_status guarded(F &&f) { return bc_guarded(std::forward<F>(f)); }

// ---------------------------------------------------------------------------
// Device buffers
// ---------------------------------------------------------------------------
void DevBuf::alloc(size_t n)
{
    release();
    if (n == 0)
        return;
    hip_check(hipMalloc(&p, n), "hipMalloc");
    bytes = n;
}

void DevBuf::release()
{
    if (p)
        (void)hipFree(p);
    p = nullptr;
    bytes = 0;
}

static void ensure_device()
{
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count < 1) {
        (void)hipGetLastError();
        throw bc_error(BC_E_DEVICE, "no HIP device available");
    }
}

static int bit_width_u64(uint64_t x)
{
    int b = 0;
    while (x) {
        ++b;
        x >>= 1;
    }
    return b;
}

// ---------------------------------------------------------------------------
// Graph ingest
// ---------------------------------------------------------------------------
static void build_transpose(int32_t n, const int64_t *row_ptr, const int32_t *col,
                            const int32_t *w, std::vector<int64_t> &trow,
                            std::vector<int32_t> &tcol, std::vector<int32_t> &tw,
                            std::vector<uint32_t> *tsrc = nullptr)
{
    const int64_t nnz = row_ptr[n];
    trow.assign((size_t)n + 1, 0);
    for (int64_t e = 0; e < nnz; ++e)
        trow[(size_t)col[e] + 1]++;
    for (int32_t v = 0; v < n; ++v)
        trow[(size_t)v + 1] += trow[(size_t)v];
    std::vector<int64_t> pos(trow.begin(), trow.end() - 1);
    tcol.resize((size_t)nnz);
    tw.resize((size_t)nnz);
    if (tsrc)
        tsrc->resize((size_t)nnz);
    for (int32_t u = 0; u < n; ++u)
        for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
            const int64_t p = pos[(size_t)col[e]]++;
            tcol[(size_t)p] = u;
            tw[(size_t)p] = w[e];
            if (tsrc)
                (*tsrc)[(size_t)p] = (uint32_t)e; // the arc this in-arc entry stands for
        }
}

// For a symmetric (undirected) CSR: rev[e] = index of the reverse arc of e
// (equal weight); parallel arcs are paired in the order they appear.
static std::vector<uint32_t> reverse_arcs(int32_t n, const int64_t *row_ptr, const int32_t *col,
                                          const int32_t *w)
{
    struct Key {
        int32_t a, b, w;
        uint32_t pos;
        bool operator<(const Key &o) const
        {
            if (a != o.a)
                return a < o.a;
            if (b != o.b)
                return b < o.b;
            if (w != o.w)
                return w < o.w;
            return pos < o.pos;
        }
    };
    const int64_t nnz = row_ptr[n];
    std::vector<Key> fwd((size_t)nnz), bwd((size_t)nnz);
    for (int32_t u = 0; u < n; ++u)
        for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
            fwd[(size_t)e] = Key{u, col[e], w[e], (uint32_t)e};
            bwd[(size_t)e] = Key{col[e], u, w[e], (uint32_t)e};
        }
    std::sort(fwd.begin(), fwd.end());
    std::sort(bwd.begin(), bwd.end());
    std::vector<uint32_t> rev((size_t)nnz);
    for (size_t i = 0; i < fwd.size(); ++i)
        rev[fwd[i].pos] = bwd[i].pos;
    return rev;
}

// Undirected input must list every edge in both directions with one weight:
// row v of the graph and row v of its transpose must be equal multisets.
static bool rows_symmetric(int32_t n, const int64_t *row_ptr, const int32_t *col,
                           const int32_t *w, const std::vector<int64_t> &trow,
                           const std::vector<int32_t> &tcol, const std::vector<int32_t> &tw)
{
    std::vector<uint64_t> a, b;
    for (int32_t v = 0; v < n; ++v) {
        const int64_t b0 = row_ptr[v], b1 = row_ptr[v + 1];
        const int64_t t0 = trow[(size_t)v], t1 = trow[(size_t)v + 1];
        if (b1 - b0 != t1 - t0)
            return false;
        a.clear();
        b.clear();
        for (int64_t e = b0; e < b1; ++e)
            a.push_back(((uint64_t)(uint32_t)col[e] << 32) | (uint32_t)w[e]);
        for (int64_t e = t0; e < t1; ++e)
            b.push_back(((uint64_t)(uint32_t)tcol[(size_t)e] << 32) | (uint32_t)tw[(size_t)e]);
        std::sort(a.begin(), a.end());
        std::sort(b.begin(), b.end());
        if (a != b)
            return false;
    }
    return true;
}

// Device layout of a graph, built on the host before anything touches the
// device: row offsets and packed arcs (out-arcs, and in-arcs for directed
// graphs), the renumbering and the edge map.
struct HostLayout {
    int32_t n = 0;
    int64_t nnz = 0;
    bool directed = false, packed = false, renumbered = false, edges = false;
    int32_t wmax = 1, maxdeg = 0;
    int wbytes = 1;
    uint32_t wshift = 0, wmask = 0;
    double avg_deg = 0.0, wmean = 1.0;
    std::vector<uint32_t> row, arc, trow, tarc;
    std::vector<int32_t> wt, twt; // only when the arcs are not packed
    std::vector<int32_t> perm, iperm;
    std::vector<uint32_t> emap;
};

// Row offsets and arc words of a CSR (head << wshift | weight - 1 when packed).
static void pack_csr(const HostLayout &L, int32_t n, const int64_t *row_ptr, const int32_t *col,
                     const int32_t *w, std::vector<uint32_t> &row, std::vector<uint32_t> &arc,
                     std::vector<int32_t> &wt)
{
    const int64_t nnz = row_ptr[n];
    row.resize((size_t)n + 1);
    for (int32_t v = 0; v <= n; ++v)
        row[(size_t)v] = (uint32_t)row_ptr[v];
    arc.resize((size_t)nnz);
    if (L.packed) {
        for (int64_t e = 0; e < nnz; ++e)
            arc[(size_t)e] = ((uint32_t)col[e] << L.wshift) | ((uint32_t)(w[e] - 1) & L.wmask);
    } else {
        for (int64_t e = 0; e < nnz; ++e)
            arc[(size_t)e] = (uint32_t)col[e];
        wt.assign(w, w + nnz);
    }
}

// Validation and the whole host-side layout (no device call).
static void build_host_layout(int32_t n, int64_t nnz, const int64_t *row_ptr, const int32_t *col,
                              const int32_t *w, uint32_t flags, HostLayout &L)
{
    if (row_ptr[0] != 0 || row_ptr[n] != nnz)
        throw bc_error(BC_E_GRAPH, "row_ptr[0] must be 0 and row_ptr[n] must equal nnz");
    int64_t maxdeg = 0;
    for (int32_t v = 0; v < n; ++v) {
        const int64_t dg = row_ptr[v + 1] - row_ptr[v];
        if (dg < 0)
            throw bc_error(BC_E_GRAPH, "row_ptr decreases at row %d", v);
        maxdeg = std::max(maxdeg, dg);
    }
    int32_t wmax = 1;
    for (int64_t e = 0; e < nnz; ++e) {
        if (col[e] < 0 || col[e] >= n)
            throw bc_error(BC_E_GRAPH, "col[%lld] = %d out of range", (long long)e, col[e]);
        if (w[e] < 1)
            throw bc_error(BC_E_WEIGHT, "w[%lld] = %d is below 1", (long long)e, w[e]);
        wmax = std::max(wmax, w[e]);
    }
    if ((int64_t)(n - 1) * (int64_t)wmax > (int64_t)INT32_MAX - 1)
        throw bc_error(BC_E_DIST_OVERFLOW, "(n-1)*max weight = %lld does not fit in int32",
                       (long long)(n - 1) * wmax);
    const bool directed = (flags & BC_DIRECTED) != 0;

    std::vector<int64_t> trow;
    std::vector<int32_t> tcol, tw;
    build_transpose(n, row_ptr, col, w, trow, tcol, tw);
    if (!directed && !rows_symmetric(n, row_ptr, col, w, trow, tcol, tw))
        throw bc_error(BC_E_GRAPH,
                       "undirected graph is not symmetric (every arc needs a reverse arc of "
                       "equal weight); pass BC_DIRECTED for one-way arcs");

    L.n = n;
    L.nnz = nnz;
    L.directed = directed;
    L.wmax = wmax;
    L.maxdeg = (int32_t)std::min<int64_t>(maxdeg, INT32_MAX);
    const int colbits = bit_width_u64((uint64_t)(n - 1));
    const int wbits = bit_width_u64((uint64_t)(wmax - 1));
    L.packed = colbits + wbits <= 32 && wbits < 32;
    L.wshift = L.packed ? (uint32_t)wbits : 0u;
    L.wmask = L.packed ? (wbits == 0 ? 0u : (uint32_t)((1ull << wbits) - 1)) : 0u;
    L.wbytes = wmax <= 255 ? 1 : (wmax <= 65535 ? 2 : 4);
    int64_t nz_rows = 0;
    for (int32_t v = 0; v < n; ++v)
        nz_rows += row_ptr[v + 1] > row_ptr[v];
    L.avg_deg = nz_rows ? (double)nnz / (double)nz_rows : 0.0;
    double wsum = 0;
    for (int64_t e = 0; e < nnz; ++e)
        wsum += w[e];
    L.wmean = nnz ? wsum / (double)nnz : 1.0;

    // Renumber skewed graphs by decreasing in-degree (ties keep the caller's
    // order): the most frequent arc heads get the lowest ids, whose distances
    // the batched kernel keeps in LDS.
    std::vector<int32_t> order;
    if (!(flags & BC_KEEP_ORDER) && n > 1) {
        std::vector<int64_t> indeg((size_t)n);
        for (int32_t v = 0; v < n; ++v)
            indeg[(size_t)v] = trow[(size_t)v + 1] - trow[(size_t)v];
        std::vector<int64_t> sorted(indeg);
        std::sort(sorted.begin(), sorted.end(), std::greater<int64_t>());
        const int32_t top = std::max<int32_t>(1, n / 100);
        int64_t top_arcs = 0;
        for (int32_t i = 0; i < top; ++i)
            top_arcs += sorted[(size_t)i];
        if (nnz > 0 && (double)top_arcs > 0.05 * (double)nnz) {
            order.resize((size_t)n);
            for (int32_t v = 0; v < n; ++v)
                order[(size_t)v] = v;
            std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
                return indeg[(size_t)a] > indeg[(size_t)b];
            });
        }
    }
    // Device numbering: the caller's or the renumbered one; ce[e] is the
    // caller's index of device arc e (needed only for edge betweenness).
    const bool want_edges = (flags & BC_EDGE_BC) != 0;
    std::vector<int64_t> rrow;
    std::vector<int32_t> rcol, rw;
    std::vector<uint32_t> ce;
    const int64_t *irow = row_ptr;
    const int32_t *icol = col, *iw = w;
    if (!order.empty()) {
        L.renumbered = true;
        L.perm = order;
        L.iperm.assign((size_t)n, 0);
        for (int32_t v = 0; v < n; ++v)
            L.iperm[(size_t)order[(size_t)v]] = v;
        rrow.assign((size_t)n + 1, 0);
        rcol.resize((size_t)nnz);
        rw.resize((size_t)nnz);
        if (want_edges)
            ce.resize((size_t)nnz);
        for (int32_t v = 0; v < n; ++v) {
            const int32_t o = order[(size_t)v];
            int64_t at = rrow[(size_t)v];
            for (int64_t e = row_ptr[o]; e < row_ptr[o + 1]; ++e, ++at) {
                rcol[(size_t)at] = L.iperm[(size_t)col[e]];
                rw[(size_t)at] = w[e];
                if (want_edges)
                    ce[(size_t)at] = (uint32_t)e;
            }
            rrow[(size_t)v + 1] = at;
        }
        irow = rrow.data();
        icol = rcol.data();
        iw = rw.data();
    }
    pack_csr(L, n, irow, icol, iw, L.row, L.arc, L.wt);
    std::vector<uint32_t> tsrc;
    if (directed) {
        if (!order.empty() || want_edges)
            build_transpose(n, irow, icol, iw, trow, tcol, tw, want_edges ? &tsrc : nullptr);
        pack_csr(L, n, trow.data(), tcol.data(), tw.data(), L.trow, L.tarc, L.twt);
    }
    L.edges = want_edges;
    if (want_edges && nnz > 0) {
        // The dependency pass records a DAG arc u -> w at a position p of w's
        // in-row; emap[p] is the caller's index of that arc.
        L.emap.resize((size_t)nnz);
        std::vector<uint32_t> rev;
        if (!directed)
            rev = reverse_arcs(n, irow, icol, iw);
        for (int64_t p = 0; p < nnz; ++p) {
            const uint32_t dev_arc = directed ? tsrc[(size_t)p] : rev[(size_t)p];
            L.emap[(size_t)p] = ce.empty() ? dev_arc : ce[dev_arc];
        }
    }
}

// Argument checks shared by both ingest paths (host and device arrays).
static void check_create_args(int32_t n, int64_t nnz, const void *row_ptr, const void *col,
                              const void *w, uint32_t flags, bc_graph **out)
{
    if (!out)
        throw bc_error(BC_E_INVAL, "out is NULL");
    if (n < 1)
        throw bc_error(BC_E_INVAL, "n must be >= 1 (got %d)", n);
    if (nnz < 0)
        throw bc_error(BC_E_INVAL, "nnz must be >= 0");
    if (nnz >= (int64_t)UINT32_MAX)
        throw bc_error(BC_E_INVAL, "nnz must be below 2^32 - 1");
    if (!row_ptr || (nnz > 0 && (!col || !w)))
        throw bc_error(BC_E_INVAL, "null CSR array");
    const uint32_t known = BC_DIRECTED | BC_KEEP_ORDER | BC_EDGE_BC;
    if (flags & ~known)
        throw bc_error(BC_E_INVAL, "unknown flag bits 0x%x", flags & ~known);
}

// Device, stream, timing events and the per-graph counter blocks.
static void init_graph_runtime(bc_graph *g)
{
    hip_check(hipGetDevice(&g->device), "hipGetDevice");
    hipDeviceProp_t prop;
    hip_check(hipGetDeviceProperties(&prop, g->device), "hipGetDeviceProperties");
    g->num_cus = prop.multiProcessorCount;
    hip_check(hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking), "hipStreamCreate");
    hip_check(hipEventCreate(&g->ev_k0), "hipEventCreate");
    hip_check(hipEventCreate(&g->ev_k1), "hipEventCreate");
    g->ctl.alloc(sizeof(DevCounters));
    g->plain_ctl.alloc(sizeof(PlainCtl));
    hip_check(hipHostMalloc((void **)&g->host_counters, sizeof(DevCounters)), "hipHostMalloc");
    hip_check(hipHostMalloc((void **)&g->host_plain, sizeof(PlainCtl)), "hipHostMalloc");
}

template <class T> static void upload(DevBuf &d, const std::vector<T> &h, const char *what)
{
    if (h.empty())
        return;
    d.alloc(h.size() * sizeof(T));
    hip_check(hipMemcpy(d.p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice), what);
}

static void create_graph(int32_t n, int64_t nnz, const int64_t *row_ptr, const int32_t *col,
                         const int32_t *w, uint32_t flags, bc_graph **out)
{
    check_create_args(n, nnz, row_ptr, col, w, flags, out);
    HostLayout L;
    build_host_layout(n, nnz, row_ptr, col, w, flags, L);

    ensure_device();
    std::unique_ptr<bc_graph> g(new bc_graph());
    init_graph_runtime(g.get());
    g->n = L.n;
    g->nnz = L.nnz;
    g->directed = L.directed;
    g->wmax = L.wmax;
    g->maxdeg = L.maxdeg;
    g->packed = L.packed;
    g->wshift = L.wshift;
    g->wmask = L.wmask;
    g->wbytes = L.wbytes;
    g->avg_deg = L.avg_deg;
    g->wmean = L.wmean;
    g->renumbered = L.renumbered;
    g->host_iperm = L.iperm;
    upload(g->perm, L.perm, "upload numbering");
    upload(g->iperm, L.iperm, "upload numbering");
    upload(g->row, L.row, "upload row offsets");
    upload(g->arc, L.arc, "upload arcs");
    upload(g->wt, L.wt, "upload weights");
    upload(g->trow, L.trow, "upload in-row offsets");
    upload(g->tarc, L.tarc, "upload in-arcs");
    upload(g->twt, L.twt, "upload in-arc weights");
    upload(g->emap, L.emap, "upload arc map");
    g->edges_ready = L.edges;
    set_inarc_bound(g.get(), g->stream);
    *out = g.release();
}

void set_inarc_bound(bc_graph *g, hipStream_t st)
{
    DevBuf b;
    b.alloc(sizeof(int));
    int v = 0;
    hip_check(launch_inarc_bound(g->view().trow, g->n, (int *)b.p, st), "in-arc bound");
    hip_check(hipMemcpyAsync(&v, b.p, sizeof v, hipMemcpyDeviceToHost, st), "in-arc bound");
    hip_check(hipStreamSynchronize(st), "graph upload");
    g->n_act = v;
}

DevGraph bc_graph::view() const
{
    DevGraph d;
    d.row = (const uint32_t *)row.p;
    d.arc = (const uint32_t *)arc.p;
    d.wt = (const int32_t *)wt.p;
    if (directed) {
        d.trow = (const uint32_t *)trow.p;
        d.tarc = (const uint32_t *)tarc.p;
        d.twt = (const int32_t *)twt.p;
    } else {
        d.trow = d.row;
        d.tarc = d.arc;
        d.twt = d.wt;
    }
    d.n = n;
    d.n_act = n_act;
    d.wshift = wshift;
    d.wmask = wmask;
    return d;
}

bc_graph::~bc_graph()
{
    if (stream) {
        (void)hipStreamSynchronize(stream);
        (void)hipStreamDestroy(stream);
    }
    if (plain_exec)
        (void)hipGraphExecDestroy(plain_exec);
    if (ev_k0)
        (void)hipEventDestroy(ev_k0);
    if (ev_k1)
        (void)hipEventDestroy(ev_k1);
    if (host_counters)
        (void)hipHostFree(host_counters);
    if (host_plain)
        (void)hipHostFree(host_plain);
}

// ---------------------------------------------------------------------------
// Workspaces
// ---------------------------------------------------------------------------
static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

SlabLayout slab_layout(int32_t n, int64_t pred_slots)
{
    SlabLayout L;
    const size_t nn = (size_t)n;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align256(o + bytes);
        return at;
    };
    L.d = take(4 * nn);
    L.rec = take(VREC_BYTES * nn);
    L.bcp = take(8 * nn);
    L.order = take(4 * nn);
    L.qa = take(4 * nn);
    L.qb = take(4 * nn);
    L.fa = take(4 * nn);
    L.fb = take(4 * nn);
    L.bx = take(8 * nn); // with fa and fb: the bucket pool of the far-bucket ring
    L.oa = take(4 * nn);
    L.ob = take(4 * nn);
    L.band_off = take(4 * (nn + 2));
    L.hdr = take(64);
    L.preds = take(4 * (size_t)std::max<int64_t>(pred_slots, 1));
    L.stride = o;
    return L;
}

static void ensure_slabs(bc_graph *g, Workspace &ws, int nslabs, hipStream_t st)
{
    if (ws.base.p && ws.nslabs >= nslabs)
        return;
    ws.base.release();
    // only the batched form records the shortest-path DAG (one slot per in-arc)
    ws.L = slab_layout(g->n, &ws == &g->batched ? g->nnz : 0);
    const size_t bytes = ws.L.stride * (size_t)nslabs;
    size_t free_b = 0, total_b = 0;
    hip_check(hipMemGetInfo(&free_b, &total_b), "hipMemGetInfo");
    if (bytes > free_b)
        throw bc_error(BC_E_NOMEM, "state slabs need %zu bytes, %zu free", bytes, free_b);
    ws.base.alloc(bytes);
    ws.nslabs = nslabs;
    hip_check(launch_slab_reset((char *)ws.base.p, ws.L, nslabs, g->n, st), "slab reset");
}

static void ensure_sources(bc_graph *g, int64_t k)
{
    const size_t need = (size_t)std::max<int64_t>(k, 1) * sizeof(int32_t);
    if (g->src_buf.bytes < need)
        g->src_buf.alloc(need);
}

// ---------------------------------------------------------------------------
// Options
// ---------------------------------------------------------------------------
int default_delta(const bc_graph *g)
{
    // Band width of the near-far split: a few mean arc weights per average
    // degree (tuned per graph by the autotuner when asked).
    const double avg = std::max(1.0, g->avg_deg);
    double d = 4.0 * (double)g->wmax / avg;
    d = std::max(d, 1.0);
    d = std::min(d, (double)INT32_MAX / 4);
    return (int)d;
}


int lds_bits_for(const bc_graph *g, int requested)
{
    if (requested == 8)
        return g->packed ? 8 : 16; // 8-bit entries are built for packed arcs only
    if (requested == 16 || requested == 32)
        return requested;
    // Graphs renumbered for skewed in-degrees are small-world: their distances
    // stay small, so 16-bit entries rarely overflow to device memory.
    return g->renumbered ? 16 : 32;
}

static size_t lds_bytes_for(int H, int bits) { return batched_lds_bytes(H, bits); }

void batched_lds_plan(const bc_graph *g, int nt, bool atomic_bc, int requested, int bits,
                      int &H, int &per_cu, int64_t want_slabs)
{
    // Workgroups per CU are set by registers (or by the sources in flight the
    // caller asked for, when those fill fewer); the LDS (160 KB per CU) is
    // then split among them for the per-source distance caches.
    int occ = batched_blocks_per_cu(g->packed, nt, atomic_bc, bits);
    if (want_slabs > 0)
        occ = (int)std::min<int64_t>(occ, (want_slabs + g->num_cus - 1) / g->num_cus);
    const size_t lds_cu = 160 * 1024, reserve = 2 * 1024;
    int cap = (int)((lds_cu / (size_t)std::max(occ, 1) - reserve) / (size_t)(bits / 8));
    cap &= ~3;
    if (requested < 0)
        H = 0;
    else if (requested > 0)
        H = std::min(requested, g->n);
    else
        H = std::min(cap, g->n);
    per_cu = H > 0 ? batched_blocks_per_cu_lds(g->packed, nt, atomic_bc, bits,
                                               lds_bytes_for(H, bits))
                   : occ;
    if (per_cu < 1) {
        H = std::min(cap, g->n);
        per_cu = batched_blocks_per_cu_lds(g->packed, nt, atomic_bc, bits, lds_bytes_for(H, bits));
    }
    per_cu = std::max(per_cu, 1);
}

int64_t batch_cap(bc_graph *g)
{
    // keep the slabs within 60% of the free device memory (the graph's own
    // slabs count as free: a larger set replaces them)
    size_t free_b = 0, total_b = 0;
    hip_check(hipMemGetInfo(&free_b, &total_b), "hipMemGetInfo");
    const size_t stride = slab_layout(g->n, g->nnz).stride;
    const size_t have = g->batched.base.p ? (size_t)g->batched.nslabs * stride : 0;
    const int64_t by_mem = (int64_t)((free_b + have) / 10 * 6 / std::max<size_t>(stride, 1));
    if (by_mem < 1)
        throw bc_error(BC_E_NOMEM, "one state slab (%zu bytes) does not fit", stride);
    return std::min<int64_t>(by_mem, 65535);
}

ResolvedOptions resolve_options(bc_graph *g, const bc_options *opt, int64_t k)
{
    ResolvedOptions r;
    bc_options o;
    memset(&o, 0, sizeof o);
    if (opt)
        o = *opt;
    if (o.mode < 0 || o.mode > BC_MODE_INTERLEAVED)
        throw bc_error(BC_E_INVAL, "unknown mode %d", o.mode);
    if (o.batch < 0 || o.delta < 0 || o.lane_max_deg < 0 || o.wg_threads < 0 ||
        o.lds_vertices < -1)
        throw bc_error(BC_E_INVAL, "negative option");
    if (o.accumulate < 0 || o.accumulate > 2)
        throw bc_error(BC_E_INVAL, "unknown accumulate mode %d", o.accumulate);
    if (o.dep_mode < 0 || o.dep_mode > 2)
        throw bc_error(BC_E_INVAL, "unknown dependency mode %d", o.dep_mode);
    if (o.virtual_warp < 0 || o.virtual_warp > 64 || (o.virtual_warp & (o.virtual_warp - 1)))
        throw bc_error(BC_E_INVAL, "virtual_warp must be 0 or a power of two up to 64");
    if (o.lds_bits != 0 && o.lds_bits != 8 && o.lds_bits != 16 && o.lds_bits != 32)
        throw bc_error(BC_E_INVAL, "lds_bits must be 0, 8, 16 or 32");
    if (o.node_parallel < 0 || o.node_parallel > 1)
        throw bc_error(BC_E_INVAL, "node_parallel must be 0 or 1");
    if (o.expand_lane_deg < 0 || o.wave_max_deg < 0 || o.wg_min_deg < 0)
        throw bc_error(BC_E_INVAL, "negative degree threshold");
    if (o.far_buckets < 0 || o.far_buckets > 2)
        throw bc_error(BC_E_INVAL, "far_buckets must be 0, 1 or 2");
    r.mode = o.mode == BC_MODE_PLAIN || o.mode == BC_MODE_INTERLEAVED ? o.mode : BC_MODE_BATCHED;
    r.stream = o.stream ? (hipStream_t)o.stream : g->stream;
    r.wg_threads = o.wg_threads ? o.wg_threads : 256;
    if (r.wg_threads != 256 && r.wg_threads != 512 && r.wg_threads != 1024)
        throw bc_error(BC_E_INVAL, "wg_threads must be 256, 512 or 1024");
    r.delta = o.delta ? o.delta : default_delta(g);
    if (r.mode == BC_MODE_INTERLEAVED && !o.delta) {
        // every band of the interleaved form costs a far-list pass and its rounds
        // a read-back each: wide bands (a few maximum weights) pay off there
        r.delta = (int)std::max<int64_t>(r.delta, std::min<int64_t>(4ll * g->wmax, INT32_MAX / 2));
    }
    r.lane_max = o.lane_max_deg ? o.lane_max_deg : 32;
    r.accumulate = o.accumulate ? o.accumulate : 1;
    r.dep_mode = o.dep_mode ? o.dep_mode : 1;
    r.vw = o.virtual_warp;
    r.node_parallel = o.node_parallel;
    // the tiers keep their order: a threshold below the one before it is raised to it
    r.lane_deg = o.expand_lane_deg ? o.expand_lane_deg : BC_DEF_LANE_DEG;
    r.wave_deg = std::max(r.lane_deg, o.wave_max_deg ? o.wave_max_deg : BC_DEF_WAVE_DEG);
    r.wg_deg = std::max(r.wave_deg, o.wg_min_deg ? o.wg_min_deg : BC_HUB_DEG);
    r.il_groups = (int)std::min<int64_t>(((int64_t)o.batch + 63) / 64, INT32_MAX);
    r.far_buckets = o.far_buckets;
    int per_cu = 1;
    r.lds_bits = lds_bits_for(g, o.lds_bits);
    batched_lds_plan(g, r.wg_threads, r.accumulate == 2, o.lds_vertices, r.lds_bits,
                     r.lds_vertices, per_cu, o.batch);
    const int fill = g->num_cus * per_cu;
    int64_t b = o.batch ? o.batch : fill;
    b = std::min<int64_t>(b, std::max<int64_t>(k, 1));
    b = std::min<int64_t>(b, batch_cap(g));
    r.batch = (int)std::max<int64_t>(b, 1);
    r.autotune = o.autotune;
    return r;
}

// ---------------------------------------------------------------------------
// Drivers
// ---------------------------------------------------------------------------
void reset_device_counters(bc_graph *g, hipStream_t st)
{
    DevCounters *c = (DevCounters *)g->ctl.p;
    hip_check(launch_fill_u64((unsigned long long *)c, sizeof(DevCounters) / 8, 0ull, st),
              "reset counters");
    hip_check(launch_fill_u64(&c->err[1], 1, (unsigned long long)INT64_MAX, st), "reset");
}

void read_device_counters(bc_graph *g, hipStream_t st, DevCounters &out)
{
    hip_check(hipMemcpyAsync(g->host_counters, g->ctl.p, sizeof(DevCounters),
                             hipMemcpyDeviceToHost, st),
              "read counters");
    hip_check(hipStreamSynchronize(st), "synchronize");
    out = *g->host_counters;
}

void fill_stats(bc_graph *g, const ResolvedOptions &r, const DevCounters &c, int64_t k,
                double ms, double kernel_ms, int64_t launches, bc_stats *st)
{
    if (!st)
        return;
    memset(st, 0, sizeof *st);
    st->ms = ms;
    st->kernel_ms = kernel_ms;
    st->kernel_launches = launches;
    st->sources = k;
    st->reached = (int64_t)c.stats.reached;
    st->arcs_out_reached = (int64_t)c.stats.arcs;
    st->dag_arcs = (int64_t)c.stats.dag;
    st->improvements = (int64_t)c.stats.improvements;
    st->bands = (int64_t)c.stats.bands;
    st->iterations = (int64_t)c.stats.iterations;
    st->sigma_rounds = (int64_t)c.stats.sigma_rounds;
    st->delta_rounds = (int64_t)c.stats.delta_rounds;
    for (int i = 0; i < 5; ++i)
        st->phase_ticks[i] = (int64_t)c.stats.ticks[i];
    st->first_bad_source = (c.err[0] & BC_ERRBIT_SIGMA) ? (int64_t)c.err[1] : -1;
    // Per-source byte model summed over sources: the n-dependent term once per source.
    st->algo_bytes = (double)k * 20.0 * (double)g->n +
                     (double)st->arcs_out_reached * (16.0 + 2.0 * g->wbytes) +
                     72.0 * (double)st->reached + 24.0 * (double)st->dag_arcs;
    st->mode = r.mode;
    st->batch = r.batch;
    st->delta = r.delta;
    st->lane_max_deg = r.lane_max;
    st->wg_threads = r.wg_threads;
    st->accumulate = r.accumulate;
    st->lds_vertices = r.lds_vertices;
    st->lds_bits = r.lds_bits;
    st->dep_mode = r.dep_mode;
    st->virtual_warp = r.vw;
    st->node_parallel = r.node_parallel;
    st->expand_lane_deg = r.lane_deg;
    st->wave_max_deg = r.wave_deg;
    st->wg_min_deg = r.wg_deg;
    int buckets = 0, nbk = 0;
    bucket_plan(g, r, buckets, nbk);
    st->far_buckets = r.mode == BC_MODE_BATCHED ? (buckets ? 1 : 2) : 0;
}

void bucket_plan(const bc_graph *g, const ResolvedOptions &r, int &buckets, int &nbk)
{
    // One bucket per band a far value can lie ahead (a value found in band b is
    // below (b + 1) delta + w_max), plus slack; the ring pays off when the
    // weights span many bands, where the pile would be rescanned many times.
    const int64_t spans = ((int64_t)g->wmax + r.delta - 1) / std::max(r.delta, 1);
    nbk = (int)std::min<int64_t>(spans + 2, BC_BUCKETS_MAX);
    // bucket keys (BUCKET_KEY) stay below the count pass's predecessor
    // encodings only while vertex ids and bucket indices stay below 2^30
    const int64_t last_bucket = (int64_t)std::max(g->n - 1, 0) * g->wmax / std::max(r.delta, 1);
    const bool keys_fit = g->n < (1 << 30) && last_bucket < (int64_t)1 << 30;
    buckets = g->packed && keys_fit &&
              (r.far_buckets == 1 || (r.far_buckets == 0 && spans >= 16));
}

void set_tier_args(const bc_graph *g, int lane_deg, int wave_deg, int wg_deg, BatchArgs &a)
{
    a.lane_deg = (uint32_t)lane_deg;
    a.wave_deg = (uint32_t)wave_deg;
    a.wg_deg = (uint32_t)wg_deg;
    a.hubs = g->maxdeg > wg_deg;
}

void check_device_errors(const DevCounters &c)
{
    if (c.err[0] & BC_ERRBIT_SOURCE)
        throw bc_error(BC_E_INVAL, "a source in the device source list is out of range");
    if (c.err[0] & BC_ERRBIT_INTERNAL)
        throw bc_error(BC_E_INTERNAL, "an internal iteration bound tripped; result invalid");
    if (c.err[0] & BC_ERRBIT_SIGMA)
        throw bc_error(BC_E_SIGMA_OVERFLOW,
                       "shortest-path count exceeded 2^64-1 (first source-list index %lld)",
                       (long long)c.err[1]);
}

void launch_batched_pass(bc_graph *g, const ResolvedOptions &r, const int32_t *src_dev,
                         int64_t k, double *bc_dev, char *slab_base, const SlabLayout &L,
                         int nslabs, double *ebc_dev, hipStream_t st)
{
    const bool atomic_bc = r.accumulate == 2;
    BatchArgs a;
    a.g = g->view();
    a.slab_base = slab_base;
    a.L = L;
    a.sources = src_dev;
    a.k = k;
    DevCounters *c = (DevCounters *)g->ctl.p;
    a.next_src = &c->next_src;
    a.bc_out = bc_dev;
    a.item_out = nullptr;
    a.item_err = nullptr;
    a.iperm = g->iperm_dev();
    a.perm = g->perm_dev();
    a.H = r.lds_vertices;
    a.lds_bits = r.lds_bits;
    set_tier_args(g, r.lane_deg, r.wave_deg, r.wg_deg, a);
    a.kahn = r.dep_mode == 1 ? 1 : 0;
    a.vw = r.vw;
    a.node_parallel = r.node_parallel;
    a.ebc = ebc_dev;
    a.emap = (const uint32_t *)g->emap.p;
    a.delta = (uint32_t)r.delta;
    a.lane_max = r.lane_max;
    a.stats = &c->stats;
    a.err = c->err;
    bucket_plan(g, r, a.buckets, a.nbk);
    // bucket pool: fa, fb and bx, contiguous in the slab
    a.bcap = (int32_t)std::min<size_t>((L.bx + 8 * (size_t)g->n - L.fa) / 4 / (size_t)a.nbk,
                                       (size_t)INT32_MAX);
    hip_check(hipEventRecord(g->ev_k0, st), "event");
    hip_check(launch_batched(a, g->packed, r.wg_threads, atomic_bc, nslabs, st), "batched kernel");
    hip_check(hipEventRecord(g->ev_k1, st), "event");
    if (!atomic_bc)
        hip_check(launch_reduce_partials(slab_base, L, nslabs, g->n, bc_dev, a.perm, st),
                  "reduce");
}

void run_batched(bc_graph *g, const ResolvedOptions &r, const int32_t *src_dev, int64_t k,
                 double *bc_dev, DevCounters &cnt, float &ms, float *kernel_ms, double *ebc_dev)
{
    hipStream_t st = r.stream;
    ensure_slabs(g, g->batched, r.batch, st);
    reset_device_counters(g, st);
    const bool atomic_bc = r.accumulate == 2;
    if (atomic_bc || k == 0)
        hip_check(launch_fill_u64((unsigned long long *)bc_dev, (size_t)g->n, 0ull, st), "zero");
    if (ebc_dev)
        hip_check(launch_fill_u64((unsigned long long *)ebc_dev, (size_t)g->nnz, 0ull, st),
                  "zero");
    hipEvent_t e0 = nullptr, e1 = nullptr;
    struct Events {
        hipEvent_t &a, &b;
        ~Events()
        {
            if (a)
                (void)hipEventDestroy(a);
            if (b)
                (void)hipEventDestroy(b);
        }
    } release{e0, e1};
    hip_check(hipEventCreate(&e0), "event");
    hip_check(hipEventCreate(&e1), "event");
    hip_check(hipEventRecord(e0, st), "event");
    if (k > 0)
        launch_batched_pass(g, r, src_dev, k, bc_dev, (char *)g->batched.base.p, g->batched.L,
                            (int)std::min<int64_t>(r.batch, k), ebc_dev, st);
    hip_check(hipEventRecord(e1, st), "event");
    read_device_counters(g, st, cnt);
    hip_check(hipEventElapsedTime(&ms, e0, e1), "event time");
    if (kernel_ms) {
        *kernel_ms = 0.f;
        if (k > 0)
            hip_check(hipEventElapsedTime(kernel_ms, g->ev_k0, g->ev_k1), "event time");
    }
}

static void run_plain(bc_graph *g, const ResolvedOptions &r, const int32_t *src_host, int64_t k,
                      double *bc_dev, DevCounters &cnt, float &ms)
{
    hipStream_t st = r.stream;
    ensure_slabs(g, g->plain, 1, st);
    reset_device_counters(g, st);
    hip_check(launch_fill_u64((unsigned long long *)bc_dev, (size_t)g->n, 0ull, st), "zero");
    PlainArgs a;
    a.g = g->view();
    a.vw = r.vw;
    a.perm = g->perm_dev();
    a.slab_base = (char *)g->plain.base.p;
    a.L = g->plain.L;
    a.ctl = (PlainCtl *)g->plain_ctl.p;
    a.bc_out = nullptr; // the output travels in the control block
    a.delta = (uint32_t)r.delta;
    a.lane_max = r.lane_max;
    a.lane_deg = (uint32_t)r.lane_deg;
    a.wave_deg = (uint32_t)r.wave_deg;
    DevCounters *c = (DevCounters *)g->ctl.p;
    a.stats = &c->stats;
    a.err = c->err;
    const int grid = g->num_cus * 4;
    if (!g->plain_ctl_ready) {
        PlainCtl init;
        memset(&init, 0, sizeof init);
        init.phase = 4;
        hip_check(hipMemcpyAsync(a.ctl, &init, sizeof init, hipMemcpyHostToDevice, st), "ctl");
        hip_check(hipStreamSynchronize(st), "ctl");
        g->plain_ctl_ready = true;
    }
    // The sweep loop of the plain form is a captured graph of (step, control)
    // pairs, replayed until the phase machine reports completion.  Its kernel
    // arguments only name per-graph buffers, so one capture serves every call
    // with the same band width and lane threshold.
    const int PLAIN_GRAPH_PAIRS = 32;
    if (!g->plain_exec || g->plain_exec_delta != a.delta || g->plain_exec_lane_max != a.lane_max ||
        g->plain_exec_vw != a.vw || g->plain_exec_slab != (const void *)a.slab_base ||
        g->plain_exec_tiers != (((uint64_t)a.lane_deg << 32) | a.wave_deg)) {
        if (g->plain_exec) {
            (void)hipGraphExecDestroy(g->plain_exec);
            g->plain_exec = nullptr;
        }
        hip_check(hipStreamSynchronize(g->stream), "synchronize");
        hip_check(hipStreamBeginCapture(g->stream, hipStreamCaptureModeThreadLocal), "capture");
        hipError_t le = launch_plain_steps(a, g->packed, grid, PLAIN_GRAPH_PAIRS, g->stream);
        hipGraph_t graph = nullptr;
        hipError_t ce = hipStreamEndCapture(g->stream, &graph);
        hip_check(le, "capture launches");
        hip_check(ce, "end capture");
        hipError_t ie = hipGraphInstantiate(&g->plain_exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        hip_check(ie, "instantiate");
        g->plain_exec_delta = a.delta;
        g->plain_exec_lane_max = a.lane_max;
        g->plain_exec_vw = a.vw;
        g->plain_exec_slab = (const void *)a.slab_base;
        g->plain_exec_tiers = ((uint64_t)a.lane_deg << 32) | a.wave_deg;
    }
    const unsigned long long iter_cap = 8ull * (unsigned long long)g->n + 1024ull;
    hipEvent_t e0, e1;
    hip_check(hipEventCreate(&e0), "event");
    hip_check(hipEventCreate(&e1), "event");
    hip_check(hipEventRecord(e0, st), "event");
    for (int64_t i = 0; i < k; ++i) {
        const bool clear = g->plain_gen_hint > (1 << 30);
        if (clear)
            g->plain_gen_hint = 0;
        hip_check(launch_plain_source(a, g->packed, grid, g->internal_id(src_host[i]),
                                      (long long)i, clear, bc_dev, st),
                  "plain setup");
        // set the iteration bound (host-side value, copied once per source)
        hip_check(launch_fill_u64(&a.ctl->iter_cap, 1, iter_cap, st), "cap");
        long long total_pairs = 0;
        for (;;) {
            hip_check(hipGraphLaunch(g->plain_exec, st), "plain sweep");
            total_pairs += PLAIN_GRAPH_PAIRS;
            hip_check(hipMemcpyAsync(g->host_plain, a.ctl, sizeof(PlainCtl),
                                     hipMemcpyDeviceToHost, st),
                      "read phase");
            hip_check(hipStreamSynchronize(st), "synchronize");
            if (g->host_plain->phase == 4)
                break;
            if (total_pairs > 64ll * (long long)iter_cap + 4096)
                throw bc_error(BC_E_INTERNAL, "plain phase machine did not finish");
        }
        g->plain_gen_hint = g->host_plain->gen;
        if (g->host_plain->abort)
            hip_check(launch_plain_clear_infar(a, st), "clear");
    }
    hip_check(hipEventRecord(e1, st), "event");
    read_device_counters(g, st, cnt);
    hip_check(hipEventElapsedTime(&ms, e0, e1), "event time");
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
}

void compute_device(bc_graph *g, const int32_t *src_dev, const int32_t *src_host, int64_t k,
                    const bc_options *opt, double *bc_dev, bc_stats *stats, double *ebc_dev)
{
    ResolvedOptions r = resolve_options(g, opt, k);
    if (ebc_dev) {
        // edge betweenness comes from the recorded-DAG dependency pass
        if (!g->edges_ready)
            throw bc_error(BC_E_INVAL, "the graph was created without BC_EDGE_BC");
        if (r.mode != BC_MODE_BATCHED)
            throw bc_error(BC_E_INVAL, "edge betweenness needs the batched form");
        r.dep_mode = 1;
        r.autotune = 0;
    }
    if (r.autotune && r.mode == BC_MODE_BATCHED && k > 0)
        autotune(g, r, opt, src_dev, k);
    DevCounters cnt;
    float ms = 0.f, kms = 0.f;
    int64_t launches = 0;
    if (r.mode == BC_MODE_PLAIN) {
        std::vector<int32_t> hs;
        if (!src_host && k > 0) {
            hs.resize((size_t)k);
            hip_check(hipMemcpyAsync(hs.data(), src_dev, (size_t)k * 4, hipMemcpyDeviceToHost,
                                     r.stream),
                      "sources to host");
            hip_check(hipStreamSynchronize(r.stream), "synchronize");
            for (int64_t i = 0; i < k; ++i)
                if (hs[(size_t)i] < 0 || hs[(size_t)i] >= g->n)
                    throw bc_error(BC_E_INVAL, "source %d out of range", hs[(size_t)i]);
            src_host = hs.data();
        }
        run_plain(g, r, src_host, k, bc_dev, cnt, ms);
        kms = ms;
        launches = 0;
    } else if (r.mode == BC_MODE_INTERLEAVED) {
        run_interleaved(g, r, src_dev, k, bc_dev, cnt, ms);
        kms = ms;
        launches = 0;
    } else {
        run_batched(g, r, src_dev, k, bc_dev, cnt, ms, &kms, ebc_dev);
        launches = k > 0 ? 1 : 0;
    }
    check_device_errors(cnt);
    fill_stats(g, r, cnt, k, (double)ms, (double)kms, launches, stats);
    g->last_stats_valid = true;
    fill_stats(g, r, cnt, k, (double)ms, (double)kms, launches, &g->last_stats);
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

bc_status bc_create_graph(int32_t n, int64_t nnz, const int64_t *row_ptr, const int32_t *col,
                          const int32_t *w, uint32_t flags, bc_graph **out)
{
    return guarded([&] { create_graph(n, nnz, row_ptr, col, w, flags, out); });
}

bc_status bc_create_graph_device(int32_t n, int64_t nnz, const int64_t *row_ptr_dev,
                                 const int32_t *col_dev, const int32_t *w_dev, uint32_t flags,
                                 void *stream, bc_graph **out)
{
    return guarded([&] {
        check_create_args(n, nnz, row_ptr_dev, col_dev, w_dev, flags, out);
        ensure_device();
        std::unique_ptr<bc_graph> g(new bc_graph());
        init_graph_runtime(g.get());
        create_graph_device(n, nnz, row_ptr_dev, col_dev, w_dev, flags,
                            stream ? (hipStream_t)stream : g->stream, g.get());
        *out = g.release();
    });
}

bc_status bc_destroy_graph(bc_graph *g)
{
    return guarded([&] {
        if (g && g->server_refs.load() > 0)
            throw bc_error(BC_E_BUSY, "the graph is held by %d live server(s); destroy them first",
                           g->server_refs.load());
        delete g;
    });
}

bc_status bc_get_graph_info(const bc_graph *g, bc_graph_info *info)
{
    return guarded([&] {
        if (!g || !info)
            throw bc_error(BC_E_INVAL, "null argument");
        bc_graph_info i;
        memset(&i, 0, sizeof i);
        i.n = g->n;
        i.nnz = g->nnz;
        i.directed = g->directed;
        i.w_max = g->wmax;
        i.max_out_degree = g->maxdeg;
        i.packed_arcs = g->packed;
        i.renumbered = g->renumbered;
        i.device_bytes = (int64_t)(g->row.bytes + g->arc.bytes + g->wt.bytes + g->trow.bytes +
                                   g->tarc.bytes + g->twt.bytes);
        i.tuned = g->tuned.valid;
        i.tuned_delta = g->tuned.delta;
        i.tuned_wg_threads = g->tuned.wg_threads;
        i.tuned_lane_max_deg = g->tuned.lane_max;
        i.tuned_dep_mode = g->tuned.dep_mode;
        i.tuned_expand_lane_deg = g->tuned.lane_deg;
        i.tuned_wave_max_deg = g->tuned.wave_deg;
        i.tuned_wg_min_deg = g->tuned.wg_deg;
        i.tuned_batch = g->tuned.batch;
        i.tuned_lds_bits = g->tuned.lds_bits;
        i.tuning_trials = g->tune_trials;
        *info = i;
    });
}

bc_status bc_compute(bc_graph *g, const int32_t *sources, int64_t k, const bc_options *opt,
                     bc_result **out)
{
    return guarded([&] {
        if (!g || !out)
            throw bc_error(BC_E_INVAL, "null argument");
        if (k < 0)
            throw bc_error(BC_E_INVAL, "k must be >= 0");
        std::vector<int32_t> all;
        if (!sources) {
            if (k != g->n && k != 0)
                throw bc_error(BC_E_INVAL, "sources may be NULL only with k = n");
            all.resize((size_t)k);
            for (int64_t i = 0; i < k; ++i)
                all[(size_t)i] = (int32_t)i;
            sources = all.data();
        }
        for (int64_t i = 0; i < k; ++i)
            if (sources[i] < 0 || sources[i] >= g->n)
                throw bc_error(BC_E_INVAL, "sources[%lld] = %d out of range", (long long)i,
                               sources[i]);
        ResolvedOptions r = resolve_options(g, opt, k);
        std::unique_ptr<bc_result> res(new bc_result());
        res->n = g->n;
        res->bc.alloc((size_t)g->n * sizeof(double));
        ensure_sources(g, k);
        if (k > 0)
            hip_check(hipMemcpyAsync(g->src_buf.p, sources, (size_t)k * 4, hipMemcpyHostToDevice,
                                     r.stream),
                      "upload sources");
        compute_device(g, (const int32_t *)g->src_buf.p, sources, k, opt, (double *)res->bc.p,
                       &res->stats);
        *out = res.release();
    });
}

bc_status bc_compute_device(bc_graph *g, const int32_t *sources_dev, int64_t k,
                            const bc_options *opt, double *bc_dev, bc_stats *stats)
{
    return guarded([&] {
        if (!g || !bc_dev || (k > 0 && !sources_dev))
            throw bc_error(BC_E_INVAL, "null argument");
        if (k < 0)
            throw bc_error(BC_E_INVAL, "k must be >= 0");
        compute_device(g, sources_dev, nullptr, k, opt, bc_dev, stats);
    });
}

bc_status bc_compute_edges_device(bc_graph *g, const int32_t *sources_dev, int64_t k,
                                  const bc_options *opt, double *bc_dev, double *ebc_dev,
                                  bc_stats *stats)
{
    return guarded([&] {
        if (!g || !bc_dev || !ebc_dev || (k > 0 && !sources_dev))
            throw bc_error(BC_E_INVAL, "null argument");
        if (k < 0)
            throw bc_error(BC_E_INVAL, "k must be >= 0");
        if (g->nnz == 0) {
            compute_device(g, sources_dev, nullptr, k, opt, bc_dev, stats);
            return;
        }
        compute_device(g, sources_dev, nullptr, k, opt, bc_dev, stats, ebc_dev);
    });
}

bc_status bc_compute_edges(bc_graph *g, const int32_t *sources, int64_t k, const bc_options *opt,
                           double *bc_host, double *ebc_host)
{
    return guarded([&] {
        if (!g || !ebc_host)
            throw bc_error(BC_E_INVAL, "null argument");
        if (k < 0)
            throw bc_error(BC_E_INVAL, "k must be >= 0");
        std::vector<int32_t> all;
        if (!sources) {
            if (k != g->n && k != 0)
                throw bc_error(BC_E_INVAL, "sources may be NULL only with k = n");
            all.resize((size_t)k);
            for (int64_t i = 0; i < k; ++i)
                all[(size_t)i] = (int32_t)i;
            sources = all.data();
        }
        for (int64_t i = 0; i < k; ++i)
            if (sources[i] < 0 || sources[i] >= g->n)
                throw bc_error(BC_E_INVAL, "sources[%lld] = %d out of range", (long long)i,
                               sources[i]);
        ResolvedOptions r = resolve_options(g, opt, k);
        ensure_sources(g, k);
        if (k > 0)
            hip_check(hipMemcpyAsync(g->src_buf.p, sources, (size_t)k * 4, hipMemcpyHostToDevice,
                                     r.stream),
                      "upload sources");
        DevBuf bc, ebc;
        bc.alloc((size_t)g->n * 8);
        ebc.alloc((size_t)std::max<int64_t>(g->nnz, 1) * 8);
        if (g->nnz == 0)
            hip_check(launch_fill_u64((unsigned long long *)ebc.p, 1, 0ull, r.stream), "zero");
        compute_device(g, (const int32_t *)g->src_buf.p, sources, k, opt, (double *)bc.p, nullptr,
                       g->nnz ? (double *)ebc.p : nullptr);
        hip_check(hipStreamSynchronize(r.stream), "synchronize");
        if (bc_host)
            hip_check(hipMemcpy(bc_host, bc.p, (size_t)g->n * 8, hipMemcpyDeviceToHost), "copy");
        if (g->nnz)
            hip_check(hipMemcpy(ebc_host, ebc.p, (size_t)g->nnz * 8, hipMemcpyDeviceToHost),
                      "copy");
    });
}

bc_status bc_result_bc(const bc_result *r, double *bc_host)
{
    return guarded([&] {
        if (!r || !bc_host)
            throw bc_error(BC_E_INVAL, "null argument");
        hip_check(hipMemcpy(bc_host, r->bc.p, (size_t)r->n * sizeof(double),
                            hipMemcpyDeviceToHost),
                  "copy result");
    });
}

bc_status bc_result_device_ptr(const bc_result *r, const double **bc_dev)
{
    return guarded([&] {
        if (!r || !bc_dev)
            throw bc_error(BC_E_INVAL, "null argument");
        *bc_dev = (const double *)r->bc.p;
    });
}

bc_status bc_result_stats(const bc_result *r, bc_stats *st)
{
    return guarded([&] {
        if (!r || !st)
            throw bc_error(BC_E_INVAL, "null argument");
        *st = r->stats;
    });
}

bc_status bc_destroy_result(bc_result *r)
{
    return guarded([&] { delete r; });
}

bc_status bc_source_state(bc_graph *g, int32_t s, const bc_options *opt, int32_t *d,
                          uint64_t *sigma, double *delta)
{
    return guarded([&] {
        if (!g)
            throw bc_error(BC_E_INVAL, "null graph");
        if (s < 0 || s >= g->n)
            throw bc_error(BC_E_INVAL, "source %d out of range", s);
        bc_options o;
        memset(&o, 0, sizeof o);
        if (opt)
            o = *opt;
        o.batch = 1;
        o.autotune = 0;
        if (o.mode == BC_MODE_INTERLEAVED)
            throw bc_error(BC_E_INVAL, "per-source state comes from the batched or plain form");
        ResolvedOptions r = resolve_options(g, &o, 1);
        ensure_sources(g, 1);
        hip_check(hipMemcpyAsync(g->src_buf.p, &s, 4, hipMemcpyHostToDevice, r.stream), "src");
        DevBuf bc, dd, ds, dl;
        bc.alloc((size_t)g->n * 8);
        compute_device(g, (const int32_t *)g->src_buf.p, &s, 1, &o, (double *)bc.p, nullptr);
        Workspace &ws = r.mode == BC_MODE_PLAIN ? g->plain : g->batched;
        dd.alloc((size_t)g->n * 4);
        ds.alloc((size_t)g->n * 8);
        dl.alloc((size_t)g->n * 8);
        hip_check(launch_export_state((char *)ws.base.p, ws.L, 0, g->n, (int32_t *)dd.p,
                                      (uint64_t *)ds.p, (double *)dl.p, g->perm_dev(), r.stream),
                  "export");
        hip_check(hipStreamSynchronize(r.stream), "synchronize");
        if (d)
            hip_check(hipMemcpy(d, dd.p, (size_t)g->n * 4, hipMemcpyDeviceToHost), "copy d");
        if (sigma)
            hip_check(hipMemcpy(sigma, ds.p, (size_t)g->n * 8, hipMemcpyDeviceToHost), "copy");
        if (delta)
            hip_check(hipMemcpy(delta, dl.p, (size_t)g->n * 8, hipMemcpyDeviceToHost), "copy");
    });
}

bc_status bc_update_arc_device(bc_graph *g_old, bc_graph *g_new, bc_graph *g_rev,
                               int32_t tail, int32_t head, int32_t w_old, int32_t w_new,
                               const bc_options *opt, double *bc_dev, int32_t *affected_dev,
                               int64_t *affected)
{
    return guarded([&] {
        if (!g_old || !g_new || !bc_dev)
            throw bc_error(BC_E_INVAL, "null argument");
        const int32_t n = g_old->n;
        if (g_new->n != n || g_new->directed != g_old->directed)
            throw bc_error(BC_E_INVAL, "the two graphs differ in size or directedness");
        if (tail < 0 || tail >= n || head < 0 || head >= n)
            throw bc_error(BC_E_INVAL, "arc %d -> %d out of range", tail, head);
        if (w_old < 0 || w_new < 0 || w_old == w_new)
            throw bc_error(BC_E_INVAL, "weights %d -> %d are not a change", w_old, w_new);
        if (g_old->directed) {
            if (!g_rev || !g_rev->directed || g_rev->n != n || g_rev->nnz != g_old->nnz)
                throw bc_error(BC_E_INVAL, "a directed graph needs its reverse (same n and nnz)");
        } else if (g_rev) {
            throw bc_error(BC_E_INVAL, "an undirected graph takes no reverse graph");
        }
        const int64_t per = g_old->directed ? 1 : 2;
        const int64_t dn = per * ((w_new > 0 ? 1 : 0) - (w_old > 0 ? 1 : 0));
        if (tail != head && g_new->nnz - g_old->nnz != dn)
            throw bc_error(BC_E_INVAL, "arc counts %lld -> %lld do not match the change",
                           (long long)g_old->nnz, (long long)g_new->nnz);
        if (tail == head) {
            if (affected)
                *affected = 0; // a self-loop lies on no shortest path
            return;
        }
        // dist(s, tail) and dist(s, head) for every s: single-source passes from
        // tail and head on the reversed graph (an undirected graph is its own)
        bc_graph *gd = g_old->directed ? g_rev : g_old;
        bc_options o;
        memset(&o, 0, sizeof o);
        if (opt)
            o = *opt;
        o.batch = 1;
        o.autotune = 0;
        if (o.mode == BC_MODE_INTERLEAVED)
            o.mode = BC_MODE_BATCHED; // the endpoint distances come from a per-source slab
        const ResolvedOptions r = resolve_options(gd, &o, 1);
        DevBuf dist, scratch, list, cnt;
        dist.alloc((size_t)n * 8);
        scratch.alloc((size_t)n * 8);
        int32_t *dt = (int32_t *)dist.p, *dh = dt + n;
        const int32_t ends[2] = {tail, head};
        ensure_sources(gd, 1);
        for (int i = 0; i < 2; ++i) {
            hip_check(hipMemcpyAsync(gd->src_buf.p, &ends[i], 4, hipMemcpyHostToDevice,
                                     r.stream),
                      "upload endpoint");
            compute_device(gd, (const int32_t *)gd->src_buf.p, &ends[i], 1, &o,
                           (double *)scratch.p, nullptr);
            Workspace &ws = r.mode == BC_MODE_PLAIN ? gd->plain : gd->batched;
            hip_check(launch_export_state((char *)ws.base.p, ws.L, 0, n, i == 0 ? dt : dh,
                                          nullptr, nullptr, gd->perm_dev(), r.stream),
                      "export distances");
        }
        list.alloc((size_t)n * 4);
        cnt.alloc(8);
        hip_check(launch_fill_u32((uint32_t *)cnt.p, 1, 0u, r.stream), "clear count");
        hip_check(launch_dynamic_affected(dt, dh, n, w_old, w_new, g_old->directed ? 0 : 1,
                                          (int32_t *)list.p, (int *)cnt.p, r.stream),
                  "affected sources");
        int k = 0;
        hip_check(hipMemcpyAsync(&k, cnt.p, 4, hipMemcpyDeviceToHost, r.stream), "count");
        hip_check(hipStreamSynchronize(r.stream), "synchronize");
        // the outputs are written once everything else has succeeded
        auto finish = [&]() {
            if (affected_dev && k > 0) {
                hip_check(hipMemcpyAsync(affected_dev, list.p, (size_t)k * 4,
                                         hipMemcpyDeviceToDevice, r.stream),
                          "copy affected sources");
                hip_check(hipStreamSynchronize(r.stream), "synchronize");
            }
            if (affected)
                *affected = k;
        };
        if (k == 0) {
            finish();
            return;
        }
        if (2 * (int64_t)k > (int64_t)n) {
            // replacing k sources costs 2k source passes: more than running
            // every source of the new graph once
            const ResolvedOptions rn = resolve_options(g_new, opt, n);
            DevBuf all;
            all.alloc((size_t)n * 4);
            hip_check(launch_iota((int32_t *)all.p, n, rn.stream), "source list");
            compute_device(g_new, (const int32_t *)all.p, nullptr, n, opt, bc_dev, nullptr);
            finish();
            return;
        }
        // the affected sources' dependencies before and after the change
        DevBuf before;
        before.alloc((size_t)n * 8);
        double *after = (double *)scratch.p;
        compute_device(g_old, (const int32_t *)list.p, nullptr, k, opt, (double *)before.p,
                       nullptr);
        compute_device(g_new, (const int32_t *)list.p, nullptr, k, opt, after, nullptr);
        const ResolvedOptions rn = resolve_options(g_new, opt, k);
        hip_check(launch_dynamic_apply(bc_dev, (const double *)before.p, after, n, rn.stream),
                  "apply");
        hip_check(hipStreamSynchronize(rn.stream), "synchronize");
        finish();
    });
}

double bc_algo_bytes(int32_t n, int32_t weight_bytes, int64_t arcs, int64_t reached,
                     int64_t dag_arcs)
{
    return (double)arcs * (16.0 + 2.0 * weight_bytes) + 72.0 * (double)reached +
           24.0 * (double)dag_arcs + 20.0 * (double)n;
}

const char *bc_last_error(void) { return g_last_error.c_str(); }

const char *bc_version(void) { return "bcgpu 0.1 (gfx950)"; }

} // extern "C"
