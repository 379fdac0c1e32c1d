/*
 * oracle.c -- CPU oracle for weighted betweenness centrality.
 *
 * TEST INFRASTRUCTURE ONLY.  This is the slow, plain reference that the GPU
 * library is checked against.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg load it; the product library never links,
 * includes or calls anything here, and this file shares no code, header,
 * table or constant with the GPU path.
 *
 * What it computes (Fan, Xu & Zhao, "A GPU-Based Solution to Fast Calculation
 * of Betweenness Centrality on Large Weighted Networks"):
 *
 *   C_B(v) = sum over ordered pairs (s, t), s != v != t, of sigma_st(v)/sigma_st
 *                                                         (Sec. 2.1, Eq. 1)
 *
 * restricted to a given multiset of sources s, computed the way the paper
 * describes it:
 *   1. per source, Dijkstra's algorithm with a binary heap (Sec. 2.2; the
 *      paper's CPU baseline uses a binary heap, Sec. 4.1) yields the
 *      distances d(s, .) and the shortest-path counts sigma_s(.): when an arc
 *      (v, u, w) gives a strictly shorter tentative distance, u's count is
 *      replaced by v's; when it gives an equal one, v's count is added
 *      (the counting rule of Alg. 2);
 *   2. the dependencies follow Brandes' recursion (Sec. 2.1)
 *          delta_s(v) = sum over successors u of v on shortest paths of
 *                       sigma_sv / sigma_su * (1 + delta_s(u)),
 *      evaluated in reverse settle order (Alg. 3), and every vertex other
 *      than the source adds its dependency to its centrality (Alg. 3).
 *
 * Readings of points the paper leaves open:
 *   - ordered pairs, no factor 1/2, no normalisation (Eq. 1 and Alg. 3 add
 *     every source's dependencies);
 *   - pairs with no path contribute nothing;
 *   - arcs are taken as given (CSR = out-arcs), which covers directed graphs
 *     (Sec. 2.1 says the method extends to them); parallel arcs are distinct
 *     paths;
 *   - weights are integers >= 1; distances are exact 64-bit integers here;
 *   - sigma is an unsigned 64-bit integer and an overflow is an error, never
 *     a wrap;
 *   - dependencies and centralities are IEEE double; sigma values are
 *     converted to double before the division, and each term is formed as
 *     (sigma_v / sigma_u) * (1 + delta_u) in that order.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_OK 0
#define ORACLE_SIGMA_OVERFLOW 1
#define ORACLE_BAD_INPUT (-1)
#define ORACLE_NOMEM (-2)

#define DIST_INF INT64_MAX

/* ---------------------------------------------------------------------- */
/* Binary min-heap keyed by tentative distance, with lazy deletion.        */
/* ---------------------------------------------------------------------- */

typedef struct {
    int64_t key;
    int32_t v;
} heap_item;

typedef struct {
    heap_item *a;
    int64_t len;
} heap;

static void heap_push(heap *h, int64_t key, int32_t v)
{
    int64_t i = h->len++;
    while (i > 0) {
        int64_t p = (i - 1) / 2;
        if (h->a[p].key <= key)
            break;
        h->a[i] = h->a[p];
        i = p;
    }
    h->a[i].key = key;
    h->a[i].v = v;
}

static heap_item heap_pop(heap *h)
{
    heap_item top = h->a[0];
    heap_item last = h->a[--h->len];
    int64_t i = 0;
    for (;;) {
        int64_t l = 2 * i + 1;
        if (l >= h->len)
            break;
        int64_t c = l;
        if (l + 1 < h->len && h->a[l + 1].key < h->a[l].key)
            c = l + 1;
        if (h->a[c].key >= last.key)
            break;
        h->a[i] = h->a[c];
        i = c;
    }
    if (h->len > 0)
        h->a[i] = last;
    return top;
}

/* ---------------------------------------------------------------------- */
/* Input validation                                                        */
/* ---------------------------------------------------------------------- */

int oracle_check_graph(int32_t n, int64_t nnz, const int64_t *row_ptr, const int32_t *col,
                       const int32_t *w)
{
    if (n < 0 || nnz < 0 || !row_ptr)
        return ORACLE_BAD_INPUT;
    if (row_ptr[0] != 0 || row_ptr[n] != nnz)
        return ORACLE_BAD_INPUT;
    for (int32_t v = 0; v < n; ++v)
        if (row_ptr[v + 1] < row_ptr[v])
            return ORACLE_BAD_INPUT;
    for (int64_t e = 0; e < nnz; ++e) {
        if (col[e] < 0 || col[e] >= n)
            return ORACLE_BAD_INPUT;
        if (w[e] < 1)
            return ORACLE_BAD_INPUT;
    }
    return ORACLE_OK;
}

/* ---------------------------------------------------------------------- */
/* Per-source forward pass: Dijkstra with shortest-path counting.          */
/* ---------------------------------------------------------------------- */

typedef struct {
    int64_t *d;       /* [n] */
    uint64_t *sigma;  /* [n] */
    double *delta;    /* [n] */
    uint8_t *done;    /* [n] */
    int32_t *order;   /* [n] settle order */
    heap h;           /* capacity nnz + 1 */
} workspace;

static int ws_alloc(workspace *ws, int32_t n, int64_t nnz)
{
    size_t nn = n > 0 ? (size_t)n : 1;
    ws->d = malloc(nn * sizeof(int64_t));
    ws->sigma = malloc(nn * sizeof(uint64_t));
    ws->delta = malloc(nn * sizeof(double));
    ws->done = malloc(nn);
    ws->order = malloc(nn * sizeof(int32_t));
    ws->h.a = malloc((size_t)(nnz + 1) * sizeof(heap_item));
    ws->h.len = 0;
    if (!ws->d || !ws->sigma || !ws->delta || !ws->done || !ws->order || !ws->h.a)
        return ORACLE_NOMEM;
    return ORACLE_OK;
}

static void ws_free(workspace *ws)
{
    free(ws->d);
    free(ws->sigma);
    free(ws->delta);
    free(ws->done);
    free(ws->order);
    free(ws->h.a);
}

/*
 * Dijkstra from s (Sec. 2.2): settle the unsettled vertex of least tentative
 * distance, then relax its arcs.  Path counts follow the rule of Alg. 2: a
 * strictly shorter distance replaces the count, an equal one adds to it.
 * With weights >= 1 every predecessor of v on a shortest path has a strictly
 * smaller distance and is settled (and has relaxed v) before v, so sigma[v]
 * is final when v is settled.  Writes the settle order; returns
 * ORACLE_SIGMA_OVERFLOW if a count exceeds 2^64 - 1.
 */
static int forward_pass(int32_t n, const int64_t *row_ptr, const int32_t *col, const int32_t *w,
                        int32_t s, workspace *ws, int32_t *n_order)
{
    int64_t *d = ws->d;
    uint64_t *sigma = ws->sigma;
    for (int32_t v = 0; v < n; ++v) {
        d[v] = DIST_INF;
        sigma[v] = 0;
        ws->done[v] = 0;
    }
    d[s] = 0;
    sigma[s] = 1;
    ws->h.len = 0;
    heap_push(&ws->h, 0, s);
    int32_t cnt = 0;
    while (ws->h.len > 0) {
        heap_item it = heap_pop(&ws->h);
        int32_t v = it.v;
        if (ws->done[v] || it.key != d[v])
            continue; /* stale heap entry */
        ws->done[v] = 1;
        ws->order[cnt++] = v;
        for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
            int32_t u = col[e];
            int64_t nd = d[v] + (int64_t)w[e];
            if (nd < d[u]) {
                d[u] = nd;
                sigma[u] = sigma[v];
                heap_push(&ws->h, nd, u);
            } else if (nd == d[u]) {
                uint64_t sum = sigma[u] + sigma[v];
                if (sum < sigma[u]) {
                    *n_order = cnt;
                    return ORACLE_SIGMA_OVERFLOW;
                }
                sigma[u] = sum;
            }
        }
    }
    *n_order = cnt;
    return ORACLE_OK;
}

/*
 * Dependency accumulation (Sec. 2.1 recursion, Alg. 3): walk the settle order
 * backwards; the successors u of v on shortest paths are the arc heads with
 * d[u] == d[v] + w(v, u).  They have larger distances, so their dependencies
 * are final.  Terms are summed in arc order.
 */
static void backward_pass(const int64_t *row_ptr, const int32_t *col, const int32_t *w,
                          workspace *ws, int32_t n_order, double *ebc)
{
    const int64_t *d = ws->d;
    const uint64_t *sigma = ws->sigma;
    double *delta = ws->delta;
    for (int32_t i = n_order - 1; i >= 0; --i) {
        int32_t v = ws->order[i];
        double acc = 0.0;
        for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
            int32_t u = col[e];
            if (d[u] != DIST_INF && d[u] == d[v] + (int64_t)w[e]) {
                double term = ((double)sigma[v] / (double)sigma[u]) * (1.0 + delta[u]);
                acc += term;
                /* edge betweenness: the same term is the dependency of source s
                   on the arc e = (v, u) (the tool's edge BC, Sec. 1) */
                if (ebc)
                    ebc[e] += term;
            }
        }
        delta[v] = acc;
    }
}

/*
 * Full per-source state: distances (DIST_INF when unreachable), path counts
 * (0 when unreachable) and dependencies (0 when unreachable).  Returns
 * ORACLE_OK, ORACLE_SIGMA_OVERFLOW or an input error.
 */
int oracle_source_state(int32_t n, int64_t nnz, const int64_t *row_ptr, const int32_t *col,
                        const int32_t *w, int32_t s, int64_t *d_out, uint64_t *sigma_out,
                        double *delta_out, int32_t *n_reached)
{
    if (s < 0 || s >= n)
        return ORACLE_BAD_INPUT;
    workspace ws;
    if (ws_alloc(&ws, n, nnz) != ORACLE_OK) {
        ws_free(&ws);
        return ORACLE_NOMEM;
    }
    int32_t cnt = 0;
    int rc = forward_pass(n, row_ptr, col, w, s, &ws, &cnt);
    if (rc == ORACLE_OK) {
        for (int32_t v = 0; v < n; ++v)
            ws.delta[v] = 0.0;
        backward_pass(row_ptr, col, w, &ws, cnt, NULL);
        memcpy(d_out, ws.d, (size_t)n * sizeof(int64_t));
        memcpy(sigma_out, ws.sigma, (size_t)n * sizeof(uint64_t));
        memcpy(delta_out, ws.delta, (size_t)n * sizeof(double));
        if (n_reached)
            *n_reached = cnt;
    }
    ws_free(&ws);
    return rc;
}

/* ---------------------------------------------------------------------- */
/* Betweenness over a multiset of sources, threaded over sources.          */
/* ---------------------------------------------------------------------- */

typedef struct {
    int32_t n;
    int64_t nnz;
    const int64_t *row_ptr;
    const int32_t *col;
    const int32_t *w;
    const int32_t *sources;
    int64_t lo, hi;         /* this thread's slice of the source list */
    double *bc;             /* this thread's partial [n] */
    double *ebc;            /* this thread's partial edge betweenness [nnz], or NULL */
    int64_t first_bad;      /* smallest source-list index that overflowed, or -1 */
    int rc;
} thread_job;

static void *bc_thread(void *arg)
{
    thread_job *job = arg;
    workspace ws;
    job->first_bad = -1;
    job->rc = ORACLE_OK;
    if (ws_alloc(&ws, job->n, job->nnz) != ORACLE_OK) {
        ws_free(&ws);
        job->rc = ORACLE_NOMEM;
        return NULL;
    }
    for (int64_t i = job->lo; i < job->hi; ++i) {
        int32_t s = job->sources[i];
        int32_t cnt = 0;
        if (forward_pass(job->n, job->row_ptr, job->col, job->w, s, &ws, &cnt) != ORACLE_OK) {
            if (job->first_bad < 0)
                job->first_bad = i;
            job->rc = ORACLE_SIGMA_OVERFLOW;
            continue;
        }
        backward_pass(job->row_ptr, job->col, job->w, &ws, cnt, job->ebc);
        for (int32_t j = 0; j < cnt; ++j) {
            int32_t v = ws.order[j];
            if (v != s)
                job->bc[v] += ws.delta[v];
        }
    }
    ws_free(&ws);
    return NULL;
}

/*
 * bc[v] = sum over the k listed sources s (with repetition) of delta_s(v),
 * v != s; when ebc is not NULL, ebc[e] receives the edge betweenness of every
 * arc e = (v, u): the sum over the sources of sigma_sv / sigma_su * (1 +
 * delta_s(u)) when e lies on a shortest path from s, i.e. the number of
 * shortest s-t paths through e divided by sigma_st, summed over all t.
 * Sources are split into contiguous slices, one per thread; the per-thread
 * partial sums are added in thread order, so the result is deterministic for
 * a fixed thread count.  *first_bad receives the smallest source-list index
 * whose path counts overflowed (or -1).
 */
int oracle_bc_edges(int32_t n, int64_t nnz, const int64_t *row_ptr, const int32_t *col,
                    const int32_t *w, const int32_t *sources, int64_t k, int32_t threads,
                    double *bc, double *ebc, int64_t *first_bad)
{
    int rc = oracle_check_graph(n, nnz, row_ptr, col, w);
    if (rc != ORACLE_OK)
        return rc;
    for (int64_t i = 0; i < k; ++i)
        if (sources[i] < 0 || sources[i] >= n)
            return ORACLE_BAD_INPUT;
    if (threads < 1)
        threads = 1;
    if ((int64_t)threads > k && k > 0)
        threads = (int32_t)k;
    for (int32_t v = 0; v < n; ++v)
        bc[v] = 0.0;
    if (ebc)
        for (int64_t e = 0; e < nnz; ++e)
            ebc[e] = 0.0;
    if (first_bad)
        *first_bad = -1;
    if (k == 0)
        return ORACLE_OK;

    thread_job *jobs = calloc((size_t)threads, sizeof(thread_job));
    pthread_t *tid = calloc((size_t)threads, sizeof(pthread_t));
    double *part = calloc((size_t)threads * (size_t)(n > 0 ? n : 1), sizeof(double));
    double *epart = ebc ? calloc((size_t)threads * (size_t)(nnz > 0 ? nnz : 1), sizeof(double))
                        : NULL;
    if (!jobs || !tid || !part || (ebc && !epart)) {
        free(jobs);
        free(tid);
        free(part);
        free(epart);
        return ORACLE_NOMEM;
    }
    for (int32_t t = 0; t < threads; ++t) {
        jobs[t].n = n;
        jobs[t].nnz = nnz;
        jobs[t].row_ptr = row_ptr;
        jobs[t].col = col;
        jobs[t].w = w;
        jobs[t].sources = sources;
        jobs[t].lo = k * t / threads;
        jobs[t].hi = k * (t + 1) / threads;
        jobs[t].bc = part + (size_t)t * (size_t)n;
        jobs[t].ebc = epart ? epart + (size_t)t * (size_t)nnz : NULL;
    }
    for (int32_t t = 1; t < threads; ++t)
        pthread_create(&tid[t], NULL, bc_thread, &jobs[t]);
    bc_thread(&jobs[0]);
    for (int32_t t = 1; t < threads; ++t)
        pthread_join(tid[t], NULL);

    rc = ORACLE_OK;
    int64_t bad = -1;
    for (int32_t t = 0; t < threads; ++t) {
        if (jobs[t].rc == ORACLE_NOMEM)
            rc = ORACLE_NOMEM;
        else if (jobs[t].rc == ORACLE_SIGMA_OVERFLOW && rc == ORACLE_OK)
            rc = ORACLE_SIGMA_OVERFLOW;
        if (jobs[t].first_bad >= 0 && (bad < 0 || jobs[t].first_bad < bad))
            bad = jobs[t].first_bad;
        for (int32_t v = 0; v < n; ++v)
            bc[v] += jobs[t].bc[v];
        if (ebc)
            for (int64_t e = 0; e < nnz; ++e)
                ebc[e] += jobs[t].ebc[e];
    }
    if (first_bad)
        *first_bad = bad;
    free(jobs);
    free(tid);
    free(part);
    free(epart);
    return rc;
}

int oracle_bc(int32_t n, int64_t nnz, const int64_t *row_ptr, const int32_t *col,
              const int32_t *w, const int32_t *sources, int64_t k, int32_t threads, double *bc,
              int64_t *first_bad)
{
    return oracle_bc_edges(n, nnz, row_ptr, col, w, sources, k, threads, bc, NULL, first_bad);
}
