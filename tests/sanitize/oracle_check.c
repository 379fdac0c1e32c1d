/*
 * The CPU oracle under the address and undefined-behaviour sanitizers: every
 * entry point on small graphs (threaded over sources), closed forms as a
 * sanity check, the overflow and bad-input paths.  Built together with
 * oracle/oracle.c by tests/test_sanitizers_cpu.py.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_bc(int32_t n, int64_t nnz, const int64_t *row_ptr, const int32_t *col,
              const int32_t *w, const int32_t *sources, int64_t k, int32_t threads, double *bc,
              int64_t *first_bad);
int oracle_bc_edges(int32_t n, int64_t nnz, const int64_t *row_ptr, const int32_t *col,
                    const int32_t *w, const int32_t *sources, int64_t k, int32_t threads,
                    double *bc, double *ebc, int64_t *first_bad);
int oracle_source_state(int32_t n, int64_t nnz, const int64_t *row_ptr, const int32_t *col,
                        const int32_t *w, int32_t s, int64_t *d_out, uint64_t *sigma_out,
                        double *delta_out, int32_t *n_reached);

static int fails = 0;
#define CHECK(c)                                                                           \
    do {                                                                                   \
        if (!(c)) {                                                                        \
            printf("FAIL %s:%d %s\n", __FILE__, __LINE__, #c);                             \
            ++fails;                                                                       \
        }                                                                                  \
    } while (0)

/* undirected path 0-1-...-(n-1), weights 1 + i % 3 */
static void path(int32_t n, int64_t *rp, int32_t *col, int32_t *w)
{
    int64_t e = 0;
    for (int32_t v = 0; v < n; ++v) {
        rp[v] = e;
        if (v > 0) {
            col[e] = v - 1;
            w[e++] = 1 + (v - 1) % 3;
        }
        if (v + 1 < n) {
            col[e] = v + 1;
            w[e++] = 1 + v % 3;
        }
    }
    rp[n] = e;
}

int main(void)
{
    enum { N = 40 };
    int64_t rp[N + 1];
    int32_t col[2 * N], w[2 * N], src[N];
    double bc[N], ebc[2 * N];
    int64_t bad = 0;
    path(N, rp, col, w);
    for (int i = 0; i < N; ++i)
        src[i] = i;
    for (int threads = 1; threads <= 8; threads *= 2) {
        CHECK(oracle_bc(N, rp[N], rp, col, w, src, N, threads, bc, &bad) == 0);
        for (int i = 0; i < N; ++i)
            CHECK(bc[i] == 2.0 * i * (N - 1 - i)); /* path closed form, ordered pairs */
        CHECK(oracle_bc_edges(N, rp[N], rp, col, w, src, N, threads, bc, ebc, &bad) == 0);
    }
    /* a random directed graph with ties, repeated sources */
    {
        enum { M = 300, E = 1500 };
        int64_t r2[M + 1];
        int32_t c2[E], w2[E], s2[64];
        uint32_t x = 12345;
        int64_t e = 0;
        for (int v = 0; v < M; ++v) {
            r2[v] = e;
            for (int j = 0; j < E / M; ++j) {
                x = x * 1103515245u + 12345u;
                c2[e] = (int32_t)((x >> 8) % M);
                w2[e++] = 1 + (int32_t)((x >> 20) % 3);
            }
        }
        r2[M] = e;
        for (int i = 0; i < 64; ++i)
            s2[i] = (i * 37) % M;
        double b2[M], eb2[E];
        CHECK(oracle_bc_edges(M, e, r2, c2, w2, s2, 64, 6, b2, eb2, &bad) == 0);
        int64_t d[M];
        uint64_t sg[M];
        double dl[M];
        int32_t nr = 0;
        CHECK(oracle_source_state(M, e, r2, c2, w2, 7, d, sg, dl, &nr) == 0);
        CHECK(nr >= 1 && d[7] == 0 && sg[7] == 1 && dl[7] == (double)(nr - 1));
    }
    /* 64 unit diamonds in a chain: the count at the end is 2^64, an overflow */
    {
        enum { K = 64, V = 3 * K + 1 };
        int64_t r3[V + 1];
        int32_t c3[8 * K], w3[8 * K];
        int64_t e = 0;
        for (int v = 0; v < V; ++v) {
            r3[v] = e;
            /* vertex 3i is the left end of diamond i; 3i+1, 3i+2 its middles */
            const int i = v / 3, r = v % 3;
            if (r == 0 && i < K) {
                c3[e] = v + 1; w3[e++] = 1;
                c3[e] = v + 2; w3[e++] = 1;
            }
            if (r == 1 || r == 2) {
                c3[e] = 3 * (i + 1); w3[e++] = 1;
            }
        }
        r3[V] = e;
        int32_t s3[3] = {1, 0, 2};
        double b3[V];
        CHECK(oracle_bc(V, e, r3, c3, w3, s3, 3, 2, b3, &bad) == 1 && bad == 1);
    }
    /* bad input */
    {
        int32_t badw[2 * N];
        for (int i = 0; i < 2 * N; ++i)
            badw[i] = w[i];
        badw[3] = 0;
        CHECK(oracle_bc(N, rp[N], rp, col, badw, src, N, 2, bc, &bad) < 0);
        int32_t badsrc[1] = {N};
        CHECK(oracle_bc(N, rp[N], rp, col, w, badsrc, 1, 2, bc, &bad) < 0);
    }
    printf("%s (%d failures)\n", fails ? "FAILED" : "OK", fails);
    return fails ? 1 : 0;
}
