// The library's host code under the address and undefined-behaviour
// sanitizers (host-side flags only; see build.build(sanitize=True)).
//
// bc_create_graph builds the whole device layout on the host (validation,
// transpose, symmetry check, renumbering, packing, edge map) before its
// first device call, so on a machine without a GPU every graph below runs
// all of that code and then stops with BC_E_DEVICE; with a GPU it is
// created and destroyed.  Argument checks of the other entry points run
// before any device work as well.
#include <cstdint>
#include <cstdio>
#include <vector>

#include "../../include/bc.h"

static int fails = 0;
#define CHECK(c)                                                                           \
    do {                                                                                   \
        if (!(c)) {                                                                        \
            std::printf("FAIL %s:%d %s (%s)\n", __FILE__, __LINE__, #c, bc_last_error());   \
            ++fails;                                                                       \
        }                                                                                  \
    } while (0)

struct Csr {
    int32_t n = 0;
    std::vector<int64_t> rp;
    std::vector<int32_t> col, w;
};

static uint32_t rnd(uint32_t &x)
{
    x = x * 1664525u + 1013904223u;
    return x >> 8;
}

// arcs (u, v, weight) -> CSR in the given order (rows not sorted)
static Csr from_arcs(int32_t n, const std::vector<int32_t> &u, const std::vector<int32_t> &v,
                     const std::vector<int32_t> &w)
{
    Csr g;
    g.n = n;
    g.rp.assign((size_t)n + 1, 0);
    for (int32_t a : u)
        g.rp[(size_t)a + 1]++;
    for (int32_t i = 0; i < n; ++i)
        g.rp[(size_t)i + 1] += g.rp[(size_t)i];
    std::vector<int64_t> at(g.rp.begin(), g.rp.end() - 1);
    g.col.resize(u.size());
    g.w.resize(u.size());
    for (size_t e = 0; e < u.size(); ++e) {
        const int64_t p = at[(size_t)u[e]]++;
        g.col[(size_t)p] = v[e];
        g.w[(size_t)p] = w[e];
    }
    return g;
}

// undirected: both arcs of every edge; skewed graphs have a few hubs
static Csr random_graph(int32_t n, int edges, bool directed, bool hubs, uint32_t seed, int wmax)
{
    std::vector<int32_t> u, v, w;
    uint32_t x = seed;
    for (int i = 0; i < edges; ++i) {
        int32_t a = (int32_t)(rnd(x) % (uint32_t)n), b = (int32_t)(rnd(x) % (uint32_t)n);
        if (hubs && (rnd(x) & 1))
            a = (int32_t)(rnd(x) % 3u); // vertices 0..2 collect most arcs
        const int32_t c = 1 + (int32_t)(rnd(x) % (uint32_t)wmax);
        u.push_back(a);
        v.push_back(b);
        w.push_back(c);
        if (!directed) {
            u.push_back(b);
            v.push_back(a);
            w.push_back(c);
        }
    }
    return from_arcs(n, u, v, w);
}

static bc_status create(const Csr &g, uint32_t flags)
{
    bc_graph *h = nullptr;
    const bc_status s = bc_create_graph(g.n, (int64_t)g.col.size(), g.rp.data(),
                                        g.col.empty() ? nullptr : g.col.data(),
                                        g.w.empty() ? nullptr : g.w.data(), flags, &h);
    if (s == BC_OK) {
        bc_graph_info info;
        CHECK(bc_get_graph_info(h, &info) == BC_OK && info.n == g.n);
        CHECK(bc_destroy_graph(h) == BC_OK);
    }
    return s;
}

int main()
{
    const uint32_t flagsets[] = {0, BC_KEEP_ORDER, BC_EDGE_BC, BC_EDGE_BC | BC_KEEP_ORDER};
    int made = 0;
    for (int directed = 0; directed < 2; ++directed)
        for (int hubs = 0; hubs < 2; ++hubs)
            for (int wmax : {1, 9, 3000, 70000})
                for (uint32_t f : flagsets) {
                    const Csr g = random_graph(500, 2500, directed, hubs, 7u + (uint32_t)wmax, wmax);
                    const bc_status s = create(g, f | (directed ? BC_DIRECTED : 0u));
                    CHECK(s == BC_OK || s == BC_E_DEVICE);
                    made += s == BC_OK;
                }
    // one vertex, no arcs; parallel arcs and self-loops
    {
        Csr one;
        one.n = 1;
        one.rp = {0, 0};
        const bc_status s = create(one, 0);
        CHECK(s == BC_OK || s == BC_E_DEVICE);
        const Csr par = from_arcs(4, {0, 0, 1, 1, 2, 2, 3}, {1, 1, 0, 0, 2, 3, 2}, {2, 2, 2, 2, 5, 1, 1});
        const bc_status t = create(par, BC_EDGE_BC);
        CHECK(t == BC_OK || t == BC_E_DEVICE);
    }
    // invalid graphs are refused before any device work
    {
        Csr g = random_graph(50, 200, false, false, 3u, 10);
        Csr bad = g;
        bad.col[5] = 50;
        CHECK(create(bad, 0) == BC_E_GRAPH);
        bad = g;
        bad.w[7] = 0;
        CHECK(create(bad, 0) == BC_E_WEIGHT);
        bad = g;
        bad.rp[10] = bad.rp[11] + 1;
        CHECK(create(bad, 0) == BC_E_GRAPH);
        bad = g;
        bad.w[0] = 11; // its reverse arc keeps the old weight
        CHECK(create(bad, 0) == BC_E_GRAPH);
        CHECK(create(bad, BC_DIRECTED) == BC_OK || create(bad, BC_DIRECTED) == BC_E_DEVICE);
        const Csr big = from_arcs(3, {0, 1, 1, 2}, {1, 0, 2, 1}, {1 << 30, 1 << 30, 1 << 30, 1 << 30});
        CHECK(create(big, 0) == BC_E_DIST_OVERFLOW);
        CHECK(create(g, 8u) == BC_E_INVAL);
        bc_graph *h = nullptr;
        CHECK(bc_create_graph(0, 0, g.rp.data(), nullptr, nullptr, 0, &h) == BC_E_INVAL);
        CHECK(bc_create_graph(g.n, -1, g.rp.data(), nullptr, nullptr, 0, &h) == BC_E_INVAL);
        CHECK(bc_create_graph(g.n, 10, g.rp.data(), nullptr, nullptr, 0, &h) == BC_E_INVAL);
        CHECK(bc_create_graph(g.n, 0, nullptr, nullptr, nullptr, 0, &h) == BC_E_INVAL);
        CHECK(bc_create_graph_device(g.n, 10, nullptr, nullptr, nullptr, 0, nullptr, &h) ==
              BC_E_INVAL);
    }
    // argument checks of the other entry points
    {
        bc_result *r = nullptr;
        double x = 0;
        CHECK(bc_compute(nullptr, nullptr, 0, nullptr, &r) == BC_E_INVAL);
        CHECK(bc_compute_device(nullptr, nullptr, 0, nullptr, &x, nullptr) == BC_E_INVAL);
        CHECK(bc_compute_edges(nullptr, nullptr, 0, nullptr, nullptr, &x) == BC_E_INVAL);
        CHECK(bc_source_state(nullptr, 0, nullptr, nullptr, nullptr, nullptr) == BC_E_INVAL);
        CHECK(bc_result_bc(nullptr, &x) == BC_E_INVAL);
        CHECK(bc_destroy_result(nullptr) == BC_OK);
        CHECK(bc_destroy_graph(nullptr) == BC_OK);
        CHECK(bc_update_arc_device(nullptr, nullptr, nullptr, 0, 1, 1, 2, nullptr, &x, nullptr,
                                   nullptr) == BC_E_INVAL);
        CHECK(bc_algo_bytes(10, 1, 20, 10, 9) == 20.0 * 18 + 72.0 * 10 + 24.0 * 9 + 20.0 * 10);
        CHECK(bc_version() != nullptr && bc_last_error() != nullptr);
    }
    std::printf("%s (%d failures, %d graphs created on a device)\n", fails ? "FAILED" : "OK",
                fails, made);
    return fails ? 1 : 0;
}
