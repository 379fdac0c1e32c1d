"""Pins for the CPU oracle, independent of the oracle itself (CPU only).

Each check compares the oracle with something the paper or mathematics fixes:
literal path enumeration and exact rational brute force (Eq. 1, Sec. 2.1),
closed forms, invariants, the worked example of Fig. 1(a) (Sec. 3.2), and
library routines (scipy's Dijkstra distances, networkx betweenness).
"""
from __future__ import annotations

import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from brute import enumerate_bc, enumerate_ebc, hop_invariant, pairwise_bc
from paper_1701_05975_amd import graphgen as gg

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def close(a, b, rel=1e-12):
    a = float(a)
    b = float(b)
    if b == 0:
        return a == 0
    return abs(a - b) <= rel * abs(b)


def small_cases():
    cases = []
    for seed in range(6):
        # weights in {1,2} force many equal-length paths
        cases.append(gg.random_graph(8, 0.45, 1, 2, seed=seed))
        cases.append(gg.random_graph(7, 0.35, 1, 3, seed=100 + seed, directed=True))
    return cases


@pytest.mark.parametrize("g", small_cases(), ids=lambda g: g.name + str(g.meta.get("seed")))
def test_oracle_matches_literal_path_enumeration(g):
    bc_exact, dist, sig = enumerate_bc(g)
    bc = oracle.oracle_bc(g, np.arange(g.n), threads=2)
    for v in range(g.n):
        assert close(bc[v], bc_exact[v]), (v, bc[v], bc_exact[v])
    for s in range(g.n):
        d, sigma, delta, nr = oracle.oracle_source_state(g, s)
        for t in range(g.n):
            if t == s:
                assert d[t] == 0 and sigma[t] == 1
            elif (s, t) in dist:
                assert d[t] == dist[(s, t)]
                assert int(sigma[t]) == sig[(s, t)]
            else:
                assert d[t] == oracle.oracle.INF64 and sigma[t] == 0 and delta[t] == 0


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("directed", [False, True])
def test_oracle_matches_pairwise_definition(seed, directed):
    n = 40
    g = gg.random_graph(n, 0.12 if directed else 0.09, 1, 3, seed=1000 + seed, directed=directed)
    srcs = list(range(0, n, 3)) + [5, 5]  # a multiset, with a repeated source
    bc_exact, D, S = pairwise_bc(g, srcs)
    bc = oracle.oracle_bc(g, srcs, threads=3)
    for v in range(n):
        assert close(bc[v], bc_exact[v], 1e-12), (v, bc[v], float(bc_exact[v]))
    for s in (0, 7):
        d, sigma, _, _ = oracle.oracle_source_state(g, s)
        for t in range(n):
            if D[s][t] == float("inf"):
                assert sigma[t] == 0
            else:
                assert d[t] == D[s][t] and int(sigma[t]) == S[s][t]


def test_fig1a_worked_example():
    """Sec. 3.2, Fig. 1(a): the text states sigma(v3) = 2."""
    lines = open(os.path.join(GOLDEN, "fig1a.txt")).read().splitlines()
    eu, ev, ew, expect = [], [], [], []
    n = s = None
    for ln in lines:
        if not ln or ln.startswith("#"):
            continue
        tok = ln.split()
        if tok[0] == "n":
            n = int(tok[1])
        elif tok[0] == "source":
            s = int(tok[1])
        elif tok[0] == "edge":
            eu.append(int(tok[1])); ev.append(int(tok[2])); ew.append(int(tok[3]))
        elif tok[0] == "expect":
            expect.append((tok[1], int(tok[2]), int(tok[3])))
    g = gg.undirected_from_edges(n, eu, ev, ew)
    d, sigma, delta, _ = oracle.oracle_source_state(g, s)
    for kind, v, val in expect:
        assert kind == "sigma" and int(sigma[v]) == val


# ---------------------------------------------------------------- closed forms

@pytest.mark.parametrize("n", [2, 3, 7, 30])
def test_star_closed_form(n):
    rng = np.random.default_rng(n)
    g = gg.star_graph(n, rng.integers(1, 50, size=n - 1))
    bc = oracle.oracle_bc(g, np.arange(n))
    assert bc[0] == (n - 1) * (n - 2)
    assert np.all(bc[1:] == 0)


@pytest.mark.parametrize("n", [2, 5, 12, 101])
def test_path_closed_form(n):
    rng = np.random.default_rng(n)
    g = gg.path_graph(n, rng.integers(1, 1000, size=n - 1))
    bc = oracle.oracle_bc(g, np.arange(n))
    for i in range(n):
        assert bc[i] == 2 * i * (n - 1 - i)


@pytest.mark.parametrize("n", [3, 4, 9, 10, 31, 64])
def test_cycle_closed_form(n):
    g = gg.cycle_graph(n)
    bc = oracle.oracle_bc(g, np.arange(n))
    want = (n - 1) * (n - 3) / 4 if n % 2 else (n - 2) ** 2 / 4
    assert np.allclose(bc, want, rtol=1e-13, atol=0)
    if n % 2 == 0:
        _, sigma, _, _ = oracle.oracle_source_state(g, 0)
        assert sigma[n // 2] == 2


def test_complete_graph_all_zero():
    g = gg.complete_graph(12)
    assert np.all(oracle.oracle_bc(g, np.arange(12)) == 0)


@pytest.mark.parametrize("a,b", [(5, 7), (34, 34)])
def test_unit_grid_corner_binomial(a, b):
    g = gg.unit_grid(a, b)
    d, sigma, _, _ = oracle.oracle_source_state(g, 0)
    for i in range(a):
        for j in range(b):
            v = i * b + j
            assert d[v] == i + j
            assert int(sigma[v]) == math.comb(i + j, i)


def test_unit_grid_35_overflows():
    g = gg.unit_grid(35, 35)
    assert math.comb(68, 34) >= 2 ** 64
    with pytest.raises(oracle.SigmaOverflow):
        oracle.oracle_source_state(g, 0)


def test_diamond_chain_limits():
    g = gg.diamond_chain(63)
    d, sigma, _, _ = oracle.oracle_source_state(g, 0)
    assert int(sigma[3 * 63]) == 2 ** 63
    g = gg.diamond_chain(64)
    with pytest.raises(oracle.SigmaOverflow) as ei:
        oracle.oracle_bc(g, [1, 0, 2])
    assert ei.value.first_bad == 1


# ---------------------------------------------------------------- invariants

@pytest.mark.parametrize("seed", range(3))
def test_sum_of_bc_is_mean_interior_count(seed):
    g = gg.random_graph(30, 0.15, 1, 2, seed=77 + seed)
    srcs = list(range(30))
    want = hop_invariant(g, srcs)
    bc = oracle.oracle_bc(g, srcs)
    assert close(bc.sum(), want, 1e-12)


@pytest.mark.parametrize("seed", range(3))
def test_source_dependency_counts_reached(seed):
    g = gg.random_graph(60, 0.05, 1, 9, seed=seed, directed=bool(seed % 2))
    for s in range(0, 60, 7):
        d, sigma, delta, nr = oracle.oracle_source_state(g, s)
        reached = int(np.sum(d != oracle.oracle.INF64))
        assert nr == reached
        assert close(delta[s], reached - 1, 1e-12)


def test_trees_give_integer_dependencies():
    """Tie-free graphs (every sigma = 1): each dependency is a subtree size."""
    g = gg.ba_graph(300, 1, 1, 50, seed=3)  # m = 1 gives a tree
    bc = oracle.oracle_bc(g, np.arange(g.n))
    assert np.all(bc == np.round(bc))


# ---------------------------------------------------------------- library routines

@pytest.mark.parametrize("name", ["er1000", "grid_small", "ba2k"])
def test_distances_match_scipy_dijkstra(name):
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import dijkstra
    if name == "er1000":
        g = gg.config_graph("er1000")
    elif name == "grid_small":
        g = gg.grid_graph(40, 50, 80, 1, 255, seed=5)
    else:
        g = gg.ba_graph(2000, 5, 1, 1000, seed=9)
    A = csr_matrix((g.w.astype(np.float64), g.col, g.row_ptr), shape=(g.n, g.n))
    srcs = [0, 17, g.n - 1]
    D = dijkstra(A, directed=True, indices=srcs)
    for i, s in enumerate(srcs):
        d, _, _, _ = oracle.oracle_source_state(g, s)
        ref = np.where(np.isinf(D[i]), oracle.oracle.INF64, D[i]).astype(np.int64)
        assert np.array_equal(d, ref)


@pytest.mark.parametrize("directed", [False, True])
def test_matches_networkx_betweenness(directed):
    nx = pytest.importorskip("networkx")
    g = gg.random_graph(120, 0.05, 1, 4, seed=11, directed=directed)
    G = nx.DiGraph() if directed else nx.Graph()
    G.add_nodes_from(range(g.n))
    for v in range(g.n):
        for e in range(g.row_ptr[v], g.row_ptr[v + 1]):
            G.add_edge(v, int(g.col[e]), weight=int(g.w[e]))
    ref = nx.betweenness_centrality(G, weight="weight", normalized=False)
    bc = oracle.oracle_bc(g, np.arange(g.n))
    scale = 1.0 if directed else 2.0  # networkx halves undirected sums
    for v in range(g.n):
        assert abs(bc[v] - scale * ref[v]) <= 1e-9 * max(1.0, abs(bc[v]))


def test_rejects_bad_input():
    g = gg.path_graph(4, [1, 0, 2])
    with pytest.raises(oracle.OracleError):
        oracle.oracle_bc(g, [0])
    g = gg.path_graph(4)
    with pytest.raises(oracle.OracleError):
        oracle.oracle_bc(g, [4])


def test_empty_source_list_and_edgeless_graph():
    g = gg.path_graph(5)
    assert np.all(oracle.oracle_bc(g, []) == 0)
    g = gg.csr_from_arcs(6, [], [], [], directed=True)
    assert np.all(oracle.oracle_bc(g, np.arange(6)) == 0)
    d, sigma, delta, nr = oracle.oracle_source_state(g, 2)
    assert nr == 1 and d[2] == 0 and sigma[2] == 1 and delta[2] == 0


def test_thread_count_does_not_change_result_beyond_rounding():
    g = gg.ba_graph(3000, 5, 1, 1000, seed=4)
    srcs = np.arange(0, 3000, 13)
    a = oracle.oracle_bc(g, srcs, threads=1)
    b = oracle.oracle_bc(g, srcs, threads=5)
    assert np.allclose(a, b, rtol=1e-12, atol=0)


# ---------------------------------------------------------------- edge betweenness

@pytest.mark.parametrize("g", small_cases()[:6], ids=lambda g: g.name + str(g.meta.get("seed")))
def test_edge_bc_matches_literal_enumeration(g):
    want = enumerate_ebc(g)
    bc, ebc = oracle.oracle_bc_edges(g, np.arange(g.n), threads=2)
    for e in range(g.nnz):
        assert close(ebc[e], want[e]), (e, ebc[e], float(want[e]))
    assert np.allclose(bc, oracle.oracle_bc(g, np.arange(g.n)), rtol=1e-14, atol=0)


def test_edge_bc_parallel_arcs_are_distinct_paths():
    g = gg.csr_from_arcs(3, [0, 0, 1], [1, 1, 2], [2, 2, 1], directed=True)
    _, ebc = oracle.oracle_bc_edges(g, np.arange(3))
    want = enumerate_ebc(g)
    assert [float(x) for x in want] == list(ebc)
    assert ebc[0] == ebc[1] == 1.0  # each parallel arc carries half of 0->1 and of 0->2


@pytest.mark.parametrize("n", [2, 6, 40])
def test_edge_bc_path_and_star_closed_forms(n):
    rng = np.random.default_rng(n)
    g = gg.path_graph(n, rng.integers(1, 100, size=n - 1))
    _, ebc = oracle.oracle_bc_edges(g, np.arange(n))
    for v in range(n):
        for e in range(g.row_ptr[v], g.row_ptr[v + 1]):
            u = int(g.col[e])
            i = min(u, v)  # the edge {i, i+1}
            assert ebc[e] == (i + 1) * (n - 1 - i)
    g = gg.star_graph(n, rng.integers(1, 100, size=n - 1))
    _, ebc = oracle.oracle_bc_edges(g, np.arange(n))
    assert np.all(ebc == n - 1)


@pytest.mark.parametrize("seed", range(3))
def test_edge_bc_sum_is_bc_sum_plus_reached_pairs(seed):
    g = gg.random_graph(50, 0.08, 1, 3, seed=500 + seed, directed=bool(seed % 2))
    srcs = np.arange(0, 50, 2)
    bc, ebc = oracle.oracle_bc_edges(g, srcs)
    pairs = 0
    for s in srcs:
        d, _, _, nr = oracle.oracle_source_state(g, int(s))
        pairs += nr - 1
    assert close(ebc.sum(), bc.sum() + pairs, 1e-12)
