"""Dynamic update of one arc (CPU, oracle only): the endpoint rule that picks
the sources to run again is exactly the set of sources whose distances or path
counts change, every other source keeps its dependencies, and the centralities
of the changed graph follow from the old ones by replacing those sources'
dependencies.  (The rule is the dynamic extension Sec. 5 leaves to future
work; it rests on the shortest-path DAG of Sec. 2.1 being the set of tight
arcs.)"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_1701_05975_amd import bc, graphgen as gg

INF = oracle.oracle.INF64

GRAPHS = [
    gg.random_graph(40, 0.12, 1, 4, seed=11),                  # undirected, many ties
    gg.random_graph(45, 0.08, 1, 9, seed=12, directed=True),
    gg.ba_graph(60, 2, 1, 6, seed=13),
    gg.grid_graph(6, 7, 5, 1, 3, seed=14),
    gg.csr_from_arcs(5, [0, 0, 1, 2, 2, 3], [1, 1, 2, 3, 3, 4], [2, 2, 1, 1, 1, 3],
                     directed=True, name="parallel"),
    gg.cycle_graph(9, 2),
]
KINDS = ["insert", "delete", "increase", "decrease"]


def endpoint_rule(g_old, tail, head, w_old, w_new):
    """Sources s for which the changed arc is tight before (d[tail] + w_old =
    d[head]) or tight or shortening after (d[tail] + w_new <= d[head]), with the
    distances from s before the change; both arcs of an undirected edge."""
    arcs = [(tail, head)] if g_old.directed else [(tail, head), (head, tail)]
    hit = []
    for s in range(g_old.n):
        d = oracle.oracle_source_state(g_old, s)[0]
        for a, b in arcs:
            if d[a] == INF:
                continue
            if (w_old > 0 and d[b] != INF and d[a] + w_old == d[b]) or \
               (w_new > 0 and (d[b] == INF or d[a] + w_new <= d[b])):
                hit.append(s)
                break
    return np.array(hit, dtype=np.int32)


def cases():
    for gi, g in enumerate(GRAPHS):
        for ki, kind in enumerate(KINDS):
            for seed in range(2):
                try:
                    ch = gg.random_arc_change(g, kind, 1, 9, seed=100 * gi + 10 * ki + seed)
                except ValueError:
                    continue
                yield pytest.param(g, ch, id=f"{g.name or gi}-{kind}-{seed}")


@pytest.mark.parametrize("g,change", list(cases()))
def test_endpoint_rule_is_the_changed_set(g, change):
    g_new = gg.change_arc(g, *change)
    want = oracle.oracle_changed_sources(g, g_new)
    got = endpoint_rule(g, *change)
    assert np.array_equal(got, want), (change, got, want)
    # sources outside the set keep their dependencies
    outside = np.setdiff1d(np.arange(g.n), want)
    for s in outside[:: max(1, outside.shape[0] // 10)]:
        d0 = oracle.oracle_source_state(g, int(s))[2]
        d1 = oracle.oracle_source_state(g_new, int(s))[2]
        np.testing.assert_allclose(d1, d0, rtol=1e-12, atol=0)


@pytest.mark.parametrize("g,change", list(cases())[::3])
def test_replacing_the_changed_sources_gives_the_new_centralities(g, change):
    g_new = gg.change_arc(g, *change)
    A = oracle.oracle_changed_sources(g, g_new)
    old = oracle.oracle_bc(g, np.arange(g.n))
    want = oracle.oracle_bc(g_new, np.arange(g.n))
    got = old - oracle.oracle_bc(g, A) + oracle.oracle_bc(g_new, A)
    # three double sums, each exact to a few ulps of its own magnitude
    assert np.all(np.abs(got - want) <= 1e-12 * (np.abs(want) + np.abs(old)) + 1e-300)


@pytest.mark.parametrize("g", GRAPHS[:2], ids=lambda g: g.name)
def test_reversed_graph_gives_distances_to_a_vertex(g):
    r = gg.reversed_graph(g)
    for x in (0, g.n // 2, g.n - 1):
        to_x = oracle.oracle_source_state(r, x)[0]
        for s in range(g.n):
            assert to_x[s] == oracle.oracle_source_state(g, s)[0][x]


def test_change_arc_edits_one_arc():
    g = GRAPHS[4]  # two parallel 0 -> 1 arcs of weight 2
    h = gg.change_arc(g, 0, 1, 2, 5)
    assert h.nnz == g.nnz and sorted(h.w[h.row_ptr[0]:h.row_ptr[1]]) == [2, 5]
    h = gg.change_arc(g, 0, 1, 2, 0)
    assert h.nnz == g.nnz - 1
    u = gg.cycle_graph(5, 1)
    h = gg.change_arc(u, 0, 2, 0, 3)
    assert h.nnz == u.nnz + 2 and not h.directed
    with pytest.raises(ValueError):
        gg.change_arc(g, 0, 1, 7, 1)


def _err(fn):
    with pytest.raises(bc.BCError) as ei:
        fn()
    return ei.value.status


def test_update_arc_rejects_bad_arguments_before_device_work():
    assert _err(lambda: bc.bc_update_arc_device(None, None, None, 0, 1, 0, 1, 0)) == bc.BC_E_INVAL
