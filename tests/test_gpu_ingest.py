"""Graphs built on the device (bc_create_graph_device from torch tensors)
against graphs built from host arrays (bc_create_graph), through the C ABI.

The device ingest must produce the same device layout: the graph information
agrees, distances and path counts are bit-identical, and centralities (node
and edge) agree with each other to 1e-12 and with the oracle to 1e-9.  The
dependency pass adds its terms with atomics, so two runs of the same graph
may differ in the last bits of a centrality; nothing else may differ.
Invalid arrays are rejected with the status the host ingest gives.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_1701_05975_amd import bc, graphgen as gg

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def rel_close(got, want, tol):
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    zero = want == 0
    assert np.all(got[zero] == 0), np.nonzero(got[zero])[0][:10]
    nz = ~zero
    err = np.abs(got[nz] - want[nz]) / np.abs(want[nz])
    assert err.size == 0 or err.max() <= tol, (float(err.max()), int(np.argmax(err)))


def tensors(csr):
    rp = torch.from_numpy(np.ascontiguousarray(csr.row_ptr, dtype=np.int64)).cuda()
    col = torch.from_numpy(np.ascontiguousarray(csr.col, dtype=np.int32)).cuda()
    w = torch.from_numpy(np.ascontiguousarray(csr.w, dtype=np.int32)).cuda()
    torch.cuda.synchronize()
    return rp, col, w


def device_graph(csr, **kw):
    rp, col, w = tensors(csr)
    stream = torch.cuda.current_stream().cuda_stream
    return bc.Graph.from_device(csr, rp, col, w, stream=stream, **kw)


def shuffled_rows(g, seed):
    """The same graph with every row's arcs in a random order (the caller's
    CSR need not be sorted by column)."""
    rng = np.random.default_rng(seed)
    col, w = g.col.copy(), g.w.copy()
    for v in range(g.n):
        a, b = int(g.row_ptr[v]), int(g.row_ptr[v + 1])
        p = rng.permutation(b - a) + a
        col[a:b], w[a:b] = g.col[p], g.w[p]
    return gg.CSRGraph(g.n, g.row_ptr.copy(), col, w, directed=g.directed, m=g.m,
                       name=g.name + "_shuffled", meta=dict(g.meta))


def cases():
    out = [
        shuffled_rows(gg.ba_graph(2000, 3, 1, 4, seed=7), seed=8),   # renumbered, unsorted rows
        shuffled_rows(gg.rmat_graph(10, 8 << 10, .57, .19, .19, 1, 3, seed=9), seed=10),
        gg.random_graph(65, 0.08, 1, 3, seed=1),                     # undirected, ties
        gg.random_graph(200, 0.03, 1, 2, seed=2, directed=True),     # directed, sinks
        gg.ba_graph(3000, 4, 1, 300, seed=3),                        # skewed: renumbered
        gg.rmat_graph(12, 8 << 12, .57, .19, .19, 1, 9, seed=4),     # directed, renumbered
        gg.random_graph(300, 0.02, 20000, 60000, seed=5),            # weights beyond 16 bits
        gg.grid_graph(60, 70, 100, 1, 255, seed=6),                  # grid, not renumbered
        gg.csr_from_arcs(70, [], [], [], directed=True),            # no arcs
        gg.csr_from_arcs(1, [], [], [], directed=False),            # one vertex
        # parallel arcs of equal and of different weights, self-loops
        gg.csr_from_arcs(6, [0, 0, 0, 1, 1, 2, 3, 3, 4, 4], [1, 1, 1, 0, 0, 3, 2, 4, 3, 4],
                         [2, 2, 5, 2, 2, 1, 1, 1, 1, 3], directed=True),
        gg.undirected_from_edges(5, [0, 0, 0, 1, 2, 3], [1, 1, 2, 2, 3, 3],
                                 [2, 3, 1, 1, 4, 2]),
    ]
    return out


@pytest.mark.parametrize("g", cases(), ids=lambda g: f"{g.name}_n{g.n}")
def test_device_ingest_matches_host_ingest(g):
    for keep in (False, True):
        H = bc.Graph(g, keep_order=keep, edges=True)
        D = device_graph(g, keep_order=keep, edges=True)
        assert D.info() == H.info()
        srcs = sorted({0, g.n // 2, g.n - 1})
        for s in srcs:
            dh, sh, lh = H.source_state(s)
            dd, sd, ld = D.source_state(s)
            assert np.array_equal(dh, dd) and np.array_equal(sh, sd), s
            rel_close(ld, lh, 1e-12)
        bh, _ = H.bc(None)
        bd, _ = D.bc(None)
        rel_close(bd, bh, 1e-12)
        rel_close(bd, oracle.oracle_bc(g, np.arange(g.n)), 1e-9)
        if g.nnz:
            _, eh = H.edge_bc(None)
            _, ed = D.edge_bc(None)
            rel_close(ed, eh, 1e-12)
        H.close()
        D.close()


def test_device_ingest_on_the_benchmark_grid_and_ba():
    for name in ("grid1000", "ba100k"):
        g = gg.config_graph(name)
        H = bc.Graph(g)
        D = device_graph(g)
        assert D.info() == H.info()
        srcs = gg.config_sources(name, g, parity=True)[:16]
        for s in srcs[:2]:
            dh, sh, _ = H.source_state(int(s))
            dd, sd, _ = D.source_state(int(s))
            assert np.array_equal(dh, dd) and np.array_equal(sh, sd)
        got, _ = D.bc(srcs)
        rel_close(got, oracle.oracle_bc(g, srcs), 1e-9)
        H.close()
        D.close()


def _status(fn):
    with pytest.raises(bc.BCError) as ei:
        fn()
    return ei.value.status


def test_device_validation_matches_host_validation():
    g = gg.path_graph(6, [3, 1, 4, 1, 5])
    bad = []
    rp = g.row_ptr.copy()
    rp[2] = rp[3] + 1                     # offsets decrease
    bad.append(("rows", gg.CSRGraph(g.n, rp, g.col, g.w, directed=False, m=g.m, name="x")))
    col = g.col.copy()
    col[3] = 6                            # head out of range
    bad.append(("col", gg.CSRGraph(g.n, g.row_ptr, col, g.w, directed=False, m=g.m, name="x")))
    w = g.w.copy()
    w[4] = 0                              # weight below 1
    bad.append(("w", gg.CSRGraph(g.n, g.row_ptr, g.col, w, directed=False, m=g.m, name="x")))
    w2 = g.w.copy()
    w2[0] = 9                             # reverse arc of another weight
    bad.append(("asym", gg.CSRGraph(g.n, g.row_ptr, g.col, w2, directed=False, m=g.m, name="x")))
    big = gg.path_graph(3, [2**30, 2**30])
    bad.append(("dist", big))
    for what, b in bad:
        hs = _status(lambda: bc.bc_create_graph(b.n, b.row_ptr, b.col, b.w,
                                                bc.BC_DIRECTED if b.directed else 0))
        rp_t, col_t, w_t = tensors(b)
        ds = _status(lambda: bc.bc_create_graph_device(
            b.n, int(col_t.numel()), rp_t.data_ptr(), col_t.data_ptr(), w_t.data_ptr(),
            bc.BC_DIRECTED if b.directed else 0))
        assert hs == ds, (what, hs, ds)
        assert ds in (bc.BC_E_GRAPH, bc.BC_E_WEIGHT, bc.BC_E_DIST_OVERFLOW), what
    # the asymmetric one is a valid directed graph
    a = bad[3][1]
    rp_t, col_t, w_t = tensors(a)
    h = bc.bc_create_graph_device(a.n, int(col_t.numel()), rp_t.data_ptr(), col_t.data_ptr(),
                                  w_t.data_ptr(), bc.BC_DIRECTED)
    bc.bc_destroy_graph(h)
