"""Edge betweenness on the GPU against the oracle (arc order of the caller's CSR)."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_1701_05975_amd import bc, graphgen as gg

pytestmark = pytest.mark.gpu


def rel_close(got, want, tol):
    zero = want == 0
    assert np.all(got[zero] == 0), np.nonzero(got[zero])[0][:10]
    err = np.abs(got[~zero] - want[~zero]) / np.abs(want[~zero])
    assert err.size == 0 or err.max() <= tol, float(err.max())


GRAPHS = [
    gg.random_graph(80, 0.06, 1, 2, seed=1),
    gg.random_graph(90, 0.05, 1, 9, seed=2, directed=True),
    gg.ba_graph(600, 3, 1, 30, seed=3),                         # renumbered on the device
    gg.rmat_graph(9, 8 << 9, .57, .19, .19, 1, 5, seed=4),      # directed, renumbered
    gg.csr_from_arcs(4, [0, 0, 1, 2, 2], [1, 1, 2, 3, 3], [2, 2, 1, 1, 1], directed=True),
]


@pytest.mark.parametrize("g", GRAPHS, ids=lambda g: g.name or "multi")
@pytest.mark.parametrize("keep_order", [False, True])
def test_edge_bc_matches_oracle(g, keep_order):
    G = bc.Graph(g, keep_order=keep_order, edges=True)
    want_bc, want_ebc = oracle.oracle_bc_edges(g, np.arange(g.n))
    for opts in (dict(), dict(accumulate=2), dict(lane_max_deg=1), dict(wg_threads=256, batch=5)):
        got_bc, got_ebc = G.edge_bc(None, **opts)
        rel_close(got_bc, want_bc, 1e-9)
        rel_close(got_ebc, want_ebc, 1e-9)


def test_edge_bc_closed_forms():
    n = 70
    g = gg.path_graph(n, np.arange(1, n))
    G = bc.Graph(g, edges=True)
    _, ebc = G.edge_bc(None)
    for v in range(n):
        for e in range(g.row_ptr[v], g.row_ptr[v + 1]):
            i = min(v, int(g.col[e]))
            assert ebc[e] == (i + 1) * (n - 1 - i)
    g = gg.star_graph(n, np.arange(1, n))
    _, ebc = bc.Graph(g, edges=True).edge_bc(None)
    assert np.all(ebc == n - 1)


def test_edge_bc_config_ba_sampled():
    g = gg.config_graph("ba100k")
    G = bc.Graph(g, edges=True)
    srcs = gg.config_sources("ba100k", g, parity=True)
    want_bc, want_ebc = oracle.oracle_bc_edges(g, srcs)
    got_bc, got_ebc = G.edge_bc(srcs)
    rel_close(got_bc, want_bc, 1e-9)
    rel_close(got_ebc, want_ebc, 1e-9)


def test_edge_bc_device_entry_and_errors():
    torch = pytest.importorskip("torch")
    g = gg.grid_graph(30, 40, 50, 1, 255, seed=6)
    G = bc.Graph(g, edges=True)
    srcs = np.arange(0, g.n, 11, dtype=np.int32)
    s_dev = torch.from_numpy(srcs).cuda()
    b = torch.empty(g.n, dtype=torch.float64, device="cuda")
    e = torch.empty(g.nnz, dtype=torch.float64, device="cuda")
    bc.bc_compute_edges_device(G.handle, s_dev.data_ptr(), len(srcs), b.data_ptr(), e.data_ptr())
    torch.cuda.synchronize()
    want_bc, want_ebc = oracle.oracle_bc_edges(g, srcs)
    rel_close(b.cpu().numpy(), want_bc, 1e-9)
    rel_close(e.cpu().numpy(), want_ebc, 1e-9)
    with pytest.raises(bc.BCError) as ei:
        G.edge_bc(srcs, mode=bc.BC_MODE_PLAIN)
    assert ei.value.status == bc.BC_E_INVAL
    H = bc.Graph(g)  # created without BC_EDGE_BC
    with pytest.raises(bc.BCError) as ei:
        H.edge_bc(srcs)
    assert ei.value.status == bc.BC_E_INVAL
