"""Source-interleaved form (BC_MODE_INTERLEAVED: 64 sources per wave, state
laid out [vertex][source]) against the oracle: centralities within 1e-9
relative, exact zero where the oracle has zero (every summand is
non-negative, so any summation order stays within that bound)."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_1701_05975_amd import bc, graphgen as gg
from test_gpu_parity import rel_close, small_graphs

pytestmark = pytest.mark.gpu

IL = bc.BC_MODE_INTERLEAVED
OPTS = [dict(mode=IL), dict(mode=IL, delta=1), dict(mode=IL, delta=1 << 28),
        dict(mode=IL, batch=64), dict(mode=IL, batch=100)]


@pytest.mark.parametrize("g", small_graphs(), ids=lambda g: f"{g.name}_s{g.meta['seed']}")
def test_small_graphs_all_sources(g):
    print(f"interleaved {g.name} n={g.n}", flush=True)
    G = bc.Graph(g)
    want = oracle.oracle_bc(g, np.arange(g.n))
    for opts in OPTS:
        got, st = G.bc(None, **opts)
        rel_close(got, want, 1e-9)
        assert st["sources"] == g.n and st["mode"] == IL
    G.close()


def test_ragged_repeated_and_keep_order():
    g = gg.ba_graph(900, 3, 1, 40, seed=31)
    rng = np.random.default_rng(3)
    srcs = rng.integers(0, g.n, size=203).astype(np.int32)   # repeats, 3 full groups + 11
    srcs[:5] = srcs[5]
    want = oracle.oracle_bc(g, srcs)
    for keep in (False, True):
        G = bc.Graph(g, keep_order=keep)
        for opts in (dict(mode=IL), dict(mode=IL, batch=70)):
            got, _ = G.bc(srcs, **opts)
            rel_close(got, want, 1e-9)


def test_closed_forms_and_degenerate_inputs():
    n = 130
    path = gg.path_graph(n, np.arange(1, n))
    got, _ = bc.Graph(path).bc(None, mode=IL)
    i = np.arange(n)
    assert np.array_equal(got, 2.0 * i * (n - 1 - i))
    star = gg.star_graph(n, np.arange(1, n))
    got, _ = bc.Graph(star).bc(None, mode=IL)
    assert got[0] == (n - 1) * (n - 2) and np.all(got[1:] == 0)
    e = gg.csr_from_arcs(70, [], [], [], directed=True)
    got, _ = bc.Graph(e).bc(None, mode=IL)
    assert np.all(got == 0)
    one = gg.csr_from_arcs(1, [], [], [], directed=False)
    got, _ = bc.Graph(one).bc(None, mode=IL)
    assert got.tolist() == [0.0]
    got, st = bc.Graph(path).bc(np.zeros(0, np.int32), mode=IL)
    assert np.all(got == 0) and st["sources"] == 0


def test_directed_sinks_parallel_arcs_and_ties():
    src = [0, 0, 0, 1, 2, 3, 3, 4]
    dst = [1, 2, 2, 3, 3, 4, 4, 5]
    w = [1, 1, 1, 1, 1, 2, 2, 1]
    g = gg.csr_from_arcs(6, src, dst, w, directed=True)
    got, _ = bc.Graph(g).bc(None, mode=IL)
    rel_close(got, oracle.oracle_bc(g, np.arange(6)), 1e-12)
    g = gg.unit_grid(20, 20)
    got, _ = bc.Graph(g).bc(None, mode=IL, delta=2)
    rel_close(got, oracle.oracle_bc(g, np.arange(g.n)), 1e-9)


def test_sigma_overflow_and_bad_sources():
    G = bc.Graph(gg.diamond_chain(64))
    with pytest.raises(bc.BCError) as ei:
        G.bc(np.array([1, 0, 2], np.int32), mode=IL)
    assert ei.value.status == bc.BC_E_SIGMA_OVERFLOW
    assert "index 1" in ei.value.msg
    got, _ = G.bc(np.array([1], np.int32), mode=IL)
    assert np.isfinite(got).all()
    with pytest.raises(bc.BCError) as ei:
        G.source_state(0, mode=IL)
    assert ei.value.status == bc.BC_E_INVAL


def test_device_sources_out_of_range_rejected():
    torch = pytest.importorskip("torch")
    g = gg.path_graph(40)
    G = bc.Graph(g)
    s = torch.tensor([0, 5, 40], dtype=torch.int32, device="cuda")
    out = torch.empty(g.n, dtype=torch.float64, device="cuda")
    with pytest.raises(bc.BCError) as ei:
        bc.bc_compute_device(G.handle, s.data_ptr(), 3, out.data_ptr(), bc.make_options(mode=IL))
    assert ei.value.status == bc.BC_E_INVAL


@pytest.mark.parametrize("name,count", [("ba100k", 256), ("grid1000", 64), ("rmat22", 64)])
def test_config_sampled_sources(name, count):
    """Each configuration's graph at full size, the first sampled sources of
    its source list (as the benchmark draws them)."""
    g = gg.config_graph(name)
    srcs = gg.config_sources(name, g, parity=True)[:count]
    print(f"interleaved {name} n={g.n} k={len(srcs)}", flush=True)
    G = bc.Graph(g)
    got, _ = G.bc(srcs, mode=IL)
    rel_close(got, oracle.oracle_bc(g, srcs), 1e-9)
