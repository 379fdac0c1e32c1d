"""GPU parity: the HIP library against the CPU oracle, through the C ABI.

Bar: distances and shortest-path counts bit-exact; per-source dependencies
within 1e-12 relative and centralities within 1e-9 relative (exact zero
where the oracle has zero).  All tests need an MI355X.
"""
from __future__ import annotations

import math

import numpy as np
import pytest

import oracle
from paper_1701_05975_amd import bc, graphgen as gg
from paper_1701_05975_amd.launch import LAUNCH
from oracle_cache import cached_oracle_bc

pytestmark = pytest.mark.gpu

INF64 = np.iinfo(np.int64).max
INT32_MAX = 2**31 - 1

# Option sets that change the schedule but never the result beyond rounding.
OPTION_SETS = [
    dict(),
    dict(mode=bc.BC_MODE_PLAIN),
    dict(delta=1),
    dict(delta=1 << 28),
    dict(lane_max_deg=1),
    dict(lane_max_deg=1 << 20),
    dict(wg_threads=1024),
    dict(wg_threads=512, batch=3),
    dict(accumulate=2),
    dict(mode=bc.BC_MODE_PLAIN, delta=1, lane_max_deg=1),
    dict(lds_vertices=-1),
    dict(lds_vertices=5, wg_threads=256),
    dict(dep_mode=2),
    dict(dep_mode=2, accumulate=2, lane_max_deg=1),
    dict(virtual_warp=1),
    dict(virtual_warp=8, node_parallel=1),
    dict(virtual_warp=64),
    dict(node_parallel=1, mode=bc.BC_MODE_BATCHED, wg_threads=512),
    dict(mode=bc.BC_MODE_PLAIN, virtual_warp=16),
    dict(lds_bits=16),
    dict(lds_bits=32),
    dict(lds_bits=16, lds_vertices=5, wg_threads=512),
    dict(lds_bits=8),
    dict(lds_bits=8, lds_vertices=5, wg_threads=512),
    dict(lds_bits=8, delta=1, far_buckets=1),
    dict(lds_bits=8, delta=1 << 28),
    dict(lds_bits=8, delta=3, far_buckets=1, accumulate=2, wg_threads=256),
    dict(far_buckets=1),
    dict(far_buckets=1, delta=1, wg_threads=256),
    dict(far_buckets=1, delta=2, lds_vertices=-1, accumulate=2),
    dict(far_buckets=2, delta=1),
    dict(far_buckets=1, delta=1, wg_threads=512, batch=7),
]


def rel_close(got, want, tol):
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    zero = want == 0
    assert np.all(got[zero] == 0), np.nonzero(got[zero])[0][:10]
    nz = ~zero
    err = np.abs(got[nz] - want[nz]) / np.abs(want[nz])
    assert err.size == 0 or err.max() <= tol, (float(err.max()), int(np.argmax(err)))


def check_state(g, G, s, **opts):
    d, sg, dl = G.source_state(s, **opts)
    od, osg, odl, nr = oracle.oracle_source_state(g, s)
    od32 = np.where(od == INF64, INT32_MAX, od).astype(np.int32)
    assert np.array_equal(d, od32), (s, np.nonzero(d != od32)[0][:10])
    assert np.array_equal(sg, osg), (s, np.nonzero(sg != osg)[0][:10])
    rel_close(dl, odl, 1e-12)


def check_bc(g, G, sources, tol=1e-9, **opts):
    got, st = G.bc(sources, **opts)
    want = oracle.oracle_bc(g, np.arange(g.n) if sources is None else sources)
    rel_close(got, want, tol)
    return got, st


# ------------------------------------------------------------------ small graphs

def small_graphs():
    out = []
    for n, p, wl, wh, seed, directed in [
        (1, 0.0, 1, 1, 0, False), (2, 1.0, 1, 5, 1, False), (7, 0.5, 1, 2, 2, False),
        (63, 0.08, 1, 2, 3, False), (64, 0.1, 1, 3, 4, True), (65, 0.06, 1, 100, 5, False),
        (200, 0.03, 1, 2, 6, True), (513, 0.012, 1, 9, 7, False), (1037, 0.006, 1, 1000, 8, True),
    ]:
        out.append(gg.random_graph(n, p, wl, wh, seed=seed, directed=directed))
    # skewed graphs: renumbered by in-degree on the device
    out.append(gg.ba_graph(700, 3, 1, 20, seed=9))
    out.append(gg.rmat_graph(10, 8 << 10, .57, .19, .19, 1, 9, seed=10))
    # heavy weights: most distances exceed 16 bits (16-bit LDS entries overflow
    # to device memory), one of them skewed so that 16-bit entries are the default
    out.append(gg.random_graph(300, 0.02, 20000, 60000, seed=11, directed=False))
    out.append(gg.ba_graph(700, 3, 1, 30000, seed=13))
    return out


@pytest.mark.parametrize("g", small_graphs(), ids=lambda g: f"{g.name}_s{g.meta['seed']}")
def test_small_graphs_all_sources_every_option_set(g):
    G = bc.Graph(g)
    want = oracle.oracle_bc(g, np.arange(g.n))
    srcs = sorted(set([0, g.n // 2, g.n - 1]))
    for opts in OPTION_SETS:
        got, st = G.bc(None, **opts)
        rel_close(got, want, 1e-9)
        assert st["sources"] == g.n
        for s in srcs:
            check_state(g, G, s, **opts)
    G.close()


def test_renumbered_graph_matches_caller_order():
    g = gg.ba_graph(3000, 4, 1, 300, seed=12)
    A = bc.Graph(g)
    B = bc.Graph(g, keep_order=True)
    assert A.info()["renumbered"] == 1 and B.info()["renumbered"] == 0
    srcs = np.arange(0, 3000, 5, dtype=np.int32)
    a, _ = A.bc(srcs)
    b, _ = B.bc(srcs)
    rel_close(a, b, 1e-12)
    for s in (0, 7, 2999):
        da, sa, la = A.source_state(s)
        db, sb, lb = B.source_state(s)
        assert np.array_equal(da, db) and np.array_equal(sa, sb)
        rel_close(la, lb, 1e-12)
    rel_close(a, oracle.oracle_bc(g, srcs), 1e-9)


def test_device_sources_out_of_range_rejected():
    torch = pytest.importorskip("torch")
    g = gg.path_graph(40)
    G = bc.Graph(g)
    out = torch.empty(g.n, dtype=torch.float64, device="cuda")
    for bad in (-1, 40):
        s_dev = torch.tensor([3, bad, 5], dtype=torch.int32, device="cuda")
        with pytest.raises(bc.BCError) as ei:
            bc.bc_compute_device(G.handle, s_dev.data_ptr(), 3, out.data_ptr())
        assert ei.value.status == bc.BC_E_INVAL
    # still usable afterwards
    got, _ = G.bc(np.array([3, 5], np.int32))
    rel_close(got, oracle.oracle_bc(g, [3, 5]), 1e-12)


def test_schedules_give_bit_identical_distances_and_counts():
    g = gg.random_graph(700, 0.01, 1, 3, seed=42)
    G = bc.Graph(g)
    ref = None
    for opts in OPTION_SETS:
        for s in (0, 123, 699):
            d, sg, _ = G.source_state(s, **opts)
            if ref is None:
                ref = {}
            if s in ref:
                assert np.array_equal(ref[s][0], d) and np.array_equal(ref[s][1], sg)
            else:
                ref[s] = (d, sg)


# ------------------------------------------------------------------ closed forms

@pytest.mark.parametrize("n", [2, 3, 65, 300])
def test_star_and_path_closed_forms(n):
    rng = np.random.default_rng(n)
    star = gg.star_graph(n, rng.integers(1, 50, size=n - 1))
    G = bc.Graph(star)
    for opts in (dict(), dict(mode=bc.BC_MODE_PLAIN)):
        got, _ = G.bc(None, **opts)
        assert got[0] == (n - 1) * (n - 2) and np.all(got[1:] == 0)
    path = gg.path_graph(n, rng.integers(1, 1000, size=n - 1))
    G = bc.Graph(path)
    for opts in (dict(), dict(mode=bc.BC_MODE_PLAIN), dict(delta=1)):
        got, _ = G.bc(None, **opts)
        assert np.array_equal(got, [2 * i * (n - 1 - i) for i in range(n)])


@pytest.mark.parametrize("n", [9, 10, 129])
def test_cycle_and_complete(n):
    G = bc.Graph(gg.cycle_graph(n))
    got, _ = G.bc(None)
    want = (n - 1) * (n - 3) / 4 if n % 2 else (n - 2) ** 2 / 4
    rel_close(got, np.full(n, want), 1e-12)
    G = bc.Graph(gg.complete_graph(40))
    got, _ = G.bc(None)
    assert np.all(got == 0)


def test_unit_grid_binomial_counts():
    g = gg.unit_grid(34, 34)
    G = bc.Graph(g)
    for opts in (dict(), dict(mode=bc.BC_MODE_PLAIN)):
        d, sg, _ = G.source_state(0, **opts)
        for i in (0, 5, 33):
            for j in (0, 17, 33):
                assert d[i * 34 + j] == i + j
                assert int(sg[i * 34 + j]) == math.comb(i + j, i)


def test_fig1a_example():
    g = gg.undirected_from_edges(4, [0, 0, 1, 2], [1, 2, 2, 3], [1, 2, 1, 1])
    G = bc.Graph(g)
    for opts in OPTION_SETS:
        _, sg, _ = G.source_state(0, **opts)
        assert int(sg[3]) == 2


# ------------------------------------------------------------------ overflow and edges

def test_sigma_overflow_reported_with_first_source():
    G = bc.Graph(gg.diamond_chain(63))
    d, sg, _ = G.source_state(0)
    assert int(sg[3 * 63]) == 2**63
    G = bc.Graph(gg.diamond_chain(64))
    for opts in (dict(), dict(mode=bc.BC_MODE_PLAIN)):
        with pytest.raises(bc.BCError) as ei:
            G.bc(np.array([1, 0, 2], np.int32), **opts)
        assert ei.value.status == bc.BC_E_SIGMA_OVERFLOW
        assert "index 1" in ei.value.msg
    # the graph stays usable after the error
    got, _ = G.bc(np.array([1], np.int32))
    assert np.isfinite(got).all()


def test_grid_35_overflows():
    G = bc.Graph(gg.unit_grid(35, 35))
    with pytest.raises(bc.BCError) as ei:
        G.bc(np.array([0], np.int32))
    assert ei.value.status == bc.BC_E_SIGMA_OVERFLOW


def test_empty_and_degenerate_inputs():
    g = gg.path_graph(5)
    G = bc.Graph(g)
    got, st = G.bc(np.zeros(0, np.int32))
    assert np.all(got == 0) and st["sources"] == 0
    got, _ = G.bc(np.zeros(0, np.int32), mode=bc.BC_MODE_PLAIN)
    assert np.all(got == 0)
    # repeated sources count once per occurrence
    got, _ = G.bc(np.array([0, 0, 4], np.int32))
    rel_close(got, oracle.oracle_bc(g, [0, 0, 4]), 1e-12)
    # edgeless directed graph; single vertex
    e = gg.csr_from_arcs(70, [], [], [], directed=True)
    G = bc.Graph(e)
    got, _ = G.bc(None)
    assert np.all(got == 0)
    d, sg, dl = G.source_state(3)
    assert d[3] == 0 and sg[3] == 1 and dl[3] == 0 and np.all(d[np.arange(70) != 3] == INT32_MAX)
    one = gg.csr_from_arcs(1, [], [], [], directed=False)
    G = bc.Graph(one)
    got, _ = G.bc(None)
    assert got.tolist() == [0.0]
    with pytest.raises(bc.BCError) as ei:
        G.bc(np.array([1], np.int32))
    assert ei.value.status == bc.BC_E_INVAL
    for bad in (dict(lds_bits=12), dict(virtual_warp=3), dict(node_parallel=2)):
        with pytest.raises(bc.BCError) as ei:
            G.bc(None, **bad)
        assert ei.value.status == bc.BC_E_INVAL, bad


def hub_graph(directed: bool):
    """Two hubs of 1500 and 900 arcs (above the workgroup-expansion threshold)
    over a sparse random graph, with tie-heavy weights."""
    rng = np.random.default_rng(21 if directed else 22)
    n = 2500
    src = [0] * 1500 + [1] * 900
    dst = list(range(2, 1502)) + list(range(1600, 2500))
    m = 4000
    a = rng.integers(0, n, size=m)
    b = rng.integers(0, n, size=m)
    keep = a != b
    src += a[keep].tolist()
    dst += b[keep].tolist()
    w = rng.integers(1, 4, size=len(src))
    if directed:
        # every leaf also points back, so the hubs have large in-degrees too
        back_s, back_d = dst[:2400], src[:2400]
        return gg.csr_from_arcs(n, src + back_s, dst + back_d,
                                np.concatenate([w, rng.integers(1, 4, size=2400)]), directed=True)
    pairs = {}
    for u, v, x in zip(src, dst, w):
        pairs.setdefault((min(u, v), max(u, v)), int(x))
    eu = [p[0] for p in pairs]
    ev = [p[1] for p in pairs]
    return gg.undirected_from_edges(n, eu, ev, list(pairs.values()))


@pytest.mark.parametrize("directed", [False, True])
def test_hub_vertices_expanded_by_the_workgroup(directed):
    g = hub_graph(directed)
    assert np.diff(g.row_ptr).max() > 512
    G = bc.Graph(g)
    want = oracle.oracle_bc(g, np.arange(g.n))
    for opts in (dict(), dict(wg_threads=256), dict(lds_bits=32), dict(dep_mode=2)):
        got, _ = G.bc(None, **opts)
        rel_close(got, want, 1e-9)
    check_state(g, G, 0)
    check_state(g, G, 1700)
    G.close()


def test_directed_sinks_and_parallel_arcs():
    # parallel equal-weight arcs are distinct shortest paths; sinks have no arcs
    src = [0, 0, 1, 1, 2, 3, 3]
    dst = [1, 1, 2, 3, 4, 4, 5]
    w = [2, 2, 1, 1, 1, 1, 7]
    g = gg.csr_from_arcs(6, src, dst, w, directed=True)
    G = bc.Graph(g)
    check_bc(g, G, None)
    for s in range(6):
        check_state(g, G, s)
    d, sg, _ = G.source_state(0)
    assert int(sg[1]) == 2 and int(sg[4]) == 4


def _tie_graphs():
    """Graphs where many vertices have several shortest-path predecessors:
    weights 1-2 with parallel arcs (equal and unequal weights) and self-loops,
    unit-weight layers of 1-12 vertices joined completely (so predecessor
    counts fall on both sides of what a vertex can keep without scanning,
    in-degree 2 and 3 included), and a unit grid (binomial counts)."""
    rng = np.random.default_rng(11)
    n = 3000
    src = rng.integers(0, n, 30000)
    dst = rng.integers(0, n, 30000)
    w = rng.integers(1, 3, 30000)
    dup = rng.choice(30000, 4500, replace=False)
    unq = rng.choice(30000, 1500, replace=False)
    src = np.concatenate([src, src[dup], src[unq]])
    dst = np.concatenate([dst, dst[dup], dst[unq]])
    w = np.concatenate([w, w[dup], w[unq] + 1])
    multi = gg.csr_from_arcs(n, src, dst, w, directed=True, name="ties-multi")
    eu, ev = [], []
    nxt = 1
    for chain in range(80):
        prev = [0]
        for layer in range(6):
            size = int(rng.integers(1, 13))
            cur = list(range(nxt, nxt + size))
            nxt += size
            for a in prev:
                for b in cur:
                    eu.append(a)
                    ev.append(b)
            prev = cur
    layers = gg.undirected_from_edges(nxt, eu, ev, np.ones(len(eu), np.int64), name="ties-layers")
    return [multi, layers, gg.unit_grid(30, 30)]


@pytest.mark.parametrize("which", [0, 1, 2], ids=["multi", "layers", "grid30"])
def test_many_tight_predecessors(which):
    # the count pass's key-and-ties shortcut against in-arc scans, every option set
    g = _tie_graphs()[which]
    G = bc.Graph(g)
    want = oracle.oracle_bc(g, np.arange(g.n))
    for opts in OPTION_SETS:
        got, _ = G.bc(None, **opts)
        rel_close(got, want, 1e-9)
    for s in (0, 1, g.n // 2, g.n - 1):
        check_state(g, G, s)
        check_state(g, G, s, far_buckets=1, delta=1)
    G.close()


def _emitters_graph(renumber_hint):
    """A directed core of 300 vertices and 200 emitters (out-arcs only) placed
    at the top ids, so the vertices without in-arcs are a suffix whether or not
    the graph is renumbered; with renumber_hint a few core hubs make the
    in-degrees skewed enough to be renumbered."""
    rng = np.random.default_rng(31 + renumber_hint)
    core, em = 300, 200
    src = list(rng.integers(0, core, 2400))
    dst = list(rng.integers(0, core, 2400))
    for e in range(core, core + em):
        k = int(rng.integers(1, 6))
        src += [e] * k
        dst += list(rng.integers(0, core, k))
    if renumber_hint:
        for hub in (7, 123, 250):
            src += list(rng.integers(0, core + em, 400))
            dst += [hub] * 400
    src, dst = np.array(src), np.array(dst)
    keep = src != dst
    w = rng.integers(1, 20, int(keep.sum()))
    return gg.csr_from_arcs(core + em, src[keep], dst[keep], w, directed=True,
                            name=f"emitters{renumber_hint}")


@pytest.mark.parametrize("hint", [0, 1])
def test_vertices_without_inarcs(hint):
    # a source's initialisation skips the vertices no source can reach (no
    # in-arcs) once the slab is in its initial state there: long runs of
    # sources per slab mixing emitters and core vertices, host and device ingest
    torch = pytest.importorskip("torch")
    g = _emitters_graph(hint)
    want = oracle.oracle_bc(g, np.arange(g.n))
    rp = torch.from_numpy(np.ascontiguousarray(g.row_ptr, dtype=np.int64)).cuda()
    col = torch.from_numpy(np.ascontiguousarray(g.col, dtype=np.int32)).cuda()
    w = torch.from_numpy(np.ascontiguousarray(g.w, dtype=np.int32)).cuda()
    torch.cuda.synchronize()
    for G in (bc.Graph(g), bc.Graph.from_device(g, rp, col, w,
                                                stream=torch.cuda.current_stream().cuda_stream)):
        srcs = np.random.default_rng(5).permutation(g.n).astype(np.int32)
        for opts in (dict(batch=3), dict(batch=1, far_buckets=1), dict(batch=2, accumulate=2),
                     dict(batch=5, wg_threads=256, lds_vertices=-1)):
            got, st = G.bc(srcs, **opts)
            rel_close(got, want, 1e-9)
        for s in (0, 299, 300, 450, g.n - 1):
            check_state(g, G, s)
        G.close()


@pytest.mark.parametrize("directed", [True, False])
def test_lds_8bit_window(directed):
    # 8-bit LDS distances relative to a window that follows the bands: every
    # vertex resident, weights far beyond the window's width (values kept in
    # device memory, brought back in at a re-base) and narrow bands (many
    # re-bases), several sources per slab; distances, counts and dependencies
    # exact at every vertex
    g = gg.random_graph(3000, 0.003, 1, 600, seed=41, directed=directed)
    G = bc.Graph(g)
    want = oracle.oracle_bc(g, np.arange(g.n))
    srcs = np.random.default_rng(3).permutation(g.n).astype(np.int32)
    for opts in (dict(delta=1), dict(delta=5, far_buckets=1), dict(delta=64, batch=2),
                 dict(delta=300, far_buckets=1, batch=3)):
        got, st = G.bc(srcs, lds_bits=8, lds_vertices=g.n, **opts)
        assert st["lds_bits"] == 8 and st["lds_vertices"] == g.n, st
        rel_close(got, want, 1e-9)
    for s in (0, 1234, g.n - 1):
        check_state(g, G, s, lds_bits=8, lds_vertices=g.n, delta=2)
        check_state(g, G, s, lds_bits=8, lds_vertices=g.n, delta=7, far_buckets=1)
    G.close()


def test_ring_key_range():
    # the far-bucket ring keeps its least bucket as a key below every predecessor
    # encoding, which needs bucket indices below 2^30: with weights up to 32767
    # on 65536 vertices, band width 1 would allow ~2^31 buckets (the pile runs
    # instead) while band width 4 keeps them below 2^30 (the ring runs)
    g = gg.random_graph(65536, 0.00006, 1, 32767, seed=51, directed=True)
    assert int(g.w.max()) > 30000
    G = bc.Graph(g)
    assert G.info()["packed_arcs"] == 1
    srcs = gg.sample_sources(g, 24, seed=52)
    want = oracle.oracle_bc(g, srcs)
    for delta, ring in ((1, False), (4, True)):
        got, st = G.bc(srcs, far_buckets=1, delta=delta)
        assert st["far_buckets"] == (1 if ring else 2), (delta, st["far_buckets"])
        rel_close(got, want, 1e-9)
    check_state(g, G, int(srcs[0]), far_buckets=1, delta=4)
    G.close()


def test_device_entry_point_with_torch_tensors():
    torch = pytest.importorskip("torch")
    g = gg.ba_graph(3000, 3, 1, 50, seed=5)
    G = bc.Graph(g)
    srcs = np.arange(0, 3000, 7, dtype=np.int32)
    s_dev = torch.from_numpy(srcs).cuda()
    out = torch.empty(g.n, dtype=torch.float64, device="cuda")
    st = bc.bc_compute_device(G.handle, s_dev.data_ptr(), srcs.shape[0], out.data_ptr(),
                              bc.make_options(stream=torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    rel_close(out.cpu().numpy(), oracle.oracle_bc(g, srcs), 1e-9)
    assert st.sources == srcs.shape[0] and st.reached > 0


# ------------------------------------------------------------------ configurations

def test_config_er1000_all_sources():
    g = gg.config_graph("er1000")
    G = bc.Graph(g)
    for opts in (LAUNCH["er1000"], dict(), dict(mode=bc.BC_MODE_PLAIN), dict(accumulate=2)):
        check_bc(g, G, None, **opts)
    for s in (0, 1, 500, 999):
        check_state(g, G, s)


def test_config_ba100k_parity_sources():
    g = gg.config_graph("ba100k")
    G = bc.Graph(g)
    srcs = gg.config_sources("ba100k", g, parity=True)
    check_bc(g, G, srcs, **LAUNCH["ba100k"])  # the benchmark's launch settings
    check_bc(g, G, srcs)
    for s in srcs[:3]:
        check_state(g, G, int(s), **LAUNCH["ba100k"])
        check_state(g, G, int(s), mode=bc.BC_MODE_PLAIN)


def test_config_ba100k_full_launch_linearity():
    """All 100k sources in the benchmark's launch configuration: BC over all
    sources equals the oracle's exact betweenness (Eq. 1, every source) and the
    sum over two halves, and sampled sources' states in that configuration
    match the oracle."""
    g = gg.config_graph("ba100k")
    G = bc.Graph(g)
    allsrc = np.arange(g.n, dtype=np.int32)
    opts = LAUNCH["ba100k"]
    full, st = G.bc(allsrc, **opts)
    rel_close(full, cached_oracle_bc(g, gg.config_sources("ba100k", g), label="ba100k"), 1e-9)
    a, _ = G.bc(allsrc[: g.n // 2], **opts)
    b, _ = G.bc(allsrc[g.n // 2:], **opts)
    assert np.all(np.isfinite(full)) and np.all(full >= 0)
    rel_close(full, a + b, 1e-9)
    assert st["reached"] == g.n * g.n  # connected graph
    for s in (0, 77_777, 99_999):
        check_state(g, G, s, **opts)


def spread(sources, count: int = 8):
    """count sources spread evenly over a source list (first and last included)."""
    idx = np.linspace(0, len(sources) - 1, count).round().astype(int)
    return [int(sources[i]) for i in idx]


def check_states(g, G, sources, **opts):
    """check_state for several sources; the oracle's single-source runs go to
    a thread pool (the ctypes calls release the interpreter lock)."""
    from concurrent.futures import ThreadPoolExecutor

    with ThreadPoolExecutor(max_workers=min(len(sources), oracle.host_threads())) as ex:
        want = list(ex.map(lambda s: oracle.oracle_source_state(g, s), sources))
    for s, (od, osg, odl, _) in zip(sources, want):
        d, sg, dl = G.source_state(s, **opts)
        od32 = np.where(od == INF64, INT32_MAX, od).astype(np.int32)
        assert np.array_equal(d, od32), (s, np.nonzero(d != od32)[0][:10])
        assert np.array_equal(sg, osg), (s, np.nonzero(sg != osg)[0][:10])
        rel_close(dl, odl, 1e-12)


def test_config_grid1000_full_source_list():
    """All 1024 sources of the grid workload in the benchmark's launch settings
    (256 sources in flight, so every slab of the launch is exercised) against
    the oracle's exact betweenness over the same list; distances and counts
    bit-exact and dependencies at 1e-12 on 8 sources spread over the list."""
    g = gg.config_graph("grid1000")
    srcs = gg.config_sources("grid1000", g)
    assert len(srcs) == 1024
    want = cached_oracle_bc(g, srcs, label="grid1000")
    G = bc.Graph(g)
    got, st = G.bc(srcs, **LAUNCH["grid1000"])
    assert st["batch"] == LAUNCH["grid1000"]["batch"] and st["sources"] == 1024
    rel_close(got, want, 1e-9)
    check_states(g, G, spread(srcs), **LAUNCH["grid1000"])
    # default options on a prefix of the list
    check_bc(g, G, srcs[:16])
    G.close()


@pytest.mark.slow
def test_config_rmat22_full_source_list():
    """All 1024 sources of the R-MAT scale-22 workload in the benchmark's launch
    settings (as many sources in flight as the launch holds) against the
    oracle's exact betweenness over the same list; distances and counts
    bit-exact and dependencies at 1e-12 on 8 sources spread over the list."""
    g = gg.config_graph("rmat22")
    srcs = gg.config_sources("rmat22", g)
    assert len(srcs) == 1024
    print(f"rmat22 n={g.n} nnz={g.nnz} sources={len(srcs)}", flush=True)
    want = cached_oracle_bc(g, srcs, label="rmat22")
    G = bc.Graph(g)
    got, st = G.bc(srcs, **LAUNCH["rmat22"])
    assert st["sources"] == 1024 and st["batch"] > 64
    rel_close(got, want, 1e-9)
    check_states(g, G, spread(srcs), **LAUNCH["rmat22"])
    G.close()
