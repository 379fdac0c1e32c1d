"""Serving form on the GPU: continuous batching over several resident graphs.

Each request's result in the mix must equal the same request computed alone
(bc_compute) within 1e-9 relative, and the oracle on the small graphs."""
from __future__ import annotations

import time

import numpy as np
import pytest

import oracle
from paper_1701_05975_amd import bc, graphgen as gg

pytestmark = pytest.mark.gpu


def rel_close(got, want, tol):
    zero = want == 0
    assert np.all(got[zero] == 0)
    err = np.abs(got[~zero] - want[~zero]) / np.abs(want[~zero])
    assert err.size == 0 or err.max() <= tol, float(err.max())


def test_mix_equals_alone_and_oracle():
    graphs = [gg.er_graph(2000, 8000, 1, 100, seed=101), gg.ba_graph(5000, 5, 1, 1000, seed=103),
              gg.grid_graph(60, 70, 80, 1, 255, seed=105),
              gg.rmat_graph(12, 16 << 12, .57, .19, .19, 1, 255, seed=107)]
    G = [bc.Graph(g) for g in graphs]
    rng = np.random.default_rng(200)
    reqs = []
    for i in range(24):
        gi = int(rng.integers(0, len(graphs)))
        g = graphs[gi]
        k = int(np.exp(rng.uniform(np.log(4), np.log(300))))
        src = gg.sample_sources(g, k, seed=1000 + i)
        reqs.append((gi, src))
    sv = bc.Server(items_per_sweep=96, slots_per_sweep=64)
    tickets = []
    for j, (gi, src) in enumerate(reqs):
        tickets.append(sv.submit(G[gi], src))
        if j % 5 == 4:
            time.sleep(0.002)  # later requests arrive while earlier ones run
    for (gi, src), t in zip(reqs, tickets):
        got, lat = sv.wait(t, graphs[gi].n)
        alone, _ = G[gi].bc(src)
        rel_close(got, alone, 1e-9)
        rel_close(got, oracle.oracle_bc(graphs[gi], src), 1e-9)
        assert lat > 0
    st = sv.stats()
    assert st["completed"] == len(reqs) and st["failed"] == 0
    assert st["p99_ms"] >= st["p50_ms"] > 0 and st["gteps"] > 0 and st["sweeps"] >= 4
    sv.close()


def test_serving_stream_requests_on_small_graphs():
    """32 requests of the benchmark's serving stream (those that fall on its
    graphs of at most 50k vertices) served together in a mix: each result
    equals the same request computed alone and the oracle, within 1e-9."""
    small = [i for i, b in enumerate(gg.SERVING_GRAPHS) if i in (0, 2, 4, 6)]
    graphs = [None] * len(gg.SERVING_GRAPHS)
    for i, g in zip(small, gg.serving_graphs(small)):
        assert g.n <= 50_000
        graphs[i] = g
    reqs = [(i, r) for i, r in enumerate(gg.serving_requests(graphs, 200)) if r[1] is not None][:32]
    assert len(reqs) == 32
    G = {i: bc.Graph(graphs[i]) for i in small}
    sv = bc.Server()
    tickets = []
    for j, (_, (gi, src)) in enumerate(reqs):
        tickets.append(sv.submit(G[gi], src))
        if j % 4 == 3:
            time.sleep(0.005)  # later requests arrive while earlier ones run
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=2) as ex:
        want = [ex.submit(oracle.oracle_bc, graphs[gi], src, oracle.host_threads())
                for _, (gi, src) in reqs]
        for (i, (gi, src)), t, w in zip(reqs, tickets, want):
            got, lat = sv.wait(t, graphs[gi].n)
            alone, _ = G[gi].bc(src)
            rel_close(got, alone, 1e-9)
            rel_close(got, w.result(), 1e-9)
            assert lat > 0, i
    st = sv.stats()
    assert st["completed"] == 32 and st["failed"] == 0
    sv.close()
    for g in G.values():
        g.close()


def test_failure_isolated_to_its_request():
    bad = bc.Graph(gg.diamond_chain(64))
    good_g = gg.path_graph(50)
    good = bc.Graph(good_g)
    sv = bc.Server()
    t_bad = sv.submit(bad, np.array([3, 0, 6], np.int32))
    t_ok = sv.submit(good, np.arange(50, dtype=np.int32))
    t_bad2 = sv.submit(bad, np.array([6], np.int32))  # shares sweeps with the failing one
    with pytest.raises(bc.BCError) as ei:
        sv.wait(t_bad, 3 * 64 + 1)
    assert ei.value.status == bc.BC_E_SIGMA_OVERFLOW and "index 1" in ei.value.msg
    got, _ = sv.wait(t_ok, 50)
    assert np.array_equal(got, [2 * i * (49 - i) for i in range(50)])
    got, _ = sv.wait(t_bad2, 3 * 64 + 1)
    assert np.isfinite(got).all()
    st = sv.stats()
    assert st["failed"] == 1 and st["completed"] == 2
    sv.close()


def test_admission_waits_for_budget():
    g = gg.ba_graph(20000, 4, 1, 100, seed=7)
    G = bc.Graph(g)
    # budget for one result at a time: requests are admitted one after another
    sv = bc.Server(result_budget_bytes=g.n * 8 + 16)
    srcs = [gg.sample_sources(g, 40, seed=s) for s in range(4)]
    tickets = [sv.submit(G, s) for s in srcs]
    outs = []
    for t in tickets:
        outs.append(sv.wait(t, g.n)[0])
    for s, o in zip(srcs, outs):
        rel_close(o, oracle.oracle_bc(g, s), 1e-9)
    st = sv.stats()
    assert st["completed"] == 4 and st["queue_ms_sum"] > 0
    with pytest.raises(bc.BCError) as ei:
        sv.submit(bc.Graph(gg.path_graph(30000)), np.array([0], np.int32))
    assert ei.value.status == bc.BC_E_BUSY
    sv.close()


def test_wait_timeout_and_empty_request():
    g = gg.grid_graph(200, 200, 0, 1, 255, seed=9)
    G = bc.Graph(g)
    sv = bc.Server(slots_per_sweep=4, items_per_sweep=4)
    t0 = sv.submit(G, np.zeros(0, np.int32))
    got, _ = sv.wait(t0, g.n)
    assert np.all(got == 0)
    t = sv.submit(G, gg.sample_sources(g, 64, seed=3))
    with pytest.raises(bc.BCError) as ei:
        sv.wait(t, g.n, timeout_us=1)
    assert ei.value.status == bc.BC_E_TIMEOUT
    got, _ = sv.wait(t, g.n)
    assert np.isfinite(got).all() and got.max() > 0
    sv.close()
