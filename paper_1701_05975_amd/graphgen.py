"""Seeded synthetic graph generators.

This module only builds inputs: CSR arrays with integer arc weights and seeded
source lists.  It computes nothing of the betweenness method itself, so both
the CPU oracle's tests and the GPU library's tests and benchmark may draw their
inputs from it.

Families follow the paper's evaluation (Sec. 4.1): Erdos-Renyi random graphs
and Kronecker-like (R-MAT) graphs, plus a scale-free Barabasi-Albert graph and
a road-like grid as further synthetic stand-ins.  Weights are uniform random
integers with inclusive bounds, as the paper assigns uniform random weights
from 1 to 10 to its unweighted networks (Sec. 4.1).

Conventions
-----------
* A graph is returned as :class:`CSRGraph`.  ``row_ptr`` is int64[n+1],
  ``col`` and ``w`` are int32[nnz]; rows are sorted by column.
* Undirected graphs store both arcs of every edge with the same weight
  (the paper treats every edge as traversable both ways, Sec. 2.1).
  ``m`` counts undirected edges once; for directed graphs ``m`` counts arcs.
* All randomness comes from ``numpy.random.default_rng(seed)`` (PCG64).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class CSRGraph:
    n: int
    row_ptr: np.ndarray  # int64[n+1]
    col: np.ndarray      # int32[nnz]
    w: np.ndarray        # int32[nnz]
    directed: bool
    m: int               # edges for throughput accounting
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])

    def out_degree(self) -> np.ndarray:
        return np.diff(self.row_ptr)


def csr_from_arcs(n: int, src, dst, wt, directed: bool, m: int | None = None,
                  name: str = "", meta: dict | None = None) -> CSRGraph:
    """Build a CSR graph from an arc list (arcs kept as given, rows sorted by column)."""
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    wt = np.asarray(wt, dtype=np.int64)
    order = np.lexsort((dst, src))
    src, dst, wt = src[order], dst[order], wt[order]
    counts = np.bincount(src, minlength=n) if n > 0 else np.zeros(0, np.int64)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    if n > 0:
        np.cumsum(counts, out=row_ptr[1:])
    return CSRGraph(n=n, row_ptr=row_ptr, col=dst.astype(np.int32), w=wt.astype(np.int32),
                    directed=directed, m=int(len(src) if m is None else m), name=name,
                    meta=dict(meta or {}))


def undirected_from_edges(n: int, eu, ev, ew, name: str = "", meta: dict | None = None) -> CSRGraph:
    """Both arcs of each undirected edge (u, v, w), same weight."""
    eu = np.asarray(eu, dtype=np.int64)
    ev = np.asarray(ev, dtype=np.int64)
    ew = np.asarray(ew, dtype=np.int64)
    src = np.concatenate([eu, ev])
    dst = np.concatenate([ev, eu])
    wt = np.concatenate([ew, ew])
    return csr_from_arcs(n, src, dst, wt, directed=False, m=len(eu), name=name, meta=meta)


# --------------------------------------------------------------------------
# Families of the benchmark configurations
# --------------------------------------------------------------------------

def er_graph(n: int, M: int, wlo: int, whi: int, seed: int) -> CSRGraph:
    """G(n, M): M distinct unordered vertex pairs without self-loops, uniform weights."""
    rng = np.random.default_rng(seed)
    if M > n * (n - 1) // 2:
        raise ValueError("too many edges for G(n, M)")
    keys = np.zeros(0, dtype=np.int64)
    while keys.shape[0] < M:
        need = M - keys.shape[0]
        a = rng.integers(0, n, size=2 * need + 16)
        b = rng.integers(0, n, size=2 * need + 16)
        ok = a != b
        lo = np.minimum(a[ok], b[ok])
        hi = np.maximum(a[ok], b[ok])
        cand = np.concatenate([keys, lo * n + hi])
        _, first = np.unique(cand, return_index=True)
        keys = cand[np.sort(first)][:M]
    eu, ev = keys // n, keys % n
    ew = rng.integers(wlo, whi + 1, size=M)
    return undirected_from_edges(n, eu, ev, ew, name=f"er_n{n}_M{M}",
                                 meta=dict(family="er", seed=seed, wlo=wlo, whi=whi))


def ba_graph(n: int, m: int, wlo: int, whi: int, seed: int) -> CSRGraph:
    """Barabasi-Albert: seed star on m+1 vertices; each new vertex attaches to m
    distinct targets drawn proportionally to degree (from the endpoint list)."""
    rng = np.random.default_rng(seed)
    n_edges = m + m * (n - m - 1)
    eu = np.empty(n_edges, dtype=np.int64)
    ev = np.empty(n_edges, dtype=np.int64)
    ep = np.empty(2 * n_edges, dtype=np.int64)
    # seed star: centre 0, leaves 1..m
    for i in range(m):
        eu[i], ev[i] = 0, i + 1
        ep[2 * i], ep[2 * i + 1] = 0, i + 1
    ne, nep = m, 2 * m
    buf = rng.random(1 << 20)
    pos = 0
    for v in range(m + 1, n):
        chosen: list[int] = []
        while len(chosen) < m:
            if pos >= buf.shape[0]:
                buf = rng.random(1 << 20)
                pos = 0
            t = int(ep[int(buf[pos] * nep)])
            pos += 1
            if t not in chosen:
                chosen.append(t)
        for t in chosen:
            eu[ne], ev[ne] = v, t
            ne += 1
            ep[nep], ep[nep + 1] = v, t
            nep += 2
    ew = rng.integers(wlo, whi + 1, size=n_edges)
    return undirected_from_edges(n, eu, ev, ew, name=f"ba_n{n}_m{m}",
                                 meta=dict(family="ba", seed=seed, wlo=wlo, whi=whi))


def grid_graph(rows: int, cols: int, remove: int, wlo: int, whi: int, seed: int) -> CSRGraph:
    """rows x cols 4-neighbour grid (id = r*cols + c) with exactly `remove`
    edges deleted uniformly at random."""
    rng = np.random.default_rng(seed)
    r, c = np.meshgrid(np.arange(rows), np.arange(cols - 1), indexing="ij")
    hu = (r * cols + c).ravel()
    hv = hu + 1
    r, c = np.meshgrid(np.arange(rows - 1), np.arange(cols), indexing="ij")
    vu = (r * cols + c).ravel()
    vv = vu + cols
    eu = np.concatenate([hu, vu]).astype(np.int64)
    ev = np.concatenate([hv, vv]).astype(np.int64)
    E = eu.shape[0]
    if remove:
        drop = rng.choice(E, size=remove, replace=False)
        keep = np.ones(E, dtype=bool)
        keep[drop] = False
        eu, ev = eu[keep], ev[keep]
    ew = rng.integers(wlo, whi + 1, size=eu.shape[0])
    return undirected_from_edges(rows * cols, eu, ev, ew, name=f"grid_{rows}x{cols}_r{remove}",
                                 meta=dict(family="grid", seed=seed, wlo=wlo, whi=whi))


def rmat_graph(scale: int, n_draws: int, a: float, b: float, c: float, wlo: int, whi: int,
               seed: int, relabel: bool = True, chunk: int = 1 << 21) -> CSRGraph:
    """Directed R-MAT (Kronecker-like): each draw picks one quadrant per bit level
    with probabilities a, b, c, 1-a-b-c; self-loops and duplicate arcs dropped;
    optional seeded vertex relabelling."""
    rng = np.random.default_rng(seed)
    n = 1 << scale
    ta, tb, tc = np.float32(a), np.float32(a + b), np.float32(a + b + c)
    keys = []
    done = 0
    while done < n_draws:
        k = min(chunk, n_draws - done)
        u = np.zeros(k, dtype=np.int64)
        v = np.zeros(k, dtype=np.int64)
        for _ in range(scale):
            x = rng.random(k, dtype=np.float32)
            bu = x >= tb                     # quadrants c, d set the row bit
            bv = ((x >= ta) & (x < tb)) | (x >= tc)   # quadrants b, d set the column bit
            u = (u << 1) | bu
            v = (v << 1) | bv
        keys.append(u * n + v)
        done += k
    key = np.concatenate(keys)
    del keys
    u, v = key // n, key % n
    del key
    if relabel:
        perm = rng.permutation(n).astype(np.int64)
        u, v = perm[u], perm[v]
    ok = u != v
    key = np.unique(u[ok] * n + v[ok])
    u, v = key // n, key % n
    del key
    ew = rng.integers(wlo, whi + 1, size=u.shape[0])
    # np.unique already sorts by (u, v)
    counts = np.bincount(u, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return CSRGraph(n=n, row_ptr=row_ptr, col=v.astype(np.int32), w=ew.astype(np.int32),
                    directed=True, m=int(u.shape[0]), name=f"rmat_s{scale}",
                    meta=dict(family="rmat", seed=seed, wlo=wlo, whi=whi, draws=n_draws))


def kronecker_graph(scale: int, edge_factor: int, wlo: int, whi: int, seed: int,
                    a: float = 0.57, b: float = 0.19, c: float = 0.19) -> CSRGraph:
    """Undirected Kronecker-like graph: R-MAT draws (edge_factor * 2^scale),
    self-loops dropped, each unordered pair kept once, uniform weights."""
    rng = np.random.default_rng(seed)
    n = 1 << scale
    draws = edge_factor * n
    ta, tb, tc = np.float32(a), np.float32(a + b), np.float32(a + b + c)
    u = np.zeros(draws, dtype=np.int64)
    v = np.zeros(draws, dtype=np.int64)
    for _ in range(scale):
        x = rng.random(draws, dtype=np.float32)
        u = (u << 1) | (x >= tb)
        v = (v << 1) | (((x >= ta) & (x < tb)) | (x >= tc))
    perm = rng.permutation(n).astype(np.int64)
    u, v = perm[u], perm[v]
    ok = u != v
    lo, hi = np.minimum(u[ok], v[ok]), np.maximum(u[ok], v[ok])
    key = np.unique(lo * n + hi)
    eu, ev = key // n, key % n
    ew = rng.integers(wlo, whi + 1, size=eu.shape[0])
    return undirected_from_edges(n, eu, ev, ew, name=f"kron_s{scale}_ef{edge_factor}",
                                 meta=dict(family="kronecker", seed=seed, wlo=wlo, whi=whi))


def random_graph(n: int, p: float, wlo: int, whi: int, seed: int, directed: bool = False) -> CSRGraph:
    """Bernoulli(p) simple graph on n vertices (small parity and pin cases)."""
    rng = np.random.default_rng(seed)
    if directed:
        a = rng.random((n, n)) < p
        np.fill_diagonal(a, False)
        su, sv = np.nonzero(a)
        wt = rng.integers(wlo, whi + 1, size=su.shape[0])
        return csr_from_arcs(n, su, sv, wt, directed=True, name=f"rand_d_n{n}",
                             meta=dict(family="random", seed=seed))
    a = np.triu(rng.random((n, n)) < p, 1)
    eu, ev = np.nonzero(a)
    ew = rng.integers(wlo, whi + 1, size=eu.shape[0])
    return undirected_from_edges(n, eu, ev, ew, name=f"rand_u_n{n}",
                                 meta=dict(family="random", seed=seed))


# --------------------------------------------------------------------------
# Small structured graphs (closed-form cases)
# --------------------------------------------------------------------------

def path_graph(n: int, weights=None) -> CSRGraph:
    w = np.ones(n - 1, dtype=np.int64) if weights is None else np.asarray(weights, np.int64)
    return undirected_from_edges(n, np.arange(n - 1), np.arange(1, n), w, name=f"path{n}")


def star_graph(n: int, weights=None) -> CSRGraph:
    w = np.ones(n - 1, dtype=np.int64) if weights is None else np.asarray(weights, np.int64)
    return undirected_from_edges(n, np.zeros(n - 1, np.int64), np.arange(1, n), w, name=f"star{n}")


def cycle_graph(n: int, weight: int = 1) -> CSRGraph:
    eu = np.arange(n)
    ev = (eu + 1) % n
    return undirected_from_edges(n, eu, ev, np.full(n, weight), name=f"cycle{n}")


def complete_graph(n: int, weight: int = 1) -> CSRGraph:
    iu, iv = np.triu_indices(n, 1)
    return undirected_from_edges(n, iu, iv, np.full(iu.shape[0], weight), name=f"K{n}")


def unit_grid(rows: int, cols: int) -> CSRGraph:
    return grid_graph(rows, cols, 0, 1, 1, seed=0)


def diamond_chain(k: int) -> CSRGraph:
    """k unit diamonds in series: hubs h_0..h_k, two parallel middle vertices
    between consecutive hubs.  From h_0, sigma(h_k) = 2**k."""
    eu, ev = [], []
    hub = lambda i: 3 * i
    for i in range(k):
        h0, h1 = hub(i), hub(i + 1)
        a, b = h0 + 1, h0 + 2
        eu += [h0, h0, a, b]
        ev += [a, b, h1, h1]
    n = 3 * k + 1
    return undirected_from_edges(n, eu, ev, np.ones(len(eu), np.int64), name=f"diamond{k}")


# --------------------------------------------------------------------------
# Graph edits (inputs of the dynamic update)
# --------------------------------------------------------------------------

def _arcs(g: CSRGraph):
    src = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(g.row_ptr))
    return src, g.col.astype(np.int64), g.w.astype(np.int64)


def reversed_graph(g: CSRGraph) -> CSRGraph:
    """Every arc (u, v, w) turned into (v, u, w)."""
    src, dst, wt = _arcs(g)
    return csr_from_arcs(g.n, dst, src, wt, directed=g.directed, m=g.m, name=g.name + "-rev")


def change_arc(g: CSRGraph, tail: int, head: int, w_old: int, w_new: int) -> CSRGraph:
    """g with one arc tail -> head of weight w_old (0: none) replaced by one of
    weight w_new (0: none); for an undirected graph both arcs of the edge."""
    src, dst, wt = _arcs(g)
    pairs = [(tail, head)] if g.directed or tail == head else [(tail, head), (head, tail)]
    keep = np.ones(src.shape[0], dtype=bool)
    add_s, add_d, add_w = [], [], []
    for a, b in pairs:
        if w_old > 0:
            hit = np.nonzero((src == a) & (dst == b) & (wt == w_old) & keep)[0]
            if hit.shape[0] == 0:
                raise ValueError(f"no arc {a} -> {b} of weight {w_old}")
            keep[hit[0]] = False
        if w_new > 0:
            add_s.append(a)
            add_d.append(b)
            add_w.append(w_new)
    src = np.concatenate([src[keep], np.asarray(add_s, np.int64)])
    dst = np.concatenate([dst[keep], np.asarray(add_d, np.int64)])
    wt = np.concatenate([wt[keep], np.asarray(add_w, np.int64)])
    dm = (1 if w_new > 0 else 0) - (1 if w_old > 0 else 0)
    return csr_from_arcs(g.n, src, dst, wt, directed=g.directed, m=g.m + dm, name=g.name)


def random_arc_change(g: CSRGraph, kind: str, wlo: int, whi: int, seed: int):
    """(tail, head, w_old, w_new) of one random change: 'insert' (a new arc
    between two distinct vertices), 'delete', 'increase' or 'decrease' (an
    existing arc, not a self-loop; a decrease needs a weight above 1)."""
    rng = np.random.default_rng(seed)
    src, dst, wt = _arcs(g)
    if kind == "insert":
        while True:
            a, b = (int(x) for x in rng.integers(0, g.n, size=2))
            if a != b:
                return a, b, 0, int(rng.integers(wlo, whi + 1))
    ok = src != dst
    if kind == "decrease":
        ok &= wt > 1
    cand = np.nonzero(ok)[0]
    if cand.shape[0] == 0:
        raise ValueError(f"no arc for a {kind}")
    e = int(cand[rng.integers(0, cand.shape[0])])
    a, b, w = int(src[e]), int(dst[e]), int(wt[e])
    if kind == "delete":
        return a, b, w, 0
    if kind == "increase":
        return a, b, w, int(w + rng.integers(1, max(whi, 2) + 1))
    if kind == "decrease":
        return a, b, w, int(rng.integers(1, w))
    raise ValueError(kind)


# --------------------------------------------------------------------------
# Benchmark configurations and source sampling
# --------------------------------------------------------------------------

def sample_sources(g: CSRGraph, k: int, seed: int) -> np.ndarray:
    """k distinct vertices with out-degree >= 1, uniform without replacement."""
    elig = np.nonzero(g.out_degree() >= 1)[0]
    rng = np.random.default_rng(seed)
    k = min(k, elig.shape[0])
    return np.sort(rng.choice(elig, size=k, replace=False)).astype(np.int32)


CONFIGS = {
    # name: (builder, source spec)
    "er1000": dict(build=lambda: er_graph(1000, 4000, 1, 100, seed=1), k=None, src_seed=None),
    "ba100k": dict(build=lambda: ba_graph(100_000, 5, 1, 1000, seed=2), k=None, src_seed=20,
                   parity_k=256),
    "grid1000": dict(build=lambda: grid_graph(1000, 1000, 39_960, 1, 255, seed=3), k=1024,
                     src_seed=30),
    "rmat22": dict(build=lambda: rmat_graph(22, 1 << 26, 0.57, 0.19, 0.19, 1, 255, seed=4),
                   k=1024, src_seed=40),
}


def config_graph(name: str) -> CSRGraph:
    return CONFIGS[name]["build"]()


def config_sources(name: str, g: CSRGraph, parity: bool = False) -> np.ndarray:
    cfg = CONFIGS[name]
    k = cfg.get("parity_k") if parity and cfg.get("parity_k") else cfg["k"]
    if k is None:
        return np.arange(g.n, dtype=np.int32)
    return sample_sources(g, k, cfg["src_seed"])


# The serving workload: eight resident graphs of the four families, n from 10k
# to 2M, and a seeded request stream over them.
SERVING_GRAPHS = [
    lambda: er_graph(10_000, 40_000, 1, 100, seed=101),
    lambda: er_graph(500_000, 2_000_000, 1, 100, seed=102),
    lambda: ba_graph(50_000, 5, 1, 1000, seed=103),
    lambda: ba_graph(1_000_000, 5, 1, 1000, seed=104),
    lambda: grid_graph(100, 100, 396, 1, 255, seed=105),
    lambda: grid_graph(1414, 1414, 79_941, 1, 255, seed=106),
    lambda: rmat_graph(14, 16 << 14, .57, .19, .19, 1, 255, seed=107),
    lambda: rmat_graph(21, 16 << 21, .57, .19, .19, 1, 255, seed=108),
]


def serving_graphs(which=None) -> list:
    """The serving graphs (all eight, or those whose indices are listed)."""
    idx = range(len(SERVING_GRAPHS)) if which is None else which
    return [SERVING_GRAPHS[i]() for i in idx]


def serving_requests(graphs: list, nreq: int) -> list:
    """The seeded request stream over the serving graphs: (graph index, source
    list) per request, the graph uniform over the eight and k log-uniform in
    [64, 4096].  Sources depend only on the request index and its graph."""
    rng = np.random.default_rng(200)
    reqs = []
    for i in range(nreq):
        gi = int(rng.integers(0, len(SERVING_GRAPHS)))
        k = int(np.floor(np.exp(rng.uniform(np.log(64), np.log(4096)))))
        g = graphs[gi]
        reqs.append((gi, sample_sources(g, k, seed=10_000 + i) if g is not None else None))
    return reqs
