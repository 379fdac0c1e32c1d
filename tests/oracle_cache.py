"""Oracle results for the full-size workloads, cached by input hash.

Test infrastructure: the exact betweenness of a workload's whole source list
(Sec. 2.1, Eq. 1 restricted to the list) takes the CPU oracle minutes on the
large graphs, so the result is stored once under ``tests/.oracle_cache/``
(not versioned) and reused while the graph, the source list and the oracle's
source are unchanged.  Every stored value is written here, by ``oracle/``
alone: nothing in this module reads a result of the HIP library.

    python tests/oracle_cache.py grid1000 rmat22     # fill the cache ahead of a GPU run
"""
from __future__ import annotations

import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from oracle.oracle import host_threads  # noqa: E402

CACHE_DIR = os.path.join(HERE, ".oracle_cache")


def input_key(g, sources) -> str:
    """Hash of the graph arrays, the source list and the oracle's C source."""
    h = hashlib.blake2b(digest_size=16)
    h.update(f"n={g.n} nnz={g.nnz} directed={int(bool(g.directed))}".encode())
    for a, dt in ((g.row_ptr, np.int64), (g.col, np.int32), (g.w, np.int32),
                  (np.asarray(sources), np.int32)):
        h.update(np.ascontiguousarray(a, dtype=dt).tobytes())
    with open(os.path.join(ROOT, "oracle", "oracle.c"), "rb") as fh:
        h.update(fh.read())
    return h.hexdigest()


def cached_oracle_bc(g, sources, label: str = "", chunk: int = 0) -> np.ndarray:
    """oracle.oracle_bc(g, sources) on every host core, stored by input key.

    With chunk > 0 the source list is run in slices of that many sources (the
    partial results are added in slice order) and progress goes to stderr."""
    sources = np.ascontiguousarray(np.asarray(sources), dtype=np.int32)
    key = input_key(g, sources)
    path = os.path.join(CACHE_DIR, f"{label or 'bc'}_{key}.npy")
    if os.path.exists(path):
        bc = np.load(path, allow_pickle=False)
        if bc.shape == (g.n,) and bc.dtype == np.float64:
            return bc
    threads = host_threads()
    t0 = time.perf_counter()
    if chunk <= 0:
        bc = oracle.oracle_bc(g, sources, threads=threads)
    else:
        bc = np.zeros(g.n, dtype=np.float64)
        for lo in range(0, sources.shape[0], chunk):
            bc += oracle.oracle_bc(g, sources[lo:lo + chunk], threads=threads)
            print(f"# oracle {label}: {min(lo + chunk, sources.shape[0])}/{sources.shape[0]} "
                  f"sources, {time.perf_counter() - t0:.0f} s", file=sys.stderr, flush=True)
    os.makedirs(CACHE_DIR, exist_ok=True)
    tmp = path + f".tmp{os.getpid()}.npy"
    np.save(tmp, bc, allow_pickle=False)
    os.replace(tmp, path)
    return bc


def main(argv):
    from paper_1701_05975_amd import graphgen as gg
    for name in argv or ["grid1000", "rmat22"]:
        t0 = time.perf_counter()
        g = gg.config_graph(name)
        srcs = gg.config_sources(name, g)
        print(f"# {name}: n={g.n} nnz={g.nnz} k={len(srcs)}, {host_threads()} threads",
              file=sys.stderr, flush=True)
        cached_oracle_bc(g, srcs, label=name, chunk=128)
        print(f"# {name}: done in {time.perf_counter() - t0:.0f} s", file=sys.stderr, flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
