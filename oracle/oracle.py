"""ctypes wrapper around oracle.c (test infrastructure only).

The C source is the oracle; this module only compiles it with gcc and
marshals numpy arrays.  See oracle.c for what is computed and which passages
of the paper each step follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
lib_path = os.path.join(_HERE, "liboracle.so")

INF64 = np.iinfo(np.int64).max


class OracleError(RuntimeError):
    pass


class SigmaOverflow(OracleError):
    def __init__(self, first_bad: int):
        super().__init__(f"shortest-path count overflow (first source index {first_bad})")
        self.first_bad = first_bad


def build(force: bool = True, extra_flags: tuple[str, ...] = (), src: str | None = None,
          out: str | None = None) -> str:
    """Compile oracle.c into a shared library with gcc; returns its path."""
    src = src or _SRC
    out = out or lib_path
    if not force and os.path.exists(out) and os.path.getmtime(out) >= os.path.getmtime(src):
        return out
    # no contraction of a product and a sum into one fused operation: every
    # term and sum is rounded as written
    cmd = ["gcc", "-O3", "-ffp-contract=off", "-std=c11", "-fPIC", "-shared", "-pthread",
           *extra_flags, src, "-o", out]
    subprocess.run(cmd, check=True)
    return out


_LIB = None


def host_threads() -> int:
    """Every host core this process may run on."""
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:
        return max(1, os.cpu_count() or 1)


def _lib(path: str | None = None):
    global _LIB
    if path is not None:
        return _bind(ctypes.CDLL(path))
    if _LIB is None:
        if not os.path.exists(lib_path) or os.path.getmtime(lib_path) < os.path.getmtime(_SRC):
            build()
        _LIB = _bind(ctypes.CDLL(lib_path))
    return _LIB


def _bind(lib):
    P = ctypes.c_void_p
    lib.oracle_bc.argtypes = [ctypes.c_int32, ctypes.c_int64, P, P, P, P, ctypes.c_int64,
                              ctypes.c_int32, P, P]
    lib.oracle_bc.restype = ctypes.c_int
    lib.oracle_bc_edges.argtypes = [ctypes.c_int32, ctypes.c_int64, P, P, P, P, ctypes.c_int64,
                                     ctypes.c_int32, P, P, P]
    lib.oracle_bc_edges.restype = ctypes.c_int
    lib.oracle_source_state.argtypes = [ctypes.c_int32, ctypes.c_int64, P, P, P, ctypes.c_int32,
                                        P, P, P, P]
    lib.oracle_source_state.restype = ctypes.c_int
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _graph_arrays(g):
    rp = np.ascontiguousarray(g.row_ptr, dtype=np.int64)
    col = np.ascontiguousarray(g.col, dtype=np.int32)
    w = np.ascontiguousarray(g.w, dtype=np.int32)
    return rp, col, w


def oracle_bc(g, sources, threads: int | None = None, lib: str | None = None) -> np.ndarray:
    """BC summed over the listed sources (ordered pairs, unnormalised)."""
    L = _lib(lib)
    rp, col, w = _graph_arrays(g)
    src = np.ascontiguousarray(np.asarray(sources), dtype=np.int32)
    bc = np.zeros(max(g.n, 1), dtype=np.float64)
    bad = ctypes.c_int64(-1)
    if threads is None:
        threads = host_threads()
    rc = L.oracle_bc(g.n, col.shape[0], _ptr(rp), _ptr(col), _ptr(w), _ptr(src), src.shape[0],
                     threads, _ptr(bc), ctypes.byref(bad))
    if rc == 1:
        raise SigmaOverflow(bad.value)
    if rc != 0:
        raise OracleError(f"oracle_bc failed with code {rc}")
    return bc[: g.n]


def oracle_bc_edges(g, sources, threads: int | None = None, lib: str | None = None):
    """(BC float64[n], edge betweenness float64[nnz] in CSR arc order) over the sources."""
    L = _lib(lib)
    rp, col, w = _graph_arrays(g)
    src = np.ascontiguousarray(np.asarray(sources), dtype=np.int32)
    bc = np.zeros(max(g.n, 1), dtype=np.float64)
    ebc = np.zeros(max(col.shape[0], 1), dtype=np.float64)
    bad = ctypes.c_int64(-1)
    if threads is None:
        threads = host_threads()
    rc = L.oracle_bc_edges(g.n, col.shape[0], _ptr(rp), _ptr(col), _ptr(w), _ptr(src),
                           src.shape[0], threads, _ptr(bc), _ptr(ebc), ctypes.byref(bad))
    if rc == 1:
        raise SigmaOverflow(bad.value)
    if rc != 0:
        raise OracleError(f"oracle_bc_edges failed with code {rc}")
    return bc[: g.n], ebc[: col.shape[0]]


def oracle_source_state(g, s: int, lib: str | None = None):
    """(d int64 with INF64 for unreachable, sigma uint64, delta float64, n_reached)."""
    L = _lib(lib)
    rp, col, w = _graph_arrays(g)
    n = g.n
    d = np.empty(n, dtype=np.int64)
    sigma = np.empty(n, dtype=np.uint64)
    delta = np.empty(n, dtype=np.float64)
    nr = ctypes.c_int32(0)
    rc = L.oracle_source_state(n, col.shape[0], _ptr(rp), _ptr(col), _ptr(w), int(s), _ptr(d),
                               _ptr(sigma), _ptr(delta), ctypes.byref(nr))
    if rc == 1:
        raise SigmaOverflow(0)
    if rc != 0:
        raise OracleError(f"oracle_source_state failed with code {rc}")
    return d, sigma, delta, int(nr.value)


def oracle_source_changed(g_old, g_new, s: int, lib: str | None = None) -> bool:
    """Whether the distances or shortest-path counts from s differ between two
    graphs.  A change of the graph can alter the dependencies delta_s, and with
    them the centralities, only through such a source."""
    d0, s0, _, _ = oracle_source_state(g_old, s, lib)
    d1, s1, _, _ = oracle_source_state(g_new, s, lib)
    return not (np.array_equal(d0, d1) and np.array_equal(s0, s1))


def oracle_changed_sources(g_old, g_new, lib: str | None = None) -> np.ndarray:
    """Sorted vertices s for which oracle_source_changed holds (every vertex
    tried: small graphs only)."""
    return np.array([s for s in range(g_old.n) if oracle_source_changed(g_old, g_new, s, lib)],
                    dtype=np.int32)
