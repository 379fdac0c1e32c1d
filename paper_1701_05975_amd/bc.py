"""Thin Python binding of the C ABI in include/bc.h (argument marshalling only).

Every computation runs in the HIP library ``libbcgpu.so``; this module only
converts numpy arrays / torch tensors to pointers and status codes to
exceptions.  There is no fallback: if the library cannot be loaded, importing
this module raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbcgpu.so")

BC_OK = 0
BC_E_INVAL = 1
BC_E_GRAPH = 2
BC_E_WEIGHT = 3
BC_E_DIST_OVERFLOW = 4
BC_E_SIGMA_OVERFLOW = 5
BC_E_NOMEM = 6
BC_E_DEVICE = 7
BC_E_BUSY = 8
BC_E_TIMEOUT = 9
BC_E_INTERNAL = 10

STATUS_NAMES = {
    0: "BC_OK", 1: "BC_E_INVAL", 2: "BC_E_GRAPH", 3: "BC_E_WEIGHT", 4: "BC_E_DIST_OVERFLOW",
    5: "BC_E_SIGMA_OVERFLOW", 6: "BC_E_NOMEM", 7: "BC_E_DEVICE", 8: "BC_E_BUSY",
    9: "BC_E_TIMEOUT", 10: "BC_E_INTERNAL",
}

BC_DIRECTED = 1
BC_KEEP_ORDER = 2
BC_EDGE_BC = 4
BC_MODE_AUTO, BC_MODE_BATCHED, BC_MODE_PLAIN, BC_MODE_INTERLEAVED = 0, 1, 2, 3

INT32_MAX = 2**31 - 1


class BCError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status
        self.msg = msg


class bc_options(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("batch", ctypes.c_int32), ("delta", ctypes.c_int32),
                ("lane_max_deg", ctypes.c_int32), ("wg_threads", ctypes.c_int32),
                ("autotune", ctypes.c_int32), ("accumulate", ctypes.c_int32),
                ("lds_vertices", ctypes.c_int32), ("dep_mode", ctypes.c_int32),
                ("virtual_warp", ctypes.c_int32), ("node_parallel", ctypes.c_int32),
                ("lds_bits", ctypes.c_int32), ("expand_lane_deg", ctypes.c_int32),
                ("wave_max_deg", ctypes.c_int32), ("wg_min_deg", ctypes.c_int32),
                ("far_buckets", ctypes.c_int32), ("stream", ctypes.c_void_p)]


class bc_stats(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double), ("sources", ctypes.c_int64),
                ("reached", ctypes.c_int64), ("arcs_out_reached", ctypes.c_int64),
                ("dag_arcs", ctypes.c_int64), ("improvements", ctypes.c_int64),
                ("bands", ctypes.c_int64), ("iterations", ctypes.c_int64),
                ("sigma_rounds", ctypes.c_int64), ("delta_rounds", ctypes.c_int64),
                ("first_bad_source", ctypes.c_int64), ("algo_bytes", ctypes.c_double),
                ("kernel_ms", ctypes.c_double), ("kernel_launches", ctypes.c_int64),
                ("phase_ticks", ctypes.c_int64 * 5),
                ("mode", ctypes.c_int32), ("batch", ctypes.c_int32), ("delta", ctypes.c_int32),
                ("lane_max_deg", ctypes.c_int32), ("wg_threads", ctypes.c_int32),
                ("accumulate", ctypes.c_int32), ("lds_vertices", ctypes.c_int32),
                ("dep_mode", ctypes.c_int32), ("virtual_warp", ctypes.c_int32),
                ("node_parallel", ctypes.c_int32), ("lds_bits", ctypes.c_int32),
                ("expand_lane_deg", ctypes.c_int32), ("wave_max_deg", ctypes.c_int32),
                ("wg_min_deg", ctypes.c_int32), ("far_buckets", ctypes.c_int32)]

    def as_dict(self) -> dict:
        d = {name: getattr(self, name) for name, _ in self._fields_}
        d["phase_ticks"] = list(self.phase_ticks)
        return d


class bc_graph_info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nnz", ctypes.c_int64), ("directed", ctypes.c_int32),
                ("w_max", ctypes.c_int32), ("max_out_degree", ctypes.c_int32),
                ("packed_arcs", ctypes.c_int32), ("renumbered", ctypes.c_int32),
                ("device_bytes", ctypes.c_int64), ("tuned", ctypes.c_int32),
                ("tuned_delta", ctypes.c_int32), ("tuned_wg_threads", ctypes.c_int32),
                ("tuned_lane_max_deg", ctypes.c_int32), ("tuned_dep_mode", ctypes.c_int32),
                ("tuned_expand_lane_deg", ctypes.c_int32), ("tuned_wave_max_deg", ctypes.c_int32),
                ("tuned_wg_min_deg", ctypes.c_int32), ("tuned_batch", ctypes.c_int32),
                ("tuned_lds_bits", ctypes.c_int32),
                ("tuning_trials", ctypes.c_int64)]


class bc_server_opts(ctypes.Structure):
    _fields_ = [("result_budget_bytes", ctypes.c_int64), ("slab_bytes_per_sweep", ctypes.c_int64),
                ("max_active", ctypes.c_int32), ("sweeps_per_graph", ctypes.c_int32),
                ("slots_per_sweep", ctypes.c_int32), ("items_per_sweep", ctypes.c_int32),
                ("compute", bc_options), ("order", ctypes.c_int32),
                ("graph_order", ctypes.c_int32), ("gpu_share", ctypes.c_double),
                ("starve_after_s", ctypes.c_double)]


class bc_server_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("failed", ctypes.c_int64), ("waiting", ctypes.c_int64),
                ("active", ctypes.c_int64), ("p50_ms", ctypes.c_double),
                ("p99_ms", ctypes.c_double), ("mean_ms", ctypes.c_double),
                ("max_ms", ctypes.c_double), ("queue_ms_sum", ctypes.c_double),
                ("gteps", ctypes.c_double), ("sweeps", ctypes.c_int64),
                ("device_bytes_in_use", ctypes.c_int64)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


def _load():
    # torch ships its own HIP runtime with the same soname as the system one;
    # loading torch first makes this library bind to that single runtime, so
    # device pointers and streams from torch tensors are valid here.
    import torch  # noqa: F401

    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_1701_05975_amd.build` (hipcc, gfx950)")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    i32, i64, u32 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
    sig = {
        "bc_create_graph": ([i32, i64, P, P, P, u32, ctypes.POINTER(P)], ctypes.c_int),
        "bc_create_graph_device": ([i32, i64, P, P, P, u32, P, ctypes.POINTER(P)], ctypes.c_int),
        "bc_destroy_graph": ([P], ctypes.c_int),
        "bc_get_graph_info": ([P, ctypes.POINTER(bc_graph_info)], ctypes.c_int),
        "bc_compute": ([P, P, i64, ctypes.POINTER(bc_options), ctypes.POINTER(P)], ctypes.c_int),
        "bc_compute_device": ([P, P, i64, ctypes.POINTER(bc_options), P,
                               ctypes.POINTER(bc_stats)], ctypes.c_int),
        "bc_compute_device_noalloc": ([P, P, i64, ctypes.POINTER(bc_options), P,
                                       ctypes.POINTER(bc_stats)], ctypes.c_int),
        "bc_compute_edges": ([P, P, i64, ctypes.POINTER(bc_options), P, P], ctypes.c_int),
        "bc_compute_edges_device": ([P, P, i64, ctypes.POINTER(bc_options), P, P,
                                     ctypes.POINTER(bc_stats)], ctypes.c_int),
        "bc_result_bc": ([P, P], ctypes.c_int),
        "bc_result_device_ptr": ([P, ctypes.POINTER(P)], ctypes.c_int),
        "bc_result_stats": ([P, ctypes.POINTER(bc_stats)], ctypes.c_int),
        "bc_destroy_result": ([P], ctypes.c_int),
        "bc_source_state": ([P, i32, ctypes.POINTER(bc_options), P, P, P], ctypes.c_int),
        "bc_update_arc_device": ([P, P, P, i32, i32, i32, i32, ctypes.POINTER(bc_options), P,
                                  P, ctypes.POINTER(i64)], ctypes.c_int),
        "bc_algo_bytes": ([i32, i32, i64, i64, i64], ctypes.c_double),
        "bc_server_create": ([ctypes.POINTER(bc_server_opts), ctypes.POINTER(P)], ctypes.c_int),
        "bc_server_submit": ([P, P, P, i64, ctypes.POINTER(ctypes.c_uint64)], ctypes.c_int),
        "bc_server_wait": ([P, ctypes.c_uint64, i64, ctypes.POINTER(P)], ctypes.c_int),
        "bc_server_get_stats": ([P, ctypes.POINTER(bc_server_stats)], ctypes.c_int),
        "bc_server_destroy": ([P], ctypes.c_int),
        "bc_last_error": ([], ctypes.c_char_p),
        "bc_version": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    return lib


_lib = _load()


def lib():
    return _lib


def _check(status: int):
    if status != BC_OK:
        raise BCError(status, _lib.bc_last_error().decode())


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def make_options(mode=0, batch=0, delta=0, lane_max_deg=0, wg_threads=0, autotune=0,
                 accumulate=0, lds_vertices=0, dep_mode=0, virtual_warp=0, node_parallel=0,
                 lds_bits=0, expand_lane_deg=0, wave_max_deg=0, wg_min_deg=0,
                 far_buckets=0, stream=None) -> bc_options:
    o = bc_options()
    o.mode, o.batch, o.delta = mode, batch, delta
    o.lane_max_deg, o.wg_threads, o.autotune, o.accumulate = lane_max_deg, wg_threads, autotune, accumulate
    o.lds_vertices = lds_vertices
    o.dep_mode = dep_mode
    o.virtual_warp = virtual_warp
    o.node_parallel = node_parallel
    o.lds_bits = lds_bits
    o.expand_lane_deg = expand_lane_deg
    o.wave_max_deg = wave_max_deg
    o.wg_min_deg = wg_min_deg
    o.far_buckets = far_buckets
    o.stream = stream
    return o


# --------------------------------------------------------------------------- ABI

def bc_create_graph(n: int, row_ptr, col, w, flags: int = 0) -> ctypes.c_void_p:
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    c = np.ascontiguousarray(col, dtype=np.int32)
    ww = np.ascontiguousarray(w, dtype=np.int32)
    out = ctypes.c_void_p()
    _check(_lib.bc_create_graph(int(n), int(c.shape[0]), _ptr(rp), _ptr(c), _ptr(ww),
                                int(flags), ctypes.byref(out)))
    return out


def bc_create_graph_device(n: int, nnz: int, row_ptr_dev_ptr: int, col_dev_ptr: int,
                           w_dev_ptr: int, flags: int = 0, stream=None) -> ctypes.c_void_p:
    """Graph from device arrays (int64 row offsets, int32 heads and weights)."""
    out = ctypes.c_void_p()
    _check(_lib.bc_create_graph_device(int(n), int(nnz), ctypes.c_void_p(row_ptr_dev_ptr),
                                       ctypes.c_void_p(col_dev_ptr or None),
                                       ctypes.c_void_p(w_dev_ptr or None), int(flags),
                                       ctypes.c_void_p(stream or None), ctypes.byref(out)))
    return out


def bc_destroy_graph(g) -> None:
    _check(_lib.bc_destroy_graph(g))


def bc_get_graph_info(g) -> dict:
    info = bc_graph_info()
    _check(_lib.bc_get_graph_info(g, ctypes.byref(info)))
    return {name: getattr(info, name) for name, _ in info._fields_}


def bc_compute(g, sources, k: int | None = None, options: bc_options | None = None):
    """Host source list (or None for all vertices); returns a result handle."""
    out = ctypes.c_void_p()
    opt = ctypes.byref(options) if options is not None else None
    if sources is None:
        _check(_lib.bc_compute(g, None, int(k), opt, ctypes.byref(out)))
    else:
        s = np.ascontiguousarray(sources, dtype=np.int32)
        _check(_lib.bc_compute(g, _ptr(s) if s.size else None, int(s.shape[0]), opt,
                               ctypes.byref(out)))
    return out


def bc_compute_device(g, sources_dev_ptr: int, k: int, bc_dev_ptr: int,
                      options: bc_options | None = None) -> bc_stats:
    st = bc_stats()
    opt = ctypes.byref(options) if options is not None else None
    _check(_lib.bc_compute_device(g, ctypes.c_void_p(sources_dev_ptr), int(k), opt,
                                  ctypes.c_void_p(bc_dev_ptr), ctypes.byref(st)))
    return st


def bc_compute_device_noalloc(g, sources_dev_ptr: int, k: int, bc_dev_ptr: int,
                              options: bc_options | None = None) -> bc_stats:
    """The batched form with its state slabs in the library's fixed device
    array (no device allocation during the call)."""
    st = bc_stats()
    opt = ctypes.byref(options) if options is not None else None
    _check(_lib.bc_compute_device_noalloc(g, ctypes.c_void_p(sources_dev_ptr), int(k), opt,
                                          ctypes.c_void_p(bc_dev_ptr), ctypes.byref(st)))
    return st


NOALLOC_SCRATCH_BYTES = 64 << 20  # BC_NOALLOC_SCRATCH_BYTES of include/bc.h


def bc_compute_edges(g, sources, n: int, nnz: int, options: bc_options | None = None):
    """(bc float64[n], edge betweenness float64[nnz] in CSR arc order)."""
    opt = ctypes.byref(options) if options is not None else None
    bc = np.empty(max(n, 1), dtype=np.float64)
    ebc = np.empty(max(nnz, 1), dtype=np.float64)
    if sources is None:
        _check(_lib.bc_compute_edges(g, None, int(n), opt, _ptr(bc), _ptr(ebc)))
    else:
        s = np.ascontiguousarray(sources, dtype=np.int32)
        _check(_lib.bc_compute_edges(g, _ptr(s) if s.size else None, int(s.shape[0]), opt,
                                     _ptr(bc), _ptr(ebc)))
    return bc[:n], ebc[:nnz]


def bc_compute_edges_device(g, sources_dev_ptr: int, k: int, bc_dev_ptr: int, ebc_dev_ptr: int,
                            options: bc_options | None = None) -> bc_stats:
    st = bc_stats()
    opt = ctypes.byref(options) if options is not None else None
    _check(_lib.bc_compute_edges_device(g, ctypes.c_void_p(sources_dev_ptr), int(k), opt,
                                        ctypes.c_void_p(bc_dev_ptr), ctypes.c_void_p(ebc_dev_ptr),
                                        ctypes.byref(st)))
    return st


def bc_result_bc(r, n: int) -> np.ndarray:
    out = np.empty(max(n, 1), dtype=np.float64)
    _check(_lib.bc_result_bc(r, _ptr(out)))
    return out[:n]


def bc_result_device_ptr(r) -> int:
    p = ctypes.c_void_p()
    _check(_lib.bc_result_device_ptr(r, ctypes.byref(p)))
    return p.value


def bc_result_stats(r) -> bc_stats:
    st = bc_stats()
    _check(_lib.bc_result_stats(r, ctypes.byref(st)))
    return st


def bc_destroy_result(r) -> None:
    _check(_lib.bc_destroy_result(r))


def bc_source_state(g, s: int, n: int, options: bc_options | None = None):
    d = np.empty(n, dtype=np.int32)
    sigma = np.empty(n, dtype=np.uint64)
    delta = np.empty(n, dtype=np.float64)
    opt = ctypes.byref(options) if options is not None else None
    _check(_lib.bc_source_state(g, int(s), opt, _ptr(d), _ptr(sigma), _ptr(delta)))
    return d, sigma, delta


def bc_update_arc_device(g_old, g_new, g_rev, tail: int, head: int, w_old: int, w_new: int,
                         bc_dev_ptr: int, affected_dev_ptr: int = 0,
                         options: bc_options | None = None) -> int:
    """Updates bc_dev (all-source centralities of g_old) to those of g_new; returns
    the number of sources run again (their ids go to affected_dev_ptr if given)."""
    k = ctypes.c_int64(0)
    opt = ctypes.byref(options) if options is not None else None
    _check(_lib.bc_update_arc_device(g_old, g_new, g_rev, int(tail), int(head), int(w_old),
                                     int(w_new), opt, ctypes.c_void_p(bc_dev_ptr),
                                     ctypes.c_void_p(affected_dev_ptr or None),
                                     ctypes.byref(k)))
    return int(k.value)


def bc_algo_bytes(n: int, weight_bytes: int, arcs: int, reached: int, dag_arcs: int) -> float:
    return _lib.bc_algo_bytes(n, weight_bytes, arcs, reached, dag_arcs)


def bc_version() -> str:
    return _lib.bc_version().decode()


# --------------------------------------------------------------------------- convenience

class Graph:
    """Owning wrapper of a bc_graph handle built from a CSR graph object."""

    def __init__(self, csr, keep_order: bool = False, edges: bool = False):
        self.n = int(csr.n)
        self.m = int(csr.m)
        self.csr = csr
        flags = (BC_DIRECTED if csr.directed else 0) | (BC_KEEP_ORDER if keep_order else 0)
        flags |= BC_EDGE_BC if edges else 0
        self.handle = bc_create_graph(csr.n, csr.row_ptr, csr.col, csr.w, flags)

    @classmethod
    def from_device(cls, csr, row_ptr_t, col_t, w_t, keep_order: bool = False,
                    edges: bool = False, stream=None) -> "Graph":
        """Graph built by bc_create_graph_device from device tensors (int64 row
        offsets, int32 heads, int32 weights) holding the CSR of `csr`."""
        self = cls.__new__(cls)
        self.n = int(csr.n)
        self.m = int(csr.m)
        self.csr = csr
        flags = (BC_DIRECTED if csr.directed else 0) | (BC_KEEP_ORDER if keep_order else 0)
        flags |= BC_EDGE_BC if edges else 0
        self.handle = None
        self.handle = bc_create_graph_device(csr.n, int(col_t.numel()), row_ptr_t.data_ptr(),
                                             col_t.data_ptr(), w_t.data_ptr(), flags, stream)
        return self

    def info(self) -> dict:
        return bc_get_graph_info(self.handle)

    def bc(self, sources=None, **opts):
        """(bc float64[n], stats dict) over the given host source list (None = all)."""
        o = make_options(**opts)
        r = bc_compute(self.handle, sources, self.n if sources is None else None, o)
        try:
            return bc_result_bc(r, self.n), bc_result_stats(r).as_dict()
        finally:
            bc_destroy_result(r)

    def edge_bc(self, sources=None, **opts):
        """(bc float64[n], edge betweenness float64[nnz]) over a host source list."""
        return bc_compute_edges(self.handle, sources, self.n, int(self.csr.nnz),
                                make_options(**opts))

    def source_state(self, s: int, **opts):
        return bc_source_state(self.handle, s, self.n, make_options(**opts))

    def close(self):
        if self.handle:
            bc_destroy_graph(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def bc_last_error() -> str:
    return _lib.bc_last_error().decode()


# --------------------------------------------------------------------------- serving

def bc_server_create(opts: bc_server_opts | None = None):
    out = ctypes.c_void_p()
    _check(_lib.bc_server_create(ctypes.byref(opts) if opts is not None else None,
                                 ctypes.byref(out)))
    return out


def bc_server_submit(sv, g, sources) -> int:
    s = np.ascontiguousarray(sources, dtype=np.int32)
    t = ctypes.c_uint64()
    _check(_lib.bc_server_submit(sv, g, _ptr(s) if s.size else None, int(s.shape[0]),
                                 ctypes.byref(t)))
    return t.value


def bc_server_wait(sv, ticket: int, timeout_us: int = -1):
    out = ctypes.c_void_p()
    _check(_lib.bc_server_wait(sv, ctypes.c_uint64(ticket), int(timeout_us), ctypes.byref(out)))
    return out


def bc_server_get_stats(sv) -> bc_server_stats:
    st = bc_server_stats()
    _check(_lib.bc_server_get_stats(sv, ctypes.byref(st)))
    return st


def bc_server_destroy(sv) -> None:
    _check(_lib.bc_server_destroy(sv))


def make_server_opts(result_budget_bytes=0, slab_bytes_per_sweep=0, max_active=0,
                     sweeps_per_graph=0, slots_per_sweep=0, items_per_sweep=0, order=0,
                     graph_order=0, gpu_share=0.0, starve_after_s=0.0,
                     **compute) -> bc_server_opts:
    o = bc_server_opts()
    o.result_budget_bytes = result_budget_bytes
    o.slab_bytes_per_sweep = slab_bytes_per_sweep
    o.max_active = max_active
    o.sweeps_per_graph = sweeps_per_graph
    o.slots_per_sweep = slots_per_sweep
    o.items_per_sweep = items_per_sweep
    o.order = order
    o.graph_order = graph_order
    o.gpu_share = gpu_share
    o.starve_after_s = starve_after_s
    o.compute = make_options(**compute)
    return o


class Server:
    """Owning wrapper of a bc_server handle."""

    def __init__(self, **opts):
        self._graphs = {}  # graphs the server holds until it is closed
        self.handle = bc_server_create(make_server_opts(**opts))

    def submit(self, graph: "Graph", sources) -> int:
        t = bc_server_submit(self.handle, graph.handle, sources)
        self._graphs[graph.handle.value] = graph
        return t

    def wait(self, ticket: int, n: int, timeout_us: int = -1):
        """(bc float64[n], latency ms) of a finished request."""
        r = bc_server_wait(self.handle, ticket, timeout_us)
        try:
            return bc_result_bc(r, n), bc_result_stats(r).ms
        finally:
            bc_destroy_result(r)

    def stats(self) -> dict:
        return bc_server_get_stats(self.handle).as_dict()

    def close(self):
        if self.handle:
            bc_server_destroy(self.handle)
            self.handle = None
        self._graphs = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
