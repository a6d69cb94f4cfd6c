"""Python binding for libhb.so: HyperBall over a LEB128 delta-compressed CSR on gfx950.

Argument marshalling only (ctypes): every step of the computation runs in the
library's HIP kernels and C++ host runtime.  The names mirror ``include/hb.h``.
There is no fallback: if ``libhb.so`` is not built, importing works but every
call raises ``HBError``.
"""
from __future__ import annotations

import atexit
import ctypes
import os
from dataclasses import dataclass

import numpy as np

__all__ = [
    "HBError", "Result", "Graph", "lib_path", "version", "device_count", "csr_encode",
    "csr_validate", "graph_load", "run", "run_batch", "release_cache", "tune_cache", "tune_clear",
    "copy_probe", "server_start", "server_stop", "unpack_nibbles",
    "server_stats", "submit", "Ticket", "HB_OK", "HB_PENDING", "HB_EINVAL", "HB_ECORRUPT",
    "HB_ENOMEM", "HB_EDEVICE", "HB_ENOTFOUND", "HB_EBUSY",
]

HB_OK, HB_PENDING = 0, 1
HB_EINVAL, HB_ECORRUPT, HB_ENOMEM, HB_EDEVICE, HB_ENOTFOUND, HB_EBUSY = -1, -2, -3, -4, -5, -6
P_MIN, P_MAX = 4, 16
STATIC_SCRATCH_BYTES = 64 << 20  # HB_STATIC_SCRATCH_BYTES in hb.h

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

u8p = ctypes.POINTER(ctypes.c_uint8)
u32p = ctypes.POINTER(ctypes.c_uint32)
u64p = ctypes.POINTER(ctypes.c_uint64)
dblp = ctypes.POINTER(ctypes.c_double)


class HBError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"[{status}] {msg}")
        self.status = status


class _CSR(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint32), ("n_edges", ctypes.c_uint64), ("offsets", u64p),
                ("degrees", u32p), ("bytes", u8p), ("comp_size", u32p), ("order", u32p),
                ("hash_ids", u32p), ("xy", ctypes.POINTER(ctypes.c_int32))]


class _Result(ctypes.Structure):
    _fields_ = [("reach", dblp), ("sum_d", dblp), ("mean_depth", dblp), ("registers", u8p),
                ("passes", ctypes.c_uint32), ("converged", ctypes.c_uint32),
                ("productive_iters", ctypes.c_uint32),
                ("c0", ctypes.c_double), ("edge_unions", ctypes.c_uint64),
                ("init_ms", ctypes.c_double), ("iter_ms", ctypes.c_double),
                ("table_ms", ctypes.c_double), ("run_ms", ctypes.c_double),
                ("union_kernel", ctypes.c_uint32), ("table_levels", ctypes.c_uint32),
                ("lanes_per_node", ctypes.c_uint32), ("nodes_per_block", ctypes.c_uint32),
                ("register_bits", ctypes.c_uint32), ("tune_ms", ctypes.c_double),
                ("t_submit_ns", ctypes.c_uint64), ("t_admit_ns", ctypes.c_uint64),
                ("t_start_ns", ctypes.c_uint64), ("t_end_ns", ctypes.c_uint64)]


class _ServerOpts(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_uint64), ("max_running", ctypes.c_uint32),
                ("union_kernel", ctypes.c_uint32), ("table_levels", ctypes.c_uint32),
                ("slow_lane_bytes", ctypes.c_uint64), ("slow_lane_running", ctypes.c_uint32)]


class _CacheStats(ctypes.Structure):
    _fields_ = [("graphs", ctypes.c_uint32), ("busy", ctypes.c_uint32), ("bytes", ctypes.c_uint64),
                ("hits", ctypes.c_uint64), ("misses", ctypes.c_uint64),
                ("evictions", ctypes.c_uint64)]


class _ServerStats(ctypes.Structure):
    _fields_ = [("running", ctypes.c_uint32), ("queued", ctypes.c_uint32),
                ("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("steps", ctypes.c_uint64), ("budget_bytes", ctypes.c_uint64),
                ("used_bytes", ctypes.c_uint64), ("peak_used_bytes", ctypes.c_uint64),
                ("edge_unions", ctypes.c_uint64)]


class _Stats(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint32), ("n_edges", ctypes.c_uint64), ("n_bytes", ctypes.c_uint64),
                ("n_runs", ctypes.c_uint64), ("table_rows", ctypes.c_uint64 * 25),
                ("local_run_reads", ctypes.c_uint64), ("group_rows", ctypes.c_uint64),
                ("group_levels", ctypes.c_uint32)]


class _RunOpts(ctypes.Structure):
    _fields_ = [("union_kernel", ctypes.c_uint32), ("table_levels", ctypes.c_uint32),
                ("tune", ctypes.c_uint32), ("lanes_per_node", ctypes.c_uint32),
                ("nodes_per_block", ctypes.c_uint32), ("register_bits", ctypes.c_uint32)]


class _TuneEntry(ctypes.Structure):
    _fields_ = [("p", ctypes.c_uint32), ("register_bits", ctypes.c_uint32),
                ("union_kernel", ctypes.c_uint32), ("batched", ctypes.c_uint32), ("log2_nodes", ctypes.c_uint32),
                ("log2_rows_per_node", ctypes.c_uint32), ("lanes_per_node", ctypes.c_uint32),
                ("nodes_per_block", ctypes.c_uint32), ("best_ms", ctypes.c_double),
                ("default_ms", ctypes.c_double)]


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class _Options(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_uint64), ("dev_alloc", _ALLOC_FN),
                ("dev_free", _FREE_FN), ("alloc_user", ctypes.c_void_p),
                ("stream", ctypes.c_void_p), ("stop_rule", ctypes.c_uint32),
                ("stop_delta", ctypes.c_double), ("tune_seed", ctypes.POINTER(_TuneEntry)),
                ("tune_seed_count", ctypes.c_uint32)]


class _MemStats(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_uint64), ("held_bytes", ctypes.c_uint64),
                ("peak_held_bytes", ctypes.c_uint64), ("pool_bytes", ctypes.c_uint64),
                ("pool_used_bytes", ctypes.c_uint64), ("pool_peak_used_bytes", ctypes.c_uint64)]


STOP_CONVERGED, STOP_DEPTH = 0, 1
TUNE_CACHED, TUNE_MEASURE, TUNE_OFF = 0, 1, 2
_TUNE = {"cached": TUNE_CACHED, "measure": TUNE_MEASURE, "off": TUNE_OFF}


def _run_opts(kernel: str, table_levels: int, tune: str, lanes_per_node: int,
              nodes_per_block: int, register_bits: int = 8) -> _RunOpts:
    return _RunOpts(_KERNELS[kernel], table_levels, _TUNE[tune], lanes_per_node, nodes_per_block,
                    register_bits)


def unpack_nibbles(regs: np.ndarray) -> np.ndarray:
    """4-bit registers (n, 2^(p-1) bytes) -> one register per byte (n, 2^p): register
    2k is the low nibble of byte k, register 2k + 1 the high nibble."""
    out = np.empty((regs.shape[0], regs.shape[1] * 2), np.uint8)
    out[:, 0::2] = regs & 0x0F
    out[:, 1::2] = regs >> 4
    return out


VGA_METRICS = ("connectivity", "control", "mean_depth", "relative_asymmetry", "integration_hh",
               "integration_tekl", "integration_pvalue", "point_first_moment",
               "point_second_moment")


class _VgaOut(ctypes.Structure):
    _fields_ = [(name, dblp) for name in VGA_METRICS]


class _LocalOut(ctypes.Structure):
    _fields_ = [("pairs", ctypes.POINTER(ctypes.c_uint64)),
                ("ball2", ctypes.POINTER(ctypes.c_uint32)),
                ("clustering", dblp), ("controllability", dblp)]


class _Job(ctypes.Structure):
    _fields_ = [("g", ctypes.c_void_p), ("p", ctypes.c_uint32), ("depth_limit", ctypes.c_uint32),
                ("hash_seed", ctypes.c_uint64)]


UNION_AUTO, UNION_EDGES, UNION_RUNS, UNION_GROUPS = 0, 1, 2, 3
_KERNELS = {"auto": UNION_AUTO, "edges": UNION_EDGES, "runs": UNION_RUNS, "groups": UNION_GROUPS}


def lib_path() -> str:
    return os.path.join(_HERE, "libhb.so")


def _lib():
    global _LIB
    if _LIB is None:
        path = lib_path()
        if not os.path.exists(path):
            raise HBError(HB_EDEVICE, f"{path} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(path)
        st = ctypes.c_int32
        L.hb_version.argtypes = []
        L.hb_version.restype = ctypes.c_char_p
        L.hb_last_error.argtypes = []
        L.hb_last_error.restype = ctypes.c_char_p
        L.hb_device_count.argtypes = [ctypes.POINTER(ctypes.c_int32)]
        L.hb_device_count.restype = st
        L.hb_csr_encode.argtypes = [ctypes.c_uint32, u64p, u32p, u64p, u32p, u8p, ctypes.c_uint64,
                                    u64p]
        L.hb_csr_encode.restype = st
        L.hb_csr_validate.argtypes = [ctypes.POINTER(_CSR), u32p]
        L.hb_csr_validate.restype = st
        L.hb_graph_load.argtypes = [ctypes.POINTER(_CSR), ctypes.POINTER(ctypes.c_void_p)]
        L.hb_graph_load.restype = st
        L.hb_graph_free.argtypes = [ctypes.c_void_p]
        L.hb_graph_free.restype = st
        L.hb_graph_info.argtypes = [ctypes.c_void_p, u32p, u64p, u64p]
        L.hb_graph_info.restype = st
        L.hb_run.argtypes = [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64,
                             ctypes.POINTER(_Result)]
        L.hb_run.restype = st
        L.hb_graph_stats.argtypes = [ctypes.c_void_p, ctypes.POINTER(_Stats)]
        L.hb_graph_stats.restype = st
        L.hb_run_with.argtypes = [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32,
                                  ctypes.c_uint64, ctypes.POINTER(_RunOpts),
                                  ctypes.POINTER(_Result)]
        L.hb_run_with.restype = st
        L.hb_run_static.argtypes = L.hb_run_with.argtypes
        L.hb_run_static.restype = st
        L.hb_gather_probe.argtypes = [ctypes.c_uint32] * 8 + [ctypes.POINTER(ctypes.c_double)]
        L.hb_gather_probe.restype = st
        L.hb_set_options.argtypes = [ctypes.POINTER(_Options)]
        L.hb_set_options.restype = st
        L.hb_get_options.argtypes = [ctypes.POINTER(_Options)]
        L.hb_get_options.restype = st
        L.hb_memory_stats.argtypes = [ctypes.c_int32, ctypes.POINTER(_MemStats)]
        L.hb_memory_stats.restype = st
        L.hb_run_batch.argtypes = [ctypes.POINTER(_Job), ctypes.c_uint32, ctypes.POINTER(_RunOpts),
                                   ctypes.POINTER(_Result)]
        L.hb_run_batch.restype = st
        L.hb_server_start.argtypes = [ctypes.POINTER(_ServerOpts)]
        L.hb_server_start.restype = st
        L.hb_server_stop.argtypes = []
        L.hb_server_stop.restype = st
        L.hb_submit.argtypes = [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64,
                                ctypes.c_uint32, ctypes.POINTER(ctypes.c_uint64)]
        L.hb_submit.restype = st
        L.hb_poll.argtypes = [ctypes.c_uint64, ctypes.POINTER(_Result)]
        L.hb_poll.restype = st
        L.hb_wait.argtypes = [ctypes.c_uint64, ctypes.POINTER(_Result)]
        L.hb_wait.restype = st
        L.hb_server_stats.argtypes = [ctypes.POINTER(_ServerStats)]
        L.hb_server_stats.restype = st
        L.hb_submit_cached.argtypes = [ctypes.c_uint64, ctypes.POINTER(_CSR), ctypes.c_uint32,
                                       ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint32,
                                       ctypes.POINTER(ctypes.c_uint64)]
        L.hb_submit_cached.restype = st
        L.hb_graph_cache_stats.argtypes = [ctypes.POINTER(_CacheStats)]
        L.hb_graph_cache_stats.restype = st
        L.hb_graph_cache_clear.argtypes = []
        L.hb_graph_cache_clear.restype = st
        L.hb_graph_cache_drop.argtypes = [ctypes.c_uint64]
        L.hb_graph_cache_drop.restype = st
        L.hb_release_cache.argtypes = []
        L.hb_release_cache.restype = st
        L.hb_tune_cache.argtypes = [ctypes.POINTER(_TuneEntry), ctypes.c_uint32, u32p]
        L.hb_tune_cache.restype = st
        L.hb_tune_clear.argtypes = []
        L.hb_tune_clear.restype = st
        L.hb_vga_metrics.argtypes = [ctypes.c_void_p, dblp, ctypes.POINTER(_VgaOut)]
        L.hb_vga_metrics.restype = st
        L.hb_local_metrics.argtypes = [ctypes.c_void_p, ctypes.POINTER(_LocalOut)]
        L.hb_local_metrics.restype = st
        L.hb_copy_probe.argtypes = [ctypes.c_uint64, ctypes.c_uint32, dblp]
        L.hb_copy_probe.restype = st
        _LIB = L
    return _LIB


def _check(status: int) -> int:
    if status < 0:
        raise HBError(status, _lib().hb_last_error().decode(errors="replace"))
    return status


def _ptr(a: np.ndarray | None, ct):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ct))


def version() -> str:
    return _lib().hb_version().decode()


def device_count() -> int:
    c = ctypes.c_int32(0)
    _check(_lib().hb_device_count(ctypes.byref(c)))
    return int(c.value)


def csr_encode(adj_offsets: np.ndarray, adj_ids: np.ndarray):
    """Sorted adjacency -> (offsets u64[n+1], degrees u32[n], bytes u8[]) via hb_csr_encode."""
    adj_offsets = np.ascontiguousarray(adj_offsets, np.uint64)
    adj_ids = np.ascontiguousarray(adj_ids, np.uint32)
    n = adj_offsets.shape[0] - 1
    offsets = np.zeros(n + 1, np.uint64)
    degrees = np.zeros(max(n, 1), np.uint32)[:n]
    blen = ctypes.c_uint64(0)
    L = _lib()
    ids_p = _ptr(adj_ids, ctypes.c_uint32) if adj_ids.size else None
    _check(L.hb_csr_encode(n, _ptr(adj_offsets, ctypes.c_uint64), ids_p,
                           _ptr(offsets, ctypes.c_uint64), _ptr(degrees, ctypes.c_uint32), None, 0,
                           ctypes.byref(blen)))
    data = np.zeros(max(1, int(blen.value)), np.uint8)
    _check(L.hb_csr_encode(n, _ptr(adj_offsets, ctypes.c_uint64), ids_p,
                           _ptr(offsets, ctypes.c_uint64), _ptr(degrees, ctypes.c_uint32),
                           _ptr(data, ctypes.c_uint8), data.shape[0], ctypes.byref(blen)))
    return offsets, degrees, data[:int(blen.value)]


def _make_csr(offsets, degrees, data, comp_size=None, n_edges=None, order=None, hash_ids=None,
              xy=None):
    offsets = np.ascontiguousarray(offsets, np.uint64)
    degrees = np.ascontiguousarray(degrees, np.uint32)
    data = np.ascontiguousarray(data, np.uint8)
    n = degrees.shape[0]
    if offsets.shape[0] != n + 1:
        raise HBError(HB_EINVAL, "offsets must have n + 1 entries")
    keep = [offsets, degrees, data]
    c = _CSR()
    c.n = n
    c.n_edges = int(degrees.sum(dtype=np.uint64)) if n_edges is None else int(n_edges)
    c.offsets = _ptr(offsets, ctypes.c_uint64)
    c.degrees = _ptr(degrees, ctypes.c_uint32)
    c.bytes = _ptr(data, ctypes.c_uint8) if data.size else None
    for name, arr in (("comp_size", comp_size), ("order", order), ("hash_ids", hash_ids)):
        if arr is not None:
            arr = np.ascontiguousarray(arr, np.uint32)
            if arr.shape != (n,):
                raise HBError(HB_EINVAL, f"{name} must have n entries")
            keep.append(arr)
            setattr(c, name, _ptr(arr, ctypes.c_uint32))
        else:
            setattr(c, name, None)
    if xy is not None:
        xy = np.ascontiguousarray(xy, np.int32)
        if xy.shape != (n, 2):
            raise HBError(HB_EINVAL, "xy must have shape (n, 2)")
        keep.append(xy)
        c.xy = _ptr(xy, ctypes.c_int32)
    else:
        c.xy = None
    return c, keep


def csr_validate(offsets, degrees, data, n_edges=None):
    """(status, bad_node) from hb_csr_validate (no exception on HB_ECORRUPT)."""
    c, keep = _make_csr(offsets, degrees, data, n_edges=n_edges)
    bad = ctypes.c_uint32(0)
    st = _lib().hb_csr_validate(ctypes.byref(c), ctypes.byref(bad))
    del keep
    if st not in (HB_OK, HB_ECORRUPT):
        _check(st)
    return int(st), int(bad.value)


@dataclass
class Result:
    reach: np.ndarray | None
    sum_d: np.ndarray | None
    mean_depth: np.ndarray | None
    registers: np.ndarray | None
    passes: int
    converged: bool
    productive_iters: int
    c0: float
    edge_unions: int
    init_ms: float
    iter_ms: float
    table_ms: float
    run_ms: float
    union_kernel: str
    table_levels: int
    lanes_per_node: int
    nodes_per_block: int
    register_bits: int
    tune_ms: float
    t_submit_ns: int
    t_admit_ns: int
    t_start_ns: int
    t_end_ns: int


class Graph:
    """A compressed CSR resident in device memory (hb_graph)."""

    def __init__(self, offsets, degrees, data, comp_size=None, n_edges=None, order=None,
                 hash_ids=None, xy=None):
        c, keep = _make_csr(offsets, degrees, data, comp_size, n_edges, order, hash_ids, xy)
        h = ctypes.c_void_p()
        _check(_lib().hb_graph_load(ctypes.byref(c), ctypes.byref(h)))
        del keep
        self._h = h
        n, e, b = ctypes.c_uint32(), ctypes.c_uint64(), ctypes.c_uint64()
        _check(_lib().hb_graph_info(h, ctypes.byref(n), ctypes.byref(e), ctypes.byref(b)))
        self.n, self.n_edges, self.n_bytes = int(n.value), int(e.value), int(b.value)

    def stats(self) -> dict:
        """hb_graph_stats: runs of consecutive ids and table rows per step for each depth K."""
        st = _Stats()
        _check(_lib().hb_graph_stats(self._h, ctypes.byref(st)))
        return {"n": st.n, "n_edges": st.n_edges, "n_bytes": st.n_bytes, "n_runs": st.n_runs,
                "table_rows": [int(x) for x in st.table_rows],
                "local_run_reads": int(st.local_run_reads), "group_rows": int(st.group_rows),
                "group_levels": int(st.group_levels)}

    def vga_metrics(self, sum_d) -> dict:
        """hb_vga_metrics: the VGA metrics of every node from a run's sum_d (Sec. 3.3)."""
        if self._h is None:
            raise HBError(HB_EINVAL, "graph was freed")
        sd = np.ascontiguousarray(sum_d, np.float64)
        if sd.shape != (self.n,):
            raise HBError(HB_EINVAL, "sum_d must have n entries")
        arrays = {name: np.empty(self.n, np.float64) for name in VGA_METRICS}
        o = _VgaOut(*[_ptr(arrays[name], ctypes.c_double) for name in VGA_METRICS])
        _check(_lib().hb_vga_metrics(self._h, _ptr(sd, ctypes.c_double), ctypes.byref(o)))
        return arrays

    def local_metrics(self) -> dict:
        """hb_local_metrics: exact local metrics of every node (Sec. 3.3) -- ordered
        adjacent neighbour pairs, |B(v, 2)| - 1, clustering, controllability."""
        if self._h is None:
            raise HBError(HB_EINVAL, "graph was freed")
        out = {"pairs": np.empty(self.n, np.uint64), "ball2": np.empty(self.n, np.uint32),
               "clustering": np.empty(self.n, np.float64),
               "controllability": np.empty(self.n, np.float64)}
        o = _LocalOut(_ptr(out["pairs"], ctypes.c_uint64), _ptr(out["ball2"], ctypes.c_uint32),
                      _ptr(out["clustering"], ctypes.c_double),
                      _ptr(out["controllability"], ctypes.c_double))
        _check(_lib().hb_local_metrics(self._h, ctypes.byref(o)))
        return out

    def free(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _check(_lib().hb_graph_free(self._h))
        self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.free()

    def _out_arrays(self, p: int, registers: bool, outputs: bool, register_bits: int = 8):
        return _out_arrays(self.n, p, registers, outputs, register_bits)

    def run(self, p: int, depth_limit: int = 0, seed: int = 0, registers: bool = False,
            outputs: bool = True, kernel: str = "auto", table_levels: int = 0,
            tune: str = "cached", lanes_per_node: int = 0, nodes_per_block: int = 0,
            register_bits: int = 8) -> Result:
        """hb_run_with: HyperBall with precision p; depth_limit 0 = until convergence.

        kernel: "auto", "edges" (gather every neighbour), "runs" (range-max table) or
        "groups" (the table's rows merged over groups of 16 nodes; counters of 256 to
        4096 bytes).
        tune: "cached" (a cached schedule pick, else the default), "measure" (measure
        the schedules first when nothing is cached) or "off"; lanes_per_node and
        nodes_per_block name a schedule explicitly.
        """
        if self._h is None:
            raise HBError(HB_EINVAL, "graph was freed")
        r, arrays = self._out_arrays(p, registers, outputs, register_bits)
        o = _run_opts(kernel, table_levels, tune, lanes_per_node, nodes_per_block, register_bits)
        _check(_lib().hb_run_with(self._h, p, depth_limit, seed & 0xFFFFFFFFFFFFFFFF,
                                  ctypes.byref(o), ctypes.byref(r)))
        return _to_result(r, arrays)

    def run_static(self, p: int, depth_limit: int = 0, seed: int = 0, registers: bool = False,
                   outputs: bool = True, kernel: str = "auto", table_levels: int = 0,
                   tune: str = "cached", lanes_per_node: int = 0, nodes_per_block: int = 0,
                   register_bits: int = 8) -> Result:
        """hb_run_static: as run(), with the counters in the library's static device
        workspace (STATIC_SCRATCH_BYTES per device); the call allocates nothing."""
        if self._h is None:
            raise HBError(HB_EINVAL, "graph was freed")
        r, arrays = self._out_arrays(p, registers, outputs, register_bits)
        o = _run_opts(kernel, table_levels, tune, lanes_per_node, nodes_per_block, register_bits)
        _check(_lib().hb_run_static(self._h, p, depth_limit, seed & 0xFFFFFFFFFFFFFFFF,
                                    ctypes.byref(o), ctypes.byref(r)))
        return _to_result(r, arrays)


def gather_probe(p: int = 10, n_nodes: int = 235770, rows_per_node: int = 1024,
                 table_rows: int = 2048, with_max: bool = True, lanes_per_node: int = 0,
                 nodes_per_block: int = 0, reps: int = 5) -> float:
    """hb_gather_probe: device ms of one launch gathering n_nodes * rows_per_node rows
    of 2^p bytes from an L2-resident table in the run kernel's shape."""
    ms = ctypes.c_double(0.0)
    _check(_lib().hb_gather_probe(p, lanes_per_node, nodes_per_block, table_rows, n_nodes,
                                  rows_per_node, 1 if with_max else 0, reps, ctypes.byref(ms)))
    return ms.value


def copy_probe(nbytes: int = 1 << 30, reps: int = 20) -> float:
    """hb_copy_probe: average device ms of one streaming copy of nbytes."""
    ms = ctypes.c_double(0.0)
    _check(_lib().hb_copy_probe(int(nbytes), int(reps), ctypes.byref(ms)))
    return float(ms.value)


def _to_result(r: _Result, arrays) -> Result:
    reach, sum_d, md, regs = arrays
    name = {UNION_EDGES: "edges", UNION_RUNS: "runs", UNION_GROUPS: "groups"}.get(
        int(r.union_kernel), "?")
    return Result(reach, sum_d, md, regs, int(r.passes), bool(r.converged),
                  int(r.productive_iters), float(r.c0),
                  int(r.edge_unions), float(r.init_ms), float(r.iter_ms), float(r.table_ms),
                  float(r.run_ms), name, int(r.table_levels), int(r.lanes_per_node),
                  int(r.nodes_per_block), int(r.register_bits), float(r.tune_ms),
                  int(r.t_submit_ns),
                  int(r.t_admit_ns), int(r.t_start_ns), int(r.t_end_ns))


def run_batch(jobs, registers: bool = False, outputs: bool = True, kernel: str = "auto",
              table_levels: int = 0, tune: str = "cached", lanes_per_node: int = 0,
              nodes_per_block: int = 0, register_bits: int = 8):
    """hb_run_batch: jobs is a list of (Graph, p, depth_limit, seed); returns Results in order."""
    n = len(jobs)
    cj = (_Job * n)()
    outs = (_Result * n)()
    keep = []
    for i, (g, p, depth, seed) in enumerate(jobs):
        if g._h is None:
            raise HBError(HB_EINVAL, "graph was freed")
        cj[i].g = g._h.value
        cj[i].p = p
        cj[i].depth_limit = depth
        cj[i].hash_seed = seed & 0xFFFFFFFFFFFFFFFF
        r, arrays = g._out_arrays(p, registers, outputs, register_bits)
        outs[i] = r
        keep.append(arrays)
    o = _run_opts(kernel, table_levels, tune, lanes_per_node, nodes_per_block, register_bits)
    _check(_lib().hb_run_batch(cj, n, ctypes.byref(o), outs))
    return [_to_result(outs[i], keep[i]) for i in range(n)]


SUBMIT_REGISTERS = 1
SUBMIT_REG4 = 2
_SERVER_STARTED = False


def server_start(hbm_budget: int = 0, max_running: int = 0, kernel: str = "auto",
                 table_levels: int = 0, slow_lane_bytes: int = 0,
                 slow_lane_running: int = 0) -> None:
    """hb_server_start: start the request loop (continuous batching)."""
    global _SERVER_STARTED
    o = _ServerOpts(hbm_budget, max_running, _KERNELS[kernel], table_levels, slow_lane_bytes,
                    slow_lane_running)
    _check(_lib().hb_server_start(ctypes.byref(o)))
    _SERVER_STARTED = True


def server_stop() -> None:
    """hb_server_stop: finish queued and running requests, then end the loop."""
    global _SERVER_STARTED
    _check(_lib().hb_server_stop())
    _SERVER_STARTED = False


def server_stats() -> dict:
    st = _ServerStats()
    _check(_lib().hb_server_stats(ctypes.byref(st)))
    return {k: int(getattr(st, k)) for k, _ in _ServerStats._fields_}


def _out_arrays(n: int, p: int, registers: bool, outputs: bool, register_bits: int = 8):
    """Host output arrays of one result and the hb_result pointing at them."""
    reach = np.empty(n, np.float64) if outputs else None
    sum_d = np.empty(n, np.float64) if outputs else None
    md = np.empty(n, np.float64) if outputs else None
    width = (1 << p) * register_bits // 8 if register_bits in (4, 8) else 0
    regs = np.empty((n, width), np.uint8) if (registers and P_MIN <= p <= P_MAX and width) \
        else None
    r = _Result()
    r.reach = _ptr(reach, ctypes.c_double)
    r.sum_d = _ptr(sum_d, ctypes.c_double)
    r.mean_depth = _ptr(md, ctypes.c_double)
    r.registers = _ptr(regs, ctypes.c_uint8)
    return r, (reach, sum_d, md, regs)


class Ticket:
    """A submitted request: poll() returns None while pending, then the Result once."""

    def __init__(self, graph: "Graph | None", p: int, registers: bool, ticket: int,
                 register_bits: int = 8, n: int | None = None):
        self.graph, self.p, self.registers, self.id = graph, p, registers, ticket
        self.register_bits = register_bits
        self.n = graph.n if n is None else n

    def _collect(self, fn) -> "Result | None":
        r, arrays = _out_arrays(self.n, self.p, self.registers, True, self.register_bits)
        st = fn(self.id, ctypes.byref(r))
        if st == HB_PENDING:
            return None
        _check(st)
        return _to_result(r, arrays)

    def poll(self):
        return self._collect(_lib().hb_poll)

    def wait(self):
        return self._collect(_lib().hb_wait)


def submit(g: "Graph", p: int, depth_limit: int = 0, seed: int = 0,
           registers: bool = False, register_bits: int = 8) -> Ticket:
    """hb_submit: queue one analysis; returns a Ticket."""
    global _SERVER_STARTED
    t = ctypes.c_uint64(0)
    flags = (SUBMIT_REGISTERS if registers else 0) | (SUBMIT_REG4 if register_bits == 4 else 0)
    _check(_lib().hb_submit(g._h, p, depth_limit, seed & 0xFFFFFFFFFFFFFFFF, flags,
                            ctypes.byref(t)))
    _SERVER_STARTED = True
    return Ticket(g, p, registers, int(t.value), register_bits)


def submit_cached(key: int, p: int, depth_limit: int = 0, seed: int = 0, csr=None,
                  registers: bool = False, register_bits: int = 8, n: int | None = None) -> Ticket:
    """hb_submit_cached: queue an analysis of the cached graph `key`.  csr is None
    (the graph must be cached) or (offsets, degrees, data[, order]) host arrays, read
    only when the key is not cached.  n: node count (from csr when given)."""
    global _SERVER_STARTED
    t = ctypes.c_uint64(0)
    flags = (SUBMIT_REGISTERS if registers else 0) | (SUBMIT_REG4 if register_bits == 4 else 0)
    cptr = None
    if csr is not None:
        off, deg, data = csr[0], csr[1], csr[2]
        order = csr[3] if len(csr) > 3 else None
        c, keep = _make_csr(off, deg, data, order=order)
        cptr = ctypes.byref(c)
        n = c.n
    if n is None:
        raise HBError(HB_EINVAL, "n is needed when no CSR is given")
    _check(_lib().hb_submit_cached(key & 0xFFFFFFFFFFFFFFFF, cptr, p, depth_limit,
                                   seed & 0xFFFFFFFFFFFFFFFF, flags, ctypes.byref(t)))
    _SERVER_STARTED = True
    return Ticket(None, p, registers, int(t.value), register_bits, n=n)


def graph_cache_stats() -> dict:
    """hb_graph_cache_stats: graphs, busy graphs, device bytes, hits, misses, evictions."""
    c = _CacheStats()
    _check(_lib().hb_graph_cache_stats(ctypes.byref(c)))
    return {f: getattr(c, f) for f, _ in _CacheStats._fields_}


def graph_cache_clear() -> None:
    """hb_graph_cache_clear: release every idle cached graph (HBError HB_EBUSY if some
    have requests; those stay)."""
    _check(_lib().hb_graph_cache_clear())


def graph_cache_drop(key: int) -> None:
    """hb_graph_cache_drop: release one idle cached graph."""
    _check(_lib().hb_graph_cache_drop(key & 0xFFFFFFFFFFFFFFFF))


@atexit.register
def _stop_server_at_exit():
    if _SERVER_STARTED and _LIB is not None:
        _LIB.hb_server_stop()


def tune_cache() -> list:
    """hb_tune_cache: the autotuner's picks, one dict per shape class."""
    cnt = ctypes.c_uint32(0)
    _check(_lib().hb_tune_cache(None, 0, ctypes.byref(cnt)))
    buf = (_TuneEntry * max(cnt.value, 1))()
    _check(_lib().hb_tune_cache(buf, cnt.value, ctypes.byref(cnt)))
    out = []
    for e in buf[:cnt.value]:
        out.append({f: getattr(e, f) for f, _ in _TuneEntry._fields_})
        out[-1]["union_kernel"] = {UNION_EDGES: "edges", UNION_RUNS: "runs"}[e.union_kernel]
    return out


# the installed allocator hooks stay referenced while the library may call them
_HOOKS = []


def set_options(hbm_budget: int = 0, dev_alloc=None, dev_free=None, stream=None,
                stop_rule: str = "converged", stop_delta: float = 0.0,
                tune_seed: list | None = None) -> None:
    """hb_set_options (all defaults when called without arguments).

    dev_alloc(bytes) -> int device pointer (0 on failure) and dev_free(ptr) are
    Python callables used for every device allocation of the library; stream is a
    hipStream_t as an int (e.g. torch.cuda.Stream().cuda_stream) for blocking runs;
    stop_rule "converged" (Alg. 1) or "depth" (run exactly the depth limit);
    stop_delta replaces the 0.5 growth threshold; tune_seed: entries as returned by
    tune_cache(), put into the pick cache.
    """
    o = _Options()
    o.hbm_budget = int(hbm_budget)
    hooks = []
    if (dev_alloc is None) != (dev_free is None):
        raise HBError(HB_EINVAL, "dev_alloc and dev_free must be given together")
    if dev_alloc is not None:
        a = _ALLOC_FN(lambda nbytes, user: int(dev_alloc(int(nbytes))) or None)
        f = _FREE_FN(lambda ptr, user: dev_free(int(ptr)))
        o.dev_alloc, o.dev_free = a, f
        hooks = [a, f]
    o.stream = int(stream) if stream else None
    o.stop_rule = {"converged": STOP_CONVERGED, "depth": STOP_DEPTH}[stop_rule]
    o.stop_delta = float(stop_delta)
    seeds = None
    if tune_seed:
        seeds = (_TuneEntry * len(tune_seed))()
        for e, d in zip(seeds, tune_seed):
            for f, _ in _TuneEntry._fields_:
                v = d[f]
                if f == "union_kernel" and isinstance(v, str):
                    v = {"edges": UNION_EDGES, "runs": UNION_RUNS}[v]
                setattr(e, f, v)
        o.tune_seed = seeds
        o.tune_seed_count = len(tune_seed)
    _check(_lib().hb_set_options(ctypes.byref(o)))
    _HOOKS.append(hooks)  # old hooks may still free what they allocated


def get_options() -> dict:
    """hb_get_options: budget, stream, stop rule and threshold in force."""
    o = _Options()
    _check(_lib().hb_get_options(ctypes.byref(o)))
    return {"hbm_budget": o.hbm_budget, "stream": o.stream or 0,
            "hooks": bool(o.dev_alloc), "stop_rule": {STOP_CONVERGED: "converged",
                                                      STOP_DEPTH: "depth"}[o.stop_rule],
            "stop_delta": o.stop_delta}


def memory_stats(device: int = 0) -> dict:
    """hb_memory_stats: device memory the library holds on one device."""
    m = _MemStats()
    _check(_lib().hb_memory_stats(device, ctypes.byref(m)))
    return {f: getattr(m, f) for f, _ in _MemStats._fields_}


def tune_clear() -> None:
    """hb_tune_clear: forget every schedule pick."""
    _check(_lib().hb_tune_clear())


def release_cache() -> None:
    """hb_release_cache: free the device workspace kept between batched calls."""
    _check(_lib().hb_release_cache())


def graph_load(offsets, degrees, data, comp_size=None, n_edges=None, order=None,
               hash_ids=None, xy=None) -> Graph:
    """hb_graph_load.  order: processing order of the nodes (a permutation; changes no
    result); hash_ids: element inserted for each node (its id before a renumbering);
    xy: (n, 2) cell coordinates, for the point second moment."""
    return Graph(offsets, degrees, data, comp_size, n_edges, order, hash_ids, xy)


def run(g: Graph, p: int, depth_limit: int = 0, seed: int = 0, registers: bool = False,
        kernel: str = "auto", table_levels: int = 0, tune: str = "cached",
        lanes_per_node: int = 0, nodes_per_block: int = 0) -> Result:
    return g.run(p, depth_limit, seed, registers, kernel=kernel, table_levels=table_levels,
                 tune=tune, lanes_per_node=lanes_per_node, nodes_per_block=nodes_per_block)
