"""CPU oracle for HyperBall over a LEB128 delta-compressed CSR (ctypes wrapper).

TEST INFRASTRUCTURE ONLY: the plain, slow reference the GPU library is checked
against.  Only the test suite, the smoke check and the benchmark's CPU-baseline leg
import this package.  It shares no code with the GPU library; see ``hb_oracle.c``
for what each function follows in the paper (Sec. 2.3, Sec. 3.2, Sec. 3.3, Eq. 1-3,
Alg. 1) and the readings taken where the paper is silent.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

C_FLAGS = ["-O3", "-march=x86-64-v3", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
           "-shared", "-fPIC", "-std=c11"]


def lib_path() -> str:
    return os.path.join(_HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    """Compile hb_oracle.c into liboracle.so with gcc."""
    out = lib_path()
    cmd = ["gcc", *C_FLAGS, "-o", out + ".tmp", os.path.join(_HERE, "hb_oracle.c"), "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


class _Info(ctypes.Structure):
    _fields_ = [("passes", ctypes.c_uint32), ("converged", ctypes.c_uint32),
                ("max_delta", ctypes.c_double)]


def _lib():
    global _LIB
    if _LIB is None:
        path = lib_path()
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(path)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        i32p = ctypes.POINTER(ctypes.c_int32)
        i64p = ctypes.POINTER(ctypes.c_int64)
        dp = ctypes.POINTER(ctypes.c_double)
        i64, u64, i32, u32 = ctypes.c_int64, ctypes.c_uint64, ctypes.c_int32, ctypes.c_uint32
        L.or_uleb_encode.argtypes = [u64, u8p]
        L.or_uleb_encode.restype = ctypes.c_int
        L.or_uleb_decode.argtypes = [u8p, u8p, u64p]
        L.or_uleb_decode.restype = ctypes.c_int
        L.or_csr_layout.argtypes = [i64, u64p, u32p, u64p, u32p]
        L.or_csr_layout.restype = u64
        L.or_csr_encode.argtypes = [i64, u64p, u32p, u64p, u8p]
        L.or_csr_encode.restype = None
        L.or_decode_row.argtypes = [u8p, u64p, i64, u32p, i64]
        L.or_decode_row.restype = i64
        L.or_splitmix64.argtypes = [u64]
        L.or_splitmix64.restype = u64
        L.or_hll_insert.argtypes = [u64, u64, ctypes.c_int, u32p, u32p]
        L.or_hll_insert.restype = None
        L.or_hll_alpha.argtypes = [ctypes.c_int]
        L.or_hll_alpha.restype = ctypes.c_double
        L.or_hll_raw.argtypes = [u8p, ctypes.c_int, u32p]
        L.or_hll_raw.restype = ctypes.c_double
        L.or_hll_estimate.argtypes = [u8p, ctypes.c_int]
        L.or_hll_estimate.restype = ctypes.c_double
        L.or_hyperball.argtypes = [i64, u64p, u32p, u8p, ctypes.c_int, u32, u64, u32p, ctypes.c_int,
                                   u8p, dp, dp,
                                   ctypes.POINTER(_Info)]
        L.or_hyperball.restype = ctypes.c_int
        L.or_vga_metrics.argtypes = [i64, u64p, u32p, u8p, u32p, dp, dp]
        L.or_vga_metrics.restype = ctypes.c_int
        L.or_point_second_moment.argtypes = [i64, u64p, u32p, u8p, ctypes.POINTER(ctypes.c_int32),
                                             dp]
        L.or_point_second_moment.restype = ctypes.c_int
        L.or_local_metrics.argtypes = [i64, u64p, u32p, u8p, u32p, i64, u64p, u32p, dp, dp]
        L.or_local_metrics.restype = ctypes.c_int
        L.or_hyperball_exact.argtypes = [i64, u64p, u32p, u8p, u32, dp, dp, ctypes.POINTER(_Info)]
        L.or_hyperball_exact.restype = ctypes.c_int
        L.or_bfs.argtypes = [i64, u64p, u32p, u8p, i64, i32p]
        L.or_bfs.restype = ctypes.c_int
        L.or_bfs_all.argtypes = [i64, u64p, u32p, u8p, i32p]
        L.or_bfs_all.restype = ctypes.c_int
        L.or_ball_registers.argtypes = [i64, i32p, i32, ctypes.c_int, u64, u8p]
        L.or_ball_registers.restype = None
        L.or_msbfs_balls.argtypes = [i64, u64p, u32p, u8p, i64p, i32, i32, ctypes.c_int, u64, u8p,
                                     u64p]
        L.or_msbfs_balls.restype = ctypes.c_int
        L.or_union_sample.argtypes = [i64, u64p, u32p, u8p, ctypes.c_int, u8p, i64p, i64, u8p, dp]
        L.or_union_sample.restype = i64
        L.or_num_threads.argtypes = []
        L.or_num_threads.restype = ctypes.c_int
        L.or_set_num_threads.argtypes = [ctypes.c_int]
        L.or_set_num_threads.restype = None
        _LIB = L
    return _LIB


def _p(a: np.ndarray, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _u8(a):
    return _p(a, ctypes.c_uint8)


def _u32(a):
    return _p(a, ctypes.c_uint32)


def _u64(a):
    return _p(a, ctypes.c_uint64)


def set_num_threads(k: int) -> None:
    """Threads of the oracle's parallel loops from now on (results do not depend on it)."""
    _lib().or_set_num_threads(int(k))


def num_threads() -> int:
    return int(_lib().or_num_threads())


# ------------------------------------------------------------------ LEB128
def uleb_encode(v: int) -> bytes:
    buf = (ctypes.c_uint8 * 16)()
    k = _lib().or_uleb_encode(int(v), buf)
    return bytes(buf[:k])


def uleb_decode(b: bytes):
    """(value, bytes used); used 0 = truncated, -1 = overlong/overflow."""
    arr = np.frombuffer(bytes(b) + b"\0", np.uint8).copy()
    v = ctypes.c_uint64(0)
    base = _u8(arr)
    end = ctypes.cast(ctypes.addressof(base.contents) + len(b), ctypes.POINTER(ctypes.c_uint8))
    used = _lib().or_uleb_decode(base, end, ctypes.byref(v))
    return int(v.value), int(used)


@dataclass
class CSR:
    """Compressed CSR (Sec. 3.2): u64 byte offsets, u32 degrees, LEB128 byte stream."""

    n: int
    offsets: np.ndarray
    degrees: np.ndarray
    bytes: np.ndarray

    @property
    def n_edges(self) -> int:
        return int(self.degrees.sum(dtype=np.uint64))


def csr_encode(n: int, adj_offsets: np.ndarray, adj_ids: np.ndarray) -> CSR:
    adj_offsets = np.ascontiguousarray(adj_offsets, np.uint64)
    adj_ids = np.ascontiguousarray(adj_ids, np.uint32)
    offsets = np.zeros(n + 1, np.uint64)
    degrees = np.zeros(n, np.uint32)
    L = _lib()
    total = L.or_csr_layout(n, _u64(adj_offsets), _u32(adj_ids), _u64(offsets), _u32(degrees))
    data = np.zeros(max(1, int(total)), np.uint8)
    L.or_csr_encode(n, _u64(adj_offsets), _u32(adj_ids), _u64(offsets), _u8(data))
    return CSR(n=n, offsets=offsets, degrees=degrees, bytes=data[:int(total)] if total else data[:0])


def _bytes_ptr(csr: CSR):
    # a non-empty buffer so the pointer is valid even for edge-free graphs
    if csr.bytes.size == 0:
        csr._pad = np.zeros(1, np.uint8)
        return _u8(csr._pad)
    return _u8(csr.bytes)


def decode_row(csr: CSR, v: int) -> np.ndarray:
    ids = np.zeros(max(1, int(csr.degrees[v]) + 1), np.uint32)
    k = _lib().or_decode_row(_bytes_ptr(csr), _u64(csr.offsets), v, _u32(ids), ids.shape[0])
    if k < 0:
        raise ValueError(f"malformed row {v}")
    return ids[:k]


def from_graph(g) -> CSR:
    """Encode a ``synth.Graph`` with the oracle's encoder."""
    return csr_encode(g.n, g.adj_offsets, g.adj_ids)


# ------------------------------------------------------------------ hash / HLL
def splitmix64(x: int) -> int:
    return int(_lib().or_splitmix64(int(x) & 0xFFFFFFFFFFFFFFFF))


def hll_insert(v: int, seed: int, p: int):
    j, r = ctypes.c_uint32(), ctypes.c_uint32()
    _lib().or_hll_insert(int(v), int(seed), p, ctypes.byref(j), ctypes.byref(r))
    return int(j.value), int(r.value)


def hll_alpha(p: int) -> float:
    return float(_lib().or_hll_alpha(p))


def hll_raw(regs: np.ndarray, p: int):
    regs = np.ascontiguousarray(regs, np.uint8)
    z = ctypes.c_uint32()
    e = _lib().or_hll_raw(_u8(regs), p, ctypes.byref(z))
    return float(e), int(z.value)


def hll_estimate(regs: np.ndarray, p: int) -> float:
    regs = np.ascontiguousarray(regs, np.uint8)
    assert regs.shape[-1] == 1 << p
    return float(_lib().or_hll_estimate(_u8(regs), p))


def hll_estimates(regs: np.ndarray, p: int) -> np.ndarray:
    regs = np.ascontiguousarray(regs, np.uint8).reshape(-1, 1 << p)
    return np.array([hll_estimate(r, p) for r in regs])


# ------------------------------------------------------------------ HyperBall
@dataclass
class HBResult:
    registers: np.ndarray | None  # u8[n, m]
    reach: np.ndarray  # f64[n]
    sum_d: np.ndarray  # f64[n]
    passes: int
    converged: bool
    max_delta: float


def hyperball(csr: CSR, p: int, depth_limit: int = 0, seed: int = 0,
              registers: bool = True, hash_ids=None, register_bits: int = 8) -> HBResult:
    """Alg. 1 (Eq. 2 union, HLL estimate, Eq. 3 accumulation, 0.5 stopping rule).

    hash_ids (n, optional): the element inserted for node v instead of v.
    register_bits: 8, or 4 for registers that saturate at 15 (returned one per byte).
    """
    if register_bits not in (8, 4):
        raise ValueError("register_bits must be 8 or 4")
    n, m = csr.n, 1 << p
    hid = None if hash_ids is None else np.ascontiguousarray(hash_ids, np.uint32)
    if hid is not None and hid.shape != (n,):
        raise ValueError("hash_ids must have n entries")
    regs = np.zeros((n, m), np.uint8) if registers else None
    reach = np.zeros(n, np.float64)
    sum_d = np.zeros(n, np.float64)
    info = _Info()
    rc = _lib().or_hyperball(n, _u64(csr.offsets), _u32(csr.degrees), _bytes_ptr(csr), p,
                             depth_limit, seed & 0xFFFFFFFFFFFFFFFF,
                             _u32(hid) if hid is not None else None, register_bits,
                             _u8(regs) if registers else None,
                             _p(reach, ctypes.c_double), _p(sum_d, ctypes.c_double),
                             ctypes.byref(info))
    if rc != 0:
        raise RuntimeError("oracle hyperball failed (malformed CSR or out of memory)")
    return HBResult(regs, reach, sum_d, int(info.passes), bool(info.converged),
                    float(info.max_delta))


def hyperball_exact(csr: CSR, depth_limit: int = 0) -> HBResult:
    """The same iteration over exact sets (bitsets, popcount): small graphs only."""
    n = csr.n
    card = np.zeros(n, np.float64)
    sum_d = np.zeros(n, np.float64)
    info = _Info()
    rc = _lib().or_hyperball_exact(n, _u64(csr.offsets), _u32(csr.degrees), _bytes_ptr(csr),
                                   depth_limit, _p(card, ctypes.c_double),
                                   _p(sum_d, ctypes.c_double), ctypes.byref(info))
    if rc != 0:
        raise RuntimeError("oracle exact hyperball failed")
    return HBResult(None, card, sum_d, int(info.passes), bool(info.converged),
                    float(info.max_delta))


# ------------------------------------------------------------------ exact BFS
def bfs(csr: CSR, src: int) -> np.ndarray:
    dist = np.empty(csr.n, np.int32)
    if _lib().or_bfs(csr.n, _u64(csr.offsets), _u32(csr.degrees), _bytes_ptr(csr), src,
                     _p(dist, ctypes.c_int32)) != 0:
        raise RuntimeError("oracle bfs failed")
    return dist


def bfs_all(csr: CSR) -> np.ndarray:
    dist = np.empty((csr.n, csr.n), np.int32)
    if _lib().or_bfs_all(csr.n, _u64(csr.offsets), _u32(csr.degrees), _bytes_ptr(csr),
                         _p(dist, ctypes.c_int32)) != 0:
        raise RuntimeError("oracle bfs failed")
    return dist


def ball_registers(dist_row: np.ndarray, t: int, p: int, seed: int = 0) -> np.ndarray:
    dist_row = np.ascontiguousarray(dist_row, np.int32)
    regs = np.zeros(1 << p, np.uint8)
    _lib().or_ball_registers(dist_row.shape[0], _p(dist_row, ctypes.c_int32), t, p,
                             seed & 0xFFFFFFFFFFFFFFFF, _u8(regs))
    return regs


def msbfs_balls(csr: CSR, sources, T: int, p: int, seed: int = 0):
    """Exact balls of up to 64 sources per call, levels 0..T.

    Returns (regs u8[ns, T+1, m], ball sizes u64[ns, T+1]).
    """
    src = np.ascontiguousarray(np.asarray(sources, np.int64))
    ns, m = src.shape[0], 1 << p
    regs = np.zeros((ns, T + 1, m), np.uint8)
    balls = np.zeros((ns, T + 1), np.uint64)
    for k0 in range(0, ns, 64):
        chunk = np.ascontiguousarray(src[k0:k0 + 64])
        r = np.zeros((chunk.shape[0], T + 1, m), np.uint8)
        b = np.zeros((chunk.shape[0], T + 1), np.uint64)
        rc = _lib().or_msbfs_balls(csr.n, _u64(csr.offsets), _u32(csr.degrees), _bytes_ptr(csr),
                                   _p(chunk, ctypes.c_int64), chunk.shape[0], T, p,
                                   seed & 0xFFFFFFFFFFFFFFFF, _u8(r), _u64(b))
        if rc != 0:
            raise RuntimeError("oracle msbfs failed")
        regs[k0:k0 + 64] = r
        balls[k0:k0 + 64] = b
    return regs, balls


def sampled_hyperball(csr: CSR, sources, T: int, p: int, seed: int = 0):
    """Per-source HyperBall outputs after T steps, from exact balls.

    Because the step-t registers of v equal the registers of the exact ball
    B(v, t), the oracle can produce any single node's registers, estimates and
    Eq. 3 sum without running the whole graph.  Returns (regs u8[ns, m] at step T,
    reach f64[ns], sum_d f64[ns], est f64[ns, T+1]).
    """
    regs, _ = msbfs_balls(csr, sources, T, p, seed)
    ns = regs.shape[0]
    est = np.array([[hll_estimate(regs[k, t], p) for t in range(T + 1)] for k in range(ns)])
    sum_d = np.zeros(ns)
    for t in range(1, T + 1):
        sum_d = sum_d + float(t) * (est[:, t] - est[:, t - 1])
    return regs[:, T], est[:, T], sum_d, est


def union_sample(csr: CSR, p: int, cur: np.ndarray, nodes: np.ndarray):
    """One Eq. 2 union + estimate for the listed nodes (the CPU-baseline unit)."""
    nodes = np.ascontiguousarray(nodes, np.int64)
    m = 1 << p
    nxt = np.zeros((nodes.shape[0], m), np.uint8)
    est = np.zeros(nodes.shape[0], np.float64)
    e = _lib().or_union_sample(csr.n, _u64(csr.offsets), _u32(csr.degrees), _bytes_ptr(csr), p,
                               _u8(cur), _p(nodes, ctypes.c_int64), nodes.shape[0], _u8(nxt),
                               _p(est, ctypes.c_double))
    if e < 0:
        raise RuntimeError("oracle union_sample failed")
    return nxt, est, int(e)


def initial_registers(n: int, p: int, seed: int = 0) -> np.ndarray:
    """Registers after inserting every node into its own counter."""
    m = 1 << p
    regs = np.zeros((n, m), np.uint8)
    for v in range(n):
        j, r = hll_insert(v, seed, p)
        regs[v, j] = r
    return regs


VGA_METRICS = ("connectivity", "control", "mean_depth", "relative_asymmetry", "integration_hh",
               "integration_tekl", "integration_pvalue", "point_first_moment")


def vga_metrics(csr: CSR, sum_d, comp_size=None) -> dict:
    """VGA metrics from the 1-hop neighbourhood and the Eq. 3 sums (Sec. 3.3)."""
    n = csr.n
    sd = np.ascontiguousarray(sum_d, np.float64)
    cs = None if comp_size is None else np.ascontiguousarray(comp_size, np.uint32)
    out = np.empty((8, n), np.float64)
    rc = _lib().or_vga_metrics(n, _u64(csr.offsets), _u32(csr.degrees), _bytes_ptr(csr),
                               _u32(cs) if cs is not None else None,
                               _p(sd, ctypes.c_double), _p(out, ctypes.c_double))
    if rc != 0:
        raise RuntimeError("oracle vga_metrics failed (malformed CSR)")
    return {name: out[i] for i, name in enumerate(VGA_METRICS)}


def point_second_moment(csr: CSR, xy) -> np.ndarray:
    """Point second moment of every node (Sec. 3.3): the sum over its neighbours of the
    squared distance between cell centres, squared cell units; xy: (n, 2) cells."""
    xy = np.ascontiguousarray(xy, np.int32)
    if xy.shape != (csr.n, 2):
        raise ValueError("xy must have shape (n, 2)")
    out = np.empty(csr.n, np.float64)
    rc = _lib().or_point_second_moment(csr.n, _u64(csr.offsets), _u32(csr.degrees),
                                       _bytes_ptr(csr), _p(xy, ctypes.c_int32),
                                       _p(out, ctypes.c_double))
    if rc != 0:
        raise RuntimeError("oracle point_second_moment failed (malformed CSR)")
    return out


def local_metrics(csr: CSR, nodes=None) -> dict:
    """Exact local metrics of the listed nodes (all when nodes is None), Sec. 3.3
    "Metric derivation": ordered adjacent neighbour pairs, two-step ball size
    (without v), clustering coefficient and controllability."""
    count = csr.n if nodes is None else len(nodes)
    nd = None if nodes is None else np.ascontiguousarray(nodes, np.uint32)
    pairs = np.empty(count, np.uint64)
    ball2 = np.empty(count, np.uint32)
    clus = np.empty(count, np.float64)
    ctrl = np.empty(count, np.float64)
    rc = _lib().or_local_metrics(csr.n, _u64(csr.offsets), _u32(csr.degrees), _bytes_ptr(csr),
                                 _u32(nd) if nd is not None else None, count, _u64(pairs),
                                 _u32(ball2), _p(clus, ctypes.c_double), _p(ctrl, ctypes.c_double))
    if rc != 0:
        raise RuntimeError("oracle local_metrics failed (malformed CSR)")
    return {"pairs": pairs, "ball2": ball2, "clustering": clus, "controllability": ctrl}
