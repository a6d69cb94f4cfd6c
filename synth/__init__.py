"""Seeded synthetic visibility graphs: the inputs shared by the oracle and the HIP path.

The paper's inputs (OpenStreetMap footprints of Valdivia, sparkSieve2 edge sets,
Sec. 3.1 and Sec. 4.1) are not available, so seeded obstacle rasters stand in for
them.  This module draws the rasters (numpy PCG64 streams, unrelated to the
method's SplitMix64 hash), keeps the main connected component, numbers its cells
in raster order and builds the sorted adjacency lists with an exact integer
visibility rule (``synth.c``; a GPU twin in ``synth_gpu.hip`` serves the largest
rasters).  It holds none of the method's arithmetic: no hashing, no registers, no
estimator and no LEB128 coding.  A graph leaves this module as plain arrays:
``adj_offsets`` (u64, n+1) and ``adj_ids`` (u32, sorted ascending per row).

Workload recipes (sizes are those of the paper's T2/T3 rows this build measures):

* ``tiny(seed)``: 32x32 grid of 1 m cells, axis-aligned rectangles with sides 3-8
  cells at uniform positions until >= 30 % of cells are covered.
* ``urban(seed)``: 230x230 cells of 3 m, perturbed street grid (streets 8-20 m
  wide, 40-90 m blocks with ragged edges) with rectangular buildings of 10-40 m
  sides filling 20 % of each block; about 42,700 nodes and 1.4e8 directed edges
  (the paper's T2 row: 42,705 cells, 161M edges).
* ``city(seed)``: the same seeded layout drawn CITY_SCALE = 2.35 times finer on a
  541x541 raster: about 236,000 nodes and 4.7e9 directed edges (the paper's
  largest T2 row: 235,983 cells, 4.8e9 edges).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None
_GPU_LIB = None

# Street/building generator parameters in metres, calibrated once on the urban
# configuration (nodes and directed edges of the paper's 42,705-cell T2 row) and
# then frozen.  The city configuration draws the same seeded layout at a spacing
# CITY_SCALE times finer, as the paper's T2 rows at 7 m and 3 m spacing cover one
# study area.
URBAN = dict(
    street_m=(8, 20),
    block_m=(40, 90),
    bldg_m=(10, 40),
    block_fill=0.20,
    jitter_m=2,
)
URBAN_EXTENT = (230, 230)
URBAN_CELL_M = 3.0
CITY_SCALE = 2.35
CITY_EXTENT = (541, 541)


C_FLAGS = ["-O3", "-march=x86-64-v3", "-fopenmp", "-shared", "-fPIC", "-std=c11"]


def lib_path() -> str:
    return os.path.join(_HERE, "libsynth.so")


def build(verbose: bool = False) -> None:
    """Compile synth.c (gcc) and synth_gpu.hip (hipcc, gfx950) in place."""
    import subprocess
    out = lib_path()
    cmd = ["gcc", *C_FLAGS, "-o", out + ".tmp", os.path.join(_HERE, "synth.c")]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    gout = gpu_lib_path()
    hip_src = os.path.join(_HERE, "synth_gpu.hip")
    if os.path.exists(hip_src):
        cmd = ["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
               "-shared", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-o", gout + ".tmp", hip_src]
        if verbose:
            print(" ".join(cmd), flush=True)
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            raise RuntimeError("hipcc failed for synth_gpu.hip:\n" + res.stderr)
        os.replace(gout + ".tmp", gout)


def gpu_lib_path() -> str:
    return os.path.join(_HERE, "libsynth_gpu.so")


def _lib():
    global _LIB
    if _LIB is None:
        path = lib_path()
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(path)
        c_u8p = ctypes.POINTER(ctypes.c_uint8)
        c_i32p = ctypes.POINTER(ctypes.c_int32)
        c_i64p = ctypes.POINTER(ctypes.c_int64)
        c_u64p = ctypes.POINTER(ctypes.c_uint64)
        c_u32p = ctypes.POINTER(ctypes.c_uint32)
        i32, i64 = ctypes.c_int32, ctypes.c_int64
        L.syn_visible.argtypes = [c_u8p, i32, i32, i32, i32, i32, i32]
        L.syn_visible.restype = ctypes.c_int
        L.syn_main_component.argtypes = [c_u8p, i32, i32, c_i32p]
        L.syn_main_component.restype = i64
        L.syn_degrees.argtypes = [c_u8p, i32, i32, c_i32p, i64, c_u64p]
        L.syn_degrees.restype = None
        L.syn_fill.argtypes = [c_u8p, i32, i32, c_i32p, i64, c_u64p, c_u32p]
        L.syn_fill.restype = None
        L.syn_degrees_sample.argtypes = [c_u8p, i32, i32, c_i32p, i64, c_i64p, i64, c_u64p]
        L.syn_degrees_sample.restype = None
        L.syn_visible_pairs.argtypes = [c_u8p, i32, i32, c_i32p, c_i64p, c_i64p, i64, c_u8p]
        L.syn_visible_pairs.restype = None
        L.syn_raster_bits.argtypes = [c_u8p, i32, i32, c_u32p]
        L.syn_raster_bits.restype = None
        L.syn_row_degrees.argtypes = [c_u32p, i64, i64, c_u64p]
        L.syn_row_degrees.restype = None
        L.syn_row_ids.argtypes = [c_u32p, i64, i64, c_u64p, c_u32p]
        L.syn_row_ids.restype = None
        L.syn_num_threads.argtypes = []
        L.syn_num_threads.restype = ctypes.c_int
        _LIB = L
    return _LIB


def _p(a: np.ndarray, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


@dataclass
class Graph:
    """A visibility graph over the main component of an obstacle raster."""

    n: int
    adj_offsets: np.ndarray  # u64[n+1]
    adj_ids: np.ndarray  # u32[adj_offsets[n]], ascending per row
    obst: np.ndarray  # u8[H, W], 1 = obstacle
    xy: np.ndarray  # i32[n, 2], (x, y) cell of each node
    name: str = ""
    params: dict = field(default_factory=dict)

    @property
    def n_edges(self) -> int:
        return int(self.adj_offsets[-1])

    @property
    def degrees(self) -> np.ndarray:
        return np.diff(self.adj_offsets).astype(np.uint32)

    def row(self, v: int) -> np.ndarray:
        return self.adj_ids[self.adj_offsets[v]: self.adj_offsets[v + 1]]


# ---------------------------------------------------------------- rasters
def _rng(seed: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64([int(seed), int(stream)]))


def tiny_raster(seed: int, W: int = 32, H: int = 32, cover: float = 0.30,
                side=(3, 8)) -> np.ndarray:
    """Rectangles with integer sides in [side] at uniform positions until cover is reached."""
    rng = _rng(seed, 1)
    obst = np.zeros((H, W), np.uint8)
    while obst.mean() < cover:
        w = int(rng.integers(side[0], side[1] + 1))
        h = int(rng.integers(side[0], side[1] + 1))
        x = int(rng.integers(0, W - w + 1))
        y = int(rng.integers(0, H - h + 1))
        obst[y:y + h, x:x + w] = 1
    return obst


def _cuts(rng, length: int, street, block, cell_m: float):
    """Alternating street / block spans along one axis, in cells: list of (b0, b1) blocks."""
    blocks = []
    pos = -int(rng.integers(0, max(1, round(block[1] / cell_m))))
    while pos < length:
        ws = max(1, round(rng.integers(street[0], street[1] + 1) / cell_m))
        wb = max(1, round(rng.integers(block[0], block[1] + 1) / cell_m))
        b0, b1 = pos + ws, pos + ws + wb
        if b1 > 0 and b0 < length:
            blocks.append((max(0, b0), min(length, b1)))
        pos = b1
    return blocks


def urban_raster(seed: int, W: int, H: int, cell_m: float = 1.0, street_m=(8, 20),
                 block_m=(40, 90), bldg_m=(10, 40), block_fill=0.20, jitter_m=2) -> np.ndarray:
    """Perturbed street grid with rectangular buildings inside the blocks.

    Streets run the full extent along both axes with widths drawn from street_m;
    each block edge is jittered by up to jitter_m so street walls are ragged; inside
    every block, rectangles with sides drawn from bldg_m are dropped at uniform
    positions until the block's built fraction reaches block_fill.
    """
    rng = _rng(seed, 2)
    obst = np.zeros((H, W), np.uint8)
    xs = _cuts(rng, W, street_m, block_m, cell_m)
    ys = _cuts(rng, H, street_m, block_m, cell_m)
    jit = max(0, round(jitter_m / cell_m))
    lo_b, hi_b = max(1, round(bldg_m[0] / cell_m)), max(1, round(bldg_m[1] / cell_m))
    for (y0, y1) in ys:
        for (x0, x1) in xs:
            if jit:
                bx0 = x0 + int(rng.integers(-jit, jit + 1))
                bx1 = x1 + int(rng.integers(-jit, jit + 1))
                by0 = y0 + int(rng.integers(-jit, jit + 1))
                by1 = y1 + int(rng.integers(-jit, jit + 1))
            else:
                bx0, bx1, by0, by1 = x0, x1, y0, y1
            bx0, by0 = max(0, bx0), max(0, by0)
            bx1, by1 = min(W, bx1), min(H, by1)
            bw, bh = bx1 - bx0, by1 - by0
            if bw < 2 or bh < 2:
                continue
            blk = np.zeros((bh, bw), np.uint8)
            tries = 0
            while blk.mean() < block_fill and tries < 200:
                tries += 1
                w = min(bw, int(rng.integers(lo_b, hi_b + 1)))
                h = min(bh, int(rng.integers(lo_b, hi_b + 1)))
                x = int(rng.integers(0, bw - w + 1))
                y = int(rng.integers(0, bh - h + 1))
                blk[y:y + h, x:x + w] = 1
            obst[by0:by1, bx0:bx1] |= blk
    return obst


# ---------------------------------------------------------------- graphs
def component(obst: np.ndarray):
    """Main 4-connected open component: (node_of_cell[H, W] int32 with -1 elsewhere, xy)."""
    obst = np.ascontiguousarray(obst, dtype=np.uint8)
    H, W = obst.shape
    node_of_cell = np.empty((H, W), np.int32)
    n = _lib().syn_main_component(_p(obst, ctypes.c_uint8), W, H, _p(node_of_cell, ctypes.c_int32))
    if n < 0:
        raise MemoryError("syn_main_component failed")
    ys, xs = np.nonzero(node_of_cell >= 0)  # row-major order == raster order
    xy = np.ascontiguousarray(np.stack([xs, ys], axis=1).astype(np.int32))
    assert xy.shape[0] == n
    return node_of_cell, xy


def graph_from_raster(obst: np.ndarray, name: str = "", params: dict | None = None,
                      device: str = "cpu") -> Graph:
    """Visibility graph of the raster's main component (CPU or GPU generator)."""
    obst = np.ascontiguousarray(obst, dtype=np.uint8)
    H, W = obst.shape
    _, xy = component(obst)
    n = xy.shape[0]
    if device == "gpu":
        off, ids = _gpu_adjacency(obst, xy)
    else:
        L = _lib()
        deg = np.empty(n, np.uint64)
        L.syn_degrees(_p(obst, ctypes.c_uint8), W, H, _p(xy, ctypes.c_int32), n,
                      _p(deg, ctypes.c_uint64))
        off = np.zeros(n + 1, np.uint64)
        np.cumsum(deg, out=off[1:])
        ids = np.empty(int(off[-1]), np.uint32)
        L.syn_fill(_p(obst, ctypes.c_uint8), W, H, _p(xy, ctypes.c_int32), n,
                   _p(off, ctypes.c_uint64), _p(ids, ctypes.c_uint32))
    return Graph(n=n, adj_offsets=off, adj_ids=ids, obst=obst, xy=xy, name=name,
                 params=dict(params or {}))


def visible_pairs(g: Graph, a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """CPU visibility rule on explicit node pairs (u8 0/1)."""
    a = np.ascontiguousarray(a, np.int64)
    b = np.ascontiguousarray(b, np.int64)
    out = np.empty(a.shape[0], np.uint8)
    H, W = g.obst.shape
    _lib().syn_visible_pairs(_p(g.obst, ctypes.c_uint8), W, H, _p(g.xy, ctypes.c_int32),
                             _p(a, ctypes.c_int64), _p(b, ctypes.c_int64), a.shape[0],
                             _p(out, ctypes.c_uint8))
    return out


def sample_degrees(obst: np.ndarray, n_src: int, seed: int = 0):
    """(n, sampled degrees) of n_src seeded source nodes; for estimating E on big rasters."""
    obst = np.ascontiguousarray(obst, dtype=np.uint8)
    H, W = obst.shape
    _, xy = component(obst)
    n = xy.shape[0]
    src = np.sort(_rng(seed, 9).choice(n, size=min(n, n_src), replace=False)).astype(np.int64)
    deg = np.empty(src.shape[0], np.uint64)
    _lib().syn_degrees_sample(_p(obst, ctypes.c_uint8), W, H, _p(xy, ctypes.c_int32), n,
                              _p(src, ctypes.c_int64), src.shape[0], _p(deg, ctypes.c_uint64))
    return n, deg


# ---------------------------------------------------------------- named workloads
def tiny(seed: int = 0) -> Graph:
    """32x32 tiny VGA graph (1 m cells, 3-8 m rectangles, >= 30 % cover)."""
    return graph_from_raster(tiny_raster(seed), name=f"tiny32-s{seed}",
                             params=dict(kind="tiny", seed=seed, W=32, H=32))


def grid_graph(seed: int, W: int, H: int, cover: float = 0.30, side=(3, 8)) -> Graph:
    """Tiny-style rectangles on a W x H raster (parity cases between tiny and urban)."""
    return graph_from_raster(tiny_raster(seed, W, H, cover, side), name=f"rect{W}x{H}-s{seed}",
                             params=dict(kind="rect", seed=seed, W=W, H=H, cover=cover))


def urban(seed: int = 0, device: str = "cpu") -> Graph:
    """230x230 urban block graph (~42,700 nodes, ~1.4e8 directed edges)."""
    W, H = URBAN_EXTENT
    obst = urban_raster(seed, W, H, cell_m=URBAN_CELL_M, **URBAN)
    return graph_from_raster(obst, name=f"urban230-s{seed}", device=device,
                             params=dict(kind="urban", seed=seed, W=W, H=H, cell_m=URBAN_CELL_M,
                                         **URBAN))


def city_raster(seed: int = 0) -> np.ndarray:
    W, H = CITY_EXTENT
    return urban_raster(seed, W, H, cell_m=URBAN_CELL_M / CITY_SCALE, **URBAN)


def city(seed: int = 0, device: str = "gpu") -> Graph:
    """541x541 city-scale graph (~236,000 nodes, ~4.7e9 directed edges)."""
    W, H = CITY_EXTENT
    return graph_from_raster(city_raster(seed), name=f"city541-s{seed}", device=device,
                             params=dict(kind="city", seed=seed, W=W, H=H, scale=CITY_SCALE,
                                         **URBAN))


def batch_spec(seed: int, n_lo: int = 500, n_hi: int = 20000, ps=(8, 10, 12),
               depths=(2, 3, 5, 0)) -> dict:
    """Seeded analysis of the batched workload: target size, cell size, p and depth.

    Sizes are log-uniform in [n_lo, n_hi] open cells; cells are 1 or 2 m (the
    street/building generator's lengths are divided by the cell size); the raster
    is square with about n / 0.8 cells (the generator leaves ~80 % of cells open).
    """
    rng = _rng(seed, 7)
    n_target = float(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi))))
    cell_m = float(rng.choice([1.0, 2.0]))
    side = max(8, int(round(np.sqrt(n_target / 0.8))))
    return dict(seed=seed, n_target=n_target, cell_m=cell_m, side=side,
                p=int(rng.choice(ps)), depth=int(rng.choice(depths)))


def batch_graph(seed: int, device: str = "gpu", **kw) -> Graph:
    """One graph of the batched workload (see batch_spec)."""
    spec = batch_spec(seed, **kw)
    obst = urban_raster(seed, spec["side"], spec["side"], cell_m=spec["cell_m"], **URBAN)
    return graph_from_raster(obst, name=f"batch{spec['side']}-s{seed}", device=device,
                             params=dict(kind="batch", **spec))


def serve_graph(seed: int, n_lo: int = 1000, n_hi: int = 120000, device: str = "gpu") -> Graph:
    """One graph of the served workload's pool: the urban generator (3 m cells) on a
    square raster sized for a log-uniform target of n_lo..n_hi open cells."""
    rng = _rng(seed, 11)
    n_target = float(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi))))
    side = max(8, int(round(np.sqrt(n_target / 0.807))))
    obst = urban_raster(seed, side, side, cell_m=URBAN_CELL_M, **URBAN)
    return graph_from_raster(obst, name=f"pool{side}-s{seed}", device=device,
                             params=dict(kind="serve", seed=seed, side=side, n_target=n_target,
                                         cell_m=URBAN_CELL_M))


# ---------------------------------------------------------------- special graphs
# ---------------------------------------------------------------- locality orders
def hilbert_index(x: np.ndarray, y: np.ndarray, bits: int) -> np.ndarray:
    """Position of cell (x, y) along a Hilbert curve over a 2^bits x 2^bits grid.

    The curve is built by quadrant recursion: at each scale s (from the largest),
    the quadrant (rx, ry) adds s^2 (3 rx XOR ry), and the remaining coordinates are
    reflected and transposed so that the sub-curve in that quadrant joins its
    neighbours end to end.  Consecutive positions are 4-adjacent cells.
    """
    x = np.asarray(x, np.int64).copy()
    y = np.asarray(y, np.int64).copy()
    d = np.zeros_like(x)
    s = 1 << (bits - 1)
    while s > 0:
        rx = (x & s) > 0
        ry = (y & s) > 0
        d += s * s * ((3 * rx.astype(np.int64)) ^ ry.astype(np.int64))
        low = ~ry
        flip = low & rx
        x[flip] = s - 1 - x[flip]
        y[flip] = s - 1 - y[flip]
        x[low], y[low] = y[low].copy(), x[low].copy()
        s >>= 1
    return d


def hilbert_order(g: "Graph") -> np.ndarray:
    """Node ids sorted along a Hilbert curve over the raster (a processing order)."""
    side = max(int(g.xy[:, 0].max(initial=0)), int(g.xy[:, 1].max(initial=0))) + 1
    bits = max(1, int(np.ceil(np.log2(side))))
    d = hilbert_index(g.xy[:, 0], g.xy[:, 1], bits)
    return np.argsort(d, kind="stable").astype(np.uint32)


def relabel(g: "Graph", order: np.ndarray) -> tuple:
    """Renumber the nodes so that new node i is old node order[i].

    Returns (graph, original_ids): the CSR is rebuilt in the new numbering (each
    row re-sorted), and original_ids[i] = order[i] is what node i inserts into its
    counter so that the results match the original numbering.
    """
    order = np.asarray(order, np.int64)
    new_of = np.empty(g.n, np.int64)
    new_of[order] = np.arange(g.n)
    deg = g.degrees[order].astype(np.uint64)
    off = np.zeros(g.n + 1, np.uint64)
    off[1:] = np.cumsum(deg)
    ids = np.empty(int(off[-1]), np.uint32)
    for i, v in enumerate(order):
        row = new_of[g.row(int(v))]
        row.sort()
        ids[int(off[i]):int(off[i + 1])] = row
    h = Graph(n=g.n, adj_offsets=off, adj_ids=ids, obst=g.obst, xy=g.xy[order].copy(),
              name=g.name + "-relabelled", params=dict(g.params, relabelled=True))
    return h, order.astype(np.uint32)


def from_edges(n: int, edges, name: str = "") -> Graph:
    """Undirected graph from an edge list (for closed-form cases: paths, stars, cliques)."""
    nbrs = [set() for _ in range(n)]
    for a, b in edges:
        if a != b:
            nbrs[a].add(b)
            nbrs[b].add(a)
    off = np.zeros(n + 1, np.uint64)
    off[1:] = np.cumsum([len(s) for s in nbrs])
    ids = np.array([v for s in nbrs for v in sorted(s)], np.uint32)
    return Graph(n=n, adj_offsets=off, adj_ids=ids, obst=np.zeros((1, 1), np.uint8),
                 xy=np.zeros((n, 2), np.int32), name=name, params=dict(kind="edges"))


def path_graph(n: int) -> Graph:
    return from_edges(n, [(i, i + 1) for i in range(n - 1)], name=f"path{n}")


def cycle_graph(n: int) -> Graph:
    return from_edges(n, [(i, (i + 1) % n) for i in range(n)], name=f"cycle{n}")


def star_graph(n: int) -> Graph:
    return from_edges(n, [(0, i) for i in range(1, n)], name=f"star{n}")


def complete_graph(n: int) -> Graph:
    return from_edges(n, [(i, j) for i in range(n) for j in range(i + 1, n)], name=f"K{n}")


def random_graph(n: int, p_edge: float, seed: int) -> Graph:
    """Seeded G(n, p) graph (may be disconnected, may have isolated nodes)."""
    rng = _rng(seed, 3)
    iu = np.triu_indices(n, 1)
    keep = rng.random(iu[0].shape[0]) < p_edge
    return from_edges(n, list(zip(iu[0][keep].tolist(), iu[1][keep].tolist())),
                      name=f"gnp{n}-{p_edge}-s{seed}")


# ---------------------------------------------------------------- GPU generator
def raster_bits(obst: np.ndarray) -> np.ndarray:
    obst = np.ascontiguousarray(obst, dtype=np.uint8)
    H, W = obst.shape
    bits = np.zeros((W * H + 31) // 32, np.uint32)
    _lib().syn_raster_bits(_p(obst, ctypes.c_uint8), W, H, _p(bits, ctypes.c_uint32))
    return bits


def _gpu_lib():
    global _GPU_LIB
    if _GPU_LIB is None:
        path = gpu_lib_path()
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(path)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        i32p = ctypes.POINTER(ctypes.c_int32)
        i32, u32 = ctypes.c_int32, ctypes.c_uint32
        L.syng_rows.argtypes = [u32p, i32, i32, i32p, u32, u32, u32, u32p]
        L.syng_rows.restype = ctypes.c_int
        L.syng_visible_host.argtypes = [u32p, i32, i32, i32, i32, i32]
        L.syng_visible_host.restype = ctypes.c_int
        L.syng_last_error.argtypes = []
        L.syng_last_error.restype = ctypes.c_char_p
        _GPU_LIB = L
    return _GPU_LIB


def gpu_walk_visible_host(obst: np.ndarray, a, b) -> int:
    """The GPU generator's division-free walk, run on the host (for cross-checks)."""
    bits = raster_bits(obst)
    return int(_gpu_lib().syng_visible_host(_p(bits, ctypes.c_uint32), obst.shape[1],
                                            int(a[0]), int(a[1]), int(b[0]), int(b[1])))


def _gpu_adjacency(obst: np.ndarray, xy: np.ndarray, batch_bytes: int = 1 << 31):
    """Adjacency from GPU-computed visibility bit rows (batched), expanded on the host."""
    L = _gpu_lib()
    H, W = obst.shape
    n = xy.shape[0]
    bits = raster_bits(obst)
    wpr = (n + 31) // 32
    rows = np.empty((n, wpr), np.uint32)
    batch = max(1, min(n, batch_bytes // (4 * wpr)))
    import sys
    import time
    t0 = time.perf_counter()
    for s0 in range(0, n, batch):
        cnt = min(batch, n - s0)
        rc = L.syng_rows(_p(bits, ctypes.c_uint32), W, H, _p(xy, ctypes.c_int32), n, s0, cnt,
                         _p(rows[s0:], ctypes.c_uint32))
        if rc != 0:
            raise RuntimeError("GPU visibility generator: " + L.syng_last_error().decode())
        if n > 20000:
            print(f"[synth] visibility rows {s0 + cnt}/{n} ({time.perf_counter() - t0:.1f}s)",
                  file=sys.stderr, flush=True)
    deg = np.empty(n, np.uint64)
    _lib().syn_row_degrees(_p(rows, ctypes.c_uint32), wpr, n, _p(deg, ctypes.c_uint64))
    off = np.zeros(n + 1, np.uint64)
    np.cumsum(deg, out=off[1:])
    ids = np.empty(int(off[-1]), np.uint32)
    _lib().syn_row_ids(_p(rows, ctypes.c_uint32), wpr, n, _p(off, ctypes.c_uint64),
                       _p(ids, ctypes.c_uint32))
    del rows
    return off, ids
