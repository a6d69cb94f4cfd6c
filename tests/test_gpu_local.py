"""Exact local metrics (hb_local_metrics) against the oracle, node by node.

Both sides count integers (adjacent neighbour pairs, the two-step ball) and form
each ratio with one double division of the same operands, so every output must
match bit for bit, NaN at the same nodes.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

KEYS = ("pairs", "ball2", "clustering", "controllability")


def _load(hb, g, **kw):
    off, deg, data = hb.csr_encode(g.adj_offsets, g.adj_ids)
    return hb.graph_load(off, deg, data, **kw)


def _compare(got, ref, what, nodes=None):
    for key in KEYS:
        a = got[key] if nodes is None else got[key][nodes]
        b = ref[key]
        assert np.array_equal(a, b, equal_nan=key in ("clustering", "controllability")), \
            f"{what} {key}: differ at {np.nonzero(~((a == b) | (np.isnan(a) & np.isnan(b))))[0][:10]}"


def _random_graph(seed, n, m, name):
    rng = np.random.default_rng(seed)
    a, b = rng.integers(0, n, m), rng.integers(0, n, m)
    return synth.from_edges(n, [(int(x), int(y)) for x, y in zip(a, b) if x != y], name=name)


def _wheel(r):
    edges = [(0, i) for i in range(1, r + 1)] + [(i, i % r + 1) for i in range(1, r + 1)]
    return synth.from_edges(r + 1, edges, name=f"wheel{r}")


@pytest.mark.parametrize("gname", ["tiny", "rect90x70", "star", "complete", "path", "wheel",
                                   "random", "isolated", "single", "pair"])
def test_local_metrics_match_oracle(hb, gname):
    g = {"tiny": lambda: synth.tiny(5),
         "rect90x70": lambda: synth.grid_graph(4, 90, 70),
         "star": lambda: synth.star_graph(500),
         "complete": lambda: synth.complete_graph(150),
         "path": lambda: synth.path_graph(300),
         "wheel": lambda: _wheel(200),
         # rows of several 64-byte chunks, runs of every length, many gaps
         "random": lambda: _random_graph(3, 3000, 120000, "random3000"),
         "isolated": lambda: synth.from_edges(9, [(0, 1), (1, 2), (0, 2), (4, 5)], name="iso"),
         "single": lambda: synth.from_edges(1, [], name="single"),
         "pair": lambda: synth.from_edges(2, [(0, 1)], name="pair"),
         }[gname]()
    ref = oracle.local_metrics(oracle.from_graph(g))
    # the neighbour runs the metrics read: sum over rows of degree x maximal runs
    deg = np.diff(g.adj_offsets).astype(np.int64)
    runs = np.array([int(np.count_nonzero(np.diff(r.astype(np.int64)) != 1)) + 1 if r.size else 0
                     for r in (g.adj_ids[g.adj_offsets[v]:g.adj_offsets[v + 1]]
                               for v in range(g.n))], np.int64)
    for order in (None, "hilbert") if gname in ("tiny", "rect90x70") else (None,):
        kw = {} if order is None else {"order": synth.hilbert_order(g)}
        G = _load(hb, g, **kw)
        print(f"[local] {g.name} order={order}", flush=True)
        assert G.stats()["local_run_reads"] == int((deg * runs).sum())
        _compare(G.local_metrics(), ref, f"{g.name} order={order}")
        G.free()


def test_local_metrics_long_runs_cross_words(hb):
    """Rows made of long id runs with ragged ends, so the bitmap ranges start and
    end at every bit position and span many 32-bit words."""
    rng = np.random.default_rng(11)
    n, edges = 4000, set()
    for v in range(0, n, 7):
        for _ in range(3):
            a = int(rng.integers(0, n - 200))
            for w in range(a, a + int(rng.integers(1, 200))):
                if w != v:
                    edges.add((min(v, w), max(v, w)))
    g = synth.from_edges(n, sorted(edges), name="longruns")
    G = _load(hb, g)
    _compare(G.local_metrics(), oracle.local_metrics(oracle.from_graph(g)), g.name)
    G.free()


def test_local_metrics_urban_sampled(hb):
    """The urban street graph (about 42,700 nodes, 1e8 directed edges): every
    node on the device, a seeded sample of 64 nodes in the oracle."""
    g = synth.urban(0, device="gpu")
    G = _load(hb, g, order=synth.hilbert_order(g))
    got = G.local_metrics()
    G.free()
    nodes = np.random.default_rng(2).choice(g.n, size=64, replace=False).astype(np.uint32)
    ref = oracle.local_metrics(oracle.from_graph(g), nodes=nodes)
    _compare(got, ref, g.name, nodes)
    assert np.all(got["ball2"] >= np.diff(g.adj_offsets))  # N(v) is inside B(v, 2)


def test_local_metrics_refuses_graphs_beyond_lds(hb):
    g = synth.path_graph(700000)
    G = _load(hb, g)
    with pytest.raises(hb.HBError) as e:
        G.local_metrics()
    assert e.value.status == hb.HB_EINVAL
    G.free()


@pytest.mark.slow
@pytest.mark.timeout(1200)
def test_local_metrics_city_sampled(hb):
    """The city graph (235,770 nodes, 4.94e9 directed edges), the size and order
    the benchmark uses: every node on the device, 16 seeded nodes in the oracle."""
    g = synth.city(0, device="gpu")
    print(f"[local] city n={g.n}", flush=True)
    G = _load(hb, g, order=synth.hilbert_order(g))
    got = G.local_metrics()
    G.free()
    nodes = np.random.default_rng(4).choice(g.n, size=16, replace=False).astype(np.uint32)
    ref = oracle.local_metrics(oracle.from_graph(g), nodes=nodes)
    _compare(got, ref, g.name, nodes)
