"""The GPU visibility generator against the CPU rule (input tooling, not the HyperBall path)."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("maker", [lambda: synth.tiny_raster(0), lambda: synth.tiny_raster(3),
                                   lambda: synth.tiny_raster(9, 64, 64),
                                   lambda: synth.urban_raster(2, 90, 70, cell_m=3.0)])
def test_gpu_generator_equals_cpu(maker):
    obst = maker()
    a = synth.graph_from_raster(obst, device="cpu")
    b = synth.graph_from_raster(obst, device="gpu")
    assert a.n == b.n
    assert np.array_equal(a.adj_offsets, b.adj_offsets)
    assert np.array_equal(a.adj_ids, b.adj_ids)


def _has_edge(g, a, b):
    row = g.row(a)
    k = np.searchsorted(row, b)
    return bool(k < row.size and row[k] == b)


def test_gpu_urban_spot_check():
    g = synth.urban(0, device="gpu")
    print(f"[synth] urban n={g.n} E={g.n_edges}", flush=True)
    assert abs(g.n - 42700) / 42700 < 0.02
    rng = np.random.default_rng(0)
    # random pairs: membership in the GPU rows vs the CPU rule
    a = rng.integers(0, g.n, 200000)
    b = rng.integers(0, g.n, 200000)
    keep = a != b
    a, b = a[keep], b[keep]
    vis = synth.visible_pairs(g, a, b).astype(bool)
    got = np.array([_has_edge(g, int(x), int(y)) for x, y in zip(a, b)])
    assert np.array_equal(got, vis)
    # whole rows of a few sources
    for s in rng.integers(0, g.n, 12):
        t = np.arange(g.n)
        t = t[t != s]
        want = t[synth.visible_pairs(g, np.full(t.size, s), t).astype(bool)]
        assert np.array_equal(g.row(int(s)), want)
