"""Decoder edge cases on the GPU: multi-byte varints, varints cut by chunk ends, long runs.

Every union kernel is checked against the oracle, byte for byte (the grouped one
where it is built: p = 8..12 at the default table depth).  Rows are built so
that the wave-cooperative decoder meets every case: 2- and 3-byte deltas, a varint
split across two 64-byte chunks, chunks that are all deltas of one, runs longer than
any table block, and a row whose only run passes over the node itself.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

RTOL = 1e-9


def _check(hb, g, p, depth, seed=0, levels=0):
    ref = oracle.hyperball(oracle.from_graph(g), p, depth, seed)
    off, deg, data = hb.csr_encode(g.adj_offsets, g.adj_ids)
    with hb.graph_load(off, deg, data) as G:
        for kernel in ("runs", "edges") + (("groups",) if 8 <= p <= 12 and levels == 0 else ()):
            print(f"[edge] {g.name} n={g.n} E={g.n_edges} p={p} d={depth} {kernel} K={levels}",
                  flush=True)
            r = G.run(p, depth, seed, registers=True, kernel=kernel, table_levels=levels)
            assert r.passes == ref.passes and r.converged == ref.converged, kernel
            bad = np.nonzero((r.registers != ref.registers).any(axis=1))[0]
            assert bad.size == 0, f"{kernel}: registers differ at {bad[:8]}"
            np.testing.assert_allclose(r.reach, ref.reach, rtol=RTOL, atol=0)
            np.testing.assert_allclose(r.sum_d, ref.sum_d, rtol=RTOL, atol=1e-9)


def test_sparse_graph_multibyte_deltas(hb):
    """n = 60,000 with ~30 random neighbours per node: most deltas need 2-3 bytes."""
    rng = np.random.default_rng(17)
    n = 60000
    a = rng.integers(0, n, 900000)
    b = rng.integers(0, n, 900000)
    g = synth.from_edges(n, list(zip(a.tolist(), b.tolist())), name="sparse60k")
    _check(hb, g, 8, 3)
    _check(hb, g, 10, 2, seed=9)


def _crafted_rows():
    """Rows that put varints across 64-byte chunk boundaries and make long runs."""
    n = 40000
    edges = []
    # node 0: ids 1..62 (62 one-byte varints), then a 3-byte jump that straddles
    # bytes 62..64, then a long run, then a 2-byte jump ending exactly at byte 127
    row = list(range(1, 63)) + [20000] + list(range(20001, 20060)) + [20300, 20301]
    edges += [(0, j) for j in row]
    # node 1: a run of 500 consecutive ids (several full chunks of deltas of one)
    edges += [(1, j) for j in range(3000, 3500)]
    # node 5: one run through the node itself (4 .. 6 without 5) plus far ids
    edges += [(5, j) for j in (2, 3, 4, 6, 7, 8, 39000, 39999)]
    # node 7: alternating gaps (no runs at all) over 200 ids
    edges += [(7, j) for j in range(100, 500, 2)]
    # a long path keeps the diameter above a few steps
    edges += [(i, i + 1) for i in range(20000, 20400)]
    return synth.from_edges(n, edges, name="crafted40k")


@pytest.mark.parametrize("levels", [0, 1, 3])
def test_crafted_chunk_boundaries(hb, levels):
    g = _crafted_rows()
    csr = oracle.from_graph(g)
    a, b = int(csr.offsets[0]), int(csr.offsets[1])
    row0 = csr.bytes[a:b]
    assert row0[62] & 0x80 and row0[63] & 0x80 and not row0[64] & 0x80  # 3-byte varint
    _check(hb, g, 9, 0, seed=4, levels=levels)
    _check(hb, g, 12, 4, seed=5, levels=levels)


def test_wide_open_area(hb):
    """An obstacle-free raster: every row is a few very long runs (runs > 2^K)."""
    g = synth.graph_from_raster(np.zeros((40, 50), np.uint8), name="open50x40")
    for levels in (2, 7):
        _check(hb, g, 8, 0, seed=1, levels=levels)


def test_very_long_row(hb):
    """A 100,001-node star: the centre's row holds 100,000 ids (about 100 KB of LEB128,
    1,563 chunks), every leaf row one id; both kernels and several shapes."""
    n = 100_001
    off = np.zeros(n + 1, np.uint64)
    off[1] = n - 1
    off[2:] = n - 1 + np.arange(1, n, dtype=np.uint64)
    ids = np.concatenate([np.arange(1, n, dtype=np.uint32), np.zeros(n - 1, np.uint32)])
    g = synth.Graph(n=n, adj_offsets=off, adj_ids=ids, obst=np.zeros((1, 1), np.uint8),
                    xy=np.zeros((n, 2), np.int32), name="star100k")
    for p, depth in ((10, 0), (4, 2), (12, 1)):
        ref = oracle.hyperball(oracle.from_graph(g), p, depth, 3)
        off_b, deg, data = hb.csr_encode(g.adj_offsets, g.adj_ids)
        assert int(off_b[1]) >= 99_000  # the centre row spans ~1,560 chunks
        with hb.graph_load(off_b, deg, data) as G:
            for kernel in ("runs", "edges") + (("groups",) if 8 <= p <= 12 else ()):
                print(f"[edge] star100k p={p} d={depth} {kernel}", flush=True)
                r = G.run(p, depth, 3, registers=True, kernel=kernel, tune="off")
                assert r.passes == ref.passes and r.converged == ref.converged
                assert np.array_equal(r.registers, ref.registers), (p, kernel)
                np.testing.assert_allclose(r.sum_d, ref.sum_d, rtol=RTOL, atol=1e-9)
