"""Union schedules and their autotuner: every schedule gives the oracle's registers.

A schedule is (lanes per node, nodes per workgroup).  The lanes spread one
counter over part of a wave (several neighbour groups per wave), one wave, or
several waves that each own a slice; the tuner only picks among them by speed,
so each one is checked against the oracle, and tuned runs against untuned ones.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

RTOL = 1e-9

# lanes per node built for each p, the default first (as documented in hb.h)
LANES = {4: [1], 5: [2], 6: [4], 7: [8], 8: [16, 8], 9: [32, 16], 10: [64, 32, 16],
         11: [64, 128, 32], 12: [64, 128, 256], 13: [128, 256], 14: [256, 512], 15: [512],
         16: [1024]}


def _schedules(p):
    for lanes in LANES[p]:
        for nb in ([4, 2, 1] if lanes <= 64 else [1]):
            yield lanes, nb


def _load(hb, g):
    off, deg, data = hb.csr_encode(g.adj_offsets, g.adj_ids)
    return hb.graph_load(off, deg, data)


def _check(res, ref, what):
    assert res.passes == ref.passes and res.converged == ref.converged, what
    bad = np.nonzero((res.registers != ref.registers).any(axis=1))[0]
    assert bad.size == 0, f"{what}: registers differ at nodes {bad[:10]}"
    np.testing.assert_allclose(res.reach, ref.reach, rtol=RTOL, atol=0, err_msg=what)
    np.testing.assert_allclose(res.sum_d, ref.sum_d, rtol=RTOL, atol=1e-9, err_msg=what)


@pytest.mark.parametrize("p", sorted(LANES))
def test_every_schedule_matches_oracle(hb, p):
    """tiny (709 nodes) and a 72x60 raster, both kernels, every built schedule.

    From p = 13 on only tiny at depth 2: the oracle's cost grows with 2^p.
    """
    cases = ((synth.tiny(1), 0, 3), (synth.grid_graph(4, 72, 60), 2, 8)) if p <= 12 else \
        ((synth.tiny(1), 2, 3),)
    for g, depth, seed in cases:
        ref = oracle.hyperball(oracle.from_graph(g), p, depth, seed)
        G = _load(hb, g)
        kernels = ("edges", "runs") if p <= 12 else ("edges",)
        for lanes, nb in _schedules(p):
            for kernel in kernels:
                what = f"{g.name} p={p} lanes={lanes} nb={nb} {kernel}"
                print(f"[sched] {what}", flush=True)
                r = G.run(p, depth, seed, registers=True, kernel=kernel, lanes_per_node=lanes,
                          nodes_per_block=nb)
                assert (r.lanes_per_node, r.nodes_per_block) == (lanes, nb), what
                _check(r, ref, what)
        G.free()


def test_schedule_on_chunked_rows(hb):
    """Rows of several 64-byte chunks with multi-byte deltas under the wide shapes."""
    rng = np.random.default_rng(5)
    n = 6000
    a = rng.integers(0, n, 120000)
    b = rng.integers(0, n, 120000)
    g = synth.from_edges(n, list(zip(a.tolist(), b.tolist())), name="sparse6k")
    G = _load(hb, g)
    for p, lanes, nb in ((10, 16, 2), (10, 32, 1), (11, 128, 1), (12, 256, 1), (12, 128, 1),
                         (8, 8, 4), (14, 512, 1)):
        ref = oracle.hyperball(oracle.from_graph(g), p, 3, 1)
        for kernel in (("edges", "runs") if p <= 12 else ("edges",)):
            what = f"p={p} lanes={lanes} nb={nb} {kernel}"
            print(f"[sched] sparse6k {what}", flush=True)
            _check(G.run(p, 3, 1, registers=True, kernel=kernel, lanes_per_node=lanes,
                         nodes_per_block=nb), ref, what)
    G.free()


def test_unbuilt_schedules_are_refused(hb):
    G = _load(hb, synth.tiny(0))
    for p, lanes, nb in ((10, 128, 1), (10, 64, 3), (12, 256, 2), (8, 64, 4), (16, 512, 1)):
        with pytest.raises(hb.HBError) as e:
            G.run(p, 1, 0, lanes_per_node=lanes, nodes_per_block=nb)
        assert e.value.status == hb.HB_EINVAL, (p, lanes, nb)
    with pytest.raises(hb.HBError) as e:
        G.run(10, 1, 0, nodes_per_block=2)  # nodes per workgroup without lanes
    assert e.value.status == hb.HB_EINVAL
    with pytest.raises(hb.HBError) as e:
        hb.run_batch([(G, 10, 1, 0), (G, 8, 1, 0)], lanes_per_node=64)  # 64 lanes: not for p=8
    assert e.value.status == hb.HB_EINVAL
    G.free()


def test_tuned_single_run(hb):
    hb.tune_clear()
    g = synth.grid_graph(3, 96, 80)
    G = _load(hb, g)
    base = G.run(12, 0, 4, registers=True, tune="off")
    first = G.run(12, 0, 4, registers=True, tune="measure")
    assert first.tune_ms > 0.0
    again = G.run(12, 0, 4, registers=True, tune="measure")
    assert again.tune_ms == 0.0  # cached
    assert (again.lanes_per_node, again.nodes_per_block) == \
        (first.lanes_per_node, first.nodes_per_block)
    assert (first.lanes_per_node, first.nodes_per_block) in set(_schedules(12))
    for r in (first, again):
        assert np.array_equal(r.registers, base.registers)
        assert np.array_equal(r.reach, base.reach) and np.array_equal(r.sum_d, base.sum_d)
        assert r.passes == base.passes and r.converged == base.converged
    cache = [e for e in hb.tune_cache() if e["batched"] == 0 and e["p"] == 12]
    assert len(cache) == 1
    e = cache[0]
    assert (e["lanes_per_node"], e["nodes_per_block"]) == \
        (first.lanes_per_node, first.nodes_per_block)
    assert 0.0 < e["best_ms"] <= e["default_ms"]
    hb.tune_clear()
    assert hb.tune_cache() == []
    G.free()


def test_tuned_batch(hb):
    hb.tune_clear()
    Gs, jobs = [], []
    for seed in range(6):
        spec = synth.batch_spec(seed)
        G = _load(hb, synth.batch_graph(seed))
        Gs.append(G)
        jobs.append((G, spec["p"], spec["depth"], seed))
    ref = hb.run_batch(jobs, registers=True, tune="off")
    tuned = hb.run_batch(jobs, registers=True, tune="measure")
    assert tuned[0].tune_ms > 0.0
    cached = hb.run_batch(jobs, registers=True, tune="cached")
    assert cached[0].tune_ms == 0.0
    for a, b, c in zip(ref, tuned, cached):
        for r in (b, c):
            assert np.array_equal(r.registers, a.registers)
            assert np.array_equal(r.reach, a.reach) and np.array_equal(r.sum_d, a.sum_d)
            assert r.passes == a.passes and r.converged == a.converged
        assert (b.lanes_per_node, b.nodes_per_block) == (c.lanes_per_node, c.nodes_per_block)
    classes = {(p, r.union_kernel) for (_, p, _, _), r in zip(jobs, tuned)}
    batched = [e for e in hb.tune_cache() if e["batched"] == 1]
    assert {(e["p"], e["union_kernel"]) for e in batched} == classes
    hb.tune_clear()
    for G in Gs:
        G.free()
