"""Batched runs (hb_run_batch): every job's result equals the oracle's run of the same
analysis (Alg. 1: registers byte for byte, passes and convergence exactly, reach and
Eq. 3 sums within 1e-9), and equals its hb_run alone bit for bit."""
import numpy as np
import pytest

import synth
from oracle_ref import assert_matches, ref

pytestmark = pytest.mark.gpu


def _load(hb, g):
    off, deg, data = hb.csr_encode(g.adj_offsets, g.adj_ids)
    return hb.graph_load(off, deg, data)


def _same(a, b, what):
    assert a.passes == b.passes, (what, a.passes, b.passes)
    assert a.converged == b.converged, what
    # kernels may differ (blocking runs at p = 10 default to the grouped kernel); every
    # kernel gives the same registers and sums
    assert np.array_equal(a.registers, b.registers), what
    assert np.array_equal(a.reach, b.reach), what
    assert np.array_equal(a.sum_d, b.sum_d), what
    np.testing.assert_array_equal(a.mean_depth, b.mean_depth)


@pytest.mark.parametrize("kernel", ["auto", "edges", "runs"])
def test_batch_equals_single_runs(hb, kernel):
    graphs = [synth.tiny(0), synth.tiny(5), synth.grid_graph(2, 64, 48), synth.star_graph(90),
              synth.random_graph(200, 0.01, 3), synth.from_edges(1, [], name="single")]
    Gs = [_load(hb, g) for g in graphs]
    ps = [4, 8, 9, 10, 12, 13] if kernel != "runs" else [4, 8, 9, 10, 12, 11]
    jobs, owners = [], []
    for i, G in enumerate(Gs):
        for k, (p, depth) in enumerate([(ps[i], 0), (ps[(i + 2) % 6], 3), (10, 1 + i % 4)]):
            jobs.append((G, p, depth, 1000 * i + k))
            owners.append(graphs[i])
    print(f"[batch] {len(jobs)} jobs kernel={kernel}", flush=True)
    res = hb.run_batch(jobs, registers=True, kernel=kernel)
    for (G, p, depth, seed), g, r in zip(jobs, owners, res):
        what = f"{g.name} p={p} depth={depth} seed={seed}"
        assert_matches(hb, r, ref(g, p, depth, seed), what)
        _same(r, G.run(p, depth, seed, registers=True, kernel=kernel), what)
    # a second batch on the same graphs leaves no state behind
    res2 = hb.run_batch(jobs[::-1], registers=True, kernel=kernel)
    for r1, r2 in zip(res, res2[::-1]):
        _same(r1, r2, "repeat")
    for G in Gs:
        G.free()


def test_batched_workload_sample(hb):
    """A slice of the batched workload (uneven sizes, 1-2 m cells, mixed p and depth)."""
    Gs, jobs, graphs = [], [], []
    for seed in range(8):
        spec = synth.batch_spec(seed)
        g = synth.batch_graph(seed)
        print(f"[batch] seed={seed} n={g.n} E={g.n_edges} p={spec['p']} d={spec['depth']}",
              flush=True)
        G = _load(hb, g)
        Gs.append(G)
        graphs.append(g)
        jobs.append((G, spec["p"], spec["depth"], seed))
    res = hb.run_batch(jobs, registers=True)
    for (G, p, depth, seed), g, r in zip(jobs, graphs, res):
        assert_matches(hb, r, ref(g, p, depth, seed), f"seed={seed} {g.name}")
        _same(r, G.run(p, depth, seed, registers=True), f"seed={seed}")
    for G in Gs:
        G.free()


def test_batch_argument_errors(hb):
    g = synth.tiny(1)
    G = _load(hb, g)
    with pytest.raises(hb.HBError) as e:
        hb.run_batch([(G, 3, 0, 0)])
    assert e.value.status == hb.HB_EINVAL
    with pytest.raises(hb.HBError) as e:
        hb.run_batch([(G, 13, 0, 0)], kernel="runs")
    assert e.value.status == hb.HB_EINVAL
    G.free()
