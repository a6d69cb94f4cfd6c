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


def _sparse_large(n=34000, n_edges=200000, seed=23):
    """Above the grouped kernel's size threshold, cheap for the oracle."""
    rng = np.random.default_rng(seed)
    a, b = rng.integers(0, n, n_edges), rng.integers(0, n, n_edges)
    return synth.from_edges(n, list(zip(a.tolist(), b.tolist())), name=f"sparse{n}")


@pytest.mark.parametrize("bits", [8, 4])
def test_batch_grouped_jobs(hb, bits):
    """Jobs on a graph of more than 32,768 nodes take the grouped kernel where it is
    built (p = 8..12 with 8-bit registers, 9..12 with 4-bit), beside run-kernel and
    per-edge jobs."""
    g = _sparse_large()
    G = _load(hb, g)
    ps = [8, 9, 10, 11, 12, 13] if bits == 8 else [8, 9, 10, 11, 12]
    jobs = [(G, p, (0, 3, 2)[i % 3], 100 + i) for i, p in enumerate(ps)]
    print(f"[batch] grouped jobs n={g.n} E={g.n_edges} bits={bits}", flush=True)
    res = hb.run_batch(jobs, registers=True, register_bits=bits)
    for (_, p, d, seed), r in zip(jobs, res):
        what = f"{g.name} p={p} d={d} seed={seed} bits={bits}"
        grouped = (8 if bits == 8 else 9) <= p <= 12
        other = "runs" if p <= 12 else "edges"
        assert r.union_kernel == ("groups" if grouped else other), (what, r.union_kernel)
        assert_matches(hb, r, ref(g, p, d, seed, register_bits=bits), what)
        _same(r, G.run(p, d, seed, registers=True, register_bits=bits, kernel=other), what)
    G.free()
