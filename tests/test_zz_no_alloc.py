"""hb_run_static, the run entry point that allocates nothing, against hb_run_with.

Its counters live in the library's static device workspace.  Two calls in a row,
the second on a smaller graph, must give exactly what hb_run_with gives on the same
arguments (registers byte for byte, pass counts, reach and sums bit for bit), and
what the oracle gives (Alg. 1), without changing the device's free memory.
"""
import numpy as np
import pytest

import hip_rt
import synth
from oracle_ref import assert_matches, ref

pytestmark = pytest.mark.gpu


def _load(hb, g):
    off, deg, data = hb.csr_encode(g.adj_offsets, g.adj_ids)
    return hb.graph_load(off, deg, data)


def _free_device_bytes():
    return hip_rt.mem_get_info()[0]


def _same(a, b, what):
    assert a.passes == b.passes and a.converged == b.converged, what
    assert a.union_kernel == b.union_kernel, what
    assert np.array_equal(a.registers, b.registers), what
    assert np.array_equal(a.reach, b.reach), what
    assert np.array_equal(a.sum_d, b.sum_d), what
    np.testing.assert_array_equal(a.mean_depth, b.mean_depth)


def test_static_runs_equal_allocating_runs(hb):
    big, small = synth.grid_graph(2, 64, 48), synth.tiny(1)
    Gb, Gs = _load(hb, big), _load(hb, small)
    cases = [(Gb, big, 10, 0, 3), (Gs, small, 10, 3, 4)]  # the second input is smaller
    assert small.n < big.n
    # the run kernel's tables fit the workspace for both graphs at p = 10
    assert 2 * 9 * big.n * 1024 <= hb.STATIC_SCRATCH_BYTES
    # one call first: the HIP runtime sets up per-kernel resources (code objects,
    # kernel-argument and scratch space) at a kernel's first launch in a process
    Gb.run_static(10, 1, 0)
    free0 = _free_device_bytes()
    held0 = hb.memory_stats(0)["held_bytes"]
    static = []
    for G, g, p, depth, seed in cases:
        print(f"[no-alloc] {g.name} n={g.n} p={p} depth={depth}", flush=True)
        static.append(G.run_static(p, depth, seed, registers=True))
    assert _free_device_bytes() == free0, "hb_run_static changed the device's free memory"
    assert hb.memory_stats(0)["held_bytes"] == held0
    for (G, g, p, depth, seed), r in zip(cases, static):
        what = f"{g.name} p={p} d={depth}"
        assert r.union_kernel == "runs", what  # small graphs: the run kernel, with its tables
        _same(r, G.run(p, depth, seed, registers=True), what)
        assert_matches(hb, r, ref(g, p, depth, seed), what)
    Gb.free()
    Gs.free()


def test_static_run_falls_back_and_refuses_what_does_not_fit(hb):
    g = synth.grid_graph(3, 100, 80)  # ~5.5k nodes
    G = _load(hb, g)
    # p = 10: the tables (2 x 9 x n KB) do not fit, the per-edge buffers do
    assert 2 * 9 * g.n * 1024 > hb.STATIC_SCRATCH_BYTES >= 2 * g.n * 1024
    print(f"[no-alloc] {g.name} n={g.n} p=10 fallback", flush=True)
    r = G.run_static(10, 2, 5, registers=True)
    assert r.union_kernel == "edges"
    _same(r, G.run(10, 2, 5, registers=True, kernel="edges"), "fallback")
    with pytest.raises(hb.HBError) as e:
        G.run_static(10, 2, 5, kernel="runs")
    assert e.value.status == hb.HB_ENOMEM and "static workspace" in str(e.value)
    # p = 14: even the per-edge buffers (2 x 16 KB per node) do not fit
    with pytest.raises(hb.HBError) as e:
        G.run_static(14, 1, 0)
    assert e.value.status == hb.HB_ENOMEM
    G.free()
