"""Library-wide options (hb_set_options): one device-memory budget for every form,
allocator hooks, a caller stream, the stopping rule and seeded tuner picks.

Results under every option are compared with the oracle: Alg. 1 for the default
rule, and the oracle's exact balls (whose per-step estimates give the step at which
any growth threshold stops the run) for the overrides.
"""
import numpy as np
import pytest

import hip_rt
import oracle
import synth
from oracle_ref import assert_matches, ref

pytestmark = pytest.mark.gpu


def _load(hb, g, **kw):
    off, deg, data = hb.csr_encode(g.adj_offsets, g.adj_ids)
    return hb.graph_load(off, deg, data, **kw)


@pytest.fixture
def reset_options(hb):
    yield
    hb.set_options()
    hb.release_cache()


def _exact_steps(g, p, seed, T):
    """Per-step registers, estimates and Eq. 3 sums of every node from exact balls."""
    csr = oracle.from_graph(g)
    regs, balls = oracle.msbfs_balls(csr, np.arange(g.n), T, p, seed)
    est = np.array([[oracle.hll_estimate(regs[v, t], p) for t in range(T + 1)]
                    for v in range(g.n)])
    return regs, est


def _sums(est, T):
    s = np.zeros(est.shape[0])
    for t in range(1, T + 1):
        s = s + float(t) * (est[:, t] - est[:, t - 1])
    return s


def test_blocking_run_while_the_server_holds_memory(hb, reset_options):
    """One budget for all forms: a blocking run finds memory while served requests run,
    and both sets of results match the oracle."""
    hb.server_start()
    try:
        gbig, gsmall = synth.grid_graph(1, 120, 100), synth.tiny(3)
        big, small = _load(hb, gbig, order=synth.hilbert_order(gbig)), _load(hb, gsmall)
        tickets = [hb.submit(big, 10, 0, s) for s in range(3)]
        r = small.run(10, 0, 7, registers=True)
        assert_matches(hb, r, ref(gsmall, 10, 0, 7), "blocking beside the server")
        for s, t in enumerate(tickets):
            assert_matches(hb, t.wait(), ref(gbig, 10, 0, s), f"served {s}")
    finally:
        hb.server_stop()
    st = hb.memory_stats(0)
    assert st["pool_used_bytes"] == 0 and st["pool_peak_used_bytes"] > 0
    big.free()
    small.free()


def test_budget_caps_all_device_memory(hb, reset_options):
    g = synth.grid_graph(2, 64, 48)
    hb.release_cache()
    base = hb.memory_stats(0)["held_bytes"]  # graphs other tests still hold
    budget = base + (96 << 20)
    hb.set_options(hbm_budget=budget)
    G = _load(hb, g)
    r = G.run(10, 3, 1, registers=True)  # tables 2 x 9 x n KB: about 38 MiB, within it
    assert r.union_kernel == "runs"  # tables within the budget (small graph: run kernel)
    assert_matches(hb, r, ref(g, 10, 3, 1), "within the budget")
    st = hb.memory_stats(0)
    assert st["budget_bytes"] == budget and st["held_bytes"] <= budget
    # p = 13 needs 2 n 8 KB = 33 MiB per-edge; with the graph that still fits, p = 15
    # (2 n 32 KB = 133 MiB) cannot
    with pytest.raises(hb.HBError) as e:
        G.run(15, 1, 0)
    assert e.value.status == hb.HB_ENOMEM
    # the auto kernel falls back to per edge when the tables do not fit
    hb.release_cache()
    hb.set_options(hbm_budget=hb.memory_stats(0)["held_bytes"] + (24 << 20))
    r = G.run(10, 2, 1, registers=True)
    assert r.union_kernel == "edges"
    assert_matches(hb, r, ref(g, 10, 2, 1), "per edge under a tight budget")
    G.free()


def test_allocator_hooks_serve_every_allocation(hb, reset_options):
    live = {}

    def alloc(nbytes):
        p = hip_rt.malloc(nbytes)
        if p:
            live[p] = nbytes
        return p

    def free(p):
        assert p in live, "freed memory the hook did not allocate"
        del live[p]
        hip_rt.free(p)

    hb.release_cache()
    hb.set_options(dev_alloc=alloc, dev_free=free)
    g = synth.tiny(2)
    G = _load(hb, g)
    assert live, "graph arrays did not come from the hook"
    r = G.run(10, 0, 3, registers=True)
    assert_matches(hb, r, ref(g, 10, 0, 3), "with allocator hooks")
    rb = hb.run_batch([(G, 8, 3, 1), (G, 12, 0, 2)], registers=True)
    assert_matches(hb, rb[0], ref(g, 8, 3, 1), "batched with hooks")
    assert_matches(hb, rb[1], ref(g, 12, 0, 2), "batched with hooks")
    G.free()
    hb.release_cache()
    assert not live, f"{len(live)} hook allocations were not freed"


def test_caller_stream(hb, reset_options):
    g = synth.tiny(4)
    G = _load(hb, g)
    s = hip_rt.stream_create()
    try:
        hb.set_options(stream=s)
        assert hb.get_options()["stream"] == s
        for p, d in ((10, 0), (8, 3)):
            assert_matches(hb, G.run(p, d, 5, registers=True), ref(g, p, d, 5), f"stream p={p}")
            assert_matches(hb, G.run_static(p, d, 5, registers=True), ref(g, p, d, 5),
                           f"stream static p={p}")
    finally:
        hb.set_options()
        hip_rt.stream_destroy(s)
    G.free()


@pytest.mark.parametrize("depth", [6, 8, 9, 17])
def test_stop_rule_depth_runs_every_step(hb, reset_options, depth):
    """HB_STOP_DEPTH: exactly depth steps, registers of the exact balls B(v, depth), and the
    Eq. 3 sums of all of those steps, in every form."""
    g = synth.tiny(0)
    p, seed = 8, 11
    regs, est = _exact_steps(g, p, seed, depth)
    hb.set_options(stop_rule="depth")
    G = _load(hb, g)
    forms = {"single": G.run(p, depth, seed, registers=True),
             "edges": G.run(p, depth, seed, registers=True, kernel="edges"),
             "static": G.run_static(p, depth, seed, registers=True),
             "batched": hb.run_batch([(G, p, depth, seed)], registers=True)[0]}
    hb.server_start()
    try:
        forms["served"] = hb.submit(G, p, depth, seed, registers=True).wait()
    finally:
        hb.server_stop()
    for name, r in forms.items():
        assert r.passes == depth, (name, r.passes)
        assert np.array_equal(r.registers, regs[:, depth]), name
        np.testing.assert_allclose(r.reach, est[:, depth], rtol=1e-9, atol=0, err_msg=name)
        np.testing.assert_allclose(r.sum_d, _sums(est, depth), rtol=1e-9, atol=1e-9,
                                   err_msg=name)
        last_growth = float(np.max(est[:, depth] - est[:, depth - 1]))
        assert r.converged == (last_growth <= 0.5), name
    with pytest.raises(hb.HBError) as e:
        G.run(p, 0, seed)
    assert e.value.status == hb.HB_EINVAL
    G.free()


@pytest.mark.parametrize("delta", [0.0, 3.0, 40.0])
def test_stop_threshold(hb, reset_options, delta):
    """stop_delta: the run stops after the first step whose largest growth is at most
    the threshold, as the exact balls' estimates say."""
    g = synth.tiny(1)
    p, seed = 10, 4
    full = ref(g, p, 0, seed)
    regs, est = _exact_steps(g, p, seed, full.passes)
    growth = np.max(est[:, 1:] - est[:, :-1], axis=0)  # growth[t - 1] of step t
    thr = delta if delta > 0 else 0.5
    T = int(np.argmax(growth <= thr)) + 1
    assert growth[T - 1] <= thr
    hb.set_options(stop_delta=delta)
    G = _load(hb, g)
    forms = {"single": G.run(p, 0, seed, registers=True),
             "batched": hb.run_batch([(G, p, 0, seed)], registers=True)[0]}
    for name, r in forms.items():
        assert r.passes == T and r.converged, (name, r.passes, T)
        assert np.array_equal(r.registers, regs[:, T]), name
        np.testing.assert_allclose(r.sum_d, _sums(est, T), rtol=1e-9, atol=1e-9, err_msg=name)
    if delta == 0.0:
        assert_matches(hb, forms["single"], full, "default threshold")
    G.free()


def test_tune_seed_sets_the_pick(hb, reset_options):
    g = synth.grid_graph(4, 60, 50)
    G = _load(hb, g)
    hb.tune_clear()
    r0 = G.run(10, 2, 0, tune="measure", kernel="runs")
    picks = [e for e in hb.tune_cache() if e["p"] == 10 and e["batched"] == 0]
    assert len(picks) == 1
    other = [(L, nb) for L, nb in ((64, 4), (32, 2), (16, 1))
             if (L, nb) != (picks[0]["lanes_per_node"], picks[0]["nodes_per_block"])][0]
    seeded = dict(picks[0], lanes_per_node=other[0], nodes_per_block=other[1])
    hb.tune_clear()
    hb.set_options(tune_seed=[seeded])
    r = G.run(10, 2, 0, registers=True, tune="cached", kernel="runs")
    assert (r.lanes_per_node, r.nodes_per_block) == other
    assert_matches(hb, r, ref(g, 10, 2, 0), "seeded pick")
    assert r.passes == r0.passes
    hb.tune_clear()
    G.free()
