"""Locality reordering (Sec. 3.2): a processing order changes no result; hash ids
make a renumbered graph reproduce the original counters, permuted.
"""
import numpy as np
import pytest

import oracle
import oracle_ref
import synth

pytestmark = pytest.mark.gpu

RTOL = 1e-9


def _load(hb, g, **kw):
    off, deg, data = hb.csr_encode(g.adj_offsets, g.adj_ids)
    return hb.graph_load(off, deg, data, **kw)


def _check(res, ref, what):
    assert res.passes == ref.passes and res.converged == ref.converged, what
    bad = np.nonzero((res.registers != ref.registers).any(axis=1))[0]
    assert bad.size == 0, f"{what}: registers differ at nodes {bad[:10]}"
    np.testing.assert_allclose(res.reach, ref.reach, rtol=RTOL, atol=0, err_msg=what)
    np.testing.assert_allclose(res.sum_d, ref.sum_d, rtol=RTOL, atol=1e-9, err_msg=what)


@pytest.mark.parametrize("gname", ["tiny", "rect100x80", "sparse5k"])
def test_processing_order_changes_nothing(hb, gname):
    if gname == "tiny":
        g = synth.tiny(3)
    elif gname == "rect100x80":
        g = synth.grid_graph(6, 100, 80)
    else:
        rng = np.random.default_rng(9)
        a, b = rng.integers(0, 5000, 60000), rng.integers(0, 5000, 60000)
        g = synth.from_edges(5000, list(zip(a.tolist(), b.tolist())), name="sparse5k")
    orders = {"random": np.random.default_rng(1).permutation(g.n).astype(np.uint32),
              "reversed": np.arange(g.n, dtype=np.uint32)[::-1].copy()}
    if gname != "sparse5k":
        orders["hilbert"] = synth.hilbert_order(g)
    for p, depth in ((8, 0), (10, 3), (12, 2), (13, 2)):
        ref = oracle.hyperball(oracle.from_graph(g), p, depth, 2)
        for oname, order in orders.items():
            G = _load(hb, g, order=order)
            kernels = (("runs", "edges") if p <= 12 else ("edges",)) + \
                (("groups",) if 8 <= p <= 12 else ())
            for kernel in kernels:
                what = f"{g.name} order={oname} p={p} d={depth} {kernel}"
                print(f"[order] {what}", flush=True)
                _check(G.run(p, depth, 2, registers=True, kernel=kernel, tune="off"), ref, what)
                if p == 10 and kernel != "groups":  # a non-default schedule walks the order too
                    _check(G.run(p, depth, 2, registers=True, kernel=kernel, lanes_per_node=32,
                                 nodes_per_block=2), ref, what + " 32x2")
            G.free()


def test_renumbered_graph_with_hash_ids(hb):
    g = synth.grid_graph(2, 90, 70)
    h, orig = synth.relabel(g, synth.hilbert_order(g))
    for p, depth in ((10, 0), (9, 3)):
        a = oracle.hyperball(oracle.from_graph(g), p, depth, 7)
        b = oracle.hyperball(oracle.from_graph(h), p, depth, 7, hash_ids=orig)
        G = _load(hb, h, hash_ids=orig)
        for kernel in ("runs", "edges") + (("groups",) if 8 <= p <= 12 else ()):
            r = G.run(p, depth, 7, registers=True, kernel=kernel, tune="off")
            what = f"renumbered p={p} d={depth} {kernel}"
            print(f"[order] {what}", flush=True)
            _check(r, b, what)
            assert np.array_equal(r.registers, a.registers[orig]), what
            assert np.array_equal(r.reach, a.reach[orig]), what
        G.free()


def test_ordered_graphs_in_batch_and_server(hb):
    graphs = [synth.tiny(0), synth.grid_graph(1, 70, 50), synth.tiny(7)]
    Gs = [_load(hb, g, order=synth.hilbert_order(g)) for g in graphs]
    jobs = [(G, p, d, 11 * i) for i, G in enumerate(Gs) for (p, d) in ((10, 0), (8, 3))]
    owners = [g for g in graphs for _ in range(2)]
    refs = [oracle_ref.ref(g, p, d, s) for g, (G, p, d, s) in zip(owners, jobs)]
    single = [G.run(p, d, s, registers=True, tune="off") for (G, p, d, s) in jobs]
    batched = hb.run_batch(jobs, registers=True, tune="off")
    for a, b, r, (G, p, d, s) in zip(single, batched, refs, jobs):
        _check(b, r, f"batched p={p} d={d} seed={s}")
        assert np.array_equal(a.registers, b.registers) and np.array_equal(a.sum_d, b.sum_d)
    hb.server_start()
    try:
        served = [hb.submit(G, p, d, s, registers=True).wait() for (G, p, d, s) in jobs]
    finally:
        hb.server_stop()
    for a, b, r, (G, p, d, s) in zip(single, served, refs, jobs):
        _check(b, r, f"served p={p} d={d} seed={s}")
        assert np.array_equal(a.registers, b.registers) and np.array_equal(a.sum_d, b.sum_d)
    for G in Gs:
        G.free()


def test_bad_orders_are_refused(hb):
    g = synth.tiny(1)
    off, deg, data = hb.csr_encode(g.adj_offsets, g.adj_ids)
    for bad in (np.zeros(g.n, np.uint32), np.arange(1, g.n + 1, dtype=np.uint32)):
        with pytest.raises(hb.HBError) as e:
            hb.graph_load(off, deg, data, order=bad)
        assert e.value.status == hb.HB_EINVAL
    with pytest.raises(hb.HBError) as e:
        hb.graph_load(off, deg, data, order=np.arange(g.n - 1, dtype=np.uint32))
    assert e.value.status == hb.HB_EINVAL
