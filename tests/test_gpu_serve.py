"""Served runs (hb_submit / hb_poll): continuous batching, admission by memory, identical results.

Every served result is compared with the oracle's run of the same analysis (Alg. 1)
and with the same analysis run alone through hb_run: a result is the same alone and
in the mix."""
import time

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
    assert np.array_equal(a.reach, b.reach), what
    assert np.array_equal(a.sum_d, b.sum_d), what
    if a.registers is not None and b.registers is not None:
        assert np.array_equal(a.registers, b.registers), what


@pytest.fixture
def server(hb):
    started = []

    def start(**kw):
        hb.server_start(**kw)
        started.append(True)

    yield start
    if started:
        hb.server_stop()


@pytest.mark.parametrize("slow_lane_bytes", [0, 1, 2**64 - 1],
                         ids=["default-lanes", "all-slow-lane", "one-lane"])
def test_served_mix_equals_single_runs(hb, server, slow_lane_bytes):
    server(slow_lane_bytes=slow_lane_bytes)
    graphs = [synth.tiny(0), synth.tiny(3), synth.grid_graph(2, 64, 48), synth.star_graph(60),
              synth.random_graph(150, 0.02, 4)]
    Gs = [_load(hb, g) for g in graphs]
    specs = []
    for i, G in enumerate(Gs):
        for k, (p, depth) in enumerate([(10, 0), (8, 3), (13, 2), (4 + i, 1)]):
            specs.append((G, p, depth, 77 * i + k))
    owner = {id(G): g for G, g in zip(Gs, graphs)}
    tickets = [hb.submit(G, p, d, sd, registers=True) for (G, p, d, sd) in specs]
    res = [t.wait() for t in tickets]
    for (G, p, d, sd), r in zip(specs, res):
        what = f"{owner[id(G)].name} p={p} d={d} seed={sd}"
        assert_matches(hb, r, ref(owner[id(G)], p, d, sd), what)
        _same(r, G.run(p, d, sd, registers=True), what)
        assert r.t_submit_ns <= r.t_admit_ns <= r.t_start_ns <= r.t_end_ns
    st = hb.server_stats()
    assert st["completed"] >= len(specs) and st["running"] == 0 and st["queued"] == 0
    for G in Gs:
        G.free()


@pytest.mark.parametrize("slow_lane_bytes", [2**64 - 1, 1 << 30], ids=["one-lane", "two-lanes"])
def test_requests_join_while_others_run(hb, server, slow_lane_bytes):
    """A long request keeps running while short ones arrive, join and finish first."""
    # the per-edge kernel keeps the long request long: about 25 GB of gathers a step
    server(slow_lane_bytes=slow_lane_bytes, kernel="edges")
    gbig, gsmall = synth.grid_graph(1, 120, 100), synth.tiny(2)
    big = _load(hb, gbig)
    small = _load(hb, gsmall)
    tb = hb.submit(big, 12, 0, 5)
    for _ in range(200000):  # until the long request has been admitted
        if hb.server_stats()["running"] >= 1:
            break
        time.sleep(0.0001)
    ts = [hb.submit(small, 8, 2, s) for s in range(6)]
    rs = [t.wait() for t in ts]
    rb = tb.wait()
    assert max(r.t_end_ns for r in rs) <= rb.t_end_ns
    assert any(r.t_admit_ns > rb.t_admit_ns for r in rs)
    assert_matches(hb, rb, ref(gbig, 12, 0, 5), "big")
    _same(rb, big.run(12, 0, 5, kernel="edges"), "big")
    for s, r in enumerate(rs):
        assert_matches(hb, r, ref(gsmall, 8, 2, s), f"small {s}")
        _same(r, small.run(8, 2, s, kernel="edges"), f"small {s}")
    big.free()
    small.free()


def test_admission_respects_the_budget(hb, server):
    g = synth.tiny(4)
    G = _load(hb, g)
    per = 2 * ((g.n * 1024 * 8 + 255) // 256 * 256) + 2 * ((8 * g.n + 255) // 256 * 256) + \
        (4 * (g.n + 2) + 255) // 256 * 256
    server(hbm_budget=2 * per + 4096)  # room for two requests at a time
    ts = [hb.submit(G, 10, 0, s) for s in range(7)]
    rs = [t.wait() for t in ts]
    st = hb.server_stats()
    assert st["peak_used_bytes"] <= st["budget_bytes"]
    assert st["peak_used_bytes"] >= per
    for s, r in enumerate(rs):
        assert_matches(hb, r, ref(g, 10, 0, s), f"seed {s}")
        _same(r, G.run(10, 0, s), f"seed {s}")
    with pytest.raises(hb.HBError) as e:
        hb.submit(_load(hb, synth.grid_graph(0, 64, 64)), 12, 0, 0)
    assert e.value.status == hb.HB_ENOMEM
    G.free()


def test_poll_and_ticket_rules(hb, server):
    server(max_running=1, kernel="edges")  # one request at a time: the second one waits
    big = _load(hb, synth.grid_graph(1, 120, 100))
    g = synth.tiny(5)
    G = _load(hb, g)
    tb = hb.submit(big, 12, 0, 3)
    t = hb.submit(G, 9, 0, 1)
    with pytest.raises(hb.HBError) as e:
        G.free()  # queued behind the long request
    assert e.value.status == hb.HB_EBUSY
    r = None
    for _ in range(2000000):
        r = t.poll()
        if r is not None:
            break
    assert r is not None
    assert tb.poll() is not None or tb.wait() is not None
    assert_matches(hb, r, ref(g, 9, 0, 1), "polled")
    _same(r, G.run(9, 0, 1, kernel="edges"), "polled")
    with pytest.raises(hb.HBError) as e:
        t.poll()
    assert e.value.status == hb.HB_ENOTFOUND
    # registers were not kept for this ticket
    t2 = hb.submit(G, 9, 1, 2)
    t2.registers = True
    with pytest.raises(hb.HBError) as e:
        t2.wait()
    assert e.value.status == hb.HB_EINVAL
    t2.registers = False
    assert t2.wait().passes == 1
    G.free()
    big.free()


# ------------------------------------------------------------ device graph cache
def _csr_of(hb, g):
    off, deg, data = hb.csr_encode(g.adj_offsets, g.adj_ids)
    return (off, deg, data)


@pytest.fixture
def fresh_cache(hb):
    hb.graph_cache_clear()
    yield
    try:
        hb.server_stop()
    except hb.HBError:
        pass  # not running
    hb.set_options()
    hb.graph_cache_clear()
    hb.release_cache()


def test_cached_graphs_load_once_and_match_the_oracle(hb, fresh_cache):
    graphs = {11: synth.tiny(0), 12: synth.grid_graph(5, 60, 40), 13: synth.star_graph(70)}
    csrs = {k: _csr_of(hb, g) for k, g in graphs.items()}
    hb.server_start()
    jobs = [(k, p, d, 31 * k + i) for i, (p, d) in enumerate([(10, 0), (8, 3), (12, 2)])
            for k in graphs]
    tickets = [hb.submit_cached(k, p, d, s, csr=csrs[k], registers=True) for (k, p, d, s) in jobs]
    for (k, p, d, s), t in zip(jobs, tickets):
        assert_matches(hb, t.wait(), ref(graphs[k], p, d, s), f"cached key {k} p={p} d={d}")
    st = hb.graph_cache_stats()
    assert st["graphs"] == 3 and st["misses"] == 3 and st["hits"] == len(jobs) - 3
    assert st["busy"] == 0 and st["bytes"] > 0
    # a cached key needs no CSR; an unknown one does
    r = hb.submit_cached(12, 9, 1, 5, n=graphs[12].n).wait()
    assert_matches(hb, r, ref(graphs[12], 9, 1, 5), "cached without csr")
    with pytest.raises(hb.HBError) as e:
        hb.submit_cached(99, 9, 1, 5, n=10)
    assert e.value.status == hb.HB_ENOTFOUND


def test_cache_releases_the_least_recently_used_idle_graph(hb, fresh_cache):
    """Under a budget that holds two of three equal graphs, loading the third releases
    the graph used least recently; the results stay those of the oracle."""
    gs = {1: synth.grid_graph(1, 100, 80), 2: synth.grid_graph(2, 100, 80),
          3: synth.grid_graph(3, 100, 80)}
    csrs = {k: _csr_of(hb, g) for k, g in gs.items()}
    hb.server_start()
    for k in (1, 2):
        assert_matches(hb, hb.submit_cached(k, 4, 2, k, csr=csrs[k]).wait(), ref(gs[k], 4, 2, k),
                       f"graph {k}")
    assert_matches(hb, hb.submit_cached(1, 4, 3, 7, n=gs[1].n).wait(), ref(gs[1], 4, 3, 7),
                   "graph 1 again")  # graph 2 is now the least recently used
    hb.release_cache()
    st = hb.graph_cache_stats()
    per = st["bytes"] // 2
    hb.set_options(hbm_budget=hb.memory_stats(0)["held_bytes"] + per // 2 + (4 << 20))
    assert_matches(hb, hb.submit_cached(3, 4, 2, 3, csr=csrs[3]).wait(), ref(gs[3], 4, 2, 3),
                   "graph 3 under the budget")
    st = hb.graph_cache_stats()
    assert st["evictions"] == 1 and st["graphs"] == 2
    with pytest.raises(hb.HBError) as e:
        hb.submit_cached(2, 4, 2, 2, n=gs[2].n)
    assert e.value.status == hb.HB_ENOTFOUND
    assert_matches(hb, hb.submit_cached(1, 4, 2, 1, n=gs[1].n).wait(), ref(gs[1], 4, 2, 1),
                   "graph 1 stayed")


def test_served_grouped_requests(hb, server):
    """Requests on a graph of more than 32,768 nodes take the grouped kernel where it is
    built, in both lanes, and match the oracle and the run kernel alone."""
    server(slow_lane_bytes=1 << 30)
    rng = np.random.default_rng(29)
    n = 34000
    a, b = rng.integers(0, n, 200000), rng.integers(0, n, 200000)
    g = synth.from_edges(n, list(zip(a.tolist(), b.tolist())), name=f"sparse{n}")
    G = _load(hb, g)
    specs = [(9, 0, 1, 8), (10, 3, 2, 8), (12, 2, 3, 8), (8, 0, 4, 8), (10, 0, 5, 4),
             (12, 3, 6, 4), (13, 2, 7, 8), (8, 3, 8, 4)]
    tickets = [hb.submit(G, p, d, sd, registers=True, register_bits=bits)
               for (p, d, sd, bits) in specs]
    for (p, d, sd, bits), t in zip(specs, tickets):
        r = t.wait()
        what = f"{g.name} p={p} d={d} seed={sd} bits={bits}"
        grouped = (8 if bits == 8 else 9) <= p <= 12
        other = "runs" if p <= 12 else "edges"
        assert r.union_kernel == ("groups" if grouped else other), (what, r.union_kernel)
        assert_matches(hb, r, ref(g, p, d, sd, register_bits=bits), what)
        _same(r, G.run(p, d, sd, registers=True, register_bits=bits, kernel=other), what)
    G.free()
