"""GPU parity: the HIP library (through the C ABI) against the CPU oracle.

Registers must match byte for byte, pass counts and the convergence flag exactly;
reach and the Eq. 3 sums within 1e-9 relative (the only floating-point step is the
estimator, whose log may differ by an ulp between host libm and the device).
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

RTOL = 1e-9


def _load(hb, g):
    off, deg, data = hb.csr_encode(g.adj_offsets, g.adj_ids)
    return hb.graph_load(off, deg, data)


def _compare(res, ref, what):
    assert res.passes == ref.passes, (what, res.passes, ref.passes)
    assert res.converged == ref.converged, (what, res.converged, ref.converged)
    # a converged run's last step only detected the fixpoint
    assert res.productive_iters == ref.passes - int(ref.converged), what
    if ref.registers is not None:
        bad = np.nonzero((res.registers != ref.registers).any(axis=1))[0]
        assert bad.size == 0, f"{what}: registers differ at nodes {bad[:10]}"
    np.testing.assert_allclose(res.reach, ref.reach, rtol=RTOL, atol=0, err_msg=what)
    np.testing.assert_allclose(res.sum_d, ref.sum_d, rtol=RTOL, atol=1e-9, err_msg=what)


def _check(hb, g, p, depth, seed=0, kernels=("edges", "runs", "groups"), table_levels=0):
    """Every union kernel that supports p against the oracle."""
    ref = oracle.hyperball(oracle.from_graph(g), p, depth, seed)
    with _load(hb, g) as G:
        for kernel in kernels:
            if kernel == "runs" and p > 12:
                continue
            if kernel == "groups" and (not 8 <= p <= 12 or table_levels not in (0, 8)):
                continue  # built for p = 8..12 and the default table depth
            print(f"[parity] {g.name} n={g.n} E={g.n_edges} p={p} depth={depth} seed={seed} "
                  f"kernel={kernel} K={table_levels}", flush=True)
            res = G.run(p, depth, seed, registers=True, kernel=kernel, table_levels=table_levels)
            assert res.union_kernel == kernel
            _compare(res, ref, f"{g.name} p={p} d={depth} seed={seed} {kernel}")
    return res, ref


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("depth", [0, 1, 2, 3])
def test_tiny_p10(hb, seed, depth):
    _check(hb, synth.tiny(seed), 10, depth, seed=0)


@pytest.mark.parametrize("p", range(4, 17))
@pytest.mark.parametrize("depth", [0, 2])
def test_tiny_all_p(hb, p, depth):
    _check(hb, synth.tiny(1), p, depth, seed=12345)


@pytest.mark.parametrize("hash_seed", [0, 1, 0xDEADBEEFCAFEF00D])
def test_hash_seeds(hb, hash_seed):
    _check(hb, synth.tiny(2), 8, 0, seed=hash_seed)


@pytest.mark.parametrize("maker,n", [(synth.path_graph, 40), (synth.cycle_graph, 33),
                                     (synth.star_graph, 50), (synth.complete_graph, 30)])
@pytest.mark.parametrize("p", [4, 10])
def test_closed_form_graphs(hb, maker, n, p):
    _check(hb, maker(n), p, 0)


def test_single_node(hb):
    g = synth.from_edges(1, [], name="single")
    res, ref = _check(hb, g, 10, 0)
    assert res.passes == 1 and res.converged


def test_isolated_nodes(hb):
    g = synth.random_graph(300, 0.004, seed=5)
    assert (g.degrees == 0).any()
    _check(hb, g, 9, 0)


@pytest.mark.parametrize("W,H,seed", [(64, 64, 0), (100, 80, 3)])
@pytest.mark.parametrize("p", [8, 10, 12])
@pytest.mark.parametrize("depth", [3, 0])
def test_rect_rasters(hb, W, H, seed, p, depth):
    _check(hb, synth.grid_graph(seed, W, H), p, depth)


@pytest.mark.parametrize("levels", [1, 2, 3, 5, 12])
@pytest.mark.parametrize("p", [4, 9, 10])
def test_run_kernel_table_depths(hb, levels, p):
    """Shallow tables force long runs to be tiled by many level-K blocks."""
    g = synth.urban_raster(4, 120, 90, cell_m=2.0)
    g = synth.graph_from_raster(g, name="urban120x90")
    _check(hb, g, p, 0, kernels=("runs",), table_levels=levels)


def test_runs_joined_across_own_node(hb):
    """Rows that skip only the node itself: one run through v, including v's counter."""
    n = 300
    edges = [(i, j) for i in range(n) for j in range(i + 1, min(n, i + 40))]
    g = synth.from_edges(n, edges, name="band40")
    _check(hb, g, 10, 0, table_levels=3)
    with _load(hb, g) as G:
        st = G.stats()
    assert st["n_runs"] == n  # every row is one run once v is joined in


def test_prefix_property(hb):
    """Registers of a depth-t run equal step t of a longer run (oracle: exact balls)."""
    g = synth.tiny(3)
    csr = oracle.from_graph(g)
    dist = oracle.bfs_all(csr)
    with _load(hb, g) as G:
        for t in (1, 2, 3, 4):
            res = G.run(10, t, 0, registers=True)
            for v in range(0, g.n, 7):
                ball = oracle.ball_registers(dist[v], t, 10, 0)
                assert np.array_equal(res.registers[v], ball), (t, v)


# ---------------------------------------------------------------- full-size graphs, sampled
def _sampled_check(hb, g, p, depth, n_src=64, seed=0, order=None, reg4=False):
    """GPU run on the whole graph; the oracle recomputes sampled nodes from exact balls.
    reg4: also run with 4-bit registers, which must equal min(8-bit registers, 15)
    at every node after the same number of steps."""
    off, deg, data = hb.csr_encode(g.adj_offsets, g.adj_ids)
    # the oracle reads its own encoding of the graph (the same bytes, checked)
    csr = oracle.from_graph(g)
    assert np.array_equal(csr.offsets, off) and np.array_equal(csr.degrees, deg)
    assert np.array_equal(csr.bytes, data)
    results = {}
    with hb.graph_load(off, deg, data, order=order) as G:
        for kernel in ("runs", "edges") + (("groups",) if 8 <= p <= 12 else ()):
            results[kernel] = G.run(p, depth, seed, registers=True, kernel=kernel)
            print(f"[parity] {kernel}: passes={results[kernel].passes} "
                  f"iter_ms={results[kernel].iter_ms:.1f}", flush=True)
        if reg4:
            r4 = G.run(p, depth, seed, registers=True, register_bits=4)
            print(f"[parity] 4-bit: passes={r4.passes} iter_ms={r4.iter_ms:.1f}", flush=True)
            assert depth > 0 and r4.passes == results["runs"].passes == depth
            assert np.array_equal(hb.unpack_nibbles(r4.registers),
                                  np.minimum(results["runs"].registers, 15))
    res = results["runs"]
    T = res.passes
    assert depth == 0 or T <= depth
    for other in [k for k in results if k != "runs"]:
        assert results[other].passes == T, other
        assert np.array_equal(results[other].registers, res.registers), other
        assert np.array_equal(results[other].sum_d, res.sum_d), other
    src = np.sort(np.random.default_rng(99).choice(g.n, n_src, replace=False))
    src = np.unique(np.concatenate([src, [0, g.n - 1, int(np.argmax(deg)), int(np.argmin(deg))]]))
    regs, reach, sum_d, _ = oracle.sampled_hyperball(csr, src, T, p, seed)
    bad = np.nonzero((res.registers[src] != regs).any(axis=1))[0]
    assert bad.size == 0, f"registers differ at sampled nodes {src[bad][:8]}"
    np.testing.assert_allclose(res.reach[src], reach, rtol=RTOL, atol=0)
    np.testing.assert_allclose(res.sum_d[src], sum_d, rtol=RTOL, atol=1e-9)
    return res


@pytest.mark.slow
@pytest.mark.parametrize("p", [8, 10, 12])
def test_urban_sampled_depth3(hb, p):
    g = _urban_graph()
    print(f"[parity] urban n={g.n} E={g.n_edges} p={p} depth=3", flush=True)
    res = _sampled_check(hb, g, p, 3)
    assert res.passes == 3


@pytest.mark.slow
def test_urban_sampled_unlimited(hb):
    g = _urban_graph()
    print(f"[parity] urban n={g.n} E={g.n_edges} p=10 unlimited", flush=True)
    res = _sampled_check(hb, g, 10, 0, n_src=32)
    assert res.converged


_URBAN = {}


def _urban_graph():
    if "g" not in _URBAN:
        _URBAN["g"] = synth.urban(0, device="gpu")
    return _URBAN["g"]


_CITY = {}


def _city_graph():
    if "g" not in _CITY:
        _CITY["g"] = synth.city(0, device="gpu")
    return _CITY["g"]


@pytest.mark.slow
@pytest.mark.timeout(1200)
def test_city_sampled_bench_config(hb):
    """The benchmark's workload and launch configuration: city graph, p = 10, depth 3,
    Hilbert processing order, default schedule."""
    g = _city_graph()
    print(f"[parity] city n={g.n} E={g.n_edges} p=10 depth=3", flush=True)
    res = _sampled_check(hb, g, 10, 3, n_src=64, order=synth.hilbert_order(g), reg4=True)
    assert res.passes == 3
    # properties at any size: registers never below a node's own insert, values <= 65-p
    assert int(res.registers.max()) <= 55
    for v in np.random.default_rng(5).choice(g.n, 200, replace=False):
        j, r = oracle.hll_insert(int(v), 0, 10)
        assert res.registers[v, j] >= r


@pytest.mark.slow
@pytest.mark.timeout(1200)
def test_city_sampled_unlimited(hb):
    """The city graph without a depth limit (Hilbert order, p = 10): the run stops by
    the 0.5 rule of Alg. 1; sampled nodes against the oracle's exact balls after the
    same number of steps, and both union kernels agree at every node."""
    g = _city_graph()
    print(f"[parity] city n={g.n} E={g.n_edges} p=10 unlimited", flush=True)
    res = _sampled_check(hb, g, 10, 0, n_src=48, order=synth.hilbert_order(g))
    print(f"[parity] city unlimited: passes={res.passes} converged={res.converged}", flush=True)
    assert res.converged and res.passes >= 4


def _has_edges(g, a, b):
    """Whether b is in row a, for arrays of pairs: a binary search inside each row."""
    lo = g.adj_offsets[a].astype(np.int64)
    hi = g.adj_offsets[a + 1].astype(np.int64)
    b = b.astype(np.uint32)
    while True:
        open_ = lo < hi
        if not open_.any():
            break
        mid = (lo + hi) // 2
        go_right = open_ & (g.adj_ids[np.minimum(mid, g.adj_ids.size - 1)] < b)
        lo = np.where(go_right, mid + 1, lo)
        hi = np.where(open_ & ~go_right, mid, hi)
    found = lo < g.adj_offsets[a + 1].astype(np.int64)
    found[found] = g.adj_ids[lo[found]] == b[found]
    return found


@pytest.mark.slow
@pytest.mark.timeout(1200)
def test_city_generator_spot_check(hb):
    """The city graph the GPU generator built against the CPU visibility rule: a million
    seeded node pairs and the whole rows of sampled nodes."""
    g = _city_graph()
    assert abs(g.n - 236000) / 236000 < 0.02
    rng = np.random.default_rng(2026)
    a = rng.integers(0, g.n, 1_000_000)
    b = rng.integers(0, g.n, 1_000_000)
    keep = a != b
    a, b = a[keep], b[keep]
    vis = synth.visible_pairs(g, a, b).astype(bool)
    got = _has_edges(g, a, b)
    print(f"[synth] city pairs={a.size} visible={int(vis.sum())}", flush=True)
    assert np.array_equal(got, vis)
    for s in rng.integers(0, g.n, 8):
        t = np.arange(g.n)
        t = t[t != s]
        want = t[synth.visible_pairs(g, np.full(t.size, s), t).astype(bool)]
        assert np.array_equal(g.row(int(s)), want), s
