"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: published code
vectors, closed forms, brute-force breadth-first search, statistical laws of the
estimator.  A plausible slip anywhere in the oracle (a dropped term, a wrong sign,
index, shift or constant) breaks at least one of them.
"""
import math
import os

import numpy as np
import pytest

import oracle
import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _rows(name):
    with open(os.path.join(GOLD, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                yield line.split()


# ------------------------------------------------------------------ LEB128 (Sec. 3.2)
def test_leb128_published_vectors():
    for val, hexb in _rows("leb128_vectors.txt"):
        v = int(val)
        assert oracle.uleb_encode(v).hex() == hexb, v
        assert oracle.uleb_decode(bytes.fromhex(hexb)) == (v, len(hexb) // 2)


def test_leb128_round_trip_random():
    rng = np.random.default_rng(7)
    vals = (rng.integers(0, 2**32, 2000).tolist() +
            [2 ** int(k) - 1 for k in rng.integers(0, 65, 500)] + [0, 1, 127, 128, 2**63])
    for v in vals:
        enc = oracle.uleb_encode(v)
        assert len(enc) == max(1, math.ceil(v.bit_length() / 7))
        assert oracle.uleb_decode(enc) == (v, len(enc))


def test_leb128_malformed():
    assert oracle.uleb_decode(bytes([0x80, 0x80]))[1] == 0  # ends inside a varint
    assert oracle.uleb_decode(b"")[1] == 0
    assert oracle.uleb_decode(bytes([0xFF] * 10 + [0x01]))[1] == -1  # more than 64 bits
    assert oracle.uleb_decode(bytes([0xFF] * 9 + [0x02]))[1] == -1  # bit 64 set


def test_row_size_model_of_the_paper():
    """13,800 one-byte deltas + 133 two-byte jumps ~ 14 KB vs 56 KB as u32 (Sec. 3.2)."""
    d = {k: int(v) for k, v in _rows("paper_row_model.txt")}
    ids, cur = [], 5000
    per_run = d["one_byte_deltas"] // (d["row_jumps"] + 1)
    for r in range(d["row_jumps"] + 1):
        for k in range(per_run):
            ids.append(cur)
            cur += 1 if k < per_run - 1 else 0
        cur += d["row_jump_delta"]
    while len(ids) < d["one_byte_deltas"] + d["row_jumps"]:
        ids.append(ids[-1] + 1)
    ids = np.unique(np.array(ids, np.uint32))
    n = int(ids.max()) + 2
    adj_off = np.zeros(n + 1, np.uint64)
    adj_off[n - 1 + 1:] = len(ids)
    csr = oracle.csr_encode(n, adj_off, ids)
    nbytes = int(csr.offsets[-1])
    raw = 4 * len(ids)
    assert abs(nbytes / 1000 - d["compressed_kb"]) < 0.5
    assert abs(raw / 1000 - d["uncompressed_kb"]) < 0.5
    assert round(raw / nbytes) == d["ratio"]
    assert np.array_equal(oracle.decode_row(csr, n - 1), ids)


def test_csr_round_trip_graphs():
    for g in (synth.tiny(0), synth.grid_graph(4, 48, 40), synth.star_graph(300)):
        csr = oracle.from_graph(g)
        assert int(csr.offsets[-1]) == csr.bytes.size
        assert np.array_equal(csr.degrees, g.degrees)
        for v in range(0, g.n, max(1, g.n // 97)):
            assert np.array_equal(oracle.decode_row(csr, v), g.row(v))


# ------------------------------------------------------------------ SplitMix64 (Sec. 3.3)
def test_splitmix64_published_sequence():
    gamma = 0x9E3779B97F4A7C15
    for k, out in _rows("splitmix64_seed0.txt"):
        k = int(k)
        assert oracle.splitmix64(((k - 1) * gamma) % 2**64) == int(out, 16)


def test_insert_index_and_rank():
    """Index = top p bits of the hash, rank = leading zeros of the rest + 1 (<= 65 - p)."""
    rng = np.random.default_rng(1)
    for v in rng.integers(0, 2**40, 300).tolist():
        for p in (4, 8, 10, 12, 16):
            seed = int(rng.integers(0, 2**63))
            j, r = oracle.hll_insert(v, seed, p)
            h = oracle.splitmix64(v ^ seed)
            assert j == h >> (64 - p)
            rest = (h << p) % 2**64
            lz = 64 - p if rest == 0 else 64 - rest.bit_length()
            assert r == min(lz, 64 - p) + 1
            assert 1 <= r <= 65 - p


def test_insert_rank_distribution():
    """P(rank = k) = 2^-k: the geometric law HLL's estimator assumes."""
    p = 10
    ranks = np.array([oracle.hll_insert(v, 99, p)[1] for v in range(200000)])
    for k in range(1, 8):
        frac = np.mean(ranks == k)
        assert abs(frac - 2.0 ** -k) < 5 * math.sqrt(2.0 ** -k / ranks.size), k
    idx = np.array([oracle.hll_insert(v, 99, 4)[0] for v in range(20000)])
    counts = np.bincount(idx, minlength=16)
    assert counts.min() > 20000 / 16 * 0.9


# ------------------------------------------------------------------ estimator (Sec. 2.3)
def test_alpha_constants():
    for p, a in _rows("hll_constants.txt"):
        assert oracle.hll_alpha(int(p)) == float(a)
    for p in range(7, 17):
        m = 2.0 ** p
        assert oracle.hll_alpha(p) == 0.7213 / (1 + 1.079 / m)


@pytest.mark.parametrize("p", [4, 6, 8, 10, 12, 16])
def test_estimator_closed_forms(p):
    m = 1 << p
    regs = np.zeros(m, np.uint8)
    assert oracle.hll_estimate(regs, p) == 0.0  # empty sketch: m ln(m/m)
    regs[m // 3] = 5
    assert oracle.hll_estimate(regs, p) == m * math.log(m / (m - 1))  # one element
    for k in (1, 3, 7, 65 - p):
        regs = np.full(m, k, np.uint8)  # no zero register: raw estimate alpha m 2^k
        assert oracle.hll_estimate(regs, p) == pytest.approx(oracle.hll_alpha(p) * m * 2.0 ** k,
                                                             rel=1e-15)


def test_estimator_linear_counting_switch():
    p, m = 8, 256
    # V zeros and the rest at 1: Z = V + (m - V)/2, E = alpha m^2 / Z
    for V in (1, 10, 100, 200, 255):
        regs = np.ones(m, np.uint8)
        regs[:V] = 0
        E = oracle.hll_alpha(p) * m * m / (V + (m - V) / 2)
        want = m * math.log(m / V) if E <= 2.5 * m else E
        assert oracle.hll_estimate(regs, p) == pytest.approx(want, rel=1e-14)
        assert oracle.hll_raw(regs, p) == (pytest.approx(E, rel=1e-14), V)
    # large registers with a zero: E > 2.5 m keeps the raw estimate
    regs = np.full(m, 20, np.uint8)
    regs[0] = 0
    E, V = oracle.hll_raw(regs, p)
    assert V == 1 and E > 2.5 * m
    assert oracle.hll_estimate(regs, p) == E


def test_exact_harmonic_sum():
    """S = sum 2^-M is formed exactly: a sum whose float accumulation would lose bits."""
    p, m = 12, 4096
    regs = np.full(m, 53, np.uint8)
    regs[0] = 1  # 0.5 + 4095 * 2^-53: a float running sum drops the small terms
    E, V = oracle.hll_raw(regs, p)
    exact = 0.5 + 4095 * 2.0 ** -53
    assert E == (oracle.hll_alpha(p) * m * m) / exact


@pytest.mark.parametrize("p", [6, 8, 10])
def test_estimator_statistics(p):
    """Raw-regime relative error: mean ~ 0, std ~ 1.04/sqrt(m) (Sec. 2.3)."""
    m = 1 << p
    n = 10 * m
    errs = []
    for trial in range(150 if p < 10 else 60):
        regs = np.zeros(m, np.uint8)
        for v in range(trial * n, (trial + 1) * n):  # a fresh set of n distinct ids per trial
            j, r = oracle.hll_insert(v, 0, p)
            if r > regs[j]:
                regs[j] = r
        errs.append(oracle.hll_estimate(regs, p) / n - 1)
    errs = np.array(errs)
    se = 1.04 / math.sqrt(m)
    assert abs(errs.mean()) < 4 * se / math.sqrt(len(errs)) + 0.01
    assert 0.7 * se < errs.std() < 1.35 * se


# ------------------------------------------------------------------ HyperBall (Alg. 1)
def _sum_dist(dist, depth=0):
    d = dist.astype(np.int64)
    keep = d > 0 if depth == 0 else (d > 0) & (d <= depth)
    return np.where(keep, d, 0).sum(axis=1).astype(np.float64)


@pytest.mark.parametrize("g", [synth.tiny(0), synth.tiny(5), synth.random_graph(120, 0.03, 2)],
                         ids=lambda g: g.name)
def test_exact_counters_give_bfs_distance_sums(g):
    """Eq. 1: with exact cardinalities the Eq. 3 accumulation equals BFS distance sums."""
    csr = oracle.from_graph(g)
    dist = oracle.bfs_all(csr)
    D = int(dist.max())
    ex = oracle.hyperball_exact(csr, 0)
    assert np.array_equal(ex.sum_d, _sum_dist(dist))
    assert np.array_equal(ex.reach, (dist >= 0).sum(axis=1).astype(float))
    assert ex.passes == D + 1 and ex.converged
    for d in (1, 2, 3):
        exd = oracle.hyperball_exact(csr, d)
        assert np.array_equal(exd.sum_d, _sum_dist(dist, d))
        assert exd.passes == min(d, D + 1)


@pytest.mark.parametrize("maker,n", [(synth.path_graph, 25), (synth.cycle_graph, 24),
                                     (synth.cycle_graph, 25), (synth.star_graph, 30),
                                     (synth.complete_graph, 20)])
def test_closed_form_distance_sums(maker, n):
    g = maker(n)
    ex = oracle.hyperball_exact(oracle.from_graph(g), 0)
    i = np.arange(n)
    if maker is synth.path_graph:
        want = i * (i + 1) / 2 + (n - 1 - i) * (n - i) / 2
        D = n - 1
    elif maker is synth.cycle_graph:
        want = np.full(n, (n * n) // 4)
        D = n // 2
    elif maker is synth.star_graph:
        want = np.where(i == 0, n - 1, 2 * n - 3)
        D = 2
    else:
        want = np.full(n, n - 1)
        D = 1
    assert np.array_equal(ex.sum_d, want.astype(float))
    assert ex.passes == D + 1


def test_hll_registers_equal_exact_ball_registers():
    """Step-t registers of v are the union of the inserts of B(v, t) (Eq. 2 by induction)."""
    g = synth.tiny(4)
    csr = oracle.from_graph(g)
    dist = oracle.bfs_all(csr)
    full = oracle.hyperball(csr, 8, 0, seed=3)
    for t in range(1, full.passes + 1):
        r = oracle.hyperball(csr, 8, t, seed=3)
        assert r.passes == t
        for v in range(g.n):
            assert np.array_equal(r.registers[v], oracle.ball_registers(dist[v], t, 8, 3)), (t, v)


def test_registers_monotone_and_fixed_after_diameter():
    g = synth.tiny(6)
    csr = oracle.from_graph(g)
    D = int(oracle.bfs_all(csr).max())
    prev = oracle.initial_registers(g.n, 10, 0)
    for t in range(1, D + 3):
        r = oracle.hyperball(csr, 10, t, seed=0)
        if r.passes < t:
            break
        assert (r.registers >= prev).all()
        if t > D:
            assert np.array_equal(r.registers, prev)
        prev = r.registers


def test_union_order_free():
    """Max-union is commutative and idempotent: reversed rows and doubled neighbours agree."""
    g = synth.tiny(7)
    csr = oracle.from_graph(g)
    n = g.n
    perm = np.arange(n)[::-1].copy()  # relabel v -> n-1-v (rows decode in reversed order)
    inv = np.argsort(perm)
    rows = [np.sort(perm[g.row(int(inv[v]))]) for v in range(n)]
    off = np.zeros(n + 1, np.uint64)
    off[1:] = np.cumsum([len(r) for r in rows])
    g2 = synth.Graph(n, off, np.concatenate(rows).astype(np.uint32), g.obst, g.xy)
    a = oracle.hyperball(csr, 8, 3, seed=11)
    # relabelling changes the hashes, so compare the multiset of exact ball sizes instead
    ex1 = oracle.hyperball_exact(csr, 3)
    ex2 = oracle.hyperball_exact(oracle.from_graph(g2), 3)
    assert np.array_equal(ex1.reach, ex2.reach[perm])
    assert a.passes == 3


def test_complete_graph_converges_in_two_passes():
    g = synth.complete_graph(64)
    for p in (4, 8, 12):
        r = oracle.hyperball(oracle.from_graph(g), p, 0, seed=1)
        assert r.passes == 2 and r.converged
        assert (r.registers == r.registers[0]).all()


def test_sampled_balls_match_full_iteration():
    """Multi-source BFS balls reproduce the full iteration's registers, reach and sums."""
    g = synth.grid_graph(2, 40, 40)
    csr = oracle.from_graph(g)
    T = 3
    full = oracle.hyperball(csr, 10, T, seed=5)
    src = np.arange(0, g.n, 37)
    regs, reach, sum_d, _ = oracle.sampled_hyperball(csr, src, T, 10, seed=5)
    assert np.array_equal(regs, full.registers[src])
    assert np.array_equal(reach, full.reach[src])
    assert np.array_equal(sum_d, full.sum_d[src])


def test_hll_distance_sums_within_error_bound():
    """HLL reach and distance sums track exact BFS on the 1.04/sqrt(m) error scale.

    All nodes of one run share most of their hashed elements, so their errors are
    correlated and the scale is checked over independent hash seeds.  The final
    reach estimates the component size with the HLL error (the raw estimator carries
    a known positive bias just above the 2.5 m switch, so 1.5 SE is allowed); the
    Eq. 3 sum T c_T - sum_{t<T} c_t weights the final estimate by T, so its relative
    error is larger by about T / MD and is held to 2.5 SE.
    """
    g = synth.grid_graph(1, 64, 64)
    csr = oracle.from_graph(g)
    dist = oracle.bfs_all(csr)
    want = _sum_dist(dist)
    for p in (8, 10):
        se = 1.04 / math.sqrt(1 << p)
        med, reach_err = [], []
        for seed in range(12):
            r = oracle.hyperball(csr, p, 0, seed=seed * 7919 + 1)
            med.append(np.median(np.abs(r.sum_d / want - 1)))
            reach_err.append(r.reach[0] / g.n - 1)
        assert math.sqrt(np.mean(np.square(reach_err))) < 1.5 * se
        assert np.mean(med) < 2.5 * se


# ------------------------------------------------------------------ reordering (Sec. 3.2)
def test_relabelled_graph_with_original_hash_ids_permutes_the_results():
    """Renumbering the nodes and hashing their original ids permutes every output.

    Node i of the renumbered graph is node perm[i] of the original; its ball is the
    image of the original ball, so with the original ids inserted its registers,
    estimates and sums must be those of perm[i], bit for bit.  Hashing the new ids
    instead must not give them at a depth limit (so the hash_ids input is really
    used).
    """
    g = synth.tiny(2)
    perm = np.random.default_rng(3).permutation(g.n).astype(np.uint32)
    h, orig = synth.relabel(g, perm)
    assert np.array_equal(orig, perm)
    for p, depth in ((8, 0), (10, 2)):
        a = oracle.hyperball(oracle.from_graph(g), p, depth, 5)
        b = oracle.hyperball(oracle.from_graph(h), p, depth, 5, hash_ids=orig)
        assert (a.passes, a.converged) == (b.passes, b.converged)
        assert np.array_equal(b.registers, a.registers[perm])
        assert np.array_equal(b.reach, a.reach[perm])
        assert np.array_equal(b.sum_d, a.sum_d[perm])
        if depth:  # a converged run's balls are the whole component under any numbering
            c = oracle.hyperball(oracle.from_graph(h), p, depth, 5)
            assert not np.array_equal(c.registers, a.registers[perm])


def test_identity_hash_ids_change_nothing():
    g = synth.tiny(4)
    a = oracle.hyperball(oracle.from_graph(g), 9, 0, 1)
    b = oracle.hyperball(oracle.from_graph(g), 9, 0, 1, hash_ids=np.arange(g.n, dtype=np.uint32))
    assert np.array_equal(a.registers, b.registers) and np.array_equal(a.sum_d, b.sum_d)


@pytest.mark.parametrize("bits", [1, 2, 3, 5])
def test_hilbert_index_is_a_curve_of_adjacent_cells(bits):
    """A bijection of the 2^bits x 2^bits grid onto 0..4^bits-1 whose steps are unit moves."""
    side = 1 << bits
    x, y = np.meshgrid(np.arange(side), np.arange(side))
    d = synth.hilbert_index(x.ravel(), y.ravel(), bits)
    assert np.array_equal(np.sort(d), np.arange(side * side))
    order = np.argsort(d)
    steps = np.abs(np.diff(x.ravel()[order])) + np.abs(np.diff(y.ravel()[order]))
    assert np.all(steps == 1)
    assert d[0] == 0  # the curve starts at the origin


def test_hilbert_order_is_a_permutation():
    g = synth.grid_graph(3, 40, 30)
    o = synth.hilbert_order(g)
    assert np.array_equal(np.sort(o), np.arange(g.n))


# ------------------------------------------------------------------ 4-bit registers (Sec. 3.4)
def _high_rank_ids(p, seed, count, rank=16):
    """Ids whose inserted rank is at least `rank` (found by search), to force saturation."""
    out, x = [], 0
    while len(out) < count:
        if oracle.hll_insert(x, seed, p)[1] >= rank:
            out.append(x)
        x += 1
    return out


def test_4bit_registers_are_the_8bit_registers_clamped_at_15():
    """max commutes with min(., 15), so after any step R4 = min(R8, 15), byte for byte.

    Some nodes insert elements of rank >= 16 (chosen through hash_ids), so the clamp
    really acts; the 8-bit run is stopped at the step where the 4-bit run stopped.
    """
    g = synth.grid_graph(5, 40, 30)
    p, seed = 8, 3
    special = _high_rank_ids(p, seed, 12)
    hid = np.arange(g.n, dtype=np.uint32) + np.uint32(10 ** 6)
    rng = np.random.default_rng(2)
    hid[rng.choice(g.n, size=len(special), replace=False)] = special
    csr = oracle.from_graph(g)
    for depth in (0, 2):
        r4 = oracle.hyperball(csr, p, depth, seed, hash_ids=hid, register_bits=4)
        r8 = oracle.hyperball(csr, p, r4.passes, seed, hash_ids=hid)
        assert r8.registers.max() >= 16  # the clamp matters in this case
        assert r4.registers.max() == 15
        assert np.array_equal(r4.registers, np.minimum(r8.registers, 15))
        # the estimator is the same formula over the clamped registers
        est = np.array([oracle.hll_estimate(row, p) for row in r4.registers])
        assert np.array_equal(est, r4.reach)


def test_4bit_equals_8bit_when_no_rank_exceeds_15():
    g = synth.tiny(6)
    csr = oracle.from_graph(g)
    a = oracle.hyperball(csr, 10, 0, 0)
    if a.registers.max() > 15:
        pytest.skip("a rank above 15 occurs on this graph")
    b = oracle.hyperball(csr, 10, 0, 0, register_bits=4)
    assert np.array_equal(a.registers, b.registers)
    assert np.array_equal(a.sum_d, b.sum_d) and a.passes == b.passes


# ------------------------------------------------------------------ VGA metrics (Sec. 3.3)
def _exact_sums(g):
    csr = oracle.from_graph(g)
    return csr, oracle.hyperball_exact(csr).sum_d


def test_vga_metrics_star_closed_forms():
    """Star of n nodes: centre k = n-1, control n-1, MD 1, RA 0; leaf k = 1,
    control 1/(n-1), MD (2n-3)/(n-1), RA 2/(n-1)."""
    n = 9
    csr, sd = _exact_sums(synth.star_graph(n))
    m = oracle.vga_metrics(csr, sd)
    assert m["connectivity"][0] == n - 1 and np.all(m["connectivity"][1:] == 1)
    assert m["control"][0] == n - 1
    np.testing.assert_allclose(m["control"][1:], 1.0 / (n - 1), rtol=1e-15)
    assert m["mean_depth"][0] == 1.0 and m["relative_asymmetry"][0] == 0.0
    assert m["integration_pvalue"][0] == 1.0 and m["integration_tekl"][0] == 0.0
    assert np.isinf(m["integration_hh"][0])
    np.testing.assert_allclose(m["mean_depth"][1:], (2 * n - 3) / (n - 1), rtol=1e-15)
    np.testing.assert_allclose(m["relative_asymmetry"][1:], 2 / (n - 1), rtol=1e-14)
    np.testing.assert_allclose(m["integration_pvalue"][1:], 1 - 2 / (n - 1), rtol=1e-14)
    np.testing.assert_allclose(m["point_first_moment"], m["mean_depth"] * m["connectivity"])


def test_vga_metrics_complete_and_path():
    csr, sd = _exact_sums(synth.complete_graph(7))
    m = oracle.vga_metrics(csr, sd)
    np.testing.assert_allclose(m["control"], 1.0, rtol=1e-15)  # six neighbours of degree 6
    assert np.all(m["relative_asymmetry"] == 0.0)
    n = 12
    csr, sd = _exact_sums(synth.path_graph(n))
    m = oracle.vga_metrics(csr, sd)
    # ends: one neighbour of degree 2; next to an end: 1/1 + 1/2; interior: 1/2 + 1/2
    np.testing.assert_allclose(m["control"][[0, -1]], 0.5)
    np.testing.assert_allclose(m["control"][[1, -2]], 1.5)
    np.testing.assert_allclose(m["control"][2:-2], 1.0)
    i = np.arange(n)
    md = (i * (i + 1) / 2 + (n - 1 - i) * (n - i) / 2) / (n - 1)
    np.testing.assert_allclose(m["mean_depth"], md, rtol=1e-15)
    np.testing.assert_allclose(m["integration_tekl"], np.log2((md + 2) / 3), rtol=1e-14)


def _diamond(levels):
    """Justified 'diamond': levels of 1, 2, 4, ..., 4, 2, 1 nodes, each level joined
    completely to the next, so the root's depth of a node is its level."""
    sizes = [2 ** i for i in range(levels + 1)] + [2 ** i for i in range(levels - 1, -1, -1)]
    start = np.cumsum([0] + sizes)
    edges = [(a, b) for L in range(len(sizes) - 1)
             for a in range(start[L], start[L + 1]) for b in range(start[L + 1], start[L + 2])]
    return synth.from_edges(int(start[-1]), edges, name=f"diamond{int(start[-1])}")


@pytest.mark.parametrize("levels", [1, 2, 3, 4])
def test_integration_hh_is_one_at_the_root_of_a_diamond(levels):
    """Hillier & Hanson's D_k is the RA of the root of the k-node diamond, so there
    RRA = 1 and integration [HH] = 1 (k = 4, 10, 22, 46)."""
    csr, sd = _exact_sums(_diamond(levels))
    m = oracle.vga_metrics(csr, sd)
    np.testing.assert_allclose(m["integration_hh"][0], 1.0, rtol=1e-13)
    assert m["integration_hh"][-1] == pytest.approx(1.0, rel=1e-13)  # the other apex


def test_vga_metrics_small_components_are_nan():
    csr, sd = _exact_sums(synth.from_edges(3, [(0, 1)]))
    m = oracle.vga_metrics(csr, sd, comp_size=np.array([2, 2, 1], np.uint32))
    assert m["mean_depth"][0] == 1.0 and np.isnan(m["relative_asymmetry"][0])
    assert np.isnan(m["mean_depth"][2]) and m["connectivity"][2] == 0 and m["control"][2] == 0


# ------------------------------------------------- local metrics (Sec. 3.3, exact)
def _adjacency(g):
    A = np.zeros((g.n, g.n), np.int64)
    for v in range(g.n):
        A[v, g.adj_ids[g.adj_offsets[v]:g.adj_offsets[v + 1]]] = 1
    return A


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_local_metrics_match_matrix_powers(seed):
    """On random graphs: the ordered adjacent neighbour pairs of v are the closed
    walks of length 3 through v, diag(A^3); the two-step ball is the support of
    row v of A + A^2, without v."""
    rng = np.random.default_rng(seed)
    n = 60
    pairs = rng.integers(0, n, size=(400 + 200 * seed, 2))
    g = synth.from_edges(n, [(int(a), int(b)) for a, b in pairs if a != b], name="rand")
    A = _adjacency(g)
    A2 = A @ A
    walks3 = np.diag(A2 @ A)
    reach = ((A + A2) > 0).astype(np.int64)
    np.fill_diagonal(reach, 0)
    k = A.sum(axis=1)
    m = oracle.local_metrics(oracle.from_graph(g))
    assert np.array_equal(m["pairs"], walks3)
    assert np.array_equal(m["ball2"], reach.sum(axis=1))
    ok = k >= 2
    np.testing.assert_allclose(m["clustering"][ok], walks3[ok] / (k[ok] * (k[ok] - 1)),
                               rtol=1e-15)
    assert np.all(np.isnan(m["clustering"][~ok]))
    np.testing.assert_allclose(m["controllability"], k / reach.sum(axis=1), rtol=1e-15)


def test_local_metrics_closed_forms():
    """K_n: clustering 1, controllability 1.  Star: centre 0 and 1; leaf NaN and
    1/(n-1).  Path: no links among neighbours; interior two-step ball of 4.
    Wheel (hub + rim cycle of r nodes): rim 2/3 and 1; hub 2/(r-1)."""
    m = oracle.local_metrics(oracle.from_graph(synth.complete_graph(7)))
    assert np.all(m["pairs"] == 30) and np.all(m["ball2"] == 6)
    assert np.all(m["clustering"] == 1.0) and np.all(m["controllability"] == 1.0)
    n = 9
    m = oracle.local_metrics(oracle.from_graph(synth.star_graph(n)))
    assert m["clustering"][0] == 0.0 and m["controllability"][0] == 1.0
    assert np.all(np.isnan(m["clustering"][1:])) and np.all(m["ball2"][1:] == n - 1)
    np.testing.assert_allclose(m["controllability"][1:], 1.0 / (n - 1), rtol=1e-15)
    m = oracle.local_metrics(oracle.from_graph(synth.path_graph(10)))
    assert np.all(m["pairs"] == 0)
    assert list(m["ball2"]) == [2, 3] + [4] * 6 + [3, 2]
    np.testing.assert_allclose(m["controllability"][2:-2], 0.5)
    r = 8
    edges = [(0, i) for i in range(1, r + 1)] + [(i, i % r + 1) for i in range(1, r + 1)]
    m = oracle.local_metrics(oracle.from_graph(synth.from_edges(r + 1, edges, name="wheel")))
    assert m["pairs"][0] == 2 * r and m["ball2"][0] == r
    np.testing.assert_allclose(m["clustering"][0], 2 / (r - 1), rtol=1e-15)
    assert np.all(m["pairs"][1:] == 4) and np.all(m["ball2"][1:] == r)
    np.testing.assert_allclose(m["clustering"][1:], 2 / 3, rtol=1e-15)
    np.testing.assert_allclose(m["controllability"][1:], 3 / r, rtol=1e-15)


def test_local_metrics_isolated_nodes_and_subsets():
    g = synth.from_edges(5, [(0, 1), (1, 2), (0, 2)], name="triangle+2")
    m = oracle.local_metrics(oracle.from_graph(g))
    assert list(m["pairs"]) == [2, 2, 2, 0, 0] and list(m["ball2"]) == [2, 2, 2, 0, 0]
    assert np.all(np.isnan(m["clustering"][3:])) and np.all(np.isnan(m["controllability"][3:]))
    g = synth.grid_graph(3, 40, 30)
    csr = oracle.from_graph(g)
    full = oracle.local_metrics(csr)
    sub = np.array([g.n - 1, 0, 17, 17, g.n // 2], np.uint32)
    part = oracle.local_metrics(csr, nodes=sub)
    for key in ("pairs", "ball2"):
        assert np.array_equal(part[key], full[key][sub])


# ------------------------------------------------ the CPU-baseline unit (one union step)
@pytest.mark.parametrize("which", ["tiny", "raster"])
def test_union_sample_is_step_one_of_the_iteration(which):
    """union_sample (one Eq. 2 union + estimate for listed nodes, the unit the CPU
    baseline times) started from the inserted counters equals step 1 of Alg. 1 at
    every node, equals the registers of the exact ball B(v, 1), and counts each
    listed node's directed edges once."""
    g = synth.tiny(0) if which == "tiny" else synth.grid_graph(3, 40, 30)
    p = 10 if which == "tiny" else 7
    csr = oracle.from_graph(g)
    cur = oracle.initial_registers(g.n, p, seed=0)
    nxt, est, edges = oracle.union_sample(csr, p, cur, np.arange(g.n))
    step1 = oracle.hyperball(csr, p, 1, 0)
    assert edges == g.n_edges
    assert np.array_equal(nxt, step1.registers)
    assert np.array_equal(est, step1.reach)
    dist = oracle.bfs_all(csr)
    for v in range(0, g.n, 5):
        assert np.array_equal(nxt[v], oracle.ball_registers(dist[v], 1, p, 0)), v
    # a shuffled subset comes back in list order, with only its own edges counted
    sub = np.random.default_rng(4).permutation(g.n)[:57]
    nxt2, est2, edges2 = oracle.union_sample(csr, p, cur, sub)
    assert edges2 == int(g.degrees[sub].sum())
    assert np.array_equal(nxt2, step1.registers[sub])
    assert np.array_equal(est2, step1.reach[sub])


def test_union_sample_keeps_the_own_counter_and_every_neighbour():
    """From arbitrary counters: the result is the byte-wise max over v and all of its
    neighbours.  Isolating one register per node shows that neither v's own counter
    nor any single neighbour is dropped."""
    g = synth.random_graph(120, 0.05, seed=8)
    p = 7
    m = 1 << p
    csr = oracle.from_graph(g)
    nodes = np.arange(g.n)
    # node u holds a single register: index u mod m, value 1 + u // m
    cur = np.zeros((g.n, m), np.uint8)
    cur[nodes, nodes % m] = 1 + nodes // m
    nxt, _, _ = oracle.union_sample(csr, p, cur, nodes)
    for v in range(g.n):
        members = [v] + list(g.adj_ids[g.adj_offsets[v]:g.adj_offsets[v + 1]])
        want = np.zeros(m, np.uint8)
        for u in members:
            want[u % m] = max(want[u % m], 1 + u // m)
        assert np.array_equal(nxt[v], want), v


# ------------------------------------------------ point second moment (Sec. 3.3)
def _sq_sum(i, L):
    """sum over cells j != i of a line of L cells of (j - i)^2, in closed form."""
    a, b = i, L - 1 - i
    return a * (a + 1) * (2 * a + 1) // 6 + b * (b + 1) * (2 * b + 1) // 6


@pytest.mark.parametrize("L", [1, 2, 7, 40])
def test_point_second_moment_corridor(L):
    """A straight corridor one cell wide: every cell sees every other one, so cell i
    has sum over j of (j - i)^2."""
    g = synth.graph_from_raster(np.zeros((1, L), np.uint8), name=f"corridor{L}")
    assert g.n == L and g.n_edges == L * (L - 1)
    psm = oracle.point_second_moment(oracle.from_graph(g), g.xy)
    want = [_sq_sum(int(x), L) for x in g.xy[:, 0]]
    assert np.array_equal(psm, np.asarray(want, np.float64))


@pytest.mark.parametrize("a,b", [(5, 5), (6, 3)])
def test_point_second_moment_rectangular_room(a, b):
    """An open a x b room: every cell sees all others; the moment splits into the x and
    y sums, b S_a(x) + a S_b(y)."""
    g = synth.graph_from_raster(np.zeros((b, a), np.uint8), name=f"room{a}x{b}")
    assert g.n == a * b and g.n_edges == a * b * (a * b - 1)
    psm = oracle.point_second_moment(oracle.from_graph(g), g.xy)
    want = [b * _sq_sum(int(x), a) + a * _sq_sum(int(y), b) for x, y in g.xy]
    assert np.array_equal(psm, np.asarray(want, np.float64))


def test_point_second_moment_by_brute_force():
    """Tiny graph with obstacles: each node against its own neighbour list."""
    g = synth.tiny(2)
    psm = oracle.point_second_moment(oracle.from_graph(g), g.xy)
    for v in range(0, g.n, 3):
        d = g.xy[g.row(v)].astype(np.int64) - g.xy[v].astype(np.int64)
        assert psm[v] == float((d * d).sum()), v
