"""4-bit packed registers (two per byte, saturating at 15) against the oracle.

Registers come back packed (low nibble = even register); they are unpacked and
compared with the oracle's 4-bit run byte for byte.  Some nodes insert ids whose
rank exceeds 15 (chosen through hash_ids), so saturation is exercised.
"""
import numpy as np
import pytest

import oracle
import oracle_ref
import synth

pytestmark = pytest.mark.gpu

RTOL = 1e-9


# the one 4-bit shape built for each p (hb.h): lanes per node
LANES4 = {5: 1, 6: 2, 7: 4, 8: 8, 9: 16, 10: 32, 11: 64, 12: 64, 13: 64, 14: 128, 15: 256,
          16: 512}


def _load(hb, g, **kw):
    off, deg, data = hb.csr_encode(g.adj_offsets, g.adj_ids)
    return hb.graph_load(off, deg, data, **kw)


def _high_rank_ids(p, seed, count):
    out, x = [], 0
    while len(out) < count:
        if oracle.hll_insert(x, seed, p)[1] >= 16:
            out.append(x)
        x += 1
    return out


def _hash_ids(g, p, seed, count=10):
    hid = np.arange(g.n, dtype=np.uint32) + np.uint32(5 * 10 ** 6)
    rng = np.random.default_rng(p)
    hid[rng.choice(g.n, size=count, replace=False)] = _high_rank_ids(p, seed, count)
    return hid


def _check(hb, res, ref, what):
    assert res.register_bits == 4, what
    assert res.passes == ref.passes and res.converged == ref.converged, what
    regs = hb.unpack_nibbles(res.registers)
    bad = np.nonzero((regs != ref.registers).any(axis=1))[0]
    assert bad.size == 0, f"{what}: registers differ at nodes {bad[:10]}"
    np.testing.assert_allclose(res.reach, ref.reach, rtol=RTOL, atol=0, err_msg=what)
    np.testing.assert_allclose(res.sum_d, ref.sum_d, rtol=RTOL, atol=1e-9, err_msg=what)


@pytest.mark.parametrize("p", [5, 8, 10, 11, 12, 13, 16])
def test_4bit_matches_oracle(hb, p):
    cases = [(synth.tiny(2), 0, 1), (synth.grid_graph(7, 80, 60), 3, 4)] if p <= 13 else \
        [(synth.tiny(2), 2, 1)]
    for g, depth, seed in cases:
        hid = _hash_ids(g, p, seed)
        ref = oracle.hyperball(oracle.from_graph(g), p, depth, seed, hash_ids=hid,
                               register_bits=4)
        assert ref.registers.max() == 15
        G = _load(hb, g, hash_ids=hid)
        kernels = (("runs", "edges") if p <= 12 else ("edges",)) + \
            (("groups",) if 9 <= p <= 12 else ())
        for kernel in kernels:
            for nb in ((4, 1) if p <= 11 and kernel != "groups" else (0,)):
                what = f"{g.name} p={p} d={depth} {kernel} nb={nb}"
                print(f"[reg4] {what}", flush=True)
                kw = {} if nb == 0 else dict(lanes_per_node=LANES4[p], nodes_per_block=nb)
                r = G.run(p, depth, seed, registers=True, kernel=kernel, register_bits=4,
                          tune="off", **kw)
                _check(hb, r, ref, what)
        G.free()


def test_4bit_clamps_the_8bit_registers(hb):
    """On the GPU too: 4-bit registers = min(8-bit registers, 15) at the same step."""
    g = synth.grid_graph(3, 70, 50)
    p, seed = 10, 2
    hid = _hash_ids(g, p, seed, 16)
    G = _load(hb, g, hash_ids=hid)
    r4 = G.run(p, 0, seed, registers=True, register_bits=4)
    r8 = G.run(p, r4.passes, seed, registers=True)
    assert r8.registers.max() >= 16
    assert np.array_equal(hb.unpack_nibbles(r4.registers), np.minimum(r8.registers, 15))
    # the grouped kernel at both widths
    g4 = G.run(p, 0, seed, registers=True, register_bits=4, kernel="groups")
    g8 = G.run(p, g4.passes, seed, registers=True, kernel="groups")
    assert g4.union_kernel == "groups" and g8.union_kernel == "groups"
    assert np.array_equal(g4.registers, r4.registers) and np.array_equal(g8.registers, r8.registers)
    G.free()


def test_4bit_batch_and_served(hb):
    graphs = [synth.tiny(0), synth.grid_graph(1, 60, 50), synth.tiny(4)]
    Gs = [_load(hb, g, order=synth.hilbert_order(g)) for g in graphs]
    jobs = [(G, p, d, 5 * i) for i, G in enumerate(Gs) for (p, d) in ((10, 0), (8, 3), (12, 2))]
    owners = [g for g in graphs for _ in range(3)]
    refs = [oracle_ref.ref(g, p, d, s, register_bits=4) for g, (G, p, d, s) in zip(owners, jobs)]
    single = [G.run(p, d, s, registers=True, register_bits=4, tune="off")
              for (G, p, d, s) in jobs]
    batched = hb.run_batch(jobs, registers=True, register_bits=4, tune="measure")
    for a, b, r, (G, p, d, s) in zip(single, batched, refs, jobs):
        assert b.register_bits == 4
        oracle_ref.assert_matches(hb, b, r, f"batched p={p} d={d} seed={s}")
        assert np.array_equal(a.registers, b.registers) and np.array_equal(a.sum_d, b.sum_d)
    hb.server_start()
    try:
        served = [hb.submit(G, p, d, s, registers=True, register_bits=4).wait()
                  for (G, p, d, s) in jobs]
    finally:
        hb.server_stop()
    for a, b, r, (G, p, d, s) in zip(single, served, refs, jobs):
        assert b.register_bits == 4
        oracle_ref.assert_matches(hb, b, r, f"served p={p} d={d} seed={s}")
        assert np.array_equal(a.registers, b.registers) and np.array_equal(a.sum_d, b.sum_d)
    hb.tune_clear()
    for G in Gs:
        G.free()


def test_4bit_argument_errors(hb):
    G = _load(hb, synth.tiny(1))
    for p, bits in ((4, 4), (10, 6)):
        with pytest.raises(hb.HBError) as e:
            G.run(p, 1, 0, register_bits=bits)
        assert e.value.status == hb.HB_EINVAL
    with pytest.raises(hb.HBError) as e:
        G.run(10, 1, 0, register_bits=4, lanes_per_node=64)  # only the default shape
    assert e.value.status == hb.HB_EINVAL
    G.free()
