"""Host-side checks of the C ABI (no GPU needed): exports, encoding, validation, errors."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import oracle
import paper_2604_08374_amd as hb
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names |= set(re.findall(r"^\s*(?:const\s+)?[\w]+\s*\**\s*(hb_\w+)\s*\(", text, flags=re.M))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    names = _declared_functions()
    assert {"hb_graph_load", "hb_run", "hb_csr_encode", "hb_csr_validate"} <= set(names)
    lib = ctypes.CDLL(hb.lib_path())
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    out = subprocess.run(["nm", "-D", "--defined-only", hb.lib_path()], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (hb_\w+)", out))
    assert set(names) <= exported


def test_version_and_errors_without_gpu_are_clean():
    assert "gfx950" in hb.version()
    assert hb.device_count() >= 0


@pytest.mark.parametrize("g", [synth.tiny(0), synth.grid_graph(3, 64, 50), synth.star_graph(200),
                               synth.random_graph(150, 0.05, 1), synth.from_edges(3, [])],
                         ids=lambda g: g.name or "empty3")
def test_encoder_matches_oracle_encoder(g):
    off, deg, data = hb.csr_encode(g.adj_offsets, g.adj_ids)
    ref = oracle.from_graph(g)
    assert np.array_equal(off, ref.offsets)
    assert np.array_equal(deg, ref.degrees)
    assert np.array_equal(data, ref.bytes)
    assert hb.csr_validate(off, deg, data) == (hb.HB_OK, 0)


def test_large_ids_round_trip_and_validate():
    """Ids up to 2^32-2 (5-byte varints): the oracle's coder and the library's validator."""
    ids = np.array([0, 1, 127, 128, 2**21, 2**28 + 5, 2**32 - 2], np.uint32)
    adj_off = np.zeros(4, np.uint64)
    adj_off[1:] = len(ids)
    csr = oracle.csr_encode(3, adj_off, ids)  # row 0 only; n is too large for dense arrays
    assert oracle.decode_row(csr, 0).tolist() == ids.tolist()
    row = csr.bytes.tolist()
    # first id absolute, then deltas 1, 126, 1, 2^21-128, 2^28-2^21+5, 2^32-2^28-7
    assert len(row) == 1 + 1 + 1 + 1 + 3 + 4 + 5
    # as node 1 of a graph with n = 2^32 - 1 nodes the row is valid: checked on a
    # one-row CSR where only the id bound matters
    off = np.array([0, 0, len(row)], np.uint64)
    deg = np.array([0, len(ids)], np.uint32)
    st, _ = hb.csr_validate(off, deg, np.array(row, np.uint8))
    assert st == hb.HB_ECORRUPT  # ids >= n = 2 and a self loop


def test_encoder_rejects_bad_adjacency():
    bad = [
        (np.array([0, 2, 2], np.uint64), np.array([1, 1], np.uint32)),  # repeated id
        (np.array([0, 2, 2], np.uint64), np.array([1, 0], np.uint32)),  # decreasing + self
        (np.array([0, 1, 1], np.uint64), np.array([5], np.uint32)),  # id >= n
        (np.array([0, 1, 2], np.uint64), np.array([1, 1], np.uint32)),  # self loop on node 1
    ]
    for off, ids in bad:
        with pytest.raises(hb.HBError) as e:
            hb.csr_encode(off, ids)
        assert e.value.status == hb.HB_EINVAL


def _tiny_csr():
    g = synth.tiny(1)
    off, deg, data = hb.csr_encode(g.adj_offsets, g.adj_ids)
    return g, off.copy(), deg.copy(), data.copy()


def _row_range(off, v):
    return int(off[v]), int(off[v + 1])


def test_validate_detects_each_corruption():
    g, off, deg, data = _tiny_csr()
    v = 17
    a, b = _row_range(off, v)

    def expect(o, d, x, node, n_edges=None):
        st, bad = hb.csr_validate(o, d, x, n_edges=n_edges)
        assert st == hb.HB_ECORRUPT
        assert bad == node

    # truncated varint: last byte of row v gets a continuation bit
    x = data.copy()
    x[b - 1] |= 0x80
    expect(off, deg, x, v)
    # repeated id: a delta of 0 (replace a one-byte delta with 0)
    x = data.copy()
    k = a + 1
    while x[k] & 0x80 or x[k - 1] & 0x80:
        k += 1
    x[k] = 0
    expect(off, deg, x, v)
    # degree mismatch
    d = deg.copy()
    d[v] += 1
    expect(off, d, data, v, n_edges=int(deg.sum()) + 1)
    # degree sum != n_edges
    expect(off, deg, data, g.n, n_edges=int(deg.sum()) + 1)
    # offsets not monotone
    o = off.copy()
    o[v + 1], o[v + 2] = o[v + 2], o[v + 1]
    st, bad = hb.csr_validate(o, deg, data)
    assert st == hb.HB_ECORRUPT
    # offsets[0] != 0
    o = off.copy()
    o[0] = 1
    assert hb.csr_validate(o, deg, data)[0] == hb.HB_ECORRUPT


def _one_row_csr(row_bytes, n, degree):
    """Node 0 holds row_bytes; the other n-1 nodes are isolated."""
    data = np.array(row_bytes, np.uint8)
    off = np.zeros(n + 1, np.uint64)
    off[1:] = len(row_bytes)
    deg = np.zeros(n, np.uint32)
    deg[0] = degree
    return off, deg, data


@pytest.mark.parametrize("row,n,degree,ok", [
    ([0x01, 0x01], 4, 2, True),                        # ids 1, 2
    ([0x01, 0x00], 4, 2, False),                       # repeated id
    ([0x00], 4, 1, False),                             # self loop (node 0)
    ([0x04], 4, 1, False),                             # id == n
    ([0x81, 0x80, 0x80, 0x80, 0x00], 4, 1, True),      # non-minimal 5-byte form of 1
    ([0x81, 0x80, 0x80, 0x80, 0x80, 0x00], 4, 1, False),  # 6-byte varint
    ([0xFF, 0xFF, 0xFF, 0xFF, 0x1F], 2**20, 1, False),  # value >= 2^32
    ([0x81], 4, 1, False),                             # truncated
    ([0x01, 0x01], 4, 1, False),                       # more varints than the degree
    ([0x01], 4, 2, False),                             # fewer varints than the degree
])
def test_validate_row_rules(row, n, degree, ok):
    off, deg, data = _one_row_csr(row, n, degree)
    st, bad = hb.csr_validate(off, deg, data)
    assert (st == hb.HB_OK) == ok, (row, st)
    if not ok:
        assert bad == 0


def test_run_argument_errors_without_graph():
    L = ctypes.CDLL(hb.lib_path())
    L.hb_run.argtypes = [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64,
                         ctypes.c_void_p]
    L.hb_run.restype = ctypes.c_int32
    assert L.hb_run(None, 10, 3, 0, None) == hb.HB_EINVAL
    L.hb_graph_free.argtypes = [ctypes.c_void_p]
    L.hb_graph_free.restype = ctypes.c_int32
    assert L.hb_graph_free(None) == hb.HB_EINVAL
    L.hb_copy_probe.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_void_p]
    L.hb_copy_probe.restype = ctypes.c_int32
    assert L.hb_copy_probe(15, 1, None) == hb.HB_EINVAL


def test_load_without_gpu_fails_loudly():
    if hb.device_count() > 0:
        pytest.skip("a GPU is present")
    g, off, deg, data = _tiny_csr()
    with pytest.raises(hb.HBError) as e:
        hb.graph_load(off, deg, data)
    assert e.value.status == hb.HB_EDEVICE


def test_set_options_checks_its_arguments():
    """hb_set_options is host-only: argument errors and the round trip need no GPU."""
    import paper_2604_08374_amd as hb

    try:
        for kw in (dict(stop_delta=-1.0),
                   dict(tune_seed=[dict(p=10, register_bits=8, union_kernel="runs", batched=0,
                                        log2_nodes=3, log2_rows_per_node=4, lanes_per_node=48,
                                        nodes_per_block=4, best_ms=1.0, default_ms=1.0)])):
            with pytest.raises(hb.HBError) as e:
                hb.set_options(**kw)
            assert e.value.status == hb.HB_EINVAL
        with pytest.raises(hb.HBError):
            hb.set_options(dev_alloc=lambda n: 0)
        hb.set_options(hbm_budget=1 << 30, stop_rule="depth", stop_delta=2.5)
        o = hb.get_options()
        assert o["hbm_budget"] == 1 << 30 and o["stop_rule"] == "depth"
        assert o["stop_delta"] == 2.5 and not o["hooks"] and o["stream"] == 0
    finally:
        hb.set_options()
    assert hb.get_options()["hbm_budget"] == 0
