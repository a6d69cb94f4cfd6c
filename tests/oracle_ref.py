"""Oracle references for the GPU tests of the batched and served forms.

Every job of a batch and every served request is compared with the CPU oracle's
run of the same (graph, p, depth limit, hash seed, register width) -- Alg. 1 with
the Eq. 2 union, the HLL estimate and the Eq. 3 sums -- on top of the check that
it equals the same analysis run alone.  References are cached per analysis, so a
test that submits one analysis many times pays for one oracle run.
"""
import hashlib

import numpy as np

import oracle

RTOL = 1e-9

_CSR = {}
_REF = {}


def _graph_key(g):
    h = hashlib.sha1()
    h.update(np.ascontiguousarray(g.adj_offsets).tobytes())
    h.update(np.ascontiguousarray(g.adj_ids).tobytes())
    return (g.name, g.n, int(g.n_edges), h.hexdigest())


def _csr(gk, g):
    if gk not in _CSR:
        _CSR[gk] = oracle.from_graph(g)
    return _CSR[gk]


def ref(g, p, depth, seed, register_bits=8, hash_ids=None):
    """The oracle's run of one analysis (registers one per byte, 4-bit ones unpacked)."""
    hk = None if hash_ids is None else np.asarray(hash_ids, np.uint32).tobytes()
    gk = _graph_key(g)
    key = (gk, p, depth, seed, register_bits, hk)
    if key not in _REF:
        _REF[key] = oracle.hyperball(_csr(gk, g), p, depth, seed, hash_ids=hash_ids,
                                     register_bits=register_bits)
    return _REF[key]


def assert_matches(hb, res, ref_run, what):
    """A GPU result against the oracle: passes and convergence exactly, registers
    byte for byte (when the result carries them), reach and sums within 1e-9."""
    assert res.passes == ref_run.passes, (what, res.passes, ref_run.passes)
    assert bool(res.converged) == bool(ref_run.converged), (what, res.converged)
    assert res.productive_iters == ref_run.passes - int(ref_run.converged), what
    if res.registers is not None:
        regs = hb.unpack_nibbles(res.registers) if res.register_bits == 4 else res.registers
        bad = np.nonzero((regs != ref_run.registers).any(axis=1))[0]
        assert bad.size == 0, f"{what}: registers differ from the oracle at nodes {bad[:10]}"
    np.testing.assert_allclose(res.reach, ref_run.reach, rtol=RTOL, atol=0, err_msg=what)
    np.testing.assert_allclose(res.sum_d, ref_run.sum_d, rtol=RTOL, atol=1e-9, err_msg=what)
