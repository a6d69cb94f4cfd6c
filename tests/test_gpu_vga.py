"""VGA metrics (hb_vga_metrics) against the oracle's formulas on the same sums.

Connectivity is exact; control is a sum of reciprocals in another order (lanes,
then a butterfly) and the log2-based metrics use the device's log2, so those are
compared within 1e-12 relative.  NaN and infinity must sit at the same nodes.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _compare(got, ref, what):
    for name in oracle.VGA_METRICS:
        a, b = got[name], ref[name]
        assert np.array_equal(np.isnan(a), np.isnan(b)), (what, name)
        assert np.array_equal(np.isinf(a), np.isinf(b)), (what, name)
        ok = np.isfinite(b)
        if name == "connectivity":
            assert np.array_equal(a, b), (what, name)
        else:
            np.testing.assert_allclose(a[ok], b[ok], rtol=1e-12, atol=0, err_msg=f"{what} {name}")


@pytest.mark.parametrize("gname", ["tiny", "rect90x70", "star", "diamond", "urban"])
def test_vga_metrics_match_oracle(hb, gname):
    comp = None
    if gname == "tiny":
        g = synth.tiny(3)
    elif gname == "rect90x70":
        g = synth.grid_graph(8, 90, 70)
    elif gname == "star":
        g = synth.star_graph(300)
    elif gname == "diamond":
        sizes = [1, 2, 4, 8, 16, 8, 4, 2, 1]
        start = np.cumsum([0] + sizes)
        edges = [(a, b) for L in range(len(sizes) - 1)
                 for a in range(start[L], start[L + 1]) for b in range(start[L + 1], start[L + 2])]
        g = synth.from_edges(int(start[-1]), edges, name="diamond")
    else:
        g = synth.urban(0, device="gpu")
    off, deg, data = hb.csr_encode(g.adj_offsets, g.adj_ids)
    raster = gname in ("tiny", "rect90x70", "urban")  # cells with coordinates
    G = hb.graph_load(off, deg, data, comp_size=comp, order=synth.hilbert_order(g),
                      xy=g.xy if raster else None)
    psm = oracle.point_second_moment(oracle.from_graph(g), g.xy) if raster else None
    for p, depth in ((10, 0), (8, 3)):
        r = G.run(p, depth, 1)
        print(f"[vga] {g.name} p={p} d={depth}", flush=True)
        got = G.vga_metrics(r.sum_d)
        ref = oracle.vga_metrics(oracle.from_graph(g), r.sum_d, comp)
        _compare(got, ref, f"{g.name} p={p} d={depth}")
        np.testing.assert_allclose(got["mean_depth"], r.mean_depth, rtol=1e-15)
        # the point second moment is an exact integer sum: equal bit for bit
        if raster:
            assert np.array_equal(got["point_second_moment"], psm), g.name
        else:
            assert np.isnan(got["point_second_moment"]).all(), g.name
    G.free()


def test_vga_metrics_with_component_sizes(hb):
    """Isolated nodes and small components: NaN where a formula has no meaning."""
    g = synth.from_edges(8, [(0, 1), (1, 2), (3, 4)])
    comp = np.array([3, 3, 3, 2, 2, 1, 1, 1], np.uint32)
    off, deg, data = hb.csr_encode(g.adj_offsets, g.adj_ids)
    G = hb.graph_load(off, deg, data, comp_size=comp)
    r = G.run(10, 0, 0)
    got = G.vga_metrics(r.sum_d)
    ref = oracle.vga_metrics(oracle.from_graph(g), r.sum_d, comp)
    _compare(got, ref, "components")
    assert np.isnan(got["relative_asymmetry"][3]) and np.isnan(got["mean_depth"][7])
    G.free()
