"""The benchmark's byte models and counter bookkeeping, on the host (no GPU).

The roofline fractions the benchmark reports divide these byte counts by measured
times, so each model is checked against a count written out by hand for a small
case, and the counter files are attached to the kernel source they were taken on.
"""
import os

import pytest

import bench


def test_per_edge_bytes_are_the_survey_model():
    # one counter row per directed edge, the LEB128 stream, offsets, own row and
    # next row per node, and 32 bytes of FP64 state per node
    n, E, nbytes, p = 10, 40, 45, 6
    m = 1 << p
    want = E * m + nbytes + 8 * (n + 1) + n * (2 * m + 32)
    assert bench.algorithmic_bytes(n, E, nbytes, p) == want


def test_run_kernel_bytes_count_table_rows_and_the_run_list():
    n, E, nbytes, p, rows, runs = 10, 40, 45, 6, 17, 9
    m = 1 << p
    want = rows * m + 8 * runs + 8 * (n + 1) + n * (2 * m + 32)
    assert bench.algorithmic_bytes(n, E, nbytes, p, rows, 8, runs, "runs") == want


@pytest.mark.parametrize("bits", [8, 4])
def test_grouped_kernel_bytes(bits):
    # each distinct (row, mask) entry: its counter row, a 4-byte row index and a
    # 2-byte mask; 8 bytes of offsets per group of 16 nodes (plus one); per node:
    # next written and 32 bytes of state (its own row is among the entries)
    n, p, rows = 33, 6, 50
    m = (1 << p) * bits // 8
    groups = (n + 15) // 16
    want = rows * (m + 6) + 8 * (groups + 1) + n * (m + 32)
    assert bench.algorithmic_bytes(n, 0, 0, p, rows, bits, 0, "groups") == want


def test_fused_table_bytes_read_each_tile_with_its_halo():
    n, p, levels = 1500, 6, 3
    m = 1 << p
    writes = sum((n - (1 << k) + 1) * m for k in range(1, levels + 1))
    span = 512 + (1 << levels) - 1
    reads = sum(min(i0 + span, n) - i0 for i0 in range(0, n, 512)) * m
    assert bench.table_bytes(n, p, levels) == writes + reads
    # 8-bit rows of 1 KB: tiles of 256 rows
    m, levels = 1024, 8
    writes = sum((n - (1 << k) + 1) * m for k in range(1, levels + 1))
    span = 256 + (1 << levels) - 1
    reads = sum(min(i0 + span, n) - i0 for i0 in range(0, n, 256)) * m
    assert bench.table_bytes(n, 10, levels) == writes + reads
    # rows narrower than 64 bytes take the per-level kernel: two reads, one write
    assert bench.table_bytes(n, 5, levels, bits=4) == 3 * sum(
        (n - (1 << k) + 1) * 16 for k in range(1, levels + 1))


def test_counters_are_dropped_once_the_kernel_source_changes(tmp_path, monkeypatch):
    src = tmp_path / "kernels.hip"
    src.write_text("__global__ void k() {}\n// a comment\n")
    from paper_2604_08374_amd.profiling import kernel_sha256

    rec = tmp_path / "counters.txt"
    rec.write_text(f"kernel union_groups_kernel<10,64,8>\nnode_order hilbert\n"
                   f"kernel_source_sha256 {kernel_sha256(str(src))}\n"
                   f"avg_launch_ns 8000000\nfabric_bytes_per_launch 1000\n")
    monkeypatch.setattr(bench, "KERNEL_SRC", str(src))
    monkeypatch.setitem(bench.COUNTERS_FILES, "groups", str(rec))
    got = bench.kernel_traffic("city", 10, 3, "groups", "union_groups_kernel<10,64,8>", "hilbert")
    assert got == {"avg_launch_ns": 8000000.0, "fabric_bytes_per_launch": 1000.0}
    # comments do not count, code does
    src.write_text("__global__ void k() {}\n// another comment\n\n")
    assert bench.kernel_traffic("city", 10, 3, "groups", "union_groups_kernel<10,64,8>",
                                "hilbert") is not None
    src.write_text("__global__ void k() { int x; }\n")
    assert bench.kernel_traffic("city", 10, 3, "groups", "union_groups_kernel<10,64,8>",
                                "hilbert") is None
    # another workload, kernel or processing order reads no counters
    src.write_text("__global__ void k() {}\n")
    assert bench.kernel_traffic("urban", 10, 3, "groups", "union_groups_kernel<10,64,8>",
                                "hilbert") is None
    assert bench.kernel_traffic("city", 10, 3, "groups", "union_groups_kernel<10,32,4>",
                                "hilbert") is None
    assert bench.kernel_traffic("city", 10, 3, "groups", "union_groups_kernel<10,64,8>",
                                "raster") is None


def test_committed_counters_match_the_current_kernel_source():
    """The counter files the default benchmark line reads were taken on this source."""
    from paper_2604_08374_amd.profiling import kernel_sha256

    sha = kernel_sha256()
    for kind, path in bench.COUNTERS_FILES.items():
        with open(path) as f:
            rec = dict(line.split(None, 1) for line in f if line.strip())
        assert rec["kernel_source_sha256"].strip() == sha, (kind, os.path.basename(path))
