"""Summaries of rocprofv3 output for the HyperBall kernels.

Reads the CSV output of three rocprofv3 runs of the same command -- one with
``--kernel-trace --stats``, one with ``--pmc FETCH_SIZE``, one with ``--pmc WRITE_SIZE``
-- and writes a short text summary: per-kernel call counts and average durations,
the byte counters per dispatch, the counter scale factors measured on the library's
plain copy kernel (which moves a known number of bytes), and the resulting bytes per
union launch between L2 and the memory fabric.  FETCH_SIZE and WRITE_SIZE count L2
misses and write-backs; the 256 MB Infinity Cache on the fabric side serves part of
those reads, so they are fabric bytes, an upper bound on HBM bytes.  An optional
run of the TCC_EA0_*_DRAM counters gives the requests L2 sent towards DRAM.  The summary also records the SHA-256 of the kernel source it was
taken on, so a later benchmark reports the traffic only while the kernel is unchanged.

Usage:
    python -m paper_2604_08374_amd.profiling --trace DIR --fetch DIR --write DIR \\
        --copy-bytes N --cmd "..." --out profiles/NAME.md --counters profiles/NAME.txt
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import os
import re
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
# MI355X: 256 CUs x 4 SIMDs at 2.4 GHz; a wave64 VALU instruction takes 4 cycles
SIMDS = 256 * 4
CLOCK_HZ = 2.4e9
VALU_CYCLES = 4
KERNEL_SRC = os.path.join(HERE, "csrc", "hb_kernels.hip")


def _find(d: str, suffix: str) -> str:
    hits = sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True))
    if not hits:
        raise FileNotFoundError(f"no *{suffix} under {d}")
    return hits[0]


def _short(name: str) -> str:
    """Kernel name without namespaces and parameters: union_runs_kernel<10,64>.

    The union kernels are templates over Cfg<p, lanes per node> (and, batched,
    the kernel kind), shown as <p,lanes> or <p,lanes,true|false>.
    """
    for key in ("batch_union_kernel", "batch_groups_kernel", "batch_table_kernel",
                "batch_init_kernel", "batch_step_end_kernel", "union_groups_kernel",
                "union_runs_kernel", "union_kernel", "table_fused_kernel", "table_level_kernel",
                "gather_probe_kernel", "init_kernel", "copy_kernel", "fill_u32_kernel",
                "vis_rows_kernel", "local_rank_kernel", "local_kernel", "row_runs_kernel",
                "vga_kernel"):
        at = name.find(key)
        if at < 0 or (at > 0 and (name[at - 1].isalnum() or name[at - 1] == "_")):
            continue
        rest = name[at + len(key):]
        if not rest.startswith("<"):
            return key
        depth, end = 0, 0
        for k, ch in enumerate(rest):
            depth += ch == "<"
            depth -= ch == ">"
            if depth == 0:
                end = k
                break
        args = rest[1:end].replace("hbk::(anonymous namespace)::", "")
        args = re.sub(r"Cfg<([^>]*)>", r"\1", args).replace(" ", "")
        return f"{key}<{args}>"
    return name[:48]


def kernel_stats(trace_dir: str):
    rows = {}
    with open(_find(trace_dir, "kernel_stats.csv")) as f:
        for r in csv.DictReader(f):
            rows[_short(r["Name"])] = (int(r["Calls"]), float(r["AverageNs"]),
                                      float(r["TotalDurationNs"]))
    return rows


def counter_means(pmc_dir: str):
    acc = defaultdict(list)
    with open(_find(pmc_dir, "counter_collection.csv")) as f:
        for r in csv.DictReader(f):
            acc[(_short(r["Kernel_Name"]), r["Counter_Name"])].append(float(r["Counter_Value"]))
    return {k: (len(v), sum(v) / len(v)) for k, v in acc.items()}


def kernel_sha256(path: str = KERNEL_SRC) -> str:
    """SHA-256 of the kernel source without comments and blank lines, so that the
    counters stay attached to the code they were taken on, not to its comments."""
    code = []
    with open(path) as f:
        for line in f:
            line = line.split("//", 1)[0].rstrip()
            if line:
                code.append(line)
    return hashlib.sha256("\n".join(code).encode()).hexdigest()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--trace", required=True)
    ap.add_argument("--fetch", default=None)
    ap.add_argument("--write", default=None)
    ap.add_argument("--hit", default=None, help="optional --pmc TCC_HIT_sum TCC_MISS_sum run")
    ap.add_argument("--copy-bytes", type=int, default=0)
    ap.add_argument("--kernel", default="union_kernel<10>")
    ap.add_argument("--algo-bytes", type=int, default=0,
                    help="algorithmic bytes per launch of --kernel (from bench.py)")
    ap.add_argument("--cmd", action="append", default=[])
    ap.add_argument("--title", default="union kernel")
    ap.add_argument("--out", required=True)
    ap.add_argument("--counters", default=None)
    ap.add_argument("--sq", default=None,
                    help="optional --pmc run of SQ_INSTS_VALU SQ_INSTS_SALU SQ_INSTS_LDS "
                         "SQ_INSTS_VMEM_RD (instruction mix of --kernel)")
    ap.add_argument("--dram", default=None,
                    help="optional --pmc run of TCC_EA0_RDREQ_DRAM_sum TCC_EA0_RDREQ_DRAM_32B_sum "
                         "TCC_EA0_WRREQ_DRAM_sum (requests from L2 towards DRAM)")
    ap.add_argument("--node-order", default="raster",
                    help="processing order of the profiled run (recorded with the counters)")
    args = ap.parse_args()

    stats = kernel_stats(args.trace)
    if not (args.fetch and args.write):
        # trace only: the per-kernel table
        lines = [f"# rocprofv3 summary: {args.title}", ""]
        lines += ["Command (run from the repository root; writes CSV under the -d directory):", ""]
        lines += [f"    {c}" for c in args.cmd]
        lines += ["", "## Kernel trace (--kernel-trace --stats)", "",
                  "| kernel | calls | avg ms | total ms |", "|---|---|---|---|"]
        for name, (c, a, t) in sorted(stats.items(), key=lambda kv: -kv[1][2]):
            lines.append(f"| {name} | {c} | {a / 1e6:.3f} | {t / 1e6:.1f} |")
        lines += ["", f"* kernel source sha256 {kernel_sha256()}", ""]
        with open(args.out, "w") as f:
            f.write("\n".join(lines))
        print("\n".join(lines))
        return
    fetch = counter_means(args.fetch)
    write = counter_means(args.write)
    copy_kib = args.copy_bytes / 1024.0
    f_fetch = copy_kib / fetch[("copy_kernel", "FETCH_SIZE")][1]
    f_write = copy_kib / write[("copy_kernel", "WRITE_SIZE")][1]
    k = args.kernel
    calls, avg_ns, _ = stats[k]
    fetch_kib = fetch[(k, "FETCH_SIZE")][1]
    write_kib = write[(k, "WRITE_SIZE")][1]
    read_b = fetch_kib * 1024 * f_fetch
    write_b = write_kib * 1024 * f_write
    traffic = read_b + write_b
    sha = kernel_sha256()

    lines = [f"# rocprofv3 summary: {args.title}", ""]
    lines += ["Commands (run from the repository root; each writes CSV under its -d directory):", ""]
    lines += [f"    {c}" for c in args.cmd]
    lines += ["", "## Kernel trace (--kernel-trace --stats)", "",
              "| kernel | calls | avg ms | total ms |", "|---|---|---|---|"]
    for name, (c, a, t) in sorted(stats.items(), key=lambda kv: -kv[1][2]):
        lines.append(f"| {name} | {c} | {a / 1e6:.3f} | {t / 1e6:.1f} |")
    lines += ["", "## Byte counters per dispatch (KiB, mean over dispatches)", "",
              "| kernel | FETCH_SIZE | WRITE_SIZE |", "|---|---|---|"]
    names = sorted({n for n, _ in fetch} | {n for n, _ in write})
    for n in names:
        fv = fetch.get((n, "FETCH_SIZE"), (0, float("nan")))[1]
        wv = write.get((n, "WRITE_SIZE"), (0, float("nan")))[1]
        lines.append(f"| {n} | {fv:.1f} | {wv:.1f} |")
    lines += ["", "## Derived", "",
              f"* copy kernel moves {args.copy_bytes} B each way per dispatch: FETCH_SIZE scale "
              f"{f_fetch:.4f}, WRITE_SIZE scale {f_write:.4f}",
              f"* {k}: average duration {avg_ns / 1e6:.3f} ms over {calls} calls",
              f"* {k}: L2-to-fabric read {read_b / 1e12:.4f} TB + write {write_b / 1e12:.4f} TB = "
              f"{traffic / 1e12:.4f} TB per launch -> {traffic / (avg_ns * 1e-9) / 1e9:.0f} GB/s"]
    dram = {}
    if args.dram:
        dc = counter_means(args.dram)
        for c in ("TCC_EA0_RDREQ_DRAM_sum", "TCC_EA0_RDREQ_DRAM_32B_sum", "TCC_EA0_WRREQ_DRAM_sum"):
            if (k, c) in dc:
                dram[c] = dc[(k, c)][1]
        if "TCC_EA0_RDREQ_DRAM_32B_sum" in dram:
            # the 32-byte count covers every sector read towards DRAM (a 128-byte line
            # counts four); the Infinity Cache sits on that side, so these are the same
            # fabric bytes, not HBM bytes alone
            rd = 32.0 * dram["TCC_EA0_RDREQ_DRAM_32B_sum"]
            dram["dram_read_bytes"] = rd
            lines.append(f"* {k}: reads towards DRAM {dram.get('TCC_EA0_RDREQ_DRAM_sum', 0):.4g} "
                         f"requests, {dram['TCC_EA0_RDREQ_DRAM_32B_sum']:.4g} 32-byte sectors = "
                         f"{rd / 1e12:.4f} TB per launch ({rd / read_b:.3f} of the FETCH_SIZE "
                         f"bytes: every L2 miss goes to the memory side)")
    if args.hit:
        hit = counter_means(args.hit)
        h = hit.get((k, "TCC_HIT_sum"), (0, 0.0))[1]
        mi = hit.get((k, "TCC_MISS_sum"), (0, 0.0))[1]
        if h + mi > 0:
            lines.append(f"* {k}: L2 hits {h:.4g}, misses {mi:.4g} per launch -> hit rate "
                         f"{h / (h + mi):.3f}")
    if args.algo_bytes:
        lines.append(f"* algorithmic bytes per launch {args.algo_bytes / 1e12:.4f} TB; measured "
                     f"traffic / algorithmic = {traffic / args.algo_bytes:.3f}")
    mix = {}
    if args.sq:
        sq = counter_means(args.sq)
        for c in ("SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_LDS", "SQ_INSTS_VMEM_RD"):
            if (k, c) in sq:
                mix[c] = sq[(k, c)][1]
        if "SQ_INSTS_VALU" in mix:
            # a wave64 VALU instruction occupies a SIMD for 4 cycles
            t_valu = mix["SQ_INSTS_VALU"] * VALU_CYCLES / (SIMDS * CLOCK_HZ)
            lines.append(f"* {k}: wave instructions per launch: " + ", ".join(
                f"{c[9:]} {v:.4g}" for c, v in mix.items()) +
                f"; VALU issue alone needs {t_valu * 1e3:.1f} ms "
                f"({t_valu / (avg_ns * 1e-9):.2f} of the launch)")
    lines += [f"* kernel source sha256 {sha}", ""]
    with open(args.out, "w") as f:
        f.write("\n".join(lines))
    with open(args.counters, "w") as f:
        f.write(f"kernel {k}\n")
        f.write(f"node_order {args.node_order}\n")
        f.write(f"kernel_source_sha256 {sha}\n")
        f.write(f"avg_launch_ns {avg_ns:.0f}\n")
        f.write(f"fetch_kib_per_launch {fetch_kib:.3f}\n")
        f.write(f"write_kib_per_launch {write_kib:.3f}\n")
        f.write(f"fetch_scale {f_fetch:.6f}\n")
        f.write(f"write_scale {f_write:.6f}\n")
        f.write(f"fabric_bytes_per_launch {traffic:.0f}\n")
        if "dram_read_bytes" in dram:
            f.write(f"dram_read_bytes_per_launch {dram['dram_read_bytes']:.0f}\n")
        for c, v in mix.items():
            f.write(f"{c.lower()}_per_launch {v:.0f}\n")
    print("\n".join(lines))


if __name__ == "__main__":
    main()
