// Internal interface between the host runtime (hb_host.cpp) and the gfx950
// kernels (hb_kernels.hip).  Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace hbk {

// Grouped union kernel: nodes are taken in groups of kGroupNodes consecutive
// nodes of the processing order; group_waves(p, bits) waves share a group, each
// on a 512-byte slice of every counter (one wave on a 256-byte counter).  Built
// where a counter is 256 to 4096 bytes (group_ok): p = 8..12 with 8-bit
// registers, p = 9..12 with 4-bit.
constexpr uint32_t kGroupNodes = 16;
constexpr uint32_t kGroupSlice = 512;
constexpr uint32_t group_counter_bytes(int p, uint32_t bits) {
    return p < 1 || p > 16 ? 0u : (1u << p) * bits / 8u;
}
constexpr bool group_ok(int p, uint32_t bits) {
    return (bits == 8u || bits == 4u) && p <= 12 &&
           group_counter_bytes(p, bits) >= kGroupSlice / 2u;
}
// waves per group: one per 512-byte slice (a 256-byte counter takes one wave)
constexpr uint32_t group_waves(int p, uint32_t bits) {
    return group_counter_bytes(p, bits) > kGroupSlice ? group_counter_bytes(p, bits) / kGroupSlice
                                                      : 1u;
}
using GroupMask = std::conditional<(kGroupNodes <= 16), uint16_t, uint32_t>::type;
static_assert(kGroupNodes <= 32, "a mask is at most 32 bits");

// One job of a batched run, in device memory.  The host fills every field
// before the first step; the step-end kernel advances t, done and converged.
struct BatchJob {
    const uint8_t *bytes;     // LEB128 stream
    const uint64_t *offsets;  // n + 1 row offsets
    const uint2 *run_list;    // run list of the rows, v joined in (run kernel)
    const uint64_t *run_off;  // n + 1 offsets into runs
    const uint32_t *order;    // processing order (a permutation of 0..n-1) or null
    const uint32_t *hash_ids; // id inserted for node v, or null for v
    uint8_t *buf[2];          // ping-pong counters (with table levels for the run kernel)
    double *c_prev;           // n estimates of the last step
    double *sum_d;            // n Eq. 3 sums
    uint32_t *flags;          // n_flags stop flags, one per step, zeroed before init
    uint64_t seed;
    uint32_t n, p, depth, levels, n_flags;
    uint32_t runs;            // 1: run kernel, 0: per-edge kernel
    uint32_t bits;            // bits per register: 8, or 4 (two per byte, saturating at 15)
    uint32_t t;               // steps completed
    uint32_t done;            // 0 while running, else the last step run
    uint32_t converged;       // 1 if the last step grew no estimate by more than stop_delta
    uint32_t depth_only;      // 1: stop at the depth limit only (ignore the growth test)
    double stop_delta;        // the growth test's threshold (Alg. 1: 0.5)
    const uint32_t *grp_rows; // grouped kernel's row lists (groups == 1), as for
    const GroupMask *grp_mask;//   launch_union_groups
    const uint64_t *grp_off;
    uint32_t groups;          // 1: grouped kernel (runs is 1 as well: its tables are built)
};

// Launch schedule of the union kernels for one precision p:
//  * lanes: lanes that share one node's counter.  Up to 64 the node sits in
//    one wave, whose 64 / lanes lane groups gather different neighbours;
//    above 64, lanes / 64 waves of one workgroup each own a slice of it.
//  * nodes_per_block: nodes per workgroup for single-wave shapes (1, 2 or 4;
//    always 1 when several waves share a node).
//  * bits: register width, 8 (one per byte) or 4 (two per byte, low nibble =
//    even register, saturating at 15; the paper's packed format).
// Every schedule of one width gives the same registers; only the speed differs.
struct Sched {
    uint32_t lanes;
    uint32_t nodes_per_block;
    uint32_t bits = 8;
};
constexpr uint32_t kMaxLaneOptions = 4;
// The lanes-per-node values compiled for (p, bits), the default first; returns the count.
uint32_t lane_options(int p, uint32_t bits, uint32_t out[kMaxLaneOptions]);
// runs: the default of the run kernel, which differs at p = 9..11 (8-bit).
Sched default_sched(int p, uint32_t bits = 8, bool runs = false);
bool sched_ok(int p, const Sched &s);

struct LaunchShape {
    uint32_t waves_per_node;  // waves sharing one counter
    uint32_t nodes_per_block; // nodes handled by one workgroup
    uint32_t threads;         // workgroup size
};
LaunchShape shape_for(int p, const Sched &s);

// Batched launches over a list of jobs of one precision p.  block_base has
// nlist + 1 entries: job list[i] owns workgroups [block_base[i], block_base[i+1])
// of the nblocks launched (shape_for(p, s).nodes_per_block nodes each).  Jobs
// whose `done` is set are skipped.
hipError_t launch_batch_init(int p, const Sched &s, BatchJob *jobs, const uint32_t *list,
                             const uint32_t *block_base, uint32_t nlist, uint32_t nblocks,
                             hipStream_t stream);
hipError_t launch_batch_union(int p, const Sched &s, bool runs, BatchJob *jobs,
                              const uint32_t *list, const uint32_t *block_base, uint32_t nlist,
                              uint32_t nblocks, hipStream_t stream);
// The grouped kernel over listed jobs of one (p, bits) with group lists: job
// list[i] owns workgroups [block_base[i], block_base[i+1]),
// group_blocks(p, bits, n) of them.
uint32_t group_blocks(int p, uint32_t bits, uint32_t n);
hipError_t launch_batch_groups(int p, uint32_t bits, BatchJob *jobs, const uint32_t *list,
                               const uint32_t *block_base, uint32_t nlist, uint32_t nblocks,
                               hipStream_t stream);
// Table level k for listed run-kernel jobs with levels >= k; job list[i] owns
// workgroups [block_base[i], block_base[i+1]), batch_table_blocks(n, p, k) of them.
uint32_t batch_table_blocks(uint32_t n, uint32_t row_bytes, uint32_t k);
hipError_t launch_batch_table(BatchJob *jobs, const uint32_t *list, const uint32_t *block_base,
                              uint32_t nlist, uint32_t nblocks, uint32_t k, hipStream_t stream);
// After a step: t += 1 and the stop decision for every listed running job.
hipError_t launch_batch_step_end(BatchJob *jobs, const uint32_t *list, uint32_t nlist,
                                 hipStream_t stream);

// Zero every counter, insert node v into its own counter (SplitMix64 of
// v ^ seed), write the one-element estimate to c_prev[v] and zero sum_d[v].
// hash_ids (n, or null): the element inserted for node v instead of v.
hipError_t launch_init(int p, const Sched &s, uint8_t *cur, double *c_prev, double *sum_d,
                       uint32_t n, uint64_t seed, const uint32_t *hash_ids, hipStream_t stream);

// One HyperBall step t: for every node v, decode its LEB128 row, take the
// byte-wise max of cur[v] and cur[w] over its neighbours w into next[v],
// estimate next[v], accumulate sum_d[v] += t (est - c_prev[v]), store est in
// c_prev[v], and set *flag_t = 1 when est - c_prev[v] > thr (Alg. 1: 0.5).
// order (n, or null): the processing order of the nodes, a permutation of 0..n-1.
// skip (or null): the previous step's flag; when it is 0 that step stopped the
// run, and this launch returns without touching anything.
hipError_t launch_union(int p, const Sched &s, const uint8_t *bytes, const uint64_t *offsets,
                        const uint8_t *cur, uint8_t *next, double *c_prev, double *sum_d,
                        uint32_t *flag_t, uint32_t n, uint32_t t, const uint32_t *order,
                        double thr, const uint32_t *skip, hipStream_t stream);

// The same step from a range-max table of cur (level-major, level 0 = cur,
// levels 1..levels built by launch_table): each run of consecutive neighbour
// ids is covered by at most two table rows.  runs / run_off: the rows' run
// lists with v joined in (launch_row_runs with join_self).  p <= 12.
hipError_t launch_union_runs(int p, const Sched &s, const uint2 *runs, const uint64_t *run_off,
                             const uint8_t *tbl, uint32_t levels, uint8_t *next, double *c_prev,
                             double *sum_d, uint32_t *flag_t, uint32_t n, uint32_t t,
                             const uint32_t *order, double thr, const uint32_t *skip,
                             hipStream_t stream);

// The same step from per-group row lists: group g holds nodes g * kGroupNodes
// .. of the processing order, and its rows grp_rows[grp_off[g] ..] (table row
// indices k n + i) with masks of the group's nodes that need them (bit w: node
// g * kGroupNodes + w; a node's own row included), rows of equal masks next to
// each other.  group_waves(p, bits) waves share a group (group_ok(p, bits)).
uint32_t group_size();
// nodes of one workgroup of the grouped kernel (group_ok(p, bits))
uint32_t group_nodes_per_block(int p, uint32_t bits);
hipError_t launch_union_groups(int p, uint32_t bits, const uint32_t *grp_rows,
                               const GroupMask *grp_mask, const uint64_t *grp_off,
                               const uint8_t *tbl, uint8_t *next, double *c_prev, double *sum_d,
                               uint32_t *flag_t, uint32_t n, uint32_t t, const uint32_t *order,
                               double thr, const uint32_t *skip, hipStream_t stream);

// Build table levels 1..levels: T[k][i] = max(T[k-1][i], T[k-1][i + 2^(k-1)]),
// i <= n - 2^k, rows of m bytes (m a multiple of 16) of `bits`-bit registers,
// T[k] at tbl + k n m.  Requires 2^levels <= n.  skip as for launch_union.
hipError_t launch_table(uint8_t *tbl, uint32_t n, uint32_t m, uint32_t levels, uint32_t bits,
                        const uint32_t *skip, hipStream_t stream);

// Gather ceiling of the run kernel's shape: n nodes each gather `rows` rows of
// a table of table_rows (a power of two) counter rows picked by a hash, with
// the byte-wise max (with_max) or loads alone; out gets WAVES x 64 words per node.
hipError_t launch_gather_probe(int p, const Sched &s, const uint8_t *tbl, uint32_t table_rows,
                               uint32_t rows, uint32_t *out, uint32_t n, uint32_t with_max,
                               hipStream_t stream);

// Streaming copy of bytes (a multiple of 16) from src to dst.
hipError_t launch_copy(const void *src, void *dst, uint64_t bytes, hipStream_t stream);

// VGA metrics of every node (Sec. 3.3): out holds 9 arrays of n doubles --
// connectivity, control, mean depth, RA, integration [HH], [Tekl], [P-value],
// point first moment, point second moment -- from the CSR, the degrees, the
// exact component sizes (null: all n), the cell coordinates (null: the second
// moment is NaN) and the Eq. 3 sums.
hipError_t launch_vga(const uint8_t *bytes, const uint64_t *offsets, const uint32_t *degrees,
                      const uint32_t *comp_size, const int32_t *xy, const double *sum_d,
                      uint32_t n, double *out, hipStream_t stream);

// Maximal runs of consecutive ids of every row (join_self: runs through v
// itself count as one).  runs == null: cnt[v] = the
// number of runs of row v.  Otherwise runs[run_off[v] ...] = the runs of row v
// as inclusive (first, last) pairs; run_off has n + 1 entries.
hipError_t launch_row_runs(const uint8_t *bytes, const uint64_t *offsets, uint32_t n,
                           bool join_self, uint32_t *cnt, const uint64_t *run_off, uint2 *runs,
                           hipStream_t stream);

// Exact local metrics of every node from the run lists (null outputs skipped):
// ordered adjacent neighbour pairs, |B(v, 2)| - 1, clustering, controllability.
// Needs 8 (n + 31) / 32 bytes of LDS, plus 12 per wave, per workgroup of
// local_threads() threads.
uint32_t local_threads();
// lds_limit: LDS bytes per workgroup on the device; n up to about lds_limit * 2
// nodes takes the kernel with constant work per neighbour run (four arrays of
// n / 32 words), larger n the one with two bitmaps.
hipError_t launch_local(const uint2 *runs, const uint64_t *run_off, const uint32_t *degrees,
                        uint32_t n, const uint32_t *order, uint64_t *pairs, uint32_t *ball2,
                        double *clustering, double *controllability, uint32_t lds_limit,
                        hipStream_t stream);

// Fill count u32 words with value (used instead of hipMemsetAsync so the
// sequence stays capturable).
hipError_t launch_fill_u32(uint32_t *dst, uint32_t value, uint64_t count, hipStream_t stream);

// Size of the static device workspace (a file-scope device array, one copy per
// device) that holds the counter buffers of the run entry point that
// allocates nothing.
constexpr uint64_t kStaticScratchBytes = 64ull << 20;
// The current device's address of that array, looked up once per device.
hipError_t static_scratch(uint8_t **ptr);

}  // namespace hbk
