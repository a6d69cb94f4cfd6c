// Internal host-side declarations shared by the runtime files (not public).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>
#include <functional>
#include <mutex>
#include <string>
#include <vector>

#include "hb.h"
#include "hb_internal.h"

namespace hbr {

extern thread_local std::string g_err;
extern std::mutex g_dev_mu;  // serialises the blocking calls that touch the GPU

hb_status fail(hb_status st, const char *fmt, ...);
hb_status hip_fail(hipError_t e, const char *what);
uint64_t now_ns();
uint32_t floor_log2(uint32_t n);

#define HB_HIP(call)                                      \
    do {                                                  \
        hipError_t e_ = (call);                           \
        if (e_ != hipSuccess) return hbr::hip_fail(e_, #call); \
    } while (0)

constexpr int kMaxLevels = 24;
// Smallest graph on which HB_UNION_AUTO picks the grouped kernel: 4,096 groups
// of 8 nodes, four waves on every SIMD of the device.
constexpr uint32_t kGroupsMinNodes = 32768;
// Steps of a blocking run enqueued between two host reads of the stop flags.
constexpr uint32_t kSegment = 8;
// Default depth K of the run kernel's range-max table (city graph, p = 10, per
// step of table build + union launch: 14.0 ms at K = 7, 13.7 at 8, 13.7 at 9,
// 15.1 at 6; deeper tables cover long runs with fewer rows but cost a level of
// build and n 2^p bytes of memory each).
constexpr uint32_t kDefaultLevels = 8;

// Runs of consecutive neighbour ids (joined across the node itself) and, for
// every table depth K, the table rows the run kernel loads to cover them.
struct RunCounts {
    uint64_t runs = 0;
    uint64_t lookups[kMaxLevels + 1] = {};
    // sum over rows w of deg(w) x (maximal runs of w, v not joined in): the
    // neighbour runs the local metrics read over all nodes
    uint64_t local_reads = 0;
    void add(uint64_t r) {
        ++runs;
        for (int k = 0; k <= kMaxLevels; ++k) {
            const uint64_t top = 1ull << k;
            if (r <= top) {
                lookups[k] += (r & (r - 1)) == 0 ? 1 : 2;  // one row if r is a power of two
            } else {
                lookups[k] += (r + top - 1) / top;
            }
        }
    }
    void merge(const RunCounts &o) {
        runs += o.runs;
        local_reads += o.local_reads;
        for (int k = 0; k <= kMaxLevels; ++k) lookups[k] += o.lookups[k];
    }
};

// ---- union-schedule autotuner (hb_tune.cpp)
// Shape class of a union launch: the key of the process-wide pick cache.
struct TuneKey {
    uint32_t p, bits, runs, batched, log_n, log_rows;
    bool operator<(const TuneKey &o) const;
};
// nodes: nodes the launch covers; rows: counter rows it gathers per step
// (table rows for the run kernel, directed edges otherwise).
TuneKey tune_key(uint32_t p, uint32_t bits, bool runs, bool batched, uint64_t nodes,
                 uint64_t rows);
struct TunePick {
    hbk::Sched s;
    double best_ms = 0.0, default_ms = 0.0;
};
bool tune_get(const TuneKey &k, hbk::Sched *s);
void tune_put(const TuneKey &k, const TunePick &v);
// Every schedule built for (p, register bits), the default first.
std::vector<hbk::Sched> tune_candidates(int p, uint32_t bits, bool runs);
// Time one union step of every candidate with `launch` (which enqueues the
// step on stream s): two launches each, the faster counts.  Fills the pick.
hb_status tune_measure(int p, uint32_t bits, bool runs, hipStream_t s,
                       const std::function<hipError_t(const hbk::Sched &)> &launch,
                       TunePick *out);

// ---- device memory and library-wide options (hb_pool.cpp)
constexpr int kMaxDevices = 64;
// The options of hb_set_options (a copy; calls take one at their start).
hb_options options();
// Allocate / free device memory of the current device through the caller's
// hooks or hipMalloc / hipFree, counted against the device's budget.  Over the
// budget (or out of memory) dmalloc first releases idle pool blocks and asks
// the evictor for memory, then returns hipErrorOutOfMemory.
hipError_t dmalloc(void **p, uint64_t bytes);
void dfree(void *p);
// Working buffers from the current device's pool (first fit in pooled blocks,
// grown within the budget).  HB_ENOMEM (with a message) when it cannot grow.
hb_status pool_take(uint64_t bytes, void **p);
void pool_give(void *p);
void pool_trim_all();  // release every idle pool block
void memory_stats(int dev, hb_memory_stats_t *out);
// Called when an allocation does not fit: free idle memory of device dev (at
// least `need` bytes if it can) and return the bytes freed.
using Evictor = std::function<uint64_t(int dev, uint64_t need)>;
void set_evictor(Evictor f);

// Free a loaded graph and its device memory (no lock taken; the caller makes
// sure nothing uses it).
void graph_release(hb_graph *g);

}  // namespace hbr

struct hb_graph {
    uint32_t n = 0;
    uint64_t n_edges = 0, n_bytes = 0;
    hbr::RunCounts runs;
    int device = 0;
    std::vector<uint32_t> comp_size;  // empty: one component of n
    uint8_t *d_bytes = nullptr;
    uint64_t *d_offsets = nullptr;
    uint32_t *d_order = nullptr;     // processing order, or null
    uint32_t *d_degrees = nullptr;   // n neighbour counts
    uint32_t *d_comp = nullptr;      // exact component sizes, or null (all n)
    uint32_t *d_hash_ids = nullptr;  // inserted ids, or null
    int32_t *d_xy = nullptr;         // 2n cell coordinates, or null
    uint32_t *d_grp_rows = nullptr;  // grouped kernel: distinct table rows per node group
    hbk::GroupMask *d_grp_mask = nullptr;  // and the group's nodes that need each
    uint64_t *d_grp_off = nullptr;   // n_groups + 1 offsets
    uint32_t grp_levels = 0;         // table depth the group lists were built for
    uint64_t grp_entries = 0;
    uint2 *d_runs = nullptr;         // run list of the rows, v joined in (run kernel)
    uint64_t *d_run_off = nullptr;   // n + 1 offsets into d_runs
    // run state, kept between runs (the counters live in a per-device workspace)
    double *d_cprev = nullptr, *d_sumd = nullptr;
    uint32_t *d_flags = nullptr;
    uint64_t n_flags = 0;
    uint32_t *h_flags = nullptr;  // pinned: the stop flags of one segment of steps
    double *h_out = nullptr;      // pinned: reach and sum_d of a blocking run (2 n), staged
                                  // here so the device copies need no pageable bounce
    hipStream_t stream = nullptr;
    hipEvent_t ev_init[2] = {nullptr, nullptr};          // around the initialisation
    hipEvent_t ev_step[hbr::kSegment][3] = {};            // per step: table, union, end
    std::atomic<uint32_t> inflight{0};  // served requests that still use this graph
    uint64_t dev_bytes = 0;             // device memory of the graph's arrays
};
