// Autotuner of the union schedule (lanes per node, nodes per workgroup).
//
// The union step's speed depends on how a node's counter is spread over
// lanes and wavefronts and on how many nodes share a workgroup, and the best
// shape varies with p, the kernel and the graph (row lengths, run lengths,
// size against the GPU).  Every shape computes identical registers, so the
// choice can be made by measurement: one union step per candidate on the
// caller's own data, the pick cached per shape class for the process.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>

#include "hb_runtime.h"

namespace hbr {

bool TuneKey::operator<(const TuneKey &o) const {
    return std::tie(p, bits, runs, batched, log_n, log_rows) <
           std::tie(o.p, o.bits, o.runs, o.batched, o.log_n, o.log_rows);
}

namespace {
std::mutex g_tune_mu;
std::map<TuneKey, TunePick> g_tune;

uint32_t log2_floor64(uint64_t x) {
    uint32_t k = 0;
    while (x >> (k + 1)) ++k;
    return k;
}
}  // namespace

TuneKey tune_key(uint32_t p, uint32_t bits, bool runs, bool batched, uint64_t nodes,
                 uint64_t rows) {
    TuneKey k;
    k.p = p;
    k.bits = bits;
    k.runs = runs ? 1u : 0u;
    k.batched = batched ? 1u : 0u;
    k.log_n = log2_floor64(std::max<uint64_t>(nodes, 1));
    k.log_rows = log2_floor64(std::max<uint64_t>(rows / std::max<uint64_t>(nodes, 1), 1));
    return k;
}

bool tune_get(const TuneKey &k, hbk::Sched *s) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    const auto it = g_tune.find(k);
    if (it == g_tune.end()) return false;
    *s = it->second.s;
    return true;
}

void tune_put(const TuneKey &k, const TunePick &v) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[k] = v;
}

std::vector<hbk::Sched> tune_candidates(int p, uint32_t bits, bool runs) {
    std::vector<hbk::Sched> c;
    const hbk::Sched d = hbk::default_sched(p, bits, runs);
    c.push_back(d);
    uint32_t lanes[hbk::kMaxLaneOptions];
    const uint32_t k = hbk::lane_options(p, bits, lanes);
    for (uint32_t i = 0; i < k; ++i) {
        const uint32_t nbs[3] = {4u, 2u, 1u};
        for (uint32_t nb : nbs) {
            hbk::Sched s{lanes[i], nb, bits};
            if (!hbk::sched_ok(p, s)) continue;
            if (s.lanes == d.lanes && s.nodes_per_block == d.nodes_per_block) continue;
            c.push_back(s);
        }
    }
    return c;
}

hb_status tune_measure(int p, uint32_t bits, bool runs, hipStream_t s,
                       const std::function<hipError_t(const hbk::Sched &)> &launch,
                       TunePick *out) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    const std::vector<hbk::Sched> cand = tune_candidates(p, bits, runs);
    TunePick best;
    best.best_ms = -1.0;
    for (size_t i = 0; i < cand.size() && e == hipSuccess; ++i) {
        double t = -1.0;
        for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {
            e = hipEventRecord(e0, s);
            if (e == hipSuccess) e = launch(cand[i]);
            if (e == hipSuccess) e = hipEventRecord(e1, s);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e == hipSuccess && (t < 0.0 || ms < t)) t = ms;
        }
        if (e != hipSuccess) break;
        if (i == 0) best.default_ms = t;
        if (best.best_ms < 0.0 || t < best.best_ms) {
            best.best_ms = t;
            best.s = cand[i];
        }
    }
    if (e1) (void)hipEventDestroy(e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e != hipSuccess) return hip_fail(e, "schedule measurement");
    *out = best;
    return HB_OK;
}

}  // namespace hbr

using namespace hbr;

extern "C" {

hb_status hb_tune_cache(hb_tune_entry *out, uint32_t cap, uint32_t *count) {
    if (!count || (!out && cap)) return fail(HB_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(g_tune_mu);
    uint32_t i = 0;
    for (const auto &kv : g_tune) {
        if (i < cap) {
            hb_tune_entry &t = out[i];
            t.p = kv.first.p;
            t.register_bits = kv.first.bits;
            t.union_kernel = kv.first.runs ? HB_UNION_RUNS : HB_UNION_EDGES;
            t.batched = kv.first.batched;
            t.log2_nodes = kv.first.log_n;
            t.log2_rows_per_node = kv.first.log_rows;
            t.lanes_per_node = kv.second.s.lanes;
            t.nodes_per_block = kv.second.s.nodes_per_block;
            t.best_ms = kv.second.best_ms;
            t.default_ms = kv.second.default_ms;
        }
        ++i;
    }
    *count = i;
    return HB_OK;
}

hb_status hb_tune_clear(void) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune.clear();
    return HB_OK;
}

}  // extern "C"
