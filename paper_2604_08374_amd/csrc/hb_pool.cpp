// Device memory and library-wide options.
//
// Every device allocation of the library goes through dmalloc / dfree: the
// caller's allocator hooks when hb_set_options installed them, else
// hipMalloc / hipFree.  All of it counts against one budget per device
// (hb_options.hbm_budget), so the blocking runs, the batched workspace, the
// served requests and the loaded graphs draw on the same memory.  Working
// buffers (counters, tables, per-node state) are carved first-fit out of
// pooled blocks of at least kMinBlock bytes (under a budget: at most a quarter
// of the budget left, or the request), which stay allocated between
// calls: a run, a batch or an admitted request then takes its buffers without
// a device allocation, and a finished one returns them without the implicit
// device synchronisation of hipFree.  Idle blocks are released by
// hb_release_cache, or when an allocation would otherwise exceed the budget.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <vector>

#include "hb.h"
#include "hb_runtime.h"

namespace hbr {

namespace {

constexpr uint64_t kMinBlock = 1ull << 30;  // pool blocks: at least 1 GiB (or the budget left)

uint64_t align_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

std::mutex g_opt_mu;
hb_options g_opt{};  // all zero: defaults

// One device allocation and the hooks that must release it.
struct Alloc {
    uint64_t bytes;
    int device;
    void (*free_fn)(void *, void *);  // null: hipFree
    void *user;
};

std::mutex g_mem_mu;  // guards g_allocs, g_held, g_peak
std::map<void *, Alloc> g_allocs;
uint64_t g_held[kMaxDevices] = {};
uint64_t g_peak[kMaxDevices] = {};

// First-fit offsets in [0, size), 256-byte granules.
class Arena {
public:
    explicit Arena(uint64_t size) {
        if (size) free_[0] = size;
        size_ = size;
    }
    bool take(uint64_t bytes, uint64_t &off) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            off = it->first;
            const uint64_t rest = it->second - bytes;
            free_.erase(it);
            if (rest) free_[off + bytes] = rest;
            used_ += bytes;
            return true;
        }
        return false;
    }
    void give(uint64_t off, uint64_t bytes) {
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    uint64_t used() const { return used_; }
    uint64_t size() const { return size_; }

private:
    std::map<uint64_t, uint64_t> free_;
    uint64_t size_ = 0, used_ = 0;
};

struct Block {
    uint8_t *base;
    Arena arena;
};

struct DevPool {
    std::vector<Block> blocks;
    std::map<void *, std::pair<size_t, uint64_t>> taken;  // pointer -> (block, bytes)
    uint64_t used = 0, peak = 0;
};

std::mutex g_pool_mu;  // guards g_pool; taken before g_mem_mu, never after it
DevPool g_pool[kMaxDevices];

std::mutex g_evict_mu;
Evictor g_evictor;

int current_device() {
    int dev = 0;
    (void)hipGetDevice(&dev);
    return dev;
}

// Release the idle blocks of dev's pool (g_pool_mu held).  Returns bytes freed.
uint64_t trim_locked(int dev) {
    DevPool &P = g_pool[dev];
    uint64_t freed = 0;
    for (size_t i = 0; i < P.blocks.size();) {
        if (P.blocks[i].arena.used() != 0) {
            ++i;
            continue;
        }
        freed += P.blocks[i].arena.size();
        dfree(P.blocks[i].base);
        P.blocks.erase(P.blocks.begin() + (ptrdiff_t)i);
        // block indices of later blocks shift down by one
        for (auto &kv : P.taken)
            if (kv.second.first > i) --kv.second.first;
    }
    return freed;
}

}  // namespace

hb_options options() {
    std::lock_guard<std::mutex> lk(g_opt_mu);
    return g_opt;
}

void set_evictor(Evictor f) {
    std::lock_guard<std::mutex> lk(g_evict_mu);
    g_evictor = std::move(f);
}

namespace {

// trim_pool: release idle pool blocks when the allocation does not fit (false
// when the caller holds g_pool_mu and trims by itself).
hipError_t dmalloc_impl(void **p, uint64_t bytes, bool trim_pool) {
    *p = nullptr;
    const int dev = current_device();
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    bytes = std::max<uint64_t>(align_up(bytes, 256), 256);
    const hb_options o = options();
    for (int attempt = 0;; ++attempt) {
        {
            std::lock_guard<std::mutex> lk(g_mem_mu);
            if (!o.hbm_budget || g_held[dev] + bytes <= o.hbm_budget) {
                void *q = nullptr;
                hipError_t e;
                if (o.dev_alloc) {
                    q = o.dev_alloc(bytes, o.alloc_user);
                    e = q ? hipSuccess : hipErrorOutOfMemory;
                } else {
                    e = hipMalloc(&q, bytes);
                }
                if (e == hipSuccess) {
                    g_allocs[q] = Alloc{bytes, dev, o.dev_alloc ? o.dev_free : nullptr,
                                        o.alloc_user};
                    g_held[dev] += bytes;
                    g_peak[dev] = std::max(g_peak[dev], g_held[dev]);
                    *p = q;
                    return hipSuccess;
                }
                if (e != hipErrorOutOfMemory) return e;
                (void)hipGetLastError();
            }
        }
        if (attempt == 1) return hipErrorOutOfMemory;
        // over the budget or out of memory: release idle pool blocks and idle
        // cached graphs, then try once more
        uint64_t freed = 0;
        if (trim_pool) {
            std::lock_guard<std::mutex> lk(g_pool_mu);
            freed += trim_locked(dev);
        }
        Evictor ev;
        {
            std::lock_guard<std::mutex> lk(g_evict_mu);
            ev = g_evictor;
        }
        if (ev) freed += ev(dev, bytes);
        if (!freed) return hipErrorOutOfMemory;
    }
}

}  // namespace

hipError_t dmalloc(void **p, uint64_t bytes) { return dmalloc_impl(p, bytes, true); }

void dfree(void *p) {
    if (!p) return;
    Alloc a{};
    bool known = false;
    {
        std::lock_guard<std::mutex> lk(g_mem_mu);
        auto it = g_allocs.find(p);
        if (it != g_allocs.end()) {
            a = it->second;
            known = true;
            g_held[a.device] -= a.bytes;
            g_allocs.erase(it);
        }
    }
    if (known && a.free_fn) {
        a.free_fn(p, a.user);
    } else {
        (void)hipFree(p);
    }
}

hb_status pool_take(uint64_t bytes, void **p) {
    *p = nullptr;
    const int dev = current_device();
    if (dev < 0 || dev >= kMaxDevices) return fail(HB_EDEVICE, "device %d out of range", dev);
    bytes = std::max<uint64_t>(align_up(bytes, 256), 256);
    std::lock_guard<std::mutex> lk(g_pool_mu);
    DevPool &P = g_pool[dev];
    auto place = [&](size_t bi, uint64_t off) {
        *p = P.blocks[bi].base + off;
        P.taken[*p] = {bi, bytes};
        P.used += bytes;
        P.peak = std::max(P.peak, P.used);
    };
    for (size_t bi = 0; bi < P.blocks.size(); ++bi) {
        uint64_t off;
        if (P.blocks[bi].arena.take(bytes, off)) {
            place(bi, off);
            return HB_OK;
        }
    }
    // a new block: kMinBlock or the request, within what the budget leaves
    const hb_options o = options();
    uint64_t held;
    {
        std::lock_guard<std::mutex> lk2(g_mem_mu);
        held = g_held[dev];
    }
    uint64_t want = std::max(align_up(bytes, 2ull << 20), kMinBlock);
    if (o.hbm_budget) {
        // under a budget a block takes at most a quarter of what is left, so
        // that graphs and other blocks still find room
        const uint64_t room = o.hbm_budget > held ? o.hbm_budget - held : 0;
        want = std::max(bytes, std::min(want, align_up(room / 4, 256)));
    }
    void *base = nullptr;
    hipError_t e = dmalloc_impl(&base, want, false);
    if (e == hipErrorOutOfMemory && want > bytes) e = dmalloc_impl(&base, want = bytes, false);
    if (e == hipErrorOutOfMemory) {
        // idle blocks may be too fragmented to hold it: release them and try
        // one block of exactly this size
        if (trim_locked(dev)) e = dmalloc_impl(&base, want = bytes, false);
    }
    if (e == hipErrorOutOfMemory)
        return fail(HB_ENOMEM,
                    "%llu bytes of device memory do not fit (held %llu, budget %llu; 0 = none)",
                    (unsigned long long)bytes, (unsigned long long)held,
                    (unsigned long long)o.hbm_budget);
    if (e != hipSuccess) return hip_fail(e, "device allocation");
    P.blocks.push_back(Block{static_cast<uint8_t *>(base), Arena(want)});
    uint64_t off;
    P.blocks.back().arena.take(bytes, off);
    place(P.blocks.size() - 1, off);
    return HB_OK;
}

void pool_give(void *p) {
    if (!p) return;
    std::lock_guard<std::mutex> lk(g_pool_mu);
    for (auto &P : g_pool) {
        auto it = P.taken.find(p);
        if (it == P.taken.end()) continue;
        Block &b = P.blocks[it->second.first];
        b.arena.give((uint64_t)(static_cast<uint8_t *>(p) - b.base), it->second.second);
        P.used -= it->second.second;
        P.taken.erase(it);
        return;
    }
}

void pool_trim_all() {
    std::lock_guard<std::mutex> lk(g_pool_mu);
    for (int d = 0; d < kMaxDevices; ++d)
        if (!g_pool[d].blocks.empty()) {
            (void)hipSetDevice(d);
            trim_locked(d);
        }
}

void memory_stats(int dev, hb_memory_stats_t *out) {
    *out = hb_memory_stats_t{};
    if (dev < 0 || dev >= kMaxDevices) return;
    const hb_options o = options();
    out->budget_bytes = o.hbm_budget;
    {
        std::lock_guard<std::mutex> lk(g_pool_mu);
        const DevPool &P = g_pool[dev];
        for (const auto &b : P.blocks) out->pool_bytes += b.arena.size();
        out->pool_used_bytes = P.used;
        out->pool_peak_used_bytes = P.peak;
    }
    std::lock_guard<std::mutex> lk(g_mem_mu);
    out->held_bytes = g_held[dev];
    out->peak_held_bytes = g_peak[dev];
}

hb_status set_options(const hb_options *o) {
    hb_options v = o ? *o : hb_options{};
    if (!v.dev_alloc != !v.dev_free)
        return fail(HB_EINVAL, "dev_alloc and dev_free must be set together");
    if (v.stop_rule > HB_STOP_DEPTH) return fail(HB_EINVAL, "unknown stop rule %u", v.stop_rule);
    if (!(v.stop_delta >= 0.0)) return fail(HB_EINVAL, "stop_delta must be >= 0");
    if (v.tune_seed_count && !v.tune_seed) return fail(HB_EINVAL, "tune_seed is NULL");
    for (uint32_t i = 0; i < v.tune_seed_count; ++i) {
        const hb_tune_entry &t = v.tune_seed[i];
        const uint32_t bits = t.register_bits ? t.register_bits : 8u;
        if (t.p < HB_P_MIN || t.p > HB_P_MAX || (bits != 8u && bits != 4u) ||
            !hbk::sched_ok((int)t.p, hbk::Sched{t.lanes_per_node, t.nodes_per_block, bits}) ||
            t.union_kernel < HB_UNION_EDGES || t.union_kernel > HB_UNION_RUNS)
            return fail(HB_EINVAL, "tune_seed[%u] names no built schedule", i);
    }
    for (uint32_t i = 0; i < v.tune_seed_count; ++i) {
        const hb_tune_entry &t = v.tune_seed[i];
        const uint32_t bits = t.register_bits ? t.register_bits : 8u;
        TuneKey k{t.p, bits, t.union_kernel == HB_UNION_RUNS ? 1u : 0u, t.batched ? 1u : 0u,
                  t.log2_nodes, t.log2_rows_per_node};
        TunePick pick;
        pick.s = hbk::Sched{t.lanes_per_node, t.nodes_per_block, bits};
        pick.best_ms = t.best_ms;
        pick.default_ms = t.default_ms;
        tune_put(k, pick);
    }
    v.tune_seed = nullptr;  // not kept: the picks are in the cache now
    v.tune_seed_count = 0;
    std::lock_guard<std::mutex> lk(g_opt_mu);
    g_opt = v;
    return HB_OK;
}

}  // namespace hbr

extern "C" {

hb_status hb_set_options(const hb_options *o) { return hbr::set_options(o); }

hb_status hb_get_options(hb_options *out) {
    if (!out) return hbr::fail(HB_EINVAL, "out is NULL");
    *out = hbr::options();
    return HB_OK;
}

hb_status hb_memory_stats(int32_t device, hb_memory_stats_t *out) {
    if (!out) return hbr::fail(HB_EINVAL, "out is NULL");
    if (device < 0 || device >= hbr::kMaxDevices) return hbr::fail(HB_EINVAL, "device %d", device);
    hbr::memory_stats(device, out);
    return HB_OK;
}

}  // extern "C"
