// Host runtime behind include/hb.h: CSR encoding and validation (host only),
// device-resident graphs, and the HyperBall run driver (Alg. 1's loop: init,
// one fused union/estimate/accumulate launch per step, a 4-byte flag read
// back after each step to decide whether to stop).
#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>
#include <time.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "hb.h"
#include "hb_internal.h"
#include "hb_runtime.h"

namespace hbr {

thread_local std::string g_err;
std::mutex g_dev_mu;

hb_status fail(hb_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

hb_status hip_fail(hipError_t e, const char *what) {
    return fail(HB_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

uint64_t now_ns() {
    timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (uint64_t)ts.tv_sec * 1000000000ull + (uint64_t)ts.tv_nsec;
}

uint32_t floor_log2(uint32_t n) {
    uint32_t lg = 0;
    while ((2ull << lg) <= n) ++lg;
    return lg;
}

}  // namespace hbr

using namespace hbr;

namespace {

unsigned host_threads() {
    unsigned h = std::thread::hardware_concurrency();
    if (h == 0) h = 1;
    return std::min(h, 16u);
}

// Run f(lo, hi) over [0, n) split into contiguous ranges, one per thread.
template <class F>
void parallel_ranges(uint64_t n, F f) {
    const unsigned nt = (unsigned)std::min<uint64_t>(host_threads(), std::max<uint64_t>(n / 1024, 1));
    if (nt <= 1) {
        f(0, n);
        return;
    }
    std::vector<std::thread> th;
    for (unsigned i = 0; i < nt; ++i) {
        const uint64_t lo = n * i / nt, hi = n * (i + 1) / nt;
        th.emplace_back([=] { f(lo, hi); });
    }
    for (auto &t : th) t.join();
}

int uleb_size(uint32_t v) {
    int k = 1;
    while (v >= 0x80u) {
        v >>= 7;
        ++k;
    }
    return k;
}

uint8_t *uleb_put(uint32_t v, uint8_t *out) {
    while (v >= 0x80u) {
        *out++ = (uint8_t)(v | 0x80u);
        v >>= 7;
    }
    *out++ = (uint8_t)v;
    return out;
}

// Check one compressed row; returns true if valid.  Counts runs into rc.
bool row_ok(const uint8_t *p, const uint8_t *end, uint32_t v, uint32_t n, uint32_t degree,
            RunCounts *rc = nullptr) {
    uint64_t prev = 0, run_start = 0, plain_runs = 0;
    uint32_t count = 0;
    while (p < end) {
        uint32_t val = 0;
        int k = 0;
        for (;;) {
            if (p >= end || k == 5) return false;  // truncated, or longer than 5 bytes
            const uint8_t b = *p++;
            if (k == 4 && (b & 0xF0u)) return false;  // beyond 32 bits
            val |= (uint32_t)(b & 0x7Fu) << (7 * k);
            ++k;
            if (!(b & 0x80u)) break;
        }
        uint64_t id;
        if (count == 0) {
            id = val;
        } else {
            if (val == 0) return false;  // repeated id
            id = prev + val;
        }
        if (id >= n || id == v) return false;
        if (rc) {
            const bool joins = count > 0 && (id == prev + 1 || (id == prev + 2 && prev + 1 == v));
            if (count > 0 && !joins) rc->add(prev - run_start + 1);
            if (count == 0 || !joins) run_start = id;
            if (count == 0 || id != prev + 1) ++plain_runs;
        }
        prev = id;
        if (++count > degree) return false;
    }
    if (rc && count > 0) rc->add(prev - run_start + 1);
    if (rc) rc->local_reads += plain_runs * degree;
    return count == degree;
}

}  // namespace

namespace {

}  // namespace

void hbr::graph_release(hb_graph *g) {
    if (!g) return;
    (void)hipSetDevice(g->device);
    if (g->stream) (void)hipStreamSynchronize(g->stream);
    for (void *p : {(void *)g->d_bytes, (void *)g->d_offsets, (void *)g->d_cprev,
                    (void *)g->d_order, (void *)g->d_hash_ids, (void *)g->d_degrees,
                    (void *)g->d_comp, (void *)g->d_runs, (void *)g->d_run_off,
                    (void *)g->d_sumd, (void *)g->d_flags, (void *)g->d_xy,
                    (void *)g->d_grp_rows, (void *)g->d_grp_mask, (void *)g->d_grp_off})
        dfree(p);
    if (g->h_flags) (void)hipHostFree(g->h_flags);
    if (g->h_out) (void)hipHostFree(g->h_out);
    for (auto &e : g->ev_init)
        if (e) (void)hipEventDestroy(e);
    for (auto &step : g->ev_step)
        for (auto &e : step)
            if (e) (void)hipEventDestroy(e);
    if (g->stream) (void)hipStreamDestroy(g->stream);
    delete g;
}

namespace {

// Run lists of g's rows, decoded on the device from the uploaded LEB128 rows:
// *runs (inclusive first/last pairs) and *off (n + 1 offsets), allocated here;
// *total runs.  join_self joins the runs on both sides of v itself.
hipError_t build_run_list(hb_graph *g, bool join_self, uint2 **runs, uint64_t **off,
                          uint64_t *total) {
    const uint32_t n = g->n;
    *runs = nullptr;
    *off = nullptr;
    std::vector<uint32_t> cnt(n);
    std::vector<uint64_t> h_off((size_t)n + 1);
    uint32_t *d_cnt = nullptr;
    hipError_t e = dmalloc((void **)&d_cnt, sizeof(uint32_t) * n);
    if (e == hipSuccess)
        e = hbk::launch_row_runs(g->d_bytes, g->d_offsets, n, join_self, d_cnt, nullptr, nullptr,
                                 g->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(cnt.data(), d_cnt, sizeof(uint32_t) * n, hipMemcpyDeviceToHost,
                           g->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
    (void)hipStreamSynchronize(g->stream);
    dfree(d_cnt);
    if (e != hipSuccess) return e;
    h_off[0] = 0;
    for (uint32_t v = 0; v < n; ++v) h_off[v + 1] = h_off[v] + cnt[v];
    *total = h_off[n];
    e = dmalloc((void **)off, sizeof(uint64_t) * (n + 1ull));
    if (e == hipSuccess) e = dmalloc((void **)runs, sizeof(uint2) * std::max<uint64_t>(h_off[n], 1));
    if (e == hipSuccess)
        e = hipMemcpyAsync(*off, h_off.data(), sizeof(uint64_t) * (n + 1ull),
                           hipMemcpyHostToDevice, g->stream);
    if (e == hipSuccess)
        e = hbk::launch_row_runs(g->d_bytes, g->d_offsets, n, join_self, nullptr, *off, *runs,
                                 g->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
    (void)hipStreamSynchronize(g->stream);  // h_off is read by the copy
    if (e != hipSuccess) {
        dfree(*off);
        dfree(*runs);
        *off = nullptr;
        *runs = nullptr;
    }
    return e;
}

// Row lists of the grouped union kernel: for every group of group_size()
// consecutive nodes of the processing order, the distinct table rows (k n + i,
// for tables of depth `levels`) that cover the runs of its nodes, each node's
// own counter row included, with a mask of the nodes that need each row; rows
// of one mask are listed together, in table position order.  Built on the host
// from the device run list; false when memory is short.
bool build_group_lists(hb_graph *g, uint32_t levels, const uint32_t *order) {
    const uint32_t n = g->n;
    const uint32_t W = hbk::kGroupNodes;
    const uint64_t total = g->runs.runs;
    if ((uint64_t)(levels + 1) * n >= (1ull << 32)) return false;  // row indices are 32-bit
    std::vector<uint64_t> roff((size_t)n + 1);
    std::vector<uint2> runs(std::max<uint64_t>(total, 1));
    if (hipMemcpy(roff.data(), g->d_run_off, sizeof(uint64_t) * (n + 1ull),
                  hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(runs.data(), g->d_runs, sizeof(uint2) * total, hipMemcpyDeviceToHost) !=
            hipSuccess)
        return false;
    const uint32_t n_groups = (n + W - 1) / W;
    const uint64_t top = 1ull << levels;
    // per thread: the entries (row << 32 | mask) of a contiguous range of groups
    const unsigned nt = (unsigned)std::min<uint64_t>(host_threads(), std::max<uint32_t>(n_groups / 64, 1));
    std::vector<std::vector<uint64_t>> part(nt);
    std::vector<uint64_t> count(n_groups, 0);
    std::vector<std::thread> th;
    for (unsigned ti = 0; ti < nt; ++ti) {
        th.emplace_back([&, ti] {
            const uint32_t g0 = (uint32_t)((uint64_t)n_groups * ti / nt);
            const uint32_t g1 = (uint32_t)((uint64_t)n_groups * (ti + 1) / nt);
            std::vector<uint64_t> tmp, merged;
            for (uint32_t gr = g0; gr < g1; ++gr) {
                tmp.clear();
                for (uint32_t w = 0; w < W; ++w) {
                    const uint64_t i = (uint64_t)gr * W + w;
                    if (i >= n) break;
                    const uint32_t v = order ? order[i] : (uint32_t)i;
                    const uint64_t bit = 1ull << w;
                    tmp.push_back(((uint64_t)v << 32) | bit);  // the node's own counter
                    for (uint64_t e = roff[v]; e < roff[v + 1]; ++e) {
                        const uint64_t x = runs[e].x, y = runs[e].y, r = y - x + 1;
                        if (r <= top) {
                            const uint32_t k = floor_log2((uint32_t)r);
                            tmp.push_back(((k * (uint64_t)n + x) << 32) | bit);
                            if (r != (1ull << k))
                                tmp.push_back(((k * (uint64_t)n + y - (1ull << k) + 1) << 32) | bit);
                            continue;
                        }
                        for (uint64_t j = x;; j += top) {
                            const uint64_t at = (j + top - 1 < y) ? j : y - top + 1;
                            tmp.push_back(((levels * (uint64_t)n + at) << 32) | bit);
                            if (at != j || j + top - 1 == y) break;
                        }
                    }
                }
                std::sort(tmp.begin(), tmp.end());
                merged.clear();
                for (size_t a = 0; a < tmp.size();) {
                    uint64_t row = tmp[a] >> 32, mask = 0;
                    while (a < tmp.size() && (tmp[a] >> 32) == row) mask |= tmp[a++] & 0xFFFFFFFFu;
                    merged.push_back((row << 32) | mask);
                }
                // by mask, then table position, then level
                std::sort(merged.begin(), merged.end(), [n](uint64_t a, uint64_t b) {
                    const uint64_t ma = a & 0xFFFFFFFFu, mb = b & 0xFFFFFFFFu;
                    if (ma != mb) return ma < mb;
                    const uint64_t ia = (a >> 32) % n, ib = (b >> 32) % n;
                    return ia != ib ? ia < ib : a < b;
                });
                part[ti].insert(part[ti].end(), merged.begin(), merged.end());
                count[gr] = merged.size();
            }
        });
    }
    for (auto &t : th) t.join();
    std::vector<uint64_t> goff((size_t)n_groups + 1, 0);
    for (uint32_t gr = 0; gr < n_groups; ++gr) goff[gr + 1] = goff[gr] + count[gr];
    const uint64_t entries = goff[n_groups];
    std::vector<uint32_t> rows(std::max<uint64_t>(entries, 1));
    std::vector<hbk::GroupMask> masks(std::max<uint64_t>(entries, 1));
    uint64_t at = 0;
    for (const auto &pv : part)
        for (uint64_t e : pv) {
            rows[at] = (uint32_t)(e >> 32);
            masks[at] = (hbk::GroupMask)(e & 0xFFFFFFFFu);
            ++at;
        }
    hipError_t e = dmalloc((void **)&g->d_grp_rows, sizeof(uint32_t) * rows.size());
    if (e == hipSuccess)
        e = dmalloc((void **)&g->d_grp_mask, sizeof(hbk::GroupMask) * masks.size());
    if (e == hipSuccess) e = dmalloc((void **)&g->d_grp_off, sizeof(uint64_t) * goff.size());
    if (e == hipSuccess)
        e = hipMemcpy(g->d_grp_rows, rows.data(), sizeof(uint32_t) * rows.size(),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(g->d_grp_mask, masks.data(), sizeof(hbk::GroupMask) * masks.size(),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(g->d_grp_off, goff.data(), sizeof(uint64_t) * goff.size(),
                      hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        dfree(g->d_grp_rows);
        dfree(g->d_grp_mask);
        dfree(g->d_grp_off);
        g->d_grp_rows = nullptr;
        g->d_grp_mask = nullptr;
        g->d_grp_off = nullptr;
        return false;
    }
    g->grp_levels = levels;
    g->grp_entries = entries;
    g->dev_bytes += (4 + sizeof(hbk::GroupMask)) * rows.size() + 8 * goff.size();
    return true;
}

hb_status have_device() {
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count < 1) return fail(HB_EDEVICE, "no GPU available");
    return HB_OK;
}

}  // namespace

namespace {
hb_status validate_impl(const hb_csr *csr, uint32_t *bad_node, RunCounts *rc_out) {
    if (bad_node) *bad_node = 0;
    if (!csr) return fail(HB_EINVAL, "csr is NULL");
    const uint32_t n = csr->n;
    if (n == 0) return fail(HB_EINVAL, "n must be >= 1");
    if (!csr->offsets || !csr->degrees) return fail(HB_EINVAL, "offsets/degrees NULL");
    if (csr->offsets[0] != 0) {
        if (bad_node) *bad_node = 0;
        return fail(HB_ECORRUPT, "offsets[0] != 0");
    }
    if (csr->offsets[n] > 0 && !csr->bytes) return fail(HB_EINVAL, "bytes is NULL");
    std::atomic<uint32_t> bad{UINT32_MAX};
    std::atomic<uint64_t> deg_sum{0};
    std::mutex rc_mu;
    parallel_ranges(n, [&](uint64_t lo, uint64_t hi) {
        uint64_t s = 0;
        RunCounts rc;
        for (uint64_t v = lo; v < hi; ++v) {
            const uint64_t a = csr->offsets[v], b = csr->offsets[v + 1];
            s += csr->degrees[v];
            if (b < a || !row_ok(csr->bytes + a, csr->bytes + b, (uint32_t)v, n, csr->degrees[v],
                                 rc_out ? &rc : nullptr)) {
                uint32_t cur = bad.load();
                while ((uint32_t)v < cur && !bad.compare_exchange_weak(cur, (uint32_t)v)) {
                }
                return;
            }
        }
        deg_sum += s;
        if (rc_out) {
            std::lock_guard<std::mutex> lk(rc_mu);
            rc_out->merge(rc);
        }
    });
    if (bad != UINT32_MAX) {
        if (bad_node) *bad_node = bad;
        return fail(HB_ECORRUPT, "row %u of the compressed CSR is malformed", (unsigned)bad.load());
    }
    if (deg_sum != csr->n_edges) {
        if (bad_node) *bad_node = n;
        return fail(HB_ECORRUPT, "degree sum %llu != n_edges %llu",
                    (unsigned long long)deg_sum.load(), (unsigned long long)csr->n_edges);
    }
    return HB_OK;
}

// The schedule named in the options for precision p, or lanes = 0 when the
// options leave it to the tuner.
hb_status explicit_sched(const hb_run_opts &o, uint32_t p, hbk::Sched *out) {
    const uint32_t bits = o.register_bits ? o.register_bits : 8u;
    *out = hbk::Sched{0u, 0u, bits};
    if (o.tune > HB_TUNE_OFF) return fail(HB_EINVAL, "unknown tune mode %u", o.tune);
    if (bits != 8u && bits != 4u) return fail(HB_EINVAL, "register_bits %u is not 8 or 4", bits);
    if (bits == 4u && p < 5) return fail(HB_EINVAL, "4-bit registers need p >= 5");
    if (o.lanes_per_node == 0) {
        if (o.nodes_per_block) return fail(HB_EINVAL, "nodes_per_block needs lanes_per_node");
        return HB_OK;
    }
    hbk::Sched s{o.lanes_per_node, o.nodes_per_block, bits};
    if (!s.nodes_per_block) s.nodes_per_block = s.lanes > 64u ? 1u : 4u;
    if (!hbk::sched_ok((int)p, s))
        return fail(HB_EINVAL, "no union schedule of %u lanes, %u nodes per workgroup for p = %u",
                    s.lanes, s.nodes_per_block, p);
    *out = s;
    return HB_OK;
}
}  // namespace

extern "C" {

const char *hb_version(void) { return "hb 0.1.0 (gfx950)"; }

const char *hb_last_error(void) { return g_err.c_str(); }

hb_status hb_device_count(int32_t *count) {
    if (!count) return fail(HB_EINVAL, "count is NULL");
    int c = 0;
    if (hipGetDeviceCount(&c) != hipSuccess) c = 0;
    *count = c;
    return HB_OK;
}

hb_status hb_csr_encode(uint32_t n, const uint64_t *adj_offsets, const uint32_t *adj_ids,
                        uint64_t *offsets, uint32_t *degrees, uint8_t *bytes, uint64_t bytes_cap,
                        uint64_t *bytes_len) {
    if (n == 0) return fail(HB_EINVAL, "n must be >= 1");
    if (!adj_offsets || !offsets || !degrees || !bytes_len)
        return fail(HB_EINVAL, "NULL argument");
    if (adj_offsets[n] > 0 && !adj_ids) return fail(HB_EINVAL, "adj_ids is NULL");
    if (adj_offsets[0] != 0) return fail(HB_EINVAL, "adj_offsets[0] != 0");
    std::vector<uint64_t> rowb(n);
    std::atomic<uint32_t> bad{UINT32_MAX};
    parallel_ranges(n, [&](uint64_t lo, uint64_t hi) {
        for (uint64_t v = lo; v < hi; ++v) {
            const uint64_t a = adj_offsets[v], b = adj_offsets[v + 1];
            if (b < a) {
                bad = std::min<uint32_t>(bad, (uint32_t)v);
                return;
            }
            uint64_t nb = 0;
            uint32_t prev = 0;
            for (uint64_t k = a; k < b; ++k) {
                const uint32_t id = adj_ids[k];
                if (id >= n || id == v || (k > a && id <= prev)) {
                    bad = std::min<uint32_t>(bad, (uint32_t)v);
                    return;
                }
                nb += (uint64_t)uleb_size(k == a ? id : id - prev);
                prev = id;
            }
            rowb[v] = nb;
            degrees[v] = (uint32_t)(b - a);
        }
    });
    if (bad != UINT32_MAX)
        return fail(HB_EINVAL, "adjacency row %u is not strictly increasing within [0, n) "
                               "without a self loop", (unsigned)bad.load());
    offsets[0] = 0;
    for (uint32_t v = 0; v < n; ++v) offsets[v + 1] = offsets[v] + rowb[v];
    *bytes_len = offsets[n];
    if (!bytes) return HB_OK;
    if (bytes_cap < offsets[n])
        return fail(HB_EINVAL, "bytes_cap %llu < %llu", (unsigned long long)bytes_cap,
                    (unsigned long long)offsets[n]);
    parallel_ranges(n, [&](uint64_t lo, uint64_t hi) {
        for (uint64_t v = lo; v < hi; ++v) {
            uint8_t *out = bytes + offsets[v];
            uint32_t prev = 0;
            for (uint64_t k = adj_offsets[v]; k < adj_offsets[v + 1]; ++k) {
                const uint32_t id = adj_ids[k];
                out = uleb_put(k == adj_offsets[v] ? id : id - prev, out);
                prev = id;
            }
        }
    });
    return HB_OK;
}

hb_status hb_csr_validate(const hb_csr *csr, uint32_t *bad_node) {
    return validate_impl(csr, bad_node, nullptr);
}


hb_status hb_graph_load(const hb_csr *csr, hb_graph **out) {
    if (!out) return fail(HB_EINVAL, "out is NULL");
    *out = nullptr;
    RunCounts rc;
    hb_status st = validate_impl(csr, nullptr, &rc);
    if (st != HB_OK) return st;
    if (csr->comp_size)
        for (uint32_t v = 0; v < csr->n; ++v)
            if (csr->comp_size[v] == 0 || csr->comp_size[v] > csr->n)
                return fail(HB_EINVAL, "comp_size[%u] outside [1, n]", v);
    if (csr->order) {
        std::vector<uint8_t> seen(csr->n, 0);
        for (uint32_t i = 0; i < csr->n; ++i) {
            const uint32_t v = csr->order[i];
            if (v >= csr->n || seen[v])
                return fail(HB_EINVAL, "order is not a permutation of 0..n-1 (entry %u)", i);
            seen[v] = 1;
        }
    }
    std::lock_guard<std::mutex> lk(g_dev_mu);
    if ((st = have_device()) != HB_OK) return st;
    hb_graph *g = new (std::nothrow) hb_graph;
    if (!g) return fail(HB_ENOMEM, "host allocation failed");
    g->n = csr->n;
    g->n_edges = csr->n_edges;
    g->n_bytes = csr->offsets[csr->n];
    g->runs = rc;
    (void)hipGetDevice(&g->device);
    if (csr->comp_size) g->comp_size.assign(csr->comp_size, csr->comp_size + csr->n);
    auto bail = [&](hipError_t e, const char *what) {
        graph_release(g);
        if (e == hipErrorOutOfMemory) return fail(HB_ENOMEM, "%s: out of device memory", what);
        return hip_fail(e, what);
    };
    hipError_t e;
    if ((e = hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking)) != hipSuccess)
        return bail(e, "hipStreamCreate");
    for (auto &ev : g->ev_init)
        if ((e = hipEventCreate(&ev)) != hipSuccess) return bail(e, "hipEventCreate");
    for (auto &step : g->ev_step)
        for (auto &ev : step)
            if ((e = hipEventCreate(&ev)) != hipSuccess) return bail(e, "hipEventCreate");
    if ((e = hipHostMalloc((void **)&g->h_flags, sizeof(uint32_t) * kSegment,
                           hipHostMallocDefault)) != hipSuccess)
        return bail(e, "hipHostMalloc");
    if ((e = hipHostMalloc((void **)&g->h_out, sizeof(double) * 2ull * std::max<uint32_t>(g->n, 1u),
                           hipHostMallocDefault)) != hipSuccess)
        return bail(e, "hipHostMalloc");
    if ((e = dmalloc((void **)&g->d_bytes, std::max<uint64_t>(g->n_bytes, 16))) != hipSuccess)
        return bail(e, "device allocation (bytes)");
    if ((e = dmalloc((void **)&g->d_offsets, sizeof(uint64_t) * ((uint64_t)g->n + 1))) != hipSuccess)
        return bail(e, "device allocation (offsets)");
    if ((e = dmalloc((void **)&g->d_cprev, sizeof(double) * g->n)) != hipSuccess)
        return bail(e, "device allocation (c_prev)");
    if ((e = dmalloc((void **)&g->d_sumd, sizeof(double) * g->n)) != hipSuccess)
        return bail(e, "device allocation (sum_d)");
    g->n_flags = (uint64_t)g->n + 2;
    if ((e = dmalloc((void **)&g->d_flags, sizeof(uint32_t) * g->n_flags)) != hipSuccess)
        return bail(e, "device allocation (flags)");
    if (g->n_bytes &&
        (e = hipMemcpy(g->d_bytes, csr->bytes, g->n_bytes, hipMemcpyHostToDevice)) != hipSuccess)
        return bail(e, "hipMemcpy(bytes)");
    if ((e = hipMemcpy(g->d_offsets, csr->offsets, sizeof(uint64_t) * ((uint64_t)g->n + 1),
                       hipMemcpyHostToDevice)) != hipSuccess)
        return bail(e, "hipMemcpy(offsets)");
    for (const auto &opt : {std::make_pair(csr->order, &g->d_order),
                            std::make_pair(csr->hash_ids, &g->d_hash_ids),
                            std::make_pair(csr->degrees, &g->d_degrees),
                            std::make_pair(csr->comp_size, &g->d_comp)}) {
        if (!opt.first) continue;
        if ((e = dmalloc((void **)opt.second, sizeof(uint32_t) * g->n)) != hipSuccess)
            return bail(e, "device allocation (per-node array)");
        if ((e = hipMemcpy(*opt.second, opt.first, sizeof(uint32_t) * g->n,
                           hipMemcpyHostToDevice)) != hipSuccess)
            return bail(e, "hipMemcpy(per-node array)");
    }
    if (csr->xy) {
        if ((e = dmalloc((void **)&g->d_xy, 8ull * g->n)) != hipSuccess)
            return bail(e, "device allocation (xy)");
        if ((e = hipMemcpy(g->d_xy, csr->xy, 8ull * g->n, hipMemcpyHostToDevice)) != hipSuccess)
            return bail(e, "hipMemcpy(xy)");
    }
    // the run kernel reads each row as its list of runs, decoded here once; a
    // graph whose run list does not fit loads without it (per-edge kernel only)
    uint64_t total = 0;
    e = build_run_list(g, true, &g->d_runs, &g->d_run_off, &total);
    if (e == hipErrorOutOfMemory) {
        (void)hipGetLastError();
    } else if (e != hipSuccess) {
        return bail(e, "run list");
    } else if (total != g->runs.runs) {
        graph_release(g);
        return fail(HB_EDEVICE, "run list: %llu runs on the device, %llu on the host",
                    (unsigned long long)total, (unsigned long long)rc.runs);
    }
    {
        const uint64_t n = g->n;
        uint64_t b = std::max<uint64_t>(g->n_bytes, 16) + 8 * (n + 1) + 16 * n + 4 * g->n_flags;
        for (const void *a : {(const void *)csr->order, (const void *)csr->hash_ids,
                              (const void *)csr->degrees, (const void *)csr->comp_size})
            if (a) b += 4 * n;
        if (g->d_runs) b += 8 * std::max<uint64_t>(total, 1) + 8 * (n + 1);
        if (csr->xy) b += 8 * n;
        g->dev_bytes = b;
    }
    // the grouped kernel's row lists, for tables of the default depth
    if (g->d_runs) (void)build_group_lists(g, std::min(kDefaultLevels, floor_log2(g->n)), csr->order);
    *out = g;
    return HB_OK;
}

hb_status hb_graph_free(hb_graph *g) {
    if (!g) return fail(HB_EINVAL, "graph is NULL");
    if (g->inflight.load() != 0)
        return fail(HB_EBUSY, "graph has %u submitted requests that have not finished",
                    g->inflight.load());
    std::lock_guard<std::mutex> lk(g_dev_mu);
    graph_release(g);
    return HB_OK;
}

hb_status hb_graph_info(const hb_graph *g, uint32_t *n, uint64_t *n_edges, uint64_t *n_bytes) {
    if (!g) return fail(HB_EINVAL, "graph is NULL");
    if (n) *n = g->n;
    if (n_edges) *n_edges = g->n_edges;
    if (n_bytes) *n_bytes = g->n_bytes;
    return HB_OK;
}

hb_status hb_graph_stats(const hb_graph *g, hb_graph_stats_t *out) {
    if (!g || !out) return fail(HB_EINVAL, "NULL argument");
    out->n = g->n;
    out->n_edges = g->n_edges;
    out->n_bytes = g->n_bytes;
    out->n_runs = g->runs.runs;
    for (int k = 0; k <= kMaxLevels; ++k) out->table_rows[k] = g->runs.lookups[k];
    out->local_run_reads = g->runs.local_reads;
    out->group_rows = g->grp_entries;
    out->group_levels = g->grp_levels;
    return HB_OK;
}

hb_status hb_run(hb_graph *g, uint32_t p, uint32_t depth_limit, uint64_t hash_seed,
                 hb_result *out) {
    return hb_run_with(g, p, depth_limit, hash_seed, nullptr, out);
}

}  // extern "C"

namespace {

// Pool memory taken for one call, returned when the call ends.
struct PoolHold {
    void *p = nullptr;
    ~PoolHold() { pool_give(p); }
};

// One blocking run (Alg. 1).  Steps are enqueued kSegment at a time without a
// host synchronisation in between: each table and union launch of step t > 1
// first reads step t - 1's stop flag and returns at once when that step grew no
// estimate by more than the threshold, so steps queued past the stopping point
// change nothing.  After each segment the host reads the segment's flags and
// either finds the step that stopped the run or queues the next segment.
// no_alloc: the counter buffers live in the static device workspace, and
// nothing is allocated on the device or the host (no schedule measurement).
hb_status run_blocking(hb_graph *g, uint32_t p, uint32_t depth_limit, uint64_t hash_seed,
                       const hb_run_opts *opts, hb_result *out, bool no_alloc) {
    const uint64_t t_start = now_ns();
    if (!g || !out) return fail(HB_EINVAL, "NULL argument");
    if (p < HB_P_MIN || p > HB_P_MAX) return fail(HB_EINVAL, "p = %u outside [4, 16]", p);
    const hb_run_opts o = opts ? *opts : hb_run_opts{};
    const hb_options lib = options();
    if (o.union_kernel > HB_UNION_GROUPS)
        return fail(HB_EINVAL, "unknown union kernel %u", o.union_kernel);
    if (o.union_kernel == HB_UNION_RUNS && p > 12)
        return fail(HB_EINVAL, "the run kernel supports p <= 12");
    if (o.union_kernel == HB_UNION_GROUPS &&
        !hbk::group_ok((int)p, o.register_bits ? o.register_bits : 8u))
        return fail(HB_EINVAL,
                    "the grouped kernel supports p = 8..12 (8-bit registers) or 9..12 (4-bit)");
    if (o.table_levels > 24) return fail(HB_EINVAL, "table_levels %u > 24", o.table_levels);
    const bool depth_only = lib.stop_rule == HB_STOP_DEPTH;
    if (depth_only && depth_limit == 0)
        return fail(HB_EINVAL, "the stop rule HB_STOP_DEPTH needs a depth limit");
    const double thr = lib.stop_delta > 0.0 ? lib.stop_delta : 0.5;
    hbk::Sched fixed{};
    hb_status st = explicit_sched(o, p, &fixed);
    if (st != HB_OK) return st;
    const uint32_t bits = fixed.bits;
    std::lock_guard<std::mutex> lk(g_dev_mu);
    HB_HIP(hipSetDevice(g->device));
    const uint32_t n = g->n;
    const uint64_t m = (1ull << p) * bits / 8u;  // bytes per counter

    // kernel choice and table depth
    uint32_t levels = o.table_levels ? o.table_levels : kDefaultLevels;
    levels = std::min(levels, floor_log2(n));
    const bool have_groups = g->d_grp_rows && levels == g->grp_levels;
    if (o.union_kernel == HB_UNION_GROUPS && !have_groups)
        return fail(HB_EINVAL, "the graph has no group lists for table depth %u", levels);
    // the grouped kernel is the default where it is built (counters of 256 to
    // 4096 bytes) and the graph has enough groups to fill the device (on a
    // 709-node graph a grouped launch takes 43 us against 12 us for the run kernel)
    bool groups = o.union_kernel == HB_UNION_GROUPS ||
                  (o.union_kernel == HB_UNION_AUTO && hbk::group_ok((int)p, bits) &&
                   have_groups && n >= kGroupsMinNodes);
    bool runs = groups || (o.union_kernel == HB_UNION_RUNS) ||
                (o.union_kernel == HB_UNION_AUTO && p <= 12);
    if (runs && (uint64_t)(levels + 1) * n >= (1ull << 32)) {
        if (o.union_kernel == HB_UNION_RUNS)
            return fail(HB_EINVAL, "table rows (levels + 1) * n must stay below 2^32");
        runs = false;
    }
    if (runs && !g->d_runs) {
        if (o.union_kernel == HB_UNION_RUNS)
            return fail(HB_ENOMEM, "the graph's run list did not fit in device memory at load");
        runs = false;
    }
    // both counter buffers (with the run kernel's table levels) in one piece
    const auto buf_bytes = [&](bool r) {
        return ((uint64_t)n * m * (r ? (levels + 1u) : 1u) + 255u) & ~255ull;
    };
    uint8_t *ws = nullptr;
    PoolHold hold;
    if (no_alloc) {
        const auto fits = [&](bool r) { return 2ull * buf_bytes(r) <= hbk::kStaticScratchBytes; };
        if (runs && !fits(true) && o.union_kernel == HB_UNION_AUTO) runs = false;
        if (!fits(runs))
            return fail(HB_ENOMEM,
                        "hb_run_static: the counters need 2 x %llu bytes; the static workspace "
                        "holds %llu bytes",
                        (unsigned long long)((uint64_t)n * m * (runs ? (levels + 1u) : 1u)),
                        (unsigned long long)hbk::kStaticScratchBytes);
        HB_HIP(hbk::static_scratch(&ws));
    } else {
        // tables beyond 64 GiB are not worth their memory; the per-edge kernel
        // needs none
        if (runs && o.union_kernel == HB_UNION_AUTO && 2ull * buf_bytes(true) > (64ull << 30))
            runs = false;
        st = pool_take(2ull * buf_bytes(runs), &hold.p);
        if (st == HB_ENOMEM && runs && o.union_kernel == HB_UNION_AUTO) {
            runs = false;
            st = pool_take(2ull * buf_bytes(false), &hold.p);
        }
        if (st != HB_OK) return st;
        ws = static_cast<uint8_t *>(hold.p);
    }
    if (!runs) {
        levels = 0;
        groups = false;  // the tables did not fit: per edge
    }
    uint8_t *const bufs[2] = {ws, ws + buf_bytes(runs)};  // step t reads bufs[(t-1)&1]
    hipStream_t s = lib.stream ? static_cast<hipStream_t>(lib.stream) : g->stream;
    const hbk::Sched init_sched = hbk::default_sched((int)p, bits);

    // ---- union schedule: explicit, cached, measured here, or the default
    const hbk::Sched union_default = hbk::default_sched((int)p, bits, runs);
    hbk::Sched sched = union_default;
    double tune_ms = 0.0;
    const TuneKey key =
        tune_key(p, bits, runs, false, n, runs ? g->runs.lookups[levels] : g->n_edges);
    if (fixed.lanes) {
        sched = fixed;
    } else if (!groups && o.tune != HB_TUNE_OFF && !tune_get(key, &sched)) {
        sched = union_default;
        if (o.tune == HB_TUNE_MEASURE && !no_alloc) {
            // step 1 of this very run, once per candidate; the state is
            // initialised again below, so the trials leave no trace
            const uint64_t t0 = now_ns();
            HB_HIP(hbk::launch_fill_u32(g->d_flags, 0u, g->n_flags, s));
            HB_HIP(hbk::launch_init((int)p, init_sched, bufs[0], g->d_cprev, g->d_sumd, n,
                                    hash_seed, g->d_hash_ids, s));
            if (runs) HB_HIP(hbk::launch_table(bufs[0], n, (uint32_t)m, levels, bits, nullptr, s));
            TunePick pick;
            st = tune_measure((int)p, bits, runs, s, [&](const hbk::Sched &c) {
                return runs ? hbk::launch_union_runs((int)p, c, g->d_runs, g->d_run_off, bufs[0],
                                                     levels, bufs[1], g->d_cprev, g->d_sumd,
                                                     g->d_flags + 1, n, 1u, g->d_order, thr,
                                                     nullptr, s)
                            : hbk::launch_union((int)p, c, g->d_bytes, g->d_offsets, bufs[0],
                                                bufs[1], g->d_cprev, g->d_sumd, g->d_flags + 1, n,
                                                1u, g->d_order, thr, nullptr, s);
            }, &pick);
            if (st != HB_OK) return st;
            tune_put(key, pick);
            sched = pick.s;
            tune_ms = (double)(now_ns() - t0) / 1e6;
        }
    }

    HB_HIP(hbk::launch_fill_u32(g->d_flags, 0u, g->n_flags, s));
    HB_HIP(hipEventRecord(g->ev_init[0], s));
    HB_HIP(hbk::launch_init((int)p, init_sched, bufs[0], g->d_cprev, g->d_sumd, n, hash_seed,
                            g->d_hash_ids, s));
    HB_HIP(hipEventRecord(g->ev_init[1], s));

    // ---- steps, kSegment at a time
    // registers are fixed after D <= n - 1 steps, so step n + 1 at the latest
    // finds no growth; flags has n + 2 entries (index 0 unused)
    const uint32_t last_step = (uint32_t)std::min<uint64_t>(
        depth_limit ? depth_limit : UINT32_MAX, g->n_flags - 2u + 1u);
    double iter_ms = 0.0, table_ms = 0.0;
    uint32_t T = 0, converged = 0, queued = 0;
    while (T == 0) {
        const uint32_t first = queued + 1u;
        const uint32_t end = std::min<uint32_t>(queued + kSegment, last_step);
        for (uint32_t t = first; t <= end; ++t) {
            hipEvent_t *ev = g->ev_step[(t - 1u) % kSegment];
            // a step after one that stopped the run returns at once
            const uint32_t *skip = (t > 1u && !depth_only) ? g->d_flags + (t - 1u) : nullptr;
            uint8_t *cur = bufs[(t - 1u) & 1u], *next = bufs[t & 1u];
            HB_HIP(hipEventRecord(ev[0], s));
            if (runs) HB_HIP(hbk::launch_table(cur, n, (uint32_t)m, levels, bits, skip, s));
            HB_HIP(hipEventRecord(ev[1], s));
            if (groups)
                HB_HIP(hbk::launch_union_groups((int)p, bits, g->d_grp_rows, g->d_grp_mask,
                                                g->d_grp_off, cur, next, g->d_cprev, g->d_sumd,
                                                g->d_flags + t, n, t, g->d_order, thr, skip, s));
            else if (runs)
                HB_HIP(hbk::launch_union_runs((int)p, sched, g->d_runs, g->d_run_off, cur, levels,
                                              next, g->d_cprev, g->d_sumd, g->d_flags + t, n, t,
                                              g->d_order, thr, skip, s));
            else
                HB_HIP(hbk::launch_union((int)p, sched, g->d_bytes, g->d_offsets, cur, next,
                                         g->d_cprev, g->d_sumd, g->d_flags + t, n, t, g->d_order,
                                         thr, skip, s));
            HB_HIP(hipEventRecord(ev[2], s));
        }
        HB_HIP(hipMemcpyAsync(g->h_flags, g->d_flags + first, sizeof(uint32_t) * (end - first + 1u),
                              hipMemcpyDeviceToHost, s));
        HB_HIP(hipStreamSynchronize(s));
        // a step after an early stop returned at once, so its flag is 0 too:
        // the first zero flag is the step that stopped the run
        for (uint32_t t = first; t <= end && T == 0; ++t) {
            const bool grew = g->h_flags[t - first] != 0u;
            if (t == last_step || (!grew && !depth_only)) {
                T = t;
                converged = grew ? 0u : 1u;
            }
        }
        queued = end;  // no stop inside the segment: the run goes on after `end`
        const uint32_t upto = T ? T : end;
        for (uint32_t t = first; t <= upto; ++t) {
            hipEvent_t *ev = g->ev_step[(t - 1u) % kSegment];
            float ms = 0.f;
            HB_HIP(hipEventElapsedTime(&ms, ev[1], ev[2]));
            iter_ms += ms;
            HB_HIP(hipEventElapsedTime(&ms, ev[0], ev[1]));
            table_ms += ms;
        }
    }
    float init_ms = 0.f, run_ms = 0.f;
    HB_HIP(hipEventElapsedTime(&init_ms, g->ev_init[0], g->ev_init[1]));
    HB_HIP(hipEventElapsedTime(&run_ms, g->ev_init[0], g->ev_step[(T - 1u) % kSegment][2]));

    // reach and sums through the graph's pinned staging buffer, then to the caller
    double *h_reach = g->h_out, *h_sum = g->h_out + n;
    if (out->reach)
        HB_HIP(hipMemcpyAsync(h_reach, g->d_cprev, sizeof(double) * n, hipMemcpyDeviceToHost, s));
    if (out->sum_d || out->mean_depth)
        HB_HIP(hipMemcpyAsync(h_sum, g->d_sumd, sizeof(double) * n, hipMemcpyDeviceToHost, s));
    if (out->registers)
        HB_HIP(hipMemcpyAsync(out->registers, bufs[T & 1u], (uint64_t)n * m, hipMemcpyDeviceToHost,
                              s));
    HB_HIP(hipStreamSynchronize(s));
    if (out->reach) memcpy(out->reach, h_reach, sizeof(double) * n);
    if (out->sum_d) memcpy(out->sum_d, h_sum, sizeof(double) * n);
    if (out->mean_depth)
        for (uint32_t v = 0; v < n; ++v) {
            const double nv = g->comp_size.empty() ? (double)n : (double)g->comp_size[v];
            out->mean_depth[v] = nv >= 2.0 ? h_sum[v] / (nv - 1.0) : NAN;
        }
    const double md = (double)(1ull << p);
    out->passes = T;
    out->converged = converged;
    out->productive_iters = converged ? T - 1u : T;
    out->c0 = md * std::log(md / (md - 1.0));
    out->edge_unions = (uint64_t)T * g->n_edges;
    out->init_ms = init_ms;
    out->iter_ms = iter_ms;
    out->table_ms = table_ms;
    out->run_ms = run_ms;
    out->union_kernel = groups ? HB_UNION_GROUPS : (runs ? HB_UNION_RUNS : HB_UNION_EDGES);
    out->table_levels = runs ? levels : 0u;
    out->lanes_per_node = groups ? 64u : sched.lanes;
    out->nodes_per_block = groups ? hbk::group_nodes_per_block((int)p, bits)
                                  : sched.nodes_per_block;
    out->register_bits = bits;
    out->tune_ms = tune_ms;
    out->t_submit_ns = t_start;
    out->t_admit_ns = t_start;
    out->t_start_ns = t_start;
    out->t_end_ns = now_ns();
    return HB_OK;
}

}  // namespace

extern "C" {

hb_status hb_run_with(hb_graph *g, uint32_t p, uint32_t depth_limit, uint64_t hash_seed,
                      const hb_run_opts *opts, hb_result *out) {
    return run_blocking(g, p, depth_limit, hash_seed, opts, out, false);
}

hb_status hb_run_static(hb_graph *g, uint32_t p, uint32_t depth_limit, uint64_t hash_seed,
                        const hb_run_opts *opts, hb_result *out) {
    return run_blocking(g, p, depth_limit, hash_seed, opts, out, true);
}

namespace {

uint64_t align256(uint64_t x) { return (x + 255u) & ~uint64_t(255u); }

// Device buffers of batched calls, kept between calls (grown on demand, held
// until hb_release_cache) so a batch does not pay for allocation every time.
// Guarded by g_dev_mu.
struct BatchCache {
    int device = -1;
    hbk::BatchJob *d_jobs = nullptr;
    hbk::BatchJob *h_jobs = nullptr;  // pinned mirror for the done checks
    uint32_t jobs_cap = 0;
    uint32_t *d_lists = nullptr;
    uint64_t lists_cap = 0;
    hipStream_t stream = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};

    void release() {
        if (device < 0) return;
        (void)hipSetDevice(device);
        if (stream) (void)hipStreamSynchronize(stream);
        for (auto &e : ev)
            if (e) (void)hipEventDestroy(e);
        if (stream) (void)hipStreamDestroy(stream);
        if (h_jobs) (void)hipHostFree(h_jobs);
        dfree(d_lists);
        dfree(d_jobs);
        *this = BatchCache{};
    }

    hipError_t reserve(int dev, uint32_t jobs_need, uint64_t lists_need) {
        if (device != dev) release();
        device = dev;
        hipError_t e = hipSuccess;
        if (!stream) e = hipStreamCreateWithFlags(&stream, hipStreamNonBlocking);
        for (auto &x : ev)
            if (e == hipSuccess && !x) e = hipEventCreate(&x);
        if (e == hipSuccess && jobs_cap < jobs_need) {
            dfree(d_jobs);
            if (h_jobs) (void)hipHostFree(h_jobs);
            d_jobs = nullptr;
            h_jobs = nullptr;
            jobs_cap = 0;
            e = dmalloc((void **)&d_jobs, sizeof(hbk::BatchJob) * jobs_need);
            if (e == hipSuccess)
                e = hipHostMalloc((void **)&h_jobs, sizeof(hbk::BatchJob) * jobs_need,
                                  hipHostMallocDefault);
            if (e == hipSuccess) jobs_cap = jobs_need;
        }
        if (e == hipSuccess && lists_cap < lists_need) {
            dfree(d_lists);
            d_lists = nullptr;
            lists_cap = 0;
            e = dmalloc((void **)&d_lists, sizeof(uint32_t) * lists_need);
            if (e == hipSuccess) lists_cap = lists_need;
        }
        return e;
    }
};
BatchCache g_batch;

// The captured step of one call, destroyed on every exit path.
struct StepGraph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ~StepGraph() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
    }
};

// Jobs of one (p, kernel) class.  Initialisation uses the default schedule,
// the union step the class's own; each has its own block bases.
struct BatchClass {
    uint32_t p;
    bool runs;
    std::vector<uint32_t> list;
    bool groups = false;                    // grouped kernel (its tables as for runs)
    uint64_t nodes = 0, rows = 0;           // tuner shape class
    hbk::Sched sched{};                     // union schedule
    bool measure = false;                   // pick it by measurement in this call
    uint32_t list_off = 0, init_off = 0, init_blocks = 0, base_off = 0, nblocks = 0;

    // Block bases under schedule s: job list[i] owns workgroups [b[i], b[i + 1]).
    std::vector<uint32_t> bases(const std::vector<hbk::BatchJob> &hj, const hbk::Sched &s) const {
        const uint32_t npb = hbk::shape_for((int)p, s).nodes_per_block;
        std::vector<uint32_t> b(1, 0u);
        for (uint32_t j : list) b.push_back(b.back() + (hj[j].n + npb - 1) / npb);
        return b;
    }
    // Block bases of the union step: the grouped kernel's, else those of s.
    std::vector<uint32_t> union_bases(const std::vector<hbk::BatchJob> &hj, const hbk::Sched &s,
                                      uint32_t bits) const {
        if (!groups) return bases(hj, s);
        std::vector<uint32_t> b(1, 0u);
        for (uint32_t j : list) b.push_back(b.back() + hbk::group_blocks((int)p, bits, hj[j].n));
        return b;
    }
};

}  // namespace

hb_status hb_run_batch(const hb_job *jobs, uint32_t n_jobs, const hb_run_opts *opts,
                       hb_result *outs) {
    const uint64_t t_start = now_ns();
    if (!jobs || !outs || n_jobs == 0) return fail(HB_EINVAL, "NULL argument or no jobs");
    if (n_jobs > 65535) return fail(HB_EINVAL, "at most 65535 jobs per batch");
    const hb_run_opts o = opts ? *opts : hb_run_opts{};
    const hb_options lib = options();
    if (o.union_kernel > HB_UNION_GROUPS)
        return fail(HB_EINVAL, "unknown union kernel %u", o.union_kernel);
    if (o.table_levels > 24) return fail(HB_EINVAL, "table_levels %u > 24", o.table_levels);
    for (uint32_t j = 0; j < n_jobs; ++j) {
        hbk::Sched fixed{};
        if (jobs[j].p >= HB_P_MIN && jobs[j].p <= HB_P_MAX) {
            const hb_status st = explicit_sched(o, jobs[j].p, &fixed);
            if (st != HB_OK) return st;
        }
        if (!jobs[j].g) return fail(HB_EINVAL, "job %u has no graph", j);
        if (lib.stop_rule == HB_STOP_DEPTH && jobs[j].depth_limit == 0)
            return fail(HB_EINVAL, "job %u: the stop rule HB_STOP_DEPTH needs a depth limit", j);
        if (jobs[j].p < HB_P_MIN || jobs[j].p > HB_P_MAX)
            return fail(HB_EINVAL, "job %u: p = %u outside [4, 16]", j, jobs[j].p);
        if (o.union_kernel == HB_UNION_RUNS && jobs[j].p > 12)
            return fail(HB_EINVAL, "job %u: the run kernel supports p <= 12", j);
        if (o.union_kernel == HB_UNION_GROUPS &&
            !hbk::group_ok((int)jobs[j].p, o.register_bits ? o.register_bits : 8u))
            return fail(HB_EINVAL, "job %u: no grouped kernel for p = %u", j, jobs[j].p);
        if (jobs[j].g->device != jobs[0].g->device)
            return fail(HB_EINVAL, "all graphs of a batch must live on one device");
    }
    const uint32_t bits = o.register_bits ? o.register_bits : 8u;  // checked per job above
    std::lock_guard<std::mutex> lk(g_dev_mu);
    HB_HIP(hipSetDevice(jobs[0].g->device));

    // ---- per-job layout in one arena; all stop flags contiguous at the end
    std::vector<hbk::BatchJob> hj(n_jobs);
    std::vector<uint64_t> off_buf(n_jobs), off_state(n_jobs), off_flags(n_jobs);
    uint64_t arena = 0, flags_words = 0;
    uint32_t max_levels = 0, max_steps = 0;
    for (uint32_t j = 0; j < n_jobs; ++j) {
        const hb_graph *g = jobs[j].g;
        const uint32_t p = jobs[j].p;
        const uint64_t m = (1ull << p) * bits / 8u;  // bytes per counter
        uint32_t levels = std::min(o.table_levels ? o.table_levels : kDefaultLevels, floor_log2(g->n));
        bool runs = o.union_kernel == HB_UNION_RUNS || o.union_kernel == HB_UNION_GROUPS ||
                    (o.union_kernel == HB_UNION_AUTO && p <= 12);
        if (runs && (uint64_t)(levels + 1) * g->n >= (1ull << 32)) {
            if (o.union_kernel == HB_UNION_RUNS)
                return fail(HB_EINVAL, "job %u: table rows (levels + 1) * n must stay below 2^32", j);
            runs = false;
        }
        if (runs && !g->d_runs) {
            if (o.union_kernel == HB_UNION_RUNS)
                return fail(HB_ENOMEM, "job %u: the graph's run list did not fit at load", j);
            runs = false;
        }
        if (!runs) levels = 0;
        // the grouped kernel where it is built and the graph has its lists for this
        // table depth, as in a blocking run
        const bool can_groups = runs && hbk::group_ok((int)p, bits) && g->d_grp_rows &&
                                levels == g->grp_levels;
        if (o.union_kernel == HB_UNION_GROUPS && !can_groups)
            return fail(HB_EINVAL, "job %u: the graph has no group lists for table depth %u", j,
                        levels);
        const bool groups = o.union_kernel == HB_UNION_GROUPS ||
                            (o.union_kernel == HB_UNION_AUTO && can_groups &&
                             g->n >= kGroupsMinNodes);
        hbk::BatchJob &b = hj[j];
        b = hbk::BatchJob{};
        b.bytes = g->d_bytes;
        b.offsets = g->d_offsets;
        b.run_list = g->d_runs;
        b.run_off = g->d_run_off;
        b.order = g->d_order;
        b.hash_ids = g->d_hash_ids;
        b.seed = jobs[j].hash_seed;
        b.n = g->n;
        b.p = p;
        b.depth = jobs[j].depth_limit;
        b.levels = levels;
        b.n_flags = (uint32_t)std::min<uint64_t>((uint64_t)g->n + 2, UINT32_MAX);
        b.runs = runs ? 1u : 0u;
        b.bits = bits;
        b.depth_only = lib.stop_rule == HB_STOP_DEPTH ? 1u : 0u;
        b.stop_delta = lib.stop_delta > 0.0 ? lib.stop_delta : 0.5;
        if (groups) {
            b.groups = 1u;
            b.grp_rows = g->d_grp_rows;
            b.grp_mask = g->d_grp_mask;
            b.grp_off = g->d_grp_off;
        }
        off_buf[j] = arena;
        arena += 2 * align256((uint64_t)g->n * m * (levels + 1u));
        off_state[j] = arena;
        arena += 2 * align256(sizeof(double) * g->n);
        off_flags[j] = flags_words;
        flags_words += b.n_flags;
        max_levels = std::max(max_levels, levels);
        max_steps = std::max(max_steps, b.depth ? b.depth : b.n_flags);
    }
    const uint64_t flags_at = arena;
    arena += align256(sizeof(uint32_t) * flags_words);
    {
        // lists: all jobs, run-kernel jobs, per-level table bases, per-class list + bases
        // (+ tuning: the block bases of every candidate schedule of a class)
        const uint64_t lists_need = 3ull * n_jobs + (uint64_t)(max_levels + 1) * (n_jobs + 1) +
                                    16ull * (n_jobs + 1) + 16ull * (n_jobs + 64);
        const hipError_t e = g_batch.reserve(jobs[0].g->device, n_jobs, lists_need);
        if (e == hipErrorOutOfMemory)
            return fail(HB_ENOMEM, "batch job tables do not fit in device memory");
        if (e != hipSuccess) return hip_fail(e, "batch workspace");
    }
    PoolHold arena_hold;  // every job's counters, tables, state and flags
    {
        const hb_status st = pool_take(arena, &arena_hold.p);
        if (st != HB_OK) return st;
    }
    BatchCache &R = g_batch;
    StepGraph SG;
    uint8_t *base = static_cast<uint8_t *>(arena_hold.p);
    uint32_t *d_flags = reinterpret_cast<uint32_t *>(base + flags_at);
    for (uint32_t j = 0; j < n_jobs; ++j) {
        const uint64_t m = (1ull << jobs[j].p) * bits / 8u;
        const uint64_t bb = align256((uint64_t)hj[j].n * m * (hj[j].levels + 1u));
        hj[j].buf[0] = base + off_buf[j];
        hj[j].buf[1] = base + off_buf[j] + bb;
        hj[j].c_prev = reinterpret_cast<double *>(base + off_state[j]);
        hj[j].sum_d = reinterpret_cast<double *>(base + off_state[j] + align256(sizeof(double) * hj[j].n));
        hj[j].flags = d_flags + off_flags[j];
    }

    // ---- classes by (p, kernel) and their union schedules
    std::vector<BatchClass> classes;
    std::vector<uint32_t> all_list(n_jobs), runs_list;
    for (uint32_t j = 0; j < n_jobs; ++j) {
        all_list[j] = j;
        if (hj[j].runs) runs_list.push_back(j);
        BatchClass *c = nullptr;
        for (auto &x : classes)
            if (x.p == hj[j].p && x.runs == (hj[j].runs != 0) && x.groups == (hj[j].groups != 0))
                c = &x;
        if (!c) {
            classes.push_back(BatchClass{hj[j].p, hj[j].runs != 0, {}});
            c = &classes.back();
            c->groups = hj[j].groups != 0;
        }
        c->list.push_back(j);
        c->nodes += hj[j].n;
        c->rows += hj[j].runs ? jobs[j].g->runs.lookups[hj[j].levels] : jobs[j].g->n_edges;
    }
    bool any_measure = false;
    for (auto &c : classes) {
        hbk::Sched fixed{};
        (void)explicit_sched(o, c.p, &fixed);
        c.sched = hbk::default_sched((int)c.p, bits, c.runs);
        if (c.groups) {
            // one launch shape: nothing to tune
        } else if (fixed.lanes) {
            c.sched = fixed;
        } else if (o.tune != HB_TUNE_OFF &&
                   !tune_get(tune_key(c.p, bits, c.runs, true, c.nodes, c.rows), &c.sched)) {
            c.sched = hbk::default_sched((int)c.p, bits, c.runs);
            c.measure = o.tune == HB_TUNE_MEASURE;
            any_measure = any_measure || c.measure;
        }
    }
    // ---- lists: all jobs, run-kernel jobs, table bases, per class list + init bases
    std::vector<uint32_t> lists(all_list);
    const uint32_t runs_off = (uint32_t)lists.size();
    lists.insert(lists.end(), runs_list.begin(), runs_list.end());
    // table level k: job runs_list[i] owns workgroups [tb[k][i], tb[k][i+1])
    std::vector<uint32_t> table_off(max_levels + 1, 0), table_blocks(max_levels + 1, 0);
    for (uint32_t k = 1; k <= max_levels; ++k) {
        table_off[k] = (uint32_t)lists.size();
        uint32_t acc = 0;
        lists.push_back(0);
        for (uint32_t j : runs_list) {
            if (k <= hj[j].levels)
                acc += hbk::batch_table_blocks(hj[j].n, (1u << hj[j].p) * bits / 8u, k);
            lists.push_back(acc);
        }
        table_blocks[k] = acc;
    }
    for (auto &c : classes) {
        c.list_off = (uint32_t)lists.size();
        lists.insert(lists.end(), c.list.begin(), c.list.end());
        const std::vector<uint32_t> ib = c.bases(hj, hbk::default_sched((int)c.p, bits));
        c.init_off = (uint32_t)lists.size();
        lists.insert(lists.end(), ib.begin(), ib.end());
        c.init_blocks = ib.back();
    }
    // the candidates' block bases of every class measured in this call
    std::vector<std::vector<hbk::Sched>> cands(classes.size());
    std::vector<std::vector<uint32_t>> cand_off(classes.size()), cand_blocks(classes.size());
    for (size_t ci = 0; ci < classes.size(); ++ci) {
        if (!classes[ci].measure) continue;
        cands[ci] = tune_candidates((int)classes[ci].p, bits, classes[ci].runs);
        for (const auto &cs : cands[ci]) {
            const std::vector<uint32_t> b = classes[ci].bases(hj, cs);
            cand_off[ci].push_back((uint32_t)lists.size());
            cand_blocks[ci].push_back(b.back());
            lists.insert(lists.end(), b.begin(), b.end());
        }
    }
    const size_t phase_a = lists.size();
    if (phase_a > R.lists_cap) return fail(HB_EDEVICE, "batch list buffer too small");
    // room for the union bases appended below: the copy of the first part may
    // still read this buffer, so it must not move
    lists.reserve(phase_a + n_jobs + classes.size());
    hipStream_t s = R.stream;
    HB_HIP(hipMemcpyAsync(R.d_jobs, hj.data(), sizeof(hbk::BatchJob) * n_jobs,
                          hipMemcpyHostToDevice, s));
    HB_HIP(hipMemcpyAsync(R.d_lists, lists.data(), sizeof(uint32_t) * lists.size(),
                          hipMemcpyHostToDevice, s));
    auto init_all = [&]() -> hb_status {
        HB_HIP(hbk::launch_fill_u32(d_flags, 0u, flags_words, s));
        for (auto &c : classes)
            HB_HIP(hbk::launch_batch_init((int)c.p, hbk::default_sched((int)c.p, bits), R.d_jobs,
                                          R.d_lists + c.list_off, R.d_lists + c.init_off,
                                          (uint32_t)c.list.size(), c.init_blocks, s));
        return HB_OK;
    };

    // ---- measure the union schedules of untuned classes on step 1 of this batch
    double tune_ms = 0.0;
    if (any_measure) {
        const uint64_t t0 = now_ns();
        hb_status st = init_all();
        if (st != HB_OK) return st;
        for (uint32_t k = 1; k <= max_levels; ++k)
            HB_HIP(hbk::launch_batch_table(R.d_jobs, R.d_lists + runs_off, R.d_lists + table_off[k],
                                           (uint32_t)runs_list.size(), table_blocks[k], k, s));
        for (size_t ci = 0; ci < classes.size(); ++ci) {
            BatchClass &c = classes[ci];
            if (!c.measure) continue;
            size_t idx = 0;
            TunePick pick;
            st = tune_measure((int)c.p, bits, c.runs, s, [&](const hbk::Sched &cs) {
                idx = 0;
                while (idx < cands[ci].size() && !(cands[ci][idx].lanes == cs.lanes &&
                                                   cands[ci][idx].nodes_per_block == cs.nodes_per_block))
                    ++idx;
                if (idx == cands[ci].size()) return hipErrorInvalidValue;
                return hbk::launch_batch_union((int)c.p, cs, c.runs, R.d_jobs,
                                               R.d_lists + c.list_off, R.d_lists + cand_off[ci][idx],
                                               (uint32_t)c.list.size(), cand_blocks[ci][idx], s);
            }, &pick);
            if (st != HB_OK) return st;
            tune_put(tune_key(c.p, bits, c.runs, true, c.nodes, c.rows), pick);
            c.sched = pick.s;
        }
        HB_HIP(hipStreamSynchronize(s));
        tune_ms = (double)(now_ns() - t0) / 1e6;
    }
    // ---- the union bases of the chosen schedules
    for (auto &c : classes) {
        const std::vector<uint32_t> b = c.union_bases(hj, c.sched, bits);
        c.base_off = (uint32_t)lists.size();
        lists.insert(lists.end(), b.begin(), b.end());
        c.nblocks = b.back();
    }
    if (lists.size() > R.lists_cap) return fail(HB_EDEVICE, "batch list buffer too small");
    HB_HIP(hipMemcpyAsync(R.d_lists + phase_a, lists.data() + phase_a,
                          sizeof(uint32_t) * (lists.size() - phase_a), hipMemcpyHostToDevice, s));

    // ---- init
    HB_HIP(hipEventRecord(R.ev[0], s));
    {
        const hb_status st = init_all();
        if (st != HB_OK) return st;
    }

    // ---- one step, captured once, replayed until every job has stopped
    HB_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    {
        hipError_t e = hipSuccess;
        for (uint32_t k = 1; k <= max_levels && e == hipSuccess; ++k)
            e = hbk::launch_batch_table(R.d_jobs, R.d_lists + runs_off, R.d_lists + table_off[k],
                                        (uint32_t)runs_list.size(), table_blocks[k], k, s);
        for (auto &c : classes) {
            if (e != hipSuccess) break;
            e = c.groups ? hbk::launch_batch_groups((int)c.p, bits, R.d_jobs,
                                                    R.d_lists + c.list_off,
                                                    R.d_lists + c.base_off,
                                                    (uint32_t)c.list.size(), c.nblocks, s)
                         : hbk::launch_batch_union((int)c.p, c.sched, c.runs, R.d_jobs,
                                                   R.d_lists + c.list_off,
                                                   R.d_lists + c.base_off,
                                                   (uint32_t)c.list.size(), c.nblocks, s);
        }
        if (e == hipSuccess) e = hbk::launch_batch_step_end(R.d_jobs, R.d_lists, n_jobs, s);
        const hipError_t e2 = hipStreamEndCapture(s, &SG.graph);
        if (e != hipSuccess) return hip_fail(e, "batched step launch");
        if (e2 != hipSuccess) return hip_fail(e2, "hipStreamEndCapture");
    }
    HB_HIP(hipGraphInstantiate(&SG.exec, SG.graph, nullptr, nullptr, 0));
    const uint32_t steps_per_check = 4;
    uint32_t steps = 0;
    for (;;) {
        for (uint32_t i = 0; i < steps_per_check; ++i) HB_HIP(hipGraphLaunch(SG.exec, s));
        steps += steps_per_check;
        HB_HIP(hipEventRecord(R.ev[1], s));
        HB_HIP(hipMemcpyAsync(R.h_jobs, R.d_jobs, sizeof(hbk::BatchJob) * n_jobs,
                              hipMemcpyDeviceToHost, s));
        HB_HIP(hipStreamSynchronize(s));
        bool all = true;
        for (uint32_t j = 0; j < n_jobs; ++j) all = all && R.h_jobs[j].done != 0u;
        if (all) break;
        if (steps > max_steps + steps_per_check)
            return fail(HB_EDEVICE, "batched run did not stop within %u steps", steps);
    }
    float run_ms = 0.f;
    HB_HIP(hipEventElapsedTime(&run_ms, R.ev[0], R.ev[1]));

    // ---- outputs
    for (uint32_t j = 0; j < n_jobs; ++j) {
        const hbk::BatchJob &b = R.h_jobs[j];
        hb_result *out = &outs[j];
        const uint32_t n = b.n;
        const uint64_t m = (1ull << b.p) * bits / 8u;
        if (out->reach)
            HB_HIP(hipMemcpy(out->reach, b.c_prev, sizeof(double) * n, hipMemcpyDeviceToHost));
        if (out->sum_d || out->mean_depth) {
            std::vector<double> tmp;
            double *sd = out->sum_d;
            if (!sd) {
                tmp.resize(n);
                sd = tmp.data();
            }
            HB_HIP(hipMemcpy(sd, b.sum_d, sizeof(double) * n, hipMemcpyDeviceToHost));
            if (out->mean_depth) {
                const hb_graph *g = jobs[j].g;
                for (uint32_t v = 0; v < n; ++v) {
                    const double nv = g->comp_size.empty() ? (double)n : (double)g->comp_size[v];
                    out->mean_depth[v] = nv >= 2.0 ? sd[v] / (nv - 1.0) : NAN;
                }
            }
        }
        if (out->registers)
            HB_HIP(hipMemcpy(out->registers, b.buf[b.done & 1u], (uint64_t)n * m,
                             hipMemcpyDeviceToHost));
        const double md = (double)(1ull << b.p);
        out->passes = b.done;
        out->converged = b.converged;
        out->productive_iters = b.converged ? b.done - 1u : b.done;
        out->c0 = md * std::log(md / (md - 1.0));
        out->edge_unions = (uint64_t)b.done * jobs[j].g->n_edges;
        out->init_ms = 0.0;
        out->iter_ms = 0.0;
        out->table_ms = 0.0;
        out->run_ms = run_ms;
        out->union_kernel = b.groups ? HB_UNION_GROUPS : (b.runs ? HB_UNION_RUNS : HB_UNION_EDGES);
        out->table_levels = b.levels;
        for (const auto &c : classes)
            if (c.p == b.p && c.runs == (b.runs != 0) && c.groups == (b.groups != 0)) {
                out->lanes_per_node = c.groups ? 64u : c.sched.lanes;
                out->nodes_per_block = c.groups ? hbk::group_nodes_per_block((int)b.p, bits)
                                                : c.sched.nodes_per_block;
            }
        out->register_bits = bits;
        out->tune_ms = tune_ms;
        out->t_submit_ns = t_start;
        out->t_admit_ns = t_start;
        out->t_start_ns = t_start;
        out->t_end_ns = now_ns();
    }
    return HB_OK;
}

hb_status hb_vga_metrics(hb_graph *g, const double *sum_d, hb_vga_out *out) {
    if (!g || !sum_d || !out) return fail(HB_EINVAL, "NULL argument");
    double *dst[9] = {out->connectivity, out->control, out->mean_depth, out->relative_asymmetry,
                      out->integration_hh, out->integration_tekl, out->integration_pvalue,
                      out->point_first_moment, out->point_second_moment};
    std::lock_guard<std::mutex> lk(g_dev_mu);
    HB_HIP(hipSetDevice(g->device));
    const uint64_t n = g->n;
    double *d_sum = nullptr, *d_out = nullptr;
    hipError_t e = dmalloc((void **)&d_sum, sizeof(double) * n);
    if (e == hipSuccess) e = dmalloc((void **)&d_out, sizeof(double) * 9 * n);
    if (e == hipSuccess) e = hipMemcpyAsync(d_sum, sum_d, sizeof(double) * n, hipMemcpyHostToDevice,
                                            g->stream);
    if (e == hipSuccess)
        e = hbk::launch_vga(g->d_bytes, g->d_offsets, g->d_degrees, g->d_comp, g->d_xy, d_sum,
                            g->n, d_out, g->stream);
    for (int i = 0; i < 9 && e == hipSuccess; ++i)
        if (dst[i])
            e = hipMemcpyAsync(dst[i], d_out + (uint64_t)i * n, sizeof(double) * n,
                               hipMemcpyDeviceToHost, g->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
    (void)hipStreamSynchronize(g->stream);
    dfree(d_out);
    dfree(d_sum);
    if (e == hipErrorOutOfMemory) return fail(HB_ENOMEM, "VGA metrics: out of device memory");
    if (e != hipSuccess) return hip_fail(e, "VGA metrics");
    return HB_OK;
}

hb_status hb_local_metrics(hb_graph *g, hb_local_out *out) {
    if (!g || !out) return fail(HB_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(g_dev_mu);
    HB_HIP(hipSetDevice(g->device));
    const uint32_t n = g->n;
    int lim = 0;
    HB_HIP(hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, g->device));
    // two bitmaps of n bits, plus 12 bytes of partial sums per wave
    const uint64_t lds = 8ull * ((n + 31ull) / 32ull) + 12ull * (hbk::local_threads() / 64u);
    if (lds > (uint64_t)lim)
        return fail(HB_EINVAL,
                    "local metrics: n = %u needs %llu bytes of LDS per workgroup; the device "
                    "has %d",
                    n, (unsigned long long)lds, lim);
    uint32_t *d_ball = nullptr;
    uint64_t *d_off = nullptr, *d_pairs = nullptr;
    uint2 *d_runs = nullptr;
    double *d_clus = nullptr, *d_ctrl = nullptr;
    // the plain maximal runs of every row (v is no neighbour of itself)
    uint64_t total = 0;
    hipError_t e = build_run_list(g, false, &d_runs, &d_off, &total);
    if (e == hipSuccess) e = dmalloc((void **)&d_pairs, sizeof(uint64_t) * n);
    if (e == hipSuccess) e = dmalloc((void **)&d_ball, sizeof(uint32_t) * n);
    if (e == hipSuccess) e = dmalloc((void **)&d_clus, sizeof(double) * n);
    if (e == hipSuccess) e = dmalloc((void **)&d_ctrl, sizeof(double) * n);
    if (e == hipSuccess)
        e = hbk::launch_local(d_runs, d_off, g->d_degrees, n, g->d_order, d_pairs, d_ball, d_clus,
                              d_ctrl, (uint32_t)lim, g->stream);
    if (e == hipSuccess && out->pairs)
        e = hipMemcpyAsync(out->pairs, d_pairs, sizeof(uint64_t) * n, hipMemcpyDeviceToHost,
                           g->stream);
    if (e == hipSuccess && out->ball2)
        e = hipMemcpyAsync(out->ball2, d_ball, sizeof(uint32_t) * n, hipMemcpyDeviceToHost,
                           g->stream);
    if (e == hipSuccess && out->clustering)
        e = hipMemcpyAsync(out->clustering, d_clus, sizeof(double) * n, hipMemcpyDeviceToHost,
                           g->stream);
    if (e == hipSuccess && out->controllability)
        e = hipMemcpyAsync(out->controllability, d_ctrl, sizeof(double) * n,
                           hipMemcpyDeviceToHost, g->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
    (void)hipStreamSynchronize(g->stream);
    for (void *p : {(void *)d_off, (void *)d_runs, (void *)d_pairs, (void *)d_ball,
                    (void *)d_clus, (void *)d_ctrl})
        dfree(p);
    if (e == hipErrorOutOfMemory) return fail(HB_ENOMEM, "local metrics: out of device memory");
    if (e != hipSuccess) return hip_fail(e, "local metrics");
    return HB_OK;
}

hb_status hb_release_cache(void) {
    std::lock_guard<std::mutex> lk(g_dev_mu);
    g_batch.release();
    pool_trim_all();
    return HB_OK;
}

hb_status hb_gather_probe(uint32_t p, uint32_t lanes_per_node, uint32_t nodes_per_block,
                          uint32_t table_rows, uint32_t n_nodes, uint32_t rows_per_node,
                          uint32_t with_max, uint32_t reps, double *avg_ms) {
    if (!avg_ms || reps == 0 || n_nodes == 0) return fail(HB_EINVAL, "bad probe arguments");
    if (p < HB_P_MIN || p > 12) return fail(HB_EINVAL, "the gather probe supports p in [4, 12]");
    if (table_rows == 0 || (table_rows & (table_rows - 1u)))
        return fail(HB_EINVAL, "table_rows must be a power of two");
    hbk::Sched sc = lanes_per_node ? hbk::Sched{lanes_per_node, nodes_per_block, 8u}
                                   : hbk::default_sched((int)p, 8u, true);
    if (!sc.nodes_per_block) sc.nodes_per_block = sc.lanes > 64u ? 1u : 4u;
    if (!hbk::sched_ok((int)p, sc))
        return fail(HB_EINVAL, "no schedule of %u lanes, %u nodes per workgroup for p = %u",
                    sc.lanes, sc.nodes_per_block, p);
    std::lock_guard<std::mutex> lk(g_dev_mu);
    hb_status st = have_device();
    if (st != HB_OK) return st;
    const uint64_t m = 1ull << p;
    const uint32_t waves = sc.lanes > 64u ? sc.lanes / 64u : 1u;
    void *tbl = nullptr, *out = nullptr;
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = dmalloc(&tbl, table_rows * m);
    if (e == hipSuccess) e = dmalloc(&out, sizeof(uint32_t) * 64ull * waves * n_nodes);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    // registers 1..4: small values like real counters
    if (e == hipSuccess)
        e = hbk::launch_fill_u32(static_cast<uint32_t *>(tbl), 0x01020304u, table_rows * m / 4, s);
    auto launch = [&]() {
        return hbk::launch_gather_probe((int)p, sc, static_cast<const uint8_t *>(tbl), table_rows,
                                        rows_per_node, static_cast<uint32_t *>(out), n_nodes,
                                        with_max ? 1u : 0u, s);
    };
    if (e == hipSuccess) e = launch();  // warm-up: the table settles in the caches
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    for (uint32_t i = 0; e == hipSuccess && i < reps; ++i) e = launch();
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e1) (void)hipEventDestroy(e1);
    if (e0) (void)hipEventDestroy(e0);
    if (s) (void)hipStreamDestroy(s);
    dfree(out);
    dfree(tbl);
    if (e == hipErrorOutOfMemory) return fail(HB_ENOMEM, "gather probe: out of device memory");
    if (e != hipSuccess) return hip_fail(e, "gather probe");
    *avg_ms = ms / reps;
    return HB_OK;
}

hb_status hb_copy_probe(uint64_t bytes, uint32_t reps, double *avg_ms) {
    if (!avg_ms || reps == 0 || bytes < 16 || bytes % 16) return fail(HB_EINVAL, "bad probe size");
    std::lock_guard<std::mutex> lk(g_dev_mu);
    hb_status st = have_device();
    if (st != HB_OK) return st;
    void *a = nullptr, *b = nullptr;
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = dmalloc(&a, bytes);
    if (e == hipSuccess) e = dmalloc(&b, bytes);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = hipMemsetAsync(a, 1, bytes, s);
    if (e == hipSuccess) e = hbk::launch_copy(a, b, bytes, s);  // warm-up
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    for (uint32_t i = 0; e == hipSuccess && i < reps; ++i) e = hbk::launch_copy(a, b, bytes, s);
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e1) (void)hipEventDestroy(e1);
    if (e0) (void)hipEventDestroy(e0);
    if (s) (void)hipStreamDestroy(s);
    dfree(a);
    dfree(b);
    if (e != hipSuccess) return hip_fail(e, "copy probe");
    *avg_ms = ms / reps;
    return HB_OK;
}

}  // extern "C"
