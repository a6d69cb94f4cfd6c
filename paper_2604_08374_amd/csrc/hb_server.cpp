// The served form: hb_submit / hb_poll over a request loop on a library thread.
//
// The loop keeps a table of running requests.  Every iteration it (1) admits
// queued requests in arrival order while their footprint can be taken from the
// library's device memory pool (within the server's own cap, if one is set,
// and the library-wide budget shared with blocking runs and graphs), (2) runs one batched
// HyperBall step over all running requests -- init for the newly admitted,
// range-max table levels for run-kernel requests, one union launch per
// (p, kernel) class, and the per-request stop decision on the device -- and
// (3) retires the requests that stopped: their reach, sums and optionally
// registers are copied to host memory owned by the request record and their
// block is freed at once.  Each request keeps its own step count, so requests
// join and leave between any two steps (continuous batching at step
// granularity).  Requests are split over two lanes by the bytes one of their
// steps gathers: each lane has its own thread, stream and running set, and both
// share the memory, so short requests never wait for the step of a very large
// one and the two kinds overlap on the device.
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <thread>
#include <unordered_map>
#include <vector>

#include "hb.h"
#include "hb_internal.h"
#include "hb_runtime.h"

using namespace hbr;

namespace {

uint64_t align256(uint64_t x) { return (x + 255u) & ~uint64_t(255u); }

enum class State { Queued, Running, Done, Failed };

struct Request {
    hb_ticket ticket = 0;
    hb_graph *g = nullptr;
    uint32_t p = 0, depth = 0, flags = 0;
    uint32_t bits = 8;  // register width
    uint64_t seed = 0;
    bool runs = false;
    bool groups = false;  // grouped kernel (its tables as for runs)
    uint32_t levels = 0;
    uint64_t footprint = 0;
    void *mem = nullptr;  // pool memory while running
    State state = State::Queued;
    hb_status error = HB_OK;
    std::string message;
    hbk::BatchJob job{};
    uint64_t t_submit = 0, t_admit = 0, t_start = 0, t_end = 0;
    std::vector<double> reach, sum_d;
    std::vector<uint8_t> regs;
};

struct Lane {
    std::deque<Request *> queue;        // guarded by Server::mu_
    std::vector<Request *> running;     // owned by the lane thread
    hbk::BatchJob *d_jobs = nullptr, *h_jobs = nullptr;
    uint32_t jobs_cap = 0;
    uint32_t *d_lists = nullptr;
    uint64_t lists_cap = 0;
    hipStream_t stream = nullptr;
    std::thread thread;
    uint32_t n_running = 0;             // guarded by Server::mu_
};

class Server {
public:
    hb_status start(const hb_server_opts *opts);
    hb_status stop();
    hb_status submit(hb_graph *g, uint32_t p, uint32_t depth, uint64_t seed, uint32_t flags,
                     hb_ticket *out);
    hb_status poll(hb_ticket t, hb_result *out, bool block);
    hb_status stats(hb_server_stats_t *out);
    ~Server() {
        // process exit without hb_server_stop: end the loops after their current step
        {
            std::lock_guard<std::mutex> lk(mu_);
            abort_ = true;
            stopping_ = true;
        }
        cv_work_.notify_all();
        for (auto &l : lanes_)
            if (l.thread.joinable()) l.thread.join();
    }

private:
    void loop(Lane &L);
    hb_status step(Lane &L);
    void fail_all(Lane &L, hb_status st, const std::string &msg);
    void retire(Lane &L, Request *r);
    hb_status footprint(const hb_graph *g, uint32_t p, uint32_t bits, bool &runs, bool &groups,
                        uint32_t &levels,
                        uint64_t &bytes) const;

    std::mutex mu_;  // guards everything below that client threads touch
    std::condition_variable cv_work_, cv_done_;
    bool running_ = false, stopping_ = false, abort_ = false;
    hb_server_opts opts_{};
    uint64_t slow_bytes_ = 0;  // a request gathering more per step goes to the slow lane
    int device_ = 0;
    uint64_t cap_ = 0;        // the server's own cap on its memory (0 = none)
    uint64_t used_ = 0, peak_used_ = 0;
    Lane lanes_[2];  // 0: fast, 1: slow
    std::unordered_map<hb_ticket, std::unique_ptr<Request>> reqs_;
    hb_ticket next_ticket_ = 1;
    uint64_t submitted_ = 0, completed_ = 0, steps_ = 0, edge_unions_ = 0;
    uint64_t device_total_ = 0;  // device memory size, for requests that could never fit
};

hb_status Server::footprint(const hb_graph *g, uint32_t p, uint32_t bits, bool &runs,
                            bool &groups, uint32_t &levels, uint64_t &bytes) const {
    const uint64_t m = (1ull << p) * bits / 8u;  // bytes per counter
    levels = std::min(opts_.table_levels ? opts_.table_levels : kDefaultLevels, floor_log2(g->n));
    runs = opts_.union_kernel == HB_UNION_RUNS || opts_.union_kernel == HB_UNION_GROUPS ||
           (opts_.union_kernel == HB_UNION_AUTO && p <= 12);
    const bool forced = opts_.union_kernel == HB_UNION_RUNS || opts_.union_kernel == HB_UNION_GROUPS;
    if (runs && (uint64_t)(levels + 1) * g->n >= (1ull << 32)) {
        if (forced)
            return fail(HB_EINVAL, "table rows (levels + 1) * n must stay below 2^32");
        runs = false;
    }
    if (runs && !g->d_runs) {
        if (forced)
            return fail(HB_ENOMEM, "the graph's run list did not fit in device memory at load");
        runs = false;
    }
    if (!runs) levels = 0;
    // the grouped kernel where it is built, as in a blocking run
    const bool can_groups = runs && hbk::group_ok((int)p, bits) && g->d_grp_rows &&
                            levels == g->grp_levels;
    if (opts_.union_kernel == HB_UNION_GROUPS && !can_groups)
        return fail(HB_EINVAL, "no grouped kernel for p = %u or no group lists for depth %u", p,
                    levels);
    groups = opts_.union_kernel == HB_UNION_GROUPS ||
             (opts_.union_kernel == HB_UNION_AUTO && can_groups && g->n >= kGroupsMinNodes);
    const uint64_t n_flags = (uint64_t)g->n + 2;
    bytes = 2 * align256((uint64_t)g->n * m * (levels + 1u)) + 2 * align256(8ull * g->n) +
            align256(4ull * n_flags);
    return HB_OK;
}

hb_status Server::start(const hb_server_opts *opts) {
    std::lock_guard<std::mutex> lk(mu_);
    if (running_) return fail(HB_EBUSY, "the request loop is already running");
    hb_server_opts o = opts ? *opts : hb_server_opts{};
    if (o.union_kernel > HB_UNION_GROUPS) return fail(HB_EINVAL, "unknown union kernel");
    if (o.table_levels > 24) return fail(HB_EINVAL, "table_levels > 24");
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count < 1) return fail(HB_EDEVICE, "no GPU available");
    HB_HIP(hipGetDevice(&device_));
    {
        size_t free_b = 0, total_b = 0;
        HB_HIP(hipMemGetInfo(&free_b, &total_b));
        device_total_ = total_b;
    }
    for (auto &l : lanes_) {
        const hipError_t e = hipStreamCreateWithFlags(&l.stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            for (auto &x : lanes_)
                if (x.stream) (void)hipStreamDestroy(x.stream), x.stream = nullptr;
            return hip_fail(e, "hipStreamCreate");
        }
    }
    opts_ = o;
    cap_ = o.hbm_budget ? align256(o.hbm_budget) : 0;
    slow_bytes_ = o.slow_lane_bytes ? o.slow_lane_bytes : (2ull << 30);
    used_ = 0;
    peak_used_ = 0;
    running_ = true;
    stopping_ = false;
    abort_ = false;
    for (auto &l : lanes_) l.thread = std::thread([this, &l] { loop(l); });
    return HB_OK;
}

hb_status Server::stop() {
    {
        std::lock_guard<std::mutex> lk(mu_);
        if (!running_) return fail(HB_ENOTFOUND, "the request loop is not running");
        stopping_ = true;
    }
    cv_work_.notify_all();
    for (auto &l : lanes_)
        if (l.thread.joinable()) l.thread.join();
    std::lock_guard<std::mutex> lk(mu_);
    running_ = false;
    return HB_OK;
}

hb_status Server::submit(hb_graph *g, uint32_t p, uint32_t depth, uint64_t seed, uint32_t flags,
                         hb_ticket *out) {
    if (!g || !out) return fail(HB_EINVAL, "NULL argument");
    if (p < HB_P_MIN || p > HB_P_MAX) return fail(HB_EINVAL, "p = %u outside [4, 16]", p);
    if (flags & ~(HB_SUBMIT_REGISTERS | HB_SUBMIT_REG4)) return fail(HB_EINVAL, "unknown submit flags");
    const uint32_t bits = (flags & HB_SUBMIT_REG4) ? 4u : 8u;
    if (bits == 4u && p < 5) return fail(HB_EINVAL, "4-bit registers need p >= 5");
    bool need_start;
    {
        std::lock_guard<std::mutex> lk(mu_);
        need_start = !running_;
    }
    if (need_start) {
        const hb_status st = start(nullptr);
        if (st != HB_OK && st != HB_EBUSY) return st;
    }
    std::lock_guard<std::mutex> lk(mu_);
    if (!running_ || stopping_) return fail(HB_EBUSY, "the request loop is stopping");
    if (g->device != device_) return fail(HB_EINVAL, "graph lives on another device");
    auto r = std::make_unique<Request>();
    if (opts_.union_kernel == HB_UNION_RUNS && p > 12)
        return fail(HB_EINVAL, "the run kernel supports p <= 12");
    hb_status st = footprint(g, p, bits, r->runs, r->groups, r->levels, r->footprint);
    if (st != HB_OK) return st;
    const hb_options lib = options();
    if (lib.stop_rule == HB_STOP_DEPTH && depth == 0)
        return fail(HB_EINVAL, "the stop rule HB_STOP_DEPTH needs a depth limit");
    const uint64_t limit = std::min({cap_ ? cap_ : UINT64_MAX,
                                     lib.hbm_budget ? lib.hbm_budget : UINT64_MAX,
                                     device_total_ ? device_total_ : UINT64_MAX});
    if (align256(r->footprint) > limit)
        return fail(HB_ENOMEM, "request needs %llu bytes, at most %llu can ever be free",
                    (unsigned long long)r->footprint, (unsigned long long)limit);
    r->ticket = next_ticket_++;
    r->g = g;
    r->p = p;
    r->depth = depth;
    r->seed = seed;
    r->flags = flags;
    r->bits = bits;
    r->t_submit = now_ns();
    // bytes one step gathers: counter rows (table rows for the run kernel, the group
    // lists' rows for the grouped one) x counter bytes
    const uint64_t rows = r->groups ? g->grp_entries
                          : r->runs ? g->runs.lookups[r->levels] : g->n_edges;
    const int lane = rows * ((1ull << p) * bits / 8u) > slow_bytes_ ? 1 : 0;
    g->inflight.fetch_add(1);
    *out = r->ticket;
    lanes_[lane].queue.push_back(r.get());
    reqs_.emplace(r->ticket, std::move(r));
    ++submitted_;
    cv_work_.notify_all();
    return HB_OK;
}

hb_status Server::poll(hb_ticket t, hb_result *out, bool block) {
    if (!out) return fail(HB_EINVAL, "out is NULL");
    std::unique_lock<std::mutex> lk(mu_);
    auto it = reqs_.find(t);
    if (it == reqs_.end()) return fail(HB_ENOTFOUND, "unknown or already collected ticket %llu",
                                       (unsigned long long)t);
    Request *r = it->second.get();
    if (block)
        cv_done_.wait(lk, [&] { return r->state == State::Done || r->state == State::Failed; });
    if (r->state == State::Queued || r->state == State::Running) return HB_PENDING;
    if (r->state == State::Failed) {
        const hb_status st = r->error;
        const std::string msg = r->message;
        reqs_.erase(it);
        return fail(st, "%s", msg.c_str());
    }
    if (out->registers && !(r->flags & HB_SUBMIT_REGISTERS))
        return fail(HB_EINVAL, "registers were not kept (submit with HB_SUBMIT_REGISTERS)");
    const uint32_t n = r->g->n;
    const double md = (double)(1u << r->p);
    if (out->reach) memcpy(out->reach, r->reach.data(), sizeof(double) * n);
    if (out->sum_d) memcpy(out->sum_d, r->sum_d.data(), sizeof(double) * n);
    if (out->mean_depth)
        for (uint32_t v = 0; v < n; ++v) {
            const double nv = r->g->comp_size.empty() ? (double)n : (double)r->g->comp_size[v];
            out->mean_depth[v] = nv >= 2.0 ? r->sum_d[v] / (nv - 1.0) : NAN;
        }
    if (out->registers) memcpy(out->registers, r->regs.data(), r->regs.size());
    out->passes = r->job.done;
    out->converged = r->job.converged;
    out->productive_iters = r->job.converged ? r->job.done - 1u : r->job.done;
    out->c0 = md * std::log(md / (md - 1.0));
    out->edge_unions = (uint64_t)r->job.done * r->g->n_edges;
    out->init_ms = out->iter_ms = out->table_ms = 0.0;
    out->run_ms = (double)(r->t_end - r->t_admit) / 1e6;
    out->union_kernel = r->groups ? HB_UNION_GROUPS : (r->runs ? HB_UNION_RUNS : HB_UNION_EDGES);
    out->table_levels = r->levels;
    out->lanes_per_node = r->groups ? 64u : hbk::default_sched((int)r->p, r->bits, r->runs).lanes;
    out->nodes_per_block = r->groups ? hbk::group_nodes_per_block((int)r->p, r->bits)
                                     : hbk::default_sched((int)r->p, r->bits, r->runs)
                                           .nodes_per_block;
    out->register_bits = r->bits;
    out->tune_ms = 0.0;
    out->t_submit_ns = r->t_submit;
    out->t_admit_ns = r->t_admit;
    out->t_start_ns = r->t_start;
    out->t_end_ns = r->t_end;
    reqs_.erase(it);
    return HB_OK;
}

hb_status Server::stats(hb_server_stats_t *out) {
    if (!out) return fail(HB_EINVAL, "out is NULL");
    std::lock_guard<std::mutex> lk(mu_);
    out->running = lanes_[0].n_running + lanes_[1].n_running;
    out->queued = (uint32_t)(lanes_[0].queue.size() + lanes_[1].queue.size());
    out->submitted = submitted_;
    out->completed = completed_;
    out->steps = steps_;
    out->budget_bytes = cap_ ? cap_ : options().hbm_budget;
    out->used_bytes = used_;
    out->peak_used_bytes = peak_used_;
    out->edge_unions = edge_unions_;
    return HB_OK;
}

void Server::fail_all(Lane &L, hb_status st, const std::string &msg) {
    std::lock_guard<std::mutex> lk(mu_);
    auto mark = [&](Request *r) {
        r->state = State::Failed;
        r->error = st;
        r->message = msg;
        r->g->inflight.fetch_sub(1);
    };
    for (Request *r : L.running) {
        mark(r);
        pool_give(r->mem);
        r->mem = nullptr;
        used_ -= align256(r->footprint);
    }
    for (Request *r : L.queue) mark(r);
    L.running.clear();
    L.queue.clear();
    L.n_running = 0;
    cv_done_.notify_all();
}

// Copy a stopped request's outputs to host memory and free its block.
void Server::retire(Lane &L, Request *r) {
    const uint32_t n = r->g->n;
    r->reach.resize(n);
    r->sum_d.resize(n);
    (void)hipMemcpyAsync(r->reach.data(), r->job.c_prev, sizeof(double) * n, hipMemcpyDeviceToHost,
                         L.stream);
    (void)hipMemcpyAsync(r->sum_d.data(), r->job.sum_d, sizeof(double) * n, hipMemcpyDeviceToHost,
                         L.stream);
    if (r->flags & HB_SUBMIT_REGISTERS) {
        r->regs.resize(((uint64_t)n << r->p) * r->bits / 8u);
        (void)hipMemcpyAsync(r->regs.data(), r->job.buf[r->job.done & 1u], r->regs.size(),
                             hipMemcpyDeviceToHost, L.stream);
    }
}

hb_status Server::step(Lane &L) {
    // ---- admit
    std::vector<Request *> admitted;
    {
        std::lock_guard<std::mutex> lk(mu_);
        const uint32_t others = lanes_[0].n_running + lanes_[1].n_running - L.n_running;
        // the slow lane runs its large requests a few at a time (default one, in
        // arrival order), each at the device's full speed
        const uint64_t lane_cap =
            &L == &lanes_[1] ? (opts_.slow_lane_running ? opts_.slow_lane_running : 1u)
                             : UINT64_MAX;
        while (!L.queue.empty() && L.running.size() + admitted.size() < lane_cap &&
               (opts_.max_running == 0 ||
                others + L.running.size() + admitted.size() < opts_.max_running)) {
            Request *r = L.queue.front();
            const uint64_t fp = align256(r->footprint);
            if (cap_ && used_ + fp > cap_) break;  // arrival order within the lane
            void *mem = nullptr;
            if (pool_take(fp, &mem) != HB_OK) break;
            L.queue.pop_front();
            r->mem = mem;
            used_ += fp;
            r->state = State::Running;
            r->t_admit = now_ns();
            admitted.push_back(r);
        }
        peak_used_ = std::max(peak_used_, used_);
        L.n_running = (uint32_t)(L.running.size() + admitted.size());
    }
    const hb_options lib = options();
    for (Request *r : admitted) {
        uint8_t *base = static_cast<uint8_t *>(r->mem);
        hb_graph *g = r->g;
        const uint64_t m = (1ull << r->p) * r->bits / 8u;
        const uint64_t bb = align256((uint64_t)g->n * m * (r->levels + 1u));
        const uint64_t sb = align256(8ull * g->n);
        hbk::BatchJob &b = r->job;
        b = hbk::BatchJob{};
        b.bytes = g->d_bytes;
        b.offsets = g->d_offsets;
        b.run_list = g->d_runs;
        b.run_off = g->d_run_off;
        b.order = g->d_order;
        b.hash_ids = g->d_hash_ids;
        b.buf[0] = base;
        b.buf[1] = base + bb;
        b.c_prev = reinterpret_cast<double *>(base + 2 * bb);
        b.sum_d = reinterpret_cast<double *>(base + 2 * bb + sb);
        b.flags = reinterpret_cast<uint32_t *>(base + 2 * bb + 2 * sb);
        b.seed = r->seed;
        b.n = g->n;
        b.p = r->p;
        b.depth = r->depth;
        b.levels = r->levels;
        b.n_flags = (uint32_t)std::min<uint64_t>((uint64_t)g->n + 2, UINT32_MAX);
        b.runs = r->runs ? 1u : 0u;
        b.bits = r->bits;
        b.depth_only = lib.stop_rule == HB_STOP_DEPTH ? 1u : 0u;
        b.stop_delta = lib.stop_delta > 0.0 ? lib.stop_delta : 0.5;
        if (r->groups) {
            b.groups = 1u;
            b.grp_rows = g->d_grp_rows;
            b.grp_mask = g->d_grp_mask;
            b.grp_off = g->d_grp_off;
        }
        L.running.push_back(r);
    }
    const uint32_t nj = (uint32_t)L.running.size();
    if (nj == 0) return HB_OK;

    // ---- job table and launch lists for this step
    if (L.jobs_cap < nj) {
        dfree(L.d_jobs);
        if (L.h_jobs) (void)hipHostFree(L.h_jobs);
        L.d_jobs = nullptr;
        L.h_jobs = nullptr;
        L.jobs_cap = 0;
        const uint32_t cap = std::max<uint32_t>(64, nj * 2);
        HB_HIP(dmalloc((void **)&L.d_jobs, sizeof(hbk::BatchJob) * cap));
        HB_HIP(hipHostMalloc((void **)&L.h_jobs, sizeof(hbk::BatchJob) * cap, hipHostMallocDefault));
        L.jobs_cap = cap;
    }
    hbk::BatchJob *h_jobs_ = L.h_jobs;
    for (uint32_t j = 0; j < nj; ++j) h_jobs_[j] = L.running[j]->job;
    struct Cls {
        uint32_t p;
        bool runs, groups;
        uint32_t bits;
        std::vector<uint32_t> list, base;
        uint32_t list_off, base_off;
    };
    std::vector<Cls> classes, inits;
    std::vector<uint32_t> all(nj), runs_list, new_list;
    uint32_t max_levels = 0;
    auto add_to = [&](std::vector<Cls> &cs, uint32_t j, bool runs, bool groups) {
        Cls *c = nullptr;
        for (auto &x : cs)
            if (x.p == h_jobs_[j].p && x.runs == runs && x.groups == groups &&
                x.bits == h_jobs_[j].bits)
                c = &x;
        if (!c) {
            cs.push_back(Cls{h_jobs_[j].p, runs, groups, h_jobs_[j].bits, {}, {0u}, 0, 0});
            c = &cs.back();
        }
        // the default schedule: a served step's class mix changes from step to step
        const int p = (int)h_jobs_[j].p;
        const uint32_t blocks =
            groups ? hbk::group_blocks(p, h_jobs_[j].bits, h_jobs_[j].n)
                   : (h_jobs_[j].n +
                      hbk::shape_for(p, hbk::default_sched(p, h_jobs_[j].bits, runs))
                          .nodes_per_block - 1) /
                         hbk::shape_for(p, hbk::default_sched(p, h_jobs_[j].bits, runs))
                             .nodes_per_block;
        c->list.push_back(j);
        c->base.push_back(c->base.back() + blocks);
    };
    for (uint32_t j = 0; j < nj; ++j) {
        all[j] = j;
        const bool is_new = j >= nj - admitted.size();
        if (is_new) {
            new_list.push_back(j);
            add_to(inits, j, false, false);
        }
        if (h_jobs_[j].runs) {
            runs_list.push_back(j);
            max_levels = std::max(max_levels, h_jobs_[j].levels);
        }
        add_to(classes, j, h_jobs_[j].runs != 0, h_jobs_[j].groups != 0);
    }
    std::vector<uint32_t> lists(all);
    const uint32_t runs_off = (uint32_t)lists.size();
    lists.insert(lists.end(), runs_list.begin(), runs_list.end());
    std::vector<uint32_t> table_off(max_levels + 1, 0), table_blocks(max_levels + 1, 0);
    for (uint32_t k = 1; k <= max_levels; ++k) {
        table_off[k] = (uint32_t)lists.size();
        uint32_t acc = 0;
        lists.push_back(0);
        for (uint32_t j : runs_list) {
            if (k <= h_jobs_[j].levels)
                acc += hbk::batch_table_blocks(
                    h_jobs_[j].n, (1u << h_jobs_[j].p) * h_jobs_[j].bits / 8u, k);
            lists.push_back(acc);
        }
        table_blocks[k] = acc;
    }
    for (auto *cs : {&classes, &inits})
        for (auto &c : *cs) {
            c.list_off = (uint32_t)lists.size();
            lists.insert(lists.end(), c.list.begin(), c.list.end());
            c.base_off = (uint32_t)lists.size();
            lists.insert(lists.end(), c.base.begin(), c.base.end());
        }
    if (L.lists_cap < lists.size()) {
        dfree(L.d_lists);
        L.d_lists = nullptr;
        L.lists_cap = 0;
        const uint64_t cap = std::max<uint64_t>(4096, lists.size() * 2);
        HB_HIP(dmalloc((void **)&L.d_lists, sizeof(uint32_t) * cap));
        L.lists_cap = cap;
    }
    hbk::BatchJob *d_jobs_ = L.d_jobs;
    uint32_t *d_lists_ = L.d_lists;
    hipStream_t s = L.stream;
    HB_HIP(hipMemcpyAsync(d_jobs_, h_jobs_, sizeof(hbk::BatchJob) * nj, hipMemcpyHostToDevice, s));
    HB_HIP(hipMemcpyAsync(d_lists_, lists.data(), sizeof(uint32_t) * lists.size(),
                          hipMemcpyHostToDevice, s));

    // ---- init the newly admitted, then one step for everyone running
    const uint64_t t_launch = now_ns();
    for (uint32_t j : new_list) {
        HB_HIP(hbk::launch_fill_u32(h_jobs_[j].flags, 0u, h_jobs_[j].n_flags, s));
        L.running[j]->t_start = t_launch;
    }
    for (auto &c : inits)
        HB_HIP(hbk::launch_batch_init((int)c.p, hbk::default_sched((int)c.p, c.bits), d_jobs_,
                                      d_lists_ + c.list_off, d_lists_ + c.base_off,
                                      (uint32_t)c.list.size(), c.base.back(), s));
    for (uint32_t k = 1; k <= max_levels; ++k)
        HB_HIP(hbk::launch_batch_table(d_jobs_, d_lists_ + runs_off, d_lists_ + table_off[k],
                                       (uint32_t)runs_list.size(), table_blocks[k], k, s));
    for (auto &c : classes) {
        if (c.groups)
            HB_HIP(hbk::launch_batch_groups((int)c.p, c.bits, d_jobs_, d_lists_ + c.list_off,
                                            d_lists_ + c.base_off, (uint32_t)c.list.size(),
                                            c.base.back(), s));
        else
            HB_HIP(hbk::launch_batch_union((int)c.p, hbk::default_sched((int)c.p, c.bits, c.runs),
                                           c.runs, d_jobs_, d_lists_ + c.list_off,
                                           d_lists_ + c.base_off, (uint32_t)c.list.size(),
                                           c.base.back(), s));
    }
    HB_HIP(hbk::launch_batch_step_end(d_jobs_, d_lists_, nj, s));
    HB_HIP(hipMemcpyAsync(h_jobs_, d_jobs_, sizeof(hbk::BatchJob) * nj, hipMemcpyDeviceToHost, s));
    HB_HIP(hipStreamSynchronize(s));

    // ---- retire the requests that stopped
    std::vector<Request *> done, still;
    for (uint32_t j = 0; j < nj; ++j) {
        Request *r = L.running[j];
        r->job = h_jobs_[j];
        if (r->job.done) {
            retire(L, r);
            done.push_back(r);
        } else {
            still.push_back(r);
        }
    }
    if (!done.empty()) HB_HIP(hipStreamSynchronize(s));
    L.running.swap(still);
    {
        std::lock_guard<std::mutex> lk(mu_);
        ++steps_;
        const uint64_t t_end = now_ns();
        for (Request *r : done) {
            r->t_end = t_end;
            r->state = State::Done;
            pool_give(r->mem);
            r->mem = nullptr;
            used_ -= align256(r->footprint);
            r->g->inflight.fetch_sub(1);
            ++completed_;
            edge_unions_ += (uint64_t)r->job.done * r->g->n_edges;
        }
        L.n_running = (uint32_t)L.running.size();
    }
    if (!done.empty()) {
        cv_done_.notify_all();
        cv_work_.notify_all();  // freed memory may let the other lane admit
    }
    return HB_OK;
}

void Server::loop(Lane &L) {
    (void)hipSetDevice(device_);
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(mu_);
            cv_work_.wait(lk, [&] { return stopping_ || !L.queue.empty() || !L.running.empty(); });
            if (abort_ || (stopping_ && L.queue.empty() && L.running.empty())) break;
            if (L.running.empty() && !L.queue.empty()) {
                // nothing of ours runs: wait until the head request fits
                const uint64_t fp = align256(L.queue.front()->footprint);
                void *mem = nullptr;
                if ((cap_ && used_ + fp > cap_) || pool_take(fp, &mem) != HB_OK) {
                    cv_work_.wait_for(lk, std::chrono::milliseconds(1));
                    continue;
                }
                pool_give(mem);
            }
        }
        const hb_status st = step(L);
        if (st != HB_OK) {
            fail_all(L, st, g_err);
            break;
        }
    }
    (void)hipStreamSynchronize(L.stream);
    dfree(L.d_lists);
    dfree(L.d_jobs);
    if (L.h_jobs) (void)hipHostFree(L.h_jobs);
    (void)hipStreamDestroy(L.stream);
    L.d_lists = nullptr;
    L.d_jobs = nullptr;
    L.h_jobs = nullptr;
    L.stream = nullptr;
    L.jobs_cap = 0;
    L.lists_cap = 0;
}

Server g_server;

// ---- device graph cache (hb_submit_cached)
// Graphs named by a caller's key stay loaded between requests.  A graph is idle
// while its inflight count is zero; the evictor, called when a device
// allocation does not fit, releases idle graphs least recently used first.  The
// lock is recursive because loading a graph may call the evictor on the same
// thread; the evictor only try-locks it, so a thread blocked elsewhere never
// waits for it.
struct CacheEntry {
    hb_graph *g;
    uint64_t last_use;
};

class GraphCache {
public:
    hb_status submit(uint64_t key, const hb_csr *csr, uint32_t p, uint32_t depth, uint64_t seed,
                     uint32_t flags, hb_ticket *out) {
        if (!out) return fail(HB_EINVAL, "NULL argument");
        hb_graph *g = nullptr;
        {
            std::lock_guard<std::recursive_mutex> lk(mu_);
            install_evictor();
            auto it = map_.find(key);
            if (it != map_.end()) {
                ++hits_;
            } else {
                if (!csr) return fail(HB_ENOTFOUND, "graph %llu is not cached and no CSR was given",
                                      (unsigned long long)key);
                hb_graph *ng = nullptr;
                const hb_status st = hb_graph_load(csr, &ng);
                if (st != HB_OK) return st;
                it = map_.emplace(key, CacheEntry{ng, 0}).first;
                ++misses_;
            }
            it->second.last_use = ++clock_;
            g = it->second.g;
            g->inflight.fetch_add(1);  // pinned until the request holds it
        }
        const hb_status st = g_server.submit(g, p, depth, seed, flags, out);
        g->inflight.fetch_sub(1);
        return st;
    }

    // Release idle graphs of device dev, oldest first, until `need` bytes are free.
    uint64_t evict(int dev, uint64_t need) {
        std::unique_lock<std::recursive_mutex> lk(mu_, std::try_to_lock);
        if (!lk.owns_lock()) return 0;
        std::vector<std::pair<uint64_t, uint64_t>> idle;  // (last use, key)
        for (const auto &kv : map_)
            if (kv.second.g->device == dev && kv.second.g->inflight.load() == 0)
                idle.emplace_back(kv.second.last_use, kv.first);
        std::sort(idle.begin(), idle.end());
        uint64_t freed = 0;
        for (const auto &e : idle) {
            if (freed >= need) break;
            hb_graph *g = map_[e.second].g;
            freed += g->dev_bytes;
            map_.erase(e.second);
            graph_release(g);
            ++evictions_;
        }
        return freed;
    }

    hb_status clear() {
        std::lock_guard<std::recursive_mutex> lk(mu_);
        uint32_t busy = 0;
        for (auto it = map_.begin(); it != map_.end();) {
            if (it->second.g->inflight.load() != 0) {
                ++busy;
                ++it;
                continue;
            }
            graph_release(it->second.g);
            it = map_.erase(it);
        }
        if (busy) return fail(HB_EBUSY, "%u cached graphs have requests and stay", busy);
        return HB_OK;
    }

    hb_status drop(uint64_t key) {
        std::lock_guard<std::recursive_mutex> lk(mu_);
        auto it = map_.find(key);
        if (it == map_.end()) return fail(HB_ENOTFOUND, "graph %llu is not cached",
                                          (unsigned long long)key);
        if (it->second.g->inflight.load() != 0)
            return fail(HB_EBUSY, "graph %llu has requests", (unsigned long long)key);
        graph_release(it->second.g);
        map_.erase(it);
        return HB_OK;
    }

    void stats(hb_graph_cache_stats_t *out) {
        std::lock_guard<std::recursive_mutex> lk(mu_);
        *out = hb_graph_cache_stats_t{};
        for (const auto &kv : map_) {
            ++out->graphs;
            out->busy += kv.second.g->inflight.load() != 0 ? 1u : 0u;
            out->bytes += kv.second.g->dev_bytes;
        }
        out->hits = hits_;
        out->misses = misses_;
        out->evictions = evictions_;
    }

private:
    void install_evictor() {
        if (evictor_set_) return;
        set_evictor([this](int dev, uint64_t need) { return evict(dev, need); });
        evictor_set_ = true;
    }

    std::recursive_mutex mu_;
    std::unordered_map<uint64_t, CacheEntry> map_;
    uint64_t clock_ = 0, hits_ = 0, misses_ = 0, evictions_ = 0;
    bool evictor_set_ = false;
};

GraphCache g_cache;

}  // namespace

extern "C" {

hb_status hb_server_start(const hb_server_opts *opts) { return g_server.start(opts); }

hb_status hb_server_stop(void) { return g_server.stop(); }

hb_status hb_submit(hb_graph *g, uint32_t p, uint32_t depth_limit, uint64_t hash_seed,
                    uint32_t flags, hb_ticket *out) {
    return g_server.submit(g, p, depth_limit, hash_seed, flags, out);
}

hb_status hb_poll(hb_ticket t, hb_result *out) { return g_server.poll(t, out, false); }

hb_status hb_wait(hb_ticket t, hb_result *out) { return g_server.poll(t, out, true); }

hb_status hb_server_stats(hb_server_stats_t *out) { return g_server.stats(out); }

hb_status hb_submit_cached(uint64_t graph_key, const hb_csr *csr, uint32_t p,
                           uint32_t depth_limit, uint64_t hash_seed, uint32_t flags,
                           hb_ticket *out) {
    return g_cache.submit(graph_key, csr, p, depth_limit, hash_seed, flags, out);
}

hb_status hb_graph_cache_stats(hb_graph_cache_stats_t *out) {
    if (!out) return fail(HB_EINVAL, "out is NULL");
    g_cache.stats(out);
    return HB_OK;
}

hb_status hb_graph_cache_clear(void) { return g_cache.clear(); }

hb_status hb_graph_cache_drop(uint64_t graph_key) { return g_cache.drop(graph_key); }

}  // extern "C"
