/*
 * hb.h -- HyperBall over a LEB128 delta-compressed CSR on one AMD Instinct GPU
 * (gfx950).  Plain C ABI: host pointers and sizes in, host arrays out; no
 * exceptions or aborts cross it.  Every call returns an hb_status; negative
 * values leave a message for hb_last_error().
 *
 * The method is HyperBall (Boldi & Vigna) as the paper "City-Scale Visibility
 * Graph Analysis via GPU-Accelerated HyperBall" applies it to visibility
 * graphs: one HyperLogLog counter of 2^p registers per node, the register-wise
 * max-union of each node's counter with its neighbours' counters per step
 * (Eq. 2), the HLL estimate of every counter after each step, and the
 * distance sum accumulated from the growth of the estimates (Eq. 3), stopped
 * by a depth limit or when no estimate grows by more than 0.5 (Alg. 1).
 *
 * Register format: one uint8 register per byte (values 0..65-p), node-major
 * rows of 2^p bytes.  Hash: SplitMix64 of (node id XOR hash_seed); register
 * index = top p bits; value = leading zeros of the remaining bits + 1.
 * Estimator: HLL raw estimate with the alpha_m constants of Flajolet et al.
 * (2007), linear counting when the raw estimate is <= 2.5 m and a register is
 * zero, computed in FP64 from an exactly summed harmonic mean.
 *
 * Threading: calls are serialised by the library; results of one call are
 * complete when it returns.
 */
#ifndef HB_H
#define HB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t hb_status;
#define HB_OK 0
#define HB_PENDING 1     /* not an error: the request is still running */
#define HB_EINVAL (-1)   /* bad argument (p outside [4,16], n = 0, NULL) */
#define HB_ECORRUPT (-2) /* the compressed CSR failed validation */
#define HB_ENOMEM (-3)   /* host or device allocation failed */
#define HB_EDEVICE (-4)  /* a HIP runtime call failed, or no GPU */
#define HB_ENOTFOUND (-5)
#define HB_EBUSY (-6)

#define HB_P_MIN 4
#define HB_P_MAX 16

/* Opaque device-resident graph. */
typedef struct hb_graph hb_graph;

/*
 * Compressed CSR (Sec. 3.2 of the paper): for node v the bytes
 * bytes[offsets[v] .. offsets[v+1]) hold degrees[v] unsigned LEB128 varints
 * (7-bit groups, least significant first, high bit = more bytes follow): the
 * first is the smallest neighbour id, each later one the positive difference
 * from the previous id, so the row lists the neighbours in increasing order.
 * All pointers are host memory, owned by the caller, read only during the
 * call.
 *
 * Two optional arrays serve the paper's locality reordering (Sec. 3.2,
 * "Optional Hilbert reordering"):
 *  - order: the order in which the union kernels process the nodes.  Nodes
 *    processed together should share neighbours (e.g. the cells sorted along
 *    a Hilbert curve), which raises cache reuse.  It changes no result.
 *    hb_graph_load returns HB_EINVAL if it is not a permutation of 0..n-1.
 *  - hash_ids: the element inserted into node v's own counter.  A graph whose
 *    nodes were renumbered (its CSR rebuilt in the new numbering) gives the
 *    same counters as the original, up to the renumbering, when hash_ids[v]
 *    is node v's original id.
 */
typedef struct {
    uint32_t n;                /* nodes, >= 1 */
    uint64_t n_edges;          /* directed edges = sum of degrees */
    const uint64_t *offsets;   /* n + 1 byte offsets, offsets[0] = 0 */
    const uint32_t *degrees;   /* n neighbour counts */
    const uint8_t *bytes;      /* offsets[n] bytes (may be NULL if offsets[n] = 0) */
    const uint32_t *comp_size; /* n exact component sizes N_v, or NULL = all n */
    const uint32_t *order;     /* n: processing order, a permutation of 0..n-1, or NULL */
    const uint32_t *hash_ids;  /* n: element inserted for node v (Alg. 1), or NULL = v */
    const int32_t *xy;         /* 2n: cell (x, y) of node v at xy[2v], xy[2v+1], or NULL
                                  (needed only by the point second moment) */
} hb_csr;

/*
 * Results of one run.  Array pointers are caller-owned host buffers of n
 * doubles (n * 2^p bytes for registers, n * 2^(p-1) with 4-bit registers),
 * or NULL to skip that output.
 * reach[v] is the final estimate of |B(v, T)|, sum_d[v] the Eq. 3 sum and
 * mean_depth[v] = sum_d[v] / (N_v - 1) (NaN when N_v < 2), as Sec. 3.3
 * defines Visual Mean Depth with the exact component size.
 */
typedef struct {
    double *reach;
    double *sum_d;
    double *mean_depth;
    uint8_t *registers;
    uint32_t passes;       /* union steps run (T) */
    uint32_t converged;    /* 1 if step T changed no estimate by more than 0.5 */
    uint32_t productive_iters; /* steps that changed some estimate by more than 0.5:
                                  passes - 1 when converged (the last step only
                                  detected the fixpoint), else passes */
    double c0;             /* estimate of a one-element counter */
    uint64_t edge_unions;  /* passes * n_edges */
    double init_ms;        /* device time of the initialisation kernel */
    double iter_ms;        /* device time summed over the passes union kernels */
    double table_ms;       /* device time summed over range-max table builds (run and
                              grouped kernels) */
    double run_ms;         /* device time from init start to the last union end */
    uint32_t union_kernel; /* kernel that ran: HB_UNION_EDGES, HB_UNION_RUNS or HB_UNION_GROUPS */
    uint32_t table_levels; /* table levels K used by the run or grouped kernel (0 otherwise) */
    uint32_t lanes_per_node;  /* union schedule that ran (see hb_run_opts); for a batch,
                                 that of the job's (p, kernel) class; for the grouped
                                 kernel 64 (a wavefront on each counter slice) */
    uint32_t nodes_per_block; /* for the grouped kernel: nodes per workgroup (16 per group) */
    uint32_t register_bits;   /* register width of the run: 8 or 4 */
    double tune_ms;        /* host time spent measuring schedules in this call (0 if none) */
    uint64_t t_submit_ns;  /* host CLOCK_MONOTONIC: hb_submit accepted it (else = t_start_ns) */
    uint64_t t_admit_ns;   /* device memory granted, joined the running steps (else = t_start_ns) */
    uint64_t t_start_ns;   /* call entry, or the first step of a served request */
    uint64_t t_end_ns;     /* results complete */
} hb_result;

/* Which union kernel a run uses. */
#define HB_UNION_AUTO 0  /* the grouped kernel where it is built (below) when the graph has
                            its group lists and at least 32,768 nodes, else the run kernel
                            when p <= 12, its table fits and the graph has its run list, else
                            per edge (in every form: blocking, batched, served) */
#define HB_UNION_EDGES 1 /* gather every neighbour's counter (Eq. 2 as written), decoding the
                            LEB128 row in the kernel */
#define HB_UNION_RUNS 2  /* cover runs of consecutive neighbour ids from a range-max table,
                            reading the run list decoded at load */
#define HB_UNION_GROUPS 3 /* the run kernel's table rows, merged at load over groups of 16
                             consecutive nodes of the processing order: each distinct row is
                             loaded once per group (counters of 256 to 4096 bytes: p = 8..12
                             with 8-bit registers, p = 9..12 with 4-bit) */

/*
 * Run options; an all-zero struct (or NULL) selects the defaults.
 * table_levels: the run kernel builds, every step, table levels 1..K with
 * T[k][i] = max of the counters i .. i + 2^k - 1 (K = table_levels, default 8,
 * capped at floor(log2 n)), costing K * n * 2^p extra bytes per counter
 * buffer.  A run of r <= 2^K consecutive neighbour ids then costs at most two
 * counter-row loads instead of r.  The registers are identical either way.
 */
typedef struct {
    uint32_t union_kernel;    /* HB_UNION_* */
    uint32_t table_levels;    /* 0 = default */
    uint32_t tune;            /* HB_TUNE_*: how the union schedule is chosen */
    uint32_t lanes_per_node;  /* 0 = by `tune`; else this schedule (HB_EINVAL if not built) */
    uint32_t nodes_per_block; /* with lanes_per_node: 1, 2 or 4 (0 = 4; must be 1 above 64 lanes) */
    uint32_t register_bits;   /* 8 (0 = default) or 4: the paper's packed format, below */
} hb_run_opts;

/*
 * Register width.  With register_bits = 8 every HLL register is a byte.  With
 * 4 (Sec. 3.4: two registers per byte) register j of a counter is the low
 * nibble of byte j/2 for even j and the high nibble for odd j, and a register
 * saturates at 15: a rank above 15 is stored as 15.  Since the register-wise
 * max commutes with that clamp, the 4-bit registers after any step are
 * exactly min(8-bit registers, 15); the estimator is the same formula over
 * them.  Counters take 2^(p-1) bytes instead of 2^p; p >= 5.  Registers
 * returned in hb_result are in the width of the run.
 */

/*
 * Union schedules.  A schedule is (lanes_per_node, nodes_per_block):
 *  - lanes_per_node: lanes that share one node's counter of 2^p bytes, 16
 *    bytes per lane slot, one to four slots per lane.  Up to 64 lanes the
 *    node sits in one wavefront, whose 64 / lanes lane groups gather
 *    different neighbours at once; above 64, lanes / 64 wavefronts of one
 *    workgroup each own a slice of the counter and read the row themselves.
 *  - nodes_per_block: nodes per workgroup (1, 2 or 4) for one-wave shapes.
 * Built lanes per p (the per-edge kernel's default first): p 4-7: 2^p / 16;
 * p 8: 16, 8; p 9: 32, 16; p 10: 64, 32, 16; p 11: 64, 128, 32; p 12: 64,
 * 128, 256; p 13: 128, 256; p 14: 256, 512; p 15: 512; p 16: 1024.  The run
 * kernel's default differs at p 9, 10 (16 lanes) and p 11 (32).  With 4-bit
 * registers one shape per p: p 5-11: 2^p / 32; p 12, 13: 64; p 14-16:
 * 2^p / 128.  Every schedule gives identical registers and estimates; only
 * the speed differs.
 *
 * The autotuner times one union step of every schedule built for p on the
 * caller's own data (two launches each, the faster counts), keeps the
 * fastest in a process-wide cache keyed by the shape class (p, kernel,
 * single or batched, floor(log2 nodes), floor(log2 gathered rows per node)),
 * then re-initialises and runs.  Tuning changes no result.
 */
#define HB_TUNE_CACHED 0  /* the cached pick for the shape class, else the default schedule */
#define HB_TUNE_MEASURE 1 /* as HB_TUNE_CACHED, but measure first when nothing is cached */
#define HB_TUNE_OFF 2     /* the default schedule */

/* One autotuner cache entry. */
typedef struct {
    uint32_t p, register_bits, union_kernel, batched; /* shape class ... */
    uint32_t log2_nodes, log2_rows_per_node;
    uint32_t lanes_per_node, nodes_per_block; /* ... and its pick */
    double best_ms;                       /* measured union step of the pick */
    double default_ms;                    /* and of the default schedule */
} hb_tune_entry;

/*
 * Library-wide options (hb_set_options); an all-zero struct selects the
 * defaults.  Every call takes a copy of them when it starts (a served request
 * when it is admitted), so changing them affects later calls only.
 *
 * Device memory.  Every device allocation of the library -- the arrays of
 * loaded graphs, the counters, range-max tables and per-node state of
 * blocking runs, the batched workspace and the memory of served requests --
 * counts against one budget per device, hbm_budget bytes (0 = no limit but
 * the device's free memory).  Working buffers are carved first-fit from
 * pooled blocks of at least 1 GiB (or what the budget leaves), kept between
 * calls so that a run, a batch or an admitted request takes memory without a
 * device allocation and returns it without hipFree's implicit device
 * synchronisation; idle blocks are released by hb_release_cache or when an
 * allocation would otherwise not fit.  A blocking call whose memory does not
 * fit returns HB_ENOMEM; a served request waits until running requests free
 * memory (hb_submit returns HB_ENOMEM only if it could never fit).
 *
 * dev_alloc / dev_free: allocator hooks for all of that memory (both or
 * neither), e.g. a framework's caching allocator.  dev_alloc returns device
 * memory of the current device aligned to 256 bytes, or NULL when it cannot;
 * memory is always released through the hooks it was allocated with.  The
 * hooks may be called from the request loop's threads.
 *
 * stream: a hipStream_t (passed as void *) on which the blocking runs
 * (hb_run, hb_run_with, hb_run_static) enqueue their work after the work the
 * caller queued there; NULL = the graph's own stream.  They still return once
 * their results are on the host.
 *
 * Stopping (Alg. 1 stops after step t when no estimate grew by more than 0.5,
 * or at the depth limit): stop_delta replaces the 0.5 (0 = 0.5);
 * stop_rule HB_STOP_DEPTH ignores the growth test and runs exactly depth_limit
 * steps (runs without a depth limit then return HB_EINVAL).  Every form
 * follows them.  `converged` still reports whether the last step grew no
 * estimate by more than the threshold.
 *
 * tune_seed: tune_seed_count autotuner picks (as hb_tune_cache returns them,
 * e.g. saved by an earlier process) put into the pick cache by this call;
 * they are not kept in the options.
 */
#define HB_STOP_CONVERGED 0 /* Alg. 1: the growth test or the depth limit, whichever first */
#define HB_STOP_DEPTH 1     /* the depth limit only */

typedef struct {
    uint64_t hbm_budget;
    void *(*dev_alloc)(uint64_t bytes, void *user);
    void (*dev_free)(void *ptr, void *user);
    void *alloc_user;
    void *stream;
    uint32_t stop_rule;
    double stop_delta;
    const hb_tune_entry *tune_seed;
    uint32_t tune_seed_count;
} hb_options;

/* Replace the options (NULL = defaults).  HB_EINVAL for a hook without its
   partner, an unknown stop rule, a negative stop_delta or a seed entry naming
   no built schedule.  Host-only. */
hb_status hb_set_options(const hb_options *o);

/* The current options (tune_seed is always NULL). */
hb_status hb_get_options(hb_options *out);

/* Device memory held by the library on one device. */
typedef struct {
    uint64_t budget_bytes;         /* hb_options.hbm_budget (0 = none) */
    uint64_t held_bytes;           /* allocated: graphs, pool blocks, small tables */
    uint64_t peak_held_bytes;
    uint64_t pool_bytes;           /* pooled blocks */
    uint64_t pool_used_bytes;      /* taken from them by runs, batches and requests */
    uint64_t pool_peak_used_bytes;
} hb_memory_stats_t;

hb_status hb_memory_stats(int32_t device, hb_memory_stats_t *out);

/* Library version string. */
const char *hb_version(void);

/* Message of the last failed call on this thread ("" if none). */
const char *hb_last_error(void);

/*
 * Number of visible GPUs (0 if none).  Host-only callers may skip it; every
 * device call returns HB_EDEVICE when no GPU is present.
 */
hb_status hb_device_count(int32_t *count);

/*
 * Encode a sorted adjacency list into the compressed CSR of Sec. 3.2.
 * adj_offsets: n+1 entries indexing adj_ids; each row strictly increasing,
 * ids < n, no self loops (HB_EINVAL otherwise).  Two-phase: call with
 * bytes == NULL to get *bytes_len (and fill offsets/degrees), then again with
 * a buffer of at least *bytes_len bytes in bytes_cap.  Host-only.
 */
hb_status hb_csr_encode(uint32_t n, const uint64_t *adj_offsets, const uint32_t *adj_ids,
                        uint64_t *offsets, uint32_t *degrees, uint8_t *bytes, uint64_t bytes_cap,
                        uint64_t *bytes_len);

/*
 * Check a compressed CSR without touching the GPU.  HB_ECORRUPT when: offsets
 * are not monotone or offsets[0] != 0; a row ends inside a varint; a varint
 * is longer than 5 bytes or exceeds 32 bits; a decoded id is >= n, repeats,
 * decreases or equals the row's own node; a row's varint count differs from
 * degrees[v]; or the degree sum differs from n_edges.  *bad_node (optional)
 * receives the first failing node (or n for a global mismatch).  Host-only.
 */
hb_status hb_csr_validate(const hb_csr *csr, uint32_t *bad_node);

/*
 * Validate csr (as hb_csr_validate) and copy it into device memory.  The
 * caller may free its arrays when this returns.  *out is library-owned until
 * hb_graph_free.  The rows are also decoded once, on the device, into the run
 * list the run kernel reads: 8 bytes per run (hb_graph_stats_t.n_runs) plus
 * 8 (n + 1) bytes of offsets.  When that list does not fit in device memory
 * the graph loads without it, and only the per-edge kernel serves it (an
 * explicit HB_UNION_RUNS request then fails with HB_ENOMEM).  HB_EDEVICE if the
 * device's run count disagrees with the host validator's.
 */
hb_status hb_graph_load(const hb_csr *csr, hb_graph **out);

/* Release a graph and its device memory. */
hb_status hb_graph_free(hb_graph *g);

/* Nodes, directed edges and compressed bytes of a loaded graph. */
hb_status hb_graph_info(const hb_graph *g, uint32_t *n, uint64_t *n_edges, uint64_t *n_bytes);

/*
 * Shape of a loaded graph, counted during hb_graph_load: runs are maximal
 * sequences of consecutive neighbour ids in a row (joined across the row's own
 * node); table_rows[K] is the number of counter rows one step of the run
 * kernel loads with a table of depth K (1 per run whose length is a power of
 * two <= 2^K, 2 per other run <= 2^K, ceil(length / 2^K) per longer run).
 */
typedef struct {
    uint32_t n;
    uint64_t n_edges;
    uint64_t n_bytes;
    uint64_t n_runs;
    uint64_t table_rows[25];
    uint64_t local_run_reads;  /* sum over rows w of deg(w) x the maximal runs of w
                                  (v not joined in): the neighbour runs that
                                  hb_local_metrics reads, 8 bytes each */
    uint64_t group_rows;       /* rows one step of the grouped kernel loads (0 when the
                                  graph has no group lists) */
    uint32_t group_levels;     /* table depth the group lists were built for */
} hb_graph_stats_t;

hb_status hb_graph_stats(const hb_graph *g, hb_graph_stats_t *out);

/*
 * Run HyperBall (Alg. 1) on a loaded graph: insert every node v into its own
 * counter, then for t = 1, 2, ...: union (Eq. 2), estimate, accumulate (Eq. 3),
 * stop after step t when no estimate grew by more than 0.5 or t ==
 * depth_limit (0 = no limit).  Blocking.  p in [4, 16].  Device memory for
 * two counter buffers (2 n 2^p bytes) and 16 n bytes of FP64 state is held by
 * the graph between runs and released by hb_graph_free.  The registers of a
 * run with depth_limit t equal the step-t registers of any longer run.
 */
hb_status hb_run(hb_graph *g, uint32_t p, uint32_t depth_limit, uint64_t hash_seed,
                 hb_result *out);

/*
 * hb_run with explicit options (opts may be NULL).  HB_EINVAL if the run
 * kernel is requested for p > 12 or table_levels > 24.
 */
hb_status hb_run_with(hb_graph *g, uint32_t p, uint32_t depth_limit, uint64_t hash_seed,
                      const hb_run_opts *opts, hb_result *out);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): hb_run_with
 * with its two counter buffers (and the run kernel's table levels) in a static
 * device workspace of HB_STATIC_SCRATCH_BYTES, one copy per device, held until
 * the process ends, instead of the run workspace grown on demand.  It calls no
 * hipMalloc, hipFree or other allocating routine and allocates no host memory;
 * the graph's per-node state (allocated by hb_graph_load) and the caller's
 * output arrays are used as by hb_run_with.  HB_UNION_AUTO takes the run kernel
 * when both buffers with their tables fit the workspace, else the per-edge
 * kernel; HB_ENOMEM (with the sizes in hb_last_error) when even the per-edge
 * kernel's 2 n 2^p bytes (n 2^(p-1) per buffer with 4-bit registers) do not
 * fit.  HB_TUNE_MEASURE acts as HB_TUNE_CACHED.  Every call on one device
 * shares that device's workspace, which keeps the last call's counters; the
 * library's device lock serialises blocking calls within a process, so calls
 * made outside it (another copy of the library in the same process) would race.
 */
#define HB_STATIC_SCRATCH_BYTES (64ull << 20)
hb_status hb_run_static(hb_graph *g, uint32_t p, uint32_t depth_limit, uint64_t hash_seed,
                        const hb_run_opts *opts, hb_result *out);

/* One analysis of a batched run. */
typedef struct {
    hb_graph *g;           /* a loaded graph; several jobs may share one */
    uint32_t p;            /* [4, 16] */
    uint32_t depth_limit;  /* 0 = until convergence */
    uint64_t hash_seed;
} hb_job;

/*
 * Run n_jobs analyses together (blocking).  All jobs advance one HyperBall
 * step per batched step: one launch per (p, union kernel) class covers the
 * nodes of every running job of that class (the union kernel of each job
 * chosen by opts->union_kernel as for hb_run_with: HB_UNION_AUTO takes the
 * grouped kernel for graphs of at least 32,768 nodes where it is built), one
 * launch per table level builds the range-max tables of all run-kernel and
 * grouped jobs, and a step-end kernel applies
 * each job's own stop rule on the device, so jobs of different sizes, p and
 * depth limits finish independently.  Each step is a captured HIP graph,
 * replayed a few steps at a time between host checks.  outs[j] is filled as
 * hb_run would fill it for job j alone, with identical registers and sums;
 * run_ms is the device time of the whole batch and iter_ms / table_ms are 0.
 * Device memory for all jobs' counters and state comes from a workspace the
 * library keeps between batched calls and grows on demand (HB_ENOMEM if it
 * does not fit); hb_release_cache returns it.  All graphs must live on one
 * device.
 */
hb_status hb_run_batch(const hb_job *jobs, uint32_t n_jobs, const hb_run_opts *opts,
                       hb_result *outs);

/*
 * Serving: a request loop on a library thread.  hb_submit queues an analysis
 * and returns at once; the loop admits queued requests in arrival order while
 * their device footprint -- 2 (K+1) n 2^p bytes of counters and tables
 * (K = 0 for the per-edge kernel), 16 n bytes of FP64 state and 4 (n+2) bytes
 * of stop flags -- fits the memory budget, and advances every admitted
 * request by one HyperBall step per batched step (continuous batching: a
 * request that arrives while others run joins at the next step, and finished
 * requests free their memory at once).  Requests whose steps gather more than
 * slow_lane_bytes run on a second lane with its own thread and stream, so
 * short requests do not wait for the steps of very large ones; that lane runs
 * slow_lane_running requests at a time (default 1: the large requests in
 * arrival order, each at the device's full speed).  Memory comes from the
 * library's pool under the budget of hb_set_options, shared with blocking runs
 * and graphs.  Results match hb_run for the same arguments bit for bit.
 * Graphs passed to hb_submit stay owned by the caller; hb_graph_free returns
 * HB_EBUSY while a submitted request still uses the graph.  hb_submit_cached
 * names graphs by a key instead and keeps them in the library's device graph
 * cache (below).
 */
typedef uint64_t hb_ticket;

typedef struct {
    uint64_t hbm_budget;      /* cap on the device bytes of running requests, within the
                                 library-wide budget; 0 = no cap of its own */
    uint32_t max_running;     /* cap on admitted requests; 0 = none */
    uint32_t union_kernel;    /* HB_UNION_* for every request */
    uint32_t table_levels;    /* 0 = default */
    uint64_t slow_lane_bytes; /* requests gathering more bytes per step run on a second lane
                                 (own thread and stream, shared memory); 0 = 2 GiB,
                                 UINT64_MAX = one lane */
    uint32_t slow_lane_running; /* requests the second lane runs at a time; 0 = 1,
                                   UINT32_MAX = no cap */
} hb_server_opts;

typedef struct {
    uint32_t running, queued;
    uint64_t submitted, completed, steps;
    uint64_t budget_bytes, used_bytes, peak_used_bytes;
    uint64_t edge_unions;  /* summed over completed requests */
} hb_server_stats_t;

#define HB_SUBMIT_REGISTERS 1u /* keep the final registers for hb_poll */
#define HB_SUBMIT_REG4 2u      /* 4-bit registers (see hb_run_opts.register_bits); p >= 5 */

/* Start the request loop (HB_EBUSY if it runs).  opts may be NULL. */
hb_status hb_server_start(const hb_server_opts *opts);

/*
 * Stop accepting requests, finish every queued and running one, release the
 * budget and end the loop.  Finished results stay available to hb_poll.
 */
hb_status hb_server_stop(void);

/*
 * Queue one analysis (starts the loop with default options if needed).
 * HB_ENOMEM if its footprint exceeds the whole budget (it could never run);
 * HB_EINVAL for bad arguments (as hb_run_with).
 */
hb_status hb_submit(hb_graph *g, uint32_t p, uint32_t depth_limit, uint64_t hash_seed,
                    uint32_t flags, hb_ticket *out);

/*
 * HB_PENDING while the request is queued or running.  When it has finished,
 * fill out (its non-NULL arrays are written as by hb_run; registers only if
 * submitted with HB_SUBMIT_REGISTERS, else HB_EINVAL) and forget the ticket:
 * later calls return HB_ENOTFOUND.  A request that failed returns its error
 * status once.
 */
hb_status hb_poll(hb_ticket t, hb_result *out);

/*
 * Device graph cache of the served form: graphs named by a caller-chosen key
 * stay device-resident between requests.  hb_submit_cached queues an analysis
 * of graph `graph_key`: when the cache holds it, csr is not read (it may be
 * NULL); otherwise csr is validated and loaded as by hb_graph_load, inside this
 * call (its time counts in the request's latency), and kept under the key.
 * HB_ENOTFOUND when the key is not cached and csr is NULL.  A cached graph is
 * idle while no request of it is queued or running; when a device allocation
 * of the library does not fit the budget (or the device), idle cached graphs
 * are released least recently used first.  Other arguments and errors as
 * hb_submit.
 */
hb_status hb_submit_cached(uint64_t graph_key, const hb_csr *csr, uint32_t p,
                           uint32_t depth_limit, uint64_t hash_seed, uint32_t flags,
                           hb_ticket *out);

typedef struct {
    uint32_t graphs;     /* graphs in the cache */
    uint32_t busy;       /* of those, graphs with queued or running requests */
    uint64_t bytes;      /* their device bytes */
    uint64_t hits, misses, evictions;
} hb_graph_cache_stats_t;

hb_status hb_graph_cache_stats(hb_graph_cache_stats_t *out);

/* Release every idle cached graph (graphs with requests stay; HB_EBUSY then). */
hb_status hb_graph_cache_clear(void);

/* Release the cached graph `graph_key` (HB_ENOTFOUND if not cached, HB_EBUSY while
   it has requests). */
hb_status hb_graph_cache_drop(uint64_t graph_key);

/* hb_poll that blocks until the request has finished. */
hb_status hb_wait(hb_ticket t, hb_result *out);

/* Counters of the request loop. */
hb_status hb_server_stats(hb_server_stats_t *out);

/*
 * Free the device workspaces kept between calls: the counter buffers of
 * blocking runs (one pair per device, shared by all graphs and sized for the
 * largest run so far) and the batched runs' workspace.
 */
hb_status hb_release_cache(void);

/*
 * VGA metrics (Sec. 3.3, "Metric derivation"), n doubles each, caller-owned
 * host arrays or NULL to skip.  k = deg(v), N = N_v (the exact component size
 * given at load, else n), MD = sum_d[v] / (N - 1):
 *  - connectivity: k;
 *  - control: the sum over neighbours w of 1 / deg(w);
 *  - mean_depth: MD (NaN if N < 2);
 *  - relative_asymmetry: RA = 2 (MD - 1) / (N - 2) (NaN if N < 3);
 *  - integration_hh: 1 / RRA with RRA = RA / D_N and Hillier & Hanson's
 *    diamond value D_N = 2 (N (log2((N + 2) / 3) - 1) + 1) / ((N - 1)(N - 2))
 *    (+inf when RA = 0; the paper names RRA but not D_N);
 *  - integration_tekl: log2((MD + 2) / 3), as the paper states it;
 *  - integration_pvalue: max(0, 1 - RA);
 *  - point_first_moment: MD k;
 *  - point_second_moment: the sum over neighbours w of (x_w - x_v)^2 + (y_w - y_v)^2,
 *    the second moment of the visible cells about v (Turner et al. 2001's isovist
 *    moment; the paper names it among the exact local metrics without a formula), in
 *    squared cell units, summed exactly in integers; NaN when the graph was loaded
 *    without hb_csr.xy.
 * connectivity, control and point_second_moment are exact; the others inherit the
 * HLL error of sum_d.
 */
typedef struct {
    double *connectivity, *control, *mean_depth, *relative_asymmetry;
    double *integration_hh, *integration_tekl, *integration_pvalue, *point_first_moment;
    double *point_second_moment;
} hb_vga_out;

/* The metrics above for every node of g from the sums of one run (n doubles). */
hb_status hb_vga_metrics(hb_graph *g, const double *sum_d, hb_vga_out *out);

/*
 * Local VGA metrics (Sec. 3.3, "Metric derivation": exact, from the
 * neighbourhoods, independent of the HLL), per node v with k = deg(v); n
 * entries each, caller-owned host arrays or NULL to skip:
 *  - pairs: ordered pairs (a, b) of neighbours of v that are adjacent, i.e. the
 *    sum over neighbours a of |N(a) intersect N(v)| (each link among the
 *    neighbours counts twice);
 *  - ball2: |B(v, 2)| - 1, the nodes other than v within two steps;
 *  - clustering: pairs / (k (k - 1)), the Watts & Strogatz (1998) coefficient
 *    (NaN for k < 2);
 *  - controllability: k / ball2, the first-step neighbourhood over the
 *    two-step one (Turner et al. 2001; NaN for an isolated node).
 * The paper names these metrics without formulas; the definitions above are the
 * standard ones it cites.  Work is the sum over edges (v, w) of the number of
 * runs of consecutive ids in w's row.  Each workgroup keeps two bitmaps of n
 * bits in LDS, so n is limited by the device's LDS per workgroup (HB_EINVAL
 * beyond it: n <= 654,592 with 160 KiB).  Temporary device memory: the run list
 * of the graph (8 bytes per run) plus 12 n bytes; HB_ENOMEM when it does not
 * fit.  Blocking: it holds the library's device lock for its whole duration
 * (8.5 s for a 236k-node, 4.9e9-edge graph), so other blocking calls (runs,
 * loads) wait for it; the served request loop does not.
 */
typedef struct {
    uint64_t *pairs;
    uint32_t *ball2;
    double *clustering, *controllability;
} hb_local_out;

hb_status hb_local_metrics(hb_graph *g, hb_local_out *out);

/*
 * Copy up to cap autotuner cache entries to out (caller-owned; NULL with
 * cap 0 only counts) and the number of entries to *count.  Host-only.
 */
hb_status hb_tune_cache(hb_tune_entry *out, uint32_t cap, uint32_t *count);

/* Forget every cached schedule pick. */
hb_status hb_tune_clear(void);

/*
 * Diagnostic: a plain streaming copy of `bytes` (a multiple of 16) between two
 * fresh device buffers, repeated reps times after one warm-up; *avg_ms is the
 * device time of one copy.  It reads and writes `bytes` each, so 2 * bytes /
 * avg_ms is the achievable device-memory bandwidth, and the copy is the
 * reference kernel for scaling hardware byte counters.  Allocates and frees
 * its own buffers.
 */
hb_status hb_copy_probe(uint64_t bytes, uint32_t reps, double *avg_ms);

/*
 * Diagnostic: the ceiling of the run kernel's gathers.  n_nodes nodes, in the
 * run kernel's launch shape for p (lanes_per_node / nodes_per_block; 0 = the
 * run kernel's default), each gather rows_per_node counter rows of 2^p bytes
 * picked by a hash from a table of table_rows rows (a power of two; 2048 rows
 * at p = 10 is 2 MiB, which stays in every L2), and take their byte-wise max
 * (with_max = 1) or only load them (0).  One warm-up launch, then reps timed
 * ones; *avg_ms is the device time of one.  n_nodes * rows_per_node * 2^p /
 * avg_ms is the rate at which that kernel's loop can gather rows that hit in
 * L2.  Allocates and frees its own buffers.  p in [4, 12].
 */
hb_status hb_gather_probe(uint32_t p, uint32_t lanes_per_node, uint32_t nodes_per_block,
                          uint32_t table_rows, uint32_t n_nodes, uint32_t rows_per_node,
                          uint32_t with_max, uint32_t reps, double *avg_ms);

#ifdef __cplusplus
}
#endif

#endif /* HB_H */
