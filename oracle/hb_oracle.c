/*
 * CPU oracle for HyperBall over a LEB128 delta-compressed CSR.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * reference that the GPU path is checked against.  Only the test suite, the
 * smoke check and the benchmark's CPU-baseline leg may load it.  It shares no
 * code, header, table or constant generator with the GPU library.
 *
 * What each part follows (the paper is "City-Scale Visibility Graph Analysis
 * via GPU-Accelerated HyperBall"):
 *   - LEB128 delta CSR ............ Sec. 3.2 "Encoding" (first neighbour
 *                                   absolute, then deltas, unsigned LEB128;
 *                                   u64 byte offsets, u32 degrees)
 *   - SplitMix64 insert ........... Sec. 3.3 "Initialisation" (node inserted
 *                                   into its own counter with SplitMix64)
 *   - HLL estimator ............... Sec. 2.3 and Sec. 3.3 "Iteration"
 *                                   (alpha_m bias correction, small-range
 *                                   linear counting; Flajolet et al. 2007)
 *   - register-wise union ......... Eq. 2 (hll-union)
 *   - distance accumulation ....... Eq. 3 (sumD)
 *   - stopping rule ............... Sec. 3.3 "Convergence" and Alg. 1
 *   - exact BFS ................... textbook breadth-first search; Eq. 1 is
 *                                   the identity HyperBall approximates
 *
 * Readings taken where the paper is silent (listed with reasons in the design
 * notes): one uint8 register per byte, no clamp; hash = full SplitMix64
 * output of (v XOR seed); register index = top p bits, value = leading zeros
 * of the remaining 64-p bits plus one (capped at 65-p); harmonic sum formed
 * exactly as a 128-bit integer and rounded once; no empirical HLL++ bias
 * table; depth_limit 0 = unlimited; stop after step t when max delta <= 0.5
 * or t == depth_limit.
 *
 * Floating point: every double op is one IEEE op in the order written; build
 * with -ffp-contract=off.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------- */
/* LEB128 (Sec. 3.2 "Encoding")                                               */
/* ------------------------------------------------------------------------- */

/* Unsigned LEB128: 7-bit groups, least significant first, high bit set on
 * every byte but the last; shortest form.  Returns the byte count. */
int or_uleb_encode(uint64_t v, uint8_t *out) {
    int k = 0;
    do {
        uint8_t b = (uint8_t)(v & 0x7F);
        v >>= 7;
        if (v != 0) b |= 0x80;
        if (out) out[k] = b;
        k++;
    } while (v != 0);
    return k;
}

/* Decode one unsigned LEB128 value from [p, end).
 * Returns the number of bytes used, 0 if the input ends inside the value,
 * -1 if the value has more than 10 groups or overflows 64 bits. */
int or_uleb_decode(const uint8_t *p, const uint8_t *end, uint64_t *v) {
    uint64_t x = 0;
    int shift = 0, k = 0;
    for (;;) {
        if (p + k >= end) return 0;
        uint8_t b = p[k++];
        uint64_t grp = (uint64_t)(b & 0x7F);
        if (shift >= 64 || (shift > 0 && (grp >> (64 - shift)) != 0)) return -1;
        x |= grp << shift;
        shift += 7;
        if (!(b & 0x80)) break;
        if (k >= 10) return -1;
    }
    *v = x;
    return k;
}

/* Bytes needed for node v's row: uleb(a_0), then uleb(a_i - a_{i-1}). */
static uint64_t row_bytes(const uint64_t *adj_off, const uint32_t *adj_ids, int64_t v) {
    uint64_t nb = 0;
    uint32_t prev = 0;
    for (uint64_t k = adj_off[v]; k < adj_off[v + 1]; ++k) {
        uint32_t a = adj_ids[k];
        uint64_t val = (k == adj_off[v]) ? (uint64_t)a : (uint64_t)(a - prev);
        nb += (uint64_t)or_uleb_encode(val, NULL);
        prev = a;
    }
    return nb;
}

/* Byte offsets (n+1) and degrees (n) of the compressed CSR of a sorted
 * adjacency list.  Returns the total byte count (= offsets[n]). */
uint64_t or_csr_layout(int64_t n, const uint64_t *adj_off, const uint32_t *adj_ids,
                       uint64_t *offsets, uint32_t *degrees) {
    offsets[0] = 0;
    for (int64_t v = 0; v < n; ++v) {
        offsets[v + 1] = offsets[v] + row_bytes(adj_off, adj_ids, v);
        degrees[v] = (uint32_t)(adj_off[v + 1] - adj_off[v]);
    }
    return offsets[n];
}

/* Write the LEB128 rows at the offsets or_csr_layout produced. */
void or_csr_encode(int64_t n, const uint64_t *adj_off, const uint32_t *adj_ids,
                   const uint64_t *offsets, uint8_t *bytes) {
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t v = 0; v < n; ++v) {
        uint8_t *out = bytes + offsets[v];
        uint32_t prev = 0;
        for (uint64_t k = adj_off[v]; k < adj_off[v + 1]; ++k) {
            uint32_t a = adj_ids[k];
            uint64_t val = (k == adj_off[v]) ? (uint64_t)a : (uint64_t)(a - prev);
            out += or_uleb_encode(val, out);
            prev = a;
        }
    }
}

/* Decode node v's row into ids (room for cap entries).  Returns the number of
 * neighbours, or -1 on a malformed row (truncated or overlong varint, more
 * than cap entries, or a running id beyond 32 bits). */
int64_t or_decode_row(const uint8_t *bytes, const uint64_t *offsets, int64_t v, uint32_t *ids,
                      int64_t cap) {
    const uint8_t *p = bytes + offsets[v], *end = bytes + offsets[v + 1];
    int64_t k = 0;
    uint64_t cur = 0;
    while (p < end) {
        uint64_t val;
        int used = or_uleb_decode(p, end, &val);
        if (used <= 0) return -1;
        p += used;
        cur = (k == 0) ? val : cur + val;
        if (cur > 0xFFFFFFFFull || k >= cap) return -1;
        ids[k++] = (uint32_t)cur;
    }
    return k;
}

/* ------------------------------------------------------------------------- */
/* SplitMix64 and HLL insert (Sec. 3.3 "Initialisation")                      */
/* ------------------------------------------------------------------------- */

/* SplitMix64 output function (Steele, Lea & Flood 2014) applied to x:
 * add the golden-gamma increment, then the two xor-shift-multiply rounds
 * and a final xor-shift.  All arithmetic mod 2^64. */
uint64_t or_splitmix64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* Register index j (top p bits of the hash) and value r (leading zeros of
 * the remaining 64-p bits, plus one; 65-p when they are all zero). */
void or_hll_insert(uint64_t v, uint64_t seed, int p, uint32_t *j, uint32_t *r) {
    uint64_t h = or_splitmix64(v ^ seed);
    uint64_t rest = h << p;
    uint32_t lz = 0;
    if (rest == 0) {
        lz = (uint32_t)(64 - p);
    } else {
        while (!(rest & 0x8000000000000000ull)) {
            rest <<= 1;
            lz++;
        }
    }
    *j = (uint32_t)(h >> (64 - p));
    *r = lz + 1;
}

/* ------------------------------------------------------------------------- */
/* HLL estimator (Sec. 2.3; Flajolet et al. 2007)                             */
/* ------------------------------------------------------------------------- */

/* Bias-correction constant alpha_m of HyperLogLog. */
double or_hll_alpha(int p) {
    const double m = (double)(1u << p);
    if (p == 4) return 0.673;
    if (p == 5) return 0.697;
    if (p == 6) return 0.709;
    return 0.7213 / (1.0 + 1.079 / m);
}

/* Raw estimate E = alpha_m m^2 / sum_j 2^-M[j] with the sum formed exactly
 * (as an integer in units of 2^-(65-p)) and rounded once; zero count in *zeros. */
double or_hll_raw(const uint8_t *regs, int p, uint32_t *zeros) {
    const uint32_t m = 1u << p;
    const int top = 65 - p; /* the largest register value */
    unsigned __int128 s = 0;
    uint32_t V = 0;
    for (uint32_t j = 0; j < m; ++j) {
        s += (unsigned __int128)1 << (top - regs[j]);
        if (regs[j] == 0) V++;
    }
    const double Z = ldexp((double)s, -top);
    const double md = (double)m;
    if (zeros) *zeros = V;
    return ((or_hll_alpha(p) * md) * md) / Z;
}

/* Cardinality estimate: raw estimate, or linear counting m*ln(m/V) when the
 * raw estimate is at most 2.5m and some register is still zero. */
double or_hll_estimate(const uint8_t *regs, int p) {
    uint32_t V;
    const double E = or_hll_raw(regs, p, &V);
    const double md = (double)(1u << p);
    if (E <= 2.5 * md && V > 0) return md * log(md / (double)V);
    return E;
}

/* ------------------------------------------------------------------------- */
/* HyperBall (Alg. 1)                                                         */
/* ------------------------------------------------------------------------- */

typedef struct {
    uint32_t passes;    /* union steps run */
    uint32_t converged; /* 1 if the last step's max delta was <= 0.5 */
    double max_delta;   /* max_v delta of the last step */
} or_hb_info;

/*
 * Alg. 1 on the compressed CSR.  regs_out (n * 2^p, optional) receives the
 * registers after the last step, reach_out (n) the last estimates, sum_d_out
 * (n) the accumulated Eq. 3 sums.  depth_limit 0 means no limit.  Node v's
 * counter starts with the element hash_ids[v] (NULL: v), as after a
 * renumbering of the nodes that keeps hashing their original ids (the
 * optional reordering of Sec. 3.2).  reg_bits is 8 or 4: 4-bit registers
 * (the paper's packed format, Sec. 3.4) hold at most 15, so an inserted rank
 * above 15 is stored as 15; every later value is a max of inserted values
 * and stays below 16 by itself.  Registers are returned one per byte.
 * Returns 0, or -1 on allocation failure / malformed rows.
 */
int or_hyperball(int64_t n, const uint64_t *offsets, const uint32_t *degrees,
                 const uint8_t *bytes, int p, uint32_t depth_limit, uint64_t seed,
                 const uint32_t *hash_ids, int reg_bits, uint8_t *regs_out, double *reach_out,
                 double *sum_d_out, or_hb_info *info) {
    const uint64_t m = 1ull << p;
    uint8_t *cur = (uint8_t *)calloc((size_t)(n * m), 1);
    uint8_t *next = (uint8_t *)calloc((size_t)(n * m), 1);
    double *c_prev = (double *)malloc(sizeof(double) * (size_t)n);
    double *c_now = (double *)malloc(sizeof(double) * (size_t)n);
    double *sum_d = (double *)calloc((size_t)n, sizeof(double));
    int bad = 0;
    if (!cur || !next || !c_prev || !c_now || !sum_d) bad = 1;

    if (!bad) {
        /* Insert v into its own counter. */
        for (int64_t v = 0; v < n; ++v) {
            uint32_t j, r;
            or_hll_insert(hash_ids ? (uint64_t)hash_ids[v] : (uint64_t)v, seed, p, &j, &r);
            if (reg_bits == 4 && r > 15) r = 15;
            cur[v * m + j] = (uint8_t)r;
        }
        /* Initial estimates c_0. */
        for (int64_t v = 0; v < n; ++v) c_prev[v] = or_hll_estimate(cur + v * m, p);
    }

    uint32_t t = 0;
    double maxd = 0.0;
    uint32_t converged = 0;
    while (!bad) {
        t++;
        /* Eq. 2: next[v] = max(cur[v], max over neighbours w of cur[w]). */
#pragma omp parallel
        {
            uint32_t *ids = NULL;
            int64_t cap = 0;
#pragma omp for schedule(dynamic, 16)
            for (int64_t v = 0; v < n; ++v) {
                if ((int64_t)degrees[v] > cap) {
                    free(ids);
                    cap = degrees[v];
                    ids = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)cap);
                }
                int64_t k = or_decode_row(bytes, offsets, v, ids, cap);
                if (k != (int64_t)degrees[v]) {
#pragma omp atomic write
                    bad = 1;
                    continue;
                }
                uint8_t *dst = next + v * m;
                memcpy(dst, cur + v * m, (size_t)m);
                for (int64_t e = 0; e < k; ++e) {
                    const uint8_t *src = cur + (uint64_t)ids[e] * m;
                    for (uint64_t j = 0; j < m; ++j)
                        if (src[j] > dst[j]) dst[j] = src[j];
                }
            }
            free(ids);
        }
        if (bad) break;
        /* Estimate c_t, then Eq. 3. */
#pragma omp parallel for schedule(static)
        for (int64_t v = 0; v < n; ++v) c_now[v] = or_hll_estimate(next + v * m, p);
        maxd = -INFINITY;
        for (int64_t v = 0; v < n; ++v) {
            const double delta = c_now[v] - c_prev[v];
            sum_d[v] = sum_d[v] + (double)t * delta;
            if (delta > maxd) maxd = delta;
            c_prev[v] = c_now[v];
        }
        if (n == 0) maxd = 0.0;
        converged = (maxd <= 0.5);
        if (converged) break;
        if (depth_limit != 0 && t == depth_limit) break;
        if (t > (uint32_t)n + 1) break; /* cannot happen: registers fix after D steps */
        uint8_t *tmp = cur;
        cur = next;
        next = tmp;
    }

    if (!bad) {
        if (regs_out) memcpy(regs_out, next, (size_t)(n * m));
        if (reach_out) memcpy(reach_out, c_prev, sizeof(double) * (size_t)n);
        if (sum_d_out) memcpy(sum_d_out, sum_d, sizeof(double) * (size_t)n);
        if (info) {
            info->passes = t;
            info->converged = converged;
            info->max_delta = maxd;
        }
    }
    free(cur);
    free(next);
    free(c_prev);
    free(c_now);
    free(sum_d);
    return bad ? -1 : 0;
}

/*
 * The same iteration with exact sets in place of HLL counters: each node's
 * counter is a bitset of the nodes it has reached, the union is bitwise OR
 * and the "estimate" is the exact popcount.  With exact cardinalities the
 * Eq. 3 accumulation must give the exact BFS distance sums of Eq. 1, which
 * pins the accumulation and stopping logic independently of the HLL.
 * card_out (n) receives |B(v, T)|, sum_d_out (n) the sums.  Small n only.
 */
int or_hyperball_exact(int64_t n, const uint64_t *offsets, const uint32_t *degrees,
                       const uint8_t *bytes, uint32_t depth_limit, double *card_out,
                       double *sum_d_out, or_hb_info *info) {
    const int64_t W = (n + 63) / 64;
    uint64_t *cur = (uint64_t *)calloc((size_t)(n * W) + 1, sizeof(uint64_t));
    uint64_t *next = (uint64_t *)calloc((size_t)(n * W) + 1, sizeof(uint64_t));
    double *c_prev = (double *)malloc(sizeof(double) * (size_t)n + 8);
    double *c_now = (double *)malloc(sizeof(double) * (size_t)n + 8);
    double *sum_d = (double *)calloc((size_t)n + 1, sizeof(double));
    uint32_t *ids = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(n + 1));
    int bad = (!cur || !next || !c_prev || !c_now || !sum_d || !ids);
    if (!bad) {
        for (int64_t v = 0; v < n; ++v) {
            cur[v * W + v / 64] |= 1ull << (v % 64);
            c_prev[v] = 1.0;
        }
    }
    uint32_t t = 0, converged = 0;
    double maxd = 0.0;
    while (!bad) {
        t++;
        for (int64_t v = 0; v < n; ++v) {
            int64_t k = or_decode_row(bytes, offsets, v, ids, n);
            if (k != (int64_t)degrees[v]) { bad = 1; break; }
            memcpy(next + v * W, cur + v * W, sizeof(uint64_t) * (size_t)W);
            for (int64_t e = 0; e < k; ++e)
                for (int64_t w = 0; w < W; ++w) next[v * W + w] |= cur[(int64_t)ids[e] * W + w];
        }
        if (bad) break;
        maxd = (n == 0) ? 0.0 : -INFINITY;
        for (int64_t v = 0; v < n; ++v) {
            int64_t c = 0;
            for (int64_t w = 0; w < W; ++w) c += __builtin_popcountll(next[v * W + w]);
            c_now[v] = (double)c;
            const double delta = c_now[v] - c_prev[v];
            sum_d[v] = sum_d[v] + (double)t * delta;
            if (delta > maxd) maxd = delta;
            c_prev[v] = c_now[v];
        }
        converged = (maxd <= 0.5);
        if (converged) break;
        if (depth_limit != 0 && t == depth_limit) break;
        if (t > (uint32_t)n + 1) break;
        uint64_t *tmp = cur;
        cur = next;
        next = tmp;
    }
    if (!bad) {
        if (card_out) memcpy(card_out, c_prev, sizeof(double) * (size_t)n);
        if (sum_d_out) memcpy(sum_d_out, sum_d, sizeof(double) * (size_t)n);
        if (info) {
            info->passes = t;
            info->converged = converged;
            info->max_delta = maxd;
        }
    }
    free(cur); free(next); free(c_prev); free(c_now); free(sum_d); free(ids);
    return bad ? -1 : 0;
}

/* ------------------------------------------------------------------------- */
/* Exact breadth-first search (textbook)                                      */
/* ------------------------------------------------------------------------- */

/* Hop distances from src (-1 = unreachable).  Returns 0 or -1. */
int or_bfs(int64_t n, const uint64_t *offsets, const uint32_t *degrees, const uint8_t *bytes,
           int64_t src, int32_t *dist) {
    int64_t *queue = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    uint32_t *ids = NULL;
    int64_t cap = 0;
    if (!queue) return -1;
    for (int64_t v = 0; v < n; ++v) dist[v] = -1;
    int64_t head = 0, tail = 0;
    dist[src] = 0;
    queue[tail++] = src;
    int bad = 0;
    while (head < tail) {
        int64_t u = queue[head++];
        if ((int64_t)degrees[u] > cap) {
            free(ids);
            cap = degrees[u];
            ids = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)cap);
        }
        int64_t k = or_decode_row(bytes, offsets, u, ids, cap);
        if (k != (int64_t)degrees[u]) { bad = 1; break; }
        for (int64_t e = 0; e < k; ++e) {
            int64_t w = ids[e];
            if (dist[w] < 0) {
                dist[w] = dist[u] + 1;
                queue[tail++] = w;
            }
        }
    }
    free(ids);
    free(queue);
    return bad ? -1 : 0;
}

/* BFS from every node (small graphs): dist is n x n, row = source. */
int or_bfs_all(int64_t n, const uint64_t *offsets, const uint32_t *degrees, const uint8_t *bytes,
               int32_t *dist) {
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t s = 0; s < n; ++s)
        if (or_bfs(n, offsets, degrees, bytes, s, dist + s * n) != 0) {
#pragma omp atomic write
            bad = 1;
        }
    return bad ? -1 : 0;
}

/*
 * Registers of the exact ball B(s, t): the union of the one-element sketches
 * of every node at hop distance <= t from s (dist from or_bfs).
 */
void or_ball_registers(int64_t n, const int32_t *dist, int32_t t, int p, uint64_t seed,
                       uint8_t *regs) {
    const uint64_t m = 1ull << p;
    memset(regs, 0, (size_t)m);
    for (int64_t u = 0; u < n; ++u) {
        if (dist[u] < 0 || dist[u] > t) continue;
        uint32_t j, r;
        or_hll_insert((uint64_t)u, seed, p, &j, &r);
        if (r > regs[j]) regs[j] = (uint8_t)r;
    }
}

/*
 * Multi-source BFS for up to 64 sources at once (one bit per source),
 * levels 0..T.  For source k and level t it writes:
 *   regs_out[(k * (T+1) + t) * m .. +m)  registers of B(s_k, t)
 *   ball_out[k * (T+1) + t]              |B(s_k, t)|
 * Cost: one pass over all edges per level.  Returns 0 or -1.
 */
int or_msbfs_balls(int64_t n, const uint64_t *offsets, const uint32_t *degrees,
                   const uint8_t *bytes, const int64_t *src, int32_t ns, int32_t T, int p,
                   uint64_t seed, uint8_t *regs_out, uint64_t *ball_out) {
    if (ns < 1 || ns > 64) return -1;
    const uint64_t m = 1ull << p;
    uint64_t *seen = (uint64_t *)calloc((size_t)n, sizeof(uint64_t));
    uint64_t *front = (uint64_t *)calloc((size_t)n, sizeof(uint64_t));
    uint64_t *nfront = (uint64_t *)calloc((size_t)n, sizeof(uint64_t));
    uint32_t *hj = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)n);
    uint32_t *hr = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)n);
    if (!seen || !front || !nfront || !hj || !hr) {
        free(seen); free(front); free(nfront); free(hj); free(hr);
        return -1;
    }
    for (int64_t u = 0; u < n; ++u) or_hll_insert((uint64_t)u, seed, p, &hj[u], &hr[u]);
    for (int32_t k = 0; k < ns; ++k) {
        seen[src[k]] |= 1ull << k;
        front[src[k]] |= 1ull << k;
    }
    int bad = 0;
    for (int32_t t = 0; t <= T && !bad; ++t) {
        if (t > 0) {
            /* pull: a node joins source k's ball if a neighbour is on k's frontier */
#pragma omp parallel
            {
                uint32_t *ids = NULL;
                int64_t cap = 0;
#pragma omp for schedule(dynamic, 64)
                for (int64_t v = 0; v < n; ++v) {
                    if ((int64_t)degrees[v] > cap) {
                        free(ids);
                        cap = degrees[v];
                        ids = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)cap);
                    }
                    int64_t k = or_decode_row(bytes, offsets, v, ids, cap);
                    if (k != (int64_t)degrees[v]) {
#pragma omp atomic write
                        bad = 1;
                        continue;
                    }
                    uint64_t acc = 0;
                    for (int64_t e = 0; e < k; ++e) acc |= front[ids[e]];
                    nfront[v] = acc & ~seen[v];
                }
                free(ids);
            }
            for (int64_t v = 0; v < n; ++v) {
                seen[v] |= nfront[v];
                front[v] = nfront[v];
            }
        }
        /* balls and registers at level t */
#pragma omp parallel for schedule(static, 1)
        for (int32_t k = 0; k < ns; ++k) {
            uint8_t *regs = regs_out + ((uint64_t)k * (uint64_t)(T + 1) + (uint64_t)t) * m;
            memset(regs, 0, (size_t)m);
            uint64_t cnt = 0;
            for (int64_t u = 0; u < n; ++u) {
                if (!((seen[u] >> k) & 1)) continue;
                cnt++;
                if (hr[u] > regs[hj[u]]) regs[hj[u]] = (uint8_t)hr[u];
            }
            ball_out[(uint64_t)k * (uint64_t)(T + 1) + (uint64_t)t] = cnt;
        }
    }
    free(seen); free(front); free(nfront); free(hj); free(hr);
    return bad ? -1 : 0;
}

/*
 * One union step (Eq. 2) plus estimate for a chosen list of nodes, timed by
 * the caller: the unit of work the CPU baseline measures.  next_out holds
 * ns * 2^p registers, est_out ns estimates.  Returns the edges processed.
 */
int64_t or_union_sample(int64_t n, const uint64_t *offsets, const uint32_t *degrees,
                        const uint8_t *bytes, int p, const uint8_t *cur, const int64_t *nodes,
                        int64_t ns, uint8_t *next_out, double *est_out) {
    (void)n;
    const uint64_t m = 1ull << p;
    int64_t edges = 0;
    int bad = 0;
#pragma omp parallel
    {
        uint32_t *ids = NULL;
        int64_t cap = 0;
#pragma omp for schedule(dynamic, 1) reduction(+ : edges)
        for (int64_t i = 0; i < ns; ++i) {
            const int64_t v = nodes[i];
            if ((int64_t)degrees[v] > cap) {
                free(ids);
                cap = degrees[v];
                ids = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)cap);
            }
            int64_t k = or_decode_row(bytes, offsets, v, ids, cap);
            if (k != (int64_t)degrees[v]) {
#pragma omp atomic write
                bad = 1;
                continue;
            }
            uint8_t *dst = next_out + (uint64_t)i * m;
            memcpy(dst, cur + (uint64_t)v * m, (size_t)m);
            for (int64_t e = 0; e < k; ++e) {
                const uint8_t *s = cur + (uint64_t)ids[e] * m;
                for (uint64_t j = 0; j < m; ++j)
                    if (s[j] > dst[j]) dst[j] = s[j];
            }
            est_out[i] = or_hll_estimate(dst, p);
            edges += k;
        }
        free(ids);
    }
    return bad ? -1 : edges;
}

int or_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads used by later parallel loops (timing only; results do not depend on it). */
void or_set_num_threads(int k) {
#ifdef _OPENMP
    if (k >= 1) omp_set_num_threads(k);
#else
    (void)k;
#endif
}

/*
 * VGA metrics (Sec. 3.3, "Metric derivation") for every node, written out one
 * by one: out holds 8 arrays of n doubles -- connectivity k = deg(v); control,
 * the sum over the neighbours w (in row order) of 1 / deg(w); MD = sum_d /
 * (N - 1) with N the exact component size (comp_size, or n); RA = 2 (MD - 1) /
 * (N - 2); integration [HH] = D_N / RA, the reciprocal of RRA = RA / D_N with
 * Hillier & Hanson's diamond value D_N = 2 (N (log2((N + 2) / 3) - 1) + 1) /
 * ((N - 1)(N - 2)); integration [Tekl] = log2((MD + 2) / 3); integration
 * [P-value] = max(0, 1 - RA); point first moment = MD k.  NaN where N is too
 * small for a formula (MD: N < 2; RA-based: N < 3).  Returns 0, or -1 on a
 * malformed row.
 */
int or_vga_metrics(int64_t n, const uint64_t *offsets, const uint32_t *degrees,
                   const uint8_t *bytes, const uint32_t *comp_size, const double *sum_d,
                   double *out) {
    int bad = 0;
#pragma omp parallel
    {
        uint32_t *ids = NULL;
        int64_t cap = 0;
#pragma omp for schedule(dynamic, 64)
        for (int64_t v = 0; v < n; ++v) {
            if ((int64_t)degrees[v] > cap) {
                free(ids);
                cap = degrees[v];
                ids = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)cap);
            }
            const int64_t k = or_decode_row(bytes, offsets, v, ids, cap);
            if (k != (int64_t)degrees[v]) {
#pragma omp atomic write
                bad = 1;
                continue;
            }
            double control = 0.0;
            for (int64_t e = 0; e < k; ++e) control += 1.0 / (double)degrees[ids[e]];
            const double N = comp_size ? (double)comp_size[v] : (double)n;
            const double md = N >= 2.0 ? sum_d[v] / (N - 1.0) : NAN;
            const double ra = N >= 3.0 ? 2.0 * (md - 1.0) / (N - 2.0) : NAN;
            const double dk = N >= 3.0 ? 2.0 * (N * (log2((N + 2.0) / 3.0) - 1.0) + 1.0) /
                                             ((N - 1.0) * (N - 2.0))
                                       : NAN;
            out[0 * n + v] = (double)k;
            out[1 * n + v] = control;
            out[2 * n + v] = md;
            out[3 * n + v] = ra;
            out[4 * n + v] = dk / ra;
            out[5 * n + v] = N >= 2.0 ? log2((md + 2.0) / 3.0) : NAN;
            out[6 * n + v] = N >= 3.0 ? fmax(0.0, 1.0 - ra) : NAN;
            out[7 * n + v] = md * (double)k;
        }
        free(ids);
    }
    return bad ? -1 : 0;
}

/*
 * Point second moment (Sec. 3.3, "Metric derivation", a local metric computed
 * exactly from the 1-hop neighbourhood), read as the second moment of the
 * visible cells about the cell itself, as Turner et al. (2001) define isovist
 * moments: PSM(v) = sum over neighbours w of (x_w - x_v)^2 + (y_w - y_v)^2, in
 * squared cell units, with xy[2v], xy[2v+1] the cell of node v.  The sum is
 * formed in 64-bit integers and converted to double once.  Returns 0, or -1 on
 * a malformed row.
 */
int or_point_second_moment(int64_t n, const uint64_t *offsets, const uint32_t *degrees,
                           const uint8_t *bytes, const int32_t *xy, double *out) {
    int bad = 0;
#pragma omp parallel
    {
        uint32_t *ids = NULL;
        int64_t cap = 0;
#pragma omp for schedule(dynamic, 64)
        for (int64_t v = 0; v < n; ++v) {
            if ((int64_t)degrees[v] > cap) {
                free(ids);
                cap = degrees[v];
                ids = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)cap);
            }
            const int64_t k = or_decode_row(bytes, offsets, v, ids, cap);
            if (k != (int64_t)degrees[v]) {
#pragma omp atomic write
                bad = 1;
                continue;
            }
            uint64_t sum = 0;
            for (int64_t e = 0; e < k; ++e) {
                const int64_t dx = (int64_t)xy[2 * ids[e]] - (int64_t)xy[2 * v];
                const int64_t dy = (int64_t)xy[2 * ids[e] + 1] - (int64_t)xy[2 * v + 1];
                sum += (uint64_t)(dx * dx + dy * dy);
            }
            out[v] = (double)sum;
        }
        free(ids);
    }
    return bad ? -1 : 0;
}

/*
 * Local VGA metrics from the neighbourhoods (Sec. 3.3, "Metric derivation":
 * computed exactly, without the HLL), for the nodes listed in nodes[0..count)
 * (nodes = NULL: every node, count = n), written out one by one per listed
 * node i:
 *   pairs[i]  = ordered pairs (a, b) of neighbours of v that are adjacent,
 *               i.e. the sum over neighbours a of |N(a) intersect N(v)|
 *               (each link among the neighbours counts twice);
 *   ball2[i]  = nodes u != v within two steps of v, |B(v, 2)| - 1;
 *   clustering[i] = pairs / (k (k - 1)) with k = deg(v), the Watts & Strogatz
 *               (1998) coefficient; NaN for k < 2;
 *   controllability[i] = k / ball2, the first-step neighbourhood over the
 *               two-step one (Turner et al. 2001); NaN for an isolated node.
 * Membership uses per-thread arrays stamped with i + 1, so a node listed twice
 * is counted afresh each time.  Any NULL output is
 * skipped.  Returns 0, or -1 on a malformed row.
 */
int or_local_metrics(int64_t n, const uint64_t *offsets, const uint32_t *degrees,
                     const uint8_t *bytes, const uint32_t *nodes, int64_t count,
                     uint64_t *pairs, uint32_t *ball2, double *clustering,
                     double *controllability) {
    int bad = 0;
    if (!nodes) count = n;
#pragma omp parallel
    {
        uint32_t *in_nv = (uint32_t *)calloc((size_t)n, sizeof(uint32_t));
        uint32_t *in_b2 = (uint32_t *)calloc((size_t)n, sizeof(uint32_t));
        uint32_t *row = NULL, *row2 = NULL;
        int64_t cap = 0, cap2 = 0;
#pragma omp for schedule(dynamic, 16)
        for (int64_t i = 0; i < count; ++i) {
            const int64_t v = nodes ? (int64_t)nodes[i] : i;
            const uint32_t stamp = (uint32_t)i + 1u;
            if ((int64_t)degrees[v] > cap) {
                free(row);
                cap = degrees[v];
                row = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)cap);
            }
            const int64_t k = or_decode_row(bytes, offsets, v, row, cap);
            if (k != (int64_t)degrees[v]) {
#pragma omp atomic write
                bad = 1;
                continue;
            }
            for (int64_t e = 0; e < k; ++e) in_nv[row[e]] = stamp;
            uint64_t links = 0;
            uint32_t reach2 = 0;
            for (int64_t e = 0; e < k; ++e) {
                const uint32_t a = row[e];
                if (in_b2[a] != stamp) {
                    in_b2[a] = stamp;
                    ++reach2;
                }
                if ((int64_t)degrees[a] > cap2) {
                    free(row2);
                    cap2 = degrees[a];
                    row2 = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)cap2);
                }
                const int64_t ka = or_decode_row(bytes, offsets, a, row2, cap2);
                if (ka != (int64_t)degrees[a]) {
#pragma omp atomic write
                    bad = 1;
                    break;
                }
                for (int64_t f = 0; f < ka; ++f) {
                    const uint32_t b = row2[f];
                    if (in_nv[b] == stamp) ++links;
                    if ((int64_t)b != v && in_b2[b] != stamp) {
                        in_b2[b] = stamp;
                        ++reach2;
                    }
                }
            }
            if (pairs) pairs[i] = links;
            if (ball2) ball2[i] = reach2;
            if (clustering)
                clustering[i] = k >= 2 ? (double)links / ((double)k * (double)(k - 1)) : NAN;
            if (controllability)
                controllability[i] = reach2 >= 1 ? (double)k / (double)reach2 : NAN;
        }
        free(row);
        free(row2);
        free(in_nv);
        free(in_b2);
    }
    return bad ? -1 : 0;
}
