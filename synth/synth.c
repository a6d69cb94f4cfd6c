/*
 * Seeded synthetic visibility-graph inputs (CPU side).
 *
 * This module builds the *input* graphs that both the CPU oracle and the HIP
 * path consume.  It holds none of the HyperBall arithmetic: no hashing, no
 * registers, no estimator, no LEB128.  Its output is a plain adjacency list
 * (u64 row offsets + sorted u32 neighbour ids) over the main connected
 * component of an obstacle raster.
 *
 * Visibility rule (the graph used in place of the paper's sparkSieve2 edge
 * sets, Sec. 3.1): two open cells a != b are joined iff the closed segment
 * between their centres meets no obstacle cell, where an obstacle cell is the
 * closed unit square it covers (touching an edge or a corner blocks).  The
 * test is exact integer arithmetic in doubled coordinates: cell (x, y) covers
 * [2x, 2x+2] x [2y, 2y+2] and its centre is (2x+1, 2y+1).
 *
 * Every cell the segment touches forms a 4-connected chain of cells, so two
 * cells are mutually visible only if they lie in the same 4-connected region
 * of open cells.  The main component of the visibility graph is therefore the
 * largest 4-connected open region; it is found with union-find (path halving,
 * union by size) over 4-neighbour pairs, the connectivity bookkeeping Sec. 3.1
 * describes.  Nodes are numbered in raster order (y outer, x inner) over that
 * component, the numbering Sec. 3.2 assumes for small deltas.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* floor(a / b) for b > 0 */
static inline int64_t fdiv(int64_t a, int64_t b) {
    int64_t q = a / b;
    if ((a % b != 0) && (a < 0)) q -= 1;
    return q;
}

/* ceil(a / b) for b > 0 */
static inline int64_t cdiv(int64_t a, int64_t b) { return -fdiv(-a, b); }

/*
 * 1 if the closed segment between the centres of cells (ax, ay) and (bx, by)
 * meets no obstacle cell, else 0.  obst is row-major W x H, nonzero = obstacle.
 * The endpoints are normalised (ax <= bx) so the test is symmetric.
 */
int syn_visible(const uint8_t *obst, int32_t W, int32_t H, int32_t ax, int32_t ay,
                int32_t bx, int32_t by) {
    (void)H;
    if (ax > bx || (ax == bx && ay > by)) {
        int32_t t;
        t = ax; ax = bx; bx = t;
        t = ay; ay = by; by = t;
    }
    const int64_t dx = (int64_t)bx - ax, dy = (int64_t)by - ay;
    if (dx == 0) {
        for (int32_t y = ay; y <= by; ++y)
            if (obst[(int64_t)y * W + ax]) return 0;
        return 1;
    }
    const int64_t x0 = 2 * (int64_t)ax + 1, x1 = 2 * (int64_t)bx + 1;
    const int64_t ybase = (2 * (int64_t)ay + 1) * dx; /* Y(x0) * dx */
    for (int64_t i = ax; i <= bx; ++i) {
        /* the part of the segment over column i, in doubled x */
        const int64_t xl = (2 * i > x0) ? 2 * i : x0;
        const int64_t xr = (2 * i + 2 < x1) ? 2 * i + 2 : x1;
        const int64_t nl = ybase + (xl - x0) * dy; /* Y(xl) * dx */
        const int64_t nr = ybase + (xr - x0) * dy;
        const int64_t lo = nl < nr ? nl : nr, hi = nl < nr ? nr : nl;
        /* rows j whose closed span [2j, 2j+2] meets [lo/dx, hi/dx] */
        const int64_t jmin = cdiv(lo, 2 * dx) - 1;
        const int64_t jmax = fdiv(hi, 2 * dx);
        for (int64_t j = jmin; j <= jmax; ++j)
            if (obst[j * W + i]) return 0;
    }
    return 1;
}

/* ---- union-find over the open cells (path halving, union by size) ---- */
static int32_t uf_find(int32_t *par, int32_t x) {
    while (par[x] != x) {
        par[x] = par[par[x]];
        x = par[x];
    }
    return x;
}

static void uf_union(int32_t *par, int32_t *sz, int32_t a, int32_t b) {
    a = uf_find(par, a);
    b = uf_find(par, b);
    if (a == b) return;
    if (sz[a] < sz[b]) { int32_t t = a; a = b; b = t; }
    par[b] = a;
    sz[a] += sz[b];
}

/*
 * Label the largest 4-connected open region.  Writes node_of_cell[W*H]
 * (raster-order node id, or -1 for cells not in the main component) and
 * returns the node count.  Ties between equal-size regions go to the region
 * holding the lowest raster cell.
 */
int64_t syn_main_component(const uint8_t *obst, int32_t W, int32_t H, int32_t *node_of_cell) {
    const int64_t C = (int64_t)W * H;
    int32_t *par = (int32_t *)malloc(sizeof(int32_t) * C);
    int32_t *sz = (int32_t *)malloc(sizeof(int32_t) * C);
    if (!par || !sz) { free(par); free(sz); return -1; }
    for (int64_t c = 0; c < C; ++c) { par[c] = (int32_t)c; sz[c] = 1; }
    for (int32_t y = 0; y < H; ++y)
        for (int32_t x = 0; x < W; ++x) {
            const int64_t c = (int64_t)y * W + x;
            if (obst[c]) continue;
            if (x + 1 < W && !obst[c + 1]) uf_union(par, sz, (int32_t)c, (int32_t)(c + 1));
            if (y + 1 < H && !obst[c + W]) uf_union(par, sz, (int32_t)c, (int32_t)(c + W));
        }
    int32_t best = -1, best_sz = 0;
    for (int64_t c = 0; c < C; ++c) {
        if (obst[c]) continue;
        const int32_t r = uf_find(par, (int32_t)c);
        if (sz[r] > best_sz) { best_sz = sz[r]; best = r; }
    }
    int64_t n = 0;
    for (int64_t c = 0; c < C; ++c) {
        if (!obst[c] && best >= 0 && uf_find(par, (int32_t)c) == best)
            node_of_cell[c] = (int32_t)n++;
        else
            node_of_cell[c] = -1;
    }
    free(par);
    free(sz);
    return n;
}

/*
 * Degree of every node (number of other nodes visible from it).
 * xy holds the node cells as (x, y) pairs in node order.
 */
void syn_degrees(const uint8_t *obst, int32_t W, int32_t H, const int32_t *xy, int64_t n,
                 uint64_t *deg) {
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t s = 0; s < n; ++s) {
        const int32_t sx = xy[2 * s], sy = xy[2 * s + 1];
        uint64_t d = 0;
        for (int64_t t = 0; t < n; ++t) {
            if (t == s) continue;
            d += (uint64_t)syn_visible(obst, W, H, sx, sy, xy[2 * t], xy[2 * t + 1]);
        }
        deg[s] = d;
    }
}

/* Neighbour ids, ascending, into ids[off[s] .. off[s+1]). */
void syn_fill(const uint8_t *obst, int32_t W, int32_t H, const int32_t *xy, int64_t n,
              const uint64_t *off, uint32_t *ids) {
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t s = 0; s < n; ++s) {
        const int32_t sx = xy[2 * s], sy = xy[2 * s + 1];
        uint64_t k = off[s];
        for (int64_t t = 0; t < n; ++t) {
            if (t == s) continue;
            if (syn_visible(obst, W, H, sx, sy, xy[2 * t], xy[2 * t + 1])) ids[k++] = (uint32_t)t;
        }
    }
}

/* Degrees of a subset of source nodes (for estimating E on large rasters). */
void syn_degrees_sample(const uint8_t *obst, int32_t W, int32_t H, const int32_t *xy,
                        int64_t n, const int64_t *src, int64_t ns, uint64_t *deg) {
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < ns; ++k) {
        const int64_t s = src[k];
        const int32_t sx = xy[2 * s], sy = xy[2 * s + 1];
        uint64_t d = 0;
        for (int64_t t = 0; t < n; ++t) {
            if (t == s) continue;
            d += (uint64_t)syn_visible(obst, W, H, sx, sy, xy[2 * t], xy[2 * t + 1]);
        }
        deg[k] = d;
    }
}

/* Visibility of explicit node pairs (for spot checks of other generators). */
void syn_visible_pairs(const uint8_t *obst, int32_t W, int32_t H, const int32_t *xy,
                       const int64_t *a, const int64_t *b, int64_t np, uint8_t *out) {
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < np; ++k)
        out[k] = (uint8_t)syn_visible(obst, W, H, xy[2 * a[k]], xy[2 * a[k] + 1], xy[2 * b[k]],
                                      xy[2 * b[k] + 1]);
}

int syn_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ---- bit-row form used by the GPU generator ---- */

/* Raster as bits: bit (y*W + x) & 31 of word (y*W + x) >> 5 set for obstacles. */
void syn_raster_bits(const uint8_t *obst, int32_t W, int32_t H, uint32_t *bits) {
    const int64_t C = (int64_t)W * H, nw = (C + 31) / 32;
    memset(bits, 0, sizeof(uint32_t) * (size_t)nw);
    for (int64_t c = 0; c < C; ++c)
        if (obst[c]) bits[c >> 5] |= 1u << (c & 31);
}

/* Degrees (popcounts) of count bit rows of wpr words. */
void syn_row_degrees(const uint32_t *rows, int64_t wpr, int64_t count, uint64_t *deg) {
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < count; ++s) {
        uint64_t d = 0;
        const uint32_t *r = rows + s * wpr;
        for (int64_t k = 0; k < wpr; ++k) d += (uint64_t)__builtin_popcount(r[k]);
        deg[s] = d;
    }
}

/* Expand bit rows into ascending ids at ids[off[s] ..) (off indexed by row). */
void syn_row_ids(const uint32_t *rows, int64_t wpr, int64_t count, const uint64_t *off,
                 uint32_t *ids) {
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t s = 0; s < count; ++s) {
        const uint32_t *r = rows + s * wpr;
        uint64_t k = off[s];
        for (int64_t w = 0; w < wpr; ++w) {
            uint32_t bitsw = r[w];
            while (bitsw) {
                const int b = __builtin_ctz(bitsw);
                ids[k++] = (uint32_t)(w * 32 + b);
                bitsw &= bitsw - 1;
            }
        }
    }
}
