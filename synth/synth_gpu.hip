// Seeded synthetic visibility graphs on the GPU (input tooling, not the
// HyperBall path).  Computes the same visibility rule as synth.c -- the closed
// segment between two cell centres meets no closed obstacle square -- for
// every ordered pair of nodes, as one bit per pair, rows of ceil(n/32) words.
//
// The walk is division-free: the problem is transposed so the segment is
// x-major (|dy| <= dx), then for each column the y-extent of the segment over
// that column is tracked as a quotient/remainder of 2*dx, which changes by at
// most one step per column.  Every row whose closed cell span meets that
// extent is tested.  synth.c computes the same cells with exact divisions; the
// two are checked against each other on the CPU (syng_visible_host) and on
// sampled pairs of GPU-built graphs.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <string>

namespace {

thread_local std::string g_err;

struct BitRaster {
    const uint32_t *bits;
    int32_t W;
    __host__ __device__ bool blocked(int32_t x, int32_t y) const {
        const uint32_t idx = (uint32_t)y * (uint32_t)W + (uint32_t)x;
        return (bits[idx >> 5] >> (idx & 31u)) & 1u;
    }
};

// Rows j (in the walk's frame) with ceil(lo/D) - 1 <= j <= floor(hi/D), where
// lo/hi are the segment's extent over the column as (quotient, remainder) of D.
__host__ __device__ inline bool column_blocked(const BitRaster &r, bool tr, int32_t i, int32_t qlo,
                                               int32_t rlo, int32_t qhi) {
    const int32_t jmin = qlo + (rlo != 0 ? 1 : 0) - 1;
    for (int32_t j = jmin; j <= qhi; ++j)
        if (tr ? r.blocked(j, i) : r.blocked(i, j)) return true;
    return false;
}

__host__ __device__ inline void step(int32_t &q, int32_t &rem, int32_t s, int32_t D) {
    rem += s;
    if (rem >= D) {
        rem -= D;
        ++q;
    } else if (rem < 0) {
        rem += D;
        --q;
    }
}

__host__ __device__ bool visible(const BitRaster &r, int32_t ax, int32_t ay, int32_t bx,
                                 int32_t by) {
    int32_t adx = bx - ax, ady = by - ay;
    adx = adx < 0 ? -adx : adx;
    ady = ady < 0 ? -ady : ady;
    const bool tr = ady > adx;
    if (tr) {
        int32_t t = ax; ax = ay; ay = t;
        t = bx; bx = by; by = t;
    }
    if (ax > bx) {
        int32_t t = ax; ax = bx; bx = t;
        t = ay; ay = by; by = t;
    }
    const int32_t dx = bx - ax, dy = by - ay;
    if (dx == 0) return !(tr ? r.blocked(ay, ax) : r.blocked(ax, ay));  // same cell
    const int32_t D = 2 * dx;
    // N(x) = (2ay+1) dx + (x - (2ax+1)) dy is the segment's y (doubled) times dx.
    // Column ax spans x in [2ax+1, 2ax+2]: N(2ax+1) = ay*D + dx.
    int32_t qa = ay, ra = dx;
    int32_t qb = qa, rb = ra;
    step(qb, rb, dy, D);
    if (dy >= 0 ? column_blocked(r, tr, ax, qa, ra, qb) : column_blocked(r, tr, ax, qb, rb, qa))
        return false;
    for (int32_t i = ax + 1; i < bx; ++i) {
        qa = qb;
        ra = rb;
        step(qb, rb, 2 * dy, D);
        if (dy >= 0 ? column_blocked(r, tr, i, qa, ra, qb) : column_blocked(r, tr, i, qb, rb, qa))
            return false;
    }
    // column bx spans x in [2bx, 2bx+1]: N(2bx+1) = by*D + dx
    qa = qb;
    ra = rb;
    qb = by;
    rb = dx;
    if (dy >= 0 ? column_blocked(r, tr, bx, qa, ra, qb) : column_blocked(r, tr, bx, qb, rb, qa))
        return false;
    return true;
}

constexpr int kThreads = 256;
constexpr uint32_t kMaxLdsWords = 16384;  // 64 KB of raster bits in LDS

template <bool LDS>
__global__ __launch_bounds__(kThreads) void vis_rows_kernel(const uint32_t *__restrict__ gbits,
                                                            uint32_t nwords, int32_t W,
                                                            const int32_t *__restrict__ xy,
                                                            uint32_t n, uint32_t wpr,
                                                            uint32_t src0,
                                                            uint32_t *__restrict__ out) {
    extern __shared__ uint32_t sbits[];
    const uint32_t *bits = gbits;
    if (LDS) {
        for (uint32_t k = threadIdx.x; k < nwords; k += kThreads) sbits[k] = gbits[k];
        __syncthreads();
        bits = sbits;
    }
    const BitRaster ras{bits, W};
    const uint32_t s = src0 + blockIdx.x;
    const int32_t sx = xy[2 * s], sy = xy[2 * s + 1];
    uint32_t *row = out + (uint64_t)blockIdx.x * wpr;
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    for (uint32_t t0 = 0; t0 < n; t0 += kThreads) {
        const uint32_t t = t0 + threadIdx.x;
        bool vis = false;
        if (t < n && t != s) vis = visible(ras, sx, sy, xy[2 * t], xy[2 * t + 1]);
        const uint64_t m = __builtin_amdgcn_ballot_w64(vis);
        const uint32_t w = (t0 + wave * 64u) >> 5;
        if (lane == 0 && w < wpr) row[w] = (uint32_t)m;
        if (lane == 32 && w + 1 < wpr) row[w + 1] = (uint32_t)(m >> 32);
    }
}

int fail(const char *msg, hipError_t e) {
    g_err = std::string(msg) + ": " + hipGetErrorString(e);
    return -1;
}

}  // namespace

extern "C" {

const char *syng_last_error(void) { return g_err.c_str(); }

// CPU build of the GPU walk, for checking it against synth.c on the host.
// bits: row-major raster, one bit per cell (bit idx & 31 of word idx >> 5).
int syng_visible_host(const uint32_t *bits, int32_t W, int32_t ax, int32_t ay, int32_t bx,
                      int32_t by) {
    const BitRaster r{bits, W};
    return visible(r, ax, ay, bx, by) ? 1 : 0;
}

// Visibility bit rows for sources [src0, src0 + count): out (host) receives
// count rows of wpr = ceil(n / 32) words; bit t of row s is 1 iff t != s and
// node t is visible from node s.  bits: raster bits as above (host).
int syng_rows(const uint32_t *bits, int32_t W, int32_t H, const int32_t *xy, uint32_t n,
              uint32_t src0, uint32_t count, uint32_t *out) {
    if (n == 0 || count == 0) return 0;
    if (src0 + (uint64_t)count > n) {
        g_err = "source range outside [0, n)";
        return -1;
    }
    const uint32_t nwords = (uint32_t)(((uint64_t)W * H + 31) / 32);
    const uint32_t wpr = (n + 31) / 32;
    uint32_t *d_bits = nullptr, *d_out = nullptr;
    int32_t *d_xy = nullptr;
    hipError_t e;
    if ((e = hipMalloc(&d_bits, sizeof(uint32_t) * nwords)) != hipSuccess)
        return fail("hipMalloc(bits)", e);
    if ((e = hipMalloc(&d_xy, sizeof(int32_t) * 2 * (uint64_t)n)) != hipSuccess) {
        (void)hipFree(d_bits);
        return fail("hipMalloc(xy)", e);
    }
    if ((e = hipMalloc(&d_out, sizeof(uint32_t) * (uint64_t)wpr * count)) != hipSuccess) {
        (void)hipFree(d_bits);
        (void)hipFree(d_xy);
        return fail("hipMalloc(out)", e);
    }
    int rc = 0;
    do {
        if ((e = hipMemcpy(d_bits, bits, sizeof(uint32_t) * nwords, hipMemcpyHostToDevice)) !=
            hipSuccess) { rc = fail("hipMemcpy(bits)", e); break; }
        if ((e = hipMemcpy(d_xy, xy, sizeof(int32_t) * 2 * (uint64_t)n, hipMemcpyHostToDevice)) !=
            hipSuccess) { rc = fail("hipMemcpy(xy)", e); break; }
        if (nwords <= kMaxLdsWords) {
            hipLaunchKernelGGL(vis_rows_kernel<true>, dim3(count), dim3(kThreads),
                               sizeof(uint32_t) * nwords, 0, d_bits, nwords, W, d_xy, n, wpr, src0,
                               d_out);
        } else {
            hipLaunchKernelGGL(vis_rows_kernel<false>, dim3(count), dim3(kThreads), 0, 0, d_bits,
                               nwords, W, d_xy, n, wpr, src0, d_out);
        }
        if ((e = hipGetLastError()) != hipSuccess) { rc = fail("vis_rows_kernel launch", e); break; }
        if ((e = hipMemcpy(out, d_out, sizeof(uint32_t) * (uint64_t)wpr * count,
                           hipMemcpyDeviceToHost)) != hipSuccess) {
            rc = fail("vis_rows_kernel / hipMemcpy(out)", e);
            break;
        }
    } while (0);
    (void)hipFree(d_bits);
    (void)hipFree(d_xy);
    (void)hipFree(d_out);
    return rc;
}

}  // extern "C"
