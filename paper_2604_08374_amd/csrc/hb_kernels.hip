// HyperBall kernels for gfx950 (CDNA4, wave64).
//
// One launch is one whole HyperBall step: the register-wise max of Eq. 2 for
// every node, with the estimator and the Eq. 3 accumulation fused into its
// epilogue.  Three union kernels give the same registers:
//
//  * the per-edge kernel is the paper's fused decode-union step (Sec. 3.4): it
//    decodes the node's LEB128 row and gathers every neighbour's counter;
//  * the run kernel (p <= 12) covers each run of consecutive neighbour ids
//    with one or two rows of a range-max table of the counters, built every
//    step, and reads the runs from a run list that the loader decodes once
//    from the LEB128 rows;
//  * the grouped kernel (the default for counters of 256 to 4096 bytes on
//    graphs of at least 32,768 nodes) reads the same table rows, merged by the
//    loader over groups of 16 nodes of the processing order, so that a row
//    that several nodes of a group need is loaded once for all of them.
//
// Design on gfx950:
//
//  * A counter of m = 2^p uint8 registers is spread over lanes in 16-byte
//    slices, so every gather is a coalesced 16 B/lane load.  Lanes per node
//    and nodes per workgroup form the schedule: up to 64 lanes a node sits in
//    one wave, whose lane groups gather different rows at once and are
//    max-reduced at the end; above 64, several waves of a workgroup share a
//    node, each owning a slice.  Several shapes are built for the autotuner,
//    and 4-bit registers (two per byte) have shapes of their own.
//  * Rows are decoded cooperatively 64 bytes at a time: a ballot of the
//    continuation bits marks varint ends, a segmented OR joins the 7-bit
//    groups (at most five per varint), a wave prefix sum turns the first id
//    and the deltas into absolute ids, and a lane permute packs them into
//    lanes 0..k-1.  Varints that straddle 64-byte chunks carry over.  The
//    shifts and prefix sums are DPP moves.
//  * Gathered rows come from readlane or from an LDS queue of table rows, so a
//    gather whose row serves the whole wave uses a scalar base address.  Tail
//    slots repeat a row already gathered (max is idempotent).
//  * Byte-wise max without unpacking: v_pk_max_u16 on the raw dword keeps the
//    max of bytes 1 and 3 in the high byte of each half, and on the dword
//    shifted left by 8 the max of bytes 0 and 2; two rows at a time go through
//    one packed fp16 three-input maximum per half instead.
//  * The estimator sums 2^(65-p-M) over the registers as an exact 128-bit
//    integer (wave butterfly with carries) and converts it to double with a
//    single rounding, so the estimate is independent of the reduction order.
//  * Workgroups are remapped across the 8 XCDs (which take workgroups
//    round-robin).  The per-edge kernel gives each XCD one contiguous range of
//    the processing order: nodes close in that order (along a Hilbert curve,
//    when the caller gives one) share most neighbours, so their gathers hit the
//    same L2.  The table kernels keep all XCDs on one stretch of the order at a
//    time, 64 workgroups each, so that the rows they share meet in the memory-
//    side cache that all XCDs share (city graph, p = 10: 7.9 against 9.0 ms
//    per grouped launch, 11.0 against 13.0 ms per run-kernel launch).
//  * The exact local metrics (clustering, controllability) walk the
//    neighbours' run lists against LDS arrays of n bits per node: a prefix
//    popcount of N(v) answers each run's intersection count in constant time,
//    and a difference array marks the words a run covers whole.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <mutex>

#include "hb_internal.h"

namespace hbk {
namespace {

constexpr int kWave = 64;
constexpr int kXcds = 8;
constexpr int kRunsMaxP = 12;  // the run kernel's tables are built for p <= 12

// Lanes that share one node's counter by default: one 16-byte slot per lane
// up to p = 10, one wave (1 to 4 slots per lane) at p = 11 and 12, and 4 KB
// wave slices beyond.  With 4-bit registers (two per byte, the paper's packed
// format) a counter has half the bytes: one slot per lane up to p = 11, one
// wave at p = 12 and 13, 4 KB slices beyond; p >= 5.
constexpr int default_lanes(int p, int bits = 8) {
    return bits == 8 ? (p <= 10 ? (1 << p) / 16 : (p <= 12 ? 64 : (1 << p) / 64))
                     : (p <= 11 ? (1 << p) / 32 : (p <= 13 ? 64 : (1 << p) / 128));
}

// Shape of one node's work for precision P with L lanes per node.  L <= 64:
// one wave holds 64 / L groups of L lanes; each group owns a whole counter
// and the groups gather different neighbours, max-reduced at the end.
// L > 64: L / 64 waves of one workgroup share the node, each owning a slice.
template <int P, int L = default_lanes(P), int B = 8>
struct Cfg {
    static constexpr int PREC = P;
    static constexpr int LANES = L;
    static constexpr int BITS = B;                               // bits per register
    static constexpr int M = (1 << P) * B / 8;                   // counter bytes
    static constexpr int WAVES = L > kWave ? L / kWave : 1;      // waves per node
    static constexpr int LPC = L > kWave ? kWave : L;            // lanes per counter in a wave
    static constexpr int G = kWave / LPC;                        // neighbour groups
    static constexpr int RPL = M / (16 * L);                     // uint4 slots per lane
    static constexpr int SLICE = M / WAVES;                      // counter bytes per wave
    static constexpr int U = RPL >= 8 ? 1 : 8 / RPL;             // gathers in flight
    static constexpr int NODES = WAVES == 1 ? 4 : 1;             // most nodes per workgroup
    static constexpr int THREADS = WAVES == 1 ? 256 : WAVES * kWave;
    static constexpr int TOP = 65 - P;                           // largest register value
    // waves per SIMD the run kernel is compiled for (its register budget):
    // 80 VGPRs with one slot per lane, 96 with two, 168 with four; 4-bit
    // accumulators take twice the registers per slot
    static constexpr int RUN_OCC = B == 8 ? (RPL == 1 ? 6 : (RPL == 2 ? 5 : 3))
                                          : (RPL == 1 ? 4 : (RPL == 2 ? 3 : 2));
    static_assert(RPL >= 1 && RPL <= 4 && M % (16 * L) == 0, "unsupported lanes per node");
};

// ---------------------------------------------------------------- helpers
__device__ __forceinline__ uint32_t lane_id() { return threadIdx.x & (kWave - 1); }

__device__ __forceinline__ uint64_t ballot(bool pred) {
    return __builtin_amdgcn_ballot_w64(pred);
}

// Data-parallel-primitive moves (VALU, no LDS round trip).  CTRL: 0x111-0x11F
// shift right within rows of 16 lanes, 0x138 shift right by one across the
// wave, 0x142 / 0x143 broadcast lane 15 / 31 of a row to the next row(s).
// Lanes with no source lane read 0.
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ uint32_t dpp(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, ROW_MASK, 0xf, false);
}

// Value of lane - 1 (0 in lane 0).
__device__ __forceinline__ uint32_t wave_shr1(uint32_t x) { return dpp<0x138>(x); }

// Inclusive prefix sum over the wave: doubling steps inside each row of 16
// lanes, then row 0's total into row 1 and row 2's into row 3, then the sum of
// rows 0-1 into rows 2 and 3.
__device__ __forceinline__ uint32_t wave_scan(uint32_t x) {
    x += dpp<0x111>(x);
    x += dpp<0x112>(x);
    x += dpp<0x114>(x);
    x += dpp<0x118>(x);
    x += dpp<0x142, 0xa>(x);
    x += dpp<0x143, 0xc>(x);
    return x;
}

__device__ __forceinline__ uint32_t shfl_idx(uint32_t x, uint32_t src) {
    return (uint32_t)__builtin_amdgcn_ds_bpermute((int)(src << 2), (int)x);
}

__device__ __forceinline__ uint32_t shfl_xor(uint32_t x, uint32_t mask) {
    return (uint32_t)__builtin_amdgcn_ds_bpermute((int)((lane_id() ^ mask) << 2), (int)x);
}

__device__ __forceinline__ uint32_t readlane(uint32_t x, uint32_t lane) {
    return (uint32_t)__builtin_amdgcn_readlane((int)x, (int)lane);
}

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t pk_max_u16(uint32_t a, uint32_t b) {
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(u16x2, a),
                                                                  __builtin_bit_cast(u16x2, b)));
}

typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));

// Max of three packed 16-bit halves, per half, as one packed fp16 maximum3.
// A half below 0x7C00 is a non-negative finite fp16 value, and on those the fp16
// order is the unsigned integer order (the kernels keep fp16 denormals, so the
// halves below 0x0400 compare exactly too).  8-bit registers are at most 61, so
// every half an 8-bit accumulator forms stays below 0x3E00.
__device__ __forceinline__ uint32_t pk_max3_u16(uint32_t a, uint32_t b, uint32_t c) {
    const f16x2 x = __builtin_bit_cast(f16x2, a);
    const f16x2 y = __builtin_bit_cast(f16x2, b);
    const f16x2 z = __builtin_bit_cast(f16x2, c);
    return __builtin_bit_cast(uint32_t,
                              __builtin_elementwise_maximum(__builtin_elementwise_maximum(x, y), z));
}

// Nibble-wise max accumulator for one dword of 8 4-bit registers.  a[k]
// holds the dword shifted left by 12 - 4k, which puts nibble k at the top of
// the low 16-bit half and nibble k + 4 at the top of the high half; a packed
// 16-bit max then keeps the max of those two nibbles (lower bits are
// don't-care).  7 VALU ops per 8 registers.
struct Max8 {
    uint32_t a[4];
    __device__ __forceinline__ void init(uint32_t w) {
        a[0] = w << 12;
        a[1] = w << 8;
        a[2] = w << 4;
        a[3] = w;
    }
    __device__ __forceinline__ void add(uint32_t w);
    __device__ __forceinline__ void add2(uint32_t w0, uint32_t w1) {
        add(w0);
        add(w1);
    }
    __device__ __forceinline__ uint32_t value() const {
        return ((a[0] >> 12) & 0x000F000Fu) | ((a[1] >> 8) & 0x00F000F0u) |
               ((a[2] >> 4) & 0x0F000F00u) | (a[3] & 0xF000F000u);
    }
};

// Byte-wise max accumulator for one dword of 4 registers.  hi tracks bytes
// 1 and 3 (the high byte of each 16-bit half); lo tracks bytes 0 and 2 after
// a left shift by 8 moves them into the high bytes.  The low bytes of both
// words are don't-care.  3 VALU ops per dword for one row, 4 for two.
struct Max4 {
    uint32_t lo, hi;
    __device__ __forceinline__ void init(uint32_t w) { lo = w << 8; hi = w; }
    __device__ __forceinline__ void add(uint32_t w) {
        hi = pk_max_u16(hi, w);
        lo = pk_max_u16(lo, w << 8);
    }
    __device__ __forceinline__ void add2(uint32_t w0, uint32_t w1) {
        hi = pk_max3_u16(hi, w0, w1);
        lo = pk_max3_u16(lo, w0 << 8, w1 << 8);
    }
    __device__ __forceinline__ uint32_t value() const {
        return ((lo >> 8) & 0x00FF00FFu) | (hi & 0xFF00FF00u);
    }
};

__device__ __forceinline__ void Max8::add(uint32_t w) {
    a[0] = pk_max_u16(a[0], w << 12);
    a[1] = pk_max_u16(a[1], w << 8);
    a[2] = pk_max_u16(a[2], w << 4);
    a[3] = pk_max_u16(a[3], w);
}

// The accumulator type of a register width.
template <int BITS> struct AccOf;
template <> struct AccOf<8> { using T = Max4; };
template <> struct AccOf<4> { using T = Max8; };

// SplitMix64 output function (Steele, Lea & Flood 2014).
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Exact partial of sum_j 2^(TOP - M[j]) (128-bit: lo, hi) and zero count.
struct EstPart {
    uint64_t lo, hi;
    uint32_t zeros;
    __device__ __forceinline__ void clear() { lo = 0; hi = 0; zeros = 0; }
    __device__ __forceinline__ void add_term(uint64_t term) {
        lo += term;
        hi += (lo < term) ? 1u : 0u;
    }
    template <int BITS>
    __device__ __forceinline__ void add_dword(uint32_t w, int top) {
        constexpr uint32_t mask = (1u << BITS) - 1u;
#pragma unroll
        for (int b = 0; b < 32 / BITS; ++b) {
            const uint32_t M = (w >> (BITS * b)) & mask;
            add_term(1ull << (top - (int)M));
            zeros += (M == 0u) ? 1u : 0u;
        }
    }
    __device__ __forceinline__ void add(const EstPart &o) {
        const uint64_t l = lo + o.lo;
        hi = hi + o.hi + ((l < lo) ? 1u : 0u);
        lo = l;
        zeros += o.zeros;
    }
    // butterfly over the whole wave: every lane ends with the wave total
    __device__ __forceinline__ void wave_reduce() {
#pragma unroll
        for (uint32_t mask = 1; mask < kWave; mask <<= 1) {
            EstPart o;
            o.lo = ((uint64_t)shfl_xor((uint32_t)(lo >> 32), mask) << 32) |
                   shfl_xor((uint32_t)lo, mask);
            o.hi = ((uint64_t)shfl_xor((uint32_t)(hi >> 32), mask) << 32) |
                   shfl_xor((uint32_t)hi, mask);
            o.zeros = shfl_xor(zeros, mask);
            add(o);
        }
    }
};

// HLL estimate from the exact sum S = hi 2^64 + lo (units of 2^-top) and the
// zero count: raw estimate alpha_m m^2 / Z, or linear counting m ln(m / V)
// when the raw estimate is at most 2.5 m and V > 0.
template <int P>
__device__ double estimate(const EstPart &e) {
    constexpr int top = Cfg<P>::TOP;
    const double md = (double)(1u << P);
    // S < 2^66: split into two exactly representable doubles, one rounding.
    const uint64_t upper = (e.hi << 32) | (e.lo >> 32);  // < 2^34
    const double s = (double)upper * 4294967296.0 + (double)(uint32_t)e.lo;
    const double Z = ldexp(s, -top);
    double alpha;
    if (P == 4) alpha = 0.673;
    else if (P == 5) alpha = 0.697;
    else if (P == 6) alpha = 0.709;
    else alpha = 0.7213 / (1.0 + 1.079 / md);
    const double E = ((alpha * md) * md) / Z;
    if (E <= 2.5 * md && e.zeros > 0u) return md * log(md / (double)e.zeros);
    return E;
}

// Workgroup index -> logical block so that XCD x (taking workgroups i with
// i % 8 == x) processes one contiguous range of logical blocks.
__device__ __forceinline__ uint32_t xcd_block(uint32_t i, uint32_t nblocks) {
    const uint32_t q = nblocks / kXcds, r = nblocks % kXcds;
    const uint32_t x = i % kXcds, k = i / kXcds;
    return (x < r) ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
}

// Workgroup index -> logical block so that the XCDs work side by side: in every
// span of kXcds * chunk workgroups, XCD x (taking workgroups i with i % 8 == x)
// processes logical blocks x * chunk .. x * chunk + chunk - 1 of the span, so
// that at any time all XCDs work on one stretch of the processing order; a
// last, partial span keeps the identity.
constexpr uint32_t kXcdSpanChunk = 64;  // 16 to 256 measured on the city graph: 64 best
__device__ __forceinline__ uint32_t xcd_span_block(uint32_t i, uint32_t nblocks,
                                                   uint32_t chunk) {
    const uint32_t span = chunk * kXcds, s = i / span;
    if ((s + 1u) * span > nblocks) return i;
    return s * span + (i % kXcds) * chunk + (i - s * span) / kXcds;
}

// Byte offset, within a counter, of lane-slot s (s < RPL) of this lane.
template <class C>
__device__ __forceinline__ uint32_t slot_offset(uint32_t slice, uint32_t lane, int s) {
    return slice * C::SLICE + (uint32_t)s * (C::LPC * 16u) + (lane % C::LPC) * 16u;
}

// Combine the estimator partials of the waves sharing a node and return the
// node total in every lane of wave 0 (others: unspecified).
template <class C>
__device__ EstPart node_total(EstPart e, uint32_t slice) {
    if (C::WAVES == 1) return e;
    __shared__ uint64_t s_lo[C::WAVES > 1 ? C::WAVES : 1];
    __shared__ uint64_t s_hi[C::WAVES > 1 ? C::WAVES : 1];
    __shared__ uint32_t s_z[C::WAVES > 1 ? C::WAVES : 1];
    if (lane_id() == 0) {
        s_lo[slice] = e.lo;
        s_hi[slice] = e.hi;
        s_z[slice] = e.zeros;
    }
    __syncthreads();
    EstPart tot;
    tot.clear();
    if (slice == 0) {
        for (int w = 0; w < C::WAVES; ++w) {
            EstPart o;
            o.lo = s_lo[w];
            o.hi = s_hi[w];
            o.zeros = s_z[w];
            tot.add(o);
        }
    }
    return tot;
}

// ---------------------------------------------------------------- init
// Zero node v's counter (this wave's slice), insert v, and set c_prev[v] to the
// estimate of the one-element counter and sum_d[v] to 0.  The inserted element
// is hash_ids[v] when given (the node's id before a relabelling), else v.
template <class C>
__device__ __forceinline__ void init_node(uint8_t *__restrict__ cur, double *__restrict__ c_prev,
                                          double *__restrict__ sum_d, uint32_t v, uint32_t slice,
                                          uint64_t seed, const uint32_t *__restrict__ hash_ids) {
    constexpr int P = C::PREC;
    const uint32_t lane = lane_id();
    const uint32_t id = hash_ids ? hash_ids[v] : v;
    const uint64_t h = splitmix64((uint64_t)id ^ seed);
    const uint32_t j = (uint32_t)(h >> (64 - P));
    const uint64_t rest = h << P;
    uint32_t r = rest ? (uint32_t)__builtin_clzll(rest) + 1u : (uint32_t)(65 - P);
    if (C::BITS == 4 && r > 15u) r = 15u;  // 4-bit registers saturate
    // register j sits in byte jb; with 4 bits, odd j in the high nibble
    const uint32_t jb = C::BITS == 8 ? j : j >> 1;
    const uint32_t sub = C::BITS == 8 ? 0u : 4u * (j & 1u);

    const bool owner = (lane / C::LPC) == 0;  // group 0 holds the counter
    EstPart e;
    e.clear();
    uint8_t *row = cur + (uint64_t)v * C::M;
#pragma unroll
    for (int s = 0; s < C::RPL; ++s) {
        const uint32_t off = slot_offset<C>(slice, lane, s);
        uint32_t w[4] = {0u, 0u, 0u, 0u};
        if (jb >= off && jb < off + 16u) w[(jb - off) >> 2] = r << (8 * ((jb - off) & 3u) + sub);
        if (owner) {
            *reinterpret_cast<uint4 *>(row + off) = make_uint4(w[0], w[1], w[2], w[3]);
#pragma unroll
            for (int k = 0; k < 4; ++k) e.template add_dword<C::BITS>(w[k], C::TOP);
        }
    }
    e.wave_reduce();
    const EstPart tot = node_total<C>(e, slice);
    if (slice == 0 && lane == 0) {
        c_prev[v] = estimate<P>(tot);
        sum_d[v] = 0.0;
    }
}

// Node and counter slice of this wave.  Single-wave shapes run blockDim / 64
// nodes per workgroup (1, 2 or 4, chosen at launch).
template <class C>
__device__ __forceinline__ void node_of(uint32_t blk, uint32_t &v, uint32_t &slice) {
    // the wave index is the same in all lanes; readfirstlane tells the compiler
    // so, which keeps v, the row bounds and every loop over the row scalar
    const uint32_t wave = (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    v = (C::WAVES == 1) ? blk * (blockDim.x / kWave) + wave : blk;
    slice = (C::WAVES == 1) ? 0u : wave;
}

template <class C>
__global__ __launch_bounds__(C::THREADS) void init_kernel(uint8_t *__restrict__ cur,
                                                          double *__restrict__ c_prev,
                                                          double *__restrict__ sum_d, uint32_t n,
                                                          uint64_t seed,
                                                          const uint32_t *__restrict__ hash_ids) {
    uint32_t v, slice;
    node_of<C>(xcd_block(blockIdx.x, gridDim.x), v, slice);
    if (v >= n) return;  // uniform per workgroup when WAVES > 1
    init_node<C>(cur, c_prev, sum_d, v, slice, seed, hash_ids);
}

// ---------------------------------------------------------------- row decoding
// Wave-cooperative LEB128 decoder of one CSR row, 64 bytes per call.  The
// carried state (wave-uniform) is the running id (the prefix sum of the first
// id and the deltas) and the bits of a varint that straddles two chunks.
struct RowDecoder {
    uint32_t run = 0;        // last absolute id decoded
    uint32_t carry_val = 0;  // low bits of a varint continued from the previous chunk
    uint32_t carry_sh = 0;   // bit position where the carried varint continues

    // Decode bytes[base, min(base + 64, end)).  Returns the decoded ids packed
    // into lanes 0..cnt-1 in increasing order (other lanes: unspecified).
    __device__ __forceinline__ uint32_t chunk(const uint8_t *__restrict__ bytes, uint64_t base,
                                              uint64_t end, uint32_t &cnt) {
        const bool valid = base + lane_id() < end;
        const uint32_t b = valid ? (uint32_t)bytes[base + lane_id()] : 0u;
        return chunk_of(b, valid, ballot(valid && !(b & 0x80u)), ballot(valid && (b & 0x80u)),
                        cnt);
    }

    // The same from this lane's byte b (0 when !valid) and the chunk's
    // terminator and continuation ballots.
    __device__ __forceinline__ uint32_t chunk_of(uint32_t b, bool valid, uint64_t term,
                                                 uint64_t cont, uint32_t &cnt) {
        (void)valid;
        const uint32_t lane = lane_id();
        const uint64_t lt_mask = (1ull << lane) - 1ull;
        const uint64_t below = term & lt_mask;
        const uint32_t start = below ? 64u - (uint32_t)__builtin_clzll(below) : 0u;
        const uint32_t pos = lane - start;
        const uint32_t sh = (below ? 0u : carry_sh) + 7u * pos;
        const uint32_t contrib = (sh < 32u) ? ((b & 0x7Fu) << sh) : 0u;
        uint32_t val = contrib;
        uint32_t x = contrib;
#pragma unroll
        for (uint32_t k = 1; k <= 4; ++k) {
            x = wave_shr1(x);  // contrib of lane - k
            if (pos >= k) val |= x;
        }
        if (!below) val |= carry_val;
        const bool is_term = (term >> lane) & 1ull;
        // inclusive prefix sum of the terminated values: first id, then deltas
        const uint32_t sum = wave_scan(is_term ? val : 0u);
        const uint32_t id = run + sum;
        run = readlane(id, kWave - 1);
        if ((cont >> (kWave - 1)) & 1ull) {
            carry_val = readlane(val, kWave - 1);
            carry_sh = readlane(sh, kWave - 1) + 7u;
        } else {
            carry_val = 0u;
            carry_sh = 0u;
        }
        // pack: terminator of rank r goes to lane r; non-terminators park on
        // lane 63, which is free whenever some lane is not a terminator
        cnt = (uint32_t)__builtin_popcountll(term);
        const uint32_t rank = (uint32_t)__builtin_popcountll(below);
        return (uint32_t)__builtin_amdgcn_ds_permute(
            (int)((is_term ? rank : (uint32_t)(kWave - 1)) << 2), (int)id);
    }
};

// ---------------------------------------------------------------- accumulator
// This lane's share of one node's running register-wise max.
template <class C>
struct NodeAcc {
    typename AccOf<C::BITS>::T m[C::RPL][4];

    __device__ __forceinline__ void init(const uint8_t *row, uint32_t slice, uint32_t lane) {
#pragma unroll
        for (int s = 0; s < C::RPL; ++s) {
            const uint4 x = *reinterpret_cast<const uint4 *>(row + slot_offset<C>(slice, lane, s));
            m[s][0].init(x.x);
            m[s][1].init(x.y);
            m[s][2].init(x.z);
            m[s][3].init(x.w);
        }
    }

    // max with the counter rows at src[u] (this lane's slots), N rows
    template <int N>
    __device__ __forceinline__ void gather(const uint8_t *const (&src)[N], uint32_t slice,
                                           uint32_t lane) {
        uint4 x[N][C::RPL];
#pragma unroll
        for (int u = 0; u < N; ++u)
#pragma unroll
            for (int s = 0; s < C::RPL; ++s)
                x[u][s] = *reinterpret_cast<const uint4 *>(src[u] + slot_offset<C>(slice, lane, s));
        // rows in pairs: a three-input max takes two rows per op
#pragma unroll
        for (int u = 0; u + 1 < N; u += 2)
#pragma unroll
            for (int s = 0; s < C::RPL; ++s) {
                m[s][0].add2(x[u][s].x, x[u + 1][s].x);
                m[s][1].add2(x[u][s].y, x[u + 1][s].y);
                m[s][2].add2(x[u][s].z, x[u + 1][s].z);
                m[s][3].add2(x[u][s].w, x[u + 1][s].w);
            }
        if (N % 2)
#pragma unroll
            for (int s = 0; s < C::RPL; ++s) {
                m[s][0].add(x[N - 1][s].x);
                m[s][1].add(x[N - 1][s].y);
                m[s][2].add(x[N - 1][s].z);
                m[s][3].add(x[N - 1][s].w);
            }
    }
};

// Final registers of node v: reduce the neighbour groups, store next[v],
// estimate it, apply Eq. 3 and the 0.5 test.
template <class C>
__device__ __forceinline__ void finish_node(NodeAcc<C> &acc, uint32_t v, uint32_t slice,
                                            uint8_t *__restrict__ next,
                                            double *__restrict__ c_prev,
                                            double *__restrict__ sum_d,
                                            uint32_t *__restrict__ flag_t, uint32_t t,
                                            double thr) {
    constexpr int P = C::PREC;
    const uint32_t lane = lane_id();
    const uint32_t grp = lane / C::LPC;
    uint32_t reg[C::RPL][4];
#pragma unroll
    for (int s = 0; s < C::RPL; ++s)
#pragma unroll
        for (int k = 0; k < 4; ++k) reg[s][k] = acc.m[s][k].value();
    if (C::G > 1) {
        // max across the groups that gathered different neighbours
#pragma unroll
        for (uint32_t mask = C::LPC; mask < kWave; mask <<= 1)
#pragma unroll
            for (int s = 0; s < C::RPL; ++s)
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    typename AccOf<C::BITS>::T mm;
                    mm.init(reg[s][k]);
                    mm.add(shfl_xor(reg[s][k], mask));
                    reg[s][k] = mm.value();
                }
    }
    EstPart e;
    e.clear();
    if (grp == 0) {
        uint8_t *row = next + (uint64_t)v * C::M;
#pragma unroll
        for (int s = 0; s < C::RPL; ++s) {
            *reinterpret_cast<uint4 *>(row + slot_offset<C>(slice, lane, s)) =
                make_uint4(reg[s][0], reg[s][1], reg[s][2], reg[s][3]);
#pragma unroll
            for (int k = 0; k < 4; ++k) e.template add_dword<C::BITS>(reg[s][k], C::TOP);
        }
    }
    e.wave_reduce();
    const EstPart tot = node_total<C>(e, slice);
    if (slice == 0 && lane == 0) {
        const double est = estimate<P>(tot);
        const double delta = est - c_prev[v];
        sum_d[v] = sum_d[v] + (double)t * delta;
        c_prev[v] = est;
        if (delta > thr &&
            __hip_atomic_load(flag_t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u)
            __hip_atomic_store(flag_t, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// ---------------------------------------------------------------- union step, per edge
// Eq. 2 as written: every neighbour's counter is gathered once per node.
template <class C>
__device__ __forceinline__ void union_node_edges(const uint8_t *__restrict__ bytes,
                                                 const uint64_t *__restrict__ offsets,
                                                 const uint8_t *__restrict__ cur,
                                                 uint8_t *__restrict__ next,
                                                 double *__restrict__ c_prev,
                                                 double *__restrict__ sum_d,
                                                 uint32_t *__restrict__ flag_t, uint32_t v,
                                                 uint32_t slice, uint32_t t, double thr) {
    const uint32_t lane = lane_id();
    const uint32_t grp = lane / C::LPC;
    NodeAcc<C> acc;  // Alg. 1: next[v] <- cur[v]
    acc.init(cur + (uint64_t)v * C::M, slice, lane);
    const uint64_t row_end = offsets[v + 1];
    RowDecoder dec;
    for (uint64_t base = offsets[v]; base < row_end; base += kWave) {
        uint32_t cnt;
        const uint32_t ids = dec.chunk(bytes, base, row_end, cnt);
        // gather-max over the cnt neighbours of this chunk; tail slots repeat
        // the batch's first id (max is idempotent)
        for (uint32_t k = 0; k < cnt; k += C::U * C::G) {
            const uint8_t *src[C::U];
#pragma unroll
            for (int u = 0; u < C::U; ++u) {
                if (C::G == 1) {
                    const uint32_t l = (k + u < cnt) ? k + u : k;
                    src[u] = cur + (uint64_t)readlane(ids, l) * C::M;
                } else {
                    const uint32_t idx = k + (uint32_t)u * C::G + grp;
                    src[u] = cur + (uint64_t)shfl_idx(ids, idx < cnt ? idx : k) * C::M;
                }
            }
            acc.gather(src, slice, lane);
        }
    }
    finish_node<C>(acc, v, slice, next, c_prev, sum_d, flag_t, t, thr);
}

template <class C>
__global__ __launch_bounds__(C::THREADS) void union_kernel(
    const uint8_t *__restrict__ bytes, const uint64_t *__restrict__ offsets,
    const uint8_t *__restrict__ cur, uint8_t *__restrict__ next, double *__restrict__ c_prev,
    double *__restrict__ sum_d, uint32_t *__restrict__ flag_t, uint32_t n, uint32_t t,
    const uint32_t *__restrict__ order, double thr, const uint32_t *__restrict__ skip) {
    if (skip && *skip == 0u) return;  // the previous step stopped the run
    uint32_t v, slice;
    node_of<C>(xcd_block(blockIdx.x, gridDim.x), v, slice);
    if (v >= n) return;  // uniform per workgroup when WAVES > 1
    if (order) v = order[v];
    union_node_edges<C>(bytes, offsets, cur, next, c_prev, sum_d, flag_t, v, slice, t, thr);
}

// ---------------------------------------------------------------- union step, per run
// In raster order most of a node's neighbours come in runs of consecutive ids
// (cells of one street segment in one raster row).  The max over a run [a, b]
// equals the max of two rows of a range-max table built from cur for this step:
// level k, row i holds max(cur[i .. i + 2^k)), so with k = floor(log2(b-a+1))
// the run is max(T[k][a], T[k][b - 2^k + 1]) -- the two blocks overlap, which
// max tolerates.  Runs longer than 2^K are covered by several level-K blocks.
// Node v itself may sit inside a run (it is no neighbour of itself, but its own
// counter is in the union anyway), so runs are joined across v.  The table is
// laid out level-major right after the counters, T[k][i] at tbl + (k n + i) m,
// and level 0 is cur itself.  The result is the same registers as the
// per-edge kernel.
//
// The runs come from a run list that the loader decodes once from the LEB128
// rows (row_runs_kernel); decoding the rows in every step, as the per-edge
// kernel does, cost more issue slots than the gathers themselves.
constexpr uint32_t kQueueCap = 384;        // table rows queued per wave (LDS)
static_assert(kQueueCap % 4 == 0, "the flush reads the queue 16 bytes at a time");
constexpr int kRunLoads = 4;               // 16 B/lane loads in flight per flush round
constexpr uint32_t kQueueFlush = kQueueCap - 2 * kWave;

template <class C>
struct RunGather {
    const uint8_t *tbl;
    uint32_t n, levels;
    uint32_t *q;   // this wave's LDS queue of table-row indices (k n + i)
    uint32_t qn;   // entries queued (wave-uniform)

    uint32_t slice;  // this wave's counter slice

    __device__ __forceinline__ void flush(NodeAcc<C> &acc, uint32_t lane) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const uint32_t grp = lane / C::LPC;
        // fewer loads in flight than the per-edge kernel: this kernel runs at
        // six waves per SIMD, where the registers of eight would spill
        constexpr int U = C::RPL >= kRunLoads ? 1 : kRunLoads / C::RPL;
        // qn is wave-uniform; saying so keeps the loop control and the index
        // clamp on the scalar unit
        const uint32_t cnt = C::G == 1 ? (uint32_t)__builtin_amdgcn_readfirstlane((int)qn) : qn;
        for (uint32_t k = 0; k < cnt; k += U * C::G) {
            const uint8_t *src[U];
            if constexpr (C::G == 1 && U == 4) {
                // the four entries in one 16-byte LDS read (k is a multiple of
                // 4 and the queue is 16-byte aligned); entries at cnt and past
                // it are stale, so they repeat entry k
                const uint4 r = *reinterpret_cast<const uint4 *>(q + k);
                const uint32_t e[4] = {r.x, r.y, r.z, r.w};
                const uint32_t r0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)e[0]);
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const uint32_t ru =
                        u == 0 ? r0 : (uint32_t)__builtin_amdgcn_readfirstlane((int)e[u]);
                    src[u] = tbl + (uint64_t)(k + (uint32_t)u < cnt ? ru : r0) * C::M;
                }
            } else {
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const uint32_t idx =
                        k + (uint32_t)u * (uint32_t)C::G + (C::G == 1 ? 0u : grp);
                    uint32_t row = q[idx < cnt ? idx : k];
                    if (C::G == 1) row = (uint32_t)__builtin_amdgcn_readfirstlane((int)row);
                    src[u] = tbl + (uint64_t)row * C::M;
                }
            }
            acc.gather(src, slice, lane);
        }
        __builtin_amdgcn_wave_barrier();
        qn = 0;
    }

    // queue the table rows covering run [a, b] (wave-uniform a, b)
    __device__ __forceinline__ void push_run(NodeAcc<C> &acc, uint32_t a, uint32_t b,
                                             uint32_t lane) {
        const uint32_t r = b - a + 1u;
        const uint32_t top = 1u << levels;
        if (r <= top) {
            const uint32_t k = 31u - (uint32_t)__builtin_clz(r);
            if (qn + 2u > kQueueCap) flush(acc, lane);
            if (lane == 0) {
                q[qn] = k * n + a;
                q[qn + 1] = k * n + (b - (1u << k) + 1u);
            }
            qn += (r == (1u << k)) ? 1u : 2u;
            return;
        }
        for (uint32_t j = a;; j += top) {
            const uint32_t i = (j + top - 1u < b) ? j : b - top + 1u;
            if (qn + 1u > kQueueCap) flush(acc, lane);
            if (lane == 0) q[qn] = levels * n + i;
            qn += 1u;
            if (i != j) break;
            if (j + top - 1u == b) break;
        }
    }
};

// Node v's step from its run list: runs[run_off[v] ..] are the maximal runs of
// its row with v itself joined in (a run that stops at v - 1 and one that
// starts at v + 1 form one run, since v's own counter is in the union anyway).
// Each lane takes one run: its table level and one or two rows go to the
// queue at offsets from a wave prefix sum.
template <class C>
__device__ __forceinline__ void union_node_runs(const uint2 *__restrict__ runs,
                                                const uint64_t *__restrict__ run_off,
                                                const uint8_t *__restrict__ tbl, uint32_t levels,
                                                uint8_t *__restrict__ next,
                                                double *__restrict__ c_prev,
                                                double *__restrict__ sum_d,
                                                uint32_t *__restrict__ flag_t, uint32_t n,
                                                uint32_t v, uint32_t slice, uint32_t t,
                                                double thr, uint32_t *queue) {
    const uint32_t lane = lane_id();
    NodeAcc<C> acc;  // Alg. 1: next[v] <- cur[v] (level 0 of the table is cur)
    acc.init(tbl + (uint64_t)v * C::M, slice, lane);
    RunGather<C> g{tbl, n, levels, queue, 0u, slice};
    const uint32_t top = 1u << levels;
    const uint64_t re = run_off[v + 1];
    uint64_t base = run_off[v];
    // each chunk's runs are loaded one chunk ahead
    uint2 x_next = base + lane < re ? runs[base + lane] : make_uint2(1u, 0u);
    for (; base < re; base += kWave) {
        const uint64_t left = re - base;
        const uint2 x = x_next;
        if (left > kWave)
            x_next = lane < left - kWave ? runs[base + kWave + lane] : make_uint2(1u, 0u);
        const bool in = (left >= kWave ? ~0ull : (1ull << left) - 1ull) >> lane & 1ull;
        const uint32_t r = x.y - x.x + 1u;  // run length (0 past the list's end)
        const bool longrun = in && r > top;
        const uint32_t k = 31u - (uint32_t)__builtin_clz(r | 1u);
        const uint32_t nl = (in && !longrun) ? ((r == (1u << k)) ? 1u : 2u) : 0u;
        const uint32_t pos = wave_scan(nl);  // inclusive prefix sum of the rows per lane
        const uint32_t total = readlane(pos, kWave - 1);
        if (g.qn > kQueueFlush) g.flush(acc, lane);
        if (nl) {
            const uint32_t at = g.qn + pos - nl;
            g.q[at] = k * n + x.x;
            if (nl == 2u) g.q[at + 1] = k * n + (x.y - (1u << k) + 1u);
        }
        g.qn += total;
        uint64_t lm = ballot(longrun);
        while (lm) {
            const uint32_t l = (uint32_t)__builtin_ctzll(lm);
            lm &= lm - 1ull;
            g.push_run(acc, readlane(x.x, l), readlane(x.y, l), lane);
        }
    }
    if (g.qn) g.flush(acc, lane);
    finish_node<C>(acc, v, slice, next, c_prev, sum_d, flag_t, t, thr);
}

// Six waves per SIMD (80 VGPRs): the run kernel hides its gather latency with
// occupancy rather than with loads in flight.  Measured per city step at p = 10:
// 39.4 ms at the four waves its natural register count allows, 33.5 ms at five,
// 32.1 ms at six with four loads in flight; eight waves spill heavily (75 ms).
// At p = 11 five waves beat four (58.0 against 60.2 ms); at p = 12 three waves
// without spills match four with them (117.4 against 118.0 ms).
// With several waves per node every wave reads the run list and queues the same
// table rows, then gathers its own slice of each.
//
// order (optional) is the processing order: logical node i is node order[i].
// Nodes that are processed together (the XCDs walk one stretch of the order
// side by side) gather overlapping table rows, so an order along a
// space-filling curve over the raster raises cache reuse; the results do not
// depend on it.
template <class C>
__global__ __launch_bounds__(C::THREADS, C::RUN_OCC) void union_runs_kernel(
    const uint2 *__restrict__ runs, const uint64_t *__restrict__ run_off,
    const uint8_t *__restrict__ tbl, uint32_t levels, uint8_t *__restrict__ next,
    double *__restrict__ c_prev, double *__restrict__ sum_d, uint32_t *__restrict__ flag_t,
    uint32_t n, uint32_t t, const uint32_t *__restrict__ order, double thr,
    const uint32_t *__restrict__ skip) {
    __shared__ __attribute__((aligned(16))) uint32_t s_queue[C::THREADS / kWave][kQueueCap];
    if (skip && *skip == 0u) return;  // the previous step stopped the run
    uint32_t v, slice;
    node_of<C>(xcd_span_block(blockIdx.x, gridDim.x, kXcdSpanChunk), v, slice);
    if (v >= n) return;  // uniform per workgroup when WAVES > 1
    if (order) v = order[v];
    union_node_runs<C>(runs, run_off, tbl, levels, next, c_prev, sum_d, flag_t, n, v, slice, t,
                       thr, s_queue[threadIdx.x / kWave]);
}

// ---------------------------------------------------------------- union step, per group
// Nodes that are processed together see almost the same cells, so their run
// lists hold many identical table rows.  The loader merges the rows of every
// group of kGroupNodes consecutive nodes of the processing order into one list
// of distinct rows, each with a bit mask of the group's nodes that need it
// (their own counters included), rows of one mask next to each other.
// group_waves(p, bits) waves handle a group, each on its own 512-byte slice of
// the counters (p = 10: two waves for 8-bit registers, one for 4-bit; p = 12,
// 8-bit: eight, in a workgroup of their own; a 256-byte counter: one wave, 4
// bytes per lane).  A wave loads every
// listed row's slice once and takes the max of the rows of one mask into a
// running value; when the mask changes, that value goes into the accumulators
// of the nodes in the mask, which sit in LDS, so that the per-node work is paid
// once per distinct mask, not once per row.
// Workgroup size for a counter of M bytes: four waves, or one group's waves
// when a group has more.
constexpr uint32_t group_block(uint32_t m) {
    return (m / kGroupSlice) * kWave > 256u ? (m / kGroupSlice) * kWave : 256u;
}
constexpr int kGroupLoads = 16;  // rows in flight per wave (one batch)

// This lane's part of one counter slice: kDw dwords (two of a 512-byte slice,
// one of a 256-byte counter).
template <uint32_t kDw> struct LaneSlice;
template <> struct LaneSlice<2> {
    uint32_t d[2];
    __device__ __forceinline__ void load(const uint8_t *p) {
        const uint2 x = *reinterpret_cast<const uint2 *>(p);
        d[0] = x.x;
        d[1] = x.y;
    }
    __device__ __forceinline__ void store(uint8_t *p) const {
        *reinterpret_cast<uint2 *>(p) = make_uint2(d[0], d[1]);
    }
};
template <> struct LaneSlice<1> {
    uint32_t d[1];
    __device__ __forceinline__ void load(const uint8_t *p) {
        d[0] = *reinterpret_cast<const uint32_t *>(p);
    }
    __device__ __forceinline__ void store(uint8_t *p) const {
        *reinterpret_cast<uint32_t *>(p) = d[0];
    }
};

// Register-wise max of the raw registers a (one dword) and the running value r.
// 8-bit: the high bytes of both 16-bit halves from one packed max, the low
// bytes (shifted up) from another, and a byte permute puts them back in place.
__device__ __forceinline__ uint32_t max_into_raw(uint32_t a, const Max4 &r) {
    const uint32_t hi = pk_max_u16(a, r.hi);
    const uint32_t lo = pk_max_u16(a << 8, r.lo);
    // bytes 0..3 of the result: lo.1, hi.1, lo.3, hi.3 (selector bytes 0-3 pick
    // from the second operand, 4-7 from the first)
    return __builtin_amdgcn_perm(hi, lo, 0x07030501u);
}
// 4-bit: the four nibble positions of each half through the accumulator's
// four shifted copies.
__device__ __forceinline__ uint32_t max_into_raw(uint32_t a, const Max8 &r) {
    Max8 b;
    b.init(a);
#pragma unroll
    for (int i = 0; i < 4; ++i) b.a[i] = pk_max_u16(b.a[i], r.a[i]);
    return b.value();
}

// One workgroup of the grouped step: logical block lb holds groups
// lb * (groups per workgroup) ..; every wave of the workgroup calls it.
template <class C>
__device__ __forceinline__ void groups_step(
    const uint32_t *__restrict__ grp_rows, const GroupMask *__restrict__ grp_mask,
    const uint64_t *__restrict__ grp_off, const uint8_t *__restrict__ tbl,
    uint8_t *__restrict__ next, double *__restrict__ c_prev, double *__restrict__ sum_d,
    uint32_t *__restrict__ flag_t, uint32_t n, uint32_t t, const uint32_t *__restrict__ order,
    double thr, uint32_t lb) {
    constexpr uint32_t W = kGroupNodes, H = group_waves(C::PREC, C::BITS);
    constexpr uint32_t kSlice = (uint32_t)C::M / H;  // counter bytes per wave
    static_assert((kSlice == kGroupSlice || (H == 1 && kSlice == kGroupSlice / 2)) && H >= 1,
                  "512-byte slices, or one 256-byte counter");
    constexpr uint32_t kDw = kSlice / kWave / 4u;    // dwords per lane
    static_assert(kDw == 1 || kDw == 2, "4 or 8 bytes per lane");
    constexpr int U = kGroupLoads;  // rows per batch
    static_assert(U * kDw <= 32, "at most 32 VGPRs of loads per batch");
    static_assert(kWave % U == 0, "a batch lies in one chunk of 64 entries");
    constexpr uint32_t kWavesPerBlock = group_block(C::M) / kWave;
    constexpr uint32_t kGroupsPerBlock = kWavesPerBlock / H;
    using Slice = LaneSlice<kDw>;
    __shared__ Slice s_acc[kWavesPerBlock][W][kWave];
    __shared__ uint64_t s_lo[kWavesPerBlock][W];
    __shared__ uint64_t s_hi[kWavesPerBlock][W];
    __shared__ uint32_t s_z[kWavesPerBlock][W];
    const uint32_t wave = (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    const uint32_t grp = lb * kGroupsPerBlock + wave / H;
    const uint32_t part = wave % H;
    const uint32_t n_groups = (n + W - 1u) / W;
    const bool active = grp < n_groups;  // every wave reaches the barrier below
    const uint32_t lane = lane_id();
    const uint32_t off = part * kSlice + lane * (kDw * 4u);
    Slice(*acc)[kWave] = s_acc[wave];  // this wave's accumulators, each lane its own
#pragma unroll
    for (uint32_t w = 0; w < W; ++w)
#pragma unroll
        for (uint32_t k = 0; k < kDw; ++k) acc[w][lane].d[k] = 0u;
    if (active) {
        const uint64_t end = grp_off[grp + 1];
        typename AccOf<C::BITS>::T run[kDw];
#pragma unroll
        for (uint32_t k = 0; k < kDw; ++k) run[k].init(0u);
        uint32_t run_mask = 0u;
        // the running value into the accumulators of the nodes in its mask
        const auto merge = [&](uint32_t mask) {
#pragma unroll 1
            while (mask) {
                const uint32_t w = (uint32_t)__builtin_ctz(mask);
                mask &= mask - 1u;
                Slice a = acc[w][lane];
#pragma unroll
                for (uint32_t k = 0; k < kDw; ++k) a.d[k] = max_into_raw(a.d[k], run[k]);
                acc[w][lane] = a;
            }
        };
        const auto process = [&](const Slice(&x)[U], const uint32_t(&mk)[U]) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (mk[u] == 0u) break;
                if (mk[u] != run_mask) {
                    merge(run_mask);
                    run_mask = mk[u];
#pragma unroll
                    for (uint32_t k = 0; k < kDw; ++k) run[k].init(x[u].d[k]);
                } else {
#pragma unroll
                    for (uint32_t k = 0; k < kDw; ++k) run[k].add(x[u].d[k]);
                }
            }
        };
        // list entries 64 at a time, one per lane, broadcast with readlane; a
        // batch of U rows in flight at a time (issuing the next batch before
        // processing this one was slower: 10.0 against 9.0 ms per city launch)
#pragma unroll 1
        for (uint64_t base = grp_off[grp]; base < end; base += kWave) {
            const uint32_t cnt = (uint32_t)((end - base < kWave) ? end - base : kWave);
            const uint32_t e_row = lane < cnt ? grp_rows[base + lane] : 0u;
            const uint32_t e_mask = lane < cnt ? (uint32_t)grp_mask[base + lane] : 0u;
#pragma unroll 1
            for (uint32_t j = 0; j < cnt; j += (uint32_t)U) {
                Slice x[U];
                uint32_t mk[U];  // the batch's masks; 0 past the list's end
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    // past the end: row j again (not used)
                    const uint32_t l = j + (uint32_t)u < cnt ? j + (uint32_t)u : j;
                    x[u].load(tbl + (uint64_t)readlane(e_row, l) * C::M + off);
                    mk[u] = j + (uint32_t)u < cnt ? readlane(e_mask, l) : 0u;
                }
                process(x, mk);
            }
        }
        merge(run_mask);
    }
    // registers of every node: store this wave's slice, estimator partials to LDS
#pragma unroll 1
    for (uint32_t w = 0; w < W; ++w) {
        const uint32_t i = grp * W + w;
        if (!active || i >= n) break;
        const uint32_t v = order ? order[i] : i;
        const Slice r = acc[w][lane];
        r.store(next + (uint64_t)v * C::M + off);
        EstPart e;
        e.clear();
#pragma unroll
        for (uint32_t k = 0; k < kDw; ++k) e.template add_dword<C::BITS>(r.d[k], C::TOP);
        e.wave_reduce();
        if (lane == 0) {
            s_lo[wave][w] = e.lo;
            s_hi[wave][w] = e.hi;
            s_z[wave][w] = e.zeros;
        }
    }
    __syncthreads();
    // lane w of the group's first wave: node w's estimate, Eq. 3 and the stop test
    const uint32_t i = grp * W + lane;
    if (active && part == 0u && lane < W && i < n) {
        EstPart tot;
        tot.clear();
#pragma unroll
        for (uint32_t h = 0; h < H; ++h) {
            EstPart o;
            o.lo = s_lo[wave + h][lane];
            o.hi = s_hi[wave + h][lane];
            o.zeros = s_z[wave + h][lane];
            tot.add(o);
        }
        const uint32_t v = order ? order[i] : i;
        const double est = estimate<C::PREC>(tot);
        const double delta = est - c_prev[v];
        sum_d[v] = sum_d[v] + (double)t * delta;
        c_prev[v] = est;
        if (delta > thr &&
            __hip_atomic_load(flag_t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u)
            __hip_atomic_store(flag_t, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

template <class C>
__global__ __launch_bounds__(group_block(C::M)) void union_groups_kernel(
    const uint32_t *__restrict__ grp_rows, const GroupMask *__restrict__ grp_mask,
    const uint64_t *__restrict__ grp_off, const uint8_t *__restrict__ tbl,
    uint8_t *__restrict__ next, double *__restrict__ c_prev, double *__restrict__ sum_d,
    uint32_t *__restrict__ flag_t, uint32_t n, uint32_t t, const uint32_t *__restrict__ order,
    double thr, const uint32_t *__restrict__ skip) {
    if (skip && *skip == 0u) return;  // the previous step stopped the run (whole launch)
    groups_step<C>(grp_rows, grp_mask, grp_off, tbl, next, c_prev, sum_d, flag_t, n, t, order,
                   thr, xcd_span_block(blockIdx.x, gridDim.x, kXcdSpanChunk));
}

// ---------------------------------------------------------------- gather ceiling
// The run kernel's gather loop without its queue or its run list: every node of
// the launch gathers `rows` counter rows of a small table (table_rows rows, a
// power of two, sized to stay in the L2 caches), picked by a hash of (node,
// row), in the run kernel's shape and with as many rows in flight, and either
// takes the byte-wise max (with_max = 1) or only xors the loaded words (the load
// path alone).  Rows gathered per second is the rate the run kernel's gathers
// can reach when every row hits in L2.
__device__ __forceinline__ uint32_t probe_hash(uint32_t x) {
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

template <class C>
__global__ __launch_bounds__(C::THREADS, C::RUN_OCC) void gather_probe_kernel(
    const uint8_t *__restrict__ tbl, uint32_t row_mask, uint32_t rows, uint32_t *__restrict__ out,
    uint32_t n, uint32_t with_max) {
    uint32_t v, slice;
    node_of<C>(xcd_block(blockIdx.x, gridDim.x), v, slice);
    if (v >= n) return;
    const uint32_t lane = lane_id();
    const uint32_t grp = lane / C::LPC;
    constexpr int U = C::RPL >= kRunLoads ? 1 : kRunLoads / C::RPL;
    const uint32_t seed = probe_hash(v * 0x9e3779b9u + slice);
    uint32_t sink = 0;
    NodeAcc<C> acc;
    acc.init(tbl + (uint64_t)(v & row_mask) * C::M, slice, lane);
    for (uint32_t k = 0; k < rows; k += U * C::G) {
        const uint8_t *src[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            uint32_t r = probe_hash(seed ^ (k + (uint32_t)u * C::G + (C::G == 1 ? 0u : grp)));
            if (C::G == 1) r = (uint32_t)__builtin_amdgcn_readfirstlane((int)r);
            src[u] = tbl + (uint64_t)(r & row_mask) * C::M;
        }
        if (with_max) {
            acc.gather(src, slice, lane);
        } else {
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int s2 = 0; s2 < C::RPL; ++s2) {
                    const uint4 x =
                        *reinterpret_cast<const uint4 *>(src[u] + slot_offset<C>(slice, lane, s2));
                    sink ^= x.x ^ x.y ^ x.z ^ x.w;
                }
        }
    }
#pragma unroll
    for (int s2 = 0; s2 < C::RPL; ++s2)
#pragma unroll
        for (int q = 0; q < 4; ++q) sink ^= acc.m[s2][q].value();
    out[(uint64_t)v * C::WAVES * kWave + slice * kWave + lane] = sink;
}

// Register-wise max of 16 bytes of two counters (8- or 4-bit registers).
template <class A>
__device__ __forceinline__ uint4 max16(const uint4 a, const uint4 b) {
    A x, y, z, w;
    x.init(a.x);
    x.add(b.x);
    y.init(a.y);
    y.add(b.y);
    z.init(a.z);
    z.add(b.z);
    w.init(a.w);
    w.add(b.w);
    return make_uint4(x.value(), y.value(), z.value(), w.value());
}

// Level k of the range-max table from level k - 1:
// T[k][i] = max(T[k-1][i], T[k-1][i + 2^(k-1)]) for i <= n - 2^k.
__global__ __launch_bounds__(256) void table_level_kernel(uint8_t *__restrict__ tbl,
                                                          uint64_t level_bytes, uint32_t k,
                                                          uint64_t count16, uint64_t half16,
                                                          uint32_t bits,
                                                          const uint32_t *__restrict__ skip) {
    if (skip && *skip == 0u) return;  // the previous step stopped the run
    const uint4 *prev = reinterpret_cast<const uint4 *>(tbl + (uint64_t)(k - 1) * level_bytes);
    uint4 *out = reinterpret_cast<uint4 *>(tbl + (uint64_t)k * level_bytes);
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count16; i += stride) {
        const uint4 a = prev[i], b = prev[i + half16];
        out[i] = bits == 4u ? max16<Max8>(a, b) : max16<Max4>(a, b);
    }
}

// All levels 1..levels (<= kFusedLevels) of the table in one launch.  A
// workgroup holds rows i0 .. i0 + kTblRows + 2^levels - 2 of a column slice of
// kTblCols x 16 bytes of cur in LDS (the output rows plus the span the largest
// block reaches past them), builds each level in place from the one before,
// and writes the level's rows i0 .. i0 + kTblRows - 1 that exist
// (i <= n - 2^k).  Level 0 is read about 1.5 times instead of twice per level,
// and no level is read back.  Two tile shapes: 512 rows of 64 bytes, or, for
// 8-bit counters of at least 1 KB, 256 rows of 128 bytes (whole 128-byte lines
// written; city graph, p = 10: 0.60 against 0.66 ms per step, while 4-bit
// counters of 512 bytes were slower with it).
constexpr uint32_t kFusedLevels = 8;

template <uint32_t kTblRows, uint32_t kTblCols>
__global__ __launch_bounds__(256) void table_fused_kernel(uint8_t *__restrict__ tbl, uint32_t n,
                                                          uint32_t m, uint32_t levels,
                                                          uint32_t bits,
                                                          const uint32_t *__restrict__ skip) {
    constexpr uint32_t kTblSpan = kTblRows + (1u << kFusedLevels) - 1u;
    constexpr uint32_t kTblPer = (kTblSpan * kTblCols + 255u) / 256u;  // LDS chunks per thread
    __shared__ uint4 lds[kTblSpan * kTblCols];
    if (skip && *skip == 0u) return;  // the previous step stopped the run
    const uint32_t slices = m / (16u * kTblCols);
    const uint32_t tile = blockIdx.x / slices, slice = blockIdx.x % slices;
    const uint64_t i0 = (uint64_t)tile * kTblRows;
    const uint64_t col = (uint64_t)slice * kTblCols * 16u;
    const uint64_t level_bytes = (uint64_t)n * m;
    const uint32_t span = kTblRows + (1u << levels) - 1u;
    for (uint32_t c = threadIdx.x; c < span * kTblCols; c += blockDim.x) {
        const uint64_t i = i0 + c / kTblCols;
        if (i < n)
            lds[c] = *reinterpret_cast<const uint4 *>(tbl + i * m + col + (c % kTblCols) * 16u);
    }
    __syncthreads();
    for (uint32_t k = 1; k <= levels; ++k) {
        // level k is exact in LDS rows 0 .. span - 2^k (their blocks end inside the span)
        const uint32_t len = (span - (1u << k) + 1u) * kTblCols;
        const uint32_t half = (1u << (k - 1)) * kTblCols;
        uint4 val[kTblPer];
#pragma unroll
        for (uint32_t t = 0; t < kTblPer; ++t) {
            const uint32_t c = threadIdx.x + t * 256u;
            if (c < len) val[t] = bits == 4u ? max16<Max8>(lds[c], lds[c + half])
                                              : max16<Max4>(lds[c], lds[c + half]);
        }
        __syncthreads();
#pragma unroll
        for (uint32_t t = 0; t < kTblPer; ++t) {
            const uint32_t c = threadIdx.x + t * 256u;
            if (c < len) lds[c] = val[t];
        }
        __syncthreads();
        uint8_t *out = tbl + (uint64_t)k * level_bytes;
        for (uint32_t c = threadIdx.x; c < kTblRows * kTblCols; c += blockDim.x) {
            const uint64_t i = i0 + c / kTblCols;
            if (i + (1ull << k) <= n)
                *reinterpret_cast<uint4 *>(out + i * m + col + (c % kTblCols) * 16u) = lds[c];
        }
    }
}

// ---------------------------------------------------------------- batched steps
// Workgroup -> (job, node block): the largest i with block_base[i] <= blk.
__device__ __forceinline__ uint32_t find_job(const uint32_t *__restrict__ block_base,
                                             uint32_t nlist, uint32_t blk) {
    uint32_t lo = 0, hi = nlist;  // block_base[lo] <= blk < block_base[hi]
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (block_base[mid] <= blk) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Workgroups are dispatched in index order, so a job's contiguous block range
// runs on all XCDs together (its working set is shared, not eight jobs'); the
// XCD of block base + l is (base + l) mod 8, a fixed rotation of l mod 8, so
// remapping the local index gives each XCD one contiguous node range of the job.
__device__ __forceinline__ uint32_t job_block(uint32_t blk, const uint32_t *__restrict__ block_base,
                                              uint32_t i) {
    return xcd_block(blk - block_base[i], block_base[i + 1] - block_base[i]);
}

template <class C>
__global__ __launch_bounds__(C::THREADS) void batch_init_kernel(
    BatchJob *__restrict__ jobs, const uint32_t *__restrict__ list,
    const uint32_t *__restrict__ block_base, uint32_t nlist) {
    const uint32_t i = find_job(block_base, nlist, blockIdx.x);
    const BatchJob &J = jobs[list[i]];
    uint32_t v, slice;
    node_of<C>(job_block(blockIdx.x, block_base, i), v, slice);
    if (v >= J.n) return;  // uniform per workgroup when WAVES > 1
    init_node<C>(J.buf[0], J.c_prev, J.sum_d, v, slice, J.seed, J.hash_ids);
}

template <class C, bool RUNS>
__global__ __launch_bounds__(C::THREADS, RUNS ? C::RUN_OCC : 1) void batch_union_kernel(
    BatchJob *__restrict__ jobs, const uint32_t *__restrict__ list,
    const uint32_t *__restrict__ block_base, uint32_t nlist) {
    __shared__ __attribute__((aligned(16))) uint32_t
        s_queue[RUNS ? C::THREADS / kWave : 1][RUNS ? kQueueCap : 1];
    const uint32_t i = find_job(block_base, nlist, blockIdx.x);
    const BatchJob &J = jobs[list[i]];
    if (J.done) return;  // uniform per workgroup
    const uint32_t t = J.t + 1u;
    uint32_t v, slice;
    node_of<C>(job_block(blockIdx.x, block_base, i), v, slice);
    if (v >= J.n) return;  // uniform per workgroup when WAVES > 1
    if (J.order) v = J.order[v];
    const uint8_t *cur = J.buf[(t - 1u) & 1u];
    uint8_t *next = J.buf[t & 1u];
    if constexpr (RUNS) {
        union_node_runs<C>(J.run_list, J.run_off, cur, J.levels, next, J.c_prev, J.sum_d,
                           J.flags + t, J.n, v, slice, t, J.stop_delta,
                           s_queue[threadIdx.x / kWave]);
    } else {
        union_node_edges<C>(J.bytes, J.offsets, cur, next, J.c_prev, J.sum_d, J.flags + t, v,
                            slice, t, J.stop_delta);
    }
}

// The grouped step for listed jobs: job list[i]'s workgroups hold its groups,
// all XCDs on one stretch of its processing order as in a single run.
template <class C>
__global__ __launch_bounds__(group_block(C::M)) void batch_groups_kernel(
    BatchJob *__restrict__ jobs, const uint32_t *__restrict__ list,
    const uint32_t *__restrict__ block_base, uint32_t nlist) {
    const uint32_t i = find_job(block_base, nlist, blockIdx.x);
    const BatchJob &J = jobs[list[i]];
    if (J.done) return;  // uniform per workgroup
    const uint32_t t = J.t + 1u;
    const uint32_t lb = xcd_span_block(blockIdx.x - block_base[i],
                                       block_base[i + 1] - block_base[i], kXcdSpanChunk);
    groups_step<C>(J.grp_rows, J.grp_mask, J.grp_off, J.buf[(t - 1u) & 1u], J.buf[t & 1u],
                   J.c_prev, J.sum_d, J.flags + t, J.n, t, J.order, J.stop_delta, lb);
}

// Table level k for a list of jobs: workgroup blk handles 16-byte chunks
// [(blk - block_base[i]) * kTableChunk, ...) of job list[i]'s level k.
constexpr uint32_t kTableChunk = 256 * 4;  // chunks per workgroup (4 per thread)

__global__ __launch_bounds__(256) void batch_table_kernel(BatchJob *__restrict__ jobs,
                                                          const uint32_t *__restrict__ list,
                                                          const uint32_t *__restrict__ block_base,
                                                          uint32_t nlist, uint32_t k) {
    const uint32_t blk = blockIdx.x;
    const uint32_t i = find_job(block_base, nlist, blk);
    const BatchJob &J = jobs[list[i]];
    if (J.done || !J.runs || k > J.levels) return;
    const uint32_t t = J.t + 1u;
    uint8_t *tbl = J.buf[(t - 1u) & 1u];
    const uint64_t m16 = ((1ull << J.p) * J.bits / 8u) / 16u;  // 16-byte chunks per counter
    const uint64_t level16 = (uint64_t)J.n * m16;
    const uint64_t count16 = ((uint64_t)J.n - (1ull << k) + 1ull) * m16;
    const uint64_t half16 = (1ull << (k - 1u)) * m16;
    const uint4 *prev = reinterpret_cast<const uint4 *>(tbl) + (uint64_t)(k - 1u) * level16;
    uint4 *out = reinterpret_cast<uint4 *>(tbl) + (uint64_t)k * level16;
    const uint64_t c0 = (uint64_t)(blk - block_base[i]) * kTableChunk;
#pragma unroll
    for (uint32_t r = 0; r < kTableChunk / 256; ++r) {
        const uint64_t c = c0 + (uint64_t)r * 256u + threadIdx.x;
        if (c >= count16) break;
        const uint4 a = prev[c], b = prev[c + half16];
        out[c] = J.bits == 4u ? max16<Max8>(a, b) : max16<Max4>(a, b);
    }
}

__global__ void batch_step_end_kernel(BatchJob *__restrict__ jobs,
                                      const uint32_t *__restrict__ list, uint32_t nlist) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nlist) return;
    BatchJob &J = jobs[list[i]];
    if (J.done) return;
    const uint32_t t = J.t + 1u;
    J.t = t;
    // converged: step t grew no estimate by more than the threshold
    J.converged = J.flags[t] == 0u ? 1u : 0u;
    if ((J.converged && !J.depth_only) || (J.depth != 0u && t == J.depth) || t + 1u >= J.n_flags)
        J.done = t;
}

// Streaming copy, 16 B per lane, grid-stride: the reference kernel for
// achievable HBM bandwidth and for scaling the HBM byte counters.
__global__ __launch_bounds__(256) void copy_kernel(const uint4 *__restrict__ src,
                                                   uint4 *__restrict__ dst, uint64_t count) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride)
        dst[i] = src[i];
}

// ---------------------------------------------------------------- VGA metrics
// Sec. 3.3, "Metric derivation": connectivity and control from the 1-hop
// neighbourhood (exact), the other metrics in closed form from the Eq. 3 sum.
// One wave per node decodes its row; each lane adds 1 / deg(w) for the
// neighbours it holds, and a fixed butterfly sums the lanes.
__device__ __forceinline__ double shfl_xor_f64(double x, uint32_t mask) {
    const uint64_t b = __builtin_bit_cast(uint64_t, x);
    const uint32_t lo = shfl_xor((uint32_t)b, mask), hi = shfl_xor((uint32_t)(b >> 32), mask);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

__global__ __launch_bounds__(256) void vga_kernel(const uint8_t *__restrict__ bytes,
                                                  const uint64_t *__restrict__ offsets,
                                                  const uint32_t *__restrict__ degrees,
                                                  const uint32_t *__restrict__ comp_size,
                                                  const int32_t *__restrict__ xy,
                                                  const double *__restrict__ sum_d, uint32_t n,
                                                  double *__restrict__ out) {
    const uint32_t wave = (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    const uint32_t lane = lane_id();
    const uint32_t v = blockIdx.x * (blockDim.x / kWave) + wave;
    if (v >= n) return;
    double part = 0.0;
    uint64_t moment2 = 0;  // squared distances to the neighbours, exact
    int32_t vx = 0, vy = 0;
    if (xy) {
        vx = xy[2ull * v];
        vy = xy[2ull * v + 1];
    }
    uint32_t k = 0;
    RowDecoder dec;
    const uint64_t row_end = offsets[v + 1];
    for (uint64_t base = offsets[v]; base < row_end; base += kWave) {
        uint32_t cnt;
        const uint32_t ids = dec.chunk(bytes, base, row_end, cnt);
        if (lane < cnt) {
            part += 1.0 / (double)degrees[ids];
            if (xy) {
                const int64_t dx = (int64_t)xy[2ull * ids] - vx;
                const int64_t dy = (int64_t)xy[2ull * ids + 1] - vy;
                moment2 += (uint64_t)(dx * dx + dy * dy);
            }
        }
        k += cnt;
    }
#pragma unroll
    for (uint32_t mask = 1; mask < kWave; mask <<= 1) {
        part += shfl_xor_f64(part, mask);
        const uint32_t lo = shfl_xor((uint32_t)moment2, mask);
        const uint32_t hi = shfl_xor((uint32_t)(moment2 >> 32), mask);
        moment2 += ((uint64_t)hi << 32) | lo;
    }
    if (lane != 0) return;
    const double nan = __builtin_nan("");
    const double N = comp_size ? (double)comp_size[v] : (double)n;  // exact N_v
    const double md = N >= 2.0 ? sum_d[v] / (N - 1.0) : nan;
    const double ra = N >= 3.0 ? 2.0 * (md - 1.0) / (N - 2.0) : nan;
    // Hillier & Hanson's diamond value D_k (k = N_v) normalises RA to RRA
    const double dk = N >= 3.0 ? 2.0 * (N * (log2((N + 2.0) / 3.0) - 1.0) + 1.0) /
                                     ((N - 1.0) * (N - 2.0))
                               : nan;
    double *o = out + v;
    o[0 * (uint64_t)n] = (double)k;                             // connectivity
    o[1 * (uint64_t)n] = part;                                  // control
    o[2 * (uint64_t)n] = md;                                    // Visual Mean Depth
    o[3 * (uint64_t)n] = ra;                                    // relative asymmetry
    o[4 * (uint64_t)n] = dk / ra;                               // integration [HH] = 1 / RRA
    o[5 * (uint64_t)n] = N >= 2.0 ? log2((md + 2.0) / 3.0) : nan;  // integration [Tekl]
    o[6 * (uint64_t)n] = N >= 3.0 ? fmax(0.0, 1.0 - ra) : nan;     // integration [P-value]
    o[7 * (uint64_t)n] = md * (double)k;                        // point first moment
    o[8 * (uint64_t)n] = xy ? (double)moment2 : nan;            // point second moment
}

// ---------------------------------------------------------------- local metrics
// Clustering and controllability need, for every node v, the neighbour lists of
// all its neighbours.  Visibility rows are mostly runs of consecutive ids, so
// each row is first turned into its maximal runs [a, b] (inclusive), and the
// metrics then work run by run on two bitmaps of n bits in LDS: N(v), and the
// union of the neighbours' rows.  One wave per node builds the run lists.
//
// Pass 1 (runs == nullptr): cnt[v] = number of runs of row v.  Pass 2: the runs
// of row v at runs[run_off[v] ...].  join_self: a run that stops at v - 1 and
// one that starts at v + 1 count as one run [a, b] through v (the run kernel's
// form; the local metrics take the plain runs).
__global__ __launch_bounds__(256) void row_runs_kernel(const uint8_t *__restrict__ bytes,
                                                       const uint64_t *__restrict__ offsets,
                                                       uint32_t n, uint32_t join_self,
                                                       uint32_t *__restrict__ cnt,
                                                       const uint64_t *__restrict__ run_off,
                                                       uint2 *__restrict__ runs) {
    const uint32_t lane = lane_id();
    const uint32_t v = blockIdx.x * (blockDim.x / kWave) +
                       (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    if (v >= n) return;
    RowDecoder dec;
    const uint64_t row_end = offsets[v + 1];
    uint64_t at = runs ? run_off[v] : 0;  // index of the next run to start
    bool open = false;                    // a run is open and ends at last
    uint32_t last = 0;
    for (uint64_t base = offsets[v]; base < row_end; base += kWave) {
        uint32_t c;
        const uint32_t ids = dec.chunk(bytes, base, row_end, c);
        if (c == 0) continue;
        const bool in = lane < c;
        uint32_t prev = wave_shr1(ids);
        if (lane == 0) prev = last;
        const bool joins = in && (lane > 0 || open) &&
                           (ids == prev + 1u || (join_self && ids == prev + 2u && prev + 1u == v));
        const uint64_t starts = ballot(in && !joins);
        if (runs) {
            const uint32_t before = (uint32_t)__builtin_popcountll(starts & ((1ull << lane) - 1ull));
            if (in && !joins) runs[at + before].x = ids;
            // lane e ends a run when lane e + 1 starts one; the chunk's last id
            // stays open
            const bool ends = lane + 1u < c && ((starts >> (lane + 1u)) & 1ull);
            if (ends) runs[at + before + ((starts >> lane) & 1ull) - 1u].y = ids;
            if (open && (starts & 1ull) && lane == 0) runs[at - 1u].y = last;
        }
        at += (uint64_t)__builtin_popcountll(starts);
        last = readlane(ids, c - 1u);
        open = true;
    }
    if (runs) {
        if (open && lane == 0) runs[at - 1u].y = last;
    } else if (lane == 0) {
        cnt[v] = (uint32_t)at;
    }
}

// One neighbour run [a, b]: the popcount of nv over [a, b], and [a, b] set in
// un (other lanes may set overlapping ranges).  The end words take no branch
// (a run inside one word gets an empty mask for its second word); only runs
// over three or more words loop, over their middle words.  A run outside
// [0, n) or reversed counts nothing (the loader validated the rows, so none
// occurs; the check keeps every LDS index in bounds).
__device__ __forceinline__ uint32_t run_popc_set(const uint32_t *nv, uint32_t *un, uint32_t a,
                                                 uint32_t b, uint32_t n) {
    if (!(a <= b && b < n)) return 0u;
    const uint32_t wa = a >> 5, wb = b >> 5;
    const uint32_t lo = ~0u << (a & 31u), hi = ~0u >> (31u - (b & 31u));
    const bool one = wa == wb;
    const uint32_t m0 = one ? (lo & hi) : lo, m1 = one ? 0u : hi;
    uint32_t c = (uint32_t)__builtin_popcount(nv[wa] & m0) +
                 (uint32_t)__builtin_popcount(nv[wb] & m1);
    atomicOr(&un[wa], m0);
    atomicOr(&un[wb], m1);
    for (uint32_t i = wa + 1u; i < wb; ++i) {
        c += (uint32_t)__builtin_popcount(nv[i]);
        atomicOr(&un[i], ~0u);
    }
    return c;
}

// Set bits [a, b] of an LDS bitmap (other lanes may set overlapping ranges).
__device__ __forceinline__ void range_set(uint32_t *bm, uint32_t a, uint32_t b) {
    const uint32_t wa = a >> 5, wb = b >> 5;
    const uint32_t lo = ~0u << (a & 31u), hi = ~0u >> (31u - (b & 31u));
    if (wa == wb) {
        atomicOr(&bm[wa], lo & hi);
        return;
    }
    atomicOr(&bm[wa], lo);
    for (uint32_t i = wa + 1u; i < wb; ++i) atomicOr(&bm[i], ~0u);
    atomicOr(&bm[wb], hi);
}

// One workgroup per node v (in the processing order when given).  LDS holds two
// bitmaps of `words` 32-bit words: N(v), and U = the union of the rows of v's
// neighbours.  The pairs count is the sum over neighbours w of |N(w) & N(v)|,
// taken run by run of N(w); B(v, 2) \ {v} is (N(v) | U) without v.  The waves
// split the neighbours; the lanes split a neighbour's runs.
// city graph, all nodes: 18.5 s at 8 waves and 1 load in flight per lane,
// 16.1 s at 8 and 4, 10.2 s at 16 and 4
constexpr uint32_t kLocalWaves = 16;
constexpr uint32_t kLocalLoads = 4;

__global__ __launch_bounds__(kLocalWaves * kWave) void local_kernel(
    const uint2 *__restrict__ runs, const uint64_t *__restrict__ run_off,
    const uint32_t *__restrict__ degrees, uint32_t n, uint32_t words,
    const uint32_t *__restrict__ order, uint64_t *__restrict__ pairs_out,
    uint32_t *__restrict__ ball2_out, double *__restrict__ clustering,
    double *__restrict__ controllability) {
    extern __shared__ uint32_t s_bits[];
    __shared__ uint64_t s_pairs[kLocalWaves];
    __shared__ uint32_t s_reach[kLocalWaves];
    uint32_t *nv = s_bits, *un = s_bits + words;
    uint32_t v = xcd_block(blockIdx.x, gridDim.x);
    if (v >= n) return;  // uniform per workgroup
    if (order) v = order[v];
    const uint32_t tid = threadIdx.x, lane = lane_id();
    const uint32_t wave = (uint32_t)__builtin_amdgcn_readfirstlane((int)(tid / kWave));
    constexpr uint32_t T = kLocalWaves * kWave;
    for (uint32_t i = tid; i < 2u * words; i += T) s_bits[i] = 0u;
    __syncthreads();
    const uint64_t rs = run_off[v], re = run_off[v + 1];
    // a run outside [0, n) or reversed is skipped (the loader validated the
    // rows, so none occurs; the check keeps every LDS index in bounds)
    for (uint64_t r = rs + tid; r < re; r += T) {
        const uint2 x = runs[r];
        if (x.x <= x.y && x.y < n) range_set(nv, x.x, x.y);
    }
    __syncthreads();
    uint64_t pairs = 0;
    // wave i takes the neighbours w = i mod kLocalWaves, so the waves work on
    // adjacent rows at the same time; its lanes take the neighbour's runs,
    // kLocalLoads per lane in flight
    for (uint64_t r = rs; r < re; ++r) {
        const uint2 x = runs[r];
        if (!(x.x <= x.y && x.y < n)) continue;
        const uint32_t w0 = x.x + (wave + kLocalWaves - x.x % kLocalWaves) % kLocalWaves;
        for (uint64_t w = w0; w <= x.y; w += kLocalWaves) {
            const uint2 *row = runs + run_off[w];
            const uint32_t cnt = (uint32_t)(run_off[w + 1] - run_off[w]);  // < 2^32 per row
            for (uint32_t q = lane; q < cnt; q += kLocalLoads * kWave) {
                uint2 y[kLocalLoads];
#pragma unroll
                for (uint32_t u = 0; u < kLocalLoads; ++u)
                    y[u] = q + u * kWave < cnt ? row[q + u * kWave] : make_uint2(1u, 0u);
#pragma unroll
                for (uint32_t u = 0; u < kLocalLoads; ++u)
                    pairs += run_popc_set(nv, un, y[u].x, y[u].y, n);
            }
        }
    }
    __syncthreads();
    uint32_t reach = 0;
    for (uint32_t i = tid; i < words; i += T) reach += (uint32_t)__builtin_popcount(nv[i] | un[i]);
#pragma unroll
    for (uint32_t mask = 1; mask < kWave; mask <<= 1) {
        reach += shfl_xor(reach, mask);
        const uint32_t lo = shfl_xor((uint32_t)pairs, mask), hi = shfl_xor((uint32_t)(pairs >> 32), mask);
        pairs += ((uint64_t)hi << 32) | lo;
    }
    if (lane == 0) {
        s_pairs[wave] = pairs;
        s_reach[wave] = reach;
    }
    __syncthreads();
    if (tid != 0) return;
    uint64_t links = 0;
    uint32_t ball = 0;
    for (uint32_t i = 0; i < kLocalWaves; ++i) {
        links += s_pairs[i];
        ball += s_reach[i];
    }
    ball -= ((nv[v >> 5] | un[v >> 5]) >> (v & 31u)) & 1u;  // v itself
    const uint32_t k = degrees[v];
    const double nan = __builtin_nan("");
    if (pairs_out) pairs_out[v] = links;
    if (ball2_out) ball2_out[v] = ball;
    if (clustering)  // Watts & Strogatz: links among neighbours over k (k - 1)
        clustering[v] = k >= 2u ? (double)links / ((double)k * (double)(k - 1u)) : nan;
    if (controllability)  // first-step neighbourhood over the two-step one
        controllability[v] = ball >= 1u ? (double)k / (double)ball : nan;
}

// The same metrics with constant work per neighbour run, for n up to a quarter
// of the LDS in 32-bit words.  LDS holds, over words+1 32-bit words each: N(v);
// P, the popcount of N(v) before each word; D, a difference array of the words
// that neighbours' runs cover whole; and U, the union of their runs' partial end
// words.  A run [a, b] then adds rank(b + 1) - rank(a) to the pairs count, with
// rank(x) = P[x / 32] + popcount(N(v) word x / 32 below bit x % 32), ORs its end
// words into U and marks its whole words in D (+1 at the first, -1 after the
// last).  At the end the prefix sums of D give the words some run covers whole,
// and B(v, 2) \ {v} is the popcount of N(v) | U | (covered words) without v.
// Every count is an exact integer, so the results equal the bitmap kernel's.
__device__ __forceinline__ uint32_t rank_bits(const uint32_t *nv, const uint32_t *pre, uint32_t x) {
    const uint32_t w = x >> 5, below = (1u << (x & 31u)) - 1u;
    return pre[w] + (uint32_t)__builtin_popcount(nv[w] & below);
}

// In-place exclusive (inclusive when `inclusive`) prefix sum of a[0 .. count)
// by the whole workgroup (T threads of kLocalWaves waves); tmp holds
// kLocalWaves words.  Every thread of the workgroup calls it.
template <uint32_t T>
__device__ void block_scan(uint32_t *a, uint32_t count, uint32_t *tmp, bool inclusive) {
    const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
    const uint32_t per = (count + T - 1u) / T;
    const uint32_t b0 = tid * per < count ? tid * per : count;
    const uint32_t b1 = b0 + per < count ? b0 + per : count;
    uint32_t sum = 0;
    for (uint32_t i = b0; i < b1; ++i) sum += a[i];
    const uint32_t incl = wave_scan(sum);
    if (lane == kWave - 1) tmp[wave] = incl;
    __syncthreads();
    uint32_t before = 0;
    for (uint32_t k = 0; k < wave; ++k) before += tmp[k];
    uint32_t run = before + incl - sum;  // exclusive prefix of this thread's chunk
    __syncthreads();                     // tmp is read before anyone reuses it
    for (uint32_t i = b0; i < b1; ++i) {
        const uint32_t x = a[i];
        a[i] = inclusive ? run + x : run;
        run += x;
    }
    __syncthreads();
}

__global__ __launch_bounds__(kLocalWaves * kWave) void local_rank_kernel(
    const uint2 *__restrict__ runs, const uint64_t *__restrict__ run_off,
    const uint32_t *__restrict__ degrees, uint32_t n, uint32_t words,
    const uint32_t *__restrict__ order, uint64_t *__restrict__ pairs_out,
    uint32_t *__restrict__ ball2_out, double *__restrict__ clustering,
    double *__restrict__ controllability) {
    extern __shared__ uint32_t s_bits[];
    __shared__ uint64_t s_pairs[kLocalWaves];
    __shared__ uint32_t s_reach[kLocalWaves];
    __shared__ uint32_t s_scan[kLocalWaves];
    constexpr uint32_t T = kLocalWaves * kWave;
    const uint32_t W1 = words + 1u;  // one word past the last, for rank(n) and D
    uint32_t *nv = s_bits, *pre = s_bits + W1, *cov = s_bits + 2u * W1, *un = s_bits + 3u * W1;
    // all XCDs on one stretch of the order, as the table kernels (4.5 against
    // 5.9 s on the city graph with one node range per XCD)
    uint32_t v = xcd_span_block(blockIdx.x, gridDim.x, kXcdSpanChunk);
    if (v >= n) return;  // uniform per workgroup
    if (order) v = order[v];
    const uint32_t tid = threadIdx.x, lane = lane_id();
    const uint32_t wave = (uint32_t)__builtin_amdgcn_readfirstlane((int)(tid / kWave));
    for (uint32_t i = tid; i < 4u * W1; i += T) s_bits[i] = 0u;
    __syncthreads();
    const uint64_t rs = run_off[v], re = run_off[v + 1];
    // a run outside [0, n) or reversed is skipped (the loader validated the
    // rows, so none occurs; the check keeps every LDS index in bounds)
    for (uint64_t r = rs + tid; r < re; r += T) {
        const uint2 x = runs[r];
        if (x.x <= x.y && x.y < n) range_set(nv, x.x, x.y);
    }
    __syncthreads();
    for (uint32_t i = tid; i < W1; i += T) pre[i] = (uint32_t)__builtin_popcount(nv[i]);
    __syncthreads();
    block_scan<T>(pre, W1, s_scan, false);
    uint64_t pairs = 0;
    // wave i takes the neighbours w = i mod kLocalWaves; its lanes take the
    // neighbour's runs, kLocalLoads per lane in flight
    for (uint64_t r = rs; r < re; ++r) {
        const uint2 x = runs[r];
        if (!(x.x <= x.y && x.y < n)) continue;
        const uint32_t w0 = x.x + (wave + kLocalWaves - x.x % kLocalWaves) % kLocalWaves;
        for (uint64_t w = w0; w <= x.y; w += kLocalWaves) {
            const uint2 *row = runs + run_off[w];
            const uint32_t cnt = (uint32_t)(run_off[w + 1] - run_off[w]);  // < 2^32 per row
            for (uint32_t q = lane; q < cnt; q += kLocalLoads * kWave) {
                uint2 y[kLocalLoads];
#pragma unroll
                for (uint32_t u = 0; u < kLocalLoads; ++u)
                    y[u] = q + u * kWave < cnt ? row[q + u * kWave] : make_uint2(1u, 0u);
#pragma unroll
                for (uint32_t u = 0; u < kLocalLoads; ++u) {
                    const uint32_t a = y[u].x, b = y[u].y;
                    if (!(a <= b && b < n)) continue;
                    pairs += rank_bits(nv, pre, b + 1u) - rank_bits(nv, pre, a);
                    const uint32_t wa = a >> 5, wb = b >> 5;
                    const uint32_t lo = ~0u << (a & 31u), hi = ~0u >> (31u - (b & 31u));
                    if (wa == wb) {
                        atomicOr(&un[wa], lo & hi);
                    } else {
                        atomicOr(&un[wa], lo);
                        atomicOr(&un[wb], hi);
                        if (wb > wa + 1u) {
                            atomicAdd(&cov[wa + 1u], 1u);
                            atomicSub(&cov[wb], 1u);
                        }
                    }
                }
            }
        }
    }
    __syncthreads();
    block_scan<T>(cov, W1, s_scan, true);
    uint32_t reach = 0;
    for (uint32_t i = tid; i < words; i += T)
        reach += (uint32_t)__builtin_popcount(nv[i] | un[i] | (cov[i] ? ~0u : 0u));
#pragma unroll
    for (uint32_t mask = 1; mask < kWave; mask <<= 1) {
        reach += shfl_xor(reach, mask);
        const uint32_t lo = shfl_xor((uint32_t)pairs, mask), hi = shfl_xor((uint32_t)(pairs >> 32), mask);
        pairs += ((uint64_t)hi << 32) | lo;
    }
    if (lane == 0) {
        s_pairs[wave] = pairs;
        s_reach[wave] = reach;
    }
    __syncthreads();
    if (tid != 0) return;
    uint64_t links = 0;
    uint32_t ball = 0;
    for (uint32_t i = 0; i < kLocalWaves; ++i) {
        links += s_pairs[i];
        ball += s_reach[i];
    }
    const uint32_t wv = nv[v >> 5] | un[v >> 5] | (cov[v >> 5] ? ~0u : 0u);
    ball -= (wv >> (v & 31u)) & 1u;  // v itself
    const uint32_t k = degrees[v];
    const double nan = __builtin_nan("");
    if (pairs_out) pairs_out[v] = links;
    if (ball2_out) ball2_out[v] = ball;
    if (clustering)  // Watts & Strogatz: links among neighbours over k (k - 1)
        clustering[v] = k >= 2u ? (double)links / ((double)k * (double)(k - 1u)) : nan;
    if (controllability)  // first-step neighbourhood over the two-step one
        controllability[v] = ball >= 1u ? (double)k / (double)ball : nan;
}

__global__ void fill_u32_kernel(uint32_t *dst, uint32_t value, uint64_t count) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) dst[i] = value;
}

// ---------------------------------------------------------------- dispatch
// Compiled shapes: (p, lanes per node, bits per register).  The first entry
// of each (p, bits) is its default; the others are the alternatives the tuner
// may pick.  4-bit registers have their default shape only.
#define HB_SHAPES(X)                                                                          \
    X(4, 1, 8) X(5, 2, 8) X(6, 4, 8) X(7, 8, 8) X(8, 16, 8) X(8, 8, 8) X(9, 32, 8)             \
    X(9, 16, 8) X(10, 64, 8) X(10, 32, 8) X(10, 16, 8) X(11, 64, 8) X(11, 128, 8)              \
    X(11, 32, 8) X(12, 64, 8) X(12, 128, 8) X(12, 256, 8) X(13, 128, 8) X(13, 256, 8)          \
    X(14, 256, 8) X(14, 512, 8) X(15, 512, 8) X(16, 1024, 8) X(5, 1, 4) X(6, 2, 4) X(7, 4, 4)  \
    X(8, 8, 4) X(9, 16, 4) X(10, 32, 4) X(11, 64, 4) X(12, 64, 4) X(13, 64, 4) X(14, 128, 4)  \
    X(15, 256, 4) X(16, 512, 4)

// Workgroups and threads of a launch over n nodes.
template <class C>
void grid_for(uint32_t n, uint32_t nb, uint32_t &blocks, uint32_t &threads) {
    const uint32_t per = C::WAVES == 1 ? nb : 1u;
    blocks = (uint32_t)(((uint64_t)n + per - 1) / per);
    threads = C::WAVES == 1 ? nb * (uint32_t)kWave : (uint32_t)C::THREADS;
}

template <class C>
hipError_t launch_init_c(uint8_t *cur, double *c_prev, double *sum_d, uint32_t n, uint64_t seed,
                         const uint32_t *hash_ids, uint32_t nb, hipStream_t stream) {
    uint32_t blocks, threads;
    grid_for<C>(n, nb, blocks, threads);
    hipLaunchKernelGGL((init_kernel<C>), dim3(blocks), dim3(threads), 0, stream, cur, c_prev,
                       sum_d, n, seed, hash_ids);
    return hipGetLastError();
}

template <class C>
hipError_t launch_union_c(const uint8_t *bytes, const uint64_t *offsets, const uint8_t *cur,
                          uint8_t *next, double *c_prev, double *sum_d, uint32_t *flag_t,
                          uint32_t n, uint32_t t, const uint32_t *order, double thr,
                          const uint32_t *skip, uint32_t nb, hipStream_t stream) {
    uint32_t blocks, threads;
    grid_for<C>(n, nb, blocks, threads);
    hipLaunchKernelGGL((union_kernel<C>), dim3(blocks), dim3(threads), 0, stream, bytes, offsets,
                       cur, next, c_prev, sum_d, flag_t, n, t, order, thr, skip);
    return hipGetLastError();
}

template <class C>
hipError_t launch_union_runs_c(const uint2 *runs, const uint64_t *run_off, const uint8_t *tbl,
                               uint32_t levels, uint8_t *next, double *c_prev, double *sum_d,
                               uint32_t *flag_t, uint32_t n, uint32_t t, const uint32_t *order,
                               double thr, const uint32_t *skip, uint32_t nb,
                               hipStream_t stream) {
    if constexpr (C::PREC <= kRunsMaxP) {
        uint32_t blocks, threads;
        grid_for<C>(n, nb, blocks, threads);
        hipLaunchKernelGGL((union_runs_kernel<C>), dim3(blocks), dim3(threads), 0, stream,
                           runs, run_off, tbl, levels, next, c_prev, sum_d, flag_t, n, t, order,
                           thr, skip);
        return hipGetLastError();
    } else {
        return hipErrorInvalidValue;
    }
}

template <class C>
hipError_t launch_gather_probe_c(const uint8_t *tbl, uint32_t row_mask, uint32_t rows,
                                 uint32_t *out, uint32_t n, uint32_t with_max, uint32_t nb,
                                 hipStream_t stream) {
    if constexpr (C::PREC <= kRunsMaxP) {
        uint32_t blocks, threads;
        grid_for<C>(n, nb, blocks, threads);
        hipLaunchKernelGGL((gather_probe_kernel<C>), dim3(blocks), dim3(threads), 0, stream, tbl,
                           row_mask, rows, out, n, with_max);
        return hipGetLastError();
    } else {
        return hipErrorInvalidValue;
    }
}

template <class C>
hipError_t launch_batch_init_c(BatchJob *jobs, const uint32_t *list, const uint32_t *block_base,
                               uint32_t nlist, uint32_t nblocks, uint32_t nb, hipStream_t stream) {
    uint32_t blocks, threads;
    grid_for<C>(1u, nb, blocks, threads);
    hipLaunchKernelGGL((batch_init_kernel<C>), dim3(nblocks), dim3(threads), 0, stream, jobs,
                       list, block_base, nlist);
    return hipGetLastError();
}

template <class C>
hipError_t launch_batch_union_c(bool runs, BatchJob *jobs, const uint32_t *list,
                                const uint32_t *block_base, uint32_t nlist, uint32_t nblocks,
                                uint32_t nb, hipStream_t stream) {
    uint32_t blocks, threads;
    grid_for<C>(1u, nb, blocks, threads);
    if (runs) {
        if constexpr (C::PREC <= kRunsMaxP) {
            hipLaunchKernelGGL((batch_union_kernel<C, true>), dim3(nblocks), dim3(threads), 0,
                               stream, jobs, list, block_base, nlist);
        } else {
            return hipErrorInvalidValue;
        }
    } else {
        hipLaunchKernelGGL((batch_union_kernel<C, false>), dim3(nblocks), dim3(threads), 0,
                           stream, jobs, list, block_base, nlist);
    }
    return hipGetLastError();
}

}  // namespace

uint32_t lane_options(int p, uint32_t bits, uint32_t out[kMaxLaneOptions]) {
    uint32_t k = 0;
#define HB_LANES(P, L, B) \
    if (p == P && bits == B && k < kMaxLaneOptions) out[k++] = L;
    HB_SHAPES(HB_LANES)
#undef HB_LANES
    return k;
}

// The run kernel's default for 8-bit registers at p = 9..11: fewer lanes per
// node, so each load instruction gathers several table rows (city graph, per
// launch: p = 9 6.45 ms at 16 lanes against 6.63 at 32; p = 10 13.4 ms at 16
// against 16.7 at 64; p = 11 30.6 ms at 32 against 43.2 at 64).
constexpr int run_default_lanes(int p, int bits) {
    return bits == 8 && p >= 9 && p <= 11 ? (p == 11 ? 32 : 16) : default_lanes(p, bits);
}

Sched default_sched(int p, uint32_t bits, bool runs) {
    Sched s;
    const bool ok = p <= 16 && ((bits == 8 && p >= 4) || (bits == 4 && p >= 5));
    s.lanes = !ok ? 0u
                  : (uint32_t)(runs ? run_default_lanes(p, (int)bits) : default_lanes(p, (int)bits));
    s.nodes_per_block = s.lanes > (uint32_t)kWave ? 1u : 4u;
    s.bits = bits;
    return s;
}

bool sched_ok(int p, const Sched &s) {
    uint32_t opts[kMaxLaneOptions];
    const uint32_t k = lane_options(p, s.bits, opts);
    bool lanes_ok = false;
    for (uint32_t i = 0; i < k; ++i) lanes_ok |= opts[i] == s.lanes;
    if (!lanes_ok) return false;
    if (s.lanes > (uint32_t)kWave) return s.nodes_per_block == 1u;
    return s.nodes_per_block == 1u || s.nodes_per_block == 2u || s.nodes_per_block == 4u;
}

LaunchShape shape_for(int p, const Sched &s) {
    LaunchShape r;
    const uint32_t m = 1u << p;
    (void)m;
    r.waves_per_node = s.lanes > (uint32_t)kWave ? s.lanes / kWave : 1u;
    r.nodes_per_block = r.waves_per_node == 1 ? s.nodes_per_block : 1u;
    r.threads = r.waves_per_node == 1 ? r.nodes_per_block * kWave : r.waves_per_node * kWave;
    return r;
}

#define HB_DISPATCH(CALL)                                                  \
    do {                                                                   \
        if (!sched_ok(p, s)) return hipErrorInvalidValue;                  \
        const uint32_t nb = s.nodes_per_block;                             \
        (void)nb;                                                          \
        HB_SHAPES(CALL)                                                    \
        return hipErrorInvalidValue;                                       \
    } while (0)

hipError_t launch_init(int p, const Sched &s, uint8_t *cur, double *c_prev, double *sum_d,
                       uint32_t n, uint64_t seed, const uint32_t *hash_ids, hipStream_t stream) {
#define HB_X(P, L, B)                                                                          \
    if (p == P && s.lanes == L && s.bits == B)                                                             \
        return launch_init_c<Cfg<P, L, B>>(cur, c_prev, sum_d, n, seed, hash_ids, nb, stream);
    HB_DISPATCH(HB_X);
#undef HB_X
}

hipError_t launch_union(int p, const Sched &s, const uint8_t *bytes, const uint64_t *offsets,
                        const uint8_t *cur, uint8_t *next, double *c_prev, double *sum_d,
                        uint32_t *flag_t, uint32_t n, uint32_t t, const uint32_t *order,
                        double thr, const uint32_t *skip, hipStream_t stream) {
#define HB_X(P, L, B)                                                                            \
    if (p == P && s.lanes == L && s.bits == B)                                                               \
        return launch_union_c<Cfg<P, L, B>>(bytes, offsets, cur, next, c_prev, sum_d, flag_t, n, \
                                         t, order, thr, skip, nb, stream);
    HB_DISPATCH(HB_X);
#undef HB_X
}

hipError_t launch_union_runs(int p, const Sched &s, const uint2 *runs, const uint64_t *run_off,
                             const uint8_t *tbl, uint32_t levels, uint8_t *next, double *c_prev,
                             double *sum_d, uint32_t *flag_t, uint32_t n, uint32_t t,
                             const uint32_t *order, double thr, const uint32_t *skip,
                             hipStream_t stream) {
#define HB_X(P, L, B)                                                                          \
    if (p == P && s.lanes == L && s.bits == B)                                                             \
        return launch_union_runs_c<Cfg<P, L, B>>(runs, run_off, tbl, levels, next, c_prev,     \
                                              sum_d, flag_t, n, t, order, thr, skip, nb, stream);
    HB_DISPATCH(HB_X);
#undef HB_X
}

uint32_t group_size() { return kGroupNodes; }
uint32_t group_nodes_per_block(int p, uint32_t bits) {
    const uint32_t m = group_counter_bytes(p, bits);
    return group_block(m) / kWave / group_waves(p, bits) * kGroupNodes;
}

namespace {
template <class C>
hipError_t launch_union_groups_c(const uint32_t *grp_rows, const GroupMask *grp_mask,
                                 const uint64_t *grp_off, const uint8_t *tbl, uint8_t *next,
                                 double *c_prev, double *sum_d, uint32_t *flag_t, uint32_t n,
                                 uint32_t t, const uint32_t *order, double thr,
                                 const uint32_t *skip, hipStream_t stream) {
    constexpr uint32_t block = group_block(C::M);
    constexpr uint32_t per_block = block / kWave / group_waves(C::PREC, C::BITS);
    const uint32_t n_groups = (n + kGroupNodes - 1u) / kGroupNodes;
    const uint32_t blocks = (n_groups + per_block - 1u) / per_block;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL((union_groups_kernel<C>), dim3(blocks), dim3(block), 0, stream, grp_rows,
                       grp_mask, grp_off, tbl, next, c_prev, sum_d, flag_t, n, t, order, thr,
                       skip);
    return hipGetLastError();
}
}  // namespace

hipError_t launch_union_groups(int p, uint32_t bits, const uint32_t *grp_rows,
                               const GroupMask *grp_mask, const uint64_t *grp_off,
                               const uint8_t *tbl, uint8_t *next, double *c_prev, double *sum_d,
                               uint32_t *flag_t, uint32_t n, uint32_t t, const uint32_t *order,
                               double thr, const uint32_t *skip, hipStream_t stream) {
    // Cfg fixes the counter size, the register width and the estimator's
    // constants; its lanes-per-node field is not used by this kernel
#define HB_G(P, L, B)                                                                         \
    if (p == P && bits == B)                                                                  \
        return launch_union_groups_c<Cfg<P, L, B>>(grp_rows, grp_mask, grp_off, tbl, next,    \
                                                   c_prev, sum_d, flag_t, n, t, order, thr,   \
                                                   skip, stream);
    HB_G(8, 16, 8)
    HB_G(9, 32, 8)
    HB_G(10, 64, 8)
    HB_G(11, 128, 8)
    HB_G(12, 256, 8)
    HB_G(9, 16, 4)
    HB_G(10, 32, 4)
    HB_G(11, 64, 4)
    HB_G(12, 128, 4)
#undef HB_G
    return hipErrorInvalidValue;
}

uint32_t group_blocks(int p, uint32_t bits, uint32_t n) {
    const uint32_t per_block =
        group_block(group_counter_bytes(p, bits)) / kWave / group_waves(p, bits);
    const uint32_t n_groups = (n + kGroupNodes - 1u) / kGroupNodes;
    return (n_groups + per_block - 1u) / per_block;
}

hipError_t launch_batch_groups(int p, uint32_t bits, BatchJob *jobs, const uint32_t *list,
                               const uint32_t *block_base, uint32_t nlist, uint32_t nblocks,
                               hipStream_t stream) {
    if (nblocks == 0) return hipSuccess;
#define HB_G(P, L, B)                                                                        \
    if (p == P && bits == B) {                                                               \
        hipLaunchKernelGGL((batch_groups_kernel<Cfg<P, L, B>>), dim3(nblocks),              \
                           dim3(group_block(Cfg<P, L, B>::M)), 0, stream, jobs, list,       \
                           block_base, nlist);                                               \
        return hipGetLastError();                                                            \
    }
    HB_G(8, 16, 8)
    HB_G(9, 32, 8)
    HB_G(10, 64, 8)
    HB_G(11, 128, 8)
    HB_G(12, 256, 8)
    HB_G(9, 16, 4)
    HB_G(10, 32, 4)
    HB_G(11, 64, 4)
    HB_G(12, 128, 4)
#undef HB_G
    return hipErrorInvalidValue;
}

hipError_t launch_gather_probe(int p, const Sched &s, const uint8_t *tbl, uint32_t table_rows,
                               uint32_t rows, uint32_t *out, uint32_t n, uint32_t with_max,
                               hipStream_t stream) {
    if (table_rows == 0 || (table_rows & (table_rows - 1u))) return hipErrorInvalidValue;
#define HB_X(P, L, B)                                                                          \
    if (p == P && s.lanes == L && s.bits == B)                                                 \
        return launch_gather_probe_c<Cfg<P, L, B>>(tbl, table_rows - 1u, rows, out, n,         \
                                                   with_max, nb, stream);
    HB_DISPATCH(HB_X);
#undef HB_X
}

hipError_t launch_table(uint8_t *tbl, uint32_t n, uint32_t m, uint32_t levels, uint32_t bits,
                        const uint32_t *skip, hipStream_t stream) {
    if (levels == 0) return hipSuccess;
    if (levels <= kFusedLevels && bits == 8u && m >= 1024u && m % 128u == 0) {
        const uint64_t tiles = ((uint64_t)n + 255u) / 256u;
        const uint64_t blocks = tiles * (m / 128u);
        hipLaunchKernelGGL((table_fused_kernel<256, 8>), dim3((uint32_t)blocks), dim3(256), 0,
                           stream, tbl, n, m, levels, bits, skip);
        return hipGetLastError();
    }
    if (levels <= kFusedLevels && m % 64u == 0) {
        const uint64_t tiles = ((uint64_t)n + 511u) / 512u;
        const uint64_t blocks = tiles * (m / 64u);
        hipLaunchKernelGGL((table_fused_kernel<512, 4>), dim3((uint32_t)blocks), dim3(256), 0,
                           stream, tbl, n, m, levels, bits, skip);
        return hipGetLastError();
    }
    const uint64_t level_bytes = (uint64_t)n * m;
    for (uint32_t k = 1; k <= levels; ++k) {
        const uint64_t rows = (uint64_t)n - (1ull << k) + 1ull;
        const uint64_t count16 = rows * (m / 16u);
        const uint64_t half16 = (1ull << (k - 1)) * (m / 16u);
        const uint32_t blocks = (uint32_t)std::min<uint64_t>((count16 + 255) / 256, 256u * 64u);
        hipLaunchKernelGGL(table_level_kernel, dim3(blocks), dim3(256), 0, stream, tbl, level_bytes,
                           k, count16, half16, bits, skip);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_batch_init(int p, const Sched &s, BatchJob *jobs, const uint32_t *list,
                             const uint32_t *block_base, uint32_t nlist, uint32_t nblocks,
                             hipStream_t stream) {
    if (nblocks == 0) return hipSuccess;
#define HB_X(P, L, B)                                                                          \
    if (p == P && s.lanes == L && s.bits == B)                                                             \
        return launch_batch_init_c<Cfg<P, L, B>>(jobs, list, block_base, nlist, nblocks, nb,  \
                                              stream);
    HB_DISPATCH(HB_X);
#undef HB_X
}

hipError_t launch_batch_union(int p, const Sched &s, bool runs, BatchJob *jobs,
                              const uint32_t *list, const uint32_t *block_base, uint32_t nlist,
                              uint32_t nblocks, hipStream_t stream) {
    if (nblocks == 0) return hipSuccess;
#define HB_X(P, L, B)                                                                            \
    if (p == P && s.lanes == L && s.bits == B)                                                               \
        return launch_batch_union_c<Cfg<P, L, B>>(runs, jobs, list, block_base, nlist, nblocks, \
                                               nb, stream);
    HB_DISPATCH(HB_X);
#undef HB_X
}

uint32_t batch_table_blocks(uint32_t n, uint32_t row_bytes, uint32_t k) {
    if (k == 0 || (1ull << k) > n) return 0;
    const uint64_t count16 = ((uint64_t)n - (1ull << k) + 1ull) * (row_bytes / 16u);
    return (uint32_t)((count16 + kTableChunk - 1) / kTableChunk);
}

hipError_t launch_batch_table(BatchJob *jobs, const uint32_t *list, const uint32_t *block_base,
                              uint32_t nlist, uint32_t nblocks, uint32_t k, hipStream_t stream) {
    if (nlist == 0 || nblocks == 0) return hipSuccess;
    hipLaunchKernelGGL(batch_table_kernel, dim3(nblocks), dim3(256), 0, stream, jobs, list,
                       block_base, nlist, k);
    return hipGetLastError();
}

hipError_t launch_batch_step_end(BatchJob *jobs, const uint32_t *list, uint32_t nlist,
                                 hipStream_t stream) {
    if (nlist == 0) return hipSuccess;
    hipLaunchKernelGGL(batch_step_end_kernel, dim3((nlist + 255) / 256), dim3(256), 0, stream,
                       jobs, list, nlist);
    return hipGetLastError();
}

hipError_t launch_copy(const void *src, void *dst, uint64_t bytes, hipStream_t stream) {
    const uint64_t count = bytes / 16;
    if (count == 0) return hipSuccess;
    const uint32_t blocks = (uint32_t)std::min<uint64_t>((count + 255) / 256, 256u * 64u);
    hipLaunchKernelGGL(copy_kernel, dim3(blocks), dim3(256), 0, stream,
                       static_cast<const uint4 *>(src), static_cast<uint4 *>(dst), count);
    return hipGetLastError();
}

hipError_t launch_vga(const uint8_t *bytes, const uint64_t *offsets, const uint32_t *degrees,
                      const uint32_t *comp_size, const int32_t *xy, const double *sum_d,
                      uint32_t n, double *out, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(vga_kernel, dim3((n + 3) / 4), dim3(256), 0, stream, bytes, offsets,
                       degrees, comp_size, xy, sum_d, n, out);
    return hipGetLastError();
}

hipError_t launch_row_runs(const uint8_t *bytes, const uint64_t *offsets, uint32_t n,
                           bool join_self, uint32_t *cnt, const uint64_t *run_off, uint2 *runs,
                           hipStream_t stream) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(row_runs_kernel, dim3((n + 3) / 4), dim3(256), 0, stream, bytes, offsets, n,
                       join_self ? 1u : 0u, cnt, run_off, runs);
    return hipGetLastError();
}

uint32_t local_threads() { return kLocalWaves * kWave; }

hipError_t launch_local(const uint2 *runs, const uint64_t *run_off, const uint32_t *degrees,
                        uint32_t n, const uint32_t *order, uint64_t *pairs, uint32_t *ball2,
                        double *clustering, double *controllability, uint32_t lds_limit,
                        hipStream_t stream) {
    if (n == 0) return hipSuccess;
    const uint32_t words = (n + 31u) / 32u;
    // constant work per run when its four arrays fit, else the two bitmaps
    const size_t lds_rank = sizeof(uint32_t) * 4u * (words + 1u);
    if (lds_rank + 16u * kLocalWaves <= lds_limit) {
        hipError_t e = hipFuncSetAttribute((const void *)local_rank_kernel,
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)lds_rank);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(local_rank_kernel, dim3(n), dim3(kLocalWaves * kWave), lds_rank,
                           stream, runs, run_off, degrees, n, words, order, pairs, ball2,
                           clustering, controllability);
        return hipGetLastError();
    }
    const size_t lds = sizeof(uint32_t) * 2u * words;
    hipError_t e = hipFuncSetAttribute((const void *)local_kernel,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(local_kernel, dim3(n), dim3(kLocalWaves * kWave), lds, stream, runs,
                       run_off, degrees, n, words, order, pairs, ball2, clustering,
                       controllability);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *dst, uint32_t value, uint64_t count, hipStream_t stream) {
    if (count == 0) return hipSuccess;
    const uint32_t threads = 256;
    const uint64_t blocks = (count + threads - 1) / threads;
    hipLaunchKernelGGL(fill_u32_kernel, dim3((uint32_t)blocks), dim3(threads), 0, stream, dst,
                       value, count);
    return hipGetLastError();
}

}  // namespace hbk

// ---------------------------------------------------------------- static workspace
// The counter buffers of the run entry point that allocates nothing: one
// file-scope device array, a copy of it on every device the library runs on,
// held until the process ends.  Host code never passes the array's name to a
// kernel (on the host it is only a stand-in for the symbol); it asks the
// runtime for each device's address once, with that device current, and uses
// that address from then on.
static __device__ __align__(256) uint8_t scratch[hbk::kStaticScratchBytes];

namespace hbk {

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint8_t *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t static_scratch(uint8_t **ptr) {
    *ptr = nullptr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = static_cast<uint8_t *>(p);
    }
    *ptr = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace hbk
