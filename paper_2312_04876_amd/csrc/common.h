// Shared device-side definitions of the gfx950 Louvain kernels.
//
// Arithmetic is exact: community weights, K' and Sigma' are int32 when the
// total weight W < 2^31 and int64 otherwise; delta-modularity scores
// W*K_{i->c} - K_i*Sigma_c (Eq. 2 scaled by W^2/2) are int64 in the first
// case and 128-bit in the second.  Sums of gains are accumulated exactly in
// 128 bits.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/louvain.h"

namespace lv {

typedef __int128 i128;

// ---------------------------------------------------------------------------
// Type configurations: WT = stored weight of the current level, ST = K',
// Sigma' and table accumulator, SC = score arithmetic, VT = value of the LDS
// tables of local moving (sums of one row's weights per community).
template <typename WT_, typename ST_, typename SC_, typename VT_ = ST_>
struct Cfg {
    typedef WT_ WT;
    typedef ST_ ST;
    typedef SC_ SC;
    typedef VT_ VT;
};
typedef Cfg<int32_t, int32_t, int64_t> CfgNarrow;  // W < 2^31, every level
typedef Cfg<int32_t, int64_t, i128> CfgWideIn;     // W >= 2^31, input level (int32 weights)
typedef Cfg<int64_t, int64_t, i128> CfgWide;       // W >= 2^31, aggregated levels
// W >= 2^31, input level, every K' below 2^31: no sum of one row's weights
// can overflow 32 bits, so local moving keeps 32-bit LDS tables (half the LDS
// of CfgWideIn, more workgroups per CU)
typedef Cfg<int32_t, int64_t, i128, int32_t> CfgWideIn32;

// ---------------------------------------------------------------------------
// Degree bins.  A vertex (or, in aggregation, a community with its total
// member degree) goes to the bin of its row length d:
//   bin 0: d in [1, 8]        moving: 1 lane per row (up to 8 entries), 16-slot LDS table
//   bin 1: d in [9, 32]       4 lanes (8 entries each), 64 slots
//   bin 2: d in [33, 128]     16 lanes (8 entries each), 256 slots
//   bin 3: d in [129, 512]    one wavefront (8 entries per lane), 1024 slots
//                             (aggregation: 8 and 32 lanes for bins 0-1, a wavefront for 2-3)
//   bin 4: d in [513, 2048]   one 256-thread workgroup, up to 4096 LDS slots
//   bin 5: d in [2049, L]     one 512-thread workgroup, LDS table of up to 2L slots
//   bin 6: d > L              hubs: pairs counting-sorted into hash partitions, each
//                             folded by one workgroup in LDS (no HBM tables)
// L (the LDS row limit) is 8192 with 4-byte table values and 4096 with 8-byte
// ones, so the bin-5 table fits the 160 KB of LDS a gfx950 workgroup may use.
// Every table has at least twice as many slots as the row has entries, so
// linear probing always finds a free slot.
constexpr int NBINS = 7;
constexpr int LDS_MAX_NARROW = 8192;
constexpr int LDS_MAX_WIDE = 4096;
constexpr int HUB_THREADS = 256;
constexpr int BLOCK_THREADS = 512;
// Hub rows in local moving are not put in HBM hashtables: each round, the
// (community, weight) pairs of a queued hub's row are counting-sorted into
// partitions by a hash of the community, and one workgroup per partition
// folds it in an LDS table of 2^hub_plog2 slots.  Partitions hold about half
// that many pairs (a table sized to twice its pairs never overflows), at most
// HUB_MAXP per hub; a workgroup of the sorting kernels handles HUB_PSLICE
// entries of a row.
constexpr int HUB_PSLICE = 8192;
constexpr int HUB_MAXP = 1024;
template <typename ST>
__host__ __device__ constexpr int hub_plog2() { return 12; }
template <typename ST>
__host__ __device__ constexpr int hub_part_pairs() { return 1 << (hub_plog2<ST>() - 1); }
// Partitions of a hub row of d entries.
template <typename ST>
__host__ __device__ inline int hub_parts(int64_t d)
{
    const int64_t p = (d + hub_part_pairs<ST>() - 1) / hub_part_pairs<ST>();
    return (int)(p < 1 ? 1 : (p > HUB_MAXP ? HUB_MAXP : p));
}
// Aggregation windows of hub communities: AGG_PSLICE = 2^AGG_PLOG2 flattened
// member entries, each folded in an LDS table of AGG_FOLD_SLOTS slots.
constexpr int AGG_PLOG2 = 12;
constexpr int AGG_PSLICE = 1 << AGG_PLOG2;
// Slots of a window's fold table: 11/8 of the window (at most 8/11 full), so
// that three 256-thread workgroups with 32-bit sums fit in one CU's LDS.
constexpr int AGG_FOLD_SLOTS = 11 * (AGG_PSLICE / 8);
// Member entries per hash partition of a hub community: windows fold repeated
// neighbours first, so partitions are cut for several times more entries than
// an LDS partition table holds pairs.
constexpr int AGG_PART_ENTRIES = 4096;
// Fast mode moves levels (in a batch: graphs) of at most SEQ_MAX vertices in
// vertex order with one wavefront (k_seq.hip); its LDS table has 2 * SEQ_MAX
// slots, enough for the distinct communities of any row of such a level.
constexpr int SEQ_LOG2 = 10;
constexpr int SEQ_MAX = 1 << SEQ_LOG2;
// Rows per workgroup of the binning and compaction kernels.
constexpr int BIN_CHUNK = 4096;
// Vertices per workgroup (and LDS table slots / 2) of the community counting kernels.
constexpr int COMM_CHUNK = 2048;
constexpr int COMM_LOG2S = 12;
// Vertices per workgroup step of the round-end apply kernel, and its LDS table
// (2^APPLY_LOG2S slots >= twice the 2 * APPLY_CHUNK community keys of their moves).
constexpr int APPLY_CHUNK = 512;
constexpr int APPLY_LOG2S = 11;
// Local-moving counters are accumulated per wavefront into NSPREAD rows of
// SPREAD_W words (row = global wavefront id mod NSPREAD), so thousands of
// wavefronts do not serialise on one address; the iteration-end kernel folds
// the rows.  Row words: [0..1] 128-bit gain sum, then per degree bin b at
// 2 + 4b: vertices, entries, distinct communities, moves.
constexpr int NSPREAD = 64;
constexpr int SPREAD_W = 32;

__host__ __device__ inline int bin_of(int64_t d, int lds_max)
{
    if (d <= 0) return -1;
    if (d <= 8) return 0;
    if (d <= 32) return 1;
    if (d <= 128) return 2;
    if (d <= 512) return 3;
    if (d <= 2048) return 4;
    if (d <= lds_max) return 5;
    return 6;
}

// log2 of the LDS table of a bin-4 row of length d: the smallest power of two
// >= 2d, at least 64 slots.
__host__ __device__ inline int block_log2s(int d)
{
    int l = 6;
    while ((1 << l) < 2 * d) ++l;
    return l;
}


// ---------------------------------------------------------------------------
// Scalars shared between kernels and the host (one copy in the workspace).
struct DevScalars {
    unsigned long long sumN[LOUVAIN_MAX_ITERATIONS + 1][2];  // 128-bit gain sums per iteration
    double dq[LOUVAIN_MAX_ITERATIONS + 1];
    unsigned long long moves[LOUVAIN_MAX_ITERATIONS + 1];
    unsigned long long processed[LOUVAIN_MAX_ITERATIONS + 1];
    unsigned long long scanned[LOUVAIN_MAX_ITERATIONS + 1];
    int32_t done;
    int32_t iters;
    int32_t bin_count[8];   // active vertices per bin in the current round
    int32_t bin_start[8];   // bin boundaries of the binning step (NBINS + 1 used)
    int32_t bin_maxlen[8];  // longest row per bin (binning step)
    int32_t running;        // batches: graphs still moving after this iteration (then reset)
    unsigned long long kmax;  // wide input level: largest K' (level setup)
    // --- fields above are cleared at the start of every local-moving phase ---
    int32_t err;            // validation: bits 0-2 offsets/targets/weights, 3 batch, 4 labels
    int32_t wmax;           // validation: largest input weight
    unsigned long long scan_total;
    unsigned long long hub_slices;   // row slices of the hub bin (sum over hubs)
    unsigned long long hub_tslices;  // table slices of the hub bin
    unsigned long long act_slices;   // sorting slices / partitions of the round's queued hubs
    unsigned long long act_parts;
    unsigned long long W;
    unsigned long long sigma;       // sum of intra-community entries
    unsigned long long s2[2];       // 128-bit sum of Sigma_c^2
    int32_t alive;                  // batches: graphs not stopped after the last aggregation test
    int32_t coloured;               // colouring: vertices coloured so far
    unsigned long long work[16][5]; // algorithmic work counters per kernel family
    int32_t fcount[3][5];   // colouring: frontier sizes per degree class, three rotating slots
    int32_t ncol;           // colouring: colours used (max colour + 1)
    // --- per-wavefront counter rows (folded and cleared by the iteration end);
    // not copied back by the host's scalar reads ---
    unsigned long long spread[NSPREAD][SPREAD_W];
};

// Work-counter slots (DevScalars::work[k]): move bins 0..NBINS-1
// [vertices, entries, community totals read, moves, -], aggregation bins
// NBINS..2*NBINS-1 [communities, members, entries, emitted, -].
constexpr int WORK_MOVE = 0;
constexpr int WORK_AGG = NBINS;

// A batch of independent graphs run as one union graph: graph g owns the
// vertex range [gvb[g], gvb[g+1]) of every level and is scored, tested for
// convergence and stopped on its own (its own W, gain sum and iteration
// count), so each graph's result is the one it would have alone.  All
// pointers are null for a single graph.
struct BatchArgs {
    const int32_t *gid;        // graph of each vertex of the level
    const int32_t *gvb;        // first vertex of each graph at this level (G + 1)
    const int64_t *gW;         // total weight (2m) per graph
    unsigned long long *gsum;  // 128-bit gain sum per graph, this iteration
    int32_t *gst;              // bit 0: converged in this pass, bit 1: stopped,
                               // bit 2: moved by a wavefront of its own in this pass
    int32_t *giter;            // iterations run in this pass
    int32_t G;
};

// ---------------------------------------------------------------------------
// Device helpers.

__device__ inline uint32_t hash32(uint32_t k) { return k * 2654435761u; }

// A second, independent bijective mix of 32-bit keys (the MurmurHash3
// finaliser); its high bits pick a hub row's partition.
__device__ inline uint32_t mix32(uint32_t k)
{
    k ^= k >> 16;
    k *= 0x85ebca6bu;
    k ^= k >> 13;
    k *= 0xc2b2ae35u;
    k ^= k >> 16;
    return k;
}
__device__ inline int part_of(int32_t c, int parts)
{
    return (int)(((uint64_t)mix32((uint32_t)c) * (uint64_t)parts) >> 32);
}

// Exact 128-bit accumulation into a two-word (lo, hi) counter: the carry out
// of the low word of this addition goes into the high word, so the total is
// exact regardless of order.
__device__ inline void atomic_add_i128(unsigned long long *acc, i128 x)
{
    if (x == 0) return;
    unsigned long long lo = (unsigned long long)x;
    unsigned long long hi = (unsigned long long)(x >> 64);
    unsigned long long old = atomicAdd(&acc[0], lo);
    unsigned long long carry = (old + lo < old) ? 1ull : 0ull;
    if (hi + carry) atomicAdd(&acc[1], hi + carry);
}

__host__ __device__ inline i128 join_i128(unsigned long long lo, unsigned long long hi)
{
    return (i128)(((unsigned __int128)hi << 64) | (unsigned __int128)lo);
}

// Correctly rounded int128 -> double: the top 64 significant bits with every
// lower bit folded into a sticky bit, converted once, then scaled exactly.
__host__ __device__ inline double i128_to_f64(i128 v)
{
    const bool neg = v < 0;
    unsigned __int128 u = neg ? (unsigned __int128)(-(v + 1)) + 1u : (unsigned __int128)v;
    const uint64_t hi = (uint64_t)(u >> 64), lo = (uint64_t)u;
    double r;
    if (hi == 0) {
        r = (double)lo;
    } else {
        const int s = __builtin_clzll(hi);
        uint64_t top = s ? (hi << s) | (lo >> (64 - s)) : hi;
        const uint64_t rest = s ? (lo << s) : lo;
        top |= (rest != 0) ? 1u : 0u;
        r = ldexp((double)top, 64 - s);
    }
    return neg ? -r : r;
}

// Iteration delta-Q as in the tolerance test of Alg. 2: 2*sumN / W^2 in FP64.
__host__ __device__ inline double iteration_dq(i128 sumN, unsigned long long W)
{
    if (W == 0) return 0.0;
    const double w = (double)(int64_t)W;
    return 2.0 * i128_to_f64(sumN) / (w * w);
}

// Round of vertex v in iteration it of pass p: the top round_bits bits of
// the SplitMix64 output (Steele, Lea and Flood 2014) for counter
// (p << 40 | it << 32 | v) under key seed.
__host__ __device__ inline int round_of(uint64_t seed, int round_bits, int pass, int it, int v)
{
    if (round_bits <= 0) return 0;
    const uint64_t ctr = ((uint64_t)(uint32_t)pass << 40) | ((uint64_t)(uint32_t)(it & 0xFF) << 32) |
                         (uint64_t)(uint32_t)v;
    uint64_t z = seed + (ctr + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (int)(z >> (64 - round_bits));
}

// Candidate order of the delta-modularity argmax: higher score first, then
// the lower community id.
template <typename SC>
__device__ inline bool better(SC s, int c, SC bs, int bc)
{
    return s > bs || (s == bs && c < bc);
}

// Mask of the lanes of this wavefront below the calling lane.
__device__ inline unsigned long long lanes_below()
{
    const int lane = threadIdx.x & 63;
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Priority of vertex v (its index within its graph) for the colouring of pass
// p: the SplitMix64 output for counter (1 << 63 | p << 40 | v) under key seed.
// Distinct vertices of a pass get distinct priorities (the counter map and
// the output mix are both one-to-one).
__host__ __device__ inline uint64_t colour_priority(uint64_t seed, int pass, int v)
{
    const uint64_t ctr = (1ull << 63) | ((uint64_t)(uint32_t)pass << 40) | (uint64_t)(uint32_t)v;
    uint64_t z = seed + (ctr + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Index h with start[h] <= k < start[h + 1] in a non-decreasing start[0..n]
// (the last such h when several starts are equal).
__device__ inline int owner_slice(const int32_t *start, int n, int k)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (start[mid] <= k)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// Row of vertex v: [off[v], off[v] + length) with length from the degree
// array of a holey level or from the next offset of a dense one.
__device__ inline int row_len(const int32_t *off, const int32_t *deg, int v)
{
    return deg ? deg[v] : off[v + 1] - off[v];
}

template <typename T>
__device__ inline T shfl_xor_t(T x, int mask);

template <>
__device__ inline int32_t shfl_xor_t<int32_t>(int32_t x, int mask)
{
    return __shfl_xor(x, mask, 64);
}

template <>
__device__ inline int64_t shfl_xor_t<int64_t>(int64_t x, int mask)
{
    const int lo = __shfl_xor((int)(uint32_t)(uint64_t)x, mask, 64);
    const int hi = __shfl_xor((int)(uint32_t)((uint64_t)x >> 32), mask, 64);
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo);
}

template <>
__device__ inline unsigned long long shfl_xor_t<unsigned long long>(unsigned long long x, int mask)
{
    return (unsigned long long)shfl_xor_t<int64_t>((int64_t)x, mask);
}

template <>
__device__ inline i128 shfl_xor_t<i128>(i128 x, int mask)
{
    const int64_t lo = shfl_xor_t<int64_t>((int64_t)(uint64_t)x, mask);
    const int64_t hi = shfl_xor_t<int64_t>((int64_t)(x >> 64), mask);
    return join_i128((unsigned long long)lo, (unsigned long long)hi);
}

// Order of wavefront-level phases that communicate through LDS: all lanes
// of the wavefront finish their LDS accesses before any lane goes on.
__device__ inline void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename T>
__device__ inline void atomic_add_t(T *p, T v);

template <>
__device__ inline void atomic_add_t<int32_t>(int32_t *p, int32_t v)
{
    atomicAdd(p, v);
}

template <>
__device__ inline void atomic_add_t<int64_t>(int64_t *p, int64_t v)
{
    atomicAdd((unsigned long long *)p, (unsigned long long)v);
}

// The same, returning the value before the add.
template <typename T>
__device__ inline T atomic_add_ret(T *p, T v);

template <>
__device__ inline int32_t atomic_add_ret<int32_t>(int32_t *p, int32_t v)
{
    return atomicAdd(p, v);
}

template <>
__device__ inline int64_t atomic_add_ret<int64_t>(int64_t *p, int64_t v)
{
    return (int64_t)atomicAdd((unsigned long long *)p, (unsigned long long)v);
}

template <typename SC>
__device__ inline SC score_min();

template <>
__device__ inline int64_t score_min<int64_t>()
{
    return INT64_MIN;
}

template <>
__device__ inline i128 score_min<i128>()
{
    return (i128)(((unsigned __int128)1) << 127);
}

// Wavefront sum of an unsigned 64-bit counter (result in every lane).
__device__ inline unsigned long long wave_sum_u64(unsigned long long x)
{
    for (int o = 32; o > 0; o >>= 1) x += shfl_xor_t<unsigned long long>(x, o);
    return x;
}

__device__ inline i128 wave_sum_i128(i128 x)
{
    for (int o = 32; o > 0; o >>= 1) x += shfl_xor_t<i128>(x, o);
    return x;
}

// Insert (c, w) into an LDS table of 2^log2s slots holding at most cap keys
// (counted in *cnt).  Returns false, inserting nothing, when c is absent and
// the table already holds cap keys.
template <typename ST>
__device__ inline bool lds_insert_capped(int32_t *keys, ST *vals, int log2s, int32_t c, ST w,
                                         int *cnt, int cap)
{
    const uint32_t mask = (1u << log2s) - 1u;
    uint32_t h = hash32((uint32_t)c) >> (32 - log2s);
    for (;;) {
        const int32_t k = __hip_atomic_load(&keys[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (k == c) {
            atomic_add_t<ST>(&vals[h], w);
            return true;
        }
        if (k < 0) {
            if (atomicAdd(cnt, 1) >= cap) {
                atomicSub(cnt, 1);
                return false;
            }
            const int32_t old = atomicCAS(&keys[h], -1, c);
            if (old < 0) {
                atomic_add_t<ST>(&vals[h], w);
                return true;
            }
            atomicSub(cnt, 1);
            if (old == c) {
                atomic_add_t<ST>(&vals[h], w);
                return true;
            }
        }
        h = (h + 1) & mask;
    }
}

}  // namespace lv
