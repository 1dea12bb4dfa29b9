// Greedy vertex colouring in decreasing hashed priority, computed in parallel
// by Jones and Plassmann's method (SIAM J. Sci. Comput. 14(3), 1993), and the
// sort of the level's rows by colour class.  The classes order the rounds of
// the colour-ordered local-moving mode (the colouring alternative cited in
// Section 2): no two neighbours share a class, so the vertices of one round
// never decide against each other.
#include "kernels.h"

namespace lv {

namespace {

__device__ inline int local_index(const BatchArgs &bt, int v)
{
    return bt.gid ? v - bt.gvb[bt.gid[v]] : v;
}

__device__ inline uint64_t prio_of(const ColourArgs &a, int v)
{
    return colour_priority(a.seed, a.pass, local_index(a.bt, v));
}

constexpr int CT = COLOUR_CT;

// Degree class of a row: bins 0, 1, 2, 3 and 4-6.
__device__ inline int degree_class(int d)
{
    return d <= 8 ? 0 : (d <= 32 ? 1 : (d <= 128 ? 2 : (d <= 512 ? 3 : 4)));
}

template <int G>
__device__ inline int group_sum(int x)
{
#pragma unroll
    for (int m = 1; m < G; m <<= 1) x += shfl_xor_t<int32_t>(x, m);
    return x;
}

template <int G>
__device__ inline unsigned long long group_or(unsigned long long x)
{
#pragma unroll
    for (int m = 1; m < G; m <<= 1) x |= shfl_xor_t<unsigned long long>(x, m);
    return x;
}

// Append v (when want) to class q's region of the next frontier; one atomic
// per wavefront and class.  Every lane of the wavefront calls this.
__device__ inline void frontier_push(bool want, int q, int v, const ColourArgs &a)
{
    const unsigned long long below = lanes_below();
    for (int k = 0; k < NCLS; ++k) {
        const bool mine = want && q == k;
        const unsigned long long m = __ballot(mine);
        if (m == 0) continue;
        const int leader = __ffsll((long long)m) - 1;
        int base = 0;
        if ((int)(threadIdx.x & 63) == leader) base = atomicAdd(&a.out_count[k], __popcll(m));
        base = __shfl(base, leader, 64);
        if (mine) a.out[a.cstart[k] + base + __popcll(m & below)] = v;
    }
}

// Class of this block and its index within the class's blocks.
__device__ inline int block_class(const ColourArgs &a, int *b, int *nblk)
{
    int q = 0;
    while (q + 1 < NCLS && (int)blockIdx.x >= a.rblk[q + 1]) ++q;
    *b = (int)blockIdx.x - a.rblk[q];
    *nblk = a.rblk[q + 1] - a.rblk[q];
    return q;
}

// Higher-priority neighbours of row v, summed over the G lanes of its group
// (G = CT: the whole block, through red).
template <int G>
__device__ inline int count_higher(const ColourArgs &a, int v, int lane, int *red)
{
    const uint64_t pv = prio_of(a, v);
    const int64_t e0 = a.off[v];
    const int64_t e1 = e0 + row_len(a.off, a.deg, v);
    int cnt = 0;
    for (int64_t e = e0 + lane; e < e1; e += G) {
        const int u = a.tgt[e];
        cnt += (u != v && prio_of(a, u) > pv) ? 1 : 0;
    }
    if (G <= 64) return group_sum<G>(cnt);
    cnt = group_sum<64>(cnt);
    if ((threadIdx.x & 63) == 0) atomicAdd(red, cnt);
    __syncthreads();
    const int total = *red;
    __syncthreads();
    if (threadIdx.x == 0) *red = 0;
    __syncthreads();
    return total;
}

// Initialisation of class q's rows: colour = -(1 + count); rows with no
// higher-priority neighbour form the first frontier.  Sweeps are uniform over
// the block so the pushes' ballots and the block reductions see every lane.
template <int G>
__device__ void init_class(const ColourArgs &a, int q, int b, int nblk, int *red)
{
    constexpr int PER = CT / G;
    const int lane = threadIdx.x & (G - 1);
    const int grp = threadIdx.x / G;
    const int64_t p0 = a.cstart[q], p1 = a.cstart[q + 1];
    const int64_t span = (int64_t)nblk * PER;
    const int64_t sweeps = (p1 - p0 + span - 1) / span;
    for (int64_t k = 0; k < sweeps; ++k) {
        const int64_t p = p0 + k * span + (int64_t)b * PER + grp;
        bool ready = false;
        int v = -1;
        if (p < p1) {  // uniform over a whole-block group (one row per block and sweep)
            v = a.binorder[p];
            const int cnt = count_higher<G>(a, v, lane, red);
            if (lane == 0) a.colour[v] = -(cnt + 1);
            ready = lane == 0 && cnt == 0;
        }
        frontier_push(ready, q, v, a);
    }
}

__global__ __launch_bounds__(CT) void k_colour_init(ColourArgs a)
{
    __shared__ int red;
    if (threadIdx.x == 0) red = 0;
    __syncthreads();
    int b, nblk;
    const int q = block_class(a, &b, &nblk);
    switch (q) {
    case 0: init_class<1>(a, q, b, nblk, &red); break;
    case 1: init_class<4>(a, q, b, nblk, &red); break;
    case 2: init_class<16>(a, q, b, nblk, &red); break;
    case 3: init_class<64>(a, q, b, nblk, &red); break;
    default: init_class<CT>(a, q, b, nblk, &red); break;
    }
}

// One step for the frontier rows of class q, G lanes per row (G <= 64).  The
// first pass over a row gathers the colours of its higher-priority
// neighbours in [0, 64 W) and counts the row off its lower-priority
// neighbours, pushing those that become ready; later passes (a row with at
// least 64 W colours below it) look at the next 64 W colours.
template <int G, int W>
__device__ void step_class(const ColourArgs &a, int q, int b, int nblk, int &top, int &done)
{
    constexpr int PER = CT / G;
    const int lane = threadIdx.x & (G - 1);
    const int grp = threadIdx.x / G;
    const int n = a.in_count[q];
    const int32_t *list = a.in + a.cstart[q];
    const int64_t span = (int64_t)nblk * PER;
    const int64_t sweeps = ((int64_t)n + span - 1) / span;
    for (int64_t k = 0; k < sweeps; ++k) {
        const int64_t i = k * span + (int64_t)b * PER + grp;
        const bool live = i < n;
        const int v = live ? list[i] : -1;
        const uint64_t pv = live ? prio_of(a, v) : 0;
        const int64_t e0 = live ? a.off[v] : 0;
        const int64_t e1 = live ? e0 + row_len(a.off, a.deg, v) : 0;
        // trips of the wavefront's longest row: the first pass is uniform over the
        // wavefront, so the pushes' ballots see every lane
        int64_t wtrips = (e1 - e0 + G - 1) / G;
        for (int m = G; m < 64; m <<= 1) wtrips = max(wtrips, shfl_xor_t<int64_t>(wtrips, m));
        int c = -1;
        for (int base = 0; c < 0; base += 64 * W) {
            unsigned long long mk[W];
#pragma unroll
            for (int w = 0; w < W; ++w) mk[w] = 0;
            for (int64_t t = 0; t < wtrips; ++t) {
                const int64_t e = e0 + t * G + lane;
                bool push = false;
                int u = -1;
                if (e < e1) {
                    u = a.tgt[e];
                    if (u != v) {
                        if (prio_of(a, u) > pv) {
                            const int cu = a.colour[u] - base;
#pragma unroll
                            for (int w = 0; w < W; ++w)
                                if ((cu >> 6) == w && cu >= 0) mk[w] |= 1ull << (cu & 63);
                        } else if (base == 0) {
                            push = atomicAdd(&a.colour[u], 1) == -2;
                        }
                    }
                }
                if (base == 0) frontier_push(push, push ? degree_class(row_len(a.off, a.deg, u)) : 0, u, a);
            }
            if (!live) break;
#pragma unroll
            for (int w = 0; w < W; ++w) mk[w] = group_or<G>(mk[w]);
#pragma unroll
            for (int w = W - 1; w >= 0; --w)
                if (mk[w] != ~0ull) c = base + 64 * w + __builtin_ctzll(~mk[w]);
        }
        if (live) {
            if (lane == 0) {
                a.colour[v] = c;
                ++done;
            }
            top = max(top, c + 1);
        }
    }
}

// Smallest colour >= base missing from the LDS bitmap bm of colours
// [base, base + 1024), or -1 if all are present.  Block-wide; returns the same
// value to every thread.
__device__ inline int bitmap_mex(const uint32_t *bm, int base, int *red)
{
    if (threadIdx.x < 64) {
        const uint32_t word = threadIdx.x < 32 ? bm[threadIdx.x] : 0xffffffffu;
        const unsigned long long m = __ballot(word != 0xffffffffu);
        if (threadIdx.x == 0) {
            int r = -1;
            if (m) {
                const int wi = __ffsll((long long)m) - 1;
                r = base + 32 * wi + __builtin_ctz(~bm[wi]);
            }
            *red = r;
        }
    }
    __syncthreads();
    const int c = *red;
    __syncthreads();
    return c;
}

// One step for the frontier rows of class 4 (longer than 512 entries), cut in
// chunks of CT entries spread over the class's blocks (chunk j of the i-th
// row goes to block (i + j) mod nblk).  A block gathers the colours its chunks
// see in an LDS bitmap and ORs it into the row's slot of cbm (32 words, then
// a chunk counter); the block that counts the last chunk in takes the
// smallest colour missing from the combined bitmap, rescanning the whole row
// for colours from 1024 up when all of [0, 1024) are taken, and clears the
// slot for the next step.  Slot updates are device-scope atomics.
__device__ void step_chunks(const ColourArgs &a, int b, int nblk, int &top, int &done, uint32_t *bm,
                            int *red, int32_t *tv, int32_t *tl)
{
    constexpr int q = NCLS - 1;
    const int n = a.in_count[q];
    const int32_t *list = a.in + a.cstart[q];
    for (int t0 = 0; t0 < n; t0 += CT) {
        // the rows of this tile and their lengths, loaded in parallel
        const int tn = min(CT, n - t0);
        if ((int)threadIdx.x < tn) {
            const int v = list[t0 + threadIdx.x];
            tv[threadIdx.x] = v;
            tl[threadIdx.x] = row_len(a.off, a.deg, v);
        }
        __syncthreads();
        for (int r = 0; r < tn; ++r) {
            const int i = t0 + r;
            const int v = tv[r];
            const int64_t len = tl[r];
            const int nch = (int)((len + CT - 1) / CT);
            const int j0 = ((b - i) % nblk + nblk) % nblk;
            if (j0 >= nch) continue;  // uniform over the block
            const uint64_t pv = prio_of(a, v);
            const int64_t e0 = a.off[v], e1 = e0 + len;
            if (threadIdx.x < 32) bm[threadIdx.x] = 0;
            __syncthreads();
            int mine = 0;
            for (int j = j0; j < nch; j += nblk, ++mine) {
                const int64_t e = e0 + (int64_t)j * CT + threadIdx.x;
                bool push = false;
                int u = -1;
                if (e < e1) {
                    u = a.tgt[e];
                    if (u != v) {
                        if (prio_of(a, u) > pv) {
                            const int cu = a.colour[u];
                            if (cu >= 0 && cu < 1024) atomicOr(&bm[cu >> 5], 1u << (cu & 31));
                        } else {
                            push = atomicAdd(&a.colour[u], 1) == -2;
                        }
                    }
                }
                frontier_push(push, push ? degree_class(row_len(a.off, a.deg, u)) : 0, u, a);
            }
            __syncthreads();
            uint32_t *g = a.cbm + (size_t)i * 33;
            if (threadIdx.x < 32 && bm[threadIdx.x]) atomicOr(&g[threadIdx.x], bm[threadIdx.x]);
            __threadfence();
            __syncthreads();
            if (threadIdx.x == 0) *red = atomicAdd(&g[32], (uint32_t)mine) + (uint32_t)mine == (uint32_t)nch;
            __syncthreads();
            const bool last = *red != 0;
            __syncthreads();
            if (!last) continue;  // uniform over the block
            __threadfence();
            if (threadIdx.x < 32) bm[threadIdx.x] = atomicOr(&g[threadIdx.x], 0u);
            __syncthreads();
            int c = bitmap_mex(bm, 0, red);
            for (int base = 1024; c < 0; base += 1024) {
                if (threadIdx.x < 32) bm[threadIdx.x] = 0;
                __syncthreads();
                for (int64_t e = e0 + threadIdx.x; e < e1; e += CT) {
                    const int u = a.tgt[e];
                    if (u != v && prio_of(a, u) > pv) {
                        const int cu = a.colour[u] - base;
                        if (cu >= 0 && cu < 1024) atomicOr(&bm[cu >> 5], 1u << (cu & 31));
                    }
                }
                __syncthreads();
                c = bitmap_mex(bm, base, red);
            }
            if (threadIdx.x <= 32) atomicExch(&g[threadIdx.x], 0u);
            if (threadIdx.x == 0) {
                a.colour[v] = c;
                ++done;
            }
            top = max(top, c + 1);
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(CT) void k_colour_step(ColourArgs a)
{
    __shared__ uint32_t bm[32];
    __shared__ int32_t tv[CT], tl[CT];
    __shared__ int red, s_max, s_done;
    if (threadIdx.x == 0) {
        s_max = 0;
        s_done = 0;
        red = 0;
        if (blockIdx.x == 0)
            for (int q = 0; q < NCLS; ++q) a.clear_count[q] = 0;
    }
    __syncthreads();
    int b, nblk;
    const int q = block_class(a, &b, &nblk);
    int top = 0, done = 0;
    switch (q) {
    case 0: step_class<1, 2>(a, q, b, nblk, top, done); break;
    case 1: step_class<4, 2>(a, q, b, nblk, top, done); break;
    case 2: step_class<16, 2>(a, q, b, nblk, top, done); break;
    case 3: step_class<64, 4>(a, q, b, nblk, top, done); break;
    default: step_chunks(a, b, nblk, top, done, bm, &red, tv, tl); break;
    }
    if (top) atomicMax(&s_max, top);
    if (done) atomicAdd(&s_done, done);
    __syncthreads();
    if (threadIdx.x == 0 && s_max) atomicMax(a.ncol, s_max);
    if (threadIdx.x == 0 && s_done) atomicAdd(a.coloured, s_done);
}

constexpr int CLASS_CHUNK = 4096;
constexpr int CLASS_KEYS = 8192;  // keys per LDS window
// Rows whose colour is not in [0, nkeys / NBINS) (only possible when rows are
// not symmetric) are left out; the caller compares the total with nb.

__device__ inline int bin_of_position(const BinInfo &bins, int64_t p)
{
    int b = 0;
    while (b + 1 < NBINS && p >= bins.start[b + 1]) ++b;
    return b;
}

__global__ __launch_bounds__(256) void k_class_count(const int32_t *binorder, int32_t nb, BinInfo bins,
                                                     const int32_t *colour, int32_t nkeys,
                                                     int32_t *kcount)
{
    __shared__ int32_t h[CLASS_KEYS];
    const int64_t base = (int64_t)blockIdx.x * CLASS_CHUNK;
    for (int kw = 0; kw < nkeys; kw += CLASS_KEYS) {
        for (int k = threadIdx.x; k < CLASS_KEYS; k += 256) h[k] = 0;
        __syncthreads();
        for (int r = threadIdx.x; r < CLASS_CHUNK; r += 256) {
            const int64_t p = base + r;
            if (p >= nb) break;
            const int key = colour[binorder[p]] * NBINS + bin_of_position(bins, p) - kw;
            if (key >= 0 && key < CLASS_KEYS && kw + key < nkeys) atomicAdd(&h[key], 1);
        }
        __syncthreads();
        for (int k = threadIdx.x; k < CLASS_KEYS && kw + k < nkeys; k += 256)
            if (h[k]) atomicAdd(&kcount[kw + k], h[k]);
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_class_fill(const int32_t *binorder, int32_t nb, BinInfo bins,
                                                    const int32_t *colour, int32_t nkeys, int32_t *kcur,
                                                    int32_t *order)
{
    __shared__ int32_t h[CLASS_KEYS];
    const int64_t base = (int64_t)blockIdx.x * CLASS_CHUNK;
    for (int kw = 0; kw < nkeys; kw += CLASS_KEYS) {
        for (int k = threadIdx.x; k < CLASS_KEYS; k += 256) h[k] = 0;
        __syncthreads();
        for (int r = threadIdx.x; r < CLASS_CHUNK; r += 256) {
            const int64_t p = base + r;
            if (p >= nb) break;
            const int key = colour[binorder[p]] * NBINS + bin_of_position(bins, p) - kw;
            if (key >= 0 && key < CLASS_KEYS && kw + key < nkeys) atomicAdd(&h[key], 1);
        }
        __syncthreads();
        // this block's range of each key, then ranks from LDS counters
        for (int k = threadIdx.x; k < CLASS_KEYS && kw + k < nkeys; k += 256)
            if (h[k]) h[k] = atomicAdd(&kcur[kw + k], h[k]);
        __syncthreads();
        for (int r = threadIdx.x; r < CLASS_CHUNK; r += 256) {
            const int64_t p = base + r;
            if (p >= nb) break;
            const int key = colour[binorder[p]] * NBINS + bin_of_position(bins, p) - kw;
            if (key >= 0 && key < CLASS_KEYS && kw + key < nkeys) order[atomicAdd(&h[key], 1)] = (int32_t)p;
        }
        __syncthreads();
    }
}

}  // namespace

void launch_colour_init(const ColourArgs &a, hipStream_t s)
{
    if (a.rblk[NCLS] > 0) k_colour_init<<<a.rblk[NCLS], CT, 0, s>>>(a);
}

void launch_colour_step(const ColourArgs &a, hipStream_t s)
{
    if (a.rblk[NCLS] > 0) k_colour_step<<<a.rblk[NCLS], CT, 0, s>>>(a);
}

__global__ void k_gather_i32(const int32_t *src, const int32_t *idx, int32_t n, int32_t *dst)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[idx[i]];
}

void launch_gather_i32(const int32_t *src, const int32_t *idx, int32_t n, int32_t *dst, hipStream_t s)
{
    if (n > 0) k_gather_i32<<<(int)std::min<int64_t>(((int64_t)n + 255) / 256, 1024), 256, 0, s>>>(src, idx, n, dst);
}

void launch_class_count(const int32_t *binorder, int32_t nb, BinInfo bins, const int32_t *colour,
                        int32_t nkeys, int32_t *kcount, hipStream_t s)
{
    if (nb > 0 && nkeys > 0)
        k_class_count<<<(nb + CLASS_CHUNK - 1) / CLASS_CHUNK, 256, 0, s>>>(binorder, nb, bins, colour,
                                                                          nkeys, kcount);
}

void launch_class_fill(const int32_t *binorder, int32_t nb, BinInfo bins, const int32_t *colour,
                       int32_t nkeys, int32_t *kcur, int32_t *order, hipStream_t s)
{
    if (nb > 0 && nkeys > 0)
        k_class_fill<<<(nb + CLASS_CHUNK - 1) / CLASS_CHUNK, 256, 0, s>>>(binorder, nb, bins, colour,
                                                                         nkeys, kcur, order);
}

}  // namespace lv
