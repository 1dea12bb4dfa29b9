// Scans, fills, validation, degree binning, row reductions, compaction and
// the small per-round / per-iteration bookkeeping kernels.
#include "kernels.h"

namespace lv {

namespace {

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_CHUNK = SCAN_THREADS * SCAN_ITEMS;

__device__ inline int64_t shfl_up_i64(int64_t x, int d)
{
    const int lo = __shfl_up((int)(uint32_t)(uint64_t)x, d, 64);
    const int hi = __shfl_up((int)(uint32_t)((uint64_t)x >> 32), d, 64);
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo);
}

// Exclusive scan of one value per thread across a 256-thread block; returns
// the exclusive prefix and stores the block total in *block_total.
__device__ inline int64_t block_exclusive_scan(int64_t x, int64_t *block_total)
{
    __shared__ int64_t wsum[SCAN_THREADS / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int64_t incl = x;
    for (int d = 1; d < 64; d <<= 1) {
        const int64_t y = shfl_up_i64(incl, d);
        if (lane >= d) incl += y;
    }
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    int64_t wbase = 0, tot = 0;
    for (int k = 0; k < SCAN_THREADS / 64; ++k) {
        if (k < wave) wbase += wsum[k];
        tot += wsum[k];
    }
    __syncthreads();
    *block_total = tot;
    return wbase + incl - x;
}

template <typename TI>
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_reduce(const TI *in, int64_t n,
                                                              int64_t *part)
{
    const int64_t base = (int64_t)blockIdx.x * SCAN_CHUNK + (int64_t)threadIdx.x * SCAN_ITEMS;
    int64_t s = 0;
    for (int k = 0; k < SCAN_ITEMS; ++k)
        if (base + k < n) s += (int64_t)in[base + k];
    int64_t tot;
    block_exclusive_scan(s, &tot);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// One block scans the block totals in place (exclusive) and records the total.
template <typename TO>
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_partials(int64_t *part, int64_t nb,
                                                                TO *out, int64_t n,
                                                                unsigned long long *total)
{
    int64_t carry = 0;
    for (int64_t b0 = 0; b0 < nb; b0 += SCAN_THREADS) {
        const int64_t i = b0 + threadIdx.x;
        const int64_t x = i < nb ? part[i] : 0;
        int64_t tot;
        const int64_t ex = block_exclusive_scan(x, &tot);
        if (i < nb) part[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) {
        out[n] = (TO)carry;
        if (total) *total = (unsigned long long)carry;
    }
}

template <typename TI, typename TO>
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_apply(const TI *in, TO *out, int64_t n,
                                                             const int64_t *part)
{
    const int64_t base = (int64_t)blockIdx.x * SCAN_CHUNK + (int64_t)threadIdx.x * SCAN_ITEMS;
    TI v[SCAN_ITEMS];
    int64_t s = 0;
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        v[k] = base + k < n ? in[base + k] : (TI)0;
        s += (int64_t)v[k];
    }
    int64_t tot;
    int64_t run = part[blockIdx.x] + block_exclusive_scan(s, &tot);
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        if (base + k < n) out[base + k] = (TO)run;
        run += (int64_t)v[k];
    }
}

inline int grid_for(int64_t n, int threads, int cap = 8192)
{
    int64_t g = (n + threads - 1) / threads;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

__global__ void k_fill_i32(int32_t *p, int32_t v, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_fill_u8(uint8_t *p, uint8_t v, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_zero_u64(unsigned long long *p, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0ull;
}

__global__ void k_iota(int32_t *p, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = (int32_t)i;
}

__global__ __launch_bounds__(256) void k_validate(int32_t n, int64_t nnz, const int32_t *off,
                                                  const int32_t *tgt, const int32_t *w,
                                                  int32_t *err, unsigned long long *W,
                                                  int32_t *wmax)
{
    int e_off = 0, e_tgt = 0, e_w = 0;
    int32_t m = 0;
    unsigned long long s = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t gid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (gid == 0 && (off[0] != 0 || (int64_t)off[n] != nnz)) e_off = 1;
    for (int64_t i = gid; i < n; i += stride)
        if (off[i] > off[i + 1]) e_off = 1;
    for (int64_t e = gid; e < nnz; e += stride) {
        const int32_t t = tgt[e];
        const int32_t x = w[e];
        if (t < 0 || t >= n) e_tgt = 1;
        if (x < 1) e_w = 1;
        s += (unsigned long long)(x > 0 ? x : 0);
        m = max(m, x);
    }
    const int bits = e_off | (e_tgt << 1) | (e_w << 2);
    if (bits) atomicOr(err, bits);
    s = wave_sum_u64(s);
    if ((threadIdx.x & 63) == 0 && s) atomicAdd(W, s);
    for (int o = 32; o > 0; o >>= 1) m = max(m, __shfl_xor(m, o, 64));
    if ((threadIdx.x & 63) == 0 && m > 0) atomicMax(wmax, m);
}

__global__ __launch_bounds__(256) void k_max_u64(const int64_t *x, int32_t n,
                                                 unsigned long long *out)
{
    unsigned long long m = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const unsigned long long v = (unsigned long long)x[i];
        m = v > m ? v : m;
    }
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long v = (unsigned long long)shfl_xor_t<int64_t>((int64_t)m, o);
        m = v > m ? v : m;
    }
    if ((threadIdx.x & 63) == 0 && m) atomicMax(out, m);
}

__global__ void k_init_vertices(int32_t n, int32_t *Cp, int32_t *size, uint8_t *fa, uint8_t *fb,
                                unsigned char *K, unsigned char *Sig, int sbytes)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        Cp[i] = (int32_t)i;
        size[i] = 1;
        fa[i] = 1;
        fb[i] = 0;
        if (sbytes == 8) {
            ((int64_t *)K)[i] = 0;
            ((int64_t *)Sig)[i] = 0;
        } else {
            ((int32_t *)K)[i] = 0;
            ((int32_t *)Sig)[i] = 0;
        }
    }
}

__device__ inline int len_of(const int32_t *off, const int32_t *deg, int v)
{
    return deg ? deg[v] : off[v + 1] - off[v];
}

// ---- degree binning as a stable counting sort over chunks of BIN_CHUNK rows:
// per-chunk bin counts, one exclusive scan over [bin][chunk], then every chunk
// writes its rows at its own offsets (no global atomics, deterministic order).

// Per-wavefront bin histogram of one round (one row per lane, b < 0 = none):
// wcnt[wave][bin] = rows of the wavefront in the bin; returns the lane's rank.
__device__ inline int wave_bin_rank(int b, int32_t (*wcnt)[NBINS])
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const unsigned long long below = lanes_below();
    int rank = 0;
    for (int bb = 0; bb < NBINS; ++bb) {
        const unsigned long long m = __ballot(b == bb);
        if (b == bb) rank = __popcll(m & below);
        if (lane == 0) wcnt[wave][bb] = __popcll(m);
    }
    return rank;
}

__global__ __launch_bounds__(256) void k_bin_count(int32_t n, const int32_t *off,
                                                   const int32_t *deg, int32_t *cnt, int32_t G,
                                                   int32_t lds_max, int32_t *maxlen)
{
    __shared__ int32_t h[NBINS];
    __shared__ int32_t mx[NBINS];
    __shared__ int32_t wcnt[4][NBINS];
    if (threadIdx.x < NBINS) {
        h[threadIdx.x] = 0;
        mx[threadIdx.x] = 0;
    }
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * BIN_CHUNK;
    for (int r = 0; r < BIN_CHUNK / 256; ++r) {
        const int64_t i = base + r * 256 + threadIdx.x;
        const int len = i < n ? len_of(off, deg, (int)i) : 0;
        const int b = bin_of(len, lds_max);
        if (b >= 0) atomicMax(&mx[b], len);
        wave_bin_rank(b, wcnt);
        __syncthreads();
        if (threadIdx.x < NBINS)
            h[threadIdx.x] += wcnt[0][threadIdx.x] + wcnt[1][threadIdx.x] + wcnt[2][threadIdx.x] +
                              wcnt[3][threadIdx.x];
        __syncthreads();
    }
    if (threadIdx.x < NBINS) {
        cnt[threadIdx.x * G + blockIdx.x] = h[threadIdx.x];
        if (mx[threadIdx.x]) atomicMax(&maxlen[threadIdx.x], mx[threadIdx.x]);
    }
}

__global__ void k_bin_starts(const int32_t *boff, int32_t G, int32_t *start)
{
    const int b = threadIdx.x;
    if (b <= NBINS) start[b] = boff[b * G];
}

__global__ __launch_bounds__(256) void k_bin_fill(int32_t n, const int32_t *off,
                                                  const int32_t *deg, const int32_t *boff,
                                                  int32_t G, int32_t lds_max, int32_t *binorder)
{
    __shared__ int32_t run[NBINS];
    __shared__ int32_t wcnt[4][NBINS];
    if (threadIdx.x < NBINS) run[threadIdx.x] = boff[threadIdx.x * G + blockIdx.x];
    __syncthreads();
    const int wave = threadIdx.x >> 6;
    const int64_t base = (int64_t)blockIdx.x * BIN_CHUNK;
    for (int r = 0; r < BIN_CHUNK / 256; ++r) {
        const int64_t i = base + r * 256 + threadIdx.x;
        const int b = i < n ? bin_of(len_of(off, deg, (int)i), lds_max) : -1;
        const int rank = wave_bin_rank(b, wcnt);
        __syncthreads();
        if (b >= 0) {
            int pos = run[b] + rank;
            for (int w = 0; w < wave; ++w) pos += wcnt[w][b];
            binorder[pos] = (int32_t)i;
        }
        __syncthreads();
        if (threadIdx.x < NBINS)
            run[threadIdx.x] += wcnt[0][threadIdx.x] + wcnt[1][threadIdx.x] + wcnt[2][threadIdx.x] +
                                wcnt[3][threadIdx.x];
        __syncthreads();
    }
}


// owner[k] = h with start[h] <= k < start[h + 1], for k < total: one thread per
// k (a giant hub owns hundreds of thousands of slices, so threads per range would
// leave one thread writing them all).
__global__ void k_owner_map(const int32_t *start, int32_t n, int32_t total, int32_t *owner)
{
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < total;
         k += (int64_t)gridDim.x * blockDim.x)
        owner[k] = owner_slice(start, n, (int)k);
}

__global__ void k_hub_move_sizes(const int32_t *binorder, int32_t hb, int32_t he,
                                 const int32_t *off, const int32_t *deg, int stbytes,
                                 int64_t *ent, int32_t *slices, int32_t *parts, int slice,
                                 int per_part)
{
    for (int64_t p = hb + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < he;
         p += (int64_t)gridDim.x * blockDim.x) {
        const int64_t d = len_of(off, deg, binorder[p]);
        ent[p - hb] = d;
        slices[p - hb] = (int32_t)((d + slice - 1) / slice);
        const int64_t q = (d + per_part - 1) / per_part;
        parts[p - hb] = (int32_t)(q < 1 ? 1 : (q > HUB_MAXP ? HUB_MAXP : q));
    }
}

// Row reductions with G lanes per row (G <= 64: groups inside a wavefront;
// G == 256: the whole workgroup).
template <class C, int G, int OP>
__global__ __launch_bounds__(256) void k_row_reduce(RowArgs<C> a)
{
    typedef typename C::ST ST;
    __shared__ unsigned long long red[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    unsigned long long acc = 0;
    if constexpr (G <= 64) {
        constexpr int GPW = 64 / G;
        const int grp = lane / G, gl = lane % G;
        const int stride = gridDim.x * 4 * GPW;
        for (int base = (blockIdx.x * 4 + wave) * GPW; base < a.count; base += stride) {
            const int idx = base + grp;
            const bool has = idx < a.count;
            int v = 0, beg = 0, d = 0;
            if (has) {
                v = a.binorder[a.begin + idx];
                beg = a.off[v];
                d = len_of(a.off, a.deg, v);
            }
            int64_t s = 0;
            const int lv = (OP == 1 && has) ? a.labels[v] : 0;
            for (int e = gl; e < d; e += G) {
                const int64_t x = (int64_t)a.w[beg + e];
                if (OP == 0 || a.labels[a.tgt[beg + e]] == lv) s += x;
            }
            for (int o = G / 2; o > 0; o >>= 1) s += shfl_xor_t<int64_t>(s, o);
            if (OP == 0) {
                if (has && gl == 0) {
                    a.K[v] = (ST)s;
                    a.Sig[v] = (ST)s;
                }
            } else if (gl == 0) {
                acc += (unsigned long long)s;
            }
        }
    } else {
        __shared__ int64_t part[4];
        for (int idx = blockIdx.x; idx < a.count; idx += gridDim.x) {
            const int v = a.binorder[a.begin + idx];
            const int beg = a.off[v];
            const int d = len_of(a.off, a.deg, v);
            const int lv = OP == 1 ? a.labels[v] : 0;
            int64_t s = 0;
            for (int e = threadIdx.x; e < d; e += 256) {
                const int64_t x = (int64_t)a.w[beg + e];
                if (OP == 0 || a.labels[a.tgt[beg + e]] == lv) s += x;
            }
            for (int o = 32; o > 0; o >>= 1) s += shfl_xor_t<int64_t>(s, o);
            if (lane == 0) part[wave] = s;
            __syncthreads();
            if (threadIdx.x == 0) {
                const int64_t t = part[0] + part[1] + part[2] + part[3];
                if (OP == 0) {
                    a.K[v] = (ST)t;
                    a.Sig[v] = (ST)t;
                } else {
                    acc += (unsigned long long)t;
                }
            }
            __syncthreads();
        }
    }
    if (OP == 1) {
        acc = wave_sum_u64(acc);
        if (lane == 0) red[wave] = acc;
        __syncthreads();
        if (threadIdx.x == 0) {
            const unsigned long long t = red[0] + red[1] + red[2] + red[3];
            if (t) atomicAdd(a.sigma, t);
        }
    }
}

// Row reductions of the hub bin, split like its local-moving scatter: slice k
// of hub h (start[h] <= k < start[h + 1]) covers entries
// [(k - start[h]) * HUB_PSLICE, +HUB_PSLICE) of the row, one workgroup at a
// time over a grid-strided slice index.  Partial sums are added atomically
// (integers, so the order does not matter); for OP 0 K' and Sigma' of the
// hub rows start at zero.
template <class C, int OP>
__global__ __launch_bounds__(256) void k_row_reduce_hub(RowArgs<C> a, const int32_t *start,
                                                        const unsigned long long *nslices)
{
    typedef typename C::ST ST;
    __shared__ int64_t part[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int total = (int)*nslices;
    unsigned long long acc = 0;
    for (int k = blockIdx.x; k < total; k += gridDim.x) {
        const int h = owner_slice(start, a.count, k);
        const int v = a.binorder[a.begin + h];
        const int beg = a.off[v];
        const int d = len_of(a.off, a.deg, v);
        const int e0 = (k - start[h]) * HUB_PSLICE;
        const int e1 = min(e0 + HUB_PSLICE, d);
        const int lv = OP == 1 ? a.labels[v] : 0;
        int64_t s = 0;
        for (int e = e0 + (int)threadIdx.x; e < e1; e += 256) {
            const int64_t x = (int64_t)a.w[beg + e];
            if (OP == 0 || a.labels[a.tgt[beg + e]] == lv) s += x;
        }
        for (int o = 32; o > 0; o >>= 1) s += shfl_xor_t<int64_t>(s, o);
        if (lane == 0) part[wave] = s;
        __syncthreads();
        if (threadIdx.x == 0) {
            const int64_t t = part[0] + part[1] + part[2] + part[3];
            if (OP == 0) {
                if (t) {
                    atomic_add_t<ST>(&a.K[v], (ST)t);
                    atomic_add_t<ST>(&a.Sig[v], (ST)t);
                }
            } else {
                acc += (unsigned long long)t;
            }
        }
        __syncthreads();
    }
    if (OP == 1 && threadIdx.x == 0 && acc) atomicAdd(a.sigma, acc);
}

template <typename ST>
__global__ __launch_bounds__(256) void k_sum_squares(const ST *Sig, int32_t n,
                                                     unsigned long long *acc)
{
    i128 s = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const i128 x = (i128)Sig[i];
        s += x * x;
    }
    s = wave_sum_i128(s);
    if ((threadIdx.x & 63) == 0) atomic_add_i128(acc, s);
}

// Active rows of one round into per-bin worklists: each workgroup takes a chunk
// of BIN_CHUNK binned rows, counts its active rows per bin, reserves space with
// one atomic per bin, and writes positions in order.  Active hubs are also
// flagged for the sliced hub kernels.
__global__ __launch_bounds__(256) void k_compact(CompactArgs a)
{
    if (*a.done) return;
    constexpr int R = BIN_CHUNK / 256;
    __shared__ int32_t bcnt[NBINS];
    __shared__ int32_t run[NBINS];
    __shared__ int32_t wcnt[4][NBINS];
    if (threadIdx.x < NBINS) bcnt[threadIdx.x] = 0;
    __syncthreads();
    const int wave = threadIdx.x >> 6;
    const int64_t base = (int64_t)blockIdx.x * BIN_CHUNK;
    // positions binorder[0, nb), or the positions order[q0, q1) of one colour class
    const int64_t len = a.order ? (int64_t)(a.q1 - a.q0) : (int64_t)a.nb;
    int sel[R];
    int32_t pos_of[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t i = base + r * 256 + threadIdx.x;
        int b = -1;
        pos_of[r] = -1;
        if (i < len) {
            const int64_t p = a.order ? (int64_t)a.order[a.q0 + i] : i;
            pos_of[r] = (int32_t)p;
            const int v = a.binorder[p];
            bool act = a.prune ? (a.flags[v] != 0) : true;
            if (a.hubs_only && p < a.bins.start[NBINS - 1]) act = false;
            int lv = v;  // index within its graph (a batch numbers each graph from 0)
            if (a.bt.gid) {
                const int g = a.bt.gid[v];
                if (a.bt.gst[g]) act = false;
                lv = v - a.bt.gvb[g];
            }
            if (act && a.round_bits > 0)
                act = round_of(a.seed, a.round_bits, a.pass, a.it, lv) == a.round;
            if (act) {
                if (a.prune) a.flags[v] = 0;
                b = 0;
                while (b + 1 < NBINS && p >= a.bins.start[b + 1]) ++b;
                if (b == NBINS - 1) a.hub_act[p - a.bins.start[NBINS - 1]] = 1;
            }
        }
        sel[r] = b;
        wave_bin_rank(b, wcnt);
        __syncthreads();
        if (threadIdx.x < NBINS)
            bcnt[threadIdx.x] += wcnt[0][threadIdx.x] + wcnt[1][threadIdx.x] + wcnt[2][threadIdx.x] +
                                 wcnt[3][threadIdx.x];
        __syncthreads();
    }
    if (threadIdx.x < NBINS)
        run[threadIdx.x] = bcnt[threadIdx.x] ? atomicAdd(&a.counts[threadIdx.x], bcnt[threadIdx.x]) : 0;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int b = sel[r];
        const int rank = wave_bin_rank(b, wcnt);
        __syncthreads();
        if (b >= 0) {
            int pos = a.bins.start[b] + run[b] + rank;
            for (int w = 0; w < wave; ++w) pos += wcnt[w][b];
            // vertex ids for bins 0-4, binorder positions for hubs (their tables are per position)
            const int32_t p = pos_of[r];
            a.worklist[pos] = b == NBINS - 1 ? p : a.binorder[p];
        }
        __syncthreads();
        if (threadIdx.x < NBINS)
            run[threadIdx.x] += wcnt[0][threadIdx.x] + wcnt[1][threadIdx.x] + wcnt[2][threadIdx.x] +
                                wcnt[3][threadIdx.x];
        __syncthreads();
    }
}

// Colour-ordered mode: every round's rows but the hubs in one pass (see
// launch_compact_keys).  Ranks come from one atomic per distinct key of a
// wavefront; keys are sorted, so a wavefront rarely holds more than two.
__global__ __launch_bounds__(256) void k_compact_keys(CompactArgs a, const int32_t *koff,
                                                      int32_t nkeys, int32_t *kact, int32_t *klist,
                                                      unsigned long long *processed)
{
    if (*a.done) return;
    const int lane = threadIdx.x & 63;
    const unsigned long long below = lanes_below();
    const int32_t hub_start = a.bins.start[NBINS - 1];
    unsigned long long nact = 0;
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t base = (int64_t)blockIdx.x * 256; base < a.nb; base += stride) {
        const int64_t i = base + threadIdx.x;
        bool act = false;
        int k = 0, v = 0;
        if (i < a.nb) {
            const int p = a.order[i];
            if (p < hub_start) {  // hub rows: the round's own compaction
                v = a.binorder[p];
                act = a.prune ? (a.flags[v] != 0) : true;
                if (a.bt.gid && a.bt.gst[a.bt.gid[v]]) act = false;
                if (act) {
                    if (a.prune) a.flags[v] = 0;
                    k = owner_slice(koff, nkeys, (int)i);
                }
            }
        }
        int rank = 0;
        unsigned long long pending = __ballot(act);
        while (pending) {  // uniform over the wavefront
            const int leader = __ffsll((long long)pending) - 1;
            const int k0 = __shfl(k, leader, 64);
            const bool mine = act && k == k0;
            const unsigned long long m = __ballot(mine);
            int b0 = 0;
            if (lane == leader) b0 = atomicAdd(&kact[k0], __popcll(m));
            b0 = __shfl(b0, leader, 64);
            if (mine) rank = b0 + __popcll(m & below);
            pending &= ~m;
        }
        if (act) {
            klist[koff[k] + rank] = v;
            ++nact;
        }
    }
    nact = wave_sum_u64(nact);
    if (lane == 0 && nact) atomicAdd(processed, nact);
}

// Slot of community c in the apply kernel's LDS table (inserted if absent; the
// inserting thread appends the slot to the chunk's list of used slots).
__device__ inline int apply_slot(int32_t *keys, int32_t c, int32_t *used, int32_t *nused)
{
    constexpr uint32_t mask = (1u << APPLY_LOG2S) - 1u;
    uint32_t h = hash32((uint32_t)c) >> (32 - APPLY_LOG2S);
    for (;;) {
        const int32_t k = __hip_atomic_load(&keys[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (k == c) return (int)h;
        if (k < 0) {
            const int32_t old = atomicCAS(&keys[h], -1, c);
            if (old < 0) used[atomicAdd(nused, 1)] = (int32_t)h;
            if (old < 0 || old == c) return (int)h;
        }
        h = (h + 1) & mask;
    }
}

template <typename ST>
__global__ __launch_bounds__(256) void k_apply(int32_t *mv_c, int32_t n, int32_t *Cp,
                                               const ST *K, ST *Sig, int32_t *size,
                                               const int32_t *done)
{
    constexpr int S = 1 << APPLY_LOG2S;
    __shared__ int32_t keys[S];
    __shared__ ST dsig[S];
    __shared__ int32_t dsz[S];
    __shared__ int32_t used[2 * APPLY_CHUNK];  // a chunk's movers name at most 2 * APPLY_CHUNK keys
    __shared__ int32_t nused;
    if (*done) return;
    for (int s = threadIdx.x; s < S; s += blockDim.x) {
        keys[s] = -1;
        dsig[s] = 0;
        dsz[s] = 0;
    }
    if (threadIdx.x == 0) nused = 0;
    __syncthreads();
    for (int64_t base = (int64_t)blockIdx.x * APPLY_CHUNK; base < n;
         base += (int64_t)gridDim.x * APPLY_CHUNK) {
        for (int q = threadIdx.x; q < APPLY_CHUNK; q += blockDim.x) {
            const int64_t v = base + q;
            if (v >= n) break;
            const int c = mv_c[v];
            if (c < 0) continue;
            // labels change only here, so Cp[v] is still the label the move was decided from
            const int d = Cp[v];
            const ST kv = K[v];
            Cp[v] = c;
            mv_c[v] = -1;
            const int sd = apply_slot(keys, d, used, &nused);
            atomic_add_t<ST>(&dsig[sd], (ST)-kv);
            atomicSub(&dsz[sd], 1);
            const int sc = apply_slot(keys, c, used, &nused);
            atomic_add_t<ST>(&dsig[sc], kv);
            atomicAdd(&dsz[sc], 1);
        }
        __syncthreads();
        // flush only the slots this chunk used
        const int nu = nused;
        for (int q = threadIdx.x; q < nu; q += blockDim.x) {
            const int s = used[q];
            const int32_t key = keys[s];
            if (dsig[s] != 0) atomic_add_t<ST>(&Sig[key], dsig[s]);
            if (dsz[s] != 0) atomicAdd(&size[key], dsz[s]);
            keys[s] = -1;
            dsig[s] = 0;
            dsz[s] = 0;
        }
        __syncthreads();
        if (threadIdx.x == 0) nused = 0;
        __syncthreads();
    }
}

__global__ void k_round_end(DevScalars *sc, int it)
{
    const int t = threadIdx.x;
    if (t < NBINS) {
        const int c = sc->bin_count[t];
        if (c) atomicAdd(&sc->processed[it], (unsigned long long)c);
        sc->bin_count[t] = 0;
    }
}

__global__ __launch_bounds__(64) void k_iter_end(DevScalars *sc, int it, double tau, int batch)
{
    if (sc->done) return;
    const int lane = threadIdx.x;  // one counter row per lane
    unsigned long long *row = sc->spread[lane];
    const i128 g = wave_sum_i128(join_i128(row[0], row[1]));
    unsigned long long moves = 0, scanned = 0;
    for (int b = 0; b < NBINS; ++b) {
        for (int k = 0; k < 4; ++k) {
            const unsigned long long x = wave_sum_u64(row[2 + 4 * b + k]);
            if (lane == 0) sc->work[WORK_MOVE + b][k] += x;
            if (k == 1) scanned += x;
            if (k == 3) moves += x;
        }
    }
    for (int f = 0; f < SPREAD_W; ++f) row[f] = 0;
    if (lane != 0) return;
    sc->sumN[it][0] = (unsigned long long)g;
    sc->sumN[it][1] = (unsigned long long)(g >> 64);
    sc->moves[it] = moves;
    sc->scanned[it] = scanned;
    const double dq = iteration_dq(g, sc->W);
    sc->dq[it] = dq;
    sc->iters = it + 1;
    if (batch) {
        // a batch stops when every graph has converged (or stopped)
        if (sc->running == 0) sc->done = 1;
        sc->running = 0;
    } else if (dq <= tau) {
        sc->done = 1;
    }
}

// ---- warm start: the first pass starts from a given partition

// err bit 4 when a label is outside [0, n), or outside its graph's vertex range in a batch.
__global__ void k_warm_check(int32_t n, const int32_t *labels, const int32_t *gid,
                             const int32_t *gvb, int32_t *err)
{
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        const int c = labels[v];
        bool bad = c < 0 || c >= n;
        if (!bad && gid) bad = c < gvb[gid[v]] || c >= gvb[gid[v] + 1];
        if (bad) atomicOr(err, 16);
    }
}

// C'[v] = labels[v]; Sigma' and the sizes of that partition (both zero on entry).
template <typename ST>
__global__ void k_warm_labels(int32_t n, const int32_t *labels, const ST *K, int32_t *Cp, ST *Sig,
                              int32_t *size)
{
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        const int c = labels[v];
        Cp[v] = c;
        atomic_add_t<ST>(&Sig[c], K[v]);
        atomicAdd(&size[c], 1);
    }
}

// ---- batches of independent graphs (see BatchArgs)

// gid[v] = graph owning vertex v (the last graph whose first vertex is <= v,
// so empty graphs own nothing).
__global__ void k_batch_gid(int32_t n, const int32_t *gvb, int32_t G, int32_t *gid)
{
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x)
        gid[v] = owner_slice(gvb, G, (int)v);
}

// Checks the graph offsets' shape and that every entry stays inside its
// graph (err bit 3), and adds every row's weight to its graph's W.
__global__ void k_batch_check(int32_t n, const int32_t *off, const int32_t *tgt, const int32_t *w,
                              const int32_t *gid, const int32_t *gvb, int64_t *gW, int32_t *err)
{
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        const int g = gid[v];
        const int lo = gvb[g], hi = gvb[g + 1];
        int64_t sum = 0;
        bool bad = false;
        for (int e = off[v]; e < off[v + 1]; ++e) {
            const int j = tgt[e];
            bad |= j < lo || j >= hi;
            sum += w[e];
        }
        if (bad) atomicOr(err, 8);
        if (sum) atomicAdd((unsigned long long *)&gW[g], (unsigned long long)sum);
    }
}

// Start of a run: every graph alive, each its own vertices as communities.
__global__ void k_batch_reset(BatchArgs b, int32_t *gcomm)
{
    for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < b.G; g += gridDim.x * blockDim.x) {
        b.gst[g] = 0;
        b.giter[g] = 0;
        gcomm[g] = b.gvb[g + 1] - b.gvb[g];
    }
}

// Start of a local-moving phase: no graph has converged in it yet.
__global__ void k_batch_pass_begin(BatchArgs b)
{
    for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < b.G; g += gridDim.x * blockDim.x) {
        b.gst[g] &= 2;
        b.giter[g] = 0;
        b.gsum[2 * g] = 0;
        b.gsum[2 * g + 1] = 0;
    }
}

// Graphs of at most max_n vertices (not stopped) are moved by a wavefront of
// their own in this pass (bit 2); the degree bins skip them from now on.
__global__ void k_batch_mark_small(BatchArgs b, int32_t max_n)
{
    for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < b.G; g += gridDim.x * blockDim.x) {
        if (b.gst[g] & 2) continue;
        const int nv = b.gvb[g + 1] - b.gvb[g];
        if (nv >= 1 && nv <= max_n) b.gst[g] |= 4;
    }
}

// End of an iteration, per graph still moving: one more iteration, then its
// own delta-Q test; counts the graphs that keep moving in sc->running.
__global__ void k_batch_iter_end(BatchArgs b, DevScalars *sc, double tau)
{
    if (sc->done) return;
    for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < b.G; g += gridDim.x * blockDim.x) {
        if (b.gst[g]) continue;
        b.giter[g] += 1;
        const double dq = iteration_dq(join_i128(b.gsum[2 * g], b.gsum[2 * g + 1]),
                                       (unsigned long long)b.gW[g]);
        b.gsum[2 * g] = 0;
        b.gsum[2 * g + 1] = 0;
        if (dq <= tau)
            b.gst[g] |= 1;
        else
            atomicAdd(&sc->running, 1);
    }
}

// After local moving and the community count of a level (idmap = exclusive
// scan of the used labels over the level's n vertices, nc in total): each
// graph's first community and count, and the stop test of Alg. 1 per graph
// (converged in one sweep, or too few merges); sc->alive counts the graphs
// that go on.
__global__ void k_batch_agg_test(BatchArgs b, const int32_t *idmap, int32_t n, int32_t nc,
                                 double aggtol, int32_t *gvb_next, int32_t *gcomm, DevScalars *sc)
{
    for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < b.G; g += gridDim.x * blockDim.x) {
        const int v0 = b.gvb[g], v1 = b.gvb[g + 1];
        const int c0 = v0 < n ? idmap[v0] : nc, c1 = v1 < n ? idmap[v1] : nc;
        gvb_next[g] = c0;
        if (g == b.G - 1) gvb_next[b.G] = nc;
        gcomm[g] = c1 - c0;
        if (b.gst[g] & 2) continue;
        if (b.giter[g] <= 1 || (double)(c1 - c0) / (double)(v1 - v0) > aggtol)
            b.gst[g] |= 2;
        else
            atomicAdd(&sc->alive, 1);
    }
}

// Graph of every super-vertex of the next level (labels already dense).
__global__ void k_batch_gid_next(int32_t n, const int32_t *labels, const int32_t *gid,
                                 int32_t *gid_next)
{
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x)
        gid_next[labels[v]] = gid[v];
}

// Per-graph modularity terms on a level with labels: sigma_g (entries inside
// a community, one wavefront per row) and S2_g (sum of squared community
// weights, 128-bit).
template <typename WT>
__global__ __launch_bounds__(256) void k_batch_sigma(int32_t n, const int32_t *off,
                                                     const int32_t *deg, const int32_t *tgt,
                                                     const WT *w, const int32_t *labels,
                                                     const int32_t *gid, unsigned long long *gsig)
{
    const int lane = threadIdx.x & 63;
    for (int64_t v = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6; v < n;
         v += ((int64_t)gridDim.x * blockDim.x) >> 6) {
        const int beg = off[v];
        const int len = deg ? deg[v] : off[v + 1] - off[v];
        const int lv = labels[v];
        unsigned long long sum = 0;
        for (int e = lane; e < len; e += 64)
            if (labels[tgt[beg + e]] == lv) sum += (unsigned long long)w[beg + e];
        sum = wave_sum_u64(sum);
        if (lane == 0 && sum) atomicAdd(&gsig[gid[v]], sum);
    }
}

template <typename ST>
__global__ void k_batch_s2(int32_t n, const ST *Sig, const int32_t *gid, unsigned long long *gs2)
{
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < n;
         c += (int64_t)gridDim.x * blockDim.x) {
        const ST x = Sig[c];
        if (x) atomic_add_i128(gs2 + 2 * gid[c], (i128)x * (i128)x);
    }
}

__global__ void k_mark_used(int32_t n, const int32_t *labels, int32_t *used)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        used[labels[i]] = 1;
}

__global__ void k_relabel(int32_t n, int32_t *labels, const int32_t *map)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        labels[i] = map[labels[i]];
}

// Slot of key c in a 2*COMM_CHUNK-slot LDS table (inserting it if absent).
__device__ inline int lds_slot(int32_t *keys, int32_t c)
{
    constexpr uint32_t mask = 2 * COMM_CHUNK - 1;
    uint32_t h = hash32((uint32_t)c) >> (32 - COMM_LOG2S);
    for (;;) {
        const int32_t k = __hip_atomic_load(&keys[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (k == c) return (int)h;
        if (k < 0) {
            const int32_t old = atomicCAS(&keys[h], -1, c);
            if (old < 0 || old == c) return (int)h;
        }
        h = (h + 1) & mask;
    }
}

// Members and total degree per community, pre-aggregated per chunk of
// COMM_CHUNK vertices in LDS so that a large community costs one global atomic
// per chunk instead of one per member.
__global__ __launch_bounds__(256) void k_comm_count(int32_t n, const int32_t *Cp, const int32_t *off,
                                                    const int32_t *deg, int32_t *ccount,
                                                    int32_t *ctot)
{
    __shared__ int32_t keys[2 * COMM_CHUNK];
    __shared__ int32_t cnt[2 * COMM_CHUNK];
    __shared__ int32_t dsum[2 * COMM_CHUNK];
    for (int s = threadIdx.x; s < 2 * COMM_CHUNK; s += 256) {
        keys[s] = -1;
        cnt[s] = 0;
        dsum[s] = 0;
    }
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * COMM_CHUNK;
    for (int r = 0; r < COMM_CHUNK / 256; ++r) {
        const int64_t i = base + r * 256 + threadIdx.x;
        if (i < n) {
            const int s = lds_slot(keys, Cp[i]);
            atomicAdd(&cnt[s], 1);
            const int d = len_of(off, deg, (int)i);
            if (d) atomicAdd(&dsum[s], d);
        }
    }
    __syncthreads();
    for (int s = threadIdx.x; s < 2 * COMM_CHUNK; s += 256) {
        const int c = keys[s];
        if (c >= 0) {
            atomicAdd(&ccount[c], cnt[s]);
            if (dsum[s]) atomicAdd(&ctot[c], dsum[s]);
        }
    }
}

// Community-vertex CSR fill: every chunk reserves one range per community it
// touches and places its members there (rank inside the chunk from LDS).
__global__ __launch_bounds__(256) void k_comm_fill(int32_t n, const int32_t *Cp, const int32_t *coff,
                                                   int32_t *cursor, int32_t *members)
{
    constexpr int R = COMM_CHUNK / 256;
    __shared__ int32_t keys[2 * COMM_CHUNK];
    __shared__ int32_t cnt[2 * COMM_CHUNK];
    for (int s = threadIdx.x; s < 2 * COMM_CHUNK; s += 256) {
        keys[s] = -1;
        cnt[s] = 0;
    }
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * COMM_CHUNK;
    int slot[R], rank[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t i = base + r * 256 + threadIdx.x;
        slot[r] = -1;
        rank[r] = 0;
        if (i < n) {
            slot[r] = lds_slot(keys, Cp[i]);
            rank[r] = atomicAdd(&cnt[slot[r]], 1);
        }
    }
    __syncthreads();
    for (int s = threadIdx.x; s < 2 * COMM_CHUNK; s += 256) {
        const int c = keys[s];
        if (c >= 0) cnt[s] = coff[c] + atomicAdd(&cursor[c], cnt[s]);
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t i = base + r * 256 + threadIdx.x;
        if (i < n) members[cnt[slot[r]] + rank[r]] = (int32_t)i;
    }
}

__global__ void k_member_degrees(int32_t n, const int32_t *members, const int32_t *off,
                                 const int32_t *deg, int32_t *mdeg)
{
    for (int64_t m = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; m < n;
         m += (int64_t)gridDim.x * blockDim.x)
        mdeg[m] = len_of(off, deg, members[m]);
}

}  // namespace

// ---------------------------------------------------------------------------
int64_t scan_scratch_elems(int64_t n) { return (n + SCAN_CHUNK - 1) / SCAN_CHUNK + 1; }

template <typename TI, typename TO>
void launch_exclusive_scan(const TI *in, TO *out, int64_t n, int64_t *scratch,
                           unsigned long long *total, hipStream_t s)
{
    const int64_t nb = (n + SCAN_CHUNK - 1) / SCAN_CHUNK;
    if (nb > 0) k_scan_reduce<TI><<<(unsigned)nb, SCAN_THREADS, 0, s>>>(in, n, scratch);
    k_scan_partials<TO><<<1, SCAN_THREADS, 0, s>>>(scratch, nb, out, n, total);
    if (nb > 0) k_scan_apply<TI, TO><<<(unsigned)nb, SCAN_THREADS, 0, s>>>(in, out, n, scratch);
}
template void launch_exclusive_scan<int32_t, int32_t>(const int32_t *, int32_t *, int64_t,
                                                      int64_t *, unsigned long long *,
                                                      hipStream_t);
template void launch_exclusive_scan<int64_t, int64_t>(const int64_t *, int64_t *, int64_t,
                                                      int64_t *, unsigned long long *,
                                                      hipStream_t);

void launch_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s)
{
    if (n > 0) k_fill_i32<<<grid_for(n, 256), 256, 0, s>>>(p, v, n);
}

void launch_fill_u8(uint8_t *p, uint8_t v, int64_t n, hipStream_t s)
{
    if (n > 0) k_fill_u8<<<grid_for(n, 256), 256, 0, s>>>(p, v, n);
}

void launch_fill_bytes_zero(void *p, int64_t bytes, hipStream_t s)
{
    // bytes is a multiple of 8 for every caller (regions are 256-byte aligned)
    const int64_t n = bytes / 8;
    if (n > 0) k_zero_u64<<<grid_for(n, 256), 256, 0, s>>>((unsigned long long *)p, n);
}

__global__ void k_hub_active_counts(const uint8_t *act, const int32_t *start_s,
                                    const int32_t *start_p, int32_t hubs,
                                    const unsigned long long *total_s,
                                    const unsigned long long *total_p, int32_t *cs, int32_t *cp)
{
    for (int64_t h = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; h < hubs;
         h += (int64_t)gridDim.x * blockDim.x) {
        const bool on = act[h] != 0;
        const int32_t es = h + 1 < hubs ? start_s[h + 1] : (int32_t)*total_s;
        const int32_t ep = h + 1 < hubs ? start_p[h + 1] : (int32_t)*total_p;
        cs[h] = on ? es - start_s[h] : 0;
        cp[h] = on ? ep - start_p[h] : 0;
    }
}

// One thread per hub writes its ranges (at most HUB_MAXP partitions and a few
// hundred slices per hub).
__global__ void k_hub_active_fill(const uint8_t *act, const int32_t *start_s,
                                  const int32_t *start_p, int32_t hubs, const int32_t *cs,
                                  const int32_t *cp, const int32_t *os, const int32_t *op,
                                  int32_t *ls, int32_t *lp)
{
    for (int64_t h = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; h < hubs;
         h += (int64_t)gridDim.x * blockDim.x) {
        if (!act[h]) continue;
        for (int32_t i = 0; i < cs[h]; ++i) ls[os[h] + i] = start_s[h] + i;
        for (int32_t i = 0; i < cp[h]; ++i) lp[op[h] + i] = start_p[h] + i;
    }
}

void launch_hub_active_lists(const uint8_t *act, const int32_t *start_s, const int32_t *start_p,
                             int32_t hubs, const unsigned long long *total_s,
                             const unsigned long long *total_p, int32_t *cs, int32_t *cp,
                             int32_t *os, int32_t *op, unsigned long long *ns,
                             unsigned long long *np, int32_t *ls, int32_t *lp, int64_t *scratch,
                             hipStream_t s)
{
    if (hubs <= 0) return;
    k_hub_active_counts<<<grid_for(hubs, 256), 256, 0, s>>>(act, start_s, start_p, hubs, total_s,
                                                            total_p, cs, cp);
    launch_exclusive_scan<int32_t, int32_t>(cs, os, hubs, scratch, ns, s);
    launch_exclusive_scan<int32_t, int32_t>(cp, op, hubs, scratch, np, s);
    k_hub_active_fill<<<grid_for(hubs, 256), 256, 0, s>>>(act, start_s, start_p, hubs, cs, cp, os,
                                                          op, ls, lp);
}

void launch_owner_map(const int32_t *start, int32_t n, int32_t total, int32_t *owner, hipStream_t s)
{
    if (n > 0 && total > 0) k_owner_map<<<grid_for(total, 256), 256, 0, s>>>(start, n, total, owner);
}

void launch_iota(int32_t *p, int64_t n, hipStream_t s)
{
    if (n > 0) k_iota<<<grid_for(n, 256), 256, 0, s>>>(p, n);
}


void launch_validate(int32_t n, int64_t nnz, const int32_t *off, const int32_t *tgt,
                     const int32_t *w, int32_t *err, unsigned long long *W, int32_t *wmax,
                     hipStream_t s)
{
    const int64_t m = nnz > n ? nnz : n;
    k_validate<<<grid_for(m + 1, 256), 256, 0, s>>>(n, nnz, off, tgt, w, err, W, wmax);
}

void launch_max_u64(const int64_t *x, int32_t n, unsigned long long *out, hipStream_t s)
{
    if (n > 0) k_max_u64<<<grid_for(n, 256, 2048), 256, 0, s>>>(x, n, out);
}

void launch_init_vertices(int32_t n, int32_t *Cp, int32_t *size, uint8_t *fa, uint8_t *fb,
                          void *K, void *Sig, int sbytes, hipStream_t s)
{
    if (n > 0)
        k_init_vertices<<<grid_for(n, 256), 256, 0, s>>>(n, Cp, size, fa, fb, (unsigned char *)K,
                                                         (unsigned char *)Sig, sbytes);
}

int32_t bin_chunks(int32_t n) { return (int32_t)(((int64_t)n + BIN_CHUNK - 1) / BIN_CHUNK); }

void launch_bin_count(int32_t n, const int32_t *off, const int32_t *deg, int32_t lds_max,
                      int32_t *cnt, int32_t *boff, int64_t *scratch, int32_t *starts,
                      int32_t *maxlen, hipStream_t s)
{
    const int32_t G = bin_chunks(n);
    k_fill_i32<<<1, 64, 0, s>>>(maxlen, 0, NBINS);
    if (G > 0) k_bin_count<<<G, 256, 0, s>>>(n, off, deg, cnt, G, lds_max, maxlen);
    launch_exclusive_scan<int32_t, int32_t>(cnt, boff, (int64_t)NBINS * G, scratch, nullptr, s);
    k_bin_starts<<<1, 64, 0, s>>>(boff, G, starts);
}

void launch_bin_fill(int32_t n, const int32_t *off, const int32_t *deg, int32_t lds_max,
                     const int32_t *boff, int32_t *binorder, hipStream_t s)
{
    const int32_t G = bin_chunks(n);
    if (G > 0) k_bin_fill<<<G, 256, 0, s>>>(n, off, deg, boff, G, lds_max, binorder);
}


void launch_hub_move_sizes(const int32_t *binorder, int32_t hb, int32_t he, const int32_t *off,
                           const int32_t *deg, int stbytes, int64_t *ent, int32_t *slices,
                           int32_t *parts, hipStream_t s, int slice, int per_part)
{
    if (per_part <= 0) per_part = stbytes == 4 ? hub_part_pairs<int32_t>() : hub_part_pairs<int64_t>();
    if (he > hb)
        k_hub_move_sizes<<<grid_for(he - hb, 256), 256, 0, s>>>(binorder, hb, he, off, deg, stbytes,
                                                                ent, slices, parts, slice, per_part);
}

void launch_member_degrees(int32_t n, const int32_t *members, const int32_t *off,
                           const int32_t *deg, int32_t *mdeg, hipStream_t s)
{
    if (n > 0) k_member_degrees<<<grid_for(n, 256), 256, 0, s>>>(n, members, off, deg, mdeg);
}

template <class C>
void launch_row_reduce(int bin, int op, const RowArgs<C> &a, hipStream_t s)
{
    if (a.count <= 0) return;
    if (bin == NBINS - 1 && a.hslice) {
        if (op == 0)
            k_row_reduce_hub<C, 0><<<2048, 256, 0, s>>>(a, a.hslice, a.nslices);
        else
            k_row_reduce_hub<C, 1><<<2048, 256, 0, s>>>(a, a.hslice, a.nslices);
        return;
    }
    const int rows_per_block[NBINS] = {32, 8, 4, 4, 1, 1, 1};
    const int grid = grid_for(a.count, rows_per_block[bin], 4096);
#define LV_ROW(G)                                                            \
    do {                                                                     \
        if (op == 0)                                                         \
            k_row_reduce<C, G, 0><<<grid, 256, 0, s>>>(a);                   \
        else                                                                 \
            k_row_reduce<C, G, 1><<<grid, 256, 0, s>>>(a);                   \
    } while (0)
    switch (bin) {
    case 0: LV_ROW(8); break;
    case 1: LV_ROW(32); break;
    case 2:
    case 3: LV_ROW(64); break;
    default: LV_ROW(256); break;
    }
#undef LV_ROW
}
template void launch_row_reduce<CfgNarrow>(int, int, const RowArgs<CfgNarrow> &, hipStream_t);
template void launch_row_reduce<CfgWideIn>(int, int, const RowArgs<CfgWideIn> &, hipStream_t);
template void launch_row_reduce<CfgWide>(int, int, const RowArgs<CfgWide> &, hipStream_t);
template void launch_row_reduce<CfgWideIn32>(int, int, const RowArgs<CfgWideIn32> &, hipStream_t);

template <typename ST>
void launch_sum_squares(const ST *Sig, int32_t n, unsigned long long *acc, hipStream_t s)
{
    if (n > 0) k_sum_squares<ST><<<grid_for(n, 256, 2048), 256, 0, s>>>(Sig, n, acc);
}
template void launch_sum_squares<int32_t>(const int32_t *, int32_t, unsigned long long *,
                                          hipStream_t);
template void launch_sum_squares<int64_t>(const int64_t *, int32_t, unsigned long long *,
                                          hipStream_t);

void launch_compact(const CompactArgs &a, hipStream_t s)
{
    const int32_t len = a.order ? a.q1 - a.q0 : a.nb;
    if (len > 0) k_compact<<<bin_chunks(len), 256, 0, s>>>(a);
}

void launch_compact_keys(const CompactArgs &a, const int32_t *koff, int32_t nkeys, int32_t *kact,
                         int32_t *klist, unsigned long long *processed, hipStream_t s)
{
    if (a.nb > 0 && nkeys > 0)
        k_compact_keys<<<grid_for(a.nb, 256, 4096), 256, 0, s>>>(a, koff, nkeys, kact, klist,
                                                                 processed);
}

template <typename ST>
void launch_apply(int32_t *mv_c, int32_t n, int32_t *Cp, const ST *K, ST *Sig, int32_t *size,
                  const int32_t *done, hipStream_t s)
{
    if (n <= 0) return;
    const int64_t chunks = ((int64_t)n + APPLY_CHUNK - 1) / APPLY_CHUNK;
    const int grid = (int)std::min<int64_t>(chunks, 2048);
    k_apply<ST><<<grid, 256, 0, s>>>(mv_c, n, Cp, K, Sig, size, done);
}
template void launch_apply<int32_t>(int32_t *, int32_t, int32_t *, const int32_t *, int32_t *,
                                    int32_t *, const int32_t *, hipStream_t);
template void launch_apply<int64_t>(int32_t *, int32_t, int32_t *, const int64_t *, int64_t *,
                                    int32_t *, const int32_t *, hipStream_t);

void launch_round_end(DevScalars *sc, int it, hipStream_t s)
{
    k_round_end<<<1, 64, 0, s>>>(sc, it);
}

void launch_iter_end(DevScalars *sc, int it, double tau, hipStream_t s, const BatchArgs *b)
{
    if (b && b->gid) k_batch_iter_end<<<grid_for(b->G, 256), 256, 0, s>>>(*b, sc, tau);
    k_iter_end<<<1, 64, 0, s>>>(sc, it, tau, b && b->gid ? 1 : 0);
}

void launch_warm_check(int32_t n, const int32_t *labels, const int32_t *gid, const int32_t *gvb,
                       int32_t *err, hipStream_t s)
{
    if (n > 0) k_warm_check<<<grid_for(n, 256), 256, 0, s>>>(n, labels, gid, gvb, err);
}

template <typename ST>
void launch_warm_labels(int32_t n, const int32_t *labels, const ST *K, int32_t *Cp, ST *Sig,
                        int32_t *size, hipStream_t s)
{
    if (n > 0) k_warm_labels<ST><<<grid_for(n, 256), 256, 0, s>>>(n, labels, K, Cp, Sig, size);
}
template void launch_warm_labels<int32_t>(int32_t, const int32_t *, const int32_t *, int32_t *,
                                          int32_t *, int32_t *, hipStream_t);
template void launch_warm_labels<int64_t>(int32_t, const int32_t *, const int64_t *, int32_t *,
                                          int64_t *, int32_t *, hipStream_t);

void launch_batch_gid(int32_t n, const int32_t *gvb, int32_t G, int32_t *gid, hipStream_t s)
{
    if (n > 0) k_batch_gid<<<grid_for(n, 256), 256, 0, s>>>(n, gvb, G, gid);
}

void launch_batch_check(int32_t n, const int32_t *off, const int32_t *tgt, const int32_t *w,
                        const int32_t *gid, const int32_t *gvb, int64_t *gW, int32_t *err,
                        hipStream_t s)
{
    if (n > 0) k_batch_check<<<grid_for(n, 256), 256, 0, s>>>(n, off, tgt, w, gid, gvb, gW, err);
}

void launch_batch_reset(const BatchArgs &b, int32_t *gcomm, hipStream_t s)
{
    if (b.G > 0) k_batch_reset<<<grid_for(b.G, 256), 256, 0, s>>>(b, gcomm);
}

void launch_batch_mark_small(const BatchArgs &b, int32_t max_n, hipStream_t s)
{
    if (b.G > 0) k_batch_mark_small<<<grid_for(b.G, 256), 256, 0, s>>>(b, max_n);
}

void launch_batch_pass_begin(const BatchArgs &b, hipStream_t s)
{
    if (b.G > 0) k_batch_pass_begin<<<grid_for(b.G, 256), 256, 0, s>>>(b);
}

void launch_batch_agg_test(const BatchArgs &b, const int32_t *idmap, int32_t n, int32_t nc,
                           double aggtol, int32_t *gvb_next, int32_t *gcomm, DevScalars *sc,
                           hipStream_t s)
{
    if (b.G > 0)
        k_batch_agg_test<<<grid_for(b.G, 256), 256, 0, s>>>(b, idmap, n, nc, aggtol, gvb_next,
                                                             gcomm, sc);
}

void launch_batch_gid_next(int32_t n, const int32_t *labels, const int32_t *gid, int32_t *gid_next,
                           hipStream_t s)
{
    if (n > 0) k_batch_gid_next<<<grid_for(n, 256), 256, 0, s>>>(n, labels, gid, gid_next);
}

template <typename WT, typename ST>
void launch_batch_modularity(int32_t n, const int32_t *off, const int32_t *deg, const int32_t *tgt,
                             const WT *w, const int32_t *labels, const ST *Sig, const int32_t *gid,
                             unsigned long long *gsig, unsigned long long *gs2, hipStream_t s)
{
    if (n <= 0) return;
    k_batch_sigma<WT><<<grid_for((int64_t)n * 64, 256), 256, 0, s>>>(n, off, deg, tgt, w, labels,
                                                                     gid, gsig);
    k_batch_s2<ST><<<grid_for(n, 256), 256, 0, s>>>(n, Sig, gid, gs2);
}
template void launch_batch_modularity<int32_t, int32_t>(int32_t, const int32_t *, const int32_t *,
                                                        const int32_t *, const int32_t *,
                                                        const int32_t *, const int32_t *,
                                                        const int32_t *, unsigned long long *,
                                                        unsigned long long *, hipStream_t);
template void launch_batch_modularity<int32_t, int64_t>(int32_t, const int32_t *, const int32_t *,
                                                        const int32_t *, const int32_t *,
                                                        const int32_t *, const int64_t *,
                                                        const int32_t *, unsigned long long *,
                                                        unsigned long long *, hipStream_t);
template void launch_batch_modularity<int64_t, int64_t>(int32_t, const int32_t *, const int32_t *,
                                                        const int32_t *, const int64_t *,
                                                        const int32_t *, const int64_t *,
                                                        const int32_t *, unsigned long long *,
                                                        unsigned long long *, hipStream_t);

void launch_mark_used(int32_t n, const int32_t *labels, int32_t *used, hipStream_t s)
{
    if (n > 0) k_mark_used<<<grid_for(n, 256), 256, 0, s>>>(n, labels, used);
}

void launch_relabel(int32_t n, int32_t *labels, const int32_t *map, hipStream_t s)
{
    if (n > 0) k_relabel<<<grid_for(n, 256), 256, 0, s>>>(n, labels, map);
}

void launch_comm_count(int32_t n, const int32_t *Cp, const int32_t *off, const int32_t *deg,
                       int32_t *ccount, int32_t *ctot, hipStream_t s)
{
    if (n > 0)
        k_comm_count<<<(unsigned)(((int64_t)n + COMM_CHUNK - 1) / COMM_CHUNK), 256, 0, s>>>(
            n, Cp, off, deg, ccount, ctot);
}

void launch_comm_fill(int32_t n, const int32_t *Cp, const int32_t *coff, int32_t *cursor,
                      int32_t *members, hipStream_t s)
{
    if (n > 0)
        k_comm_fill<<<(unsigned)(((int64_t)n + COMM_CHUNK - 1) / COMM_CHUNK), 256, 0, s>>>(
            n, Cp, coff, cursor, members);
}

}  // namespace lv
