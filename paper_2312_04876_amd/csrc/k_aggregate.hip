// Aggregation kernels (Alg. 3): for every community c of one bin (binned by
// the total degree of its members), scan the rows of all members into a
// community table keyed by the neighbour's community (scanCommunities with
// the self-loop kept) and write the table out as row c of the holey
// super-vertex CSR, whose row capacity is the total member degree.
//
// The members' rows are walked as one flattened sequence: a chunk of G
// members is loaded, their row lengths are prefix-summed, and every lane
// takes entries t = lane, lane + G, ... finding its member by binary search
// over the prefix sums, so short rows do not leave lanes idle.
#include "kernels.h"

namespace lv {

namespace {

template <typename ST>
__device__ inline void lds_add(int32_t *keys, ST *vals, int log2s, int32_t c, ST w)
{
    const uint32_t mask = (1u << log2s) - 1u;
    uint32_t h = hash32((uint32_t)c) >> (32 - log2s);
    for (;;) {
        const int32_t k = __hip_atomic_load(&keys[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (k == c) {
            atomic_add_t<ST>(&vals[h], w);
            return;
        }
        if (k < 0) {
            const int32_t old = atomicCAS(&keys[h], -1, c);
            if (old < 0 || old == c) {
                atomic_add_t<ST>(&vals[h], w);
                return;
            }
        }
        h = (h + 1) & mask;
    }
}

// lds_add over a table of any size ns (not only a power of two): the start slot
// scales the hash into [0, ns).
template <typename ST>
__device__ inline void lds_add_n(int32_t *keys, ST *vals, uint32_t ns, int32_t c, ST w)
{
    uint32_t h = (uint32_t)(((uint64_t)hash32((uint32_t)c) * ns) >> 32);
    for (;;) {
        const int32_t k = __hip_atomic_load(&keys[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (k == c) {
            atomic_add_t<ST>(&vals[h], w);
            return;
        }
        if (k < 0) {
            const int32_t old = atomicCAS(&keys[h], -1, c);
            if (old < 0 || old == c) {
                atomic_add_t<ST>(&vals[h], w);
                return;
            }
        }
        h = h + 1 == ns ? 0 : h + 1;
    }
}

// Position of the member owning flattened entry t: the first lane whose
// inclusive prefix exceeds t.
__device__ inline int owner_of(const int32_t *incl, int n, int t)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (incl[mid] > t)
            hi = mid;
        else
            lo = mid + 1;
    }
    return lo;
}

// Entries folded per lane at a time: their targets, weights and target
// communities are loaded together, so several dependent gathers are in flight
// per lane instead of one (more in the hub windows, whose large LDS tables
// leave few workgroups per CU).
constexpr int AGG_U = 4;
constexpr int AGG_HUB_U = 16;

// For CSR entries e[] (-1 for none): add(C'[target], weight) for each.
template <class C, typename VT, int U, class F>
__device__ inline void fold_entries(const AggArgs<C> &a, const int (&e)[U], F add)
{
    int j[U], c[U];
    VT w[U];
#pragma unroll
    for (int u = 0; u < U; ++u) j[u] = e[u] >= 0 ? a.tgt[e[u]] : -1;
#pragma unroll
    for (int u = 0; u < U; ++u) w[u] = e[u] >= 0 ? (VT)a.w[e[u]] : (VT)0;
#pragma unroll
    for (int u = 0; u < U; ++u) c[u] = j[u] >= 0 ? a.Cp[j[u]] : -1;
#pragma unroll
    for (int u = 0; u < U; ++u)
        if (c[u] >= 0) add(c[u], w[u]);
}

// Inclusive prefix sum of x over the G lanes of a group (G <= 64).
template <int G>
__device__ inline int group_inclusive_scan(int x, int gl)
{
    for (int d = 1; d < G; d <<= 1) {
        const int y = __shfl_up(x, d, G);
        if (gl >= d) x += y;
    }
    return x;
}

// Bins 0-3: G lanes per community with a private LDS table of 2^LOG2S slots.
template <class C, int G, int LOG2S>
__global__ __launch_bounds__(256) void k_agg_wave(AggArgs<C> a)
{
    typedef typename C::ST ST;
    constexpr int S = 1 << LOG2S;
    constexpr int GPW = 64 / G;
    constexpr int NG = 4 * GPW;
    __shared__ ST s_vals[NG * S];
    __shared__ int32_t s_keys[NG * S];
    __shared__ int32_t s_incl[NG * G];
    __shared__ int32_t s_rb[NG * G];
    __shared__ int32_t s_cnt[NG];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int grp = lane / G, gl = lane % G;
    const int gid = wave * GPW + grp;
    int32_t *keys = s_keys + gid * S;
    ST *vals = s_vals + gid * S;
    int32_t *incl = s_incl + gid * G;
    int32_t *rbs = s_rb + gid * G;
    for (int s = gl; s < S; s += G) {
        keys[s] = -1;
        vals[s] = 0;
    }
    if (gl == 0) s_cnt[gid] = 0;
    wave_sync();
    unsigned long long nc_ = 0, nm_ = 0, ne_ = 0, no_ = 0;
    const int stride = gridDim.x * NG;
    for (int base = (blockIdx.x * 4 + wave) * GPW; base < a.count; base += stride) {
        const int idx = base + grp;
        const bool has = idx < a.count;
        const int c = has ? a.cbinorder[a.begin + idx] : 0;
        const int mb = has ? a.coff[c] : 0;
        const int me = has ? a.coff[c + 1] : 0;
        for (int m0 = mb; m0 < me; m0 += G) {
            const int mi = m0 + gl;
            int rl = 0, rb = 0;
            if (mi < me) {
                const int u = a.members[mi];
                rb = a.off[u];
                rl = row_len(a.off, a.deg, u);
            }
            const int inc = group_inclusive_scan<G>(rl, gl);
            const int total = __shfl(inc, G - 1, G);
            incl[gl] = inc;
            rbs[gl] = rb;
            wave_sync();
            for (int t0 = gl; t0 < total; t0 += AGG_U * G) {
                int e[AGG_U];
#pragma unroll
                for (int u = 0; u < AGG_U; ++u) {
                    const int t = t0 + u * G;
                    const int L = t < total ? owner_of(incl, G, t) : 0;
                    e[u] = t < total ? rbs[L] + (t - (L ? incl[L - 1] : 0)) : -1;
                }
                fold_entries<C, ST, AGG_U>(a, e,
                                           [&](int32_t c, ST w) { lds_add<ST>(keys, vals, LOG2S, c, w); });
            }
            ne_ += total > gl ? (total - gl + G - 1) / G : 0;
            nm_ += mi < me ? 1 : 0;
            wave_sync();
        }
        const int ybeg = has ? a.yoff[c] : 0;
        for (int s = gl; s < S; s += G) {
            const int k = keys[s];
            if (k >= 0) {
                const int pos = atomicAdd(&s_cnt[gid], 1);
                a.ytgt[ybeg + pos] = k;
                a.yw[ybeg + pos] = vals[s];
                keys[s] = -1;
                vals[s] = 0;
            }
        }
        wave_sync();
        if (has && gl == 0) {
            const int n_out = s_cnt[gid];
            a.ydeg[c] = n_out;
            s_cnt[gid] = 0;
            no_ += (unsigned long long)n_out;
            ++nc_;
        }
        wave_sync();
    }
    nc_ = wave_sum_u64(nc_);
    nm_ = wave_sum_u64(nm_);
    ne_ = wave_sum_u64(ne_);
    no_ = wave_sum_u64(no_);
    if (lane == 0) {
        if (nc_) atomicAdd(&a.work[0], nc_);
        if (nm_) atomicAdd(&a.work[1], nm_);
        if (ne_) atomicAdd(&a.work[2], ne_);
        if (no_) atomicAdd(&a.work[3], no_);
    }
}

// Exclusive scan of one int per thread across the 256-thread block (total in *tot).
__device__ inline int block_scan_int(int x, int *wsum, int *tot)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int inc = x;
    for (int d = 1; d < 64; d <<= 1) {
        const int y = __shfl_up(inc, d, 64);
        if (lane >= d) inc += y;
    }
    if (lane == 63) wsum[wave] = inc;
    __syncthreads();
    int wb = 0, t = 0;
    for (int k = 0; k < 4; ++k) {
        if (k < wave) wb += wsum[k];
        t += wsum[k];
    }
    *tot = t;
    return wb + inc;  // inclusive
}

// Bins 4-5: one workgroup per community with an LDS table (dynamic shared
// memory of 2^log2s_max slots) of block_log2s(total member degree) slots.
template <class C>
__global__ __launch_bounds__(256) void k_agg_block(AggArgs<C> a, int log2s_max)
{
    typedef typename C::ST ST;
    extern __shared__ __align__(16) unsigned char smem[];
    const int S = 1 << log2s_max;
    ST *s_vals = (ST *)smem;
    int32_t *s_keys = (int32_t *)(smem + (size_t)S * sizeof(ST));
    __shared__ int32_t s_incl[256];
    __shared__ int32_t s_rb[256];
    __shared__ int32_t wsum[4];
    __shared__ int32_t s_cnt;
    for (int s = threadIdx.x; s < S; s += 256) {
        s_keys[s] = -1;
        s_vals[s] = 0;
    }
    if (threadIdx.x == 0) s_cnt = 0;
    __syncthreads();
    unsigned long long nc_ = 0, nm_ = 0, ne_ = 0, no_ = 0;
    for (int idx = blockIdx.x; idx < a.count; idx += gridDim.x) {
        const int c = a.cbinorder[a.begin + idx];
        const int mb = a.coff[c], me = a.coff[c + 1];
        const int log2s = block_log2s(a.yoff[c + 1] - a.yoff[c]);
        for (int m0 = mb; m0 < me; m0 += 256) {
            const int mi = m0 + threadIdx.x;
            int rl = 0, rb = 0;
            if (mi < me) {
                const int u = a.members[mi];
                rb = a.off[u];
                rl = row_len(a.off, a.deg, u);
                ++nm_;
            }
            int total;
            const int inc = block_scan_int(rl, wsum, &total);
            s_incl[threadIdx.x] = inc;
            s_rb[threadIdx.x] = rb;
            __syncthreads();
            for (int t0 = threadIdx.x; t0 < total; t0 += AGG_U * 256) {
                int e[AGG_U];
#pragma unroll
                for (int u = 0; u < AGG_U; ++u) {
                    const int t = t0 + u * 256;
                    const int L = t < total ? owner_of(s_incl, 256, t) : 0;
                    e[u] = t < total ? s_rb[L] + (t - (L ? s_incl[L - 1] : 0)) : -1;
                    ne_ += t < total ? 1 : 0;
                }
                fold_entries<C, ST, AGG_U>(
                    a, e, [&](int32_t c, ST w) { lds_add<ST>(s_keys, s_vals, log2s, c, w); });
            }
            __syncthreads();
        }
        const int ybeg = a.yoff[c];
        for (int s = threadIdx.x; s < (1 << log2s); s += 256) {
            const int k = s_keys[s];
            if (k >= 0) {
                const int pos = atomicAdd(&s_cnt, 1);
                a.ytgt[ybeg + pos] = k;
                a.yw[ybeg + pos] = s_vals[s];
                s_keys[s] = -1;
                s_vals[s] = 0;
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            a.ydeg[c] = s_cnt;
            no_ += (unsigned long long)s_cnt;
            s_cnt = 0;
            ++nc_;
        }
        __syncthreads();
    }
    nc_ = wave_sum_u64(nc_);
    nm_ = wave_sum_u64(nm_);
    ne_ = wave_sum_u64(ne_);
    no_ = wave_sum_u64(no_);
    if ((threadIdx.x & 63) == 0) {
        if (nc_) atomicAdd(&a.work[0], nc_);
        if (nm_) atomicAdd(&a.work[1], nm_);
        if (ne_) atomicAdd(&a.work[2], ne_);
        if (no_) atomicAdd(&a.work[3], no_);
    }
}

// Hub communities (bin 6) are folded like hub rows in local moving: the
// flattened member rows of each community, folded per window, are
// counting-sorted into hash partitions, and one workgroup per partition folds
// it in LDS and appends its keys to the community's row.

// Walks the flattened entries t in [w0, w1) of community c's member rows
// (members m0..me, m0 the first whose row reaches past w0; flattened offsets
// mpre - base): f(e) for AGG_HUB_U CSR entries
// e[] per thread at a time (-1 past the end).  All threads of the workgroup
// call this.
struct Window {
    int32_t start[257];
    int32_t rb[256];
};

template <class C, class F>
__device__ inline void walk_window(const AggArgs<C> &a, Window &W, int m0, int me, int base, int w0,
                                   int w1, unsigned long long *nm_, F f)
{
    int m = m0;
    for (;;) {
        const int cnt = min(256, me - m);
        if ((int)threadIdx.x < cnt) {
            const int u = a.members[m + threadIdx.x];
            W.rb[threadIdx.x] = a.off[u];
            const int st = a.mpre[m + threadIdx.x] - base;
            W.start[threadIdx.x] = st;
            if (nm_ && st >= w0 && st < w1 && a.mpre[m + threadIdx.x + 1] - base > st) ++*nm_;
        }
        if (threadIdx.x == 0) W.start[cnt] = a.mpre[m + cnt] - base;
        __syncthreads();
        const int t_lo = max(w0, W.start[0]);
        const int t_hi = min(w1, W.start[cnt]);
        for (int t0 = t_lo + (int)threadIdx.x; t0 < t_hi; t0 += AGG_HUB_U * 256) {
            int e[AGG_HUB_U];
#pragma unroll
            for (int u = 0; u < AGG_HUB_U; ++u) {
                const int t = t0 + u * 256;
                const int L = t < t_hi ? owner_slice(W.start, cnt, t) : 0;
                e[u] = t < t_hi ? W.rb[L] + (t - W.start[L]) : -1;
            }
            f(e);
        }
        const bool more = W.start[cnt] < w1 && m + cnt < me;
        __syncthreads();
        if (!more) break;
        m += cnt;
    }
}

// Sorting window k of the hub bin: community idx (in the bin), c, members,
// flattened range [w0, w1), partitions.
template <class C>
__device__ inline void agg_window(const AggArgs<C> &a, int nh, int k, int *idx, int *c, int *mb,
                                  int *me, int *base, int *w0, int *w1, int *parts, int *gp0)
{
    *idx = a.sown[k];
    *c = a.cbinorder[a.begin + *idx];
    *mb = a.coff[*c];
    *me = a.coff[*c + 1];
    *base = a.mpre[*mb];
    const int tot = a.mpre[*me] - *base;
    *w0 = (k - a.cslice[*idx]) * AGG_PSLICE;
    *w1 = min(*w0 + AGG_PSLICE, tot);
    *gp0 = a.tslice[*idx];
    *parts = (*idx + 1 < nh ? a.tslice[*idx + 1] : (int)*a.tslices) - *gp0;
}

// Step 1: one workgroup per AGG_PSLICE flattened entries of a hub community
// folds its window in an LDS table (dynamic shared memory of AGG_FOLD_SLOTS
// slots), stages the window's distinct (community, weight) pairs at the
// window's flattened offset (count in wcnt), and adds their count per
// partition into pcount.  Folding first keeps a community's many entries
// into the same neighbour (its internal edges above all) to one pair per
// window.  VT is the table's value type: 32-bit whenever AGG_PSLICE times the
// largest weight stays below 2^31 (no window sum can overflow), which halves
// the table of 64-bit configurations and doubles the workgroups per CU.
template <class C, class VT>
__global__ __launch_bounds__(256) void k_agg_hub_count(AggArgs<C> a, int32_t nh)
{
    typedef typename C::ST ST;
    constexpr int S = AGG_FOLD_SLOTS;
    extern __shared__ __align__(16) unsigned char smem[];
    VT *vals = (VT *)smem;
    int32_t *keys = (int32_t *)(smem + (size_t)S * sizeof(VT));
    __shared__ Window W;
    __shared__ int32_t hist[HUB_MAXP];
    __shared__ int s_n;
    int idx, c, mb, me, base, w0, w1, parts, gp0;
    agg_window(a, nh, (int)blockIdx.x, &idx, &c, &mb, &me, &base, &w0, &w1, &parts, &gp0);
    for (int p = threadIdx.x; p < parts; p += 256) hist[p] = 0;
    for (int q = threadIdx.x; q < S; q += 256) {
        keys[q] = -1;
        vals[q] = 0;
    }
    if (threadIdx.x == 0) s_n = 0;
    unsigned long long ne_ = 0, nm_ = 0;
    walk_window(a, W, a.wm0[blockIdx.x], me, base, w0, w1, &nm_, [&](const int (&e)[AGG_HUB_U]) {
        fold_entries<C, VT, AGG_HUB_U>(a, e, [&](int32_t c, VT w) {
            lds_add_n<VT>(keys, vals, (uint32_t)S, c, w);
            ++ne_;
        });
    });
    int32_t *sk = a.hstage + base + w0;
    ST *sw = a.hstage_w + base + w0;
    for (int q = threadIdx.x; q < S; q += 256) {
        const int32_t key = keys[q];
        if (key < 0) continue;
        const int i = atomicAdd(&s_n, 1);
        sk[i] = key;
        sw[i] = (ST)vals[q];
        atomicAdd(&hist[part_of(key, parts)], 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) a.wcnt[blockIdx.x] = s_n;
    for (int p = threadIdx.x; p < parts; p += 256)
        if (hist[p]) atomicAdd(&a.pcount[gp0 + p], hist[p]);
    nm_ = wave_sum_u64(nm_);
    ne_ = wave_sum_u64(ne_);
    if ((threadIdx.x & 63) == 0) {
        if (nm_) atomicAdd(&a.work[1], nm_);
        if (ne_) atomicAdd(&a.work[2], ne_);
    }
}

// Step 2 (after the exclusive scan pcount -> poff): the same workgroups
// reserve room in every partition and move their staged pairs there.
template <class C>
__global__ __launch_bounds__(256) void k_agg_hub_fill(AggArgs<C> a, int32_t nh)
{
    typedef typename C::ST ST;
    __shared__ int32_t hist[HUB_MAXP];
    int idx, c, mb, me, base, w0, w1, parts, gp0;
    agg_window(a, nh, (int)blockIdx.x, &idx, &c, &mb, &me, &base, &w0, &w1, &parts, &gp0);
    for (int p = threadIdx.x; p < parts; p += 256) hist[p] = 0;
    __syncthreads();
    const int n = a.wcnt[blockIdx.x];
    const int32_t *sk = a.hstage + base + w0;
    const ST *sw = a.hstage_w + base + w0;
    for (int i = threadIdx.x; i < n; i += 256) atomicAdd(&hist[part_of(sk[i], parts)], 1);
    __syncthreads();
    for (int p = threadIdx.x; p < parts; p += 256)
        if (hist[p]) hist[p] = a.poff[gp0 + p] + atomicAdd(&a.pcur[gp0 + p], hist[p]);
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += 256) {
        const int32_t key = sk[i];
        const int pos = atomicAdd(&hist[part_of(key, parts)], 1);
        a.pk[pos] = key;
        a.pw[pos] = sw[i];
    }
}

// Step 3: one workgroup per partition folds its pairs into an LDS table of
// 2^hub_plog2 slots and appends the keys to row c (position from an atomic on
// ydeg[c], zero on entry).  A partition with more distinct keys than 3/4 of
// the slots is folded in passes over halved ranges of a third key hash.
template <class C>
__global__ __launch_bounds__(256) void k_agg_hub_part(AggArgs<C> a, int32_t nh)
{
    typedef typename C::ST ST;
    constexpr int LOG2S = hub_plog2<ST>();
    constexpr int S = 1 << LOG2S;
    __shared__ ST vals[S];
    __shared__ int32_t keys[S];
    __shared__ uint64_t st_lo[40], st_hi[40];
    __shared__ int s_sp, s_cnt, s_over, s_pos, s_base;
    const int gp = (int)blockIdx.x;
    const int idx = a.pown[gp];
    const int c = a.cbinorder[a.begin + idx];
    const int pb = a.poff[gp], pn = a.pcount[gp];
    // table of 2^lg slots: twice the pairs (so no overflow) when that fits
    int lg = 8;
    while (lg < LOG2S && (1 << lg) < 2 * pn) ++lg;
    const int Su = 1 << lg, capu = 3 * (Su / 4);
    for (int s = threadIdx.x; s < Su; s += 256) {
        keys[s] = -1;
        vals[s] = 0;
    }
    if (threadIdx.x == 0) {
        st_lo[0] = 0;
        st_hi[0] = 1ull << 32;
        s_sp = 1;
    }
    unsigned long long emitted = 0;
    for (;;) {
        __syncthreads();
        const int sp = s_sp;
        if (sp == 0) break;
        const uint64_t lo = st_lo[sp - 1], hi = st_hi[sp - 1];
        __syncthreads();
        if (threadIdx.x == 0) {
            s_sp = sp - 1;
            s_cnt = 0;
            s_over = 0;
            s_pos = 0;
        }
        __syncthreads();
        const bool all = lo == 0 && hi == (1ull << 32);
        for (int i0 = threadIdx.x; i0 < pn; i0 += 4 * 256) {
            // four pairs per thread loaded together, then inserted
            int32_t kq[4];
            ST wq[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) kq[q] = i0 + q * 256 < pn ? a.pk[pb + i0 + q * 256] : -1;
#pragma unroll
            for (int q = 0; q < 4; ++q) wq[q] = kq[q] >= 0 ? a.pw[pb + i0 + q * 256] : (ST)0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int32_t key = kq[q];
                if (key < 0) continue;
                if (!all) {
                    const uint64_t x = hash32(mix32((uint32_t)key) ^ 0x5bd1e995u);
                    if (x < lo || x >= hi) continue;
                }
                if (!lds_insert_capped<ST>(keys, vals, lg, key, wq[q], &s_cnt, capu)) s_over = 1;
            }
        }
        __syncthreads();
        if (s_over) {
            for (int s = threadIdx.x; s < Su; s += 256) {
                keys[s] = -1;
                vals[s] = 0;
            }
            if (threadIdx.x == 0) {
                const uint64_t mid = lo + (hi - lo) / 2;
                st_lo[s_sp] = lo;
                st_hi[s_sp] = mid;
                st_lo[s_sp + 1] = mid;
                st_hi[s_sp + 1] = hi;
                s_sp += 2;
            }
            continue;
        }
        if (threadIdx.x == 0) s_base = s_cnt ? atomicAdd(&a.ydeg[c], s_cnt) : 0;
        __syncthreads();
        const int64_t ybeg = (int64_t)a.yoff[c] + s_base;
        for (int s = threadIdx.x; s < Su; s += 256) {
            const int32_t key = keys[s];
            if (key < 0) continue;
            const int q = atomicAdd(&s_pos, 1);
            a.ytgt[ybeg + q] = key;
            a.yw[ybeg + q] = vals[s];
            keys[s] = -1;
            vals[s] = 0;
            ++emitted;
        }
    }
    emitted = wave_sum_u64(emitted);
    if ((threadIdx.x & 63) == 0 && emitted) atomicAdd(&a.work[3], emitted);
    if (threadIdx.x == 0 && gp == a.tslice[idx]) atomicAdd(&a.work[0], 1ull);
}

// First member of each window (one thread per window): the first member of its
// community whose row ends after the window's first flattened entry.
template <class C>
__global__ __launch_bounds__(256) void k_window_first_member(AggArgs<C> a, int32_t nh, int32_t windows)
{
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < windows; k += gridDim.x * blockDim.x) {
        int idx, c, mb, me, base, w0, w1, parts, gp0;
        agg_window(a, nh, k, &idx, &c, &mb, &me, &base, &w0, &w1, &parts, &gp0);
        int lo = mb, hi = me - 1;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (a.mpre[mid + 1] - base > w0)
                hi = mid;
            else
                lo = mid + 1;
        }
        a.wm0[k] = lo;
    }
}

inline int agg_grid(int count, int per_block)
{
    int64_t g = ((int64_t)count + per_block - 1) / per_block;
    if (g > 4096) g = 4096;
    if (g < 1) g = 1;
    return (int)g;
}

}  // namespace

template <class C>
void launch_aggregate(int bin, const AggArgs<C> &a, int log2s_max, hipStream_t s)
{
    if (a.count <= 0) return;
    switch (bin) {
    // few lanes per community keep many small communities in flight (measured
    // against 8, 32 and 64 lanes for bins 0-2); bin 2 with 8-byte sums takes 16
    // lanes so that its tables leave room for more than one workgroup per CU
    case 0: k_agg_wave<C, 4, 4><<<agg_grid(a.count, 64), 256, 0, s>>>(a); break;
    case 1: k_agg_wave<C, 4, 6><<<agg_grid(a.count, 64), 256, 0, s>>>(a); break;
    case 2:
        if (sizeof(typename C::ST) > 4)
            k_agg_wave<C, 16, 8><<<agg_grid(a.count, 16), 256, 0, s>>>(a);
        else
            k_agg_wave<C, 8, 8><<<agg_grid(a.count, 32), 256, 0, s>>>(a);
        break;
    case 3: k_agg_wave<C, 64, 10><<<agg_grid(a.count, 4), 256, 0, s>>>(a); break;
    case 4:
    case 5: {
        const size_t bytes = ((size_t)1 << log2s_max) * (sizeof(typename C::ST) + 4);
        if (bytes > 65536) {
            // raise the dynamic-LDS limit of this kernel to what the launch asks for;
            // a failure shows up as a launch error at the caller's check
            if (hipFuncSetAttribute((const void *)&k_agg_block<C>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) !=
                hipSuccess)
                (void)hipGetLastError();
        }
        k_agg_block<C><<<agg_grid(a.count, 1), 256, bytes, s>>>(a, log2s_max);
        break;
    }
    default: break;  // hub communities: launch_aggregate_hub
    }
}

template <class C, class VT>
void launch_agg_hub_count(const AggArgs<C> &a, int32_t sort_slices, hipStream_t s)
{
    const size_t bytes = (size_t)AGG_FOLD_SLOTS * (sizeof(VT) + 4);
    if (bytes > 32768) {
        // raise the dynamic-LDS limit of this kernel to what the launch asks for; a
        // failure shows up as a launch error at the caller's check
        if (hipFuncSetAttribute((const void *)&k_agg_hub_count<C, VT>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess)
            (void)hipGetLastError();
    }
    k_agg_hub_count<C, VT><<<sort_slices, 256, bytes, s>>>(a, a.count);
}

template <class C>
void launch_aggregate_hub(const AggArgs<C> &a, int32_t sort_slices, int32_t parts,
                          int64_t wmax, int64_t *scratch, hipStream_t s)
{
    if (a.count <= 0 || sort_slices <= 0 || parts <= 0) return;
    typedef typename C::ST ST;
    launch_fill_bytes_zero(a.pcount, 2 * (int64_t)parts * sizeof(int32_t), s);  // pcount, pcur
    launch_owner_map(a.cslice, a.count, sort_slices, a.sown, s);
    launch_owner_map(a.tslice, a.count, parts, a.pown, s);
    k_window_first_member<C><<<(sort_slices + 255) / 256, 256, 0, s>>>(a, a.count, sort_slices);
    if (sizeof(ST) > 4 && wmax > 0 && wmax * AGG_PSLICE < ((int64_t)1 << 31))
        launch_agg_hub_count<C, int32_t>(a, sort_slices, s);
    else
        launch_agg_hub_count<C, ST>(a, sort_slices, s);
    launch_exclusive_scan<int32_t, int32_t>(a.pcount, a.poff, parts, scratch, nullptr, s);
    k_agg_hub_fill<C><<<sort_slices, 256, 0, s>>>(a, a.count);
    k_agg_hub_part<C><<<parts, 256, 0, s>>>(a, a.count);
}

template void launch_aggregate<CfgNarrow>(int, const AggArgs<CfgNarrow> &, int, hipStream_t);
template void launch_aggregate<CfgWideIn>(int, const AggArgs<CfgWideIn> &, int, hipStream_t);
template void launch_aggregate<CfgWide>(int, const AggArgs<CfgWide> &, int, hipStream_t);
template void launch_aggregate_hub<CfgNarrow>(const AggArgs<CfgNarrow> &, int32_t, int32_t,
                                              int64_t, int64_t *, hipStream_t);
template void launch_aggregate_hub<CfgWideIn>(const AggArgs<CfgWideIn> &, int32_t, int32_t,
                                              int64_t, int64_t *, hipStream_t);
template void launch_aggregate_hub<CfgWide>(const AggArgs<CfgWide> &, int32_t, int32_t,
                                            int64_t, int64_t *, hipStream_t);

}  // namespace lv
