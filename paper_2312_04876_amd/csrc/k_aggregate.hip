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

template <typename ST>
__device__ inline void hbm_add(int32_t *keys, ST *vals, uint32_t T, int32_t c, ST w)
{
    uint32_t h = (uint32_t)(((uint64_t)hash32((uint32_t)c) * (uint64_t)T) >> 32);
    for (;;) {
        const int32_t k = __hip_atomic_load(&keys[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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
        h = (h + 1 == T) ? 0u : h + 1;
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
            for (int t = gl; t < total; t += G) {
                const int L = owner_of(incl, G, t);
                const int e = rbs[L] + (t - (L ? incl[L - 1] : 0));
                lds_add<ST>(keys, vals, LOG2S, a.Cp[a.tgt[e]], (ST)a.w[e]);
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
            for (int t = threadIdx.x; t < total; t += 256) {
                const int L = owner_of(s_incl, 256, t);
                const int e = s_rb[L] + (t - (L ? s_incl[L - 1] : 0));
                lds_add<ST>(s_keys, s_vals, log2s, a.Cp[a.tgt[e]], (ST)a.w[e]);
                ++ne_;
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

// Bin 5 (hub communities), step 1: one workgroup per HUB_SLICE-entry window of
// the concatenated member rows of a community (window w of community idx is
// slice cslice[idx] + w); the window is folded into an LDS table and the table
// is added into the community's HBM table of hub_slots(min(total, |Gamma|))
// slots at hoff[idx].
template <class C>
__global__ __launch_bounds__(256) void k_agg_hub_scatter(AggArgs<C> a, int32_t nh)
{
    typedef typename C::ST ST;
    constexpr int S = 1 << HUB_LOG2S;
    __shared__ ST s_vals[S];
    __shared__ int32_t s_keys[S];
    __shared__ int32_t s_start[257];
    __shared__ int32_t s_rb[256];
    __shared__ int32_t s_m0;
    const int k = (int)blockIdx.x;
    const int idx = owner_slice(a.cslice, nh, k);
    const int c = a.cbinorder[a.begin + idx];
    const int mb = a.coff[c], me = a.coff[c + 1];
    const int base = a.mpre[mb];
    const int tot = a.mpre[me] - base;
    const int w0 = (k - a.cslice[idx]) * HUB_SLICE;
    const int w1 = min(w0 + HUB_SLICE, tot);
    for (int s = threadIdx.x; s < S; s += 256) {
        s_keys[s] = -1;
        s_vals[s] = 0;
    }
    if (threadIdx.x == 0) {
        // first member whose row ends after w0
        int lo = mb, hi = me - 1;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (a.mpre[mid + 1] - base > w0)
                hi = mid;
            else
                lo = mid + 1;
        }
        s_m0 = lo;
    }
    __syncthreads();
    unsigned long long ne_ = 0, nm_ = 0;
    int m = s_m0;
    for (;;) {
        const int cnt = min(256, me - m);
        if ((int)threadIdx.x < cnt) {
            const int u = a.members[m + threadIdx.x];
            s_rb[threadIdx.x] = a.off[u];
            const int st = a.mpre[m + threadIdx.x] - base;
            s_start[threadIdx.x] = st;
            if (st >= w0 && st < w1 && a.mpre[m + threadIdx.x + 1] - base > st) ++nm_;
        }
        if (threadIdx.x == 0) s_start[cnt] = a.mpre[m + cnt] - base;
        __syncthreads();
        const int t_lo = max(w0, s_start[0]);
        const int t_hi = min(w1, s_start[cnt]);
        for (int t = t_lo + (int)threadIdx.x; t < t_hi; t += 256) {
            const int L = owner_slice(s_start, cnt, t);
            const int e = s_rb[L] + (t - s_start[L]);
            lds_add<ST>(s_keys, s_vals, HUB_LOG2S, a.Cp[a.tgt[e]], (ST)a.w[e]);
            ++ne_;
        }
        const bool more = s_start[cnt] < w1 && m + cnt < me;
        __syncthreads();
        if (!more) break;
        m += cnt;
    }
    int64_t cap = tot;
    if (cap > a.ncomm) cap = a.ncomm;
    const uint32_t T = (uint32_t)hub_slots(cap);
    const int64_t t0 = a.hoff[idx];
    for (int s = threadIdx.x; s < S; s += 256) {
        const int key = s_keys[s];
        if (key >= 0) hbm_add<ST>(a.hkeys + t0, a.hvals + t0, T, key, s_vals[s]);
    }
    nm_ = wave_sum_u64(nm_);
    ne_ = wave_sum_u64(ne_);
    if ((threadIdx.x & 63) == 0) {
        if (nm_) atomicAdd(&a.work[1], nm_);
        if (ne_) atomicAdd(&a.work[2], ne_);
    }
}

// Bin 5, step 2: one workgroup per HUB_SLICE slots of a community's HBM table
// (slice tslice[idx] + j) appends the occupied slots to row c of the
// super-vertex graph (position from an atomic on ydeg[c], zero on entry) and
// clears them.
template <class C>
__global__ __launch_bounds__(256) void k_agg_hub_emit(AggArgs<C> a, int32_t nh)
{
    typedef typename C::ST ST;
    __shared__ ST s_v[HUB_SLICE];
    __shared__ int32_t s_k[HUB_SLICE];
    __shared__ int32_t s_cnt, s_base;
    const int k = (int)blockIdx.x;
    const int idx = owner_slice(a.tslice, nh, k);
    const int c = a.cbinorder[a.begin + idx];
    int64_t cap = a.yoff[c + 1] - a.yoff[c];
    if (cap > a.ncomm) cap = a.ncomm;
    const uint32_t T = (uint32_t)hub_slots(cap);
    const int64_t t0 = a.hoff[idx];
    int32_t *keys = a.hkeys + t0;
    ST *vals = a.hvals + t0;
    const uint32_t s0 = (uint32_t)(k - a.tslice[idx]) * HUB_SLICE;
    const uint32_t s1 = min(s0 + (uint32_t)HUB_SLICE, T);
    if (threadIdx.x == 0) s_cnt = 0;
    __syncthreads();
    for (uint32_t s = s0 + threadIdx.x; s < s1; s += 256) {
        const int key = __hip_atomic_load(&keys[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (key >= 0) {
            const ST x = __hip_atomic_load(&vals[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const int pos = atomicAdd(&s_cnt, 1);
            s_k[pos] = key;
            s_v[pos] = x;
            keys[s] = -1;
            vals[s] = 0;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        s_base = s_cnt ? atomicAdd(&a.ydeg[c], s_cnt) : 0;
        if (s_cnt) atomicAdd(&a.work[3], (unsigned long long)s_cnt);
        if (s0 == 0) atomicAdd(&a.work[0], 1ull);
    }
    __syncthreads();
    const int ybeg = a.yoff[c] + s_base;
    for (int i = threadIdx.x; i < s_cnt; i += 256) {
        a.ytgt[ybeg + i] = s_k[i];
        a.yw[ybeg + i] = s_v[i];
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
    case 0: k_agg_wave<C, 8, 4><<<agg_grid(a.count, 32), 256, 0, s>>>(a); break;
    case 1: k_agg_wave<C, 32, 6><<<agg_grid(a.count, 8), 256, 0, s>>>(a); break;
    case 2: k_agg_wave<C, 64, 8><<<agg_grid(a.count, 4), 256, 0, s>>>(a); break;
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

template <class C>
void launch_aggregate_hub(const AggArgs<C> &a, int32_t row_slices, int32_t table_slices,
                          hipStream_t s)
{
    if (a.count <= 0 || row_slices <= 0) return;
    k_agg_hub_scatter<C><<<row_slices, 256, 0, s>>>(a, a.count);
    k_agg_hub_emit<C><<<table_slices, 256, 0, s>>>(a, a.count);
}

template void launch_aggregate<CfgNarrow>(int, const AggArgs<CfgNarrow> &, int, hipStream_t);
template void launch_aggregate<CfgWideIn>(int, const AggArgs<CfgWideIn> &, int, hipStream_t);
template void launch_aggregate<CfgWide>(int, const AggArgs<CfgWide> &, int, hipStream_t);
template void launch_aggregate_hub<CfgNarrow>(const AggArgs<CfgNarrow> &, int32_t, int32_t,
                                              hipStream_t);
template void launch_aggregate_hub<CfgWideIn>(const AggArgs<CfgWideIn> &, int32_t, int32_t,
                                              hipStream_t);
template void launch_aggregate_hub<CfgWide>(const AggArgs<CfgWide> &, int32_t, int32_t,
                                            hipStream_t);

}  // namespace lv
