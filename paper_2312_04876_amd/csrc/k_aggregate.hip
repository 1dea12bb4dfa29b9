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

// Bins 4 and 5: one workgroup per community; the table is in LDS (bin 4,
// 2^log2s slots) or in HBM (bin 5, hub_slots(min(total degree, |Gamma|))).
template <class C, bool HBM>
__global__ __launch_bounds__(256) void k_agg_block(AggArgs<C> a, int32_t ncomm)
{
    typedef typename C::ST ST;
    constexpr int S = HBM ? 1 : (1 << BLOCK_LOG2S_MAX);
    __shared__ ST s_vals[S];
    __shared__ int32_t s_keys[S];
    __shared__ int32_t s_incl[256];
    __shared__ int32_t s_rb[256];
    __shared__ int32_t wsum[4];
    __shared__ int32_t s_cnt;
    if (!HBM) {
        for (int s = threadIdx.x; s < S; s += 256) {
            s_keys[s] = -1;
            s_vals[s] = 0;
        }
    }
    if (threadIdx.x == 0) s_cnt = 0;
    __syncthreads();
    unsigned long long nc_ = 0, nm_ = 0, ne_ = 0, no_ = 0;
    for (int idx = blockIdx.x; idx < a.count; idx += gridDim.x) {
        const int c = a.cbinorder[a.begin + idx];
        const int mb = a.coff[c], me = a.coff[c + 1];
        int32_t *keys;
        ST *vals;
        uint32_t T = 0;
        int log2s = 0;
        if (HBM) {
            const int64_t t0 = a.hoff[idx];
            int64_t cap = (int64_t)(a.yoff[c + 1] - a.yoff[c]);
            if (cap > ncomm) cap = ncomm;
            T = (uint32_t)hub_slots(cap);
            keys = a.hkeys + t0;
            vals = a.hvals + t0;
        } else {
            const int tot = a.yoff[c + 1] - a.yoff[c];
            log2s = 32 - __clz(2 * tot - 1);
            if (log2s < 6) log2s = 6;
            keys = s_keys;
            vals = s_vals;
        }
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
                const int k = a.Cp[a.tgt[e]];
                if (HBM)
                    hbm_add<ST>(keys, vals, T, k, (ST)a.w[e]);
                else
                    lds_add<ST>(keys, vals, log2s, k, (ST)a.w[e]);
                ++ne_;
            }
            __syncthreads();
        }
        if (HBM) __threadfence();
        const int ybeg = a.yoff[c];
        const uint32_t n_slots = HBM ? T : (1u << log2s);
        for (uint32_t s = threadIdx.x; s < n_slots; s += 256) {
            int k;
            ST x;
            if (HBM) {
                k = __hip_atomic_load(&keys[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                x = k >= 0 ? __hip_atomic_load(&vals[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0;
            } else {
                k = keys[s];
                x = k >= 0 ? vals[s] : 0;
            }
            if (k >= 0) {
                const int pos = atomicAdd(&s_cnt, 1);
                a.ytgt[ybeg + pos] = k;
                a.yw[ybeg + pos] = x;
                keys[s] = -1;
                vals[s] = 0;
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            a.ydeg[c] = s_cnt;
            no_ += (unsigned long long)s_cnt;
            s_cnt = 0;
            ++nc_;
        }
        if (HBM) __threadfence();
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

inline int agg_grid(int count, int per_block)
{
    int64_t g = ((int64_t)count + per_block - 1) / per_block;
    if (g > 4096) g = 4096;
    if (g < 1) g = 1;
    return (int)g;
}

}  // namespace

template <class C>
void launch_aggregate(int bin, const AggArgs<C> &a, hipStream_t s)
{
    if (a.count <= 0) return;
    switch (bin) {
    case 0: k_agg_wave<C, 8, 4><<<agg_grid(a.count, 32), 256, 0, s>>>(a); break;
    case 1: k_agg_wave<C, 32, 6><<<agg_grid(a.count, 8), 256, 0, s>>>(a); break;
    case 2: k_agg_wave<C, 64, 8><<<agg_grid(a.count, 4), 256, 0, s>>>(a); break;
    case 3: k_agg_wave<C, 64, 10><<<agg_grid(a.count, 4), 256, 0, s>>>(a); break;
    case 4: k_agg_block<C, false><<<agg_grid(a.count, 1), 256, 0, s>>>(a, 0); break;
    default: break;
    }
}

template <class C>
void launch_aggregate_hub(const AggArgs<C> &a, int32_t ncomm, hipStream_t s)
{
    if (a.count <= 0) return;
    k_agg_block<C, true><<<agg_grid(a.count, 1), 256, 0, s>>>(a, ncomm);
}

template void launch_aggregate<CfgNarrow>(int, const AggArgs<CfgNarrow> &, hipStream_t);
template void launch_aggregate<CfgWideIn>(int, const AggArgs<CfgWideIn> &, hipStream_t);
template void launch_aggregate<CfgWide>(int, const AggArgs<CfgWide> &, hipStream_t);
template void launch_aggregate_hub<CfgNarrow>(const AggArgs<CfgNarrow> &, int32_t, hipStream_t);
template void launch_aggregate_hub<CfgWideIn>(const AggArgs<CfgWideIn> &, int32_t, hipStream_t);
template void launch_aggregate_hub<CfgWide>(const AggArgs<CfgWide> &, int32_t, hipStream_t);

}  // namespace lv
