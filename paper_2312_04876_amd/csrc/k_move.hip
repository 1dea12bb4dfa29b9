// Local-moving kernels (Alg. 2): for every active vertex of one degree bin,
// scatter the weights of its row into a per-vertex community table
// (scanCommunities without the self-loop), take the delta-modularity argmax
// over the table (Eq. 2 in exact integers, ties to the lowest community
// id), and move / mark the row's vertices for the next iteration (pruning).
//
// Table placement by bin: groups of 8/32/64 lanes with private LDS tables
// (bins 0-3), one workgroup with an LDS table of up to 8192 slots (bin 4),
// one workgroup with an open-addressing table in HBM (bin 5, hubs).
//
// FAST = true applies each move at once (live C', Sigma', size; asynchronous
// semantics); FAST = false records the move for the apply kernel so every
// decision of a round sees the state at the start of the round.
#include <climits>

#include "kernels.h"

namespace lv {

namespace {

// Insert (c, w) into a power-of-two LDS table of 2^log2s slots (linear probing).
// Returns 1 if c was a new key.
template <typename ST>
__device__ inline int lds_insert(int32_t *keys, ST *vals, int log2s, int32_t c, ST w)
{
    const uint32_t mask = (1u << log2s) - 1u;
    uint32_t h = hash32((uint32_t)c) >> (32 - log2s);
    for (;;) {
        const int32_t k = __hip_atomic_load(&keys[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (k == c) {
            atomic_add_t<ST>(&vals[h], w);
            return 0;
        }
        if (k < 0) {
            const int32_t old = atomicCAS(&keys[h], -1, c);
            if (old < 0 || old == c) {
                atomic_add_t<ST>(&vals[h], w);
                return old < 0 ? 1 : 0;
            }
        }
        h = (h + 1) & mask;
    }
}

// Insert into an HBM table of T slots (T >= 2 * row length); index by the
// high half of hash * T.
template <typename ST>
__device__ inline int hbm_insert(int32_t *keys, ST *vals, uint32_t T, int32_t c, ST w)
{
    uint32_t h = (uint32_t)(((uint64_t)hash32((uint32_t)c) * (uint64_t)T) >> 32);
    for (;;) {
        const int32_t k = __hip_atomic_load(&keys[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (k == c) {
            atomic_add_t<ST>(&vals[h], w);
            return 0;
        }
        if (k < 0) {
            const int32_t old = atomicCAS(&keys[h], -1, c);
            if (old < 0 || old == c) {
                atomic_add_t<ST>(&vals[h], w);
                return old < 0 ? 1 : 0;
            }
        }
        h = (h + 1 == T) ? 0u : h + 1;
    }
}

// Candidate order: higher score first, then lower community id.
template <typename SC>
__device__ inline bool better(SC s, int c, SC bs, int bc)
{
    return s > bs || (s == bs && c < bc);
}

// Decision for vertex v once the group knows (best score, its community,
// weight to the own community, non-self entries).  Returns true to move and
// sets the gain N = best - stay.
template <class C>
__device__ inline bool decide(const MoveArgs<C> &a, int v, int dc, typename C::ST kv,
                              typename C::SC best, int bc, typename C::ST hd, int nonself,
                              typename C::SC *gain)
{
    typedef typename C::SC SC;
    if (nonself <= 0 || bc == INT_MAX) return false;
    const SC stay = (SC)a.W * (SC)hd - (SC)kv * ((SC)a.Sig[dc] - (SC)kv);
    if (!(best > stay)) return false;
    if (a.rule && a.size[dc] == 1 && a.size[bc] == 1 && bc > dc) return false;
    *gain = best - stay;
    return true;
}

template <class C, bool FAST>
__device__ inline void commit(const MoveArgs<C> &a, int v, int dc, int bc, typename C::ST kv)
{
    typedef typename C::ST ST;
    if (FAST) {
        a.Cp[v] = bc;
        atomic_add_t<ST>(&a.Sig[dc], (ST)-kv);
        atomic_add_t<ST>(&a.Sig[bc], kv);
        atomicSub(&a.size[dc], 1);
        atomicAdd(&a.size[bc], 1);
    } else {
        const int m = atomicAdd(a.mv_count, 1);
        a.mv_v[m] = v;
        a.mv_c[m] = bc;
    }
}

// Flush per-lane counters of a 256-thread block.
template <class C>
__device__ inline void flush_counters(const MoveArgs<C> &a, typename C::SC gain,
                                      unsigned long long nv, unsigned long long ne,
                                      unsigned long long nk, unsigned long long nm)
{
    const i128 g = wave_sum_i128((i128)gain);
    nv = wave_sum_u64(nv);
    ne = wave_sum_u64(ne);
    nk = wave_sum_u64(nk);
    nm = wave_sum_u64(nm);
    if ((threadIdx.x & 63) == 0) {
        atomic_add_i128(a.sumN, g);
        if (nv) atomicAdd(&a.work[0], nv);
        if (ne) {
            atomicAdd(&a.work[1], ne);
            atomicAdd(a.it_scanned, ne);
        }
        if (nk) atomicAdd(&a.work[2], nk);
        if (nm) {
            atomicAdd(&a.work[3], nm);
            atomicAdd(a.it_moves, nm);
        }
    }
}

// Bins 0-3: G lanes per vertex, 64/G vertices per wavefront, LDS table of
// 2^LOG2S slots per group.
template <class C, int G, int LOG2S, bool FAST>
__global__ __launch_bounds__(256) void k_move_wave(MoveArgs<C> a)
{
    typedef typename C::ST ST;
    typedef typename C::SC SC;
    constexpr int S = 1 << LOG2S;
    constexpr int GPW = 64 / G;
    constexpr int NG = 4 * GPW;
    __shared__ ST s_vals[NG * S];
    __shared__ int32_t s_keys[NG * S];
    if (*a.done) return;
    const int count = *a.count;
    if (count == 0) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int grp = lane / G, gl = lane % G;
    int32_t *keys = s_keys + (wave * GPW + grp) * S;
    ST *vals = s_vals + (wave * GPW + grp) * S;
    for (int s = gl; s < S; s += G) {
        keys[s] = -1;
        vals[s] = 0;
    }
    wave_sync();
    SC gain_acc = 0;
    unsigned long long nv = 0, ne = 0, nk = 0, nm = 0;
    const int stride = gridDim.x * NG;
    for (int base = (blockIdx.x * 4 + wave) * GPW; base < count; base += stride) {
        const int idx = base + grp;
        const bool has = idx < count;
        int v = 0, beg = 0, d = 0;
        if (has) {
            v = a.binorder[a.worklist[a.list_begin + idx]];
            beg = a.off[v];
            d = row_len(a.off, a.deg, v);
        }
        int nonself = 0;
        for (int e = gl; e < d; e += G) {
            const int j = a.tgt[beg + e];
            ++ne;
            if (j == v) continue;
            ++nonself;
            nk += lds_insert<ST>(keys, vals, LOG2S, a.Cp[j], (ST)a.w[beg + e]);
        }
        wave_sync();
        const int dc = has ? a.Cp[v] : -1;
        const ST kv = has ? a.K[v] : (ST)0;
        SC best = score_min<SC>();
        int bc = INT_MAX;
        ST hd = 0;
        for (int s = gl; s < S; s += G) {
            const int k = keys[s];
            if (k >= 0) {
                const ST x = vals[s];
                keys[s] = -1;
                vals[s] = 0;
                if (k == dc) {
                    hd = x;
                } else {
                    const SC sc = (SC)a.W * (SC)x - (SC)kv * (SC)a.Sig[k];
                    if (better(sc, k, best, bc)) {
                        best = sc;
                        bc = k;
                    }
                }
            }
        }
        for (int o = G / 2; o > 0; o >>= 1) {
            const SC ob = shfl_xor_t<SC>(best, o);
            const int oc = __shfl_xor(bc, o, 64);
            if (better(ob, oc, best, bc)) {
                best = ob;
                bc = oc;
            }
            hd += shfl_xor_t<ST>(hd, o);
            nonself += __shfl_xor(nonself, o, 64);
        }
        SC gain = 0;
        const bool mv = has && decide<C>(a, v, dc, kv, best, bc, hd, nonself, &gain);
        if (has && gl == 0) {
            ++nv;
            if (mv) {
                gain_acc += gain;
                ++nm;
                commit<C, FAST>(a, v, dc, bc, kv);
            }
        }
        if (mv)
            for (int e = gl; e < d; e += G) a.flags_next[a.tgt[beg + e]] = 1;
        wave_sync();
    }
    flush_counters<C>(a, gain_acc, nv, ne, nk, nm);
}

// Block-wide argmax: every thread passes its (best, bc, hd, nonself); the
// result is left in the shared slots r_*[0].
template <typename SC, typename ST>
struct BlockRed {
    SC best[4];
    int bc[4];
    ST hd[4];
    int nonself[4];
    int move;
    int target;
};

template <typename SC, typename ST>
__device__ inline void block_reduce(BlockRed<SC, ST> &r, SC best, int bc, ST hd, int nonself)
{
    for (int o = 32; o > 0; o >>= 1) {
        const SC ob = shfl_xor_t<SC>(best, o);
        const int oc = __shfl_xor(bc, o, 64);
        if (better(ob, oc, best, bc)) {
            best = ob;
            bc = oc;
        }
        hd += shfl_xor_t<ST>(hd, o);
        nonself += __shfl_xor(nonself, o, 64);
    }
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        r.best[wave] = best;
        r.bc[wave] = bc;
        r.hd[wave] = hd;
        r.nonself[wave] = nonself;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < 4; ++k) {
            if (better(r.best[k], r.bc[k], r.best[0], r.bc[0])) {
                r.best[0] = r.best[k];
                r.bc[0] = r.bc[k];
            }
            r.hd[0] += r.hd[k];
            r.nonself[0] += r.nonself[k];
        }
    }
}

// Bin 4: one workgroup per vertex, LDS table of the smallest power of two
// >= 2 * row length (at most 8192 slots).
template <class C, bool FAST>
__global__ __launch_bounds__(256) void k_move_block(MoveArgs<C> a)
{
    typedef typename C::ST ST;
    typedef typename C::SC SC;
    constexpr int S = 1 << BLOCK_LOG2S_MAX;
    __shared__ ST s_vals[S];
    __shared__ int32_t s_keys[S];
    __shared__ BlockRed<SC, ST> r;
    if (*a.done) return;
    const int count = *a.count;
    if (count == 0) return;
    for (int s = threadIdx.x; s < S; s += 256) {
        s_keys[s] = -1;
        s_vals[s] = 0;
    }
    __syncthreads();
    SC gain_acc = 0;
    unsigned long long nv = 0, ne = 0, nk = 0, nm = 0;
    for (int idx = blockIdx.x; idx < count; idx += gridDim.x) {
        const int v = a.binorder[a.worklist[a.list_begin + idx]];
        const int beg = a.off[v];
        const int d = row_len(a.off, a.deg, v);
        int log2s = 32 - __clz(2 * d - 1);
        if (log2s < 6) log2s = 6;
        const int S_eff = 1 << log2s;
        int nonself = 0;
        for (int e = threadIdx.x; e < d; e += 256) {
            const int j = a.tgt[beg + e];
            ++ne;
            if (j == v) continue;
            ++nonself;
            nk += lds_insert<ST>(s_keys, s_vals, log2s, a.Cp[j], (ST)a.w[beg + e]);
        }
        __syncthreads();
        const int dc = a.Cp[v];
        const ST kv = a.K[v];
        SC best = score_min<SC>();
        int bc = INT_MAX;
        ST hd = 0;
        for (int s = threadIdx.x; s < S_eff; s += 256) {
            const int k = s_keys[s];
            if (k >= 0) {
                const ST x = s_vals[s];
                s_keys[s] = -1;
                s_vals[s] = 0;
                if (k == dc) {
                    hd = x;
                } else {
                    const SC sc = (SC)a.W * (SC)x - (SC)kv * (SC)a.Sig[k];
                    if (better(sc, k, best, bc)) {
                        best = sc;
                        bc = k;
                    }
                }
            }
        }
        block_reduce<SC, ST>(r, best, bc, hd, nonself);
        if (threadIdx.x == 0) {
            SC gain = 0;
            const bool mv = decide<C>(a, v, dc, kv, r.best[0], r.bc[0], r.hd[0], r.nonself[0], &gain);
            r.move = mv ? 1 : 0;
            r.target = r.bc[0];
            ++nv;
            if (mv) {
                gain_acc += gain;
                ++nm;
                commit<C, FAST>(a, v, dc, r.bc[0], kv);
            }
        }
        __syncthreads();
        if (r.move)
            for (int e = threadIdx.x; e < d; e += 256) a.flags_next[a.tgt[beg + e]] = 1;
        __syncthreads();
    }
    flush_counters<C>(a, gain_acc, nv, ne, nk, nm);
}

// Bin 5 (hubs): one workgroup per vertex, open-addressing table in HBM at
// hkeys/hvals + hoff[position in the bin]; the workgroup clears the slots it
// read, so the table is empty again for the next user.
template <class C, bool FAST>
__global__ __launch_bounds__(HUB_THREADS) void k_move_hub(MoveArgs<C> a)
{
    typedef typename C::ST ST;
    typedef typename C::SC SC;
    __shared__ BlockRed<SC, ST> r;
    if (*a.done) return;
    const int count = *a.count;
    SC gain_acc = 0;
    unsigned long long nv = 0, ne = 0, nk = 0, nm = 0;
    for (int idx = blockIdx.x; idx < count; idx += gridDim.x) {
        const int p = a.worklist[a.list_begin + idx];
        const int v = a.binorder[p];
        const int beg = a.off[v];
        const int d = row_len(a.off, a.deg, v);
        const int64_t t0 = a.hoff[p - a.list_begin];
        const uint32_t T = (uint32_t)hub_slots(d);
        int32_t *keys = a.hkeys + t0;
        ST *vals = a.hvals + t0;
        int nonself = 0;
        for (int e = threadIdx.x; e < d; e += HUB_THREADS) {
            const int j = a.tgt[beg + e];
            ++ne;
            if (j == v) continue;
            ++nonself;
            nk += hbm_insert<ST>(keys, vals, T, a.Cp[j], (ST)a.w[beg + e]);
        }
        __threadfence_block();
        __syncthreads();
        const int dc = a.Cp[v];
        const ST kv = a.K[v];
        SC best = score_min<SC>();
        int bc = INT_MAX;
        ST hd = 0;
        for (uint32_t s = threadIdx.x; s < T; s += HUB_THREADS) {
            const int k = __hip_atomic_load(&keys[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (k >= 0) {
                const ST x = __hip_atomic_load(&vals[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                keys[s] = -1;
                vals[s] = 0;
                if (k == dc) {
                    hd = x;
                } else {
                    const SC sc = (SC)a.W * (SC)x - (SC)kv * (SC)a.Sig[k];
                    if (better(sc, k, best, bc)) {
                        best = sc;
                        bc = k;
                    }
                }
            }
        }
        block_reduce<SC, ST>(r, best, bc, hd, nonself);
        if (threadIdx.x == 0) {
            SC gain = 0;
            const bool mv = decide<C>(a, v, dc, kv, r.best[0], r.bc[0], r.hd[0], r.nonself[0], &gain);
            r.move = mv ? 1 : 0;
            ++nv;
            if (mv) {
                gain_acc += gain;
                ++nm;
                commit<C, FAST>(a, v, dc, r.bc[0], kv);
            }
        }
        __syncthreads();
        if (r.move)
            for (int e = threadIdx.x; e < d; e += HUB_THREADS) a.flags_next[a.tgt[beg + e]] = 1;
        __threadfence();
        __syncthreads();
    }
    flush_counters<C>(a, gain_acc, nv, ne, nk, nm);
}

template <class C, bool FAST>
void launch_move_t(int bin, const MoveArgs<C> &a, int grid, hipStream_t s)
{
    switch (bin) {
    case 0: k_move_wave<C, 8, 4, FAST><<<grid, 256, 0, s>>>(a); break;
    case 1: k_move_wave<C, 32, 6, FAST><<<grid, 256, 0, s>>>(a); break;
    case 2: k_move_wave<C, 64, 8, FAST><<<grid, 256, 0, s>>>(a); break;
    case 3: k_move_wave<C, 64, 10, FAST><<<grid, 256, 0, s>>>(a); break;
    case 4: k_move_block<C, FAST><<<grid, 256, 0, s>>>(a); break;
    default: k_move_hub<C, FAST><<<grid, HUB_THREADS, 0, s>>>(a); break;
    }
}

}  // namespace

int move_rows_per_block(int bin)
{
    static const int rows[NBINS] = {32, 8, 4, 4, 1, 1};
    return rows[bin];
}

template <class C>
void launch_move(int bin, bool fast, const MoveArgs<C> &a, int grid, hipStream_t s)
{
    if (grid <= 0) return;
    if (fast)
        launch_move_t<C, true>(bin, a, grid, s);
    else
        launch_move_t<C, false>(bin, a, grid, s);
}
template void launch_move<CfgNarrow>(int, bool, const MoveArgs<CfgNarrow> &, int, hipStream_t);
template void launch_move<CfgWideIn>(int, bool, const MoveArgs<CfgWideIn> &, int, hipStream_t);
template void launch_move<CfgWide>(int, bool, const MoveArgs<CfgWide> &, int, hipStream_t);

}  // namespace lv
