// Local moving of small levels, one wavefront per graph, every iteration of
// the level in one launch (Alg. 2 called from Alg. 1).
//
// On a level of a few hundred or thousand vertices the concurrent degree bins
// would decide most vertices at the same moment.  Fast mode then lets each
// one see the community totals of the others at the start of the kernel:
// many pick the same attractive community together, and a level can collapse
// into a few giant communities (measured on coarse levels of batched
// planted-partition graphs: 66 communities folded into 7).  Deterministic
// mode is safe from that, but pays a launch sequence per round and
// iteration for a few hundred vertices.  Both run such levels here instead:
//
// - k_seq_level (fast mode): the paper's asynchronous sweep as one thread
//   executes it, one vertex at a time in ascending id against the live state
//   left by the previous ones, a mover re-marking its neighbours (later ones
//   in the same sweep); iterations until delta-Q <= tau.  This is the
//   oracle's sequential mode for that level, bit for bit.
// - k_sync_level (deterministic mode): the synchronous rounds of the degree
//   bins, decided one vertex at a time against the round's state (no move is
//   applied before the round ends), then applied together; bit-identical to
//   the rounds of the bins and to the oracle's synchronous mode.
//
// A row is scanned by the 64 lanes into an LDS table keyed by community; the
// lane whose insert creates a key lists its slot, so scoring and clearing
// touch only the row's distinct communities.  Isolated vertices are never
// visited (as in the bins).
#include <climits>

#include "kernels.h"

namespace lv {

namespace {

// LDS of one wavefront: a table of 2 * SEQ_MAX slots (a row of a level of at
// most SEQ_MAX vertices has at most that many distinct communities) and the
// list of the slots in use.
template <typename VT>
struct WaveTable {
    int32_t keys[2 * SEQ_MAX];
    VT vals[2 * SEQ_MAX];
    int32_t list[SEQ_MAX];
    int32_t nlist;
};

// Best move of vertex v (row beg, length d, label dc, weight kv) against the
// current C', Sigma' and sizes: every lane returns the same (move, c*, gain).
// With rule set, a singleton may join another singleton only if that
// community's id is smaller.
template <class C>
__device__ inline bool wave_decide(const SeqArgs<C> &a, WaveTable<typename C::VT> &t, int v,
                                   int beg, int d, int dc, typename C::ST kv, int64_t W, bool rule,
                                   int *cstar, i128 *gain)
{
    typedef typename C::ST ST;
    typedef typename C::SC SC;
    typedef typename C::VT VT;
    constexpr int TS = 2 * SEQ_MAX;
    constexpr int LOG2S = SEQ_LOG2 + 1;
    const int lane = threadIdx.x;
    int nonself = 0;
    for (int e0 = 0; e0 < d; e0 += 64 * 4) {
        int j[4], c[4];
        VT w[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int e = e0 + lane + 64 * k;
            j[k] = e < d ? a.tgt[beg + e] : -1;
            w[k] = e < d ? (VT)a.w[beg + e] : (VT)0;
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) c[k] = (j[k] >= 0 && j[k] != v) ? a.Cp[j[k]] : -1;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (c[k] < 0) continue;
            ++nonself;
            uint32_t h = hash32((uint32_t)c[k]) >> (32 - LOG2S);
            for (;;) {
                const int32_t key = __hip_atomic_load(&t.keys[h], __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_WORKGROUP);
                if (key == c[k]) break;
                if (key < 0) {
                    const int32_t old = atomicCAS(&t.keys[h], -1, c[k]);
                    if (old < 0) {
                        t.list[atomicAdd(&t.nlist, 1)] = (int32_t)h;
                        break;
                    }
                    if (old == c[k]) break;
                }
                h = (h + 1) & (uint32_t)(TS - 1);
            }
            atomic_add_t<VT>(&t.vals[h], w[k]);
        }
    }
    wave_sync();
    const int nk = t.nlist;
    SC best = score_min<SC>();
    int bc = INT_MAX;
    ST hd = 0;
    for (int q = lane; q < nk; q += 64) {
        const int slot = t.list[q];
        const int key = t.keys[slot];
        const ST x = (ST)t.vals[slot];
        t.keys[slot] = -1;
        t.vals[slot] = 0;
        if (key == dc) {
            hd = x;
        } else {
            const SC sc = (SC)W * (SC)x - (SC)kv * (SC)a.Sig[key];
            if (better(sc, key, best, bc)) {
                best = sc;
                bc = key;
            }
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        const SC ob = shfl_xor_t<SC>(best, o);
        const int oc = __shfl_xor(bc, o, 64);
        if (better(ob, oc, best, bc)) {
            best = ob;
            bc = oc;
        }
        const ST oh = shfl_xor_t<ST>(hd, o);
        hd = oh > hd ? oh : hd;  // only the lane that held the own community is non-zero
        nonself += __shfl_xor(nonself, o, 64);
    }
    wave_sync();
    if (lane == 0) t.nlist = 0;
    // Eq. 2: move only for a strictly positive gain over staying
    if (nonself <= 0 || bc == INT_MAX) return false;
    const SC stay = (SC)W * (SC)hd - (SC)kv * ((SC)a.Sig[dc] - (SC)kv);
    if (!(best > stay)) return false;
    if (rule && a.size[dc] == 1 && a.size[bc] == 1 && bc > dc) return false;
    *cstar = bc;
    *gain = (i128)(best - stay);
    return true;
}

// The graph of this wavefront: its vertex range and W, or false when it is not
// moved here (stopped, empty, or larger than max_n).
template <class C>
__device__ inline bool wave_graph(const SeqArgs<C> &a, int *vb, int *ve, int64_t *W)
{
    const int g = blockIdx.x;
    *vb = 0;
    *ve = a.n;
    *W = a.W;
    if (a.bt.gid) {
        if (g >= a.bt.G || a.bt.gst[g]) return false;
        *vb = a.bt.gvb[g];
        *ve = a.bt.gvb[g + 1];
        *W = a.bt.gW[g];
    } else if (g > 0) {
        return false;
    }
    const int nv = *ve - *vb;
    return nv > 0 && nv <= a.max_n;
}

// Per-iteration record (a single graph) and the end of the level's phase.
template <class C>
__device__ inline void wave_record(const SeqArgs<C> &a, int it, i128 sumN, double dq,
                                   unsigned long long moves, unsigned long long processed,
                                   unsigned long long scanned)
{
    if (threadIdx.x != 0 || a.bt.gid || it >= LOUVAIN_MAX_ITERATIONS) return;
    a.sc->sumN[it][0] = (unsigned long long)sumN;
    a.sc->sumN[it][1] = (unsigned long long)(sumN >> 64);
    a.sc->dq[it] = dq;
    a.sc->moves[it] = moves;
    a.sc->processed[it] = processed;
    a.sc->scanned[it] = scanned;
}

template <class C>
__device__ inline void wave_finish(const SeqArgs<C> &a, int iters)
{
    if (threadIdx.x != 0) return;
    if (a.bt.gid) {
        a.bt.giter[blockIdx.x] = iters;
        a.bt.gst[blockIdx.x] |= 1;  // converged in this pass: the degree bins skip it
    } else {
        a.sc->iters = iters;
        a.sc->done = 1;
    }
}

template <class C>
__global__ __launch_bounds__(64) void k_seq_level(SeqArgs<C> a)
{
    typedef typename C::ST ST;
    __shared__ WaveTable<typename C::VT> t;
    const int lane = threadIdx.x;
    int vb, ve;
    int64_t W;
    if (!wave_graph(a, &vb, &ve, &W)) return;
    for (int q = lane; q < 2 * SEQ_MAX; q += 64) {
        t.keys[q] = -1;
        t.vals[q] = 0;
    }
    if (lane == 0) t.nlist = 0;
    for (int v = vb + lane; v < ve; v += 64) a.act[v] = 1;
    wave_sync();
    int it = 0;
    while (it < a.max_iter) {
        if (!a.prune)
            for (int v = vb + lane; v < ve; v += 64) a.act[v] = 1;
        wave_sync();
        i128 sumN = 0;
        unsigned long long moves = 0, processed = 0, scanned = 0;
        for (int v = vb; v < ve; ++v) {
            if (!a.act[v]) continue;  // uniform: every lane reads the same flag
            const int d = row_len(a.off, a.deg, v);
            wave_sync();
            if (lane == 0) a.act[v] = 0;
            if (d == 0) continue;  // isolated: never moves
            ++processed;
            scanned += (unsigned long long)d;
            const int beg = a.off[v];
            const int dc = a.Cp[v];
            const ST kv = a.K[v];
            int bc = 0;
            i128 gain = 0;
            if (wave_decide<C>(a, t, v, beg, d, dc, kv, W, false, &bc, &gain)) {
                if (lane == 0) {
                    a.Sig[dc] -= kv;
                    a.Sig[bc] += kv;
                    a.size[dc] -= 1;
                    a.size[bc] += 1;
                    a.Cp[v] = bc;
                }
                sumN += gain;
                ++moves;
                for (int e = lane; e < d; e += 64) a.act[a.tgt[beg + e]] = 1;
            }
            wave_sync();
        }
        const double dq = iteration_dq(sumN, (unsigned long long)W);
        wave_record(a, it, sumN, dq, moves, processed, scanned);
        ++it;
        if (dq <= a.tau) break;
    }
    wave_finish(a, it);
}

template <class C>
__global__ __launch_bounds__(64) void k_sync_level(SeqArgs<C> a)
{
    typedef typename C::ST ST;
    __shared__ WaveTable<typename C::VT> t;
    __shared__ int32_t nmv;
    const int lane = threadIdx.x;
    int vb, ve;
    int64_t W;
    if (!wave_graph(a, &vb, &ve, &W)) return;
    for (int q = lane; q < 2 * SEQ_MAX; q += 64) {
        t.keys[q] = -1;
        t.vals[q] = 0;
    }
    if (lane == 0) {
        t.nlist = 0;
        nmv = 0;
    }
    for (int v = vb + lane; v < ve; v += 64) {
        a.act[v] = 1;
        a.mark[v] = 0;
    }
    wave_sync();
    const int rounds = 1 << a.round_bits;
    int it = 0;
    while (it < a.max_iter) {
        if (!a.prune)
            for (int v = vb + lane; v < ve; v += 64) a.act[v] = 1;
        wave_sync();
        i128 sumN = 0;
        unsigned long long moves = 0, processed = 0, scanned = 0;
        for (int r = 0; r < rounds; ++r) {
            // decide every active vertex of the round against the round's state; the
            // moves wait in mv_v / mv_c (this graph's range) until the round ends
            for (int v = vb; v < ve; ++v) {
                if (!a.act[v]) continue;
                if (round_of(a.seed, a.round_bits, a.pass, it, v - vb) != r) continue;
                const int d = row_len(a.off, a.deg, v);
                wave_sync();
                if (lane == 0) a.act[v] = 0;
                if (d == 0) continue;
                ++processed;
                scanned += (unsigned long long)d;
                int bc = 0;
                i128 gain = 0;
                if (wave_decide<C>(a, t, v, a.off[v], d, a.Cp[v], a.K[v], W, a.rule != 0, &bc,
                                   &gain)) {
                    if (lane == 0) {
                        a.mv_v[vb + nmv] = v;
                        a.mv_c[vb + nmv] = bc;
                        nmv += 1;
                    }
                    sumN += gain;
                    ++moves;
                }
                wave_sync();
            }
            // the round's moves together: totals, sizes and labels, and the rows of
            // the movers marked for the next iteration
            const int nm = nmv;
            for (int k = lane; k < nm; k += 64) {
                const int v = a.mv_v[vb + k], c = a.mv_c[vb + k], dc = a.Cp[v];
                const ST kv = a.K[v];
                atomic_add_t<ST>(&a.Sig[dc], (ST)-kv);
                atomic_add_t<ST>(&a.Sig[c], kv);
                atomicSub(&a.size[dc], 1);
                atomicAdd(&a.size[c], 1);
            }
            wave_sync();
            for (int k = lane; k < nm; k += 64) a.Cp[a.mv_v[vb + k]] = a.mv_c[vb + k];
            for (int k = 0; k < nm; ++k) {
                const int v = a.mv_v[vb + k];
                const int beg = a.off[v], d = row_len(a.off, a.deg, v);
                for (int e = lane; e < d; e += 64) a.mark[a.tgt[beg + e]] = 1;
            }
            wave_sync();
            if (lane == 0) nmv = 0;
            wave_sync();
        }
        // the next iteration's active set: the rows of this iteration's movers
        for (int v = vb + lane; v < ve; v += 64)
            if (a.mark[v]) {
                a.act[v] = 1;
                a.mark[v] = 0;
            }
        const double dq = iteration_dq(sumN, (unsigned long long)W);
        wave_record(a, it, sumN, dq, moves, processed, scanned);
        ++it;
        if (dq <= a.tau) break;
    }
    wave_finish(a, it);
}

}  // namespace

template <class C>
void launch_seq_level(const SeqArgs<C> &a, bool fast, int graphs, hipStream_t s)
{
    if (graphs <= 0) return;
    if (fast)
        k_seq_level<C><<<graphs, 64, 0, s>>>(a);
    else
        k_sync_level<C><<<graphs, 64, 0, s>>>(a);
}
template void launch_seq_level<CfgNarrow>(const SeqArgs<CfgNarrow> &, bool, int, hipStream_t);
template void launch_seq_level<CfgWideIn>(const SeqArgs<CfgWideIn> &, bool, int, hipStream_t);
template void launch_seq_level<CfgWide>(const SeqArgs<CfgWide> &, bool, int, hipStream_t);
template void launch_seq_level<CfgWideIn32>(const SeqArgs<CfgWideIn32> &, bool, int, hipStream_t);

}  // namespace lv
