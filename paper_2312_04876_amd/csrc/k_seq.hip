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
// iteration for a few hundred vertices.  Both can run such levels here:
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
// The level's state of the graph (labels, community totals and sizes, vertex
// weights, row offsets and lengths, active flags) is loaded into LDS once and
// written back at the end, so a vertex costs one round trip to HBM (its row)
// and LDS work.  Labels and communities are held as indices within the graph.
// A row is scanned by the 64 lanes into an LDS table keyed by community; the
// lane whose insert creates a key lists its slot, so scoring and clearing
// touch only the row's distinct communities.  Isolated vertices are never
// visited (as in the bins).
#include <climits>

#include "kernels.h"

namespace lv {

namespace {

// LDS of one wavefront: the graph's state (at most MAXV vertices), a table
// of 2 * MAXV slots (a row has at most MAXV distinct communities) and the
// list of the slots in use.  Two sizes: 256 vertices (small enough for many
// wavefronts per CU) and SEQ_MAX.  The deterministic kernel keeps its round's
// move list in LDS of its own, so the sequential one fits three graphs of
// SEQ_MAX vertices per CU.
template <class C, int MAXV>
struct WaveLds {
    typedef typename C::ST ST;
    typedef typename C::VT VT;
    static constexpr int LOG2S = MAXV == 256 ? 9 : SEQ_LOG2 + 1;  // 2 * MAXV slots
    static_assert((1 << LOG2S) == 2 * MAXV, "table of twice MAXV slots");
    int32_t keys[2 * MAXV];
    VT vals[2 * MAXV];
    ST sig[MAXV];
    ST k[MAXV];
    int32_t list[MAXV];
    int32_t lab[MAXV];
    int32_t size[MAXV];
    int32_t beg[MAXV];
    int32_t len[MAXV];
    uint8_t act[MAXV];
    uint8_t mark[MAXV];
    int32_t nlist, nmv;
};

// Best move of local vertex i (row beg, length d) against the LDS state: every
// lane returns the same (move, c*, gain), communities as local indices.  With
// rule set, a singleton may join another singleton only if that community's
// index is smaller.
// The first 256 entries of a row (4 per lane), loaded ahead of the decision
// that needs them: target (local index, -1 past the row) and weight.
template <typename VT>
struct RowChunk {
    int j[4];
    VT w[4];
};

template <class C>
__device__ inline RowChunk<typename C::VT> load_chunk(const SeqArgs<C> &a, int vb, int beg, int d,
                                                      int e0)
{
    typedef typename C::VT VT;
    RowChunk<VT> r;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int e = e0 + (int)threadIdx.x + 64 * k;
        r.j[k] = e < d ? a.tgt[beg + e] - vb : -1;
        r.w[k] = e < d ? (VT)a.w[beg + e] : (VT)0;
    }
    return r;
}

template <class C, int MAXV>
__device__ inline bool wave_decide(const SeqArgs<C> &a, WaveLds<C, MAXV> &t, int vb, int i, int beg,
                                   int d, const RowChunk<typename C::VT> &first, int64_t W,
                                   bool rule, int *cstar, i128 *gain)
{
    typedef typename C::ST ST;
    typedef typename C::SC SC;
    typedef typename C::VT VT;
    constexpr int TS = 2 * MAXV;
    constexpr int LOG2S = WaveLds<C, MAXV>::LOG2S;
    const int lane = threadIdx.x;
    const int dc = t.lab[i];
    const ST kv = t.k[i];
    int nonself = 0;
    for (int e0 = 0; e0 < d; e0 += 64 * 4) {
        const RowChunk<VT> ch = e0 == 0 ? first : load_chunk(a, vb, beg, d, e0);
        const int *j = ch.j;
        const VT *w = ch.w;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (j[k] < 0 || j[k] == i) continue;
            const int c = t.lab[j[k]];
            ++nonself;
            uint32_t h = hash32((uint32_t)c) >> (32 - LOG2S);
            for (;;) {
                const int32_t key = __hip_atomic_load(&t.keys[h], __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_WORKGROUP);
                if (key == c) break;
                if (key < 0) {
                    const int32_t old = atomicCAS(&t.keys[h], -1, c);
                    if (old < 0) {
                        t.list[atomicAdd(&t.nlist, 1)] = (int32_t)h;
                        break;
                    }
                    if (old == c) break;
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
            const SC sc = (SC)W * (SC)x - (SC)kv * (SC)t.sig[key];
            // ties to the lower community id: local indices keep the order of the ids
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
    const SC stay = (SC)W * (SC)hd - (SC)kv * ((SC)t.sig[dc] - (SC)kv);
    if (!(best > stay)) return false;
    if (rule && t.size[dc] == 1 && t.size[bc] == 1 && bc > dc) return false;
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
        // the graphs marked for this pass (launch_batch_mark_small)
        if (g >= a.bt.G || !(a.bt.gst[g] & 4)) return false;
        *vb = a.bt.gvb[g];
        *ve = a.bt.gvb[g + 1];
        *W = a.bt.gW[g];
    } else if (g > 0) {
        return false;
    }
    const int nv = *ve - *vb;
    return nv > 0 && nv <= a.max_n;
}

// Graphs of the size class of a kernel: more than lo and at most MAXV vertices.
__device__ inline bool in_class(int nv, int lo, int maxv) { return nv > lo && nv <= maxv; }

// The graph's state into LDS (labels and communities as local indices).
template <class C, int MAXV>
__device__ inline void wave_load(const SeqArgs<C> &a, WaveLds<C, MAXV> &t, int vb, int nv)
{
    for (int q = threadIdx.x; q < 2 * MAXV; q += 64) {
        t.keys[q] = -1;
        t.vals[q] = 0;
    }
    for (int i = threadIdx.x; i < nv; i += 64) {
        const int v = vb + i;
        t.lab[i] = a.Cp[v] - vb;
        t.sig[i] = a.Sig[v];
        t.size[i] = a.size[v];
        t.k[i] = a.K[v];
        t.beg[i] = a.off[v];
        t.len[i] = row_len(a.off, a.deg, v);
        t.act[i] = 1;
        t.mark[i] = 0;
    }
    if (threadIdx.x == 0) {
        t.nlist = 0;
        t.nmv = 0;
    }
    wave_sync();
}

// The state back to HBM, the per-iteration record (a single graph) and the end
// of the level's phase.
template <class C, int MAXV>
__device__ inline void wave_store(const SeqArgs<C> &a, WaveLds<C, MAXV> &t, int vb, int nv, int iters)
{
    wave_sync();
    for (int i = threadIdx.x; i < nv; i += 64) {
        const int v = vb + i;
        a.Cp[v] = t.lab[i] + vb;
        a.Sig[v] = t.sig[i];
        a.size[v] = t.size[i];
    }
    if (threadIdx.x != 0) return;
    if (a.bt.gid) {
        a.bt.giter[blockIdx.x] = iters;
        a.bt.gst[blockIdx.x] |= 1;  // converged in this pass
    } else {
        a.sc->iters = iters;
        a.sc->done = 1;
    }
}

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

// First vertex >= from that is active (and, with round >= 0, in that round of
// iteration it), or nv; every lane returns the same.
template <class C, int MAXV>
__device__ inline int next_active(const SeqArgs<C> &a, const WaveLds<C, MAXV> &t, int from, int nv,
                                  int round, int it)
{
    for (int b = from; b < nv; b += 64) {
        const int i = b + (int)threadIdx.x;
        bool on = i < nv && t.act[i] != 0;
        if (on && round >= 0) on = round_of(a.seed, a.round_bits, a.pass, it, i) == round;
        const unsigned long long m = __ballot(on);
        if (m) return b + __ffsll((long long)m) - 1;
    }
    return nv;
}

template <class C, int MAXV>
__global__ __launch_bounds__(64) void k_seq_level(SeqArgs<C> a)
{
    typedef typename C::ST ST;
    __shared__ WaveLds<C, MAXV> t;
    const int lane = threadIdx.x;
    int vb, ve;
    int64_t W;
    if (!wave_graph(a, &vb, &ve, &W)) return;
    const int nv = ve - vb;
    if (!in_class(nv, MAXV == SEQ_MAX ? 256 : 0, MAXV)) return;
    wave_load(a, t, vb, nv);
    int it = 0;
    while (it < a.max_iter) {
        if (!a.prune)
            for (int i = lane; i < nv; i += 64) t.act[i] = 1;
        wave_sync();
        i128 sumN = 0;
        unsigned long long moves = 0, processed = 0, scanned = 0;
        // the active vertices in ascending order; the next one's row is loaded while
        // the current one decides (a move that activates a vertex in between reloads)
        int i = next_active(a, t, 0, nv, -1, it);
        RowChunk<typename C::VT> cur = load_chunk(a, vb, i < nv ? t.beg[i] : 0, i < nv ? t.len[i] : 0, 0);
        while (i < nv) {
            const int d = t.len[i], beg = t.beg[i];
            int ni = next_active(a, t, i + 1, nv, -1, it);
            RowChunk<typename C::VT> nxt = load_chunk(a, vb, ni < nv ? t.beg[ni] : 0, ni < nv ? t.len[ni] : 0, 0);
            wave_sync();
            if (lane == 0) t.act[i] = 0;
            if (d > 0) {  // isolated vertices never move
                ++processed;
                scanned += (unsigned long long)d;
                int bc = 0;
                i128 gain = 0;
                if (wave_decide<C, MAXV>(a, t, vb, i, beg, d, cur, W, false, &bc, &gain)) {
                    if (lane == 0) {
                        const int dc = t.lab[i];
                        const ST kv = t.k[i];
                        t.sig[dc] -= kv;
                        t.sig[bc] += kv;
                        t.size[dc] -= 1;
                        t.size[bc] += 1;
                        t.lab[i] = bc;
                    }
                    sumN += gain;
                    ++moves;
                    for (int e = lane; e < d; e += 64) t.act[a.tgt[beg + e] - vb] = 1;
                    wave_sync();
                    const int n2 = next_active(a, t, i + 1, nv, -1, it);
                    if (n2 != ni) {
                        ni = n2;
                        nxt = load_chunk(a, vb, t.beg[ni], t.len[ni], 0);
                    }
                }
            }
            wave_sync();
            i = ni;
            cur = nxt;
        }
        const double dq = iteration_dq(sumN, (unsigned long long)W);
        wave_record(a, it, sumN, dq, moves, processed, scanned);
        ++it;
        if (dq <= a.tau) break;
    }
    wave_store(a, t, vb, nv, it);
}

template <class C, int MAXV>
__global__ __launch_bounds__(64) void k_sync_level(SeqArgs<C> a)
{
    typedef typename C::ST ST;
    __shared__ WaveLds<C, MAXV> t;
    __shared__ int32_t mv_v[MAXV], mv_c[MAXV];  // a round's moves (vertex, community)
    const int lane = threadIdx.x;
    int vb, ve;
    int64_t W;
    if (!wave_graph(a, &vb, &ve, &W)) return;
    const int nv = ve - vb;
    if (!in_class(nv, MAXV == SEQ_MAX ? 256 : 0, MAXV)) return;
    wave_load(a, t, vb, nv);
    const int rounds = 1 << a.round_bits;
    int it = 0;
    while (it < a.max_iter) {
        if (!a.prune)
            for (int i = lane; i < nv; i += 64) t.act[i] = 1;
        wave_sync();
        i128 sumN = 0;
        unsigned long long moves = 0, processed = 0, scanned = 0;
        for (int r = 0; r < rounds; ++r) {
            // decide every active vertex of the round against the round's state; the
            // moves wait in the LDS list until the round ends
            // (no decision changes the flags of this round: the next vertex's row is
            // loaded while the current one decides)
            int i = next_active(a, t, 0, nv, r, it);
            RowChunk<typename C::VT> cur = load_chunk(a, vb, i < nv ? t.beg[i] : 0, i < nv ? t.len[i] : 0, 0);
            while (i < nv) {
                const int d = t.len[i];
                const int ni = next_active(a, t, i + 1, nv, r, it);
                const RowChunk<typename C::VT> nxt =
                    load_chunk(a, vb, ni < nv ? t.beg[ni] : 0, ni < nv ? t.len[ni] : 0, 0);
                wave_sync();
                if (lane == 0) t.act[i] = 0;
                if (d > 0) {
                    ++processed;
                    scanned += (unsigned long long)d;
                    int bc = 0;
                    i128 gain = 0;
                    if (wave_decide<C, MAXV>(a, t, vb, i, t.beg[i], d, cur, W, a.rule != 0, &bc,
                                       &gain)) {
                        if (lane == 0) {
                            mv_v[t.nmv] = i;
                            mv_c[t.nmv] = bc;
                            t.nmv += 1;
                        }
                        sumN += gain;
                        ++moves;
                    }
                }
                wave_sync();
                i = ni;
                cur = nxt;
            }
            // the round's moves together: totals, sizes and labels, and the rows of
            // the movers marked for the next iteration
            const int nm = t.nmv;
            for (int k = lane; k < nm; k += 64) {
                const int i = mv_v[k], c = mv_c[k], dc = t.lab[i];
                const ST kv = t.k[i];
                atomic_add_t<ST>(&t.sig[dc], (ST)-kv);
                atomic_add_t<ST>(&t.sig[c], kv);
                atomicSub(&t.size[dc], 1);
                atomicAdd(&t.size[c], 1);
            }
            wave_sync();
            for (int k = lane; k < nm; k += 64) t.lab[mv_v[k]] = mv_c[k];
            for (int k = 0; k < nm; ++k) {
                const int i = mv_v[k];
                const int beg = t.beg[i], d = t.len[i];
                for (int e = lane; e < d; e += 64) t.mark[a.tgt[beg + e] - vb] = 1;
            }
            wave_sync();
            if (lane == 0) t.nmv = 0;
            wave_sync();
        }
        // the next iteration's active set: the rows of this iteration's movers
        for (int i = lane; i < nv; i += 64)
            if (t.mark[i]) {
                t.act[i] = 1;
                t.mark[i] = 0;
            }
        const double dq = iteration_dq(sumN, (unsigned long long)W);
        wave_record(a, it, sumN, dq, moves, processed, scanned);
        ++it;
        if (dq <= a.tau) break;
    }
    wave_store(a, t, vb, nv, it);
}

}  // namespace

template <class C>
void launch_seq_level(const SeqArgs<C> &a, bool fast, int graphs, hipStream_t s)
{
    if (graphs <= 0) return;
    // graphs of up to 256 vertices in the small LDS layout, the others up to max_n in
    // the large one
    if (fast) {
        k_seq_level<C, 256><<<graphs, 64, 0, s>>>(a);
        if (a.max_n > 256) k_seq_level<C, SEQ_MAX><<<graphs, 64, 0, s>>>(a);
    } else {
        k_sync_level<C, 256><<<graphs, 64, 0, s>>>(a);
        if (a.max_n > 256) k_sync_level<C, SEQ_MAX><<<graphs, 64, 0, s>>>(a);
    }
}
template void launch_seq_level<CfgNarrow>(const SeqArgs<CfgNarrow> &, bool, int, hipStream_t);
template void launch_seq_level<CfgWideIn>(const SeqArgs<CfgWideIn> &, bool, int, hipStream_t);
template void launch_seq_level<CfgWide>(const SeqArgs<CfgWide> &, bool, int, hipStream_t);
template void launch_seq_level<CfgWideIn32>(const SeqArgs<CfgWideIn32> &, bool, int, hipStream_t);

}  // namespace lv
