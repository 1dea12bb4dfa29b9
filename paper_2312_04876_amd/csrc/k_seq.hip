// Local moving of small levels, one wavefront per graph (Alg. 2 with the
// paper's asynchronous semantics, executed in vertex order).
//
// On a level of a few hundred or thousand vertices the GPU would decide most
// vertices at the same moment: each sees the community totals of the others
// at the start of the kernel, many of them pick the same attractive community
// together, and the level can collapse into a few giant communities (measured
// on coarse levels of batched planted-partition graphs: 66 communities folded
// into 7).  A level this small costs microseconds per vertex when visited in
// order, so fast mode runs it the way the paper's Alg. 2 reads: one vertex at
// a time in ascending id, each against the live state left by the previous
// ones, a mover re-marking its neighbours (later ones in the same sweep),
// iterations until delta-Q <= tau.  The rows are scanned by the 64 lanes of
// the wavefront into an LDS table; the lane whose insert created a
// community's slot lists it, so scoring and clearing touch only the keys.
// The result is the oracle's sequential sweep for that level, bit for bit.
#include <climits>

#include "kernels.h"

namespace lv {

namespace {

template <class C>
__global__ __launch_bounds__(64) void k_seq_level(SeqArgs<C> a)
{
    typedef typename C::ST ST;
    typedef typename C::SC SC;
    typedef typename C::VT VT;
    constexpr int TS = 2 * SEQ_MAX;  // slots: twice the most distinct communities of a row
    constexpr int LOG2S = SEQ_LOG2 + 1;
    __shared__ int32_t keys[TS];
    __shared__ VT vals[TS];
    __shared__ int32_t list[SEQ_MAX];
    __shared__ int32_t nlist;
    const int lane = threadIdx.x;
    const int g = blockIdx.x;
    int vb = 0, ve = a.n;
    int64_t W = a.W;
    if (a.bt.gid) {
        if (g >= a.bt.G || a.bt.gst[g]) return;  // stopped graph
        vb = a.bt.gvb[g];
        ve = a.bt.gvb[g + 1];
        W = a.bt.gW[g];
    } else if (g > 0) {
        return;
    }
    const int nv = ve - vb;
    if (nv <= 0 || nv > a.max_n) return;  // empty, or left to the degree bins
    for (int q = lane; q < TS; q += 64) {
        keys[q] = -1;
        vals[q] = 0;
    }
    if (lane == 0) nlist = 0;
    for (int v = vb + lane; v < ve; v += 64) a.act[v] = 1;
    wave_sync();
    int it = 0;
    for (; it < a.max_iter; ++it) {
        if (!a.prune)
            for (int v = vb + lane; v < ve; v += 64) a.act[v] = 1;
        wave_sync();
        i128 sumN = 0;
        unsigned long long moves = 0, processed = 0, scanned = 0;
        for (int v = vb; v < ve; ++v) {
            if (!a.act[v]) continue;  // uniform: every lane reads the same flag
            wave_sync();
            if (lane == 0) a.act[v] = 0;
            ++processed;
            const int beg = a.off[v];
            const int d = row_len(a.off, a.deg, v);
            const int dc = a.Cp[v];
            const ST kv = a.K[v];
            scanned += (unsigned long long)d;
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
                    const uint32_t mask = (uint32_t)TS - 1u;
                    uint32_t h = hash32((uint32_t)c[k]) >> (32 - LOG2S);
                    for (;;) {
                        const int32_t key = __hip_atomic_load(&keys[h], __ATOMIC_RELAXED,
                                                              __HIP_MEMORY_SCOPE_WORKGROUP);
                        if (key == c[k]) break;
                        if (key < 0) {
                            const int32_t old = atomicCAS(&keys[h], -1, c[k]);
                            if (old < 0) {
                                list[atomicAdd(&nlist, 1)] = (int32_t)h;
                                break;
                            }
                            if (old == c[k]) break;
                        }
                        h = (h + 1) & mask;
                    }
                    atomic_add_t<VT>(&vals[h], w[k]);
                }
            }
            wave_sync();
            const int nk = nlist;
            SC best = score_min<SC>();
            int bc = INT_MAX;
            ST hd = 0;
            for (int q = lane; q < nk; q += 64) {
                const int slot = list[q];
                const int key = keys[slot];
                const ST x = (ST)vals[slot];
                keys[slot] = -1;
                vals[slot] = 0;
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
            if (lane == 0) nlist = 0;
            // Eq. 2: move only for a strictly positive gain (no singleton rule: the
            // vertices decide one at a time)
            bool mv = false;
            SC gain = 0;
            if (nonself > 0 && bc != INT_MAX) {
                const SC stay = (SC)W * (SC)hd - (SC)kv * ((SC)a.Sig[dc] - (SC)kv);
                if (best > stay) {
                    mv = true;
                    gain = best - stay;
                }
            }
            if (mv) {
                if (lane == 0) {
                    a.Sig[dc] -= kv;
                    a.Sig[bc] += kv;
                    a.size[dc] -= 1;
                    a.size[bc] += 1;
                    a.Cp[v] = bc;
                }
                sumN += (i128)gain;
                ++moves;
                for (int e = lane; e < d; e += 64) a.act[a.tgt[beg + e]] = 1;
            }
            wave_sync();
        }
        const double dq = iteration_dq(sumN, (unsigned long long)W);
        if (lane == 0) {
            if (a.bt.gid) {
                // a batch graph records its gains in its own sum (the per-iteration
                // trace is the union's)
            } else if (it < LOUVAIN_MAX_ITERATIONS) {
                a.sc->sumN[it][0] = (unsigned long long)sumN;
                a.sc->sumN[it][1] = (unsigned long long)(sumN >> 64);
                a.sc->dq[it] = dq;
                a.sc->moves[it] = moves;
                a.sc->processed[it] = processed;
                a.sc->scanned[it] = scanned;
            }
        }
        if (dq <= a.tau) {
            ++it;
            break;
        }
    }
    if (lane == 0) {
        if (a.bt.gid) {
            a.bt.giter[g] = it;
            a.bt.gst[g] |= 1;  // converged in this pass: the degree bins skip it
        } else {
            a.sc->iters = it;
            a.sc->done = 1;
        }
    }
}

}  // namespace

template <class C>
void launch_seq_level(const SeqArgs<C> &a, int graphs, hipStream_t s)
{
    if (graphs <= 0) return;
    k_seq_level<C><<<graphs, 64, 0, s>>>(a);
}
template void launch_seq_level<CfgNarrow>(const SeqArgs<CfgNarrow> &, int, hipStream_t);
template void launch_seq_level<CfgWideIn>(const SeqArgs<CfgWideIn> &, int, hipStream_t);
template void launch_seq_level<CfgWide>(const SeqArgs<CfgWide> &, int, hipStream_t);
template void launch_seq_level<CfgWideIn32>(const SeqArgs<CfgWideIn32> &, int, hipStream_t);

}  // namespace lv
