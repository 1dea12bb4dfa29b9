// Local-moving kernels (Alg. 2): for every active vertex of one degree bin,
// scatter the weights of its row into a per-vertex community table
// (scanCommunities without the self-loop), take the delta-modularity argmax
// over the table (Eq. 2 in exact integers, ties to the lowest community
// id), and move / mark the row's vertices for the next iteration (pruning).
//
// Table placement by bin: groups of 1/4/16/64 lanes with private LDS tables
// (bins 0-3), one workgroup with an LDS table (bins 4-5), and for hubs the
// row's (community, weight) pairs counting-sorted into hash partitions that one
// workgroup each folds in LDS.  Every lane first loads its share
// of the row (targets, weights, then the communities of the targets) into
// registers so the independent loads are in flight together, then inserts.
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

// W (2m) of vertex v's graph: the level's W, or in a batch its own graph's.
template <class C>
__device__ inline int64_t vertex_W(const MoveArgs<C> &a, int v)
{
    return a.bt.gid ? a.bt.gW[a.bt.gid[v]] : a.W;
}

// A batch adds each mover's gain to its graph's sum (the per-graph
// convergence test); a single graph only uses the per-wavefront counters.
template <class C>
__device__ inline void graph_gain(const MoveArgs<C> &a, int v, typename C::SC gain)
{
    if (a.bt.gid) atomic_add_i128(a.bt.gsum + 2 * a.bt.gid[v], (i128)gain);
}

// The same for a whole wavefront (every lane calls this; gain 0 where the lane
// adds nothing).  A wavefront's vertices are consecutive worklist entries, so
// they nearly always lie in one or two graphs: the wavefront adds one sum per
// graph it holds instead of one atomic per mover, which would all land on the
// few graph sums that the vertices in flight share.
template <class C>
__device__ inline void wave_graph_gain(const MoveArgs<C> &a, int v, typename C::SC gain)
{
    if (!a.bt.gid) return;
    const int g = gain != 0 ? a.bt.gid[v] : -1;
    unsigned long long left = __ballot(g >= 0);
    while (left) {
        const int leader = __ffsll((long long)left) - 1;
        const int gl = __shfl(g, leader, 64);
        const bool mine = g == gl;
        const i128 s = wave_sum_i128(mine ? (i128)gain : (i128)0);
        if ((threadIdx.x & 63) == leader) atomic_add_i128(a.bt.gsum + 2 * gl, s);
        left &= ~__ballot(mine);
    }
}

// A community total or size as a decision reads it.  Fast mode reads the live
// value coherently at agent scope (past the non-coherent L1 and the per-XCD
// L2s): movers update totals with memory-side atomics and publish labels only
// afterwards (fast_apply), so a reader that sees a neighbour's new label and
// then loads the total of that community (its address depends on the label)
// sees the mover's weight in it.  A plain load could return a line its XCD
// cached before the update, i.e. a label ahead of its total, the case that
// drags neighbours after movers.  Deterministic mode reads the round's
// snapshot, which no kernel of the round writes, with plain loads.
template <bool FAST, typename T>
__device__ inline T live_load(const T *p)
{
    if (FAST) return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return *p;
}

// A fast-mode label store, coherent at agent scope (written through the
// writer's L2, so readers on the other XCDs see it).
__device__ inline void live_store(int32_t *p, int32_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Decision for vertex v once the group knows (best score, its community,
// weight to the own community, non-self entries).  sd is the own community's
// total as the caller read it; fast mode reads the live total again here.
// Returns true to move and sets the gain N = best - stay.
template <class C, bool FAST>
__device__ inline bool decide(const MoveArgs<C> &a, int64_t W, int dc, typename C::ST kv,
                              typename C::SC best, int bc, typename C::ST hd, int nonself,
                              typename C::ST sd, typename C::SC *gain)
{
    typedef typename C::SC SC;
    if (nonself <= 0 || bc == INT_MAX) return false;
    if (FAST) sd = live_load<FAST>(&a.Sig[dc]);
    const SC stay = (SC)W * (SC)hd - (SC)kv * ((SC)sd - (SC)kv);
    if (!(best > stay)) return false;
    if (a.rule && live_load<FAST>(&a.size[dc]) == 1 && live_load<FAST>(&a.size[bc]) == 1 &&
        bc > dc)
        return false;
    *gain = best - stay;
    return true;
}

// Fast mode applies a move at once: both community weights and both sizes
// (HBM atomics), then the label, so every vertex decided later reads the new
// state.  The label goes last, once the atomics have completed: a reader that
// sees the new label of a neighbour must not score its new community
// against a total that still lacks the neighbour's weight (with the label
// ahead of the totals, every such reader over-rates the mover's community
// and under-rates its old one, and movers pull their neighbours after them;
// a CPU model of that delay loses 0.04-0.06 of Q on a heavy-weight R-MAT
// graph, against under 0.001 when both are published together).
template <class C>
__device__ inline void fast_apply(const MoveArgs<C> &a, int v, int dc, int bc, typename C::ST kv)
{
    typedef typename C::ST ST;
    atomic_add_t<ST>(&a.Sig[dc], (ST)-kv);
    atomic_add_t<ST>(&a.Sig[bc], kv);
    atomicSub(&a.size[dc], 1);
    atomicAdd(&a.size[bc], 1);
    __builtin_amdgcn_s_waitcnt(0);  // the atomics have completed before the label is stored
    live_store(&a.Cp[v], bc);
}

// Fast mode, bins 4-5 (one deciding thread per vertex): the join is checked
// against the destination's total at the moment it is committed.  The atomic
// add of K_v to Sigma'[bc] returns the total just before the join; if movers
// that joined bc after the vertex read its total raised it, the score drops by
// K_v times their weight, and a move that no longer beats staying is withdrawn
// (the weight taken back out, no size or label written), as if the vertex had
// been decided after them.  Otherwise the rest of the move follows, the label
// last (fast_apply).  *gain is the gain over staying as decided; it becomes
// the gain at the commit.
template <class C>
__device__ inline bool fast_commit(const MoveArgs<C> &a, int v, int dc, int bc, typename C::ST kv,
                                   typename C::ST sg, typename C::SC *gain)
{
    typedef typename C::ST ST;
    typedef typename C::SC SC;
    const ST now = atomic_add_ret<ST>(&a.Sig[bc], kv);
    const SC g = *gain - (SC)kv * ((SC)now - (SC)sg);
    if (!(g > 0)) {
        atomic_add_t<ST>(&a.Sig[bc], (ST)-kv);
        return false;
    }
    *gain = g;
    atomic_add_t<ST>(&a.Sig[dc], (ST)-kv);
    atomicSub(&a.size[dc], 1);
    atomicAdd(&a.size[bc], 1);
    __builtin_amdgcn_s_waitcnt(0);  // the atomics have completed before the label is stored
    live_store(&a.Cp[v], bc);
    return true;
}

// Commits the moves decided by the lanes with m set (one lane per vertex);
// every lane of the wavefront calls this.  Deterministic mode writes the new
// label into the round's per-vertex move table (no vertex is decided twice in
// a round), applied when the round ends.
template <class C, bool FAST>
__device__ inline void record_moves(const MoveArgs<C> &a, bool m, int v, int dc, int bc,
                                    typename C::ST kv)
{
    if (!m) return;
    if (FAST)
        fast_apply<C>(a, v, dc, bc, kv);
    else
        a.mv_c[v] = bc;
}

// The same for a single deciding thread.
template <class C, bool FAST>
__device__ inline void record_move(const MoveArgs<C> &a, int v, int dc, int bc,
                                   typename C::ST kv)
{
    if (FAST)
        fast_apply<C>(a, v, dc, bc, kv);
    else
        a.mv_c[v] = bc;
}

// Fast mode, bins 0-3: a workgroup adds the community weight and size changes
// of its moves into an LDS table and applies them with one HBM atomic per
// community every few steps; the movers' labels wait in an LDS list and are
// published after those atomics, so labels and totals become visible together
// (labels never ahead of the totals, see fast_apply).  A GPU decides
// thousands of vertices against the same state anyway, so this adds little
// delay, while it folds the many moves into one popular community (atomics
// performed at the memory side, each also evicting the line every scoring
// lane reads) into a few.
template <typename ST>
__device__ inline void pending_add(int32_t *keys, ST *dsig, int32_t *dsz, int log2s, int32_t c,
                                   ST dk, int ds)
{
    const uint32_t mask = (1u << log2s) - 1u;
    uint32_t h = hash32((uint32_t)c) >> (32 - log2s);
    for (;;) {
        const int32_t k = __hip_atomic_load(&keys[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (k == c) break;
        if (k < 0) {
            const int32_t old = atomicCAS(&keys[h], -1, c);
            if (old < 0 || old == c) break;
        }
        h = (h + 1) & mask;
    }
    atomic_add_t<ST>(&dsig[h], dk);
    atomicAdd(&dsz[h], ds);
}

// Publishes the pending totals, then the pending labels (mv_v[k] -> mv_c[k]
// for k < *mv_n); every thread of the workgroup calls this between barriers.
template <class C>
__device__ inline void pending_flush(const MoveArgs<C> &a, int32_t *keys, typename C::ST *dsig,
                                     int32_t *dsz, int slots, const int32_t *mv_v,
                                     const int32_t *mv_c, int32_t *mv_n)
{
    typedef typename C::ST ST;
    for (int q = threadIdx.x; q < slots; q += blockDim.x) {
        const int32_t c = keys[q];
        if (c < 0) continue;
        if (dsig[q] != 0) atomic_add_t<ST>(&a.Sig[c], dsig[q]);
        if (dsz[q] != 0) atomicAdd(&a.size[c], dsz[q]);
        keys[q] = -1;
        dsig[q] = 0;
        dsz[q] = 0;
    }
    const int nm = *mv_n;
    if (nm == 0) return;  // uniform: read by every thread before the barrier below
    // every wave's totals have completed (vmcnt drained) before any label is stored
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    for (int k = threadIdx.x; k < nm; k += blockDim.x) live_store(&a.Cp[mv_v[k]], mv_c[k]);
    __syncthreads();
    if (threadIdx.x == 0) *mv_n = 0;
}

// Counter row of the calling wavefront.
template <class C>
__device__ inline unsigned long long *counter_row(const MoveArgs<C> &a)
{
    const unsigned wid = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    return a.spread + (size_t)(wid & (NSPREAD - 1)) * SPREAD_W;
}

// Flush per-lane counters (all lanes of every wavefront call this).
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
        unsigned long long *row = counter_row(a);
        unsigned long long *col = row + 2 + 4 * a.bin;
        if (g != 0) atomic_add_i128(row, g);
        if (nv) atomicAdd(&col[0], nv);
        if (ne) atomicAdd(&col[1], ne);
        if (nk) atomicAdd(&col[2], nk);
        if (nm) atomicAdd(&col[3], nm);
    }
}

// Score of one table slot for vertex with label dc and weight kv; updates the
// running best or the weight to the own community.
template <class C>
__device__ inline void consider(const MoveArgs<C> &a, int64_t W, int dc, typename C::ST kv, int k,
                                typename C::ST x, typename C::ST sig, typename C::SC &best,
                                int &bc, typename C::ST &hd)
{
    typedef typename C::SC SC;
    if (k < 0) return;
    if (k == dc) {
        hd = x;
        return;
    }
    const SC sc = (SC)W * (SC)x - (SC)kv * (SC)sig;
    if (better(sc, k, best, bc)) {
        best = sc;
        bc = k;
    }
}

// Score bound (Eq. 2 in the integer form of `consider`).  A community total is
// a sum of non-negative vertex weights, so a candidate's score W*x - K_i*Sigma_c
// never exceeds W*x.  A candidate with W*x <= stay therefore cannot make a
// move, and one with W*x below a score already found cannot be or tie the
// best; neither needs its total read.  Reading the totals of the candidates
// whose bound reaches the floor (stay + 1, raised to the best score of a first
// round over the heaviest candidates) leaves every decision as it was: the
// best candidate and every candidate tying it are read, and when the best
// does not beat staying no move happens either way.
template <class C>
__device__ inline bool worth_reading(int64_t W, typename C::ST x, typename C::SC floor)
{
    typedef typename C::SC SC;
    return (SC)W * (SC)x >= floor;
}

// The floor of the candidates' scores: one above the score of staying.
template <class C>
__device__ inline typename C::SC score_floor(int64_t W, typename C::ST hd, typename C::ST kv,
                                             typename C::ST sd)
{
    typedef typename C::SC SC;
    return (SC)W * (SC)hd - (SC)kv * ((SC)sd - (SC)kv) + 1;
}

// Maximum over a workgroup of NW wavefronts, returned to every thread; buf
// holds NW values in LDS.  Every thread of the workgroup calls this.
template <typename T, int NW>
__device__ inline T block_max(T v, T *buf)
{
    for (int o = 32; o > 0; o >>= 1) {
        const T ov = shfl_xor_t<T>(v, o);
        v = ov > v ? ov : v;
    }
    if ((threadIdx.x & 63) == 0) buf[threadIdx.x >> 6] = v;
    __syncthreads();
    T m = buf[0];
    for (int k = 1; k < NW; ++k) m = buf[k] > m ? buf[k] : m;
    __syncthreads();
    return m;
}

// Insert (c, w) into a power-of-two LDS table; returns the slot, and sets
// *own when this call created the key.
template <typename ST>
__device__ inline int lds_insert_slot(int32_t *keys, ST *vals, int log2s, int32_t c, ST w,
                                      bool *own)
{
    const uint32_t mask = (1u << log2s) - 1u;
    uint32_t h = hash32((uint32_t)c) >> (32 - log2s);
    for (;;) {
        const int32_t k = __hip_atomic_load(&keys[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (k == c) {
            atomic_add_t<ST>(&vals[h], w);
            *own = false;
            return (int)h;
        }
        if (k < 0) {
            const int32_t old = atomicCAS(&keys[h], -1, c);
            if (old < 0 || old == c) {
                atomic_add_t<ST>(&vals[h], w);
                *own = old < 0;
                return (int)h;
            }
        }
        h = (h + 1) & mask;
    }
}

// Bins 0-3: G lanes per vertex (64/G vertices per wavefront), lane l holding
// entries l, l+G, ... (up to E of them), LDS table of 2^LOG2S slots per group
// (groups padded by one slot to spread LDS banks).  The lane whose insert
// created a community's slot scores that community (one read of its total
// per distinct community), so the table is never scanned.
template <class C, int G, int E, int LOG2S, bool FAST>
__global__ __launch_bounds__(256) void k_move_wave(MoveArgs<C> a)
{
    typedef typename C::ST ST;
    typedef typename C::SC SC;
    constexpr int S = 1 << LOG2S;
    constexpr int SP = S + 1;  // padded group stride
    constexpr int GPW = 64 / G;
    constexpr int NG = 4 * GPW;
    // fast mode: community updates pending in LDS, flushed every FL steps
    constexpr int FL = NG >= 64 ? 1 : 64 / NG;
    constexpr int PLOG2 = 4 * NG * FL <= 256 ? 8 : (4 * NG * FL <= 512 ? 9 : 10);  // >= 4 slots/vertex
    constexpr int PS = FAST ? 1 << PLOG2 : 1;
    static_assert(!FAST || PS >= 4 * NG * FL, "pending table too small");
    typedef typename C::VT VT;
    __shared__ VT s_vals[NG * SP];
    __shared__ int32_t s_keys[NG * SP];
    __shared__ int32_t p_keys[PS];
    __shared__ ST p_sig[PS];
    __shared__ int32_t p_sz[PS];
    constexpr int PM = FAST ? NG * FL : 1;  // movers of one flush window
    __shared__ int32_t p_mv[PM], p_mc[PM];
    __shared__ int32_t p_nm;
    if (*a.done) return;
    const int count = *a.count;
    if (count == 0) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int grp = lane / G, gl = lane % G;
    int32_t *keys = s_keys + (wave * GPW + grp) * SP;
    VT *vals = s_vals + (wave * GPW + grp) * SP;
    for (int q = gl; q < S; q += G) {
        keys[q] = -1;
        vals[q] = 0;
    }
    if (FAST) {
        for (int q = threadIdx.x; q < PS; q += 256) {
            p_keys[q] = -1;
            p_sig[q] = 0;
            p_sz[q] = 0;
        }
        if (threadIdx.x == 0) p_nm = 0;
    }
    __syncthreads();
    SC gain_acc = 0;
    unsigned long long nv = 0, ne = 0, nk = 0, nm = 0;
    const int stride = gridDim.x * NG;
    int step = 0;
    for (int b0 = blockIdx.x * NG; b0 < count; b0 += stride, ++step) {
        const int base = b0 + wave * GPW;
        const int idx = base + grp;
        const bool has = idx < count;
        const int v = has ? a.worklist[a.list_begin + idx] : 0;
        int beg = 0, d = 0, dc = -1;
        ST kv = 0, sd = 0;
        int64_t Wv = a.W;
        if (has) {
            beg = a.off[v];
            d = row_len(a.off, a.deg, v);
            dc = a.Cp[v];
            kv = a.K[v];
            Wv = vertex_W(a, v);
        }
        int j[E], c[E], slot[E];
        bool own[E];
        ST w[E];
#pragma unroll
        for (int k = 0; k < E; ++k) {
            const bool in = gl + k * G < d;
            j[k] = in ? a.tgt[beg + gl + k * G] : -1;
            w[k] = in ? (ST)a.w[beg + gl + k * G] : (ST)0;
        }
        if (has) sd = live_load<FAST>(&a.Sig[dc]);
#pragma unroll
        for (int k = 0; k < E; ++k)
            c[k] = (j[k] >= 0 && j[k] != v) ? live_load<FAST>(&a.Cp[j[k]]) : -1;
        int nonself = 0;
#pragma unroll
        for (int k = 0; k < E; ++k) {
            ne += j[k] >= 0 ? 1 : 0;
            slot[k] = -1;
            own[k] = false;
            if (c[k] >= 0) {
                ++nonself;
                slot[k] = lds_insert_slot<VT>(keys, vals, LOG2S, c[k], (VT)w[k], &own[k]);
            }
        }
        wave_sync();
        // each distinct community is held by the lane that created its slot
        ST x[E];
        ST hd = 0, xm = 0;
#pragma unroll
        for (int k = 0; k < E; ++k) {
            x[k] = own[k] ? (ST)vals[slot[k]] : (ST)0;
            if (own[k] && c[k] == dc) hd = x[k];
            if (own[k] && c[k] != dc && x[k] > xm) xm = x[k];
        }
        wave_sync();
#pragma unroll
        for (int k = 0; k < E; ++k)
            if (own[k]) {
                keys[slot[k]] = -1;
                vals[slot[k]] = 0;
            }
        // the group's weight to its own community (one lane holds it) and its
        // heaviest candidate weight
        for (int o = G / 2; o > 0; o >>= 1) {
            const ST oh = shfl_xor_t<ST>(hd, o);
            hd = oh > hd ? oh : hd;
            const ST ox = shfl_xor_t<ST>(xm, o);
            xm = ox > xm ? ox : xm;
            nonself += __shfl_xor(nonself, o, 64);
        }
        // totals of the candidates whose score bound reaches the floor: those of
        // weight at least half the heaviest first, then the rest against the
        // best score found
        SC floor = score_floor<C>(Wv, hd, kv, sd);
        SC best = score_min<SC>();
        int bc = INT_MAX;
#pragma unroll
        for (int ph = 0; ph < 2; ++ph) {
            bool rd[E];
            ST sg[E];
#pragma unroll
            for (int k = 0; k < E; ++k) {
                const bool heavy = x[k] >= xm - x[k];
                rd[k] = own[k] && c[k] != dc && (ph == 0 ? heavy : !heavy) &&
                        worth_reading<C>(Wv, x[k], floor);
            }
#pragma unroll
            for (int k = 0; k < E; ++k) sg[k] = rd[k] ? live_load<FAST>(&a.Sig[c[k]]) : (ST)0;
#pragma unroll
            for (int k = 0; k < E; ++k) {
                if (!rd[k]) continue;
                ++nk;
                const SC sc = (SC)Wv * (SC)x[k] - (SC)kv * (SC)sg[k];
                if (better(sc, c[k], best, bc)) {
                    best = sc;
                    bc = c[k];
                }
            }
            for (int o = G / 2; o > 0; o >>= 1) {
                const SC ob = shfl_xor_t<SC>(best, o);
                const int oc = __shfl_xor(bc, o, 64);
                if (better(ob, oc, best, bc)) {
                    best = ob;
                    bc = oc;
                }
            }
            if (best > floor) floor = best;
        }
        SC gain = 0;
        const bool mv = has && decide<C, FAST>(a, Wv, dc, kv, best, bc, hd, nonself, sd, &gain);
        wave_graph_gain<C>(a, v, mv && gl == 0 ? gain : (SC)0);
        if (has && gl == 0) {
            ++nv;
            if (mv) {
                gain_acc += gain;
                ++nm;
            }
        }
        if (mv) {
#pragma unroll
            for (int k = 0; k < E; ++k)
                if (j[k] >= 0) a.flags_next[j[k]] = 1;
        }
        if (FAST) {
            if (mv && gl == 0) {
                const int k = atomicAdd(&p_nm, 1);  // < NG * FL: one row per group and step
                p_mv[k] = v;
                p_mc[k] = bc;
                pending_add<ST>(p_keys, p_sig, p_sz, PLOG2, dc, (ST)-kv, -1);
                pending_add<ST>(p_keys, p_sig, p_sz, PLOG2, bc, kv, 1);
            }
            if (step % FL == FL - 1 || b0 + stride >= count) {  // uniform over the block
                __syncthreads();
                pending_flush<C>(a, p_keys, p_sig, p_sz, PS, p_mv, p_mc, &p_nm);
                __syncthreads();
            }
        } else {
            record_moves<C, FAST>(a, mv && gl == 0, v, dc, bc, kv);
        }
        wave_sync();
    }
    flush_counters<C>(a, gain_acc, nv, ne, nk, nm);
}

// Block-wide argmax over NW wavefronts; the result is left in r.*[0].
// The best candidate's community total as scored travels with it (sg).
template <typename SC, typename ST, int NW>
struct BlockRed {
    SC best[NW];
    int bc[NW];
    ST sg[NW];
    ST hd[NW];
    int nonself[NW];
    int move;
};

template <typename SC, typename ST, int NW>
__device__ inline void block_reduce(BlockRed<SC, ST, NW> &r, SC best, int bc, ST hd, int nonself,
                                    ST sg = 0)
{
    for (int o = 32; o > 0; o >>= 1) {
        const SC ob = shfl_xor_t<SC>(best, o);
        const int oc = __shfl_xor(bc, o, 64);
        const ST og = shfl_xor_t<ST>(sg, o);
        if (better(ob, oc, best, bc)) {
            best = ob;
            bc = oc;
            sg = og;
        }
        hd += shfl_xor_t<ST>(hd, o);
        nonself += __shfl_xor(nonself, o, 64);
    }
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        r.best[wave] = best;
        r.bc[wave] = bc;
        r.sg[wave] = sg;
        r.hd[wave] = hd;
        r.nonself[wave] = nonself;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < NW; ++k) {
            if (better(r.best[k], r.bc[k], r.best[0], r.bc[0])) {
                r.best[0] = r.best[k];
                r.bc[0] = r.bc[k];
                r.sg[0] = r.sg[k];
            }
            r.hd[0] += r.hd[k];
            r.nonself[0] += r.nonself[k];
        }
    }
}

// Bins 4-5: one workgroup of BT threads per vertex, LDS table (dynamic shared
// memory of 2^log2s_max slots) of block_log2s(row length) slots per vertex.
template <class C, int BT, bool FAST>
__global__ __launch_bounds__(BT) void k_move_block(MoveArgs<C> a, int log2s_max)
{
    typedef typename C::ST ST;
    typedef typename C::SC SC;
    constexpr int NW = BT / 64;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ BlockRed<SC, ST, NW> r;
    __shared__ ST s_mx[NW];
    __shared__ SC s_mb[NW];
    typedef typename C::VT VT;
    const int S_max = 1 << log2s_max;
    VT *s_vals = (VT *)smem;
    int32_t *s_keys = (int32_t *)(smem + (size_t)S_max * sizeof(VT));
    if (*a.done) return;
    const int count = *a.count;
    if (count == 0) return;
    for (int s = threadIdx.x; s < S_max; s += BT) {
        s_keys[s] = -1;
        s_vals[s] = 0;
    }
    __syncthreads();
    SC gain_acc = 0;
    unsigned long long nv = 0, ne = 0, nk = 0, nm = 0;
    for (int idx = blockIdx.x; idx < count; idx += gridDim.x) {
        const int v = a.worklist[a.list_begin + idx];
        const int beg = a.off[v];
        const int d = row_len(a.off, a.deg, v);
        const int dc = a.Cp[v];
        const ST kv = a.K[v];
        const int64_t Wv = vertex_W(a, v);
        const int log2s = block_log2s(d);
        const ST sd = live_load<FAST>(&a.Sig[dc]);
        int nonself = 0;
        for (int e0 = threadIdx.x; e0 < d; e0 += 4 * BT) {
            int j[4], c[4];
            ST w[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) j[k] = e0 + k * BT < d ? a.tgt[beg + e0 + k * BT] : -1;
#pragma unroll
            for (int k = 0; k < 4; ++k) w[k] = j[k] >= 0 ? (ST)a.w[beg + e0 + k * BT] : (ST)0;
#pragma unroll
            for (int k = 0; k < 4; ++k)
                c[k] = (j[k] >= 0 && j[k] != v) ? live_load<FAST>(&a.Cp[j[k]]) : -1;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                ne += j[k] >= 0 ? 1 : 0;
                if (c[k] >= 0) {
                    ++nonself;
                    lds_insert<VT>(s_keys, s_vals, log2s, c[k], (VT)w[k]);
                }
            }
        }
        __syncthreads();
        const int S = 1 << log2s;
        // weight to the own community and the heaviest candidate weight
        ST hd = 0, xm = 0;
        for (int s = threadIdx.x; s < S; s += BT) {
            const int k = s_keys[s];
            if (k < 0) continue;
            const ST x = (ST)s_vals[s];
            if (k == dc)
                hd = x;
            else if (x > xm)
                xm = x;
        }
        hd = block_max<ST, NW>(hd, s_mx);
        xm = block_max<ST, NW>(xm, s_mx);
        // totals of the candidates whose score bound reaches the floor: those of
        // weight at least half the heaviest first, then the rest against the best
        // score found (the second scan also clears the table)
        SC floor = score_floor<C>(Wv, hd, kv, sd);
        SC best = score_min<SC>();
        int bc = INT_MAX;
        ST sgb = 0;
        for (int ph = 0; ph < 2; ++ph) {
            for (int s0 = threadIdx.x; s0 < S; s0 += 4 * BT) {
                int kk[4];
                ST xx[4], sg[4];
                bool rd[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int s = s0 + q * BT;
                    kk[q] = s < S ? s_keys[s] : -1;
                    xx[q] = kk[q] >= 0 ? (ST)s_vals[s] : (ST)0;
                    if (ph == 1 && kk[q] >= 0) {
                        s_keys[s] = -1;
                        s_vals[s] = 0;
                    }
                    const bool heavy = xx[q] >= xm - xx[q];
                    rd[q] = kk[q] >= 0 && kk[q] != dc && (ph == 0 ? heavy : !heavy) &&
                            worth_reading<C>(Wv, xx[q], floor);
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) sg[q] = rd[q] ? live_load<FAST>(&a.Sig[kk[q]]) : (ST)0;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if (!rd[q]) continue;
                    ++nk;
                    const SC sc = (SC)Wv * (SC)xx[q] - (SC)kv * (SC)sg[q];
                    if (better(sc, kk[q], best, bc)) {
                        best = sc;
                        bc = kk[q];
                        sgb = sg[q];
                    }
                }
            }
            if (ph == 0) {
                const SC b1 = block_max<SC, NW>(best, s_mb);
                if (b1 > floor) floor = b1;
            }
        }
        block_reduce<SC, ST, NW>(r, best, bc, threadIdx.x == 0 ? hd : (ST)0, nonself, sgb);
        if (threadIdx.x == 0) {
            SC gain = 0;
            bool mv = decide<C, FAST>(a, Wv, dc, kv, r.best[0], r.bc[0], r.hd[0], r.nonself[0], sd,
                                      &gain);
            if (FAST && mv) mv = fast_commit<C>(a, v, dc, r.bc[0], kv, r.sg[0], &gain);
            if (mv) graph_gain<C>(a, v, gain);
            r.move = mv ? 1 : 0;
            ++nv;
            if (mv) {
                gain_acc += gain;
                ++nm;
                if (!FAST) record_move<C, FAST>(a, v, dc, r.bc[0], kv);
            }
        }
        __syncthreads();
        if (r.move)
            for (int e = threadIdx.x; e < d; e += BT) a.flags_next[a.tgt[beg + e]] = 1;
        __syncthreads();
    }
    flush_counters<C>(a, gain_acc, nv, ne, nk, nm);
}

// Sorting slice k of the hub bin: hub h, entries [e0, e1) of its row.
template <class C>
__device__ inline bool hub_slice(const MoveArgs<C> &a, int k, int *h, int *v, int *beg, int *e0,
                                 int *e1, int *parts, int *gp0)
{
    *h = a.sown[k];
    if (!a.hub_act[*h]) return false;
    *v = a.binorder[a.list_begin + *h];
    *beg = a.off[*v];
    const int d = row_len(a.off, a.deg, *v);
    *e0 = (k - a.hslice[*h]) * HUB_PSLICE;
    *e1 = min(*e0 + HUB_PSLICE, d);
    *gp0 = a.htslice[*h];
    *parts = (*h + 1 < a.nhubs ? a.htslice[*h + 1] : (int)*a.htslices) - *gp0;
    return true;
}

// Hubs, step 1: one workgroup per HUB_PSLICE entries of a queued hub's row
// stages the community of every entry (-1 for a self-loop) and adds the
// slice's pair count per partition into pcount.
template <class C>
__global__ __launch_bounds__(256) void k_hub_count(MoveArgs<C> a)
{
    __shared__ int32_t hist[HUB_MAXP];
    if (*a.done) return;
    const int na = (int)*a.n_act_s;
    unsigned long long ne = 0;
    for (int q = blockIdx.x; q < na; q += gridDim.x) {  // uniform over the workgroup
        int h, v, beg, e0, e1, parts, gp0;
        if (!hub_slice(a, a.act_s[q], &h, &v, &beg, &e0, &e1, &parts, &gp0)) continue;
        for (int p = threadIdx.x; p < parts; p += 256) hist[p] = 0;
        __syncthreads();
        int32_t *stage = a.hstage + a.hoff[h];
        for (int c0 = e0; c0 < e1; c0 += 256 * 8) {
            int j[8], c[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int e = c0 + (int)threadIdx.x + k * 256;
                j[k] = e < e1 ? a.tgt[beg + e] : -1;
            }
#pragma unroll
            for (int k = 0; k < 8; ++k) c[k] = (j[k] >= 0 && j[k] != v) ? a.Cp[j[k]] : -1;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int e = c0 + (int)threadIdx.x + k * 256;
                if (j[k] < 0) continue;
                ++ne;
                stage[e] = c[k];
                if (c[k] >= 0) atomicAdd(&hist[part_of(c[k], parts)], 1);
            }
        }
        __syncthreads();
        for (int p = threadIdx.x; p < parts; p += 256)
            if (hist[p]) atomicAdd(&a.pcount[gp0 + p], hist[p]);
        __syncthreads();  // hist is cleared for the next slice
    }
    ne = wave_sum_u64(ne);
    if ((threadIdx.x & 63) == 0 && ne) atomicAdd(&counter_row(a)[2 + 4 * a.bin + 1], ne);
}

// Hubs, step 2 (after the exclusive scan pcount -> poff): the same workgroups
// reserve room for their pairs in every partition and write them.
template <class C>
__global__ __launch_bounds__(256) void k_hub_fill(MoveArgs<C> a)
{
    typedef typename C::ST ST;
    __shared__ int32_t hist[HUB_MAXP];
    if (*a.done) return;
    const int na = (int)*a.n_act_s;
    for (int q = blockIdx.x; q < na; q += gridDim.x) {  // uniform over the workgroup
        int h, v, beg, e0, e1, parts, gp0;
        if (!hub_slice(a, a.act_s[q], &h, &v, &beg, &e0, &e1, &parts, &gp0)) continue;
        for (int p = threadIdx.x; p < parts; p += 256) hist[p] = 0;
        __syncthreads();
        int32_t *stage = a.hstage + a.hoff[h];
        const int dc = a.Cp[v];
        ST hd = 0;  // weight of the slice's entries into the hub's own community
        for (int e = e0 + (int)threadIdx.x; e < e1; e += 256) {
            const int c = stage[e];
            if (c >= 0) atomicAdd(&hist[part_of(c, parts)], 1);
        }
        __syncthreads();
        for (int p = threadIdx.x; p < parts; p += 256)
            if (hist[p]) hist[p] = a.poff[gp0 + p] + atomicAdd(&a.pcur[gp0 + p], hist[p]);
        __syncthreads();
        for (int c0 = e0; c0 < e1; c0 += 256 * 8) {
            int c[8];
            ST w[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int e = c0 + (int)threadIdx.x + k * 256;
                c[k] = e < e1 ? stage[e] : -1;
            }
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int e = c0 + (int)threadIdx.x + k * 256;
                w[k] = c[k] >= 0 ? (ST)a.w[beg + e] : (ST)0;
            }
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int e = c0 + (int)threadIdx.x + k * 256;
                if (e >= e1) continue;
                if (c[k] >= 0) {
                    const int pos = atomicAdd(&hist[part_of(c[k], parts)], 1);
                    a.pk[pos] = c[k];
                    a.pw[pos] = w[k];
                    if (c[k] == dc) hd += w[k];
                }
            }
        }
        hd = (ST)wave_sum_u64((unsigned long long)(int64_t)hd);
        if ((threadIdx.x & 63) == 0 && hd != 0) atomic_add_t<ST>(&a.hub_hd[h], hd);
        __syncthreads();  // hist is cleared for the next slice
    }
}

// Hubs, step 3: one workgroup per partition of a queued hub folds the
// partition's pairs into an LDS table (dynamic shared memory of 2^hub_plog2
// slots) and leaves its best candidate in hpart.  A partition with more
// distinct communities than 3/4 of the slots (only for skewed keys) is
// folded in several passes over sub-ranges of a third key hash, halving any
// range that still overflows.
template <class C>
__global__ __launch_bounds__(256) void k_hub_part(MoveArgs<C> a)
{
    typedef typename C::ST ST;
    typedef typename C::SC SC;
    typedef typename C::VT VT;
    constexpr int LOG2S = hub_plog2<ST>();
    constexpr int S = 1 << LOG2S;
    extern __shared__ __align__(16) unsigned char smem[];
    VT *vals = (VT *)smem;
    int32_t *keys = (int32_t *)(smem + (size_t)S * sizeof(VT));
    __shared__ BlockRed<SC, ST, 4> r;
    __shared__ uint64_t st_lo[40], st_hi[40];
    __shared__ int s_sp, s_cnt, s_over;
    if (*a.done) return;
    const int na = (int)*a.n_act_p;
    for (int qi = blockIdx.x; qi < na; qi += gridDim.x) {  // uniform over the workgroup
        const int gp = a.act_p[qi];
        const int h = a.pown[gp];
        if (!a.hub_act[h]) continue;
        const int v = a.binorder[a.list_begin + h];
        const int dc = a.Cp[v];
        const ST kv = a.K[v];
        const int64_t Wv = vertex_W(a, v);
        // candidates of this partition whose score bound cannot exceed staying are
        // not read (the hub's weight to its own community is complete after k_hub_fill)
        const SC floor = score_floor<C>(Wv, a.hub_hd[h], kv, a.Sig[dc]);
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
        SC best = score_min<SC>();
        int bc = INT_MAX;
        ST hd = 0;
        int nk = 0;
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
                    const int32_t c = kq[q];
                    if (c < 0) continue;
                    if (!all) {
                        const uint64_t x = hash32(mix32((uint32_t)c) ^ 0x5bd1e995u);
                        if (x < lo || x >= hi) continue;
                    }
                    if (!lds_insert_capped<VT>(keys, vals, lg, c, (VT)wq[q], &s_cnt, capu)) s_over = 1;
                }
            }
            __syncthreads();
            if (s_over) {
                // clear and split the range (a range of one hash value holds one key, so
                // the splitting ends)
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
            for (int s0 = threadIdx.x; s0 < Su; s0 += 4 * 256) {
                int kk[4];
                ST xx[4], sg[4];
                bool rd[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int s = s0 + q * 256;
                    kk[q] = s < Su ? keys[s] : -1;
                    xx[q] = kk[q] >= 0 ? (ST)vals[s] : (ST)0;
                    if (kk[q] >= 0) {
                        keys[s] = -1;
                        vals[s] = 0;
                    }
                    rd[q] = kk[q] >= 0 && kk[q] != dc && worth_reading<C>(Wv, xx[q], floor);
                    nk += rd[q] ? 1 : 0;
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) sg[q] = rd[q] ? a.Sig[kk[q]] : (ST)0;
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (rd[q] || kk[q] == dc)
                        consider<C>(a, Wv, dc, kv, kk[q], xx[q], sg[q], best, bc, hd);
            }
        }
        block_reduce<SC, ST, 4>(r, best, bc, hd, nk);
        if (threadIdx.x == 0) {
            HubPart<C> p;
            p.best = r.best[0];
            p.bc = r.bc[0];
            p.hd = r.hd[0];
            p.nk = r.nonself[0];
            ((HubPart<C> *)a.hpart)[gp] = p;
        }
        __syncthreads();  // the table, the stack and r are reused by the next partition
    }
}

// Hubs, step 4: one workgroup per queued hub takes the argmax over its
// partitions and moves.
template <class C, bool FAST>
__global__ __launch_bounds__(HUB_THREADS) void k_move_hub(MoveArgs<C> a)
{
    typedef typename C::ST ST;
    typedef typename C::SC SC;
    constexpr int NW = HUB_THREADS / 64;
    __shared__ BlockRed<SC, ST, NW> r;
    if (*a.done) return;
    const int count = *a.count;
    const HubPart<C> *part = (const HubPart<C> *)a.hpart;
    SC gain_acc = 0;
    unsigned long long nv = 0, nk = 0, nm = 0;
    for (int idx = blockIdx.x; idx < count; idx += gridDim.x) {
        const int p = a.worklist[a.list_begin + idx];
        const int h = p - a.list_begin;
        const int v = a.binorder[p];
        const int q1 = h + 1 < a.nhubs ? a.htslice[h + 1] : (int)*a.htslices;
        const int dc = a.Cp[v];
        const ST kv = a.K[v];
        const int64_t Wv = vertex_W(a, v);
        SC best = score_min<SC>();
        int bc = INT_MAX;
        ST hd = 0;
        int keys = 0;
        for (int q = a.htslice[h] + threadIdx.x; q < q1; q += HUB_THREADS) {
            const HubPart<C> pp = part[q];
            if (better(pp.best, pp.bc, best, bc)) {
                best = pp.best;
                bc = pp.bc;
            }
            hd += pp.hd;
            keys += pp.nk;
        }
        block_reduce<SC, ST, NW>(r, best, bc, hd, keys);
        if (threadIdx.x == 0) {
            nk += (unsigned long long)r.nonself[0];
            // a hub row holds more than the LDS row limit of distinct targets, so
            // it always has an entry other than a self-loop
            SC gain = 0;
            const bool mv = decide<C, FAST>(a, Wv, dc, kv, r.best[0], r.bc[0], r.hd[0], 1,
                                            FAST ? (ST)0 : a.Sig[dc], &gain);
            if (mv) graph_gain<C>(a, v, gain);
            ++nv;
            if (mv) {
                gain_acc += gain;
                ++nm;
                record_move<C, FAST>(a, v, dc, r.bc[0], kv);
            }
            // k_hub_mark marks the rows of the movers (2) over their sorting slices
            a.hub_act[h] = mv ? 2 : 0;
        }
        __syncthreads();
    }
    flush_counters<C>(a, gain_acc, nv, 0, nk, nm);
}

// Hubs, step 5: one workgroup per sorting slice of a hub that moved marks the
// slice's entries active for the next iteration (pruning), so a giant row is
// marked by many workgroups instead of the one that decided it.
template <class C>
__global__ __launch_bounds__(256) void k_hub_mark(MoveArgs<C> a)
{
    if (*a.done) return;
    const int na = (int)*a.n_act_s;
    for (int q = blockIdx.x; q < na; q += gridDim.x) {
        int h, v, beg, e0, e1, parts, gp0;
        if (!hub_slice(a, a.act_s[q], &h, &v, &beg, &e0, &e1, &parts, &gp0)) continue;
        if (a.hub_act[h] != 2) continue;
        for (int e = e0 + (int)threadIdx.x; e < e1; e += 256) a.flags_next[a.tgt[beg + e]] = 1;
    }
}

template <class C, int BT, bool FAST>
void launch_block(const MoveArgs<C> &a, int grid, int log2s_max, hipStream_t s)
{
    const size_t bytes = ((size_t)1 << log2s_max) * (sizeof(typename C::VT) + 4);
    if (bytes > 65536) {
        // raise the dynamic-LDS limit of this kernel to what the launch asks for; a
        // failure shows up as a launch error at the caller's check
        if (hipFuncSetAttribute((const void *)&k_move_block<C, BT, FAST>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) !=
            hipSuccess)
            (void)hipGetLastError();
    }
    k_move_block<C, BT, FAST><<<grid, BT, bytes, s>>>(a, log2s_max);
}

template <class C, bool FAST>
void launch_move_t(int bin, const MoveArgs<C> &a, int grid, int log2s_max, hipStream_t s)
{
    switch (bin) {
    case 0: k_move_wave<C, 1, 8, 4, FAST><<<grid, 256, 0, s>>>(a); break;
    case 1: k_move_wave<C, 4, 8, 6, FAST><<<grid, 256, 0, s>>>(a); break;
    case 2: k_move_wave<C, 16, 8, 8, FAST><<<grid, 256, 0, s>>>(a); break;
    case 3: k_move_wave<C, 64, 8, 10, FAST><<<grid, 256, 0, s>>>(a); break;
    case 4: launch_block<C, 256, FAST>(a, grid, log2s_max, s); break;
    case 5: launch_block<C, BLOCK_THREADS, FAST>(a, grid, log2s_max, s); break;
    default: break;  // hubs: launch_move_hubs
    }
}

}  // namespace

int move_rows_per_block(int bin)
{
    static const int rows[NBINS] = {256, 64, 16, 4, 1, 1, 1};
    return rows[bin];
}

template <class C>
void launch_move(int bin, bool fast, const MoveArgs<C> &a, int grid, int log2s_max,
                 hipStream_t s)
{
    if (grid <= 0) return;
    if (fast)
        launch_move_t<C, true>(bin, a, grid, log2s_max, s);
    else
        launch_move_t<C, false>(bin, a, grid, log2s_max, s);
}
template void launch_move<CfgNarrow>(int, bool, const MoveArgs<CfgNarrow> &, int, int,
                                     hipStream_t);
template void launch_move<CfgWideIn>(int, bool, const MoveArgs<CfgWideIn> &, int, int,
                                     hipStream_t);
template void launch_move<CfgWide>(int, bool, const MoveArgs<CfgWide> &, int, int, hipStream_t);
template void launch_move<CfgWideIn32>(int, bool, const MoveArgs<CfgWideIn32> &, int, int,
                                       hipStream_t);

template <class C>
void launch_move_hubs(bool fast, const MoveArgs<C> &a, int32_t sort_slices, int32_t parts,
                      int grid, int64_t *scratch, hipStream_t s)
{
    typedef typename C::ST ST;
    if (sort_slices <= 0 || parts <= 0 || grid <= 0) return;
    // the launch covers sorting slices [slice_base, + sort_slices) and partitions
    // [part_base, + parts): all hubs, or the hubs of one colour class
    const int pb = a.part_base;
    // (the region holds 8 bytes per vertex, so the size rounds up to whole words)
    launch_fill_bytes_zero(a.hub_hd, ((int64_t)a.nhubs * (int64_t)sizeof(ST) + 7) & ~(int64_t)7, s);
    if (pb == 0 && a.pcur == a.pcount + parts) {
        launch_fill_bytes_zero(a.pcount + pb, 2 * (int64_t)parts * sizeof(int32_t), s);  // pcount, pcur
    } else {
        launch_fill_i32(a.pcount + pb, 0, parts, s);
        launch_fill_i32(a.pcur + pb, 0, parts, s);
    }
    // the slices and partitions of the round's queued hubs: the sorting kernels loop
    // over these lists instead of launching a workgroup for every slice of every hub
    int32_t *tmp = a.act_tmp;
    launch_hub_active_lists(a.hub_act, a.hslice, a.htslice, a.nhubs, a.hslices, a.htslices, tmp,
                            tmp + a.nhubs, tmp + 2 * a.nhubs, tmp + 3 * a.nhubs, a.n_act_s,
                            a.n_act_p, a.act_s, a.act_p, scratch, s);
    const int gs = sort_slices < 8192 ? sort_slices : 8192;
    const int gpt = parts < 4096 ? parts : 4096;
    k_hub_count<C><<<gs, 256, 0, s>>>(a);
    launch_exclusive_scan<int32_t, int32_t>(a.pcount + pb, a.poff + pb, parts, scratch, nullptr, s);
    k_hub_fill<C><<<gs, 256, 0, s>>>(a);
    const size_t bytes = ((size_t)1 << hub_plog2<ST>()) * (sizeof(typename C::VT) + 4);
    if (bytes > 65536) {
        // raise the dynamic-LDS limit of this kernel to what the launch asks for; a
        // failure shows up as a launch error at the caller's check
        if (hipFuncSetAttribute((const void *)&k_hub_part<C>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess)
            (void)hipGetLastError();
    }
    k_hub_part<C><<<gpt, 256, bytes, s>>>(a);
    if (fast)
        k_move_hub<C, true><<<grid, HUB_THREADS, 0, s>>>(a);
    else
        k_move_hub<C, false><<<grid, HUB_THREADS, 0, s>>>(a);
    k_hub_mark<C><<<gs, 256, 0, s>>>(a);
    launch_fill_u8(a.hub_act, 0, a.nhubs, s);  // every hub inactive again for the next round
}
template void launch_move_hubs<CfgNarrow>(bool, const MoveArgs<CfgNarrow> &, int32_t, int32_t,
                                          int, int64_t *, hipStream_t);
template void launch_move_hubs<CfgWideIn>(bool, const MoveArgs<CfgWideIn> &, int32_t, int32_t,
                                          int, int64_t *, hipStream_t);
template void launch_move_hubs<CfgWide>(bool, const MoveArgs<CfgWide> &, int32_t, int32_t, int,
                                        int64_t *, hipStream_t);
template void launch_move_hubs<CfgWideIn32>(bool, const MoveArgs<CfgWideIn32> &, int32_t, int32_t,
                                            int, int64_t *, hipStream_t);

}  // namespace lv
