// Host side of the C ABI: context, workspace layout, the pass loop of Alg. 1
// around the local-moving (Alg. 2) and aggregation (Alg. 3) kernels.
//
// Control stays on the device within a pass: every iteration ends with a
// one-thread kernel that applies the tolerance test of Alg. 2 and raises a
// done flag that all later kernels of the pass check, so the host enqueues
// iterations ahead and only reads the flag one iteration behind.  The host
// synchronises once per level (degree-bin sizes), once per pass (community
// count for the aggregation tolerance of Alg. 1) and once for the community
// bins of the aggregation.
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <cmath>
#include <new>
#include <vector>

#include "kernels.h"

using namespace lv;

namespace {

constexpr size_t ALIGN = 256;

struct Layout {
    size_t total;
    int sb;  // bytes of K', Sigma', table values and aggregated weights (4 or 8)
    int64_t scratch_elems;
    size_t scalars, Cp, top, K, Sig, size, fa, fb, binorder, worklist, vtmp, mv_c;
    size_t used, idmap, ccount, coff, ctot, cursor, members, cbinorder;
    size_t offA, offB, degA, degB, tgtA, tgtB, wA, wB;
    size_t hstage, hstage_w, wcnt, pk, pw, hsz, hoff, scratch;
    size_t bincnt, binoff, slA, slB, mpre, hub_act, hub_hd, hpart, pcnt, poff, sown, pown, wm0, act_s,
        act_p, act_tmp;
    size_t colour, front, corder, kcnt, koff, cbm;  // colour-ordered mode
    int64_t kmax;                              // (colour, bin) keys that fit kcnt / koff
    size_t gid[3], gvb[3], gW, gsum, gst, giter, gcomm, gsig, gs2;  // batches
};

Layout make_layout(int32_t n, int64_t nnz, int sb, int32_t G = 0)
{
    Layout L;
    memset(&L, 0, sizeof(L));
    size_t cur = 0;
    auto take = [&](size_t bytes) {
        const size_t o = cur;
        cur += (bytes + ALIGN - 1) / ALIGN * ALIGN;
        return o;
    };
    const size_t n1 = (size_t)n + 1;
    const size_t z = (size_t)(nnz > 0 ? nnz : 1);
    L.sb = sb;
    // a greedy colouring with k colours has an edge between every two classes, so
    // k(k - 1) <= nnz and k <= 1 + sqrt(nnz)
    L.kmax = (int64_t)NBINS * (2 + (int64_t)std::sqrt((double)z)) + 8;
    L.scratch_elems = scan_scratch_elems(std::max<int64_t>((int64_t)n1, L.kmax + 1));
    L.scalars = take(sizeof(DevScalars));
    L.Cp = take(4 * n1);
    L.top = take(4 * n1);
    L.K = take((size_t)sb * n1);
    L.Sig = take((size_t)sb * n1);
    L.size = take(4 * n1);
    L.fa = take(n1);
    L.fb = take(n1);
    L.binorder = take(4 * n1);
    L.worklist = take(4 * n1);
    L.vtmp = take(4 * n1);
    L.mv_c = take(4 * n1);
    L.used = take(4 * (n1 + 1));
    L.idmap = take(4 * (n1 + 1));
    L.ccount = take(4 * (n1 + 1));
    L.coff = take(4 * (n1 + 1));
    L.ctot = take(4 * (n1 + 1));
    L.cursor = take(4 * n1);
    L.members = take(4 * n1);
    L.cbinorder = take(4 * n1);
    L.offA = take(4 * (n1 + 1));
    L.offB = take(4 * (n1 + 1));
    L.degA = take(4 * n1);
    L.degB = take(4 * n1);
    L.tgtA = take(4 * z);
    L.tgtB = take(4 * z);
    L.wA = take((size_t)sb * z);
    L.wB = take((size_t)sb * z);
    // hub rows / hub communities: staged communities and partitioned pairs
    L.hstage = take(4 * z);
    L.hstage_w = take((size_t)sb * z);
    L.wcnt = take(4 * ((size_t)z / 1024 + 64));  // per aggregation window (>= 1/4096 entries)
    L.pk = take(4 * z);
    L.pw = take((size_t)sb * z);
    L.hsz = take(8 * (n1 + 1));
    L.hoff = take(8 * (n1 + 1));
    L.scratch = take(8 * (size_t)L.scratch_elems);
    const size_t nchunks = (size_t)bin_chunks(n) + 1;
    L.bincnt = take(4 * ((size_t)NBINS * nchunks + 8));
    L.binoff = take(4 * ((size_t)NBINS * nchunks + 8));
    L.slA = take(4 * (n1 + 1));
    L.slB = take(4 * (n1 + 1));
    L.mpre = take(4 * (n1 + 1));
    L.hub_act = take(n1);
    L.hub_hd = take(8 * n1);
    L.colour = take(4 * n1);
    L.front = take(4 * 2 * n1);
    L.corder = take(4 * n1);
    L.kcnt = take(4 * ((size_t)L.kmax + 1));
    L.koff = take(4 * ((size_t)L.kmax + 1));
    L.cbm = take(4 * 33 * ((size_t)z / 513 + 1));  // rows longer than 512 entries
    if (G > 0) {
        // batches: graph of each vertex and first vertex of each graph, for the
        // input level (0) and two ping-ponged aggregated levels
        const size_t g1 = (size_t)G + 1;
        for (int k = 0; k < 3; ++k) {
            L.gid[k] = take(4 * n1);
            L.gvb[k] = take(4 * g1);
        }
        L.gW = take(8 * g1);
        L.gsum = take(16 * g1);
        L.gst = take(4 * g1);
        L.giter = take(4 * g1);
        L.gcomm = take(4 * g1);
        L.gsig = take(8 * g1);
        L.gs2 = take(16 * g1);
    }
    // per partition of the hub rows (at most one per 2048 entries, plus one per hub)
    const size_t parts = (size_t)z / 512 + 64;
    L.hpart = take(32 * parts);
    L.pcnt = take(4 * 2 * parts);  // pcount then pcur
    L.poff = take(4 * parts);
    // owner of each partition, and of each sorting slice or window with the first
    // member reaching into it (hubs and hub communities hold more than 2048 entries,
    // so there are fewer than nnz/8192 + nnz/2048 slices and nnz/4096 + nnz/2048
    // windows)
    L.pown = take(4 * parts);
    L.sown = take(4 * (z / 1024 + 64));
    L.wm0 = take(4 * (z / 1024 + 64));
    // the round's queued hubs: their slices and partitions, and per-hub counts and
    // offsets (fewer than nnz/2048 hubs)
    L.act_s = take(4 * (z / 1024 + 64));
    L.act_p = take(4 * parts);
    L.act_tmp = take(4 * 4 * (z / 2048 + 64));
    L.total = cur;
    return L;
}

enum State { S_READY = 0, S_MOVED = 1, S_STOPPED = 2, S_EXHAUSTED = 3, S_DONE = 4 };

struct LevelH {
    int32_t n;
    const int32_t *off, *deg, *tgt;
    const void *w;
    int wbytes;
    int buf;  // -1 input, 0 = A, 1 = B
    int64_t entries;
};

// Kernel families timed with HIP events when profiling.
enum Fam {
    F_MOVE0 = 0,       // .. F_MOVE0 + NBINS - 1
    F_AGG0 = NBINS,    // .. F_AGG0 + NBINS - 1
    F_COMPACT = 2 * NBINS,
    F_APPLY,
    F_ITER,
    F_SETUP,
    F_AGGPREP,
    F_FINAL,
    F_COLOUR,
    F_SEQ,
    F_COUNT
};
const char *FAM_NAMES[F_COUNT] = {
    "move_bin0_1lane", "move_bin1_4lanes", "move_bin2_16lanes", "move_bin3_wave",
    "move_bin4_block", "move_bin5_bigblock", "move_bin6_hub", "agg_bin0_4lanes",
    "agg_bin1_4lanes", "agg_bin2_8lanes", "agg_bin3_wave", "agg_bin4_block",
    "agg_bin5_bigblock", "agg_bin6_hub", "compact", "apply", "iteration_end", "level_setup",
    "aggregate_prep", "final", "colour", "move_seq"};
static_assert(F_COUNT == 2 * NBINS + 8, "family names");

struct Pending {
    int fam;
    hipEvent_t a, b;
    int pass;  // pass whose phase the launch belongs to
};

// Phase of a kernel family in the per-pass split of louvain_stats (the split
// of Section 5.3: local moving, aggregation, other): 0 local moving, 1
// aggregation (renumbering and the community-vertex CSR included), 2 other
// (level setup, modularity).
int phase_of(int fam)
{
    if (fam >= F_MOVE0 && fam < F_MOVE0 + NBINS) return 0;
    if (fam == F_COMPACT || fam == F_APPLY || fam == F_ITER || fam == F_COLOUR || fam == F_SEQ)
        return 0;
    if (fam >= F_AGG0 && fam < F_AGG0 + NBINS) return 1;
    if (fam == F_AGGPREP) return 1;
    return 2;
}

thread_local const char *g_last_hip_error = "no HIP error";

// Pinned host blocks for the scalar read-backs, kept in a process-wide pool:
// freeing pinned memory synchronises the whole device, which would make
// contexts created and destroyed next to running ones (a server's batches)
// wait for every stream.  A block goes back to the pool when its context is
// destroyed and is reused by the next one; the pool is held until the
// process ends.
struct PinnedBlock {
    DevScalars *hsc;
    int32_t *done;
};
std::mutex g_pinned_mu;
std::vector<PinnedBlock> g_pinned_pool;

bool pinned_take(PinnedBlock *b)
{
    {
        std::lock_guard<std::mutex> lk(g_pinned_mu);
        if (!g_pinned_pool.empty()) {
            *b = g_pinned_pool.back();
            g_pinned_pool.pop_back();
            return true;
        }
    }
    b->hsc = nullptr;
    b->done = nullptr;
    if (hipHostMalloc((void **)&b->hsc, sizeof(DevScalars), hipHostMallocDefault) == hipSuccess &&
        hipHostMalloc((void **)&b->done, sizeof(int32_t) * (LOUVAIN_MAX_ITERATIONS + 1),
                      hipHostMallocDefault) == hipSuccess)
        return true;
    // allocation failure (rare): give back what was obtained
    if (b->hsc) (void)hipHostFree(b->hsc);
    b->hsc = nullptr;
    b->done = nullptr;
    return false;
}

// Both pointers come from one pinned_take.
void pinned_give(DevScalars *hsc, int32_t *done)
{
    if (!hsc || !done) return;
    std::lock_guard<std::mutex> lk(g_pinned_mu);
    g_pinned_pool.push_back(PinnedBlock{hsc, done});
}

}  // namespace

struct louvain_ctx {
    louvain_params p;
    hipStream_t s;
    // batches: a second stream on which the small graphs' wavefront kernel runs beside
    // the degree bins of the others, with the events that fork and join it
    hipStream_t s2;
    hipEvent_t fork_ev, join_ev;
    int32_t n;
    int64_t nnz;
    const int32_t *in_off, *in_tgt, *in_w;
    unsigned char *ws;
    Layout L;
    DevScalars *sc;
    DevScalars *hsc;  // pinned host copy
    int32_t *pinned_done;
    hipEvent_t it_ev[2];
    // louvain_run_noalloc: read-backs into this pageable memory instead of a
    // pinned block, and no events (the host waits on the stream each iteration)
    bool noalloc;
    DevScalars own_hsc;
    int32_t own_done[LOUVAIN_MAX_ITERATIONS + 1];
    int32_t *Cp, *top, *size, *binorder, *worklist, *vtmp, *mv_c;
    int32_t *used, *idmap, *ccount, *coff, *ctot, *cursor, *members, *cbinorder;
    uint8_t *fa, *fb;
    void *K, *Sig;
    int32_t *off_buf[2], *deg_buf[2], *tgt_buf[2];
    void *w_buf[2];
    int32_t *hstage, *pk, *wcnt;
    void *pw, *hstage_w;
    int64_t *hsz, *hoff, *scratch;
    int32_t *bincnt, *binoff, *slA, *slB, *mpre;
    void *hpart;
    int32_t *pcnt, *poff;
    int32_t *sown, *pown, *wm0;  // owners of hub slices / partitions, first member per window
    int32_t *act_s, *act_p, *act_tmp;  // the round's queued hubs: slices, partitions, scratch
    int64_t owner_cap, part_cap; // their capacities
    uint8_t *hub_act;
    unsigned char *hub_hd;  // per hub: weight into its own community (moving, 4 or 8 bytes)
    // colour-ordered mode: colour of each row, frontier lists of the colouring,
    // rows sorted by (colour, bin), key counts and offsets (device and host)
    int32_t *colour, *front, *corder, *kcnt, *koff;
    uint32_t *cbm;
    int32_t ncol;        // colours of the current level
    std::vector<int32_t> koff_h;
    std::vector<int32_t> hub_sl_h, hub_pt_h;  // first sorting slice / partition per hub (hubs + 1)
    // batches of independent graphs (G = 0 for a single graph)
    int32_t G;
    int32_t *gid[3], *gvb[3];
    int64_t *gW;
    unsigned long long *gsum, *gsig, *gs2;
    int32_t *gst, *giter, *gcomm;
    int glev;                 // which gid/gvb pair the current level uses (0 = input)
    const int32_t *warm;      // labels the first pass starts from (louvain_set_membership)
    std::vector<double> gq;   // per-graph modularity of the finished run
    int32_t hub_slices;  // row slices of the current level's hubs
    int32_t hub_tslices; // partitions of the current level's hub rows
    int64_t W;
    int32_t wmax;        // largest input weight
    bool wide;
    unsigned long long kmax_in;  // largest K' of the input level (wide graphs, after its setup)
    int32_t lds_max;     // LDS row limit of the bins (LDS_MAX_NARROW or LDS_MAX_WIDE)
    int32_t bin_maxlen[NBINS];
    int state;
    int pass;
    double tau;
    int32_t iters_last;
    double dq_last;
    LevelH lev;
    BinInfo bins;
    int32_t nb;
    louvain_stats st;
    // per-iteration trace of the last move
    std::vector<i128> tr_sum;
    std::vector<int64_t> tr_moves, tr_proc;
    // profiling
    std::vector<hipEvent_t> ev_free;
    std::vector<Pending> pending;
    double fam_ms[F_COUNT];
    int64_t fam_launches[F_COUNT];
    double fam_bytes[F_COUNT];
    hipError_t last_err;
};

namespace {

#define CK(x)                                                   \
    do {                                                        \
        hipError_t e_ = (x);                                    \
        if (e_ != hipSuccess) {                                 \
            ctx->last_err = e_;                                 \
            g_last_hip_error = hipGetErrorString(e_);           \
            return LOUVAIN_EHIP;                                \
        }                                                       \
    } while (0)

#define CKL() CK(hipGetLastError())

#define TRY(x)                          \
    do {                                \
        int r_ = (x);                   \
        if (r_ != LOUVAIN_OK) return r_; \
    } while (0)

int bins_of(louvain_ctx *ctx, int b) { return ctx->bins.start[b + 1] - ctx->bins.start[b]; }

// Batch arguments of the current level (all null for a single graph).
BatchArgs batch_args(louvain_ctx *ctx)
{
    BatchArgs b;
    memset(&b, 0, sizeof(b));
    if (ctx->G <= 0) return b;
    b.gid = ctx->gid[ctx->glev];
    b.gvb = ctx->gvb[ctx->glev];
    b.gW = ctx->gW;
    b.gsum = ctx->gsum;
    b.gst = ctx->gst;
    b.giter = ctx->giter;
    b.G = ctx->G;
    return b;
}

// ---------------------------------------------------------------- profiling
int prof_begin(louvain_ctx *ctx, hipEvent_t *ev)
{
    *ev = nullptr;
    if (!ctx->p.profile) return LOUVAIN_OK;
    if (ctx->ev_free.empty()) {
        hipEvent_t e;
        CK(hipEventCreate(&e));
        ctx->ev_free.push_back(e);
    }
    *ev = ctx->ev_free.back();
    ctx->ev_free.pop_back();
    CK(hipEventRecord(*ev, ctx->s));
    return LOUVAIN_OK;
}

int prof_end(louvain_ctx *ctx, int fam, hipEvent_t a)
{
    if (!ctx->p.profile || !a) return LOUVAIN_OK;
    hipEvent_t b;
    if (ctx->ev_free.empty()) {
        CK(hipEventCreate(&b));
    } else {
        b = ctx->ev_free.back();
        ctx->ev_free.pop_back();
    }
    CK(hipEventRecord(b, ctx->s));
    ctx->pending.push_back(Pending{fam, a, b, ctx->pass});
    return LOUVAIN_OK;
}

// Called after the stream has been synchronised.
int prof_collect(louvain_ctx *ctx)
{
    for (const Pending &q : ctx->pending) {
        float ms = 0.f;
        CK(hipEventElapsedTime(&ms, q.a, q.b));
        ctx->fam_ms[q.fam] += ms;
        ctx->fam_launches[q.fam] += 1;
        // the modularity after the last pass goes to that pass
        int p = q.pass;
        if (q.fam == F_FINAL && p >= ctx->st.passes && ctx->st.passes > 0) p = ctx->st.passes - 1;
        if (p < LOUVAIN_MAX_PASSES) {
            const int ph = phase_of(q.fam);
            double *acc = ph == 0 ? ctx->st.ms_move : (ph == 1 ? ctx->st.ms_aggregate : ctx->st.ms_other);
            acc[p] += ms;
        }
        ctx->ev_free.push_back(q.a);
        ctx->ev_free.push_back(q.b);
    }
    ctx->pending.clear();
    return LOUVAIN_OK;
}

int sync_stream(louvain_ctx *ctx)
{
    CK(hipStreamSynchronize(ctx->s));
    return prof_collect(ctx);
}

int read_scalars(louvain_ctx *ctx)
{
    CK(hipMemcpyAsync(ctx->hsc, ctx->sc, offsetof(DevScalars, spread), hipMemcpyDeviceToHost,
                      ctx->s));
    return sync_stream(ctx);
}

template <class C>
const typename C::WT *lev_w(const LevelH &l)
{
    return (const typename C::WT *)l.w;
}

// Staging offsets, sorting slices and partitions of the hub rows in binorder
// order (cursor and ccount are free during moving).
template <class C>
int hub_layout(louvain_ctx *ctx)
{
    hipStream_t s = ctx->s;
    const LevelH &l = ctx->lev;
    const int hubs = bins_of(ctx, NBINS - 1);
    launch_hub_move_sizes(ctx->binorder, ctx->bins.start[NBINS - 1], ctx->bins.start[NBINS], l.off, l.deg,
                          (int)sizeof(typename C::ST), ctx->hsz, ctx->cursor, ctx->ccount, s, HUB_PSLICE,
                          ctx->p.hub_part_pairs);
    launch_exclusive_scan<int64_t, int64_t>(ctx->hsz, ctx->hoff, hubs, ctx->scratch, nullptr, s);
    launch_exclusive_scan<int32_t, int32_t>(ctx->cursor, ctx->slA, hubs, ctx->scratch,
                                            &ctx->sc->hub_slices, s);
    launch_exclusive_scan<int32_t, int32_t>(ctx->ccount, ctx->slB, hubs, ctx->scratch,
                                            &ctx->sc->hub_tslices, s);
    launch_fill_u8(ctx->hub_act, 0, hubs, s);
    CKL();
    return LOUVAIN_OK;
}

// ---------------------------------------------------------------- level setup (Alg. 1 per-pass reset)
template <class C>
int setup_level(louvain_ctx *ctx)
{
    hipStream_t s = ctx->s;
    const LevelH &l = ctx->lev;
    hipEvent_t ev;
    TRY(prof_begin(ctx, &ev));
    launch_fill_bytes_zero(ctx->sc, offsetof(DevScalars, err), s);
    CKL();
    launch_fill_bytes_zero(ctx->sc->spread, sizeof(ctx->sc->spread), s);
    CKL();
    if (ctx->G > 0) {
        launch_batch_pass_begin(batch_args(ctx), s);
        CKL();
    }
    launch_init_vertices(l.n, ctx->Cp, ctx->size, ctx->fa, ctx->fb, ctx->K, ctx->Sig, ctx->L.sb, s);
    launch_fill_i32(ctx->mv_c, -1, l.n, s);  // no deferred move (deterministic rounds)
    launch_bin_count(l.n, l.off, l.deg, ctx->lds_max, ctx->bincnt, ctx->binoff, ctx->scratch,
                     ctx->sc->bin_start, ctx->sc->bin_maxlen, s);
    CKL();
    TRY(prof_end(ctx, F_SETUP, ev));
    TRY(read_scalars(ctx));
    for (int b = 0; b <= NBINS; ++b) ctx->bins.start[b] = ctx->hsc->bin_start[b];
    for (int b = 0; b < NBINS; ++b) ctx->bin_maxlen[b] = ctx->hsc->bin_maxlen[b];
    ctx->nb = ctx->bins.start[NBINS];
    TRY(prof_begin(ctx, &ev));
    launch_bin_fill(l.n, l.off, l.deg, ctx->lds_max, ctx->binoff, ctx->binorder, s);
    CKL();
    const int hubs = bins_of(ctx, NBINS - 1);
    ctx->hub_slices = 0;
    ctx->hub_tslices = 0;
    if (hubs > 0) TRY(hub_layout<C>(ctx));
    for (int b = 0; b < NBINS; ++b) {
        RowArgs<C> r;
        r.off = l.off;
        r.deg = l.deg;
        r.tgt = l.tgt;
        r.w = lev_w<C>(l);
        r.binorder = ctx->binorder;
        r.begin = ctx->bins.start[b];
        r.count = bins_of(ctx, b);
        r.K = (typename C::ST *)ctx->K;
        r.Sig = (typename C::ST *)ctx->Sig;
        r.labels = nullptr;
        r.sigma = nullptr;
        r.hslice = b == NBINS - 1 ? ctx->slA : nullptr;  // hub_layout above
        r.nslices = &ctx->sc->hub_slices;
        launch_row_reduce<C>(b, 0, r, s);
        CKL();
    }
    if (ctx->pass == 0 && ctx->warm) {
        // warm start: the first pass starts from the caller's partition
        launch_fill_bytes_zero(ctx->Sig, (int64_t)ctx->L.sb * l.n, s);
        launch_fill_bytes_zero(ctx->size, 4 * (int64_t)l.n, s);
        launch_warm_labels<typename C::ST>(l.n, ctx->warm, (const typename C::ST *)ctx->K,
                                           ctx->Cp, (typename C::ST *)ctx->Sig, ctx->size, s);
        CKL();
    }
    // the input level of a wide graph: its largest K' decides the width of the
    // local-moving tables
    const bool want_kmax = ctx->wide && l.buf < 0;
    if (want_kmax) {
        launch_max_u64((const int64_t *)ctx->K, l.n, &ctx->sc->kmax, s);
        CKL();
    }
    TRY(prof_end(ctx, F_SETUP, ev));
    if (hubs > 0 || want_kmax) {
        TRY(read_scalars(ctx));
        if (hubs > 0) {
            ctx->hub_slices = (int32_t)ctx->hsc->hub_slices;
            ctx->hub_tslices = (int32_t)ctx->hsc->hub_tslices;
            // excluded by the layout's bounds on slices and partitions
            if (ctx->hub_slices > ctx->owner_cap || ctx->hub_tslices > ctx->part_cap)
                return LOUVAIN_EINVAL;
            launch_owner_map(ctx->slA, hubs, ctx->hub_slices, ctx->sown, s);
            launch_owner_map(ctx->slB, hubs, ctx->hub_tslices, ctx->pown, s);
            CKL();
        }
        if (want_kmax) ctx->kmax_in = ctx->hsc->kmax;
    }
    return LOUVAIN_OK;
}

// ---------------------------------------------------------------- colouring
// Colour the level's rows (Jones-Plassmann frontiers until one is empty), then
// sort the rows by (colour, bin) and read the key offsets back: round r of an
// iteration visits order[koff[r * NBINS], koff[(r + 1) * NBINS]).  With
// symmetric rows the uncoloured vertex of highest priority is always in the
// frontier, so the frontiers empty exactly when every row is coloured; rows
// that are not symmetric can leave vertices waiting forever, which is
// reported as LOUVAIN_EINVAL.
template <class C>
int colour_level(louvain_ctx *ctx)
{
    hipStream_t s = ctx->s;
    const LevelH &l = ctx->lev;
    hipEvent_t ev;
    TRY(prof_begin(ctx, &ev));
    ColourArgs a;
    memset(&a, 0, sizeof(a));
    a.off = l.off;
    a.deg = l.deg;
    a.tgt = l.tgt;
    a.binorder = ctx->binorder;
    a.colour = ctx->colour;
    a.ncol = &ctx->sc->ncol;
    a.coloured = &ctx->sc->coloured;
    a.cbm = ctx->cbm;
    a.seed = ctx->p.seed;
    a.pass = ctx->pass;
    a.bt = batch_args(ctx);
    // degree classes: bins 0, 1, 2, 3 and 4-6
    a.cstart[0] = ctx->bins.start[0];
    a.cstart[1] = ctx->bins.start[1];
    a.cstart[2] = ctx->bins.start[2];
    a.cstart[3] = ctx->bins.start[3];
    a.cstart[4] = ctx->bins.start[4];
    a.cstart[5] = ctx->bins.start[NBINS];
    static_assert(offsetof(DevScalars, ncol) == offsetof(DevScalars, fcount) + 3 * NCLS * sizeof(int32_t),
                  "ncol follows the frontier counts");
    // blocks per class for frontiers of the given sizes (at least one per
    // non-empty class, since a frontier can grow between two host reads)
    auto set_grid = [&](const int32_t *sizes) {
        int nb = 0;
        for (int q = 0; q < NCLS; ++q) {
            a.rblk[q] = nb;
            const int64_t cls = (int64_t)a.cstart[q + 1] - a.cstart[q];
            if (cls <= 0) continue;
            const int per = COLOUR_CT / colour_lanes(q);
            int64_t g = ((int64_t)std::min<int64_t>(sizes[q], cls) + per - 1) / per;
            if (q == NCLS - 1) g = std::max<int64_t>(8, 4 * g);  // chunks of long rows
            nb += (int)std::max<int64_t>(1, std::min<int64_t>(g, 256));
        }
        a.rblk[NCLS] = nb;
    };
    const size_t stride = (size_t)ctx->n + 1;  // each frontier list holds up to nb <= n rows
    launch_fill_i32(&ctx->sc->fcount[0][0], 0, 3 * NCLS + 1, s);  // counts and ncol
    launch_fill_i32(&ctx->sc->coloured, 0, 1, s);
    launch_fill_i32((int32_t *)ctx->cbm, 0, 33 * ((int64_t)a.cstart[NCLS] - a.cstart[NCLS - 1]), s);
    int32_t est[NCLS];
    for (int q = 0; q < NCLS; ++q) est[q] = a.cstart[q + 1] - a.cstart[q];
    set_grid(est);
    a.out = ctx->front;
    a.out_count = ctx->sc->fcount[0];
    launch_colour_init(a, s);
    CKL();
    int64_t k = 0;  // steps launched; step k reads list k & 1 and count slot k % 3
    int group = 8;
    for (;;) {
        for (int j = 0; j < group; ++j, ++k) {
            a.in = ctx->front + (size_t)(k & 1) * stride;
            a.in_count = ctx->sc->fcount[k % 3];
            a.out = ctx->front + (size_t)((k + 1) & 1) * stride;
            a.out_count = ctx->sc->fcount[(k + 1) % 3];
            a.clear_count = ctx->sc->fcount[(k + 2) % 3];
            launch_colour_step(a, s);
        }
        CKL();
        CK(hipMemcpyAsync(&ctx->hsc->fcount[0][0], &ctx->sc->fcount[0][0],
                          (3 * NCLS + 1) * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        CK(hipMemcpyAsync(&ctx->hsc->coloured, &ctx->sc->coloured, sizeof(int32_t),
                          hipMemcpyDeviceToHost, s));
        CK(hipStreamSynchronize(s));
        const int32_t *f = ctx->hsc->fcount[k % 3];  // the frontier the last step produced
        int64_t total = 0;
        for (int q = 0; q < NCLS; ++q) total += f[q];
        if (total == 0) break;
        set_grid(f);
        group = total < 4096 ? 32 : 8;
    }
    if (ctx->hsc->coloured != ctx->nb) return LOUVAIN_EINVAL;
    ctx->ncol = ctx->hsc->ncol;
    const int hubs = bins_of(ctx, NBINS - 1);
    if (hubs > 0) {
        // order the hubs by colour (stable), so that each colour's hubs are
        // consecutive and a round launches the hub kernels over their slices only
        int32_t *hub_ids = ctx->binorder + ctx->bins.start[NBINS - 1];
        std::vector<int32_t> ids(hubs), col(hubs);
        launch_gather_i32(ctx->colour, hub_ids, hubs, ctx->vtmp, s);
        CKL();
        CK(hipMemcpyAsync(ids.data(), hub_ids, hubs * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        CK(hipMemcpyAsync(col.data(), ctx->vtmp, hubs * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        CK(hipStreamSynchronize(s));
        std::vector<int32_t> idx(hubs);
        for (int h = 0; h < hubs; ++h) idx[h] = h;
        std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) { return col[x] < col[y]; });
        std::vector<int32_t> sorted(hubs);
        for (int h = 0; h < hubs; ++h) sorted[h] = ids[idx[h]];
        CK(hipMemcpyAsync(hub_ids, sorted.data(), hubs * sizeof(int32_t), hipMemcpyHostToDevice, s));
        TRY(hub_layout<C>(ctx));
        // same totals as before the reordering; the owners follow the new order
        launch_owner_map(ctx->slA, hubs, ctx->hub_slices, ctx->sown, s);
        launch_owner_map(ctx->slB, hubs, ctx->hub_tslices, ctx->pown, s);
        CKL();
        ctx->hub_sl_h.assign((size_t)hubs + 1, 0);
        ctx->hub_pt_h.assign((size_t)hubs + 1, 0);
        CK(hipMemcpyAsync(ctx->hub_sl_h.data(), ctx->slA, ((size_t)hubs + 1) * sizeof(int32_t),
                          hipMemcpyDeviceToHost, s));
        CK(hipMemcpyAsync(ctx->hub_pt_h.data(), ctx->slB, ((size_t)hubs + 1) * sizeof(int32_t),
                          hipMemcpyDeviceToHost, s));
        CK(hipStreamSynchronize(s));
    }
    const int64_t nkeys = (int64_t)ctx->ncol * NBINS;
    if (nkeys > ctx->L.kmax) return LOUVAIN_EINVAL;  // excluded by the bound on colours
    if (nkeys > 0) {
        launch_fill_i32(ctx->kcnt, 0, nkeys + 1, s);
        launch_class_count(ctx->binorder, ctx->nb, ctx->bins, ctx->colour, (int32_t)nkeys, ctx->kcnt,
                           s);
        launch_exclusive_scan<int32_t, int32_t>(ctx->kcnt, ctx->koff, nkeys, ctx->scratch, nullptr, s);
        CK(hipMemcpyAsync(ctx->kcnt, ctx->koff, (size_t)nkeys * sizeof(int32_t),
                          hipMemcpyDeviceToDevice, s));
        launch_class_fill(ctx->binorder, ctx->nb, ctx->bins, ctx->colour, (int32_t)nkeys, ctx->kcnt,
                          ctx->corder, s);
        CKL();
    }
    ctx->koff_h.assign((size_t)nkeys + 1, 0);
    if (nkeys > 0)
        CK(hipMemcpyAsync(ctx->koff_h.data(), ctx->koff, ((size_t)nkeys + 1) * sizeof(int32_t),
                          hipMemcpyDeviceToHost, s));
    CK(hipStreamSynchronize(s));
    if (nkeys > 0 && ctx->koff_h[(size_t)nkeys] != ctx->nb) return LOUVAIN_EINVAL;
    TRY(prof_end(ctx, F_COLOUR, ev));
    return LOUVAIN_OK;
}

// ---------------------------------------------------------------- local moving (Alg. 2)
template <class C>
int move_phase(louvain_ctx *ctx, bool level_ready = false)
{
    typedef typename C::ST ST;
    hipStream_t s = ctx->s;
    const LevelH &l = ctx->lev;
    if (!level_ready) TRY(setup_level<C>(ctx));
    const bool fast = ctx->p.mode == LOUVAIN_FAST;
    const bool coloured = ctx->p.mode == LOUVAIN_COLOURED;
    if (coloured) TRY(colour_level<C>(ctx));
    const int rounds = coloured ? ctx->ncol : 1 << ctx->p.round_bits;
    const int max_it = ctx->p.max_iterations;
    MoveArgs<C> a;
    a.off = l.off;
    a.deg = l.deg;
    a.tgt = l.tgt;
    a.w = lev_w<C>(l);
    a.binorder = ctx->binorder;
    a.worklist = ctx->worklist;
    a.Cp = ctx->Cp;
    a.K = (const ST *)ctx->K;
    a.Sig = (ST *)ctx->Sig;
    a.size = ctx->size;
    a.mv_c = ctx->mv_c;
    a.spread = &ctx->sc->spread[0][0];
    a.hstage = ctx->hstage;
    a.pcount = ctx->pcnt;
    a.pcur = ctx->pcnt + ctx->hub_tslices;  // zeroed together with pcount every round
    a.poff = ctx->poff;
    a.pk = ctx->pk;
    a.pw = (ST *)ctx->pw;
    a.hoff = ctx->hoff;
    a.hslice = ctx->slA;
    a.htslice = ctx->slB;
    a.sown = ctx->sown;
    a.pown = ctx->pown;
    a.act_s = ctx->act_s;
    a.act_p = ctx->act_p;
    a.act_tmp = ctx->act_tmp;
    a.n_act_s = &ctx->sc->act_slices;
    a.n_act_p = &ctx->sc->act_parts;
    a.hslices = &ctx->sc->hub_slices;
    a.htslices = &ctx->sc->hub_tslices;
    a.hpart = ctx->hpart;
    a.hub_act = ctx->hub_act;
    a.hub_hd = (ST *)ctx->hub_hd;
    a.nhubs = bins_of(ctx, NBINS - 1);
    a.done = &ctx->sc->done;
    a.W = ctx->W;
    a.rule = coloured ? 0 : 1;  // min-label singleton rule: only where neighbours share rounds
    a.slice_base = 0;
    a.part_base = 0;
    int32_t hub0 = 0;  // colour-ordered rounds: first hub (in binorder) of the round's colour
    a.bt = batch_args(ctx);
    int grid[NBINS], log2s[NBINS];
    for (int b = 0; b < NBINS; ++b) {
        const int cnt = bins_of(ctx, b);
        const int per = move_rows_per_block(b);
        int g = (cnt + per - 1) / per;
        const int cap = b >= 4 ? 1024 : 2048;
        grid[b] = std::min(g, cap);
        log2s[b] = block_log2s(ctx->bin_maxlen[b]);
    }
    // levels (in a batch: graphs) of at most `small` vertices are moved by one
    // wavefront each, every iteration in one launch (fast mode: in vertex order;
    // deterministic mode: in the same synchronous rounds); the bins below handle the rest
    // (default: fast mode SEQ_MAX, for its quality; deterministic mode none, whose
    // result is the same either way and whose bins are faster on the measured batches)
    const int small = ctx->p.small_level == 0 ? (fast ? SEQ_MAX : 0)
                                              : (ctx->p.small_level < 0 ? 0 : ctx->p.small_level);
    bool seq_all = false;
    bool seq_joined = true;
    if (!coloured && small > 0 && (ctx->G > 0 || (l.n >= 1 && l.n <= small))) {
        SeqArgs<C> q;
        q.off = l.off;
        q.deg = l.deg;
        q.tgt = l.tgt;
        q.w = lev_w<C>(l);
        q.Cp = ctx->Cp;
        q.K = (const ST *)ctx->K;
        q.Sig = (ST *)ctx->Sig;
        q.size = ctx->size;
        q.act = ctx->fa;  // the flags of iteration 0 (graphs left to the rounds keep theirs)
        q.mark = ctx->fb;
        q.rule = 1;
        q.seed = ctx->p.seed;
        q.round_bits = ctx->p.round_bits;
        q.pass = ctx->pass;
        q.n = l.n;
        q.max_n = small;
        q.W = ctx->W;
        q.tau = ctx->tau;
        q.max_iter = max_it;
        q.prune = ctx->p.prune;
        q.sc = ctx->sc;
        q.bt = a.bt;
        if (ctx->G == 0) {
            hipEvent_t ev;
            TRY(prof_begin(ctx, &ev));
            launch_seq_level<C>(q, fast, 1, s);
            CKL();
            TRY(prof_end(ctx, F_SEQ, ev));
            seq_all = true;
        } else {
            launch_batch_mark_small(a.bt, small, s);
            CKL();
            if (ctx->s2) {
                // the small graphs on the second stream, beside the bins of the others
                // (disjoint vertex ranges); joined before the phase ends
                CK(hipEventRecord(ctx->fork_ev, s));
                CK(hipStreamWaitEvent(ctx->s2, ctx->fork_ev, 0));
                launch_seq_level<C>(q, fast, ctx->G, ctx->s2);
                CKL();
                CK(hipEventRecord(ctx->join_ev, ctx->s2));
                seq_joined = false;
            } else {
                launch_seq_level<C>(q, fast, ctx->G, s);
                CKL();
            }
        }
    }
    int it;
    for (it = 0; !seq_all && it < max_it; ++it) {
        uint8_t *cur = (it & 1) ? ctx->fb : ctx->fa;
        uint8_t *nxt = (it & 1) ? ctx->fa : ctx->fb;
        a.flags_next = nxt;
        if (coloured && ctx->ncol > 0) {
            // every round's rows but the hubs, compacted once: the active set of an
            // iteration is fixed when it starts (movers flag the next one)
            const int32_t nkeys = ctx->ncol * NBINS;
            CompactArgs ka;
            memset(&ka, 0, sizeof(ka));
            ka.binorder = ctx->binorder;
            ka.nb = ctx->nb;
            ka.bins = ctx->bins;
            ka.flags = cur;
            ka.prune = ctx->p.prune;
            ka.pass = ctx->pass;
            ka.it = it;
            ka.seed = ctx->p.seed;
            ka.order = ctx->corder;
            ka.q0 = 0;
            ka.q1 = ctx->nb;
            ka.hub_act = ctx->hub_act;
            ka.done = &ctx->sc->done;
            ka.bt = a.bt;
            hipEvent_t ev;
            TRY(prof_begin(ctx, &ev));
            launch_fill_i32(ctx->kcnt, 0, nkeys, s);
            launch_compact_keys(ka, ctx->koff, nkeys, ctx->kcnt, ctx->front, &ctx->sc->processed[it], s);
            CKL();
            TRY(prof_end(ctx, F_COMPACT, ev));
        }
        for (int r = 0; r < rounds; ++r) {
            int rgrid[NBINS];
            int32_t hub1 = 0;
            for (int b = 0; b < NBINS; ++b) rgrid[b] = grid[b];
            CompactArgs ca;
            ca.order = nullptr;
            ca.q0 = ca.q1 = 0;
            if (coloured) {
                // round r: the rows of colour r, per bin from the (colour, bin) key offsets
                const int32_t *ko = &ctx->koff_h[(size_t)r * NBINS];
                ca.order = ctx->corder;
                ca.q0 = ko[0];
                ca.q1 = ko[NBINS];
                for (int b = 0; b < NBINS; ++b) {
                    const int per = move_rows_per_block(b);
                    const int64_t g = ((int64_t)ko[b + 1] - ko[b] + per - 1) / per;
                    rgrid[b] = (int)std::min<int64_t>(g, b >= 4 ? 1024 : 2048);
                }
                if (r == 0) hub0 = 0;
                hub1 = hub0 + (ko[NBINS] - ko[NBINS - 1]);
            }
            ca.binorder = ctx->binorder;
            ca.nb = ctx->nb;
            ca.bins = ctx->bins;
            ca.flags = cur;
            ca.prune = ctx->p.prune;
            ca.round = r;
            ca.round_bits = coloured ? 0 : ctx->p.round_bits;  // a colour class is the whole round
            ca.pass = ctx->pass;
            ca.it = it;
            ca.seed = ctx->p.seed;
            ca.worklist = ctx->worklist;
            ca.counts = ctx->sc->bin_count;
            ca.hub_act = ctx->hub_act;
            ca.done = &ctx->sc->done;
            ca.bt = a.bt;
            ca.hubs_only = coloured ? 1 : 0;  // the other rows: launch_compact_keys above
            hipEvent_t ev;
            if (!coloured || hub1 > hub0) {
                TRY(prof_begin(ctx, &ev));
                launch_compact(ca, s);
                CKL();
                TRY(prof_end(ctx, F_COMPACT, ev));
            }
            for (int b = 0; b < NBINS; ++b) {
                if (rgrid[b] <= 0) continue;
                if (coloured && b < NBINS - 1) {
                    // round r's rows of bin b, from the per-iteration keyed compaction
                    a.worklist = ctx->front;
                    a.list_begin = ctx->koff_h[(size_t)r * NBINS + b];
                    a.count = ctx->kcnt + (size_t)r * NBINS + b;
                } else {
                    a.worklist = ctx->worklist;
                    a.list_begin = ctx->bins.start[b];
                    a.count = &ctx->sc->bin_count[b];
                }
                a.bin = b;
                TRY(prof_begin(ctx, &ev));
                if (b < NBINS - 1) {
                    launch_move<C>(b, fast, a, rgrid[b], log2s[b], s);
                } else if (!coloured) {
                    launch_move_hubs<C>(fast, a, ctx->hub_slices, ctx->hub_tslices, rgrid[b],
                                        ctx->scratch, s);
                } else {
                    // the round's hubs are hubs [hub0, hub1) of the colour-sorted hub bin
                    a.slice_base = ctx->hub_sl_h[hub0];
                    a.part_base = ctx->hub_pt_h[hub0];
                    launch_move_hubs<C>(fast, a, ctx->hub_sl_h[hub1] - a.slice_base,
                                        ctx->hub_pt_h[hub1] - a.part_base, rgrid[b], ctx->scratch, s);
                    a.slice_base = 0;
                    a.part_base = 0;
                }
                CKL();
                TRY(prof_end(ctx, F_MOVE0 + b, ev));
            }
            TRY(prof_begin(ctx, &ev));
            if (!fast) {
                launch_apply<ST>(ctx->mv_c, l.n, ctx->Cp, (const ST *)ctx->K, (ST *)ctx->Sig,
                                 ctx->size, &ctx->sc->done, s);
                CKL();
            }
            launch_round_end(ctx->sc, it, s);
            hub0 = hub1;
            CKL();
            TRY(prof_end(ctx, F_APPLY, ev));
        }
        hipEvent_t ev;
        TRY(prof_begin(ctx, &ev));
        launch_iter_end(ctx->sc, it, ctx->tau, s, &a.bt);
        CKL();
        TRY(prof_end(ctx, F_ITER, ev));
        CK(hipMemcpyAsync(&ctx->pinned_done[it], &ctx->sc->done, sizeof(int32_t),
                          hipMemcpyDeviceToHost, s));
        if (ctx->noalloc) {
            // no events: wait for this iteration (kernels after the done flag are no-ops
            // anyway, so the result is the same)
            CK(hipStreamSynchronize(s));
            if (ctx->pinned_done[it]) break;
            continue;
        }
        CK(hipEventRecord(ctx->it_ev[it & 1], s));
        // look one iteration behind so the device always has queued work
        if (it >= 1) {
            CK(hipEventSynchronize(ctx->it_ev[(it - 1) & 1]));
            if (ctx->pinned_done[it - 1]) break;
        }
    }
    if (!seq_joined) CK(hipStreamWaitEvent(s, ctx->join_ev, 0));
    TRY(read_scalars(ctx));
    const DevScalars &h = *ctx->hsc;
    ctx->iters_last = h.iters;
    ctx->dq_last = h.iters > 0 ? h.dq[h.iters - 1] : 0.0;
    ctx->tr_sum.assign(h.iters, 0);
    ctx->tr_moves.assign(h.iters, 0);
    ctx->tr_proc.assign(h.iters, 0);
    int64_t mv = 0, pr = 0, scn = 0;
    for (int k = 0; k < h.iters; ++k) {
        ctx->tr_sum[k] = join_i128(h.sumN[k][0], h.sumN[k][1]);
        ctx->tr_moves[k] = (int64_t)h.moves[k];
        ctx->tr_proc[k] = (int64_t)h.processed[k];
        mv += (int64_t)h.moves[k];
        pr += (int64_t)h.processed[k];
        scn += (int64_t)h.scanned[k];
    }
    const int P = ctx->pass;
    if (P < LOUVAIN_MAX_PASSES) {
        ctx->st.passes = P + 1;
        ctx->st.iterations[P] = h.iters;
        ctx->st.vertices[P] = l.n;
        ctx->st.entries[P] = l.entries;
        ctx->st.dq_last[P] = ctx->dq_last;
        ctx->st.moves[P] = mv;
        ctx->st.processed[P] = pr;
        ctx->st.scanned[P] = scn;
        ctx->st.colours[P] = coloured ? ctx->ncol : 0;
    }
    return LOUVAIN_OK;
}

// Dense order-preserving renumbering of labels[0..n) (values < range) in place.
int renumber_dense(louvain_ctx *ctx, int32_t *labels, int32_t n, int32_t range)
{
    hipStream_t s = ctx->s;
    launch_fill_i32(ctx->used, 0, (int64_t)range + 1, s);
    launch_mark_used(n, labels, ctx->used, s);
    launch_exclusive_scan<int32_t, int32_t>(ctx->used, ctx->idmap, range, ctx->scratch,
                                            &ctx->sc->scan_total, s);
    launch_relabel(n, labels, ctx->idmap, s);
    CKL();
    return LOUVAIN_OK;
}

// ---------------------------------------------------------------- aggregation (Alg. 1 tail + Alg. 3)
template <class C>
int aggregate_phase(louvain_ctx *ctx, int32_t *communities, int32_t *stop)
{
    typedef typename C::ST ST;
    hipStream_t s = ctx->s;
    const LevelH l = ctx->lev;
    hipEvent_t ev;
    TRY(prof_begin(ctx, &ev));
    // number of communities |Gamma| after local moving
    launch_fill_i32(ctx->used, 0, (int64_t)l.n + 1, s);
    launch_mark_used(l.n, ctx->Cp, ctx->used, s);
    launch_exclusive_scan<int32_t, int32_t>(ctx->used, ctx->idmap, l.n, ctx->scratch,
                                            &ctx->sc->scan_total, s);
    CKL();
    TRY(prof_end(ctx, F_AGGPREP, ev));
    TRY(read_scalars(ctx));
    const int32_t nc = (int32_t)ctx->hsc->scan_total;
    const int P = ctx->pass;
    if (P < LOUVAIN_MAX_PASSES) ctx->st.communities[P] = nc;
    if (communities) *communities = nc;
    // Alg. 1: globally converged, or too few merges (per graph in a batch, which
    // stops when every graph has)
    const int gnext = ctx->glev == 1 ? 2 : 1;
    bool stopped;
    if (ctx->G > 0) {
        launch_fill_bytes_zero(&ctx->sc->alive, sizeof(int32_t), s);
        launch_batch_agg_test(batch_args(ctx), ctx->idmap, l.n, nc, ctx->p.aggregation_tolerance,
                              ctx->gvb[gnext], ctx->gcomm, ctx->sc, s);
        CKL();
        TRY(read_scalars(ctx));
        stopped = ctx->hsc->alive == 0;
    } else {
        stopped = ctx->iters_last <= 1 || (double)nc / (double)l.n > ctx->p.aggregation_tolerance;
    }
    if (stopped) {
        ctx->state = S_STOPPED;
        if (stop) *stop = 1;
        return LOUVAIN_OK;
    }
    const int nbuf = l.buf == 0 ? 1 : 0;
    int32_t *yoff = ctx->off_buf[nbuf], *ydeg = ctx->deg_buf[nbuf], *ytgt = ctx->tgt_buf[nbuf];
    ST *yw = (ST *)ctx->w_buf[nbuf];
    TRY(prof_begin(ctx, &ev));
    // renumber communities (prefix sum over used ids) and look up the dendrogram
    launch_relabel(l.n, ctx->Cp, ctx->idmap, s);
    launch_relabel(ctx->n, ctx->top, ctx->Cp, s);
    if (ctx->G > 0) launch_batch_gid_next(l.n, ctx->Cp, ctx->gid[ctx->glev], ctx->gid[gnext], s);
    // community-vertex CSR: count, exclusive scan, fill
    launch_fill_i32(ctx->ccount, 0, (int64_t)nc + 1, s);
    launch_fill_i32(ctx->ctot, 0, (int64_t)nc + 1, s);
    launch_comm_count(l.n, ctx->Cp, l.off, l.deg, ctx->ccount, ctx->ctot, s);
    launch_exclusive_scan<int32_t, int32_t>(ctx->ccount, ctx->coff, nc, ctx->scratch, nullptr, s);
    launch_exclusive_scan<int32_t, int32_t>(ctx->ctot, yoff, nc, ctx->scratch, nullptr, s);
    launch_fill_i32(ctx->cursor, 0, nc, s);
    launch_comm_fill(l.n, ctx->Cp, ctx->coff, ctx->cursor, ctx->members, s);
    // bins of communities by total degree
    launch_bin_count(nc, nullptr, ctx->ctot, ctx->lds_max, ctx->bincnt, ctx->binoff, ctx->scratch,
                     ctx->sc->bin_start, ctx->sc->bin_maxlen, s);
    launch_fill_i32(ydeg, 0, nc, s);
    CKL();
    TRY(prof_end(ctx, F_AGGPREP, ev));
    TRY(read_scalars(ctx));
    BinInfo cb;
    for (int b = 0; b <= NBINS; ++b) cb.start[b] = ctx->hsc->bin_start[b];
    TRY(prof_begin(ctx, &ev));
    int cmax[NBINS];
    for (int b = 0; b < NBINS; ++b) cmax[b] = ctx->hsc->bin_maxlen[b];
    launch_bin_fill(nc, nullptr, ctx->ctot, ctx->lds_max, ctx->binoff, ctx->cbinorder, s);
    const int hubs = cb.start[NBINS] - cb.start[NBINS - 1];
    int32_t row_slices = 0, table_slices = 0;
    if (hubs > 0) {
        // member row lengths prefix (flattened member rows of hub communities),
        // sorting slices (in cursor) and partitions (in ccount)
        launch_member_degrees(l.n, ctx->members, l.off, l.deg, ctx->cursor, s);
        launch_exclusive_scan<int32_t, int32_t>(ctx->cursor, ctx->mpre, l.n, ctx->scratch, nullptr,
                                                s);
        launch_hub_move_sizes(ctx->cbinorder, cb.start[NBINS - 1], cb.start[NBINS], nullptr,
                              ctx->ctot, (int)sizeof(ST), ctx->hsz, ctx->cursor, ctx->ccount, s,
                              AGG_PSLICE, AGG_PART_ENTRIES);
        launch_exclusive_scan<int32_t, int32_t>(ctx->cursor, ctx->slA, hubs, ctx->scratch,
                                                &ctx->sc->hub_slices, s);
        launch_exclusive_scan<int32_t, int32_t>(ctx->ccount, ctx->slB, hubs, ctx->scratch,
                                                &ctx->sc->hub_tslices, s);
    }
    CKL();
    TRY(prof_end(ctx, F_AGGPREP, ev));
    if (hubs > 0) {
        TRY(read_scalars(ctx));
        row_slices = (int32_t)ctx->hsc->hub_slices;
        table_slices = (int32_t)ctx->hsc->hub_tslices;
        // excluded by the layout's bounds on windows and partitions
        if (row_slices > ctx->owner_cap || table_slices > ctx->part_cap) return LOUVAIN_EINVAL;
    }
    unsigned long long emitted0 = 0;
    for (int b = 0; b < NBINS; ++b) emitted0 += ctx->hsc->work[WORK_AGG + b][3];
    AggArgs<C> g;
    g.off = l.off;
    g.deg = l.deg;
    g.tgt = l.tgt;
    g.w = lev_w<C>(l);
    g.Cp = ctx->Cp;
    g.coff = ctx->coff;
    g.members = ctx->members;
    g.cbinorder = ctx->cbinorder;
    g.yoff = yoff;
    g.ydeg = ydeg;
    g.ytgt = ytgt;
    g.yw = yw;
    g.hstage = ctx->hstage;
    g.hstage_w = (ST *)ctx->hstage_w;
    g.wcnt = ctx->wcnt;
    g.pk = ctx->pk;
    g.pw = (ST *)ctx->pw;
    g.pcount = ctx->pcnt;
    g.pcur = ctx->pcnt + table_slices;  // zeroed together with pcount
    g.poff = ctx->poff;
    g.tslices = &ctx->sc->hub_tslices;
    g.mpre = ctx->mpre;
    g.cslice = ctx->slA;
    g.tslice = ctx->slB;
    g.sown = ctx->sown;
    g.pown = ctx->pown;
    g.wm0 = ctx->wm0;
    g.ncomm = nc;
    for (int b = 0; b < NBINS; ++b) {
        g.begin = cb.start[b];
        g.count = cb.start[b + 1] - cb.start[b];
        if (g.count <= 0) continue;
        g.work = ctx->sc->work[WORK_AGG + b];
        TRY(prof_begin(ctx, &ev));
        if (b < NBINS - 1)
            launch_aggregate<C>(b, g, block_log2s(cmax[b]), s);
        else
            launch_aggregate_hub<C>(g, row_slices, table_slices, l.buf < 0 ? ctx->wmax : 0,
                                    ctx->scratch, s);
        CKL();
        TRY(prof_end(ctx, F_AGG0 + b, ev));
    }
    // the super-vertex graph becomes the next level (Alg. 1: G' <- G'')
    TRY(read_scalars(ctx));
    unsigned long long emitted1 = 0;
    for (int b = 0; b < NBINS; ++b) emitted1 += ctx->hsc->work[WORK_AGG + b][3];
    LevelH nl;
    nl.n = nc;
    nl.off = yoff;
    nl.deg = ydeg;
    nl.tgt = ytgt;
    nl.w = yw;
    nl.wbytes = ctx->L.sb;
    nl.buf = nbuf;
    nl.entries = (int64_t)(emitted1 - emitted0);
    ctx->lev = nl;
    if (ctx->G > 0) ctx->glev = gnext;
    ctx->tau = ctx->tau / ctx->p.tolerance_drop;
    ctx->pass += 1;
    const bool more = ctx->pass < ctx->p.max_passes;
    ctx->state = more ? S_READY : S_EXHAUSTED;
    if (stop) *stop = more ? 0 : 1;
    return LOUVAIN_OK;
}

// Q of the current state (Eq. 1): on the last level with its labels (after an
// early stop) or with singletons (after the last pass aggregated).
template <class C>
int modularity_t(louvain_ctx *ctx, double *q)
{
    typedef typename C::ST ST;
    hipStream_t s = ctx->s;
    if (ctx->state == S_EXHAUSTED) TRY(setup_level<C>(ctx));
    const LevelH &l = ctx->lev;
    hipEvent_t ev;
    TRY(prof_begin(ctx, &ev));
    launch_fill_bytes_zero(&ctx->sc->sigma, 3 * sizeof(unsigned long long), s);
    for (int b = 0; b < NBINS; ++b) {
        RowArgs<C> r;
        r.off = l.off;
        r.deg = l.deg;
        r.tgt = l.tgt;
        r.w = lev_w<C>(l);
        r.binorder = ctx->binorder;
        r.begin = ctx->bins.start[b];
        r.count = bins_of(ctx, b);
        r.K = nullptr;
        r.Sig = nullptr;
        r.labels = ctx->Cp;
        r.sigma = &ctx->sc->sigma;
        // the level's hub layout: from its setup, which an early stop leaves in
        // place (aggregation rebuilds the slices only after its stop test)
        r.hslice = b == NBINS - 1 ? ctx->slA : nullptr;
        r.nslices = &ctx->sc->hub_slices;
        launch_row_reduce<C>(b, 1, r, s);
    }
    launch_sum_squares<ST>((const ST *)ctx->Sig, l.n, ctx->sc->s2, s);
    CKL();
    TRY(prof_end(ctx, F_FINAL, ev));
    TRY(read_scalars(ctx));
    const i128 sigma = (i128)ctx->hsc->sigma;
    const i128 s2 = join_i128(ctx->hsc->s2[0], ctx->hsc->s2[1]);
    const i128 W = (i128)ctx->W;
    const i128 num = sigma * W - s2;
    const i128 den = W * W;
    *q = den == 0 ? 0.0 : i128_to_f64(num) / i128_to_f64(den);
    if (ctx->G > 0) {
        // each graph's own Q (its own W) from per-graph sigma and S2
        const int G = ctx->G;
        launch_fill_bytes_zero(ctx->gsig, 8 * (int64_t)G, s);
        launch_fill_bytes_zero(ctx->gs2, 16 * (int64_t)G, s);
        launch_batch_modularity<typename C::WT, ST>(l.n, l.off, l.deg, l.tgt, lev_w<C>(l), ctx->Cp,
                                                    (const ST *)ctx->Sig, ctx->gid[ctx->glev],
                                                    ctx->gsig, ctx->gs2, s);
        CKL();
        std::vector<unsigned long long> sig(G), sq(2 * (size_t)G);
        std::vector<int64_t> gw(G);
        CK(hipMemcpyAsync(sig.data(), ctx->gsig, 8 * (size_t)G, hipMemcpyDeviceToHost, s));
        CK(hipMemcpyAsync(sq.data(), ctx->gs2, 16 * (size_t)G, hipMemcpyDeviceToHost, s));
        CK(hipMemcpyAsync(gw.data(), ctx->gW, 8 * (size_t)G, hipMemcpyDeviceToHost, s));
        TRY(sync_stream(ctx));
        ctx->gq.assign(G, 0.0);
        for (int g = 0; g < G; ++g) {
            const i128 Wg = (i128)gw[g];
            const i128 ng = (i128)sig[g] * Wg - join_i128(sq[2 * g], sq[2 * g + 1]);
            ctx->gq[g] = Wg == 0 ? 0.0 : i128_to_f64(ng) / i128_to_f64(Wg * Wg);
        }
    }
    return LOUVAIN_OK;
}

template <class C>
int dispatch_move(louvain_ctx *ctx)
{
    return move_phase<C>(ctx);
}

int do_move(louvain_ctx *ctx)
{
    if (!ctx->wide) return move_phase<CfgNarrow>(ctx);
    if (ctx->lev.buf < 0) {
        // set the level up first: its largest K' bounds every sum of one row's
        // weights, so below 2^31 the LDS tables can hold 32-bit sums
        TRY(setup_level<CfgWideIn>(ctx));
        if (ctx->kmax_in < (1ull << 31)) return move_phase<CfgWideIn32>(ctx, true);
        return move_phase<CfgWideIn>(ctx, true);
    }
    return move_phase<CfgWide>(ctx);
}

int do_aggregate(louvain_ctx *ctx, int32_t *nc, int32_t *stop)
{
    if (!ctx->wide) return aggregate_phase<CfgNarrow>(ctx, nc, stop);
    if (ctx->lev.buf < 0) return aggregate_phase<CfgWideIn>(ctx, nc, stop);
    return aggregate_phase<CfgWide>(ctx, nc, stop);
}

int do_modularity(louvain_ctx *ctx, double *q)
{
    if (!ctx->wide) return modularity_t<CfgNarrow>(ctx, q);
    if (ctx->lev.buf < 0) return modularity_t<CfgWideIn>(ctx, q);
    return modularity_t<CfgWide>(ctx, q);
}

// Rounds per iteration when the caller leaves round_bits at -1.  Fast mode on one
// graph: 8 (measured on R-MAT-24: 2 rounds 334 ms and Q 0.0269, 8 rounds 277-291 ms and
// Q 0.0280 against 0.0289 for the sequential oracle; on a 10^6-vertex planted-partition
// graph 2 rounds end 0.02-0.06 below the sequential Q, 8 within 0.0003: fewer
// neighbours decide at the same moment, and the better partition needs fewer
// iterations).  Fast mode on a batch: 2 (its graphs' vertices are interleaved anyway;
// 8 rounds made the 4096-graph batch 27% slower and no better).  Deterministic mode: 2,
// its reference schedule (another round count is another, equally deterministic,
// result).
int default_round_bits(int32_t mode, bool batch)
{
    return mode == LOUVAIN_FAST && !batch ? 3 : 1;
}

int check_params(const louvain_params *p)
{
    if (p->mode != LOUVAIN_DETERMINISTIC && p->mode != LOUVAIN_FAST && p->mode != LOUVAIN_COLOURED)
        return LOUVAIN_EINVAL;
    if (p->max_passes < 0 || p->max_passes > LOUVAIN_MAX_PASSES) return LOUVAIN_EINVAL;
    if (p->max_iterations < 1 || p->max_iterations > LOUVAIN_MAX_ITERATIONS) return LOUVAIN_EINVAL;
    if (p->round_bits < -1 || p->round_bits > 4) return LOUVAIN_EINVAL;
    if (p->hub_rows != 0 && (p->hub_rows < 2048 || p->hub_rows > LDS_MAX_NARROW)) return LOUVAIN_EINVAL;
    if (p->hub_part_pairs != 0 && (p->hub_part_pairs < 1024 || p->hub_part_pairs > hub_part_pairs<int64_t>()))
        return LOUVAIN_EINVAL;
    if (p->small_level < -1 || p->small_level > SEQ_MAX) return LOUVAIN_EINVAL;
    if (!(p->tolerance_drop > 0.0) || p->aggregation_tolerance != p->aggregation_tolerance ||
        p->tolerance != p->tolerance)
        return LOUVAIN_EINVAL;
    return LOUVAIN_OK;
}

void reset_state(louvain_ctx *ctx)
{
    ctx->state = S_READY;
    ctx->pass = 0;
    ctx->tau = ctx->p.tolerance;
    ctx->iters_last = 0;
    ctx->dq_last = 0.0;
    LevelH l;
    l.n = ctx->n;
    l.off = ctx->in_off;
    l.deg = nullptr;
    l.tgt = ctx->in_tgt;
    l.w = ctx->in_w;
    l.wbytes = 4;
    l.buf = -1;
    l.entries = ctx->nnz;
    ctx->lev = l;
    ctx->glev = 0;
    memset(&ctx->st, 0, sizeof(ctx->st));
    ctx->tr_sum.clear();
    ctx->tr_moves.clear();
    ctx->tr_proc.clear();
    if (ctx->p.max_passes == 0) ctx->state = S_EXHAUSTED;
}

}  // namespace

// ======================================================================= C ABI
extern "C" {

void louvain_default_params(louvain_params *p)
{
    if (!p) return;
    memset(p, 0, sizeof(*p));
    p->mode = LOUVAIN_DETERMINISTIC;
    p->max_passes = 10;
    p->max_iterations = 20;
    p->prune = 1;
    p->tolerance = 0.01;
    p->tolerance_drop = 10.0;
    p->aggregation_tolerance = 0.8;
    p->seed = 0;
    p->round_bits = -1;  // the mode's own (default_round_bits)
    p->profile = 0;
    p->hub_rows = 0;
    p->hub_part_pairs = 0;
    p->small_level = 0;
}

int louvain_workspace_size(int32_t n, int64_t nnz, int64_t total_weight, const louvain_params *p,
                           size_t *bytes)
{
    if (!bytes || n < 0 || nnz < 0) return LOUVAIN_EINVAL;
    if (nnz > INT32_MAX) return LOUVAIN_EOVERFLOW;
    if (p) {
        const int r = check_params(p);
        if (r) return r;
    }
    const int sb = (total_weight >= 0 && total_weight < ((int64_t)1 << 31)) ? 4 : 8;
    *bytes = make_layout(n, nnz, sb).total;
    return LOUVAIN_OK;
}

}  // extern "C"

namespace {

int init_ctx(louvain_ctx **out, int32_t G, const int32_t *graph_offsets, int32_t n, int64_t nnz,
             const int32_t *offsets, const int32_t *targets, const int32_t *weights,
             void *workspace, size_t workspace_bytes, const louvain_params *p, void *stream,
             bool noalloc = false)
{
    if (!out) return LOUVAIN_EINVAL;
    *out = nullptr;
    if (n < 0 || nnz < 0 || !offsets || !workspace) return LOUVAIN_EINVAL;
    if (nnz > 0 && (!targets || !weights)) return LOUVAIN_EINVAL;
    if (nnz > INT32_MAX) return LOUVAIN_EOVERFLOW;
    louvain_params prm;
    if (p)
        prm = *p;
    else
        louvain_default_params(&prm);
    if (check_params(&prm)) return LOUVAIN_EINVAL;
    if (prm.round_bits < 0) prm.round_bits = default_round_bits(prm.mode, G > 0);
    if (G < 0 || (G > 0 && !graph_offsets)) return LOUVAIN_EINVAL;
    const size_t need4 = make_layout(n, nnz, 4, G).total;
    if (workspace_bytes < need4) return LOUVAIN_ENOSPC;

    louvain_ctx *ctx = new (std::nothrow) louvain_ctx();
    if (!ctx) return LOUVAIN_EINVAL;
    ctx->p = prm;
    ctx->s = (hipStream_t)stream;
    ctx->n = n;
    ctx->nnz = nnz;
    ctx->in_off = offsets;
    ctx->in_tgt = targets;
    ctx->in_w = weights;
    ctx->ws = (unsigned char *)workspace;
    ctx->last_err = hipSuccess;
    ctx->G = G;
    for (int f = 0; f < F_COUNT; ++f) {
        ctx->fam_ms[f] = 0.0;
        ctx->fam_launches[f] = 0;
        ctx->fam_bytes[f] = 0.0;
    }
    auto fail = [&](int code) {
        louvain_destroy(ctx);
        return code;
    };
    ctx->noalloc = noalloc;
    if (noalloc) {
        ctx->hsc = &ctx->own_hsc;
        ctx->pinned_done = ctx->own_done;
    } else {
        PinnedBlock pb;
        const bool pinned = pinned_take(&pb);
        ctx->hsc = pb.hsc;
        ctx->pinned_done = pb.done;
        if (!pinned ||
            hipEventCreateWithFlags(&ctx->it_ev[0], hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&ctx->it_ev[1], hipEventDisableTiming) != hipSuccess) {
            g_last_hip_error = "host-side allocation failed";
            return fail(LOUVAIN_EHIP);
        }
    }
    // validation and W with the narrow layout's scalar block (same offset in both layouts)
    ctx->L = make_layout(n, nnz, 4, G);
    ctx->sc = (DevScalars *)(ctx->ws + ctx->L.scalars);
    launch_fill_bytes_zero(ctx->sc, sizeof(DevScalars), ctx->s);
    launch_validate(n, nnz, offsets, targets, weights, &ctx->sc->err, &ctx->sc->W, &ctx->sc->wmax,
                    ctx->s);
    if (hipGetLastError() != hipSuccess) return fail(LOUVAIN_EHIP);
    if (hipMemcpyAsync(ctx->hsc, ctx->sc, sizeof(DevScalars), hipMemcpyDeviceToHost, ctx->s) !=
            hipSuccess ||
        hipStreamSynchronize(ctx->s) != hipSuccess) {
        g_last_hip_error = "validation kernel failed";
        return fail(LOUVAIN_EHIP);
    }
    if (ctx->hsc->err) return fail(LOUVAIN_EINVAL);
    const unsigned long long W = ctx->hsc->W;
    if (W >= (1ull << 62)) return fail(LOUVAIN_EOVERFLOW);
    ctx->W = (int64_t)W;
    ctx->wmax = ctx->hsc->wmax;
    ctx->wide = W >= (1ull << 31);
    ctx->lds_max = ctx->wide ? LDS_MAX_WIDE : LDS_MAX_NARROW;
    if (prm.hub_rows) ctx->lds_max = std::min(ctx->lds_max, prm.hub_rows);
    ctx->L = make_layout(n, nnz, ctx->wide ? 8 : 4, G);
    if (workspace_bytes < ctx->L.total) return fail(LOUVAIN_ENOSPC);
    const Layout &L = ctx->L;
    unsigned char *b = ctx->ws;
    ctx->sc = (DevScalars *)(b + L.scalars);
    ctx->Cp = (int32_t *)(b + L.Cp);
    ctx->top = (int32_t *)(b + L.top);
    ctx->K = b + L.K;
    ctx->Sig = b + L.Sig;
    ctx->size = (int32_t *)(b + L.size);
    ctx->fa = b + L.fa;
    ctx->fb = b + L.fb;
    ctx->binorder = (int32_t *)(b + L.binorder);
    ctx->worklist = (int32_t *)(b + L.worklist);
    ctx->vtmp = (int32_t *)(b + L.vtmp);
    ctx->mv_c = (int32_t *)(b + L.mv_c);
    ctx->used = (int32_t *)(b + L.used);
    ctx->idmap = (int32_t *)(b + L.idmap);
    ctx->ccount = (int32_t *)(b + L.ccount);
    ctx->coff = (int32_t *)(b + L.coff);
    ctx->ctot = (int32_t *)(b + L.ctot);
    ctx->cursor = (int32_t *)(b + L.cursor);
    ctx->members = (int32_t *)(b + L.members);
    ctx->cbinorder = (int32_t *)(b + L.cbinorder);
    ctx->off_buf[0] = (int32_t *)(b + L.offA);
    ctx->off_buf[1] = (int32_t *)(b + L.offB);
    ctx->deg_buf[0] = (int32_t *)(b + L.degA);
    ctx->deg_buf[1] = (int32_t *)(b + L.degB);
    ctx->tgt_buf[0] = (int32_t *)(b + L.tgtA);
    ctx->tgt_buf[1] = (int32_t *)(b + L.tgtB);
    ctx->w_buf[0] = b + L.wA;
    ctx->w_buf[1] = b + L.wB;
    ctx->hstage = (int32_t *)(b + L.hstage);
    ctx->hstage_w = b + L.hstage_w;
    ctx->wcnt = (int32_t *)(b + L.wcnt);
    ctx->pk = (int32_t *)(b + L.pk);
    ctx->pw = b + L.pw;
    ctx->hsz = (int64_t *)(b + L.hsz);
    ctx->hoff = (int64_t *)(b + L.hoff);
    ctx->scratch = (int64_t *)(b + L.scratch);
    ctx->bincnt = (int32_t *)(b + L.bincnt);
    ctx->binoff = (int32_t *)(b + L.binoff);
    ctx->slA = (int32_t *)(b + L.slA);
    ctx->slB = (int32_t *)(b + L.slB);
    ctx->hpart = (void *)(b + L.hpart);
    ctx->pcnt = (int32_t *)(b + L.pcnt);
    ctx->poff = (int32_t *)(b + L.poff);
    ctx->sown = (int32_t *)(b + L.sown);
    ctx->pown = (int32_t *)(b + L.pown);
    ctx->wm0 = (int32_t *)(b + L.wm0);
    ctx->act_s = (int32_t *)(b + L.act_s);
    ctx->act_p = (int32_t *)(b + L.act_p);
    ctx->act_tmp = (int32_t *)(b + L.act_tmp);
    ctx->owner_cap = (nnz > 0 ? nnz : 1) / 1024 + 64;  // as sized in make_layout
    ctx->part_cap = (nnz > 0 ? nnz : 1) / 512 + 64;
    ctx->mpre = (int32_t *)(b + L.mpre);
    ctx->hub_act = b + L.hub_act;
    ctx->hub_hd = b + L.hub_hd;
    ctx->colour = (int32_t *)(b + L.colour);
    ctx->front = (int32_t *)(b + L.front);
    ctx->corder = (int32_t *)(b + L.corder);
    ctx->kcnt = (int32_t *)(b + L.kcnt);
    ctx->koff = (int32_t *)(b + L.koff);
    ctx->cbm = (uint32_t *)(b + L.cbm);
    if (G > 0) {
        for (int k = 0; k < 3; ++k) {
            ctx->gid[k] = (int32_t *)(b + L.gid[k]);
            ctx->gvb[k] = (int32_t *)(b + L.gvb[k]);
        }
        ctx->gW = (int64_t *)(b + L.gW);
        ctx->gsum = (unsigned long long *)(b + L.gsum);
        ctx->gst = (int32_t *)(b + L.gst);
        ctx->giter = (int32_t *)(b + L.giter);
        ctx->gcomm = (int32_t *)(b + L.gcomm);
        ctx->gsig = (unsigned long long *)(b + L.gsig);
        ctx->gs2 = (unsigned long long *)(b + L.gs2);
        // graph offsets: 0 = first <= ... <= last = n
        std::vector<int32_t> go((size_t)G + 1);
        if (hipMemcpyAsync(go.data(), graph_offsets, sizeof(int32_t) * go.size(), hipMemcpyDefault,
                           ctx->s) != hipSuccess ||
            hipStreamSynchronize(ctx->s) != hipSuccess) {
            g_last_hip_error = "reading the graph offsets failed";
            return fail(LOUVAIN_EHIP);
        }
        bool ok = go[0] == 0 && go[G] == n;
        for (int g = 0; g < G && ok; ++g) ok = go[g] <= go[g + 1];
        if (!ok) return fail(LOUVAIN_EINVAL);
        if (hipMemcpyAsync(ctx->gvb[0], go.data(), sizeof(int32_t) * go.size(),
                           hipMemcpyHostToDevice, ctx->s) != hipSuccess ||
            hipStreamSynchronize(ctx->s) != hipSuccess) {
            g_last_hip_error = "copying the graph offsets failed";
            return fail(LOUVAIN_EHIP);
        }
        launch_batch_gid(n, ctx->gvb[0], G, ctx->gid[0], ctx->s);
        launch_fill_bytes_zero(ctx->gW, 8 * (int64_t)G, ctx->s);
        launch_batch_check(n, offsets, targets, weights, ctx->gid[0], ctx->gvb[0], ctx->gW,
                           &ctx->sc->err, ctx->s);
        if (hipGetLastError() != hipSuccess ||
            hipMemcpyAsync(ctx->hsc, ctx->sc, offsetof(DevScalars, spread), hipMemcpyDeviceToHost,
                           ctx->s) != hipSuccess ||
            hipStreamSynchronize(ctx->s) != hipSuccess) {
            g_last_hip_error = "batch validation failed";
            return fail(LOUVAIN_EHIP);
        }
        if (ctx->hsc->err) return fail(LOUVAIN_EINVAL);
        if (!noalloc &&
            (hipStreamCreateWithFlags(&ctx->s2, hipStreamNonBlocking) != hipSuccess ||
             hipEventCreateWithFlags(&ctx->fork_ev, hipEventDisableTiming) != hipSuccess ||
             hipEventCreateWithFlags(&ctx->join_ev, hipEventDisableTiming) != hipSuccess)) {
            g_last_hip_error = "creating the second stream failed";
            return fail(LOUVAIN_EHIP);
        }
    }
    launch_iota(ctx->top, n, ctx->s);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(ctx->s) != hipSuccess) {
        g_last_hip_error = "workspace initialisation failed";
        return fail(LOUVAIN_EHIP);
    }
    reset_state(ctx);
    if (G > 0) {
        launch_batch_reset(batch_args(ctx), ctx->gcomm, ctx->s);
        if (hipGetLastError() != hipSuccess || hipStreamSynchronize(ctx->s) != hipSuccess) {
            g_last_hip_error = "workspace initialisation failed";
            return fail(LOUVAIN_EHIP);
        }
    }
    *out = ctx;
    return LOUVAIN_OK;
}

}  // namespace

extern "C" {

int louvain_init(louvain_ctx **out, int32_t n, int64_t nnz, const int32_t *offsets,
                 const int32_t *targets, const int32_t *weights, void *workspace,
                 size_t workspace_bytes, const louvain_params *p, void *stream)
{
    return init_ctx(out, 0, nullptr, n, nnz, offsets, targets, weights, workspace, workspace_bytes,
                    p, stream);
}

int louvain_batch_workspace_size(int32_t graphs, int32_t n, int64_t nnz, int64_t total_weight,
                                 const louvain_params *p, size_t *bytes)
{
    if (!bytes || graphs < 1 || n < 0 || nnz < 0) return LOUVAIN_EINVAL;
    if (nnz > INT32_MAX) return LOUVAIN_EOVERFLOW;
    if (p) {
        const int r = check_params(p);
        if (r) return r;
    }
    const int sb = (total_weight >= 0 && total_weight < ((int64_t)1 << 31)) ? 4 : 8;
    *bytes = make_layout(n, nnz, sb, graphs).total;
    return LOUVAIN_OK;
}

int louvain_init_batch(louvain_ctx **out, int32_t graphs, const int32_t *graph_offsets, int32_t n,
                       int64_t nnz, const int32_t *offsets, const int32_t *targets,
                       const int32_t *weights, void *workspace, size_t workspace_bytes,
                       const louvain_params *p, void *stream)
{
    if (graphs < 1) return LOUVAIN_EINVAL;
    return init_ctx(out, graphs, graph_offsets, n, nnz, offsets, targets, weights, workspace,
                    workspace_bytes, p, stream);
}

int louvain_set_membership(louvain_ctx *ctx, const int32_t *labels)
{
    if (!ctx) return LOUVAIN_EINVAL;
    if (ctx->state != S_READY || ctx->pass != 0) return LOUVAIN_ESTATE;
    if (!labels) {
        ctx->warm = nullptr;
        return LOUVAIN_OK;
    }
    launch_fill_bytes_zero(&ctx->sc->err, sizeof(int32_t), ctx->s);
    const BatchArgs b = batch_args(ctx);
    launch_warm_check(ctx->n, labels, b.gid, b.gvb, &ctx->sc->err, ctx->s);
    CKL();
    TRY(read_scalars(ctx));
    if (ctx->hsc->err) return LOUVAIN_EINVAL;
    ctx->warm = labels;
    return LOUVAIN_OK;
}

int louvain_batch_results(louvain_ctx *ctx, double *modularity, int32_t *communities)
{
    if (!ctx || ctx->G <= 0) return LOUVAIN_EINVAL;
    if (ctx->state != S_DONE) return LOUVAIN_ESTATE;
    if (modularity)
        for (int g = 0; g < ctx->G; ++g) modularity[g] = ctx->gq[g];
    if (communities) {
        CK(hipMemcpyAsync(communities, ctx->gcomm, sizeof(int32_t) * (size_t)ctx->G,
                          hipMemcpyDeviceToHost, ctx->s));
        TRY(sync_stream(ctx));
    }
    return LOUVAIN_OK;
}

int louvain_move(louvain_ctx *ctx, int32_t *iterations, double *delta_q)
{
    if (!ctx) return LOUVAIN_EINVAL;
    if (ctx->state != S_READY) return LOUVAIN_ESTATE;
    if (ctx->pass == 0) {
        launch_iota(ctx->top, ctx->n, ctx->s);
        CKL();
    }
    TRY(do_move(ctx));
    ctx->state = S_MOVED;
    if (iterations) *iterations = ctx->iters_last;
    if (delta_q) *delta_q = ctx->dq_last;
    return LOUVAIN_OK;
}

int louvain_aggregate(louvain_ctx *ctx, int32_t *communities, int32_t *stop)
{
    if (!ctx) return LOUVAIN_EINVAL;
    if (ctx->state != S_MOVED) return LOUVAIN_ESTATE;
    return do_aggregate(ctx, communities, stop);
}

int louvain_run(louvain_ctx *ctx, int32_t *membership, double *modularity, louvain_stats *stats)
{
    if (!ctx || !membership) return LOUVAIN_EINVAL;
    if (ctx->state == S_DONE) return LOUVAIN_ESTATE;
    while (ctx->state == S_READY || ctx->state == S_MOVED) {
        if (ctx->state == S_READY) TRY(louvain_move(ctx, nullptr, nullptr));
        int32_t stop = 0;
        TRY(louvain_aggregate(ctx, nullptr, &stop));
    }
    hipStream_t s = ctx->s;
    if (ctx->state == S_STOPPED) {
        // final dendrogram lookup (Alg. 1), only after an early stop
        launch_relabel(ctx->n, ctx->top, ctx->Cp, s);
        CKL();
    }
    double q = 0.0;
    TRY(do_modularity(ctx, &q));
    TRY(renumber_dense(ctx, ctx->top, ctx->n, ctx->lev.n > 0 ? ctx->lev.n : 1));
    CK(hipMemcpyAsync(membership, ctx->top, sizeof(int32_t) * (size_t)ctx->n,
                      hipMemcpyDeviceToDevice, s));
    TRY(sync_stream(ctx));
    ctx->state = S_DONE;
    if (modularity) *modularity = q;
    if (stats) *stats = ctx->st;
    return LOUVAIN_OK;
}

int louvain_membership(louvain_ctx *ctx, int32_t *membership)
{
    if (!ctx || !membership) return LOUVAIN_EINVAL;
    hipStream_t s = ctx->s;
    CK(hipMemcpyAsync(membership, ctx->top, sizeof(int32_t) * (size_t)ctx->n,
                      hipMemcpyDeviceToDevice, s));
    if (ctx->state == S_MOVED || ctx->state == S_STOPPED) launch_relabel(ctx->n, membership, ctx->Cp, s);
    CKL();
    const int32_t range = ctx->state == S_DONE ? ctx->n : ctx->lev.n;
    TRY(renumber_dense(ctx, membership, ctx->n, range > 0 ? range : 1));
    TRY(sync_stream(ctx));
    return LOUVAIN_OK;
}

int louvain_level_labels(louvain_ctx *ctx, int32_t *labels)
{
    if (!ctx || !labels) return LOUVAIN_EINVAL;
    if (ctx->state != S_MOVED && ctx->state != S_STOPPED) return LOUVAIN_ESTATE;
    CK(hipMemcpyAsync(labels, ctx->Cp, sizeof(int32_t) * (size_t)ctx->lev.n,
                      hipMemcpyDeviceToDevice, ctx->s));
    TRY(sync_stream(ctx));
    return LOUVAIN_OK;
}

int louvain_level_graph(louvain_ctx *ctx, const int32_t **offsets, const int32_t **degree,
                        const int32_t **targets, const void **weights, int32_t *n_level,
                        int32_t *weight_bytes)
{
    if (!ctx) return LOUVAIN_EINVAL;
    if (offsets) *offsets = ctx->lev.off;
    if (degree) *degree = ctx->lev.deg;
    if (targets) *targets = ctx->lev.tgt;
    if (weights) *weights = ctx->lev.w;
    if (n_level) *n_level = ctx->lev.n;
    if (weight_bytes) *weight_bytes = ctx->lev.wbytes;
    return LOUVAIN_OK;
}

int louvain_move_trace(louvain_ctx *ctx, int32_t max, int64_t *sumN_hi, uint64_t *sumN_lo,
                       int64_t *moves, int64_t *processed, int32_t *count)
{
    if (!ctx || max < 0) return LOUVAIN_EINVAL;
    const int32_t k = std::min<int32_t>(max, (int32_t)ctx->tr_sum.size());
    for (int32_t i = 0; i < k; ++i) {
        if (sumN_hi) sumN_hi[i] = (int64_t)(ctx->tr_sum[i] >> 64);
        if (sumN_lo) sumN_lo[i] = (uint64_t)ctx->tr_sum[i];
        if (moves) moves[i] = ctx->tr_moves[i];
        if (processed) processed[i] = ctx->tr_proc[i];
    }
    if (count) *count = (int32_t)ctx->tr_sum.size();
    return LOUVAIN_OK;
}

int louvain_reset(louvain_ctx *ctx)
{
    if (!ctx) return LOUVAIN_EINVAL;
    reset_state(ctx);
    ctx->warm = nullptr;
    launch_iota(ctx->top, ctx->n, ctx->s);
    CKL();
    if (ctx->G > 0) {
        launch_batch_reset(batch_args(ctx), ctx->gcomm, ctx->s);
        CKL();
    }
    TRY(sync_stream(ctx));
    return LOUVAIN_OK;
}

int louvain_total_weight(louvain_ctx *ctx, int64_t *W)
{
    if (!ctx || !W) return LOUVAIN_EINVAL;
    *W = ctx->W;
    return LOUVAIN_OK;
}

int louvain_get_stats(louvain_ctx *ctx, louvain_stats *stats)
{
    if (!ctx || !stats) return LOUVAIN_EINVAL;
    *stats = ctx->st;
    return LOUVAIN_OK;
}

int louvain_kernel_stats(louvain_ctx *ctx, louvain_kernel_stat *out, int32_t max, int32_t *count)
{
    if (!ctx || max < 0 || (max > 0 && !out)) return LOUVAIN_EINVAL;
    // algorithmic bytes from the work counters (whole context lifetime)
    if (hipMemcpyAsync(ctx->hsc, ctx->sc, sizeof(DevScalars), hipMemcpyDeviceToHost, ctx->s) !=
            hipSuccess ||
        hipStreamSynchronize(ctx->s) != hipSuccess)
        return LOUVAIN_EHIP;
    const double sb = ctx->L.sb;
    const double wb_in = 4.0;
    int32_t k = 0;
    for (int f = 0; f < F_COUNT; ++f) {
        double bytes = 0.0;
        if (f >= F_MOVE0 && f < F_MOVE0 + NBINS) {
            const unsigned long long *w = ctx->hsc->work[WORK_MOVE + f - F_MOVE0];
            // per vertex: row offsets 8, K' sb, C' 4, its community's Sigma' sb, active flag
            // 1; per entry: target 4, weight, C'[j] 4; per candidate total read (those whose
            // score bound reaches the floor): Sigma' sb; per move: C' 4, two Sigma' updates
            // 2*sb, two size updates 8
            bytes = (double)w[0] * (8 + 2 * sb + 4 + 1) + (double)w[1] * (4 + wb_in + 4) +
                    (double)w[2] * sb + (double)w[3] * (4 + 2 * sb + 8);
        } else if (f >= F_AGG0 && f < F_AGG0 + NBINS) {
            const unsigned long long *w = ctx->hsc->work[WORK_AGG + f - F_AGG0];
            // per community: member offsets 8, row offset 8, row length 4; per member: id 4,
            // its row offsets 8; per entry: target 4, weight, C'[j] 4; per emitted entry:
            // target 4 and weight sb
            bytes = (double)w[0] * 20 + (double)w[1] * 12 + (double)w[2] * (4 + wb_in + 4) +
                    (double)w[3] * (4 + sb);
        }
        ctx->fam_bytes[f] = bytes;
        if (k < max) {
            memset(&out[k], 0, sizeof(out[k]));
            strncpy(out[k].name, FAM_NAMES[f], sizeof(out[k].name) - 1);
            out[k].launches = ctx->fam_launches[f];
            out[k].ms = ctx->fam_ms[f];
            out[k].bytes = bytes;
        }
        ++k;
    }
    if (count) *count = k;
    return LOUVAIN_OK;
}

void louvain_destroy(louvain_ctx *ctx)
{
    if (!ctx) return;
    for (const Pending &q : ctx->pending) {
        hipEventDestroy(q.a);
        hipEventDestroy(q.b);
    }
    for (hipEvent_t e : ctx->ev_free) hipEventDestroy(e);
    if (!ctx->noalloc) pinned_give(ctx->hsc, ctx->pinned_done);
    for (int k = 0; k < 2; ++k)
        if (ctx->it_ev[k]) hipEventDestroy(ctx->it_ev[k]);
    if (ctx->s2) {
        (void)hipStreamSynchronize(ctx->s2);
        hipStreamDestroy(ctx->s2);
    }
    if (ctx->fork_ev) hipEventDestroy(ctx->fork_ev);
    if (ctx->join_ev) hipEventDestroy(ctx->join_ev);
    delete ctx;
}

}  // extern "C"

// ---------------------------------------------------------------- no-allocation entry point
//
// The device scratch array of louvain_run_noalloc: one per GPU the library runs
// on, held until the process ends.  In host code `scratch` names a host-side
// stand-in, not the device array: its device address comes from
// hipGetSymbolAddress once per device (noalloc_scratch) and only that address
// is ever handed to kernels or copies.
static __device__ __align__(256) unsigned char scratch[LOUVAIN_NOALLOC_BYTES];

namespace {

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[NOALLOC_MAX_DEVICES];

// Device address of the current device's scratch array (looked up on the
// first call on that device), or nullptr on failure.
void *noalloc_scratch()
{
    int dev = -1;
    const hipError_t ed = hipGetDevice(&dev);
    if (ed != hipSuccess) {
        g_last_hip_error = hipGetErrorString(ed);
        return nullptr;
    }
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) {
        g_last_hip_error = "device index beyond the scratch-address table";
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            g_last_hip_error = e != hipSuccess ? hipGetErrorString(e)
                                               : "hipGetSymbolAddress gave a null address";
            return nullptr;
        }
        g_scratch_ptr[dev] = ptr;
    }
    return g_scratch_ptr[dev];
}

}  // namespace

extern "C" int louvain_run_noalloc(int32_t n, int64_t nnz, const int32_t *offsets,
                                   const int32_t *targets, const int32_t *weights,
                                   const louvain_params *p, int32_t *membership,
                                   double *modularity, louvain_stats *stats, void *stream)
{
    if (p && p->profile) return LOUVAIN_EINVAL;  // profiling creates events
    size_t need = 0;
    // sized for 8-byte totals, whatever the weights: the total weight is only known
    // after validation, and the array must hold either layout
    const int r = louvain_workspace_size(n, nnz, -1, p, &need);
    if (r) return r;
    if (need > (size_t)LOUVAIN_NOALLOC_BYTES) return LOUVAIN_ENOSPC;
    void *ws = noalloc_scratch();
    if (!ws) return LOUVAIN_EHIP;
    louvain_ctx *ctx = nullptr;
    int rc = init_ctx(&ctx, 0, nullptr, n, nnz, offsets, targets, weights, ws,
                      (size_t)LOUVAIN_NOALLOC_BYTES, p, stream, true);
    if (rc) return rc;
    rc = louvain_run(ctx, membership, modularity, stats);
    louvain_destroy(ctx);
    return rc;
}

extern "C" {

const char *louvain_strerror(int code)
{
    switch (code) {
    case LOUVAIN_OK: return "ok";
    case LOUVAIN_EINVAL: return "invalid argument or malformed graph";
    case LOUVAIN_EOVERFLOW: return "size or total weight out of range";
    case LOUVAIN_ENOSPC: return "workspace too small";
    case LOUVAIN_EHIP: return g_last_hip_error;
    case LOUVAIN_ESTATE: return "call out of order";
    default: return "unknown status";
    }
}

}  // extern "C"
