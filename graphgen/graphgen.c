/*
 * Seeded synthetic graph generators (R-MAT and planted-partition SBM) that
 * produce symmetric CSR graphs with int32 targets and int32 weights.
 *
 * Holds none of the community-detection arithmetic: it only draws edges.
 *
 * Random numbers: a counter-based use of SplitMix64 (Steele, Lea and Flood,
 * "Fast splittable pseudorandom number generators", OOPSLA 2014).  The k-th
 * output of a stream whose state starts at `key` is mix64(key + (k+1)*gamma),
 * gamma = 0x9E3779B97F4A7C15, so every draw is a pure function of
 * (seed, stream, counter) and the graph does not depend on the thread count.
 *
 * R-MAT (Chakrabarti, Zhan and Faloutsos, SDM 2004): for each of M draws
 * pick one quadrant per level with probabilities a, b, c, d (one FP64
 * uniform per level, thresholds a, a+b, a+b+c), then relabel vertices by a
 * seeded random permutation; self-loops are dropped, each edge is stored in
 * both directions and duplicates are merged by summing their weights.
 *
 * SBM: vertex v is in block floor(v*k/n); each unordered pair u < v is an
 * edge with probability p_in (same block) or p_out, drawn by geometric
 * skipping (Batagelj and Brandes, Phys. Rev. E 71, 2005).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define GAMMA 0x9E3779B97F4A7C15ULL

static inline uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static inline uint64_t draw(uint64_t key, uint64_t ctr)
{
    return mix64(key + (ctr + 1) * GAMMA);
}

static inline double u01(uint64_t x) { return (double)(x >> 11) * 0x1.0p-53; }

static uint64_t stream_key(uint64_t seed, uint64_t stream)
{
    return mix64(mix64(seed + GAMMA) ^ (stream * 0xD1B54A32D192ED03ULL));
}

/* uniform integer in [0, bound) by the high half of a 64x64 product */
static inline uint64_t below(uint64_t x, uint64_t bound)
{
    return (uint64_t)(((unsigned __int128)x * bound) >> 64);
}

enum { S_QUAD = 1, S_WEIGHT = 2, S_PERM = 3, S_SBM = 4 };

/* Exposed for the generator's own tests. */
uint64_t gg_splitmix_draw(uint64_t key, uint64_t ctr) { return draw(key, ctr); }
uint64_t gg_splitmix_next(uint64_t *state)
{
    *state += GAMMA;
    return mix64(*state);
}

typedef struct {
    int64_t n;
    int64_t nnz;
    int64_t *off;  /* n+1 */
    int32_t *tgt;  /* nnz */
    int32_t *w;    /* nnz */
    int status;    /* 0 ok, -1 alloc, -2 weight overflow, -3 bad args */
} gg_graph;

typedef struct {
    int kind; /* 0 rmat, 1 sbm */
    /* rmat */
    int scale;
    int64_t draws;
    double a, b, c;
    int32_t wmax;
    int32_t *perm;
    /* sbm */
    int64_t n;
    int64_t k;
    double p_in, p_out;
    uint64_t seed;
} gen_spec;

/* R-MAT edge e: endpoints after relabelling and its weight; returns 0 if self-loop */
static inline int rmat_edge(const gen_spec *s, uint64_t kq, uint64_t kw, int64_t e,
                            int32_t *u, int32_t *v, int32_t *w)
{
    uint64_t src = 0, dst = 0;
    const double ab = s->a + s->b, abc = s->a + s->b + s->c;
    for (int l = 0; l < s->scale; ++l) {
        double r = u01(draw(kq, (uint64_t)e * (uint64_t)s->scale + (uint64_t)l));
        uint64_t rb, cb;
        if (r < s->a) { rb = 0; cb = 0; }
        else if (r < ab) { rb = 0; cb = 1; }
        else if (r < abc) { rb = 1; cb = 0; }
        else { rb = 1; cb = 1; }
        src = (src << 1) | rb;
        dst = (dst << 1) | cb;
    }
    if (src == dst) return 0;
    *u = s->perm[src];
    *v = s->perm[dst];
    *w = s->wmax > 1 ? 1 + (int32_t)below(draw(kw, (uint64_t)e), (uint64_t)s->wmax) : 1;
    return 1;
}

static inline int64_t sbm_block(const gen_spec *s, int64_t v)
{
    return (int64_t)(((unsigned __int128)v * (uint64_t)s->k) / (uint64_t)s->n);
}

/* first vertex of the block after v's block */
static inline int64_t sbm_block_end(const gen_spec *s, int64_t v)
{
    int64_t b = sbm_block(s, v) + 1;
    /* smallest x with floor(x*k/n) >= b  is ceil(b*n/k) */
    return (int64_t)(((unsigned __int128)b * (uint64_t)s->n + (uint64_t)s->k - 1) / (uint64_t)s->k);
}

/*
 * Walk the SBM pairs (u, v > u) of vertex u.  Geometric skipping: the gap to
 * the next success of a Bernoulli(p) sequence is floor(log(1-r)/log(1-p)).
 * fill = 0 counts degrees into deg[]; fill = 1 places entries using cur[].
 */
static void sbm_row(const gen_spec *s, uint64_t key, int64_t u, int fill,
                    int64_t *deg, int64_t *cur, uint64_t *ent)
{
    uint64_t ctr = (uint64_t)u << 32;
    int64_t be = sbm_block_end(s, u);
    if (be > s->n) be = s->n;
    const int64_t seg_lo[2] = {u + 1, be}, seg_hi[2] = {be, s->n};
    const double seg_p[2] = {s->p_in, s->p_out};
    for (int sg = 0; sg < 2; ++sg) {
        double p = seg_p[sg];
        if (p <= 0.0 || seg_lo[sg] >= seg_hi[sg]) continue;
        double lq = p >= 1.0 ? 0.0 : log1p(-p);
        int64_t pos = seg_lo[sg] - 1;
        for (;;) {
            int64_t skip = 0;
            if (p < 1.0) {
                double r = u01(draw(key, ctr++));
                double gap = floor(log1p(-r) / lq);
                if (gap > (double)(seg_hi[sg] - pos)) break;
                skip = (int64_t)gap;
            }
            pos += skip + 1;
            if (pos >= seg_hi[sg]) break;
            int64_t v = pos;
            if (!fill) {
#pragma omp atomic
                deg[u + 1] += 1;
#pragma omp atomic
                deg[v + 1] += 1;
            } else {
                int64_t pu, pv;
#pragma omp atomic capture
                pu = cur[u]++;
#pragma omp atomic capture
                pv = cur[v]++;
                ent[pu] = ((uint64_t)(uint32_t)v << 32) | 1u;
                ent[pv] = ((uint64_t)(uint32_t)u << 32) | 1u;
            }
        }
    }
}

static int cmp_u64(const void *x, const void *y)
{
    uint64_t a = *(const uint64_t *)x, b = *(const uint64_t *)y;
    return (a > b) - (a < b);
}

static void set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

/* Build the symmetric CSR of a generator spec: count, fill, sort rows, merge. */
static gg_graph *assemble(gen_spec *s)
{
    gg_graph *g = (gg_graph *)calloc(1, sizeof(gg_graph));
    if (!g) return NULL;
    int64_t n = s->kind == 0 ? ((int64_t)1 << s->scale) : s->n;
    g->n = n;
    int64_t *deg = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    if (!deg) { g->status = -1; return g; }
    uint64_t kq = stream_key(s->seed, S_QUAD), kw = stream_key(s->seed, S_WEIGHT);
    uint64_t ks = stream_key(s->seed, S_SBM);

    /* pass 1: degrees */
    if (s->kind == 0) {
#pragma omp parallel for schedule(static)
        for (int64_t e = 0; e < s->draws; ++e) {
            int32_t u, v, w;
            if (!rmat_edge(s, kq, kw, e, &u, &v, &w)) continue;
#pragma omp atomic
            deg[u + 1] += 1;
#pragma omp atomic
            deg[v + 1] += 1;
        }
    } else {
#pragma omp parallel for schedule(dynamic, 64)
        for (int64_t u = 0; u < n; ++u) sbm_row(s, ks, u, 0, deg, NULL, NULL);
    }
    for (int64_t i = 0; i < n; ++i) deg[i + 1] += deg[i];
    int64_t raw = deg[n];
    uint64_t *ent = (uint64_t *)malloc((size_t)(raw > 0 ? raw : 1) * sizeof(uint64_t));
    int64_t *cur = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    if (!ent || !cur) { free(ent); free(cur); free(deg); g->status = -1; return g; }
    memcpy(cur, deg, (size_t)n * sizeof(int64_t));

    /* pass 2: fill entries as (target << 32 | weight) */
    if (s->kind == 0) {
#pragma omp parallel for schedule(static)
        for (int64_t e = 0; e < s->draws; ++e) {
            int32_t u, v, w;
            int64_t pu, pv;
            if (!rmat_edge(s, kq, kw, e, &u, &v, &w)) continue;
#pragma omp atomic capture
            pu = cur[u]++;
#pragma omp atomic capture
            pv = cur[v]++;
            ent[pu] = ((uint64_t)(uint32_t)v << 32) | (uint32_t)w;
            ent[pv] = ((uint64_t)(uint32_t)u << 32) | (uint32_t)w;
        }
    } else {
#pragma omp parallel for schedule(dynamic, 64)
        for (int64_t u = 0; u < n; ++u) sbm_row(s, ks, u, 1, NULL, cur, ent);
    }
    free(cur);

    /* sort each row, merge duplicates in place, record merged row lengths */
    int64_t *len = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    int bad = 0;
    if (!len) { free(ent); free(deg); g->status = -1; return g; }
#pragma omp parallel for schedule(dynamic, 256) reduction(| : bad)
    for (int64_t i = 0; i < n; ++i) {
        uint64_t *r = ent + deg[i];
        int64_t m = deg[i + 1] - deg[i];
        if (m > 1) qsort(r, (size_t)m, sizeof(uint64_t), cmp_u64);
        int64_t o = 0;
        for (int64_t k = 0; k < m;) {
            uint64_t t = r[k] >> 32;
            int64_t sw = 0;
            while (k < m && (r[k] >> 32) == t) { sw += (int64_t)(uint32_t)r[k]; ++k; }
            if (sw > INT32_MAX) bad = 1;
            r[o++] = (t << 32) | (uint32_t)(sw > INT32_MAX ? INT32_MAX : sw);
        }
        len[i + 1] = o;
    }
    if (bad) { free(ent); free(deg); free(len); g->status = -2; return g; }
    for (int64_t i = 0; i < n; ++i) len[i + 1] += len[i];
    g->nnz = len[n];
    g->off = len;
    g->tgt = (int32_t *)malloc((size_t)(g->nnz > 0 ? g->nnz : 1) * sizeof(int32_t));
    g->w = (int32_t *)malloc((size_t)(g->nnz > 0 ? g->nnz : 1) * sizeof(int32_t));
    if (!g->tgt || !g->w) { free(ent); free(deg); g->status = -1; return g; }
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t i = 0; i < n; ++i) {
        const uint64_t *r = ent + deg[i];
        int64_t o = len[i], m = len[i + 1] - len[i];
        for (int64_t k = 0; k < m; ++k) {
            g->tgt[o + k] = (int32_t)(r[k] >> 32);
            g->w[o + k] = (int32_t)(uint32_t)r[k];
        }
    }
    free(ent);
    free(deg);
    return g;
}

gg_graph *gg_rmat(int32_t scale, int64_t draws, double a, double b, double c,
                  int32_t wmax, uint64_t seed, int32_t nthreads)
{
    if (scale < 1 || scale > 30 || draws < 0 || wmax < 1 || a < 0 || b < 0 || c < 0 ||
        a + b + c > 1.0) {
        gg_graph *g = (gg_graph *)calloc(1, sizeof(gg_graph));
        if (g) g->status = -3;
        return g;
    }
    set_threads(nthreads);
    gen_spec s;
    memset(&s, 0, sizeof(s));
    s.kind = 0;
    s.scale = scale;
    s.draws = draws;
    s.a = a;
    s.b = b;
    s.c = c;
    s.wmax = wmax;
    s.seed = seed;
    int64_t n = (int64_t)1 << scale;
    s.perm = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    if (!s.perm) {
        gg_graph *g = (gg_graph *)calloc(1, sizeof(gg_graph));
        if (g) g->status = -1;
        return g;
    }
    /* Fisher-Yates shuffle driven by the permutation stream */
    uint64_t kp = stream_key(seed, S_PERM);
    for (int64_t i = 0; i < n; ++i) s.perm[i] = (int32_t)i;
    for (int64_t i = n - 1; i > 0; --i) {
        int64_t j = (int64_t)below(draw(kp, (uint64_t)i), (uint64_t)(i + 1));
        int32_t t = s.perm[i];
        s.perm[i] = s.perm[j];
        s.perm[j] = t;
    }
    gg_graph *g = assemble(&s);
    free(s.perm);
    return g;
}

gg_graph *gg_sbm(int64_t n, int64_t k, double p_in, double p_out, uint64_t seed,
                 int32_t nthreads)
{
    if (n < 0 || n > INT32_MAX || k < 1 || (n > 0 && k > n) || p_in < 0 || p_in > 1 ||
        p_out < 0 || p_out > 1) {
        gg_graph *g = (gg_graph *)calloc(1, sizeof(gg_graph));
        if (g) g->status = -3;
        return g;
    }
    set_threads(nthreads);
    gen_spec s;
    memset(&s, 0, sizeof(s));
    s.kind = 1;
    s.n = n;
    s.k = k;
    s.p_in = p_in;
    s.p_out = p_out;
    s.seed = seed;
    return assemble(&s);
}

int gg_status(const gg_graph *g) { return g ? g->status : -1; }
int64_t gg_n(const gg_graph *g) { return g->n; }
int64_t gg_nnz(const gg_graph *g) { return g->nnz; }

void gg_copy(const gg_graph *g, int64_t *off, int32_t *tgt, int32_t *w)
{
    memcpy(off, g->off, (size_t)(g->n + 1) * sizeof(int64_t));
    if (g->nnz > 0) {
        memcpy(tgt, g->tgt, (size_t)g->nnz * sizeof(int32_t));
        memcpy(w, g->w, (size_t)g->nnz * sizeof(int32_t));
    }
}

void gg_free(gg_graph *g)
{
    if (!g) return;
    free(g->off);
    free(g->tgt);
    free(g->w);
    free(g);
}
