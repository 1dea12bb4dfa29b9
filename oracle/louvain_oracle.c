/*
 * Louvain oracle: a plain, slow, serial CPU implementation of the method of
 * "GVE-Louvain: Fast Louvain Algorithm for Community Detection in Shared
 * Memory Setting" (Sahu, arXiv 2312.04876).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code with
 * the GPU path and nothing in the GPU path may call it.
 *
 * Arithmetic: every quantity is an exact integer (int64, or __int128 where a
 * product of two weights can exceed 63 bits); the only floating-point values
 * are the per-iteration delta-modularity compared with the tolerance and the
 * returned modularity, each a single FP64 expression over exact integers.
 *
 * Conventions (paper Section 3, "Preliminaries"):
 *   - A CSR entry (i -> j, w) is one directed entry; an undirected edge is
 *     stored twice, a self-loop once.
 *   - K_i is the sum of the weights in row i (self-loop included) and
 *     W = 2m = sum_i K_i.
 *   - sigma_c sums the entries whose two ends lie in c; Sigma_c = sum of K_i
 *     over the members of c.
 *
 * Modularity (Eq. 1, second form):  Q = sum_c [ sigma_c/W - (Sigma_c/W)^2 ]
 *   = (sigma_tot*W - sum_c Sigma_c^2) / W^2, evaluated as one FP64 division
 *   of the two exactly computed integers.
 *
 * Delta-modularity (Eq. 2) of moving i from d to c, scaled by W^2/2:
 *   N = [W*K_{i->c} - K_i*Sigma_c] - [W*K_{i->d} - K_i*(Sigma_d - K_i)]
 *   where K_{i->x} leaves out i's self-loop, so that dQ = 2N/W^2 exactly.
 *
 * Synchronous (deterministic) iteration -- not in the paper, which runs
 * asynchronously (Section 4.1).  Iteration l of pass p visits the active
 * vertices in R = 2^sample_bits rounds; vertex i belongs to round r = the top
 * `sample_bits` bits of the SplitMix64 output (Steele, Lea and Flood, OOPSLA
 * 2014) for counter (p << 40 | l << 32 | i) under key `seed`.  In a round,
 * each of its vertices decides against the state at the start of the round,
 * a singleton may join another singleton community only if that community's
 * id is smaller (the min-label heuristic of Lu et al. 2015, cited in
 * Section 2), and the round's moves are applied together before the next
 * round.  Movers mark their rows for the next iteration; the tolerance test
 * sees the gains of all rounds.
 *
 * Colour-ordered iteration -- the colouring alternative of Section 2, also
 * not the paper's own choice.  Each pass colours its graph greedily in
 * decreasing order of a SplitMix64 priority per vertex (counter
 * 1 << 63 | p << 40 | i under `seed`): the colouring Jones and Plassmann's
 * parallel algorithm (SIAM J. Sci. Comput. 1993) produces.  Iteration l then
 * runs one synchronous round per colour class in ascending colour order; no
 * two vertices of a round are neighbours, so the singleton rule is off.
 *
 * parity pins: modularity, the move gain, the sequential sweep, renumbering,
 * the community-vertex CSR, aggregation and the whole pass loop are each
 * checked against independent definitions in the CPU test-suite; the
 * synchronous and colour-ordered iterations are pinned by hand-worked cases,
 * invariants and a brute-force recomputation of whole iterations on small
 * graphs (gains from the pairwise form of modularity, rounds from the
 * generator module's SplitMix64, the decision rule restated); the colouring
 * is pinned by its defining properties (proper, greedy-minimal in priority
 * order) and the colour-ordered iteration also by its reduction to the
 * sequential sweep when priorities fall with the vertex id on a clique.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef __int128 i128;

enum { ORACLE_SYNC = 0, ORACLE_SEQ = 1, ORACLE_COLOUR = 2 };

static void split128(i128 x, int64_t *hi, uint64_t *lo)
{
    *lo = (uint64_t)x;
    *hi = (int64_t)(x >> 64);
}

/* SplitMix64 output function (Steele, Lea and Flood 2014). */
static uint64_t splitmix_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* The synchronous iteration's round of vertex i in iteration l of pass p (the
 * hashed-round reading of the synchronous mode, which the paper does not have). */
static int32_t sync_round(uint64_t seed, int32_t sample_bits, int32_t p, int32_t l, int32_t i)
{
    if (sample_bits <= 0) return 0;
    uint64_t ctr = ((uint64_t)(uint32_t)p << 40) | ((uint64_t)(uint32_t)(l & 0xFF) << 32) |
                   (uint64_t)(uint32_t)i;
    uint64_t x = splitmix_mix(seed + (ctr + 1) * 0x9E3779B97F4A7C15ULL);
    return (int32_t)(x >> (64 - sample_bits));
}

/* Priority of vertex v in pass p for the colouring of the colour-ordered reading
 * (distinct for distinct v). */
static uint64_t colour_priority(uint64_t seed, int32_t p, int32_t v)
{
    uint64_t ctr = (1ULL << 63) | ((uint64_t)(uint32_t)p << 40) | (uint64_t)(uint32_t)v;
    return splitmix_mix(seed + (ctr + 1) * 0x9E3779B97F4A7C15ULL);
}

typedef struct {
    uint64_t prio;
    int32_t v;
} prio_v;

static int cmp_prio_desc(const void *a, const void *b)
{
    uint64_t x = ((const prio_v *)a)->prio, y = ((const prio_v *)b)->prio;
    return x < y ? 1 : (x > y ? -1 : 0);
}

/* Greedy colouring in decreasing priority order (the colouring Jones and
 * Plassmann's parallel algorithm computes): every vertex takes the smallest
 * colour no higher-priority neighbour has.  Self-loops are ignored.  Returns
 * the number of colours, or -1 on allocation failure. */
int32_t oracle_colour(int32_t n, const int64_t *off, const int32_t *tgt, uint64_t seed,
                      int32_t pass_index, int32_t *colour)
{
    size_t m = (size_t)(n > 0 ? n : 1);
    prio_v *order = (prio_v *)malloc(m * sizeof(prio_v));
    int32_t *stamp = (int32_t *)malloc((m + 1) * sizeof(int32_t));
    if (!order || !stamp) {
        free(order);
        free(stamp);
        return -1;
    }
    for (int32_t v = 0; v < n; ++v) {
        order[v].prio = colour_priority(seed, pass_index, v);
        order[v].v = v;
        colour[v] = -1;
    }
    for (size_t c = 0; c <= m; ++c) stamp[c] = -1;
    qsort(order, (size_t)n, sizeof(prio_v), cmp_prio_desc);
    int32_t ncol = 0;
    for (int32_t k = 0; k < n; ++k) {
        int32_t v = order[k].v;
        for (int64_t e = off[v]; e < off[v + 1]; ++e) {
            int32_t u = tgt[e];
            if (u != v && colour[u] >= 0) stamp[colour[u]] = v;
        }
        int32_t c = 0;
        while (stamp[c] == v) ++c;
        colour[v] = c;
        if (c + 1 > ncol) ncol = c + 1;
    }
    free(order);
    free(stamp);
    return ncol;
}

/* K_i = row sums (Alg. 1, vertexWeights); returns W = sum_i K_i. */
int64_t oracle_vertex_weights(int32_t n, const int64_t *off, const int64_t *w,
                              int64_t *K)
{
    int64_t W = 0;
    for (int32_t i = 0; i < n; ++i) {
        int64_t s = 0;
        for (int64_t e = off[i]; e < off[i + 1]; ++e) s += w[e];
        K[i] = s;
        W += s;
    }
    return W;
}

/*
 * Modularity, Eq. 1 (second form), as the exact fraction num/den with
 * num = sigma_tot*W - sum_c Sigma_c^2 and den = W^2.  Labels C[i] must lie in
 * [0, n).  Returns 0 on success, -1 on a label out of range or on allocation
 * failure.
 */
int oracle_modularity_exact(int32_t n, const int64_t *off, const int32_t *tgt,
                            const int64_t *w, const int32_t *C,
                            int64_t *num_hi, uint64_t *num_lo,
                            int64_t *den_hi, uint64_t *den_lo)
{
    int64_t *Sig = (int64_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
    if (!Sig) return -1;
    int64_t W = 0, sigma = 0;
    for (int32_t i = 0; i < n; ++i) {
        if (C[i] < 0 || C[i] >= n) { free(Sig); return -1; }
        for (int64_t e = off[i]; e < off[i + 1]; ++e) {
            W += w[e];
            Sig[C[i]] += w[e];
            if (C[tgt[e]] == C[i]) sigma += w[e];
        }
    }
    i128 s2 = 0;
    for (int32_t c = 0; c < n; ++c) s2 += (i128)Sig[c] * (i128)Sig[c];
    i128 num = (i128)sigma * (i128)W - s2;
    i128 den = (i128)W * (i128)W;
    split128(num, num_hi, num_lo);
    split128(den, den_hi, den_lo);
    free(Sig);
    return 0;
}

/* Eq. 1 as a double: (double)num / (double)den, and 0 for an edgeless graph. */
double oracle_modularity(int32_t n, const int64_t *off, const int32_t *tgt,
                         const int64_t *w, const int32_t *C)
{
    int64_t nh, dh;
    uint64_t nl, dl;
    if (oracle_modularity_exact(n, off, tgt, w, C, &nh, &nl, &dh, &dl) != 0)
        return -2.0;
    i128 num = ((i128)nh << 64) | (i128)nl;
    i128 den = ((i128)dh << 64) | (i128)dl;
    if (den == 0) return 0.0;
    return (double)num / (double)den;
}

/*
 * Per-vertex scratch for scanCommunities (Alg. 2): a dense accumulator indexed
 * by community id plus the list of keys touched, reset after each use.
 */
typedef struct {
    int64_t *acc;
    uint8_t *seen;
    int32_t *keys;
    int32_t nk;
} scan_table;

static int table_init(scan_table *t, int32_t n)
{
    size_t m = (size_t)(n > 0 ? n : 1);
    t->acc = (int64_t *)calloc(m, sizeof(int64_t));
    t->seen = (uint8_t *)calloc(m, 1);
    t->keys = (int32_t *)malloc(m * sizeof(int32_t));
    t->nk = 0;
    return (t->acc && t->seen && t->keys) ? 0 : -1;
}

static void table_free(scan_table *t)
{
    free(t->acc);
    free(t->seen);
    free(t->keys);
}

static void table_add(scan_table *t, int32_t c, int64_t w)
{
    if (!t->seen[c]) {
        t->seen[c] = 1;
        t->acc[c] = 0;
        t->keys[t->nk++] = c;
    }
    t->acc[c] += w;
}

static void table_clear(scan_table *t)
{
    for (int32_t k = 0; k < t->nk; ++k) t->seen[t->keys[k]] = 0;
    t->nk = 0;
}

/*
 * scanCommunities (Alg. 2): accumulate the weight from i to each community
 * of its neighbours; self = 0 leaves out i's self-loop (local moving),
 * self = 1 keeps it (aggregation).  Returns the number of entries added.
 */
static int64_t scan_communities(scan_table *t, const int64_t *off,
                                const int32_t *tgt, const int64_t *w,
                                const int32_t *C, int32_t i, int self)
{
    int64_t added = 0;
    for (int64_t e = off[i]; e < off[i + 1]; ++e) {
        int32_t j = tgt[e];
        if (!self && j == i) continue;
        table_add(t, C[j], w[e]);
        ++added;
    }
    return added;
}

/*
 * Best community for vertex i (Alg. 2, choice of c* and its gain).
 * Candidates are the neighbour communities other than d = C[i]; the score of
 * c is W*K_{i->c} - K_i*Sigma_c and ties go to the smallest id.  The vertex
 * moves only if the best score strictly exceeds the score of staying,
 * W*K_{i->d} - K_i*(Sigma_d - K_i).  With min_label set, a singleton may join
 * another singleton community only if that community's id is smaller.
 * Returns 1 and fills (cstar, N) for a move, 0 to stay.
 */
static int decide(scan_table *t, const int64_t *off, const int32_t *tgt,
                  const int64_t *w, const int64_t *K, int64_t W,
                  const int32_t *C, const int64_t *Sig, const int32_t *size,
                  int min_label, int32_t i, int32_t *cstar, i128 *N)
{
    int32_t d = C[i];
    int64_t nonself = scan_communities(t, off, tgt, w, C, i, 0);
    int moved = 0;
    if (nonself > 0) {
        i128 Ki = K[i];
        i128 hd = t->seen[d] ? t->acc[d] : 0;
        i128 stay = (i128)W * hd - Ki * ((i128)Sig[d] - Ki);
        int found = 0;
        int32_t bc = -1;
        i128 best = 0;
        for (int32_t k = 0; k < t->nk; ++k) {
            int32_t c = t->keys[k];
            if (c == d) continue;
            i128 s = (i128)W * (i128)t->acc[c] - Ki * (i128)Sig[c];
            if (!found || s > best || (s == best && c < bc)) {
                found = 1;
                best = s;
                bc = c;
            }
        }
        if (found && best > stay) {
            if (!(min_label && size[d] == 1 && size[bc] == 1 && bc > d)) {
                *cstar = bc;
                *N = best - stay;
                moved = 1;
            }
        }
    }
    table_clear(t);
    return moved;
}

/*
 * Exact gain N (Eq. 2 scaled by W^2/2) of moving vertex i from C[i] to c,
 * with Sigma recomputed from the membership C (labels in [0, n)).  Returns
 * 0 on success.
 */
int oracle_move_gain(int32_t n, const int64_t *off, const int32_t *tgt,
                     const int64_t *w, const int32_t *C, int32_t i, int32_t c,
                     int64_t *N_hi, uint64_t *N_lo)
{
    int64_t *K = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    int64_t *Sig = (int64_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
    if (!K || !Sig) { free(K); free(Sig); return -1; }
    int64_t W = oracle_vertex_weights(n, off, w, K);
    for (int32_t v = 0; v < n; ++v) Sig[C[v]] += K[v];
    int32_t d = C[i];
    i128 kc = 0, kd = 0;
    for (int64_t e = off[i]; e < off[i + 1]; ++e) {
        int32_t j = tgt[e];
        if (j == i) continue;
        if (C[j] == c) kc += w[e];
        if (C[j] == d) kd += w[e];
    }
    i128 Ki = K[i];
    i128 N;
    if (c == d) {
        N = 0;
    } else {
        N = ((i128)W * kc - Ki * (i128)Sig[c]) -
            ((i128)W * kd - Ki * ((i128)Sig[d] - Ki));
    }
    split128(N, N_hi, N_lo);
    free(K);
    free(Sig);
    return 0;
}

/* The tolerance test of Alg. 2: dQ = 2*sumN / W^2 in FP64 (0 if W = 0). */
static double iteration_dq(i128 sumN, int64_t W)
{
    if (W == 0) return 0.0;
    return 2.0 * (double)sumN / ((double)W * (double)W);
}

/*
 * louvainMove (Alg. 2) from the given state, updating C, Sigma, size and the
 * active flags in place.
 *   mode ORACLE_SEQ : asynchronous semantics on one thread, vertices visited
 *                     in ascending id order against the live state; a mover
 *                     re-marks its neighbours, who may run later in the same
 *                     sweep.
 *   mode ORACLE_SYNC: the active vertices are split into 2^sample_bits
 *                     rounds (seed, pass_index; see the file header); each
 *                     round decides against the state at its start
 *                     (min-label singleton rule on) and then applies its
 *                     moves; the next iteration's active set is the rows of
 *                     the movers.
 *   colour != NULL  : synchronous rounds, round r = the vertices of colour r
 *                     (r < ncolour), singleton rule off.
 * prune = 0 processes every vertex in every sweep.
 * Per-sweep traces (length max_iter, may be NULL): sumN split in hi/lo,
 * number of moves, number of vertices processed.
 * Returns the number of sweeps run (l_i), or -1 on allocation failure.
 */
static int32_t move_impl(int32_t mode, int32_t n, const int64_t *off,
                         const int32_t *tgt, const int64_t *w, const int64_t *K,
                         int64_t W, int64_t *Sig, int32_t *C, int32_t *size,
                         uint8_t *active, int32_t prune, double tau,
                         int32_t max_iter, uint64_t seed, int32_t pass_index,
                         int32_t sample_bits, const int32_t *colour, int32_t ncolour,
                         int64_t *tr_hi, uint64_t *tr_lo,
                         int32_t *tr_moves, int32_t *tr_processed)
{
    scan_table t;
    size_t m = (size_t)(n > 0 ? n : 1);
    int32_t *C0 = (int32_t *)malloc(m * sizeof(int32_t));
    int64_t *S0 = (int64_t *)malloc(m * sizeof(int64_t));
    int32_t *z0 = (int32_t *)malloc(m * sizeof(int32_t));
    int32_t *mv_i = (int32_t *)malloc(m * sizeof(int32_t));
    int32_t *mv_c = (int32_t *)malloc(m * sizeof(int32_t));
    i128 *mv_N = (i128 *)malloc(m * sizeof(i128));
    uint8_t *mark = (uint8_t *)malloc(m);
    /* one scan table per thread for the decisions of a synchronous round
     * (a single table without OpenMP) */
#ifdef _OPENMP
    const int nt = mode == ORACLE_SEQ ? 1 : omp_get_max_threads();
#else
    const int nt = 1;
#endif
    scan_table *tt = (scan_table *)calloc((size_t)nt, sizeof(scan_table));
    int tables_ok = tt != NULL;
    for (int k = 0; tt && k < nt; ++k)
        if (table_init(&tt[k], n) != 0) tables_ok = 0;
    if (table_init(&t, n) != 0 || !tables_ok || !C0 || !S0 || !z0 || !mv_i || !mv_c || !mv_N ||
        !mark) {
        table_free(&t);
        for (int k = 0; tt && k < nt; ++k) table_free(&tt[k]);
        free(tt);
        free(C0); free(S0); free(z0); free(mv_i); free(mv_c); free(mv_N); free(mark);
        return -1;
    }
    int32_t l = 0;
    for (int32_t it = 0; it < max_iter; ++it) {
        l = it + 1;
        i128 sumN = 0;
        int32_t moves = 0, processed = 0;
        if (!prune) memset(active, 1, (size_t)n);
        if (mode == ORACLE_SEQ) {
            for (int32_t i = 0; i < n; ++i) {
                if (!active[i]) continue;
                active[i] = 0;
                ++processed;
                int32_t c;
                i128 N;
                if (!decide(&t, off, tgt, w, K, W, C, Sig, size, 0, i, &c, &N))
                    continue;
                int32_t d = C[i];
                Sig[d] -= K[i];
                Sig[c] += K[i];
                size[d] -= 1;
                size[c] += 1;
                C[i] = c;
                sumN += N;
                ++moves;
                for (int64_t e = off[i]; e < off[i + 1]; ++e) active[tgt[e]] = 1;
            }
        } else {
            /* colour-ordered mode: one round per colour class, so no two
             * neighbours ever move together and the singleton rule is not needed */
            int32_t rounds = colour ? ncolour : 1 << (sample_bits > 0 ? sample_bits : 0);
            memset(mark, 0, (size_t)n);
            for (int32_t r = 0; r < rounds; ++r) {
                memcpy(C0, C, (size_t)n * sizeof(int32_t));
                memcpy(S0, Sig, (size_t)n * sizeof(int64_t));
                memcpy(z0, size, (size_t)n * sizeof(int32_t));
                /* every decision of the round reads only the snapshot (C0, S0, z0),
                 * so the decisions are independent: vertex i's choice goes to
                 * mv_c[i] (-1 to stay) and its gain to mv_N[i].  A build with
                 * OpenMP takes them on several threads; the moves are then listed
                 * and applied in ascending vertex order either way. */
                int32_t nproc = 0;
#pragma omp parallel for schedule(dynamic, 1024) reduction(+ : nproc)
                for (int32_t i = 0; i < n; ++i) {
                    mv_c[i] = -1;
                    if (!active[i]) continue;
                    if ((colour ? colour[i] : sync_round(seed, sample_bits, pass_index, it, i)) != r)
                        continue;
                    active[i] = 0;
                    ++nproc;
#ifdef _OPENMP
                    scan_table *ti = &tt[omp_get_thread_num()];
#else
                    scan_table *ti = &tt[0];
#endif
                    int32_t c;
                    i128 N;
                    if (decide(ti, off, tgt, w, K, W, C0, S0, z0, colour ? 0 : 1, i, &c, &N)) {
                        mv_c[i] = c;
                        mv_N[i] = N;
                    }
                }
                processed += nproc;
                int32_t nm = 0;
                for (int32_t i = 0; i < n; ++i)
                    if (mv_c[i] >= 0) mv_i[nm++] = i;
                for (int32_t k = 0; k < nm; ++k) {
                    int32_t i = mv_i[k], c = mv_c[i], d = C[i];
                    Sig[d] -= K[i];
                    Sig[c] += K[i];
                    size[d] -= 1;
                    size[c] += 1;
                    C[i] = c;
                    sumN += mv_N[i];
                    for (int64_t e = off[i]; e < off[i + 1]; ++e) mark[tgt[e]] = 1;
                }
                moves += nm;
            }
            for (int32_t i = 0; i < n; ++i)
                if (mark[i]) active[i] = 1;
        }
        if (tr_hi) split128(sumN, &tr_hi[it], &tr_lo[it]);
        if (tr_moves) tr_moves[it] = moves;
        if (tr_processed) tr_processed[it] = processed;
        if (iteration_dq(sumN, W) <= tau) break;
    }
    table_free(&t);
    for (int k = 0; k < nt; ++k) table_free(&tt[k]);
    free(tt);
    free(C0); free(S0); free(z0); free(mv_i); free(mv_c); free(mv_N); free(mark);
    return l;
}

int32_t oracle_move(int32_t mode, int32_t n, const int64_t *off,
                    const int32_t *tgt, const int64_t *w, const int64_t *K,
                    int64_t W, int64_t *Sig, int32_t *C, int32_t *size,
                    uint8_t *active, int32_t prune, double tau,
                    int32_t max_iter, uint64_t seed, int32_t pass_index,
                    int32_t sample_bits, int64_t *tr_hi, uint64_t *tr_lo,
                    int32_t *tr_moves, int32_t *tr_processed)
{
    return move_impl(mode, n, off, tgt, w, K, W, Sig, C, size, active, prune, tau, max_iter,
                     seed, pass_index, sample_bits, NULL, 0, tr_hi, tr_lo, tr_moves,
                     tr_processed);
}

/* Colour-ordered local moving: synchronous rounds, round r = the vertices of
 * colour r (colour[i] in [0, ncolour)). */
int32_t oracle_move_coloured(int32_t n, const int64_t *off, const int32_t *tgt,
                             const int64_t *w, const int64_t *K, int64_t W, int64_t *Sig,
                             int32_t *C, int32_t *size, uint8_t *active, int32_t prune,
                             double tau, int32_t max_iter, const int32_t *colour,
                             int32_t ncolour, int64_t *tr_hi, uint64_t *tr_lo,
                             int32_t *tr_moves, int32_t *tr_processed)
{
    return move_impl(ORACLE_SYNC, n, off, tgt, w, K, W, Sig, C, size, active, prune, tau,
                     max_iter, 0, 0, 0, colour, ncolour, tr_hi, tr_lo, tr_moves, tr_processed);
}

/*
 * Renumber communities (Alg. 1): each used label c < n becomes the number of
 * used labels below it, so the order of labels is kept.  Returns the number
 * of communities, or -1 on a label out of range.
 */
int32_t oracle_renumber(int32_t n, int32_t *C)
{
    int32_t *id = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    if (!id) return -1;
    for (int32_t c = 0; c < n; ++c) id[c] = -1;
    for (int32_t i = 0; i < n; ++i) {
        if (C[i] < 0 || C[i] >= n) { free(id); return -1; }
        id[C[i]] = 0;
    }
    int32_t nc = 0;
    for (int32_t c = 0; c < n; ++c)
        if (id[c] == 0) id[c] = nc++;
    for (int32_t i = 0; i < n; ++i) C[i] = id[C[i]];
    free(id);
    return nc;
}

/*
 * Community-vertex CSR (Alg. 3): count members per community, exclusive
 * scan, then place each vertex; here vertices are placed in ascending order.
 * C must be dense in [0, nc).
 */
void oracle_community_vertices(int32_t n, const int32_t *C, int32_t nc,
                               int64_t *coff, int32_t *members)
{
    for (int32_t c = 0; c <= nc; ++c) coff[c] = 0;
    for (int32_t i = 0; i < n; ++i) coff[C[i] + 1] += 1;
    for (int32_t c = 0; c < nc; ++c) coff[c + 1] += coff[c];
    int64_t *cur = (int64_t *)malloc((size_t)(nc > 0 ? nc : 1) * sizeof(int64_t));
    for (int32_t c = 0; c < nc; ++c) cur[c] = coff[c];
    for (int32_t i = 0; i < n; ++i) members[cur[C[i]]++] = i;
    free(cur);
}

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/*
 * louvainAggregate (Alg. 3): the super-vertex graph of a dense membership C
 * (labels in [0, nc)).  Row c holds, for every community d linked to a member
 * of c (self-loops kept), the total weight between c and d.  Output is the
 * canonical CSR: rows sorted by target, no gaps.  Returns the number of
 * entries written, or -1 if cap is too small or allocation fails.
 */
int64_t oracle_aggregate(int32_t n, const int64_t *off, const int32_t *tgt,
                         const int64_t *w, const int32_t *C, int32_t nc,
                         int64_t *out_off, int32_t *out_tgt, int64_t *out_w,
                         int64_t cap)
{
    scan_table t = {0};
    int64_t *coff = (int64_t *)malloc((size_t)(nc + 1) * sizeof(int64_t));
    int32_t *members = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    if (!coff || !members || table_init(&t, nc) != 0) {
        free(coff); free(members); table_free(&t);
        return -1;
    }
    oracle_community_vertices(n, C, nc, coff, members);
    int64_t pos = 0;
    out_off[0] = 0;
    for (int32_t c = 0; c < nc; ++c) {
        for (int64_t k = coff[c]; k < coff[c + 1]; ++k)
            scan_communities(&t, off, tgt, w, C, members[k], 1);
        if (pos + t.nk > cap) {
            free(coff); free(members); table_free(&t);
            return -1;
        }
        qsort(t.keys, (size_t)t.nk, sizeof(int32_t), cmp_i32);
        for (int32_t k = 0; k < t.nk; ++k) {
            out_tgt[pos] = t.keys[k];
            out_w[pos] = t.acc[t.keys[k]];
            ++pos;
        }
        table_clear(&t);
        out_off[c + 1] = pos;
    }
    free(coff);
    free(members);
    table_free(&t);
    return pos;
}

/*
 * The whole method (Alg. 1): passes of local moving and aggregation with
 * threshold scaling, the global-convergence and aggregation-tolerance tests,
 * and the dendrogram lookup.  The final lookup is applied only when the pass
 * loop ended early (when it runs out of passes, the last pass already folded
 * its membership in).  The returned membership is renumbered densely in
 * label order; Q is the modularity of that membership on the input.
 * Per-pass records (arrays of length max_passes, may be NULL): sweeps run,
 * vertices of the level, communities after local moving.
 * Returns the number of passes whose local-moving phase ran, or a negative
 * value on failure.
 */
/* Alg. 1, optionally warm-started: with `initial` non-NULL the first pass's
 * local moving starts from those labels (each in [0, n)) instead of
 * singletons, with Sigma and the community sizes of that partition; later
 * passes start from singletons of their aggregated graph as usual. */
int32_t oracle_louvain_from(int32_t mode, int32_t max_passes, int32_t max_iter,
                            int32_t prune, double tolerance, double tolerance_drop,
                            double aggregation_tolerance, uint64_t seed,
                            int32_t sample_bits, int32_t n,
                            const int64_t *off, const int32_t *tgt,
                            const int64_t *w, const int32_t *initial,
                            int32_t *membership, double *Q,
                            int32_t *rec_iters, int32_t *rec_vertices,
                            int32_t *rec_comms)
{
    int64_t nnz = off[n];
    size_t m = (size_t)(n > 0 ? n : 1);
    size_t mz = (size_t)(nnz > 0 ? nnz : 1);
    int64_t *offA = (int64_t *)malloc((m + 1) * sizeof(int64_t));
    int32_t *tgtA = (int32_t *)malloc(mz * sizeof(int32_t));
    int64_t *wA = (int64_t *)malloc(mz * sizeof(int64_t));
    int64_t *offB = (int64_t *)malloc((m + 1) * sizeof(int64_t));
    int32_t *tgtB = (int32_t *)malloc(mz * sizeof(int32_t));
    int64_t *wB = (int64_t *)malloc(mz * sizeof(int64_t));
    int64_t *K = (int64_t *)malloc(m * sizeof(int64_t));
    int64_t *Sig = (int64_t *)malloc(m * sizeof(int64_t));
    int32_t *Cp = (int32_t *)malloc(m * sizeof(int32_t));
    int32_t *size = (int32_t *)malloc(m * sizeof(int32_t));
    uint8_t *active = (uint8_t *)malloc(m);
    int32_t *colour = (int32_t *)malloc(m * sizeof(int32_t));
    int32_t *top = membership;
    if (!offA || !tgtA || !wA || !offB || !tgtB || !wB || !K || !Sig || !Cp ||
        !size || !active || !colour) {
        free(offA); free(tgtA); free(wA); free(offB); free(tgtB); free(wB);
        free(K); free(Sig); free(Cp); free(size); free(active); free(colour);
        return -1;
    }
    /* G' <- G (level buffers are copies so that the input stays untouched) */
    memcpy(offA, off, (size_t)(n + 1) * sizeof(int64_t));
    if (nnz > 0) {
        memcpy(tgtA, tgt, (size_t)nnz * sizeof(int32_t));
        memcpy(wA, w, (size_t)nnz * sizeof(int64_t));
    }
    int64_t *loff = offA, *noff = offB, *lw = wA, *nw = wB;
    int32_t *ltgt = tgtA, *ntgt = tgtB;
    int32_t ln = n;
    for (int32_t v = 0; v < n; ++v) top[v] = v;
    double tau = tolerance;
    int broke = 0;
    int32_t passes = 0;
    int32_t rc = 0;
    for (int32_t p = 0; p < max_passes; ++p) {
        int64_t W = oracle_vertex_weights(ln, loff, lw, K);
        for (int32_t i = 0; i < ln; ++i) {
            Sig[i] = K[i];
            Cp[i] = i;
            size[i] = 1;
            active[i] = 1;
        }
        if (p == 0 && initial) {
            for (int32_t i = 0; i < ln; ++i) {
                Sig[i] = 0;
                size[i] = 0;
            }
            for (int32_t i = 0; i < ln; ++i) {
                Cp[i] = initial[i];
                Sig[initial[i]] += K[i];
                size[initial[i]] += 1;
            }
        }
        int32_t l;
        if (mode == ORACLE_COLOUR) {
            int32_t ncol = oracle_colour(ln, loff, ltgt, seed, p, colour);
            l = ncol < 0 ? -1
                         : move_impl(ORACLE_SYNC, ln, loff, ltgt, lw, K, W, Sig, Cp, size, active,
                                     prune, tau, max_iter, seed, p, sample_bits, colour, ncol,
                                     NULL, NULL, NULL, NULL);
        } else {
            l = move_impl(mode, ln, loff, ltgt, lw, K, W, Sig, Cp, size, active, prune, tau,
                          max_iter, seed, p, sample_bits, NULL, 0, NULL, NULL, NULL, NULL);
        }
        if (l < 0) { rc = -1; break; }
        passes = p + 1;
        if (rec_iters) rec_iters[p] = l;
        if (rec_vertices) rec_vertices[p] = ln;
        /* number of distinct labels after moving */
        memset(active, 0, (size_t)ln);
        int32_t nc = 0;
        for (int32_t i = 0; i < ln; ++i)
            if (!active[Cp[i]]) { active[Cp[i]] = 1; ++nc; }
        if (rec_comms) rec_comms[p] = nc;
        if (l <= 1) { broke = 1; break; }
        if ((double)nc / (double)ln > aggregation_tolerance) { broke = 1; break; }
        oracle_renumber(ln, Cp);
        for (int32_t v = 0; v < n; ++v) top[v] = Cp[top[v]];
        int64_t got = oracle_aggregate(ln, loff, ltgt, lw, Cp, nc, noff, ntgt,
                                       nw, nnz);
        if (got < 0) { rc = -1; break; }
        /* ping-pong the two level buffers */
        int64_t *t64 = loff; loff = noff; noff = t64;
        t64 = lw; lw = nw; nw = t64;
        int32_t *t32 = ltgt; ltgt = ntgt; ntgt = t32;
        ln = nc;
        tau = tau / tolerance_drop;
    }
    if (rc == 0) {
        if (broke)
            for (int32_t v = 0; v < n; ++v) top[v] = Cp[top[v]];
        oracle_renumber(n, top);
        *Q = oracle_modularity(n, off, tgt, w, top);
    }
    free(offA); free(tgtA); free(wA); free(offB); free(tgtB); free(wB);
    free(K); free(Sig); free(Cp); free(size); free(active); free(colour);
    return rc == 0 ? passes : rc;
}

/* Alg. 1 from singletons (oracle_louvain_from without a warm start). */
int32_t oracle_louvain(int32_t mode, int32_t max_passes, int32_t max_iter,
                       int32_t prune, double tolerance, double tolerance_drop,
                       double aggregation_tolerance, uint64_t seed,
                       int32_t sample_bits, int32_t n,
                       const int64_t *off, const int32_t *tgt,
                       const int64_t *w, int32_t *membership, double *Q,
                       int32_t *rec_iters, int32_t *rec_vertices,
                       int32_t *rec_comms)
{
    return oracle_louvain_from(mode, max_passes, max_iter, prune, tolerance,
                               tolerance_drop, aggregation_tolerance, seed,
                               sample_bits, n, off, tgt, w, NULL, membership, Q,
                               rec_iters, rec_vertices, rec_comms);
}
