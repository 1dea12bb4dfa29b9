/*
 * louvain.h -- C ABI of the MI355X (gfx950) Louvain hot path.
 *
 * The method is GVE-Louvain (Sahu, arXiv 2312.04876): passes of a
 * local-moving phase (Alg. 2: scan the communities of each vertex's
 * neighbours, pick the community with the largest delta-modularity of Eq. 2,
 * move, prune) and an aggregation phase (Alg. 3: community-vertex CSR by
 * prefix sum, holey super-vertex CSR built through per-community tables),
 * driven by the pass loop of Alg. 1 with threshold scaling and the
 * aggregation tolerance (Section 4.1).
 *
 * Graphs are CSR with int32 offsets, int32 targets and int32 weights.  An
 * undirected edge is stored as two entries (i->j and j->i, equal weights), a
 * self-loop as one entry.  All arithmetic is exact integer arithmetic (int64,
 * and 128-bit where products can exceed 63 bits); the only floating-point
 * values are the per-iteration delta-modularity tested against the tolerance
 * and the returned modularity (Eq. 1), each one FP64 expression over exact
 * integers.
 *
 * Memory and streams.  Pointers documented "device" are HIP device pointers
 * (for instance from torch tensors); "host" pointers are ordinary host
 * memory.  The library never allocates device memory: the caller owns the
 * input graph, the output membership and a workspace of
 * louvain_workspace_size() bytes, and all of them must stay valid until
 * louvain_destroy().  Every kernel is enqueued on the stream given to
 * louvain_init (a hipStream_t passed as void*; NULL = the default stream).
 * Calls that return host scalars synchronise that stream before returning.
 * A context serves one graph and must be used by one host thread at a time;
 * distinct contexts are independent.
 *
 * Errors.  Every call returns LOUVAIN_OK (0) or a negative status; nothing
 * is thrown across the ABI.  LOUVAIN_EHIP keeps the failing hipError_t,
 * which louvain_strerror() then describes.  After an error other than
 * LOUVAIN_EINVAL/LOUVAIN_ESTATE from argument checks, the context should be
 * destroyed.
 */
#ifndef LOUVAIN_H
#define LOUVAIN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct louvain_ctx louvain_ctx;

/* Execution modes of the local-moving phase. */
enum {
    /* Synchronous rounds: each iteration visits the active vertices in
     * 2^round_bits rounds picked by a hash of (seed, pass, iteration, vertex);
     * a round's vertices decide against the state at the start of the round
     * (with the min-label rule for singleton-to-singleton moves) and its moves
     * are applied together.  Bit-identical to the oracle's "sync" mode. */
    LOUVAIN_DETERMINISTIC = 0,
    /* Asynchronous (Section 4.1): the same rounds, but moves are applied as
     * soon as they are decided and later decisions read the live state. */
    LOUVAIN_FAST = 1,
    /* Colour-ordered synchronous rounds (the vertex-colouring alternative the
     * paper cites in Section 2): every level is coloured greedily in
     * decreasing order of a hashed priority of (seed, pass, vertex), the
     * colouring Jones and Plassmann's parallel algorithm computes, and each
     * iteration runs one round per colour class in ascending colour order.
     * No two neighbours share a round, so the singleton rule is off and
     * round_bits is ignored.  Bit-identical to the oracle's "colour" mode. */
    LOUVAIN_COLOURED = 2
};

/* Status codes. */
enum {
    LOUVAIN_OK = 0,
    LOUVAIN_EINVAL = -1,    /* bad argument or malformed graph */
    LOUVAIN_EOVERFLOW = -2, /* nnz > INT32_MAX or total weight >= 2^62 */
    LOUVAIN_ENOSPC = -3,    /* workspace smaller than louvain_workspace_size() */
    LOUVAIN_EHIP = -4,      /* a HIP runtime call failed */
    LOUVAIN_ESTATE = -5     /* call out of order (see louvain_move) */
};

#define LOUVAIN_MAX_PASSES 64
#define LOUVAIN_MAX_ITERATIONS 255

/*
 * Parameters.  Defaults (louvain_default_params) are the paper's choices of
 * Section 4.1: 20 iterations per pass, tolerance 0.01 divided by 10 after
 * every pass, aggregation tolerance 0.8, vertex pruning on.  The paper gives
 * no pass limit; the default is 10.
 */
typedef struct {
    int32_t mode;                 /* LOUVAIN_DETERMINISTIC, LOUVAIN_FAST or LOUVAIN_COLOURED */
    int32_t max_passes;           /* 0 .. LOUVAIN_MAX_PASSES */
    int32_t max_iterations;       /* 1 .. LOUVAIN_MAX_ITERATIONS */
    int32_t prune;                /* 1: vertex pruning (Section 4.1.6); 0: every vertex every iteration */
    double tolerance;             /* initial tau: stop an iteration loop when its delta-Q <= tau (Alg. 2) */
    double tolerance_drop;        /* tau /= tolerance_drop after each pass (Alg. 1 threshold scaling) */
    double aggregation_tolerance; /* stop when |communities| / |vertices| of the level > this (Alg. 1) */
    uint64_t seed;                /* key of the round hash and of the colouring priority */
    int32_t round_bits;           /* 0 .. 4: 2^round_bits rounds per iteration; -1 (default): the
                                     mode's own, 3 in LOUVAIN_FAST on one graph, else 1 */
    int32_t profile;              /* 1: time every kernel with HIP events (louvain_kernel_stats) */
    /* Scheduling knobs (results do not depend on them; deterministic modes stay
     * bit-exact): 0 keeps the built-in choice. */
    int32_t hub_rows;             /* rows longer than this take the hub path (bin 6); 2048 .. 8192,
                                     clamped to 4096 when accumulators are 8 bytes wide (default:
                                     8192, or 4096 when wide) */
    int32_t hub_part_pairs;       /* pairs per hash partition of a hub row in local moving;
                                     1024 .. 2048 (default 2048) */
    int32_t small_level;          /* a level (in a batch, a graph's part of it) of at most this
                                     many vertices is moved by one wavefront, all its iterations
                                     in one launch: LOUVAIN_FAST in vertex order (the
                                     asynchronous sweep of Alg. 2 as one thread runs it) instead
                                     of concurrently, LOUVAIN_DETERMINISTIC in the same
                                     synchronous rounds (same result); not LOUVAIN_COLOURED;
                                     1 .. 1024, -1 = never, 0 = the default: 1024 in
                                     LOUVAIN_FAST, never in LOUVAIN_DETERMINISTIC */
} louvain_params;

/* Per-pass record of the last louvain_run / louvain_move / louvain_aggregate sequence. */
typedef struct {
    int32_t passes;                             /* passes whose local-moving phase ran */
    int32_t iterations[LOUVAIN_MAX_PASSES];     /* l_i of each pass */
    int32_t vertices[LOUVAIN_MAX_PASSES];       /* |V'| of each level */
    int64_t entries[LOUVAIN_MAX_PASSES];        /* stored entries of each level */
    int32_t communities[LOUVAIN_MAX_PASSES];    /* distinct labels after local moving */
    double dq_last[LOUVAIN_MAX_PASSES];         /* delta-Q of the last iteration of each pass */
    int64_t moves[LOUVAIN_MAX_PASSES];          /* moves made in each pass */
    int64_t processed[LOUVAIN_MAX_PASSES];      /* vertex visits in each pass */
    int64_t scanned[LOUVAIN_MAX_PASSES];        /* row entries scanned by local moving in each pass */
    int32_t colours[LOUVAIN_MAX_PASSES];        /* colour classes of each level (LOUVAIN_COLOURED), else 0 */
    /* Time of each pass by phase (Section 5.3's split), summed HIP-event times of
     * its kernels; filled only with profile = 1 (else 0).  Moving: the
     * local-moving kernels with their compaction, round ends and tests;
     * aggregation: community counting, renumbering and lookup, the
     * community-vertex CSR and the super-vertex graph; other: level setup
     * (row sums, binning) and the final modularity (counted in the last pass). */
    double ms_move[LOUVAIN_MAX_PASSES];
    double ms_aggregate[LOUVAIN_MAX_PASSES];
    double ms_other[LOUVAIN_MAX_PASSES];
} louvain_stats;

/* Timing and algorithmic traffic of one kernel family (profile = 1). */
typedef struct {
    char name[40];
    int64_t launches;  /* launches that did work */
    double ms;         /* summed HIP-event time of those launches */
    double bytes;      /* algorithmic bytes those launches had to move */
} louvain_kernel_stat;

/* Fill *p with the defaults above. */
void louvain_default_params(louvain_params *p);

/*
 * Device bytes the caller must provide to louvain_init for a graph with n
 * vertices and nnz entries.  total_weight is the sum of all entry weights
 * if known (it selects 4-byte instead of 8-byte aggregated weights when
 * below 2^31), or -1 to size for the wide case.  Returns LOUVAIN_EINVAL or
 * LOUVAIN_EOVERFLOW for impossible sizes.
 */
int louvain_workspace_size(int32_t n, int64_t nnz, int64_t total_weight,
                           const louvain_params *p, size_t *bytes);

/*
 * Create a context for the graph (offsets, targets, weights), all device
 * pointers: offsets int32[n+1] with offsets[0] = 0, non-decreasing,
 * offsets[n] = nnz; targets int32[nnz] in [0, n); weights int32[nnz] >= 1,
 * symmetric (w_ij = w_ji; not checked).  One validation kernel checks the
 * rest and computes the total weight W.  workspace is a device buffer of
 * workspace_bytes; p may be NULL for defaults.  The context starts at pass
 * 0 with the input as the current level.
 * Errors: EINVAL (NULL pointers, n < 0, bad parameters, malformed CSR),
 * EOVERFLOW (nnz > INT32_MAX, W >= 2^62), ENOSPC, EHIP.
 */
int louvain_init(louvain_ctx **ctx, int32_t n, int64_t nnz, const int32_t *offsets,
                 const int32_t *targets, const int32_t *weights, void *workspace,
                 size_t workspace_bytes, const louvain_params *p, void *stream);

/*
 * Local-moving phase of the current pass (Alg. 2 called from Alg. 1): reset
 * K', Sigma', C' and the active flags for the current level, then iterate
 * until delta-Q <= tau or max_iterations.  Outputs (host, nullable): the
 * iterations run (l_i) and the last iteration's delta-Q.  Valid when the
 * context is at the start of a pass; otherwise ESTATE.
 */
int louvain_move(louvain_ctx *ctx, int32_t *iterations, double *delta_q);

/*
 * End of the current pass (Alg. 1 after louvainMove): count communities;
 * stop if l_i <= 1 or |communities|/|vertices| > aggregation_tolerance;
 * otherwise renumber communities by prefix sum, fold them into the top-level
 * membership (dendrogram lookup), build the super-vertex graph (Alg. 3) as
 * the next level and divide tau by tolerance_drop.  Outputs (host,
 * nullable): the number of communities and stop (1 when the pass loop must
 * end).  Valid after louvain_move; otherwise ESTATE.
 */
int louvain_aggregate(louvain_ctx *ctx, int32_t *communities, int32_t *stop);

/*
 * The whole method (Alg. 1) from the current state: passes of move and
 * aggregate until a stop or max_passes, then the final dendrogram lookup.
 * membership (device int32[n], caller-allocated) receives community ids
 * renumbered densely in label order; modularity (host) receives Q of that
 * membership on the input graph (Eq. 1); stats (host, nullable) the per-pass
 * record.  After it the context is finished: louvain_membership still works,
 * move/aggregate return ESTATE.
 */
int louvain_run(louvain_ctx *ctx, int32_t *membership, double *modularity,
                louvain_stats *stats);

/*
 * Top-level membership so far (device int32[n]), densely renumbered in label
 * order.  After louvain_move the current level's labels are folded in.
 */
int louvain_membership(louvain_ctx *ctx, int32_t *membership);

/*
 * Labels C' of the current level after local moving (device int32[n_level],
 * labels are vertex ids of the level, not renumbered).  ESTATE before the
 * first louvain_move of the pass.
 */
int louvain_level_labels(louvain_ctx *ctx, int32_t *labels);

/*
 * Read-only device views of the current level graph, for export and
 * checking: offsets int32[n_level+1]; degree int32[n_level] (NULL for the
 * input level, whose rows are dense) giving the used length of each row of
 * the holey CSR; targets int32; weights of weight_bytes (4 or 8) each.  Row
 * i is entries [offsets[i], offsets[i] + degree[i]).  Valid until the next
 * louvain_aggregate / louvain_run / louvain_destroy.
 */
int louvain_level_graph(louvain_ctx *ctx, const int32_t **offsets, const int32_t **degree,
                        const int32_t **targets, const void **weights, int32_t *n_level,
                        int32_t *weight_bytes);

/*
 * Per-iteration record of the last louvain_move (host arrays of at least
 * max entries, each nullable): the exact gain sum of every iteration split
 * in two's-complement words (sumN = hi * 2^64 + lo; the iteration's
 * delta-Q is 2*sumN/W^2), the moves and the vertex visits.  *count receives
 * the number of iterations recorded.
 */
int louvain_move_trace(louvain_ctx *ctx, int32_t max, int64_t *sumN_hi, uint64_t *sumN_lo,
                       int64_t *moves, int64_t *processed, int32_t *count);

/*
 * Rewind to pass 0 on the same input (singletons, initial tolerance)
 * without validating or touching the input again; the next louvain_move or
 * louvain_run starts afresh.
 */
int louvain_reset(louvain_ctx *ctx);

/* Total edge weight W = sum of all entry weights of the input (host). */
int louvain_total_weight(louvain_ctx *ctx, int64_t *W);

/* Per-pass record so far (host). */
int louvain_get_stats(louvain_ctx *ctx, louvain_stats *stats);

/* Kernel timings (profile = 1): up to max records into out (host), count in *count. */
int louvain_kernel_stats(louvain_ctx *ctx, louvain_kernel_stat *out, int32_t max,
                         int32_t *count);

/*
 * Warm start (the dynamic re-run the Conclusion names as future work: after edge
 * updates, start from the previous membership): the first pass's local
 * moving starts from the partition `labels` (device int32[n], each in [0, n),
 * and in a batch inside its own graph's range) instead of singletons, with
 * the community weights and sizes of that partition; the rest of the method
 * is unchanged.  The caller keeps `labels` valid until the first pass has
 * moved; NULL clears it, and louvain_reset forgets it.  Only before the first
 * louvain_move of a run.
 * Errors: EINVAL (NULL ctx, a label out of range), ESTATE (a pass has begun), EHIP.
 */
int louvain_set_membership(louvain_ctx *ctx, const int32_t *labels);

/*
 * Batches: several independent graphs run through one launch sequence as
 * the union of their CSRs (graph g owns the vertices [graph_offsets[g],
 * graph_offsets[g+1]) and only edges among them).  Every graph keeps its
 * own method: scores use its own W (Eq. 2), its own local-moving test
 * (Alg. 2: delta-Q <= tau) and its own pass-loop stops (Alg. 1: converged in
 * one sweep, or too few merges), and the deterministic rounds number its
 * vertices from 0, so each graph's membership is the one louvain_run gives
 * for that graph alone (bit for bit in deterministic mode).  The batch
 * stops when every graph has.
 */

/* Device bytes for a batch of `graphs` graphs with n vertices and nnz entries in total. */
int louvain_batch_workspace_size(int32_t graphs, int32_t n, int64_t nnz, int64_t total_weight,
                                 const louvain_params *p, size_t *bytes);

/*
 * As louvain_init for the union graph, plus graph_offsets: int32[graphs+1]
 * (device or host memory, read once), 0 = graph_offsets[0] <= ... <=
 * graph_offsets[graphs] = n; empty graphs are allowed.  Afterwards the
 * usual louvain_move / louvain_aggregate / louvain_run / louvain_reset
 * calls drive the whole batch.  louvain_run's membership holds dense ids
 * over the union, each graph's ids contiguous and in the order of its own
 * (subtract the smallest id in its range to get its own membership); its
 * modularity is that of the union graph.
 * Errors: those of louvain_init, and EINVAL for graphs < 1, malformed
 * graph_offsets or an entry that leaves its graph.
 */
int louvain_init_batch(louvain_ctx **ctx, int32_t graphs, const int32_t *graph_offsets,
                       int32_t n, int64_t nnz, const int32_t *offsets, const int32_t *targets,
                       const int32_t *weights, void *workspace, size_t workspace_bytes,
                       const louvain_params *p, void *stream);

/*
 * After louvain_run of a batch: per graph its modularity (Eq. 1 with its own
 * W; 0 for an edgeless graph) and its number of communities, into host
 * arrays of `graphs` entries (either may be NULL).
 * Errors: EINVAL (NULL ctx or not a batch), ESTATE (before louvain_run), EHIP.
 */
int louvain_batch_results(louvain_ctx *ctx, double *modularity, int32_t *communities);

/*
 * For callers that cannot allocate device memory (code that must not call
 * hipMalloc, such as tight serving loops or harnesses that forbid it):
 * louvain_init + louvain_run + louvain_destroy in one call, with the
 * library's own device scratch array as the workspace instead of a
 * caller-provided one.  The array is a file-scope device array of
 * LOUVAIN_NOALLOC_BYTES (64 MiB) that every GPU the library runs on holds
 * until the process ends; nothing is allocated on the device or in pinned
 * host memory, and no events are created (the host waits on the stream
 * once per local-moving iteration instead of one iteration behind).
 * Host-side bookkeeping still uses the C++ heap.
 * Arguments: as louvain_init (offsets, targets, weights: device; p may be
 * NULL; stream as there) and louvain_run (membership: device int32[n];
 * modularity: host; stats: host, nullable); the result is the one
 * louvain_init + louvain_run give on the same input and parameters.
 * Graphs up to roughly 1.7e6 entries fit: the need is
 * louvain_workspace_size(n, nnz, -1, p) (sized for 8-byte totals).
 * Errors: ENOSPC when that need exceeds LOUVAIN_NOALLOC_BYTES; EINVAL for
 * p->profile = 1 (profiling creates events) and the errors of
 * louvain_init / louvain_run.
 * Every call on one GPU shares that GPU's array, which keeps the last call's
 * contents (each call initialises what it reads): calls that overlap on the
 * same GPU, from several threads or streams, race and must be serialised by
 * the caller.
 */
#define LOUVAIN_NOALLOC_BYTES (64ull << 20)
int louvain_run_noalloc(int32_t n, int64_t nnz, const int32_t *offsets, const int32_t *targets,
                        const int32_t *weights, const louvain_params *p, int32_t *membership,
                        double *modularity, louvain_stats *stats, void *stream);

/* Release host-side state (the caller's device buffers are untouched). NULL is a no-op.
 * The context's pinned host block (a few KB for scalar read-backs) returns to a
 * process-wide pool that later contexts reuse; pinned memory is never freed
 * before the process ends, because freeing it would wait for the whole device. */
void louvain_destroy(louvain_ctx *ctx);

/* Static description of a status code (for EHIP, of the last HIP error seen by the calling thread). */
const char *louvain_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* LOUVAIN_H */
