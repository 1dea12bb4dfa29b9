// Launchers of the gfx950 Louvain kernels (internal to the library).
#pragma once

#include "common.h"

namespace lv {

// Bin boundaries of one level: bin b holds binorder[start[b] .. start[b+1]).
struct BinInfo {
    int32_t start[NBINS + 1];
};

// ----------------------------------------------------------------- scans
// Exclusive prefix sum of in[0..n) into out[0..n], out[n] = total; the total
// is also stored in *total (device).  Scratch needs scan_scratch_elems(n)
// int64 elements.
int64_t scan_scratch_elems(int64_t n);
template <typename TI, typename TO>
void launch_exclusive_scan(const TI *in, TO *out, int64_t n, int64_t *scratch,
                           unsigned long long *total, hipStream_t s);

// ----------------------------------------------------------------- fills / setup
void launch_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s);
void launch_fill_u8(uint8_t *p, uint8_t v, int64_t n, hipStream_t s);
void launch_fill_bytes_zero(void *p, int64_t bytes, hipStream_t s);
void launch_iota(int32_t *p, int64_t n, hipStream_t s);

// Validation of the input CSR; sets bits of *err, adds weights into *W and
// raises *wmax to the largest weight (both start at zero).
void launch_validate(int32_t n, int64_t nnz, const int32_t *off, const int32_t *tgt,
                     const int32_t *w, int32_t *err, unsigned long long *W, int32_t *wmax,
                     hipStream_t s);

// *out = max(*out, max of x[0..n)) for non-negative x.
void launch_max_u64(const int64_t *x, int32_t n, unsigned long long *out, hipStream_t s);

// Per-level reset: C' = iota, size = 1, flagsA = 1, flagsB = 0, K = Sigma = 0.
void launch_init_vertices(int32_t n, int32_t *Cp, int32_t *size, uint8_t *fa, uint8_t *fb,
                          void *K, void *Sig, int sbytes, hipStream_t s);

// Degree binning as a stable counting sort over chunks of BIN_CHUNK rows.
// Row length: deg[v] if deg, else off[v+1]-off[v].  launch_bin_count writes
// per-chunk bin counts (cnt, NBINS * bin_chunks(n)), their exclusive scan
// (boff, one more element) and the bin boundaries starts[0..NBINS] (device);
// launch_bin_fill then writes binorder.
// lds_max is the LDS row limit L of the bins; maxlen[0..NBINS) receives the
// longest row of every bin.
int32_t bin_chunks(int32_t n);
void launch_bin_count(int32_t n, const int32_t *off, const int32_t *deg, int32_t lds_max,
                      int32_t *cnt, int32_t *boff, int64_t *scratch, int32_t *starts,
                      int32_t *maxlen, hipStream_t s);
void launch_bin_fill(int32_t n, const int32_t *off, const int32_t *deg, int32_t lds_max,
                     const int32_t *boff, int32_t *binorder, hipStream_t s);
// Hub bin rows binorder[hb .. he) (row lengths from off/deg, or from deg alone
// when off is null): length (ent), sorting slices of `slice` entries (slices)
// and hash partitions of about per_part entries each (parts; 0 = the LDS
// partition size for table values of stbytes bytes), at most HUB_MAXP.
void launch_hub_move_sizes(const int32_t *binorder, int32_t hb, int32_t he, const int32_t *off,
                           const int32_t *deg, int stbytes, int64_t *ent, int32_t *slices,
                           int32_t *parts, hipStream_t s, int slice = HUB_PSLICE,
                           int per_part = 0);

// The sorting slices and partitions of the queued hubs (act != 0) of a round, in hub
// order: counts per hub (cs, cp), their exclusive scans (os, op; totals in *ns, *np)
// and the lists (ls, lp).  start_s / start_p: first slice / partition per hub, totals
// *total_s / *total_p (device).
void launch_hub_active_lists(const uint8_t *act, const int32_t *start_s, const int32_t *start_p,
                             int32_t hubs, const unsigned long long *total_s,
                             const unsigned long long *total_p, int32_t *cs, int32_t *cp,
                             int32_t *os, int32_t *op, unsigned long long *ns,
                             unsigned long long *np, int32_t *ls, int32_t *lp, int64_t *scratch,
                             hipStream_t s);

// owner[k] = h for every k in [start[h], start[h + 1]) (the last range ends at
// total): the hub, or hub community, of each sorting slice or partition, so the
// sorting kernels read it instead of searching start[].
void launch_owner_map(const int32_t *start, int32_t n, int32_t total, int32_t *owner, hipStream_t s);

// mdeg[m] = row length of members[m].
void launch_member_degrees(int32_t n, const int32_t *members, const int32_t *off,
                           const int32_t *deg, int32_t *mdeg, hipStream_t s);

// Row reductions over the rows of one bin.
//   op 0: K[v] = Sigma[v] = sum of row weights
//   op 1: *sigma += sum of row weights whose target has the same label
template <class C>
struct RowArgs {
    const int32_t *off, *deg, *tgt;
    const typename C::WT *w;
    const int32_t *binorder;
    int32_t begin, count;
    typename C::ST *K, *Sig;
    const int32_t *labels;
    unsigned long long *sigma;
    // hub bin: exclusive prefix of HUB_PSLICE-entry slices per row and its total
    // (device); null runs one workgroup per hub row
    const int32_t *hslice;
    const unsigned long long *nslices;
};
template <class C>
void launch_row_reduce(int bin, int op, const RowArgs<C> &a, hipStream_t s);

// Sum of Sigma_c^2 (128-bit) over c < n into acc[2].
template <typename ST>
void launch_sum_squares(const ST *Sig, int32_t n, unsigned long long *acc, hipStream_t s);

// ----------------------------------------------------------------- local moving
// ----------------------------------------------------------------- colouring
// Jones and Plassmann's colouring with readiness counters.  While v is
// uncoloured, colour[v] = -(1 + its uncoloured higher-priority neighbours);
// a vertex whose count reaches zero joins the next frontier, and a frontier
// vertex takes the smallest colour none of its (all coloured) higher-priority
// neighbours holds, then counts itself off its lower-priority neighbours.
// Rows fall in five degree classes (bins 0, 1, 2, 3 and 4-6) worked by 1, 4,
// 16 and 64 lanes per vertex and, for class 4, by chunks of 1024 entries
// spread over blocks (initialisation: a block per row); one launch covers all classes, blocks
// [rblk[q], rblk[q + 1]) taking class q.  A frontier list holds class q at
// [cstart[q], cstart[q + 1]).
constexpr int NCLS = 5;
constexpr int COLOUR_CT = 1024;  // threads per colouring block
struct ColourArgs {
    const int32_t *off, *deg, *tgt;
    const int32_t *binorder;
    int32_t cstart[NCLS + 1];  // class regions (also the classes' binorder ranges)
    int32_t rblk[NCLS + 1];    // first block of each class; rblk[NCLS] = grid
    const int32_t *in;         // frontier of this step (vertex ids)
    const int32_t *in_count;   // per class
    int32_t *out;              // next frontier
    int32_t *out_count;        // per class (zero on entry)
    int32_t *clear_count;      // per class: zeroed for the step after next
    int32_t *colour;
    int32_t *ncol;             // raised to max colour + 1
    int32_t *coloured;         // vertices coloured (summed per block)
    uint32_t *cbm;             // class 4: per frontier slot a 1024-colour bitmap and a chunk
                               // counter (33 words, zero between steps)
    uint64_t seed;
    int32_t pass;
    BatchArgs bt;              // batches: priorities by index within the graph
};
// Lanes per vertex of class q.
constexpr int colour_lanes(int q) { return q == 0 ? 1 : (q == 1 ? 4 : (q == 2 ? 16 : (q == 3 ? 64 : 1024))); }
// Initialisation over every binned row (binorder positions), then one step.
void launch_colour_init(const ColourArgs &a, hipStream_t s);
void launch_colour_step(const ColourArgs &a, hipStream_t s);

// Positions binorder[0, nb) sorted by (colour, bin) into order[0, nb): key
// k = colour * NBINS + bin, koff = exclusive scan of the key counts
// (kcount, nkeys + 1 entries; the scan's total in koff[nkeys]), kcur a copy
// of koff used as fill cursors.  Order within a key is arbitrary.
void launch_class_count(const int32_t *binorder, int32_t nb, BinInfo bins, const int32_t *colour,
                        int32_t nkeys, int32_t *kcount, hipStream_t s);
// dst[i] = src[idx[i]] for i < n.
void launch_gather_i32(const int32_t *src, const int32_t *idx, int32_t n, int32_t *dst, hipStream_t s);
void launch_class_fill(const int32_t *binorder, int32_t nb, BinInfo bins, const int32_t *colour,
                       int32_t nkeys, int32_t *kcur, int32_t *order, hipStream_t s);

struct CompactArgs {
    const int32_t *binorder;
    int32_t nb;  // rows in bins (binorder[0..nb))
    BinInfo bins;
    uint8_t *flags;  // active flags of this iteration (cleared as they are taken)
    int32_t prune;
    int32_t round, round_bits, pass, it;
    uint64_t seed;
    const int32_t *order;   // if set: visit the positions order[q0, q1) (one colour class)
                            // instead of 0 .. nb - 1
    int32_t q0, q1;
    int32_t *worklist;  // per bin at bins.start[b]: vertex ids (bins 0-4), binorder positions (hubs)
    int32_t *counts;    // per-bin count of this round (zero on entry)
    uint8_t *hub_act;   // per hub (position - bins.start[NBINS-1]): queued this round
    const int32_t *done;
    BatchArgs bt;       // batches: skip graphs that converged or stopped; rounds by local index
    int32_t hubs_only;  // take only hub rows (the other rows were taken by launch_compact_keys)
};
void launch_compact(const CompactArgs &a, hipStream_t s);

// Colour-ordered mode: the rows of every round at once, hub rows excepted.  Position
// i of a.order (keys sorted (colour, bin); key k owns [koff[k], koff[k + 1])) goes,
// when active, to klist[koff[k] + rank] with rank from kact[k] (zero on entry); the
// order within a key is free.  Adds the rows taken to *processed.
void launch_compact_keys(const CompactArgs &a, const int32_t *koff, int32_t nkeys, int32_t *kact,
                         int32_t *klist, unsigned long long *processed, hipStream_t s);

// Best candidate of one partition of a hub row.
template <class C>
struct HubPart {
    typename C::SC best;
    typename C::ST hd;   // weight to the own community, if its key is in the partition
    int32_t bc;
    int32_t nk;          // distinct communities in the partition
};

template <class C>
struct MoveArgs {
    const int32_t *off, *deg, *tgt;
    const typename C::WT *w;
    const int32_t *binorder, *worklist;
    int32_t list_begin;
    const int32_t *count;
    int32_t *Cp;
    const typename C::ST *K;
    typename C::ST *Sig;
    int32_t *size;
    uint8_t *flags_next;
    int32_t *mv_c;                      // deferred moves: new label per vertex, -1 if none
    // hub bin: row entries are counting-sorted into partitions by community
    int32_t *hstage;                   // community of each hub entry (-1 between rounds)
    const int64_t *hoff;               // first staged entry per hub (scan of row lengths)
    const int32_t *hslice;             // first sorting slice per hub (HUB_PSLICE entries)
    const int32_t *htslice;            // first partition per hub
    const int32_t *sown, *pown;        // hub of each sorting slice / of each partition
    int32_t *act_s, *act_p;            // sorting slices / partitions of the round's queued hubs
    unsigned long long *n_act_s, *n_act_p;  // their counts
    int32_t *act_tmp;                  // 4 * (hubs) ints: per-hub counts and offsets of the lists
    const unsigned long long *hslices; // total sorting slices of the level
    const unsigned long long *htslices;  // total partitions
    int32_t slice_base, part_base;     // first sorting slice and partition of this launch's hubs
    int32_t *pcount, *pcur, *poff;     // pairs per partition, fill cursors, offsets
    int32_t *pk;                       // partitioned pairs (community, weight)
    typename C::ST *pw;
    void *hpart;                       // HubPart<C> per partition
    uint8_t *hub_act;                  // hub queued in this round (2 once it has moved)
    typename C::ST *hub_hd;            // per hub: weight of its row into its own community
    int32_t nhubs;
    unsigned long long *spread;        // NSPREAD counter rows of SPREAD_W words
    int32_t bin;                       // degree bin of this launch (counter columns)
    const int32_t *done;
    int64_t W;
    int32_t rule;                      // min-label rule for singleton moves
    BatchArgs bt;                      // batches: per-graph W and gain sums
};
// Bins 0-4; grid: workgroups to launch for this bin (each loops over the device count);
// log2s_max: LDS table size of bin 4 (block_log2s of the bin's longest row).
template <class C>
void launch_move(int bin, bool fast, const MoveArgs<C> &a, int grid, int log2s_max,
                 hipStream_t s);
int move_rows_per_block(int bin);
// Hub bin: the queued hubs' rows are counted and sorted into partitions
// (workgroups over all hubs' sorting slices; inactive hubs exit), one
// workgroup per partition finds its best candidate, then one workgroup per
// queued hub takes the argmax over its partitions and moves.
template <class C>
void launch_move_hubs(bool fast, const MoveArgs<C> &a, int32_t sort_slices, int32_t parts,
                      int grid, int64_t *scratch, hipStream_t s);

// Small levels: one wavefront per graph (one in total for a single graph)
// runs the whole local-moving phase of a level of at most max_n vertices, in
// vertex order (fast mode: Alg. 2 as one thread executes it) or in the
// synchronous rounds of the degree bins (deterministic mode), then marks the
// graph converged for the pass; larger graphs are left to the degree bins.
template <class C>
struct SeqArgs {
    const int32_t *off, *deg, *tgt;
    const typename C::WT *w;
    int32_t *Cp;
    const typename C::ST *K;
    typename C::ST *Sig;
    int32_t *size;
    uint8_t *act;        // active flags of the level
    uint8_t *mark;       // deterministic mode: rows of this iteration's movers
    int32_t n;           // vertices of the level (a single graph)
    int32_t max_n;       // largest graph moved here (at most SEQ_MAX)
    int64_t W;           // total weight (a single graph; a batch uses bt.gW)
    double tau;
    int32_t max_iter, prune;
    int32_t rule;        // deterministic mode: min-label rule for singleton moves
    uint64_t seed;       // deterministic mode: round hash of (seed, pass, iteration, vertex)
    int32_t round_bits, pass;
    DevScalars *sc;      // a single graph: per-iteration trace, iterations, done
    BatchArgs bt;
};
// grid: graphs (1 for a single graph).
template <class C>
void launch_seq_level(const SeqArgs<C> &a, bool fast, int graphs, hipStream_t s);

// Deferred moves of a round (deterministic mode): every vertex v < n with
// mv_c[v] >= 0 relabelled to mv_c[v] (mv_c[v] reset to -1), the community
// weights and sizes updated, each workgroup combining the updates of
// APPLY_CHUNK vertices per community in LDS before one HBM atomic per community.
template <typename ST>
void launch_apply(int32_t *mv_c, int32_t n, int32_t *Cp, const ST *K, ST *Sig, int32_t *size,
                  const int32_t *done, hipStream_t s);

// End of a round: processed += counts, counts = 0.
void launch_round_end(DevScalars *sc, int it, hipStream_t s);
// End of an iteration: folds the per-wavefront counter rows into the
// iteration's gain sum, moves, scanned entries and the work counters, clears
// them, then the delta-Q test against tau and the done / iters update.
void launch_iter_end(DevScalars *sc, int it, double tau, hipStream_t s,
                     const BatchArgs *b = nullptr);

// ----------------------------------------------------------------- warm start
// err bit 4 for a label outside [0, n) (or outside its graph's range when gid is non-null).
void launch_warm_check(int32_t n, const int32_t *labels, const int32_t *gid, const int32_t *gvb,
                       int32_t *err, hipStream_t s);
// C' = labels, Sigma' and sizes of that partition (Sig and size zero on entry).
template <typename ST>
void launch_warm_labels(int32_t n, const int32_t *labels, const ST *K, int32_t *Cp, ST *Sig,
                        int32_t *size, hipStream_t s);

// ----------------------------------------------------------------- batches
// gid[v] for a level whose graph g owns vertices [gvb[g], gvb[g+1]).
void launch_batch_gid(int32_t n, const int32_t *gvb, int32_t G, int32_t *gid, hipStream_t s);
// Input check (err bit 3: an entry leaves its graph) and per-graph W (zero on entry).
void launch_batch_check(int32_t n, const int32_t *off, const int32_t *tgt, const int32_t *w,
                        const int32_t *gid, const int32_t *gvb, int64_t *gW, int32_t *err,
                        hipStream_t s);
// Start of a run: all graphs alive, gcomm[g] = vertices of graph g.
void launch_batch_reset(const BatchArgs &b, int32_t *gcomm, hipStream_t s);
// Start of a local-moving phase: converged bits, iteration counts and gain sums cleared.
void launch_batch_pass_begin(const BatchArgs &b, hipStream_t s);
// Marks the graphs of at most max_n vertices (not stopped) for the small-level
// kernels of this pass (gst bit 2), which the degree bins then skip.
void launch_batch_mark_small(const BatchArgs &b, int32_t max_n, hipStream_t s);
// Per-graph community bases (gvb_next), counts (gcomm) and stop test; sc->alive (zero on
// entry) counts the graphs that go on.
void launch_batch_agg_test(const BatchArgs &b, const int32_t *idmap, int32_t n, int32_t nc,
                           double aggtol, int32_t *gvb_next, int32_t *gcomm, DevScalars *sc,
                           hipStream_t s);
// gid of the next level from the dense labels.
void launch_batch_gid_next(int32_t n, const int32_t *labels, const int32_t *gid, int32_t *gid_next,
                           hipStream_t s);
// Per-graph sigma and S2 (both zero on entry) of a level with labels.
template <typename WT, typename ST>
void launch_batch_modularity(int32_t n, const int32_t *off, const int32_t *deg, const int32_t *tgt,
                             const WT *w, const int32_t *labels, const ST *Sig, const int32_t *gid,
                             unsigned long long *gsig, unsigned long long *gs2, hipStream_t s);

// ----------------------------------------------------------------- aggregation
void launch_mark_used(int32_t n, const int32_t *labels, int32_t *used, hipStream_t s);
void launch_relabel(int32_t n, int32_t *labels, const int32_t *map, hipStream_t s);
void launch_comm_count(int32_t n, const int32_t *Cp, const int32_t *off, const int32_t *deg,
                       int32_t *ccount, int32_t *ctot, hipStream_t s);
void launch_comm_fill(int32_t n, const int32_t *Cp, const int32_t *coff, int32_t *cursor,
                      int32_t *members, hipStream_t s);

template <class C>
struct AggArgs {
    const int32_t *off, *deg, *tgt;   // level G'
    const typename C::WT *w;
    const int32_t *Cp;                // dense labels of G'
    const int32_t *coff, *members;    // community-vertex CSR
    const int32_t *cbinorder;         // communities grouped by bin
    int32_t begin, count;             // this bin's segment of cbinorder
    const int32_t *yoff;              // holey offsets of G''
    int32_t *ydeg;                    // used length of each row of G''
    int32_t *ytgt;
    typename C::ST *yw;
    // hub bin: flattened member rows counting-sorted into partitions by community
    const int32_t *mpre;              // exclusive scan of member row lengths
    const int32_t *cslice, *tslice;   // first sorting slice / partition per community
    int32_t *sown, *pown;             // community (in the bin) of each window / partition
    int32_t *wm0;                     // first member whose row reaches into each window
    const unsigned long long *tslices;  // total partitions
    int32_t *hstage;                  // distinct pairs of each window (at its flattened offset)
    typename C::ST *hstage_w;
    int32_t *wcnt;                    // pairs staged per window
    int32_t *pcount, *pcur, *poff;    // pairs per partition, fill cursors, offsets
    int32_t *pk;                      // partitioned pairs (community, weight)
    typename C::ST *pw;
    int32_t ncomm;                    // |Gamma|
    unsigned long long *work;         // [communities, members, entries, emitted]
};
// Bins 0-4 (LDS tables); the hub bin goes through launch_aggregate_hub.
// log2s_max: LDS table size of bin 4.
template <class C>
void launch_aggregate(int bin, const AggArgs<C> &a, int log2s_max, hipStream_t s);
// Hub bin: one workgroup per AGG_PSLICE flattened entries of a community's
// member rows folds and stages them and then sorts them into partitions; one
// workgroup per partition folds it and appends its keys to the community's row.
// wmax: the largest weight of the level when known (input weights), else 0; it
// lets the first fold use 32-bit sums.
template <class C>
void launch_aggregate_hub(const AggArgs<C> &a, int32_t sort_slices, int32_t parts,
                          int64_t wmax, int64_t *scratch, hipStream_t s);

}  // namespace lv
