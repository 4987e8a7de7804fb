/*
 * famsa_lcs.h -- all-pairs LCS similarity stage of FAMSA on gfx950 (MI355X).
 *
 * FAMSA (Deorowicz, Debudaj-Grabysz, Gudys; arXiv 1603.06958) measures the
 * similarity of every pair of sequences in a family by the length of a
 * longest common subsequence, computed bit-parallel (Methods, "Pairwise
 * similarities calculation"), and feeds the similarities, as they are
 * produced, into a single-linkage guide-tree builder that keeps O(k) memory
 * (Methods, "Determination of the guide tree").  This library computes the
 * exact int32 LCS length of every pair i < j inside each family on one GPU
 * and hands the results to the caller as row tiles, so the k x k matrix is
 * never stored.  Around that core: tiles of indel distances or similarities
 * instead of LCS values; two single-linkage consumers (SLINK on the host, an
 * exact maximum spanning forest on the GPU) and the guide tree they give;
 * the gapped sequence representation the progressive stage builds profiles
 * with; and a continuous-batching server for many families.
 *
 * Conventions for every call:
 *  - Functions return 0 (FAMSA_LCS_OK) or a negative famsa_lcs_status; the
 *    text of the last error on the calling thread is famsa_lcs_last_error().
 *    Nothing is reported through errno or exceptions.
 *  - Argument validation happens before any HIP call, so invalid input is
 *    rejected with FAMSA_LCS_EINVAL even on a machine without a GPU.
 *  - Host pointers are read during the call only; the library copies what it
 *    keeps.  Device and pinned memory the library allocates belongs to the
 *    object that allocated it and is freed by its release/destroy call.
 *  - Sequence i of a batch is codes[seq_off[i] .. seq_off[i+1]); codes are
 *    symbol indices in [0, alphabet_size).  The paper's alphabet has 32
 *    codes (twenty amino acids plus special symbols; Methods, "Progressive
 *    construction of the alignment"); two codes match only when equal.
 *  - Lengths are limited to FAMSA_LCS_MAX_LEN residues; empty sequences are
 *    allowed and have LCS 0 with everything.
 */
#ifndef FAMSA_LCS_H
#define FAMSA_LCS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FAMSA_LCS_ABI_VERSION 1
#define FAMSA_LCS_MAX_LEN 65535u
#define FAMSA_LCS_MAX_ALPHABET 32u

typedef enum famsa_lcs_status {
  FAMSA_LCS_OK = 0,
  FAMSA_LCS_EINVAL = -1,     /* bad argument; nothing was done */
  FAMSA_LCS_ENOMEM = -2,     /* host, pinned or device allocation failed, or the HBM budget is too small */
  FAMSA_LCS_EDEVICE = -3,    /* a HIP call failed (no GPU, fault, ...) */
  FAMSA_LCS_ECANCELED = -4,  /* a tile callback returned nonzero */
  FAMSA_LCS_EBUSY = -5       /* object already in use on this or another thread */
} famsa_lcs_status;

/* Option flags. */
#define FAMSA_LCS_PLAIN        0x1u  /* baseline: one pair per lane, 64-bit words, masks from global memory,
                                        one launch per tile, no work queue, no autotune, no graph */
#define FAMSA_LCS_DESCENDING   0x2u  /* deliver each family's row tiles from the last to the first */
#define FAMSA_LCS_DEVICE_TILES 0x4u  /* deliver device pointers (no copy to host); valid during the callback,
                                        whose GPU work must be ordered on famsa_lcs_tile.stream */
#define FAMSA_LCS_NO_GRAPH     0x8u  /* launch kernels directly (timed per kernel class) instead of replaying
                                        one captured hipGraph per launch step */
#define FAMSA_LCS_NO_AUTOTUNE  0x10u /* use the built-in launch parameters; ignore the tuning cache */
#define FAMSA_LCS_ONE_STREAM   0x20u /* run every launch step on one compute stream: the default; the flag is
                                        accepted and changes nothing (excludes FAMSA_LCS_TWO_STREAMS) */
#define FAMSA_LCS_OUT_INDEL    0x40u /* tiles hold indel = |A| + |B| - 2 LCS (int32) instead of LCS */
#define FAMSA_LCS_OUT_SIM      0x80u /* tiles hold the similarity LCS / indel^2 as float32 (the float rounding
                                        of the correctly rounded double; +infinity when indel = 0) instead of
                                        LCS (Methods, "Pairwise similarities calculation"); excludes OUT_INDEL */
#define FAMSA_LCS_PLAIN_ASYNC  0x100u /* with FAMSA_LCS_PLAIN only: two output buffers on one compute stream, and
                                         each tile's launch is issued without waiting for the previous tile's
                                         delivery (the plain kernels with no host synchronisation between them) */
#define FAMSA_LCS_TWO_STREAMS  0x200u /* alternate consecutive launch steps between two compute streams, so a
                                         step's tail overlaps the next step's head (on a single family of
                                         k = 100,000 this is 3% slower with graphs and equal without) */
#define FAMSA_LCS_LONG_SEGMENTED 0x400u /* rows longer than one lane holds (896 residues; 512 for alphabets over
                                           20) go to the segmented long-row kernel only, not to the
                                           lanes-per-row mode (several lanes per row, carries passed across
                                           lanes); results are the same */

/* What a tile's values are (famsa_lcs_tile.values). */
#define FAMSA_LCS_VALUES_LCS   0u
#define FAMSA_LCS_VALUES_INDEL 1u
#define FAMSA_LCS_VALUES_SIM   2u

typedef struct famsa_lcs_options {
  uint32_t struct_size;    /* sizeof(famsa_lcs_options) as the caller compiled it */
  uint32_t alphabet_size;  /* 1..32; every code must be below it (default 20) */
  uint32_t tile_rows;      /* rows per tile, >= 1 (default 1024) */
  int32_t device;          /* HIP device ordinal (default 0) */
  void* stream;            /* hipStream_t the caller orders its own work on, or NULL (library stream) */
  uint64_t hbm_budget;     /* device bytes the plan may hold; 0 = 90% of free memory at plan time */
  uint32_t flags;          /* FAMSA_LCS_* flags above */
  uint32_t cols_per_item;  /* columns per work item, 0 = tuned/default */
  uint64_t step_values;    /* int32 values per launch step (several tiles), 0 = default (2^27) */
  uint64_t step_cells;     /* server only: cells |A||B| per scheduler step, which bounds how long a
                              step runs and so how long a new job waits; the server's tiles then
                              also hold at most this many cells (fewer than tile_rows rows for
                              jobs of long rows, at least one row), and a step still takes at
                              least one tile; 0 = no bound (plans ignore it) */
} famsa_lcs_options;

/* Fill *opt with the defaults above. */
void famsa_lcs_default_options(famsa_lcs_options* opt);

/* Opaque handles, owned by the library.  (The call that makes a plan is
 * famsa_lcs_plan, so the type carries a _t suffix.) */
typedef struct famsa_lcs_plan_s famsa_lcs_plan_t;

/*
 * Validate the batch, copy it to the device, build the per-symbol match
 * bit masks and the work lists, allocate tile buffers, and return a plan.
 * The quantity a plan computes is the one the first stage of the method
 * defines (Methods, "Pairwise similarities calculation"): the length of a
 * longest common subsequence of every pair of sequences of a family, found
 * bit-parallel, w DP cells per machine word.
 *   codes      nseq sequences back to back (may be NULL if all are empty)
 *   seq_off    nseq + 1 non-decreasing offsets into codes
 *   fam_off    nfam + 1 non-decreasing offsets into the sequence list with
 *              fam_off[0] = 0 and fam_off[nfam] = nseq; NULL means one
 *              family of all nseq sequences (then nfam is ignored)
 *   opt        options, or NULL for the defaults
 *   out        receives the plan; set to NULL on failure
 * Errors: EINVAL (bad offsets, code >= alphabet_size, length over
 * FAMSA_LCS_MAX_LEN, bad options), ENOMEM (budget or allocation), EDEVICE.
 */
int famsa_lcs_plan(const uint8_t* codes, const uint64_t* seq_off, uint32_t nseq,
                    const uint32_t* fam_off, uint32_t nfam, const famsa_lcs_options* opt,
                    famsa_lcs_plan_t** out);

/* One row tile: rows [row_begin, row_end) of family `family`; row i holds
 * LCS(i, j) for j = i+1 .. k-1 (family-local indices, the caller's order),
 * rows back to back, `count` int32 values in total. */
typedef struct famsa_lcs_tile {
  uint64_t tile_index;   /* position in the plan's delivery order (resume point) */
  uint32_t family;       /* family id (serving: job id) */
  uint32_t k;            /* family size */
  uint32_t row_begin, row_end;
  const int32_t* lcs;    /* host memory, or device memory under FAMSA_LCS_DEVICE_TILES; int32 LCS values,
                            or indel / float32 similarity bits as `values` says */
  uint64_t count;
  void* stream;          /* hipStream_t the tile was produced on */
  uint32_t values;       /* FAMSA_LCS_VALUES_*: LCS unless the plan asked for OUT_INDEL or OUT_SIM */
} famsa_lcs_tile;

/* Tile consumer; return 0 to continue, nonzero to cancel. */
typedef int (*famsa_lcs_tile_fn)(void* user, const famsa_lcs_tile* tile);

/*
 * Compute and deliver every tile with index >= first_tile, in order, calling
 * fn(user, tile) on the calling thread.  Tiles are streamed so a consumer
 * can build the single-linkage guide tree as the similarities arrive,
 * without the k x k matrix (Methods, "Determination of the guide tree":
 * the first two stages run together in O(k) memory).  The tile memory is valid only during
 * the callback.  While a callback runs, the next tiles are being computed.
 * Errors: EINVAL (NULL plan/fn, first_tile > tile count), EBUSY (plan in
 * use, e.g. called from inside its own callback), ECANCELED, EDEVICE.
 * After any error the plan is still valid and can be run again.
 */
int famsa_lcs_tiles(famsa_lcs_plan_t* plan, uint64_t first_tile, famsa_lcs_tile_fn fn, void* user);

/* Free everything the plan holds (its device batch, masks, work lists and
 * tile buffers: the memory of the first stage of the method, Methods,
 * "Determination of the guide tree").  NULL is a no-op. */
void famsa_lcs_release(famsa_lcs_plan_t* plan);

/* Thread-local text of the last error ("" if none). */
const char* famsa_lcs_last_error(void);

typedef struct famsa_lcs_plan_info {
  uint64_t ntiles;         /* tiles delivered by a full famsa_lcs_tiles call */
  uint64_t nsteps;         /* launch steps (each one kernel launch per length class) */
  uint64_t pairs;          /* sum over families of k(k-1)/2 */
  uint64_t cells;          /* sum over pairs of |A||B| */
  uint64_t device_bytes;   /* device memory the plan holds */
  uint64_t pinned_bytes;   /* pinned host memory the plan holds */
  uint64_t max_tile_values;
  uint32_t nfam, max_len;
  uint32_t cols_per_item;  /* launch parameters in force */
  uint32_t waves_per_group[4];
} famsa_lcs_plan_info;

int famsa_lcs_plan_get_info(const famsa_lcs_plan_t* plan, famsa_lcs_plan_info* info);

/* Dry run: the same validation and host-side planning as famsa_lcs_plan
 * (tiles, launch steps, per-step work lists for the kernels) with no HIP
 * call at all, for inspecting a decomposition on any machine.  Device
 * fields of *info (device_bytes, pinned_bytes, waves) are 0.  If dump_path
 * is not NULL the work lists are written there (binary: the magic
 * "FLCSDMP1", then for each array a uint64 count, a uint64 element size and
 * the elements: tiles, steps, step ranges, groups, lanes, items, plain rows,
 * column map, row bases, sequence lengths, family offsets).
 * Errors: EINVAL as for famsa_lcs_plan, or when the file cannot be written. */
int famsa_lcs_plan_dry_run(const uint8_t* codes, const uint64_t* seq_off, uint32_t nseq, const uint32_t* fam_off,
                           uint32_t nfam, const famsa_lcs_options* opt, const char* dump_path,
                           famsa_lcs_plan_info* info);

/* Timing of the last famsa_lcs_tiles call, from HIP events on the compute
 * streams.  Per-kernel times are recorded only for plans that launch without
 * a graph (FAMSA_LCS_NO_GRAPH or FAMSA_LCS_PLAIN); step_ms is always there. */
typedef struct famsa_lcs_stats {
  double kernel_ms[5];     /* summed duration per kernel: [0] rows of <= 256 residues, [1] <= 384, [2] <= 896
                              (<= 512 with more than 20 symbols), [3] longer rows, in segments,
                              [4] plain one-pair-per-lane baseline (FAMSA_LCS_PLAIN) */
  uint64_t launches[5];
  uint64_t cells[5];       /* algorithmic cells |A||B| assigned to each kernel over the whole plan */
  double step_ms;          /* summed device time of the launch steps (all kernels of a step) */
  uint64_t steps;
  double wall_ms;          /* first launch to last callback return */
  uint64_t tiles;
} famsa_lcs_stats;

int famsa_lcs_get_stats(const famsa_lcs_plan_t* plan, famsa_lcs_stats* stats);

/* ------------------------------------------------------------------------
 * Single-linkage consumer (Methods, "Determination of the guide tree": the
 * tree is built incrementally by SLINK in O(k^2) time and O(k) memory, fed
 * while the similarities are produced).  Similarity is LCS / indel^2 with
 * indel = |A| + |B| - 2 LCS (the two equations of "Pairwise similarities
 * calculation"); indel = 0 (identical sequences) counts as +infinity.
 * Points are inserted from k-1 down to 0, so the consumer needs the tiles of
 * one family in descending order (FAMSA_LCS_DESCENDING); it keeps the
 * pointer representation pi(i) (the later point i joins) and lambda(i) (the
 * similarity at which it joins) as exact rationals L/indel^2, ordered by the
 * correctly rounded double of the ratio (exact for lengths up to
 * FAMSA_LCS_MAX_LEN: different ratios never round to the same double).
 * ------------------------------------------------------------------------ */
typedef struct famsa_slink_s famsa_slink_t;

/* lengths: k sequence lengths of the family (copied). */
int famsa_slink_create(const uint32_t* lengths, uint32_t k, famsa_slink_t** out);
/* A famsa_lcs_tile_fn: pass the famsa_slink_t* as `user`.  Host tiles only.
 * Returns nonzero (cancel) if tiles arrive out of order. */
int famsa_slink_consume(void* slink, const famsa_lcs_tile* tile);
/* After all rows are in, by original index i: pi[i] (the root, index 0,
 * points to itself) and lambda[i] = lambda_num[i] / lambda_den[i]; den 0 with
 * num >= 0 is +infinity (identical sequences), and the root has num -1,
 * den 0 (never joins).  NULL outputs are skipped.  EINVAL before all rows. */
int famsa_slink_result(const famsa_slink_t* s, uint32_t* pi, int64_t* lambda_num, int64_t* lambda_den);
/* The guide tree from the pointer representation: every point i but the
 * root joins the cluster of pi[i] at similarity lambda[i]; as
 * famsa_guide_tree over the pairs (i, pi[i]).  Arrays of k-1; EINVAL before
 * all rows. */
int famsa_slink_guide_tree(const famsa_slink_t* s, uint32_t* left, uint32_t* right, int64_t* lambda_num,
                           int64_t* lambda_den, uint32_t* nmerges);
/* Rows inserted so far. */
uint32_t famsa_slink_rows_done(const famsa_slink_t* s);
void famsa_slink_destroy(famsa_slink_t* s);

/* ------------------------------------------------------------------------
 * Single linkage on the GPU.  Single linkage merges clusters in the order of
 * the maximum spanning tree of the similarities, so instead of SLINK's
 * pointer representation this consumer keeps that tree on the device: after
 * each device tile (FAMSA_LCS_DEVICE_TILES) it replaces its forest with the
 * maximum spanning forest of the forest plus the tile's pairs (Boruvka
 * rounds on the GPU, one pass over the tile per round).  Device memory is
 * O(k) plus per-round partial results of about k * R / 50 entries for tiles
 * of R rows (R <= 65535); tiles may come in any order.  Similarities are
 * ordered exactly; equal similarities are ordered by the pair (u, v), u < v,
 * so the tree is unique.
 * ------------------------------------------------------------------------ */
typedef struct famsa_mst_s famsa_mst_t;

/* lengths: the k sequence lengths of the family (copied to `device`). */
int famsa_mst_create(const uint32_t* lengths, uint32_t k, int device, famsa_mst_t** out);
/* A famsa_lcs_tile_fn for device tiles: pass the famsa_mst_t* as `user`.
 * Orders its GPU work on tile->stream, after the previous tile's merge
 * whatever stream that one came on, and returns once that work has finished
 * reading the tile (nonzero on a bad tile or a HIP error); calls on one
 * famsa_mst_t must not overlap.  famsa_mst_result, _guide_tree and
 * _get_stats wait for the last merge, not for the whole device. */
int famsa_mst_consume(void* mst, const famsa_lcs_tile* tile);
/* The forest's edges (k-1 of them once every pair has been seen): endpoints
 * u < v (family-local), their LCS and indel^2 (similarity LCS / indel^2).
 * Arrays hold k entries; NULL ones are skipped. */
int famsa_mst_result(const famsa_mst_t* mst, uint32_t* u, uint32_t* v, int64_t* lcs, int64_t* indel2,
                     uint32_t* nedges);
/* The guide tree of the forest (famsa_guide_tree below), arrays of k-1. */
int famsa_mst_guide_tree(const famsa_mst_t* mst, uint32_t* left, uint32_t* right, int64_t* lcs, int64_t* indel2,
                         uint32_t* nmerges);
/* Tiles merged so far and the Boruvka rounds that joined components. */
int famsa_mst_get_stats(const famsa_mst_t* mst, uint64_t* tiles, uint64_t* rounds);
void famsa_mst_destroy(famsa_mst_t* mst);

/* ------------------------------------------------------------------------
 * Guide tree (Methods, "Determination of the guide tree"; the progressive
 * stage merges profiles in the tree's bottom-up order).  Host code, no GPU.
 *
 * Input: nedges <= k-1 edges (u[e], v[e]) of a spanning forest of the k
 * sequences (family-local indices, u != v) with similarity num[e] / den[e]
 * (den 0 = +infinity, e.g. LCS and indel^2).  Output: the single-linkage
 * merges, most similar first, equal similarities by the edge (min, max)
 * lexicographically: merge t joins clusters left[t] (holding the edge's
 * smaller end) and right[t] into cluster k + t; clusters 0..k-1 are the
 * sequences.  merge_num/merge_den receive each merge's similarity;
 * *nmerges = nedges.  Output arrays hold nedges entries, NULL ones are
 * skipped.  EINVAL if an edge is out of range, has a negative similarity, or
 * closes a cycle.
 * ------------------------------------------------------------------------ */
int famsa_guide_tree(uint32_t k, const uint32_t* u, const uint32_t* v, const int64_t* num, const int64_t* den,
                     uint32_t nedges, uint32_t* left, uint32_t* right, int64_t* merge_num, int64_t* merge_den,
                     uint32_t* nmerges);
/* The maximum spanning forest of any nedges edges (u, v, num/den as above,
 * cycles allowed) under the same order: most similar first, equal
 * similarities by the pair (min, max).  Out arrays hold up to k-1 edges,
 * written as (min, max); *nout is their number.  Because the forest of a
 * union of edge sets equals the forest of the union of their forests, the
 * forests that several consumers (one per GPU, say) build from disjoint
 * shares of a family's tiles merge here into the forest of all its pairs. */
int famsa_spanning_forest(uint32_t k, const uint32_t* u, const uint32_t* v, const int64_t* num, const int64_t* den,
                          uint64_t nedges, uint32_t* out_u, uint32_t* out_v, int64_t* out_num, int64_t* out_den,
                          uint32_t* nout);
/* The leaves in depth-first order, left subtree first (order[0..k-1]), and
 * for every cluster c (0 .. k+nmerges-1) the range first[c] .. first[c] +
 * size[c] - 1 its leaves take in that order: with the sequences laid out in
 * this order (e.g. in a famsa_gapped_t) every profile of the progressive
 * stage is a contiguous range, and two merging profiles are adjacent.
 * Several roots (a forest) follow each other.  NULL outputs are skipped.
 * EINVAL if the merges do not each join two current clusters. */
int famsa_guide_tree_leaf_order(uint32_t k, const uint32_t* left, const uint32_t* right, uint32_t nmerges,
                                uint32_t* order, uint32_t* first, uint32_t* size);
/* The tree in Newick form, leaves named by index ("((0,1),2);"; a forest is
 * wrapped in one more pair of parentheses).  *needed = its length + 1; the
 * text is written when buf holds that many bytes (buf may be NULL to ask). */
int famsa_guide_tree_newick(uint32_t k, const uint32_t* left, const uint32_t* right, uint32_t nmerges, char* buf,
                            uint64_t buf_size, uint64_t* needed);

/* ------------------------------------------------------------------------
 * Gapped sequence representation (Methods, "Progressive construction of the
 * alignment", Fig. 1): the form in which the progressive stage moves whole
 * sequences between profiles and inserts gap columns without copying them.
 * Each sequence is kept on the device as its symbols behind a guard
 * (position 0), a gap counter per position -- the gap columns right after
 * that position's symbol (position 0: leading gaps), as the figure's numbers
 * have it -- and the tree of column counts dps: with P the positions rounded
 * up to a power of two (>= 2), leaf P/2 + j counts the columns of positions
 * 2j and 2j+1 and dps[v] = dps[2v] + dps[2v+1]; dps[1] counts every column,
 * the guard's included.  Column 0 is the guard's; the alignment's columns
 * are 1..width.  Calls return when their GPU work is done.
 * ------------------------------------------------------------------------ */
typedef struct famsa_gapped_s famsa_gapped_t;

/* nseq sequences (codes, seq_off as for famsa_lcs_plan; lengths <= 65535)
 * with no gaps, on `device`.  EINVAL on bad input, EDEVICE without a GPU. */
int famsa_gapped_create(const uint8_t* codes, const uint64_t* seq_off, uint32_t nseq, int device,
                        famsa_gapped_t** out);
/* Insert gap runs into sequences first..first+count-1: run r puts len[r] gap
 * columns before column col[r].  Columns are those before this call, sorted
 * ascending, 1 <= col[r] <= width + 1 of every sequence touched (width + 1
 * appends).  One GPU thread per sequence; O(nruns log n) each. */
int famsa_gapped_insert(famsa_gapped_t* g, uint32_t first, uint32_t count, const uint32_t* col, const uint32_t* len,
                        uint32_t nruns);
/* width[i] = the alignment columns of sequence i (the guard's excluded). */
int famsa_gapped_width(const famsa_gapped_t* g, uint32_t* width);
/* pos[q] = the position (0 = guard, i = symbol i) whose span -- its symbol
 * column and the gap run after it -- holds column col[q] (0..width) of
 * sequence seq[q]: a walk down the tree per query. */
int famsa_gapped_locate(famsa_gapped_t* g, const uint32_t* seq, const uint32_t* col, uint32_t nq, uint32_t* pos);
/* The gapped rows of sequences first..first+count-1 into host memory: row t
 * (row_bytes apart) gets columns 1..width of sequence first+t, symbol codes
 * and 0xFF for gaps; bytes past the width are left as they were. */
int famsa_gapped_decode(famsa_gapped_t* g, uint32_t first, uint32_t count, uint8_t* out, uint64_t row_bytes);
/* Copies of sequence s's gap counters (npos entries) and tree (ptree
 * entries, index 0 unused); NULL outputs are skipped. */
int famsa_gapped_state(famsa_gapped_t* g, uint32_t s, uint32_t* no_gaps, uint32_t* dps, uint32_t* npos,
                       uint32_t* ptree);
void famsa_gapped_destroy(famsa_gapped_t* g);

/* ------------------------------------------------------------------------
 * Serving: similarity jobs (each one family) are admitted while their device
 * footprint fits the budget, kept resident, and batched together: every
 * scheduler step gathers the next tiles of all admitted jobs into one launch
 * per length class, so a job that arrives while others run joins on the next
 * step.  Results are identical to running each job alone.
 * ------------------------------------------------------------------------ */
typedef struct famsa_lcs_server_s famsa_lcs_server_t;

/* opt->hbm_budget bounds the resident jobs plus step buffers (0 = 90% of free). */
int famsa_lcs_server_create(const famsa_lcs_options* opt, famsa_lcs_server_t** out);
/* Queue a job (one family); inputs are copied.  *job_id receives its id.
 * EINVAL as for famsa_lcs_plan_create; ENOMEM if the job alone can never fit. */
int famsa_lcs_server_submit(famsa_lcs_server_t* srv, const uint8_t* codes, const uint64_t* seq_off,
                            uint32_t nseq, uint32_t* job_id);
/* Admit queued jobs that fit, run one step over all admitted jobs, deliver its
 * tiles (tile.family = job id, per-job tile_index; a job's tiles cover its
 * rows in order, tile_rows at a time, or fewer under a step_cells bound),
 * retire finished jobs.
 * *active receives the number of jobs still admitted or queued. */
int famsa_lcs_server_step(famsa_lcs_server_t* srv, famsa_lcs_tile_fn fn, void* user, uint32_t* active);
/* Job state: 0 queued, 1 admitted, 2 done. */
int famsa_lcs_server_job_state(const famsa_lcs_server_t* srv, uint32_t job_id, int* state);
/* Device bytes held now and the high-water mark. */
int famsa_lcs_server_memory(const famsa_lcs_server_t* srv, uint64_t* in_use, uint64_t* peak);
void famsa_lcs_server_destroy(famsa_lcs_server_t* srv);

/* ------------------------------------------------------------------------
 * Autotuning: time candidate launch parameters (waves per workgroup per
 * length class, columns per work item, and for long rows the most dwords a
 * lane holds in the lanes-per-row mode, which fixes the lanes per row and
 * the rows per wave, or the segmented kernel) on the plan's first launch
 * step and store the winner in a text cache, one line per GPU architecture
 * and alphabet size ("arch/sigmaN waves0 waves1 waves2 cols long_dwords
 * waves3"; path: cache_path, else FAMSA_LCS_TUNE_CACHE, else none).
 * Results never change.
 * ------------------------------------------------------------------------ */
int famsa_lcs_autotune(famsa_lcs_plan_t* plan, const char* cache_path);

/* ------------------------------------------------------------------------
 * Integer-VALU ceiling (Methods, "Pairwise similarities calculation": the
 * bit-parallel step costs O(|A||B|/w); on gfx950 it is three 32-bit VALU
 * instructions per 32 cells).  Runs long register-only chains of exactly
 * those instructions on every CU and reports their rate and the shader
 * clock measured inside the kernel (s_memtime over s_memrealtime).
 *   variant        0 the recurrence (v_and_b32, v_addc_co_u32 chained over 8
 *                  dwords, v_bitop3_b32), 1 v_and_b32 only, 2 v_addc_co_u32
 *                  only, 3 v_bitop3_b32 only
 *   blocks_per_cu  workgroups of 256 threads per CU (1..32)
 *   iters          loop iterations, 192 instructions per lane each (1..2^24)
 * Errors: EINVAL (bad argument), EDEVICE (no GPU or a HIP failure).
 * ------------------------------------------------------------------------ */
typedef struct famsa_valu_peak_result {
  double ms;                       /* event-timed kernel duration */
  double lane_ops;                 /* 32-bit lane operations executed */
  double ops_per_s;                /* lane_ops / duration */
  double clock_ghz;                /* mean shader clock over the workgroups' loops */
  double mean_loop_cycles;         /* mean shader-clock cycles of a workgroup's loop */
  double lane_ops_per_clk_per_cu;  /* ops_per_s / (clock * CUs) */
  uint32_t cus;
} famsa_valu_peak_result;

int famsa_valu_peak(int device, uint32_t variant, uint32_t blocks_per_cu, uint32_t iters,
                    famsa_valu_peak_result* out);

/* ------------------------------------------------------------------------
 * Aligning one sequence to a profile: the specialised DP the progressive
 * stage runs when one side of a merge is a single sequence (Methods,
 * "Progressive construction of the alignment"), with affine terminal and
 * non-terminal gap costs and gap-type corrections ("Gap types and costs
 * determination").  A batch of independent problems (one level of the guide
 * tree) runs in one call.  Problem p:
 *   sequence   seqs[seq_off[p] .. seq_off[p+1]), m codes < alphabet_size
 *   profile    nrows[p] >= 1 gapped rows of width[p] columns, row-major at
 *              rows + rows_off[p]; each byte a code < alphabet_size or
 *              FAMSA_PROFILE_GAP
 *   subst      alphabet_size x alphabet_size scores, S[x][a] at
 *              subst[x * alphabet_size + a]; |S| <= FAMSA_PROFILE_MAX_SUBST
 *   gap_costs  To, Te, Go, Ge (terminal open, terminal extension, open,
 *              extension), already scaled (famsa_gap_costs_scaled);
 *              |cost| <= FAMSA_PROFILE_MAX_GAP
 * The score of an alignment sums, over the profile's rows, the pair score
 * with the sequence: S[x][a] where residue a faces residue x; a gap run in
 * the sequence against columns costs each column's residue count times To
 * or Go for the first column and Te or Ge for the rest (terminal before
 * the first and after the last residue); a run of new gap columns inserted
 * into the profile at a boundary costs each row, for the first column, Te
 * or To in its terminal region (next to a gap or opening) and Ge or Go
 * inside, and Te or Ge for the others.  The DP maximises it; among optimal
 * alignments it returns the one that prefers, at every cell, M over D over
 * I (the first maximum in that order).
 * Outputs: score[p]; ops + ops_off[p] (room for m + width[p] bytes) gets
 * the alignment from its first column: FAMSA_PROFILE_OP_M residue against
 * column, _D column against a gap in the sequence, _I residue against a new
 * gap column; nops[p] its length.  Synchronous; inputs are host memory.
 * Errors: EINVAL (bad argument), ENOMEM, EDEVICE.
 * ------------------------------------------------------------------------ */
#define FAMSA_PROFILE_GAP 0xFFu
#define FAMSA_PROFILE_OP_M 0u
#define FAMSA_PROFILE_OP_D 1u
#define FAMSA_PROFILE_OP_I 2u
#define FAMSA_PROFILE_MAX_PROBLEMS (1u << 20)
#define FAMSA_PROFILE_MAX_ROWS (1u << 20)
#define FAMSA_PROFILE_MAX_SUBST 1024u
#define FAMSA_PROFILE_MAX_GAP (1u << 20)
int famsa_profile_align(uint32_t nprob, const uint8_t* seqs, const uint64_t* seq_off, const uint8_t* rows,
                        const uint64_t* rows_off, const uint32_t* nrows, const uint32_t* width,
                        uint32_t alphabet_size, const int32_t* subst, const int64_t* gap_costs, int device,
                        int64_t* score, uint8_t* ops, const uint64_t* ops_off, uint32_t* nops);
/* Duration in ms (HIP events) of the DP launch of the last famsa_profile_align
 * call in this process. */
double famsa_profile_last_dp_ms(void);
/* The gap costs scaled by the family size (same section): every cost times
 * g_scale = 1 + ln(k / gl) / gd (the paper's defaults gl = 45, gd = 7),
 * rounded to the nearest integer, halves away from zero.
 * Errors: EINVAL (k = 0, gl <= 0, gd = 0, a result beyond FAMSA_PROFILE_MAX_GAP). */
int famsa_gap_costs_scaled(uint32_t k, const double* base, double gl, double gd, int64_t* out);

/* ------------------------------------------------------------------------
 * For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): the LCS of every pair
 * i < j of one family, the values famsa_lcs_plan + famsa_lcs_tiles give for
 * a single tile of all rows, computed with no allocation of any kind.  Its
 * working memory is one static device array per GPU of
 * FAMSA_LCS_NOALLOC_SCRATCH_BYTES (about 32 MiB), held from the library's
 * first use of that GPU until the process ends; planning runs on the device.
 *   codes      DEVICE pointer: sequence i is codes[seq_off[i] .. seq_off[i+1])
 *   seq_off    DEVICE pointer: nseq + 1 offsets
 *   nseq       <= FAMSA_LCS_NOALLOC_MAX_SEQ
 *   out        DEVICE pointer: nseq (nseq - 1) / 2 int32, row-major upper
 *              triangle, LCS(i, j) at i nseq - i (i + 1) / 2 + (j - i - 1)
 *   status     DEVICE pointer to one int32 or NULL: 0 when every value was
 *              computed, FAMSA_LCS_EINVAL when the device found the input
 *              invalid (decreasing offsets, a length over the limit below, a
 *              code >= alphabet_size); then every value of out is -1
 *   device     HIP ordinal; stream: hipStream_t or NULL.  The work is queued
 *              on the stream and the call returns without waiting.
 * Limits: lengths <= FAMSA_LCS_NOALLOC_MAX_LEN for alphabet_size <= 20,
 * <= FAMSA_LCS_NOALLOC_MAX_LEN_S32 for alphabet_size 21..32.
 * Calls on one GPU share its array: two calls whose work overlaps on the
 * device (different streams, or different host threads) race and give wrong
 * results; calls ordered on one stream are safe.
 * Errors (returned, nothing queued): EINVAL (alphabet_size, nseq over the
 * limit, NULL pointer, bad device), EDEVICE (a HIP call failed).
 * ------------------------------------------------------------------------ */
#define FAMSA_LCS_NOALLOC_MAX_SEQ 8192u
#define FAMSA_LCS_NOALLOC_MAX_LEN 896u
#define FAMSA_LCS_NOALLOC_MAX_LEN_S32 512u
#define FAMSA_LCS_NOALLOC_SCRATCH_BYTES 33757440u
int famsa_lcs_family_noalloc(const uint8_t* codes, const uint64_t* seq_off, uint32_t nseq,
                             uint32_t alphabet_size, int32_t* out, int32_t* status, int device, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* FAMSA_LCS_H */
