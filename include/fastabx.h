/*
 * fastabx-hip: ABX discriminability on AMD Instinct MI355X (gfx950).
 *
 * C ABI of the hot path.  The calls follow the paper's pipeline (Poli, Chemla,
 * Dupoux, "fastabx: A library for efficient computation of ABX
 * discriminability", library-overview section and its pipeline figure):
 *
 *   dataset  -- labels plus a way to reach each item's features (Dataset)
 *   task     -- every cell for given ON / BY / ACROSS conditions (Task)
 *   score    -- d(x,a), d(x,b) for every triple of every cell, D_C per cell (Score)
 *   collapse -- cell-size weighted average, or averaging level by level (collapse)
 *
 * Conventions
 * -----------
 *  - Every call that can fail returns an int status: FABX_OK (0) or a negative
 *    FABX_E* code.  fabx_last_error() then returns a message for the calling
 *    thread.  No C++ exception crosses this boundary.
 *  - Pointers documented "device" are HIP device pointers on the context's
 *    device; every other pointer is host memory.
 *  - Objects returned through an out-parameter are owned by the library and
 *    released with the matching *_destroy / *_free call.  A task keeps its
 *    dataset alive, a result keeps its task alive; releasing the parent first
 *    is allowed (the child holds a reference).
 *  - Work runs on the context's HIP stream.  fabx_score blocks until the
 *    per-cell results are on the host.
 *  - Threads: calls on different tasks and results may come from different
 *    threads at once, also on one context (say one thread building the next
 *    tasks while another launches scores and collapses results).  A task's
 *    scores are serialised by the task itself (a new score first waits for
 *    the one still pending), and a result completes once, whichever thread
 *    asks first.  Destroying an object while another thread still uses it
 *    is not allowed.  The server documents its own rules.
 */
#ifndef FASTABX_H
#define FASTABX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ status codes */
#define FABX_OK 0
#define FABX_EINVAL (-1)     /* bad argument or task specification */
#define FABX_ENOMEM (-2)     /* device or host allocation failed, or over budget */
#define FABX_EDOMAIN (-3)    /* a frame (or pooled mean) has zero norm: its angle is undefined */
#define FABX_EAGAIN (-4)     /* server: job accepted but not finished / not yet admitted */
#define FABX_EHIP (-5)       /* a HIP runtime call failed */
#define FABX_ECANCELED (-6)  /* server: job was cancelled */
#define FABX_ENOTFOUND (-7)  /* server: unknown job id */

/* ------------------------------------------------------------------ enums */
#define FABX_DTYPE_F32 0
#define FABX_DTYPE_BF16 1
#define FABX_DTYPE_UNITS 2           /* int32 discrete unit codes, dim 1 */

#define FABX_DISTANCE_ANGULAR 0      /* theta(u, v) / pi, in [0, 1] */
#define FABX_DISTANCE_EUCLIDEAN 1    /* |u - v| of the raw frames (or means) */
#define FABX_DISTANCE_UNITS 2        /* discrete units: 0 for equal codes, else 1 */

#define FABX_MODE_DTW 0              /* align frames with DTW */
#define FABX_MODE_POOLED 1           /* mean over time, one vector per item */

#define FABX_PREC_FP32 0             /* plain form: FP32 distances, FP32 DTW */
#define FABX_PREC_BF16_RECHECK 1     /* BF16 MFMA distances, FP32 DTW, FP64 recheck of near ties */

#define FABX_NORM_PATH 0             /* DTW cost divided by the optimal path's length */
#define FABX_NORM_NONE 1             /* raw DTW cost */

/* Longest item (in frames) DTW mode accepts.  The BF16 kernels evaluate pairs
 * of items of at most 64 frames; a pair with a longer item is computed in FP64
 * from the raw features instead (rows in chunks of 64, each chunk handing its
 * last row of costs and path lengths to the next), and the plain FP32 form
 * runs its DTW in the same row chunks.  The streaming kernel (fused_cols 512,
 * 1024, 2048) takes items of at most 64 frames. */
#define FABX_MAX_ITEM_FRAMES 1024

typedef struct fabx_ctx fabx_ctx;
typedef struct fabx_dataset fabx_dataset;
typedef struct fabx_task fabx_task;
typedef struct fabx_result fabx_result;

/* Thread-local message for the last failed call on this thread ("" if none). */
const char *fabx_last_error(void);

/* Library version string. */
const char *fabx_version(void);

/* Host threads.  The library runs the parallel parts of its host work (task
 * builds, collapses, table packing) on one shared pool of host threads; a
 * call made while another thread's parallel region runs does its part on the
 * calling thread.  fabx_set_thread_serial(1) makes every later call from the
 * calling thread run its host work on that thread alone, so that it never
 * takes the pool from another thread (e.g. a thread that collapses results
 * beside a thread that builds the next tasks); 0 restores the default.
 * Returns the previous setting of the calling thread.  Results do not depend
 * on it. */
int fabx_set_thread_serial(int serial);

/* --------------------------------------------------------------- context */

/* Create a context on HIP device `device`.  `hip_stream` is a hipStream_t on
 * that device (borrowed, must outlive the context) or NULL for the device's
 * null stream.  Every device operation of the context (uploads, kernels,
 * copies) is enqueued on that stream, after whatever the caller enqueued there
 * before the call: features written by earlier work on the same stream are
 * read in order, with no host synchronisation needed.  fabx_score waits for
 * its own work on the stream before it returns.  Errors: EINVAL (bad device),
 * EHIP. */
int fabx_create(fabx_ctx **out, int device, void *hip_stream);
void fabx_destroy(fabx_ctx *ctx);

/* --------------------------------------------------------------- dataset */

/* A dataset: ragged feature sequences plus an integer attribute table
 * (the Dataset class: "labels and a way to access the representations").
 *
 *  features  device pointer, [n_frames][dim] row-major, dtype F32 or BF16;
 *            or, for discrete representations (the paper says ABX works with
 *            them but gives no distance), FABX_DTYPE_UNITS: one int32 unit
 *            code per frame, dim = 1, scored with FABX_DISTANCE_UNITS in DTW
 *            mode (frame distance 0 for equal codes, 1 otherwise; the DTW
 *            costs are then exact integers and every comparison is exact).
 *            BORROWED: it must stay valid and unchanged while the dataset
 *            (or any task / result made from it) is alive.
 *  offsets   host int64 [n_items + 1]; item i owns frames offsets[i] ..
 *            offsets[i+1]-1.  offsets[0] = 0, offsets[n_items] = n_frames,
 *            strictly increasing (every item has at least one frame) and,
 *            for FABX_MODE_DTW, no item longer than FABX_MAX_ITEM_FRAMES.
 *            Copied.
 *  attrs     host int32 [n_items][n_attr], label-encoded attribute columns
 *            (any int32 values).  Copied.
 * Errors: EINVAL for a null pointer, n_items < 1, dim < 1, n_attr < 1, an
 * unknown dtype, or offsets that break the rules above.  Zero-norm frames are
 * reported by fabx_score (EDOMAIN). */
typedef struct fabx_dataset_desc {
    const void *features;
    int32_t dtype;
    int64_t n_frames;
    int32_t dim;
    const int64_t *offsets;
    int64_t n_items;
    const int32_t *attrs;
    int32_t n_attr;
} fabx_dataset_desc;

int fabx_dataset_create(fabx_ctx *ctx, const fabx_dataset_desc *desc, fabx_dataset **out);

/* The same dataset with items given as windows of the feature rows: item i
 * owns frames item_start[i] .. item_start[i] + item_len[i] - 1.  Windows may
 * overlap and need not cover every row (say consecutive triphones sliced
 * from the features of whole utterances, see fabx_slice_frames): nothing is
 * copied.  features / dtype / n_frames / dim / attrs / n_attr as in
 * fabx_dataset_desc (features BORROWED, item arrays and attrs copied).
 * Errors: EINVAL for a null pointer, n_items < 1, dim < 1, n_attr < 1, an
 * unknown dtype, an item_len < 1, or a window outside [0, n_frames). */
int fabx_dataset_create_windows(fabx_ctx *ctx, const void *features, int32_t dtype, int64_t n_frames,
                                int32_t dim, const int64_t *item_start, const int64_t *item_len,
                                int64_t n_items, const int32_t *attrs, int32_t n_attr, fabx_dataset **out);
void fabx_dataset_destroy(fabx_dataset *ds);

/* Frames of aligned units (the "Slicing features" appendix).  Frame i of an
 * utterance stands for time t_i = dt / 2 + i dt (dt: the constant step
 * between feature frames, e.g. 0.02 s); unit k, [onset[k], offset[k]] in
 * seconds, keeps the frames with onset <= t_i <= offset, i.e. i_start =
 * ceil(onset / dt - 1/2) .. i_end = floor(offset / dt - 1/2), both included,
 * computed in FP64 (i_start no lower than 0).  libri_light != 0 reproduces
 * the slicing of the Libri-Light evaluation, which dropped frame i_end.
 * Outputs start[k] = i_start and len[k] = frames kept (0 when none; the
 * caller decides what an empty unit means).  Errors: EINVAL for a null
 * pointer, n < 0, dt not positive and finite, or a unit without 0 <= onset
 * <= offset (finite). */
int fabx_slice_frames(const double *onset, const double *offset, int64_t n, double dt, int libri_light,
                      int64_t *start, int64_t *len);

/* ------------------------------------------------------------------ task */

/* Build every cell for ON attribute `on`, BY attributes `by[n_by]` and ACROSS
 * attributes `across[n_across]` (attribute = column of the attrs table).
 *
 * Triple predicate (Background section, ABX figure caption and Table 1):
 * a and x share the ON value, b does not; a, b, x share every BY value; a and
 * b share every ACROSS value and x differs from them in every ACROSS
 * attribute.  Without ACROSS the X set is A itself and a == x is excluded
 * (x is compared with *another* a), so |C| = |A|(|A|-1)|B|; with ACROSS
 * |C| = |A||B||X|.  Cells are ordered pairs (on_ax, on_b); cells with no
 * triple are not built.  Cells are numbered in ascending order of
 * (by..., on_ax, on_b, across_ab..., across_x...).
 *
 * This is host work only (integer sort and grouping); device tables are
 * uploaded on the first fabx_score.  Zero cells is valid (num_cells = 0).
 * Errors: EINVAL for a column out of range, a repeated column among on / by /
 * across, or n_by / n_across < 0. */
int fabx_task_create(fabx_dataset *ds, int32_t on, const int32_t *by, int32_t n_by,
                     const int32_t *across, int32_t n_across, fabx_task **out);
void fabx_task_destroy(fabx_task *task);

/* The Subsampler of the Task interface (library overview, "Task" paragraph):
 * it caps the number of a, b and x independently in each cell, and, when
 * ACROSS attributes are given, limits the number of distinct values x takes
 * for them (the paper writes "for the ON attribute"; x's ON value is fixed in
 * a cell, and the Libri-Light evaluation this reproduces limits x's speaker,
 * i.e. its ACROSS value).  A cap of 0 means no cap.
 *
 *  seed          key of the draws.
 *  max_a, max_b  per cell, at most this many items of A / B.
 *  max_x         per cell, at most this many items of X.  Without ACROSS, X is
 *                A itself: the one set is capped by both max_a and max_x and
 *                stays the same set.
 *  max_x_across  ACROSS tasks: of the cells sharing (on_ax, on_b, by...,
 *                across_ab...), which differ only in across_x, at most this
 *                many are kept.
 *
 * Draws: Philox4x32-10 (Salmon et al., "Parallel random numbers: as easy as
 * 1, 2, 3", SC'11) keyed by the seed (low word first), first output word, at
 * counter (c, s, j, 0) where c is the cell's index in the full task (cells
 * numbered as fabx_task_create numbers them), s = 0 / 1 / 2 for A / B / X
 * and j the item's position in the set (items in ascending id), or s = 3 and
 * j the cell's rank in its family for the ACROSS limit, with c the family's
 * first cell.  A capped set keeps the items with the smallest draws (position
 * breaking ties); the family keeps its cells with the smallest draws.  Cells
 * left without a triple (fewer than 2 items in A without ACROSS) are dropped;
 * the cells kept keep their order and keys. */
typedef struct fabx_subsampler {
    uint64_t seed;
    int32_t max_a, max_b, max_x;
    int32_t max_x_across;
} fabx_subsampler;

/* fabx_task_create followed by the Subsampler.  The task's cells are the
 * kept cells with their capped sets (fabx_task_cell_sizes reports the capped
 * |A|, |B|, |X| and |C|); a cell whose sets were reduced is scored on its own
 * sampled items only.  fabx_result_pairs on such a task looks each item up
 * where it first occurs.  Errors: those of fabx_task_create; EINVAL for a
 * NULL subsampler or a negative cap. */
int fabx_task_create_subsampled(fabx_dataset *ds, int32_t on, const int32_t *by, int32_t n_by,
                                const int32_t *across, int32_t n_across, const fabx_subsampler *sub,
                                fabx_task **out);

int64_t fabx_task_num_cells(const fabx_task *task);
/* Number of int32 columns of a cell key: 2 + n_by + 2 * n_across. */
int32_t fabx_task_key_width(const fabx_task *task);
/* Cell keys into host int32 out[num_cells][key_width]:
 * (on_ax, on_b, by..., across_ab..., across_x...), attribute values as given. */
int fabx_task_cell_keys(const fabx_task *task, int32_t *out);
/* Cell sizes into host int64 out[num_cells] (|C|), and the item counts
 * |A|, |B|, |X| into host int32 abx[num_cells][3] (either may be NULL). */
int fabx_task_cell_sizes(const fabx_task *task, int64_t *n_triplets, int32_t *abx);

/* ----------------------------------------------------------------- score */

typedef struct fabx_score_opts {
    int32_t distance;    /* FABX_DISTANCE_ANGULAR | FABX_DISTANCE_EUCLIDEAN.  The
                            Euclidean BF16_RECHECK form takes the unit-vector cosine
                            of the MFMA Gram tile and each frame's FP32 length:
                            |u - v|^2 = (|u| - |v|)^2 + 2 |u| |v| (1 - cos); zero
                            frames are legal there.  Not with the stream kernel
                            (fused_cols >= 512: FABX_EINVAL). */
    int32_t mode;        /* FABX_MODE_DTW | FABX_MODE_POOLED */
    int32_t precision;   /* FABX_PREC_FP32 | FABX_PREC_BF16_RECHECK */
    int32_t dtw_norm;    /* FABX_NORM_PATH | FABX_NORM_NONE */
    double margin;       /* BF16_RECHECK: a comparison with |d(x,a) - d(x,b)| <= margin
                            is re-decided on FP64 distances; < 0 selects the default
                            2e-2 / sqrt(dim), times 2 L - 1 (L: the longest item, at
                            most 64) for the raw DTW cost (FABX_NORM_NONE), a sum of up
                            to 2 L - 1 frame distances.  Euclidean: in units of the
                            largest frame (or mean) length S, found on the device; the
                            default is pi times the angular one (an angle error e
                            moves a Euclidean frame distance by at most S e). */
    double delta;        /* BF16_RECHECK + PATH: cumulative-cost window within which
                            alternative DTW predecessors must agree on the path length,
                            else the pair is recomputed in FP64; < 0 selects the default
                            4e-2 / sqrt(dim) (Euclidean: pi times that, in units of S) */
    int32_t keep_pairs;  /* nonzero: keep the per-pair distances for fabx_result_pairs */
    int32_t fused_cols;  /* BF16 DTW launch choice: 128 or 256 = the tile kernel with
                            column blocks of that many frames; 512, 1024 or 2048 = the
                            stream kernel, each wave streaming segments of about that
                            many column frames; 0 takes the context's tuning table
                            (fabx_autotune), as does 0 with a nonzero grid.  Results do
                            not depend on it. */
    int32_t fused_blocks_per_cu; /* its grid: 0 = one block per work unit (stream
                                    kernel: a wave per segment), 1..64 = a persistent
                                    grid of that many blocks per CU */
} fabx_score_opts;

/* Defaults: ANGULAR, DTW, BF16_RECHECK, PATH, margin/delta = -1 (library
 * defaults), keep_pairs = 0, fused_cols = fused_blocks_per_cu = 0 (tuning
 * table).  FABX_EINVAL for a fused_cols other than 0, 128, 256, 512, 1024 or
 * 2048, or a grid outside 0..64. */
int fabx_score_opts_default(fabx_score_opts *opts);

/* Score every cell: for each cell C and each triple (a, b, x) in it, compare
 * d(x, a) with d(x, b) and accumulate W_C = sum 2[d(x,a) < d(x,b)] +
 * [d(x,a) = d(x,b)] in int64 "half units", so that D_C = W_C / (2 |C|)
 * (the cell discriminability formula of the Background section).
 *
 * d is the distance between frames named by opts->distance (angular: theta /
 * pi; Euclidean: |u - v|, the other distance the Score interface names),
 * aligned with DTW (c[0][0] = d00, cumulative first row and column, c[i][j] =
 * d[i][j] + min(c[i-1][j-1], c[i][j-1], c[i-1][j]), "Dynamic Time Warping on
 * GPU" section) and divided by the optimal path length for FABX_NORM_PATH, or
 * the distance between time-averaged frames for FABX_MODE_POOLED.
 *
 * Synchronous on the context stream.  Errors: EINVAL (bad opts), EDOMAIN
 * (zero-norm frame / mean with the angular distance), ENOMEM (device
 * workspace), EHIP. */
int fabx_score(fabx_task *task, const fabx_score_opts *opts, fabx_result **out);

/* The same score, returned as soon as its work is enqueued on the context
 * stream (task tables are uploaded first if the task has not been scored
 * before).  The result completes in fabx_result_wait, or implicitly in the
 * first fabx_result_cells / _pairs / _stats / fabx_collapse call; num_cells,
 * key_width and cell_keys do not wait.  Errors found on completion (EDOMAIN,
 * EHIP) are returned there, every time it is asked.  A later score of the
 * same task first waits for this one (the task's device workspace is reused).
 * Freeing a pending result waits for its work.  Lets a caller build the next
 * task or collapse the previous result while the device works.  Errors at
 * launch: EINVAL, ENOMEM, EHIP. */
int fabx_score_async(fabx_task *task, const fabx_score_opts *opts, fabx_result **out);

/* Wait for a result and report its status (FABX_OK at once for a finished
 * result).  Errors: EINVAL (NULL), EDOMAIN, EHIP. */
int fabx_result_wait(fabx_result *res);

void fabx_result_free(fabx_result *res);

/* Number of cells of the scored task, and its cell keys (same layout as
 * fabx_task_cell_keys); useful for results returned by the server. */
int64_t fabx_result_num_cells(const fabx_result *res);
int32_t fabx_result_key_width(const fabx_result *res);
int fabx_result_cell_keys(const fabx_result *res, int32_t *out);

/* Per-cell results into caller-owned host buffers of length num_cells (any
 * may be NULL): W_C (half units), |C|, and D_C = W_C / (2|C|). */
int fabx_result_cells(const fabx_result *res, int64_t *half_units, int64_t *n_triplets,
                      double *score);

/* Distances of item pairs (x = row item, y = column item, original item ids,
 * both in the same BY group of the task and both used by some cell) from a
 * result scored with keep_pairs != 0.  out_f32[n]: the GPU distance;
 * flags[n] (may be NULL): bit 0 = the pair's DTW path length was not robust,
 * bit 1 = the pair was recomputed in FP64; out_f64[n] (may be NULL): the FP64
 * recomputed distance where bit 1 is set, else the FP32 value widened.
 * Errors: EINVAL (keep_pairs was 0, or a pair outside the task). */
int fabx_result_pairs(const fabx_result *res, int64_t n, const int64_t *x_items,
                      const int64_t *y_items, float *out_f32, uint8_t *flags, double *out_f64);

typedef struct fabx_stats {
    int64_t n_cells;
    int64_t n_triplets;         /* sum of |C| */
    int64_t n_items;            /* items that take part in some cell */
    int64_t n_frames;           /* their frames */
    int64_t n_pairs;            /* item pairs scored (x, y), both orientations */
    int64_t dtw_cells;          /* sum over the unique pairs the cells need of len(x) * len(y) */
    int64_t computed_dtw_cells; /* DTW cells the kernels actually evaluated */
    int64_t n_nonrobust_pairs;  /* pairs whose DTW path length was not robust */
    int64_t n_recheck_pairs;    /* pairs recomputed in FP64 */
    int64_t n_recount_rows;     /* (cell, x) rows re-counted with FP64 distances */
    int64_t workspace_bytes;    /* device workspace held by the task */
    double ms_total;            /* first kernel to per-cell results on the host */
    double ms_normalize;
    double ms_distance;         /* frame distances + DTW (or pooled distances) */
    double ms_triplets;
    double ms_recheck;          /* FP64 recheck + recount */
    double ms_host_setup;       /* host: work plans, table uploads, workspace (before the first kernel) */
    double ms_host_finish;      /* host: after the results reached the host, until fabx_score returns */
    double margin;              /* near-tie margin used (BF16 form; 0 for FP32; Euclidean: in
                                   units of the largest frame length) */
    double delta;               /* path-length window used (BF16 form, DTW; else 0; the same
                                   units as margin) */
    int32_t fused_cols;         /* fused kernel column block width used (BF16 DTW; else 0) */
    int32_t fused_blocks_per_cu;/* its grid: blocks per CU, 0 = one block per work unit */
    int64_t dtw_cells_sym;      /* sum over the unordered pairs {x, y} of which some cell needs
                                   (x, y) or (y, x) of len(x) * len(y): the DTW cells needed
                                   when each pair's DTW, which is symmetric, is evaluated once */
} fabx_stats;

int fabx_result_stats(const fabx_result *res, fabx_stats *stats);

/* Bytes of the per-device scratch array behind fabx_score_noalloc (256 MiB). */
#define FABX_NOALLOC_SCRATCH_BYTES (256 * 1024 * 1024)

/* fabx_score for callers that cannot allocate memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  It computes
 * exactly what fabx_score computes (same kernels, same per-cell counts W_C)
 * but lays every device buffer of the score -- the task's tables, the fused
 * kernel's column plan and the whole workspace -- in one library-owned
 * scratch array of FABX_NOALLOC_SCRATCH_BYTES per device, which each device
 * the library runs on holds until the process ends.  It calls no hipMalloc,
 * hipFree, pinned-memory allocation or allocating library routine.
 *
 *  task        a task of a device context (the dataset's features are read
 *              on the context's stream, as by fabx_score).
 *  opts        as fabx_score (NULL: defaults); keep_pairs must be 0.
 *  half_units  host int64 [num_cells], caller-owned: W_C of every cell.
 *  stats       host, may be NULL: as fabx_result_stats, without stage times.
 *
 * Synchronous: returns once the counts are on the host.  Calls on one device
 * share its scratch array, which keeps the last call's contents; they are
 * serialised by a per-device lock held for the whole call, so calls from
 * several threads do not overlap, but any other use of the same memory (a
 * graph replay still running, say) would race.  Errors: EINVAL (bad opts,
 * keep_pairs set, host-only context), ENOMEM (the task needs more scratch
 * than FABX_NOALLOC_SCRATCH_BYTES; fabx_score has no such limit), EDOMAIN,
 * EHIP. */
int fabx_score_noalloc(fabx_task *task, const fabx_score_opts *opts, int64_t *half_units,
                       fabx_stats *stats);

/* ------------------------------------------------------------- autotune */

/* Launch choices of the fused BF16 DTW kernel (batching of uneven cells in one
 * persistent launch): the column block width in frames (128 or 256; wider
 * blocks give each DTW wave a longer column stream, narrower ones keep more
 * blocks resident) and the grid (blocks_per_cu > 0: a persistent grid of that
 * many blocks per compute unit; 0: one block per work unit). */
typedef struct fabx_tune_entry {
    int32_t cols;
    int32_t blocks_per_cu;
    double ms_distance;   /* best of three runs, distance + DTW stage, device time */
} fabx_tune_entry;

typedef struct fabx_tune_report {
    int32_t n_tried;      /* 0: nothing to tune for these options */
    int32_t best;         /* index into tried, -1 if none */
    int32_t key_dim_pad, key_max_len, key_frames_log2;  /* shape class the choice is kept for */
    fabx_tune_entry tried[8];
} fabx_tune_report;

/* Score the task with every candidate configuration in three interleaved
 * rounds (one when the default's distance stage takes 100 ms or more),
 * keeping each one's fastest run, check that every candidate gives
 * identical per-cell counts, and keep the default (tried[0]) unless another
 * candidate is faster by more than 2%, then the fastest, for the task's
 * shape class (padded dim, longest item rounded up
 * to 8 frames, log2 of mean frames per BY group, DTW normalisation) in the
 * context's table; later scores of tasks in that class use it.  If the
 * environment variable FABX_AUTOTUNE_CACHE names a file when the context is
 * created, the table is read from it and rewritten after each new entry.
 * Only the BF16 DTW form has choices; other options return FABX_OK with
 * n_tried = 0.  keep_pairs is ignored.  Errors: as fabx_score; EINVAL if two
 * candidates disagree (a defect). */
int fabx_autotune(fabx_task *task, const fabx_score_opts *opts, fabx_tune_report *report);

/* HBM streaming probe, for measurement only: converts n_rows rows of dim FP32
 * values (src, device, [n_rows][dim]) to BF16 rows of dim_pad = the multiple
 * of 64 at or above dim (dst, device, [n_rows][dim_pad]; the padding columns
 * are written as zeros) with the access widths and order of the normalise
 * kernel but none of its arithmetic, on `hip_stream` (NULL: the null stream),
 * asynchronously.  It moves 4 dim bytes in and 2 dim_pad bytes out per row,
 * the normalise kernel's traffic for FP32 features, so the achievable
 * bandwidth and the byte counters' scaling for that access pattern can be
 * measured beside it.  Both buffers are caller-owned.  Errors: EINVAL (null
 * pointer, n_rows < 0, dim not a positive multiple of 4 or above 2048),
 * EHIP. */
int fabx_probe_stream(const float *src, uint16_t *dst, int64_t n_rows, int32_t dim, void *hip_stream);

/* -------------------------------------------------------------- collapse */

/* ABX error rate 1 - D (Score.collapse).  n_levels = 0: D is the cell-size
 * weighted mean, sum W / (2 sum |C|).  Otherwise level k names
 * level_len[k] attributes, listed one after another in level_attr; for each
 * level in order, the key columns of its attributes (both the _ab and _x
 * columns of an ACROSS attribute) are removed and D_C is averaged, unweighted,
 * over the rows sharing the remaining key; D is the unweighted mean of what is
 * left.  Errors: EINVAL if a level names the ON attribute or an attribute that
 * is not a BY / ACROSS attribute of the task, or the task has no cell. */
int fabx_collapse(const fabx_result *res, const int32_t *level_attr, const int32_t *level_len,
                  int32_t n_levels, double *error_rate);

/* ---------------------------------------------------------------- server */

/* Continuous-batching job server on one context.  Jobs (dataset + task spec
 * + options) are queued by fabx_server_submit.  Whenever one of `n_streams`
 * HIP streams of the context's device is free, the first queued job whose
 * device-memory footprint fits in `hbm_budget_bytes` next to the jobs already
 * running is admitted: a smaller job may start before a larger one queued
 * ahead of it, but a job passed over 8 times is not passed again (it starts
 * as soon as it fits).  Admitted jobs run concurrently.  A job's result is
 * identical to what fabx_score returns for it alone, and a job that fails
 * (say EDOMAIN) does not change the others.  When a job ends, its device
 * memory goes back to the context's pool.
 *
 * Thread rules: submit / poll / wait / cancel may be called from any thread.
 * A dataset passed to submit must stay alive until the job completes or is
 * cancelled (the job holds a reference to it; the features are borrowed). */
typedef struct fabx_server fabx_server;

int fabx_server_create(fabx_ctx *ctx, int64_t hbm_budget_bytes, int32_t n_streams,
                       fabx_server **out);
/* Stops accepting jobs, cancels queued ones, waits for running ones. */
void fabx_server_destroy(fabx_server *srv);

/* Queue a job.  The job's kernels run on the server's own streams, after all
 * work enqueued on the context's stream before this call (an event recorded
 * there at submit), so features produced on that stream are read in order.
 * Errors: EINVAL (bad spec), ENOMEM (the job's footprint exceeds the whole
 * budget, so it could never run), EHIP. */
int fabx_server_submit(fabx_server *srv, fabx_dataset *ds, int32_t on, const int32_t *by,
                       int32_t n_by, const int32_t *across, int32_t n_across,
                       const fabx_score_opts *opts, uint64_t *job_id);
/* FABX_OK and *out set when finished (caller frees the result); EAGAIN while
 * queued or running; ECANCELED; ENOTFOUND; or the job's own error code.  Once
 * an outcome other than EAGAIN has been returned, the server forgets the job:
 * asking again gives ENOTFOUND. */
int fabx_server_poll(fabx_server *srv, uint64_t job_id, fabx_result **out);
/* Like poll, but blocks until the job is no longer queued or running. */
int fabx_server_wait(fabx_server *srv, uint64_t job_id, fabx_result **out);
/* Cancel a queued job (running jobs finish).  Errors: ENOTFOUND, EAGAIN if
 * already running or finished. */
int fabx_server_cancel(fabx_server *srv, uint64_t job_id);

typedef struct fabx_server_stats {
    int64_t submitted, completed, cancelled, failed, queued, running;
    int64_t hbm_in_use, hbm_high_water;
    double p50_ms, p99_ms;        /* completion - entry into fabx_server_submit, over completed jobs */
    double p50_queue_ms, p99_queue_ms; /* queue wait: end of the submit call -> admission */
    double mean_build_ms;         /* task build inside fabx_server_submit */
    double mean_queue_ms;         /* queue wait */
    double mean_run_ms;           /* admission -> completion (device work and result copy) */
} fabx_server_stats;

int fabx_server_stats_get(fabx_server *srv, fabx_server_stats *st);

#ifdef __cplusplus
}
#endif
#endif /* FASTABX_H */
