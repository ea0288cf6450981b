// Host-side launchers of the HIP kernels.  Each launcher checks the launch
// shape it relies on and enqueues on `stream`; none synchronises.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.h"

namespace fabx {
namespace kern {

// Blocks for `work` items handled `per_block` at a time, capped (the kernels
// loop); threads * blocks always fits the 32-bit dispatch grid.
inline unsigned grid_for(int64_t work, int64_t per_block, int64_t cap = int64_t(1) << 20) {
    int64_t b = (work + per_block - 1) / per_block;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return unsigned(b);
}

// Per-item task tables on the device.
struct ItemTables {
    const int64_t *src;    // first source frame of each task item
    const int32_t *len;    // frames per item
    const int64_t *dst;    // first packed frame
    int64_t n_items;
};

// Per-group tables on the device (n_groups entries; *_prefix arrays have n_groups + 1).
struct GroupTables {
    const int64_t *item0, *n_items, *frame0, *n_frames, *pair_base;
    int64_t n_groups;
    int64_t n_pair_slots;
};

// --- k_prep.hip
// Pack every frame of every task item into the packed buffer (row stride
// dim_pad, zero padded).  out_form = 0: F32 unit rows; 1: BF16 unit rows plus
// rinv[f] = 1 / ||bf16 row|| (F32); 2: F32 rows unscaled (Euclidean distance,
// FP32 form); 3: form 1 plus len_out[f] = ||frame|| (F32) and *scale = the
// largest length (F32 bits; *scale zero before the call), a zero frame packed
// as zeros with rinv 0 (Euclidean distance, BF16 form).  In forms 0 and 1 a
// zero-norm frame sets err[0] = 1 and lowers err_item (unsigned long long) to
// its task item.  len_out and scale may be null outside form 3.
void normalize(hipStream_t s, const void *features, int dtype, int dim, int dim_pad,
               const ItemTables &it, void *out, int out_form, float *rinv, int *err,
               unsigned long long *err_item, float *len_out, unsigned int *scale);

// HBM streaming probe: rows [n_rows][dim] FP32 -> [n_rows][dim_pad] BF16 with
// the normalise kernel's access widths (dim a multiple of 4, <= 2048).
void probe_stream(hipStream_t s, const float *src, int dim, int64_t n_rows, uint16_t *out);

// Discrete units: the int32 code of every frame of every task item, packed in
// task order into out [task frames].
void pack_units(hipStream_t s, const int32_t *codes, const ItemTables &it, int32_t *out);

// Time pooling: mean of each item's frames (F32 accumulation), then the same
// packing; one packed row per task item.
void pool_normalize(hipStream_t s, const void *features, int dtype, int dim, int dim_pad,
                    const ItemTables &it, void *out, int out_form, float *rinv, int *err,
                    unsigned long long *err_item, float *len_out, unsigned int *scale);

// --- k_plain.hip (plain FP32 form)
// Segments of Gram output: segment s holds the distances of packed rows
// [row0[s], row0[s] + nrows[s]) against packed rows [col0[s], col0[s] + ncols[s])
// at out[base[s] + r * ncols[s] + c].  Tiles are 64 x 64; tile_prefix has n + 1
// entries, and the launch covers tiles [tile_prefix[0], tile_prefix[n]).
struct GramSegments {
    const int64_t *row0, *nrows, *col0, *ncols, *base, *tile_prefix;
    int64_t n;
    int64_t n_tiles;  // tile_prefix[n] - tile_prefix[0] (host copy, sizes the grid)
};
// theta/pi of unit rows (euclid = 0) or the length of the difference of raw
// rows (euclid = 1) for every (row, column) of every segment.  Pooled mode:
// one segment per group (its item vectors against themselves, base = the
// group's pair matrix); DTW mode: one segment per strip (below).
void gram_angular_f32(hipStream_t s, const float *xn, int dim_pad, const GramSegments &seg, float *out,
                      int euclid);

// Plain DTW mode: a group's frame distance matrix is made in strips of rows
// (the frames of consecutive items of the group) against all the group's
// frames, and strips are processed in batches whose matrices fit the dmat
// buffer.  Strip s: group[s], its first pair slot slot0[s] (n + 1 entries, a
// prefix: the slots of the strip's row items), its first row's packed frame
// row0[s] and its matrix offset base[s] in the batch's dmat buffer.
struct PlainStrips {
    const int64_t *group, *slot0, *row0, *base;
    int64_t n;
    int64_t n_slots;  // slot0[n] - slot0[0] (host copy, sizes the grid)
};
// One wave per ordered item pair of the strips' slots: anti-diagonal DTW over
// the strip's F32 distance matrix (lane = row), exact diagonal > left > up
// predecessor order.  norm: FABX_NORM_PATH / FABX_NORM_NONE.  has_long: some
// item has more than 64 frames (rows then go in chunks of 64).  exact: the
// costs are integers (discrete units); the path-normalised value is their
// double quotient rounded once.
void dtw_plain(hipStream_t s, const float *dmat, const PlainStrips &st, const GroupTables &g,
               const ItemTables &it, int norm, bool has_long, bool exact, float *p32);
// Discrete units: the GramSegments tiles of [code_row != code_col] (0 or 1) from
// the packed codes.
void unit_mismatch(hipStream_t s, const int32_t *codes, const GramSegments &seg, float *out);

// --- k_fused.hip (BF16 form)
struct FusedPlan {
    const int32_t *rb;        // row blocks: [n_rb][4] = group, first item (task), n items, n frames
    const int32_t *cb;        // col blocks: same layout
    const int64_t *unit_prefix; // per band: prefix of its work units, n_bands + 1
    const int32_t *band_rb;     // band b = row blocks [band_rb[b], band_rb[b + 1]) of one group
    const int32_t *g_cb0;       // per group: first column block
    const int32_t *rb_cstart;   // per row block: its first kept column block (counted in the group)
    // A band's units: column block c (from its first row block's rb_cstart on)
    // x its row blocks, row block fastest; a unit with c before its row block's
    // rb_cstart is skipped.
    int64_t n_bands;
    int64_t n_units;
    int cols;            // column block width the blocks were packed for: 128 or 256
    int blocks_per_cu;   // persistent grid of blocks_per_cu * n_cu blocks; 0: one block per unit
    int n_cu;
};
// unit_ctr: 8 counters, zero at launch (the XCDs' next units of a persistent grid)
// flen (non-null: Euclidean distance): FP32 frame lengths; scale: the largest
// (FP32 bits), delta being in units of it.
void fused_bf16(hipStream_t s, const uint16_t *xn, const float *rinv, int dim_pad,
                const GroupTables &g, const ItemTables &it, const FusedPlan &plan, int norm,
                float delta, float *p32, uint8_t *flags, unsigned int *nonrobust_n,
                unsigned int *unit_ctr, const float *flen, const unsigned int *scale);

// --- k_stream.hip (BF16 form, DTW mode: the column-stream kernel)
// Per task frame: bit 31 first frame of its item, bit 30 last frame, bits
// 6..29 the item's place in its BY group, bits 0..5 the frame's index in
// its item.
void frame_info(hipStream_t s, const ItemTables &it, const int32_t *item_group, const int64_t *g_item0,
                uint32_t *finfo);
struct StreamPlan {
    const int32_t *rb;              // row blocks: [n_rb][4] = group, first item (task), n items, n frames
    const int64_t *rb_unit_prefix;  // per row block: prefix of its stream segments, n_rb + 1
    int64_t n_rb;
    int64_t n_units;
    int seg_len;         // nominal segment length (frames)
    int blocks_per_cu;   // persistent grid of blocks_per_cu * n_cu blocks (4 waves each); 0: a wave per unit
    int n_cu;
};
// unit_ctr: 8 counters, zero at launch.  delta_q: the path-length window in
// units of 1 / 65535.
void stream_bf16(hipStream_t s, const uint16_t *xn, const float *rinv, int dim_pad, const uint32_t *finfo,
                 const GroupTables &g, const ItemTables &it, const StreamPlan &plan, int norm, uint32_t delta_q,
                 float *p32, uint8_t *flags, unsigned int *nonrobust_n, unsigned int *unit_ctr);

// Pooled mode, BF16 MFMA: theta/pi between pooled item vectors of each group
// (flen non-null: the Euclidean distance of the means, from the cosine and
// their FP32 lengths); flags[slot] = 1 (non-robust) for a nearly parallel or
// antiparallel pair (flags zeroed before).
void gram_angular_bf16(hipStream_t s, const uint16_t *xn, const float *rinv, int dim_pad,
                       const int64_t *row0, const int64_t *nrows, const int64_t *base,
                       const int64_t *tile_prefix, int64_t n_groups, int64_t n_tiles, float *out,
                       uint8_t *flags, const float *flen);

// --- k_triplets.hip
// One wave per unit [cell, x_begin, x_end): W[cell] += sum over the unit's rows of
// 2[d(x,a) < d(x,b)] + [d(x,a) == d(x,b)].  With flags != nullptr (BF16 form), a row
// holding a comparison with |d(x,a) - d(x,b)| <= margin, or a non-robust pair, is
// not counted: its pairs get flag bit 1 and (cell, x) is appended to recount.
// scale (may be null): margin is in units of *scale (FP32 bits; the Euclidean
// BF16 form's largest frame length).
void triplets(hipStream_t s, const CellDev *cells, const int32_t *units, int64_t n_units,
              const GroupTables &g, const float *p32, unsigned long long *W, uint8_t *flags,
              float margin, int32_t *recount, unsigned int *recount_n, int64_t recount_cap,
              const unsigned int *scale);
// Large cells, one x per unit: the same counts and marks from the row's B
// distances sorted in LDS (|B| <= kSortedMaxB).
void triplets_sorted(hipStream_t s, const CellDev *cells, const int32_t *units, int64_t n_units,
              const GroupTables &g, const float *p32, unsigned long long *W, uint8_t *flags,
              float margin, int32_t *recount, unsigned int *recount_n, int64_t recount_cap,
              const unsigned int *scale);

// Zeroes W [n_cells] and the 64 counter bytes after it (the u64 at byte 8 of
// those, the error item, is set to all ones).
void init_score(hipStream_t s, unsigned long long *W, int64_t n_cells);

// Pair slots whose flag bit 1 is set -> list (order unspecified); nothing when
// *recount_n is 0 (no row was sent to the recount, so no pair is marked).
void collect_marked(hipStream_t s, const uint8_t *flags, int64_t n_slots, int64_t *list,
                    unsigned int *count, int64_t cap, const unsigned int *recount_n);

// Re-count rows (cell, x): a comparison of two recomputed pairs (flag bit 1 on both)
// uses their FP64 values, any other comparison the FP32 ones.
void recount(hipStream_t s, const CellDev *cells, const int32_t *rows, const unsigned int *n_rows,
             int64_t max_rows, const GroupTables &g, const float *p32, const double *p64,
             const uint8_t *flags, unsigned long long *W);

// --- k_recheck.hip
// FP64 distance of each listed pair slot from the raw features (unit vectors
// by division by the sequential-sum norm, cosine as a sequential sum, acos or
// the half-chord atan2 form near |cos| = 1, DTW with diagonal > left > up).
// has_long: the task has items of more than 64 frames (DTW mode); their pairs
// go through the tiled kernel of long_dtw.  euclid: the Euclidean distance.
void recheck_fp64(hipStream_t s, const void *features, int dtype, int dim, const GroupTables &g,
                  const ItemTables &it, const int64_t *list, const unsigned int *count,
                  int64_t max_count, int mode, int norm, bool has_long, int euclid, double *p64);
// The same FP64 DTW for the listed slots whose pair has an item of more than
// 64 frames (up to FABX_MAX_ITEM_FRAMES); others are skipped.  count: device
// count of listed slots, or null for max_count.  p32 and flags (may be null)
// also receive the value and 0 (robust, unmarked).
void long_dtw(hipStream_t s, const void *features, int dtype, int dim, const GroupTables &g,
              const ItemTables &it, const int64_t *list, const unsigned int *count, int64_t max_count, int norm,
              int euclid, double *p64, float *p32, uint8_t *flags);

}  // namespace kern
}  // namespace fabx
