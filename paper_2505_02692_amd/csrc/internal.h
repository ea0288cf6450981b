// Internal types of the fastabx-hip runtime (host side).
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <atomic>
#include <cstdint>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "fastabx.h"
#include "host_pool.h"

namespace fabx {

// Errors travel as exceptions inside the library and become status codes at
// the C boundary (api.cpp); nothing throws across extern "C".
struct Error {
    int code;
    std::string msg;
};

[[noreturn]] void fail(int code, const std::string &msg);
void set_last_error(const std::string &msg);

#define FABX_HIP(call)                                                                    \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess)                                                             \
            ::fabx::fail(FABX_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));  \
    } while (0)

// Caching device allocator of one context: freed blocks are kept and handed
// out again to later requests of a similar size, so scoring a new task does
// not go back to hipMalloc for its (multi-GB) workspace.  Thread-safe.
struct Pool {
    std::mutex mu;
    std::vector<std::pair<size_t, void *>> free_blocks;  // (bytes, ptr)
    size_t held = 0;                                     // bytes owned (free + in use)
    void *alloc(size_t n, size_t *got);
    void free(void *p, size_t n);
    void trim();  // return every free block to the runtime
    ~Pool();
};

// Grow-only device buffer (from a context pool when one is attached).
struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    Pool *pool = nullptr;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() { release(); }
    void release();
    // Ensure capacity >= n bytes (contents are not preserved on growth).
    void ensure(size_t n);
    template <typename T>
    T *as() const { return static_cast<T *>(ptr); }
};

// Reusable HIP events of one context (stage timers of concurrent scores).
struct EventPool {
    std::mutex mu;
    std::vector<hipEvent_t> free_events;
    hipEvent_t get();
    void put(hipEvent_t e);
    ~EventPool();
};

// Pinned host buffer that uploads go through.  An upload returns once its DMA
// is enqueued; the next one waits for that DMA before writing the buffer.
struct Staging {
    std::mutex mu;
    void *host = nullptr;
    size_t cap = 0;
    hipEvent_t done = nullptr;
    bool in_flight = false;   // a DMA out of `host` may still run (done not yet waited for)
    void reserve(size_t n);   // caller holds mu; waits for an in-flight DMA first
    ~Staging();
};

// Pinned host blocks for device-to-host result copies, cached by size class
// (so a result can be copied back asynchronously without a hipHostMalloc per
// score).
struct PinnedPool {
    std::mutex mu;
    std::vector<std::pair<size_t, void *>> free_blocks;  // (bytes, ptr)
    size_t cached = 0;
    // bytes held by tasks' packed tables (PinnedBlock with `packed`): kept
    // below what the cache takes back, so that returning them frees nothing
    // (hipHostFree waits for the device)
    std::atomic<size_t> packed_bytes{0};
    void *get(size_t n, size_t *got);
    void put(void *p, size_t n);
    ~PinnedPool();
};

// BF16 DTW kernels: frames per row block (one DTW lane per frame row), and the
// column widths of the launch choices.  Items are never split across row
// blocks, so items are <= 64 frames.
constexpr int kFusedRowFrames = 64;
constexpr int kSortedMaxB = 4096;      // largest |B| counted from sorted rows (sorted in LDS)
constexpr int kFusedColFrames = 128;  // default: tile kernel, 128-frame column blocks (the other is 256)
constexpr int kStreamMinCols = 512;   // cols at or above this select the stream kernel
// Units of a group with at least kBandMinCols column blocks go in bands of
// kBandRows row blocks (see ColPlan); smaller groups fit L2 as they are.
constexpr int kBandRows = 16, kBandMinCols = 24;

// Launch choices of the fused kernel: column block width (128 or 256 frames)
// and grid (blocks_per_cu > 0: a persistent grid of that many blocks per CU;
// 0: one block per work unit).  Results do not depend on them.
struct FusedConfig {
    int cols = 0;           // 0: not set
    int blocks_per_cu = 0;
};

// Shape class of a task for tuning the fused kernel.
struct TuneKey {
    int dim_pad = 0, max_len = 0, frames_log2 = 0, path = 0;
    bool operator<(const TuneKey &o) const {
        if (dim_pad != o.dim_pad) return dim_pad < o.dim_pad;
        if (max_len != o.max_len) return max_len < o.max_len;
        if (frames_log2 != o.frames_log2) return frames_log2 < o.frames_log2;
        return path < o.path;
    }
};

// Best fused-kernel configuration per shape class, filled by fabx_autotune and
// kept in the file named by FABX_AUTOTUNE_CACHE (read at context creation,
// rewritten on each new entry).  Untuned shapes get the default.
class Tuner {
public:
    void load(const std::string &path);
    FusedConfig lookup(const TuneKey &k);
    void record(const TuneKey &k, const FusedConfig &c);
    static FusedConfig default_config() { return FusedConfig{kFusedColFrames, 0}; }

private:
    std::mutex mu_;
    std::string path_;
    std::map<TuneKey, FusedConfig> table_;
    void save_locked();
};

struct CtxImpl {
    int device = 0;
    hipStream_t stream = nullptr;  // borrowed; nullptr = the null stream
    // owned, non-blocking: uploads of task tables, so that the next score's
    // tables travel while the current score's kernels run; `stream` waits for them
    hipStream_t copy_stream = nullptr;
    int n_cu = 0;
    Pool pool;
    EventPool events;
    Staging staging;
    PinnedPool pinned;
    Tuner tuner;
    ~CtxImpl();
};

// A block of a context's pinned pool and the last DMA out of it; the block
// goes back to the pool once that DMA has completed.
struct PinnedBlock {
    std::shared_ptr<CtxImpl> ctx;
    void *p = nullptr;
    size_t cap = 0, bytes = 0;
    hipEvent_t done = nullptr;  // from ctx->events, recorded after the DMA
    bool packed = false;        // counted in ctx->pinned.packed_bytes (cap bytes)
    PinnedBlock(std::shared_ptr<CtxImpl> c, size_t n);
    PinnedBlock(const PinnedBlock &) = delete;
    PinnedBlock &operator=(const PinnedBlock &) = delete;
    ~PinnedBlock();
};

struct DatasetImpl {
    std::shared_ptr<CtxImpl> ctx;
    const void *features = nullptr;   // borrowed device pointer
    int dtype = FABX_DTYPE_F32;
    int64_t n_frames = 0;
    int dim = 0;
    int64_t n_items = 0;
    int n_attr = 0;
    int max_len = 0;
    std::vector<int64_t> item_start;  // [n_items]: first frame of each item
    std::vector<int32_t> item_len;    // [n_items]: its frames (>= 1); items may overlap
    std::vector<int32_t> attrs;       // [n_items * n_attr]
};

// One BY group that holds at least one cell.  Items of a group are
// contiguous in task order, and so are their packed frames.
struct Group {
    int64_t item0;      // first task item
    int64_t n_items;
    int64_t frame0;     // first packed frame
    int64_t n_frames;
    int64_t pair_base;  // offset of the group's [n_items x n_items] pair matrix
};

// A cell on the device: item positions are local to the group.
struct CellDev {
    int32_t group;
    int32_t a0, na;
    int32_t b0, nb;
    int32_t x0, nx;
    int32_t exclude_self;  // X is A: skip a == x
};
static_assert(sizeof(CellDev) == 32, "CellDev layout");

// Device copy of the task tables: one buffer, uploaded with one copy on the
// task's first score; the pointers below point into it.
// Byte offsets of the task tables in their device buffer.
struct TableLayout {
    size_t item_src = 0, item_len = 0, item_dst = 0, item_group = 0;
    std::array<size_t, 5> g{};  // item0, n_items (+ sentinel), frame0, n_frames, pair_base (+ total)
    size_t cells = 0, units = 0, rb = 0, g_rb0 = 0;
    std::array<size_t, 5> plan{};  // cb, unit_prefix, g_cb0, rb_cstart, band_rb of `plan_cols`
    int plan_cols = 0;             // 0: no column plan in the buffer
};

struct TaskDevice {
    DevBuf blob;
    const int64_t *item_src = nullptr, *item_dst = nullptr;
    const int32_t *item_len = nullptr, *item_group = nullptr;
    const int64_t *g_item0 = nullptr, *g_n = nullptr, *g_frame0 = nullptr, *g_nframes = nullptr,
                  *g_pair_base = nullptr;
    const CellDev *cells = nullptr;
    const int32_t *units = nullptr, *rb = nullptr, *g_rb0 = nullptr;
    bool uploaded = false;
};

// Device workspace kept by a task between scores.
struct Workspace {
    DevBuf xn;          // packed normalised frames (F32 or BF16) [n_frames x dim_pad]
    DevBuf rinv;        // F32 [n_frames]: 1 / ||bf16 frame|| (BF16 form)
    DevBuf dmat;        // plain form: F32 frame distances of one batch of group strips
    DevBuf p32;         // F32 [n_pair_slots]
    DevBuf flags;       // uint8 [n_pair_slots]: bit0 non-robust, bit1 marked for FP64
    DevBuf p64;         // F64 [n_pair_slots]
    DevBuf half_units;  // uint64 [n_cells], then the score's 64 counter bytes
    DevBuf finfo;       // uint32 [n_frames]: frame info of the stream kernel
    DevBuf flen;        // F32 [rows]: frame (or mean) lengths (Euclidean BF16 form)
    DevBuf recheck_list, recount_list;
    size_t total() const;
    void release();
};

struct ResultImpl;

// Work plan of the BF16 DTW kernel for one launch choice `cols`.
//  cols 128 / 256 (tile kernel): column blocks of whole items packed into
//    <= cols frames per group, and the work units (row block x column block)
//    they make with the task's row blocks (below).
//  cols 512 / 1024 / 2048 (stream kernel): each row block's column stream
//    (the group's frames from the row block's first frame on) cut into
//    segments of about `cols` frames; only unit_prefix (segments per row
//    block) and cells are used.
struct ColPlan {
    int cols = 0;
    hvec<int32_t> cb;                    // [n_cb][4] = group, first item (task), n items, n frames
    std::vector<int32_t> g_cb0, g_ncb;   // per group: first column block, count
    // Work units: the (row block, column block) pairs of a group whose column
    // block ends after the row block's first item.  A group's pair matrix is
    // symmetric, so the units wholly below its diagonal are not computed: the
    // kernel writes each pair (x, y) with x before y, or x = y, at both (x, y)
    // and (y, x).  Per row block: its first kept column block (counted in the
    // group).
    hvec<int32_t> rb_cstart;             // [n_rb]
    // Order of the units (tile kernel): bands of up to kBandRows consecutive
    // row blocks of one group (band b = row blocks [band_rb[b], band_rb[b+1])),
    // each band's units by column block, then row block, from its first row
    // block's first kept column block on, so that the units in flight share a
    // few row and column blocks in L2.  A unit whose column block comes before
    // its own row block's first kept one is skipped by the kernel.
    // unit_prefix: units per band, prefix; stream kernel: segments per row
    // block, prefix (band_rb empty).
    hvec<int32_t> band_rb;               // [n_bands + 1]
    hvec<int64_t> unit_prefix;           // [n_bands + 1], stream kernel [n_rb + 1]
    int64_t cells = 0;                   // frame pairs the kept units cover (stream kernel: lanes x
                                         // stream columns, 64 per column)
    DevBuf dev;                          // device copy of the above, made on first use
    const int32_t *d_cb = nullptr, *d_g_cb0 = nullptr, *d_rb_cstart = nullptr, *d_band_rb = nullptr;
    const int64_t *d_unit_prefix = nullptr;
};

struct TaskImpl {
    std::shared_ptr<DatasetImpl> ds;
    int32_t on = 0;
    std::vector<int32_t> by, across;
    std::vector<int32_t> key_attr;  // attribute behind each key column
    int32_t key_width = 0;

    // task items (those in groups with cells), in task order
    hvec<int64_t> items;     // original ids
    hvec<int32_t> item_len;
    hvec<int64_t> item_src;  // first source frame
    hvec<int64_t> item_dst;  // first packed frame
    hvec<int32_t> item_group;
    hvec<int64_t> item_pos_of;  // original id -> task position, -1 if absent

    hvec<Group> groups;
    hvec<CellDev> cells;
    hvec<int64_t> n_triplets;
    std::vector<std::vector<int32_t>> key_values;  // per key column: attribute value of each rank
    hvec<uint32_t> rkeys;    // [n_cells * key_width]: dense ranks of the key values
                             // (cell keys are key_values[c][rank]; collapse works on ranks)
    std::vector<int> key_bits;      // bits of each key column's ranks
    std::vector<uint32_t> key_card; // distinct values of each key column (ranks are 0 .. card - 1)

    // work plans, fixed for the task
    hvec<int32_t> units;     // triplet units [n][3]: cell, x_begin, x_end; the first
                             // n_units_small are counted by brute force, the rest
                             // (one x each, large cells) from sorted rows
    int64_t n_units_small = 0;
    int64_t sum_nx = 0;             // sum over cells of |X|
    hvec<int32_t> rb;               // fused kernel row blocks [n][4] (<= 64 frames)
    std::vector<int64_t> long_slots;  // pair slots with an item of more than 64 frames (FP64 kernel)
    std::vector<int32_t> g_rb0, g_nrb;
    std::vector<std::unique_ptr<ColPlan>> col_plans;  // by column block width, made on demand
    int64_t fused_cells = 0;        // frame pairs the fused kernel covers

    int64_t n_frames = 0;
    int64_t n_pair_slots = 0;       // sum over groups of n_items^2
    int64_t n_dmat = 0;             // sum over groups of n_frames^2 (frame pairs of the plain form)
    int64_t n_pairs_needed = 0;     // unique ordered pairs some cell uses
    int64_t dtw_cells_needed = 0;   // sum of len(x) * len(y) over those pairs
    int64_t dtw_cells_sym = 0;      // the same over unordered pairs {x, y} needed in either order
    int64_t total_triplets = 0;
    int max_len = 0;
    bool subsampled = false;        // made by the Subsampler: items may repeat across groups

    TaskDevice dev;
    // device tables packed in pinned memory when the task is made (tables up
    // to a few tens of MB), so that the first score only enqueues their DMA
    std::unique_ptr<PinnedBlock> packed;
    TableLayout packed_layout;
    Workspace ws;
    std::mutex mu;                  // one score launch at a time per task
    std::weak_ptr<ResultImpl> pending;  // the score whose kernels may still use ws
};

struct PendingScore;  // launched work of a score not finished yet (score.cpp)

struct ResultImpl {
    std::shared_ptr<TaskImpl> task;
    hvec<int64_t> half_units;
    fabx_stats stats{};
    bool has_pairs = false;
    hvec<float> p32;
    hvec<uint8_t> flags;
    hvec<double> p64;
    FusedConfig fused;  // fused kernel configuration used (BF16 DTW)
    // Completion: a launched score stays pending until finish_score; its
    // status (an error found on completion) is kept and reported again.
    std::mutex mu;
    std::unique_ptr<PendingScore> pending;
    int status = FABX_OK;
    std::string status_msg;
    ResultImpl();
    ~ResultImpl();
};

// task.cpp
// Cell keys (attribute values) of cells [0, n) into out [n * key_width].
void cell_keys(const TaskImpl &t, int32_t *out);
// The task's column plan for `cols` (128 or 256), built on first use; the caller
// holds the task's mutex.
ColPlan &col_plan(TaskImpl &t, int cols);
// score.cpp: packs the task's device tables (and its default column plan) into
// a pinned block of the context, for a task on a device context.
void prepack_tables(TaskImpl &t);
std::shared_ptr<TaskImpl> build_task(const std::shared_ptr<DatasetImpl> &ds, int32_t on,
                                     const int32_t *by, int32_t n_by, const int32_t *across,
                                     int32_t n_across);
// Row blocks of the DTW kernels and the default work plan, from the task's
// groups and items (the last step of a task build).
void plan_blocks(TaskImpl &t);
// subsample.cpp: the task the Subsampler makes from a full task `t`.
std::shared_ptr<TaskImpl> subsample_task(const TaskImpl &t, const fabx_subsampler &sub);

// score.cpp
struct ScoreParams {
    int mode, precision, dtw_norm;
    int distance;  // FABX_DISTANCE_*
    double margin, delta;
    bool keep_pairs;
    FusedConfig fused;  // cols > 0: use this instead of the tuning table
};
ScoreParams resolve_opts(const fabx_score_opts *opts, const DatasetImpl &ds);
TuneKey tune_key(const TaskImpl &t, const ScoreParams &p);
// launch_score enqueues the whole score on `stream` and returns a pending
// result; finish_score waits for it and fills the result (idempotent, throws
// the score's error every time it is called on a failed result).  run_score
// is both.
std::shared_ptr<ResultImpl> launch_score(const std::shared_ptr<TaskImpl> &task, const ScoreParams &p,
                                         hipStream_t stream);
void finish_score(ResultImpl &res);
std::shared_ptr<ResultImpl> run_score(const std::shared_ptr<TaskImpl> &task, const ScoreParams &p,
                                      hipStream_t stream);
// Device bytes a score of this task would hold (admission control).
int64_t footprint_bytes(const TaskImpl &task, const ScoreParams &p);
// The whole score of fabx_score with every device buffer (task tables, column
// plan, workspace) laid out in `base` [cap bytes] instead of the context's
// pool: allocates no device or pinned memory.  Synchronous on `stream`; per-cell
// counts into host half_units [n_cells]; stats (may be null) without stage
// times.  ENOMEM if the task needs more than `cap` bytes.
void score_in_scratch(TaskImpl &task, const ScoreParams &p, char *base, size_t cap, hipStream_t stream,
                      int64_t *half_units, fabx_stats *stats);
// noalloc.hip: device address of the fabx_score_noalloc scratch array on
// `device` (looked up once per device, with that device current).
char *scratch_setup(int device);
// Gives the task's device memory (workspace, tables, column plans) and its
// pinned packed tables back to the context's pools, after waiting for its
// pending score.  A later score uploads the tables again.
void release_device(TaskImpl &task);

// collapse.cpp
double collapse(const ResultImpl &res, const int32_t *level_attr, const int32_t *level_len,
                int32_t n_levels);

}  // namespace fabx

// Opaque handle types of the C ABI.
struct fabx_ctx {
    std::shared_ptr<fabx::CtxImpl> p;
};
struct fabx_dataset {
    std::shared_ptr<fabx::DatasetImpl> p;
};
struct fabx_task {
    std::shared_ptr<fabx::TaskImpl> p;
};
struct fabx_result {
    std::shared_ptr<fabx::ResultImpl> p;
};
