// Score orchestration: device tables, workspace, work plans and the launch
// sequence of one fabx_score call.
#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <exception>

#include "host_pool.h"
#include "kernels.h"

namespace fabx {

namespace {

// Default near-tie margin and DTW path-length window of the BF16 form, as
// k / sqrt(dim): rounding unit vectors to BF16 (8-bit mantissa) perturbs a
// cosine by about 2^-9 * sqrt(2 / dim) (one sigma), i.e. about 1e-3 / sqrt(dim)
// in theta / pi at typical angles.  The margin must exceed twice the largest
// pair-distance error (so a comparison decided outside it is right), the
// window twice the largest cumulative-cost error; both constants leave a
// wide safety factor over the errors measured by the parity tests.
constexpr double kMarginK = 2e-2;
constexpr double kDeltaK = 4e-2;
constexpr double kPi = 3.14159265358979323846;
int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

// Collects host arrays (256-byte aligned pieces) into one layout.  copy_to
// writes them to pinned memory (a task's packed block, made when the task is
// built); upload sends them to one device buffer with a single DMA copy
// through the context's pinned staging buffer.  Either copy runs on the
// context's copy stream and the compute stream waits for it.  The destination
// is a buffer of this task or score, so no earlier kernel still on the compute
// stream can be reading it.
struct Packer {
    struct Piece {
        const void *src;
        size_t bytes, off;
    };
    std::vector<Piece> pieces;
    size_t total = 0;
    template <typename T>
    size_t add(const T *p, size_t n) {
        const size_t off = (total + 255) & ~size_t(255);
        pieces.push_back({p, n * sizeof(T), off});
        total = off + std::max<size_t>(n * sizeof(T), 16);
        return off;
    }
    template <typename T, typename A>
    size_t add(const std::vector<T, A> &v) { return add(v.data(), v.size()); }
    // host copy of all pieces to h [total], in 1 MiB slices on the host pool
    void copy_to(char *h) const {
        constexpr size_t kSlice = size_t(1) << 20;
        std::vector<std::pair<size_t, size_t>> slices;  // (piece, offset in piece)
        for (size_t i = 0; i < pieces.size(); ++i)
            for (size_t o = 0; o < pieces[i].bytes; o += kSlice) slices.push_back({i, o});
        HostPool::get().parallel_for(int(slices.size()), [&](int k) {
            const Piece &p = pieces[slices[size_t(k)].first];
            const size_t o = slices[size_t(k)].second;
            std::memcpy(h + p.off + o, static_cast<const char *>(p.src) + o, std::min(kSlice, p.bytes - o));
        });
    }
    void upload(DevBuf &dst, Staging &stg, hipStream_t copy, hipStream_t compute) {
        dst.ensure(total);
        std::lock_guard<std::mutex> lk(stg.mu);
        stg.reserve(total);
        char *h = static_cast<char *>(stg.host);
        copy_to(h);
        FABX_HIP(hipMemcpyAsync(dst.ptr, h, total, hipMemcpyHostToDevice, copy));
        FABX_HIP(hipEventRecord(stg.done, copy));
        stg.in_flight = true;  // the next upload waits for this DMA before reusing the buffer
        FABX_HIP(hipStreamWaitEvent(compute, stg.done, 0));
    }
    template <typename T>
    static const T *at(const DevBuf &b, size_t off) {
        return reinterpret_cast<const T *>(b.as<char>() + off);
    }
};

// Host side of the task tables: adds them (and `plan`, if any) to `pk`; the
// group columns are built in `gcols`, which must live until the copy is made.
TableLayout add_task_tables(const TaskImpl &t, const ColPlan *plan, Packer &pk,
                            std::array<std::vector<int64_t>, 5> &gcols) {
    const size_t G = t.groups.size();
    for (auto &v : gcols) v.resize(G);
    gcols[1].resize(G + 1);
    gcols[4].resize(G + 1);
    for (size_t i = 0; i < G; ++i) {
        const Group &g = t.groups[i];
        gcols[0][i] = g.item0;
        gcols[1][i] = g.n_items;
        gcols[2][i] = g.frame0;
        gcols[3][i] = g.n_frames;
        gcols[4][i] = g.pair_base;
    }
    gcols[1][G] = 0;
    gcols[4][G] = t.n_pair_slots;
    TableLayout L;
    L.item_src = pk.add(t.item_src);
    L.item_len = pk.add(t.item_len);
    L.item_dst = pk.add(t.item_dst);
    L.item_group = pk.add(t.item_group);
    for (size_t k = 0; k < 5; ++k) L.g[k] = pk.add(gcols[k]);
    L.cells = pk.add(t.cells);
    L.units = pk.add(t.units);
    L.rb = pk.add(t.rb);
    L.g_rb0 = pk.add(t.g_rb0);
    if (plan) {
        L.plan = {pk.add(plan->cb), pk.add(plan->unit_prefix), pk.add(plan->g_cb0), pk.add(plan->rb_cstart),
                  pk.add(plan->band_rb)};
        L.plan_cols = plan->cols;
    }
    return L;
}

void set_col_plan(ColPlan &cp, const DevBuf &buf, const std::array<size_t, 5> &o) {
    cp.d_cb = Packer::at<int32_t>(buf, o[0]);
    cp.d_unit_prefix = Packer::at<int64_t>(buf, o[1]);
    cp.d_g_cb0 = Packer::at<int32_t>(buf, o[2]);
    cp.d_rb_cstart = Packer::at<int32_t>(buf, o[3]);
    cp.d_band_rb = Packer::at<int32_t>(buf, o[4]);
}

// Device pointers of the task tables in dv.blob (and of the column plan packed
// with them).
void set_task_tables(TaskImpl &t, const TableLayout &L) {
    TaskDevice &dv = t.dev;
    dv.item_src = Packer::at<int64_t>(dv.blob, L.item_src);
    dv.item_len = Packer::at<int32_t>(dv.blob, L.item_len);
    dv.item_dst = Packer::at<int64_t>(dv.blob, L.item_dst);
    dv.item_group = Packer::at<int32_t>(dv.blob, L.item_group);
    dv.g_item0 = Packer::at<int64_t>(dv.blob, L.g[0]);
    dv.g_n = Packer::at<int64_t>(dv.blob, L.g[1]);
    dv.g_frame0 = Packer::at<int64_t>(dv.blob, L.g[2]);
    dv.g_nframes = Packer::at<int64_t>(dv.blob, L.g[3]);
    dv.g_pair_base = Packer::at<int64_t>(dv.blob, L.g[4]);
    dv.cells = Packer::at<CellDev>(dv.blob, L.cells);
    dv.units = Packer::at<int32_t>(dv.blob, L.units);
    dv.rb = Packer::at<int32_t>(dv.blob, L.rb);
    dv.g_rb0 = Packer::at<int32_t>(dv.blob, L.g_rb0);
    if (L.plan_cols)
        for (auto &cp : t.col_plans)
            if (cp->cols == L.plan_cols && !cp->d_cb) set_col_plan(*cp, dv.blob, L.plan);
}

// Task tables larger than this are sent through the staging buffer on the
// first score instead of being packed when the task is made; so are those of
// a task made while other tasks' packed tables already hold kPrepackBudget.
constexpr size_t kPrepackMaxBytes = size_t(64) << 20;
constexpr size_t kPrepackBudget = size_t(128) << 20;

// Gram tile prefix per group for the pooled mode (64 x 64 FP32 or 64 x 128
// BF16 tiles of items).
std::vector<int64_t> tile_prefix(const TaskImpl &t, const ScoreParams &p) {
    const bool bf16 = p.precision == FABX_PREC_BF16_RECHECK;
    const int64_t G = int64_t(t.groups.size());
    std::vector<int64_t> pre(size_t(G) + 1, 0);
    for (int64_t gi = 0; gi < G; ++gi) {
        const int64_t n = t.groups[size_t(gi)].n_items;
        const int64_t tr = (n + 63) / 64;
        const int64_t tc = bf16 ? (n + 127) / 128 : tr;
        pre[size_t(gi) + 1] = pre[size_t(gi)] + tr * tc;
    }
    return pre;
}

// Frame distances of the plain DTW form, per batch of strips: a strip is the
// frames of consecutive items of one group (rows) against all the group's
// frames (columns).  A group whose squared frame count fits `cap` cells is one
// strip; consecutive strips form a batch while their matrices total at most
// `cap` cells, so the distance buffer never holds more than that.
struct PlainPlan {
    // per strip; slot0 and tiles are prefixes with one more entry
    std::vector<int64_t> group, slot0, row0, nrows, col0, ncols, base, tiles;
    std::vector<std::pair<int64_t, int64_t>> batches;                          // strip ranges
    int64_t max_cells = 0;                                                     // largest batch
};

PlainPlan plain_plan(const TaskImpl &t, int64_t cap) {
    PlainPlan pl;
    pl.tiles.push_back(0);
    int64_t batch_cells = 0, batch_first = 0;
    // strip of group g: its items from local position x0 on, rows r0 .. r0 + nr - 1
    auto add_strip = [&](size_t g, int64_t x0, int64_t r0, int64_t nr) {
        const Group &gr = t.groups[g];
        const int64_t cells = nr * gr.n_frames;
        const int64_t k = int64_t(pl.group.size());
        if (batch_cells > 0 && batch_cells + cells > cap) {
            pl.batches.push_back({batch_first, k});
            batch_first = k;
            batch_cells = 0;
        }
        pl.group.push_back(int64_t(g));
        pl.slot0.push_back(gr.pair_base + x0 * gr.n_items);
        pl.row0.push_back(r0);
        pl.nrows.push_back(nr);
        pl.col0.push_back(gr.frame0);
        pl.ncols.push_back(gr.n_frames);
        pl.base.push_back(batch_cells);
        pl.tiles.push_back(pl.tiles.back() + ((nr + 63) / 64) * ((gr.n_frames + 63) / 64));
        batch_cells += cells;
        pl.max_cells = std::max(pl.max_cells, batch_cells);
    };
    for (size_t g = 0; g < t.groups.size(); ++g) {
        const Group &gr = t.groups[g];
        const int64_t rows_cap = std::max<int64_t>(1, cap / std::max<int64_t>(gr.n_frames, 1));
        int64_t x0 = 0, r0 = gr.frame0, nr = 0;
        for (int64_t k = 0; k < gr.n_items; ++k) {
            const int64_t L = t.item_len[size_t(gr.item0 + k)];
            if (nr > 0 && nr + L > rows_cap) {
                add_strip(g, x0, r0, nr);
                x0 = k;
                r0 += nr;
                nr = 0;
            }
            nr += L;
        }
        add_strip(g, x0, r0, nr);
    }
    if (!pl.group.empty()) pl.batches.push_back({batch_first, int64_t(pl.group.size())});
    pl.slot0.push_back(t.n_pair_slots);  // n + 1 entries: the slots of strip k are [slot0[k], slot0[k+1])
    return pl;
}

// Cells (4 bytes each) of the plain form's distance buffer: 4 GiB.  The
// environment variable FABX_PLAIN_DMAT_CELLS (read when a score starts, at
// least 4096) sets another size, so that small tasks can run in many batches.
constexpr int64_t kPlainDmatCells = int64_t(1) << 30;
int64_t plain_dmat_cells() {
    if (const char *e = std::getenv("FABX_PLAIN_DMAT_CELLS")) {
        const long long v = std::atoll(e);
        if (v >= 4096) return int64_t(v);
    }
    return kPlainDmatCells;
}

struct Timer {
    hipEvent_t ev[8];
    int n = 0;
    hipStream_t s;
    EventPool &pool;
    Timer(hipStream_t st, EventPool &p) : s(st), pool(p) {
        for (auto &e : ev) e = pool.get();
    }
    ~Timer() {
        for (auto &e : ev) pool.put(e);
    }
    void mark() { FABX_HIP(hipEventRecord(ev[n++], s)); }
    double ms(int a, int b) {
        float v = 0.f;
        FABX_HIP(hipEventElapsedTime(&v, ev[a], ev[b]));
        return double(v);
    }
};

}  // namespace

ScoreParams resolve_opts(const fabx_score_opts *opts, const DatasetImpl &ds) {
    fabx_score_opts o;
    fabx_score_opts_default(&o);
    if (opts) o = *opts;
    if (o.distance != FABX_DISTANCE_ANGULAR && o.distance != FABX_DISTANCE_EUCLIDEAN &&
        o.distance != FABX_DISTANCE_UNITS)
        fail(FABX_EINVAL, "bad distance");
    // discrete units: the 0 / 1 mismatch of unit codes, in DTW mode only; the
    // costs are exact integers, so the scores take the plain kernels and every
    // comparison is exact (no BF16 stage, nothing to recheck)
    const bool units = ds.dtype == FABX_DTYPE_UNITS;
    if (units != (o.distance == FABX_DISTANCE_UNITS))
        fail(FABX_EINVAL, "FABX_DISTANCE_UNITS goes with FABX_DTYPE_UNITS datasets, and only with them");
    if (units && o.mode != FABX_MODE_DTW) fail(FABX_EINVAL, "discrete units are scored in DTW mode only");
    if (units) o.precision = FABX_PREC_FP32;
    if (o.mode != FABX_MODE_DTW && o.mode != FABX_MODE_POOLED) fail(FABX_EINVAL, "bad mode");
    if (o.precision != FABX_PREC_FP32 && o.precision != FABX_PREC_BF16_RECHECK)
        fail(FABX_EINVAL, "bad precision");
    if (o.dtw_norm != FABX_NORM_PATH && o.dtw_norm != FABX_NORM_NONE) fail(FABX_EINVAL, "bad dtw_norm");
    if (std::isnan(o.margin) || std::isnan(o.delta)) fail(FABX_EINVAL, "margin / delta is NaN");
    ScoreParams p;
    p.mode = o.mode;
    p.precision = o.precision;
    p.dtw_norm = o.dtw_norm;
    p.distance = o.distance;
    // the raw DTW cost (FABX_NORM_NONE) sums up to 2 L - 1 frame distances
    // (L: the longest item the BF16 kernels take; pairs of longer items are
    // computed in FP64), each with its own error: its default margin is that
    // many times the per-distance one
    const double path_cells = p.mode == FABX_MODE_DTW && p.dtw_norm == FABX_NORM_NONE
                                  ? double(2 * std::clamp(ds.max_len, 1, kFusedRowFrames) - 1) : 1.0;
    // BF16 form of the Euclidean distance: margin and delta are in units of the
    // largest frame (or mean) length S, and an angle error e moves a frame
    // distance by at most S e, so the angular bounds are scaled by pi (the
    // angular distance being the angle / pi)
    const double unit = p.distance == FABX_DISTANCE_EUCLIDEAN ? kPi : 1.0;
    p.margin = o.margin < 0 ? unit * kMarginK / std::sqrt(double(ds.dim)) * path_cells : o.margin;
    p.delta = o.delta < 0 ? unit * kDeltaK / std::sqrt(double(ds.dim)) : o.delta;
    p.keep_pairs = o.keep_pairs != 0;
    if (o.fused_cols != 0 && o.fused_cols != 128 && o.fused_cols != 256 && o.fused_cols != 512 &&
        o.fused_cols != 1024 && o.fused_cols != 2048)
        fail(FABX_EINVAL, "fused_cols must be 0, 128, 256, 512, 1024 or 2048");
    if (o.fused_blocks_per_cu < 0 || o.fused_blocks_per_cu > 64)
        fail(FABX_EINVAL, "fused_blocks_per_cu must be in 0..64");
    p.fused = FusedConfig{o.fused_cols, o.fused_blocks_per_cu};  // cols 0: the tuning table
    if (p.mode == FABX_MODE_DTW && ds.max_len > FABX_MAX_ITEM_FRAMES)
        fail(FABX_EINVAL, "an item is longer than FABX_MAX_ITEM_FRAMES frames (DTW mode)");
    if (p.mode == FABX_MODE_DTW && p.fused.cols >= kStreamMinCols && ds.max_len > kFusedRowFrames)
        fail(FABX_EINVAL, "the streaming DTW kernel (fused_cols >= 512) takes items of at most 64 frames");
    if (p.fused.cols >= kStreamMinCols && p.distance == FABX_DISTANCE_EUCLIDEAN)
        fail(FABX_EINVAL, "the streaming DTW kernel (fused_cols >= 512) computes the angular distance only");
    if (ds.dim > 2048) fail(FABX_EINVAL, "feature dim above 2048 is not supported");
    return p;
}

int64_t footprint_bytes(const TaskImpl &t, const ScoreParams &p) {
    const bool bf16 = p.precision == FABX_PREC_BF16_RECHECK;
    const int64_t dim_pad = round_up(t.ds->dim, 64);
    const int64_t rows = p.mode == FABX_MODE_DTW ? t.n_frames : int64_t(t.items.size());
    int64_t b = p.distance == FABX_DISTANCE_UNITS ? rows * 4 : rows * dim_pad * (bf16 ? 2 : 4) + rows * 4;
    if (bf16 && p.distance == FABX_DISTANCE_EUCLIDEAN) b += rows * 4;  // frame lengths
    if (p.mode == FABX_MODE_DTW && !bf16) b += std::min(t.n_dmat, plain_dmat_cells()) * 4;
    b += t.n_pair_slots * 4;
    if (bf16) b += t.n_pair_slots * (1 + 8 + 8) + int64_t(t.long_slots.size()) * 8;
    b += int64_t(t.cells.size()) * (8 + 32) + int64_t(t.units.size()) * 4 + t.sum_nx * 8 +
         int64_t(t.items.size()) * 24;
    return b + (1 << 20);
}

size_t Workspace::total() const {
    const DevBuf *all[] = {&xn, &rinv, &dmat, &p32, &flags, &p64, &half_units,
                           &recheck_list, &recount_list, &finfo, &flen};
    size_t s = 0;
    for (auto *b : all) s += b->bytes;
    return s;
}

void Workspace::release() {
    DevBuf *all[] = {&xn, &rinv, &dmat, &p32, &flags, &p64, &half_units,
                     &recheck_list, &recount_list, &finfo, &flen};
    for (auto *b : all) b->release();
}

// Launched work of a score, kept until finish_score.
struct PendingScore {
    std::shared_ptr<TaskImpl> task;
    std::shared_ptr<CtxImpl> ctx;
    hipStream_t stream = nullptr;
    std::unique_ptr<Timer> tm;
    DevBuf plan_d;                 // Gram tile prefix read by the plain / pooled kernels
    void *host = nullptr;          // pinned: half_units [n_cells] then 64 counter bytes
    size_t host_bytes = 0;
    std::unique_ptr<PinnedBlock> packed;  // the task's packed tables, if this score sent them
    bool bf16 = false, dtw = false, keep_pairs = false;
    std::chrono::steady_clock::time_point t_enter, t_launch;
    ~PendingScore() {
        if (host) ctx->pinned.put(host, host_bytes);
    }
};

ResultImpl::ResultImpl() = default;

ResultImpl::~ResultImpl() {
    // a result dropped while its kernels run must not let the memory go first
    try {
        finish_score(*this);
    } catch (...) {
    }
}

void prepack_tables(TaskImpl &t) {
    const std::shared_ptr<CtxImpl> &ctx = t.ds->ctx;
    if (!ctx || ctx->device < 0 || t.cells.empty()) return;
    Trace tr("prepack");
    Packer pk;
    std::array<std::vector<int64_t>, 5> gcols;
    const ColPlan *plan = t.col_plans.empty() ? nullptr : t.col_plans.front().get();
    const TableLayout L = add_task_tables(t, plan, pk, gcols);
    if (pk.total > kPrepackMaxBytes || ctx->pinned.packed_bytes.load() + pk.total > kPrepackBudget) return;
    FABX_HIP(hipSetDevice(ctx->device));
    std::unique_ptr<PinnedBlock> blk;
    try {
        blk = std::make_unique<PinnedBlock>(ctx, pk.total);
    } catch (const Error &) {
        return;  // no pinned memory to spare: the first score sends the tables through the staging buffer
    }
    blk->packed = true;
    ctx->pinned.packed_bytes += blk->cap;
    blk->bytes = pk.total;
    tr.mark("alloc");
    pk.copy_to(static_cast<char *>(blk->p));
    tr.mark("copy");
    t.packed = std::move(blk);
    t.packed_layout = L;
}

namespace {

// Device addresses a score's kernels use: the task tables, the column plan of
// the fused kernel, the plan of the pooled / plain kernels, and the workspace.
struct DevPtrs {
    kern::ItemTables it{};
    kern::GroupTables gt{};
    const CellDev *cells = nullptr;
    const int32_t *units = nullptr, *rb = nullptr, *item_group = nullptr;
    const int32_t *cb = nullptr, *g_cb0 = nullptr, *rb_cstart = nullptr;
    const int32_t *band_rb = nullptr;
    const int64_t *unit_prefix = nullptr;
    const int64_t *tiles = nullptr;             // pooled: Gram tile prefix per group
    const int64_t *long_slots = nullptr;        // BF16 DTW: slots of pairs with an item over 64 frames
    std::array<const int64_t *, 8> strips{};    // plain DTW: group, slot0, row0, nrows, col0, ncols, base, tiles
    void *xn = nullptr;
    float *rinv = nullptr, *dmat = nullptr, *p32 = nullptr;
    uint8_t *flags = nullptr;
    double *p64 = nullptr;
    int64_t *recheck_list = nullptr;
    int32_t *recount_list = nullptr;
    unsigned long long *half_units = nullptr;   // [n_cells], then the score's 64 counter bytes
    uint32_t *finfo = nullptr;                  // stream kernel: frame info [n_frames]
    float *flen = nullptr;                      // Euclidean BF16 form: frame (or mean) lengths
};

// Byte offsets of the pooled tile prefix or of the plain form's strip columns.
struct PlanLayout {
    size_t tiles = 0, long_slots = 0;
    std::array<size_t, 8> strips{};
    bool has_tiles = false, has_strips = false, has_long = false;
};

PlanLayout add_plan(Packer &pk, const std::vector<int64_t> &tiles, const PlainPlan &strips,
                    const std::vector<int64_t> &long_slots) {
    PlanLayout L;
    if (!long_slots.empty()) {
        L.long_slots = pk.add(long_slots);
        L.has_long = true;
    }
    if (!tiles.empty()) {
        L.tiles = pk.add(tiles);
        L.has_tiles = true;
    }
    if (!strips.group.empty()) {
        const std::vector<int64_t> *cols[8] = {&strips.group, &strips.slot0, &strips.row0, &strips.nrows,
                                               &strips.col0,  &strips.ncols, &strips.base, &strips.tiles};
        for (size_t k = 0; k < 8; ++k) L.strips[k] = pk.add(*cols[k]);
        L.has_strips = true;
    }
    return L;
}

void set_plan(DevPtrs &d, const char *base, const PlanLayout &L) {
    if (L.has_tiles) d.tiles = reinterpret_cast<const int64_t *>(base + L.tiles);
    if (L.has_long) d.long_slots = reinterpret_cast<const int64_t *>(base + L.long_slots);
    if (L.has_strips)
        for (size_t k = 0; k < 8; ++k) d.strips[k] = reinterpret_cast<const int64_t *>(base + L.strips[k]);
}

// Workspace bytes of one score (0 for buffers the form does not use).
struct WorkspaceSizes {
    size_t xn = 0, rinv = 0, dmat = 0, p32 = 0, flags = 0, p64 = 0, recheck_list = 0, recount_list = 0,
           half_units = 0, finfo = 0, flen = 0;
    size_t total_aligned() const {
        size_t s = 0;
        for (size_t b : {xn, rinv, dmat, p32, flags, p64, recheck_list, recount_list, half_units, finfo, flen})
            s += (b + 255) & ~size_t(255);
        return s;
    }
};

WorkspaceSizes workspace_sizes(const TaskImpl &t, const ScoreParams &p, const PlainPlan &strips, bool stream) {
    const bool bf16 = p.precision == FABX_PREC_BF16_RECHECK;
    const bool dtw = p.mode == FABX_MODE_DTW;
    const int64_t dim_pad = round_up(t.ds->dim, 64);
    const int64_t rows = dtw ? t.n_frames : int64_t(t.items.size());
    WorkspaceSizes w;
    w.xn = p.distance == FABX_DISTANCE_UNITS ? size_t(rows) * 4  // packed codes
                                             : size_t(rows) * size_t(dim_pad) * (bf16 ? 2 : 4);
    if (bf16) w.rinv = size_t(rows) * 4;
    if (dtw && !bf16) w.dmat = size_t(std::max<int64_t>(strips.max_cells, 1)) * 4;
    w.p32 = size_t(t.n_pair_slots) * 4;
    if (bf16) {
        w.flags = size_t(t.n_pair_slots);
        w.p64 = size_t(t.n_pair_slots) * 8;
        w.recheck_list = size_t(t.n_pair_slots) * 8;
        w.recount_list = size_t(std::max<int64_t>(t.sum_nx, 1)) * 8;
    }
    // per-cell counts, then 64 counter bytes: both come back with one copy
    w.half_units = t.cells.size() * 8 + 64;
    if (stream) w.finfo = size_t(t.n_frames) * 4;
    if (bf16 && p.distance == FABX_DISTANCE_EUCLIDEAN) w.flen = size_t(rows) * 4;
    return w;
}

// Enqueues every kernel of a score on `stream` and the copy of the per-cell
// counts and the 64 counter bytes into `host` [n_cells * 8 + 64].  `tm` (may
// be null) records the stage events 0..6.
void enqueue_score(const TaskImpl &t, const ScoreParams &p, const FusedConfig &fcfg, const ColPlan *cplan,
                   const std::vector<int64_t> &tiles, const PlainPlan &strips, const DevPtrs &d,
                   hipStream_t stream, Timer *tm, void *host, fabx_stats &st) {
    const DatasetImpl &ds = *t.ds;
    const bool bf16 = p.precision == FABX_PREC_BF16_RECHECK;
    const bool dtw = p.mode == FABX_MODE_DTW;
    const bool plain_dtw = dtw && !bf16;
    const int dim = ds.dim;
    const int dim_pad = int(round_up(dim, 64));
    const int64_t n_cells = int64_t(t.cells.size());
    const int64_t n_units = int64_t(t.units.size() / 3);
    const int64_t G = int64_t(t.groups.size());
    const kern::ItemTables &it = d.it;
    const kern::GroupTables &gt = d.gt;
    char *counters = reinterpret_cast<char *>(d.half_units) + size_t(n_cells) * 8;
    int *err = reinterpret_cast<int *>(counters);
    unsigned long long *err_item = reinterpret_cast<unsigned long long *>(counters + 8);
    unsigned int *recount_n = reinterpret_cast<unsigned int *>(counters + 16);
    unsigned int *marked_n = reinterpret_cast<unsigned int *>(counters + 20);
    unsigned int *nonrobust_n = reinterpret_cast<unsigned int *>(counters + 24);
    unsigned int *unit_ctr = reinterpret_cast<unsigned int *>(counters + 32);  // [8]
    const bool euclid = p.distance == FABX_DISTANCE_EUCLIDEAN;
    // Euclidean BF16 form: frame lengths and the largest one (FP32 bits)
    float *flen = bf16 && euclid ? d.flen : nullptr;
    unsigned int *scale = bf16 && euclid ? reinterpret_cast<unsigned int *>(counters + 28) : nullptr;
    auto mark = [&] {
        if (tm) tm->mark();
    };
    mark();  // 0
    kern::init_score(stream, d.half_units, n_cells);
    if (bf16 && !dtw) FABX_HIP(hipMemsetAsync(d.flags, 0, size_t(t.n_pair_slots), stream));
    mark();  // 1
    const int out_form = bf16 ? (euclid ? 3 : 1) : euclid ? 2 : 0;
    const bool units = p.distance == FABX_DISTANCE_UNITS;
    if (units)
        kern::pack_units(stream, static_cast<const int32_t *>(ds.features), it, static_cast<int32_t *>(d.xn));
    else if (dtw)
        kern::normalize(stream, ds.features, ds.dtype, dim, dim_pad, it, d.xn, out_form, d.rinv, err, err_item,
                        flen, scale);
    else
        kern::pool_normalize(stream, ds.features, ds.dtype, dim, dim_pad, it, d.xn, out_form, d.rinv, err,
                             err_item, flen, scale);
    mark();  // 2
    const auto &sp = d.strips;
    if (plain_dtw) {
        // one batch of strips at a time through the distance buffer (stream order
        // keeps a batch's Gram from overwriting the previous batch's DTW input)
        for (const auto &b : strips.batches) {
            const size_t k0 = size_t(b.first);
            const int64_t ns = b.second - b.first;
            const kern::GramSegments seg{sp[2] + k0, sp[3] + k0, sp[4] + k0, sp[5] + k0, sp[6] + k0, sp[7] + k0, ns,
                                         strips.tiles[size_t(b.second)] - strips.tiles[k0]};
            if (units)
                kern::unit_mismatch(stream, static_cast<const int32_t *>(d.xn), seg, d.dmat);
            else
                kern::gram_angular_f32(stream, static_cast<const float *>(d.xn), dim_pad, seg, d.dmat,
                                       euclid ? 1 : 0);
            const kern::PlainStrips ps{sp[0] + k0, sp[1] + k0, sp[2] + k0, sp[6] + k0, ns,
                                       strips.slot0[size_t(b.second)] - strips.slot0[k0]};
            kern::dtw_plain(stream, d.dmat, ps, gt, it, p.dtw_norm, t.max_len > kFusedRowFrames, units, d.p32);
        }
        st.computed_dtw_cells = t.n_dmat;
    } else if (dtw && fcfg.cols >= kStreamMinCols) {
        kern::frame_info(stream, it, d.item_group, gt.item0, d.finfo);
        const kern::StreamPlan sp{d.rb, d.unit_prefix, int64_t(t.rb.size() / 4), cplan->unit_prefix.back(),
                                  fcfg.cols, fcfg.blocks_per_cu, ds.ctx->n_cu};
        const uint32_t delta_q = uint32_t(std::ceil(p.delta * 65535.0));
        kern::stream_bf16(stream, static_cast<const uint16_t *>(d.xn), d.rinv, dim_pad, d.finfo, gt, it, sp,
                          p.dtw_norm, delta_q, d.p32, d.flags, nonrobust_n, unit_ctr);
        st.computed_dtw_cells = cplan->cells;
    } else if (dtw) {
        kern::FusedPlan fp{d.rb, d.cb, d.unit_prefix, d.band_rb, d.g_cb0, d.rb_cstart,
                           int64_t(cplan->band_rb.size()) - 1, cplan->unit_prefix.back(), fcfg.cols,
                           fcfg.blocks_per_cu, ds.ctx->n_cu};
        kern::fused_bf16(stream, static_cast<const uint16_t *>(d.xn), d.rinv, dim_pad, gt, it, fp, p.dtw_norm,
                         float(p.delta), d.p32, d.flags, nonrobust_n, unit_ctr, flen, scale);
        // pairs with an item over 64 frames: FP64 from the raw features
        kern::long_dtw(stream, ds.features, ds.dtype, dim, gt, it, d.long_slots, nullptr,
                       int64_t(t.long_slots.size()), p.dtw_norm, euclid ? 1 : 0, d.p64, d.p32, d.flags);
        st.computed_dtw_cells = cplan->cells;
    } else if (!bf16) {
        const kern::GramSegments seg{gt.item0, gt.n_items, gt.item0, gt.n_items, gt.pair_base, d.tiles, G,
                                     tiles.back()};
        kern::gram_angular_f32(stream, static_cast<const float *>(d.xn), dim_pad, seg, d.p32, euclid ? 1 : 0);
    } else {
        kern::gram_angular_bf16(stream, static_cast<const uint16_t *>(d.xn), d.rinv, dim_pad, gt.item0,
                                gt.n_items, gt.pair_base, d.tiles, G, tiles.back(), d.p32, d.flags, flen);
    }
    mark();  // 3
    uint8_t *flags = bf16 ? d.flags : nullptr;
    int32_t *recount = bf16 ? d.recount_list : nullptr;
    kern::triplets(stream, d.cells, d.units, t.n_units_small, gt, d.p32, d.half_units, flags, float(p.margin),
                   recount, recount_n, t.sum_nx, scale);
    kern::triplets_sorted(stream, d.cells, d.units + 3 * t.n_units_small, n_units - t.n_units_small, gt, d.p32,
                          d.half_units, flags, float(p.margin), recount, recount_n, t.sum_nx, scale);
    mark();  // 4
    if (bf16) {
        kern::collect_marked(stream, d.flags, t.n_pair_slots, d.recheck_list, marked_n, t.n_pair_slots, recount_n);
        kern::recheck_fp64(stream, ds.features, ds.dtype, dim, gt, it, d.recheck_list, marked_n, t.n_pair_slots,
                           p.mode, p.dtw_norm, dtw && t.max_len > kFusedRowFrames, euclid ? 1 : 0, d.p64);
        kern::recount(stream, d.cells, d.recount_list, recount_n, t.sum_nx, gt, d.p32, d.p64, d.flags,
                      d.half_units);
    }
    mark();  // 5
    FABX_HIP(hipMemcpyAsync(host, d.half_units, size_t(n_cells) * 8 + 64, hipMemcpyDeviceToHost, stream));
    mark();  // 6
}

// The score's counters in the host copy (after the per-cell counts): EDOMAIN
// if a zero-norm frame was met, else the recheck / recount / non-robust counts.
void read_counters(const TaskImpl &t, const char *host, size_t n_cells, bool dtw, fabx_stats &st) {
    const unsigned char *counters = reinterpret_cast<const unsigned char *>(host + n_cells * 8);
    int err_h;
    unsigned long long err_item_h;
    unsigned int recount_h, marked_h, nonrobust_h;
    std::memcpy(&err_h, counters, 4);
    std::memcpy(&err_item_h, counters + 8, 8);
    std::memcpy(&recount_h, counters + 16, 4);
    std::memcpy(&marked_h, counters + 20, 4);
    std::memcpy(&nonrobust_h, counters + 24, 4);
    if (err_h) {
        const int64_t bad = err_item_h < uint64_t(t.items.size()) ? t.items[size_t(err_item_h)] : -1;
        fail(FABX_EDOMAIN, "zero-norm " + std::string(dtw ? "frame" : "mean") + " in item " + std::to_string(bad) +
                               ": its angle is undefined");
    }
    st.n_recheck_pairs = marked_h;
    st.n_recount_rows = recount_h;
    st.n_nonrobust_pairs = nonrobust_h;
}

}  // namespace

std::shared_ptr<ResultImpl> launch_score(const std::shared_ptr<TaskImpl> &tp, const ScoreParams &p,
                                         hipStream_t stream) {
    using clock = std::chrono::steady_clock;
    const auto t_enter = clock::now();
    TaskImpl &t = *tp;
    std::lock_guard<std::mutex> lock(t.mu);
    // the workspace is reused: the task's previous score must have completed
    if (auto prev = t.pending.lock()) {
        try {
            finish_score(*prev);
        } catch (const Error &) {
            // that score's error stays with its own result
        }
    }
    const DatasetImpl &ds = *t.ds;
    auto res = std::make_shared<ResultImpl>();
    res->task = tp;
    const int64_t n_cells = int64_t(t.cells.size());
    res->half_units.assign(size_t(n_cells), 0);
    fabx_stats &st = res->stats;
    st.n_cells = n_cells;
    st.n_triplets = t.total_triplets;
    st.n_items = int64_t(t.items.size());
    st.n_frames = t.n_frames;
    st.n_pairs = t.n_pairs_needed;
    st.dtw_cells = p.mode == FABX_MODE_DTW ? t.dtw_cells_needed : 0;
    st.dtw_cells_sym = p.mode == FABX_MODE_DTW ? t.dtw_cells_sym : 0;
    st.margin = p.precision == FABX_PREC_BF16_RECHECK ? p.margin : 0.0;
    st.delta = p.precision == FABX_PREC_BF16_RECHECK && p.mode == FABX_MODE_DTW ? p.delta : 0.0;
    if (n_cells == 0) return res;
    if (ds.ctx->device < 0) fail(FABX_EINVAL, "context has no device (host-only context)");
    FABX_HIP(hipSetDevice(ds.ctx->device));

    auto pend = std::make_unique<PendingScore>();
    pend->task = tp;
    pend->ctx = ds.ctx;
    pend->stream = stream;
    pend->t_enter = t_enter;
    const bool bf16 = p.precision == FABX_PREC_BF16_RECHECK;
    const bool dtw = p.mode == FABX_MODE_DTW;
    pend->bf16 = bf16;
    pend->dtw = dtw;
    pend->keep_pairs = p.keep_pairs;
    const int dim = ds.dim;
    const int dim_pad = int(round_up(dim, 64));
    const int64_t n_items = int64_t(t.items.size());
    const int64_t G = int64_t(t.groups.size());
    Trace tr("score");
    const int64_t n_units = int64_t(t.units.size() / 3);
    const bool pooled = !dtw;
    const bool plain_dtw = dtw && !bf16;
    const std::vector<int64_t> tiles = pooled ? tile_prefix(t, p) : std::vector<int64_t>();
    const PlainPlan strips = plain_dtw ? plain_plan(t, plain_dmat_cells()) : PlainPlan();
    tr.mark("plans");

    // ---- device tables (items / groups / cells are fixed for the task): one copy
    TaskDevice &dv = t.dev;
    Pool *pool = &ds.ctx->pool;
    if (!dv.blob.ptr) dv.blob.pool = pool;
    for (DevBuf *b : {&t.ws.xn, &t.ws.rinv, &t.ws.dmat, &t.ws.p32, &t.ws.flags, &t.ws.p64,
                      &t.ws.half_units, &t.ws.recheck_list, &t.ws.recount_list, &t.ws.finfo, &t.ws.flen})
        if (!b->ptr) b->pool = pool;
    // fused kernel: tile width and grid from the tuning table (or the caller),
    // and the task's column blocks for that width (uploaded on first use)
    FusedConfig fcfg;
    ColPlan *cplan = nullptr;
    if (dtw && bf16) {
        fcfg = p.fused.cols > 0 ? p.fused : ds.ctx->tuner.lookup(tune_key(t, p));
        if (fcfg.cols >= kStreamMinCols && t.max_len > kFusedRowFrames)
            fail(FABX_EINVAL, "the streaming DTW kernel (fused_cols >= 512) takes items of at most 64 frames");
        cplan = &col_plan(t, fcfg.cols);
        res->fused = fcfg;
        st.fused_cols = fcfg.cols;
        st.fused_blocks_per_cu = fcfg.blocks_per_cu;
    }
    if (!dv.uploaded) {
        // one DMA for the task's tables (and the column plan this score uses)
        if (t.packed) {
            PinnedBlock &pb = *t.packed;
            dv.blob.ensure(pb.bytes);
            FABX_HIP(hipMemcpyAsync(dv.blob.ptr, pb.p, pb.bytes, hipMemcpyHostToDevice, ds.ctx->copy_stream));
            pb.done = ds.ctx->events.get();
            FABX_HIP(hipEventRecord(pb.done, ds.ctx->copy_stream));
            FABX_HIP(hipStreamWaitEvent(stream, pb.done, 0));
            set_task_tables(t, t.packed_layout);
            pend->packed = std::move(t.packed);  // back to the pool when this score is done
        } else {
            Packer pk;
            std::array<std::vector<int64_t>, 5> gcols;
            const TableLayout L = add_task_tables(t, cplan && !cplan->d_cb ? cplan : nullptr, pk, gcols);
            pk.upload(dv.blob, ds.ctx->staging, ds.ctx->copy_stream, stream);
            set_task_tables(t, L);
        }
        dv.uploaded = true;
    }
    if (cplan && !cplan->d_cb) {  // another column width for an already uploaded task
        Packer pc;
        const std::array<size_t, 5> o{pc.add(cplan->cb), pc.add(cplan->unit_prefix), pc.add(cplan->g_cb0),
                                      pc.add(cplan->rb_cstart), pc.add(cplan->band_rb)};
        cplan->dev.pool = pool;
        pc.upload(cplan->dev, ds.ctx->staging, ds.ctx->copy_stream, stream);
        set_col_plan(*cplan, cplan->dev, o);
    }
    // Gram tile prefix of this score (pooled mode), or the strips of the plain DTW form
    DevBuf &plan_d = pend->plan_d;
    plan_d.pool = pool;
    DevPtrs d;
    static const std::vector<int64_t> no_slots;
    const std::vector<int64_t> &long_slots = dtw && bf16 ? t.long_slots : no_slots;
    if (pooled || plain_dtw || !long_slots.empty()) {
        Packer pp;
        const PlanLayout pl = add_plan(pp, tiles, strips, long_slots);
        pp.upload(plan_d, ds.ctx->staging, ds.ctx->copy_stream, stream);
        set_plan(d, plan_d.as<char>(), pl);
    }
    tr.mark("upload");

    // ---- workspace
    Workspace &ws = t.ws;
    const WorkspaceSizes wz = workspace_sizes(t, p, strips, cplan && fcfg.cols >= kStreamMinCols);
    // buffers the form does not use keep what an earlier score left (or nothing)
    for (auto bs : {std::make_pair(&ws.xn, wz.xn), std::make_pair(&ws.rinv, wz.rinv),
                    std::make_pair(&ws.dmat, wz.dmat), std::make_pair(&ws.p32, wz.p32),
                    std::make_pair(&ws.flags, wz.flags), std::make_pair(&ws.p64, wz.p64),
                    std::make_pair(&ws.recheck_list, wz.recheck_list),
                    std::make_pair(&ws.recount_list, wz.recount_list),
                    std::make_pair(&ws.half_units, wz.half_units), std::make_pair(&ws.finfo, wz.finfo),
                    std::make_pair(&ws.flen, wz.flen)})
        if (bs.second) bs.first->ensure(bs.second);
    st.workspace_bytes = int64_t(ws.total());
    pend->host_bytes = size_t(n_cells) * 8 + 64;
    pend->host = ds.ctx->pinned.get(pend->host_bytes, &pend->host_bytes);

    d.it = kern::ItemTables{dv.item_src, dv.item_len, dv.item_dst, n_items};
    d.gt = kern::GroupTables{dv.g_item0, dv.g_n, dv.g_frame0, dv.g_nframes, dv.g_pair_base, G, t.n_pair_slots};
    d.cells = dv.cells;
    d.units = dv.units;
    d.rb = dv.rb;
    d.item_group = dv.item_group;
    if (cplan) {
        d.cb = cplan->d_cb;
        d.g_cb0 = cplan->d_g_cb0;
        d.rb_cstart = cplan->d_rb_cstart;
        d.unit_prefix = cplan->d_unit_prefix;
        d.band_rb = cplan->d_band_rb;
    }
    d.xn = ws.xn.ptr;
    d.rinv = ws.rinv.as<float>();
    d.dmat = ws.dmat.as<float>();
    d.p32 = ws.p32.as<float>();
    d.flags = ws.flags.as<uint8_t>();
    d.p64 = ws.p64.as<double>();
    d.recheck_list = ws.recheck_list.as<int64_t>();
    d.recount_list = ws.recount_list.as<int32_t>();
    d.half_units = ws.half_units.as<unsigned long long>();
    d.finfo = ws.finfo.as<uint32_t>();
    d.flen = ws.flen.as<float>();

    pend->tm = std::make_unique<Timer>(stream, ds.ctx->events);
    tr.mark("workspace");
    // on an error after launches, drain the stream before plan_d goes back to the pool
    struct DrainOnError {
        hipStream_t s;
        ~DrainOnError() {
            if (std::uncaught_exceptions() > 0) (void)hipStreamSynchronize(s);
        }
    } drain{stream};
    enqueue_score(t, p, fcfg, cplan, tiles, strips, d, stream, pend->tm.get(), pend->host, st);
    tr.mark("launch");
    pend->t_launch = clock::now();
    res->pending = std::move(pend);
    t.pending = res;
    return res;
}

void finish_score(ResultImpl &res) {
    using clock = std::chrono::steady_clock;
    std::lock_guard<std::mutex> lk(res.mu);
    if (!res.pending) {
        if (res.status != FABX_OK) fail(res.status, res.status_msg);
        return;
    }
    std::unique_ptr<PendingScore> pend = std::move(res.pending);
    try {
        TaskImpl &t = *pend->task;
        Timer &tm = *pend->tm;
        FABX_HIP(hipSetDevice(pend->ctx->device));
        FABX_HIP(hipEventSynchronize(tm.ev[6]));
        const auto t_synced = clock::now();
        const size_t n_cells = res.half_units.size();
        const char *host = static_cast<const char *>(pend->host);
        std::memcpy(res.half_units.data(), host, n_cells * 8);
        fabx_stats &st = res.stats;
        read_counters(t, host, n_cells, pend->dtw, st);
        st.ms_normalize = tm.ms(1, 2);
        st.ms_distance = tm.ms(2, 3);
        st.ms_triplets = tm.ms(3, 4);
        st.ms_recheck = tm.ms(4, 5);
        st.ms_total = tm.ms(0, 6);
        if (pend->keep_pairs) {
            // the task's workspace still holds this score: a later score on the task
            // finishes this one before it touches the workspace
            res.has_pairs = true;
            res.p32.resize(size_t(t.n_pair_slots));
            FABX_HIP(hipMemcpy(res.p32.data(), t.ws.p32.ptr, res.p32.size() * 4, hipMemcpyDeviceToHost));
            if (pend->bf16) {
                res.flags.resize(size_t(t.n_pair_slots));
                FABX_HIP(hipMemcpy(res.flags.data(), t.ws.flags.ptr, res.flags.size(), hipMemcpyDeviceToHost));
                res.p64.resize(size_t(t.n_pair_slots));
                FABX_HIP(hipMemcpy(res.p64.data(), t.ws.p64.ptr, res.p64.size() * 8, hipMemcpyDeviceToHost));
            }
        }
        st.ms_host_setup = std::chrono::duration<double, std::milli>(pend->t_launch - pend->t_enter).count();
        st.ms_host_finish = std::chrono::duration<double, std::milli>(clock::now() - t_synced).count();
    } catch (const Error &e) {
        // make sure nothing of the score still runs before its buffers are released
        (void)hipStreamSynchronize(pend->stream);
        res.status = e.code;
        res.status_msg = e.msg;
        throw;
    }
}

void score_in_scratch(TaskImpl &t, const ScoreParams &p, char *base, size_t cap, hipStream_t stream,
                      int64_t *half_units, fabx_stats *stats) {
    std::lock_guard<std::mutex> lock(t.mu);
    const DatasetImpl &ds = *t.ds;
    if (ds.ctx->device < 0) fail(FABX_EINVAL, "context has no device (host-only context)");
    fabx_stats st{};
    const int64_t n_cells = int64_t(t.cells.size());
    st.n_cells = n_cells;
    st.n_triplets = t.total_triplets;
    st.n_items = int64_t(t.items.size());
    st.n_frames = t.n_frames;
    st.n_pairs = t.n_pairs_needed;
    st.dtw_cells = p.mode == FABX_MODE_DTW ? t.dtw_cells_needed : 0;
    st.dtw_cells_sym = p.mode == FABX_MODE_DTW ? t.dtw_cells_sym : 0;
    st.margin = p.precision == FABX_PREC_BF16_RECHECK ? p.margin : 0.0;
    st.delta = p.precision == FABX_PREC_BF16_RECHECK && p.mode == FABX_MODE_DTW ? p.delta : 0.0;
    if (n_cells == 0) {
        if (stats) *stats = st;
        return;
    }
    FABX_HIP(hipSetDevice(ds.ctx->device));
    const bool bf16 = p.precision == FABX_PREC_BF16_RECHECK;
    const bool dtw = p.mode == FABX_MODE_DTW;
    FusedConfig fcfg;
    ColPlan *cplan = nullptr;
    if (dtw && bf16) {
        fcfg = p.fused.cols > 0 ? p.fused : ds.ctx->tuner.lookup(tune_key(t, p));
        if (fcfg.cols >= kStreamMinCols && t.max_len > kFusedRowFrames)
            fail(FABX_EINVAL, "the streaming DTW kernel (fused_cols >= 512) takes items of at most 64 frames");
        cplan = &col_plan(t, fcfg.cols);
        st.fused_cols = fcfg.cols;
        st.fused_blocks_per_cu = fcfg.blocks_per_cu;
    }
    const std::vector<int64_t> tiles = dtw ? std::vector<int64_t>() : tile_prefix(t, p);
    const bool stream_k = cplan && fcfg.cols >= kStreamMinCols;
    // Layout in the scratch buffer: tables (task, column plan, plan), then the
    // workspace.  The plain DTW form's distance buffer takes what is left, at
    // most its usual size; its strips are planned for that size.
    auto layout = [&](const PlainPlan &strips, Packer &pk, TableLayout &tl, PlanLayout &pl,
                      std::array<std::vector<int64_t>, 5> &gcols) {
        tl = add_task_tables(t, cplan, pk, gcols);
        static const std::vector<int64_t> no_slots;  // the packer keeps pointers: no temporaries
        pl = add_plan(pk, tiles, strips, dtw && bf16 ? t.long_slots : no_slots);
        const size_t tables = (pk.total + 255) & ~size_t(255);
        return tables + workspace_sizes(t, p, strips, stream_k).total_aligned();
    };
    Packer pk;
    TableLayout tl;
    PlanLayout pl;
    std::array<std::vector<int64_t>, 5> gcols;
    PlainPlan strips;
    if (dtw && !bf16) {
        strips = plain_plan(t, plain_dmat_cells());
        Packer probe;
        std::array<std::vector<int64_t>, 5> gc2;
        const size_t need = layout(strips, probe, tl, pl, gc2);
        if (need > cap) {
            // the distance buffer gets what the rest leaves (1 MiB kept for the longer strip tables)
            const size_t rest = need - ((size_t(std::max<int64_t>(strips.max_cells, 1)) * 4 + 255) & ~size_t(255));
            const int64_t cells = rest + (size_t(1) << 20) < cap ? int64_t((cap - rest - (size_t(1) << 20)) / 4) : 0;
            if (cells < 4096) fail(FABX_ENOMEM, "task needs more scratch than the no-allocation limit");
            strips = plain_plan(t, cells);
        }
    }
    const size_t need = layout(strips, pk, tl, pl, gcols);
    if (need > cap)
        fail(FABX_ENOMEM, "task needs " + std::to_string(need) + " bytes of scratch; the no-allocation limit is " +
                              std::to_string(cap));
    // tables: packed on the host, one copy (from pageable memory) into the scratch
    std::vector<char> h(pk.total);
    pk.copy_to(h.data());
    FABX_HIP(hipMemcpyAsync(base, h.data(), pk.total, hipMemcpyHostToDevice, stream));
    DevPtrs d;
    auto at = [&](size_t off) { return base + off; };
    d.it = kern::ItemTables{reinterpret_cast<const int64_t *>(at(tl.item_src)),
                            reinterpret_cast<const int32_t *>(at(tl.item_len)),
                            reinterpret_cast<const int64_t *>(at(tl.item_dst)), int64_t(t.items.size())};
    d.gt = kern::GroupTables{reinterpret_cast<const int64_t *>(at(tl.g[0])),
                             reinterpret_cast<const int64_t *>(at(tl.g[1])),
                             reinterpret_cast<const int64_t *>(at(tl.g[2])),
                             reinterpret_cast<const int64_t *>(at(tl.g[3])),
                             reinterpret_cast<const int64_t *>(at(tl.g[4])), int64_t(t.groups.size()),
                             t.n_pair_slots};
    d.cells = reinterpret_cast<const CellDev *>(at(tl.cells));
    d.units = reinterpret_cast<const int32_t *>(at(tl.units));
    d.rb = reinterpret_cast<const int32_t *>(at(tl.rb));
    d.item_group = reinterpret_cast<const int32_t *>(at(tl.item_group));
    if (cplan) {
        d.cb = reinterpret_cast<const int32_t *>(at(tl.plan[0]));
        d.unit_prefix = reinterpret_cast<const int64_t *>(at(tl.plan[1]));
        d.g_cb0 = reinterpret_cast<const int32_t *>(at(tl.plan[2]));
        d.rb_cstart = reinterpret_cast<const int32_t *>(at(tl.plan[3]));
        d.band_rb = reinterpret_cast<const int32_t *>(at(tl.plan[4]));
    }
    set_plan(d, base, pl);
    const WorkspaceSizes wz = workspace_sizes(t, p, strips, stream_k);
    size_t off = (pk.total + 255) & ~size_t(255);
    auto take = [&](size_t bytes) -> char * {
        if (!bytes) return nullptr;
        char *q = base + off;
        off += (bytes + 255) & ~size_t(255);
        return q;
    };
    d.xn = take(wz.xn);
    d.rinv = reinterpret_cast<float *>(take(wz.rinv));
    d.dmat = reinterpret_cast<float *>(take(wz.dmat));
    d.p32 = reinterpret_cast<float *>(take(wz.p32));
    d.flags = reinterpret_cast<uint8_t *>(take(wz.flags));
    d.p64 = reinterpret_cast<double *>(take(wz.p64));
    d.recheck_list = reinterpret_cast<int64_t *>(take(wz.recheck_list));
    d.recount_list = reinterpret_cast<int32_t *>(take(wz.recount_list));
    d.half_units = reinterpret_cast<unsigned long long *>(take(wz.half_units));
    d.finfo = reinterpret_cast<uint32_t *>(take(wz.finfo));
    d.flen = reinterpret_cast<float *>(take(wz.flen));
    st.workspace_bytes = int64_t(wz.total_aligned());
    std::vector<char> host(size_t(n_cells) * 8 + 64);
    try {
        enqueue_score(t, p, fcfg, cplan, tiles, strips, d, stream, nullptr, host.data(), st);
        FABX_HIP(hipStreamSynchronize(stream));
    } catch (...) {
        (void)hipStreamSynchronize(stream);  // nothing may still use the scratch or `h`
        throw;
    }
    read_counters(t, host.data(), size_t(n_cells), dtw, st);
    std::memcpy(half_units, host.data(), size_t(n_cells) * 8);
    if (stats) *stats = st;
}

void release_device(TaskImpl &t) {
    std::lock_guard<std::mutex> lock(t.mu);
    if (auto prev = t.pending.lock()) {
        try {
            finish_score(*prev);
        } catch (const Error &) {
            // that score's error stays with its own result
        }
    }
    t.ws.release();
    TaskDevice &dv = t.dev;
    dv.blob.release();
    dv.uploaded = false;
    for (auto &cp : t.col_plans) {
        cp->dev.release();
        cp->d_cb = nullptr;
        cp->d_g_cb0 = nullptr;
        cp->d_rb_cstart = nullptr;
        cp->d_unit_prefix = nullptr;
        cp->d_band_rb = nullptr;
    }
    t.packed.reset();
}

std::shared_ptr<ResultImpl> run_score(const std::shared_ptr<TaskImpl> &tp, const ScoreParams &p,
                                      hipStream_t stream) {
    auto res = launch_score(tp, p, stream);
    finish_score(*res);
    return res;
}

}  // namespace fabx
