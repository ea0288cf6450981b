// C ABI of fastabx-hip: argument checks, handle management, error codes.
#include <algorithm>
#include <cstdint>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>

#include "internal.h"
#include "kernels.h"

namespace fabx {

namespace {
thread_local std::string g_last_error;
}

void set_last_error(const std::string &msg) { g_last_error = msg; }
const char *last_error_cstr() { return g_last_error.c_str(); }

[[noreturn]] void fail(int code, const std::string &msg) { throw Error{code, msg}; }

static void *raw_alloc(size_t n) {
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, n);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return p;
}

void *Pool::alloc(size_t n, size_t *got) {
    n = (n + (size_t(2) << 20) - 1) & ~((size_t(2) << 20) - 1);  // 2 MiB granules
    {
        std::lock_guard<std::mutex> lk(mu);
        // best fit among free blocks no larger than twice the request
        size_t best = free_blocks.size();
        for (size_t i = 0; i < free_blocks.size(); ++i)
            if (free_blocks[i].first >= n && free_blocks[i].first <= 2 * n &&
                (best == free_blocks.size() || free_blocks[i].first < free_blocks[best].first))
                best = i;
        if (best != free_blocks.size()) {
            auto b = free_blocks[best];
            free_blocks.erase(free_blocks.begin() + long(best));
            *got = b.first;
            return b.second;
        }
    }
    void *p = raw_alloc(n);
    if (!p) {
        trim();  // give cached blocks back and try once more
        p = raw_alloc(n);
    }
    if (!p) fail(FABX_ENOMEM, "device allocation of " + std::to_string(n) + " bytes failed");
    std::lock_guard<std::mutex> lk(mu);
    held += n;
    *got = n;
    return p;
}

void Pool::free(void *p, size_t n) {
    std::lock_guard<std::mutex> lk(mu);
    free_blocks.push_back({n, p});
}

void Pool::trim() {
    std::lock_guard<std::mutex> lk(mu);
    for (auto &b : free_blocks) {
        (void)hipFree(b.second);
        held -= b.first;
    }
    free_blocks.clear();
}

Pool::~Pool() { trim(); }

void DevBuf::release() {
    if (ptr) {
        if (pool) pool->free(ptr, bytes);
        else (void)hipFree(ptr);
    }
    ptr = nullptr;
    bytes = 0;
}

void DevBuf::ensure(size_t n) {
    if (n <= bytes && ptr) return;
    release();
    if (n == 0) n = 16;
    if (pool) {
        ptr = pool->alloc(n, &bytes);
        return;
    }
    ptr = raw_alloc(n);
    if (!ptr) fail(FABX_ENOMEM, "device allocation of " + std::to_string(n) + " bytes failed");
    bytes = n;
}

hipEvent_t EventPool::get() {
    {
        std::lock_guard<std::mutex> lk(mu);
        if (!free_events.empty()) {
            hipEvent_t e = free_events.back();
            free_events.pop_back();
            return e;
        }
    }
    hipEvent_t e;
    FABX_HIP(hipEventCreate(&e));
    return e;
}

void EventPool::put(hipEvent_t e) {
    std::lock_guard<std::mutex> lk(mu);
    free_events.push_back(e);
}

EventPool::~EventPool() {
    for (auto e : free_events) (void)hipEventDestroy(e);
}

void Staging::reserve(size_t n) {
    if (!done) FABX_HIP(hipEventCreateWithFlags(&done, hipEventDisableTiming));
    if (in_flight) {
        FABX_HIP(hipEventSynchronize(done));
        in_flight = false;
    }
    if (n <= cap) return;
    if (host) (void)hipHostFree(host);
    host = nullptr;
    cap = 0;
    const size_t want = std::max(n, size_t(8) << 20);
    if (hipHostMalloc(&host, want, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        host = nullptr;
        fail(FABX_ENOMEM, "pinned staging allocation of " + std::to_string(want) + " bytes failed");
    }
    cap = want;
}

void *PinnedPool::get(size_t n, size_t *got) {
    n = std::max<size_t>(n, 4096);
    {
        std::lock_guard<std::mutex> lk(mu);
        size_t best = free_blocks.size();
        for (size_t i = 0; i < free_blocks.size(); ++i)
            if (free_blocks[i].first >= n && free_blocks[i].first <= 2 * n &&
                (best == free_blocks.size() || free_blocks[i].first < free_blocks[best].first))
                best = i;
        if (best != free_blocks.size()) {
            auto b = free_blocks[best];
            free_blocks.erase(free_blocks.begin() + long(best));
            cached -= b.first;
            *got = b.first;
            return b.second;
        }
    }
    void *p = nullptr;
    if (hipHostMalloc(&p, n, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        fail(FABX_ENOMEM, "pinned host allocation of " + std::to_string(n) + " bytes failed");
    }
    *got = n;
    return p;
}

void PinnedPool::put(void *p, size_t n) {
    {
        std::lock_guard<std::mutex> lk(mu);
        if (cached + n <= (size_t(256) << 20)) {
            free_blocks.push_back({n, p});
            cached += n;
            return;
        }
    }
    (void)hipHostFree(p);
}

PinnedPool::~PinnedPool() {
    for (auto &b : free_blocks) (void)hipHostFree(b.second);
}

PinnedBlock::PinnedBlock(std::shared_ptr<CtxImpl> c, size_t n) : ctx(std::move(c)) {
    p = ctx->pinned.get(n, &cap);
}

PinnedBlock::~PinnedBlock() {
    if (done) {
        (void)hipEventSynchronize(done);
        ctx->events.put(done);
    }
    if (p) ctx->pinned.put(p, cap);
    if (packed) ctx->pinned.packed_bytes -= cap;
}

Staging::~Staging() {
    if (in_flight) (void)hipEventSynchronize(done);
    if (host) (void)hipHostFree(host);
    if (done) (void)hipEventDestroy(done);
}

CtxImpl::~CtxImpl() {
    if (copy_stream) {
        (void)hipStreamSynchronize(copy_stream);
        (void)hipStreamDestroy(copy_stream);
    }
    pool.trim();
}

// Runs `f`, converting internal errors into status codes.
template <typename F>
int guarded(F &&f) {
    try {
        f();
        set_last_error("");
        return FABX_OK;
    } catch (const Error &e) {
        set_last_error(e.msg);
        return e.code;
    } catch (const std::bad_alloc &) {
        set_last_error("host allocation failed");
        return FABX_ENOMEM;
    } catch (const std::exception &e) {
        set_last_error(e.what());
        return FABX_EINVAL;
    } catch (...) {
        set_last_error("unknown internal error");
        return FABX_EINVAL;
    }
}

}  // namespace fabx

using namespace fabx;

extern "C" {

const char *fabx_last_error(void) { return last_error_cstr(); }

const char *fabx_version(void) { return "fastabx-hip 0.1.0 (gfx950)"; }

int fabx_set_thread_serial(int serial) {
    bool &f = HostPool::caller_serial();
    const int prev = f ? 1 : 0;
    f = serial != 0;
    return prev;
}

int fabx_create(fabx_ctx **out, int device, void *hip_stream) {
    return guarded([&] {
        if (!out) fail(FABX_EINVAL, "out is NULL");
        *out = nullptr;
        auto c = std::make_shared<CtxImpl>();
        c->device = device;
        if (device >= 0) {
            int n = 0;
            if (hipGetDeviceCount(&n) != hipSuccess || device >= n) {
                (void)hipGetLastError();
                fail(FABX_EINVAL, "no HIP device " + std::to_string(device));
            }
            FABX_HIP(hipSetDevice(device));
            hipDeviceProp_t prop;
            FABX_HIP(hipGetDeviceProperties(&prop, device));
            c->n_cu = prop.multiProcessorCount;
            FABX_HIP(hipStreamCreateWithFlags(&c->copy_stream, hipStreamNonBlocking));
            (void)scratch_setup(device);  // the device address of fabx_score_noalloc's scratch
            const char *tune_file = std::getenv("FABX_AUTOTUNE_CACHE");
            if (tune_file && *tune_file) c->tuner.load(tune_file);
            // NULL is the device's null stream, as everywhere in HIP: the context's
            // work is then ordered after what the caller enqueued there
            c->stream = static_cast<hipStream_t>(hip_stream);
        } else if (device != -1) {
            fail(FABX_EINVAL, "device must be >= 0 (or -1 for a host-only context)");
        }
        *out = new fabx_ctx{c};
    });
}

void fabx_destroy(fabx_ctx *ctx) { delete ctx; }

namespace {

// The checks and fields common to both dataset constructors; items are filled
// by the caller.
std::shared_ptr<DatasetImpl> new_dataset(fabx_ctx *ctx, const void *features, int32_t dtype, int64_t n_frames,
                                         int32_t dim, int64_t n_items, const int32_t *attrs, int32_t n_attr) {
    if (n_items < 1) fail(FABX_EINVAL, "n_items must be >= 1");
    if (dim < 1) fail(FABX_EINVAL, "dim must be >= 1");
    if (n_attr < 1) fail(FABX_EINVAL, "n_attr must be >= 1");
    if (dtype != FABX_DTYPE_F32 && dtype != FABX_DTYPE_BF16 && dtype != FABX_DTYPE_UNITS)
        fail(FABX_EINVAL, "unknown dtype");
    if (dtype == FABX_DTYPE_UNITS && dim != 1) fail(FABX_EINVAL, "unit codes (FABX_DTYPE_UNITS) have dim 1");
    if (!attrs) fail(FABX_EINVAL, "attrs is NULL");
    if (!features && ctx->p->device >= 0) fail(FABX_EINVAL, "features is NULL");
    auto ds = std::make_shared<DatasetImpl>();
    ds->ctx = ctx->p;
    ds->features = features;
    ds->dtype = dtype;
    ds->n_frames = n_frames;
    ds->dim = dim;
    ds->n_items = n_items;
    ds->n_attr = n_attr;
    ds->attrs.assign(attrs, attrs + n_items * int64_t(n_attr));
    ds->item_start.resize(size_t(n_items));
    ds->item_len.resize(size_t(n_items));
    return ds;
}

void set_item(DatasetImpl &ds, int64_t i, int64_t start, int64_t len) {
    if (len < 1) fail(FABX_EINVAL, "item " + std::to_string(i) + " has no frame");
    if (len > INT32_MAX) fail(FABX_EINVAL, "item " + std::to_string(i) + " is too long");
    if (start < 0 || start > ds.n_frames - len)
        fail(FABX_EINVAL, "item " + std::to_string(i) + " lies outside the feature rows");
    ds.item_start[size_t(i)] = start;
    ds.item_len[size_t(i)] = int32_t(len);
    if (len > ds.max_len) ds.max_len = int(len);
}

}  // namespace

int fabx_dataset_create(fabx_ctx *ctx, const fabx_dataset_desc *d, fabx_dataset **out) {
    return guarded([&] {
        if (!ctx || !d || !out) fail(FABX_EINVAL, "null argument");
        *out = nullptr;
        if (!d->offsets) fail(FABX_EINVAL, "offsets is NULL");
        auto ds = new_dataset(ctx, d->features, d->dtype, d->n_frames, d->dim, d->n_items, d->attrs, d->n_attr);
        if (d->offsets[0] != 0) fail(FABX_EINVAL, "offsets[0] must be 0");
        for (int64_t i = 0; i < d->n_items; ++i) set_item(*ds, i, d->offsets[i], d->offsets[i + 1] - d->offsets[i]);
        if (d->offsets[d->n_items] != d->n_frames) fail(FABX_EINVAL, "offsets[n_items] != n_frames");
        *out = new fabx_dataset{ds};
    });
}

int fabx_dataset_create_windows(fabx_ctx *ctx, const void *features, int32_t dtype, int64_t n_frames,
                                int32_t dim, const int64_t *item_start, const int64_t *item_len,
                                int64_t n_items, const int32_t *attrs, int32_t n_attr, fabx_dataset **out) {
    return guarded([&] {
        if (!ctx || !out || !item_start || !item_len) fail(FABX_EINVAL, "null argument");
        *out = nullptr;
        auto ds = new_dataset(ctx, features, dtype, n_frames, dim, n_items, attrs, n_attr);
        for (int64_t i = 0; i < n_items; ++i) set_item(*ds, i, item_start[i], item_len[i]);
        *out = new fabx_dataset{ds};
    });
}

int fabx_slice_frames(const double *onset, const double *offset, int64_t n, double dt, int libri_light,
                      int64_t *start, int64_t *len) {
    return guarded([&] {
        if (n < 0 || (n > 0 && (!onset || !offset || !start || !len))) fail(FABX_EINVAL, "null argument");
        if (!(dt > 0.0) || !std::isfinite(dt)) fail(FABX_EINVAL, "the frame step must be positive and finite");
        for (int64_t k = 0; k < n; ++k) {
            const double a = onset[k], b = offset[k];
            if (!std::isfinite(a) || !std::isfinite(b) || a < 0.0 || a > b)
                fail(FABX_EINVAL, "unit " + std::to_string(k) + ": need 0 <= onset <= offset");
            // frame i has time dt / 2 + i dt; kept when onset <= t_i <= offset
            const double first = std::ceil(a / dt - 0.5), last = std::floor(b / dt - 0.5);
            if (first > 9.0e15 || last > 9.0e15) fail(FABX_EINVAL, "unit " + std::to_string(k) + " is too far");
            const int64_t i0 = std::max<int64_t>(0, int64_t(first));
            const int64_t i1 = int64_t(last) - (libri_light ? 1 : 0);
            start[k] = i0;
            len[k] = std::max<int64_t>(0, i1 - i0 + 1);
        }
    });
}

int fabx_probe_stream(const float *src, uint16_t *dst, int64_t n_rows, int32_t dim, void *hip_stream) {
    return guarded([&] {
        if (!src || !dst || n_rows < 0 || dim <= 0) fail(FABX_EINVAL, "bad probe arguments");
        fabx::kern::probe_stream(static_cast<hipStream_t>(hip_stream), src, dim, n_rows, dst);
    });
}

void fabx_dataset_destroy(fabx_dataset *ds) { delete ds; }

int fabx_task_create(fabx_dataset *ds, int32_t on, const int32_t *by, int32_t n_by,
                     const int32_t *across, int32_t n_across, fabx_task **out) {
    return guarded([&] {
        if (!ds || !out) fail(FABX_EINVAL, "null argument");
        *out = nullptr;
        auto t = build_task(ds->p, on, by, n_by, across, n_across);
        prepack_tables(*t);
        *out = new fabx_task{t};
    });
}

int fabx_task_create_subsampled(fabx_dataset *ds, int32_t on, const int32_t *by, int32_t n_by,
                                const int32_t *across, int32_t n_across, const fabx_subsampler *sub,
                                fabx_task **out) {
    return guarded([&] {
        if (!ds || !out || !sub) fail(FABX_EINVAL, "null argument");
        *out = nullptr;
        if (sub->max_a < 0 || sub->max_b < 0 || sub->max_x < 0 || sub->max_x_across < 0)
            fail(FABX_EINVAL, "subsampler caps must be >= 0 (0: no cap)");
        auto full = build_task(ds->p, on, by, n_by, across, n_across);
        auto t = subsample_task(*full, *sub);
        full.reset();
        prepack_tables(*t);
        *out = new fabx_task{t};
    });
}

void fabx_task_destroy(fabx_task *t) { delete t; }

int64_t fabx_task_num_cells(const fabx_task *t) { return t ? int64_t(t->p->cells.size()) : -1; }

int32_t fabx_task_key_width(const fabx_task *t) { return t ? t->p->key_width : -1; }

int fabx_task_cell_keys(const fabx_task *t, int32_t *out) {
    return guarded([&] {
        if (!t || !out) fail(FABX_EINVAL, "null argument");
        cell_keys(*t->p, out);
    });
}

int fabx_task_cell_sizes(const fabx_task *t, int64_t *n_triplets, int32_t *abx) {
    return guarded([&] {
        if (!t) fail(FABX_EINVAL, "null task");
        const auto &T = *t->p;
        for (size_t c = 0; c < T.cells.size(); ++c) {
            if (n_triplets) n_triplets[c] = T.n_triplets[c];
            if (abx) {
                abx[3 * c] = T.cells[c].na;
                abx[3 * c + 1] = T.cells[c].nb;
                abx[3 * c + 2] = T.cells[c].nx;
            }
        }
    });
}

int fabx_score_opts_default(fabx_score_opts *o) {
    if (!o) return FABX_EINVAL;
    o->distance = FABX_DISTANCE_ANGULAR;
    o->mode = FABX_MODE_DTW;
    o->precision = FABX_PREC_BF16_RECHECK;
    o->dtw_norm = FABX_NORM_PATH;
    o->margin = -1.0;
    o->delta = -1.0;
    o->keep_pairs = 0;
    o->fused_cols = 0;
    o->fused_blocks_per_cu = 0;
    return FABX_OK;
}

int fabx_score(fabx_task *t, const fabx_score_opts *opts, fabx_result **out) {
    return guarded([&] {
        if (!t || !out) fail(FABX_EINVAL, "null argument");
        *out = nullptr;
        ScoreParams p = resolve_opts(opts, *t->p->ds);
        auto r = run_score(t->p, p, t->p->ds->ctx->stream);
        *out = new fabx_result{r};
    });
}

int fabx_score_async(fabx_task *t, const fabx_score_opts *opts, fabx_result **out) {
    return guarded([&] {
        if (!t || !out) fail(FABX_EINVAL, "null argument");
        *out = nullptr;
        ScoreParams p = resolve_opts(opts, *t->p->ds);
        auto r = launch_score(t->p, p, t->p->ds->ctx->stream);
        *out = new fabx_result{r};
    });
}

int fabx_result_wait(fabx_result *r) {
    return guarded([&] {
        if (!r) fail(FABX_EINVAL, "null result");
        finish_score(*r->p);
    });
}

void fabx_result_free(fabx_result *r) { delete r; }

int64_t fabx_result_num_cells(const fabx_result *r) { return r ? int64_t(r->p->half_units.size()) : -1; }

int32_t fabx_result_key_width(const fabx_result *r) { return r ? r->p->task->key_width : -1; }

int fabx_result_cell_keys(const fabx_result *r, int32_t *out) {
    return guarded([&] {
        if (!r || !out) fail(FABX_EINVAL, "null argument");
        cell_keys(*r->p->task, out);
    });
}

int fabx_result_cells(const fabx_result *r, int64_t *half_units, int64_t *n_triplets, double *score) {
    return guarded([&] {
        if (!r) fail(FABX_EINVAL, "null result");
        finish_score(*r->p);
        const auto &R = *r->p;
        const auto &T = *R.task;
        for (size_t c = 0; c < R.half_units.size(); ++c) {
            if (half_units) half_units[c] = R.half_units[c];
            if (n_triplets) n_triplets[c] = T.n_triplets[c];
            if (score) score[c] = double(R.half_units[c]) / (2.0 * double(T.n_triplets[c]));
        }
    });
}

int fabx_result_pairs(const fabx_result *r, int64_t n, const int64_t *xs, const int64_t *ys,
                      float *out_f32, uint8_t *flags, double *out_f64) {
    return guarded([&] {
        if (!r || (n > 0 && (!xs || !ys || !out_f32))) fail(FABX_EINVAL, "null argument");
        finish_score(*r->p);
        const auto &R = *r->p;
        if (!R.has_pairs) fail(FABX_EINVAL, "result was scored without keep_pairs");
        const auto &T = *R.task;
        for (int64_t k = 0; k < n; ++k) {
            const int64_t x = xs[k], y = ys[k];
            if (x < 0 || y < 0 || x >= T.ds->n_items || y >= T.ds->n_items)
                fail(FABX_EINVAL, "item id out of range");
            const int64_t px = T.item_pos_of[x], py = T.item_pos_of[y];
            if (px < 0 || py < 0 || T.item_group[px] != T.item_group[py])
                fail(FABX_EINVAL, "pair not in one BY group of the task");
            const Group &g = T.groups[T.item_group[px]];
            const int64_t slot = g.pair_base + (px - g.item0) * g.n_items + (py - g.item0);
            out_f32[k] = R.p32[slot];
            const uint8_t f = R.flags.empty() ? 0 : R.flags[slot];
            if (flags) flags[k] = f;
            if (out_f64) out_f64[k] = (f & 2) ? R.p64[slot] : double(R.p32[slot]);
        }
    });
}

int fabx_result_stats(const fabx_result *r, fabx_stats *st) {
    return guarded([&] {
        if (!r || !st) fail(FABX_EINVAL, "null argument");
        finish_score(*r->p);
        *st = r->p->stats;
    });
}

int fabx_collapse(const fabx_result *r, const int32_t *level_attr, const int32_t *level_len,
                  int32_t n_levels, double *error_rate) {
    return guarded([&] {
        if (!r || !error_rate) fail(FABX_EINVAL, "null argument");
        if (n_levels < 0 || (n_levels > 0 && (!level_attr || !level_len))) fail(FABX_EINVAL, "bad levels");
        finish_score(*r->p);
        *error_rate = collapse(*r->p, level_attr, level_len, n_levels);
    });
}

}  // extern "C"
