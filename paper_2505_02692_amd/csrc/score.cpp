// Score orchestration: device tables, workspace, work plans and the launch
// sequence of one fabx_score call.
#include <algorithm>
#include <cmath>
#include <cstring>

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
constexpr int kRowBlock = 64;    // fused kernel: frames per row block
constexpr int kColBlock = 128;   // fused kernel: frames per column block
constexpr int64_t kUnitBudget = 8192;  // comparisons per triplet work unit (at least one x)

int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

template <typename T>
void upload(DevBuf &b, const std::vector<T> &v, hipStream_t s) {
    b.ensure(std::max<size_t>(v.size() * sizeof(T), 16));
    if (!v.empty())
        FABX_HIP(hipMemcpyAsync(b.ptr, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
}

struct Plans {
    std::vector<int32_t> units;                 // triplets: [n][3]
    std::vector<int64_t> tiles_prefix;          // Gram tile prefix (plain / pooled)
    std::vector<int32_t> rb, cb;                // fused: blocks [n][4]
    std::vector<int32_t> g_rb0, g_cb0, g_nrb, g_ncb;
    std::vector<int64_t> unit_prefix;
    int64_t sum_nx = 0;
    int64_t fused_cells = 0;                    // DTW cells the fused kernel evaluates
};

void pack_blocks(const TaskImpl &t, const Group &g, int limit, std::vector<int32_t> &out) {
    int64_t k = g.item0, end = g.item0 + g.n_items;
    while (k < end) {
        int32_t first = int32_t(k), frames = 0, n = 0;
        while (k < end && frames + t.item_len[k] <= limit) {
            frames += t.item_len[k];
            ++n;
            ++k;
        }
        out.insert(out.end(), {int32_t(&g - t.groups.data()), first, n, frames});
    }
}

Plans make_plans(const TaskImpl &t, const ScoreParams &p) {
    Plans pl;
    // triplet units: split the X set of big cells so one unit does <= kUnitBudget comparisons
    for (size_t c = 0; c < t.cells.size(); ++c) {
        const CellDev &cd = t.cells[c];
        const int64_t per_x = std::max<int64_t>(1, int64_t(cd.na) * cd.nb);
        const int64_t chunk = std::max<int64_t>(1, kUnitBudget / per_x);
        for (int64_t x = 0; x < cd.nx; x += chunk)
            pl.units.insert(pl.units.end(),
                            {int32_t(c), int32_t(x), int32_t(std::min<int64_t>(cd.nx, x + chunk))});
        pl.sum_nx += cd.nx;
    }
    const bool bf16 = p.precision == FABX_PREC_BF16_RECHECK;
    const int64_t G = int64_t(t.groups.size());
    if (p.mode == FABX_MODE_DTW && bf16) {
        pl.unit_prefix.assign(size_t(G + 1), 0);
        for (int64_t gi = 0; gi < G; ++gi) {
            const Group &g = t.groups[gi];
            pl.g_rb0.push_back(int32_t(pl.rb.size() / 4));
            pl.g_cb0.push_back(int32_t(pl.cb.size() / 4));
            pack_blocks(t, g, kRowBlock, pl.rb);
            pack_blocks(t, g, kColBlock, pl.cb);
            const int32_t nrb = int32_t(pl.rb.size() / 4) - pl.g_rb0.back();
            const int32_t ncb = int32_t(pl.cb.size() / 4) - pl.g_cb0.back();
            pl.g_nrb.push_back(nrb);
            pl.g_ncb.push_back(ncb);
            pl.unit_prefix[gi + 1] = pl.unit_prefix[gi] + int64_t(nrb) * ncb;
            pl.fused_cells += g.n_frames * g.n_frames;
        }
    } else {
        // plain Gram tiles (64 x 64), or BF16 pooled tiles (64 x 128)
        pl.tiles_prefix.assign(size_t(G + 1), 0);
        for (int64_t gi = 0; gi < G; ++gi) {
            const Group &g = t.groups[gi];
            const int64_t n = p.mode == FABX_MODE_DTW ? g.n_frames : g.n_items;
            const int64_t tr = (n + 63) / 64;
            const int64_t tc = bf16 ? (n + 127) / 128 : tr;
            pl.tiles_prefix[gi + 1] = pl.tiles_prefix[gi] + tr * tc;
        }
    }
    return pl;
}

struct Timer {
    hipEvent_t ev[8];
    int n = 0;
    hipStream_t s;
    explicit Timer(hipStream_t st) : s(st) {
        for (auto &e : ev) FABX_HIP(hipEventCreate(&e));
    }
    ~Timer() {
        for (auto &e : ev) (void)hipEventDestroy(e);
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
    if (o.distance != FABX_DISTANCE_ANGULAR) fail(FABX_EINVAL, "only the angular distance is implemented");
    if (o.mode != FABX_MODE_DTW && o.mode != FABX_MODE_POOLED) fail(FABX_EINVAL, "bad mode");
    if (o.precision != FABX_PREC_FP32 && o.precision != FABX_PREC_BF16_RECHECK)
        fail(FABX_EINVAL, "bad precision");
    if (o.dtw_norm != FABX_NORM_PATH && o.dtw_norm != FABX_NORM_NONE) fail(FABX_EINVAL, "bad dtw_norm");
    if (std::isnan(o.margin) || std::isnan(o.delta)) fail(FABX_EINVAL, "margin / delta is NaN");
    ScoreParams p;
    p.mode = o.mode;
    p.precision = o.precision;
    p.dtw_norm = o.dtw_norm;
    p.margin = o.margin < 0 ? kMarginK / std::sqrt(double(ds.dim)) : o.margin;
    p.delta = o.delta < 0 ? kDeltaK / std::sqrt(double(ds.dim)) : o.delta;
    p.keep_pairs = o.keep_pairs != 0;
    if (p.mode == FABX_MODE_DTW && ds.max_len > FABX_MAX_ITEM_FRAMES)
        fail(FABX_EINVAL, "an item is longer than FABX_MAX_ITEM_FRAMES frames (DTW mode)");
    if (ds.dim > 2048) fail(FABX_EINVAL, "feature dim above 2048 is not supported");
    return p;
}

int64_t footprint_bytes(const TaskImpl &t, const ScoreParams &p) {
    const bool bf16 = p.precision == FABX_PREC_BF16_RECHECK;
    const int64_t dim_pad = round_up(t.ds->dim, 64);
    const int64_t rows = p.mode == FABX_MODE_DTW ? t.n_frames : int64_t(t.items.size());
    int64_t b = rows * dim_pad * (bf16 ? 2 : 4) + rows * 4;
    if (p.mode == FABX_MODE_DTW && !bf16) b += t.n_dmat * 4;
    b += t.n_pair_slots * 4;
    if (bf16) b += t.n_pair_slots * (1 + 8 + 8);
    int64_t sum_nx = 0;
    for (auto &c : t.cells) sum_nx += c.nx;
    b += int64_t(t.cells.size()) * (8 + 32 + 12) + sum_nx * 8 + int64_t(t.items.size()) * 24;
    return b + (1 << 20);
}

size_t Workspace::total() const {
    const DevBuf *all[] = {&xn, &rinv, &dmat, &p32, &flags, &p64, &half_units, &counters,
                           &recheck_list, &recount_list};
    size_t s = 0;
    for (auto *b : all) s += b->bytes;
    return s;
}

void Workspace::release() {
    DevBuf *all[] = {&xn, &rinv, &dmat, &p32, &flags, &p64, &half_units, &counters,
                     &recheck_list, &recount_list};
    for (auto *b : all) b->release();
}

std::shared_ptr<ResultImpl> run_score(const std::shared_ptr<TaskImpl> &tp, const ScoreParams &p,
                                      hipStream_t stream) {
    TaskImpl &t = *tp;
    std::lock_guard<std::mutex> lock(t.mu);
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
    st.margin = p.precision == FABX_PREC_BF16_RECHECK ? p.margin : 0.0;
    st.delta = p.precision == FABX_PREC_BF16_RECHECK && p.mode == FABX_MODE_DTW ? p.delta : 0.0;
    if (n_cells == 0) return res;
    if (ds.ctx->device < 0) fail(FABX_EINVAL, "context has no device (host-only context)");
    FABX_HIP(hipSetDevice(ds.ctx->device));

    const bool bf16 = p.precision == FABX_PREC_BF16_RECHECK;
    const bool dtw = p.mode == FABX_MODE_DTW;
    const int dim = ds.dim;
    const int dim_pad = int(round_up(dim, 64));
    const int64_t n_items = int64_t(t.items.size());
    const int64_t G = int64_t(t.groups.size());
    Plans pl = make_plans(t, p);
    const int64_t n_units = int64_t(pl.units.size() / 3);

    // ---- device tables (items / groups / cells are fixed for the task)
    TaskDevice &dv = t.dev;
    for (DevBuf *b : {&dv.item_src, &dv.item_len, &dv.item_dst, &dv.item_group, &dv.g_item0, &dv.g_n,
                      &dv.g_frame0, &dv.g_nframes, &dv.g_pair_base, &dv.g_dmat_base, &dv.cells})
        if (!b->ptr) b->pool = &ds.ctx->pool;
    for (DevBuf *b : {&t.ws.xn, &t.ws.rinv, &t.ws.dmat, &t.ws.p32, &t.ws.flags, &t.ws.p64,
                      &t.ws.half_units, &t.ws.counters, &t.ws.recheck_list, &t.ws.recount_list})
        if (!b->ptr) b->pool = &ds.ctx->pool;
    if (!dv.uploaded) {
        upload(dv.item_src, t.item_src, stream);
        upload(dv.item_len, t.item_len, stream);
        upload(dv.item_dst, t.item_dst, stream);
        upload(dv.item_group, t.item_group, stream);
        const size_t ng = static_cast<size_t>(G);
        std::vector<int64_t> a(ng), b(ng + 1), c(ng), d(ng), e(ng), f(ng + 1);
        for (int64_t i = 0; i < G; ++i) {
            a[i] = t.groups[i].item0;
            b[i] = t.groups[i].n_items;
            c[i] = t.groups[i].frame0;
            d[i] = t.groups[i].n_frames;
            e[i] = t.groups[i].dmat_base;
            f[i] = t.groups[i].pair_base;
        }
        b[G] = 0;
        f[G] = t.n_pair_slots;
        upload(dv.g_item0, a, stream);
        upload(dv.g_n, b, stream);
        upload(dv.g_frame0, c, stream);
        upload(dv.g_nframes, d, stream);
        upload(dv.g_dmat_base, e, stream);
        upload(dv.g_pair_base, f, stream);
        upload(dv.cells, t.cells, stream);
        dv.uploaded = true;
    }
    DevBuf units_d, tiles_d, rb_d, cb_d, up_d, grb_d, gcb_d, gncb_d;
    Pool *pool = &ds.ctx->pool;
    for (DevBuf *b : {&units_d, &tiles_d, &rb_d, &cb_d, &up_d, &grb_d, &gcb_d, &gncb_d}) b->pool = pool;
    upload(units_d, pl.units, stream);
    if (!pl.tiles_prefix.empty()) upload(tiles_d, pl.tiles_prefix, stream);
    if (!pl.unit_prefix.empty()) {
        upload(rb_d, pl.rb, stream);
        upload(cb_d, pl.cb, stream);
        upload(up_d, pl.unit_prefix, stream);
        upload(grb_d, pl.g_rb0, stream);
        upload(gcb_d, pl.g_cb0, stream);
        upload(gncb_d, pl.g_ncb, stream);
    }

    // ---- workspace
    Workspace &ws = t.ws;
    const int64_t rows = dtw ? t.n_frames : n_items;
    ws.xn.ensure(size_t(rows) * dim_pad * (bf16 ? 2 : 4));
    if (bf16) ws.rinv.ensure(size_t(rows) * 4);
    if (dtw && !bf16) ws.dmat.ensure(size_t(std::max<int64_t>(t.n_dmat, 1)) * 4);
    ws.p32.ensure(size_t(t.n_pair_slots) * 4);
    if (bf16) {
        ws.flags.ensure(size_t(t.n_pair_slots));
        ws.p64.ensure(size_t(t.n_pair_slots) * 8);
        ws.recheck_list.ensure(size_t(t.n_pair_slots) * 8);
        ws.recount_list.ensure(size_t(pl.sum_nx) * 8);
    }
    ws.half_units.ensure(size_t(n_cells) * 8);
    ws.counters.ensure(64);
    int *err = ws.counters.as<int>();
    unsigned long long *err_item = reinterpret_cast<unsigned long long *>(ws.counters.as<char>() + 8);
    unsigned int *recount_n = reinterpret_cast<unsigned int *>(ws.counters.as<char>() + 16);
    unsigned int *marked_n = reinterpret_cast<unsigned int *>(ws.counters.as<char>() + 20);
    unsigned int *nonrobust_n = reinterpret_cast<unsigned int *>(ws.counters.as<char>() + 24);
    st.workspace_bytes = int64_t(ws.total());

    kern::ItemTables it{dv.item_src.as<int64_t>(), dv.item_len.as<int32_t>(), dv.item_dst.as<int64_t>(),
                        n_items};
    kern::GroupTables gt{dv.g_item0.as<int64_t>(), dv.g_n.as<int64_t>(), dv.g_frame0.as<int64_t>(),
                         dv.g_nframes.as<int64_t>(), dv.g_pair_base.as<int64_t>(),
                         dv.g_dmat_base.as<int64_t>(), G, t.n_pair_slots};

    Timer tm(stream);
    tm.mark();  // 0
    FABX_HIP(hipMemsetAsync(ws.counters.ptr, 0, 64, stream));
    FABX_HIP(hipMemsetAsync(err_item, 0xFF, 8, stream));
    FABX_HIP(hipMemsetAsync(ws.half_units.ptr, 0, size_t(n_cells) * 8, stream));
    if (bf16 && !dtw) FABX_HIP(hipMemsetAsync(ws.flags.ptr, 0, size_t(t.n_pair_slots), stream));
    tm.mark();  // 1
    if (dtw)
        kern::normalize(stream, ds.features, ds.dtype, dim, dim_pad, it, ws.xn.ptr, bf16 ? 1 : 0,
                        ws.rinv.as<float>(), err, err_item);
    else
        kern::pool_normalize(stream, ds.features, ds.dtype, dim, dim_pad, it, ws.xn.ptr, bf16 ? 1 : 0,
                             ws.rinv.as<float>(), err, err_item);
    tm.mark();  // 2
    if (dtw && !bf16) {
        kern::gram_angular_f32(stream, ws.xn.as<float>(), dim_pad, gt.frame0, gt.n_frames, gt.dmat_base,
                               tiles_d.as<int64_t>(), G, pl.tiles_prefix.back(), ws.dmat.as<float>());
        kern::dtw_plain(stream, ws.dmat.as<float>(), gt, it, p.dtw_norm, ws.p32.as<float>());
        st.computed_dtw_cells = t.n_dmat;
    } else if (dtw) {
        kern::FusedPlan fp{rb_d.as<int32_t>(), cb_d.as<int32_t>(), up_d.as<int64_t>(), grb_d.as<int32_t>(),
                           gcb_d.as<int32_t>(), nullptr, gncb_d.as<int32_t>(), pl.unit_prefix.back()};
        kern::fused_bf16(stream, ws.xn.as<uint16_t>(), ws.rinv.as<float>(), dim_pad, gt, it, fp,
                         p.dtw_norm, float(p.delta), ws.p32.as<float>(), ws.flags.as<uint8_t>(),
                         nonrobust_n);
        st.computed_dtw_cells = pl.fused_cells;
    } else if (!bf16) {
        kern::gram_angular_f32(stream, ws.xn.as<float>(), dim_pad, gt.item0, gt.n_items, gt.pair_base,
                               tiles_d.as<int64_t>(), G, pl.tiles_prefix.back(), ws.p32.as<float>());
    } else {
        kern::gram_angular_bf16(stream, ws.xn.as<uint16_t>(), ws.rinv.as<float>(), dim_pad, gt.item0,
                                gt.n_items, gt.pair_base, tiles_d.as<int64_t>(), G,
                                pl.tiles_prefix.back(), ws.p32.as<float>());
    }
    tm.mark();  // 3
    kern::triplets(stream, dv.cells.as<CellDev>(), units_d.as<int32_t>(), n_units, gt,
                   ws.p32.as<float>(), ws.half_units.as<unsigned long long>(),
                   bf16 ? ws.flags.as<uint8_t>() : nullptr, float(p.margin),
                   bf16 ? ws.recount_list.as<int32_t>() : nullptr, recount_n, pl.sum_nx);
    tm.mark();  // 4
    if (bf16) {
        kern::collect_marked(stream, ws.flags.as<uint8_t>(), t.n_pair_slots, ws.recheck_list.as<int64_t>(),
                             marked_n, t.n_pair_slots);
        kern::recheck_fp64(stream, ds.features, ds.dtype, dim, gt, it, ws.recheck_list.as<int64_t>(),
                           marked_n, t.n_pair_slots, p.mode, p.dtw_norm, ws.p64.as<double>());
        kern::recount(stream, dv.cells.as<CellDev>(), ws.recount_list.as<int32_t>(), recount_n, pl.sum_nx,
                      gt, ws.p32.as<float>(), ws.p64.as<double>(), ws.flags.as<uint8_t>(),
                      ws.half_units.as<unsigned long long>());
    }
    tm.mark();  // 5
    unsigned char counters[64];
    FABX_HIP(hipMemcpyAsync(res->half_units.data(), ws.half_units.ptr, size_t(n_cells) * 8,
                            hipMemcpyDeviceToHost, stream));
    FABX_HIP(hipMemcpyAsync(counters, ws.counters.ptr, 64, hipMemcpyDeviceToHost, stream));
    tm.mark();  // 6
    FABX_HIP(hipStreamSynchronize(stream));
    int err_h;
    unsigned long long err_item_h;
    unsigned int recount_h, marked_h, nonrobust_h;
    std::memcpy(&err_h, counters, 4);
    std::memcpy(&nonrobust_h, counters + 24, 4);
    std::memcpy(&err_item_h, counters + 8, 8);
    std::memcpy(&recount_h, counters + 16, 4);
    std::memcpy(&marked_h, counters + 20, 4);
    if (err_h) {
        const int64_t bad = err_item_h < uint64_t(n_items) ? t.items[size_t(err_item_h)] : -1;
        fail(FABX_EDOMAIN, "zero-norm " + std::string(dtw ? "frame" : "mean") + " in item " +
                               std::to_string(bad) + ": its angle is undefined");
    }
    st.ms_normalize = tm.ms(1, 2);
    st.ms_distance = tm.ms(2, 3);
    st.ms_triplets = tm.ms(3, 4);
    st.ms_recheck = tm.ms(4, 5);
    st.ms_total = tm.ms(0, 6);
    st.n_recheck_pairs = marked_h;
    st.n_recount_rows = recount_h;
    st.n_nonrobust_pairs = nonrobust_h;
    if (p.keep_pairs) {
        res->has_pairs = true;
        res->p32.resize(size_t(t.n_pair_slots));
        FABX_HIP(hipMemcpy(res->p32.data(), ws.p32.ptr, res->p32.size() * 4, hipMemcpyDeviceToHost));
        if (bf16) {
            res->flags.resize(size_t(t.n_pair_slots));
            FABX_HIP(hipMemcpy(res->flags.data(), ws.flags.ptr, res->flags.size(), hipMemcpyDeviceToHost));
            res->p64.resize(size_t(t.n_pair_slots));
            FABX_HIP(hipMemcpy(res->p64.data(), ws.p64.ptr, res->p64.size() * 8, hipMemcpyDeviceToHost));
        }
    }
    return res;
}

}  // namespace fabx
