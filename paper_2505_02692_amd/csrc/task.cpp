// Task construction: group items by BY value, split groups into classes of
// equal (ON, ACROSS) value, and enumerate the cells (Background section: the
// ON / BY / ACROSS conditions, and the cell A x B x X).
//
// All host integer work.  Items are ordered once by a composite key
// (by..., on, across...) with an LSD radix sort, so every BY group and every
// class is a contiguous run; a cell is then three runs (A, B, X).
#include <algorithm>
#include <cstring>
#include <numeric>

#include "internal.h"

namespace fabx {
namespace {

struct RankedColumn {
    std::vector<int32_t> values;   // sorted unique attribute values
    std::vector<uint32_t> rank;    // per item: index into values
    int bits = 0;                  // bits needed to hold a rank
};

RankedColumn rank_column(const DatasetImpl &ds, int col) {
    RankedColumn rc;
    const int64_t n = ds.n_items;
    rc.values.resize(n);
    for (int64_t i = 0; i < n; ++i) rc.values[i] = ds.attrs[i * ds.n_attr + col];
    std::vector<int32_t> raw = rc.values;
    std::sort(rc.values.begin(), rc.values.end());
    rc.values.erase(std::unique(rc.values.begin(), rc.values.end()), rc.values.end());
    rc.rank.resize(n);
    for (int64_t i = 0; i < n; ++i)
        rc.rank[i] = uint32_t(std::lower_bound(rc.values.begin(), rc.values.end(), raw[i]) -
                              rc.values.begin());
    uint64_t u = rc.values.size();
    while ((uint64_t(1) << rc.bits) < u) ++rc.bits;
    return rc;
}

// Stable LSD radix sort of items by a 64-bit key (8-bit digits, only the
// digits the key uses).  Ties keep ascending item order.
void radix_sort(std::vector<uint64_t> &key, std::vector<int64_t> &idx, int key_bits) {
    const size_t n = key.size();
    std::vector<uint64_t> k2(n);
    std::vector<int64_t> i2(n);
    for (int shift = 0; shift < key_bits; shift += 8) {
        size_t count[257] = {0};
        for (size_t i = 0; i < n; ++i) ++count[((key[i] >> shift) & 0xFF) + 1];
        for (int b = 0; b < 256; ++b) count[b + 1] += count[b];
        for (size_t i = 0; i < n; ++i) {
            size_t d = count[(key[i] >> shift) & 0xFF]++;
            k2[d] = key[i];
            i2[d] = idx[i];
        }
        key.swap(k2);
        idx.swap(i2);
    }
}

struct ClassRun {
    int64_t start;      // position in sorted order
    int64_t count;
    uint32_t on_rank;
    int64_t first;      // one item of the class (for its ACROSS ranks)
};

}  // namespace

std::shared_ptr<TaskImpl> build_task(const std::shared_ptr<DatasetImpl> &ds, int32_t on,
                                     const int32_t *by, int32_t n_by, const int32_t *across,
                                     int32_t n_across) {
    if (n_by < 0 || n_across < 0) fail(FABX_EINVAL, "n_by and n_across must be >= 0");
    if ((n_by > 0 && !by) || (n_across > 0 && !across)) fail(FABX_EINVAL, "null by/across array");
    std::vector<int32_t> cols;
    cols.push_back(on);
    for (int i = 0; i < n_by; ++i) cols.push_back(by[i]);
    for (int i = 0; i < n_across; ++i) cols.push_back(across[i]);
    for (int32_t c : cols)
        if (c < 0 || c >= ds->n_attr) fail(FABX_EINVAL, "attribute column out of range");
    {
        std::vector<int32_t> s = cols;
        std::sort(s.begin(), s.end());
        if (std::adjacent_find(s.begin(), s.end()) != s.end())
            fail(FABX_EINVAL, "ON, BY and ACROSS attributes must be distinct");
    }

    auto t = std::make_shared<TaskImpl>();
    t->ds = ds;
    t->on = on;
    t->by.assign(by, by + n_by);
    t->across.assign(across, across + n_across);
    t->key_attr = {on, on};
    for (int32_t c : t->by) t->key_attr.push_back(c);
    for (int32_t c : t->across) t->key_attr.push_back(c);
    for (int32_t c : t->across) t->key_attr.push_back(c);
    t->key_width = int32_t(t->key_attr.size());

    const int64_t n = ds->n_items;
    // ---- composite key: by fields (high), on, across fields (low)
    std::vector<RankedColumn> rby, racr;
    for (int32_t c : t->by) rby.push_back(rank_column(*ds, c));
    RankedColumn ron = rank_column(*ds, on);
    for (int32_t c : t->across) racr.push_back(rank_column(*ds, c));
    int acr_bits = 0;
    std::vector<int> acr_shift(n_across);
    for (int k = n_across - 1; k >= 0; --k) {
        acr_shift[k] = acr_bits;
        acr_bits += racr[k].bits;
    }
    int low_bits = acr_bits + ron.bits;
    int total_bits = low_bits;
    for (auto &r : rby) total_bits += r.bits;

    std::vector<int64_t> order(n);
    std::iota(order.begin(), order.end(), int64_t(0));
    std::vector<uint64_t> by_part(n, 0), cls_part(n, 0);   // BY tuple id / (on, across) class id
    if (total_bits <= 64) {
        std::vector<uint64_t> key(n);
        for (int64_t i = 0; i < n; ++i) {
            uint64_t k = 0;
            for (auto &r : rby) k = (k << r.bits) | r.rank[i];
            k = (k << ron.bits) | ron.rank[i];
            uint64_t a = 0;
            for (int j = 0; j < n_across; ++j) a |= uint64_t(racr[j].rank[i]) << acr_shift[j];
            key[i] = (k << acr_bits) | a;
        }
        radix_sort(key, order, total_bits);
        for (int64_t s = 0; s < n; ++s) {
            by_part[s] = low_bits >= 64 ? 0 : key[s] >> low_bits;
            cls_part[s] = key[s];
        }
    } else {
        // Key too wide for one word: comparison sort on the rank tuple.
        std::stable_sort(order.begin(), order.end(), [&](int64_t x, int64_t y) {
            for (auto &r : rby)
                if (r.rank[x] != r.rank[y]) return r.rank[x] < r.rank[y];
            if (ron.rank[x] != ron.rank[y]) return ron.rank[x] < ron.rank[y];
            for (auto &r : racr)
                if (r.rank[x] != r.rank[y]) return r.rank[x] < r.rank[y];
            return false;
        });
        uint64_t gid = 0, cid = 0;
        for (int64_t s = 0; s < n; ++s) {
            if (s > 0) {
                int64_t x = order[s - 1], y = order[s];
                bool same_by = true;
                for (auto &r : rby) same_by = same_by && r.rank[x] == r.rank[y];
                bool same_cls = same_by && ron.rank[x] == ron.rank[y];
                for (auto &r : racr) same_cls = same_cls && r.rank[x] == r.rank[y];
                gid += !same_by;
                cid += !same_cls;
            }
            by_part[s] = gid;
            cls_part[s] = cid;
        }
    }
    // ACROSS tuples of two items: lexicographic order (the sort order) and "differ in every one"
    auto across_cmp = [&](int64_t a, int64_t b) {
        for (int j = 0; j < n_across; ++j)
            if (racr[j].rank[a] != racr[j].rank[b]) return racr[j].rank[a] < racr[j].rank[b] ? -1 : 1;
        return 0;
    };
    auto across_all_differ = [&](int64_t a, int64_t b) {
        for (int j = 0; j < n_across; ++j)
            if (racr[j].rank[a] == racr[j].rank[b]) return false;
        return true;
    };

    // ---- walk groups and classes
    std::vector<int64_t> kept_pos;   // sorted positions of items kept, in task order
    kept_pos.reserve(n);
    std::vector<ClassRun> cls;
    std::vector<uint8_t> need;       // class-pair need matrix of the current group
    int64_t g0 = 0;
    while (g0 < n) {
        int64_t g1 = g0 + 1;
        while (g1 < n && by_part[g1] == by_part[g0]) ++g1;
        cls.clear();
        for (int64_t s = g0; s < g1;) {
            int64_t e = s + 1;
            while (e < g1 && cls_part[e] == cls_part[s]) ++e;
            cls.push_back({s, e - s, ron.rank[order[s]], order[s]});
            s = e;
        }
        const int64_t K = int64_t(cls.size());
        const int32_t group_id = int32_t(t->groups.size());
        const int64_t cells_before = int64_t(t->cells.size());
        // class-pair need matrix (ACROSS tasks only; within tasks use a closed form)
        const bool use_need = n_across > 0 && K <= 8192;
        if (use_need) need.assign(size_t(K * K), 0);
        std::vector<std::pair<int64_t, int64_t>> need_list;
        auto add_cell = [&](int64_t ia, int64_t ib, int64_t ix, bool excl) {
            CellDev c;
            c.group = group_id;
            c.a0 = int32_t(cls[ia].start - g0);
            c.na = int32_t(cls[ia].count);
            c.b0 = int32_t(cls[ib].start - g0);
            c.nb = int32_t(cls[ib].count);
            c.x0 = int32_t(cls[ix].start - g0);
            c.nx = int32_t(cls[ix].count);
            c.exclude_self = excl ? 1 : 0;
            t->cells.push_back(c);
            int64_t nt = excl ? c.na * int64_t(c.na - 1) * c.nb : int64_t(c.na) * c.nb * c.nx;
            t->n_triplets.push_back(nt);
            t->total_triplets += nt;
            const int64_t ia0 = order[cls[ia].start], ib0 = order[cls[ib].start],
                          ix0 = order[cls[ix].start];
            t->keys.push_back(ds->attrs[ia0 * ds->n_attr + on]);
            t->keys.push_back(ds->attrs[ib0 * ds->n_attr + on]);
            for (int32_t b : t->by) t->keys.push_back(ds->attrs[ia0 * ds->n_attr + b]);
            for (int32_t a : t->across) t->keys.push_back(ds->attrs[ia0 * ds->n_attr + a]);
            for (int32_t a : t->across) t->keys.push_back(ds->attrs[ix0 * ds->n_attr + a]);
            if (use_need) {
                need[size_t(ix * K + ia)] = 1;
                need[size_t(ix * K + ib)] = 1;
            } else if (n_across > 0) {
                need_list.push_back({ix, ia});
                need_list.push_back({ix, ib});
            }
        };
        if (n_across == 0) {
            for (int64_t i = 0; i < K; ++i) {
                if (cls[i].count < 2) continue;
                for (int64_t j = 0; j < K; ++j)
                    if (j != i) add_cell(i, j, i, true);
            }
        } else {
            // classes are sorted by (on, across): runs of equal on
            std::vector<std::pair<int64_t, int64_t>> runs;
            for (int64_t i = 0; i < K;) {
                int64_t e = i + 1;
                while (e < K && cls[e].on_rank == cls[i].on_rank) ++e;
                runs.push_back({i, e});
                i = e;
            }
            for (auto &r1 : runs)
                for (auto &r2 : runs) {
                    if (r1.first == r2.first) continue;
                    for (int64_t ia = r1.first; ia < r1.second; ++ia) {
                        // B: same across value, other on value
                        int64_t lo = r2.first, hi = r2.second;
                        while (lo < hi) {
                            int64_t mid = (lo + hi) / 2;
                            if (across_cmp(cls[mid].first, cls[ia].first) < 0) lo = mid + 1; else hi = mid;
                        }
                        if (lo == r2.second || across_cmp(cls[lo].first, cls[ia].first) != 0) continue;
                        for (int64_t ix = r1.first; ix < r1.second; ++ix)
                            if (across_all_differ(cls[ix].first, cls[ia].first))
                                add_cell(ia, lo, ix, false);
                    }
                }
        }
        if (int64_t(t->cells.size()) > cells_before) {
            Group g;
            g.item0 = int64_t(kept_pos.size());
            g.n_items = g1 - g0;
            g.frame0 = 0;
            g.n_frames = 0;
            g.pair_base = t->n_pair_slots;
            g.dmat_base = 0;
            t->n_pair_slots += g.n_items * g.n_items;
            // unique needed pairs and their DTW cells
            std::vector<int64_t> cframes(size_t(K), 0);
            for (int64_t i = 0; i < K; ++i)
                for (int64_t s = cls[i].start; s < cls[i].start + cls[i].count; ++s) {
                    int64_t it = order[s];
                    cframes[size_t(i)] += ds->offsets[it + 1] - ds->offsets[it];
                }
            auto count_pair = [&](int64_t ix, int64_t iy) {
                if (ix == iy) {   // X x A with a != x
                    t->n_pairs_needed += cls[ix].count * (cls[ix].count - 1);
                    int64_t sq = 0;
                    for (int64_t s = cls[ix].start; s < cls[ix].start + cls[ix].count; ++s) {
                        int64_t L = ds->offsets[order[s] + 1] - ds->offsets[order[s]];
                        sq += L * L;
                    }
                    t->dtw_cells_needed += cframes[size_t(ix)] * cframes[size_t(ix)] - sq;
                } else {
                    t->n_pairs_needed += cls[ix].count * cls[iy].count;
                    t->dtw_cells_needed += cframes[size_t(ix)] * cframes[size_t(iy)];
                }
            };
            if (n_across == 0) {
                // every item of a class with >= 2 items is an x; it needs every other item
                for (int64_t ix = 0; ix < K; ++ix) {
                    if (cls[ix].count < 2) continue;
                    for (int64_t iy = 0; iy < K; ++iy) count_pair(ix, iy);
                }
            } else if (use_need) {
                for (int64_t ix = 0; ix < K; ++ix)
                    for (int64_t iy = 0; iy < K; ++iy)
                        if (need[size_t(ix * K + iy)]) count_pair(ix, iy);
            } else {
                std::sort(need_list.begin(), need_list.end());
                need_list.erase(std::unique(need_list.begin(), need_list.end()), need_list.end());
                for (auto &pr : need_list) count_pair(pr.first, pr.second);
            }
            for (int64_t s = g0; s < g1; ++s) kept_pos.push_back(s);
            t->groups.push_back(g);
        }
        g0 = g1;
    }

    // ---- task items in task order, packed frame offsets
    const int64_t nt = int64_t(kept_pos.size());
    t->items.resize(nt);
    t->item_len.resize(nt);
    t->item_src.resize(nt);
    t->item_dst.resize(nt);
    t->item_group.resize(nt);
    t->item_pos_of.assign(size_t(n), -1);
    int64_t frame = 0;
    for (size_t gi = 0; gi < t->groups.size(); ++gi) {
        Group &g = t->groups[gi];
        g.frame0 = frame;
        for (int64_t k = g.item0; k < g.item0 + g.n_items; ++k) {
            int64_t it = order[kept_pos[k]];
            t->items[k] = it;
            t->item_pos_of[it] = k;
            t->item_src[k] = ds->offsets[it];
            t->item_len[k] = int32_t(ds->offsets[it + 1] - ds->offsets[it]);
            t->item_dst[k] = frame;
            t->item_group[k] = int32_t(gi);
            t->max_len = std::max(t->max_len, t->item_len[k]);
            frame += t->item_len[k];
        }
        g.n_frames = frame - g.frame0;
        g.dmat_base = t->n_dmat;
        t->n_dmat += g.n_frames * g.n_frames;
    }
    t->n_frames = frame;
    return t;
}

}  // namespace fabx
