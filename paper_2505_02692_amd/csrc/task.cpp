// Task construction: group items by BY value, split groups into classes of
// equal (ON, ACROSS) value, and enumerate the cells (Background section: the
// ON / BY / ACROSS conditions, and the cell A x B x X).
//
// All host integer work.  Items are ordered once by a composite key
// (by..., on, across...) with an LSD radix sort, so every BY group and every
// class is a contiguous run; a cell is then three runs (A, B, X).
#include <algorithm>
#include <climits>
#include <cstring>
#include <functional>
#include <numeric>
#include <thread>

#include "host_pool.h"
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
    rc.rank.resize(n);
    int32_t mn = INT32_MAX, mx = INT32_MIN;
    for (int64_t i = 0; i < n; ++i) {
        const int32_t v = ds.attrs[i * ds.n_attr + col];
        mn = std::min(mn, v);
        mx = std::max(mx, v);
    }
    const int64_t range = int64_t(mx) - int64_t(mn) + 1;
    if (range <= std::max<int64_t>(4 * n, 1 << 16)) {
        // dense value range: rank by a direct table
        std::vector<int32_t> table(size_t(range), -1);
        for (int64_t i = 0; i < n; ++i) table[size_t(ds.attrs[i * ds.n_attr + col] - int64_t(mn))] = 0;
        int32_t r = 0;
        for (int64_t v = 0; v < range; ++v)
            if (table[size_t(v)] == 0) {
                table[size_t(v)] = r++;
                rc.values.push_back(int32_t(v + mn));
            }
        for (int64_t i = 0; i < n; ++i)
            rc.rank[i] = uint32_t(table[size_t(ds.attrs[i * ds.n_attr + col] - int64_t(mn))]);
    } else {
        rc.values.resize(n);
        for (int64_t i = 0; i < n; ++i) rc.values[i] = ds.attrs[i * ds.n_attr + col];
        std::sort(rc.values.begin(), rc.values.end());
        rc.values.erase(std::unique(rc.values.begin(), rc.values.end()), rc.values.end());
        for (int64_t i = 0; i < n; ++i)
            rc.rank[i] = uint32_t(std::lower_bound(rc.values.begin(), rc.values.end(),
                                                   ds.attrs[i * ds.n_attr + col]) -
                                  rc.values.begin());
    }
    uint64_t u = rc.values.size();
    while ((uint64_t(1) << rc.bits) < u) ++rc.bits;
    return rc;
}

// Stable LSD radix sort of items by a 64-bit key (12-bit digits, only the
// digits the key uses).  Ties keep ascending item order.
void radix_sort(std::vector<uint64_t> &key, std::vector<int64_t> &idx, int key_bits) {
    constexpr int kDigit = 12;
    constexpr size_t kBuckets = size_t(1) << kDigit;
    const size_t n = key.size();
    std::vector<uint64_t> k2(n);
    std::vector<int64_t> i2(n);
    std::vector<size_t> count(kBuckets + 1);
    for (int shift = 0; shift < key_bits; shift += kDigit) {
        std::fill(count.begin(), count.end(), 0);
        for (size_t i = 0; i < n; ++i) ++count[((key[i] >> shift) & (kBuckets - 1)) + 1];
        for (size_t b = 0; b < kBuckets; ++b) count[b + 1] += count[b];
        for (size_t i = 0; i < n; ++i) {
            size_t d = count[(key[i] >> shift) & (kBuckets - 1)]++;
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


template <typename F>
void parallel_for(int n, F &&f) {
    const std::function<void(int)> fn = f;
    HostPool::get().parallel_for(n, fn);
}

// Output of one thread's share of the group walk (group ids and pair-slot
// bases local to the share; stitched together afterwards).
struct WalkOut {
    std::vector<CellDev> cells;
    std::vector<int64_t> ntrip;
    std::vector<int32_t> keys;
    std::vector<uint32_t> rkeys;
    std::vector<int32_t> units;                     // [n][3], cell ids local to this share
    std::vector<Group> groups;
    std::vector<std::pair<int64_t, int64_t>> kept;  // sorted-order range of each kept group
    int64_t total_triplets = 0, pairs_needed = 0, dtw_needed = 0, pair_slots = 0, sum_nx = 0;
    void swap(WalkOut &o) {
        cells.swap(o.cells);
        ntrip.swap(o.ntrip);
        keys.swap(o.keys);
        rkeys.swap(o.rkeys);
        units.swap(o.units);
        groups.swap(o.groups);
        kept.swap(o.kept);
    }
};

constexpr int64_t kUnitBudget = 8192;  // comparisons per triplet work unit (at least one x)

struct WalkCtx {
    const DatasetImpl *ds;
    const TaskImpl *t;
    const std::vector<int64_t> *order;
    const std::vector<uint64_t> *by_part, *cls_part;
    const std::vector<uint32_t> *on_rank;
    const std::vector<const std::vector<uint32_t> *> *by_rank, *across_rank;
    const std::vector<int64_t> *pf, *pq;
    int32_t on;
    int32_t n_across;
    std::function<int(int64_t, int64_t)> across_cmp;
    std::function<bool(int64_t, int64_t)> across_all_differ;
};

// Cells of the groups that start in sorted positions [s_begin, s_end).
void walk_groups(const WalkCtx &w, int64_t s_begin, int64_t s_end, WalkOut &out) {
    const auto &order = *w.order;
    const auto &by_part = *w.by_part;
    const auto &cls_part = *w.cls_part;
    const auto &pf = *w.pf;
    const auto &pq = *w.pq;
    const int32_t *A = w.ds->attrs.data();
    const int NA = w.ds->n_attr;
    const TaskImpl &t = *w.t;
    std::vector<ClassRun> cls;
    std::vector<uint8_t> need;
    std::vector<std::pair<int64_t, int64_t>> need_list, runs;
    int64_t g0 = s_begin;
    while (g0 < s_end) {
        int64_t g1 = g0 + 1;
        while (g1 < s_end && by_part[g1] == by_part[g0]) ++g1;
        cls.clear();
        for (int64_t s = g0; s < g1;) {
            int64_t e = s + 1;
            while (e < g1 && cls_part[e] == cls_part[s]) ++e;
            cls.push_back({s, e - s, (*w.on_rank)[order[s]], order[s]});
            s = e;
        }
        const int64_t K = int64_t(cls.size());
        const int32_t group_id = int32_t(out.groups.size());
        const size_t cells_before = out.cells.size();
        const bool use_need = w.n_across > 0 && K <= 8192;
        if (use_need) need.assign(size_t(K * K), 0);
        need_list.clear();
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
            out.cells.push_back(c);
            const int64_t nt = excl ? c.na * int64_t(c.na - 1) * c.nb : int64_t(c.na) * c.nb * c.nx;
            out.ntrip.push_back(nt);
            out.total_triplets += nt;
            const int32_t *ka = A + cls[ia].first * NA;
            const int32_t *kb = A + cls[ib].first * NA;
            const int32_t *kx = A + cls[ix].first * NA;
            out.keys.push_back(ka[w.on]);
            out.keys.push_back(kb[w.on]);
            for (int32_t b : t.by) out.keys.push_back(ka[b]);
            for (int32_t a : t.across) out.keys.push_back(ka[a]);
            for (int32_t a : t.across) out.keys.push_back(kx[a]);
            const int64_t ia0 = cls[ia].first, ib0 = cls[ib].first, ix0 = cls[ix].first;
            out.rkeys.push_back((*w.on_rank)[ia0]);
            out.rkeys.push_back((*w.on_rank)[ib0]);
            for (auto *r : *w.by_rank) out.rkeys.push_back((*r)[ia0]);
            for (auto *r : *w.across_rank) out.rkeys.push_back((*r)[ia0]);
            for (auto *r : *w.across_rank) out.rkeys.push_back((*r)[ix0]);
            // triplet work units: split X so one unit does <= kUnitBudget comparisons
            const int64_t per_x = std::max<int64_t>(1, int64_t(c.na) * c.nb);
            const int64_t chunk = std::max<int64_t>(1, kUnitBudget / per_x);
            const int32_t cid = int32_t(out.cells.size() - 1);
            for (int64_t x = 0; x < c.nx; x += chunk) {
                out.units.push_back(cid);
                out.units.push_back(int32_t(x));
                out.units.push_back(int32_t(std::min<int64_t>(c.nx, x + chunk)));
            }
            out.sum_nx += c.nx;
            if (use_need) {
                need[size_t(ix * K + ia)] = 1;
                need[size_t(ix * K + ib)] = 1;
            } else if (w.n_across > 0) {
                need_list.push_back({ix, ia});
                need_list.push_back({ix, ib});
            }
        };
        if (w.n_across == 0) {
            for (int64_t i = 0; i < K; ++i) {
                if (cls[i].count < 2) continue;
                for (int64_t j = 0; j < K; ++j)
                    if (j != i) add_cell(i, j, i, true);
            }
        } else {
            // classes are sorted by (on, across): runs of equal on
            runs.clear();
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
                            if (w.across_cmp(cls[mid].first, cls[ia].first) < 0) lo = mid + 1; else hi = mid;
                        }
                        if (lo == r2.second || w.across_cmp(cls[lo].first, cls[ia].first) != 0) continue;
                        for (int64_t ix = r1.first; ix < r1.second; ++ix)
                            if (w.across_all_differ(cls[ix].first, cls[ia].first))
                                add_cell(ia, lo, ix, false);
                    }
                }
        }
        if (out.cells.size() > cells_before) {
            Group g{};
            g.n_items = g1 - g0;
            g.pair_base = out.pair_slots;
            out.pair_slots += g.n_items * g.n_items;
            // unique needed pairs and their DTW cells, from prefix sums over sorted positions
            auto cnt = [&](int64_t i) { return cls[i].count; };
            auto frames = [&](int64_t i) { return pf[cls[i].start + cls[i].count] - pf[cls[i].start]; };
            auto sq = [&](int64_t i) { return pq[cls[i].start + cls[i].count] - pq[cls[i].start]; };
            auto count_pair = [&](int64_t ix, int64_t iy) {
                if (ix == iy) {   // X x A with a != x
                    out.pairs_needed += cnt(ix) * (cnt(ix) - 1);
                    out.dtw_needed += frames(ix) * frames(ix) - sq(ix);
                } else {
                    out.pairs_needed += cnt(ix) * cnt(iy);
                    out.dtw_needed += frames(ix) * frames(iy);
                }
            };
            if (w.n_across == 0) {
                // every item of a class with >= 2 items is an x; it needs every other item
                const int64_t all_items = g1 - g0, all_frames = pf[g1] - pf[g0];
                for (int64_t ix = 0; ix < K; ++ix) {
                    if (cnt(ix) < 2) continue;
                    out.pairs_needed += cnt(ix) * (all_items - 1);
                    out.dtw_needed += frames(ix) * all_frames - sq(ix);
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
            out.kept.push_back({g0, g1});
            out.groups.push_back(g);
        }
        g0 = g1;
    }
}

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

    Trace tr("task");
    const int64_t n = ds->n_items;
    // ---- composite key: by fields (high), on, across fields (low)
    std::vector<RankedColumn> rby(t->by.size()), racr(t->across.size());
    RankedColumn ron;
    {
        std::vector<int32_t> all_cols = cols;   // on, by..., across...
        std::vector<RankedColumn> ranked(all_cols.size());
        parallel_for(int(all_cols.size()), [&](int k) { ranked[size_t(k)] = rank_column(*ds, all_cols[size_t(k)]); });
        ron = std::move(ranked[0]);
        for (size_t i = 0; i < rby.size(); ++i) rby[i] = std::move(ranked[1 + i]);
        for (size_t i = 0; i < racr.size(); ++i) racr[i] = std::move(ranked[1 + rby.size() + i]);
    }
    int acr_bits = 0;
    std::vector<int> acr_shift(n_across);
    for (int k = n_across - 1; k >= 0; --k) {
        acr_shift[k] = acr_bits;
        acr_bits += racr[k].bits;
    }
    int low_bits = acr_bits + ron.bits;
    int total_bits = low_bits;
    for (auto &r : rby) total_bits += r.bits;

    tr.mark("rank");
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
    std::function<int(int64_t, int64_t)> across_cmp = [&](int64_t a, int64_t b) {
        for (int j = 0; j < n_across; ++j)
            if (racr[j].rank[a] != racr[j].rank[b]) return racr[j].rank[a] < racr[j].rank[b] ? -1 : 1;
        return 0;
    };
    std::function<bool(int64_t, int64_t)> across_all_differ = [&](int64_t a, int64_t b) {
        for (int j = 0; j < n_across; ++j)
            if (racr[j].rank[a] == racr[j].rank[b]) return false;
        return true;
    };

    tr.mark("sort");
    // ---- per sorted position: length, and prefix sums of frames and squared lengths
    std::vector<int32_t> len_s(static_cast<size_t>(n));
    std::vector<int64_t> pf(static_cast<size_t>(n) + 1, 0), pq(static_cast<size_t>(n) + 1, 0);
    for (int64_t s = 0; s < n; ++s) {
        const int64_t L = ds->offsets[order[s] + 1] - ds->offsets[order[s]];
        len_s[s] = int32_t(L);
        pf[s + 1] = pf[s] + L;
        pq[s + 1] = pq[s] + L * L;
    }

    // ---- walk the groups: chunks of whole groups in parallel, then stitch
    const int n_threads = int(std::min<int64_t>(HostPool::get().size(), std::max<int64_t>(1, n / 4096)));
    // more shares than threads: the pool hands them out dynamically (group sizes vary)
    const int n_shares = int(std::min<int64_t>(4 * int64_t(n_threads), std::max<int64_t>(1, n / 1024)));
    std::vector<int64_t> cut(size_t(n_shares) + 1, n);
    cut[0] = 0;
    for (int k = 1; k < n_shares; ++k) {
        int64_t c = std::max(cut[k - 1], n * k / n_shares);
        while (c > 0 && c < n && by_part[c] == by_part[c - 1]) ++c;   // move to a group start
        cut[k] = c;
    }
    std::vector<WalkOut> parts(static_cast<size_t>(n_shares));
    std::vector<const std::vector<uint32_t> *> by_rank_p, across_rank_p;
    for (auto &r : rby) by_rank_p.push_back(&r.rank);
    for (auto &r : racr) across_rank_p.push_back(&r.rank);
    WalkCtx wc{ds.get(), t.get(), &order, &by_part, &cls_part, &ron.rank, &by_rank_p, &across_rank_p,
               &pf, &pq, on, n_across, across_cmp, across_all_differ};
    t->key_bits = {ron.bits, ron.bits};
    for (auto &r : rby) t->key_bits.push_back(r.bits);
    for (auto &r : racr) t->key_bits.push_back(r.bits);
    for (auto &r : racr) t->key_bits.push_back(r.bits);
    parallel_for(n_shares, [&](int k) { walk_groups(wc, cut[k], cut[k + 1], parts[size_t(k)]); });

    tr.mark("walk");
    size_t n_cells = 0, n_groups = 0;
    for (auto &p : parts) {
        n_cells += p.cells.size();
        n_groups += p.groups.size();
    }
    size_t n_unit_ints = 0;
    for (auto &p : parts) n_unit_ints += p.units.size();
    t->cells.resize(n_cells);
    t->n_triplets.resize(n_cells);
    t->keys.resize(n_cells * size_t(t->key_width));
    t->rkeys.resize(n_cells * size_t(t->key_width));
    t->units.resize(n_unit_ints);
    std::vector<size_t> unit_off(parts.size());
    t->groups.resize(n_groups);
    std::vector<std::pair<int64_t, int64_t>> kept(n_groups);
    std::vector<size_t> cell_off(parts.size()), group_off(parts.size());
    std::vector<int64_t> slot_off(parts.size());
    {
        size_t co = 0, go = 0;
        int64_t so = 0;
        for (size_t k = 0; k < parts.size(); ++k) {
            cell_off[k] = co;
            group_off[k] = go;
            slot_off[k] = so;
            co += parts[k].cells.size();
            go += parts[k].groups.size();
            t->sum_nx += parts[k].sum_nx;
            so += parts[k].pair_slots;
            t->total_triplets += parts[k].total_triplets;
            t->n_pairs_needed += parts[k].pairs_needed;
            t->dtw_cells_needed += parts[k].dtw_needed;
        }
        t->n_pair_slots = so;
        size_t uo = 0;
        for (size_t k = 0; k < parts.size(); ++k) {
            unit_off[k] = uo;
            uo += parts[k].units.size();
        }
    }
    parallel_for(n_shares, [&](int k) {
        WalkOut &p = parts[size_t(k)];
        for (size_t c = 0; c < p.cells.size(); ++c) {
            CellDev cd = p.cells[c];
            cd.group += int32_t(group_off[size_t(k)]);
            t->cells[cell_off[size_t(k)] + c] = cd;
        }
        std::copy(p.ntrip.begin(), p.ntrip.end(), t->n_triplets.begin() + long(cell_off[size_t(k)]));
        std::copy(p.keys.begin(), p.keys.end(), t->keys.begin() + long(cell_off[size_t(k)] * size_t(t->key_width)));
        std::copy(p.rkeys.begin(), p.rkeys.end(), t->rkeys.begin() + long(cell_off[size_t(k)] * size_t(t->key_width)));
        for (size_t u = 0; u < p.units.size(); u += 3) {
            t->units[unit_off[size_t(k)] + u] = p.units[u] + int32_t(cell_off[size_t(k)]);
            t->units[unit_off[size_t(k)] + u + 1] = p.units[u + 1];
            t->units[unit_off[size_t(k)] + u + 2] = p.units[u + 2];
        }
        for (size_t g = 0; g < p.groups.size(); ++g) {
            Group gg = p.groups[g];
            gg.pair_base += slot_off[size_t(k)];
            t->groups[group_off[size_t(k)] + g] = gg;
            kept[group_off[size_t(k)] + g] = p.kept[g];
        }
        WalkOut().swap(p);
    });

    tr.mark("stitch");
    // ---- task items in task order, packed frame offsets
    int64_t nt = 0, frame_total = 0;
    for (size_t gi = 0; gi < t->groups.size(); ++gi) {
        Group &g = t->groups[gi];
        g.item0 = nt;
        g.n_items = kept[gi].second - kept[gi].first;
        g.frame0 = frame_total;
        g.n_frames = pf[kept[gi].second] - pf[kept[gi].first];
        g.dmat_base = t->n_dmat;
        t->n_dmat += g.n_frames * g.n_frames;
        nt += g.n_items;
        frame_total += g.n_frames;
    }
    t->items.resize(size_t(nt));
    t->item_len.resize(size_t(nt));
    t->item_src.resize(size_t(nt));
    t->item_dst.resize(size_t(nt));
    t->item_group.resize(size_t(nt));
    t->item_pos_of.assign(size_t(n), -1);
    std::vector<int> max_len_part(static_cast<size_t>(n_threads), 0);
    const int64_t G = int64_t(t->groups.size());
    parallel_for(n_threads, [&](int k) {
        int ml = 0;
        for (int64_t gi = G * k / n_threads; gi < G * (k + 1) / n_threads; ++gi) {
            const Group &g = t->groups[size_t(gi)];
            int64_t frame = g.frame0, q = g.item0;
            for (int64_t s = kept[size_t(gi)].first; s < kept[size_t(gi)].second; ++s, ++q) {
                const int64_t it = order[s];
                t->items[q] = it;
                t->item_pos_of[it] = q;
                t->item_src[q] = ds->offsets[it];
                t->item_len[q] = len_s[s];
                t->item_dst[q] = frame;
                t->item_group[q] = int32_t(gi);
                ml = std::max(ml, len_s[s]);
                frame += len_s[s];
            }
        }
        max_len_part[size_t(k)] = ml;
    });
    for (int ml : max_len_part) t->max_len = std::max(t->max_len, ml);
    const int64_t frame = frame_total;

    // fused-kernel blocks: whole items packed into <= 64-frame row blocks and
    // <= 128-frame column blocks per group; work units = row x column blocks
    t->unit_prefix.assign(size_t(G) + 1, 0);
    for (int64_t gi = 0; gi < G; ++gi) {
        const Group &g = t->groups[size_t(gi)];
        t->g_rb0.push_back(int32_t(t->rb.size() / 4));
        t->g_cb0.push_back(int32_t(t->cb.size() / 4));
        for (int pass = 0; pass < 2; ++pass) {
            const int limit = pass == 0 ? kFusedRowFrames : kFusedColFrames;
            std::vector<int32_t> &out = pass == 0 ? t->rb : t->cb;
            int64_t k = g.item0;
            const int64_t end = g.item0 + g.n_items;
            while (k < end) {
                const int32_t first = int32_t(k);
                int32_t frames = 0, cnt = 0;
                // at least one item per block (an item above the limit is only legal in
                // pooled mode, which does not use these blocks)
                while (k < end && (cnt == 0 || frames + t->item_len[size_t(k)] <= limit)) {
                    frames += t->item_len[size_t(k)];
                    ++cnt;
                    ++k;
                }
                out.insert(out.end(), {int32_t(gi), first, cnt, frames});
            }
        }
        const int32_t nrb = int32_t(t->rb.size() / 4) - t->g_rb0.back();
        const int32_t ncb = int32_t(t->cb.size() / 4) - t->g_cb0.back();
        t->g_ncb.push_back(ncb);
        t->unit_prefix[size_t(gi) + 1] = t->unit_prefix[size_t(gi)] + int64_t(nrb) * ncb;
        t->fused_cells += g.n_frames * g.n_frames;
    }
    t->n_frames = frame;
    tr.mark("items");
    return t;
}

}  // namespace fabx
