// Task construction: group items by BY value, split groups into classes of
// equal (ON, ACROSS) value, and enumerate the cells (Background section: the
// ON / BY / ACROSS conditions, and the cell A x B x X).
//
// All host integer work.  Items are ordered once by a composite key
// (by..., on, across...) with an LSD radix sort, so every BY group and every
// class is a contiguous run; a cell is then three runs (A, B, X).
#include <algorithm>
#include <atomic>
#include <climits>
#include <cstring>
#include <functional>
#include <numeric>
#include <thread>

#if defined(__x86_64__)
#include <immintrin.h>
#endif

#include "host_pool.h"
#include "internal.h"

namespace fabx {
namespace {

struct RankedColumn {
    std::vector<int32_t> values;   // sorted unique attribute values
    hvec<uint32_t> rank;           // per item: index into values
    int bits = 0;                  // bits needed to hold a rank
};

template <typename F>
void parallel_for(int n, F &&f);

// Items per chunk of a per-item parallel loop: up to four chunks per pool
// thread, at least 1024 items each.  Loops chunked this way compute the same
// per-item results whatever the chunk size.
int64_t item_chunk(int64_t n) {
    const int64_t parts = 4 * int64_t(HostPool::get().size());
    return std::max<int64_t>(1024, (n + parts - 1) / parts);
}

// Groups per chunk of a loop over BY groups: about 8 chunks per pool thread
// (group sizes vary), at least 16 groups each.  Per-group results do not
// depend on it.
int64_t group_chunk(int64_t n_groups) {
    const int64_t parts = 8 * int64_t(HostPool::get().size());
    return std::max<int64_t>(16, (n_groups + parts - 1) / parts);
}

// Dense ranks of attribute columns `cols`, all columns per pass over the
// item rows, each pass parallel over fixed row chunks: per-chunk minima and
// maxima; then, for a column whose value range is small, the values present
// (marked in a byte table) numbered in value order, else its sorted unique
// values; then every item's rank.
std::vector<RankedColumn> rank_columns(const DatasetImpl &ds, const std::vector<int32_t> &cols) {
    const int64_t n = ds.n_items;
    const size_t nc = cols.size(), na = size_t(ds.n_attr);
    std::vector<RankedColumn> out(nc);
    for (auto &rc : out) rc.rank.resize(size_t(n));
    if (n == 0 || nc == 0) return out;
    const int32_t *A = ds.attrs.data();
    const int64_t kChunk = item_chunk(n);
    const int n_chunks = int((n + kChunk - 1) / kChunk);
    auto rows = [&](int c) { return std::make_pair(c * kChunk, std::min<int64_t>(n, (c + 1) * kChunk)); };
    std::vector<int32_t> cmn(size_t(n_chunks) * nc, INT32_MAX), cmx(size_t(n_chunks) * nc, INT32_MIN);
    parallel_for(n_chunks, [&](int c) {
        // one column at a time in locals; chunks' results share cache lines
        const auto [i0, i1] = rows(c);
        for (size_t j = 0; j < nc; ++j) {
            const size_t col = size_t(cols[j]);
            int32_t mn = INT32_MAX, mx = INT32_MIN;
            for (int64_t i = i0; i < i1; ++i) {
                const int32_t v = A[size_t(i) * na + col];
                mn = std::min(mn, v);
                mx = std::max(mx, v);
            }
            cmn[size_t(c) * nc + j] = mn;
            cmx[size_t(c) * nc + j] = mx;
        }
    });
    std::vector<int32_t> lo(nc, INT32_MAX), hi(nc, INT32_MIN);
    std::vector<char> dense(nc);
    std::vector<std::vector<int32_t>> table(nc);  // dense: value - lo -> rank
    std::vector<std::vector<uint8_t>> seen(nc);
    for (size_t j = 0; j < nc; ++j) {
        for (int c = 0; c < n_chunks; ++c) {
            lo[j] = std::min(lo[j], cmn[size_t(c) * nc + j]);
            hi[j] = std::max(hi[j], cmx[size_t(c) * nc + j]);
        }
        const int64_t range = int64_t(hi[j]) - int64_t(lo[j]) + 1;
        dense[j] = range <= std::max<int64_t>(4 * n, 1 << 16);
        if (dense[j]) seen[j].assign(size_t(range), 0);
    }
    parallel_for(n_chunks, [&](int c) {
        const auto [i0, i1] = rows(c);
        for (size_t j = 0; j < nc; ++j) {
            if (!dense[j]) continue;
            uint8_t *sj = seen[j].data();
            const int64_t l = lo[j];
            // store only when unset: the few values of a label column then stay
            // in shared cache lines instead of bouncing between threads
            for (int64_t i = i0; i < i1; ++i) {
                uint8_t *e = sj + (A[size_t(i) * na + size_t(cols[j])] - l);
                if (!__atomic_load_n(e, __ATOMIC_RELAXED)) __atomic_store_n(e, uint8_t(1), __ATOMIC_RELAXED);
            }
        }
    });
    parallel_for(int(nc), [&](int jj) {
        const size_t j = size_t(jj);
        RankedColumn &rc = out[j];
        if (dense[j]) {
            table[j].assign(seen[j].size(), 0);
            int32_t r = 0;
            for (size_t v = 0; v < seen[j].size(); ++v)
                if (seen[j][v]) {
                    table[j][v] = r++;
                    rc.values.push_back(int32_t(int64_t(v) + lo[j]));
                }
        } else {
            rc.values.resize(size_t(n));
            for (int64_t i = 0; i < n; ++i) rc.values[size_t(i)] = A[size_t(i) * na + size_t(cols[j])];
            std::sort(rc.values.begin(), rc.values.end());
            rc.values.erase(std::unique(rc.values.begin(), rc.values.end()), rc.values.end());
        }
        uint64_t u = rc.values.size();
        while ((uint64_t(1) << rc.bits) < u) ++rc.bits;
    });
    parallel_for(n_chunks, [&](int c) {
        const auto [i0, i1] = rows(c);
        for (size_t j = 0; j < nc; ++j) {
            uint32_t *rk = out[j].rank.data();
            const size_t col = size_t(cols[j]);
            if (dense[j]) {
                const int32_t *tb = table[j].data();
                const int64_t l = lo[j];
                for (int64_t i = i0; i < i1; ++i) rk[i] = uint32_t(tb[A[size_t(i) * na + col] - l]);
            } else {
                const auto &vals = out[j].values;
                for (int64_t i = i0; i < i1; ++i)
                    rk[i] = uint32_t(std::lower_bound(vals.begin(), vals.end(), A[size_t(i) * na + col]) -
                                     vals.begin());
            }
        }
    });
    return out;
}

// Stable LSD radix sort of items by a key of key_bits bits (digits of at
// most 11 bits, as few passes as that allows), parallel over fixed chunks:
// each chunk counts its digits, one prefix over (digit, chunk) gives every
// chunk its output positions, and each chunk scatters its elements in order.
// Ties keep ascending item order, whatever the thread count.
template <typename K, typename I>
void radix_sort(hvec<K> &key, hvec<I> &idx, int key_bits) {
    const size_t n = key.size();
    if (key_bits <= 0 || n < 2) return;
    const int passes = (key_bits + 10) / 11;
    const int digit = (key_bits + passes - 1) / passes;
    const size_t buckets = size_t(1) << digit;
    const size_t n_chunks = std::min<size_t>(64, std::max<size_t>(1, n / 8192));
    hvec<K> k2(n);
    hvec<I> i2(n);
    std::vector<size_t> hist(n_chunks * buckets);
    auto bounds = [&](size_t c) { return std::make_pair(n * c / n_chunks, n * (c + 1) / n_chunks); };
    for (int shift = 0; shift < key_bits; shift += digit) {
        const K mask = K(buckets - 1);
        HostPool::get().parallel_for(int(n_chunks), [&](int c) {
            size_t *h = hist.data() + size_t(c) * buckets;
            std::fill(h, h + buckets, size_t(0));
            const auto [b0, b1] = bounds(size_t(c));
            for (size_t i = b0; i < b1; ++i) ++h[(key[i] >> shift) & mask];
        });
        size_t run = 0;
        for (size_t b = 0; b < buckets; ++b)
            for (size_t c = 0; c < n_chunks; ++c) {
                const size_t v = hist[c * buckets + b];
                hist[c * buckets + b] = run;
                run += v;
            }
        HostPool::get().parallel_for(int(n_chunks), [&](int c) {
            size_t *h = hist.data() + size_t(c) * buckets;
            const auto [b0, b1] = bounds(size_t(c));
            for (size_t i = b0; i < b1; ++i) {
                const size_t d = h[(key[i] >> shift) & mask]++;
                k2[d] = key[i];
                i2[d] = idx[i];
            }
        });
        key.swap(k2);
        idx.swap(i2);
    }
}

struct ClassRun {
    int64_t start;      // position in sorted order
    int64_t count;
    uint32_t on_rank;
};


template <typename F>
void parallel_for(int n, F &&f) {
    const std::function<void(int)> fn = f;
    HostPool::get().parallel_for(n, fn);
}

// One share of the group walk.  The walk runs twice over the same share:
// first counting (cells, unit ints, kept groups and the task totals), then,
// after prefix sums over the shares, writing straight into the task's arrays
// at the share's offsets.
struct Sink {
    size_t n_cells = 0, n_unit_ints = 0, n_big_unit_ints = 0, n_groups = 0;
    int64_t total_triplets = 0, pairs_needed = 0, dtw_needed = 0, dtw_sym = 0, pair_slots = 0, sum_nx = 0;
    // write pass: destinations, and the share's first cell / unit int / group / pair slot
    CellDev *cells = nullptr;
    int64_t *ntrip = nullptr;
    uint32_t *rkeys = nullptr;
    int32_t *units = nullptr;
    Group *groups = nullptr;
    std::pair<int64_t, int64_t> *kept = nullptr;
    size_t cell_base = 0, unit_base = 0, big_unit_base = 0, group_base = 0, key_width = 0;
    int64_t slot_base = 0;
};

constexpr int64_t kUnitBudget = 8192;  // comparisons per triplet work unit (at least one x)
// Cells with at least this many comparisons per x, and |B| within the sort
// capacity, are counted from sorted rows (one unit per x, after the others).
constexpr int64_t kSortedMinPerX = 8192;

struct WalkCtx {
    const DatasetImpl *ds;
    const TaskImpl *t;
    const hvec<int64_t> *order;
    const hvec<uint64_t> *by_part, *cls_part;
    // ranks per sorted position, [n x W]: ON, then BY..., then ACROSS...
    const uint32_t *srank;
    int W;
    const hvec<int64_t> *pf, *pq;
    int32_t n_across;
};

// Cells of the groups that start in sorted positions [s_begin, s_end).
template <bool kWrite>
void walk_groups(const WalkCtx &w, int64_t s_begin, int64_t s_end, Sink &out) {
    const auto &by_part = *w.by_part;
    const auto &cls_part = *w.cls_part;
    const auto &pf = *w.pf;
    const auto &pq = *w.pq;
    const TaskImpl &t = *w.t;
    const uint32_t *SR = w.srank;
    const size_t W = size_t(w.W);
    std::vector<ClassRun> cls;
    std::vector<uint8_t> need;
    std::vector<std::pair<int64_t, int64_t>> need_list, runs;
    // key ranks, read once per group (BY) and per class (ACROSS)
    const int n_by = int(t.by.size()), n_ac = w.n_across;
    std::vector<uint32_t> gbyr(static_cast<size_t>(n_by)), cacr;
    int64_t g0 = s_begin;
    while (g0 < s_end) {
        int64_t g1 = g0 + 1;
        while (g1 < s_end && by_part[g1] == by_part[g0]) ++g1;
        cls.clear();
        for (int64_t s = g0; s < g1;) {
            int64_t e = s + 1;
            while (e < g1 && cls_part[e] == cls_part[s]) ++e;
            cls.push_back({s, e - s, SR[size_t(s) * W]});
            s = e;
        }
        const int64_t K = int64_t(cls.size());
        const int32_t group_id = int32_t(out.group_base + out.n_groups);
        {
            const uint32_t *r0 = SR + size_t(g0) * W;
            for (int j = 0; j < n_by; ++j) gbyr[size_t(j)] = r0[1 + j];
            cacr.resize(size_t(K * n_ac));
            for (int64_t i = 0; i < K; ++i) {
                const uint32_t *ri = SR + size_t(cls[size_t(i)].start) * W;
                for (int j = 0; j < n_ac; ++j) cacr[size_t(i * n_ac + j)] = ri[1 + n_by + j];
            }
        }
        // ACROSS tuples of two classes: lexicographic order (the sort order) and
        // "differ in every attribute"
        auto across_cmp = [&](int64_t a, int64_t b) {
            for (int j = 0; j < n_ac; ++j) {
                const uint32_t x = cacr[size_t(a * n_ac + j)], y = cacr[size_t(b * n_ac + j)];
                if (x != y) return x < y ? -1 : 1;
            }
            return 0;
        };
        auto across_all_differ = [&](int64_t a, int64_t b) {
            for (int j = 0; j < n_ac; ++j)
                if (cacr[size_t(a * n_ac + j)] == cacr[size_t(b * n_ac + j)]) return false;
            return true;
        };
        const size_t cells_before = out.n_cells;
        // the unique pairs a group needs are only counted in the first pass
        const bool use_need = !kWrite && w.n_across > 0 && K <= 8192;
        if (use_need) need.assign(size_t(K * K), 0);
        need_list.clear();
        auto add_cell = [&](int64_t ia, int64_t ib, int64_t ix, bool excl) {
            const int64_t na = cls[ia].count, nb = cls[ib].count, nx = cls[ix].count;
            const int64_t nt = excl ? na * (na - 1) * nb : na * nb * nx;
            const size_t cid = out.cell_base + out.n_cells;
            // triplet work units: split X so one unit does <= kUnitBudget comparisons;
            // large cells get one unit per x, in the sorted-row region
            const int64_t per_x = std::max<int64_t>(1, na * nb);
            const bool big = per_x >= kSortedMinPerX && nb <= kSortedMaxB;
            // nx * per_x <= budget (the usual case): one unit for the whole cell,
            // which is what the division below gives, without dividing
            const bool one = !big && nx >= 1 && nx * per_x <= kUnitBudget;
            const int64_t chunk = one ? nx : big ? 1 : std::max<int64_t>(1, kUnitBudget / per_x);
            const int64_t n_units_cell = one ? 1 : (nx + chunk - 1) / chunk;
            if (kWrite) {
                // The task's per-cell arrays are far larger than the caches and
                // are read back only later (upload, collapse): streaming stores
                // write them without first reading their lines.
                auto put = [](auto *dst, auto v) { __builtin_nontemporal_store(v, dst); };
                int32_t *c = reinterpret_cast<int32_t *>(out.cells + cid);
                put(c + 0, group_id);
                put(c + 1, int32_t(cls[ia].start - g0));
                put(c + 2, int32_t(na));
                put(c + 3, int32_t(cls[ib].start - g0));
                put(c + 4, int32_t(nb));
                put(c + 5, int32_t(cls[ix].start - g0));
                put(c + 6, int32_t(nx));
                put(c + 7, int32_t(excl ? 1 : 0));
                put(out.ntrip + cid, int64_t(nt));
                uint32_t *rk = out.rkeys + cid * out.key_width;
                put(rk + 0, cls[size_t(ia)].on_rank);
                put(rk + 1, cls[size_t(ib)].on_rank);
                for (int j = 0; j < n_by; ++j) put(rk + 2 + j, gbyr[size_t(j)]);
                for (int j = 0; j < n_ac; ++j) {
                    put(rk + 2 + n_by + j, cacr[size_t(ia * n_ac + j)]);
                    put(rk + 2 + n_by + n_ac + j, cacr[size_t(ix * n_ac + j)]);
                }
                int32_t *u = big ? out.units + out.big_unit_base + out.n_big_unit_ints
                                 : out.units + out.unit_base + out.n_unit_ints;
                for (int64_t x = 0; x < nx; x += chunk, u += 3) {
                    put(u + 0, int32_t(cid));
                    put(u + 1, int32_t(x));
                    put(u + 2, int32_t(std::min<int64_t>(nx, x + chunk)));
                }
            }
            (big ? out.n_big_unit_ints : out.n_unit_ints) += size_t(3 * n_units_cell);
            ++out.n_cells;
            out.total_triplets += nt;
            out.sum_nx += nx;
            if (use_need) {
                need[size_t(ix * K + ia)] = 1;
                need[size_t(ix * K + ib)] = 1;
            } else if (!kWrite && w.n_across > 0) {
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
                            if (across_cmp(mid, ia) < 0) lo = mid + 1; else hi = mid;
                        }
                        if (lo == r2.second || across_cmp(lo, ia) != 0) continue;
                        for (int64_t ix = r1.first; ix < r1.second; ++ix)
                            if (across_all_differ(ix, ia))
                                add_cell(ia, lo, ix, false);
                    }
                }
        }
        if (out.n_cells > cells_before) {
            Group g{};
            g.n_items = g1 - g0;
            g.pair_base = out.slot_base + out.pair_slots;
            out.pair_slots += g.n_items * g.n_items;
            if (kWrite) {
                out.groups[out.group_base + out.n_groups] = g;
                out.kept[out.group_base + out.n_groups] = {g0, g1};
            }
            ++out.n_groups;
        }
        if (!kWrite && out.n_cells > cells_before) {
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
            // unordered class pair {ix, iy} (ix <= iy) needed in either order
            auto count_sym = [&](int64_t ix, int64_t iy) {
                out.dtw_sym += ix == iy ? (frames(ix) * frames(ix) - sq(ix)) / 2 : frames(ix) * frames(iy);
            };
            if (w.n_across == 0) {
                // every item of a class with >= 2 items is an x; it needs every other item
                const int64_t all_items = g1 - g0, all_frames = pf[g1] - pf[g0];
                const int64_t all_sq = pq[g1] - pq[g0];
                int64_t single_frames = 0, single_sq = 0;  // items of one-item classes
                for (int64_t ix = 0; ix < K; ++ix) {
                    if (cnt(ix) < 2) {
                        single_frames += frames(ix);
                        single_sq += sq(ix);
                        continue;
                    }
                    out.pairs_needed += cnt(ix) * (all_items - 1);
                    out.dtw_needed += frames(ix) * all_frames - sq(ix);
                }
                // unordered pairs of distinct items with at least one in a class of >= 2
                out.dtw_sym += (all_frames * all_frames - all_sq) / 2 -
                               (single_frames * single_frames - single_sq) / 2;
            } else if (use_need) {
                for (int64_t ix = 0; ix < K; ++ix)
                    for (int64_t iy = 0; iy < K; ++iy)
                        if (need[size_t(ix * K + iy)]) count_pair(ix, iy);
                for (int64_t ix = 0; ix < K; ++ix)
                    for (int64_t iy = ix; iy < K; ++iy)
                        if (need[size_t(ix * K + iy)] || need[size_t(iy * K + ix)]) count_sym(ix, iy);
            } else {
                std::sort(need_list.begin(), need_list.end());
                need_list.erase(std::unique(need_list.begin(), need_list.end()), need_list.end());
                for (auto &pr : need_list) count_pair(pr.first, pr.second);
                for (auto &pr : need_list)
                    if (pr.first > pr.second) std::swap(pr.first, pr.second);
                std::sort(need_list.begin(), need_list.end());
                need_list.erase(std::unique(need_list.begin(), need_list.end()), need_list.end());
                for (auto &pr : need_list) count_sym(pr.first, pr.second);
            }
        }
        g0 = g1;
    }
}

// Whole items of group gi packed, in task order, into blocks of at most
// `limit` frames.  Items of more than kFusedRowFrames frames are left out (a
// block ends before such an item and the next starts after it): their pairs
// are computed by the FP64 long-item kernel.  Writes [n][4] = group, first
// item, n items, n frames to `out` if given; returns the count.
int32_t pack_blocks(const TaskImpl &t, int64_t gi, int limit, int32_t *out) {
    const Group &g = t.groups[size_t(gi)];
    int32_t nb = 0;
    int64_t k = g.item0;
    const int64_t end = g.item0 + g.n_items;
    while (k < end) {
        if (t.item_len[size_t(k)] > kFusedRowFrames) {
            ++k;
            continue;
        }
        const int32_t first = int32_t(k);
        int32_t frames = 0, cnt = 0;
        while (k < end && t.item_len[size_t(k)] <= kFusedRowFrames &&
               (cnt == 0 || frames + t.item_len[size_t(k)] <= limit)) {
            frames += t.item_len[size_t(k)];
            ++cnt;
            ++k;
        }
        if (out) {
            int32_t *o = out + 4 * size_t(nb);
            o[0] = int32_t(gi);
            o[1] = first;
            o[2] = cnt;
            o[3] = frames;
        }
        ++nb;
    }
    return nb;
}

}  // namespace

void cell_keys(const TaskImpl &t, int32_t *out) {
    const size_t K = size_t(t.key_width), n = t.cells.size();
    const size_t kChunk = size_t(1) << 15;
    parallel_for(int((n + kChunk - 1) / kChunk), [&](int c) {
        for (size_t i = size_t(c) * kChunk; i < std::min(n, size_t(c + 1) * kChunk); ++i)
            for (size_t k = 0; k < K; ++k) out[i * K + k] = t.key_values[k][t.rkeys[i * K + k]];
    });
}

// Kept work units of a column plan (see ColPlan): for each row block, the
// first column block of its group that ends after the row block's first item
// (a suffix of the group's column blocks; row blocks ascend, so one pointer
// per group walks the column blocks), and the frame pairs they cover; then
// the bands the units are ordered in, and the prefix of units over bands.
void plan_units(const TaskImpl &t, ColPlan &cp) {
    const int64_t G = int64_t(t.groups.size());
    const size_t n_rb = t.rb.size() / 4;
    cp.rb_cstart.resize(n_rb);
    const int64_t kGroups = group_chunk(G);
    const int n_gc = int((G + kGroups - 1) / kGroups);
    std::vector<int64_t> part_cells(static_cast<size_t>(std::max(n_gc, 1)), 0);
    parallel_for(n_gc, [&](int c) {
        int64_t cells = 0;
        for (int64_t gi = c * kGroups; gi < std::min<int64_t>(G, (c + 1) * kGroups); ++gi) {
            const size_t r0 = size_t(t.g_rb0[size_t(gi)]), c0 = size_t(cp.g_cb0[size_t(gi)]);
            const int32_t nr = t.g_nrb[size_t(gi)], nc = cp.g_ncb[size_t(gi)];
            int64_t suffix = 0;  // frames of column blocks [k, nc)
            for (int32_t k = 0; k < nc; ++k) suffix += cp.cb[4 * (c0 + size_t(k)) + 3];
            int32_t k = 0;
            for (int32_t r = 0; r < nr; ++r) {
                const int32_t *rbe = t.rb.data() + 4 * (r0 + size_t(r));
                const int32_t ri0 = rbe[1];
                while (k < nc) {
                    const int32_t *cbe = cp.cb.data() + 4 * (c0 + size_t(k));
                    if (cbe[1] + cbe[2] > ri0) break;   // ends after the row block starts: kept
                    suffix -= cbe[3];
                    ++k;
                }
                cp.rb_cstart[r0 + size_t(r)] = k;
                cells += int64_t(rbe[3]) * suffix;
            }
        }
        part_cells[size_t(c)] = cells;
    });
    cp.cells = 0;
    for (int64_t v : part_cells) cp.cells += v;
    // Bands: runs of kBandRows row blocks in groups of at least kBandMinCols
    // column blocks, else one row block each.  A band's units are its rows x
    // the column blocks from its first row block's first kept one (the least
    // of the band's, as they ascend with the row block) to the group's last.
    cp.band_rb.clear();
    cp.unit_prefix.clear();
    cp.unit_prefix.push_back(0);
    for (int64_t gi = 0; gi < G; ++gi) {
        const int32_t r0 = t.g_rb0[size_t(gi)], nr = t.g_nrb[size_t(gi)], nc = cp.g_ncb[size_t(gi)];
        const int32_t rows_per_band = nc >= kBandMinCols ? kBandRows : 1;
        for (int32_t r = 0; r < nr; r += rows_per_band) {
            const int32_t rows = std::min(rows_per_band, nr - r);
            cp.band_rb.push_back(r0 + r);
            cp.unit_prefix.push_back(cp.unit_prefix.back() + int64_t(rows) * (nc - cp.rb_cstart[size_t(r0 + r)]));
        }
    }
    cp.band_rb.push_back(int32_t(n_rb));
}

// Stream kernel: segments of about `cols` frames of each row block's column
// stream (the group's frames from the row block's first frame on).
void plan_stream(const TaskImpl &t, ColPlan &cp) {
    const int64_t G = int64_t(t.groups.size());
    for (const Group &g : t.groups)
        if (g.n_items > 0xFFFFFF) fail(FABX_EINVAL, "a BY group holds more than 2^24 - 1 items");
    const size_t n_rb = t.rb.size() / 4;
    cp.unit_prefix.resize(n_rb + 1);
    cp.unit_prefix[0] = 0;
    const int64_t kGroups = group_chunk(G);
    const int n_gc = int((G + kGroups - 1) / kGroups);
    std::vector<int64_t> part_cells(static_cast<size_t>(std::max(n_gc, 1)), 0);
    parallel_for(n_gc, [&](int c) {
        int64_t cells = 0;
        for (int64_t gi = c * kGroups; gi < std::min<int64_t>(G, (c + 1) * kGroups); ++gi) {
            const Group &g = t.groups[size_t(gi)];
            const size_t r0 = size_t(t.g_rb0[size_t(gi)]);
            for (int32_t r = 0; r < t.g_nrb[size_t(gi)]; ++r) {
                const int32_t *rbe = t.rb.data() + 4 * (r0 + size_t(r));
                const int64_t S = g.frame0 + g.n_frames - t.item_dst[size_t(rbe[1])];
                cp.unit_prefix[r0 + size_t(r) + 1] = (S + cp.cols - 1) / cp.cols;
                cells += int64_t(kFusedRowFrames) * S;
            }
        }
        part_cells[size_t(c)] = cells;
    });
    for (size_t i = 0; i < n_rb; ++i) cp.unit_prefix[i + 1] += cp.unit_prefix[i];
    cp.cells = 0;
    for (int64_t v : part_cells) cp.cells += v;
}

ColPlan &col_plan(TaskImpl &t, int cols) {
    for (auto &p : t.col_plans)
        if (p->cols == cols) return *p;
    auto cp = std::make_unique<ColPlan>();
    cp->cols = cols;
    if (cols >= kStreamMinCols) {
        plan_stream(t, *cp);
        t.col_plans.push_back(std::move(cp));
        return *t.col_plans.back();
    }
    const int64_t G = int64_t(t.groups.size());
    cp->g_cb0.assign(size_t(G), 0);
    cp->g_ncb.assign(size_t(G), 0);
    const int64_t kGroups = group_chunk(G);
    const int n_gc = int((G + kGroups - 1) / kGroups);
    parallel_for(n_gc, [&](int c) {
        for (int64_t gi = c * kGroups; gi < std::min<int64_t>(G, (c + 1) * kGroups); ++gi)
            cp->g_ncb[size_t(gi)] = pack_blocks(t, gi, cols, nullptr);
    });
    int32_t total = 0;
    for (int64_t gi = 0; gi < G; ++gi) {
        cp->g_cb0[size_t(gi)] = total;
        total += cp->g_ncb[size_t(gi)];
    }
    cp->cb.resize(4 * size_t(total));
    parallel_for(n_gc, [&](int c) {
        for (int64_t gi = c * kGroups; gi < std::min<int64_t>(G, (c + 1) * kGroups); ++gi)
            pack_blocks(t, gi, cols, cp->cb.data() + 4 * size_t(cp->g_cb0[size_t(gi)]));
    });
    plan_units(t, *cp);
    t.col_plans.push_back(std::move(cp));
    return *t.col_plans.back();
}

void plan_blocks(TaskImpl &t) {
    const int64_t G = int64_t(t.groups.size());
    // DTW row blocks (whole items packed into <= 64 frames per group), counted
    // in one parallel pass and written in another; then the default work plan
    // (other launch choices are planned by col_plan on demand)
    std::vector<int32_t> nrb(static_cast<size_t>(G));
    const int64_t kGroups = group_chunk(G);
    const int n_gc = int((G + kGroups - 1) / kGroups);
    parallel_for(n_gc, [&](int c) {
        for (int64_t gi = c * kGroups; gi < std::min<int64_t>(G, (c + 1) * kGroups); ++gi)
            nrb[size_t(gi)] = pack_blocks(t, gi, kFusedRowFrames, nullptr);
    });
    t.g_rb0.assign(size_t(G), 0);
    t.g_nrb.assign(nrb.begin(), nrb.end());
    int32_t rb_total = 0;
    for (int64_t gi = 0; gi < G; ++gi) {
        t.g_rb0[size_t(gi)] = rb_total;
        rb_total += nrb[size_t(gi)];
    }
    t.rb.resize(4 * size_t(rb_total));
    parallel_for(n_gc, [&](int c) {
        for (int64_t gi = c * kGroups; gi < std::min<int64_t>(G, (c + 1) * kGroups); ++gi)
            pack_blocks(t, gi, kFusedRowFrames, t.rb.data() + 4 * size_t(t.g_rb0[size_t(gi)]));
    });
    t.fused_cells = col_plan(t, Tuner::default_config().cols).cells;
    // pair slots with an item of more than kFusedRowFrames frames, both
    // orientations, (x, x) left out: the FP64 long-item kernel's list
    t.long_slots.clear();
    if (t.max_len > kFusedRowFrames) {
        for (const Group &g : t.groups) {
            const int64_t n = g.n_items;
            for (int64_t a = 0; a < n; ++a) {
                const bool la = t.item_len[size_t(g.item0 + a)] > kFusedRowFrames;
                for (int64_t b = a + 1; b < n; ++b) {
                    if (!la && t.item_len[size_t(g.item0 + b)] <= kFusedRowFrames) continue;
                    t.long_slots.push_back(g.pair_base + a * n + b);
                    t.long_slots.push_back(g.pair_base + b * n + a);
                }
            }
        }
    }
}

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
        std::vector<RankedColumn> ranked = rank_columns(*ds, all_cols);
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
    hvec<int64_t> order(n);
    hvec<uint64_t> by_part(n), cls_part(n);   // BY tuple id / (on, across) class id
    if (total_bits <= 64) {
        // packed key: BY ranks (high), ON rank, ACROSS ranks (low); sorted as
        // 32-bit keys and item ids when it fits, which halves the bytes moved
        const int64_t kChunk = item_chunk(n);
        const int n_chunks = int((n + kChunk - 1) / kChunk);
        // rank arrays and shifts of the key's fields, most significant first
        std::vector<const uint32_t *> fr;
        std::vector<int> fs;
        for (auto &r : rby) {
            fr.push_back(r.rank.data());
            fs.push_back(r.bits);
        }
        fr.push_back(ron.rank.data());
        fs.push_back(ron.bits);
        for (int j = 0; j < n_across; ++j) {
            fr.push_back(racr[size_t(j)].rank.data());
            fs.push_back(racr[size_t(j)].bits);
        }
        const size_t nf = fr.size();
        auto packed = [&](int64_t i) {
            uint64_t k = 0;
            for (size_t f = 0; f < nf; ++f) k = (k << fs[f]) | fr[f][i];
            return k;
        };
        auto split = [&](int64_t s, uint64_t k) {
            by_part[s] = low_bits >= 64 ? 0 : k >> low_bits;
            cls_part[s] = k;
        };
        if (total_bits <= 32 && n <= INT32_MAX) {
            hvec<uint32_t> key(n), ord(n);
            parallel_for(n_chunks, [&](int c) {
                for (int64_t i = c * kChunk; i < std::min<int64_t>(n, (c + 1) * kChunk); ++i) {
                    key[i] = uint32_t(packed(i));
                    ord[i] = uint32_t(i);
                }
            });
            tr.mark("keys");
            radix_sort(key, ord, total_bits);
            tr.mark("radix");
            parallel_for(n_chunks, [&](int c) {
                for (int64_t s = c * kChunk; s < std::min<int64_t>(n, (c + 1) * kChunk); ++s) {
                    order[s] = ord[s];
                    split(s, key[s]);
                }
            });
        } else {
            hvec<uint64_t> key(n);
            parallel_for(n_chunks, [&](int c) {
                for (int64_t i = c * kChunk; i < std::min<int64_t>(n, (c + 1) * kChunk); ++i) {
                    key[i] = packed(i);
                    order[i] = i;
                }
            });
            tr.mark("keys");
            radix_sort(key, order, total_bits);
            tr.mark("radix");
            parallel_for(n_chunks, [&](int c) {
                for (int64_t s = c * kChunk; s < std::min<int64_t>(n, (c + 1) * kChunk); ++s) split(s, key[s]);
            });
        }
    } else {
        // Key too wide for one word: comparison sort on the rank tuple.
        std::iota(order.begin(), order.end(), int64_t(0));
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
    tr.mark("parts");
    // ---- ranks per sorted position (from the packed key when there is one)
    const int W = 1 + n_by + n_across;
    hvec<uint32_t> srank(static_cast<size_t>(n) * size_t(W));
    {
        const size_t nw = static_cast<size_t>(W);
        std::vector<int> shift(nw), bits(nw);
        std::vector<const hvec<uint32_t> *> src(nw);
        shift[0] = acr_bits;
        bits[0] = ron.bits;
        src[0] = &ron.rank;
        int sh = low_bits;
        for (int j = n_by - 1; j >= 0; --j) {
            shift[size_t(1 + j)] = sh;
            bits[size_t(1 + j)] = rby[size_t(j)].bits;
            src[size_t(1 + j)] = &rby[size_t(j)].rank;
            sh += rby[size_t(j)].bits;
        }
        for (int j = 0; j < n_across; ++j) {
            shift[size_t(1 + n_by + j)] = acr_shift[size_t(j)];
            bits[size_t(1 + n_by + j)] = racr[size_t(j)].bits;
            src[size_t(1 + n_by + j)] = &racr[size_t(j)].rank;
        }
        const bool packed = total_bits <= 64;
        const int64_t kChunk = item_chunk(n);
        parallel_for(int((n + kChunk - 1) / kChunk), [&](int c) {
            const int64_t s0 = c * kChunk, s1 = std::min<int64_t>(n, s0 + kChunk);
            for (int64_t s = s0; s < s1; ++s) {
                uint32_t *o = srank.data() + size_t(s) * size_t(W);
                for (int k = 0; k < W; ++k)
                    o[k] = packed ? uint32_t((cls_part[size_t(s)] >> shift[size_t(k)]) &
                                             ((uint64_t(1) << bits[size_t(k)]) - 1))
                                  : (*src[size_t(k)])[size_t(order[size_t(s)])];
            }
        });
    }
    tr.mark("srank");
    // ---- per sorted position: length, and prefix sums of frames and squared lengths
    hvec<int32_t> len_s(static_cast<size_t>(n));
    hvec<int64_t> pf(static_cast<size_t>(n) + 1), pq(static_cast<size_t>(n) + 1);
    {
        // two-level scan over fixed chunks: chunk sums, their prefix, then the fill
        const int64_t kChunk = item_chunk(n);
        const int nc = int((n + kChunk - 1) / kChunk);
        std::vector<int64_t> cf(size_t(nc) + 1, 0), cq(size_t(nc) + 1, 0);
        parallel_for(nc, [&](int c) {
            int64_t f = 0, q = 0;
            for (int64_t s = c * kChunk; s < std::min<int64_t>(n, (c + 1) * kChunk); ++s) {
                const int64_t L = ds->item_len[size_t(order[s])];
                len_s[s] = int32_t(L);
                f += L;
                q += L * L;
            }
            cf[size_t(c) + 1] = f;
            cq[size_t(c) + 1] = q;
        });
        for (int c = 0; c < nc; ++c) {
            cf[size_t(c) + 1] += cf[size_t(c)];
            cq[size_t(c) + 1] += cq[size_t(c)];
        }
        pf[0] = pq[0] = 0;
        parallel_for(nc, [&](int c) {
            int64_t f = cf[size_t(c)], q = cq[size_t(c)];
            for (int64_t s = c * kChunk; s < std::min<int64_t>(n, (c + 1) * kChunk); ++s) {
                f += len_s[s];
                q += int64_t(len_s[s]) * len_s[s];
                pf[s + 1] = f;
                pq[s + 1] = q;
            }
        });
    }

    tr.mark("lengths");
    // ---- walk the groups: chunks of whole groups in parallel, then stitch
    const int n_threads = int(std::min<int64_t>(HostPool::get().size(), std::max<int64_t>(1, n / 4096)));
    // more shares than threads: the pool hands them out dynamically (group sizes vary)
    const int n_shares = int(std::min<int64_t>(16 * int64_t(n_threads), std::max<int64_t>(1, n / 512)));
    std::vector<int64_t> cut(size_t(n_shares) + 1, n);
    cut[0] = 0;
    for (int k = 1; k < n_shares; ++k) {
        int64_t c = std::max(cut[k - 1], n * k / n_shares);
        while (c > 0 && c < n && by_part[c] == by_part[c - 1]) ++c;   // move to a group start
        cut[k] = c;
    }
    std::vector<Sink> parts(static_cast<size_t>(n_shares));
    WalkCtx wc{ds.get(), t.get(), &order, &by_part, &cls_part, srank.data(), W, &pf, &pq, n_across};
    t->key_values = {ron.values, ron.values};
    for (auto &r : rby) t->key_values.push_back(r.values);
    for (auto &r : racr) t->key_values.push_back(r.values);
    for (auto &r : racr) t->key_values.push_back(r.values);
    t->key_bits = {ron.bits, ron.bits};
    for (auto &r : rby) t->key_bits.push_back(r.bits);
    for (auto &r : racr) t->key_bits.push_back(r.bits);
    for (auto &r : racr) t->key_bits.push_back(r.bits);
    t->key_card = {uint32_t(ron.values.size()), uint32_t(ron.values.size())};
    for (auto &r : rby) t->key_card.push_back(uint32_t(r.values.size()));
    for (auto &r : racr) t->key_card.push_back(uint32_t(r.values.size()));
    for (auto &r : racr) t->key_card.push_back(uint32_t(r.values.size()));
    parallel_for(n_shares, [&](int k) { walk_groups<false>(wc, cut[k], cut[k + 1], parts[size_t(k)]); });
    tr.mark("walk");
    size_t n_cells = 0, n_groups = 0, n_unit_ints = 0, n_big_ints = 0;
    int64_t n_slots = 0;
    for (auto &p : parts) n_unit_ints += p.n_unit_ints;   // small-cell units first
    const size_t n_small_ints = n_unit_ints;
    n_unit_ints = 0;
    for (auto &p : parts) {
        p.cell_base = n_cells;
        p.unit_base = n_unit_ints;
        p.big_unit_base = n_small_ints + n_big_ints;
        n_big_ints += p.n_big_unit_ints;
        p.group_base = n_groups;
        p.slot_base = n_slots;
        n_cells += p.n_cells;
        n_unit_ints += p.n_unit_ints;
        n_groups += p.n_groups;
        n_slots += p.pair_slots;
        t->sum_nx += p.sum_nx;
        t->total_triplets += p.total_triplets;
        t->n_pairs_needed += p.pairs_needed;
        t->dtw_cells_needed += p.dtw_needed;
        t->dtw_cells_sym += p.dtw_sym;
    }
    t->n_pair_slots = n_slots;
    t->cells.resize(n_cells);
    t->n_triplets.resize(n_cells);
    t->rkeys.resize(n_cells * size_t(t->key_width));
    t->units.resize(n_unit_ints + n_big_ints);
    t->n_units_small = int64_t(n_unit_ints / 3);
    t->groups.resize(n_groups);
    hvec<std::pair<int64_t, int64_t>> kept(n_groups);
    std::atomic<bool> mismatch{false};
    parallel_for(n_shares, [&](int k) {
        Sink &p = parts[size_t(k)];
        const Sink counted = p;
        p.n_cells = p.n_unit_ints = p.n_big_unit_ints = p.n_groups = 0;
        p.pair_slots = 0;
        p.cells = t->cells.data();
        p.ntrip = t->n_triplets.data();
        p.rkeys = t->rkeys.data();
        p.units = t->units.data();
        p.groups = t->groups.data();
        p.kept = kept.data();
        p.key_width = size_t(t->key_width);
        walk_groups<true>(wc, cut[k], cut[k + 1], p);
        // the walk's streaming stores are weakly ordered: make them visible
        // before the region ends and other threads read the arrays
#if defined(__x86_64__)
        _mm_sfence();
#endif
        std::atomic_thread_fence(std::memory_order_seq_cst);
        if (p.n_cells != counted.n_cells || p.n_unit_ints != counted.n_unit_ints ||
            p.n_big_unit_ints != counted.n_big_unit_ints || p.n_groups != counted.n_groups)
            mismatch = true;  // both passes walk the same share: cannot happen
    });
    if (mismatch) fail(FABX_EINVAL, "internal error: task walk passes disagree");

    tr.mark("stitch");
    // ---- task items in task order, packed frame offsets
    int64_t nt = 0, frame_total = 0;
    for (size_t gi = 0; gi < t->groups.size(); ++gi) {
        Group &g = t->groups[gi];
        g.item0 = nt;
        g.n_items = kept[gi].second - kept[gi].first;
        g.frame0 = frame_total;
        g.n_frames = pf[kept[gi].second] - pf[kept[gi].first];
        t->n_dmat += g.n_frames * g.n_frames;
        nt += g.n_items;
        frame_total += g.n_frames;
    }
    tr.mark("groups");
    t->items.resize(size_t(nt));
    t->item_len.resize(size_t(nt));
    t->item_src.resize(size_t(nt));
    t->item_dst.resize(size_t(nt));
    t->item_group.resize(size_t(nt));
    t->item_pos_of.resize(size_t(n));
    {
        const int64_t kChunk = item_chunk(n);
        parallel_for(int((n + kChunk - 1) / kChunk), [&](int c) {
            std::fill(t->item_pos_of.begin() + c * kChunk,
                      t->item_pos_of.begin() + std::min<int64_t>(n, (c + 1) * kChunk), int64_t(-1));
        });
    }
    // task items in balanced chunks of task positions; a chunk may start inside
    // a group, whose first frame offset then comes from the frame prefix
    const int64_t G = int64_t(t->groups.size());
    const int64_t q_chunk = item_chunk(nt);
    const int n_qc = int(std::max<int64_t>(1, (nt + q_chunk - 1) / q_chunk));
    std::vector<int> max_len_part(static_cast<size_t>(n_qc), 0);
    parallel_for(n_qc, [&](int k) {
        const int64_t q0 = int64_t(k) * q_chunk, q1 = std::min<int64_t>(nt, q0 + q_chunk);
        if (q0 >= q1) return;
        // group holding task position q0: the last with item0 <= q0
        int64_t lo = 0, hi = G;
        while (hi - lo > 1) {
            const int64_t mid = (lo + hi) / 2;
            if (t->groups[size_t(mid)].item0 <= q0) lo = mid; else hi = mid;
        }
        int ml = 0;
        int64_t q = q0;
        for (int64_t gi = lo; q < q1; ++gi) {
            const Group &g = t->groups[size_t(gi)];
            const int64_t s_first = kept[size_t(gi)].first;
            const int64_t s0 = s_first + (q - g.item0);
            const int64_t s1 = std::min<int64_t>(kept[size_t(gi)].second, s_first + (q1 - g.item0));
            int64_t frame = g.frame0 + (pf[s0] - pf[s_first]);
            for (int64_t s = s0; s < s1; ++s, ++q) {
                const int64_t it = order[s];
                t->items[q] = it;
                t->item_pos_of[it] = q;
                t->item_src[q] = ds->item_start[size_t(it)];
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
    tr.mark("items");

    t->n_frames = frame;
    plan_blocks(*t);
    tr.mark("blocks");
    return t;
}

}  // namespace fabx
