// Aggregation of cell scores into the ABX error rate (Background section: the
// overall discriminability D is a weighted average over cells; the phoneme
// task averages over contexts, then speakers, then phonemes; Score.collapse
// offers cell-size weighting or averaging level by level).  FP64 on the host.
//
// Level by level: every key value is replaced by its dense rank (computed by
// the task builder); for a level, the ranks of the columns that remain form
// one key.  Rows with equal keys are averaged (unweighted): when the key space
// is small, through a direct table indexed by the mixed-radix key (one pass,
// no sort; with many rows per key, fixed row ranges are accumulated in
// parallel and merged in range order), otherwise after a stable radix sort of
// the bit-packed key (summed in row order).  The averaged rows, in key order,
// carry on to the next level; the last rows are averaged flat.
#include <algorithm>
#include <numeric>

#include "host_pool.h"
#include "host_sort.h"
#include "internal.h"

namespace fabx {

double collapse(const ResultImpl &res, const int32_t *level_attr, const int32_t *level_len,
                int32_t n_levels) {
    const TaskImpl &t = *res.task;
    const size_t n = res.half_units.size();
    if (n == 0) fail(FABX_EINVAL, "the task has no cell");
    if (n_levels == 0) {
        // D = sum W / (2 sum |C|): each triple weighs the same
        long double w = 0, c = 0;
        for (size_t i = 0; i < n; ++i) {
            w += (long double)res.half_units[i];
            c += (long double)t.n_triplets[i];
        }
        return double(1.0L - w / (2.0L * c));
    }
    // validate levels: BY / ACROSS attributes of the task only
    std::vector<std::vector<int32_t>> levels;
    int64_t off = 0;
    for (int32_t l = 0; l < n_levels; ++l) {
        if (level_len[l] < 1) fail(FABX_EINVAL, "empty collapse level");
        std::vector<int32_t> lv(level_attr + off, level_attr + off + level_len[l]);
        off += level_len[l];
        for (int32_t a : lv) {
            const bool is_by = std::find(t.by.begin(), t.by.end(), a) != t.by.end();
            const bool is_ac = std::find(t.across.begin(), t.across.end(), a) != t.across.end();
            if (!is_by && !is_ac)
                fail(FABX_EINVAL, "collapse level names attribute " + std::to_string(a) +
                                      ", which is not a BY or ACROSS attribute of the task");
        }
        levels.push_back(lv);
    }
    Trace tr("collapse");
    const size_t K = size_t(t.key_width);
    // Dense ranks of the key values (from the task builder), row-major [n x K].
    // A row after a level stands for a run of cells that agree on every column
    // still present, so it is represented by one of those cells (rep[i]) and
    // its ranks are read from that cell's row.
    const uint32_t *R = t.rkeys.data();
    hvec<uint32_t> rep(n);
    std::iota(rep.begin(), rep.end(), 0u);
    std::vector<size_t> cols(K);  // key columns still present
    std::iota(cols.begin(), cols.end(), size_t(0));
    hvec<double> score(n);
    for (size_t i = 0; i < n; ++i) score[i] = double(res.half_units[i]) / (2.0 * double(t.n_triplets[i]));
    for (const auto &lv : levels) {
        std::vector<size_t> kept;
        for (size_t c : cols)
            if (std::find(lv.begin(), lv.end(), t.key_attr[c]) == lv.end()) kept.push_back(c);
        int total_bits = 0;
        for (size_t c : kept) total_bits += t.key_bits[c];
        const size_t m = score.size();
        hvec<double> nscore;
        hvec<uint32_t> nrep;
        auto rank = [&](size_t i, size_t c) { return R[size_t(rep[i]) * K + c]; };
        uint64_t space = 1;  // mixed-radix key space of the kept columns
        for (size_t c : kept) space = std::min<uint64_t>(space * std::max<uint32_t>(t.key_card[c], 1), uint64_t(1) << 40);
        if (space <= (uint64_t(1) << 24) && space <= 2 * uint64_t(m) + 4096) {
            struct Acc {
                double sum;
                uint32_t cnt, first;
            };
            auto mixed = [&](size_t i) {
                uint64_t k = 0;
                for (size_t c : kept) k = k * t.key_card[c] + rank(i, c);
                return k;
            };
            const size_t nk = size_t(space);
            // Many rows per key: fixed row ranges (independent of the thread count)
            // fill tables in parallel, merged in range order.
            const size_t n_tab = m >= 16 * nk && m >= (size_t(1) << 18) ? 8 : 1;
            std::vector<hvec<Acc>> tabs(n_tab);
            auto fill = [&](size_t r) {
                hvec<Acc> &tab = tabs[r];
                tab.assign(nk, Acc{0.0, 0u, 0u});
                const size_t i0 = m * r / n_tab, i1 = m * (r + 1) / n_tab;
                for (size_t i = i0; i < i1; ++i) {
                    Acc &a = tab[mixed(i)];
                    if (a.cnt++ == 0) a.first = uint32_t(i);
                    a.sum += score[i];
                }
            };
            if (n_tab > 1) HostPool::get().parallel_for(int(n_tab), [&](int r) { fill(size_t(r)); });
            else fill(0);
            hvec<Acc> &tab = tabs[0];
            for (size_t r = 1; r < n_tab; ++r)
                for (size_t k = 0; k < nk; ++k) {
                    const Acc &b = tabs[r][k];
                    if (!b.cnt) continue;
                    Acc &a = tab[k];
                    if (!a.cnt) a.first = b.first;
                    a.cnt += b.cnt;
                    a.sum += b.sum;
                }
            nscore.reserve(m);
            nrep.reserve(m);
            for (size_t k = 0; k < nk; ++k)
                if (tab[k].cnt) {
                    nscore.push_back(tab[k].sum / double(tab[k].cnt));
                    nrep.push_back(rep[tab[k].first]);
                }
        } else {
            hvec<uint32_t> order(m);
            std::iota(order.begin(), order.end(), 0u);
            hvec<uint64_t> key(m);
            if (total_bits <= 64) {
                for (size_t i = 0; i < m; ++i) {
                    uint64_t k = 0;
                    for (size_t c : kept)
                        if (t.key_bits[c]) k = (k << t.key_bits[c]) | rank(i, c);
                    key[i] = k;
                }
                radix_sort_pairs(key, order, total_bits);
            } else {
                std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) {
                    for (size_t c : kept)
                        if (rank(a, c) != rank(b, c)) return rank(a, c) < rank(b, c);
                    return false;
                });
                uint64_t id = 0;  // run ids as keys
                for (size_t i = 0; i < m; ++i) {
                    if (i > 0)
                        for (size_t c : kept)
                            if (rank(order[i], c) != rank(order[i - 1], c)) {
                                ++id;
                                break;
                            }
                    key[i] = id;
                }
            }
            // average each run of equal keys, summed in row order
            nscore.reserve(m);
            nrep.reserve(m);
            for (size_t i = 0; i < m;) {
                size_t j = i;
                double sacc = 0.0;
                while (j < m && key[j] == key[i]) sacc += score[order[j++]];
                nscore.push_back(sacc / double(j - i));
                nrep.push_back(rep[order[i]]);
                i = j;
            }
        }
        score.swap(nscore);
        rep.swap(nrep);
        cols = kept;
        tr.mark("level");
    }
    double s = 0.0;
    for (double v : score) s += v;
    return 1.0 - s / double(score.size());
}

}  // namespace fabx
