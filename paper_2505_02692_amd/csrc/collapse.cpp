// Aggregation of cell scores into the ABX error rate (Background section: the
// overall discriminability D is a weighted average over cells; the phoneme
// task averages over contexts, then speakers, then phonemes; Score.collapse
// offers cell-size weighting or averaging level by level).  FP64 on the host.
//
// Level by level: every key value is replaced by its dense rank (computed by
// the task builder); for a level, the ranks of the columns that remain are
// packed into one key.  Rows with equal keys are averaged (unweighted, summed
// in row order): when the key space is small, through a direct table indexed
// by the key (one pass, no sort), otherwise after a stable radix sort.  The
// averaged rows, in key order, carry on to the next level; the last rows are
// averaged flat.
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
    // rows: dense ranks of the key values (from the task builder), row-major [m x K]
    const uint32_t *rows = t.rkeys.data();
    std::vector<uint32_t> own;  // rows after the first level
    std::vector<size_t> cols(K);  // key columns still present
    std::iota(cols.begin(), cols.end(), size_t(0));
    std::vector<double> score(n);
    for (size_t i = 0; i < n; ++i) score[i] = double(res.half_units[i]) / (2.0 * double(t.n_triplets[i]));
    for (const auto &lv : levels) {
        std::vector<size_t> kept;
        for (size_t c : cols)
            if (std::find(lv.begin(), lv.end(), t.key_attr[c]) == lv.end()) kept.push_back(c);
        int total_bits = 0;
        for (size_t c : kept) total_bits += t.key_bits[c];
        const size_t m = score.size();
        std::vector<double> nscore;
        std::vector<uint32_t> nrows;
        auto pack = [&](size_t i) {
            uint64_t k = 0;
            for (size_t c : kept)
                if (t.key_bits[c]) k = (k << t.key_bits[c]) | rows[i * K + c];
            return k;
        };
        if (total_bits <= 22 && (uint64_t(1) << total_bits) <= 8 * uint64_t(m) + 4096) {
            // direct table: sum and count per key, first row of each key for its ranks
            const size_t nk = size_t(1) << total_bits;
            std::vector<double> sum(nk, 0.0);
            std::vector<uint32_t> cnt(nk, 0), first(nk, 0);
            for (size_t i = 0; i < m; ++i) {
                const uint64_t k = pack(i);
                if (cnt[k]++ == 0) first[k] = uint32_t(i);
                sum[k] += score[i];
            }
            nscore.reserve(m);
            nrows.reserve(m * K);
            for (size_t k = 0; k < nk; ++k)
                if (cnt[k]) {
                    nscore.push_back(sum[k] / double(cnt[k]));
                    nrows.insert(nrows.end(), rows + size_t(first[k]) * K, rows + size_t(first[k]) * K + K);
                }
        } else {
            std::vector<uint32_t> order(m);
            std::iota(order.begin(), order.end(), 0u);
            std::vector<uint64_t> key(m, 0);
            if (total_bits <= 64) {
                for (size_t i = 0; i < m; ++i) key[i] = pack(i);
                radix_sort_pairs(key, order, total_bits);
            } else {
                std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) {
                    for (size_t c : kept)
                        if (rows[a * K + c] != rows[b * K + c]) return rows[a * K + c] < rows[b * K + c];
                    return false;
                });
                uint64_t id = 0;  // run ids as keys
                for (size_t i = 0; i < m; ++i) {
                    if (i > 0)
                        for (size_t c : kept)
                            if (rows[size_t(order[i]) * K + c] != rows[size_t(order[i - 1]) * K + c]) {
                                ++id;
                                break;
                            }
                    key[i] = id;
                }
            }
            // average each run of equal keys; the new rows keep the ranks of the kept columns
            nscore.reserve(m);
            nrows.reserve(m * K);
            for (size_t i = 0; i < m;) {
                size_t j = i;
                double sacc = 0.0;
                while (j < m && key[j] == key[i]) sacc += score[order[j++]];
                nscore.push_back(sacc / double(j - i));
                nrows.insert(nrows.end(), rows + size_t(order[i]) * K, rows + size_t(order[i]) * K + K);
                i = j;
            }
        }
        score.swap(nscore);
        own.swap(nrows);
        rows = own.data();
        cols = kept;
        tr.mark("level");
    }
    double s = 0.0;
    for (double v : score) s += v;
    return 1.0 - s / double(score.size());
}

}  // namespace fabx
