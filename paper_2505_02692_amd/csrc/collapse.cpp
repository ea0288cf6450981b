// Aggregation of cell scores into the ABX error rate (Background section: the
// overall discriminability D is a weighted average over cells; the phoneme
// task averages over contexts, then speakers, then phonemes; Score.collapse
// offers cell-size weighting or averaging level by level).  FP64 on the host.
//
// Level by level: the rows (key tuple, score) are sorted by the key columns
// that remain after removing the level's attributes, equal runs are averaged
// (unweighted), and the averaged rows carry on to the next level.
#include <algorithm>
#include <numeric>

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
    const int K = t.key_width;
    // current rows: keys [m x width] (width = cols.size()), scores [m]
    std::vector<int> cols(static_cast<size_t>(K));
    std::iota(cols.begin(), cols.end(), 0);
    std::vector<int32_t> keys = t.keys;
    std::vector<double> score(n);
    for (size_t i = 0; i < n; ++i) score[i] = double(res.half_units[i]) / (2.0 * double(t.n_triplets[i]));
    size_t width = size_t(K);
    for (const auto &lv : levels) {
        std::vector<size_t> keep;  // positions (in the current key) of the kept columns
        std::vector<int> kept_cols;
        for (size_t p = 0; p < cols.size(); ++p)
            if (std::find(lv.begin(), lv.end(), t.key_attr[size_t(cols[p])]) == lv.end()) {
                keep.push_back(p);
                kept_cols.push_back(cols[p]);
            }
        const size_t m = score.size();
        std::vector<size_t> idx(m);
        std::iota(idx.begin(), idx.end(), size_t(0));
        auto less = [&](size_t a, size_t b) {
            for (size_t p : keep) {
                const int32_t x = keys[a * width + p], y = keys[b * width + p];
                if (x != y) return x < y;
            }
            return a < b;
        };
        auto same = [&](size_t a, size_t b) {
            for (size_t p : keep)
                if (keys[a * width + p] != keys[b * width + p]) return false;
            return true;
        };
        std::sort(idx.begin(), idx.end(), less);
        std::vector<int32_t> nkeys;
        std::vector<double> nscore;
        for (size_t i = 0; i < m;) {
            size_t j = i;
            double s = 0.0;
            while (j < m && same(idx[i], idx[j])) s += score[idx[j++]];
            for (size_t p : keep) nkeys.push_back(keys[idx[i] * width + p]);
            nscore.push_back(s / double(j - i));
            i = j;
        }
        keys.swap(nkeys);
        score.swap(nscore);
        cols = kept_cols;
        width = keep.size();
    }
    double s = 0.0;
    for (double v : score) s += v;
    return 1.0 - s / double(score.size());
}

}  // namespace fabx
