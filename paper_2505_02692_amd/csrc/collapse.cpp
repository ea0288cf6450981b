// Aggregation of cell scores into the ABX error rate (Background section: the
// overall discriminability D is a weighted average over cells; the phoneme
// task averages over contexts, then speakers, then phonemes; Score.collapse
// offers cell-size weighting or averaging level by level).  FP64 on the host.
#include <algorithm>
#include <map>
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
    // rows: remaining key columns -> mean score
    std::vector<int> cols(static_cast<size_t>(K));
    std::iota(cols.begin(), cols.end(), 0);
    std::map<std::vector<int32_t>, double> rows;
    for (size_t i = 0; i < n; ++i) {
        std::vector<int32_t> k(t.keys.begin() + int64_t(i) * K, t.keys.begin() + int64_t(i + 1) * K);
        rows[k] = double(res.half_units[i]) / (2.0 * double(t.n_triplets[i]));
    }
    for (const auto &lv : levels) {
        std::vector<int> keep_pos;  // positions (in the current key) of kept columns
        std::vector<int> kept;
        for (size_t p = 0; p < cols.size(); ++p)
            if (std::find(lv.begin(), lv.end(), t.key_attr[size_t(cols[p])]) == lv.end()) {
                keep_pos.push_back(int(p));
                kept.push_back(cols[p]);
            }
        std::map<std::vector<int32_t>, std::pair<double, int64_t>> acc;
        for (const auto &kv : rows) {
            std::vector<int32_t> k;
            k.reserve(keep_pos.size());
            for (int p : keep_pos) k.push_back(kv.first[size_t(p)]);
            auto &a = acc[k];
            a.first += kv.second;
            a.second += 1;
        }
        rows.clear();
        for (auto &kv : acc) rows[kv.first] = kv.second.first / double(kv.second.second);
        cols = kept;
    }
    double s = 0.0;
    for (auto &kv : rows) s += kv.second;
    return 1.0 - s / double(rows.size());
}

}  // namespace fabx
