// Aggregation of cell scores into the ABX error rate (Background section: the
// overall discriminability D is a weighted average over cells; the phoneme
// task averages over contexts, then speakers, then phonemes; Score.collapse
// offers cell-size weighting or averaging level by level).  FP64 on the host.
//
// Level by level: every key value is replaced by its dense rank (computed by
// the task builder); for a level, the ranks of the columns that remain form
// one key.  Rows with equal keys are averaged (unweighted, summed in row
// order): when the key space is small, through a direct table indexed by the
// mixed-radix key (no sort; threads own key ranges of the table), otherwise
// after a stable radix sort of the bit-packed key.  The averaged rows, in key order,
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
    {
        const size_t kChunk = size_t(1) << 16;
        HostPool::get().parallel_for(int((n + kChunk - 1) / kChunk), [&](int c) {
            for (size_t i = size_t(c) * kChunk; i < std::min(n, size_t(c + 1) * kChunk); ++i)
                score[i] = double(res.half_units[i]) / (2.0 * double(t.n_triplets[i]));
        });
    }
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
            // Each part owns a contiguous key range of the table: it scans all
            // keys in row order and accumulates its own, so every key's sum is
            // formed in row order whatever the part count.
            hvec<uint32_t> keyv(m);
            const size_t kChunk = size_t(1) << 16;
            HostPool &hp = HostPool::get();
            hp.parallel_for(int((m + kChunk - 1) / kChunk), [&](int c) {
                for (size_t i = size_t(c) * kChunk; i < std::min(m, size_t(c + 1) * kChunk); ++i)
                    keyv[i] = uint32_t(mixed(i));
            });
            // parts of at least 4096 keys, and only when there are many rows
            const size_t n_parts = m >= (size_t(1) << 15)
                                       ? std::max<size_t>(1, std::min<size_t>(size_t(hp.size()), nk / 4096))
                                       : 1;
            hvec<Acc> tab(nk);
            std::vector<size_t> part_rows(n_parts + 1, 0);
            hp.parallel_for(int(n_parts), [&](int r) {
                const size_t k0 = nk * size_t(r) / n_parts, k1 = nk * size_t(r + 1) / n_parts;
                for (size_t k = k0; k < k1; ++k) tab[k] = Acc{0.0, 0u, 0u};
                for (size_t i = 0; i < m; ++i) {
                    const size_t k = keyv[i];
                    if (k < k0 || k >= k1) continue;
                    Acc &acc = tab[k];
                    if (acc.cnt++ == 0) acc.first = uint32_t(i);
                    acc.sum += score[i];
                }
                size_t used = 0;
                for (size_t k = k0; k < k1; ++k) used += tab[k].cnt != 0;
                part_rows[size_t(r) + 1] = used;
            });
            for (size_t r = 0; r < n_parts; ++r) part_rows[r + 1] += part_rows[r];
            nscore.resize(part_rows[n_parts]);
            nrep.resize(part_rows[n_parts]);
            hp.parallel_for(int(n_parts), [&](int r) {
                const size_t k0 = nk * size_t(r) / n_parts, k1 = nk * size_t(r + 1) / n_parts;
                size_t o = part_rows[size_t(r)];
                for (size_t k = k0; k < k1; ++k)
                    if (tab[k].cnt) {
                        nscore[o] = tab[k].sum / double(tab[k].cnt);
                        nrep[o] = rep[tab[k].first];
                        ++o;
                    }
            });
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
