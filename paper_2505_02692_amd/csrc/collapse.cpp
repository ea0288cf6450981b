// Aggregation of cell scores into the ABX error rate (Background section: the
// overall discriminability D is a weighted average over cells; the phoneme
// task averages over contexts, then speakers, then phonemes; Score.collapse
// offers cell-size weighting or averaging level by level).  FP64 on the host.
//
// Level by level: every key value is replaced by its dense rank (computed by
// the task builder); for a level, the ranks of the columns that remain form
// one key.  Rows with equal keys are averaged (unweighted, summed in row
// order): when the key space is small, through a direct table indexed by the
// mixed-radix key (no sort; parts of the table's key range run in parallel),
// otherwise after a stable radix sort of the bit-packed key.  The averaged
// rows, in key order and with the ranks of the columns they keep, carry on to
// the next level; the last rows are averaged flat.
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
    HostPool &hp = HostPool::get();
    // Ranks of the key columns still present, row-major [m x w]: at first the
    // task's dense ranks of every key column ([n x K], read in place); after a
    // level, the kept columns of each averaged row, copied from one of the
    // rows it averages (all of them agree on those columns).
    const size_t K = size_t(t.key_width);
    const uint32_t *C = t.rkeys.data();
    size_t w = K;
    std::vector<size_t> cols(K);  // key column (of the task) at each position of a row
    std::iota(cols.begin(), cols.end(), size_t(0));
    hvec<uint32_t> cur;
    hvec<double> score(n);
    {
        const size_t kChunk = size_t(1) << 16;
        hp.parallel_for(int((n + kChunk - 1) / kChunk), [&](int c) {
            for (size_t i = size_t(c) * kChunk; i < std::min(n, size_t(c + 1) * kChunk); ++i)
                score[i] = double(res.half_units[i]) / (2.0 * double(t.n_triplets[i]));
        });
    }
    for (const auto &lv : levels) {
        std::vector<size_t> kept_pos;  // positions (in the current rows) of the kept columns
        for (size_t j = 0; j < cols.size(); ++j)
            if (std::find(lv.begin(), lv.end(), t.key_attr[cols[j]]) == lv.end()) kept_pos.push_back(j);
        const size_t nw = kept_pos.size();
        int total_bits = 0;
        for (size_t j : kept_pos) total_bits += t.key_bits[cols[j]];
        const size_t m = score.size();
        hvec<double> nscore;
        hvec<uint32_t> ncur;
        // next rows: ranks of the kept columns of current row `src`, into row `o`
        auto carry = [&](size_t o, size_t src) {
            const uint32_t *r = C + src * w;
            uint32_t *d = ncur.data() + o * nw;
            for (size_t j = 0; j < nw; ++j) d[j] = r[kept_pos[j]];
        };
        uint64_t space = 1;  // mixed-radix key space of the kept columns
        for (size_t j : kept_pos)
            space = std::min<uint64_t>(space * std::max<uint32_t>(t.key_card[cols[j]], 1), uint64_t(1) << 40);
        if (space <= (uint64_t(1) << 24) && space <= 2 * uint64_t(m) + 4096) {
            struct Acc {
                double sum;
                uint32_t cnt, first;
            };
            std::vector<uint32_t> card(nw);
            for (size_t j = 0; j < nw; ++j) card[j] = t.key_card[cols[kept_pos[j]]];
            auto mixed = [&](size_t i) {
                const uint32_t *r = C + i * w;
                uint32_t k = 0;
                for (size_t j = 0; j < nw; ++j) k = k * card[j] + r[kept_pos[j]];
                return k;
            };
            // add row i to its key (sums per key in row order; first row kept)
            auto add = [&](Acc *tab, uint32_t k, size_t i) {
                Acc &acc = tab[k];
                acc.first = acc.cnt == 0 ? uint32_t(i) : acc.first;
                acc.cnt += 1;
                acc.sum += score[i];
            };
            const size_t nk = size_t(space);
            hvec<Acc> tab(nk);
            // Parts own contiguous key ranges of the table (part = key >> shift);
            // they are formed only for many rows and when the pool would run
            // them in parallel.  Rows are first grouped by part, stably, so each
            // part adds its rows in row order: every key's sum is formed in row
            // order whatever the part count.
            int shift = 12;
            while ((nk >> shift) >= 16) ++shift;
            const size_t n_parts =
                m >= (size_t(1) << 15) && hp.would_run_parallel() ? ((nk - 1) >> shift) + 1 : 1;
            std::vector<size_t> part_rows(n_parts + 1, 0);
            if (n_parts == 1) {
                shift = 62;  // one part: every key
                for (size_t k = 0; k < nk; ++k) tab[k] = Acc{0.0, 0u, 0u};
                // keys run kAhead rows ahead of the adds, whose table entries are
                // prefetched meanwhile (the table is larger than the L2 cache)
                constexpr size_t kAhead = 16;
                uint32_t ring[kAhead];
                const size_t pre = std::min(m, kAhead);
                for (size_t i = 0; i < pre; ++i) {
                    ring[i] = mixed(i);
                    __builtin_prefetch(&tab[ring[i]], 1);
                }
                for (size_t i = 0; i < m; ++i) {
                    const uint32_t k = ring[i % kAhead];
                    if (i + kAhead < m) {
                        const uint32_t kn = mixed(i + kAhead);
                        ring[i % kAhead] = kn;
                        __builtin_prefetch(&tab[kn], 1);
                    }
                    add(tab.data(), k, i);
                }
                size_t used = 0;
                for (size_t k = 0; k < nk; ++k) used += tab[k].cnt != 0;
                part_rows[1] = used;
            } else {
                // rows in fixed chunks: keys and per-(chunk, part) counts, then a
                // stable scatter of row ids by part
                const size_t kRowChunk = size_t(1) << 13;
                const size_t n_rc = (m + kRowChunk - 1) / kRowChunk;
                hvec<uint32_t> keyv(m), prow(m);
                std::vector<size_t> cnt(n_rc * n_parts, 0);
                hp.parallel_for(int(n_rc), [&](int c) {
                    size_t *h = cnt.data() + size_t(c) * n_parts;
                    for (size_t i = size_t(c) * kRowChunk; i < std::min(m, size_t(c + 1) * kRowChunk); ++i) {
                        const uint32_t k = mixed(i);
                        keyv[i] = k;
                        ++h[k >> shift];
                    }
                });
                std::vector<size_t> part_begin(n_parts + 1, 0);
                size_t run = 0;
                for (size_t r = 0; r < n_parts; ++r) {
                    part_begin[r] = run;
                    for (size_t c = 0; c < n_rc; ++c) {
                        const size_t v = cnt[c * n_parts + r];
                        cnt[c * n_parts + r] = run;
                        run += v;
                    }
                }
                part_begin[n_parts] = run;
                hp.parallel_for(int(n_rc), [&](int c) {
                    size_t *o = cnt.data() + size_t(c) * n_parts;
                    for (size_t i = size_t(c) * kRowChunk; i < std::min(m, size_t(c + 1) * kRowChunk); ++i)
                        prow[o[keyv[i] >> shift]++] = uint32_t(i);
                });
                hp.parallel_for(int(n_parts), [&](int r) {
                    const size_t k0 = size_t(r) << shift, k1 = std::min(nk, size_t(r + 1) << shift);
                    for (size_t k = k0; k < k1; ++k) tab[k] = Acc{0.0, 0u, 0u};
                    for (size_t j = part_begin[size_t(r)]; j < part_begin[size_t(r) + 1]; ++j) {
                        const size_t i = prow[j];
                        add(tab.data(), keyv[i], i);
                    }
                    size_t used = 0;
                    for (size_t k = k0; k < k1; ++k) used += tab[k].cnt != 0;
                    part_rows[size_t(r) + 1] = used;
                });
            }
            tr.mark("level.table");
            for (size_t r = 0; r < n_parts; ++r) part_rows[r + 1] += part_rows[r];
            nscore.resize(part_rows[n_parts]);
            ncur.resize(part_rows[n_parts] * nw);
            hp.parallel_for(int(n_parts), [&](int r) {
                const size_t k0 = n_parts == 1 ? 0 : size_t(r) << shift;
                const size_t k1 = n_parts == 1 ? nk : std::min(nk, size_t(r + 1) << shift);
                size_t o = part_rows[size_t(r)];
                for (size_t k = k0; k < k1; ++k)
                    if (tab[k].cnt) {
                        nscore[o] = tab[k].sum / double(tab[k].cnt);
                        carry(o, tab[k].first);
                        ++o;
                    }
            });
        } else {
            hvec<uint32_t> order(m);
            std::iota(order.begin(), order.end(), 0u);
            hvec<uint64_t> key(m);
            auto rank = [&](size_t i, size_t j) { return C[i * w + kept_pos[j]]; };
            if (total_bits <= 64) {
                for (size_t i = 0; i < m; ++i) {
                    uint64_t k = 0;
                    for (size_t j = 0; j < nw; ++j) {
                        const int b = t.key_bits[cols[kept_pos[j]]];
                        if (b) k = (k << b) | rank(i, j);
                    }
                    key[i] = k;
                }
                radix_sort_pairs(key, order, total_bits);
            } else {
                std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) {
                    for (size_t j = 0; j < nw; ++j)
                        if (rank(a, j) != rank(b, j)) return rank(a, j) < rank(b, j);
                    return false;
                });
                uint64_t id = 0;  // run ids as keys
                for (size_t i = 0; i < m; ++i) {
                    if (i > 0)
                        for (size_t j = 0; j < nw; ++j)
                            if (rank(order[i], j) != rank(order[i - 1], j)) {
                                ++id;
                                break;
                            }
                    key[i] = id;
                }
            }
            // average each run of equal keys, summed in row order
            nscore.reserve(m);
            ncur.reserve(m * nw);
            for (size_t i = 0; i < m;) {
                size_t j = i;
                double sacc = 0.0;
                while (j < m && key[j] == key[i]) sacc += score[order[j++]];
                const size_t o = nscore.size();
                nscore.push_back(sacc / double(j - i));
                ncur.resize((o + 1) * nw);
                carry(o, order[i]);
                i = j;
            }
        }
        score.swap(nscore);
        cur.swap(ncur);
        C = cur.data();
        w = nw;
        std::vector<size_t> ncols;
        for (size_t j : kept_pos) ncols.push_back(cols[j]);
        cols.swap(ncols);
        tr.mark("level");
    }
    double s = 0.0;
    for (double v : score) s += v;
    return 1.0 - s / double(score.size());
}

}  // namespace fabx
