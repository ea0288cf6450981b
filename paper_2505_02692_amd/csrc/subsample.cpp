// The Subsampler of the Task interface (library overview, "Task" paragraph):
// per cell, caps on the number of a, b and x (drawn independently), and, with
// ACROSS conditions, a limit on the distinct ACROSS values x takes.
//
// Reading of the paper: the limit is on x's ACROSS value (its ON value is
// fixed within a cell); without ACROSS, X is A itself, so the one set is
// capped by both the a and the x cap and stays the same set; cells left
// without a triple are dropped.  Every random choice is a draw of the
// counter-based generator Philox4x32-10 (Salmon, Moraes, Dror, Shaw,
// "Parallel random numbers: as easy as 1, 2, 3", SC'11) at a counter made of
// the cell's index in the full task, the set (0 = A, 1 = B, 2 = X, 3 = the
// ACROSS limit) and the position, keyed by the seed: a subsample is a pure
// function of those, so scores are reproducible and checkable.  A capped set
// keeps the items with the smallest draws (position breaks ties), in their
// original order.
//
// Layout: a cell whose sets are not reduced keeps its BY group; a cell with a
// reduced set gets a group of its own holding only its sampled items (A, B,
// and X when it is a set of its own), so the DTW kernels compute just the
// pairs such a cell needs.  Items of those groups repeat items of the dataset.
#include <algorithm>
#include <cstring>

#include "internal.h"

namespace fabx {
namespace {

// Philox4x32-10: ten rounds of two 32x32 -> 64-bit multiplications of
// counter words 0 and 2, their high halves mixed into words 1 and 3 with the
// key, a word permutation, and the key advanced by the Weyl constants.
struct Philox {
    uint32_t k0, k1;
    explicit Philox(uint64_t seed) : k0(uint32_t(seed)), k1(uint32_t(seed >> 32)) {}
    uint32_t first(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3 = 0) const {
        uint32_t a = k0, b = k1;
        for (int r = 0; r < 10; ++r) {
            const uint64_t p0 = uint64_t(0xD2511F53u) * c0, p1 = uint64_t(0xCD9E8D57u) * c2;
            const uint32_t n0 = uint32_t(p1 >> 32) ^ c1 ^ a, n2 = uint32_t(p0 >> 32) ^ c3 ^ b;
            c1 = uint32_t(p1);
            c3 = uint32_t(p0);
            c0 = n0;
            c2 = n2;
            a += 0x9E3779B9u;
            b += 0xBB67AE85u;
        }
        return c0;
    }
};

// Positions 0..n-1 kept by a cap: all when cap <= 0 or n <= cap, else the cap
// positions with the smallest draws at (cell, which, position), ascending.
std::vector<int32_t> pick(const Philox &ph, int64_t cell, int which, int32_t n, int32_t cap) {
    std::vector<int32_t> pos(static_cast<size_t>(n));
    for (int32_t i = 0; i < n; ++i) pos[size_t(i)] = i;
    if (cap <= 0 || n <= cap) return pos;
    std::vector<std::pair<uint32_t, int32_t>> r(static_cast<size_t>(n));
    for (int32_t i = 0; i < n; ++i) r[size_t(i)] = {ph.first(uint32_t(cell), uint32_t(which), uint32_t(i)), i};
    std::nth_element(r.begin(), r.begin() + cap, r.end());
    pos.resize(size_t(cap));
    for (int32_t i = 0; i < cap; ++i) pos[size_t(i)] = r[size_t(i)].second;
    std::sort(pos.begin(), pos.end());
    return pos;
}

constexpr int64_t kUnitBudget = 8192;     // as the task build: comparisons per triplet work unit
constexpr int64_t kSortedMinPerX = 8192;  // cells counted from sorted rows

}  // namespace

std::shared_ptr<TaskImpl> subsample_task(const TaskImpl &t, const fabx_subsampler &sub) {
    const int n_across = int(t.across.size());
    const size_t K = size_t(t.key_width);
    const int64_t n_cells = int64_t(t.cells.size());
    const Philox ph(sub.seed);
    // ---- 1. the ACROSS limit: of each family of cells (equal key but for the
    // across_x columns, consecutive in cell order), keep max_x_across
    std::vector<char> keep(size_t(n_cells), 1);
    if (n_across > 0 && sub.max_x_across > 0) {
        const size_t fw = K - size_t(n_across);
        int64_t c = 0;
        while (c < n_cells) {
            int64_t e = c + 1;
            while (e < n_cells && std::memcmp(&t.rkeys[size_t(e) * K], &t.rkeys[size_t(c) * K], fw * 4) == 0) ++e;
            if (e - c > sub.max_x_across) {
                const std::vector<int32_t> kept = pick(ph, c, 3, int32_t(e - c), sub.max_x_across);
                std::fill(keep.begin() + c, keep.begin() + e, 0);
                for (int32_t j : kept) keep[size_t(c + j)] = 1;
            }
            c = e;
        }
    }
    // ---- 2. caps per cell (positions inside the cell's A / B / X ranges)
    int32_t cap_ax = 0;  // without ACROSS: the shared A = X set's cap
    for (int32_t v : {sub.max_a, sub.max_x})
        if (v > 0) cap_ax = cap_ax > 0 ? std::min(cap_ax, v) : v;
    struct Sampled {
        int64_t cell;
        std::vector<int32_t> a, b, x;  // group-local positions
        bool own_group;
    };
    std::vector<Sampled> cells;
    for (int64_t c = 0; c < n_cells; ++c) {
        if (!keep[size_t(c)]) continue;
        const CellDev &cd = t.cells[size_t(c)];
        Sampled s{c, {}, {}, {}, false};
        const bool within = cd.exclude_self != 0;
        const std::vector<int32_t> pa = pick(ph, c, 0, cd.na, within ? cap_ax : sub.max_a);
        const std::vector<int32_t> pb = pick(ph, c, 1, cd.nb, sub.max_b);
        if (within && pa.size() < 2) continue;
        for (int32_t i : pa) s.a.push_back(cd.a0 + i);
        for (int32_t i : pb) s.b.push_back(cd.b0 + i);
        if (within) {
            s.x = s.a;
        } else {
            for (int32_t i : pick(ph, c, 2, cd.nx, sub.max_x)) s.x.push_back(cd.x0 + i);
        }
        s.own_group = int32_t(s.a.size()) < cd.na || int32_t(s.b.size()) < cd.nb || int32_t(s.x.size()) < cd.nx;
        cells.push_back(std::move(s));
    }
    // ---- 3. the new task: BY groups still used whole, then one group per reduced cell
    auto out = std::make_shared<TaskImpl>();
    TaskImpl &u = *out;
    u.ds = t.ds;
    u.on = t.on;
    u.by = t.by;
    u.across = t.across;
    u.key_attr = t.key_attr;
    u.key_width = t.key_width;
    u.key_values = t.key_values;
    u.key_bits = t.key_bits;
    u.key_card = t.key_card;
    u.subsampled = true;
    std::vector<int32_t> new_gid(t.groups.size(), -1);
    std::vector<std::vector<int64_t>> gitems;  // per new group: task items of `t`
    for (const Sampled &s : cells) {
        if (s.own_group) continue;
        const int32_t g = t.cells[size_t(s.cell)].group;
        if (new_gid[size_t(g)] < 0) {
            new_gid[size_t(g)] = int32_t(gitems.size());
            const Group &gr = t.groups[size_t(g)];
            std::vector<int64_t> it(size_t(gr.n_items));
            for (int64_t i = 0; i < gr.n_items; ++i) it[size_t(i)] = gr.item0 + i;
            gitems.push_back(std::move(it));
        }
    }
    u.cells.resize(cells.size());
    u.n_triplets.resize(cells.size());
    u.rkeys.resize(cells.size() * K);
    std::vector<int32_t> cell_gid(cells.size());
    for (size_t k = 0; k < cells.size(); ++k) {
        const Sampled &s = cells[k];
        const CellDev &cd = t.cells[size_t(s.cell)];
        const bool within = cd.exclude_self != 0;
        CellDev nc = cd;
        if (!s.own_group) {
            nc.group = new_gid[size_t(cd.group)];
        } else {
            const Group &gr = t.groups[size_t(cd.group)];
            std::vector<int64_t> it;
            for (int32_t p : s.a) it.push_back(gr.item0 + p);
            for (int32_t p : s.b) it.push_back(gr.item0 + p);
            if (!within)
                for (int32_t p : s.x) it.push_back(gr.item0 + p);
            nc.group = int32_t(gitems.size());
            nc.a0 = 0;
            nc.na = int32_t(s.a.size());
            nc.b0 = nc.na;
            nc.nb = int32_t(s.b.size());
            nc.x0 = within ? 0 : nc.na + nc.nb;
            nc.nx = int32_t(s.x.size());
            gitems.push_back(std::move(it));
        }
        cell_gid[k] = nc.group;
        u.cells[k] = nc;
        const int64_t na = nc.na, nb = nc.nb, nx = nc.nx;
        u.n_triplets[k] = within ? na * (na - 1) * nb : na * nb * nx;
        u.total_triplets += u.n_triplets[k];
        u.sum_nx += nx;
        std::memcpy(&u.rkeys[k * K], &t.rkeys[size_t(s.cell) * K], K * 4);
    }
    // triplet work units, as the task build makes them: small cells first (one
    // unit per run of x with at most kUnitBudget comparisons), then one unit per
    // x of the cells counted from sorted rows
    std::vector<int32_t> small_u, big_u;
    for (size_t k = 0; k < cells.size(); ++k) {
        const CellDev &nc = u.cells[k];
        const int64_t per_x = std::max<int64_t>(1, int64_t(nc.na) * nc.nb);
        const bool big = per_x >= kSortedMinPerX && nc.nb <= kSortedMaxB;
        const int64_t chunk = big ? 1 : std::max<int64_t>(1, kUnitBudget / per_x);
        auto &dst = big ? big_u : small_u;
        for (int64_t x = 0; x < nc.nx; x += chunk) {
            dst.push_back(int32_t(k));
            dst.push_back(int32_t(x));
            dst.push_back(int32_t(std::min<int64_t>(nc.nx, x + chunk)));
        }
    }
    u.n_units_small = int64_t(small_u.size() / 3);
    u.units.resize(small_u.size() + big_u.size());
    std::copy(small_u.begin(), small_u.end(), u.units.begin());
    std::copy(big_u.begin(), big_u.end(), u.units.begin() + std::ptrdiff_t(small_u.size()));
    // items and groups
    int64_t n_items = 0;
    for (auto &v : gitems) n_items += int64_t(v.size());
    u.items.resize(size_t(n_items));
    u.item_len.resize(size_t(n_items));
    u.item_src.resize(size_t(n_items));
    u.item_dst.resize(size_t(n_items));
    u.item_group.resize(size_t(n_items));
    u.item_pos_of.assign(t.item_pos_of.size(), int64_t(-1));
    u.groups.resize(gitems.size());
    int64_t q = 0, frame = 0, slots = 0;
    for (size_t g = 0; g < gitems.size(); ++g) {
        Group &gr = u.groups[g];
        gr.item0 = q;
        gr.n_items = int64_t(gitems[g].size());
        gr.frame0 = frame;
        gr.pair_base = slots;
        for (int64_t ti : gitems[g]) {
            u.items[size_t(q)] = t.items[size_t(ti)];
            if (u.item_pos_of[size_t(t.items[size_t(ti)])] < 0) u.item_pos_of[size_t(t.items[size_t(ti)])] = q;
            u.item_len[size_t(q)] = t.item_len[size_t(ti)];
            u.item_src[size_t(q)] = t.item_src[size_t(ti)];
            u.item_dst[size_t(q)] = frame;
            u.item_group[size_t(q)] = int32_t(g);
            u.max_len = std::max(u.max_len, int(t.item_len[size_t(ti)]));
            frame += t.item_len[size_t(ti)];
            ++q;
        }
        gr.n_frames = frame - gr.frame0;
        u.n_dmat += gr.n_frames * gr.n_frames;
        slots += gr.n_items * gr.n_items;
    }
    u.n_frames = frame;
    u.n_pair_slots = slots;
    // the pairs the cells need (x with a != x, x with b), per group, in one
    // bitmap per group: counts of ordered and unordered pairs and their DTW cells
    std::vector<std::vector<size_t>> gcells(gitems.size());
    for (size_t k = 0; k < cells.size(); ++k) gcells[size_t(cell_gid[k])].push_back(k);
    for (size_t g = 0; g < gitems.size(); ++g) {
        const Group &gr = u.groups[g];
        const int64_t n = gr.n_items;
        std::vector<uint8_t> need(size_t(n * n), 0);
        for (size_t k : gcells[g]) {
            const CellDev &nc = u.cells[k];
            for (int32_t x = nc.x0; x < nc.x0 + nc.nx; ++x) {
                for (int32_t a = nc.a0; a < nc.a0 + nc.na; ++a)
                    if (!(nc.exclude_self && a == x)) need[size_t(x * n + a)] = 1;
                for (int32_t b = nc.b0; b < nc.b0 + nc.nb; ++b) need[size_t(x * n + b)] = 1;
            }
        }
        auto L = [&](int64_t p) { return int64_t(u.item_len[size_t(gr.item0 + p)]); };
        for (int64_t x = 0; x < n; ++x)
            for (int64_t y = 0; y < n; ++y) {
                const bool nxy = need[size_t(x * n + y)] != 0;
                if (nxy) {
                    ++u.n_pairs_needed;
                    u.dtw_cells_needed += L(x) * L(y);
                }
                if (x <= y && (nxy || need[size_t(y * n + x)])) u.dtw_cells_sym += L(x) * L(y);
            }
    }
    plan_blocks(u);
    return out;
}

}  // namespace fabx
