// Host-side integer sorting helpers shared by the task builder and collapse.
#pragma once

#include <algorithm>
#include <cstdint>
#include <vector>

namespace fabx {

// Stable LSD radix sort of (key, idx) pairs by a key of `key_bits` bits
// (12-bit digits, only the digits the key uses).  Ties keep their input order.
template <typename KeyVec, typename IdxVec>
void radix_sort_pairs(KeyVec &key, IdxVec &idx, int key_bits) {
    constexpr int kDigit = 12;
    constexpr size_t kBuckets = size_t(1) << kDigit;
    const size_t n = key.size();
    if (key_bits <= 0 || n < 2) return;
    KeyVec k2(n);
    IdxVec i2(n);
    std::vector<size_t> count(kBuckets + 1);
    for (int shift = 0; shift < key_bits; shift += kDigit) {
        std::fill(count.begin(), count.end(), 0);
        for (size_t i = 0; i < n; ++i) ++count[((key[i] >> shift) & (kBuckets - 1)) + 1];
        for (size_t b = 0; b < kBuckets; ++b) count[b + 1] += count[b];
        for (size_t i = 0; i < n; ++i) {
            const size_t d = count[(key[i] >> shift) & (kBuckets - 1)]++;
            k2[d] = key[i];
            i2[d] = idx[i];
        }
        key.swap(k2);
        idx.swap(i2);
    }
}

// Dense ranks (0 .. u-1, in value order) of an int32 column; returns the bits
// needed to hold a rank.  A direct table is used when the value range is small.
inline int dense_ranks(const int32_t *vals, size_t n, size_t stride, std::vector<uint32_t> &rank) {
    rank.resize(n);
    if (n == 0) return 0;
    int32_t mn = vals[0], mx = vals[0];
    for (size_t i = 0; i < n; ++i) {
        mn = std::min(mn, vals[i * stride]);
        mx = std::max(mx, vals[i * stride]);
    }
    const int64_t range = int64_t(mx) - int64_t(mn) + 1;
    uint64_t u = 0;
    if (range <= std::max<int64_t>(4 * int64_t(n), 1 << 16)) {
        std::vector<int32_t> table(size_t(range), -1);
        for (size_t i = 0; i < n; ++i) table[size_t(int64_t(vals[i * stride]) - mn)] = 0;
        for (auto &t : table)
            if (t == 0) t = int32_t(u++);
        for (size_t i = 0; i < n; ++i) rank[i] = uint32_t(table[size_t(int64_t(vals[i * stride]) - mn)]);
    } else {
        std::vector<int32_t> sorted(n);
        for (size_t i = 0; i < n; ++i) sorted[i] = vals[i * stride];
        std::sort(sorted.begin(), sorted.end());
        sorted.erase(std::unique(sorted.begin(), sorted.end()), sorted.end());
        u = sorted.size();
        for (size_t i = 0; i < n; ++i)
            rank[i] = uint32_t(std::lower_bound(sorted.begin(), sorted.end(), vals[i * stride]) - sorted.begin());
    }
    int bits = 0;
    while ((uint64_t(1) << bits) < u) ++bits;
    return bits;
}

}  // namespace fabx
