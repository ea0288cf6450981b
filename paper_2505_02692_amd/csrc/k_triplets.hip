// Triplet comparison and per-cell reduction (cell discriminability formula of
// the Background section), in integer half units: each triple adds
// 2 [d(x,a) < d(x,b)] + [d(x,a) == d(x,b)].
//
// Work unit = (cell, range of x), one wave each.  When |A| x |B| fits the
// wave, a pass covers as many whole rows x as fit, |A| x |B| lanes per row;
// otherwise a row's grid is walked in passes of 64 lanes.  Both distances come
// from the row of x in the group's pair matrix (a few hundred bytes, in L1/L2).
// A row with a near tie or a non-robust pair is left to the FP64 recount (one
// ballot per pass finds it); the other rows' counts stay in the lanes and are
// reduced once per unit, then added with one 64-bit atomic, so the result does
// not depend on scheduling.
#include "device_common.h"
#include "kernels.h"

namespace fabx {
namespace kern {
namespace {

using dev::kWave;

constexpr uint8_t kNonRobust = 1;
constexpr uint8_t kMarked = 2;

__global__ __launch_bounds__(256) void k_triplets(const CellDev *__restrict__ cells,
                                                  const int32_t *__restrict__ units, int64_t n_units,
                                                  const int64_t *__restrict__ g_pair_base,
                                                  const int64_t *__restrict__ g_n,
                                                  const float *__restrict__ p32,
                                                  unsigned long long *__restrict__ W,
                                                  uint8_t *flags, float margin,
                                                  int32_t *__restrict__ recount,
                                                  unsigned int *__restrict__ recount_n,
                                                  int64_t recount_cap,
                                                  const unsigned int *__restrict__ scale) {
    const int lane = threadIdx.x % kWave;
    if (scale) margin *= __uint_as_float(*scale);  // margin in units of the largest frame length
    // one wave per unit; the loop bound is uniform across the wave
    for (int64_t unit = int64_t(blockIdx.x) * 4 + threadIdx.x / kWave; unit < n_units;
         unit += int64_t(gridDim.x) * 4) {
    const int32_t cell_id = units[3 * unit];
    const int32_t xb = units[3 * unit + 1], xe = units[3 * unit + 2];
    const CellDev c = cells[cell_id];
    const int64_t base = g_pair_base[c.group];
    const int64_t n = g_n[c.group];
    const int na = c.na, nb = c.nb;
    if (na <= 0 || nb <= 0) continue;  // uniform: no comparisons
    // lane sums of 2 [d_xa < d_xb] + [d_xa == d_xb] over the rows kept
    unsigned long long acc = 0;
    // one comparison of row xl at (al, bl); returns its half units, sets dirty
    auto compare = [&](int xl, int al, int bl, int &dirty) -> unsigned int {
        const float *row = p32 + base + int64_t(xl) * n;
        const float da = row[al], db = row[bl];
        if (flags) {
            uint8_t *frow = flags + base + int64_t(xl) * n;
            const uint8_t fa = frow[al], fb = frow[bl];
            if (fabsf(da - db) <= margin || ((fa | fb) & kNonRobust)) {
                dirty = 1;
                if (!(fa & kMarked)) frow[al] = fa | kMarked;
                if (!(fb & kMarked)) frow[bl] = fb | kMarked;
            }
        }
        return da < db ? 2u : (da == db ? 1u : 0u);
    };
    auto push_row = [&](int xi) {
        const unsigned int k = atomicAdd(recount_n, 1u);
        if (int64_t(k) < recount_cap) {
            recount[2 * int64_t(k)] = cell_id;
            recount[2 * int64_t(k) + 1] = xi;
        }
    };
    const int per_x = na * nb;
    if (per_x <= kWave) {
        // `rows` whole rows per pass: lane = r * per_x + (a * nb + b)
        const int rows = kWave / per_x;
        const int r = lane / per_x, kk = lane - r * per_x;
        const int a = kk / nb, b = kk - a * nb;
        const bool lane_on = r < rows;
        const unsigned long long seg =
            lane_on ? (per_x == kWave ? ~0ull : ((1ull << per_x) - 1ull) << (r * per_x)) : 0ull;
        const int al = c.a0 + a, bl = c.b0 + b;
        unsigned int cnt = 0;
        for (int x0 = xb; x0 < xe; x0 += rows) {
            const int xi = x0 + r;
            const bool row_on = lane_on && xi < xe;
            const int xl = c.x0 + xi;
            int dirty = 0;
            unsigned int add = 0;
            if (row_on && !(c.exclude_self && al == xl)) add = compare(xl, al, bl, dirty);
            if (flags) {
                const unsigned long long dmask = __ballot(dirty);
                if (dmask & seg) {
                    add = 0;
                    if (row_on && kk == 0) push_row(xi);
                }
            }
            cnt += add;
        }
        acc = cnt;
    } else {
        // one row at a time, its |A| x |B| grid in passes of 64 lanes
        const int step_a = kWave / nb, step_b = kWave % nb;
        for (int xi = xb; xi < xe; ++xi) {
            const int xl = c.x0 + xi;
            int a = lane / nb, b = lane % nb;
            unsigned long long cnt = 0;
            int dirty = 0;
            while (a < na) {
                const int al = c.a0 + a, bl = c.b0 + b;
                if (!(c.exclude_self && al == xl)) cnt += compare(xl, al, bl, dirty);
                a += step_a;
                b += step_b;
                if (b >= nb) { b -= nb; ++a; }
            }
            if (flags && dev::wave_any(dirty)) {
                if (lane == 0) push_row(xi);
                continue;
            }
            acc += cnt;
        }
    }
    const unsigned long long total = dev::wave_sum_u64(acc);
    if (lane == 0 && total) atomicAdd(&W[cell_id], total);
    }
}

// Count of sorted values v[0..n) below `key` (strict: v < key) or at most `key`.
__device__ __forceinline__ int count_below(const float *v, int n, float key, bool inclusive) {
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        const bool left = inclusive ? v[mid] <= key : v[mid] < key;
        if (left) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// Large cells, one block per unit (cell, one x): the row's distances to B are
// sorted in LDS (bitonic, with their B positions), then each a adds
// 2|B| - #(d_xb < d_xa) - #(d_xb <= d_xa), which equals the sum over b of
// 2[d_xa < d_xb] + [d_xa == d_xb].  Near ties and non-robust pairs are found as
// in k_triplets (the b within margin of d_xa form one sorted range) and make
// the row go to the FP64 recount with the involved pairs marked.
__global__ __launch_bounds__(256) void k_triplets_sorted(const CellDev *__restrict__ cells,
                                                         const int32_t *__restrict__ units, int64_t n_units,
                                                         const int64_t *__restrict__ g_pair_base,
                                                         const int64_t *__restrict__ g_n,
                                                         const float *__restrict__ p32,
                                                         unsigned long long *__restrict__ W,
                                                         uint8_t *flags, float margin,
                                                         int32_t *__restrict__ recount,
                                                         unsigned int *__restrict__ recount_n,
                                                         int64_t recount_cap,
                                                         const unsigned int *__restrict__ scale) {
    if (scale) margin *= __uint_as_float(*scale);  // margin in units of the largest frame length
    __shared__ float sv[kSortedMaxB];
    __shared__ uint16_t si[kSortedMaxB];
    __shared__ unsigned long long red[4];
    __shared__ int bad[4];
    const int tid = threadIdx.x, lane = tid % kWave, w = tid / kWave;
    for (int64_t unit = blockIdx.x; unit < n_units; unit += gridDim.x) {
        const int32_t cell_id = units[3 * unit];
        const int32_t xi = units[3 * unit + 1];
        const CellDev c = cells[cell_id];
        const int64_t base = g_pair_base[c.group];
        const int64_t n = g_n[c.group];
        const int nb = c.nb;
        int nb2 = 2;
        while (nb2 < nb) nb2 <<= 1;
        const int xl = c.x0 + xi;
        const float *row = p32 + base + int64_t(xl) * n;
        uint8_t *frow = flags ? flags + base + int64_t(xl) * n : nullptr;
        for (int j = tid; j < nb2; j += 256) {
            sv[j] = j < nb ? row[c.b0 + j] : __builtin_inff();
            si[j] = uint16_t(j);
        }
        __syncthreads();
        for (int k = 2; k <= nb2; k <<= 1)
            for (int jj = k >> 1; jj > 0; jj >>= 1) {
                for (int i = tid; i < nb2; i += 256) {
                    const int l = i ^ jj;
                    if (l > i) {
                        const bool up = (i & k) == 0;
                        const float vi = sv[i], vl = sv[l];
                        if ((vi > vl) == up) {
                            sv[i] = vl;
                            sv[l] = vi;
                            const uint16_t t = si[i];
                            si[i] = si[l];
                            si[l] = t;
                        }
                    }
                }
                __syncthreads();
            }
        // count, near ties, non-robust pairs
        unsigned long long cnt = 0;
        int dirty = 0, all_b = 0, all_a = 0;
        for (int a = tid; a < c.na; a += 256) {
            const int al = c.a0 + a;
            if (c.exclude_self && al == xl) continue;
            const float da = row[al];
            const int lb = count_below(sv, nb, da, false), ub = count_below(sv, nb, da, true);
            cnt += unsigned(2 * nb - lb - ub);
            if (frow) {
                const uint8_t fa = frow[al];
                if (fa & kNonRobust) {
                    dirty = all_b = 1;
                    frow[al] = fa | kMarked;
                }
                const int lo = count_below(sv, nb, da - margin, false);
                const int hi = count_below(sv, nb, da + margin, true);
                if (lo < hi) {
                    dirty = 1;
                    frow[al] = frow[al] | kMarked;
                    for (int k = lo; k < hi; ++k) {
                        const int bl = c.b0 + si[k];
                        frow[bl] = frow[bl] | kMarked;
                    }
                }
            }
        }
        if (frow)
            for (int b = tid; b < nb; b += 256)
                if (frow[c.b0 + b] & kNonRobust) {
                    dirty = all_a = 1;
                    frow[c.b0 + b] = frow[c.b0 + b] | kMarked;
                }
        const unsigned long long wsum = dev::wave_sum_u64(cnt);
        const int wflags = (dev::wave_any(dirty) ? 1 : 0) | (dev::wave_any(all_b) ? 2 : 0) |
                           (dev::wave_any(all_a) ? 4 : 0);
        if (lane == 0) {
            red[w] = wsum;
            bad[w] = wflags;
        }
        __syncthreads();
        const unsigned long long total = red[0] + red[1] + red[2] + red[3];
        const int f = bad[0] | bad[1] | bad[2] | bad[3];
        if (f & 2)  // a non-robust (x, a): every comparison it takes part in is a near tie
            for (int b = tid; b < nb; b += 256) frow[c.b0 + b] = frow[c.b0 + b] | kMarked;
        if (f & 4)  // a non-robust (x, b)
            for (int a = tid; a < c.na; a += 256) {
                const int al = c.a0 + a;
                if (!(c.exclude_self && al == xl)) frow[al] = frow[al] | kMarked;
            }
        if (tid == 0) {
            if (f & 1) {
                const unsigned int k = atomicAdd(recount_n, 1u);
                if (int64_t(k) < recount_cap) {
                    recount[2 * int64_t(k)] = cell_id;
                    recount[2 * int64_t(k) + 1] = xi;
                }
            } else if (total) {
                atomicAdd(&W[cell_id], total);
            }
        }
        __syncthreads();  // the next unit reuses the sort buffers and reductions
    }
}

// Zeroes the per-cell counts W [n_cells] and the score's 64 counter bytes
// that follow them, except the error item (the word at byte 8), which starts
// at all ones.
__global__ __launch_bounds__(256) void k_init(unsigned long long *__restrict__ W, int64_t n_cells) {
    const int64_t n = n_cells + 8;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
        W[i] = i == n_cells + 1 ? ~0ull : 0ull;
}

// Marked pairs into `list`.  Every pair the triplet kernels mark belongs to a
// row they also send to the recount, so with no such row there is nothing to
// collect.
__global__ __launch_bounds__(256) void k_collect_marked(const uint8_t *__restrict__ flags, int64_t n_slots,
                                                        int64_t *__restrict__ list,
                                                        unsigned int *__restrict__ count, int64_t cap,
                                                        const unsigned int *__restrict__ recount_n) {
    if (*recount_n == 0) return;
    const int lane = threadIdx.x % kWave;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
         i - lane < n_slots; i += int64_t(gridDim.x) * blockDim.x) {
        const bool m = i < n_slots && (flags[i] & kMarked);
        const unsigned long long ball = __ballot(m);
        if (!ball) continue;
        unsigned int base = 0;
        if (lane == 0) base = atomicAdd(count, unsigned(__popcll(ball)));
        base = __shfl(base, 0, kWave);
        if (m) {
            const unsigned int k = base + unsigned(__popcll(ball & ((1ull << lane) - 1ull)));
            if (int64_t(k) < cap) list[k] = i;
        }
    }
}

__global__ __launch_bounds__(256) void k_recount(const CellDev *__restrict__ cells,
                                                 const int32_t *__restrict__ rows,
                                                 const unsigned int *__restrict__ n_rows,
                                                 int64_t max_rows,
                                                 const int64_t *__restrict__ g_pair_base,
                                                 const int64_t *__restrict__ g_n,
                                                 const float *__restrict__ p32,
                                                 const double *__restrict__ p64,
                                                 const uint8_t *__restrict__ flags,
                                                 unsigned long long *__restrict__ W) {
    const int lane = threadIdx.x % kWave;
    const int64_t total = min(int64_t(*n_rows), max_rows);
    const int64_t n_waves = int64_t(gridDim.x) * 4;
    for (int64_t r = int64_t(blockIdx.x) * 4 + threadIdx.x / kWave; r < total; r += n_waves) {
        const int32_t cell_id = rows[2 * r], xi = rows[2 * r + 1];
        const CellDev c = cells[cell_id];
        const int64_t base = g_pair_base[c.group];
        const int64_t n = g_n[c.group];
        const int xl = c.x0 + xi;
        const int64_t roff = base + int64_t(xl) * n;
        const int nb = c.nb;
        const int step_a = kWave / nb, step_b = kWave % nb;
        int a = lane / nb, b = lane % nb;
        unsigned int cnt = 0;
        while (a < c.na) {
            const int al = c.a0 + a, bl = c.b0 + b;
            if (!(c.exclude_self && al == xl)) {
                // FP64 when both pairs were recomputed; otherwise this comparison was
                // already decided far from a tie in FP32 (gap > margin >= 2 x error)
                const bool both = (flags[roff + al] & kMarked) && (flags[roff + bl] & kMarked);
                const double da = both ? p64[roff + al] : double(p32[roff + al]);
                const double db = both ? p64[roff + bl] : double(p32[roff + bl]);
                cnt += da < db ? 2u : (da == db ? 1u : 0u);
            }
            a += step_a;
            b += step_b;
            if (b >= nb) { b -= nb; ++a; }
        }
        const unsigned long long row_total = dev::wave_sum_u64(cnt);
        if (lane == 0 && row_total) atomicAdd(&W[cell_id], row_total);
    }
}

}  // namespace

void triplets(hipStream_t s, const CellDev *cells, const int32_t *units, int64_t n_units,
              const GroupTables &g, const float *p32, unsigned long long *W, uint8_t *flags,
              float margin, int32_t *recount, unsigned int *recount_n, int64_t recount_cap,
              const unsigned int *scale) {
    if (n_units <= 0) return;
    hipLaunchKernelGGL(k_triplets, dim3(grid_for(n_units, 4)), dim3(256), 0, s, cells, units, n_units,
                       g.pair_base, g.n_items, p32, W, flags, margin, recount, recount_n,
                       recount_cap, scale);
    FABX_HIP(hipGetLastError());
}

void triplets_sorted(hipStream_t s, const CellDev *cells, const int32_t *units, int64_t n_units,
                     const GroupTables &g, const float *p32, unsigned long long *W, uint8_t *flags,
                     float margin, int32_t *recount, unsigned int *recount_n, int64_t recount_cap,
                     const unsigned int *scale) {
    if (n_units <= 0) return;
    hipLaunchKernelGGL(k_triplets_sorted, dim3(grid_for(n_units, 1)), dim3(256), 0, s, cells, units, n_units,
                       g.pair_base, g.n_items, p32, W, flags, margin, recount, recount_n, recount_cap, scale);
    FABX_HIP(hipGetLastError());
}

void init_score(hipStream_t s, unsigned long long *W, int64_t n_cells) {
    const int64_t blocks = std::min<int64_t>((n_cells + 8 + 255) / 256, 4096);
    hipLaunchKernelGGL(k_init, dim3(unsigned(blocks)), dim3(256), 0, s, W, n_cells);
    FABX_HIP(hipGetLastError());
}

void collect_marked(hipStream_t s, const uint8_t *flags, int64_t n_slots, int64_t *list,
                    unsigned int *count, int64_t cap, const unsigned int *recount_n) {
    if (n_slots <= 0) return;
    const int64_t blocks = std::min<int64_t>((n_slots + 255) / 256, 4096);
    hipLaunchKernelGGL(k_collect_marked, dim3(unsigned(blocks)), dim3(256), 0, s, flags, n_slots,
                       list, count, cap, recount_n);
    FABX_HIP(hipGetLastError());
}

void recount(hipStream_t s, const CellDev *cells, const int32_t *rows, const unsigned int *n_rows,
             int64_t max_rows, const GroupTables &g, const float *p32, const double *p64,
             const uint8_t *flags, unsigned long long *W) {
    if (max_rows <= 0) return;
    const int64_t blocks = std::min<int64_t>((max_rows + 3) / 4, 2048);
    hipLaunchKernelGGL(k_recount, dim3(unsigned(blocks)), dim3(256), 0, s, cells, rows, n_rows,
                       max_rows, g.pair_base, g.n_items, p32, p64, flags, W);
    FABX_HIP(hipGetLastError());
}

}  // namespace kern
}  // namespace fabx
