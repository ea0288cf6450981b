// Triplet comparison and per-cell reduction (cell discriminability formula of
// the Background section), in integer half units: each triple adds
// 2 [d(x,a) < d(x,b)] + [d(x,a) == d(x,b)].
//
// Work unit = (cell, range of x).  A wave walks the flattened |A| x |B| grid
// of one x with one (a, b) per lane, so short B sets still fill the wave;
// both distances come from the row of x in the group's pair matrix (the row
// is a few hundred bytes and stays in L1/L2).  Counts are reduced in the wave
// and added once per unit with a 64-bit atomic, so the result does not depend
// on scheduling.
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
                                                  int64_t recount_cap) {
    const int lane = threadIdx.x % kWave;
    // one wave per unit; the loop bound is uniform across the wave
    for (int64_t unit = int64_t(blockIdx.x) * 4 + threadIdx.x / kWave; unit < n_units;
         unit += int64_t(gridDim.x) * 4) {
    const int32_t cell_id = units[3 * unit];
    const int32_t xb = units[3 * unit + 1], xe = units[3 * unit + 2];
    const CellDev c = cells[cell_id];
    const int64_t base = g_pair_base[c.group];
    const int64_t n = g_n[c.group];
    const int nb = c.nb;
    const int step_a = kWave / nb, step_b = kWave % nb;
    unsigned long long acc = 0;
    for (int xi = xb; xi < xe; ++xi) {
        const int xl = c.x0 + xi;
        const float *row = p32 + base + int64_t(xl) * n;
        uint8_t *frow = flags ? flags + base + int64_t(xl) * n : nullptr;
        int a = lane / nb, b = lane % nb;
        unsigned int cnt = 0;
        int dirty = 0;
        while (a < c.na) {
            const int al = c.a0 + a, bl = c.b0 + b;
            if (!(c.exclude_self && al == xl)) {
                const float da = row[al], db = row[bl];
                cnt += da < db ? 2u : (da == db ? 1u : 0u);
                if (frow) {
                    const uint8_t fa = frow[al], fb = frow[bl];
                    if (fabsf(da - db) <= margin || ((fa | fb) & kNonRobust)) {
                        dirty = 1;
                        if (!(fa & kMarked)) frow[al] = fa | kMarked;
                        if (!(fb & kMarked)) frow[bl] = fb | kMarked;
                    }
                }
            }
            a += step_a;
            b += step_b;
            if (b >= nb) { b -= nb; ++a; }
        }
        const unsigned long long row_total = dev::wave_sum_u64(cnt);
        if (flags && dev::wave_any(dirty)) {
            if (lane == 0) {
                const unsigned int k = atomicAdd(recount_n, 1u);
                if (int64_t(k) < recount_cap) {
                    recount[2 * int64_t(k)] = cell_id;
                    recount[2 * int64_t(k) + 1] = xi;
                }
            }
            continue;
        }
        acc += row_total;
    }
    if (lane == 0 && acc) atomicAdd(&W[cell_id], acc);
    }
}

__global__ __launch_bounds__(256) void k_collect_marked(const uint8_t *__restrict__ flags, int64_t n_slots,
                                                        int64_t *__restrict__ list,
                                                        unsigned int *__restrict__ count, int64_t cap) {
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
              float margin, int32_t *recount, unsigned int *recount_n, int64_t recount_cap) {
    if (n_units <= 0) return;
    hipLaunchKernelGGL(k_triplets, dim3(grid_for(n_units, 4)), dim3(256), 0, s, cells, units, n_units,
                       g.pair_base, g.n_items, p32, W, flags, margin, recount, recount_n,
                       recount_cap);
    FABX_HIP(hipGetLastError());
}

void collect_marked(hipStream_t s, const uint8_t *flags, int64_t n_slots, int64_t *list,
                    unsigned int *count, int64_t cap) {
    if (n_slots <= 0) return;
    const int64_t blocks = std::min<int64_t>((n_slots + 255) / 256, 4096);
    hipLaunchKernelGGL(k_collect_marked, dim3(unsigned(blocks)), dim3(256), 0, s, flags, n_slots,
                       list, count, cap);
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
