// FP64 recomputation of the item-pair distances whose triplet comparisons
// were too close to call in BF16 / FP32, or whose DTW path length was not
// robust.  Works from the raw features (F32 or BF16 widened exactly):
//   unit vector  u times 1 / ||u||, ||u|| = sqrt of the sum of squares
//   cosine       sum of products of the unit vectors
//   angle        acos(cos) when |cos| < 1 - 2^-20, else the half-chord form
//                2 atan2(||u - v||, ||u + v||), which stays accurate near 0 and pi
//   distance     angle / pi; DTW with the diagonal > left > up predecessor order
// Contraction into FMA is disabled.
//
// Persistent grid: each 256-thread block takes listed pairs in turn.  The
// sums run over the lanes of a wave and end in one butterfly; they differ
// from the strictly sequential sums of the definition only in rounding
// (about 1e-16 relative), and every pair goes through the same arithmetic, so
// equal inputs (exact copies) still give equal distances.
#include "device_common.h"
#include "kernels.h"

#pragma clang fp contract(off)

namespace fabx {
namespace kern {
namespace {

constexpr int kMaxL = FABX_MAX_ITEM_FRAMES;
constexpr double kPi = 3.14159265358979323846;

template <typename T>
__device__ __forceinline__ double ld(const T *p, int64_t i);
template <>
__device__ __forceinline__ double ld<float>(const float *p, int64_t i) { return double(p[i]); }
template <>
__device__ __forceinline__ double ld<uint16_t>(const uint16_t *p, int64_t i) {
    return double(__uint_as_float(uint32_t(p[i]) << 16));
}

__device__ double angle_over_pi_units(double c, double sm, double sp) {
    const double th = fabs(c) < 1.0 - 0x1p-20 ? acos(c) : 2.0 * atan2(sqrt(sm), sqrt(sp));
    return th / kPi;
}

// Sum of a double over the wave (butterfly; every lane gets the sum).
__device__ __forceinline__ double wave_sum_f64(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, dev::kWave);
    return v;
}

// One 256-thread block per listed pair: the four waves share the N + M frame
// norms and then the N x M frame distances (a wave per frame pair at a time,
// its 64 lanes splitting the feature dimension, one butterfly sum each), held
// in LDS; then one wave runs the DTW over anti-diagonals (lane = row i), with
// the diagonal > left > up predecessor order on exact ties.
template <typename T>
__global__ __launch_bounds__(256) void k_recheck_dtw(const T *__restrict__ feat, int dim,
                                                     const int64_t *__restrict__ g_item0,
                                                     const int64_t *__restrict__ g_n,
                                                     const int64_t *__restrict__ g_pair_base,
                                                     int64_t n_groups,
                                                     const int64_t *__restrict__ item_src,
                                                     const int32_t *__restrict__ item_len,
                                                     const int64_t *__restrict__ list,
                                                     const unsigned int *__restrict__ count,
                                                     int64_t max_count, int norm,
                                                     double *__restrict__ p64) {
    __shared__ double inrm[2 * kMaxL];     // 1 / ||frame|| of the N rows, then the M columns
    __shared__ double dm[kMaxL * kMaxL];   // frame distances, row-major [N][M]
    const int lane = threadIdx.x % dev::kWave, w = threadIdx.x / dev::kWave;
    const int64_t total = min(int64_t(*count), max_count);
    for (int64_t e = blockIdx.x; e < total; e += gridDim.x) {
        const int64_t slot = list[e];
        const int64_t g = dev::find_segment(g_pair_base, n_groups, slot);
        const int64_t n = g_n[g];
        const int64_t local = slot - g_pair_base[g];
        const int64_t x = g_item0[g] + local / n, y = g_item0[g] + local % n;
        const int N = item_len[x], M = item_len[y];
        const T *fx = feat + item_src[x] * int64_t(dim);
        const T *fy = feat + item_src[y] * int64_t(dim);
        auto frame = [&](int f) { return f < N ? fx + int64_t(f) * dim : fy + int64_t(f - N) * dim; };
        // norms of the N + M frames, a wave per frame
        for (int f = w; f < N + M; f += 4) {
            const T *row = frame(f);
            double s = 0.0;
            for (int k = lane; k < dim; k += dev::kWave) {
                const double v = ld(row, k);
                s += v * v;
            }
            s = wave_sum_f64(s);
            if (lane == 0) inrm[f] = 1.0 / sqrt(s);
        }
        __syncthreads();
        // frame distances, a wave per (i, j)
        for (int cidx = w; cidx < N * M; cidx += 4) {
            const int i = cidx / M, j = cidx % M;
            const T *u = fx + int64_t(i) * dim;
            const T *v = fy + int64_t(j) * dim;
            const double su = inrm[i], sv = inrm[N + j];
            double c = 0.0;
            for (int k = lane; k < dim; k += dev::kWave) c += (ld(u, k) * su) * (ld(v, k) * sv);
            c = wave_sum_f64(c);
            double sm = 0.0, sp = 0.0;
            if (!(fabs(c) < 1.0 - 0x1p-20)) {   // wave-uniform: c is the same in every lane
                for (int k = lane; k < dim; k += dev::kWave) {
                    const double a = ld(u, k) * su, b = ld(v, k) * sv;
                    sm += (a - b) * (a - b);
                    sp += (a + b) * (a + b);
                }
                sm = wave_sum_f64(sm);
                sp = wave_sum_f64(sp);
            }
            if (lane == 0) dm[cidx] = angle_over_pi_units(c, sm, sp);
        }
        __syncthreads();
        if (w == 0) {
            // lane i is on column t - i at step t: c[i-1][j] comes from lane i - 1
            // one step earlier, c[i-1][j-1] two steps earlier
            const int i = lane;
            double c = 0.0, up_prev = 0.0;
            int len = 0, lup_prev = 0;
            for (int t = 0; t < N + M - 1; ++t) {
                const int j = t - i;
                const double up = __shfl_up(c, 1, dev::kWave);   // lane i - 1's cost, step t - 1
                const int lup = __shfl_up(len, 1, dev::kWave);
                const double diag = up_prev, left = c;
                const int ldiag = lup_prev, lleft = len;
                up_prev = up;
                lup_prev = lup;
                if (i < N && j >= 0 && j < M) {
                    const double d = dm[i * M + j];
                    if (i == 0 && j == 0) {
                        c = d;
                        len = 1;
                    } else if (i == 0) {
                        c = left + d;
                        len = lleft + 1;
                    } else if (j == 0) {
                        c = up + d;
                        len = lup + 1;
                    } else if (diag <= left && diag <= up) {
                        c = diag + d;
                        len = ldiag + 1;
                    } else if (left <= up) {
                        c = left + d;
                        len = lleft + 1;
                    } else {
                        c = up + d;
                        len = lup + 1;
                    }
                }
            }
            if (i == N - 1) p64[slot] = norm == FABX_NORM_PATH ? c / double(len) : c;
        }
        __syncthreads();
    }
}

// One block per listed pair: the two items' mean frames (threads over the
// feature dimension), then wave 0 takes their norms, cosine and, near +-1,
// the half-chord sums, its lanes splitting the dimension.
template <typename T>
__global__ __launch_bounds__(256) void k_recheck_pooled(const T *__restrict__ feat, int dim,
                                                        const int64_t *__restrict__ g_item0,
                                                        const int64_t *__restrict__ g_n,
                                                        const int64_t *__restrict__ g_pair_base,
                                                        int64_t n_groups,
                                                        const int64_t *__restrict__ item_src,
                                                        const int32_t *__restrict__ item_len,
                                                        const int64_t *__restrict__ list,
                                                        const unsigned int *__restrict__ count,
                                                        int64_t max_count, double *__restrict__ p64) {
    __shared__ double mx[2048];
    __shared__ double my[2048];
    const int lane = threadIdx.x % dev::kWave;
    const int64_t total = min(int64_t(*count), max_count);
    for (int64_t e = blockIdx.x; e < total; e += gridDim.x) {
        const int64_t slot = list[e];
        const int64_t g = dev::find_segment(g_pair_base, n_groups, slot);
        const int64_t n = g_n[g];
        const int64_t local = slot - g_pair_base[g];
        const int64_t x = g_item0[g] + local / n, y = g_item0[g] + local % n;
        const int N = item_len[x], M = item_len[y];
        const T *fx = feat + item_src[x] * int64_t(dim);
        const T *fy = feat + item_src[y] * int64_t(dim);
        for (int k = threadIdx.x; k < dim; k += blockDim.x) {
            double sx = 0.0, sy = 0.0;
            for (int t = 0; t < N; ++t) sx += ld(fx, int64_t(t) * dim + k);
            for (int t = 0; t < M; ++t) sy += ld(fy, int64_t(t) * dim + k);
            mx[k] = sx / double(N);
            my[k] = sy / double(M);
        }
        __syncthreads();
        if (threadIdx.x < dev::kWave) {
            double sx = 0.0, sy = 0.0;
            for (int k = lane; k < dim; k += dev::kWave) {
                sx += mx[k] * mx[k];
                sy += my[k] * my[k];
            }
            const double ix = 1.0 / sqrt(wave_sum_f64(sx)), iy = 1.0 / sqrt(wave_sum_f64(sy));
            double c = 0.0;
            for (int k = lane; k < dim; k += dev::kWave) c += (mx[k] * ix) * (my[k] * iy);
            c = wave_sum_f64(c);
            double sm = 0.0, sp = 0.0;
            if (!(fabs(c) < 1.0 - 0x1p-20)) {
                for (int k = lane; k < dim; k += dev::kWave) {
                    const double a = mx[k] * ix, b = my[k] * iy;
                    sm += (a - b) * (a - b);
                    sp += (a + b) * (a + b);
                }
                sm = wave_sum_f64(sm);
                sp = wave_sum_f64(sp);
            }
            if (lane == 0) p64[slot] = angle_over_pi_units(c, sm, sp);
        }
        __syncthreads();
    }
}

}  // namespace

void recheck_fp64(hipStream_t s, const void *features, int dtype, int dim, const GroupTables &g,
                  const ItemTables &it, const int64_t *list, const unsigned int *count,
                  int64_t max_count, int mode, int norm, double *p64) {
    if (max_count <= 0) return;
    if (mode == FABX_MODE_POOLED && dim > 2048) fail(FABX_EINVAL, "pooled recheck supports dim <= 2048");
    const unsigned blocks = unsigned(std::min<int64_t>(max_count, 4096));
    if (mode == FABX_MODE_DTW) {
        if (dtype == FABX_DTYPE_F32)
            hipLaunchKernelGGL(k_recheck_dtw<float>, dim3(blocks), dim3(256), 0, s,
                               static_cast<const float *>(features), dim, g.item0, g.n_items,
                               g.pair_base, g.n_groups, it.src, it.len, list, count, max_count, norm,
                               p64);
        else
            hipLaunchKernelGGL(k_recheck_dtw<uint16_t>, dim3(blocks), dim3(256), 0, s,
                               static_cast<const uint16_t *>(features), dim, g.item0, g.n_items,
                               g.pair_base, g.n_groups, it.src, it.len, list, count, max_count, norm,
                               p64);
    } else {
        if (dtype == FABX_DTYPE_F32)
            hipLaunchKernelGGL(k_recheck_pooled<float>, dim3(blocks), dim3(256), 0, s,
                               static_cast<const float *>(features), dim, g.item0, g.n_items,
                               g.pair_base, g.n_groups, it.src, it.len, list, count, max_count, p64);
        else
            hipLaunchKernelGGL(k_recheck_pooled<uint16_t>, dim3(blocks), dim3(256), 0, s,
                               static_cast<const uint16_t *>(features), dim, g.item0, g.n_items,
                               g.pair_base, g.n_groups, it.src, it.len, list, count, max_count, p64);
    }
    FABX_HIP(hipGetLastError());
}

}  // namespace kern
}  // namespace fabx
