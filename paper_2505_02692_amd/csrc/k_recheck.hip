// FP64 recomputation of the item-pair distances whose triplet comparisons
// were too close to call in BF16 / FP32, or whose DTW path length was not
// robust.  Works from the raw features (F32 or BF16 widened exactly):
//   unit vector  u / ||u||, ||u|| = sqrt of the sequential sum of squares
//   cosine       sequential sum of products of the unit vectors
//   angle        acos(cos) when |cos| < 1 - 2^-20, else the half-chord form
//                2 atan2(||u - v||, ||u + v||), which stays accurate near 0 and pi
//   distance     angle / pi; DTW with the diagonal > left > up predecessor order
// Contraction into FMA is disabled so each sum is the plain sequential sum.
//
// Persistent grid: each 256-thread block takes listed pairs in turn.
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
    __shared__ double nrm[2 * kMaxL];
    __shared__ double dm[kMaxL * kMaxL];
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
        // norms of the N + M frames, one thread per frame
        for (int f = threadIdx.x; f < N + M; f += blockDim.x) {
            const T *row = f < N ? fx + int64_t(f) * dim : fy + int64_t(f - N) * dim;
            double s = 0.0;
            for (int k = 0; k < dim; ++k) {
                const double v = ld(row, k);
                s += v * v;
            }
            nrm[f] = sqrt(s);
        }
        __syncthreads();
        for (int cidx = threadIdx.x; cidx < N * M; cidx += blockDim.x) {
            const int i = cidx / M, j = cidx % M;
            const T *u = fx + int64_t(i) * dim;
            const T *v = fy + int64_t(j) * dim;
            const double nu = nrm[i], nv = nrm[N + j];
            double c = 0.0;
            for (int k = 0; k < dim; ++k) c += (ld(u, k) / nu) * (ld(v, k) / nv);
            double sm = 0.0, sp = 0.0;
            if (!(fabs(c) < 1.0 - 0x1p-20)) {
                for (int k = 0; k < dim; ++k) {
                    const double a = ld(u, k) / nu, b = ld(v, k) / nv;
                    sm += (a - b) * (a - b);
                    sp += (a + b) * (a + b);
                }
            }
            dm[cidx] = angle_over_pi_units(c, sm, sp);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            // in place: dm becomes the cumulative cost, lens kept in a local array per row
            int len_prev[kMaxL], len_cur[kMaxL];
            for (int j = 0; j < M; ++j) {
                if (j > 0) dm[j] = dm[j - 1] + dm[j];
                len_prev[j] = j + 1;
            }
            for (int i = 1; i < N; ++i) {
                double *cr = dm + i * M;
                const double *pr = dm + (i - 1) * M;
                cr[0] = pr[0] + cr[0];
                len_cur[0] = i + 1;
                for (int j = 1; j < M; ++j) {
                    const double dg = pr[j - 1], lf = cr[j - 1], up = pr[j];
                    double best;
                    int lb;
                    if (dg <= lf && dg <= up) { best = dg; lb = len_prev[j - 1]; }
                    else if (lf <= up) { best = lf; lb = len_cur[j - 1]; }
                    else { best = up; lb = len_prev[j]; }
                    cr[j] = cr[j] + best;
                    len_cur[j] = lb + 1;
                }
                for (int j = 0; j < M; ++j) len_prev[j] = len_cur[j];
            }
            const double cost = dm[N * M - 1];
            p64[slot] = norm == FABX_NORM_PATH ? cost / double(len_prev[M - 1]) : cost;
        }
        __syncthreads();
    }
}

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
        if (threadIdx.x == 0) {
            double sx = 0.0, sy = 0.0;
            for (int k = 0; k < dim; ++k) { sx += mx[k] * mx[k]; sy += my[k] * my[k]; }
            const double nx = sqrt(sx), ny = sqrt(sy);
            double c = 0.0;
            for (int k = 0; k < dim; ++k) c += (mx[k] / nx) * (my[k] / ny);
            double sm = 0.0, sp = 0.0;
            if (!(fabs(c) < 1.0 - 0x1p-20)) {
                for (int k = 0; k < dim; ++k) {
                    const double a = mx[k] / nx, b = my[k] / ny;
                    sm += (a - b) * (a - b);
                    sp += (a + b) * (a + b);
                }
            }
            p64[slot] = angle_over_pi_units(c, sm, sp);
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
