// FP64 recomputation of the item-pair distances whose triplet comparisons
// were too close to call in BF16 / FP32, or whose DTW path length was not
// robust.  Works from the raw features (F32 or BF16 widened exactly):
//   unit vector  u times 1 / ||u||, ||u|| = sqrt of the sum of squares
//   cosine       sum of products of the unit vectors
//   angle        acos(cos) when |cos| < 1 - 2^-20, else the half-chord form
//                2 atan2(||u - v||, ||u + v||), which stays accurate near 0 and pi
//   distance     angle / pi; DTW with the diagonal > left > up predecessor order
// or, for the Euclidean distance (euclid != 0), the square root of the sum of
// squared differences of the raw frames (or means).
// Contraction into FMA is disabled.
//
// Persistent grid: each 256-thread block takes listed pairs in turn.  The
// frame norms and most frame products are sums over the lanes of a wave
// ending in one butterfly; the frame products of k_recheck_dtw for pairs of
// more than 256 frame pairs are sequential sums per frame pair.  Either
// differs from the strictly sequential sums of the definition only in
// rounding (about 1e-16 relative), and every pair of a kernel goes through
// the same arithmetic (exact copies have equal lengths, so they meet in the
// same kernel), so equal inputs still give equal distances.
#include "device_common.h"
#include "kernels.h"

#pragma clang fp contract(off)

namespace fabx {
namespace kern {
namespace {

constexpr int kMaxL = 64;                    // items of at most this many frames: k_recheck_dtw
constexpr int kLongMax = FABX_MAX_ITEM_FRAMES;  // longer ones (up to this): k_long_dtw
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

// The per-lane loops over the features below are unrolled so that the loads
// of several features are in flight at once; each lane still adds its terms
// in feature order.

// Sum of a double over the wave (butterfly; every lane gets the sum).
__device__ __forceinline__ double wave_sum_f64(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, dev::kWave);
    return v;
}

// 1 / ||frame|| (the whole wave; every lane gets it).
template <typename T>
__device__ __forceinline__ double wave_inv_norm(const T *row, int dim, int lane) {
    double s = 0.0;
#pragma unroll 4
    for (int k = lane; k < dim; k += dev::kWave) {
        const double v = ld(row, k);
        s += v * v;
    }
    return 1.0 / sqrt(wave_sum_f64(s));
}

// Angular distance of frames u and v with inverse norms su and sv (the whole
// wave, its lanes splitting the dimension; every lane gets it).
template <typename T>
__device__ __forceinline__ double wave_frame_distance(const T *u, const T *v, double su, double sv, int dim,
                                                      int lane) {
    double c = 0.0;
#pragma unroll 4
    for (int k = lane; k < dim; k += dev::kWave) c += (ld(u, k) * su) * (ld(v, k) * sv);
    c = wave_sum_f64(c);
    double sm = 0.0, sp = 0.0;
    if (!(fabs(c) < 1.0 - 0x1p-20)) {   // wave-uniform: c is the same in every lane
#pragma unroll 4
        for (int k = lane; k < dim; k += dev::kWave) {
            const double a = ld(u, k) * su, b = ld(v, k) * sv;
            sm += (a - b) * (a - b);
            sp += (a + b) * (a + b);
        }
        sm = wave_sum_f64(sm);
        sp = wave_sum_f64(sp);
    }
    return angle_over_pi_units(c, sm, sp);
}

// Euclidean distance of frames u and v (the whole wave; every lane gets it).
template <typename T>
__device__ __forceinline__ double wave_euclid_distance(const T *u, const T *v, int dim, int lane) {
    double s = 0.0;
#pragma unroll 4
    for (int k = lane; k < dim; k += dev::kWave) {
        const double a = ld(u, k) - ld(v, k);
        s += a * a;
    }
    return sqrt(wave_sum_f64(s));
}

// The DTW update of cell (i, j) from its neighbours' costs and path lengths,
// with the first row and column accumulating along themselves and the
// diagonal > left > up order on exact ties.
__device__ __forceinline__ void dtw_update(int i, int j, double d, double diag, int ldiag, double left,
                                           int lleft, double up, int lup, double &c, int &len) {
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

// LDS staging of k_recheck_dtw's frame products: room for 132 rows (N + M
// frames and the tiles' overreach of up to 3 rows) of 32 features (+1 pad);
// fewer rows take longer feature chunks
constexpr int kRstage = (2 * kMaxL + 4) * 33;
constexpr int kRper = 8;  // staging loads a thread has in flight at once

// One 256-thread block per listed pair of items of at most kMaxL frames (the
// others are left to k_long_dtw).  The four waves share the N + M frame norms
// (a wave per frame, its lanes splitting the dimension).  The N x M frame
// products are then a register-tiled FP64 product: the frames go through LDS
// in chunks of features (as many as kRstage holds for N + M + 3 rows; each
// thread issues kRper loads before their stores), as unit-vector
// components (or raw values for the Euclidean distance), and a thread
// accumulates T x T frame pairs, each a sequential sum over the features in
// order, so every pair gets the same arithmetic whatever its tile: T = 2
// (thread t on (2 (t / 16) + r, 2 (t % 16) + c)) when both items have at most
// 32 frames, else T = 4.  Pairs of at most kSmallPairs frame pairs go to the
// kTiled = false instantiation instead, whose small footprint keeps more
// blocks per CU: there a wave takes a frame pair at a time, its lanes
// splitting the features (one butterfly sum).  The class depends on N * M
// only, so both orientations of a pair, and copies, share the arithmetic;
// each instantiation skips the other's pairs.  A frame pair whose cosine is within 2^-20 of +-1 is
// finished by a wave (lanes splitting the dimension) with the half-chord
// sums.  The distances stay in LDS; one wave then runs the DTW over
// anti-diagonals (lane = row i), with the diagonal > left > up predecessor
// order on exact ties.
constexpr int kSmallPairs = 256;  // pairs of at most this many frame pairs: a wave per frame pair

template <typename T, bool kTiled>
__global__ __launch_bounds__(256) void k_recheck_dtw(const T *__restrict__ feat, int dim,
                                                     const int64_t *__restrict__ g_item0,
                                                     const int64_t *__restrict__ g_n,
                                                     const int64_t *__restrict__ g_pair_base,
                                                     int64_t n_groups,
                                                     const int64_t *__restrict__ item_src,
                                                     const int32_t *__restrict__ item_len,
                                                     const int64_t *__restrict__ list,
                                                     const unsigned int *__restrict__ count,
                                                     int64_t max_count, int norm, int euclid,
                                                     double *__restrict__ p64) {
    constexpr int kDm = kTiled ? kMaxL * kMaxL : kSmallPairs;  // room for N * M distances
    __shared__ double inrm[2 * kMaxL];     // 1 / ||frame|| of the N rows, then the M columns
    __shared__ double dm[kDm];             // frame distances, row-major [N][M]
    __shared__ double st[kTiled ? kRstage : 1];  // a feature chunk of the N + M frames
    __shared__ uint8_t near[kDm];                // cosine within 2^-20 of +-1
    const int lane = threadIdx.x % dev::kWave, w = threadIdx.x / dev::kWave;
    const int ti = threadIdx.x / 16, tj = threadIdx.x % 16;  // this thread's tile of frame pairs
    const int64_t total = min(int64_t(*count), max_count);
    for (int64_t e = blockIdx.x; e < total; e += gridDim.x) {
        const int64_t slot = list[e];
        const int64_t g = dev::find_segment_wave(g_pair_base, n_groups, slot);
        const int64_t n = g_n[g];
        const int64_t local = slot - g_pair_base[g];
        const int64_t x = g_item0[g] + local / n, y = g_item0[g] + local % n;
        const int N = item_len[x], M = item_len[y];
        if (N > kMaxL || M > kMaxL || (N * M <= kSmallPairs) == kTiled) continue;  // block-uniform
        const T *fx = feat + item_src[x] * int64_t(dim);
        const T *fy = feat + item_src[y] * int64_t(dim);
        auto frame = [&](int f) { return f < N ? fx + int64_t(f) * dim : fy + int64_t(f - N) * dim; };
        // norms of the N + M frames, a wave per frame (angular distance)
        if (!euclid)
            for (int f = w; f < N + M; f += 4) {
                const double r = wave_inv_norm(frame(f), dim, lane);
                if (lane == 0) inrm[f] = r;
            }
        __syncthreads();
        // frame products.  Rows of st: 0..N-1 the x frames, N..N+M-1 the y
        // frames; a tile reaching past them (i >= N or j >= M) reads at most 3
        // rows further (inside st, whatever they hold) and its sums are dropped.
        const int kc = min(dim, kRstage / (N + M + 3) - 1);  // features per chunk
        const int pad = kc + 1;
        auto products = [&](auto tile_tag) {
            constexpr int kT = decltype(tile_tag)::value;
            const int i0 = kT * ti, j0 = kT * tj;
            const bool active = i0 < N && j0 < M;
            double acc[kT][kT];
#pragma unroll
            for (int r = 0; r < kT; ++r)
#pragma unroll
                for (int c = 0; c < kT; ++c) acc[r][c] = 0.0;
            for (int k0 = 0; k0 < dim; k0 += kc) {
                const int kn = min(kc, dim - k0);
                // kRper loads in flight per thread before their stores
                const int nq = (N + M) * kc;
                for (int q0 = 0; q0 < nq; q0 += 256 * kRper) {
                    double v[kRper];
#pragma unroll
                    for (int u = 0; u < kRper; ++u) {
                        const int q = q0 + threadIdx.x + 256 * u, f = q / kc, kk = q - f * kc;
                        v[u] = q < nq && kk < kn ? ld(frame(f), k0 + kk) : 0.0;
                    }
#pragma unroll
                    for (int u = 0; u < kRper; ++u) {
                        const int q = q0 + threadIdx.x + 256 * u, f = q / kc, kk = q - f * kc;
                        if (q < nq) st[f * pad + kk] = euclid ? v[u] : v[u] * inrm[f];
                    }
                }
                __syncthreads();
                if (active) {
                    const double *sa = st + i0 * pad;
                    const double *sb = st + (N + j0) * pad;
                    for (int kk = 0; kk < kn; ++kk) {
                        double a[kT], b[kT];
#pragma unroll
                        for (int r = 0; r < kT; ++r) a[r] = sa[r * pad + kk];
#pragma unroll
                        for (int c = 0; c < kT; ++c) b[c] = sb[c * pad + kk];
#pragma unroll
                        for (int r = 0; r < kT; ++r)
#pragma unroll
                            for (int c = 0; c < kT; ++c) {
                                if (euclid) {
                                    const double d = a[r] - b[c];
                                    acc[r][c] = acc[r][c] + d * d;
                                } else {
                                    acc[r][c] = acc[r][c] + a[r] * b[c];
                                }
                            }
                    }
                }
                __syncthreads();
            }
            if (active) {
#pragma unroll
                for (int r = 0; r < kT; ++r)
#pragma unroll
                    for (int c = 0; c < kT; ++c) {
                        const int i = i0 + r, j = j0 + c;
                        if (i < N && j < M) {
                            const double v = acc[r][c];
                            if (euclid) {
                                dm[i * M + j] = sqrt(v);
                                near[i * M + j] = 0;
                            } else {
                                const bool nr = !(fabs(v) < 1.0 - 0x1p-20);
                                dm[i * M + j] = nr ? 0.0 : acos(v) / kPi;
                                near[i * M + j] = nr ? 1 : 0;
                            }
                        }
                    }
            }
        };
        if constexpr (!kTiled) {
            // few frame pairs: a wave per pair, its lanes splitting the features
            // (one butterfly sum), which keeps the lanes busy where tiles would not
            for (int cidx = w; cidx < N * M; cidx += 4) {
                const int i = cidx / M, j = cidx % M;
                const T *u = fx + int64_t(i) * dim, *v = fy + int64_t(j) * dim;
                const double d = euclid ? wave_euclid_distance(u, v, dim, lane)
                                        : wave_frame_distance(u, v, inrm[i], inrm[N + j], dim, lane);
                if (lane == 0) {
                    dm[cidx] = d;
                    near[cidx] = 0;
                }
            }
        } else if (N <= 32 && M <= 32) {
            products(std::integral_constant<int, 2>{});
        } else {
            products(std::integral_constant<int, 4>{});
        }
        __syncthreads();
        // near-parallel pairs: the half-chord form, a wave per pair
        if (!euclid)
            for (int cidx = w; cidx < N * M; cidx += 4) {
                if (!near[cidx]) continue;  // wave-uniform
                const int i = cidx / M, j = cidx % M;
                const double d = wave_frame_distance(fx + int64_t(i) * dim, fy + int64_t(j) * dim, inrm[i],
                                                     inrm[N + j], dim, lane);
                if (lane == 0) dm[cidx] = d;
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
                if (i < N && j >= 0 && j < M)
                    dtw_update(i, j, dm[i * M + j], diag, ldiag, left, lleft, up, lup, c, len);
            }
            if (i == N - 1) p64[slot] = norm == FABX_NORM_PATH ? c / double(len) : c;
        }
        __syncthreads();
    }
}

// One 256-thread block per listed pair in which an item has more than kMaxL
// frames (pairs of shorter items are skipped): the same arithmetic as
// k_recheck_dtw, tiled.  Rows go in chunks of 64 (lane = row), each chunk
// sweeping all M columns along anti-diagonals; a chunk hands its last row's
// costs and path lengths to the next one through LDS (`rowc`, `rowl`).  The
// frame distances of a chunk are made 32 columns at a time by the four waves
// into a ring of three 32-column tiles: at step s lane i reads column s - i,
// so the steps of tile k (s in [32k, 32k + 32)) read tiles k - 2 .. k only,
// and tile k + 1 may overwrite tile k - 2 once those steps are done.
// The result of pair `slot` goes to p64, and also to p32 and flags (0: robust,
// unmarked) when they are given (the first computation of such a pair).
template <typename T>
__global__ __launch_bounds__(256) void k_long_dtw(const T *__restrict__ feat, int dim,
                                                  const int64_t *__restrict__ g_item0,
                                                  const int64_t *__restrict__ g_n,
                                                  const int64_t *__restrict__ g_pair_base,
                                                  int64_t n_groups,
                                                  const int64_t *__restrict__ item_src,
                                                  const int32_t *__restrict__ item_len,
                                                  const int64_t *__restrict__ list,
                                                  const unsigned int *__restrict__ count,
                                                  int64_t max_count, int norm, int euclid,
                                                  double *__restrict__ p64, float *__restrict__ p32,
                                                  uint8_t *__restrict__ flags) {
    constexpr int kTc = 32, kRing = 3, kRingCols = kRing * kTc;
    __shared__ double dm[dev::kWave * kRingCols];  // [row of chunk][ring column]
    __shared__ double rinv_r[dev::kWave], rinv_c[kTc];
    __shared__ double rowc[kLongMax];              // previous chunk's last row: costs
    __shared__ int rowl[kLongMax];                 // and path lengths
    const int lane = threadIdx.x % dev::kWave, w = threadIdx.x / dev::kWave;
    const int64_t total = count ? min(int64_t(*count), max_count) : max_count;
    for (int64_t e = blockIdx.x; e < total; e += gridDim.x) {
        const int64_t slot = list[e];
        const int64_t g = dev::find_segment_wave(g_pair_base, n_groups, slot);
        const int64_t n = g_n[g];
        const int64_t local = slot - g_pair_base[g];
        const int64_t x = g_item0[g] + local / n, y = g_item0[g] + local % n;
        const int N = item_len[x], M = item_len[y];
        if (N <= kMaxL && M <= kMaxL) continue;  // block-uniform: k_recheck_dtw's pairs
        const T *fx = feat + item_src[x] * int64_t(dim);
        const T *fy = feat + item_src[y] * int64_t(dim);
        const int n_tiles = (M + kTc - 1) / kTc;
        double c = 0.0;
        int len = 0;
        for (int r0 = 0; r0 < N; r0 += dev::kWave) {
            const int nr = min(dev::kWave, N - r0);
            __syncthreads();  // the previous chunk's steps are done with the norms and the ring
            if (!euclid)
                for (int f = w; f < nr; f += 4) {
                    const double r = wave_inv_norm(fx + int64_t(r0 + f) * dim, dim, lane);
                    if (lane == 0) rinv_r[f] = r;
                }
            // wave 0's sweep state: lane i holds row r0 + i at column s - i
            const int i = lane;
            double up_prev = 0.0;
            int lup_prev = 0;
            c = 0.0;
            len = 0;
            int s = 0;
            const int steps = M + nr - 1;
            for (int k = 0; k < n_tiles; ++k) {
                const int c0 = k * kTc, nc = min(kTc, M - c0);
                const int ring0 = (k % kRing) * kTc;
                __syncthreads();  // tile k - 2's steps are done (and the row norms are in)
                if (!euclid)
                    for (int f = w; f < nc; f += 4) {
                        const double r = wave_inv_norm(fy + int64_t(c0 + f) * dim, dim, lane);
                        if (lane == 0) rinv_c[f] = r;
                    }
                __syncthreads();
                for (int cidx = w; cidx < nr * nc; cidx += 4) {
                    const int ii = cidx / nc, jj = cidx % nc;
                    const T *u = fx + int64_t(r0 + ii) * dim, *v = fy + int64_t(c0 + jj) * dim;
                    const double d = euclid ? wave_euclid_distance(u, v, dim, lane)
                                            : wave_frame_distance(u, v, rinv_r[ii], rinv_c[jj], dim, lane);
                    if (lane == 0) dm[ii * kRingCols + ring0 + jj] = d;
                }
                __syncthreads();
                if (w == 0) {
                    const int s_end = k == n_tiles - 1 ? steps : c0 + kTc;
                    for (; s < s_end; ++s) {
                        const int j = s - i;
                        double up = __shfl_up(c, 1, dev::kWave);   // lane i - 1's cost, step s - 1
                        int lup = __shfl_up(len, 1, dev::kWave);
                        if (i == 0) {  // the row above the chunk, read before this step's store
                            const bool in = r0 > 0 && j >= 0 && j < M;
                            up = in ? rowc[j] : 0.0;
                            lup = in ? rowl[j] : 0;
                        }
                        const double diag = up_prev, left = c;
                        const int ldiag = lup_prev, lleft = len;
                        up_prev = up;
                        lup_prev = lup;
                        if (i < nr && j >= 0 && j < M) {
                            const double d = dm[i * kRingCols + ((j / kTc) % kRing) * kTc + j % kTc];
                            dtw_update(r0 + i, j, d, diag, ldiag, left, lleft, up, lup, c, len);
                            if (i == nr - 1) {  // this chunk's last row, for the next chunk
                                rowc[j] = c;
                                rowl[j] = len;
                            }
                        }
                    }
                }
            }
        }
        // lane (N - 1) % 64 of wave 0 ended on cell (N - 1, M - 1)
        if (w == 0 && lane == (N - 1) % dev::kWave) {
            const double v = norm == FABX_NORM_PATH ? c / double(len) : c;
            p64[slot] = v;
            if (p32) p32[slot] = float(v);
            if (flags) flags[slot] = 0;
        }
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
                                                        int64_t max_count, int euclid,
                                                        double *__restrict__ p64) {
    __shared__ double mx[2048];
    __shared__ double my[2048];
    const int lane = threadIdx.x % dev::kWave;
    const int64_t total = min(int64_t(*count), max_count);
    for (int64_t e = blockIdx.x; e < total; e += gridDim.x) {
        const int64_t slot = list[e];
        const int64_t g = dev::find_segment_wave(g_pair_base, n_groups, slot);
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
        if (threadIdx.x < dev::kWave && euclid) {
            double sd = 0.0;
            for (int k = lane; k < dim; k += dev::kWave) sd += (mx[k] - my[k]) * (mx[k] - my[k]);
            sd = wave_sum_f64(sd);
            if (lane == 0) p64[slot] = sqrt(sd);
        } else if (threadIdx.x < dev::kWave) {
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

void long_dtw(hipStream_t s, const void *features, int dtype, int dim, const GroupTables &g,
              const ItemTables &it, const int64_t *list, const unsigned int *count, int64_t max_count, int norm,
              int euclid, double *p64, float *p32, uint8_t *flags) {
    if (max_count <= 0) return;
    const unsigned blocks = unsigned(std::min<int64_t>(max_count, 4096));
    if (dtype == FABX_DTYPE_F32)
        hipLaunchKernelGGL(k_long_dtw<float>, dim3(blocks), dim3(256), 0, s, static_cast<const float *>(features),
                           dim, g.item0, g.n_items, g.pair_base, g.n_groups, it.src, it.len, list, count,
                           max_count, norm, euclid, p64, p32, flags);
    else
        hipLaunchKernelGGL(k_long_dtw<uint16_t>, dim3(blocks), dim3(256), 0, s,
                           static_cast<const uint16_t *>(features), dim, g.item0, g.n_items, g.pair_base,
                           g.n_groups, it.src, it.len, list, count, max_count, norm, euclid, p64, p32, flags);
    FABX_HIP(hipGetLastError());
}

void recheck_fp64(hipStream_t s, const void *features, int dtype, int dim, const GroupTables &g,
                  const ItemTables &it, const int64_t *list, const unsigned int *count,
                  int64_t max_count, int mode, int norm, bool has_long, int euclid, double *p64) {
    if (max_count <= 0) return;
    if (mode == FABX_MODE_POOLED && dim > 2048) fail(FABX_EINVAL, "pooled recheck supports dim <= 2048");
    const unsigned blocks = unsigned(std::min<int64_t>(max_count, 4096));
    if (mode == FABX_MODE_DTW && has_long)
        long_dtw(s, features, dtype, dim, g, it, list, count, max_count, norm, euclid, p64, nullptr, nullptr);
    if (mode == FABX_MODE_DTW) {
        // pairs of short items, then the others (each kernel skips the other's)
        if (dtype == FABX_DTYPE_F32) {
            hipLaunchKernelGGL((k_recheck_dtw<float, false>), dim3(blocks), dim3(256), 0, s,
                               static_cast<const float *>(features), dim, g.item0, g.n_items, g.pair_base,
                               g.n_groups, it.src, it.len, list, count, max_count, norm, euclid, p64);
            hipLaunchKernelGGL((k_recheck_dtw<float, true>), dim3(blocks), dim3(256), 0, s,
                               static_cast<const float *>(features), dim, g.item0, g.n_items, g.pair_base,
                               g.n_groups, it.src, it.len, list, count, max_count, norm, euclid, p64);
        } else {
            hipLaunchKernelGGL((k_recheck_dtw<uint16_t, false>), dim3(blocks), dim3(256), 0, s,
                               static_cast<const uint16_t *>(features), dim, g.item0, g.n_items, g.pair_base,
                               g.n_groups, it.src, it.len, list, count, max_count, norm, euclid, p64);
            hipLaunchKernelGGL((k_recheck_dtw<uint16_t, true>), dim3(blocks), dim3(256), 0, s,
                               static_cast<const uint16_t *>(features), dim, g.item0, g.n_items, g.pair_base,
                               g.n_groups, it.src, it.len, list, count, max_count, norm, euclid, p64);
        }
    } else {
        if (dtype == FABX_DTYPE_F32)
            hipLaunchKernelGGL(k_recheck_pooled<float>, dim3(blocks), dim3(256), 0, s,
                               static_cast<const float *>(features), dim, g.item0, g.n_items,
                               g.pair_base, g.n_groups, it.src, it.len, list, count, max_count, euclid, p64);
        else
            hipLaunchKernelGGL(k_recheck_pooled<uint16_t>, dim3(blocks), dim3(256), 0, s,
                               static_cast<const uint16_t *>(features), dim, g.item0, g.n_items,
                               g.pair_base, g.n_groups, it.src, it.len, list, count, max_count, euclid, p64);
    }
    FABX_HIP(hipGetLastError());
}

}  // namespace kern
}  // namespace fabx
