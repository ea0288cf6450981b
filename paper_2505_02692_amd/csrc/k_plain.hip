// Plain FP32 form: the straightforward GPU pipeline the BF16 form is
// measured against.
//
//  gram_angular_f32: per segment (a BY group's pooled items, or a strip of a
//    group's frames against all its frames), every pair of unit rows ->
//    theta / pi in FP32 (64 x 64 output tile per 256-thread block, 4 x 4 per
//    thread, K staged through LDS in steps of 16), written to HBM.  For the Euclidean distance
//    the same tiles sum (u_k - v_k)^2 over raw rows (no cancellation of a
//    norms-minus-dot form) and take the square root.
//  unit_mismatch: the same segments and tiles for discrete unit codes: 0 for
//    equal codes, 1 otherwise (exact in FP32).
//  dtw_plain: one wave per ordered item pair; lane i owns row i of the DTW
//    matrix and the wave sweeps the anti-diagonals t = i + j, reading the
//    distance matrix from HBM: the paper's wavefront scheme (one pair per
//    block, the cells of a diagonal in parallel), with the previous two
//    diagonals held in registers of neighbouring lanes.  The distance
//    matrices of a task can far exceed device memory (the sum of the squared
//    frame counts of its groups), so they are made and consumed in batches
//    of strips that fit one buffer.
#include "device_common.h"
#include "kernels.h"

namespace fabx {
namespace kern {
namespace {

using dev::kInf;
using dev::kWave;

constexpr int kTile = 64;
constexpr int kK = 16;

template <bool kEuclid>
__global__ __launch_bounds__(256) void k_gram_angular_f32(const float *__restrict__ xn, int dim_pad,
                                                          const int64_t *__restrict__ row0,
                                                          const int64_t *__restrict__ nrows,
                                                          const int64_t *__restrict__ col0,
                                                          const int64_t *__restrict__ ncols,
                                                          const int64_t *__restrict__ base,
                                                          const int64_t *__restrict__ tile_prefix,
                                                          int64_t n_seg, float *__restrict__ out) {
    __shared__ float As[kK][kTile + 4];
    __shared__ float Bs[kK][kTile + 4];
    const int64_t t_hi = tile_prefix[n_seg];
    for (int64_t tile = tile_prefix[0] + blockIdx.x; tile < t_hi; tile += gridDim.x) {
    const int64_t sg = dev::find_segment(tile_prefix, n_seg, tile);
    const int64_t nr = nrows[sg], nc = ncols[sg];
    const int64_t ntc = (nc + kTile - 1) / kTile;
    const int64_t local = tile - tile_prefix[sg];
    const int64_t r0 = (local / ntc) * kTile, c0 = (local % ntc) * kTile;
    const float *rows = xn + row0[sg] * int64_t(dim_pad);
    const float *cols = xn + col0[sg] * int64_t(dim_pad);
    const int tid = threadIdx.x;
    const int ty = tid / 16, tx = tid % 16;
    float acc[4][4] = {};
    // staging: each thread loads 4 consecutive k of one row for A and for B
    const int lr = tid / 4, lk = (tid % 4) * 4;
    for (int k0 = 0; k0 < dim_pad; k0 += kK) {
        float4 a = make_float4(0.f, 0.f, 0.f, 0.f), b = a;
        if (r0 + lr < nr) a = *reinterpret_cast<const float4 *>(rows + (r0 + lr) * dim_pad + k0 + lk);
        if (c0 + lr < nc) b = *reinterpret_cast<const float4 *>(cols + (c0 + lr) * dim_pad + k0 + lk);
        As[lk + 0][lr] = a.x; As[lk + 1][lr] = a.y; As[lk + 2][lr] = a.z; As[lk + 3][lr] = a.w;
        Bs[lk + 0][lr] = b.x; Bs[lk + 1][lr] = b.y; Bs[lk + 2][lr] = b.z; Bs[lk + 3][lr] = b.w;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kK; ++k) {
            float av[4], bv[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) av[i] = As[k][ty * 4 + i];
#pragma unroll
            for (int j = 0; j < 4; ++j) bv[j] = Bs[k][tx * 4 + j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    if (kEuclid) {
                        const float d = av[i] - bv[j];
                        acc[i][j] = fmaf(d, d, acc[i][j]);
                    } else {
                        acc[i][j] = fmaf(av[i], bv[j], acc[i][j]);
                    }
                }
        }
        __syncthreads();
    }
    float *o = out + base[sg];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int64_t r = r0 + ty * 4 + i;
        if (r >= nr) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t c = c0 + tx * 4 + j;
            if (c >= nc) continue;
            if (kEuclid) {
                o[r * nc + c] = __builtin_sqrtf(acc[i][j]);
            } else {
                const float cs = fminf(fmaxf(acc[i][j], -1.0f), 1.0f);
                o[r * nc + c] = acosf(cs) * dev::kInvPi;
            }
        }
    }
    }
}

// Discrete units: d = [code_row != code_col], one 64 x 64 tile per block at a
// time (a thread per element, 16 each).
__global__ __launch_bounds__(256) void k_unit_mismatch(const int32_t *__restrict__ codes,
                                                       const int64_t *__restrict__ row0,
                                                       const int64_t *__restrict__ nrows,
                                                       const int64_t *__restrict__ col0,
                                                       const int64_t *__restrict__ ncols,
                                                       const int64_t *__restrict__ base,
                                                       const int64_t *__restrict__ tile_prefix,
                                                       int64_t n_seg, float *__restrict__ out) {
    const int64_t t_hi = tile_prefix[n_seg];
    for (int64_t tile = tile_prefix[0] + blockIdx.x; tile < t_hi; tile += gridDim.x) {
        const int64_t sg = dev::find_segment(tile_prefix, n_seg, tile);
        const int64_t nr = nrows[sg], nc = ncols[sg];
        const int64_t ntc = (nc + kTile - 1) / kTile;
        const int64_t local = tile - tile_prefix[sg];
        const int64_t r0 = (local / ntc) * kTile, c0 = (local % ntc) * kTile;
        float *o = out + base[sg];
        for (int e = threadIdx.x; e < kTile * kTile; e += 256) {
            const int64_t r = r0 + e / kTile, c = c0 + e % kTile;
            if (r < nr && c < nc) o[r * nc + c] = codes[row0[sg] + r] != codes[col0[sg] + c] ? 1.0f : 0.0f;
        }
    }
}

// One wave per pair slot of a strip: lane i is on row i, column t - i at step
// t (anti-diagonals), reading the strip's frame distances.  kLong: items may
// have more than 64 frames; rows then go in chunks of 64, each sweeping all
// columns, and a chunk hands its last row's costs and path lengths to the
// next one through the wave's LDS row buffer.  exact (discrete units, whose
// costs are integers): the path-normalised value is the double quotient
// rounded once to float, so equal fractions give equal values and different
// ones (which differ by at least 1 / (N + M)^2, two float ulps or more) stay apart,
// whatever the float division's rounding.
template <bool kLong>
__global__ __launch_bounds__(256) void k_dtw_plain(const float *__restrict__ dmat,
                                                   const int64_t *__restrict__ s_group,
                                                   const int64_t *__restrict__ s_slot0,
                                                   const int64_t *__restrict__ s_row0,
                                                   const int64_t *__restrict__ s_base, int64_t n_strips,
                                                   const int64_t *__restrict__ g_item0,
                                                   const int64_t *__restrict__ g_n,
                                                   const int64_t *__restrict__ g_frame0,
                                                   const int64_t *__restrict__ g_nframes,
                                                   const int64_t *__restrict__ g_pair_base,
                                                   const int32_t *__restrict__ item_len,
                                                   const int64_t *__restrict__ item_dst, int norm,
                                                   int exact, float *__restrict__ p32) {
    constexpr int kRowBuf = kLong ? FABX_MAX_ITEM_FRAMES : 1;
    __shared__ float rowc_s[4][kRowBuf];  // per wave: the previous chunk's last row (costs)
    __shared__ int rowl_s[4][kRowBuf];    // and path lengths
    const int i = threadIdx.x % kWave, wv = threadIdx.x / kWave;
    float *rowc = rowc_s[wv];
    int *rowl = rowl_s[wv];
    const int64_t slot_lo = s_slot0[0], slot_hi = s_slot0[n_strips];
    // one wave per slot; the loop bound is uniform across the wave
    for (int64_t slot = slot_lo + int64_t(blockIdx.x) * 4 + wv; slot < slot_hi;
         slot += int64_t(gridDim.x) * 4) {
    const int64_t sg = dev::find_segment(s_slot0, n_strips, slot);
    const int64_t g = s_group[sg];
    const int64_t n = g_n[g];
    const int64_t local = slot - g_pair_base[g];
    const int64_t x = g_item0[g] + local / n, y = g_item0[g] + local % n;
    const int N = item_len[x], M = item_len[y];
    const int64_t F = g_nframes[g];
    const float *d = dmat + s_base[sg] + (item_dst[x] - s_row0[sg]) * F + (item_dst[y] - g_frame0[g]);

    float c = kInf;          // c[i][j-1] (own value of the previous step)
    int len = 0;
    for (int r0 = 0; r0 < N; r0 += kWave) {
    const int nr = min(kWave, N - r0);
    const int gi = r0 + i;   // this lane's row
    c = kInf;
    len = 0;
    float up_prev = kInf;    // c[i-1][j-1]
    int lup_prev = 0;
    for (int t = 0; t < nr + M - 1; ++t) {
        const int j = t - i;
        float up = __shfl_up(c, 1, kWave);  // c[i-1][j]: lane i-1 at step t-1
        int lup = __shfl_up(len, 1, kWave);
        if (i == 0) {  // the row above the chunk (none above row 0)
            const bool in = kLong && r0 > 0 && j >= 0 && j < M;
            up = in ? rowc[in ? j : 0] : kInf;
            lup = in ? rowl[in ? j : 0] : 0;
        }
        float diag = up_prev, left = c;
        int ldiag = lup_prev, lleft = len;
        if (gi == 0) diag = kInf;
        if (j == 0) { left = kInf; diag = kInf; }
        up_prev = up;
        lup_prev = lup;
        if (i < nr && j >= 0 && j < M) {
            const float dv = d[int64_t(gi) * F + j];
            if (gi == 0 && j == 0) {
                c = dv;
                len = 1;
            } else {
                float best;
                int lb;
                if (diag <= left && diag <= up) { best = diag; lb = ldiag; }
                else if (left <= up) { best = left; lb = lleft; }
                else { best = up; lb = lup; }
                c = dv + best;
                len = lb + 1;
            }
            if (kLong && i == nr - 1) {  // this chunk's last row, for the next chunk
                rowc[j] = c;
                rowl[j] = len;
            }
        }
    }
    }
    if (i == (N - 1) % kWave)
        p32[slot] = norm != FABX_NORM_PATH ? c : exact ? float(double(c) / double(len)) : c / float(len);
    }
}

}  // namespace

void gram_angular_f32(hipStream_t s, const float *xn, int dim_pad, const GramSegments &seg, float *out,
                      int euclid) {
    if (seg.n <= 0 || seg.n_tiles <= 0) return;
    if (dim_pad % kK) fail(FABX_EINVAL, "padded dim must be a multiple of 16");
    const dim3 grid(grid_for(seg.n_tiles, 1)), block(256);
    if (euclid)
        hipLaunchKernelGGL(k_gram_angular_f32<true>, grid, block, 0, s, xn, dim_pad, seg.row0, seg.nrows,
                           seg.col0, seg.ncols, seg.base, seg.tile_prefix, seg.n, out);
    else
        hipLaunchKernelGGL(k_gram_angular_f32<false>, grid, block, 0, s, xn, dim_pad, seg.row0, seg.nrows,
                           seg.col0, seg.ncols, seg.base, seg.tile_prefix, seg.n, out);
    FABX_HIP(hipGetLastError());
}

void unit_mismatch(hipStream_t s, const int32_t *codes, const GramSegments &seg, float *out) {
    if (seg.n <= 0 || seg.n_tiles <= 0) return;
    hipLaunchKernelGGL(k_unit_mismatch, dim3(grid_for(seg.n_tiles, 1)), dim3(256), 0, s, codes, seg.row0,
                       seg.nrows, seg.col0, seg.ncols, seg.base, seg.tile_prefix, seg.n, out);
    FABX_HIP(hipGetLastError());
}

void dtw_plain(hipStream_t s, const float *dmat, const PlainStrips &st, const GroupTables &g,
               const ItemTables &it, int norm, bool has_long, bool exact, float *p32) {
    if (st.n <= 0 || st.n_slots <= 0) return;
    hipLaunchKernelGGL(has_long ? k_dtw_plain<true> : k_dtw_plain<false>, dim3(grid_for(st.n_slots, 4)),
                       dim3(256), 0, s, dmat, st.group, st.slot0, st.row0, st.base, st.n, g.item0, g.n_items,
                       g.frame0, g.n_frames, g.pair_base, it.len, it.dst, norm, exact ? 1 : 0, p32);
    FABX_HIP(hipGetLastError());
}

}  // namespace kern
}  // namespace fabx
