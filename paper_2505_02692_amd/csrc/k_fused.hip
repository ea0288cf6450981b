// BF16 form: frame distances on MFMA fused with the DTW wavefront.
//
// Work unit = (row block, column block) of one BY group.  A row block packs
// whole items into at most 64 frames (one DTW lane per frame row); a column
// block packs whole items into at most kCols frames.  For each unit:
//
//  1. Gram tile on MFMA: S = Xr (64 x D) * Xc^T (D x kCols), BF16 operands
//     staged through LDS in K chunks of 64, FP32 accumulation
//     (v_mfma_f32_32x32x16_bf16; wave w owns columns [32w, 32w + 32) of a
//     128-column tile, two 32 x 32 accumulators for the 64 rows).
//  2. Epilogue: cos = S * rinv_r * rinv_c, d = acos(cos) / pi (Abramowitz &
//     Stegun 4.4.46), written to an LDS tile; it never reaches HBM.
//  3. DTW wavefront (the recurrence of the "Dynamic Time Warping on GPU"
//     section), laid out for wave64 instead of one pair per block: lane r
//     owns frame row r of the row block, whatever item it belongs to, and
//     each wave streams the columns of its share of the column items past
//     all 64 rows.  Lane r works on column t - i_r at step t (i_r = row
//     index inside its own item), so the value above comes from lane r - 1
//     one step earlier (DPP wave_shr:1) and the diagonal one from two steps
//     earlier; a column that starts a new item resets the left neighbour.
//     Every step all lanes do useful work except the fill and drain of the
//     longest row item.
//
// Path length (FABX_NORM_PATH): with BF16 distances the predecessor chosen in
// FP32 can differ from the FP64 one when their cumulative costs are within
// the error bound, and then the length (the divisor) changes.  Each cell
// therefore carries the interval [Lmin, Lmax] of lengths over all
// predecessors within `delta` of the minimum (packed as two u16 halves,
// high = Lmax, low = 0xFFFF - Lmin, so one packed max merges both ends).
// If delta is at least twice the cumulative-cost error, the FP64 length lies
// in the interval; a pair whose interval is not a single value is flagged
// non-robust (flag bit 0) and recomputed in FP64.
#include "device_common.h"
#include "kernels.h"

namespace fabx {
namespace kern {
namespace {

using dev::kInf;
using dev::kWave;

typedef short bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

constexpr int kRows = 64;             // row block frames = DTW lanes
// Near-parallel (or antiparallel) frames: acos is ill-conditioned at
// |cos| = 1, where the BF16 cosine's rounding (about 1e-7) moves the angle by
// up to about 1e-4.  |cos| above kNearCos (an angle under about 3e-3 rad from
// 0 or pi, a distance within kNearD of 0 or 1) sends the pair to the FP64
// recheck.
constexpr float kNearCos = 1.0f - 4.7e-6f;
constexpr float kNearD = 9.8e-4f;
constexpr int kKc = 64;               // K chunk (bf16 elements) staged in LDS
constexpr int kLdsRow = kKc + 8;      // padded LDS row of a K chunk (bf16)

// Tile geometry for a column block of kC frames (128 or 256): wave w owns
// columns [kWaveCols * w, kWaveCols * (w + 1)) of the Gram tile, kCT tiles of
// 32 columns.
template <int kC>
struct Tile {
    static constexpr int kCols = kC;
    static constexpr int kWaveCols = kC / 4;
    static constexpr int kCT = kWaveCols / 32;
    static constexpr int kDStride = kC + 2;  // LDS distance tile stride (floats)
    static constexpr int kStageBytes = (kRows + kC) * kLdsRow * 2;
    // distance tile + a tail guard: the DTW loop reads up to 67 columns past a
    // row's end (64 of drain, 3 of read-ahead)
    static constexpr int kTileBytes = (kRows * kDStride + kWave + 4) * 4;
    // column flags: a zero guard of one wave before the span and one wave + 4 after
    static constexpr int kFlagLen = kWave + kC + kWave + 4;
    static constexpr int kSmemBytes = kStageBytes > kTileBytes ? kStageBytes : kTileBytes;
};

// Value of lane - 1 (DPP wave_shr:1 with bound_ctrl); lane 0 reads 0.  The add
// that consumes it folds the move into one DPP instruction.
__device__ __forceinline__ float shr1z(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xf, 0xf, true));
}
__device__ __forceinline__ uint32_t shr1uz(uint32_t v) {
    return uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0x138, 0xf, 0xf, true));
}

__device__ __forceinline__ uint32_t pk_max(uint32_t a, uint32_t b) {
    u16x2 x = __builtin_bit_cast(u16x2, a), y = __builtin_bit_cast(u16x2, b);
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(x, y));
}
__device__ __forceinline__ uint32_t pk_step(uint32_t a) {
    // Lmax + 1 (high half), (0xFFFF - Lmin) - 1 (low half), each half wrapping
    u16x2 x = __builtin_bit_cast(u16x2, a);
    u16x2 inc = {(unsigned short)0xFFFF, (unsigned short)1};
    return __builtin_bit_cast(uint32_t, x + inc);
}

// A K chunk of the tile's rows, held in registers between its global load
// and its store to LDS: each thread owns kN * kKc / 8 / 256 pieces of 16 bytes.
template <int kN>
struct Chunk {
    static constexpr int kPer = kN * (kKc / 8) / 256;
    // one vector value, not an array, so it stays in registers
    typedef uint32_t Vec __attribute__((ext_vector_type(4 * kPer)));
    Vec v;
    // rows beyond nr (>= 1) repeat row nr - 1: finite values whose products
    // only reach accumulator rows or columns that are never used, or that are
    // scaled by a zero inverse norm (no zero fill, no masked loads)
    __device__ __forceinline__ void load(const uint16_t *__restrict__ xn, int dim_pad, int64_t row0, int nr,
                                         int k0) {
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const int p = threadIdx.x + 256 * i;
            const int r = min(p / (kKc / 8), nr - 1), q = p % (kKc / 8);
            const uint4 t = *reinterpret_cast<const uint4 *>(xn + (row0 + r) * dim_pad + k0 + q * 8);
            v[4 * i] = t.x;
            v[4 * i + 1] = t.y;
            v[4 * i + 2] = t.z;
            v[4 * i + 3] = t.w;
        }
    }
    __device__ __forceinline__ void store(uint16_t *lds) const {
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const int p = threadIdx.x + 256 * i;
            const int r = p / (kKc / 8), q = p % (kKc / 8);
            *reinterpret_cast<uint4 *>(lds + r * kLdsRow + q * 8) =
                make_uint4(v[4 * i], v[4 * i + 1], v[4 * i + 2], v[4 * i + 3]);
        }
    }
};

// acc[h][ct] = rows [32h, 32h + 32) against columns kWaveCols * w + 32 ct + [0, 32).
// Software-pipelined: the next K chunk is loaded from memory into registers
// while the MFMAs consume the current one from LDS.  Column tiles that lie
// past nc skip their MFMAs, and so does the second row half when nr <= 32
// (those accumulators are never read).  Every product accumulates its K
// range in the same order whatever the tile width, so results do not depend
// on it.  Column tiles wholly below c_lo (columns nobody reads) skip their
// MFMAs too.  `stash` runs once, after the first chunk is stored and before the
// barrier that publishes it, so LDS it writes is visible to the epilogue.
template <int kC, typename Stash>
__device__ __forceinline__ void gram_tile(uint16_t *smem, const uint16_t *__restrict__ xn, int dim_pad,
                                          int64_t r0, int nr, int64_t c0, int nc, int c_lo,
                                          f32x16 (&acc)[2][Tile<kC>::kCT], Stash &&stash) {
    using T = Tile<kC>;
    const int lane = threadIdx.x % kWave;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const bool do1 = nr > 32;
    uint16_t *As = smem;
    uint16_t *Bs = smem + kRows * kLdsRow;
#pragma unroll
    for (int ct = 0; ct < T::kCT; ++ct)
        for (int i = 0; i < 16; ++i) { acc[0][ct][i] = 0.0f; acc[1][ct][i] = 0.0f; }
    Chunk<kRows> ca;
    Chunk<kC> cb;
    ca.load(xn, dim_pad, r0, nr, 0);
    cb.load(xn, dim_pad, c0, nc, 0);
    for (int k0 = 0; k0 < dim_pad; k0 += kKc) {
        ca.store(As);
        cb.store(Bs);
        if (k0 == 0) stash();
        __syncthreads();
        if (k0 + kKc < dim_pad) {
            ca.load(xn, dim_pad, r0, nr, k0 + kKc);
            cb.load(xn, dim_pad, c0, nc, k0 + kKc);
        }
#pragma unroll
        for (int ct = 0; ct < T::kCT; ++ct) {
            const int col0 = T::kWaveCols * w + 32 * ct;
            if (col0 < nc && col0 + 32 > c_lo) {
#pragma unroll
                for (int ks = 0; ks < kKc / 16; ++ks) {
                    const int kk = ks * 16 + (lane / 32) * 8;
                    const bf16x8 a0 = *reinterpret_cast<const bf16x8 *>(As + (lane % 32) * kLdsRow + kk);
                    const bf16x8 b = *reinterpret_cast<const bf16x8 *>(Bs + (col0 + lane % 32) * kLdsRow + kk);
                    acc[0][ct] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b, acc[0][ct], 0, 0, 0);
                    if (do1) {
                        const bf16x8 a1 =
                            *reinterpret_cast<const bf16x8 *>(As + (32 + lane % 32) * kLdsRow + kk);
                        acc[1][ct] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b, acc[1][ct], 0, 0, 0);
                    }
                }
            }
        }
        __syncthreads();
    }
}

// Inverse norms of a unit's kRows row frames and kC column frames (zero past
// nr / nc), loaded into registers before the Gram tile and written to LDS by
// its stash hook, so the epilogue reads them from LDS instead of issuing one
// dependent global load per element.
template <int kC>
struct NormStage {
    static constexpr int kN = kRows + kC;
    static constexpr int kPer = (kN + 255) / 256;
    float v[kPer];
    __device__ __forceinline__ void load(const float *__restrict__ rinv, int64_t r0, int nr, int64_t c0,
                                         int nc) {
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const int j = threadIdx.x + 256 * i;
            v[i] = 0.0f;
            if (j < kRows) {
                if (j < nr) v[i] = rinv[r0 + j];
            } else if (j < kN && j - kRows < nc) {
                v[i] = rinv[c0 + j - kRows];
            }
        }
    }
    __device__ __forceinline__ void store(float *lds) const {
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const int j = threadIdx.x + 256 * i;
            if (j < kN) lds[j] = v[i];
        }
    }
};

// Row (within the 32 x 32 tile) of accumulator element i of this lane.
__device__ __forceinline__ int acc_row(int i, int lane) { return 8 * (i / 4) + 4 * (lane / 32) + (i % 4); }

// kEuclid: the Euclidean distance of the raw frames, from the same unit-vector
// cosine and each frame's FP32 length (flen): |u - v|^2 = (|u| - |v|)^2 +
// 2 |u| |v| (1 - cos).  A near-parallel element is stored with its sign bit
// set (the DTW of a careful unit takes its magnitude and notes it), and delta
// is in units of the largest frame length (*scale, FP32 bits).
template <int kC, bool kPath, bool kEuclid>
__global__ __launch_bounds__(256, 4) void k_fused(const uint16_t *__restrict__ xn,
                                                  const float *__restrict__ rinv, int dim_pad,
                                                  const int64_t *__restrict__ g_item0,
                                                  const int64_t *__restrict__ g_n,
                                                  const int64_t *__restrict__ g_pair_base,
                                                  const int32_t *__restrict__ item_len,
                                                  const int64_t *__restrict__ item_dst,
                                                  const int32_t *__restrict__ rb,
                                                  const int32_t *__restrict__ cb,
                                                  const int64_t *__restrict__ unit_prefix,
                                                  const int32_t *__restrict__ band_rb,
                                                  const int32_t *__restrict__ g_cb0,
                                                  const int32_t *__restrict__ rb_cstart,
                                                  int64_t n_bands, int64_t n_units, int64_t grid_q,
                                                  float delta, float *__restrict__ p32,
                                                  uint8_t *__restrict__ flags,
                                                  unsigned int *__restrict__ nonrobust_n,
                                                  unsigned int *__restrict__ unit_ctr,
                                                  const float *__restrict__ flen,
                                                  const unsigned int *__restrict__ scale) {
    using T = Tile<kC>;
    constexpr int kDStride = T::kDStride, kFlagLen = T::kFlagLen;
    __shared__ __attribute__((aligned(16))) unsigned char smem_raw[T::kSmemBytes];
    __shared__ uint32_t colflag[4][kFlagLen];
    __shared__ __attribute__((aligned(16))) float norm_s[kRows + kC];  // row then column inverse norms
    __shared__ __attribute__((aligned(16))) float len_s[kEuclid ? kRows + kC : 1];  // and lengths
    if constexpr (kEuclid) delta *= __uint_as_float(*scale);
    __shared__ int near_s;  // the unit holds a near-parallel frame pair
    // XCD-aware order: the 8 XCDs take blocks round-robin, so XCD x works
    // through the contiguous unit range [x * grid_q, (x+1) * grid_q) (units of
    // one group share its frames in that XCD's L2).  gridDim.x is a multiple
    // of 8.  With a block per unit the block's index gives its unit; with
    // fewer blocks (a persistent grid) the blocks of an XCD take the range's
    // units in order from the XCD's counter (zero at launch), so the units in
    // flight stay together; each block stops once its counter passes the range.
    const int64_t xcd = blockIdx.x % 8, n_m = gridDim.x / 8;
    const bool take = n_m < grid_q;
    __shared__ int64_t taken_s;
    // next unit index for this block: written by thread 0, read by every
    // thread between two barriers (a skipped unit has no barrier of its own)
    auto next = [&](int64_t j) -> int64_t {
        if (!take) return j + n_m;
        if (threadIdx.x == 0) taken_s = int64_t(atomicAdd(unit_ctr + xcd, 1u));
        __syncthreads();
        const int64_t v = taken_s;
        __syncthreads();
        return v;
    };
    const int lane = threadIdx.x % kWave;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    // the band of the block's previous unit and its unit range: a persistent
    // block's next unit usually lies in it, which spares the band search
    int64_t band_c = -1, band_lo = 0, band_hi = 0;
    for (int64_t j = take ? next(0) : int64_t(blockIdx.x / 8); j < grid_q; j = next(j)) {
    const int64_t unit = xcd * grid_q + j;
    if (unit >= n_units) break;  // uniform across the block; later units are larger

    // the unit's band, row block, group and column block: within a band,
    // column blocks from the band's first kept one on, row blocks fastest
    if (band_c < 0 || unit < band_lo || unit >= band_hi) {  // uniform
        band_c = dev::find_segment_wave(unit_prefix, n_bands, unit);
        band_lo = unit_prefix[band_c];
        band_hi = unit_prefix[band_c + 1];
    }
    const int64_t bi = band_c;
    const int rb0 = band_rb[bi], band_rows = band_rb[bi + 1] - rb0;
    const int64_t local = unit - band_lo;
    // 32-bit division whenever the offset fits (a band holds fewer than 2^32
    // units unless a group has hundreds of millions of column blocks)
    int64_t rbi;
    int c_local;
    if (local < (int64_t(1) << 32)) {
        const uint32_t l32 = uint32_t(local), br = uint32_t(band_rows);
        rbi = rb0 + int64_t(l32 % br);
        c_local = rb_cstart[rb0] + int(l32 / br);
    } else {
        rbi = rb0 + local % band_rows;
        c_local = rb_cstart[rb0] + int(local / band_rows);
    }
    if (c_local < rb_cstart[rbi]) continue;  // uniform: wholly below the group's diagonal
    const int64_t g = rb[4 * rbi];
    const int cbi = g_cb0[g] + c_local;
    const int r_item0 = rb[4 * rbi + 1], r_nitems = rb[4 * rbi + 2], r_frames = rb[4 * rbi + 3];
    const int c_item0 = cb[4 * cbi + 1], c_nitems = cb[4 * cbi + 2], c_frames = cb[4 * cbi + 3];
    const int64_t r_frame0 = item_dst[r_item0], c_frame0 = item_dst[c_item0];

    if (threadIdx.x == 0) near_s = 0;  // read after the barriers of the Gram tile and the epilogue
    // 1. Gram tile
    NormStage<kC> ns, ls;
    ns.load(rinv, r_frame0, r_frames, c_frame0, c_frames);
    if constexpr (kEuclid) ls.load(flen, r_frame0, r_frames, c_frame0, c_frames);
    // column items before the row block's first item pair only with rows after
    // them, which other units write: their columns (the first c_skip of the
    // block) are not needed
    const int k_first = max(0, r_item0 - c_item0);
    int c_skip = 0;
    for (int k = 0; k < min(k_first, c_nitems); ++k) c_skip += item_len[c_item0 + k];
    f32x16 acc[2][T::kCT];
    gram_tile<kC>(reinterpret_cast<uint16_t *>(smem_raw), xn, dim_pad, r_frame0, r_frames, c_frame0,
                  c_frames, c_skip, acc, [&] {
                      ns.store(norm_s);
                      if constexpr (kEuclid) ls.store(len_s);
                  });

    // 2. epilogue -> LDS distance tile (the staging buffers are dead now).  Only
    // the rows and column waves that hold frames are written; the DTW reads the
    // others only in lanes and steps whose results are discarded.
    // Rows and columns past the block's frames have zero inverse norms, so their
    // cosines are 0 and never count as near-parallel.
    float *dt = reinterpret_cast<float *>(smem_raw);
    // Largest |cos| this lane wrote, leaving out a frame against itself: that
    // element (row frame = column frame, only in units on the diagonal of the
    // group's pair matrix, for the pair (x, x) that is never compared) is
    // parallel by construction.  In the sub-tile of rows 32h + acc_row(i, lane)
    // and columns col0 + lane % 32 the element is a frame against itself when
    // acc_row(i, lane) - lane % 32 equals e = (column block start + col0) -
    // (row block start + 32h), which needs |e| < 32.  The Euclidean epilogue
    // tests each element (it also marks near-parallel ones); the angular one
    // takes the maximum over all elements and redoes it for the rare sub-tiles
    // with |e| < 32 without those elements.
    // (kept as bits: the values are >= 0, whose bit patterns order like them)
    uint32_t cmax = 0;
    const int lane_term = 4 * (lane / 32) - lane % 32;
#pragma unroll
    for (int ct = 0; ct < T::kCT; ++ct) {
        const int col0 = T::kWaveCols * w + 32 * ct;
        if (col0 >= c_frames || col0 + 32 <= c_skip) continue;
        const int col = col0 + lane % 32;
        const float rc = norm_s[kRows + col];
        const float lc = kEuclid ? len_s[kRows + col] : 0.0f;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            if (h == 1 && r_frames <= 32) break;
            uint32_t cmax_t = 0;  // this sub-tile's largest |cos| (bits)
            // a sub-tile within 32 frames of the diagonal may hold frames against
            // themselves (uniform over the wave; rare)
            const int64_t e = c_frame0 - r_frame0 + col0 - 32 * h;
            const bool on_diag = e > -32 && e < 32;
            const int q = on_diag ? int(e) - lane_term : 1 << 20;  // 1 << 20: no such element
            // rows past the block's frames belong to no item (their DTW lanes are
            // discarded): the groups of 8 rows (4 elements) from the first that
            // starts past them on are skipped (uniform over the wave)
#pragma unroll
            for (int g4 = 0; g4 < 4; ++g4) {
                if (32 * h + 8 * g4 >= r_frames) break;
#pragma unroll
                for (int i = 4 * g4; i < 4 * g4 + 4; ++i) {
                    const int r = 32 * h + acc_row(i, lane);
                    const float raw = acc[h][ct][i] * norm_s[r] * rc;
                    if constexpr (kEuclid) {
                        const float cs = fminf(fmaxf(raw, -1.0f), 1.0f);
                        const float ac = 8 * (i / 4) + (i % 4) == q ? 0.0f : fabsf(cs);
                        cmax_t = max(cmax_t, __float_as_uint(ac));
                        const float lr = len_s[r], dl = lr - lc;
                        const float d =
                            __builtin_sqrtf(fmaxf(fmaf(dl, dl, 2.0f * lr * lc * (1.0f - cs)), 0.0f));
                        dt[r * kDStride + col] = ac > kNearCos ? -d : d;  // the sign marks it
                    } else {
                        const float ax = fminf(fabsf(raw), 1.0f);  // |cos|, clamped
                        cmax_t = max(cmax_t, __float_as_uint(ax));
                        dt[r * kDStride + col] = dev::acos_over_pi_abs(ax, raw);
                    }
                }
            }
            // angular: the loop above took every element; on the diagonal the
            // sub-tile's largest |cos| is taken again without a frame against itself
            if (!kEuclid && on_diag) {
                cmax_t = 0;
#pragma unroll
                for (int g4 = 0; g4 < 4; ++g4) {
                    if (32 * h + 8 * g4 >= r_frames) break;
#pragma unroll
                    for (int i = 4 * g4; i < 4 * g4 + 4; ++i) {
                        const int r = 32 * h + acc_row(i, lane);
                        const float ax = fminf(fabsf(acc[h][ct][i] * norm_s[r] * rc), 1.0f);
                        cmax_t = max(cmax_t, 8 * (i / 4) + (i % 4) == q ? 0u : __float_as_uint(ax));
                    }
                }
            }
            cmax = max(cmax, cmax_t);
        }
    }
    if (__ballot(__uint_as_float(cmax) > kNearCos) != 0 && lane == 0) atomicOr(&near_s, 1);

    // 3. DTW.  Column items of this block split over the 4 waves by start frame.
    // Lane constants: the row item of lane `lane`.
    int ir = 0, nx = 0, x_task = -1;
    {
        int start = 0;
        for (int k = 0; k < r_nitems; ++k) {
            const int L = item_len[r_item0 + k];
            if (lane >= start && lane < start + L) { ir = lane - start; nx = L; x_task = r_item0 + k; }
            start += L;
        }
    }
    int max_n = 0;
    for (int k = 0; k < r_nitems; ++k) max_n = max(max_n, item_len[r_item0 + k]);
    // this wave's column items: those whose first frame falls in its quarter of
    // the needed columns (from item k_first on).  A lane reads distances at most
    // 63 columns left of its span's start only in steps whose cells are never
    // used (an item's first column resets the left and diagonal neighbours);
    // those columns may hold stale values when their tiles were skipped.
    int y_begin = 0, y_end = 0, s_begin = 0, s_end = 0;
    {
        const int skip = c_skip;
        const int kept = max(c_frames - skip, 1);
        // item k belongs to wave floor(4 (start - skip) / kept), tested as
        // w kept <= 4 (start - skip) < (w + 1) kept without a division
        const int own_lo = w * kept, own_hi = own_lo + kept;
        int start = skip;
        bool seen = false;
        for (int k = k_first; k < c_nitems; ++k) {
            const int L = item_len[c_item0 + k];
            const int a4 = 4 * (start - skip);
            if (a4 >= own_lo && a4 < own_hi) {
                if (!seen) { y_begin = k; s_begin = start; seen = true; }
                y_end = k + 1;
                s_end = start + L;
            }
            start += L;
        }
        // column c of this wave's span is entry kWave + c: byte 0 = 1 at the
        // first column of an item (tested with one byte-select compare), bits
        // 8..21 = the item's index in the column block, bit 31 =
        // last column.  The guards read as 0 (no item start, no output).
        // Same-wave LDS stores land in issue order.
        for (int j = lane; j < kFlagLen; j += kWave) colflag[w][j] = 0;
        if (seen) {
            int start2 = s_begin;
            for (int k = y_begin; k < y_end; ++k) {
                const int L = item_len[c_item0 + k];
                for (int j = lane; j < L; j += kWave)
                    colflag[w][kWave + start2 - s_begin + j] =
                        uint32_t((j == 0 ? 1u : 0u) | (uint32_t(k) << 8) | (j == L - 1 ? 0x80000000u : 0u));
                start2 += L;
            }
        }
    }
    __syncthreads();
    const int S = s_end - s_begin;
    if (S > 0) {  // this wave has column items

    const int64_t pbase = g_pair_base[g];
    const int64_t gn = g_n[g];
    const int64_t gitem0 = g_item0[g];
    const bool row_valid = x_task >= 0;
    const bool top = ir == 0;
    const bool last_row = row_valid && ir == nx - 1;
    // The first row of an item has no row above: it adds +inf to whatever the
    // lane above sends (the last row of another item, or a row past the
    // block's frames; lane 0 reads 0).  That lane may be on columns outside its
    // span, where the tile holds values of no use (possibly stale LDS), so the
    // sum may be a quiet NaN; a first row's up neighbour only enters fminf
    // (which returns the other operand for a NaN) and <= tests (false for a
    // NaN, as for +inf below a finite threshold), and its own cost, the one
    // it sends, is always finite on its columns.
    const float top_pen = top ? kInf : 0.0f;
    const float diag_first = top ? 0.0f : kInf;       // virtual c[-1][-1] = 0 at an item start
    const uint32_t pd_first = top ? 0x0000FFFFu : 0u;  // its length interval: Lmin = Lmax = 0
    const int64_t px = row_valid ? int64_t(x_task) - gitem0 : 0;  // row item's position in the group
    // at step t the lane is on column t - ir of the wave's span: distance
    // dcol[t], flags fcol[t], read four steps ahead.  ir <= lane, so dcol[0] is
    // inside the tile; the last read-ahead is at most max_n + 2 <= 66 columns
    // past the span: row 63 then ends 3 floats short of the tile's tail guard,
    // and the flags' zero guard covers it.
    const float *dcol = dt + lane * kDStride + s_begin - ir;
    const uint32_t *fcol = &colflag[w][kWave - ir];
    // a cell is output on the item's last row and last column: flags >=
    // 0x80000000 (flags never reach 0xFFFFFFFF)
    const uint32_t out_min = last_row ? 0x80000000u : 0xFFFFFFFFu;

    // Cells outside a lane's column range are computed too (on guard columns)
    // but never read: the first column of every item resets left and diagonal.
    float c = kInf, up = kInf, up_prev = kInf;
    uint32_t P = 0, Pup = 0, Pup_prev = 0;
    const int steps = S + max_n - 1;
    // A unit with a near-parallel frame pair ORs a "near" bit over each pair's
    // cells (the wavefront's left and up neighbours), and a pair with a near
    // cell goes to the FP64 recheck.
    uint32_t nz = 0;
    auto run = [&](auto careful_tag) {
    constexpr bool careful = decltype(careful_tag)::value;
    auto step = [&](const uint32_t cf, const float dv) {
        const bool first = uint8_t(cf) != 0;
        up = shr1z(c) + top_pen;
        // (lane 0 reads 0: a first row, whose up interval is never taken)
        if (kPath) Pup = shr1uz(P);
        const float diag = first ? diag_first : up_prev;
        const float left = first ? kInf : c;
        const float m = fminf(fminf(diag, left), up);
        if (kPath) {
            const uint32_t Pd = first ? pd_first : Pup_prev;
            const float thr = m + delta;
            const uint32_t sd = diag <= thr ? Pd : 0u;
            const uint32_t sl = left <= thr ? P : 0u;
            const uint32_t su = up <= thr ? Pup : 0u;
            P = pk_step(pk_max(pk_max(sd, sl), su));
        }
        float dvc = dv;
        if constexpr (careful) {
            const uint32_t nup = top ? 0u : shr1uz(nz);
            uint32_t nq;
            if constexpr (kEuclid) {
                nq = __float_as_uint(dv) >> 31;  // marked by the epilogue
                dvc = fabsf(dv);
            } else {
                nq = (dv < kNearD || dv > 1.0f - kNearD) ? 1u : 0u;
            }
            nz = nq | nup | (first ? 0u : nz);
        }
        c = dvc + m;
        up_prev = up;
        Pup_prev = Pup;
        // Pair (x, y) of the group, x the row item: kept when x comes before y
        // (or is y) and written at (x, y) and (y, x), the distance being
        // symmetric (a pair whose path length is ambiguous is flagged in both
        // slots and recomputed in FP64 in each orientation).  Each slot has one
        // writer: the pairs with x after y are written by the unit holding
        // (y, x).
        if (cf >= out_min) {
            const int64_t py = int64_t(c_item0) + ((cf >> 8) & 0x3FFF) - gitem0;
            if (px <= py) {
                const int64_t slot = pbase + px * gn + py, mirror = pbase + py * gn + px;
                float v;
                uint8_t fl = 0;
                if (kPath) {
                    const uint32_t lmax = P >> 16, lmin = 0xFFFFu - (P & 0xFFFFu);
                    v = c * __builtin_amdgcn_rcpf(float(lmin));
                    fl = lmin == lmax ? 0 : 1;
                } else {
                    v = c;
                }
                if (careful && nz && px != py) fl = 1;  // (x, x) is never compared
                if (fl) atomicAdd(nonrobust_n, px < py ? 2u : 1u);
                p32[slot] = v;
                flags[slot] = fl;
                if (px < py) {
                    p32[mirror] = v;
                    flags[mirror] = fl;
                }
            }
        }
    };
    // four steps at a time from one of two register buffers while the other
    // takes the next four (read ahead up to step steps + 3); the buffers
    // alternate, so no values are copied between them
    auto load4 = [&](uint32_t (&f)[4], float (&d)[4], int t0) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            f[k] = fcol[t0 + k];
            d[k] = dcol[t0 + k];
        }
    };
    auto run4 = [&](const uint32_t (&f)[4], const float (&d)[4]) {
#pragma unroll
        for (int k = 0; k < 4; ++k) step(f[k], d[k]);
    };
    auto tail = [&](const uint32_t (&f)[4], const float (&d)[4], int n) {
#pragma unroll
        for (int k = 0; k < 3; ++k)
            if (k < n) step(f[k], d[k]);
    };
    uint32_t fa[4], fb[4];
    float da[4], db[4];
    load4(fa, da, 0);
    for (int t = 0;;) {
        if (t + 4 > steps) {
            tail(fa, da, steps - t);
            break;
        }
        load4(fb, db, t + 4);
        run4(fa, da);
        t += 4;
        if (t + 4 > steps) {
            tail(fb, db, steps - t);
            break;
        }
        load4(fa, da, t + 4);
        run4(fb, db);
        t += 4;
    }
    };
    if (near_s != 0)  // uniform: written before the barrier above
        run(std::true_type{});
    else
        run(std::false_type{});
    }  // S > 0
    __syncthreads();  // the next unit overwrites the LDS tile and column flags
    }
}

// Pooled mode: MFMA Gram tile of pooled unit vectors, angular distance straight
// into the pair matrix (64 x 128 item tile per block).  |cos| above kNearCos
// flags the pair non-robust, for the FP64 recheck.  kEuclid: the Euclidean
// distance of the means from the same cosine and their FP32 lengths (flen).
template <bool kEuclid>
__global__ __launch_bounds__(256, 2) void k_gram_angular_bf16(const uint16_t *__restrict__ xn,
                                                              const float *__restrict__ rinv,
                                                              int dim_pad,
                                                              const int64_t *__restrict__ row0,
                                                              const int64_t *__restrict__ nrows,
                                                              const int64_t *__restrict__ base,
                                                              const int64_t *__restrict__ tile_prefix,
                                                              int64_t n_groups, int64_t n_tiles,
                                                              float *__restrict__ out,
                                                              uint8_t *__restrict__ flags,
                                                              const float *__restrict__ flen) {
    using T = Tile<128>;
    constexpr int kCols = T::kCols;
    __shared__ __attribute__((aligned(16))) unsigned char smem_raw[T::kStageBytes];
    __shared__ __attribute__((aligned(16))) float norm_s[kRows + kCols];
    __shared__ __attribute__((aligned(16))) float len_s[kEuclid ? kRows + kCols : 1];
    for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
    const int64_t g = dev::find_segment_wave(tile_prefix, n_groups, tile);
    const int64_t n = nrows[g];
    const int64_t ntc = (n + kCols - 1) / kCols;
    const int64_t local = tile - tile_prefix[g];
    const int64_t r0 = (local / ntc) * kRows, c0 = (local % ntc) * kCols;
    const int nr = int(min<int64_t>(kRows, n - r0)), nc = int(min<int64_t>(kCols, n - c0));
    NormStage<128> ns, ls;
    ns.load(rinv, row0[g] + r0, nr, row0[g] + c0, nc);
    if constexpr (kEuclid) ls.load(flen, row0[g] + r0, nr, row0[g] + c0, nc);
    f32x16 acc[2][1];
    gram_tile<128>(reinterpret_cast<uint16_t *>(smem_raw), xn, dim_pad, row0[g] + r0, nr, row0[g] + c0, nc, 0,
                   acc, [&] {
                       ns.store(norm_s);
                       if constexpr (kEuclid) ls.store(len_s);
                   });
    const f32x16 &acc0 = acc[0][0], &acc1 = acc[1][0];
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    const int col = 32 * w + lane % 32;
    if (col < nc) {
        const float rc = norm_s[kRows + col];
        float *o = out + base[g];
        uint8_t *fo = flags + base[g];
        // near-parallel (or antiparallel) means: acos is ill-conditioned at
        // |cos| = 1, so such a pair is flagged non-robust and recomputed in FP64
        auto put = [&](int r, float a) {
            const float cs = fminf(fmaxf(a * norm_s[r] * rc, -1.0f), 1.0f);
            const int64_t at = (r0 + r) * n + c0 + col;
            if constexpr (kEuclid) {
                const float lr = len_s[r], lc = len_s[kRows + col], dl = lr - lc;
                o[at] = __builtin_sqrtf(fmaxf(fmaf(dl, dl, 2.0f * lr * lc * (1.0f - cs)), 0.0f));
            } else {
                o[at] = dev::acos_over_pi(cs);
            }
            if (fabsf(cs) > kNearCos) fo[at] = 1;
        };
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int ra = acc_row(i, lane), rb2 = 32 + ra;
            if (ra < nr) put(ra, acc0[i]);
            if (rb2 < nr) put(rb2, acc1[i]);
        }
    }
    __syncthreads();  // the next tile overwrites the inverse norms
    }
}

template <int kC>
void launch_fused(hipStream_t s, const uint16_t *xn, const float *rinv, int dim_pad, const GroupTables &g,
                  const ItemTables &it, const FusedPlan &plan, int norm, float delta, float *p32,
                  uint8_t *flags, unsigned int *nonrobust_n, unsigned int *unit_ctr, const float *flen,
                  const unsigned int *scale) {
    // units are split into 8 contiguous ranges, one per XCD; blocks of XCD x take
    // the units of range x in turn
    const int64_t q = (plan.n_units + 7) / 8;
    int64_t per_xcd = std::min<int64_t>(q, dev::kMaxBlocks / 8);
    if (plan.blocks_per_cu > 0)
        per_xcd = std::min<int64_t>(per_xcd, std::max<int64_t>(1, int64_t(plan.blocks_per_cu) * plan.n_cu / 8));
    const dim3 grid(unsigned(8 * per_xcd)), block(256);
    auto go = [&](auto kernel) {
        hipLaunchKernelGGL(kernel, grid, block, 0, s, xn, rinv, dim_pad, g.item0, g.n_items, g.pair_base, it.len,
                           it.dst, plan.rb, plan.cb, plan.unit_prefix, plan.band_rb, plan.g_cb0, plan.rb_cstart,
                           plan.n_bands, plan.n_units, q, delta, p32, flags, nonrobust_n, unit_ctr, flen, scale);
    };
    const bool path = norm == FABX_NORM_PATH;
    if (flen)
        path ? go(k_fused<kC, true, true>) : go(k_fused<kC, false, true>);
    else
        path ? go(k_fused<kC, true, false>) : go(k_fused<kC, false, false>);
}

}  // namespace

void fused_bf16(hipStream_t s, const uint16_t *xn, const float *rinv, int dim_pad,
                const GroupTables &g, const ItemTables &it, const FusedPlan &plan, int norm,
                float delta, float *p32, uint8_t *flags, unsigned int *nonrobust_n,
                unsigned int *unit_ctr, const float *flen, const unsigned int *scale) {
    if (plan.n_units <= 0) return;
    if (dim_pad % kKc) fail(FABX_EINVAL, "padded dim must be a multiple of 64");
    if (plan.cols == 128)
        launch_fused<128>(s, xn, rinv, dim_pad, g, it, plan, norm, delta, p32, flags, nonrobust_n, unit_ctr,
                          flen, scale);
    else if (plan.cols == 256)
        launch_fused<256>(s, xn, rinv, dim_pad, g, it, plan, norm, delta, p32, flags, nonrobust_n, unit_ctr,
                          flen, scale);
    else
        fail(FABX_EINVAL, "fused kernel column block must be 128 or 256 frames");
    FABX_HIP(hipGetLastError());
}

void gram_angular_bf16(hipStream_t s, const uint16_t *xn, const float *rinv, int dim_pad,
                       const int64_t *row0, const int64_t *nrows, const int64_t *base,
                       const int64_t *tile_prefix, int64_t n_groups, int64_t n_tiles, float *out,
                       uint8_t *flags, const float *flen) {
    if (n_tiles <= 0) return;
    if (dim_pad % kKc) fail(FABX_EINVAL, "padded dim must be a multiple of 64");
    hipLaunchKernelGGL(flen ? k_gram_angular_bf16<true> : k_gram_angular_bf16<false>, dim3(grid_for(n_tiles, 1)),
                       dim3(256), 0, s, xn, rinv, dim_pad, row0, nrows, base, tile_prefix, n_groups, n_tiles, out,
                       flags, flen);
    FABX_HIP(hipGetLastError());
}

}  // namespace kern
}  // namespace fabx
