// BF16 form, DTW mode: frame distances on MFMA fused with the DTW wavefront,
// one wave per work unit, each wave streaming a long run of column frames
// past a block of up to 64 row frames.
//
// Work unit = (row block, segment of its column stream) of one BY group.  A
// row block packs whole items into at most 64 frames (lane r = frame row r).
// Its column stream is every frame of the group from the row block's first
// frame on: the pairs (x, y) with x in the row block and y at or after x's
// place in the group are exactly the pairs the symmetric evaluation keeps
// (each is written at (x, y) and (y, x)).  The stream is cut into segments of
// about L frames; a segment starts at the first item that starts in its
// nominal range, so no item straddles two segments.  The wave walks its
// segment in tiles of 64 columns:
//   1. Gram tile on MFMA: 64 column frames x 64 row frames, BF16 operands
//      loaded straight into registers (v_mfma_f32_32x32x16_bf16, FP32
//      accumulation); with the column frames as the first operand, each lane
//      ends up holding one row's distances to 16 columns, four consecutive
//      columns at a time;
//   2. epilogue: cos = S * rinv_row * rinv_col, d = acos(cos) / pi (Abramowitz
//      & Stegun 4.4.46), stored as the 16-bit fixed-point value
//      q = round(65535 d) in a ring of two tiles in LDS;
//   3. 64 DTW steps: lane r is on column t - i_r at step t (i_r = its row index
//      inside its item), so the cell above comes from lane r - 1 one step
//      earlier (one DPP shift) and a lane still behind finds its columns in
//      the previous tile of the ring.  DTW costs are sums of q, exact integers
//      in 32 bits (at most 127 * 65535): the recurrence adds no rounding, and
//      its ties are exact ties of the quantized distances.
// Lanes idle only in the fill at a segment's start and the drain at its end.
//
// Path length (FABX_NORM_PATH): as in the tile kernel, each cell carries the
// interval [Lmin, Lmax] of path lengths over the predecessors within `delta`
// of the minimum (u16 halves: high = Lmax, low = 0xFFFF - Lmin; one packed
// max merges both ends); a pair whose interval is not one value is flagged
// non-robust and recomputed in FP64.
//
// Near-parallel frames: acos is ill-conditioned at cos = +-1, so there the
// BF16 cosine's rounding (about 1e-7) turns into an angle error of order
// 1e-4.  A tile whose distances come within kNearQ / 65535 of 0 or 1 makes the
// DTW rounds that read it also OR a "near" bit over each pair's cells (the
// same wavefront shape: left, up); a pair with such a cell is flagged for the
// FP64 recheck.
#include "device_common.h"
#include "kernels.h"

namespace fabx {
namespace kern {
namespace {

using dev::kWave;

typedef short bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

constexpr int kRows = 64;          // row block frames = DTW lanes
constexpr int kTile = 64;          // columns per tile
constexpr int kRing = 128;         // columns in the ring (two tiles)
constexpr int kPitch = 136;        // u16 per ring row: 272 B, 16-byte aligned, rows 4 banks apart
constexpr float kQScale = 65535.0f;
constexpr uint32_t kInfQ = 0x3FFFFFFFu;      // "no predecessor"
constexpr uint32_t kAboveOr = 0x40000000u;   // the row above belongs to another item
constexpr uint32_t kNearQ = 64;              // |d| or |1 - d| below 64 / 65535 counts as near-parallel

struct WaveLds {
    uint16_t ring[kRows * kPitch];  // q of rows 0..63, ring columns 0..127
    uint32_t fring[kRing];          // frame info of the ring's columns (0: no column)
};

__device__ __forceinline__ uint32_t shr1(uint32_t v) {
    // value of lane - 1 (DPP wave_shr:1, bound_ctrl: lane 0 reads 0)
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
__device__ __forceinline__ uint32_t umin3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_elementwise_min(__builtin_elementwise_min(a, b), c);
}
__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, kWave));
    return v;
}
__device__ __forceinline__ bf16x8 ld8(const uint16_t *p, bool ok) {
    bf16x8 v = {0, 0, 0, 0, 0, 0, 0, 0};
    if (ok) v = *reinterpret_cast<const bf16x8 *>(p);
    return v;
}

template <bool kPath>
__global__ __launch_bounds__(256, 2) void k_stream(const uint16_t *__restrict__ xn, const float *__restrict__ rinv,
                                                   int dim_pad, const uint32_t *__restrict__ finfo,
                                                   const int32_t *__restrict__ rb,
                                                   const int64_t *__restrict__ item_dst,
                                                   const int64_t *__restrict__ g_frame0,
                                                   const int64_t *__restrict__ g_nframes,
                                                   const int64_t *__restrict__ g_n,
                                                   const int64_t *__restrict__ g_pair_base,
                                                   const int64_t *__restrict__ rb_unit_prefix, int64_t n_rb,
                                                   int64_t n_units, int64_t grid_q, int seg_len,
                                                   uint32_t delta_q, float *__restrict__ p32,
                                                   uint8_t *__restrict__ flags,
                                                   unsigned int *__restrict__ nonrobust_n,
                                                   unsigned int *__restrict__ unit_ctr) {
    __shared__ __attribute__((aligned(16))) WaveLds lds_all[4];
    const int lane = threadIdx.x % kWave;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    WaveLds &L = lds_all[w];
    // XCD-aware order: the 8 XCDs take blocks round-robin, so XCD x works
    // through the contiguous unit range [x * grid_q, (x+1) * grid_q): the units
    // of a row block, and the row blocks of a group, run close together in
    // that XCD's L2.  With fewer waves than units in the range, each wave
    // takes the range's next unit from the XCD's counter (zero at launch).
    const int64_t xcd = blockIdx.x % 8;
    const int64_t n_w = int64_t(gridDim.x / 8) * 4;   // waves per XCD
    const bool take = n_w < grid_q;
    auto next = [&](int64_t j) -> int64_t {
        if (!take) return j + n_w;
        unsigned int v = 0;
        if (lane == 0) v = atomicAdd(unit_ctr + xcd, 1u);
        return int64_t(__builtin_amdgcn_readfirstlane(int(v)));
    };
    for (int64_t j = take ? next(0) : int64_t(blockIdx.x / 8) * 4 + w; j < grid_q; j = next(j)) {
        const int64_t u = xcd * grid_q + j;
        if (u >= n_units) break;  // uniform across the wave; later units are beyond too

        // ---- the unit: row block, its stream, the segment's item-aligned bounds
        const int64_t rbi = dev::find_segment_wave(rb_unit_prefix, n_rb, u);
        const int64_t s = u - rb_unit_prefix[rbi];
        const int g = rb[4 * rbi];
        const int n_rows = rb[4 * rbi + 3];
        const int64_t row_f0 = item_dst[rb[4 * rbi + 1]];
        const int64_t S = g_frame0[g] + g_nframes[g] - row_f0;  // stream length
        // first item start at or after a (S past the last one); items are at
        // most 64 frames, so one starts within any 64 frames of the stream
        auto item_start = [&](int64_t a) -> int64_t {
            if (a >= S) return S;
            const int64_t f = a + lane;
            const bool st = f >= S || int32_t(finfo[row_f0 + f]) < 0;
            const unsigned long long b = __ballot(st);
            return a + __builtin_ctzll(b);
        };
        const int64_t a = item_start(s * seg_len);
        const int len = int(item_start((s + 1) * seg_len) - a);
        if (len <= 0) continue;
        const int64_t col_f0 = row_f0 + a;

        // ---- row lanes
        const bool row_valid = lane < n_rows;
        const uint32_t rfi = row_valid ? finfo[row_f0 + lane] : 0u;
        const int ir = row_valid ? int(rfi & 63u) : 0;
        const bool top = ir == 0;
        const bool last_row = row_valid && (rfi & 0x40000000u);
        const int64_t px = int64_t((rfi >> 6) & 0xFFFFFFu);
        const int skew = wave_max(ir);
        const int64_t gn = g_n[g];
        const int64_t pbase = g_pair_base[g];
        // MFMA operands: the first is 32 column frames (lane: column l % 32, k
        // offset 8 (l / 32)), the second 32 row frames; rows past n_rows read as 0
        const int lr = lane % 32, lk = 8 * (lane / 32);
        const uint16_t *brow0 = xn + (row_f0 + lr) * int64_t(dim_pad) + lk;
        const uint16_t *brow1 = xn + (row_f0 + 32 + lr) * int64_t(dim_pad) + lk;
        const bool rv0 = lr < n_rows, rv1 = 32 + lr < n_rows;
        const float rr0 = rv0 ? rinv[row_f0 + lr] : 0.0f;
        const float rr1 = rv1 ? rinv[row_f0 + 32 + lr] : 0.0f;

        // negative columns (lanes behind at the segment's start) read ring half 1:
        // no item starts or ends there
        L.fring[kTile + lane] = 0u;

        const int n_tiles = (len + kTile - 1) / kTile;
        const int total = len + skew;
        const int n_rounds = (total + kTile - 1) / kTile;
        uint32_t near_tiles = 0;  // bit h: ring half h holds a near-parallel distance

        // DTW state of this lane's row
        uint32_t c = kInfQ, P = 0u, up_prev = kInfQ, Pup_prev = 0u, nz = 0u;
        const uint32_t above_or = top ? kAboveOr : 0u;       // the row above is another item
        const uint32_t above_and = top ? 0u : 0xFFFFFFFFu;
        const uint32_t diag_first = top ? 0u : kInfQ;        // virtual c[-1][-1] = 0 at an item start
        const uint32_t pd_first = top ? 0x0000FFFFu : 0u;    // its length interval: Lmin = Lmax = 0
        const uint32_t out_mask = last_row ? 0x40000000u : 0u;
        const uint16_t *qrow = L.ring + lane * kPitch;

        for (int k = 0; k < n_rounds; ++k) {
            const int half = k & 1;
            if (k < n_tiles) {
                // ---- 1. Gram tile k: columns [64k, 64k + 64) of the segment
                const int cc0 = kTile * k + lr, cc1 = cc0 + 32;
                const bool cv0 = cc0 < len, cv1 = cc1 < len;
                const uint16_t *acol0 = xn + (col_f0 + cc0) * int64_t(dim_pad) + lk;
                const uint16_t *acol1 = xn + (col_f0 + cc1) * int64_t(dim_pad) + lk;
                f32x16 acc00, acc01, acc10, acc11;
#pragma unroll
                for (int i = 0; i < 16; ++i) acc00[i] = acc01[i] = acc10[i] = acc11[i] = 0.0f;
                bf16x8 A0 = ld8(acol0, cv0), A1 = ld8(acol1, cv1), B0 = ld8(brow0, rv0), B1 = ld8(brow1, rv1);
                for (int kk = 0; kk < dim_pad; kk += 16) {
                    bf16x8 nA0 = A0, nA1 = A1, nB0 = B0, nB1 = B1;
                    if (kk + 16 < dim_pad) {
                        nA0 = ld8(acol0 + kk + 16, cv0);
                        nA1 = ld8(acol1 + kk + 16, cv1);
                        nB0 = ld8(brow0 + kk + 16, rv0);
                        nB1 = ld8(brow1 + kk + 16, rv1);
                    }
                    acc00 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A0, B0, acc00, 0, 0, 0);
                    acc01 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A0, B1, acc01, 0, 0, 0);
                    acc10 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A1, B0, acc10, 0, 0, 0);
                    acc11 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A1, B1, acc11, 0, 0, 0);
                    A0 = nA0;
                    A1 = nA1;
                    B0 = nB0;
                    B1 = nB1;
                }
                // ---- 2. epilogue: lane holds row 32h + l % 32 against columns
                // 32 ct + 8 (v / 4) + 4 (l / 32) + v % 4 of the tile
                bool near = false;
                auto epi = [&](const f32x16 &acc, int ct, int h, float rr) {
                    uint16_t *dst = L.ring + (32 * h + lr) * kPitch + kTile * half + 32 * ct + 4 * (lane / 32);
#pragma unroll
                    for (int gq = 0; gq < 4; ++gq) {
                        const int col = kTile * k + 32 * ct + 8 * gq + 4 * (lane / 32);  // segment column
                        float rc[4];
                        if (col + 3 < len) {
                            const float4 v = *reinterpret_cast<const float4 *>(rinv + col_f0 + col);
                            rc[0] = v.x; rc[1] = v.y; rc[2] = v.z; rc[3] = v.w;
                        } else {
#pragma unroll
                            for (int e = 0; e < 4; ++e) rc[e] = col + e < len ? rinv[col_f0 + col + e] : 0.0f;
                        }
                        uint32_t q[4];
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            const float cs = fminf(fmaxf(acc[4 * gq + e] * rr * rc[e], -1.0f), 1.0f);
                            q[e] = uint32_t(__builtin_rintf(dev::acos_over_pi(cs) * kQScale));
                            near |= (q[e] - kNearQ) > (65535u - 2u * kNearQ);  // q < 64 or q > 65471
                        }
                        *reinterpret_cast<uint2 *>(dst + 8 * gq) = make_uint2(q[0] | (q[1] << 16), q[2] | (q[3] << 16));
                    }
                };
                epi(acc00, 0, 0, rr0);
                epi(acc01, 0, 1, rr1);
                epi(acc10, 1, 0, rr0);
                epi(acc11, 1, 1, rr1);
                // rows past n_rows hold products with zero rows: never read by a valid lane
                const bool nr_any = __ballot(near && (lr < n_rows)) != 0;
                near_tiles = (near_tiles & ~(1u << half)) | (nr_any ? (1u << half) : 0u);
                const int cc = kTile * k + lane;
                L.fring[kTile * half + lane] = cc < len ? finfo[col_f0 + cc] : 0u;
            } else {
                L.fring[kTile * half + lane] = 0u;  // drain: columns past the segment
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();

            // ---- 3. DTW steps [64k, 64k + 64) of the segment
            const int t0 = kTile * k, t1 = min(t0 + kTile, total);
            const bool careful = near_tiles != 0;  // this round reads a tile with near-parallel frames
            auto step = [&](uint32_t q, uint32_t cf) {
                const bool first = int32_t(cf) < 0;
                const uint32_t up = shr1(c) | above_or;
                const uint32_t diag = first ? diag_first : up_prev;
                const uint32_t left = first ? kInfQ : c;
                const uint32_t m = umin3(diag, left, up);
                if (kPath) {
                    const uint32_t Pup = shr1(P);
                    const uint32_t Pd = first ? pd_first : Pup_prev;
                    const uint32_t thr = m + delta_q;
                    const uint32_t sd = diag <= thr ? Pd : 0u;
                    const uint32_t sl = left <= thr ? P : 0u;
                    const uint32_t su = up <= thr ? Pup : 0u;
                    P = pk_step(pk_max(pk_max(sd, sl), su));
                    Pup_prev = Pup;
                }
                if (careful) {
                    // near bit ORed over the pair's cells so far (left, up)
                    const uint32_t nup = shr1(nz) & above_and;
                    const uint32_t nq = (q - kNearQ) > (65535u - 2u * kNearQ) ? 1u : 0u;
                    nz = nq | nup | (first ? 0u : nz);
                }
                c = q + m;
                up_prev = up;
                if (cf & out_mask) {
                    // pair (x, y): x = this lane's item, y = the column's item (its
                    // place in the group); kept when x is at or before y and
                    // written at (x, y) and (y, x)
                    const int64_t py = int64_t((cf >> 6) & 0xFFFFFFu);
                    if (px <= py) {
                        float v;
                        uint8_t fl = 0;
                        if (kPath) {
                            const uint32_t lmax = P >> 16, lmin = 0xFFFFu - (P & 0xFFFFu);
                            v = float(c) * __builtin_amdgcn_rcpf(kQScale * float(lmin));
                            fl = lmin == lmax ? 0 : 1;
                        } else {
                            v = float(c) * (1.0f / kQScale);
                        }
                        if (careful && nz) fl = 1;
                        if (fl) atomicAdd(nonrobust_n, px < py ? 2u : 1u);
                        const int64_t slot = pbase + px * gn + py, mirror = pbase + py * gn + px;
                        p32[slot] = v;
                        flags[slot] = fl;
                        if (px < py) {
                            p32[mirror] = v;
                            flags[mirror] = fl;
                        }
                    }
                }
            };
            // column t - ir of the segment at step t; reads run two steps ahead
            int t = t0;
            int ci = (t - ir) & (kRing - 1);
            uint32_t qa = qrow[ci], fa = L.fring[ci];
            ci = (t + 1 - ir) & (kRing - 1);
            uint32_t qb = qrow[ci], fb = L.fring[ci];
            for (; t + 1 < t1; t += 2) {
                const uint32_t q0 = qa, f0 = fa, q1 = qb, f1 = fb;
                ci = (t + 2 - ir) & (kRing - 1);
                qa = qrow[ci];
                fa = L.fring[ci];
                ci = (t + 3 - ir) & (kRing - 1);
                qb = qrow[ci];
                fb = L.fring[ci];
                step(q0, f0);
                step(q1, f1);
            }
            if (t < t1) step(qa, fa);
            // the next tile overwrites the ring half this round's lagging lanes read
            __builtin_amdgcn_wave_barrier();
        }
    }
}

__global__ __launch_bounds__(256) void k_frame_info(const int64_t *__restrict__ item_dst,
                                                    const int32_t *__restrict__ item_len,
                                                    const int32_t *__restrict__ item_group,
                                                    const int64_t *__restrict__ g_item0, int64_t n_items,
                                                    uint32_t *__restrict__ finfo) {
    for (int64_t i = int64_t(blockIdx.x) * 4 + threadIdx.x / kWave; i < n_items; i += int64_t(gridDim.x) * 4) {
        const int lane = threadIdx.x % kWave;
        const int len = item_len[i];
        const uint32_t pos = uint32_t(i - g_item0[item_group[i]]);
        if (lane < len)
            finfo[item_dst[i] + lane] = (lane == 0 ? 0x80000000u : 0u) | (lane == len - 1 ? 0x40000000u : 0u) |
                                        (pos << 6) | uint32_t(lane);
    }
}

}  // namespace

void frame_info(hipStream_t s, const ItemTables &it, const int32_t *item_group, const int64_t *g_item0,
                uint32_t *finfo) {
    if (it.n_items <= 0) return;
    hipLaunchKernelGGL(k_frame_info, dim3(grid_for(it.n_items, 4)), dim3(256), 0, s, it.dst, it.len, item_group,
                       g_item0, it.n_items, finfo);
    FABX_HIP(hipGetLastError());
}

void stream_bf16(hipStream_t s, const uint16_t *xn, const float *rinv, int dim_pad, const uint32_t *finfo,
                 const GroupTables &g, const ItemTables &it, const StreamPlan &plan, int norm, uint32_t delta_q,
                 float *p32, uint8_t *flags, unsigned int *nonrobust_n, unsigned int *unit_ctr) {
    if (plan.n_units <= 0) return;
    if (dim_pad % 16) fail(FABX_EINVAL, "padded dim must be a multiple of 16");
    if (plan.seg_len < kTile) fail(FABX_EINVAL, "stream segment shorter than an item can be");
    // units are split into 8 contiguous ranges, one per XCD; the 4 waves of a
    // block take the units of their XCD's range in turn
    const int64_t q = (plan.n_units + 7) / 8;
    int64_t blocks_per_xcd = std::min<int64_t>((q + 3) / 4, dev::kMaxBlocks / 8);
    if (plan.blocks_per_cu > 0)
        blocks_per_xcd = std::min<int64_t>(blocks_per_xcd, std::max<int64_t>(1, int64_t(plan.blocks_per_cu) * plan.n_cu / 8));
    const dim3 grid(unsigned(8 * blocks_per_xcd)), block(256);
    if (norm == FABX_NORM_PATH)
        hipLaunchKernelGGL((k_stream<true>), grid, block, 0, s, xn, rinv, dim_pad, finfo, plan.rb, it.dst,
                           g.frame0, g.n_frames, g.n_items, g.pair_base, plan.rb_unit_prefix, plan.n_rb,
                           plan.n_units, q, plan.seg_len, delta_q, p32, flags, nonrobust_n, unit_ctr);
    else
        hipLaunchKernelGGL((k_stream<false>), grid, block, 0, s, xn, rinv, dim_pad, finfo, plan.rb, it.dst,
                           g.frame0, g.n_frames, g.n_items, g.pair_base, plan.rb_unit_prefix, plan.n_rb,
                           plan.n_units, q, plan.seg_len, delta_q, p32, flags, nonrobust_n, unit_ctr);
    FABX_HIP(hipGetLastError());
}

}  // namespace kern
}  // namespace fabx
