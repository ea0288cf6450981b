// Frame normalisation and time pooling.
//
// The angular distance only depends on directions, so every frame is scaled
// to unit length once and packed in task order (frames of a BY group are
// contiguous, row stride padded to a multiple of 64 with zeros) so that a
// group's frame-distance matrix is one dense Gram product.  For the Euclidean
// distance the frames (or means) are packed the same way, unscaled.
//
// out_form: kUnitF32 (FP32 unit rows), kUnitBF16 (BF16 unit rows + 1 / norm
// of the rounded row), kRawF32 (FP32 rows as they are; no zero-norm check,
// since a zero vector has a length), kUnitBF16Len (the BF16 form of the
// Euclidean distance: kUnitBF16 plus each row's FP32 length and the largest
// length over all rows; a zero row is legal there and packs as zeros with
// 1 / norm = 0).
//
// HBM-bound: one read of each feature row, one write of the packed row.
// One 256-thread block per task item, each wave takes every 4th frame.
#include "device_common.h"
#include "kernels.h"

namespace fabx {
namespace kern {
namespace {

using dev::kWave;

constexpr int kUnitF32 = 0, kUnitBF16 = 1, kRawF32 = 2, kUnitBF16Len = 3;

template <typename Tin>
__device__ __forceinline__ void load_row_chunk(const Tin *row, int k, int dim, float v[4]);

template <>
__device__ __forceinline__ void load_row_chunk<float>(const float *row, int k, int dim, float v[4]) {
    if (k + 3 < dim && (dim & 3) == 0) {
        float4 q = *reinterpret_cast<const float4 *>(row + k);
        v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
    } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] = (k + e < dim) ? row[k + e] : 0.0f;
    }
}

template <>
__device__ __forceinline__ void load_row_chunk<uint16_t>(const uint16_t *row, int k, int dim, float v[4]) {
    if (k + 3 < dim && (dim & 3) == 0) {
        uint2 q = *reinterpret_cast<const uint2 *>(row + k);
        v[0] = __uint_as_float(q.x << 16);
        v[1] = __uint_as_float(q.x & 0xFFFF0000u);
        v[2] = __uint_as_float(q.y << 16);
        v[3] = __uint_as_float(q.y & 0xFFFF0000u);
    } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] = (k + e < dim) ? dev::bf16_to_f32(row[k + e]) : 0.0f;
    }
}

// Scale one row held as 4-element chunks (k = 4 * (lane + 64 * c)) and store it.
template <int kChunks>
__device__ __forceinline__ void store_unit_row(float (&v)[kChunks][4], float ss, int lane, int dim_pad,
                                               int64_t out_row, void *out, int out_form,
                                               float *rinv) {
    const float r = out_form == kRawF32 ? 1.0f : ss > 0.0f ? 1.0f / __builtin_sqrtf(ss) : 0.0f;
    if (out_form != kUnitBF16 && out_form != kUnitBF16Len) {
        float *o = static_cast<float *>(out) + out_row * dim_pad;
#pragma unroll
        for (int c = 0; c < kChunks; ++c) {
            int k = 4 * (lane + kWave * c);
            if (k < dim_pad)
                *reinterpret_cast<float4 *>(o + k) =
                    make_float4(v[c][0] * r, v[c][1] * r, v[c][2] * r, v[c][3] * r);
        }
    } else {
        uint16_t *o = static_cast<uint16_t *>(out) + out_row * dim_pad;
        float ss16 = 0.0f;
#pragma unroll
        for (int c = 0; c < kChunks; ++c) {
            int k = 4 * (lane + kWave * c);
            if (k < dim_pad) {
                uint16_t h[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    h[e] = dev::f32_to_bf16(v[c][e] * r);
                    float b = dev::bf16_to_f32(h[e]);
                    ss16 = fmaf(b, b, ss16);
                }
                uint2 q;
                q.x = uint32_t(h[0]) | (uint32_t(h[1]) << 16);
                q.y = uint32_t(h[2]) | (uint32_t(h[3]) << 16);
                *reinterpret_cast<uint2 *>(o + k) = q;
            }
        }
        ss16 = dev::wave_sum(ss16);
        if (lane == 0) rinv[out_row] = ss16 > 0.0f ? 1.0f / __builtin_sqrtf(ss16) : 0.0f;
    }
}

// Largest row length of a block into *scale (FP32 bits; lengths are >= 0, so
// their bit patterns order like the values): one atomic per block.
__device__ __forceinline__ void block_max_to(float m, unsigned int *scale) {
    __shared__ float wmax[4];
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, kWave));
    if (lane == 0) wmax[wave] = m;
    __syncthreads();
    if (threadIdx.x == 0)
        atomicMax(scale, __float_as_uint(fmaxf(fmaxf(wmax[0], wmax[1]), fmaxf(wmax[2], wmax[3]))));
}

// kChunks * 256 >= dim_pad: each lane keeps its 4 * kChunks elements in registers.
template <typename Tin, int kChunks>
__global__ __launch_bounds__(256) void k_normalize(const Tin *__restrict__ src, int dim, int dim_pad,
                                                   const int64_t *__restrict__ item_src,
                                                   const int32_t *__restrict__ item_len,
                                                   const int64_t *__restrict__ item_dst,
                                                   void *out, int out_form, float *rinv, int *err,
                                                   int64_t n_items, unsigned long long *err_item,
                                                   float *len_out, unsigned int *scale) {
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    float lmax = 0.0f;  // kUnitBF16Len: the largest row length this thread saw
    for (int64_t item = blockIdx.x; item < n_items; item += gridDim.x) {
    const int L = item_len[item];
    const int64_t s0 = item_src[item], d0 = item_dst[item];
    // two frames per wave in flight (t and t + 4) to keep more loads outstanding
    for (int t = wave; t < L; t += 8) {
        const bool two = t + 4 < L;
        const Tin *row0 = src + (s0 + t) * int64_t(dim);
        const Tin *row1 = src + (s0 + (two ? t + 4 : t)) * int64_t(dim);
        float v[kChunks][4], u[kChunks][4];
#pragma unroll
        for (int c = 0; c < kChunks; ++c) {
            const int k = 4 * (lane + kWave * c);
            load_row_chunk<Tin>(row0, k, dim, v[c]);
            load_row_chunk<Tin>(row1, k, dim, u[c]);
        }
        float ss = 0.0f, su = 0.0f;
#pragma unroll
        for (int c = 0; c < kChunks; ++c)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                ss = fmaf(v[c][e], v[c][e], ss);
                su = fmaf(u[c][e], u[c][e], su);
            }
        ss = dev::wave_sum(ss);
        su = dev::wave_sum(su);
        if (out_form == kUnitBF16Len) {
            if (lane == 0) {
                len_out[d0 + t] = __builtin_sqrtf(ss);
                if (two) len_out[d0 + t + 4] = __builtin_sqrtf(su);
            }
            lmax = fmaxf(lmax, __builtin_sqrtf(fmaxf(ss, su)));
        } else if (out_form != kRawF32 && (!(ss > 0.0f) || !(su > 0.0f))) {
            if (lane == 0) {
                atomicExch(err, 1);
                atomicMin(err_item, (unsigned long long)item);
            }
            ss = ss > 0.0f ? ss : 1.0f;
            su = su > 0.0f ? su : 1.0f;
        }
        store_unit_row<kChunks>(v, ss, lane, dim_pad, d0 + t, out, out_form, rinv);
        if (two) store_unit_row<kChunks>(u, su, lane, dim_pad, d0 + t + 4, out, out_form, rinv);
    }
    }
    if (out_form == kUnitBF16Len) block_max_to(lmax, scale);  // uniform over the block
}

template <typename Tin, int kChunks>
__global__ __launch_bounds__(256) void k_pool_normalize(const Tin *__restrict__ src, int dim, int dim_pad,
                                                        const int64_t *__restrict__ item_src,
                                                        const int32_t *__restrict__ item_len,
                                                        int64_t n_items, void *out, int out_form,
                                                        float *rinv, int *err,
                                                        unsigned long long *err_item, float *len_out,
                                                        unsigned int *scale) {
    // one wave per item
    const int lane = threadIdx.x % kWave;
    float lmax = 0.0f;  // kUnitBF16Len: the largest mean length this thread saw
    for (int64_t item = int64_t(blockIdx.x) * 4 + threadIdx.x / kWave; item < n_items;
         item += int64_t(gridDim.x) * 4) {
    const int L = item_len[item];
    const int64_t s0 = item_src[item];
    float v[kChunks][4];
#pragma unroll
    for (int c = 0; c < kChunks; ++c)
#pragma unroll
        for (int e = 0; e < 4; ++e) v[c][e] = 0.0f;
    for (int t = 0; t < L; ++t) {
        const Tin *row = src + (s0 + t) * int64_t(dim);
#pragma unroll
        for (int c = 0; c < kChunks; ++c) {
            float w[4];
            load_row_chunk<Tin>(row, 4 * (lane + kWave * c), dim, w);
#pragma unroll
            for (int e = 0; e < 4; ++e) v[c][e] += w[e];
        }
    }
    const float invL = 1.0f / float(L);
    float ss = 0.0f;
#pragma unroll
    for (int c = 0; c < kChunks; ++c)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            v[c][e] *= invL;
            ss = fmaf(v[c][e], v[c][e], ss);
        }
    ss = dev::wave_sum(ss);
    if (out_form == kUnitBF16Len) {
        if (lane == 0) len_out[item] = __builtin_sqrtf(ss);
        lmax = fmaxf(lmax, __builtin_sqrtf(ss));
    } else if (out_form != kRawF32 && !(ss > 0.0f)) {
        if (lane == 0) {
            atomicExch(err, 1);
            atomicMin(err_item, (unsigned long long)item);
        }
        ss = 1.0f;
    }
    store_unit_row<kChunks>(v, ss, lane, dim_pad, item, out, out_form, rinv);
    }
    if (out_form == kUnitBF16Len) block_max_to(lmax, scale);  // uniform over the block
}

// Discrete units: each task item's int32 codes, copied into task order (one
// block per item at a time).
__global__ __launch_bounds__(256) void k_pack_units(const int32_t *__restrict__ src,
                                                    const int64_t *__restrict__ item_src,
                                                    const int32_t *__restrict__ item_len,
                                                    const int64_t *__restrict__ item_dst, int64_t n_items,
                                                    int32_t *__restrict__ out) {
    for (int64_t item = blockIdx.x; item < n_items; item += gridDim.x) {
        const int L = item_len[item];
        const int64_t s0 = item_src[item], d0 = item_dst[item];
        for (int f = threadIdx.x; f < L; f += blockDim.x) out[d0 + f] = src[s0 + f];
    }
}

// HBM streaming probe with k_normalize's access widths and order: a block takes
// 8 rows at a time, each wave two rows in flight, 16-byte FP32 loads per lane
// and 8-byte BF16 stores, but no arithmetic beyond the conversion: it reads
// 4 x dim and writes 2 x dim_pad bytes per row, the normalise kernel's
// traffic for FP32 input, so the two can be compared and the byte counters
// calibrated on this access pattern.
template <int kChunks>
__global__ __launch_bounds__(256) void k_probe_stream(const float *__restrict__ src, int dim, int dim_pad,
                                                      int64_t n_rows, uint16_t *__restrict__ out) {
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    for (int64_t r0 = int64_t(blockIdx.x) * 8; r0 < n_rows; r0 += int64_t(gridDim.x) * 8) {
        const int64_t ra = r0 + wave, rb = r0 + wave + 4;
        float v[kChunks][4], u[kChunks][4];
#pragma unroll
        for (int c = 0; c < kChunks; ++c) {
            const int k = 4 * (lane + kWave * c);
            load_row_chunk<float>(src + min(ra, n_rows - 1) * int64_t(dim), k, dim, v[c]);
            load_row_chunk<float>(src + min(rb, n_rows - 1) * int64_t(dim), k, dim, u[c]);
        }
        auto put = [&](int64_t row, float (&w)[kChunks][4]) {
            uint16_t *o = out + row * dim_pad;
#pragma unroll
            for (int c = 0; c < kChunks; ++c) {
                const int k = 4 * (lane + kWave * c);
                if (k < dim_pad) {
                    uint2 q;
                    q.x = uint32_t(dev::f32_to_bf16(w[c][0])) | (uint32_t(dev::f32_to_bf16(w[c][1])) << 16);
                    q.y = uint32_t(dev::f32_to_bf16(w[c][2])) | (uint32_t(dev::f32_to_bf16(w[c][3])) << 16);
                    *reinterpret_cast<uint2 *>(o + k) = q;
                }
            }
        };
        if (ra < n_rows) put(ra, v);
        if (rb < n_rows) put(rb, u);
    }
}

template <int kChunks>
void launch_probe(hipStream_t s, const float *src, int dim, int dim_pad, int64_t n_rows, uint16_t *out) {
    hipLaunchKernelGGL(k_probe_stream<kChunks>, dim3(grid_for((n_rows + 7) / 8, 1)), dim3(256), 0, s, src, dim,
                       dim_pad, n_rows, out);
}

template <int kChunks>
void launch_norm(hipStream_t s, const void *features, int dtype, int dim, int dim_pad,
                 const ItemTables &it, void *out, int out_form, float *rinv, int *err,
                 unsigned long long *err_item, float *len_out, unsigned int *scale, bool pooled) {
    if (pooled) {
        dim3 grid(grid_for(it.n_items, 4));
        if (dtype == FABX_DTYPE_F32)
            hipLaunchKernelGGL((k_pool_normalize<float, kChunks>), grid, dim3(256), 0, s,
                               static_cast<const float *>(features), dim, dim_pad, it.src, it.len,
                               it.n_items, out, out_form, rinv, err, err_item, len_out, scale);
        else
            hipLaunchKernelGGL((k_pool_normalize<uint16_t, kChunks>), grid, dim3(256), 0, s,
                               static_cast<const uint16_t *>(features), dim, dim_pad, it.src,
                               it.len, it.n_items, out, out_form, rinv, err, err_item, len_out, scale);
    } else {
        dim3 grid(grid_for(it.n_items, 1));
        if (dtype == FABX_DTYPE_F32)
            hipLaunchKernelGGL((k_normalize<float, kChunks>), grid, dim3(256), 0, s,
                               static_cast<const float *>(features), dim, dim_pad, it.src, it.len,
                               it.dst, out, out_form, rinv, err, it.n_items, err_item, len_out, scale);
        else
            hipLaunchKernelGGL((k_normalize<uint16_t, kChunks>), grid, dim3(256), 0, s,
                               static_cast<const uint16_t *>(features), dim, dim_pad, it.src,
                               it.len, it.dst, out, out_form, rinv, err, it.n_items, err_item, len_out, scale);
    }
    FABX_HIP(hipGetLastError());
}

void dispatch(hipStream_t s, const void *features, int dtype, int dim, int dim_pad,
              const ItemTables &it, void *out, int out_form, float *rinv, int *err,
              unsigned long long *err_item, float *len_out, unsigned int *scale, bool pooled) {
    if (it.n_items <= 0) return;
    // chunks of 256 elements per wave pass
    const int chunks = (dim_pad + 255) / 256;
    switch (chunks) {
        case 1: launch_norm<1>(s, features, dtype, dim, dim_pad, it, out, out_form, rinv, err, err_item, len_out, scale, pooled); break;
        case 2: launch_norm<2>(s, features, dtype, dim, dim_pad, it, out, out_form, rinv, err, err_item, len_out, scale, pooled); break;
        case 3: launch_norm<3>(s, features, dtype, dim, dim_pad, it, out, out_form, rinv, err, err_item, len_out, scale, pooled); break;
        case 4: launch_norm<4>(s, features, dtype, dim, dim_pad, it, out, out_form, rinv, err, err_item, len_out, scale, pooled); break;
        case 5: launch_norm<5>(s, features, dtype, dim, dim_pad, it, out, out_form, rinv, err, err_item, len_out, scale, pooled); break;
        case 6: launch_norm<6>(s, features, dtype, dim, dim_pad, it, out, out_form, rinv, err, err_item, len_out, scale, pooled); break;
        case 7: launch_norm<7>(s, features, dtype, dim, dim_pad, it, out, out_form, rinv, err, err_item, len_out, scale, pooled); break;
        case 8: launch_norm<8>(s, features, dtype, dim, dim_pad, it, out, out_form, rinv, err, err_item, len_out, scale, pooled); break;
        default: fail(FABX_EINVAL, "feature dim above 2048 is not supported");
    }
}

}  // namespace

void normalize(hipStream_t s, const void *features, int dtype, int dim, int dim_pad,
               const ItemTables &it, void *out, int out_form, float *rinv, int *err,
               unsigned long long *err_item, float *len_out, unsigned int *scale) {
    dispatch(s, features, dtype, dim, dim_pad, it, out, out_form, rinv, err, err_item, len_out, scale, false);
}

void probe_stream(hipStream_t s, const float *src, int dim, int64_t n_rows, uint16_t *out) {
    if (n_rows <= 0) return;
    if (dim % 4 != 0 || dim > 2048) fail(FABX_EINVAL, "the streaming probe takes dim a multiple of 4, at most 2048");
    const int dim_pad = int((dim + 63) / 64 * 64);
    switch ((dim_pad + 255) / 256) {
        case 1: launch_probe<1>(s, src, dim, dim_pad, n_rows, out); break;
        case 2: launch_probe<2>(s, src, dim, dim_pad, n_rows, out); break;
        case 3: launch_probe<3>(s, src, dim, dim_pad, n_rows, out); break;
        case 4: launch_probe<4>(s, src, dim, dim_pad, n_rows, out); break;
        case 5: launch_probe<5>(s, src, dim, dim_pad, n_rows, out); break;
        case 6: launch_probe<6>(s, src, dim, dim_pad, n_rows, out); break;
        case 7: launch_probe<7>(s, src, dim, dim_pad, n_rows, out); break;
        default: launch_probe<8>(s, src, dim, dim_pad, n_rows, out); break;
    }
    FABX_HIP(hipGetLastError());
}

void pack_units(hipStream_t s, const int32_t *codes, const ItemTables &it, int32_t *out) {
    if (it.n_items <= 0) return;
    hipLaunchKernelGGL(k_pack_units, dim3(grid_for(it.n_items, 1)), dim3(256), 0, s, codes, it.src, it.len,
                       it.dst, it.n_items, out);
    FABX_HIP(hipGetLastError());
}

void pool_normalize(hipStream_t s, const void *features, int dtype, int dim, int dim_pad,
                    const ItemTables &it, void *out, int out_form, float *rinv, int *err,
                    unsigned long long *err_item, float *len_out, unsigned int *scale) {
    dispatch(s, features, dtype, dim, dim_pad, it, out, out_form, rinv, err, err_item, len_out, scale, true);
}

}  // namespace kern
}  // namespace fabx
