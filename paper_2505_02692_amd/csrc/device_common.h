// Device helpers shared by the HIP kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace fabx {
namespace dev {

constexpr int kWave = 64;

// Launches use at most this many blocks and loop over their work: an AQL
// dispatch holds the grid as a 32-bit count of work-items, so a grid sized by
// the work (pairs, tiles, units) could silently wrap.
constexpr int64_t kMaxBlocks = int64_t(1) << 20;
constexpr float kInf = __builtin_huge_valf();
constexpr float kInvPi = 0.318309886183790671537767526745f;

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

__device__ __forceinline__ int wave_any(int pred) { return __any(pred); }

// Index g with prefix[g] <= id < prefix[g + 1] (prefix has n + 1 ascending entries).
__device__ __forceinline__ int64_t find_segment(const int64_t *__restrict__ prefix, int64_t n,
                                                int64_t id) {
    int64_t lo = 0, hi = n;  // answer in [lo, hi)
    while (hi - lo > 1) {
        int64_t mid = (lo + hi) >> 1;
        if (prefix[mid] <= id) lo = mid; else hi = mid;
    }
    return lo;
}

// The same search done by a whole wave: each step compares `id` with 64 pivots
// spread over the remaining range, one per lane, and keeps the part between the
// last pivot at or below `id` and the next pivot, so about log64(n) dependent
// loads instead of log2(n) (three for up to 250,000 segments).  Every lane
// must pass the same arguments and gets the result; prefix[0] <= id.
__device__ __forceinline__ int64_t find_segment_wave(const int64_t *__restrict__ prefix, int64_t n,
                                                     int64_t id) {
    const int lane = threadIdx.x % kWave;
    int64_t lo = 0, hi = n;  // answer in [lo, hi)
    while (hi - lo > 1) {
        const int64_t span = hi - lo;
        const int64_t p = lo + (span * lane + 63) / 64;
        const bool le = p < hi && prefix[p] <= id;
        const unsigned long long ball = __ballot(le);  // bit 0 set: prefix[lo] <= id
        const int kmax = 63 - __clzll(ball);
        const int64_t nlo = lo + (span * kmax + 63) / 64;
        const int64_t nhi = kmax == 63 ? hi : min(hi, lo + (span * (kmax + 1) + 63) / 64);
        lo = nlo;
        hi = nhi;
    }
    return lo;
}

// float -> bf16 bits, round to nearest even (finite inputs).
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return uint16_t(u >> 16);
}

__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float(uint32_t(h) << 16); }

template <typename T>
__device__ __forceinline__ float load_as_f32(const T *p);
template <>
__device__ __forceinline__ float load_as_f32<float>(const float *p) { return *p; }
template <>
__device__ __forceinline__ float load_as_f32<uint16_t>(const uint16_t *p) { return bf16_to_f32(*p); }

// acos(x) / pi for x in [-1, 1], from Abramowitz & Stegun formula 4.4.46:
// acos(x) = sqrt(1 - x) * (a0 + a1 x + ... + a7 x^7) + e, |e| <= 2e-8 on [0, 1],
// with acos(-x) = pi - acos(x).  The coefficients below are the published
// ones divided by pi.
__device__ __forceinline__ float acos_over_pi(float x) {
    const float ax = fminf(fabsf(x), 1.0f);
    float p = -0.0012624911f * kInvPi;
    p = fmaf(p, ax, 0.0066700901f * kInvPi);
    p = fmaf(p, ax, -0.0170881256f * kInvPi);
    p = fmaf(p, ax, 0.0308918810f * kInvPi);
    p = fmaf(p, ax, -0.0501743046f * kInvPi);
    p = fmaf(p, ax, 0.0889789874f * kInvPi);
    p = fmaf(p, ax, -0.2145988016f * kInvPi);
    p = fmaf(p, ax, 1.5707963050f * kInvPi);
    // hardware square root (about 1 ulp); its error is far below the
    // polynomial's and the BF16 operands'
    const float r = __builtin_amdgcn_sqrtf(1.0f - ax) * p;
    return x < 0.0f ? 1.0f - r : r;
}

// acos_over_pi from ax = |x| (at most 1) and the sign of x, taken from s,
// with the reflection folded into the last steps: r = acos(ax) / pi as above
// lies in [0, 1/2], so h = r - 1/2 <= 0 and acos(x) / pi = 1/2 - copysign(h, s)
// (r for x >= 0, 1 - r below).  One fused multiply-add, a sign transfer and a
// subtraction replace the product, the subtraction and the select (the result
// moves by at most one rounding of a value below 1).  ax arrives in a
// register, so the multiply-adds take their coefficients as literals.
__device__ __forceinline__ float acos_over_pi_abs(float ax, float s) {
    float p = -0.0012624911f * kInvPi;
    p = fmaf(p, ax, 0.0066700901f * kInvPi);
    p = fmaf(p, ax, -0.0170881256f * kInvPi);
    p = fmaf(p, ax, 0.0308918810f * kInvPi);
    p = fmaf(p, ax, -0.0501743046f * kInvPi);
    p = fmaf(p, ax, 0.0889789874f * kInvPi);
    p = fmaf(p, ax, -0.2145988016f * kInvPi);
    p = fmaf(p, ax, 1.5707963050f * kInvPi);
    const float h = fmaf(__builtin_amdgcn_sqrtf(1.0f - ax), p, -0.5f);
    return 0.5f - copysignf(h, s);
}

}  // namespace dev
}  // namespace fabx
