// Shared device/host helpers of the SPCG library (gfx950).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace spcg {

enum Dtype : int { DT_F64 = 0, DT_F32 = 1, DT_BF16 = 2, DT_FP8 = 3 };

inline int dtype_bytes(int dt) {
    switch (dt) {
        case DT_F64: return 8;
        case DT_F32: return 4;
        case DT_BF16: return 2;
        case DT_FP8: return 1;
        default: return 0;
    }
}

// Storage tags: the element type in memory and how it widens to float/double.
struct bf16_t {
    uint16_t bits;
};
struct fp8_t {
    uint8_t bits;
};

__device__ __forceinline__ float bf16_bits_to_f32(uint32_t h) { return __uint_as_float(h << 16); }

// OCP e4m3fn: s.eeee.mmm, bias 7.  The 7 magnitude bits placed at bit 20 of
// a binary32 give (1 + m/8) 2^(e - 127) for e > 0 and m 2^-129 for e = 0,
// i.e. the value times 2^-120; one multiply by 2^120 restores it exactly
// (subnormals included).  NaN (0x7f / 0xff) is not decoded; inputs are
// finite by contract.
__device__ __forceinline__ float fp8e4m3_bits_to_f32(uint32_t v) {
    uint32_t u = ((v & 0x7Fu) << 20) | ((v & 0x80u) << 24);
    return __uint_as_float(u) * 1.329227995784916e36f;  // 2^120
}

// ---- wave-level reductions over groups of W lanes (W a power of two <= 64)
template <int W>
__device__ __forceinline__ float group_sum(float v) {
#pragma unroll
    for (int o = W / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, W);
    return v;
}
template <int W>
__device__ __forceinline__ double group_sum(double v) {
#pragma unroll
    for (int o = W / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, W);
    return v;
}

// ---- full-wave sums through DPP (no LDS round trips) ----------------------
// Sum over the 64 lanes, returned uniformly: row_shr 1, 2, 4, 8 leave each
// 16-lane row's total in its lane 15 (lanes shifted in from outside the
// row read 0), row_bcast 15 / 31 fold the rows into lane 63, and readlane
// broadcasts it.  The order of the additions is fixed.
template <int CTRL, int ROWMASK = 0xf>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWMASK, 0xf, true);
}
__device__ __forceinline__ float wave_sum(float v) {
    v += __uint_as_float(dpp_u32<0x111>(__float_as_uint(v)));
    v += __uint_as_float(dpp_u32<0x112>(__float_as_uint(v)));
    v += __uint_as_float(dpp_u32<0x114>(__float_as_uint(v)));
    v += __uint_as_float(dpp_u32<0x118>(__float_as_uint(v)));
    v += __uint_as_float(dpp_u32<0x142, 0xa>(__float_as_uint(v)));
    v += __uint_as_float(dpp_u32<0x143, 0xc>(__float_as_uint(v)));
    return __uint_as_float((uint32_t)__builtin_amdgcn_readlane((int)__float_as_uint(v), 63));
}
template <int CTRL, int ROWMASK = 0xf>
__device__ __forceinline__ double dpp_f64(double v) {
    const uint64_t u = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = dpp_u32<CTRL, ROWMASK>((uint32_t)u);
    const uint32_t hi = dpp_u32<CTRL, ROWMASK>((uint32_t)(u >> 32));
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}
__device__ __forceinline__ double wave_sum(double v) {
    v += dpp_f64<0x111>(v);
    v += dpp_f64<0x112>(v);
    v += dpp_f64<0x114>(v);
    v += dpp_f64<0x118>(v);
    v += dpp_f64<0x142, 0xa>(v);
    v += dpp_f64<0x143, 0xc>(v);
    const uint64_t u = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, 63);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), 63);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// f(std::integral_constant<int, I>) for I = B .. E-1, unrolled at compile time
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
__host__ __device__ inline int64_t round_up(int64_t a, int64_t b) { return ceil_div(a, b) * b; }

}  // namespace spcg
