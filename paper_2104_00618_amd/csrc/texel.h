// Storage-type conversions of pyramid texels (float32, float16, bfloat16 RGBA).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "vct.h"

typedef _Float16 vct_half4 __attribute__((ext_vector_type(4)));

// Index hook for host-side verification builds (empty in the library).
#ifndef VCT_CHECK_TEXEL
#define VCT_CHECK_TEXEL(idx)
#endif

// float32 -> bfloat16 bits, round to nearest even (NaN stays a quiet NaN).
__device__ __forceinline__ uint32_t vct_f32_to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (u >> 16) | 0x40u;
    u += 0x7fffu + ((u >> 16) & 1u);
    return u >> 16;
}

template <int DT>
__device__ __forceinline__ float4 vct_load_texel(const void* __restrict__ pyr, uint32_t idx) {
    VCT_CHECK_TEXEL(idx);
    if constexpr (DT == VCT_F32) {
        return reinterpret_cast<const float4*>(pyr)[idx];
    } else if constexpr (DT == VCT_F16) {
        vct_half4 h = reinterpret_cast<const vct_half4*>(pyr)[idx];
        return make_float4((float)h.x, (float)h.y, (float)h.z, (float)h.w);
    } else {
        uint2 v = reinterpret_cast<const uint2*>(pyr)[idx];
        return make_float4(__uint_as_float(v.x << 16), __uint_as_float(v.x & 0xffff0000u),
                           __uint_as_float(v.y << 16), __uint_as_float(v.y & 0xffff0000u));
    }
}

template <int DT>
__device__ __forceinline__ void vct_store_texel(void* __restrict__ pyr, uint32_t idx, float4 v) {
    VCT_CHECK_TEXEL(idx);
    if constexpr (DT == VCT_F32) {
        reinterpret_cast<float4*>(pyr)[idx] = v;
    } else if constexpr (DT == VCT_F16) {
        vct_half4 h;
        h.x = (_Float16)v.x;
        h.y = (_Float16)v.y;
        h.z = (_Float16)v.z;
        h.w = (_Float16)v.w;
        reinterpret_cast<vct_half4*>(pyr)[idx] = h;
    } else {
        uint2 u;
        u.x = vct_f32_to_bf16(v.x) | (vct_f32_to_bf16(v.y) << 16);
        u.y = vct_f32_to_bf16(v.z) | (vct_f32_to_bf16(v.w) << 16);
        reinterpret_cast<uint2*>(pyr)[idx] = u;
    }
}
