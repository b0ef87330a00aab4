// Storage-type conversions of pyramid texels (float32, float16, bfloat16 RGBA).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "vct.h"

typedef _Float16 vct_half4 __attribute__((ext_vector_type(4)));
typedef int32_t vct_v4i __attribute__((ext_vector_type(4)));
typedef int32_t vct_v2i __attribute__((ext_vector_type(2)));
typedef float vct_v4f __attribute__((ext_vector_type(4)));

// Buffer resource (V#) words of a structured buffer over the pyramid: one
// record of `texel_bytes` per texel and `n_texels` records, so a load takes the
// 32-bit texel index and the hardware forms the 64-bit address; an index past
// the last record reads as zero.  Word 3 is the untyped 32-bit data format of
// the CDNA buffer descriptor.
inline vct_v4i vct_pyr_rsrc(const void* pyr, int texel_bytes, uint32_t n_texels) {
    const uint64_t base = (uint64_t)(uintptr_t)pyr;
    vct_v4i r;
    r.x = (int32_t)(uint32_t)base;
    r.y = (int32_t)((uint32_t)(base >> 32) & 0xffffu) | (texel_bytes << 16);
    r.z = (int32_t)n_texels;
    r.w = 0x00020000;
    return r;
}

// Raw (byte-offset) resource over the same pyramid, for loads that span two
// neighbouring 8-byte texels: stride 0, `bytes` records of one byte (at most
// 2^32 - 1; dwords past it read as zero).
inline vct_v4i vct_pyr_raw_rsrc(const void* pyr, uint64_t bytes) {
    const uint64_t base = (uint64_t)(uintptr_t)pyr;
    vct_v4i r;
    r.x = (int32_t)(uint32_t)base;
    r.y = (int32_t)((uint32_t)(base >> 32) & 0xffffu);
    r.z = (int32_t)(uint32_t)(bytes > 0xffffffffull ? 0xffffffffull : bytes);
    r.w = 0x00020000;
    return r;
}

// The raw resource r with its base moved `by` bytes forward and its range
// shortened by as much (empty once `by` reaches it), so that an offset o into
// the result reads what offset by + o reads from r.  Used with wave-uniform
// values, where it is a handful of scalar instructions.
__host__ __device__ inline vct_v4i vct_rebase_raw(vct_v4i r, uint64_t by) {
    const uint64_t base = ((uint64_t)(uint32_t)r.x | ((uint64_t)((uint32_t)r.y & 0xffffu) << 32)) + by;
    const uint32_t n = (uint32_t)r.z;
    vct_v4i o;
    o.x = (int32_t)(uint32_t)base;
    o.y = (int32_t)(((uint32_t)(base >> 32) & 0xffffu) | ((uint32_t)r.y & 0xffff0000u));
    o.z = (int32_t)(by < (uint64_t)n ? n - (uint32_t)by : 0u);
    o.w = r.w;
    return o;
}

#ifndef VCT_HOST_EMULATION
// buffer_load_dwordx4 / _dwordx2 with offen (voffset = byte offset)
__device__ vct_v4i vct_raw_load_v4i32(vct_v4i rsrc, int32_t voffset, int32_t soffset,
                                      int32_t aux) __asm("llvm.amdgcn.raw.buffer.load.v4i32");
__device__ vct_v2i vct_raw_load_v2i32(vct_v4i rsrc, int32_t voffset, int32_t soffset,
                                      int32_t aux) __asm("llvm.amdgcn.raw.buffer.load.v2i32");
// buffer_load_dwordx4 / _dwordx2 with idxen (vindex = record index)
__device__ vct_v4f vct_struct_load_v4f32(vct_v4i rsrc, int32_t vindex, int32_t voffset, int32_t soffset,
                                         int32_t aux) __asm("llvm.amdgcn.struct.buffer.load.v4f32");
__device__ vct_v2i vct_struct_load_v2i32(vct_v4i rsrc, int32_t vindex, int32_t voffset, int32_t soffset,
                                         int32_t aux) __asm("llvm.amdgcn.struct.buffer.load.v2i32");
// s_buffer_load_dwordx4 / _dwordx2 (byte offset): a read whose resource and
// offset are the same in every lane of the wave, through the scalar data
// cache into scalar registers; dwords past the resource's range read as zero.
__device__ vct_v4i vct_scalar_load_v4i32(vct_v4i rsrc, int32_t offset,
                                         int32_t aux) __asm("llvm.amdgcn.s.buffer.load.v4i32");
__device__ vct_v2i vct_scalar_load_v2i32(vct_v4i rsrc, int32_t offset,
                                         int32_t aux) __asm("llvm.amdgcn.s.buffer.load.v2i32");
#else
// host-side verification builds supply these
vct_v4i vct_raw_load_v4i32(vct_v4i rsrc, int32_t voffset, int32_t soffset, int32_t aux);
vct_v2i vct_raw_load_v2i32(vct_v4i rsrc, int32_t voffset, int32_t soffset, int32_t aux);
vct_v4f vct_struct_load_v4f32(vct_v4i rsrc, int32_t vindex, int32_t voffset, int32_t soffset, int32_t aux);
vct_v2i vct_struct_load_v2i32(vct_v4i rsrc, int32_t vindex, int32_t voffset, int32_t soffset, int32_t aux);
vct_v4i vct_scalar_load_v4i32(vct_v4i rsrc, int32_t offset, int32_t aux);
vct_v2i vct_scalar_load_v2i32(vct_v4i rsrc, int32_t offset, int32_t aux);
#endif

// float16 / bfloat16 texel from its two 32-bit words (the decode of vct_fetch_texel).
template <int DT>
__device__ __forceinline__ float4 vct_decode_texel(uint32_t x, uint32_t y) {
    if constexpr (DT == VCT_F16) {
        vct_v2i u;
        u.x = (int32_t)x;
        u.y = (int32_t)y;
        const vct_half4 h = __builtin_bit_cast(vct_half4, u);
        return make_float4((float)h.x, (float)h.y, (float)h.z, (float)h.w);
    } else {
        return make_float4(__uint_as_float(x << 16), __uint_as_float(x & 0xffff0000u), __uint_as_float(y << 16),
                           __uint_as_float(y & 0xffff0000u));
    }
}

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

// Fetch-path flag carried in the storage-type template argument: a structured
// buffer load forms its byte offset (index * record size) in 32 bits, so a
// pyramid of more than 4 GiB is read with 64-bit global addresses instead
// (the base address is the one in the resource's first two words).
constexpr int VCT_WIDE = 16;

// Texel `idx` through the pyramid's buffer resource.
template <int DT>
__device__ __forceinline__ float4 vct_fetch_texel(const vct_v4i& rsrc, uint32_t idx) {
    VCT_CHECK_TEXEL(idx);
    if constexpr ((DT & VCT_WIDE) != 0) {
        const uint64_t base = (uint64_t)(uint32_t)rsrc.x | ((uint64_t)((uint32_t)rsrc.y & 0xffffu) << 32);
        return vct_load_texel<DT & ~VCT_WIDE>(reinterpret_cast<const void*>(base), idx);
    } else if constexpr (DT == VCT_F32) {
        const vct_v4f v = vct_struct_load_v4f32(rsrc, (int32_t)idx, 0, 0, 0);
        return make_float4(v.x, v.y, v.z, v.w);
    } else if constexpr (DT == VCT_F16) {
        const vct_v2i u = vct_struct_load_v2i32(rsrc, (int32_t)idx, 0, 0, 0);
        vct_half4 h = __builtin_bit_cast(vct_half4, u);
        return make_float4((float)h.x, (float)h.y, (float)h.z, (float)h.w);
    } else {
        const vct_v2i u = vct_struct_load_v2i32(rsrc, (int32_t)idx, 0, 0, 0);
        const uint32_t x = (uint32_t)u.x, y = (uint32_t)u.y;
        return make_float4(__uint_as_float(x << 16), __uint_as_float(x & 0xffff0000u), __uint_as_float(y << 16),
                           __uint_as_float(y & 0xffff0000u));
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
