// Forward cone trace: one lane per pixel, each lane marches all cones of its
// pixel (u diffuse, specular, occlusion) and writes the 8-float epilogue
// (D.rgb, D.a, S.rgb, O).  Sections 4.2, 4.3.2, 4.5 and 5.4.4; with an
// anisotropic pyramid the samples weight its directional levels by the cone
// axis (Section 5.1.3).
//
// Launch: 256-thread workgroups over 16x16-pixel tiles (a wave is an 8x8
// quadrant, so the 64 lanes of a wave start from neighbouring surface points
// and, for the fixed-aperture cones, step through the same LOD schedule),
// tiles ordered so that each XCD gets a contiguous run of the image.
#include "march.h"

namespace {

using namespace vct;

template <int DT, bool COUNT, bool ANISO>
__global__ __launch_bounds__(256) void k_trace(TraceArgs a, float4* __restrict__ out,
                                               unsigned long long* __restrict__ count) {
    __shared__ LevelTable T;
    __shared__ DirSlot<ANISO> D;
    __shared__ unsigned long long s_cnt;
    load_level_table(a, &T);
    load_dir_table(a, &D);
    if (COUNT && threadIdx.x == 0) s_cnt = 0;
    __syncthreads();

    const int tile = xcd_tile(blockIdx.x, a.n_tiles);
    int view, y, x;
    tile_pixel(a, tile, threadIdx.x, view, y, x);
    const bool inb = x < a.w && y < a.h;
    unsigned int ksum = 0;
    float4 o0, o1;
    const size_t pix = ((size_t)view * a.h + y) * a.w + x;
    if (inb) trace_pixel<DT, ANISO>(a, T, view, pix, o0, o1, ksum, dir_ptr(D));
    if constexpr (COUNT) {
        if (ksum) atomicAdd(&s_cnt, (unsigned long long)ksum);
        __syncthreads();
        if (threadIdx.x == 0 && s_cnt) atomicAdd(count, s_cnt);
    } else {
        if (inb) {
            out[2 * pix] = o0;
            out[2 * pix + 1] = o1;
        }
    }
}

__global__ void k_zero_u64(unsigned long long* p) { *p = 0ull; }

template <int DT, bool ANISO>
hipError_t run_trace(const TraceArgs& a, float* out, unsigned long long* count, hipStream_t s, EventSink& es) {
    dim3 grid(a.n_tiles), block(256);
    if (count) {
        es.mark(s);
        hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(1), 0, s, count);
        if (a.n_tiles > 0) {
            es.mark(s);
            hipLaunchKernelGGL((k_trace<DT, true, ANISO>), grid, block, 0, s, a, nullptr, count);
        }
    } else if (a.n_tiles > 0) {
        es.mark(s);
        hipLaunchKernelGGL((k_trace<DT, false, ANISO>), grid, block, 0, s, a, reinterpret_cast<float4*>(out),
                           nullptr);
    }
    es.mark(s);
    return hipGetLastError();
}

template <int DT>
hipError_t run_trace_any(const TraceArgs& a, float* out, unsigned long long* count, hipStream_t s, EventSink& es) {
    return a.aniso ? run_trace<DT, true>(a, out, count, s, es) : run_trace<DT, false>(a, out, count, s, es);
}

}  // namespace

hipError_t vct_launch_trace(const TraceArgs& a, int dtype, float* out, unsigned long long* count, hipStream_t s,
                            EventSink& es) {
    return vct_dispatch_dt(dtype, a.wide != 0,
                           [&](auto dt) { return run_trace_any<decltype(dt)::value>(a, out, count, s, es); });
}
