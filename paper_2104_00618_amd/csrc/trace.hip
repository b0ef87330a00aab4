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

// COUNT: no output; count[0] += the cone samples taken, and with two
// counters count[1] += those that read two levels.
template <int DT, bool COUNT, bool ANISO>
__global__ __launch_bounds__(256) void k_trace(TraceArgs a, float4* __restrict__ out,
                                               unsigned long long* __restrict__ count, int n_counts) {
    __shared__ LevelTable T;
    __shared__ DirSlot<ANISO> D;
    __shared__ unsigned long long s_cnt[2];
    load_level_table(a, &T);
    load_dir_table(a, &D);
    if (COUNT && threadIdx.x < 2) s_cnt[threadIdx.x] = 0;
    __syncthreads();

    const int tile = xcd_tile(blockIdx.x, a.n_tiles);
    int view, y, x;
    tile_pixel(a, tile, threadIdx.x, view, y, x);
    const bool inb = x < a.w && y < a.h;
    unsigned int ksum = 0, k2sum = 0;
    float4 o0, o1;
    const size_t pix = ((size_t)view * a.h + y) * a.w + x;
    if (inb) trace_pixel<DT, ANISO>(a, T, view, pix, o0, o1, ksum, k2sum, dir_ptr(D));
    if constexpr (COUNT) {
        if (ksum) atomicAdd(&s_cnt[0], (unsigned long long)ksum);
        if (k2sum) atomicAdd(&s_cnt[1], (unsigned long long)k2sum);
        __syncthreads();
        if ((int)threadIdx.x < n_counts && s_cnt[threadIdx.x]) atomicAdd(&count[threadIdx.x], s_cnt[threadIdx.x]);
    } else {
        if (inb) {
            out[2 * pix] = o0;
            out[2 * pix + 1] = o1;
        }
    }
}

__global__ void k_zero_u64(unsigned long long* p, int n) {
    if ((int)threadIdx.x < n) p[threadIdx.x] = 0ull;
}

template <int DT, bool ANISO>
hipError_t run_trace(const TraceArgs& a, float* out, unsigned long long* count, int n_counts, hipStream_t s,
                     EventSink& es) {
    dim3 grid(a.n_tiles), block(256);
    if (count) {
        es.mark(s);
        hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, count, n_counts);
        if (a.n_tiles > 0) {
            es.mark(s);
            hipLaunchKernelGGL((k_trace<DT, true, ANISO>), grid, block, 0, s, a, nullptr, count, n_counts);
        }
    } else if (a.n_tiles > 0) {
        es.mark(s);
        hipLaunchKernelGGL((k_trace<DT, false, ANISO>), grid, block, 0, s, a, reinterpret_cast<float4*>(out),
                           nullptr, 0);
    }
    es.mark(s);
    return hipGetLastError();
}

template <int DT>
hipError_t run_trace_any(const TraceArgs& a, float* out, unsigned long long* count, int n_counts, hipStream_t s,
                         EventSink& es) {
    return a.aniso ? run_trace<DT, true>(a, out, count, n_counts, s, es)
                   : run_trace<DT, false>(a, out, count, n_counts, s, es);
}

}  // namespace

hipError_t vct_launch_trace(const TraceArgs& a, int dtype, float* out, unsigned long long* count, int n_counts,
                            hipStream_t s, EventSink& es) {
    return vct_dispatch_dt(dtype, a.wide != 0, [&](auto dt) {
        return run_trace_any<decltype(dt)::value>(a, out, count, n_counts, s, es);
    });
}
