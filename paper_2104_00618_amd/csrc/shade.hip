// Final shading with the thesis's cone variants (Section 5.4.4, "Cone Tracing"):
// per G-buffer pixel, u diffuse cones (optionally stopping at the first
// sample whose alpha exceeds a threshold and returning its colour), one
// specular cone weighted per light by the angular-grace BRDF, and one
// occlusion cone per light (optionally with each sampled alpha scaled by a
// Hermite step of sqrt(distance) times a shadow strength), combined as
//   L = o_min * sum_q w_q C_diff,q + sum_s f_spec,s C_spec
//       + sum_s V_s (c_d i_d,s max(0, L_s.N) + c_s i_s,s max(0, R_s.w)^shininess),
// V_s = 1 - occlusion alpha, o_min = min_s V_s.  Output float4 (L.rgb, o_min).
//
// The specular cone is traced once: every light's specular cone has the same
// axis and aperture, so the per-light traces of the thesis are one trace
// weighted by the sum of the per-light BRDF values.
//
// Launch: the tiles, waves and XCD order of the forward trace.  With an
// anisotropic pyramid every cone samples its directional levels (Section 5.1.3).
#include "shade_pixel.h"

namespace {

using namespace vct;

// COUNT: instead of the shaded pixels, add the number of cone samples every
// march takes (diffuse, specular, one occlusion cone per light) to *count.
template <int DT, bool ANISO, bool COUNT>
__global__ __launch_bounds__(256) void k_shade(TraceArgs a, ShadeArgs s, float4* __restrict__ out,
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
    const size_t pix = ((size_t)view * a.h + y) * a.w + x;
    unsigned int n = 0;
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (inb) {
        const float4 nr = a.normal[pix];
        if (nr.w != 0.0f) v = shade_pixel<DT, ANISO>(a, T, dir_ptr(D), s, view, pix, nr, n);
    }
    if constexpr (COUNT) {
        if (n) atomicAdd(&s_cnt, (unsigned long long)n);
        __syncthreads();
        if (threadIdx.x == 0 && s_cnt) atomicAdd(count, s_cnt);
    } else {
        if (inb) out[pix] = v;
    }
}

__global__ void k_zero_count(unsigned long long* p) { *p = 0ull; }

template <int DT, bool ANISO>
void launch_shade(const TraceArgs& a, const ShadeArgs& s, float* out, unsigned long long* count, hipStream_t st) {
    if (count)
        hipLaunchKernelGGL((k_shade<DT, ANISO, true>), dim3(a.n_tiles), dim3(256), 0, st, a, s, nullptr, count);
    else
        hipLaunchKernelGGL((k_shade<DT, ANISO, false>), dim3(a.n_tiles), dim3(256), 0, st, a, s,
                           reinterpret_cast<float4*>(out), nullptr);
}

template <int DT>
hipError_t run_shade(const TraceArgs& a, const ShadeArgs& s, float* out, unsigned long long* count, hipStream_t st,
                     EventSink& es) {
    if (count) {
        es.mark(st);
        hipLaunchKernelGGL(k_zero_count, dim3(1), dim3(1), 0, st, count);
    }
    if (a.n_tiles > 0) {
        es.mark(st);
        if (a.aniso)
            launch_shade<DT, true>(a, s, out, count, st);
        else
            launch_shade<DT, false>(a, s, out, count, st);
    }
    es.mark(st);
    return hipGetLastError();
}

}  // namespace

hipError_t vct_launch_shade(const TraceArgs& a, int dtype, const vct_shade_params* p, const float* material,
                            float* out, unsigned long long* count, hipStream_t st, EventSink& es) {
    ShadeArgs s{};
    s.n_lights = p->n_lights;
    const double scale = (double)a.scale_hi + (double)a.scale_lo;
    for (int l = 0; l < p->n_lights; ++l)
        for (int i = 0; i < 3; ++i) {
            const double lt = ((double)p->light_pos[l][i] - (double)a.origin[i]) * scale;
            s.light_tex[l][i][0] = (float)lt;
            s.light_tex[l][i][1] = (float)(lt - (double)s.light_tex[l][i][0]);
            s.light_pos[l][i] = p->light_pos[l][i];
            s.light_diffuse[l][i] = p->light_diffuse[l][i];
            s.light_specular[l][i] = p->light_specular[l][i];
        }
    for (int i = 0; i < 3; ++i) s.specular_color[i] = p->specular_color[i];
    s.first_hit = p->diffuse_first_hit != 0;
    s.falloff = p->occlusion_falloff != 0;
    s.brdf = p->specular_brdf != 0;
    s.first_hit_alpha = p->first_hit_alpha;
    s.shadow_strength = p->shadow_strength;
    s.grace = p->grace_per_shininess;
    s.q = p->shininess_falloff;
    s.material = reinterpret_cast<const float4*>(material);
    return vct_dispatch_dt(dtype, a.wide != 0,
                           [&](auto dt) { return run_shade<decltype(dt)::value>(a, s, out, count, st, es); });
}
