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

template <int DT, bool ANISO>
__global__ __launch_bounds__(256) void k_shade(TraceArgs a, ShadeArgs s, float4* __restrict__ out) {
    __shared__ LevelTable T;
    __shared__ DirSlot<ANISO> D;
    load_level_table(a, &T);
    load_dir_table(a, &D);
    __syncthreads();
    const int tile = xcd_tile(blockIdx.x, a.n_tiles);
    int view, y, x;
    tile_pixel(a, tile, threadIdx.x, view, y, x);
    if (!(x < a.w && y < a.h)) return;
    const size_t pix = ((size_t)view * a.h + y) * a.w + x;
    const float4 nr = a.normal[pix];
    out[pix] = nr.w == 0.0f ? make_float4(0.f, 0.f, 0.f, 0.f) : shade_pixel<DT, ANISO>(a, T, dir_ptr(D), s, view, pix, nr);
}

template <int DT>
hipError_t run_shade(const TraceArgs& a, const ShadeArgs& s, float* out, hipStream_t st, EventSink& es) {
    if (a.n_tiles > 0) {
        es.mark(st);
        if (a.aniso)
            hipLaunchKernelGGL((k_shade<DT, true>), dim3(a.n_tiles), dim3(256), 0, st, a, s,
                               reinterpret_cast<float4*>(out));
        else
            hipLaunchKernelGGL((k_shade<DT, false>), dim3(a.n_tiles), dim3(256), 0, st, a, s,
                               reinterpret_cast<float4*>(out));
    }
    es.mark(st);
    return hipGetLastError();
}

}  // namespace

hipError_t vct_launch_shade(const TraceArgs& a, int dtype, const vct_shade_params* p, const float* material,
                            float* out, hipStream_t st, EventSink& es) {
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
                           [&](auto dt) { return run_shade<decltype(dt)::value>(a, s, out, st, es); });
}
