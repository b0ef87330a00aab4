// Per-pixel body of the final shading pass (Section 5.4.4, "Cone Tracing"):
// the modified diffuse and occlusion cones and the shading equation.  Included
// by shade.hip.
#pragma once

#include "march.h"

namespace vct {

struct ShadeArgs {
    int32_t n_lights;
    float light_tex[VCT_MAX_LIGHTS][3][2];   // light positions in texel units, double-float per axis
    float light_pos[VCT_MAX_LIGHTS][3];      // world
    float light_diffuse[VCT_MAX_LIGHTS][3];
    float light_specular[VCT_MAX_LIGHTS][3];
    float specular_color[3];
    int32_t first_hit, falloff, brdf;
    float first_hit_alpha, shadow_strength, grace, q;
    const float4* material;                  // [b][h][w]: c_d.rgb, shininess
};

// First-hit diffuse cone: march until a sample's alpha exceeds `thresh` and
// return that sample's (premultiplied) colour; 0 if none before t_max.  The
// samples taken are added to n.
template <int DT, bool ANISO>
__device__ __forceinline__ float3 march_first_hit(const TraceArgs& a, const LevelTable& T, const DirTable* dirs,
                                                  const Cone& c, float thresh, unsigned int& n) {
    float3 rgb = make_float3(0.f, 0.f, 0.f);
    df t = {a.t0, 0.0f};
    for (int k = 0; k < a.max_steps; ++k) {
        if (!t_within(t, c.tmax)) break;
        const float d = fmaxf(c.two_tan * t.hi, a.voxel);
        const float4 s = sample_at<DT, ANISO, kShareFootprint<DT>>(a, T, c, t, lod_of(a, d), dirs);
        ++n;
        if (s.w > thresh) {
            rgb = make_float3(s.x, s.y, s.z);
            break;
        }
        t = df_add(t, a.step_factor * d);
    }
    return rgb;
}

// Occlusion cone with distance falloff: A += (1 - A) s.a smoothstep(0,
// max_dist, sqrt(t) * strength) while t <= t_max and A < alpha_thresh.  The
// samples taken are added to n.
template <int DT, bool ANISO>
__device__ __forceinline__ float march_falloff(const TraceArgs& a, const LevelTable& T, const DirTable* dirs,
                                               const Cone& c, float strength, unsigned int& n) {
    float A = 0.f;
    df t = {a.t0, 0.0f};
    const float inv = 1.0f / a.max_dist;
    for (int k = 0; k < a.max_steps; ++k) {
        if (!t_within(t, c.tmax) || !(A < a.alpha_thresh)) break;
        const float d = fmaxf(c.two_tan * t.hi, a.voxel);
        const float4 s = sample_at<DT, ANISO, kShareFootprint<DT>>(a, T, c, t, lod_of(a, d), dirs);
        ++n;
        const float h = fminf(fmaxf(sqrtf(t.hi) * strength * inv, 0.0f), 1.0f);
        A = __builtin_fmaf(1.0f - A, s.w * (h * h * (3.0f - 2.0f * h)), A);
        t = df_add(t, a.step_factor * d);
    }
    return A;
}

// Occlusion cone of one light: axis toward it, t_max = min(max_dist, distance).
__device__ __forceinline__ Cone light_cone(const TraceArgs& a, const PixelSetup& P, const float (&L)[3][2]) {
    const float dx = (L[0][0] - P.Ox.hi) + (L[0][1] - P.Ox.lo);
    const float dy = (L[1][0] - P.Oy.hi) + (L[1][1] - P.Oy.lo);
    const float dz = (L[2][0] - P.Oz.hi) + (L[2][1] - P.Oz.lo);
    const float len = sqrtf(dx * dx + dy * dy + dz * dz);
    const float dist = len / a.scale_hi;
    const float3 w = len > 0.f ? make_float3(dx / len, dy / len, dz / len) : make_float3(0.f, 0.f, 0.f);
    return make_cone(a, P, w, a.occ_aperture, fminf(a.max_dist, dist));
}

// (L.rgb, o_min) of one valid pixel; the samples of all its cones are added to n.
template <int DT, bool ANISO>
__device__ __forceinline__ float4 shade_pixel(const TraceArgs& a, const LevelTable& T, const DirTable* dirs,
                                              const ShadeArgs& s, int view, size_t pix, float4 nr, unsigned int& n) {
    const float4 pr = a.pos_rough[pix];
    const float4 mat = s.material[pix];
    const PixelSetup P = pixel_setup(a, pr, nr);
    const float3 cam = make_float3(a.cam_pos[3 * view], a.cam_pos[3 * view + 1], a.cam_pos[3 * view + 2]);

    // indirect diffuse
    float3 D = make_float3(0.f, 0.f, 0.f);
    for (int q = 0; q < a.n_diffuse; ++q) {
        const Cone c = cone_for_slot(a, P, q, cam);
        float3 col;
        if (s.first_hit) {
            col = march_first_hit<DT, ANISO>(a, T, dirs, c, s.first_hit_alpha, n);
        } else {
            const MarchResult m = march<DT, ANISO, kShareFootprint<DT>>(a, T, c, dirs);
            col = make_float3(m.r, m.g, m.b);
            n += (unsigned int)m.k;
        }
        const float wq = a.weight[q];
        D.x = __builtin_fmaf(wq, col.x, D.x);
        D.y = __builtin_fmaf(wq, col.y, D.y);
        D.z = __builtin_fmaf(wq, col.z, D.z);
    }
    // indirect specular: one trace along the reflection axis
    const MarchResult ms = march<DT, ANISO, kShareFootprint<DT>>(a, T, cone_for_slot(a, P, a.n_diffuse, cam), dirs);
    n += (unsigned int)ms.k;
    // unit reflection axis (as in the specular cone) and view direction
    const float3 v = normalize3(P.px - cam.x, P.py - cam.y, P.pz - cam.z);
    const float vn = v.x * P.nx + v.y * P.ny + v.z * P.nz;
    const float3 r = normalize3(v.x - 2.f * vn * P.nx, v.y - 2.f * vn * P.ny, v.z - 2.f * vn * P.nz);
    const float3 wv = make_float3(-v.x, -v.y, -v.z);
    const float shin = mat.w;

    float omin = 1.0f, fsum = 0.0f;
    float3 direct = make_float3(0.f, 0.f, 0.f);
    for (int l = 0; l < s.n_lights; ++l) {
        const Cone co = light_cone(a, P, s.light_tex[l]);
        float A;
        if (s.falloff) {
            A = march_falloff<DT, ANISO>(a, T, dirs, co, s.shadow_strength, n);
        } else {
            const MarchResult mo = march<DT, ANISO, kShareFootprint<DT>>(a, T, co, dirs);
            A = mo.a;
            n += (unsigned int)mo.k;
        }
        const float V = 1.0f - A;
        omin = fminf(omin, V);
        const float3 L = normalize3(s.light_pos[l][0] - P.px, s.light_pos[l][1] - P.py, s.light_pos[l][2] - P.pz);
        const float ndl = P.nx * L.x + P.ny * L.y + P.nz * L.z;
        const float3 R = make_float3(2.f * ndl * P.nx - L.x, 2.f * ndl * P.ny - L.y, 2.f * ndl * P.nz - L.z);
        const float rdw = fmaxf(R.x * wv.x + R.y * wv.y + R.z * wv.z, 0.0f);
        const float lam = fmaxf(ndl, 0.0f);
        const float phong = shin == 0.0f ? 1.0f : powf(rdw, shin);
        direct.x += V * (mat.x * s.light_diffuse[l][0] * lam + s.specular_color[0] * s.light_specular[l][0] * phong);
        direct.y += V * (mat.y * s.light_diffuse[l][1] * lam + s.specular_color[1] * s.light_specular[l][1] * phong);
        direct.z += V * (mat.z * s.light_diffuse[l][2] * lam + s.specular_color[2] * s.light_specular[l][2] * phong);
        if (s.brdf) {
            // gamma = angle(r, L) from atan2(|r x L|, r.L): accurate near 0 and pi
            const float cx = r.y * L.z - r.z * L.y, cy = r.z * L.x - r.x * L.z, cz = r.x * L.y - r.y * L.x;
            const float gamma = atan2f(sqrtf(cx * cx + cy * cy + cz * cz), r.x * L.x + r.y * L.y + r.z * L.z);
            const float g = fmaxf(gamma - s.grace * shin, 0.0f);
            fsum += powf(1.0f - g * 0.31830988618379067f, s.q);   // 1 / pi
        }
    }
    if (!s.brdf) fsum = 1.0f;
    return make_float4(__builtin_fmaf(omin, D.x, __builtin_fmaf(fsum, ms.r, direct.x)),
                       __builtin_fmaf(omin, D.y, __builtin_fmaf(fsum, ms.g, direct.y)),
                       __builtin_fmaf(omin, D.z, __builtin_fmaf(fsum, ms.b, direct.z)), omin);
}

}  // namespace vct
