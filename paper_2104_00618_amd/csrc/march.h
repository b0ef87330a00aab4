// Per-lane cone setup, quadrilinear sampler and front-to-back march shared by
// the forward and backward kernels (Section 4.3.2 cone-trace function,
// Section 4.5 colour supersampler, Sections 4.2 / 5.4.4 cone set).
//
// Precision.  Tap weights are frac(p * N_l - 1/2), so a world-space position
// error dp becomes a weight error dp * N_l.  Float32 positions near 1 carry
// 6e-8 of rounding, i.e. ~1.5e-5 texel at N = 256, too much for 1e-5 parity at
// hard 0/1 opacity edges.  The march therefore keeps the distance t and the
// texel-space origin as double-floats (hi + lo float pairs, Knuth's TwoSum and
// Dekker's TwoProduct via fma) and forms texel coordinates U = O + t W as a
// double-float before floor/frac.  Directions stay float32: once the LOD
// follows the cone diameter, a direction error dw moves a tap by only
// dw / (2 tan(aperture / 2)) texels of the sampled level.
#pragma once

#include <type_traits>

#include "texel.h"
#include "vct_internal.h"

namespace vct {

struct df {
    float hi, lo;
};

__device__ __forceinline__ df two_sum(float a, float b) {
#pragma clang fp contract(off)
    float s = a + b;
    float bp = s - a;
    float e = (a - (s - bp)) + (b - bp);
    return {s, e};
}

__device__ __forceinline__ df fast_two_sum(float a, float b) {
#pragma clang fp contract(off)
    float s = a + b;
    float e = b - (s - a);
    return {s, e};
}

__device__ __forceinline__ df two_prod(float a, float b) {
#pragma clang fp contract(off)
    float p = a * b;
    float e = __builtin_fmaf(a, b, -p);
    return {p, e};
}

// a + b for a double-float a and a float b
__device__ __forceinline__ df df_add(df a, float b) {
#pragma clang fp contract(off)
    df s = two_sum(a.hi, b);
    float lo = s.lo + a.lo;
    return fast_two_sum(s.hi, lo);
}

// O + t * W per axis (double-float O and t, float W)
__device__ __forceinline__ df df_axis(df O, df t, float W) {
#pragma clang fp contract(off)
    df p = two_prod(t.hi, W);
    float plo = __builtin_fmaf(t.lo, W, p.lo);
    df s = two_sum(O.hi, p.hi);
    float lo = s.lo + (O.lo + plo);
    return fast_two_sum(s.hi, lo);
}

// a * b for a double-float a and b
__device__ __forceinline__ df df_mul(df a, df b) {
#pragma clang fp contract(off)
    df p = two_prod(a.hi, b.hi);
    float lo = p.lo + (a.hi * b.lo + a.lo * b.hi);
    return fast_two_sum(p.hi, lo);
}

__device__ __forceinline__ float3 normalize3(float x, float y, float z) {
    float r = sqrtf(x * x + y * y + z * z);
    return make_float3(x / r, y / r, z / r);
}

// Shared-memory copy of the level table (per-lane levels index it).
struct LevelTable {
    float top[VCT_MAX_LEVELS];       // index of the last texel per axis (side - 1), as a float
    int32_t lnb[VCT_MAX_LEVELS];     // log2 of bricks per axis
    uint32_t off[VCT_MAX_LEVELS];
};

// (Both table loaders stride over the workgroup, so they fill every entry for
// any workgroup size; the caller synchronises before the tables are read.)
__device__ __forceinline__ void load_level_table(const TraceArgs& a, LevelTable* t) {
    for (int l = (int)threadIdx.x; l < VCT_MAX_LEVELS; l += (int)blockDim.x) {
        t->top[l] = (float)(a.lv[l].n - 1);
        t->lnb[l] = 31 - __builtin_clz(a.lv[l].nb);
        t->off[l] = a.lv[l].off;
    }
}

// Texel-space coordinate split into base tap and fraction, for level scale 2^-l.
struct Axis {
    int i0, i1;
    float w1;  // weight of i1; i0 gets 1 - w1
};

__device__ __forceinline__ Axis axis_taps(df U, float sc, float top) {
    float u = U.hi * sc - 0.5f;          // exact: power-of-two scale, and u >= -1/4 whenever it matters
    float ulo = U.lo * sc;
    float fl = floorf(u);
    float ph = (u - fl) + ulo;           // in (-1, 2): renormalise without branches
    float c = floorf(ph);
    ph -= c;
    // clamp-to-edge in float before converting: both taps inside [0, top]; an
    // integer-valued fi is exact below 2^24 and clamps to an edge above
    const float fi = fl + c;
    Axis a;
    a.i0 = (int)__builtin_amdgcn_fmed3f(fi, 0.0f, top);
    a.i1 = (int)__builtin_amdgcn_fmed3f(fi + 1.0f, 0.0f, top);
    a.w1 = ph;
    return a;
}

struct Taps {
    uint32_t idx[8];
    float w[8];
    int clamp;   // bit a set: both taps of axis a (x, y, z) fell on the same texel
};

// The 8 taps and trilinear weights of level l at texel-space position U (level-0 texels).
__device__ __forceinline__ void level_taps(const LevelTable& T, int l, df Ux, df Uy, df Uz, Taps& tp) {
    const float top = T.top[l];
    const int lnb = T.lnb[l];
    const uint32_t off = T.off[l];
    const float sc = __int_as_float((127 - l) << 23);   // 2^-l
    Axis ax = axis_taps(Ux, sc, top);
    Axis ay = axis_taps(Uy, sc, top);
    Axis az = axis_taps(Uz, sc, top);
    const float wx0 = 1.0f - ax.w1, wy0 = 1.0f - ay.w1, wz0 = 1.0f - az.w1;
    tp.clamp = (ax.i0 == ax.i1 ? 1 : 0) | (ay.i0 == ay.i1 ? 2 : 0) | (az.i0 == az.i1 ? 4 : 0);
    // brick layout: ((bz * nb + by) * nb + bx) * 64 + (z & 3) * 16 + (y & 3) * 4 + (x & 3), nb = 2^lnb
    const uint32_t cx[2] = {(uint32_t)(((ax.i0 >> 2) << 6) | (ax.i0 & 3)), (uint32_t)(((ax.i1 >> 2) << 6) | (ax.i1 & 3))};
    const uint32_t cy[2] = {(uint32_t)(((ay.i0 >> 2) << (6 + lnb)) | ((ay.i0 & 3) << 2)),
                            (uint32_t)(((ay.i1 >> 2) << (6 + lnb)) | ((ay.i1 & 3) << 2))};
    const uint32_t cz[2] = {(uint32_t)(((az.i0 >> 2) << (6 + 2 * lnb)) | ((az.i0 & 3) << 4)),
                            (uint32_t)(((az.i1 >> 2) << (6 + 2 * lnb)) | ((az.i1 & 3) << 4))};
    const float wxy[4] = {wx0 * wy0, ax.w1 * wy0, wx0 * ay.w1, ax.w1 * ay.w1};
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        int dz = q >> 2, dy = (q >> 1) & 1, dx = q & 1;
        tp.idx[q] = off + cx[dx] + cy[dy] + cz[dz];
        tp.w[q] = wxy[q & 3] * (dz ? az.w1 : wz0);
    }
}

// Anisotropic pyramids: per direction and level, the texel offset relative to
// the +x pyramid's level (which is what LevelTable::off holds); 0 at level 0.
struct DirTable {
    uint32_t delta[6][VCT_MAX_LEVELS];
};

// LDS slot of the table: a DirTable in anisotropic kernels, an empty struct otherwise.
struct NoDirTable {};
template <bool ANISO>
using DirSlot = typename std::conditional<ANISO, DirTable, NoDirTable>::type;
__device__ __forceinline__ const DirTable* dir_ptr(const DirTable& t) { return &t; }
__device__ __forceinline__ const DirTable* dir_ptr(const NoDirTable&) { return nullptr; }
__device__ __forceinline__ void load_dir_table(const TraceArgs&, NoDirTable*) {}

__device__ __forceinline__ void load_dir_table(const TraceArgs& a, DirTable* t) {
    for (int i = (int)threadIdx.x; i < 6 * VCT_MAX_LEVELS; i += (int)blockDim.x)
        t->delta[i / VCT_MAX_LEVELS][i % VCT_MAX_LEVELS] = a.ddelta[i / VCT_MAX_LEVELS][i % VCT_MAX_LEVELS];
}

// s += w * v on the four channels (the accumulation step of every gather).
__device__ __forceinline__ void acc_tap(float4& s, float w, float4 v) {
    s.x = __builtin_fmaf(w, v.x, s.x);
    s.y = __builtin_fmaf(w, v.y, s.y);
    s.z = __builtin_fmaf(w, v.z, s.z);
    s.w = __builtin_fmaf(w, v.w, s.w);
}

// Storage types whose forward marches (trace, shading, bounce) take SHARE
// below: float32.  float16 / bfloat16 marches already halve their requests
// with paired loads, and there the check and the registers it holds cost
// more than the loads it saves.
template <int DT>
constexpr bool kShareFootprint = (DT & ~VCT_WIDE) == VCT_F32;

// SHARE: when every active lane of the wave samples the same 8 texels (same
// level, base texel and clamp pattern, as the lanes of a wave usually do on
// the coarse levels), the texel addresses are wave-uniform, so the 8 texels
// are read once with scalar loads and every lane's FMAs take them from scalar
// registers, instead of every lane issuing texture-address requests (which
// bound these marches).  Same texels, same accumulation order, so the same
// sample bits.  The scalar loads go through a copy of the raw resource whose
// base is moved to the footprint's base texel (wave-uniform 64-bit arithmetic
// in scalar registers), so each load's offset is the tap's small step inside
// the level, never a byte offset of 2 GiB or more, whatever the pyramid's size
// below 4 GiB.  (Pyramids above 4 GiB keep the vector loads.)
// True when `differs` is false in every active lane of the wave (a hook: a
// host-emulation build gives each lane its own view).
#ifndef VCT_WAVE_AGREES
#define VCT_WAVE_AGREES(differs) (__ballot(differs) == 0)
#endif

template <int DT, bool SHARE = false>
__device__ __forceinline__ float4 gather(const TraceArgs& a, const Taps& tp) {
    float4 s = make_float4(0.f, 0.f, 0.f, 0.f);
    if constexpr (SHARE && (DT & VCT_WIDE) == 0) {
        const uint32_t i0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)tp.idx[0]);
        const int c0 = __builtin_amdgcn_readfirstlane(tp.clamp);
        if (VCT_WAVE_AGREES(tp.idx[0] != i0 || tp.clamp != c0)) {
            // (the steps to the +x / +y / +z taps follow from the base texel and
            // the clamp pattern, so they are wave-uniform too)
            const uint32_t d1 = (uint32_t)__builtin_amdgcn_readfirstlane((int)(tp.idx[1] - tp.idx[0]));
            const uint32_t d2 = (uint32_t)__builtin_amdgcn_readfirstlane((int)(tp.idx[2] - tp.idx[0]));
            const uint32_t d4 = (uint32_t)__builtin_amdgcn_readfirstlane((int)(tp.idx[4] - tp.idx[0]));
            constexpr uint32_t tb = DT == VCT_F32 ? 16u : 8u;
            const vct_v4i rs = vct_rebase_raw(a.rraw, (uint64_t)i0 * tb);
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const uint32_t step = ((q & 1) ? d1 : 0u) + ((q & 2) ? d2 : 0u) + ((q & 4) ? d4 : 0u);
                VCT_CHECK_TEXEL(i0 + step);
                if constexpr (DT == VCT_F32) {
                    const vct_v4i v = vct_scalar_load_v4i32(rs, (int32_t)(step * tb), 0);
                    acc_tap(s, tp.w[q], make_float4(__int_as_float(v.x), __int_as_float(v.y), __int_as_float(v.z),
                                                    __int_as_float(v.w)));
                } else {
                    const vct_v2i v = vct_scalar_load_v2i32(rs, (int32_t)(step * tb), 0);
                    acc_tap(s, tp.w[q], vct_decode_texel<DT>((uint32_t)v.x, (uint32_t)v.y));
                }
            }
            return s;
        }
    }
    if constexpr (DT == VCT_F16 || DT == VCT_BF16) {
        // 8-byte texels: the two x taps of a (y, z) row are the neighbouring
        // texels idx and idx + 1 unless the pair crosses a brick (x0 = 3 mod
        // 4) or x clamps (one texel twice), so one 16-byte load fetches both;
        // lanes of those two kinds (the clamp only at the grid's edge) load
        // the second texel on their own, over the upper half of the pair.
        // (Texture-address requests per level: 4 plus those lanes' instead of
        // 8.)  Taps are accumulated in the order 0..7 of the other paths.
        const bool apart = tp.idx[1] - tp.idx[0] != 1u;
        vct_v4i pr[4];
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            VCT_CHECK_TEXEL(tp.idx[2 * p]);
            pr[p] = vct_raw_load_v4i32(a.rraw, (int32_t)(tp.idx[2 * p] * 8u), 0, 0);
        }
        if (apart) {
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                VCT_CHECK_TEXEL(tp.idx[2 * p + 1]);
                const vct_v2i u = vct_raw_load_v2i32(a.rraw, (int32_t)(tp.idx[2 * p + 1] * 8u), 0, 0);
                pr[p].z = u.x;
                pr[p].w = u.y;
            }
        }
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            acc_tap(s, tp.w[2 * p], vct_decode_texel<DT>((uint32_t)pr[p].x, (uint32_t)pr[p].y));
            acc_tap(s, tp.w[2 * p + 1], vct_decode_texel<DT>((uint32_t)pr[p].z, (uint32_t)pr[p].w));
        }
    } else {
#pragma unroll
        for (int q = 0; q < 8; ++q) acc_tap(s, tp.w[q], vct_fetch_texel<DT>(a.rsrc, tp.idx[q]));
    }
    return s;
}

// LOD of a diameter d (world units): lambda = clamp(log2(d / voxel), 0, L - 1).
// d >= voxel, so d / voxel >= 1 is never denormal and the hardware log2 applies directly.
__device__ __forceinline__ float lod_of(const TraceArgs& a, float d) {
    float lam = __builtin_amdgcn_logf(d * a.scale_hi);
    return fminf(fmaxf(lam, 0.0f), (float)(a.levels - 1));
}

// One cone, fully set up.
struct Cone {
    df Ox, Oy, Oz;        // origin, level-0 texel units
    float Wx, Wy, Wz;     // axis times N / extent
    float two_tan;        // 2 tan(aperture / 2)
    float tmax;
};

// Per-pixel setup shared by all cones of the pixel.
struct PixelSetup {
    df Ox, Oy, Oz;
    float nx, ny, nz;                 // unit normal
    float tx, ty, tz, bx, by, bz;     // tangent frame
    float px, py, pz;                 // surface point (world)
    float rough;
};

__device__ __forceinline__ df to_texel(const TraceArgs& a, float x, int ax) {
    // (x - origin) * N / extent as a double-float
    df d = two_sum(x, -a.origin[ax]);
    df sc = {a.scale_hi, a.scale_lo};
    return df_mul(d, sc);
}

// Unit normal and tangent frame of a cone origin (frame helper axis x if the
// normal is near +-y, else y).
__device__ __forceinline__ void set_frame(PixelSetup& P, float4 nr) {
    float3 n = normalize3(nr.x, nr.y, nr.z);
    P.nx = n.x;
    P.ny = n.y;
    P.nz = n.z;
    float ax = 0.f, ay = 1.f;
    if (fabsf(n.y) > 0.9f) {
        ax = 1.f;
        ay = 0.f;
    }
    // t = normalize(a x n) with a = (ax, ay, 0)
    float3 t = normalize3(ay * n.z, -ax * n.z, ax * n.y - ay * n.x);
    P.tx = t.x;
    P.ty = t.y;
    P.tz = t.z;
    // b = n x t
    P.bx = n.y * t.z - n.z * t.y;
    P.by = n.z * t.x - n.x * t.z;
    P.bz = n.x * t.y - n.y * t.x;
}

// Cone origin offset from texel-space point X along the unit normal:
// o = x + n * normal_offset * voxel, i.e. X + n * normal_offset in texel units.
__device__ __forceinline__ void set_origin(const TraceArgs& a, PixelSetup& P, df X, df Y, df Z) {
    P.Ox = df_add(X, P.nx * a.normal_offset);
    P.Oy = df_add(Y, P.ny * a.normal_offset);
    P.Oz = df_add(Z, P.nz * a.normal_offset);
}

__device__ __forceinline__ PixelSetup pixel_setup(const TraceArgs& a, float4 pr, float4 nr) {
    PixelSetup P;
    set_frame(P, nr);
    P.px = pr.x;
    P.py = pr.y;
    P.pz = pr.z;
    P.rough = pr.w;
    set_origin(a, P, to_texel(a, pr.x, 0), to_texel(a, pr.y, 1), to_texel(a, pr.z, 2));
    return P;
}

__device__ __forceinline__ Cone make_cone(const TraceArgs& a, const PixelSetup& P, float3 w, float aperture,
                                          float tmax) {
    Cone c;
    c.Ox = P.Ox;
    c.Oy = P.Oy;
    c.Oz = P.Oz;
    c.Wx = w.x * a.scale_hi;
    c.Wy = w.y * a.scale_hi;
    c.Wz = w.z * a.scale_hi;
    c.two_tan = 2.0f * tanf(0.5f * aperture);
    c.tmax = tmax;
    return c;
}

// Axis of cone slot `slot` of a pixel (0..u-1 diffuse, u specular, u+1 occlusion);
// sets aperture and t_max.
__device__ __forceinline__ Cone cone_for_slot(const TraceArgs& a, const PixelSetup& P, int slot, float3 cam) {
    if (slot < a.n_diffuse) {
        float dx = a.dir[slot][0], dy = a.dir[slot][1], dz = a.dir[slot][2];
        float3 w = normalize3(P.tx * dx + P.bx * dy + P.nx * dz, P.ty * dx + P.by * dy + P.ny * dz,
                              P.tz * dx + P.bz * dy + P.nz * dz);
        return make_cone(a, P, w, a.diffuse_aperture, a.max_dist);
    }
    if (slot == a.n_diffuse) {
        float3 v = normalize3(P.px - cam.x, P.py - cam.y, P.pz - cam.z);
        float vn = v.x * P.nx + v.y * P.ny + v.z * P.nz;
        float3 r = normalize3(v.x - 2.f * vn * P.nx, v.y - 2.f * vn * P.ny, v.z - 2.f * vn * P.nz);
        return make_cone(a, P, r, P.rough * a.spec_aperture_scale, a.max_dist);
    }
    // occlusion: toward the light, in texel units
    df Lx = {a.light_tex[0][0], a.light_tex[0][1]};
    df Ly = {a.light_tex[1][0], a.light_tex[1][1]};
    df Lz = {a.light_tex[2][0], a.light_tex[2][1]};
    float dx = (Lx.hi - P.Ox.hi) + (Lx.lo - P.Ox.lo);
    float dy = (Ly.hi - P.Oy.hi) + (Ly.lo - P.Oy.lo);
    float dz = (Lz.hi - P.Oz.hi) + (Lz.lo - P.Oz.lo);
    float len = sqrtf(dx * dx + dy * dy + dz * dz);
    float dist = len / a.scale_hi;
    float3 w = len > 0.f ? make_float3(dx / len, dy / len, dz / len) : make_float3(0.f, 0.f, 0.f);
    return make_cone(a, P, w, a.occ_aperture, fminf(a.max_dist, dist));
}

// Trilinear sample of level l.  Anisotropic pyramids above level 0: the sum
// over the three axes of w_a^2 times the sample of the direction sign(w_a)
// (the taps are the same in every direction, only the level's offset moves);
// axes with w_a = 0 are skipped.
template <int DT, bool ANISO, bool SHARE = false>
__device__ __forceinline__ float4 level_sample(const TraceArgs& a, const LevelTable& T, const DirTable* D,
                                               const Cone& c, int l, df Ux, df Uy, df Uz) {
    Taps tp;
    level_taps(T, l, Ux, Uy, Uz, tp);
    if constexpr (ANISO) {
        if (l > 0) {
            const float W[3] = {c.Wx, c.Wy, c.Wz};
            float4 s = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) {
                const float wt = W[ax] * W[ax] * a.inv_scale2;
                if (wt == 0.0f) continue;
                const uint32_t delta = D->delta[2 * ax + (W[ax] < 0.0f ? 1 : 0)][l];
                Taps td = tp;
#pragma unroll
                for (int q = 0; q < 8; ++q) td.idx[q] += delta;
                const float4 g = gather<DT, SHARE>(a, td);
                s.x = __builtin_fmaf(wt, g.x, s.x);
                s.y = __builtin_fmaf(wt, g.y, s.y);
                s.z = __builtin_fmaf(wt, g.z, s.z);
                s.w = __builtin_fmaf(wt, g.w, s.w);
            }
            return s;
        }
    }
    return gather<DT, SHARE>(a, tp);
}

// Quadrilinear sample at distance t along the cone (SHARE: see gather).
template <int DT, bool ANISO = false, bool SHARE = false>
__device__ __forceinline__ float4 sample_at(const TraceArgs& a, const LevelTable& T, const Cone& c, df t,
                                            float lam, const DirTable* D = nullptr) {
    df Ux = df_axis(c.Ox, t, c.Wx);
    df Uy = df_axis(c.Oy, t, c.Wy);
    df Uz = df_axis(c.Oz, t, c.Wz);
    int l0 = (int)lam;
    float f = lam - (float)l0;
    float4 s0 = level_sample<DT, ANISO, SHARE>(a, T, D, c, l0, Ux, Uy, Uz);
    if (f > 0.0f) {
        int l1 = min(l0 + 1, a.levels - 1);
        float4 s1 = level_sample<DT, ANISO, SHARE>(a, T, D, c, l1, Ux, Uy, Uz);
        float g = 1.0f - f;
        s0.x = __builtin_fmaf(f, s1.x, g * s0.x);
        s0.y = __builtin_fmaf(f, s1.y, g * s0.y);
        s0.z = __builtin_fmaf(f, s1.z, g * s0.z);
        s0.w = __builtin_fmaf(f, s1.w, g * s0.w);
    }
    return s0;
}

__device__ __forceinline__ bool t_within(df t, float tmax) {
    return t.hi < tmax || (t.hi == tmax && t.lo <= 0.0f);
}

struct MarchResult {
    float r, g, b, a;
    int k;    // samples taken
    int k2;   // of those, samples that read two levels (fractional LOD)
};

// Forward march of one cone (Section 4.3.2): sample while t <= t_max and
// A < alpha_thresh; C += (1 - A) s.rgb, A += (1 - A) s.a, t += beta d.
template <int DT, bool ANISO = false, bool SHARE = false>
__device__ __forceinline__ MarchResult march(const TraceArgs& a, const LevelTable& T, const Cone& c,
                                             const DirTable* D = nullptr) {
    MarchResult m = {0.f, 0.f, 0.f, 0.f, 0, 0};
    df t = {a.t0, 0.0f};
    for (int k = 0; k < a.max_steps; ++k) {
        if (!t_within(t, c.tmax) || !(m.a < a.alpha_thresh)) break;
        float d = fmaxf(c.two_tan * t.hi, a.voxel);
        float lam = lod_of(a, d);
        float4 s = sample_at<DT, ANISO, SHARE>(a, T, c, t, lam, D);
        float tr = 1.0f - m.a;
        m.r = __builtin_fmaf(tr, s.x, m.r);
        m.g = __builtin_fmaf(tr, s.y, m.g);
        m.b = __builtin_fmaf(tr, s.z, m.b);
        m.a = __builtin_fmaf(tr, s.w, m.a);
        m.k = k + 1;
        m.k2 += lam > (float)(int)lam ? 1 : 0;   // (sample_at reads level l0 + 1 too)
        t = df_add(t, a.step_factor * d);
    }
    return m;
}

// All cones of one pixel (slots 0..u-1 diffuse, specular, occlusion); the
// 8-float epilogue (D.rgb, D.a, S.rgb, O) goes to o0, o1, the sample count to
// ksum and the count of two-level samples to k2sum.
template <int DT, bool ANISO = false>
__device__ __forceinline__ void trace_pixel(const TraceArgs& a, const LevelTable& T, int view, size_t pix,
                                            float4& o0, float4& o1, unsigned int& ksum, unsigned int& k2sum,
                                            const DirTable* D = nullptr) {
    o0 = make_float4(0.f, 0.f, 0.f, 0.f);
    o1 = o0;
    ksum = 0;
    k2sum = 0;
    float4 nr = a.normal[pix];
    if (nr.w == 0.0f) return;
    float4 pr = a.pos_rough[pix];
    PixelSetup P = pixel_setup(a, pr, nr);
    float3 cam = make_float3(a.cam_pos[3 * view], a.cam_pos[3 * view + 1], a.cam_pos[3 * view + 2]);
    for (int q = 0; q < a.n_diffuse; ++q) {
        Cone c = cone_for_slot(a, P, q, cam);
        MarchResult m = march<DT, ANISO, kShareFootprint<DT>>(a, T, c, D);
        float wq = a.weight[q];
        o0.x = __builtin_fmaf(wq, m.r, o0.x);
        o0.y = __builtin_fmaf(wq, m.g, o0.y);
        o0.z = __builtin_fmaf(wq, m.b, o0.z);
        o0.w = __builtin_fmaf(wq, m.a, o0.w);
        ksum += m.k;
        k2sum += m.k2;
    }
    if (a.enable_spec) {
        Cone c = cone_for_slot(a, P, a.n_diffuse, cam);
        MarchResult m = march<DT, ANISO, kShareFootprint<DT>>(a, T, c, D);
        o1.x = m.r;
        o1.y = m.g;
        o1.z = m.b;
        ksum += m.k;
        k2sum += m.k2;
    }
    if (a.enable_occ) {
        Cone c = cone_for_slot(a, P, a.n_diffuse + 1, cam);
        MarchResult m = march<DT, ANISO, kShareFootprint<DT>>(a, T, c, D);
        o1.w = m.a;
        ksum += m.k;
        k2sum += m.k2;
    }
}

// XCD-aware tile order: hardware dispatches workgroup i to XCD i % 8; give each
// XCD a contiguous run of tiles so neighbouring tiles share an L2.
__device__ __forceinline__ int xcd_tile(int bid, int nt) {
    int q = nt >> 3, r = nt & 7;
    int xcd = bid & 7, k = bid >> 3;
    return xcd < r ? xcd * (q + 1) + k : r * (q + 1) + (xcd - r) * q + k;
}

// Pixel of thread `tid` in tile `tile`: 16x16 pixels per 256-thread workgroup,
// each wave an 8x8 quadrant.
__device__ __forceinline__ void tile_pixel(const TraceArgs& a, int tile, int tid, int& view, int& y, int& x) {
    int tpv = a.tiles_x * a.tiles_y;
    view = tile / tpv;
    int r = tile - view * tpv;
    int ty = r / a.tiles_x, tx = r - ty * a.tiles_x;
    int wv = tid >> 6, lane = tid & 63;
    x = tx * 16 + (wv & 1) * 8 + (lane & 7);
    y = ty * 16 + (wv >> 1) * 8 + (lane >> 3);
}

}  // namespace vct
