// Per-pixel bodies of the adjoint (see backward.hip for the method).
#pragma once

#include "march.h"

// Index hook for host-side verification builds (empty in the library).
#ifndef VCT_CHECK_ACC
#define VCT_CHECK_ACC(idx)
#endif

namespace vct {

// End state of one cone after its forward march (40 bytes stored).
struct LaneState {
    float4 hi;   // C_K.hi (rgb), A_K
    float4 lo;   // C_K.lo (rgb), K (as int bits)
    float2 cf;   // (alpha, beta) of the contribution bound (lane_coefs)
};

__device__ __forceinline__ size_t n_pixels(const TraceArgs& a) { return (size_t)a.b * a.h * a.w; }

// Lane states are stored field-major, so that the 64 pixels of a wave read and
// write contiguous runs: float4 number (2 q + f) * n_pix + p holds field f
// (hi, lo) of cone q of pixel p; after those 2 * nslots * n_pix float4s,
// float2 number q * n_pix + p holds its bound coefficients.  The backward's
// bound pass reads only the coefficients, the scatter pass only hi and lo.
__device__ __forceinline__ const float2* lane_coefs_base(const TraceArgs& a, const LaneState* state) {
    return reinterpret_cast<const float2*>(reinterpret_cast<const float4*>(state) +
                                           (size_t)2 * (a.n_diffuse + 2) * n_pixels(a));
}

__device__ __forceinline__ LaneState lane_get(const TraceArgs& a, const LaneState* __restrict__ state, size_t pix,
                                              int slot) {
    const size_t np = n_pixels(a);
    const float4* f = reinterpret_cast<const float4*>(state) + (size_t)slot * 2 * np + pix;
    LaneState s;
    s.hi = f[0];
    s.lo = f[np];
    s.cf = make_float2(0.f, 0.f);
    return s;
}

__device__ __forceinline__ float2 lane_get_coefs(const TraceArgs& a, const LaneState* __restrict__ state, size_t pix,
                                                 int slot) {
    return lane_coefs_base(a, state)[(size_t)slot * n_pixels(a) + pix];
}

__device__ __forceinline__ void lane_put(const TraceArgs& a, LaneState* __restrict__ state, size_t pix, int slot,
                                         const LaneState& s) {
    const size_t np = n_pixels(a);
    float4* f = reinterpret_cast<float4*>(state) + (size_t)slot * 2 * np + pix;
    f[0] = s.hi;
    f[np] = s.lo;
    const_cast<float2*>(lane_coefs_base(a, state))[(size_t)slot * np + pix] = s.cf;
}

// dL/dC (3) and dL/dA of cone `slot` from the pixel's dL/d(out) = (g0, g1).
__device__ __forceinline__ void slot_grads(const TraceArgs& a, int slot, float4 g0, float4 g1, float gc[3],
                                           float& ga) {
    if (slot < a.n_diffuse) {
        float wq = a.weight[slot];
        gc[0] = wq * g0.x;
        gc[1] = wq * g0.y;
        gc[2] = wq * g0.z;
        ga = wq * g0.w;
    } else if (slot == a.n_diffuse) {
        gc[0] = g1.x;
        gc[1] = g1.y;
        gc[2] = g1.z;
        ga = 0.f;
    } else {
        gc[0] = gc[1] = gc[2] = 0.f;
        ga = g1.w;
    }
}

__device__ __forceinline__ bool slot_enabled(const TraceArgs& a, int slot) {
    if (slot < a.n_diffuse) return true;
    if (slot == a.n_diffuse) return a.enable_spec != 0;
    return a.enable_occ != 0;
}

// Compensated colour accumulation C += T * s (per channel).
__device__ __forceinline__ void acc_colour(df& C, float T, float s) {
    df p = two_prod(T, s);
    C = df_add(C, p.hi);
    C.lo += p.lo;
}

struct Pass1Out {
    df C[3];
    float A, Tlast, ST, SQ, MC;
    int K;
};

// Recompute one cone (same A recurrence as the forward, so the same K),
// with C as a double-float and the sums needed for the contribution bound.
template <int DT, bool ANISO = false>
__device__ __forceinline__ Pass1Out pass1_march(const TraceArgs& a, const LevelTable& T, const Cone& c,
                                                const DirTable* D = nullptr) {
    Pass1Out r;
    for (int i = 0; i < 3; ++i) r.C[i] = {0.f, 0.f};
    r.A = 0.f;
    r.Tlast = 1.f;
    r.ST = 0.f;
    r.SQ = 0.f;
    r.MC = 0.f;
    r.K = 0;
    df t = {a.t0, 0.0f};
    for (int k = 0; k < a.max_steps; ++k) {
        if (!t_within(t, c.tmax) || !(r.A < a.alpha_thresh)) break;
        float d = fmaxf(c.two_tan * t.hi, a.voxel);
        float lam = lod_of(a, d);
        // (wave-uniform footprint reads on float32 pyramids: the forward that
        // keeps lane states ran 4.9 -> 4.0 ms with them on anisotropic
        // pyramids, 1.99 -> 1.96 ms on isotropic ones)
        float4 s = sample_at<DT, ANISO, kShareFootprint<DT>>(a, T, c, t, lam, D);
        float tr = 1.0f - r.A;
        // |T_{k-1}| / |T_k| for every sample k that follows another (T_k >= 2^-24
        // here, so the hardware reciprocal is within 1 ulp; the bound's 1.001
        // covers that as it covers the rounding of the sums)
        if (k > 0) r.SQ += fabsf(r.Tlast) * __builtin_amdgcn_rcpf(fabsf(tr));
        acc_colour(r.C[0], tr, s.x);
        acc_colour(r.C[1], tr, s.y);
        acc_colour(r.C[2], tr, s.z);
        r.A = __builtin_fmaf(tr, s.w, r.A);
        r.ST += fabsf(tr);
        r.MC = fmaxf(r.MC, fmaxf(fabsf(r.C[0].hi), fmaxf(fabsf(r.C[1].hi), fabsf(r.C[2].hi))));
        r.Tlast = tr;
        r.K = k + 1;
        t = df_add(t, a.step_factor * d);
    }
    return r;
}

// Bound on sum_k |dL/dc_k|_1 + |dL/da_k| of one cone, linear in its
// gradient: |dL/dc_k| = |T_k| |dL/dC|, and for k < K-1
// |dL/da_k| <= |T_k / T_{k+1}| (|dL/dC|_1 (|C_K| + max|C|) + |dL/dA| |T_K|);
// the last sample gives |T_{K-1} dL/dA|.  So the sum is at most
// alpha |dL/dC|_1 + beta |dL/dA| with
//   alpha = sum_k |T_k| + sum_{k<K-1} |T_k / T_{k+1}| (|C_K| + max_k |C_k|),
//   beta  = sum_{k<K-1} |T_k / T_{k+1}| |T_K| + |T_{K-1}|  (K > 0),
// which the forward stores so that the backward's bound pass reads 8 bytes
// per cone.
__device__ __forceinline__ float2 lane_coefs(const Pass1Out& r) {
    const float CK = fmaxf(fabsf(r.C[0].hi), fmaxf(fabsf(r.C[1].hi), fabsf(r.C[2].hi)));
    const float TK = 1.0f - r.A;
    const float alpha = r.ST + r.SQ * (CK + r.MC);
    const float beta = r.SQ * fabsf(TK) + (r.K > 0 ? fabsf(r.Tlast) : 0.f);
    return make_float2(alpha, beta);
}

__device__ __forceinline__ LaneState lane_state(const Pass1Out& r) {
    LaneState out;
    out.hi = make_float4(r.C[0].hi, r.C[1].hi, r.C[2].hi, r.A);
    out.lo = make_float4(r.C[0].lo, r.C[1].lo, r.C[2].lo, __int_as_float(r.K));
    out.cf = lane_coefs(r);
    return out;
}

__device__ __forceinline__ LaneState zero_lane_state() {
    LaneState z;
    z.hi = make_float4(0.f, 0.f, 0.f, 0.f);
    z.lo = z.hi;
    z.cf = make_float2(0.f, 0.f);
    return z;
}

// The bound of one cone for dL/d(out) = (g0, g1) of its pixel (1.001 covers
// the float32 rounding of the sums).
__device__ __forceinline__ float lane_bound(const TraceArgs& a, int slot, float2 cf, float4 g0, float4 g1) {
    float gc[3], ga;
    slot_grads(a, slot, g0, g1, gc, ga);
    const float gc1 = fabsf(gc[0]) + fabsf(gc[1]) + fabsf(gc[2]);
    return (cf.x * gc1 + cf.y * fabsf(ga)) * 1.001f;
}

// Pass 1 for one pixel: stores the lane states of its cones and returns the
// bound on sum_k |dL/dc_k|_1 + |dL/da_k| over them.
template <int DT, bool ANISO = false>
__device__ __forceinline__ float pass1_pixel(const TraceArgs& a, const LevelTable& T, const float4* __restrict__ gout,
                                             LaneState* __restrict__ state, int view, size_t pix,
                                             const DirTable* D = nullptr) {
    const int nslots = a.n_diffuse + 2;
    float4 nr = a.normal[pix];
    float bound = 0.f;
    if (nr.w == 0.0f) {
        for (int slot = 0; slot < nslots; ++slot) lane_put(a, state, pix, slot, zero_lane_state());
        return 0.f;
    }
    float4 pr = a.pos_rough[pix];
    float4 g0 = gout[2 * pix], g1 = gout[2 * pix + 1];
    PixelSetup P = pixel_setup(a, pr, nr);
    float3 cam = make_float3(a.cam_pos[3 * view], a.cam_pos[3 * view + 1], a.cam_pos[3 * view + 2]);
    for (int slot = 0; slot < nslots; ++slot) {
        LaneState out = zero_lane_state();
        if (slot_enabled(a, slot)) {
            Cone c = cone_for_slot(a, P, slot, cam);
            out = lane_state(pass1_march<DT, ANISO>(a, T, c, D));
            bound += lane_bound(a, slot, out.cf, g0, g1);
        }
        lane_put(a, state, pix, slot, out);
    }
    return bound;
}

// Bound of one pixel's cones from saved lane states.
__device__ __forceinline__ float saved_bound_pixel(const TraceArgs& a, const float4* __restrict__ gout,
                                                   const LaneState* __restrict__ state, size_t pix) {
    if (a.normal[pix].w == 0.0f) return 0.f;
    const int nslots = a.n_diffuse + 2;
    const float4 g0 = gout[2 * pix], g1 = gout[2 * pix + 1];
    float bound = 0.f;
    for (int slot = 0; slot < nslots; ++slot)
        if (slot_enabled(a, slot)) bound += lane_bound(a, slot, lane_get_coefs(a, state, pix, slot), g0, g1);
    return bound;
}

// Forward for one pixel that also saves its cones' end states (for the
// backward): the same march as pass 1, with the epilogue of trace_pixel.
template <int DT, bool ANISO = false>
__device__ __forceinline__ void trace_save_pixel(const TraceArgs& a, const LevelTable& T, int view, size_t pix,
                                                 LaneState* __restrict__ state, float4& o0, float4& o1,
                                                 const DirTable* D = nullptr) {
    o0 = make_float4(0.f, 0.f, 0.f, 0.f);
    o1 = o0;
    const int nslots = a.n_diffuse + 2;
    float4 nr = a.normal[pix];
    if (nr.w == 0.0f) {
        for (int slot = 0; slot < nslots; ++slot) lane_put(a, state, pix, slot, zero_lane_state());
        return;
    }
    PixelSetup P = pixel_setup(a, a.pos_rough[pix], nr);
    float3 cam = make_float3(a.cam_pos[3 * view], a.cam_pos[3 * view + 1], a.cam_pos[3 * view + 2]);
    for (int slot = 0; slot < nslots; ++slot) {
        LaneState out = zero_lane_state();
        if (slot_enabled(a, slot)) {
            Cone c = cone_for_slot(a, P, slot, cam);
            Pass1Out r = pass1_march<DT, ANISO>(a, T, c, D);
            out = lane_state(r);
            const float cr = r.C[0].hi + r.C[0].lo, cg = r.C[1].hi + r.C[1].lo, cb = r.C[2].hi + r.C[2].lo;
            if (slot < a.n_diffuse) {
                const float wq = a.weight[slot];
                o0.x = __builtin_fmaf(wq, cr, o0.x);
                o0.y = __builtin_fmaf(wq, cg, o0.y);
                o0.z = __builtin_fmaf(wq, cb, o0.z);
                o0.w = __builtin_fmaf(wq, r.A, o0.w);
            } else if (slot == a.n_diffuse) {
                o1.x = cr;
                o1.y = cg;
                o1.z = cb;
            } else {
                o1.w = r.A;
            }
        }
        lane_put(a, state, pix, slot, out);
    }
}

// Pass-2 state of one cone of one lane.
struct Pass2Lane {
    Cone c;
    df C[3];
    df CK[3];
    df t;
    float A, TK;
    float gc[3], ga;
    int K;
};

// Set up the re-march of cone `slot`; K = 0 when the cone receives no gradient.
__device__ __forceinline__ void pass2_init(const TraceArgs& a, const PixelSetup& P, float3 cam, float4 g0, float4 g1,
                                           const LaneState& S, int slot, Pass2Lane& L) {
    slot_grads(a, slot, g0, g1, L.gc, L.ga);
    const bool zero = L.gc[0] == 0.f && L.gc[1] == 0.f && L.gc[2] == 0.f && L.ga == 0.f;
    L.K = zero ? 0 : min(max(__float_as_int(S.lo.w), 0), a.max_steps);
    L.CK[0] = {S.hi.x, S.lo.x};
    L.CK[1] = {S.hi.y, S.lo.y};
    L.CK[2] = {S.hi.z, S.lo.z};
    L.TK = 1.0f - S.hi.w;
    L.c = cone_for_slot(a, P, slot, cam);
    for (int i = 0; i < 3; ++i) L.C[i] = {0.f, 0.f};
    L.A = 0.f;
    L.t = {a.t0, 0.0f};
}

// One level's 8 taps in factored form: base texel (tap 0), the index steps to
// the +x / +y / +z neighbours (0 on an axis that clamps) and the per-axis
// weights of the upper taps.
struct LevelGeom {
    uint32_t base, dx, dy, dz;
    float wx, wy, wz;
    int level;
};

__device__ __forceinline__ LevelGeom level_geom(const LevelTable& T, int l, df Ux, df Uy, df Uz) {
    const float top = T.top[l];
    const int lnb = T.lnb[l];
    const float sc = __int_as_float((127 - l) << 23);   // 2^-l
    const Axis ax = axis_taps(Ux, sc, top);
    const Axis ay = axis_taps(Uy, sc, top);
    const Axis az = axis_taps(Uz, sc, top);
    // brick layout: ((bz * nb + by) * nb + bx) * 64 + (z & 3) * 16 + (y & 3) * 4 + (x & 3), nb = 2^lnb
    const uint32_t cx0 = ((ax.i0 >> 2) << 6) | (ax.i0 & 3), cx1 = ((ax.i1 >> 2) << 6) | (ax.i1 & 3);
    const uint32_t cy0 = ((ay.i0 >> 2) << (6 + lnb)) | ((ay.i0 & 3) << 2);
    const uint32_t cy1 = ((ay.i1 >> 2) << (6 + lnb)) | ((ay.i1 & 3) << 2);
    const uint32_t cz0 = ((az.i0 >> 2) << (6 + 2 * lnb)) | ((az.i0 & 3) << 4);
    const uint32_t cz1 = ((az.i1 >> 2) << (6 + 2 * lnb)) | ((az.i1 & 3) << 4);
    LevelGeom g;
    g.base = T.off[l] + cx0 + cy0 + cz0;
    g.dx = cx1 - cx0;
    g.dy = cy1 - cy0;
    g.dz = cz1 - cz0;
    g.wx = ax.w1;
    g.wy = ay.w1;
    g.wz = az.w1;
    g.level = l;
    return g;
}

// The level's sample: the same taps, weights and products as level_taps +
// gather of the forward, so the recomputed samples equal the forward's.
// (Per-tap loads for every storage type: the forward's paired float16 /
// bfloat16 loads would save texture-address requests here too, but this pass
// is bound by VALU issue, and their extra branch made it 2-3 % slower.  The
// texels and the accumulation order are the same, so the samples are too.)
// SPLIT (float32): taps 4..7 are loaded after taps 0..3 are accumulated, so
// at most four 16-byte texels are in flight; with the held emissions of the
// scatter pass the kernel is at its register cap, and the full set of eight
// made it slower (7.14 -> 8.08 ms, against 6.62 -> 6.09 ms split).
template <int DT, bool SPLIT = false>
__device__ __forceinline__ float4 gather_geom(const TraceArgs& a, const LevelGeom& g) {
    const float wx0 = 1.0f - g.wx, wy0 = 1.0f - g.wy, wz0 = 1.0f - g.wz;
    const float wxy[4] = {wx0 * wy0, g.wx * wy0, wx0 * g.wy, g.wx * g.wy};
    float4 s = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const uint32_t idx = g.base + ((q & 1) ? g.dx : 0u) + ((q & 2) ? g.dy : 0u) + ((q & 4) ? g.dz : 0u);
        acc_tap(s, wxy[q & 3] * ((q & 4) ? g.wz : wz0), vct_fetch_texel<DT>(a.rsrc, idx));
        if (SPLIT && (DT & ~VCT_WIDE) == VCT_F32 && q == 3) __builtin_amdgcn_sched_barrier(0);
    }
    return s;
}

// gather_geom with wave-uniform footprints read once through the scalar
// cache (float32 narrow pyramids; the same taps, weights and order, so the
// same bits): when every active lane has the same base texel and steps.
// Used by the anisotropic re-march, which reads three directions per level
// and is bound by its texture requests (15.3 -> 13.4 ms for the scatter pass
// at 1080p / 256^3); the isotropic one is bound by VALU issue and the
// atomics, and measured slower with it.
template <int DT>
__device__ __forceinline__ float4 gather_geom_shared(const TraceArgs& a, const LevelGeom& g) {
    if constexpr (DT == VCT_F32) {
        const uint32_t b0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)g.base);
        const uint32_t dx = (uint32_t)__builtin_amdgcn_readfirstlane((int)g.dx);
        const uint32_t dy = (uint32_t)__builtin_amdgcn_readfirstlane((int)g.dy);
        const uint32_t dz = (uint32_t)__builtin_amdgcn_readfirstlane((int)g.dz);
        if (VCT_WAVE_AGREES(g.base != b0 || g.dx != dx || g.dy != dy || g.dz != dz)) {
            const float wx0 = 1.0f - g.wx, wy0 = 1.0f - g.wy, wz0 = 1.0f - g.wz;
            const float wxy[4] = {wx0 * wy0, g.wx * wy0, wx0 * g.wy, g.wx * g.wy};
            const vct_v4i rs = vct_rebase_raw(a.rraw, (uint64_t)b0 * 16u);
            float4 s = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const uint32_t step = ((q & 1) ? dx : 0u) + ((q & 2) ? dy : 0u) + ((q & 4) ? dz : 0u);
                VCT_CHECK_TEXEL(b0 + step);
                const vct_v4i v = vct_scalar_load_v4i32(rs, (int32_t)(step * 16u), 0);
                acc_tap(s, wxy[q & 3] * ((q & 4) ? g.wz : wz0),
                        make_float4(__int_as_float(v.x), __int_as_float(v.y), __int_as_float(v.z),
                                    __int_as_float(v.w)));
            }
            return s;
        }
    }
    return gather_geom<DT>(a, g);
}

// Anisotropic pyramids: the level's sample as level_sample<.., true> forms it
// (level 0 plain; above, the axes with w_a^2 > 0 in order, each gathered at
// its direction's offset and added with an FMA), from the factored taps.
template <int DT>
__device__ __forceinline__ float4 gather_geom_aniso(const TraceArgs& a, const DirTable* D, const Cone& c,
                                                    const LevelGeom& g) {
    if (g.level == 0) return gather_geom_shared<DT>(a, g);
    const float W[3] = {c.Wx, c.Wy, c.Wz};
    float4 s = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        const float wt = W[ax] * W[ax] * a.inv_scale2;
        if (wt == 0.0f) continue;
        LevelGeom gd = g;
        gd.base += D->delta[2 * ax + (W[ax] < 0.0f ? 1 : 0)][g.level];
        const float4 v = gather_geom_shared<DT>(a, gd);
        s.x = __builtin_fmaf(wt, v.x, s.x);
        s.y = __builtin_fmaf(wt, v.y, s.y);
        s.z = __builtin_fmaf(wt, v.z, s.z);
        s.w = __builtin_fmaf(wt, v.w, s.w);
    }
    return s;
}

// Sample k of a pass-2 cone: its taps on one or two levels and the gradient
// g = (dL/dc_k, dL/da_k) of the sample; advances the march.
struct Pass2Step {
    LevelGeom g0, g1;   // levels l0 and l1 (g1 only when f > 0)
    float f;            // weight of level l1 (0: single level)
    float g[4];
};

template <int DT, bool ANISO = false>
__device__ __forceinline__ void pass2_step(const TraceArgs& a, const LevelTable& T, Pass2Lane& L, int k,
                                           Pass2Step& st, const DirTable* D = nullptr) {
    const float d = fmaxf(L.c.two_tan * L.t.hi, a.voxel);
    const float lam = lod_of(a, d);
    const df Ux = df_axis(L.c.Ox, L.t, L.c.Wx);
    const df Uy = df_axis(L.c.Oy, L.t, L.c.Wy);
    const df Uz = df_axis(L.c.Oz, L.t, L.c.Wz);
    const int l0 = (int)lam;
    st.f = lam - (float)l0;
    st.g0 = level_geom(T, l0, Ux, Uy, Uz);
    float4 s = ANISO ? gather_geom_aniso<DT>(a, D, L.c, st.g0) : gather_geom<DT, true>(a, st.g0);
    if (st.f > 0.0f) {
        st.g1 = level_geom(T, min(l0 + 1, a.levels - 1), Ux, Uy, Uz);
        float4 s1 = ANISO ? gather_geom_aniso<DT>(a, D, L.c, st.g1) : gather_geom<DT, true>(a, st.g1);
        float gg = 1.0f - st.f;
        s.x = __builtin_fmaf(st.f, s1.x, gg * s.x);
        s.y = __builtin_fmaf(st.f, s1.y, gg * s.y);
        s.z = __builtin_fmaf(st.f, s1.z, gg * s.z);
        s.w = __builtin_fmaf(st.f, s1.w, gg * s.w);
    }
    const float tr = 1.0f - L.A;
    acc_colour(L.C[0], tr, s.x);
    acc_colour(L.C[1], tr, s.y);
    acc_colour(L.C[2], tr, s.z);
    L.A = __builtin_fmaf(tr, s.w, L.A);
    st.g[0] = tr * L.gc[0];
    st.g[1] = tr * L.gc[1];
    st.g[2] = tr * L.gc[2];
    if (k == L.K - 1) {
        st.g[3] = tr * L.ga;
    } else {
        const float tn = 1.0f - L.A;
        float dot = 0.f;
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            float diff = (L.CK[ch].hi - L.C[ch].hi) + (L.CK[ch].lo - L.C[ch].lo);
            dot = __builtin_fmaf(L.gc[ch], diff, dot);
        }
        st.g[3] = -tr * (dot - L.ga * L.TK) * __builtin_amdgcn_rcpf(tn);   // tn >= 2^-24: rcp is 1 ulp
    }
    L.t = df_add(L.t, a.step_factor * d);
}

// round(v * 2^e) as a 64-bit integer (float32 ops only: the float64 units of
// gfx950 run at a fraction of the float32 rate).
__device__ __forceinline__ long long fixed_point(float v, int e) { return (long long)rintf(ldexpf(v, e)); }

}  // namespace vct
