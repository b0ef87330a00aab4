// Per-pixel bodies of the adjoint (see backward.hip for the method).
#pragma once

#include "march.h"

// Index hook for host-side verification builds (empty in the library).
#ifndef VCT_CHECK_ACC
#define VCT_CHECK_ACC(idx)
#endif

namespace vct {

struct LaneState {
    float4 hi;   // C_K.hi (rgb), A_K
    float4 lo;   // C_K.lo (rgb), K (as int bits)
};

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
template <int DT>
__device__ __forceinline__ Pass1Out pass1_march(const TraceArgs& a, const LevelTable& T, const Cone& c) {
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
        float4 s = sample_at<DT>(a, T, c, t, lam);
        float tr = 1.0f - r.A;
        // |T_{k-1}| / |T_k| for every sample k that follows another (T_k >= 2^-24 here)
        if (k > 0) r.SQ += fabsf(r.Tlast) / fabsf(tr);
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

// Pass 1 for one pixel: stores the lane states of its cones and returns the
// bound on sum_k |dL/dc_k|_1 + |dL/da_k| over them.
template <int DT>
__device__ __forceinline__ float pass1_pixel(const TraceArgs& a, const LevelTable& T, const float4* __restrict__ gout,
                                             LaneState* __restrict__ state, int view, size_t pix) {
    const int nslots = a.n_diffuse + 2;
    LaneState* st = state + pix * nslots;
    float4 nr = a.normal[pix];
    float bound = 0.f;
    if (nr.w == 0.0f) {
        for (int slot = 0; slot < nslots; ++slot) {
            LaneState z;
            z.hi = make_float4(0.f, 0.f, 0.f, 0.f);
            z.lo = make_float4(0.f, 0.f, 0.f, 0.f);
            st[slot] = z;
        }
        return 0.f;
    }
    float4 pr = a.pos_rough[pix];
    float4 g0 = gout[2 * pix], g1 = gout[2 * pix + 1];
    PixelSetup P = pixel_setup(a, pr, nr);
    float3 cam = make_float3(a.cam_pos[3 * view], a.cam_pos[3 * view + 1], a.cam_pos[3 * view + 2]);
    for (int slot = 0; slot < nslots; ++slot) {
        LaneState out;
        out.hi = make_float4(0.f, 0.f, 0.f, 0.f);
        out.lo = make_float4(0.f, 0.f, 0.f, 0.f);
        if (slot_enabled(a, slot)) {
            Cone c = cone_for_slot(a, P, slot, cam);
            Pass1Out r = pass1_march<DT>(a, T, c);
            out.hi = make_float4(r.C[0].hi, r.C[1].hi, r.C[2].hi, r.A);
            out.lo = make_float4(r.C[0].lo, r.C[1].lo, r.C[2].lo, __int_as_float(r.K));
            float gc[3], ga;
            slot_grads(a, slot, g0, g1, gc, ga);
            float gc1 = fabsf(gc[0]) + fabsf(gc[1]) + fabsf(gc[2]);
            float TK = 1.0f - r.A;
            float CK = fmaxf(fabsf(r.C[0].hi), fmaxf(fabsf(r.C[1].hi), fabsf(r.C[2].hi)));
            // sum_k |dL/dc_k|_1 + |dL/da_k| <= this; the last sample uses T_{K-1} dL/dA
            float b = r.ST * gc1 + r.SQ * (gc1 * (CK + r.MC) + fabsf(ga) * fabsf(TK)) +
                      (r.K > 0 ? fabsf(ga) * fabsf(r.Tlast) : 0.f);
            bound += b * 1.001f;
        }
        st[slot] = out;
    }
    return bound;
}

// Add round(v * 2^e) to a 64-bit fixed-point accumulator for each channel.
__device__ __forceinline__ void emit(unsigned long long* __restrict__ acc, uint32_t idx, float wt, const float g[4],
                                     int e) {
    VCT_CHECK_ACC(idx);
    unsigned long long* p = acc + (size_t)idx * 4;
#pragma unroll
    for (int ch = 0; ch < 4; ++ch) {
        float v = ldexpf(wt * g[ch], e);
        long long q = (long long)rintf(v);
        if (q) atomicAdd(p + ch, (unsigned long long)q);
    }
}

// Pass 2 for one pixel: re-march every cone with a nonzero output gradient
// and scatter the fixed-point tap contributions.
template <int DT>
__device__ __forceinline__ void pass2_pixel(const TraceArgs& a, const LevelTable& T, const float4* __restrict__ gout,
                                            const LaneState* __restrict__ state, int E,
                                            unsigned long long* __restrict__ acc, int view, size_t pix) {
    float4 nr = a.normal[pix];
    if (nr.w == 0.0f) return;
    const int nslots = a.n_diffuse + 2;
    float4 pr = a.pos_rough[pix];
    float4 g0 = gout[2 * pix], g1 = gout[2 * pix + 1];
    PixelSetup P = pixel_setup(a, pr, nr);
    float3 cam = make_float3(a.cam_pos[3 * view], a.cam_pos[3 * view + 1], a.cam_pos[3 * view + 2]);
    const LaneState* st = state + pix * nslots;
    for (int slot = 0; slot < nslots; ++slot) {
        if (!slot_enabled(a, slot)) continue;
        float gc[3], ga;
        slot_grads(a, slot, g0, g1, gc, ga);
        if (gc[0] == 0.f && gc[1] == 0.f && gc[2] == 0.f && ga == 0.f) continue;
        LaneState S = st[slot];
        const int K = min(max(__float_as_int(S.lo.w), 0), a.max_steps);
        const df CK[3] = {{S.hi.x, S.lo.x}, {S.hi.y, S.lo.y}, {S.hi.z, S.lo.z}};
        const float TK = 1.0f - S.hi.w;
        Cone c = cone_for_slot(a, P, slot, cam);
        df C[3] = {{0.f, 0.f}, {0.f, 0.f}, {0.f, 0.f}};
        float A = 0.f;
        df t = {a.t0, 0.0f};
        for (int k = 0; k < K; ++k) {
            float d = fmaxf(c.two_tan * t.hi, a.voxel);
            float lam = lod_of(a, d);
            df Ux = df_axis(c.Ox, t, c.Wx);
            df Uy = df_axis(c.Oy, t, c.Wy);
            df Uz = df_axis(c.Oz, t, c.Wz);
            int l0 = (int)lam;
            float f = lam - (float)l0;
            int l1 = min(l0 + 1, a.levels - 1);
            Taps tp0, tp1;
            level_taps(T, l0, Ux, Uy, Uz, tp0);
            float4 s = gather<DT>(a.pyr, tp0);
            if (f > 0.0f) {
                level_taps(T, l1, Ux, Uy, Uz, tp1);
                float4 s1 = gather<DT>(a.pyr, tp1);
                float gg = 1.0f - f;
                s.x = __builtin_fmaf(f, s1.x, gg * s.x);
                s.y = __builtin_fmaf(f, s1.y, gg * s.y);
                s.z = __builtin_fmaf(f, s1.z, gg * s.z);
                s.w = __builtin_fmaf(f, s1.w, gg * s.w);
            }
            const float tr = 1.0f - A;
            acc_colour(C[0], tr, s.x);
            acc_colour(C[1], tr, s.y);
            acc_colour(C[2], tr, s.z);
            A = __builtin_fmaf(tr, s.w, A);
            float g[4];
            g[0] = tr * gc[0];
            g[1] = tr * gc[1];
            g[2] = tr * gc[2];
            if (k == K - 1) {
                g[3] = tr * ga;
            } else {
                const float tn = 1.0f - A;
                float dot = 0.f;
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) {
                    float diff = (CK[ch].hi - C[ch].hi) + (CK[ch].lo - C[ch].lo);
                    dot = __builtin_fmaf(gc[ch], diff, dot);
                }
                g[3] = -tr * (dot - ga * TK) / tn;
            }
            const int e0 = E - 3 * l0;
            const float w0 = 1.0f - f;
#pragma unroll
            for (int q = 0; q < 8; ++q) emit(acc, tp0.idx[q], w0 * tp0.w[q], g, e0);
            if (f > 0.0f) {
                const int e1 = E - 3 * l1;
#pragma unroll
                for (int q = 0; q < 8; ++q) emit(acc, tp1.idx[q], f * tp1.w[q], g, e1);
            }
            t = df_add(t, a.step_factor * d);
        }
    }
}

}  // namespace vct
