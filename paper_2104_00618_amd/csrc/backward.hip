// Adjoint of the cone trace with respect to the base grid (step counts held
// fixed), transmittance recomputed by re-marching instead of stored.
//
// Per cone with samples s_k = (c_k, a_k), T_k = 1 - A_k and totals (C_K, A_K):
//   dL/dc_k = T_k dL/dC
//   dL/da_k = -T_k (dL/dC . (C_K - C_{k+1}) - dL/dA T_K) / T_{k+1}   (k < K-1)
//   dL/da_{K-1} = T_{K-1} dL/dA
// (derivatives of the front-to-back recurrences of Section 4.3.2).  While a
// cone continues, A_{k+1} < alpha_thresh, so T_{k+1} > 1 - alpha_thresh and,
// since T is computed as 1 - A in float32, T_{k+1} >= 2^-24 in any case.
// C is accumulated as a double-float in both passes so that C_K - C_{k+1} is
// accurate to ~1e-14 of C_K.
//
// Deterministic reduction: every tap contribution g * w is converted to a
// 64-bit fixed-point integer with a per-call power-of-two scale 2^E (level l
// uses 2^(E - 3l), folding the 1/8 of each mip level into the scale) and added
// with integer atomics.  Integer addition is exact and associative, so the
// result is bitwise independent of execution order.  E is chosen from a bound
// on the sum of |contributions| computed in pass 1 so that no partial sum can
// exceed 2^62.  The mip adjoint (each child receives 1/8 of its parent's
// gradient) is then a gather: grad_base[x] = 2^-E * sum_l acc_l[ancestor_l(x)].
//
// Kernels, in stream order:
//   k_fill_zero   clear the accumulator
//   k_bwd_pass1   per pixel: re-march every cone, store (C_K, A_K, K), and the
//                 workgroup's sum of per-cone contribution bounds
//   k_bwd_scale   one workgroup: fixed-order sum of the bounds -> E
//   k_bwd_pass2   per pixel: re-march, emit fixed-point tap gradients
//   k_mip_adjoint per 2x2x2 block of base texels: gather over levels, convert to float32
//
// Anisotropic pyramids (Section 5.1.3) use the same kernels instantiated for
// six directional pyramids: every level accumulates at the scale 2^E, and
// k_aniso_adjoint, one launch per level from the top, replaces k_mip_adjoint
// (the adjoint of a directional texel depends on the stored texels, so it is
// no longer a fixed factor per level).
#include "bwd_pixel.h"

namespace {

using namespace vct;

constexpr int kThreads = 256;

template <int DT, bool ANISO>
__global__ __launch_bounds__(kThreads, 4) void k_bwd_pass1(TraceArgs a, const float4* __restrict__ gout,
                                                        LaneState* __restrict__ state, float* __restrict__ part) {
    __shared__ LevelTable T;
    __shared__ DirSlot<ANISO> D;
    __shared__ float s_part[kThreads / 64];
    load_level_table(a, &T);
    load_dir_table(a, &D);
    __syncthreads();
    const int tile = xcd_tile(blockIdx.x, a.n_tiles);
    int view, y, x;
    tile_pixel(a, tile, threadIdx.x, view, y, x);
    float bound = 0.f;
    if (x < a.w && y < a.h)
        bound = pass1_pixel<DT, ANISO>(a, T, gout, state, view, ((size_t)view * a.h + y) * a.w + x, dir_ptr(D));
    // fixed-order workgroup sum
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int o = 32; o > 0; o >>= 1) bound += __shfl_xor(bound, o, 64);
    if (lane == 0) s_part[wv] = bound;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = (s_part[0] + s_part[1]) + (s_part[2] + s_part[3]);
}

// Forward that also saves every cone's end state (training path: the
// backward then skips pass 1).
template <int DT, bool ANISO>
__global__ __launch_bounds__(kThreads, 4) void k_trace_save(TraceArgs a, float4* __restrict__ out,
                                                         LaneState* __restrict__ state) {
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
    float4 o0, o1;
    trace_save_pixel<DT, ANISO>(a, T, view, pix, state, o0, o1, dir_ptr(D));
    out[2 * pix] = o0;
    out[2 * pix + 1] = o1;
}

// Per-workgroup bound sums from saved lane states (same tiles and summation
// order as pass 1, so the scale exponent is the same).
__global__ __launch_bounds__(kThreads) void k_bwd_bound(TraceArgs a, const float4* __restrict__ gout,
                                                        const LaneState* __restrict__ state, float* __restrict__ part) {
    __shared__ float s_part[kThreads / 64];
    const int tile = xcd_tile(blockIdx.x, a.n_tiles);
    int view, y, x;
    tile_pixel(a, tile, threadIdx.x, view, y, x);
    float bound = 0.f;
    if (x < a.w && y < a.h) bound = saved_bound_pixel(a, gout, state, ((size_t)view * a.h + y) * a.w + x);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int o = 32; o > 0; o >>= 1) bound += __shfl_xor(bound, o, 64);
    if (lane == 0) s_part[wv] = bound;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = (s_part[0] + s_part[1]) + (s_part[2] + s_part[3]);
}

// ctl[0] = E, ctl[1] = 1 if the bound is not finite
__global__ __launch_bounds__(kThreads) void k_bwd_scale(const float* __restrict__ part, int n, int* __restrict__ ctl) {
    __shared__ float s[kThreads];
    float acc = 0.f;
    for (int i = threadIdx.x; i < n; i += kThreads) acc += part[i];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        float total = s[0];
        int E = 0, bad = 0;
        if (!isfinite(total)) {
            bad = 1;
        } else if (total > 0.f) {
            int ex;
            frexpf(total, &ex);     // total < 2^ex
            E = 61 - ex;            // total * 2^E < 2^61
        }
        ctl[0] = E;
        ctl[1] = bad;
    }
}

// Cross-lane moves of the reduction butterfly.  Each pairs lane i with
// i ^ mask: row_mirror (^15), row_half_mirror (^7) and the quad permutes (^2,
// ^1) are DPP modifiers of ordinary VALU instructions; ^16 and ^32 are the
// permlane16 / permlane32 swaps of gfx950.
template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, true));
}
constexpr int kDppXor15 = 0x140;   // row_mirror
constexpr int kDppXor7 = 0x141;    // row_half_mirror
constexpr int kDppXor2 = 0x4E;     // quad_perm [2,3,0,1]
constexpr int kDppXor1 = 0xB1;     // quad_perm [1,0,3,2]

// Given lo and hi, lanes with bit 4 clear return lo[i] + lo[i ^ 16] and lanes
// with bit 4 set hi[i ^ 16] + hi[i] (the swap exchanges the odd 16-lane rows
// of its first operand with the even rows of its second).
__device__ __forceinline__ float split16(float lo, float hi) {
    const auto s = __builtin_amdgcn_permlane16_swap(__float_as_uint(lo), __float_as_uint(hi), false, false);
    return __uint_as_float(s[0]) + __uint_as_float(s[1]);
}
// v[i] + v[i ^ 16] and v[i] + v[i ^ 32] in every lane.
__device__ __forceinline__ float sum16(float v) { return split16(v, v); }
__device__ __forceinline__ float sum32(float v) {
    const auto s = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    return __uint_as_float(s[0]) + __uint_as_float(s[1]);
}

// Role of a lane in the tap-gradient butterfly.  The 32 values of a sample
// are w[q] * g[c] (tap q = 4 z + 2 y + x, channel c).  Lane i keeps the value
// (q, c) in register slot 4 (q ^ qm) + (c ^ cm), where every bit of the masks
// is the parity of a set of lane bits: z = i3, y = i2 ^ i3, x = i1 ^ i2 and
// channel bit 1 = i0 ^ i2.  Each of these parities flips under the lane mask
// of the butterfly stage that splits on its bit (15, 7, 2, 1) and under no
// earlier or later stage, so partners always hold the same value in the same
// slot and every stage adds the partner's upper half to the own lower half,
// with no per-lane selects.  The final split (^16) is a permlane16 swap, after
// which lane i holds tap qm, channel cm + i4; lanes i and i ^ 32 agree.
struct EmitLane {
    bool xf, yf, zf;        // tap bits of the sum this lane ends with
    bool cf;                // channel bit 1 of that sum
    uint32_t xm, ym, zm;    // all-ones where xf / yf / zf
    int ch;                 // channel of that sum
};

__device__ __forceinline__ EmitLane emit_lane(int lane) {
    const int b0 = lane & 1, b1 = (lane >> 1) & 1, b2 = (lane >> 2) & 1, b3 = (lane >> 3) & 1, b4 = (lane >> 4) & 1;
    EmitLane e;
    e.zf = b3;
    e.yf = b2 ^ b3;
    e.xf = b1 ^ b2;
    e.cf = b0 ^ b2;
    e.xm = e.xf ? ~0u : 0u;
    e.ym = e.yf ? ~0u : 0u;
    e.zm = e.zf ? ~0u : 0u;
    e.ch = (b0 ^ b2) * 2 + b4;
    return e;
}

// Sum over the wave of w[q] * g[c] for this lane's (q, c) (see EmitLane):
// wp = the lane's weights in slot order, wpart[k] = wp[k + 4] of the ^15
// partner, g = the lane's gradient in slot order (zero outside the group).
// 4 DPP moves, 32 multiply-adds, 14 DPP adds and two permlane swaps; the
// addition order is fixed, so the sums are reproducible.
__device__ __forceinline__ float bfly32(const float wp[8], const float wpart[4], const float g[4]) {
    float gpart[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) gpart[m] = dpp<kDppXor15>(g[m]);
    float r[16];
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int m = 0; m < 4; ++m) r[4 * k + m] = __builtin_fmaf(wp[k], g[m], wpart[k] * gpart[m]);
#pragma unroll
    for (int i = 0; i < 8; ++i) r[i] += dpp<kDppXor7>(r[i + 8]);
#pragma unroll
    for (int i = 0; i < 4; ++i) r[i] += dpp<kDppXor2>(r[i + 4]);
#pragma unroll
    for (int i = 0; i < 2; ++i) r[i] += dpp<kDppXor1>(r[i + 2]);
    return sum32(split16(r[0], r[1]));
}

// Alpha-only variant (occlusion cones carry no colour gradient): the sum of
// w[q] * ga for q = qm; lanes with bits 0, 4 and 5 clear emit it.
__device__ __forceinline__ float bfly8(const float wp[8], const float wpart[4], float g) {
    const float gpart = dpp<kDppXor15>(g);
    float r[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) r[k] = __builtin_fmaf(wp[k], g, wpart[k] * gpart);
    r[0] += dpp<kDppXor7>(r[2]);
    r[1] += dpp<kDppXor7>(r[3]);
    r[0] += dpp<kDppXor2>(r[1]);
    r[0] += dpp<kDppXor1>(r[0]);
    return sum32(sum16(r[0]));
}

// The lane's slot-ordered weights of one level's 8 taps, level weight wl
// folded in (an axis that clamps has both taps on one texel, each with its
// own weight).
__device__ __forceinline__ void emit_weights(const LevelGeom& g, float wl, const EmitLane& e, float wp[8]) {
    const float x0 = 1.0f - g.wx, y0 = 1.0f - g.wy, z0 = 1.0f - g.wz;
    const float xa = e.xf ? g.wx : x0, xb = e.xf ? x0 : g.wx;
    const float ya = e.yf ? g.wy : y0, yb = e.yf ? y0 : g.wy;
    const float za = e.zf ? g.wz : z0, zb = e.zf ? z0 : g.wz;
    const float wxy[4] = {xa * ya, xb * ya, xa * yb, xb * yb};
#pragma unroll
    for (int k = 0; k < 8; ++k) wp[k] = wl * (wxy[k & 3] * ((k >> 2) ? zb : za));
}

// A group's fixed-point values held back while the wave's next samples on the
// same level parity fall on the same footprint (same base texel and clamp
// pattern): they are summed in registers and added to the accumulator once.
// Integer addition is associative, so the accumulator ends bitwise the same
// as with one atomic per sample.  The key and the index steps are
// wave-uniform; qv is the lane's value (zero outside the emitting lanes).
struct Held {
    uint32_t key;          // base texel, kNoKey when empty
    int kc;                // clamp pattern
    uint32_t dx, dy, dz;   // index steps of the footprint
    long long qv;
};
constexpr uint32_t kNoKey = 0xffffffffu;

// Add a lane's value for texel idx, channel ch to the workgroup's LDS table
// (coarse levels) or to the global accumulator.
__device__ __forceinline__ void add_fixed(uint32_t idx, int ch, long long qv, unsigned long long* __restrict__ acc,
                                          unsigned long long* small, uint32_t small_off) {
    VCT_CHECK_ACC(idx);
    if (qv != 0 && idx >= small_off) atomicAdd(&small[(idx - small_off) * 4 + ch], (unsigned long long)qv);
    if (qv != 0 && idx < small_off) atomicAdd(&acc[(size_t)idx * 4 + ch], (unsigned long long)qv);
}

__device__ __forceinline__ void flush_held(Held& h, const EmitLane& e, int ch, unsigned long long* __restrict__ acc,
                                           unsigned long long* small, uint32_t small_off) {
    if (h.key != kNoKey)
        add_fixed(h.key + (h.dx & e.xm) + (h.dy & e.ym) + (h.dz & e.zm), ch, h.qv, acc, small, small_off);
    h.key = kNoKey;
}

__device__ __forceinline__ void hold(Held& h, uint32_t k, int kc, uint32_t dx, uint32_t dy, uint32_t dz, long long qv,
                                     const EmitLane& e, int ch, unsigned long long* __restrict__ acc,
                                     unsigned long long* small, uint32_t small_off) {
    if (h.key == k && h.kc == kc) {
        h.qv += qv;
        return;
    }
    flush_held(h, e, ch, acc, small, small_off);
    h.key = k;
    h.kc = kc;
    h.dx = dx;
    h.dy = dy;
    h.dz = dz;
    h.qv = qv;
}

// The group loop of one level's emission.  Lanes whose samples share the
// same base texel and clamp pattern have the same 8 taps; each such group is
// summed across the wave (fixed order), after which 32 lanes (8 for alpha
// only) hold its taps x channels.  sink(k, kc, lev, dx, dy, dz, sum, emitter,
// ch) receives each group: its base texel, clamp pattern, level and index
// steps (wave-uniform), the lane's sum, whether the lane emits it, and its
// channel.
template <bool ALPHA_ONLY, typename Sink>
__device__ __forceinline__ void emit_groups(bool live, const LevelGeom& geo, float wl, const float gs[4],
                                            const EmitLane& e, int lane, Sink&& sink) {
    unsigned long long mask = __ballot(live);
    if (mask == 0) return;   // (wave-uniform: no lane emits on this level)
    float wp[8];
    emit_weights(geo, wl, e, wp);
    float wpart[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) wpart[k] = dpp<kDppXor15>(wp[k + 4]);
    const uint32_t key = live ? geo.base : 0xffffffffu;
    const int kcl = (geo.dx == 0 ? 1 : 0) | (geo.dy == 0 ? 2 : 0) | (geo.dz == 0 ? 4 : 0);
    const bool emitter = ALPHA_ONLY ? ((lane & 0x31) == 0) : (lane < 32);
    const int ch = ALPHA_ONLY ? 3 : e.ch;
    while (mask) {
        const int leader = __builtin_ctzll(mask);
        const uint32_t k = (uint32_t)__builtin_amdgcn_readlane((int)key, leader);
        const int kc = __builtin_amdgcn_readlane(kcl, leader);
        const bool in = live && key == k && kcl == kc;
        const unsigned long long gm = __ballot(in);
        float sum;
        if (ALPHA_ONLY) {
            sum = bfly8(wp, wpart, in ? gs[3] : 0.f);
        } else {
            float g[4];
#pragma unroll
            for (int m = 0; m < 4; ++m) g[m] = in ? gs[m] : 0.f;
            sum = bfly32(wp, wpart, g);
        }
        const int lev = __builtin_amdgcn_readlane(geo.level, leader);
        const uint32_t dx = (uint32_t)__builtin_amdgcn_readlane((int)geo.dx, leader);
        const uint32_t dy = (uint32_t)__builtin_amdgcn_readlane((int)geo.dy, leader);
        const uint32_t dz = (uint32_t)__builtin_amdgcn_readlane((int)geo.dz, leader);
        sink(k, kc, lev, dx, dy, dz, sum, emitter, ch);
        mask &= ~gm;
    }
}

// Emit one level's tap gradients of the wave as fixed-point integers: to the
// workgroup's LDS table for the coarse levels (side <= 8), to the global
// accumulator otherwise.
template <bool ALPHA_ONLY, bool HOLD = false>
__device__ __forceinline__ void emit_level(bool live, const LevelGeom& geo, float wl, const float gs[4],
                                           const EmitLane& e, int E, int lev_shift,
                                           unsigned long long* __restrict__ acc, unsigned long long* small,
                                           uint32_t small_off, int lane, Held* held = nullptr) {
    emit_groups<ALPHA_ONLY>(live, geo, wl, gs, e, lane,
                            [&](uint32_t k, int kc, int lev, uint32_t dx, uint32_t dy, uint32_t dz, float sum,
                                bool emitter, int ch) {
        const long long qv = emitter ? fixed_point(sum, E - lev_shift * lev) : 0;
        if constexpr (HOLD) {
            // (the two levels of a sample differ in parity, and a level keeps
            // its parity stream as the march moves up)
            if (lev & 1)
                hold(held[1], k, kc, dx, dy, dz, qv, e, ch, acc, small, small_off);
            else
                hold(held[0], k, kc, dx, dy, dz, qv, e, ch, acc, small, small_off);
        } else {
            add_fixed(k + (dx & e.xm) + (dy & e.ym) + (dz & e.zm), ch, qv, acc, small, small_off);
        }
    });
}

// Anisotropic pyramids above level 0, when every emitting lane of the wave has
// the same cone axis (so the same direction weights w_a^2 and direction
// signs): the three directions' sums are the axis-free sum times w_a^2, so
// each group runs one butterfly and adds it at the three directions' offsets.
template <bool ALPHA_ONLY>
__device__ __forceinline__ void emit_level_dirs(bool live, const LevelGeom& geo, float wl, const float gs[4],
                                                const EmitLane& e, int E, const float wt[3], const int dsel[3],
                                                const DirTable* D, unsigned long long* __restrict__ acc,
                                                unsigned long long* small, uint32_t small_off, int lane) {
    emit_groups<ALPHA_ONLY>(live, geo, wl, gs, e, lane,
                            [&](uint32_t k, int, int lev, uint32_t dx, uint32_t dy, uint32_t dz, float sum,
                                bool emitter, int ch) {
        const uint32_t tap = k + (dx & e.xm) + (dy & e.ym) + (dz & e.zm);
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            if (wt[ax] == 0.0f) continue;
            const long long qv = emitter ? fixed_point(sum * wt[ax], E) : 0;
            add_fixed(tap + D->delta[dsel[ax]][lev], ch, qv, acc, small, small_off);
        }
    });
}

// Anisotropic pyramids above level 0, when the wave's lanes have different
// cone axes: lanes are grouped by footprint and by the signs of their axis
// (which pick the three directional pyramids, so each direction's offset is
// uniform in a group), once for the three directions; each group then runs
// one butterfly per axis, with the lane's gradient scaled by its w_a^2 for
// that axis, and adds the sum at that direction's offset.  (Grouping once in
// place of once per direction: the group loop, the slot-order weights and the
// clamp key are shared by the three.)
template <bool ALPHA_ONLY>
__device__ __forceinline__ void emit_level_axes(bool live, const LevelGeom& geo, float wl, const float gs[4],
                                                const EmitLane& e, int E, const float wt[3], int sgn,
                                                const DirTable* D, unsigned long long* __restrict__ acc,
                                                unsigned long long* small, uint32_t small_off, int lane) {
    unsigned long long mask = __ballot(live);
    if (mask == 0) return;   // (wave-uniform)
    float wp[8];
    emit_weights(geo, wl, e, wp);
    float wpart[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) wpart[k] = dpp<kDppXor15>(wp[k + 4]);
    const uint32_t key = live ? geo.base : 0xffffffffu;
    const int kcl = (geo.dx == 0 ? 1 : 0) | (geo.dy == 0 ? 2 : 0) | (geo.dz == 0 ? 4 : 0) | (sgn << 3);
    const bool emitter = ALPHA_ONLY ? ((lane & 0x31) == 0) : (lane < 32);
    const int ch = ALPHA_ONLY ? 3 : e.ch;
    while (mask) {
        const int leader = __builtin_ctzll(mask);
        const uint32_t k = (uint32_t)__builtin_amdgcn_readlane((int)key, leader);
        const int kc = __builtin_amdgcn_readlane(kcl, leader);
        const bool in = live && key == k && kcl == kc;
        const unsigned long long gm = __ballot(in);
        const int lev = __builtin_amdgcn_readlane(geo.level, leader);
        const uint32_t dx = (uint32_t)__builtin_amdgcn_readlane((int)geo.dx, leader);
        const uint32_t dy = (uint32_t)__builtin_amdgcn_readlane((int)geo.dy, leader);
        const uint32_t dz = (uint32_t)__builtin_amdgcn_readlane((int)geo.dz, leader);
        const uint32_t tap = k + (dx & e.xm) + (dy & e.ym) + (dz & e.zm);
        const int sg = kc >> 3;
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            float sum;
            if (ALPHA_ONLY) {
                sum = bfly8(wp, wpart, in ? gs[3] * wt[ax] : 0.f);
            } else {
                float g[4];
#pragma unroll
                for (int m = 0; m < 4; ++m) g[m] = in ? gs[m] * wt[ax] : 0.f;
                sum = bfly32(wp, wpart, g);
            }
            const long long qv = emitter ? fixed_point(sum, E) : 0;
            add_fixed(tap + D->delta[2 * ax + ((sg >> ax) & 1)][lev], ch, qv, acc, small, small_off);
        }
        mask &= ~gm;
    }
}

// One level's emission.  Isotropic pyramids: level l's integers carry the
// scale 2^(E - 3l) (the 1/8 per level of the mip adjoint folded in).
// Anisotropic pyramids: scale 2^E at every level (their mip adjoint is not a
// fixed factor); above level 0 the sample read the three directions of its
// axis signs with weights w_a^2, so each gets the gradient with that weight at
// its direction's offset: with one butterfly per group when the wave's lanes
// share their axis (emit_level_dirs), else one per axis in a group keyed by the
// footprint and the axis's signs (emit_level_axes).
template <bool ALPHA_ONLY, bool ANISO, bool HOLD>
__device__ __forceinline__ void emit_dirs(const TraceArgs& a, const DirTable* D, const Cone& c, bool live,
                                          const LevelGeom& geo, float wl, const float gs[4], const EmitLane& e, int E,
                                          unsigned long long* __restrict__ acc, unsigned long long* small,
                                          uint32_t small_off, int lane, Held* held) {
    if constexpr (!ANISO) {
        emit_level<ALPHA_ONLY, HOLD>(live, geo, wl, gs, e, E, 3, acc, small, small_off, lane, held);
    } else {
        const bool base_level = live && geo.level == 0;
        emit_level<ALPHA_ONLY>(base_level, geo, wl, gs, e, E, 0, acc, small, small_off, lane);
        const float W[3] = {c.Wx, c.Wy, c.Wz};
        const bool up = live && !base_level;
        const unsigned long long upm = __ballot(up);
        if (upm == 0) return;
        const int ld = __builtin_ctzll(upm);
        const float Wl[3] = {__int_as_float(__builtin_amdgcn_readlane(__float_as_int(W[0]), ld)),
                             __int_as_float(__builtin_amdgcn_readlane(__float_as_int(W[1]), ld)),
                             __int_as_float(__builtin_amdgcn_readlane(__float_as_int(W[2]), ld))};
        const bool same = __float_as_int(W[0]) == __float_as_int(Wl[0]) &&
                          __float_as_int(W[1]) == __float_as_int(Wl[1]) &&
                          __float_as_int(W[2]) == __float_as_int(Wl[2]);
        if (__ballot(up && !same) == 0) {
            float wt[3];
            int dsel[3];
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) {
                wt[ax] = Wl[ax] * Wl[ax] * a.inv_scale2;
                dsel[ax] = 2 * ax + (Wl[ax] < 0.0f ? 1 : 0);
            }
            emit_level_dirs<ALPHA_ONLY>(up, geo, wl, gs, e, E, wt, dsel, D, acc, small, small_off, lane);
            return;
        }
        // (a lane of a pixel with no surface has no cone and its W is whatever
        // the registers held: its axis weights and signs are only read through
        // the group test, which such a lane never passes)
        float wt[3];
        int sgn = 0;
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            wt[ax] = W[ax] * W[ax] * a.inv_scale2;
            sgn |= (W[ax] < 0.0f ? 1 : 0) << ax;
        }
        emit_level_axes<ALPHA_ONLY>(up, geo, wl, gs, e, E, wt, sgn, D, acc, small, small_off, lane);
    }
}

constexpr int kSmallMax = 704;        // texels of all levels with side <= 8 (8^3 + 3 bricks of 64)
constexpr int kSmallMaxAniso = 1152;  // anisotropic: levels with side <= 4 of six directions (6 x 3 bricks)

template <int DT, bool ANISO>
__global__ __launch_bounds__(kThreads, 4) void k_bwd_pass2(TraceArgs a, const float4* __restrict__ gout,
                                                        const LaneState* __restrict__ state,
                                                        const int* __restrict__ ctl,
                                                        unsigned long long* __restrict__ acc, uint32_t small_off,
                                                        int small_n) {
    __shared__ LevelTable T;
    __shared__ DirSlot<ANISO> D;
    __shared__ unsigned long long s_small[(ANISO ? kSmallMaxAniso : kSmallMax) * 4];
    load_level_table(a, &T);
    load_dir_table(a, &D);
    for (int i = threadIdx.x; i < small_n * 4; i += kThreads) s_small[i] = 0ull;
    __syncthreads();
    const int E = ctl[0];
    const int lane = threadIdx.x & 63;
    const int tile = xcd_tile(blockIdx.x, a.n_tiles);
    int view, y, x;
    tile_pixel(a, tile, threadIdx.x, view, y, x);
    const bool inb = x < a.w && y < a.h;
    const size_t pix = inb ? ((size_t)view * a.h + y) * a.w + x : 0;
    const bool valid = inb && a.normal[pix].w != 0.0f;
    const int nslots = a.n_diffuse + 2;
    const EmitLane e = emit_lane(lane);
    for (int slot = 0; slot < nslots; ++slot) {
        if (!slot_enabled(a, slot)) continue;
        Pass2Lane L;
        L.K = 0;
        if (valid) {
            // pixel setup and dL/d(out) are reloaded per cone to keep registers free
            const PixelSetup P = pixel_setup(a, a.pos_rough[pix], a.normal[pix]);
            const float3 cam = make_float3(a.cam_pos[3 * view], a.cam_pos[3 * view + 1], a.cam_pos[3 * view + 2]);
            pass2_init(a, P, cam, gout[2 * pix], gout[2 * pix + 1], lane_get(a, state, pix, slot), slot,
                       L);
        }
        int Kw = L.K;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) Kw = max(Kw, __shfl_xor(Kw, o));
        Kw = __builtin_amdgcn_readfirstlane(Kw);   // (equal in every lane: the loop is wave-uniform)
        const bool occ = slot == a.n_diffuse + 1;
        // Held emissions (isotropic pyramids; the anisotropic ones emit four
        // interleaved direction keys per level and add every group at once).
        constexpr bool kHold = !ANISO;
        Held held[2];
        held[0].key = held[1].key = kNoKey;
        held[0].kc = held[1].kc = 0;
        held[0].dx = held[0].dy = held[0].dz = held[1].dx = held[1].dy = held[1].dz = 0u;
        held[0].qv = held[1].qv = 0;
        for (int k = 0; k < Kw; ++k) {
            const bool live = k < L.K;
            // lanes past their K only need finite weights for the butterfly
            Pass2Step st;
            st.f = 0.f;
            st.g0.wx = st.g0.wy = st.g0.wz = 0.f;
            st.g1.wx = st.g1.wy = st.g1.wz = 0.f;
            if constexpr (ANISO) st.g0.level = st.g1.level = 0;   // (a dead lane's direction-table row)
            if (live) pass2_step<DT, ANISO>(a, T, L, k, st, dir_ptr(D));
            if (occ) {
                emit_dirs<true, ANISO, kHold>(a, dir_ptr(D), L.c, live, st.g0, 1.0f - st.f, st.g, e, E, acc,
                                              s_small, small_off, lane, held);
                emit_dirs<true, ANISO, kHold>(a, dir_ptr(D), L.c, live && st.f > 0.0f, st.g1, st.f, st.g, e, E,
                                              acc, s_small, small_off, lane, held);
            } else {
                // gradient in the lane's slot order (channel bit 1 flipped where cf);
                // selects on values: an index select would move st to scratch memory
                const float g0 = st.g[0], g1 = st.g[1], g2 = st.g[2], g3 = st.g[3];
                const float gs[4] = {e.cf ? g2 : g0, e.cf ? g3 : g1, e.cf ? g0 : g2, e.cf ? g1 : g3};
                emit_dirs<false, ANISO, kHold>(a, dir_ptr(D), L.c, live, st.g0, 1.0f - st.f, gs, e, E, acc,
                                               s_small, small_off, lane, held);
                emit_dirs<false, ANISO, kHold>(a, dir_ptr(D), L.c, live && st.f > 0.0f, st.g1, st.f, gs, e, E,
                                               acc, s_small, small_off, lane, held);
            }
        }
        if constexpr (kHold) {
            // (the occlusion cone's values are all channel 3)
            flush_held(held[0], e, occ ? 3 : e.ch, acc, s_small, small_off);
            flush_held(held[1], e, occ ? 3 : e.ch, acc, s_small, small_off);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < small_n * 4; i += kThreads) {
        const unsigned long long v = s_small[i];
        if (v) atomicAdd(&acc[(size_t)small_off * 4 + i], v);
    }
}

__global__ void k_fill_zero(uint4* __restrict__ p, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = make_uint4(0u, 0u, 0u, 0u);
}

struct AdjArgs {
    int32_t n, levels;
    int32_t nb[VCT_MAX_LEVELS];
    uint32_t off[VCT_MAX_LEVELS];
};

// Two threads per 2x2x2 block of base texels (a level-1 texel), one for each
// x half: the sum of the block's ancestors on levels >= 1 is shared by the
// four children a thread writes, so the coarse levels are read twice per block
// rather than once per texel.  Lane pairs take the two x halves, so every
// store instruction writes whole 128-byte rows of the gradient (8 texels in
// x), and a wave reads whole lines of the base-level accumulator.  Integer
// sums, so the result does not depend on this grouping.
__global__ __launch_bounds__(256) void k_mip_adjoint(AdjArgs m, const long long* __restrict__ acc,
                                                     const int* __restrict__ ctl, float4* __restrict__ grad) {
    const int E = ctl[0];
    const bool bad = ctl[1] != 0;
    const int n = m.n;
    const int nh = (n + 1) >> 1;             // blocks a side
    const uint32_t nbh = (uint32_t)(nh + 3) >> 2;
    const uint32_t total = nbh * nbh * nbh * 128u;
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < total; t += gridDim.x * blockDim.x) {
        const uint32_t brick = t >> 7, w = (t >> 1) & 63u;
        const int dx = (int)(t & 1u);
        const int bx = (int)(brick % nbh) * 4 + (int)(w & 3u);
        const int by = (int)((brick / nbh) % nbh) * 4 + (int)((w >> 2) & 3u);
        const int bz = (int)(brick / (nbh * nbh)) * 4 + (int)(w >> 4);
        const int x = 2 * bx + dx;
        if (bx >= nh || by >= nh || bz >= nh || x >= n) continue;   // (x >= n: n = 1)
        long long a0 = 0, a1 = 0, a2 = 0, a3 = 0;
#pragma unroll
        for (int l = 1; l < VCT_MAX_LEVELS; ++l) {
            if (l < m.levels) {
                const uint32_t idx = m.off[l] + vct_brick_index(bx >> (l - 1), by >> (l - 1), bz >> (l - 1), m.nb[l]);
                const longlong2 u = reinterpret_cast<const longlong2*>(acc + (size_t)idx * 4)[0];
                const longlong2 v = reinterpret_cast<const longlong2*>(acc + (size_t)idx * 4)[1];
                a0 += u.x;
                a1 += u.y;
                a2 += v.x;
                a3 += v.y;
            }
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int y = 2 * by + (c & 1), z = 2 * bz + (c >> 1);
            if (y >= n || z >= n) continue;   // (n = 1)
            const long long* p = acc + (size_t)(m.off[0] + vct_brick_index(x, y, z, m.nb[0])) * 4;
            const longlong2 u = reinterpret_cast<const longlong2*>(p)[0];
            const longlong2 v = reinterpret_cast<const longlong2*>(p)[1];
            float4 g;
            if (bad) {
                g = make_float4(__int_as_float(0x7fc00000), __int_as_float(0x7fc00000), __int_as_float(0x7fc00000),
                                __int_as_float(0x7fc00000));
            } else {
                g = make_float4(ldexpf((float)(a0 + u.x), -E), ldexpf((float)(a1 + u.y), -E),
                                ldexpf((float)(a2 + v.x), -E), ldexpf((float)(a3 + v.y), -E));
            }
            grad[((size_t)z * n + y) * n + x] = g;
        }
    }
}

// Mip adjoint of anisotropic pyramids, one launch per level from the top
// down.  The gradient of a directional texel is its own accumulated sum plus
// what its parent (same direction, one level up) passes through the
// linearised front-to-back composite: parent = (1/4) sum over the four child
// pairs along the direction's axis of over(f, b) = f + (1 - f.a) b, so the
// front child gets (G - e_a (G . b)) / 4 and the back child (1 - f.a) G / 4,
// with f, b the stored texels of the pair.  Levels >= 1 keep their float32
// gradient in the first 16 bytes of their own accumulator slot (one writer
// per slot, parents final before their children run); level 0 sums the six
// directions' contributions in order and writes the base gradient.
struct AnisoAdj {
    int32_t n, levels, level;          // level processed (its parents are level + 1)
    int32_t nb[VCT_MAX_LEVELS];
    uint32_t doff[6][VCT_MAX_LEVELS];
};

__device__ __forceinline__ float4 scaled(const long long* p, int E) {
    const longlong2 u = reinterpret_cast<const longlong2*>(p)[0];
    const longlong2 v = reinterpret_cast<const longlong2*>(p)[1];
    return make_float4(ldexpf((float)u.x, -E), ldexpf((float)u.y, -E), ldexpf((float)v.x, -E),
                       ldexpf((float)v.y, -E));
}

template <int DT>
__device__ __forceinline__ float4 from_parent(const AnisoAdj& m, const void* pyr, const long long* acc, int d, int x,
                                              int y, int z) {
    const int c = m.level, nbp = m.nb[c + 1];
    const float4 G = *reinterpret_cast<const float4*>(
        acc + (size_t)(m.doff[d][c + 1] + vct_brick_index(x >> 1, y >> 1, z >> 1, nbp)) * 4);
    const int axis = d >> 1;
    const int coord = axis == 0 ? x : (axis == 1 ? y : z);
    const bool front = ((coord & 1) == 0) == ((d & 1) == 0);
    const int px = axis == 0 ? x ^ 1 : x, py = axis == 1 ? y ^ 1 : y, pz = axis == 2 ? z ^ 1 : z;
    const float4 q = vct_load_texel<DT & ~VCT_WIDE>(pyr, m.doff[d][c] + vct_brick_index(px, py, pz, m.nb[c]));
    if (front) {
        const float gb = G.x * q.x + G.y * q.y + G.z * q.z + G.w * q.w;
        return make_float4(0.25f * G.x, 0.25f * G.y, 0.25f * G.z, 0.25f * (G.w - gb));
    }
    const float t = 0.25f * (1.0f - q.w);
    return make_float4(t * G.x, t * G.y, t * G.z, t * G.w);
}

template <int DT>
__global__ __launch_bounds__(256) void k_aniso_adjoint(AnisoAdj m, long long* __restrict__ acc, const void* pyr,
                                                       const int* __restrict__ ctl, float4* __restrict__ grad) {
    const int E = ctl[0];
    const bool bad = ctl[1] != 0;
    const int c = m.level, side = m.n >> c, nb = m.nb[c];
    const bool top = c == m.levels - 1;
    const uint32_t t = blockIdx.x * 256u + threadIdx.x;
    const uint32_t brick = t >> 6, w = t & 63u;
    if (brick >= (uint32_t)nb * nb * nb) return;
    const int x = (int)(brick % nb) * 4 + (int)(w & 3u), y = (int)((brick / nb) % nb) * 4 + (int)((w >> 2) & 3u),
              z = (int)(brick / ((uint32_t)nb * nb)) * 4 + (int)(w >> 4);
    if (x >= side || y >= side || z >= side) return;
    const uint32_t at = vct_brick_index(x, y, z, nb);
    if (c == 0) {
        float4 g = scaled(acc + (size_t)at * 4, E);
        if (!top)
            for (int d = 0; d < 6; ++d) {
                const float4 p = from_parent<DT>(m, pyr, acc, d, x, y, z);
                g.x += p.x;
                g.y += p.y;
                g.z += p.z;
                g.w += p.w;
            }
        if (bad) g = make_float4(__int_as_float(0x7fc00000), __int_as_float(0x7fc00000), __int_as_float(0x7fc00000),
                                 __int_as_float(0x7fc00000));
        grad[((size_t)z * m.n + y) * m.n + x] = g;
        return;
    }
    for (int d = 0; d < 6; ++d) {
        long long* slot = acc + (size_t)(m.doff[d][c] + at) * 4;
        float4 g = scaled(slot, E);
        if (!top) {
            const float4 p = from_parent<DT>(m, pyr, acc, d, x, y, z);
            g.x += p.x;
            g.y += p.y;
            g.z += p.z;
            g.w += p.w;
        }
        *reinterpret_cast<float4*>(slot) = g;
    }
}

template <int DT, bool ANISO>
hipError_t run_backward(const PyrLayout& L, const TraceArgs& a, const BackwardPlan& P, const float* grad_out,
                        float* grad_base, void* ws, const void* saved, hipStream_t s, EventSink& es) {
    char* w = static_cast<char*>(ws);
    unsigned long long* acc = reinterpret_cast<unsigned long long*>(w + P.acc_off);
    LaneState* state = saved ? reinterpret_cast<LaneState*>(const_cast<void*>(saved))
                             : reinterpret_cast<LaneState*>(w + P.state_off);
    float* part = reinterpret_cast<float*>(w + P.part_off);
    int* ctl = reinterpret_cast<int*>(w + P.ctl_off);
    size_t n16 = (size_t)P.acc_bytes / 16;
    int fb = (int)((n16 + 255) / 256);
    if (fb > 8192) fb = 8192;
    es.mark(s);
    hipLaunchKernelGGL(k_fill_zero, dim3(fb), dim3(256), 0, s, reinterpret_cast<uint4*>(acc), n16);
    const float4* g4 = reinterpret_cast<const float4*>(grad_out);
    es.mark(s);
    if (a.n_tiles > 0) {
        if (saved)
            hipLaunchKernelGGL(k_bwd_bound, dim3(a.n_tiles), dim3(kThreads), 0, s, a, g4, state, part);
        else
            hipLaunchKernelGGL((k_bwd_pass1<DT, ANISO>), dim3(a.n_tiles), dim3(kThreads), 0, s, a, g4, state, part);
    }
    es.mark(s);
    hipLaunchKernelGGL(k_bwd_scale, dim3(1), dim3(kThreads), 0, s, part, (int)P.n_blocks, ctl);
    // coarse levels accumulate per workgroup in LDS first: side <= 8, or for
    // anisotropic pyramids the levels 1.. with side <= 4 of all six directions
    // (stored together at the end of the pyramid)
    int ls = L.levels;
    for (int l = ANISO ? 1 : 0; l < L.levels; ++l)
        if ((L.n >> l) <= (ANISO ? VCT_ANISO_SMALL_SIDE : 8)) {
            ls = l;
            break;
        }
    const uint32_t small_off = (uint32_t)(ls < L.levels ? L.doff[0][ls] : L.total_texels);
    const int small_n = (int)(L.total_texels - small_off);
    if (small_n > (ANISO ? kSmallMaxAniso : kSmallMax)) return hipErrorInvalidValue;
    es.mark(s);
    if (a.n_tiles > 0) {
        hipLaunchKernelGGL((k_bwd_pass2<DT, ANISO>), dim3(a.n_tiles), dim3(kThreads), 0, s, a, g4, state, ctl, acc,
                           small_off, small_n);
    }
    if constexpr (ANISO) {
        AnisoAdj m{};
        m.n = L.n;
        m.levels = L.levels;
        for (int l = 0; l < L.levels; ++l) {
            m.nb[l] = L.nb[l];
            for (int d = 0; d < 6; ++d) m.doff[d][l] = (uint32_t)L.doff[d][l];
        }
        es.mark(s);
        for (int c = L.levels - 1; c >= 0; --c) {
            m.level = c;
            const uint32_t threads = (uint32_t)L.nb[c] * L.nb[c] * L.nb[c] * 64u;
            hipLaunchKernelGGL(k_aniso_adjoint<DT>, dim3((threads + 255u) / 256u), dim3(256), 0, s, m,
                               reinterpret_cast<long long*>(acc), a.pyr, ctl, reinterpret_cast<float4*>(grad_base));
        }
        es.mark(s);
        return hipGetLastError();
    }
    AdjArgs m{};
    m.n = L.n;
    m.levels = L.levels;
    for (int l = 0; l < L.levels; ++l) {
        m.nb[l] = L.nb[l];
        m.off[l] = (uint32_t)L.off[l];
    }
    const uint32_t nbh = (uint32_t)((L.n + 1) / 2 + 3) / 4;
    const uint32_t total = nbh * nbh * nbh * 128u;   // threads: two per block of 2x2x2 base texels, brick order
    int blocks = (int)((total + 255) / 256);
    if (blocks > 65536) blocks = 65536;
    es.mark(s);
    hipLaunchKernelGGL(k_mip_adjoint, dim3(blocks), dim3(256), 0, s, m, reinterpret_cast<const long long*>(acc), ctl,
                       reinterpret_cast<float4*>(grad_base));
    es.mark(s);
    return hipGetLastError();
}

int64_t align256(int64_t v) { return (v + 255) & ~int64_t(255); }

}  // namespace

BackwardPlan vct_plan_backward(const PyrLayout& L, const TraceArgs& a) {
    BackwardPlan P{};
    int64_t npix = (int64_t)a.b * a.h * a.w;
    int nslots = a.n_diffuse + 2;
    P.n_lanes = npix * nslots;
    P.n_blocks = a.n_tiles;
    int64_t off = 0;
    P.acc_off = off;
    P.acc_bytes = align256(L.total_texels * 32);
    off += P.acc_bytes;
    P.part_off = off;
    P.part_bytes = align256(P.n_blocks * 4 + 4);
    off += P.part_bytes;
    P.ctl_off = off;
    P.ctl_bytes = 256;
    off += P.ctl_bytes;
    P.state_off = off;            // last, so that the saved-state variant needs only state_off bytes
    P.state_bytes = vct_lane_state_bytes(P.n_lanes);
    off += P.state_bytes;
    P.bytes = off;
    return P;
}

// hi and lo (32 bytes) and the bound coefficients (8 bytes) of every lane
int64_t vct_lane_state_bytes(int64_t n_lanes) { return align256(n_lanes * 40); }

hipError_t vct_launch_backward(const PyrLayout& L, const TraceArgs& a, const BackwardPlan& P, const float* grad_out,
                               float* grad_base, void* ws, const void* saved, hipStream_t s, EventSink& es) {
    return vct_dispatch_dt(L.dtype, a.wide != 0, [&](auto dt) {
        constexpr int DT = decltype(dt)::value;
        return a.aniso ? run_backward<DT, true>(L, a, P, grad_out, grad_base, ws, saved, s, es)
                       : run_backward<DT, false>(L, a, P, grad_out, grad_base, ws, saved, s, es);
    });
}

hipError_t vct_launch_trace_save(const TraceArgs& a, int dtype, float* out, void* state, hipStream_t s,
                                 EventSink& es) {
    if (a.n_tiles > 0) {
        es.mark(s);
        float4* o = reinterpret_cast<float4*>(out);
        LaneState* st = reinterpret_cast<LaneState*>(state);
        (void)vct_dispatch_dt(dtype, a.wide != 0, [&](auto dt) {   // (launch errors: hipGetLastError below)
            constexpr int DT = decltype(dt)::value;
            if (a.aniso)
                hipLaunchKernelGGL((k_trace_save<DT, true>), dim3(a.n_tiles), dim3(kThreads), 0, s, a, o, st);
            else
                hipLaunchKernelGGL((k_trace_save<DT, false>), dim3(a.n_tiles), dim3(kThreads), 0, s, a, o, st);
            return hipSuccess;
        });
    }
    es.mark(s);
    return hipGetLastError();
}
