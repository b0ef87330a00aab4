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
//   k_mip_adjoint per base texel: gather over levels, convert to float32
#include "bwd_pixel.h"

namespace {

using namespace vct;

constexpr int kThreads = 256;

template <int DT>
__global__ __launch_bounds__(kThreads) void k_bwd_pass1(TraceArgs a, const float4* __restrict__ gout,
                                                        LaneState* __restrict__ state, float* __restrict__ part) {
    __shared__ LevelTable T;
    __shared__ float s_part[kThreads / 64];
    load_level_table(a, &T);
    __syncthreads();
    const int tile = xcd_tile(blockIdx.x, a.n_tiles);
    int view, y, x;
    tile_pixel(a, tile, threadIdx.x, view, y, x);
    float bound = 0.f;
    if (x < a.w && y < a.h) bound = pass1_pixel<DT>(a, T, gout, state, view, ((size_t)view * a.h + y) * a.w + x);
    // fixed-order workgroup sum
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int o = 32; o > 0; o >>= 1) bound += __shfl_xor(bound, o, 64);
    if (lane == 0) s_part[wv] = bound;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = (s_part[0] + s_part[1]) + (s_part[2] + s_part[3]);
}

// Forward that also saves every cone's end state (training path: the
// backward then skips pass 1).
template <int DT>
__global__ __launch_bounds__(kThreads) void k_trace_save(TraceArgs a, float4* __restrict__ out,
                                                         LaneState* __restrict__ state) {
    __shared__ LevelTable T;
    load_level_table(a, &T);
    __syncthreads();
    const int tile = xcd_tile(blockIdx.x, a.n_tiles);
    int view, y, x;
    tile_pixel(a, tile, threadIdx.x, view, y, x);
    if (!(x < a.w && y < a.h)) return;
    const size_t pix = ((size_t)view * a.h + y) * a.w + x;
    float4 o0, o1;
    trace_save_pixel<DT>(a, T, view, pix, state, o0, o1);
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
// i ^ mask: row_mirror (^15) and row_half_mirror (^7) and quad permutes (^2,
// ^1) are DPP modifiers of ordinary VALU instructions; ^16 is a ds_swizzle in
// bitmask mode and ^32 a single bpermute.
template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, true));
}
constexpr int kDppXor15 = 0x140;   // row_mirror
constexpr int kDppXor7 = 0x141;    // row_half_mirror
constexpr int kDppXor2 = 0x4E;     // quad_perm [2,3,0,1]
constexpr int kDppXor1 = 0xB1;     // quad_perm [1,0,3,2]
__device__ __forceinline__ float swz_xor16(float v) {
    return __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), 0x401F));
}

// After xpose_sum32, lanes 0..31 hold the sums of value index
// xpose_index(lane) (lanes j and j + 32 hold the same sum).
__device__ __forceinline__ int xpose_index(int lane) {
    return ((lane >> 3) & 1) * 16 + ((lane >> 2) & 1) * 8 + ((lane >> 1) & 1) * 4 + (lane & 1) * 2 +
           ((lane >> 4) & 1);
}

// Butterfly step: pair lanes by `mask`; the lane whose `up` bit is set keeps
// the upper half of its values, its partner the lower half.
template <int N, typename X>
__device__ __forceinline__ void halve(float* r, bool up, X xmove) {
#pragma unroll
    for (int i = 0; i < N / 2; ++i) {
        float keep = up ? r[N / 2 + i] : r[i];
        float send = up ? r[i] : r[N / 2 + i];
        r[i] = keep + xmove(send);
    }
}

// Sum over the lanes with `in` set of the 32 values w[q] * g[ch] (index
// 4q + ch), transposed across the wave: 16 + 8 + 4 + 2 DPP moves, one swizzle
// and one bpermute.  The masks 15, 7, 2, 1, 16, 32 each flip only bits not
// yet used to split the values, so partners always hold the same indices;
// the addition order is fixed, so the sums are reproducible.
__device__ __forceinline__ float xpose_sum32(const float w[8], const float g[4], bool in, int lane) {
    float r[16];
    {
        // First split is on the tap's z bit (value index bit 4): a lane with
        // lane bit 3 set keeps taps 4..7, so it swaps tap q with q + 4 up front
        // instead of selecting among the 32 products.
        const bool up = (lane & 8) != 0;
        float wk[4], ws[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float a = in ? w[q] : 0.f, b = in ? w[q + 4] : 0.f;
            wk[q] = up ? b : a;
            ws[q] = up ? a : b;
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) r[i] = ws[i >> 2] * g[i & 3];
#pragma unroll
        for (int i = 0; i < 16; ++i) r[i] = __builtin_fmaf(wk[i >> 2], g[i & 3], dpp<kDppXor15>(r[i]));
    }
    halve<16>(r, (lane & 4) != 0, [](float v) { return dpp<kDppXor7>(v); });
    halve<8>(r, (lane & 2) != 0, [](float v) { return dpp<kDppXor2>(v); });
    halve<4>(r, (lane & 1) != 0, [](float v) { return dpp<kDppXor1>(v); });
    halve<2>(r, (lane & 16) != 0, [](float v) { return swz_xor16(v); });
    return r[0] + __shfl_xor(r[0], 32);
}

// Alpha-only variant (occlusion cones carry no colour gradient): the sum over
// the lanes with `in` set of w[q] * ga for the 8 taps.  Lanes with bits 0, 4, 5
// clear end with the sum of tap 4 b3 + 2 b2 + b1.
__device__ __forceinline__ float xpose_sum8(const float w[8], float ga, bool in, int lane) {
    float r[4];
    {
        const bool up = (lane & 8) != 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float a = in ? w[q] * ga : 0.f, b = in ? w[q + 4] * ga : 0.f;
            r[q] = (up ? b : a) + dpp<kDppXor15>(up ? a : b);
        }
    }
    halve<4>(r, (lane & 4) != 0, [](float v) { return dpp<kDppXor7>(v); });
    halve<2>(r, (lane & 2) != 0, [](float v) { return dpp<kDppXor2>(v); });
    float x = r[0] + dpp<kDppXor1>(r[0]);
    x += swz_xor16(x);
    return x + __shfl_xor(x, 32);
}

// Emit one level's tap gradients of the wave.  Lanes whose samples share the
// same (level, base texel) have the same 8 taps; each such group is summed
// across the wave (fixed order) and 32 lanes then add its 8 taps x 4 channels
// as fixed-point integers: to the workgroup's LDS table for the coarse levels
// (side <= 8), to the global accumulator otherwise.
template <bool ALPHA_ONLY>
__device__ __forceinline__ void emit_level(bool live, const LevelTable& T, int level, df Ux, df Uy, df Uz, float wl,
                                           const float g[4], int E, unsigned long long* __restrict__ acc,
                                           unsigned long long* small, uint32_t small_off, int lane) {
    Taps tp;
    level_taps(T, level, Ux, Uy, Uz, tp);
    float w[8];
    folded_weights(tp, wl, w);
    // The 8 taps are fixed by the base texel together with which axes clamp
    // (a clamped axis repeats the base texel instead of stepping to i0 + 1).
    const uint32_t key = live ? tp.idx[0] : 0xffffffffu;
    const int kcl = tp.clamp;
    unsigned long long mask = __ballot(live);
    const int j = ALPHA_ONLY ? (((lane >> 3) & 1) * 4 + ((lane >> 2) & 1) * 2 + ((lane >> 1) & 1)) : xpose_index(lane);
    const int tq = ALPHA_ONLY ? j : (j >> 2), ch = ALPHA_ONLY ? 3 : (j & 3);
    const bool emitter = ALPHA_ONLY ? ((lane & 0x31) == 0) : (lane < 32);
    while (mask) {
        const int leader = __builtin_ctzll(mask);
        const uint32_t k = (uint32_t)__builtin_amdgcn_readlane((int)key, leader);
        const int kc = __builtin_amdgcn_readlane(kcl, leader);
        const bool in = live && key == k && kcl == kc;
        const unsigned long long gm = __ballot(in);
        const float sum = ALPHA_ONLY ? xpose_sum8(w, g[3], in, lane) : xpose_sum32(w, g, in, lane);
        const int lev = __builtin_amdgcn_readlane(level, leader);
        uint32_t idx = 0;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            uint32_t iq = (uint32_t)__builtin_amdgcn_readlane((int)tp.idx[q], leader);
            idx = tq == q ? iq : idx;
        }
        const long long qv = emitter ? fixed_point(sum, E - 3 * lev) : 0;
        VCT_CHECK_ACC(idx);
        if (qv != 0 && idx >= small_off) atomicAdd(&small[(idx - small_off) * 4 + ch], (unsigned long long)qv);
        if (qv != 0 && idx < small_off) atomicAdd(&acc[(size_t)idx * 4 + ch], (unsigned long long)qv);
        mask &= ~gm;
    }
}

constexpr int kSmallMax = 704;   // texels of all levels with side <= 8 (8^3 + 3 bricks of 64)

template <int DT>
__global__ __launch_bounds__(kThreads, 4) void k_bwd_pass2(TraceArgs a, const float4* __restrict__ gout,
                                                        const LaneState* __restrict__ state,
                                                        const int* __restrict__ ctl,
                                                        unsigned long long* __restrict__ acc, uint32_t small_off,
                                                        int small_n) {
    __shared__ LevelTable T;
    __shared__ unsigned long long s_small[kSmallMax * 4];
    load_level_table(a, &T);
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
    for (int slot = 0; slot < nslots; ++slot) {
        if (!slot_enabled(a, slot)) continue;
        Pass2Lane L;
        L.K = 0;
        if (valid) {
            // pixel setup and dL/d(out) are reloaded per cone to keep registers free
            const PixelSetup P = pixel_setup(a, a.pos_rough[pix], a.normal[pix]);
            const float3 cam = make_float3(a.cam_pos[3 * view], a.cam_pos[3 * view + 1], a.cam_pos[3 * view + 2]);
            pass2_init(a, P, cam, gout[2 * pix], gout[2 * pix + 1], state[pix * nslots + slot], slot, L);
        }
        int Kw = L.K;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) Kw = max(Kw, __shfl_xor(Kw, o));
        const bool occ = slot == a.n_diffuse + 1;
        for (int k = 0; k < Kw; ++k) {
            const bool live = k < L.K;
            Pass2Step st = {};
            if (live) pass2_step<DT>(a, T, L, k, st);
            if (occ) {
                emit_level<true>(live, T, st.l0, st.Ux, st.Uy, st.Uz, 1.0f - st.f, st.g, E, acc, s_small, small_off, lane);
                emit_level<true>(live && st.f > 0.0f, T, st.l1, st.Ux, st.Uy, st.Uz, st.f, st.g, E, acc, s_small,
                                 small_off, lane);
            } else {
                emit_level<false>(live, T, st.l0, st.Ux, st.Uy, st.Uz, 1.0f - st.f, st.g, E, acc, s_small, small_off,
                                  lane);
                emit_level<false>(live && st.f > 0.0f, T, st.l1, st.Ux, st.Uy, st.Uz, st.f, st.g, E, acc, s_small,
                                  small_off, lane);
            }
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

__global__ __launch_bounds__(256) void k_mip_adjoint(AdjArgs m, const long long* __restrict__ acc,
                                                     const int* __restrict__ ctl, float4* __restrict__ grad) {
    const int E = ctl[0];
    const bool bad = ctl[1] != 0;
    const uint32_t n = m.n;
    const uint32_t total = n * n * n;
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < total; t += gridDim.x * blockDim.x) {
        int x = t % n, y = (t / n) % n, z = t / (n * n);
        long long s0 = 0, s1 = 0, s2 = 0, s3 = 0;
#pragma unroll
        for (int l = 0; l < VCT_MAX_LEVELS; ++l) {
            if (l < m.levels) {
                uint32_t idx = m.off[l] + vct_brick_index(x >> l, y >> l, z >> l, m.nb[l]);
                const long long* p = acc + (size_t)idx * 4;
                longlong2 u = reinterpret_cast<const longlong2*>(p)[0];
                longlong2 v = reinterpret_cast<const longlong2*>(p)[1];
                s0 += u.x;
                s1 += u.y;
                s2 += v.x;
                s3 += v.y;
            }
        }
        float4 g;
        if (bad) {
            g = make_float4(__int_as_float(0x7fc00000), __int_as_float(0x7fc00000), __int_as_float(0x7fc00000),
                            __int_as_float(0x7fc00000));
        } else {
            g = make_float4(ldexpf((float)s0, -E), ldexpf((float)s1, -E), ldexpf((float)s2, -E),
                            ldexpf((float)s3, -E));
        }
        grad[t] = g;
    }
}

template <int DT>
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
            hipLaunchKernelGGL(k_bwd_pass1<DT>, dim3(a.n_tiles), dim3(kThreads), 0, s, a, g4, state, part);
    }
    es.mark(s);
    hipLaunchKernelGGL(k_bwd_scale, dim3(1), dim3(kThreads), 0, s, part, (int)P.n_blocks, ctl);
    // coarse levels (side <= 8) accumulate per workgroup in LDS first
    int ls = L.levels;
    for (int l = 0; l < L.levels; ++l)
        if ((L.n >> l) <= 8) {
            ls = l;
            break;
        }
    const uint32_t small_off = (uint32_t)(ls < L.levels ? L.off[ls] : L.total_texels);
    const int small_n = (int)(L.total_texels - small_off);
    if (small_n > kSmallMax) return hipErrorInvalidValue;
    es.mark(s);
    if (a.n_tiles > 0) {
        hipLaunchKernelGGL(k_bwd_pass2<DT>, dim3(a.n_tiles), dim3(kThreads), 0, s, a, g4, state, ctl, acc, small_off,
                           small_n);
    }
    AdjArgs m{};
    m.n = L.n;
    m.levels = L.levels;
    for (int l = 0; l < L.levels; ++l) {
        m.nb[l] = L.nb[l];
        m.off[l] = (uint32_t)L.off[l];
    }
    uint32_t total = (uint32_t)L.n * L.n * L.n;
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

int64_t vct_lane_state_bytes(int64_t n_lanes) { return align256(n_lanes * (int64_t)sizeof(LaneState)); }

hipError_t vct_launch_backward(const PyrLayout& L, const TraceArgs& a, const BackwardPlan& P, const float* grad_out,
                               float* grad_base, void* ws, const void* saved, hipStream_t s, EventSink& es) {
    switch (L.dtype) {
        case VCT_F32: return run_backward<VCT_F32>(L, a, P, grad_out, grad_base, ws, saved, s, es);
        case VCT_F16: return run_backward<VCT_F16>(L, a, P, grad_out, grad_base, ws, saved, s, es);
        default: return run_backward<VCT_BF16>(L, a, P, grad_out, grad_base, ws, saved, s, es);
    }
}

hipError_t vct_launch_trace_save(const TraceArgs& a, int dtype, float* out, void* state, hipStream_t s,
                                 EventSink& es) {
    if (a.n_tiles > 0) {
        es.mark(s);
        float4* o = reinterpret_cast<float4*>(out);
        LaneState* st = reinterpret_cast<LaneState*>(state);
        switch (dtype) {
            case VCT_F32: hipLaunchKernelGGL(k_trace_save<VCT_F32>, dim3(a.n_tiles), dim3(kThreads), 0, s, a, o, st); break;
            case VCT_F16: hipLaunchKernelGGL(k_trace_save<VCT_F16>, dim3(a.n_tiles), dim3(kThreads), 0, s, a, o, st); break;
            default: hipLaunchKernelGGL(k_trace_save<VCT_BF16>, dim3(a.n_tiles), dim3(kThreads), 0, s, a, o, st); break;
        }
    }
    es.mark(s);
    return hipGetLastError();
}
