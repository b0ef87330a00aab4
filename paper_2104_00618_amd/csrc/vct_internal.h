// Internal layout, argument blocks and device helpers of libvct (gfx950).
#pragma once

#include <stdint.h>

#include <type_traits>

#include <hip/hip_runtime.h>

#include "texel.h"
#include "vct.h"

#define VCT_MAX_LEVELS 11   // N <= 1024
#define VCT_BRICK 4          // bricks of 4^3 texels
#define VCT_BRICK_TEXELS 64

// ---------------------------------------------------------------------------
// Pyramid layout.  Level l (N_l = N >> l texels a side) is stored as
// nb_l^3 bricks, nb_l = ceil(N_l / 4), brick (bz, by, bx) at linear index
// (bz * nb_l + by) * nb_l + bx, texels inside a brick at (z&3)*16 + (y&3)*4 + (x&3).
// A 2x2x2 trilinear footprint therefore touches at most 8 bricks and usually
// one, and a brick of float16 texels is 512 contiguous bytes.
// After the last level comes a float32 staging area of two buffers of
// (N/16)^3 texels used by the multi-pass mip build.
// An anisotropic pyramid stores level 0 once, then the levels 1.. with more
// than 4 texels a side of each of the six directions (+x, -x, +y, -y, +z, -z)
// in turn, then the levels with at most 4 of each direction in turn (so the
// adjoint can keep all coarse levels in one LDS table); off[] then describes
// the +x pyramid and doff[d][] every direction (doff[d][0] = 0).
#define VCT_ANISO_SMALL_SIDE 4
// ---------------------------------------------------------------------------
struct PyrLayout {
    int32_t n, levels, dtype, texel_bytes, aniso;
    int32_t nb[VCT_MAX_LEVELS];        // bricks per axis of each level
    int64_t off[VCT_MAX_LEVELS];       // texel offset of each level
    int64_t doff[6][VCT_MAX_LEVELS];   // texel offset of each level of each direction
    int64_t total_texels;              // all levels
    int64_t stage_off_bytes[2];        // byte offsets of the two staging buffers
    int64_t stage_texels;              // capacity of each staging buffer (float4 texels)
    int64_t bytes;                     // whole buffer
};

static inline int vct_log2i(int v) {
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

static inline PyrLayout vct_make_layout(int n, int levels, int dtype, int aniso = 0) {
    PyrLayout p{};
    p.n = n;
    p.levels = levels;
    p.dtype = dtype;
    p.aniso = aniso ? 1 : 0;
    p.texel_bytes = dtype == VCT_F32 ? 16 : 8;
    int64_t off = 0;
    // (every level stays 256-byte aligned: a brick is >= 512 bytes)
    for (int l = 0; l < levels; ++l) {
        int nl = n >> l;
        int nb = (nl + VCT_BRICK - 1) / VCT_BRICK;
        p.nb[l] = nb;
    }
    if (!p.aniso) {
        for (int l = 0; l < levels; ++l) {
            p.doff[0][l] = off;
            off += (int64_t)p.nb[l] * p.nb[l] * p.nb[l] * VCT_BRICK_TEXELS;
        }
    } else {
        off += (int64_t)p.nb[0] * p.nb[0] * p.nb[0] * VCT_BRICK_TEXELS;   // level 0, shared
        for (int pass = 0; pass < 2; ++pass)                              // large levels, then small ones
            for (int d = 0; d < 6; ++d)
                for (int l = 1; l < levels; ++l)
                    if (((n >> l) <= VCT_ANISO_SMALL_SIDE) == (pass == 1)) {
                        p.doff[d][l] = off;
                        off += (int64_t)p.nb[l] * p.nb[l] * p.nb[l] * VCT_BRICK_TEXELS;
                    }
    }
    for (int d = 0; d < 6; ++d)
        for (int l = 0; l < levels; ++l) {
            if (!p.aniso) p.doff[d][l] = p.doff[0][l];
            if (l == 0) p.doff[d][0] = 0;
        }
    for (int l = 0; l < levels; ++l) p.off[l] = p.doff[0][l];
    p.total_texels = off;
    int64_t bytes = off * p.texel_bytes;
    bytes = (bytes + 255) & ~int64_t(255);
    int64_t ns = n / 16 > 0 ? n / 16 : 1;
    p.stage_texels = ns * ns * ns;
    p.stage_off_bytes[0] = bytes;
    bytes += ((p.stage_texels * 16 + 255) & ~int64_t(255));
    p.stage_off_bytes[1] = bytes;
    bytes += ((p.stage_texels * 16 + 255) & ~int64_t(255));
    p.bytes = bytes;
    return p;
}

// Texel index inside a level (brick layout above).
__host__ __device__ static inline uint32_t vct_brick_index(int x, int y, int z, int nb) {
    return (uint32_t)((((z >> 2) * nb + (y >> 2)) * nb + (x >> 2)) << 6) +
           (uint32_t)(((z & 3) << 4) | ((y & 3) << 2) | (x & 3));
}

// ---------------------------------------------------------------------------
// Kernel argument blocks (passed by value).
// ---------------------------------------------------------------------------
struct LevelInfo {
    int32_t n;        // texels a side
    int32_t nb;       // bricks a side
    uint32_t off;     // texel offset of the level in the pyramid (< 2^31 for N <= 1024)
    int32_t pad;
};

struct TraceArgs {
    // grid
    int32_t n, levels;
    float origin[3];
    float scale_hi, scale_lo;      // N / extent as a double-float
    float voxel;                   // extent / N (world size of a base texel)
    LevelInfo lv[VCT_MAX_LEVELS];
    const void* pyr;
    vct_v4i rsrc;                  // structured buffer resource over pyr (one record per texel)
    vct_v4i rraw;                  // raw (byte-offset) resource over pyr (paired float16 / bfloat16 loads)
    uint32_t ddelta[6][VCT_MAX_LEVELS];   // anisotropic: texel offset of direction d's level l minus lv[l].off
    float inv_scale2;              // (extent / N)^2: unit-axis weights w_a^2 = W_a^2 * inv_scale2
    int32_t aniso;                 // six directional pyramids (levels >= 1)
    int32_t wide;                  // pyramid of more than 4 GiB: fetch through 64-bit addresses
    // G-buffer
    int32_t b, h, w;
    int32_t tiles_x, tiles_y, n_tiles;   // 16x16-pixel tiles
    const float4* pos_rough;
    const float4* normal;
    const float* cam_pos;
    // cone set
    int32_t n_diffuse, enable_spec, enable_occ;
    float dir[VCT_MAX_DIFFUSE][3];
    float weight[VCT_MAX_DIFFUSE];
    float diffuse_aperture, spec_aperture_scale, occ_aperture;
    float light_tex[3][2];         // light position in texel units, double-float per axis
    float step_factor, t0, normal_offset, max_dist, alpha_thresh;
    int32_t max_steps;             // hard bound on samples per cone
};

// Calls f(std::integral_constant<int, DT>) with the kernel template argument
// of a pyramid: its storage type, plus VCT_WIDE when it needs 64-bit fetches.
template <typename F>
static inline hipError_t vct_dispatch_dt(int dtype, bool wide, F&& f) {
    using std::integral_constant;
    switch (dtype) {
        case VCT_F32:
            return wide ? f(integral_constant<int, VCT_F32 | VCT_WIDE>{}) : f(integral_constant<int, VCT_F32>{});
        case VCT_F16:
            return wide ? f(integral_constant<int, VCT_F16 | VCT_WIDE>{}) : f(integral_constant<int, VCT_F16>{});
        default:
            return wide ? f(integral_constant<int, VCT_BF16 | VCT_WIDE>{}) : f(integral_constant<int, VCT_BF16>{});
    }
}

// Optional per-kernel event recording (diagnostics): mark() records the next
// registered event on the stream, before each kernel and after the last.
struct EventSink {
    hipEvent_t* ev = nullptr;
    int n = 0, next = 0;
    void mark(hipStream_t s) {
        if (next < n) (void)hipEventRecord(ev[next++], s);
    }
};

// Launch helpers implemented in the .hip files.
hipError_t vct_launch_build_mips(const PyrLayout& L, const float* base, void* pyr, hipStream_t s, EventSink& es);
hipError_t vct_launch_unpack(const PyrLayout& L, const void* pyr, int level, int direction, float* out,
                             hipStream_t s);
// count != nullptr: no output; count[0] = the cone samples taken and, with
// n_counts = 2, count[1] = those that read two levels
hipError_t vct_launch_trace(const TraceArgs& a, int dtype, float* out, unsigned long long* count, int n_counts,
                            hipStream_t s, EventSink& es);
size_t vct_voxelize_acc_bytes(int n, bool surface);
size_t vct_voxelize_workspace_size(int n, long long n_tris, bool surface);
hipError_t vct_launch_voxelize(const vct_grid* g, const float* tris, const float* colors, long long n_tris,
                               const vct_voxelize_params* p, float* base, float* normal, float* albedo, void* ws,
                               hipStream_t s, EventSink& es);
size_t vct_bounce_workspace_size(int n);
hipError_t vct_launch_bounce(const TraceArgs& a, int dtype, const float* base, const float* normal,
                             const float* albedo, float* out, void* ws, hipStream_t s, EventSink& es);
// count != nullptr: no shading; *count = the cone samples all marches take
hipError_t vct_launch_shade(const TraceArgs& a, int dtype, const vct_shade_params* p, const float* material,
                            float* out, unsigned long long* count, hipStream_t s, EventSink& es);

struct BackwardPlan {
    int64_t n_lanes;          // pixels * cones
    int64_t acc_off, acc_bytes;       // int64 x4 accumulator over the pyramid texels
    int64_t state_off, state_bytes;   // per-lane forward state
    int64_t part_off, part_bytes;     // per-block bound partial sums
    int64_t ctl_off, ctl_bytes;       // scale exponent and flags
    int64_t n_blocks;
    int64_t bytes;
};

BackwardPlan vct_plan_backward(const PyrLayout& L, const TraceArgs& a);
int64_t vct_lane_state_bytes(int64_t n_lanes);
// saved == nullptr: recompute the lane states (pass 1); else read them from `saved`
hipError_t vct_launch_backward(const PyrLayout& L, const TraceArgs& a, const BackwardPlan& P,
                               const float* grad_out, float* grad_base, void* ws, const void* saved, hipStream_t s,
                               EventSink& es);
hipError_t vct_launch_trace_save(const TraceArgs& a, int dtype, float* out, void* state, hipStream_t s, EventSink& es);
