/*
 * vct.h - C ABI of the voxel-cone-tracing hot path for AMD Instinct MI355X (gfx950).
 *
 * The library computes the data-parallel core of voxel cone tracing as defined in
 * arXiv 2104.00618 ("Real-Time Global Illumination Using OpenGL And Voxel Cone
 * Tracing"): a mip pyramid of a premultiplied RGBA voxel grid, and for every
 * G-buffer pixel u diffuse cones, one specular cone and one occlusion cone that
 * march through that pyramid, sampling quadrilinearly and compositing front to
 * back; plus the adjoint of the march with respect to the base grid.
 *
 * Conventions shared by every entry point
 *   - Data pointers are DEVICE pointers unless marked "host".  Struct pointers
 *     (vct_grid, vct_gbuffer, vct_cone_params) point to host memory and are read
 *     during the call only.
 *   - Work is enqueued on `stream` (a hipStream_t; 0 = the null stream) and runs
 *     asynchronously; the call returns before it completes.  The library never
 *     synchronises the device or the stream.
 *   - The caller owns every buffer.  The library allocates no memory that the
 *     caller can see and keeps no pointer after a call returns.
 *   - Every entry point returns VCT_OK (0) or a negative error code.  All
 *     arguments are validated before anything is enqueued, so a call that fails
 *     validation has no side effects.  vct_last_error() then gives a
 *     "function: message" string (thread-local, valid until the next call on
 *     that thread).  No C++ exception or abort crosses this interface.
 *   - Grids are cubes of N^3 texels, N = 2^k with 1 <= N <= 1024, covering the
 *     world-space cube [origin, origin + extent]^3.  Texel (i, j, k) of level l
 *     has its centre at origin + (i + 1/2, j + 1/2, k + 1/2) * extent / N_l with
 *     N_l = N >> l.  Logical grid buffers are contiguous float32
 *     [z][y][x][4] (x fastest) holding premultiplied (r*a, g*a, b*a, a).
 *   - Non-finite grid, G-buffer or gradient VALUES are not checked (that would
 *     need a device synchronisation); they propagate into the results, and every
 *     march stays bounded in time regardless.
 */
#ifndef VCT_H
#define VCT_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define VCT_OK 0
#define VCT_EINVAL (-1)        /* a shape, size or parameter is out of range, or a pointer is null */
#define VCT_EWORKSPACE (-2)    /* a caller buffer is smaller than the size query requires */
#define VCT_EDEVICE (-3)       /* the HIP runtime refused a launch; the message carries its error */
#define VCT_EUNSUPPORTED (-4)  /* valid request that the library does not implement (kept for ABI
                                  stability; no entry point returns it at present) */

#define VCT_MAX_DIFFUSE 16
#define VCT_MAX_N 1024
#define VCT_MAX_STEPS (1 << 20) /* bound on max_dist / (step_factor * voxel size) */
#define VCT_MAX_LIGHTS 8

/* Storage type of the mip pyramid.  Sampling, compositing and gradients are
 * always float32; reduced-precision pyramids are rounded to nearest even. */
typedef enum { VCT_F32 = 0, VCT_F16 = 1, VCT_BF16 = 2 } vct_dtype;

/* The voxel grid and its pyramid (the thesis's VoxelMap 3D texture and its
 * mipmaps; Section 4.3.3 "Mipmaps", Section 5.4.4 "Additional components"). */
typedef struct {
    int32_t n;         /* base resolution N = 2^k, 1..1024 */
    int32_t levels;    /* pyramid levels L, 1 <= L <= log2(N) + 1 (level l has N >> l texels a side) */
    int32_t dtype;     /* vct_dtype of the pyramid storage */
    float origin[3];   /* world position of the grid's minimum corner */
    float extent;      /* side length of the grid cube, world units, finite and > 0 */
    int32_t anisotropic; /* 0: one pyramid of 2x2x2 means; 1: six directional pyramids sharing level 0
                            (see vct_build_mips); every entry point accepts both */
} vct_grid;

/* Deferred-shading G-buffer: one cone origin per pixel (Section 5.1.3 adopts
 * deferred shading; the cone-trace fragment inputs are position, normal,
 * material and camera, Section 5.4.4 "Cone Tracing"). */
typedef struct {
    int32_t b, h, w;          /* views, rows, columns; any may be 0 (nothing to do) */
    const float* pos_rough;   /* device [b][h][w][4] = (x, y, z, roughness) in world units */
    const float* normal;      /* device [b][h][w][4] = (nx, ny, nz, valid); valid == 0 marks background */
    const float* cam_pos;     /* device [b][3] camera position of each view */
} vct_gbuffer;

/* Cone set and march parameters.  The thesis groups an initial offset t0, an
 * aperture and a step factor per cone class (Section 5.4.4 "Additional
 * components") and traces u diffuse cones, a specular cone in the reflection
 * direction and an occlusion cone toward the light (Section 4.2). */
typedef struct {
    int32_t n_diffuse;                           /* u, 0..16 */
    float diffuse_dir[VCT_MAX_DIFFUSE][3];       /* tangent-frame axes (x = tangent, y = bitangent, z = normal) */
    float diffuse_weight[VCT_MAX_DIFFUSE];       /* weight of each diffuse cone in the D output */
    float diffuse_aperture;                      /* radians, finite, >= 0 */
    int32_t enable_spec;                         /* nonzero: trace the specular cone */
    int32_t enable_occ;                          /* nonzero: trace the occlusion cone */
    float spec_aperture_scale;                   /* specular aperture = roughness * scale (radians), >= 0 */
    float occ_aperture;                          /* radians, finite, >= 0 */
    float light_pos[3];                          /* point light, world units */
    float step_factor;                           /* beta > 0: t += beta * d */
    float t0;                                    /* initial offset along the axis, >= 0 */
    float normal_offset;                         /* cone origin = x + n * normal_offset * voxel size */
    float max_dist;                              /* > 0: samples only at t <= max_dist */
    float alpha_thresh;                          /* > 0: samples only while accumulated alpha < alpha_thresh */
} vct_cone_params;

/* Lights, specular colour and cone-variant flags of the final shading pass
 * (Section 5.4.4, "Cone Tracing": the modified occlusion, specular and
 * diffuse cones of the implementation and the shading equation that combines
 * them with a Lambert + Phong direct term per light). */
typedef struct {
    int32_t n_lights;                            /* 0..8; each light gets an occlusion cone */
    float light_pos[VCT_MAX_LIGHTS][3];          /* point lights, world units */
    float light_diffuse[VCT_MAX_LIGHTS][3];      /* i_d per light (rgb) */
    float light_specular[VCT_MAX_LIGHTS][3];     /* i_s per light (rgb) */
    float specular_color[3];                     /* c_s of the Phong term (rgb) */
    int32_t diffuse_first_hit;                   /* nonzero: a diffuse cone stops at the first sample with
                                                    alpha > first_hit_alpha and returns its colour */
    float first_hit_alpha;                       /* in [0, 1); 0.01 in the thesis */
    int32_t occlusion_falloff;                   /* nonzero: each occlusion sample's alpha is scaled by
                                                    smoothstep(0, max_dist, sqrt(t) * shadow_strength) */
    float shadow_strength;                       /* >= 0 */
    int32_t specular_brdf;                       /* nonzero: the specular cone is weighted per light by
                                                    (1 - max(0, gamma - grace * shininess) / pi)^falloff,
                                                    gamma the angle between its axis and the light;
                                                    zero: added once with weight 1 */
    float grace_per_shininess;                   /* >= 0; 0.008 pi in the thesis */
    float shininess_falloff;                     /* exponent q >= 0 */
} vct_shade_params;

/* Lights and material strengths of voxelization with direct-light injection
 * (Section 4.4 "Voxelization Process", 3D texture storage: the Phong model of
 * Section 3.2 without its glossy term, with distance attenuation). */
typedef struct {
    int32_t n_lights;                            /* 0..8 */
    float light_pos[VCT_MAX_LIGHTS][3];          /* world units */
    float light_color[VCT_MAX_LIGHTS][3];        /* rgb, finite */
    float attenuation[VCT_MAX_LIGHTS][3];        /* (constant, linear, quadratic), >= 0, not all 0 */
    float ambient;                               /* ambient strength, >= 0 */
    float diffuse;                               /* diffuse strength, >= 0 */
} vct_voxelize_params;

/* Bytes of the opaque pyramid buffer for `grid` (host only, enqueues nothing).
 * Layout (informative): each level stored as 4^3-texel bricks in the storage
 * type, levels concatenated at 256-byte alignment, followed by a small float32
 * staging area used while the pyramid is built. */
int vct_pyramid_bytes(const vct_grid* grid, size_t* bytes);

/* Build the mip pyramid: level 0 = `base`, level l+1 = mean of the 2x2x2
 * children of level l (sum in float32 as ((c0+c1)+(c2+c3))+((c4+c5)+(c6+c7)),
 * times 1/8), every level computed from float32 parents and then rounded once
 * to the storage type.  Texture filtering, Section 4.3.3; mipmaps generated
 * after voxelization, Sections 4.5 and 5.4.4.
 *   base          device float32 [N][N][N][4], premultiplied RGBA, read only
 *   pyramid       device buffer of at least vct_pyramid_bytes(grid) bytes, overwritten
 *   pyramid_bytes its size (VCT_EWORKSPACE if too small) */
int vct_build_mips(const vct_grid* grid, const float* base, void* pyramid, size_t pyramid_bytes,
                   hipStream_t stream);
/* Anisotropic pyramids (grid->anisotropic = 1; the mipmaps built with
 * anisotropic filtering of Section 5.1.3, "Villegas"): six pyramids, one per
 * direction +x, -x, +y, -y, +z, -z, sharing level 0 = base.  A texel of level
 * l + 1 in direction d composites its two children along the axis of d front
 * to back as seen by a ray travelling along d (c = c_f + (1 - a_f) c_b on all
 * four premultiplied channels; "+x" puts the smaller-x child in front) and
 * averages the four pairs ((p0 + p1) + (p2 + p3)) / 4 in float32.  Level 1 is
 * computed from the float32 base; level l + 1 >= 2 from the stored level l (so
 * for float16 / bfloat16 storage it is rounded once per level).  A cone with
 * unit axis w samples sum_a w_a^2 * (quadrilinear sample of the pyramid of
 * direction sign(w_a) along axis a); at level 0 all six coincide.  Storage:
 * level 0 plus six copies of levels 1..L-1 (about 1.86x the base for full
 * pyramids, vct_pyramid_bytes). */

/* Copy level `level` of a built pyramid out as logical float32
 * [N_l][N_l][N_l][4] (test and inspection hook; the thesis's
 * VoxelMap::retrieveData, Section 5.4.4). */
int vct_unpack_level(const vct_grid* grid, const void* pyramid, int32_t level, float* out,
                     hipStream_t stream);
/* Same for one direction of an anisotropic pyramid: direction 0..5 = +x, -x,
 * +y, -y, +z, -z (level 0 is the same for all six).  For an isotropic grid
 * direction must be 0 and this equals vct_unpack_level. */
int vct_unpack_level_dir(const vct_grid* grid, const void* pyramid, int32_t level, int32_t direction,
                         float* out, hipStream_t stream);

/* Forward cone trace (Section 4.3.2 cone-trace function; sampler of Section
 * 4.5; cone set of Sections 4.2 and 5.4.4).  For every pixel with valid != 0:
 *   o = x + normalize(n) * normal_offset * voxel;  frame t = normalize(a x n),
 *   b = n x t with a = (1,0,0) if |n_y| > 0.9 else (0,1,0);
 *   diffuse q: axis normalize(t*d.x + b*d.y + n*d.z), aperture diffuse_aperture;
 *   specular:  axis reflect(normalize(x - cam), n), aperture roughness * scale;
 *   occlusion: axis toward light_pos, t_max = min(max_dist, |light - o|).
 * Each cone: t = t0, C = 0, A = 0; while t <= t_max and A < alpha_thresh:
 *   d = max(2 t tan(aperture / 2), voxel); lod = clamp(log2(d / voxel), 0, L - 1);
 *   s = quadrilinear sample at o + t * axis (clamp-to-edge);
 *   C += (1 - A) s.rgb; A += (1 - A) s.a; t += step_factor * d.
 *   out        device float32 [b][h][w][8], overwritten:
 *              (sum_q w_q C_q, sum_q w_q A_q, C_spec, A_occ); background pixels and
 *              disabled cones give 0.  May be null when b*h*w == 0. */
int vct_trace(const vct_grid* grid, const void* pyramid, const vct_gbuffer* gbuf,
              const vct_cone_params* params, float* out, hipStream_t stream);

/* Same march as vct_trace, but instead of radiance it writes the total number
 * of cone samples taken over all pixels and cones to *count (device uint64,
 * overwritten).  Used to state throughput in samples per second. */
int vct_count_samples(const vct_grid* grid, const void* pyramid, const vct_gbuffer* gbuf,
                      const vct_cone_params* params, unsigned long long* count, hipStream_t stream);

/* The same count split by the levels a sample reads (Section 4.3.3: linear
 * blend of the two levels around the LOD): counts[0] = all cone samples,
 * counts[1] = those whose LOD is fractional, so that they read two levels
 * (the others read one).  counts: device uint64 [2], overwritten.  Used to
 * state the arithmetic a march performs.  Errors: those of vct_count_samples. */
int vct_count_sample_levels(const vct_grid* grid, const void* pyramid, const vct_gbuffer* gbuf,
                            const vct_cone_params* params, unsigned long long* counts, hipStream_t stream);

/* Device workspace bytes needed by vct_trace_backward for these shapes (host only). */
int vct_backward_workspace_bytes(const vct_grid* grid, const vct_gbuffer* gbuf,
                                 const vct_cone_params* params, size_t* bytes);

/* Adjoint of vct_build_mips followed by vct_trace with respect to `base`,
 * holding the number of samples of every cone fixed.  Per cone, with
 * T_k = 1 - A_k: dL/dc_k = T_k dL/dC and
 * dL/da_k = -T_k (dL/dC . (C_K - C_{k+1}) - dL/dA T_K) / T_{k+1}
 * (dL/da_{K-1} = T_{K-1} dL/dA), transmittance recomputed by re-marching, never
 * stored; each sample's gradient is spread over its 16 taps with the tap
 * weights and reduced deterministically (64-bit fixed point, exact integer
 * sums: bitwise identical results on every run); then carried through the mip
 * reduction (each child receives 1/8 of its parent's gradient).  For float16 or
 * bfloat16 pyramids the sampled values are the stored ones and the rounding is
 * treated as the identity.  Anisotropic pyramids: a sample above level 0 sends
 * its gradient to the three directions it read, weighted by w_a^2, and each
 * direction's level gradients reach the level below through the transpose of
 * the linearised front-to-back composite of the two children (front child
 * (G - e_alpha (G . b)) / 4, back child (1 - f.alpha) G / 4, with f, b the
 * stored texels), computed in float32 from the top level down with one writer
 * per texel, so the result is still the same on every run.
 *   grad_out   device float32 [b][h][w][8] = dL/d(out of vct_trace)
 *   grad_base  device float32 [N][N][N][4], overwritten (not accumulated)
 *   workspace  device buffer of at least vct_backward_workspace_bytes bytes */
int vct_trace_backward(const vct_grid* grid, const void* pyramid, const vct_gbuffer* gbuf,
                       const vct_cone_params* params, const float* grad_out, float* grad_base,
                       void* workspace, size_t workspace_bytes, hipStream_t stream);

/* Training path: a forward that also keeps every cone's end state so that the
 * backward need not re-march once more to recover it.
 *
 * vct_lane_state_bytes: bytes of the lane-state buffer for these shapes (host
 * only); (b*h*w) * (n_diffuse + 2) states of 40 bytes, rounded up to 256.
 *
 * vct_trace_save: the forward of vct_trace (same cones, same sample counts),
 * with the colour accumulated as a double-float, so that `out` agrees with
 * vct_trace to float32 rounding rather than bit for bit; it also writes the
 * lane states (C_K, A_K, K and the two coefficients of the bound that sets
 * the fixed-point scale of the adjoint) to `lane_state` (device, opaque,
 * overwritten).  Per-sample
 * transmittance is not stored; the backward still recomputes it.
 *
 * vct_trace_backward_saved: vct_trace_backward given those lane states (same
 * grid, pyramid, G-buffer and parameters as the vct_trace_save call).  Its
 * result is bitwise equal to vct_trace_backward's.  The workspace needs
 * vct_backward_workspace_bytes - vct_lane_state_bytes bytes. */
int vct_lane_state_bytes(const vct_gbuffer* gbuf, const vct_cone_params* params, size_t* bytes);
int vct_trace_save(const vct_grid* grid, const void* pyramid, const vct_gbuffer* gbuf,
                   const vct_cone_params* params, float* out, void* lane_state, size_t lane_state_bytes,
                   hipStream_t stream);
int vct_trace_backward_saved(const vct_grid* grid, const void* pyramid, const vct_gbuffer* gbuf,
                             const vct_cone_params* params, const void* lane_state, size_t lane_state_bytes,
                             const float* grad_out, float* grad_base, void* workspace, size_t workspace_bytes,
                             hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops and harnesses that forbid hipMalloc): the same
 * backward as vct_trace_backward_saved, bitwise the same result, with no
 * workspace argument.  Its accumulator, bound partials and control word live
 * in a device array of VCT_NOALLOC_SCRATCH_BYTES inside the library, one per
 * GPU (each GPU the library runs on holds it until the process ends); the
 * call allocates nothing and clears what it uses with kernels.
 *   - Shapes whose workspace (vct_backward_workspace_bytes minus
 *     vct_lane_state_bytes) exceeds VCT_NOALLOC_SCRATCH_BYTES are rejected with
 *     VCT_EWORKSPACE before anything is enqueued (128 MiB covers a 128^3
 *     grid, isotropic or anisotropic, with any G-buffer up to 2 million
 *     16x16 tiles).
 *   - Every call on a GPU shares that GPU's array: calls that overlap on one
 *     GPU (on different streams, or from several threads) race and corrupt
 *     each other's result; serialise them.
 *   - `stream` must belong to the current device (else VCT_EINVAL); the first
 *     call on a device looks up the array's address there (VCT_EDEVICE if the
 *     runtime refuses). */
#define VCT_NOALLOC_SCRATCH_BYTES (128ull << 20)
int vct_trace_backward_saved_noalloc(const vct_grid* grid, const void* pyramid, const vct_gbuffer* gbuf,
                                     const vct_cone_params* params, const void* lane_state, size_t lane_state_bytes,
                                     const float* grad_out, float* grad_base, hipStream_t stream);

/* Shaded radiance with the thesis's cone variants (Section 5.4.4, "Cone
 * Tracing", the implemented shading equation):
 *   L = o_min * sum_q w_q C_diff,q + sum_s f_spec,s C_spec
 *       + sum_s V_s (c_d i_d,s max(0, L_s . N) + c_s i_s,s max(0, R_s . w)^shininess)
 * with the u diffuse cones of `params` (first-hit or accumulated), one specular
 * cone along the reflection axis (aperture roughness * spec_aperture_scale),
 * one occlusion cone per light (aperture occ_aperture, t_max = min(max_dist,
 * distance), with or without falloff), V_s = 1 - its alpha, o_min = min_s V_s
 * (1 with no light), L_s the unit direction to light s, R_s = reflect(-L_s, N)
 * and w the unit direction to the camera.  `params`'s light_pos and enable
 * flags are not used here; its march parameters are.
 *   material  device [b][h][w][4] = (c_d.r, c_d.g, c_d.b, shininess)
 *   out       device [b][h][w][4] = (L.r, L.g, L.b, o_min), overwritten; 0 for background pixels
 * Errors: VCT_EINVAL for a null pointer with pixels present, n_lights outside
 * 0..8, a non-finite light or flag parameter, first_hit_alpha outside [0, 1)
 * or a negative strength, grace or falloff. */
int vct_shade(const vct_grid* grid, const void* pyramid, const vct_gbuffer* gbuf, const float* material,
              const vct_cone_params* params, const vct_shade_params* shade, float* out, hipStream_t stream);

/* Same marches as vct_shade (diffuse cones first-hit or accumulated, the
 * specular cone, one occlusion cone per light with or without falloff), but
 * instead of radiance it writes the total number of cone samples they take
 * over all pixels to *count (device uint64, overwritten; 0 with no pixels).
 * Used to state the shading pass's throughput in samples per second.
 * Errors: those of vct_shade, with `count` in place of `out`. */
int vct_count_shade_samples(const vct_grid* grid, const void* pyramid, const vct_gbuffer* gbuf,
                            const float* material, const vct_cone_params* params, const vct_shade_params* shade,
                            unsigned long long* count, hipStream_t stream);

/* Voxelize a triangle mesh with direct-light injection into a base grid
 * (Section 4.4 "Voxelization Process": rasterization onto an N x N viewport,
 * dominant axis selection, 3D texture storage; Section 5.4.4 "Voxelization").
 * Every triangle is rasterized once along the largest component of its normal
 * (ties to x, then y, then z; frames x: (z, y | x), y: (x, z | y), z: (x, y | z));
 * a pixel centre inside the projected triangle is a fragment in the voxel
 * (pixel, floor(depth)), with colour
 *   c_tri * sum_l (ambient + diffuse max(0, N . L_l)) light_color_l / (c_l + l_l d_l + q_l d_l^2)
 * (N the unit normal of the triangle as wound, L_l and d_l direction and
 * distance to light l) and alpha 1.  Coverage and depth are exact: vertices
 * snapped to 1/256 voxel (round((p - origin) * 256 N / extent) in float32),
 * integer edge functions with the top-left rule (a centre on an edge belongs to
 * the triangle when the counter-clockwise edge runs upward, or horizontally
 * leftward), exact floor of the plane depth.  Fragments in one voxel are
 * averaged (deterministic fixed-point sums and a count); other voxels are 0.
 * Triangles with a non-finite vertex or a snapped coordinate beyond 2^19 are
 * skipped; per-fragment colours are clamped to +-2^28.
 * Optional surface attributes (the further 3D texture of surface normals that
 * more light bounces need, Section 6.2.2; albedo and normal textures of
 * deferred voxel cone tracing, Section 5.1.3): per voxel the average of its
 * fragments' unit triangle normals (not renormalised: opposite faces in one
 * voxel cancel) and of their triangle colours, w = 1 where a fragment landed,
 * else all 0; same fixed-point averaging.
 *   tris       device float32 [n_tris][3][3] vertex positions, world units
 *   colors     device float32 [n_tris][3] triangle colours
 *   base       device float32 [N][N][N][4] premultiplied RGBA, overwritten (a vct_build_mips input);
 *              while the call runs it also holds the accumulator index of each reached voxel, so it
 *              must not overlap tris, colors, normal, albedo or the workspace
 *   normal     device float32 [N][N][N][4] average normal, overwritten; or null (no surface attributes)
 *   albedo     device float32 [N][N][N][4] average colour, overwritten; null exactly when normal is
 *   workspace  device, vct_voxelize_workspace_bytes(grid, n_tris, surface) bytes (room for an accumulator
 *              of 32 bytes per voxel, 48 more with surface attributes, about 160 per triangle; only the
 *              accumulators of voxels the mesh reaches are cleared and used); surface != 0 sizes it for
 *              normal/albedo output
 * Errors: VCT_EINVAL for a bad grid, n_tris outside [0, 2^31), null buffers,
 * only one of normal / albedo given, n_lights outside 0..8, non-finite or
 * negative light parameters or attenuation all 0, or two of base, normal,
 * albedo and the workspace's first vct_voxelize_workspace_bytes bytes
 * overlapping each other or tris / colors; VCT_EWORKSPACE if the workspace is
 * too small. */
int vct_voxelize_workspace_bytes(const vct_grid* grid, int64_t n_tris, int32_t surface, size_t* bytes);
int vct_voxelize(const vct_grid* grid, const float* tris, const float* colors, int64_t n_tris,
                 const vct_voxelize_params* params, float* base, float* normal, float* albedo, void* workspace,
                 size_t workspace_bytes, hipStream_t stream);

/* One further light bounce inside the voxel grid (Section 6.2.2 "Algorithm
 * Limitations": more bounces need a texture of average surface normals, with
 * cones traced again from the voxels hit about that normal; Sections 6.2.4
 * and 5.1.3: indirect light inserted into a further 3D texture).  Every
 * surface voxel -- base alpha > 0 and |normal.xyz| >= 1/100 -- traces the
 * diffuse cones of `params` (frame, apertures, t0, step factor, max_dist,
 * alpha_thresh and normal_offset as in vct_trace; specular and occlusion cones
 * are not traced) from its centre about normalize(normal.xyz), through
 * `pyramid`, and
 *   out.rgb = base.rgb + base.a * albedo.rgb * sum_q w_q C_q,   out.a = base.a;
 * every other voxel gets its base value.  For k bounces call it k times with
 * the same base (the direct light) and the pyramid of the previous result.
 *   pyramid    built by vct_build_mips for `grid` (e.g. from base, or from the previous bounce)
 *   base       device float32 [N][N][N][4] premultiplied direct light, read only
 *   normal     device float32 [N][N][N][4] average surface normal (xyz; w unused), read only
 *   albedo     device float32 [N][N][N][4] surface colour (rgb; w unused), read only
 *   out        device float32 [N][N][N][4], overwritten; may be base itself (in place), must not
 *              overlap normal, albedo, pyramid or workspace otherwise
 *   workspace  device, vct_bounce_workspace_bytes(grid) bytes (about 4.1 per voxel: a list entry for
 *              every voxel that could be a surface voxel, and a flag bit)
 * The cones' terms are summed in cone order, as in vct_trace's D, so the result
 * is the same on every run.
 * Errors: VCT_EINVAL for a bad grid or cone parameters, a null pointer, the
 * workspace's first vct_bounce_workspace_bytes bytes overlapping any buffer,
 * or out overlapping pyramid, normal, albedo or (other than exactly) base;
 * VCT_EWORKSPACE if the workspace is too small. */
int vct_bounce_workspace_bytes(const vct_grid* grid, size_t* bytes);
int vct_bounce(const vct_grid* grid, const void* pyramid, const float* base, const float* normal,
               const float* albedo, const vct_cone_params* params, float* out, void* workspace,
               size_t workspace_bytes, hipStream_t stream);

/* Diagnostics: per-kernel timing.  Registers `count` events (a host array of
 * hipEvent_t created by the caller) for the NEXT enqueuing call on this thread
 * (any entry point that enqueues kernels).  That call records events[i] on its
 * stream just before its i-th kernel and, after its last kernel, records the
 * next unused event; events beyond its kernel count are left untouched.
 * Kernel order of vct_trace_backward: clear accumulator, pass 1 (recompute),
 * scale, pass 2 (re-march and scatter), mip adjoint; of vct_bounce: flag,
 * scan, list, gather.  The registration is consumed by that call (also if it fails).
 * count = 0 clears it.  Recording costs one hipEventRecord per kernel. */
int vct_record_kernel_events(hipEvent_t* events, int32_t count);

/* Message of the last failed call on this thread ("" if none). */
const char* vct_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* VCT_H */
