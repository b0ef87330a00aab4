// C ABI of libvct: argument validation, pyramid layout, launch planning.
// Every entry point validates all arguments before enqueuing anything and
// reports failures through a return code plus a thread-local
// "function: message" string (the thesis's checkErrors(context) convention,
// Section 5.4.1 "IoObject").
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <string>

#include "vct_internal.h"

// Scratch of the allocation-free backward (vct_trace_backward_saved_noalloc):
// its accumulator, bound partials and control word, in place of a caller
// workspace.  Every GPU the library runs on holds its own copy until the
// process ends.  Host code must not use this name as a device address: the
// address on each device comes from hipGetSymbolAddress (scratch_on_device).
static __device__ __align__(256) unsigned char scratch[VCT_NOALLOC_SCRATCH_BYTES];

namespace {

thread_local std::string g_err;
thread_local hipEvent_t* g_events = nullptr;
thread_local int g_n_events = 0;

// The event registration (diagnostics) applies to one enqueuing call only.
EventSink take_events() {
    EventSink es;
    es.ev = g_events;
    es.n = g_n_events;
    g_events = nullptr;
    g_n_events = 0;
    return es;
}

int fail(int code, const char* fn, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = std::string(fn) + ": " + buf;
    return code;
}

void ok() { g_err.clear(); }

bool finite(float v) { return isfinite(v); }

// A named byte range of a caller's buffer.
struct Span {
    const char* name;
    const void* p;
    size_t bytes;
};

// Fails with VCT_EINVAL if two of the spans share a byte (null or empty spans
// share none).  Used where kernels index through values other kernels of the
// same call wrote to device memory: an output that aliased their storage
// would turn into indices past a buffer's end.
int check_disjoint(const char* fn, const Span* s, int n) {
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) {
            if (!s[i].p || !s[j].p || !s[i].bytes || !s[j].bytes) continue;
            const uintptr_t a = (uintptr_t)s[i].p, b = (uintptr_t)s[j].p;
            if (a < b + s[j].bytes && b < a + s[i].bytes)
                return fail(VCT_EINVAL, fn, "%s and %s overlap", s[i].name, s[j].name);
        }
    return 0;
}

int check_grid(const char* fn, const vct_grid* g) {
    if (!g) return fail(VCT_EINVAL, fn, "grid is null");
    if (g->n < 1 || g->n > VCT_MAX_N || (g->n & (g->n - 1)))
        return fail(VCT_EINVAL, fn, "grid n = %d must be a power of two in [1, %d]", g->n, VCT_MAX_N);
    int lmax = vct_log2i(g->n) + 1;
    if (g->levels < 1 || g->levels > lmax)
        return fail(VCT_EINVAL, fn, "grid levels = %d must be in [1, %d] for n = %d", g->levels, lmax, g->n);
    if (g->dtype != VCT_F32 && g->dtype != VCT_F16 && g->dtype != VCT_BF16)
        return fail(VCT_EINVAL, fn, "grid dtype = %d is not VCT_F32, VCT_F16 or VCT_BF16", g->dtype);
    for (int i = 0; i < 3; ++i)
        if (!finite(g->origin[i])) return fail(VCT_EINVAL, fn, "grid origin[%d] is not finite", i);
    if (!finite(g->extent) || !(g->extent > 0.f))
        return fail(VCT_EINVAL, fn, "grid extent must be finite and > 0");
    if (g->anisotropic != 0 && g->anisotropic != 1)
        return fail(VCT_EINVAL, fn, "grid anisotropic = %d must be 0 or 1", g->anisotropic);
    return VCT_OK;
}

int check_gbuffer(const char* fn, const vct_gbuffer* gb) {
    if (!gb) return fail(VCT_EINVAL, fn, "gbuffer is null");
    if (gb->b < 0 || gb->h < 0 || gb->w < 0)
        return fail(VCT_EINVAL, fn, "gbuffer shape (%d, %d, %d) has a negative extent", gb->b, gb->h, gb->w);
    if (gb->h > 32768 || gb->w > 32768 || gb->b > 4096)
        return fail(VCT_EINVAL, fn, "gbuffer shape (%d, %d, %d) exceeds (4096, 32768, 32768)", gb->b, gb->h, gb->w);
    long long np = (long long)gb->b * gb->h * gb->w;
    if (np > (1ll << 30)) return fail(VCT_EINVAL, fn, "gbuffer has %lld pixels, more than 2^30", np);
    if (np > 0 && (!gb->pos_rough || !gb->normal || !gb->cam_pos))
        return fail(VCT_EINVAL, fn, "gbuffer pos_rough, normal and cam_pos must be non-null");
    return VCT_OK;
}

int check_params(const char* fn, const vct_grid* g, const vct_cone_params* p) {
    if (!p) return fail(VCT_EINVAL, fn, "params is null");
    if (p->n_diffuse < 0 || p->n_diffuse > VCT_MAX_DIFFUSE)
        return fail(VCT_EINVAL, fn, "n_diffuse = %d must be in [0, %d]", p->n_diffuse, VCT_MAX_DIFFUSE);
    for (int q = 0; q < p->n_diffuse; ++q) {
        for (int i = 0; i < 3; ++i)
            if (!finite(p->diffuse_dir[q][i])) return fail(VCT_EINVAL, fn, "diffuse_dir[%d] is not finite", q);
        float l2 = p->diffuse_dir[q][0] * p->diffuse_dir[q][0] + p->diffuse_dir[q][1] * p->diffuse_dir[q][1] +
                   p->diffuse_dir[q][2] * p->diffuse_dir[q][2];
        if (!(l2 > 0.f)) return fail(VCT_EINVAL, fn, "diffuse_dir[%d] is the zero vector", q);
        if (!finite(p->diffuse_weight[q])) return fail(VCT_EINVAL, fn, "diffuse_weight[%d] is not finite", q);
    }
    struct {
        const char* name;
        float v;
    } nonneg[] = {{"diffuse_aperture", p->diffuse_aperture},
                  {"spec_aperture_scale", p->spec_aperture_scale},
                  {"occ_aperture", p->occ_aperture},
                  {"t0", p->t0}};
    for (auto& e : nonneg)
        if (!finite(e.v) || e.v < 0.f) return fail(VCT_EINVAL, fn, "%s must be finite and >= 0", e.name);
    for (int i = 0; i < 3; ++i)
        if (!finite(p->light_pos[i])) return fail(VCT_EINVAL, fn, "light_pos[%d] is not finite", i);
    if (!finite(p->normal_offset)) return fail(VCT_EINVAL, fn, "normal_offset is not finite");
    if (!finite(p->step_factor) || !(p->step_factor > 0.f))
        return fail(VCT_EINVAL, fn, "step_factor must be finite and > 0");
    if (!finite(p->max_dist) || !(p->max_dist > 0.f)) return fail(VCT_EINVAL, fn, "max_dist must be finite and > 0");
    if (!finite(p->alpha_thresh) || !(p->alpha_thresh > 0.f))
        return fail(VCT_EINVAL, fn, "alpha_thresh must be finite and > 0");
    double voxel = (double)g->extent / g->n;
    double steps = (double)p->max_dist / ((double)p->step_factor * voxel);
    if (steps > VCT_MAX_STEPS)
        return fail(VCT_EINVAL, fn, "max_dist / (step_factor * voxel) = %.3g exceeds %d samples per cone", steps,
                    VCT_MAX_STEPS);
    return VCT_OK;
}

void split(double v, float& hi, float& lo) {
    hi = (float)v;
    lo = (float)(v - (double)hi);
}

TraceArgs make_args(const vct_grid* g, const PyrLayout& L, const void* pyr, const vct_gbuffer* gb,
                    const vct_cone_params* p) {
    TraceArgs a{};
    a.n = g->n;
    a.levels = g->levels;
    for (int i = 0; i < 3; ++i) a.origin[i] = g->origin[i];
    double scale = (double)g->n / (double)g->extent;
    split(scale, a.scale_hi, a.scale_lo);
    a.voxel = (float)((double)g->extent / g->n);
    for (int l = 0; l < VCT_MAX_LEVELS; ++l) {
        if (l < g->levels) {
            a.lv[l].n = g->n >> l;
            a.lv[l].nb = L.nb[l];
            a.lv[l].off = (uint32_t)L.off[l];
        } else {
            a.lv[l].n = 1;
            a.lv[l].nb = 1;
            a.lv[l].off = 0;
        }
    }
    a.pyr = pyr;
    a.rsrc = vct_pyr_rsrc(pyr, g->dtype == VCT_F32 ? 16 : 8, (uint32_t)L.total_texels);
    a.rraw = vct_pyr_raw_rsrc(pyr, (uint64_t)L.total_texels * (uint64_t)L.texel_bytes);
    for (int d = 0; d < 6; ++d)
        for (int l = 0; l < VCT_MAX_LEVELS; ++l)
            a.ddelta[d][l] = l < g->levels ? (uint32_t)(L.doff[d][l] - L.off[l]) : 0u;
    a.inv_scale2 = (float)(((double)g->extent / g->n) * ((double)g->extent / g->n));
    a.aniso = g->anisotropic ? 1 : 0;
    // (narrow pyramids keep every byte offset below 2^32, within the raw
    // resource's range of 2^32 - 1 bytes)
    a.wide = L.total_texels * (int64_t)L.texel_bytes >= (int64_t(1) << 32) ? 1 : 0;
    a.b = gb->b;
    a.h = gb->h;
    a.w = gb->w;
    a.tiles_x = (gb->w + 15) / 16;
    a.tiles_y = (gb->h + 15) / 16;
    a.n_tiles = a.tiles_x * a.tiles_y * gb->b;
    a.pos_rough = reinterpret_cast<const float4*>(gb->pos_rough);
    a.normal = reinterpret_cast<const float4*>(gb->normal);
    a.cam_pos = gb->cam_pos;
    a.n_diffuse = p->n_diffuse;
    a.enable_spec = p->enable_spec ? 1 : 0;
    a.enable_occ = p->enable_occ ? 1 : 0;
    for (int q = 0; q < p->n_diffuse; ++q) {
        for (int i = 0; i < 3; ++i) a.dir[q][i] = p->diffuse_dir[q][i];
        a.weight[q] = p->diffuse_weight[q];
    }
    a.diffuse_aperture = p->diffuse_aperture;
    a.spec_aperture_scale = p->spec_aperture_scale;
    a.occ_aperture = p->occ_aperture;
    for (int i = 0; i < 3; ++i) {
        double lt = ((double)p->light_pos[i] - (double)g->origin[i]) * scale;
        split(lt, a.light_tex[i][0], a.light_tex[i][1]);
    }
    a.step_factor = p->step_factor;
    a.t0 = p->t0;
    a.normal_offset = p->normal_offset;
    a.max_dist = p->max_dist;
    a.alpha_thresh = p->alpha_thresh;
    double voxel = (double)g->extent / g->n;
    a.max_steps = (int)ceil((double)p->max_dist / ((double)p->step_factor * voxel)) + 2;
    return a;
}

int device_error(const char* fn, hipError_t e) {
    return fail(VCT_EDEVICE, fn, "HIP error %d (%s)", (int)e, hipGetErrorString(e));
}

// Device address of `scratch` on the current device, looked up once per
// device (with that device current) and kept; the stream must belong to the
// current device.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

int scratch_on_device(const char* fn, hipStream_t stream, void** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return device_error(fn, e);
    if (dev < 0 || dev >= kMaxDevices)
        return fail(VCT_EDEVICE, fn, "device %d is beyond the %d devices the scratch table covers", dev, kMaxDevices);
    if (stream) {
        hipDevice_t sdev = -1;
        e = hipStreamGetDevice(stream, &sdev);
        if (e != hipSuccess) return device_error(fn, e);
        if (sdev != dev)
            return fail(VCT_EINVAL, fn, "stream belongs to device %d but device %d is current", (int)sdev, dev);
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return device_error(fn, e);
        if (!p) return fail(VCT_EDEVICE, fn, "hipGetSymbolAddress gave a null scratch address on device %d", dev);
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return VCT_OK;
}

}  // namespace

extern "C" {

int vct_pyramid_bytes(const vct_grid* grid, size_t* bytes) {
    const char* fn = "vct_pyramid_bytes";
    if (int r = check_grid(fn, grid)) return r;
    if (!bytes) return fail(VCT_EINVAL, fn, "bytes is null");
    *bytes = (size_t)vct_make_layout(grid->n, grid->levels, grid->dtype, grid->anisotropic).bytes;
    ok();
    return VCT_OK;
}

int vct_build_mips(const vct_grid* grid, const float* base, void* pyramid, size_t pyramid_bytes,
                   hipStream_t stream) {
    const char* fn = "vct_build_mips";
    EventSink es = take_events();
    if (int r = check_grid(fn, grid)) return r;
    if (!base || !pyramid) return fail(VCT_EINVAL, fn, "base and pyramid must be non-null");
    PyrLayout L = vct_make_layout(grid->n, grid->levels, grid->dtype, grid->anisotropic);
    if (pyramid_bytes < (size_t)L.bytes)
        return fail(VCT_EWORKSPACE, fn, "pyramid buffer has %zu bytes, needs %lld", pyramid_bytes,
                    (long long)L.bytes);
    hipError_t e = vct_launch_build_mips(L, base, pyramid, stream, es);
    if (e != hipSuccess) return device_error(fn, e);
    ok();
    return VCT_OK;
}

static int unpack_common(const char* fn, const vct_grid* grid, const void* pyramid, int32_t level, int32_t direction,
                         float* out, hipStream_t stream) {
    if (int r = check_grid(fn, grid)) return r;
    if (!pyramid || !out) return fail(VCT_EINVAL, fn, "pyramid and out must be non-null");
    if (level < 0 || level >= grid->levels)
        return fail(VCT_EINVAL, fn, "level = %d must be in [0, %d]", level, grid->levels - 1);
    if (direction < 0 || direction >= (grid->anisotropic ? 6 : 1))
        return fail(VCT_EINVAL, fn, "direction = %d must be in [0, %d]", direction, grid->anisotropic ? 5 : 0);
    PyrLayout L = vct_make_layout(grid->n, grid->levels, grid->dtype, grid->anisotropic);
    hipError_t e = vct_launch_unpack(L, pyramid, level, direction, out, stream);
    if (e != hipSuccess) return device_error(fn, e);
    ok();
    return VCT_OK;
}

int vct_unpack_level(const vct_grid* grid, const void* pyramid, int32_t level, float* out, hipStream_t stream) {
    return unpack_common("vct_unpack_level", grid, pyramid, level, 0, out, stream);
}

int vct_unpack_level_dir(const vct_grid* grid, const void* pyramid, int32_t level, int32_t direction, float* out,
                         hipStream_t stream) {
    return unpack_common("vct_unpack_level_dir", grid, pyramid, level, direction, out, stream);
}

static int trace_common(const char* fn, const vct_grid* grid, const void* pyramid, const vct_gbuffer* gbuf,
                        const vct_cone_params* params, float* out, unsigned long long* count, int n_counts,
                        hipStream_t stream) {
    const bool counting = n_counts > 0;
    EventSink es = take_events();
    if (int r = check_grid(fn, grid)) return r;
    if (int r = check_gbuffer(fn, gbuf)) return r;
    if (int r = check_params(fn, grid, params)) return r;
    long long np = (long long)gbuf->b * gbuf->h * gbuf->w;
    if (counting && !count) return fail(VCT_EINVAL, fn, "count is null");
    if (!counting && !out && np > 0) return fail(VCT_EINVAL, fn, "out is null");
    if (!pyramid) return fail(VCT_EINVAL, fn, "pyramid is null");
    PyrLayout L = vct_make_layout(grid->n, grid->levels, grid->dtype, grid->anisotropic);
    TraceArgs a = make_args(grid, L, pyramid, gbuf, params);
    if (a.n_tiles == 0 && !count) {
        ok();
        return VCT_OK;
    }
    hipError_t e = vct_launch_trace(a, grid->dtype, out, counting ? count : nullptr, n_counts, stream, es);
    if (e != hipSuccess) return device_error(fn, e);
    ok();
    return VCT_OK;
}

int vct_trace(const vct_grid* grid, const void* pyramid, const vct_gbuffer* gbuf, const vct_cone_params* params,
              float* out, hipStream_t stream) {
    return trace_common("vct_trace", grid, pyramid, gbuf, params, out, nullptr, 0, stream);
}

int vct_count_samples(const vct_grid* grid, const void* pyramid, const vct_gbuffer* gbuf,
                      const vct_cone_params* params, unsigned long long* count, hipStream_t stream) {
    return trace_common("vct_count_samples", grid, pyramid, gbuf, params, nullptr, count, 1, stream);
}

int vct_count_sample_levels(const vct_grid* grid, const void* pyramid, const vct_gbuffer* gbuf,
                            const vct_cone_params* params, unsigned long long* counts, hipStream_t stream) {
    return trace_common("vct_count_sample_levels", grid, pyramid, gbuf, params, nullptr, counts, 2, stream);
}

static int shade_common(const char* fn, const vct_grid* grid, const void* pyramid, const vct_gbuffer* gbuf,
                        const float* material, const vct_cone_params* params, const vct_shade_params* shade,
                        float* out, unsigned long long* count, bool counting, hipStream_t stream) {
    EventSink es = take_events();
    if (int r = check_grid(fn, grid)) return r;
    if (int r = check_gbuffer(fn, gbuf)) return r;
    if (int r = check_params(fn, grid, params)) return r;
    if (!shade) return fail(VCT_EINVAL, fn, "shade is null");
    if (shade->n_lights < 0 || shade->n_lights > VCT_MAX_LIGHTS)
        return fail(VCT_EINVAL, fn, "n_lights = %d must be in [0, %d]", shade->n_lights, VCT_MAX_LIGHTS);
    for (int l = 0; l < shade->n_lights; ++l)
        for (int i = 0; i < 3; ++i)
            if (!finite(shade->light_pos[l][i]) || !finite(shade->light_diffuse[l][i]) ||
                !finite(shade->light_specular[l][i]))
                return fail(VCT_EINVAL, fn, "light %d has a non-finite position or intensity", l);
    for (int i = 0; i < 3; ++i)
        if (!finite(shade->specular_color[i])) return fail(VCT_EINVAL, fn, "specular_color is not finite");
    if (!finite(shade->first_hit_alpha) || shade->first_hit_alpha < 0.f || shade->first_hit_alpha >= 1.f)
        return fail(VCT_EINVAL, fn, "first_hit_alpha must be in [0, 1)");
    struct {
        const char* name;
        float v;
    } nonneg[] = {{"shadow_strength", shade->shadow_strength},
                  {"grace_per_shininess", shade->grace_per_shininess},
                  {"shininess_falloff", shade->shininess_falloff}};
    for (auto& e : nonneg)
        if (!finite(e.v) || e.v < 0.f) return fail(VCT_EINVAL, fn, "%s must be finite and >= 0", e.name);
    long long np = (long long)gbuf->b * gbuf->h * gbuf->w;
    if (counting && !count) return fail(VCT_EINVAL, fn, "count is null");
    if (np > 0 && (!pyramid || !material || (!counting && !out)))
        return fail(VCT_EINVAL, fn, counting ? "pyramid and material must be non-null"
                                             : "pyramid, material and out must be non-null");
    PyrLayout L = vct_make_layout(grid->n, grid->levels, grid->dtype, grid->anisotropic);
    TraceArgs a = make_args(grid, L, pyramid, gbuf, params);
    if (a.n_tiles == 0 && !counting) {
        ok();
        return VCT_OK;
    }
    hipError_t e = vct_launch_shade(a, grid->dtype, shade, material, counting ? nullptr : out,
                                    counting ? count : nullptr, stream, es);
    if (e != hipSuccess) return device_error(fn, e);
    ok();
    return VCT_OK;
}

int vct_shade(const vct_grid* grid, const void* pyramid, const vct_gbuffer* gbuf, const float* material,
              const vct_cone_params* params, const vct_shade_params* shade, float* out, hipStream_t stream) {
    return shade_common("vct_shade", grid, pyramid, gbuf, material, params, shade, out, nullptr, false, stream);
}

int vct_count_shade_samples(const vct_grid* grid, const void* pyramid, const vct_gbuffer* gbuf,
                            const float* material, const vct_cone_params* params, const vct_shade_params* shade,
                            unsigned long long* count, hipStream_t stream) {
    return shade_common("vct_count_shade_samples", grid, pyramid, gbuf, material, params, shade, nullptr, count,
                        true, stream);
}

int vct_voxelize_workspace_bytes(const vct_grid* grid, int64_t n_tris, int32_t surface, size_t* bytes) {
    const char* fn = "vct_voxelize_workspace_bytes";
    if (int r = check_grid(fn, grid)) return r;
    if (n_tris < 0 || n_tris >= (int64_t(1) << 31))
        return fail(VCT_EINVAL, fn, "n_tris = %lld must be in [0, 2^31)", (long long)n_tris);
    if (!bytes) return fail(VCT_EINVAL, fn, "bytes is null");
    *bytes = vct_voxelize_workspace_size(grid->n, n_tris, surface != 0);
    ok();
    return VCT_OK;
}

int vct_voxelize(const vct_grid* grid, const float* tris, const float* colors, int64_t n_tris,
                 const vct_voxelize_params* params, float* base, float* normal, float* albedo, void* workspace,
                 size_t workspace_bytes, hipStream_t stream) {
    const char* fn = "vct_voxelize";
    EventSink es = take_events();
    if (int r = check_grid(fn, grid)) return r;
    if (n_tris < 0 || n_tris >= (int64_t(1) << 31))
        return fail(VCT_EINVAL, fn, "n_tris = %lld must be in [0, 2^31)", (long long)n_tris);
    if (!params) return fail(VCT_EINVAL, fn, "params is null");
    if (params->n_lights < 0 || params->n_lights > VCT_MAX_LIGHTS)
        return fail(VCT_EINVAL, fn, "n_lights = %d must be in [0, %d]", params->n_lights, VCT_MAX_LIGHTS);
    for (int l = 0; l < params->n_lights; ++l) {
        for (int i = 0; i < 3; ++i)
            if (!finite(params->light_pos[l][i]) || !finite(params->light_color[l][i]) ||
                !finite(params->attenuation[l][i]) || params->attenuation[l][i] < 0.f)
                return fail(VCT_EINVAL, fn, "light %d: position and colour must be finite, attenuation finite and >= 0",
                            l);
        if (!(params->attenuation[l][0] + params->attenuation[l][1] + params->attenuation[l][2] > 0.f))
            return fail(VCT_EINVAL, fn, "light %d: attenuation terms are all 0", l);
    }
    if (!finite(params->ambient) || params->ambient < 0.f || !finite(params->diffuse) || params->diffuse < 0.f)
        return fail(VCT_EINVAL, fn, "ambient and diffuse must be finite and >= 0");
    if (!base || !workspace) return fail(VCT_EINVAL, fn, "base and workspace must be non-null");
    if (n_tris > 0 && (!tris || !colors)) return fail(VCT_EINVAL, fn, "tris and colors must be non-null");
    if ((normal == nullptr) != (albedo == nullptr))
        return fail(VCT_EINVAL, fn, "normal and albedo must both be null or both be non-null");
    const bool surface = normal != nullptr;
    const size_t need = vct_voxelize_workspace_size(grid->n, n_tris, surface);
    if (workspace_bytes < need)
        return fail(VCT_EWORKSPACE, fn, "workspace has %zu bytes, needs %zu", workspace_bytes, need);
    {
        // outputs and workspace pairwise apart, and apart from the mesh (tris
        // and colors are only read, so they may share memory)
        const size_t grid_bytes = (size_t)grid->n * grid->n * grid->n * 16;
        const Span out[] = {{"base", base, grid_bytes}, {"normal", normal, grid_bytes},
                            {"albedo", albedo, grid_bytes}, {"workspace", workspace, need}};
        if (int r = check_disjoint(fn, out, 4)) return r;
        for (const Span& in : {Span{"tris", tris, (size_t)n_tris * 36}, Span{"colors", colors, (size_t)n_tris * 12}})
            for (const Span& o : out) {
                const Span pair[] = {o, in};
                if (int r = check_disjoint(fn, pair, 2)) return r;
            }
    }
    hipError_t e = vct_launch_voxelize(grid, tris, colors, n_tris, params, base, normal, albedo, workspace, stream,
                                       es);
    if (e != hipSuccess) return device_error(fn, e);
    ok();
    return VCT_OK;
}

int vct_backward_workspace_bytes(const vct_grid* grid, const vct_gbuffer* gbuf, const vct_cone_params* params,
                                 size_t* bytes) {
    const char* fn = "vct_backward_workspace_bytes";
    if (int r = check_grid(fn, grid)) return r;
    if (int r = check_gbuffer(fn, gbuf)) return r;
    if (int r = check_params(fn, grid, params)) return r;
    if (!bytes) return fail(VCT_EINVAL, fn, "bytes is null");
    PyrLayout L = vct_make_layout(grid->n, grid->levels, grid->dtype, grid->anisotropic);
    TraceArgs a = make_args(grid, L, nullptr, gbuf, params);
    *bytes = (size_t)vct_plan_backward(L, a).bytes;
    ok();
    return VCT_OK;
}

int vct_lane_state_bytes(const vct_gbuffer* gbuf, const vct_cone_params* params, size_t* bytes) {
    const char* fn = "vct_lane_state_bytes";
    if (int r = check_gbuffer(fn, gbuf)) return r;
    if (!params) return fail(VCT_EINVAL, fn, "params is null");
    if (params->n_diffuse < 0 || params->n_diffuse > VCT_MAX_DIFFUSE)
        return fail(VCT_EINVAL, fn, "n_diffuse = %d must be in [0, %d]", params->n_diffuse, VCT_MAX_DIFFUSE);
    if (!bytes) return fail(VCT_EINVAL, fn, "bytes is null");
    int64_t lanes = (int64_t)gbuf->b * gbuf->h * gbuf->w * (params->n_diffuse + 2);
    *bytes = (size_t)vct_lane_state_bytes(lanes);
    ok();
    return VCT_OK;
}

int vct_trace_save(const vct_grid* grid, const void* pyramid, const vct_gbuffer* gbuf, const vct_cone_params* params,
                   float* out, void* lane_state, size_t lane_state_bytes, hipStream_t stream) {
    const char* fn = "vct_trace_save";
    EventSink es = take_events();
    if (int r = check_grid(fn, grid)) return r;
    if (int r = check_gbuffer(fn, gbuf)) return r;
    if (int r = check_params(fn, grid, params)) return r;
    long long np = (long long)gbuf->b * gbuf->h * gbuf->w;
    if (np > 0 && (!out || !lane_state || !pyramid))
        return fail(VCT_EINVAL, fn, "pyramid, out and lane_state must be non-null");
    int64_t need = vct_lane_state_bytes(np * (params->n_diffuse + 2));
    if (lane_state_bytes < (size_t)need)
        return fail(VCT_EWORKSPACE, fn, "lane_state has %zu bytes, needs %lld", lane_state_bytes, (long long)need);
    PyrLayout L = vct_make_layout(grid->n, grid->levels, grid->dtype, grid->anisotropic);
    TraceArgs a = make_args(grid, L, pyramid, gbuf, params);
    hipError_t e = vct_launch_trace_save(a, grid->dtype, out, lane_state, stream, es);
    if (e != hipSuccess) return device_error(fn, e);
    ok();
    return VCT_OK;
}

// noalloc: the workspace is the library's device scratch (workspace and
// workspace_bytes are ignored); sizes beyond it are rejected.
static int backward_common(const char* fn, const vct_grid* grid, const void* pyramid, const vct_gbuffer* gbuf,
                           const vct_cone_params* params, const void* lane_state, size_t lane_state_bytes,
                           bool saved, const float* grad_out, float* grad_base, void* workspace,
                           size_t workspace_bytes, hipStream_t stream, bool noalloc = false) {
    EventSink es = take_events();
    if (int r = check_grid(fn, grid)) return r;
    if (int r = check_gbuffer(fn, gbuf)) return r;
    if (int r = check_params(fn, grid, params)) return r;
    if (!(params->alpha_thresh <= 1.0f))
        return fail(VCT_EINVAL, fn, "alpha_thresh = %g: the adjoint needs alpha_thresh <= 1 (transmittance of a "
                    "continuing cone must stay positive)", (double)params->alpha_thresh);
    if (!pyramid || !grad_base || (!noalloc && !workspace))
        return fail(VCT_EINVAL, fn, noalloc ? "pyramid and grad_base must be non-null"
                                            : "pyramid, grad_base and workspace must be non-null");
    long long np = (long long)gbuf->b * gbuf->h * gbuf->w;
    if (np > 0 && !grad_out) return fail(VCT_EINVAL, fn, "grad_out is null");
    PyrLayout L = vct_make_layout(grid->n, grid->levels, grid->dtype, grid->anisotropic);
    TraceArgs a = make_args(grid, L, pyramid, gbuf, params);
    BackwardPlan P = vct_plan_backward(L, a);
    const int64_t need = saved ? P.state_off : P.bytes;
    if (noalloc && need > (int64_t)VCT_NOALLOC_SCRATCH_BYTES)
        return fail(VCT_EWORKSPACE, fn, "these shapes need %lld bytes of scratch; the allocation-free entry point "
                    "has %lld (VCT_NOALLOC_SCRATCH_BYTES): use vct_trace_backward_saved with a workspace",
                    (long long)need, (long long)VCT_NOALLOC_SCRATCH_BYTES);
    if (!noalloc && workspace_bytes < (size_t)need)
        return fail(VCT_EWORKSPACE, fn, "workspace has %zu bytes, needs %lld", workspace_bytes, (long long)need);
    if (saved) {
        if (np > 0 && !lane_state) return fail(VCT_EINVAL, fn, "lane_state is null");
        if (lane_state_bytes < (size_t)P.state_bytes)
            return fail(VCT_EWORKSPACE, fn, "lane_state has %zu bytes, needs %lld", lane_state_bytes,
                        (long long)P.state_bytes);
    }
    if (noalloc)
        if (int r = scratch_on_device(fn, stream, &workspace)) return r;
    hipError_t e = vct_launch_backward(L, a, P, grad_out, grad_base, workspace, saved ? lane_state : nullptr, stream,
                                       es);
    if (e != hipSuccess) return device_error(fn, e);
    ok();
    return VCT_OK;
}

int vct_trace_backward(const vct_grid* grid, const void* pyramid, const vct_gbuffer* gbuf,
                       const vct_cone_params* params, const float* grad_out, float* grad_base, void* workspace,
                       size_t workspace_bytes, hipStream_t stream) {
    return backward_common("vct_trace_backward", grid, pyramid, gbuf, params, nullptr, 0, false, grad_out, grad_base,
                           workspace, workspace_bytes, stream);
}

int vct_trace_backward_saved(const vct_grid* grid, const void* pyramid, const vct_gbuffer* gbuf,
                             const vct_cone_params* params, const void* lane_state, size_t lane_state_bytes,
                             const float* grad_out, float* grad_base, void* workspace, size_t workspace_bytes,
                             hipStream_t stream) {
    return backward_common("vct_trace_backward_saved", grid, pyramid, gbuf, params, lane_state, lane_state_bytes,
                           true, grad_out, grad_base, workspace, workspace_bytes, stream);
}

int vct_trace_backward_saved_noalloc(const vct_grid* grid, const void* pyramid, const vct_gbuffer* gbuf,
                                     const vct_cone_params* params, const void* lane_state, size_t lane_state_bytes,
                                     const float* grad_out, float* grad_base, hipStream_t stream) {
    return backward_common("vct_trace_backward_saved_noalloc", grid, pyramid, gbuf, params, lane_state,
                           lane_state_bytes, true, grad_out, grad_base, nullptr, 0, stream, true);
}

int vct_bounce_workspace_bytes(const vct_grid* grid, size_t* bytes) {
    const char* fn = "vct_bounce_workspace_bytes";
    if (int r = check_grid(fn, grid)) return r;
    if (!bytes) return fail(VCT_EINVAL, fn, "bytes is null");
    *bytes = vct_bounce_workspace_size(grid->n);
    ok();
    return VCT_OK;
}

int vct_bounce(const vct_grid* grid, const void* pyramid, const float* base, const float* normal,
               const float* albedo, const vct_cone_params* params, float* out, void* workspace,
               size_t workspace_bytes, hipStream_t stream) {
    const char* fn = "vct_bounce";
    EventSink es = take_events();
    if (int r = check_grid(fn, grid)) return r;
    if (int r = check_params(fn, grid, params)) return r;
    if (!pyramid || !base || !normal || !albedo || !out || !workspace)
        return fail(VCT_EINVAL, fn, "pyramid, base, normal, albedo, out and workspace must be non-null");
    const size_t need = vct_bounce_workspace_size(grid->n);
    if (workspace_bytes < need)
        return fail(VCT_EWORKSPACE, fn, "workspace has %zu bytes, needs %zu", workspace_bytes, need);
    PyrLayout L = vct_make_layout(grid->n, grid->levels, grid->dtype, grid->anisotropic);
    {
        // the workspace apart from every buffer, out apart from every input
        // but base (out == base is the in-place form); the inputs are only read
        const size_t grid_bytes = (size_t)grid->n * grid->n * grid->n * 16;
        const Span ins[] = {{"pyramid", pyramid, (size_t)L.bytes}, {"base", base, grid_bytes},
                            {"normal", normal, grid_bytes}, {"albedo", albedo, grid_bytes}};
        const Span ws{"workspace", workspace, need}, o{"out", out, grid_bytes};
        const Span pair_wo[] = {ws, o};
        if (int r = check_disjoint(fn, pair_wo, 2)) return r;
        for (const Span& in : ins) {
            const Span pair_w[] = {ws, in};
            if (int r = check_disjoint(fn, pair_w, 2)) return r;
            if (in.p == base && out == base) continue;
            const Span pair_o[] = {o, in};
            if (int r = check_disjoint(fn, pair_o, 2)) return r;
        }
    }
    const vct_gbuffer none{};
    TraceArgs a = make_args(grid, L, pyramid, &none, params);
    a.enable_spec = 0;
    a.enable_occ = 0;
    hipError_t e = vct_launch_bounce(a, grid->dtype, base, normal, albedo, out, workspace, stream, es);
    if (e != hipSuccess) return device_error(fn, e);
    ok();
    return VCT_OK;
}

int vct_record_kernel_events(hipEvent_t* events, int32_t count) {
    const char* fn = "vct_record_kernel_events";
    if (count < 0 || count > 64) return fail(VCT_EINVAL, fn, "count = %d must be in [0, 64]", count);
    if (count > 0 && !events) return fail(VCT_EINVAL, fn, "events is null");
    g_events = count > 0 ? events : nullptr;
    g_n_events = count;
    ok();
    return VCT_OK;
}

const char* vct_last_error(void) { return g_err.c_str(); }

}  // extern "C"
