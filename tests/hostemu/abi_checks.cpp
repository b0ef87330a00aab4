// The C ABI's argument validation, run inside the host build (so with
// AddressSanitizer and UndefinedBehaviorSanitizer when the build has them):
// every entry point is called with null, negative, non-finite, oversized and
// overflowing arguments, and must return the documented code with a
// "function: message" error string, without reading or writing any buffer
// (the pointers handed in for that are not allocations, so an access would
// fail the emulator's range check).  Valid size queries must succeed and
// clear the error string.
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>

#include "emu.h"
#include "vct.h"

namespace {

int g_checks = 0;

void expect(int rc, int want, const char* fn, const char* needle, int line) {
    ++g_checks;
    const char* err = vct_last_error();
    if (rc != want) emu_fail("abi check at line %d: %s returned %d, expected %d (%s)", line, fn, rc, want, err);
    if (want == VCT_OK) {
        if (err[0] != '\0') emu_fail("abi check at line %d: %s succeeded but left the error \"%s\"", line, fn, err);
        return;
    }
    const std::string prefix = std::string(fn) + ":";
    if (strncmp(err, prefix.c_str(), prefix.size()) != 0)
        emu_fail("abi check at line %d: error \"%s\" does not start with \"%s\"", line, err, prefix.c_str());
    if (needle && !strstr(err, needle))
        emu_fail("abi check at line %d: error \"%s\" does not mention \"%s\"", line, err, needle);
}

#define EXPECT(call, want, fn, needle) expect((call), (want), (fn), (needle), __LINE__)

vct_grid grid16() {
    vct_grid g{};
    g.n = 16;
    g.levels = 5;
    g.dtype = VCT_F32;
    g.extent = 1.0f;
    return g;
}

vct_cone_params params() {
    vct_cone_params p{};
    p.n_diffuse = 1;
    p.diffuse_dir[0][2] = 1.0f;
    p.diffuse_weight[0] = 1.0f;
    p.diffuse_aperture = 1.0f;
    p.enable_spec = 1;
    p.enable_occ = 1;
    p.spec_aperture_scale = 0.5f;
    p.occ_aperture = 0.3f;
    p.light_pos[1] = 2.0f;
    p.step_factor = 0.5f;
    p.t0 = 0.001f;
    p.normal_offset = 1.0f;
    p.max_dist = 1.0f;
    p.alpha_thresh = 0.99f;
    return p;
}

vct_shade_params shade_params() {
    vct_shade_params s{};
    s.n_lights = 1;
    s.light_pos[0][1] = 2.0f;
    s.light_diffuse[0][0] = s.light_diffuse[0][1] = s.light_diffuse[0][2] = 1.0f;
    s.first_hit_alpha = 0.01f;
    s.shadow_strength = 1.0f;
    s.grace_per_shininess = 0.025f;
    s.shininess_falloff = 1.0f;
    return s;
}

}  // namespace

// Returns the number of checks that passed (each failure ends the process).
int run_abi_checks() {
    // Distinct non-null addresses that are not allocations: the calls below
    // must reject their arguments before touching any buffer.
    float* const fake = reinterpret_cast<float*>(uintptr_t(1) << 40);
    void* const vfake = fake;
    size_t bytes = 0;
    const float nan = std::nanf(""), inf = INFINITY;

    // grids
    EXPECT(vct_pyramid_bytes(nullptr, &bytes), VCT_EINVAL, "vct_pyramid_bytes", "grid is null");
    for (int n : {0, -4, 3, 12, 2048, INT_MIN, INT_MAX}) {
        vct_grid g = grid16();
        g.n = n;
        EXPECT(vct_pyramid_bytes(&g, &bytes), VCT_EINVAL, "vct_pyramid_bytes", "power of two");
    }
    for (int l : {0, -1, 6, INT_MAX}) {
        vct_grid g = grid16();
        g.levels = l;
        EXPECT(vct_pyramid_bytes(&g, &bytes), VCT_EINVAL, "vct_pyramid_bytes", "levels");
    }
    for (int d : {-1, 3, 16, INT_MAX}) {
        vct_grid g = grid16();
        g.dtype = d;
        EXPECT(vct_pyramid_bytes(&g, &bytes), VCT_EINVAL, "vct_pyramid_bytes", "dtype");
    }
    for (float e : {0.0f, -1.0f, nan, inf}) {
        vct_grid g = grid16();
        g.extent = e;
        EXPECT(vct_pyramid_bytes(&g, &bytes), VCT_EINVAL, "vct_pyramid_bytes", "extent");
    }
    {
        vct_grid g = grid16();
        g.origin[2] = -inf;
        EXPECT(vct_pyramid_bytes(&g, &bytes), VCT_EINVAL, "vct_pyramid_bytes", "origin[2]");
        g = grid16();
        g.anisotropic = 2;
        EXPECT(vct_pyramid_bytes(&g, &bytes), VCT_EINVAL, "vct_pyramid_bytes", "anisotropic");
        g = grid16();
        EXPECT(vct_pyramid_bytes(&g, nullptr), VCT_EINVAL, "vct_pyramid_bytes", "bytes is null");
        for (int n : {1, 1024}) {
            for (int a : {0, 1}) {
                g.n = n;
                g.levels = (int)std::lround(std::log2((double)n)) + 1;
                g.anisotropic = a;
                g.dtype = VCT_F32;
                EXPECT(vct_pyramid_bytes(&g, &bytes), VCT_OK, "vct_pyramid_bytes", nullptr);
            }
        }
    }

    // mip build and unpack
    vct_grid g = grid16();
    size_t pyr = 0;
    EXPECT(vct_pyramid_bytes(&g, &pyr), VCT_OK, "vct_pyramid_bytes", nullptr);
    EXPECT(vct_build_mips(&g, nullptr, vfake, pyr, nullptr), VCT_EINVAL, "vct_build_mips", "non-null");
    EXPECT(vct_build_mips(&g, fake, vfake, pyr - 1, nullptr), VCT_EWORKSPACE, "vct_build_mips", "needs");
    for (int l : {-1, 5, INT_MIN}) EXPECT(vct_unpack_level(&g, vfake, l, fake, nullptr), VCT_EINVAL, "vct_unpack_level", "level");
    EXPECT(vct_unpack_level_dir(&g, vfake, 1, 1, fake, nullptr), VCT_EINVAL, "vct_unpack_level_dir", "direction");
    EXPECT(vct_unpack_level(&g, nullptr, 0, fake, nullptr), VCT_EINVAL, "vct_unpack_level", "non-null");

    // G-buffers
    vct_cone_params p = params();
    vct_gbuffer gb{1, 4, 4, fake, fake, fake};
    const int shapes[][3] = {{-1, 4, 4}, {1, -4, 4}, {1, 4, INT_MIN}, {4097, 1, 1}, {1, 32769, 1},
                             {INT_MAX, INT_MAX, INT_MAX}, {4096, 32768, 32768}};
    for (const auto& s : shapes) {
        vct_gbuffer bad{s[0], s[1], s[2], fake, fake, fake};
        EXPECT(vct_trace(&g, vfake, &bad, &p, fake, nullptr), VCT_EINVAL, "vct_trace", "gbuffer");
    }
    EXPECT(vct_trace(&g, vfake, nullptr, &p, fake, nullptr), VCT_EINVAL, "vct_trace", "gbuffer is null");
    {
        vct_gbuffer bad = gb;
        bad.normal = nullptr;
        EXPECT(vct_trace(&g, vfake, &bad, &p, fake, nullptr), VCT_EINVAL, "vct_trace", "non-null");
    }
    EXPECT(vct_trace(&g, vfake, &gb, &p, nullptr, nullptr), VCT_EINVAL, "vct_trace", "out is null");
    EXPECT(vct_trace(&g, nullptr, &gb, &p, fake, nullptr), VCT_EINVAL, "vct_trace", "pyramid is null");
    EXPECT(vct_count_samples(&g, vfake, &gb, &p, nullptr, nullptr), VCT_EINVAL, "vct_count_samples", "count");
    EXPECT(vct_count_sample_levels(&g, vfake, &gb, &p, nullptr, nullptr), VCT_EINVAL, "vct_count_sample_levels",
           "count");

    // cone parameters
    {
        struct Case { void (*edit)(vct_cone_params&); const char* msg; };
        const Case cases[] = {
            {[](vct_cone_params& q) { q.n_diffuse = 17; }, "n_diffuse"},
            {[](vct_cone_params& q) { q.n_diffuse = -1; }, "n_diffuse"},
            {[](vct_cone_params& q) { q.diffuse_dir[0][2] = 0.0f; }, "zero vector"},
            {[](vct_cone_params& q) { q.diffuse_dir[0][0] = NAN; }, "diffuse_dir[0]"},
            {[](vct_cone_params& q) { q.diffuse_weight[0] = INFINITY; }, "diffuse_weight[0]"},
            {[](vct_cone_params& q) { q.diffuse_aperture = -0.5f; }, "diffuse_aperture"},
            {[](vct_cone_params& q) { q.occ_aperture = NAN; }, "occ_aperture"},
            {[](vct_cone_params& q) { q.light_pos[2] = INFINITY; }, "light_pos[2]"},
            {[](vct_cone_params& q) { q.normal_offset = NAN; }, "normal_offset"},
            {[](vct_cone_params& q) { q.step_factor = 0.0f; }, "step_factor"},
            {[](vct_cone_params& q) { q.max_dist = 0.0f; }, "max_dist"},
            {[](vct_cone_params& q) { q.alpha_thresh = 0.0f; }, "alpha_thresh"},
            {[](vct_cone_params& q) { q.step_factor = 1e-30f; }, "samples per cone"},
            {[](vct_cone_params& q) { q.max_dist = 3e38f; }, "samples per cone"},
        };
        for (const auto& c : cases) {
            vct_cone_params q = params();
            c.edit(q);
            EXPECT(vct_trace(&g, vfake, &gb, &q, fake, nullptr), VCT_EINVAL, "vct_trace", c.msg);
        }
        EXPECT(vct_trace(&g, vfake, &gb, nullptr, fake, nullptr), VCT_EINVAL, "vct_trace", "params is null");
    }

    // backward, saved path, allocation-free backward
    size_t ws = 0, ls = 0;
    EXPECT(vct_backward_workspace_bytes(&g, &gb, &p, &ws), VCT_OK, "vct_backward_workspace_bytes", nullptr);
    EXPECT(vct_backward_workspace_bytes(&g, &gb, &p, nullptr), VCT_EINVAL, "vct_backward_workspace_bytes",
           "bytes is null");
    EXPECT(vct_trace_backward(&g, vfake, &gb, &p, fake, fake, vfake, ws - 1, nullptr), VCT_EWORKSPACE,
           "vct_trace_backward", "workspace");
    {
        vct_cone_params q = params();
        q.alpha_thresh = 1.5f;
        EXPECT(vct_trace_backward(&g, vfake, &gb, &q, fake, fake, vfake, ws, nullptr), VCT_EINVAL,
               "vct_trace_backward", "alpha_thresh");
    }
    EXPECT(vct_lane_state_bytes(&gb, &p, &ls), VCT_OK, "vct_lane_state_bytes", nullptr);
    {
        vct_cone_params q = params();
        q.n_diffuse = 40;
        EXPECT(vct_lane_state_bytes(&gb, &q, &ls), VCT_EINVAL, "vct_lane_state_bytes", "n_diffuse");
        EXPECT(vct_lane_state_bytes(&gb, &p, &ls), VCT_OK, "vct_lane_state_bytes", nullptr);
    }
    EXPECT(vct_trace_save(&g, vfake, &gb, &p, fake, vfake, ls - 1, nullptr), VCT_EWORKSPACE, "vct_trace_save",
           "lane_state");
    EXPECT(vct_trace_backward_saved(&g, vfake, &gb, &p, vfake, ls - 1, fake, fake, vfake, ws, nullptr),
           VCT_EWORKSPACE, "vct_trace_backward_saved", "lane_state");
    EXPECT(vct_trace_backward_saved(&g, vfake, &gb, &p, vfake, ls, fake, fake, vfake, 64, nullptr),
           VCT_EWORKSPACE, "vct_trace_backward_saved", "workspace");
    {
        vct_grid big = grid16();
        big.n = 256;
        big.levels = 9;
        EXPECT(vct_trace_backward_saved_noalloc(&big, vfake, &gb, &p, vfake, ls, fake, fake, nullptr),
               VCT_EWORKSPACE, "vct_trace_backward_saved_noalloc", "VCT_NOALLOC_SCRATCH_BYTES");
        EXPECT(vct_trace_backward_saved_noalloc(&g, vfake, &gb, &p, vfake, ls - 1, fake, fake, nullptr),
               VCT_EWORKSPACE, "vct_trace_backward_saved_noalloc", "lane_state");
    }

    // shading
    {
        vct_shade_params s = shade_params();
        EXPECT(vct_shade(&g, vfake, &gb, fake, &p, nullptr, fake, nullptr), VCT_EINVAL, "vct_shade", "shade is null");
        s.n_lights = 9;
        EXPECT(vct_shade(&g, vfake, &gb, fake, &p, &s, fake, nullptr), VCT_EINVAL, "vct_shade", "n_lights");
        s = shade_params();
        s.light_pos[0][0] = nan;
        EXPECT(vct_shade(&g, vfake, &gb, fake, &p, &s, fake, nullptr), VCT_EINVAL, "vct_shade", "light 0");
        s = shade_params();
        s.first_hit_alpha = 1.0f;
        EXPECT(vct_shade(&g, vfake, &gb, fake, &p, &s, fake, nullptr), VCT_EINVAL, "vct_shade", "first_hit_alpha");
        s = shade_params();
        s.shininess_falloff = -1.0f;
        EXPECT(vct_shade(&g, vfake, &gb, fake, &p, &s, fake, nullptr), VCT_EINVAL, "vct_shade", "shininess_falloff");
        s = shade_params();
        EXPECT(vct_shade(&g, vfake, &gb, nullptr, &p, &s, fake, nullptr), VCT_EINVAL, "vct_shade", "material");
        EXPECT(vct_count_shade_samples(&g, vfake, &gb, fake, &p, &s, nullptr, nullptr), VCT_EINVAL,
               "vct_count_shade_samples", "count");
    }

    // voxelization and bounce
    {
        vct_voxelize_params v{};
        v.n_lights = 1;
        v.light_color[0][0] = 1.0f;
        v.attenuation[0][0] = 1.0f;
        v.ambient = 0.1f;
        v.diffuse = 1.0f;
        for (long long nt : {-1ll, 1ll << 31, LLONG_MAX, LLONG_MIN})
            EXPECT(vct_voxelize_workspace_bytes(&g, (int64_t)nt, 0, &bytes), VCT_EINVAL,
                   "vct_voxelize_workspace_bytes", "n_tris");
        size_t vws = 0;
        EXPECT(vct_voxelize_workspace_bytes(&g, 10, 1, &vws), VCT_OK, "vct_voxelize_workspace_bytes", nullptr);
        EXPECT(vct_voxelize(&g, nullptr, fake, 10, &v, fake, fake, fake, vfake, vws, nullptr), VCT_EINVAL,
               "vct_voxelize", "tris and colors");
        EXPECT(vct_voxelize(&g, fake, fake, 10, &v, fake, fake, nullptr, vfake, vws, nullptr), VCT_EINVAL,
               "vct_voxelize", "both be null");
        EXPECT(vct_voxelize(&g, fake, fake, 10, &v, fake, fake, fake, vfake, vws - 1, nullptr), VCT_EWORKSPACE,
               "vct_voxelize", "workspace");
        v.attenuation[0][0] = 0.0f;
        EXPECT(vct_voxelize(&g, fake, fake, 10, &v, fake, nullptr, nullptr, vfake, vws, nullptr), VCT_EINVAL,
               "vct_voxelize", "attenuation");
        v.attenuation[0][0] = 1.0f;
        v.n_lights = -1;
        EXPECT(vct_voxelize(&g, fake, fake, 10, &v, fake, nullptr, nullptr, vfake, vws, nullptr), VCT_EINVAL,
               "vct_voxelize", "n_lights");
        EXPECT(vct_bounce_workspace_bytes(&g, nullptr), VCT_EINVAL, "vct_bounce_workspace_bytes", "bytes is null");
        size_t bws = 0;
        EXPECT(vct_bounce_workspace_bytes(&g, &bws), VCT_OK, "vct_bounce_workspace_bytes", nullptr);
        EXPECT(vct_bounce(&g, vfake, fake, fake, fake, &p, fake, vfake, bws - 1, nullptr), VCT_EWORKSPACE,
               "vct_bounce", "workspace");
        // overlapping buffers (rejected before anything is enqueued; addresses only, never dereferenced)
        v.n_lights = 1;
        {
            const uintptr_t A = uintptr_t(1) << 40;
            const size_t gbytes = (size_t)g.n * g.n * g.n * 16;
            auto at = [&](size_t off) { return reinterpret_cast<float*>(A + off); };
            EXPECT(vct_voxelize(&g, at(8 * gbytes), at(9 * gbytes), 10, &v, at(0), at(gbytes / 2), at(2 * gbytes),
                                at(3 * gbytes), vws, nullptr),
                   VCT_EINVAL, "vct_voxelize", "base and normal overlap");
            EXPECT(vct_voxelize(&g, at(gbytes - 8), at(9 * gbytes), 10, &v, at(0), at(gbytes), at(2 * gbytes),
                                at(3 * gbytes), vws, nullptr),
                   VCT_EINVAL, "vct_voxelize", "base and tris overlap");
            size_t pbytes = 0;
            EXPECT(vct_pyramid_bytes(&g, &pbytes), VCT_OK, "vct_pyramid_bytes", nullptr);
            EXPECT(vct_bounce(&g, at(0), at(pbytes), at(pbytes + gbytes), at(pbytes + 2 * gbytes), &p,
                              at(pbytes + gbytes + 64), at(pbytes + 4 * gbytes), bws, nullptr),
                   VCT_EINVAL, "vct_bounce", "out and normal overlap");
            EXPECT(vct_bounce(&g, at(0), at(pbytes), at(pbytes + gbytes), at(pbytes + 2 * gbytes), &p, at(pbytes),
                              at(64), bws, nullptr),
                   VCT_EINVAL, "vct_bounce", "workspace and pyramid overlap");
        }
    }

    // diagnostics
    for (int c : {-1, 65, 3})
        EXPECT(vct_record_kernel_events(nullptr, c), VCT_EINVAL, "vct_record_kernel_events", "events");
    EXPECT(vct_record_kernel_events(nullptr, 0), VCT_OK, "vct_record_kernel_events", nullptr);
    return g_checks;
}
