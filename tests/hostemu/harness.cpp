// Checked CPU build: drives the library's C ABI, compiled for the host with
// the emulation of emu.h, on one case directory written by the test:
//   meta.txt   key value lines (grid, G-buffer shape, cone parameters, what to run)
//   base.bin pos_rough.bin normal.bin cam.bin dirs.bin weights.bin gout.bin material.bin
// and writes trace.bin, save.bin, count.bin, grad.bin, shade.bin and the
// decoded levels level_<d>_<l>.bin next to them.  With --abi instead of a
// directory it runs the argument-validation battery of abi_checks.cpp, and
// with --voxelize <dir> the voxelization case of voxelize_case.cpp.
#include <sys/mman.h>

#include <map>
#include <string>
#include <vector>

#include "emu.h"
#include "vct_internal.h"

void emu_register(const void* p, size_t n, const char* name);
void emu_clear_allocations();
void emu_set_limits(uint64_t texels, uint64_t acc);
void emu_shutdown();
int run_abi_checks();
int run_voxelize_case(const char* dir);

namespace {

std::string g_dir;
std::map<std::string, std::string> g_meta;

double num(const char* k, double def = NAN) {
    auto it = g_meta.find(k);
    if (it == g_meta.end()) {
        if (std::isnan(def)) emu_fail("meta.txt lacks %s", k);
        return def;
    }
    return atof(it->second.c_str());
}

std::vector<char> read_file(const char* name, size_t expect) {
    std::string p = g_dir + "/" + name;
    FILE* f = fopen(p.c_str(), "rb");
    if (!f) emu_fail("cannot open %s", p.c_str());
    std::vector<char> v(expect);
    if (expect && fread(v.data(), 1, expect, f) != expect) emu_fail("%s is shorter than %zu bytes", p.c_str(), expect);
    fclose(f);
    return v;
}

void write_file(const char* name, const void* p, size_t n) {
    std::string path = g_dir + "/" + name;
    FILE* f = fopen(path.c_str(), "wb");
    if (!f || fwrite(p, 1, n, f) != n) emu_fail("cannot write %s", path.c_str());
    fclose(f);
}

// Buffer registered with the emulator (the "device" memory of a call).  Up to
// 256 MiB: heap memory (seen by AddressSanitizer), poisoned so that nothing
// can rely on fresh memory being zero.  Larger: anonymous mappings, left
// unpoisoned (the kernels write all of it before reading it; pages never
// written cost nothing to read).
constexpr size_t kBigBuf = size_t(256) << 20;
struct Buf {
    char* p = nullptr;
    size_t n = 0;
    bool mapped = false;
    Buf(size_t bytes, const char* name) : n(bytes) {
        if (bytes > kBigBuf) {
            void* m = mmap(nullptr, bytes, PROT_READ | PROT_WRITE, MAP_PRIVATE | MAP_ANONYMOUS | MAP_NORESERVE, -1, 0);
            if (m == MAP_FAILED) emu_fail("out of host memory (%zu bytes for %s)", bytes, name);
            p = static_cast<char*>(m);
            mapped = true;
        } else {
            p = static_cast<char*>(malloc(bytes ? bytes : 1));
            if (!p) emu_fail("out of host memory (%zu bytes for %s)", bytes, name);
            memset(p, 0xA5, bytes);
        }
        emu_register(p, bytes, name);
    }
    Buf(const Buf&) = delete;
    ~Buf() {
        if (mapped) munmap(p, n);
        else free(p);
    }
    template <typename T>
    T* as() { return reinterpret_cast<T*>(p); }
};

void read_into(const char* name, void* dst, size_t n) {
    std::string p = g_dir + "/" + name;
    FILE* f = fopen(p.c_str(), "rb");
    if (!f) emu_fail("cannot open %s", p.c_str());
    if (n && fread(dst, 1, n, f) != n) emu_fail("%s is shorter than %zu bytes", p.c_str(), n);
    fclose(f);
}

void check(int rc, const char* what) {
    if (rc != VCT_OK) emu_fail("%s returned %d: %s", what, rc, vct_last_error());
}

}  // namespace

int main(int argc, char** argv) {
    if (argc == 3 && strcmp(argv[1], "--voxelize") == 0) {
        run_voxelize_case(argv[2]);
        emu_shutdown();
        printf("EMU OK\n");
        return 0;
    }
    if (argc != 2) {
        fprintf(stderr, "usage: %s <case dir> | --abi | --voxelize <case dir>\n", argv[0]);
        return 2;
    }
    if (strcmp(argv[1], "--abi") == 0) {
        const int n = run_abi_checks();
        printf("abi checks passed: %d\n", n);
        emu_shutdown();
        return 0;
    }
    g_dir = argv[1];
    {
        FILE* f = fopen((g_dir + "/meta.txt").c_str(), "r");
        if (!f) emu_fail("no meta.txt in %s", argv[1]);
        char k[128], v[128];
        while (fscanf(f, "%127s %127s", k, v) == 2) g_meta[k] = v;
        fclose(f);
    }
    vct_grid g{};
    g.n = (int)num("n");
    g.levels = (int)num("levels");
    g.dtype = (int)num("dtype");
    g.origin[0] = (float)num("origin0", 0.0);
    g.origin[1] = (float)num("origin1", 0.0);
    g.origin[2] = (float)num("origin2", 0.0);
    g.extent = (float)num("extent", 1.0);
    g.anisotropic = (int)num("aniso", 0.0);
    const size_t nvox = (size_t)g.n * g.n * g.n;
    const int B = (int)num("b"), H = (int)num("h"), W = (int)num("w");
    const size_t npix = (size_t)B * H * W;

    vct_cone_params p{};
    p.n_diffuse = (int)num("n_diffuse");
    {
        auto dirs = read_file("dirs.bin", sizeof(float) * 3 * p.n_diffuse);
        auto wts = read_file("weights.bin", sizeof(float) * p.n_diffuse);
        memcpy(p.diffuse_dir, dirs.data(), dirs.size());
        memcpy(p.diffuse_weight, wts.data(), wts.size());
    }
    p.diffuse_aperture = (float)num("diffuse_aperture");
    p.enable_spec = (int)num("enable_spec");
    p.enable_occ = (int)num("enable_occ");
    p.spec_aperture_scale = (float)num("spec_aperture_scale");
    p.occ_aperture = (float)num("occ_aperture");
    p.light_pos[0] = (float)num("light0");
    p.light_pos[1] = (float)num("light1");
    p.light_pos[2] = (float)num("light2");
    p.step_factor = (float)num("step_factor");
    p.t0 = (float)num("t0");
    p.normal_offset = (float)num("normal_offset");
    p.max_dist = (float)num("max_dist");
    p.alpha_thresh = (float)num("alpha_thresh");

    // base.bin holds the whole grid, or with block_origin w0 only the corner
    // block [w0, n)^3 of a grid that is zero elsewhere
    Buf base(nvox * 16, "base");
    const int w0 = (int)num("block_origin", 0.0);
    if (w0 == 0) {
        read_into("base.bin", base.p, nvox * 16);
    } else {
        if (base.n <= kBigBuf) memset(base.p, 0, base.n);   // (mapped memory starts zero)
        const size_t m = (size_t)(g.n - w0);
        std::vector<float> blk(m * m * m * 4);
        read_into("base.bin", blk.data(), blk.size() * 4);
        for (size_t z = 0; z < m; ++z)
            for (size_t y = 0; y < m; ++y)
                memcpy(base.p + ((((z + w0) * g.n + (y + w0)) * g.n + w0) * 16), &blk[((z * m + y) * m) * 4], m * 16);
    }
    Buf pos(npix * 16, "pos_rough"), nrm(npix * 16, "normal"), cam((size_t)B * 12, "cam_pos");
    {
        auto a = read_file("pos_rough.bin", npix * 16);
        auto b = read_file("normal.bin", npix * 16);
        auto c = read_file("cam.bin", (size_t)B * 12);
        memcpy(pos.p, a.data(), a.size());
        memcpy(nrm.p, b.data(), b.size());
        memcpy(cam.p, c.data(), c.size());
    }
    vct_gbuffer gb{};
    gb.b = B, gb.h = H, gb.w = W;
    gb.pos_rough = pos.as<float>();
    gb.normal = nrm.as<float>();
    gb.cam_pos = cam.as<float>();

    size_t pyr_bytes = 0;
    check(vct_pyramid_bytes(&g, &pyr_bytes), "vct_pyramid_bytes");
    Buf pyr(pyr_bytes, "pyramid");
    // texel and accumulator indices stay below the layout's texel count
    const PyrLayout lay = vct_make_layout(g.n, g.levels, g.dtype, g.anisotropic);
    emu_set_limits((uint64_t)lay.total_texels, (uint64_t)lay.total_texels);
    check(vct_build_mips(&g, base.as<float>(), pyr.p, pyr.n, nullptr), "vct_build_mips");
    fprintf(stderr, "built mips (%zu bytes)\n", pyr.n);
    for (int d = 0; d < (g.anisotropic ? 6 : 1); ++d)
        for (int l = 0; l < g.levels; ++l) {
            if (!(int)num("dump_levels", 0.0)) break;
            const size_t nl = (size_t)(g.n >> l);
            Buf lv(nl * nl * nl * 16, "level");
            check(vct_unpack_level_dir(&g, pyr.p, l, d, lv.as<float>(), nullptr), "vct_unpack_level_dir");
            char name[64];
            snprintf(name, sizeof name, "level_%d_%d.bin", d, l);
            write_file(name, lv.p, lv.n);
        }

    Buf out(npix * 32, "out");
    check(vct_trace(&g, pyr.p, &gb, &p, out.as<float>(), nullptr), "vct_trace");
    write_file("trace.bin", out.p, out.n);
    fprintf(stderr, "traced %zu pixels\n", npix);
    Buf cnt(16, "counts");
    check(vct_count_sample_levels(&g, pyr.p, &gb, &p, cnt.as<unsigned long long>(), nullptr),
          "vct_count_sample_levels");
    write_file("count.bin", cnt.p, 16);

    if ((int)num("backward", 1.0)) {
        size_t st_bytes = 0, ws_bytes = 0;
        check(vct_lane_state_bytes(&gb, &p, &st_bytes), "vct_lane_state_bytes");
        check(vct_backward_workspace_bytes(&g, &gb, &p, &ws_bytes), "vct_backward_workspace_bytes");
        Buf state(st_bytes, "lane states");
        Buf ws((int)num("save_only", 0.0) ? 0 : ws_bytes - st_bytes, "workspace");
        Buf out2(npix * 32, "out (save)");
        check(vct_trace_save(&g, pyr.p, &gb, &p, out2.as<float>(), state.p, state.n, nullptr), "vct_trace_save");
        write_file("save.bin", out2.p, out2.n);
        if ((int)num("save_only", 0.0)) {
            emu_clear_allocations();
            emu_shutdown();
            printf("EMU OK\n");
            return 0;
        }
        Buf gout(npix * 32, "grad_out"), grad(nvox * 16, "grad_base");
        {
            auto v = read_file("gout.bin", npix * 32);
            memcpy(gout.p, v.data(), v.size());
        }
        check(vct_trace_backward_saved(&g, pyr.p, &gb, &p, state.p, state.n, gout.as<float>(), grad.as<float>(), ws.p,
                                       ws.n, nullptr),
              "vct_trace_backward_saved");
        if (w0 == 0) {
            write_file("grad.bin", grad.p, grad.n);
        } else {
            // the block's gradient, and the count of nonzero values outside it
            const size_t m = (size_t)(g.n - w0);
            std::vector<float> blk(m * m * m * 4);
            unsigned long long outside = 0;
            const float* G = grad.as<float>();
            for (size_t z = 0; z < (size_t)g.n; ++z)
                for (size_t y = 0; y < (size_t)g.n; ++y)
                    for (size_t x = 0; x < (size_t)g.n; ++x) {
                        const float* v = G + ((z * g.n + y) * g.n + x) * 4;
                        if (z >= (size_t)w0 && y >= (size_t)w0 && x >= (size_t)w0)
                            memcpy(&blk[(((z - w0) * m + (y - w0)) * m + (x - w0)) * 4], v, 16);
                        else
                            outside += (v[0] != 0.f) + (v[1] != 0.f) + (v[2] != 0.f) + (v[3] != 0.f);
                    }
            write_file("grad.bin", blk.data(), blk.size() * 4);
            write_file("grad_outside_nonzero.bin", &outside, sizeof outside);
        }
        fprintf(stderr, "backward done\n");
        if ((int)num("noalloc", 0.0)) {
            Buf grad2(nvox * 16, "grad_base (allocation-free)");
            check(vct_trace_backward_saved_noalloc(&g, pyr.p, &gb, &p, state.p, state.n, gout.as<float>(),
                                                   grad2.as<float>(), nullptr),
                  "vct_trace_backward_saved_noalloc");
            write_file("grad_noalloc.bin", grad2.p, grad2.n);
        }
    }
    if ((int)num("shade", 0.0)) {
        vct_shade_params sp{};
        sp.n_lights = (int)num("n_lights");
        auto lights = read_file("lights.bin", sizeof(float) * 9 * sp.n_lights);
        const float* L = reinterpret_cast<const float*>(lights.data());
        for (int l = 0; l < sp.n_lights; ++l)
            for (int i = 0; i < 3; ++i) {
                sp.light_pos[l][i] = L[9 * l + i];
                sp.light_diffuse[l][i] = L[9 * l + 3 + i];
                sp.light_specular[l][i] = L[9 * l + 6 + i];
            }
        for (int i = 0; i < 3; ++i) sp.specular_color[i] = 1.0f;
        sp.diffuse_first_hit = (int)num("diffuse_first_hit");
        sp.first_hit_alpha = (float)num("first_hit_alpha");
        sp.occlusion_falloff = (int)num("occlusion_falloff");
        sp.shadow_strength = (float)num("shadow_strength");
        sp.specular_brdf = (int)num("specular_brdf");
        sp.grace_per_shininess = (float)num("grace_per_shininess");
        sp.shininess_falloff = (float)num("shininess_falloff");
        Buf mat(npix * 16, "material"), sout(npix * 16, "shade out");
        {
            auto v = read_file("material.bin", npix * 16);
            memcpy(mat.p, v.data(), v.size());
        }
        check(vct_shade(&g, pyr.p, &gb, mat.as<float>(), &p, &sp, sout.as<float>(), nullptr), "vct_shade");
        write_file("shade.bin", sout.p, sout.n);
        fprintf(stderr, "shaded\n");
    }
    if ((int)num("bounce", 0.0)) {
        // one further bounce of the base grid through its own pyramid
        Buf nrmg(nvox * 16, "normal grid"), albg(nvox * 16, "albedo grid"), bout(nvox * 16, "bounced");
        read_into("normal_grid.bin", nrmg.p, nrmg.n);
        read_into("albedo_grid.bin", albg.p, albg.n);
        size_t ws_bytes = 0;
        check(vct_bounce_workspace_bytes(&g, &ws_bytes), "vct_bounce_workspace_bytes");
        Buf ws(ws_bytes, "bounce workspace");
        check(vct_bounce(&g, pyr.p, base.as<float>(), nrmg.as<float>(), albg.as<float>(), &p, bout.as<float>(), ws.p,
                         ws.n, nullptr),
              "vct_bounce");
        write_file("bounce.bin", bout.p, bout.n);
        fprintf(stderr, "bounced\n");
    }
    emu_clear_allocations();
    emu_shutdown();
    printf("EMU OK\n");
    return 0;
}
