// Checked CPU build, voxelization: runs vct_voxelize on the case directory
// <dir> written by the test (vmeta.txt: n, n_tris, surface, n_lights, ambient,
// diffuse; tris.bin, colors.bin, lights.bin = [n_lights][9] position, colour,
// attenuation) and writes vox_base.bin, and with surface attributes
// vox_normal.bin and vox_albedo.bin.  The output grids start poisoned and the
// workspace is registered with the emulator like every other buffer.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "emu.h"
#include "vct.h"

void emu_register(const void* p, size_t n, const char* name);
void emu_clear_allocations();

namespace {

std::vector<char> slurp(const std::string& path, size_t n) {
    std::vector<char> v(n ? n : 1);
    FILE* f = fopen(path.c_str(), "rb");
    if (!f) emu_fail("cannot open %s", path.c_str());
    if (n && fread(v.data(), 1, n, f) != n) emu_fail("%s is shorter than %zu bytes", path.c_str(), n);
    fclose(f);
    return v;
}

void spill(const std::string& path, const void* p, size_t n) {
    FILE* f = fopen(path.c_str(), "wb");
    if (!f || fwrite(p, 1, n, f) != n) emu_fail("cannot write %s", path.c_str());
    fclose(f);
}

char* buffer(size_t n, const char* name) {
    char* p = static_cast<char*>(malloc(n ? n : 1));
    if (!p) emu_fail("out of host memory for %s", name);
    memset(p, 0xA5, n);
    emu_register(p, n, name);
    return p;
}

}  // namespace

int run_voxelize_case(const char* dir) {
    const std::string d = dir;
    std::map<std::string, double> m;
    {
        FILE* f = fopen((d + "/vmeta.txt").c_str(), "r");
        if (!f) emu_fail("no vmeta.txt in %s", dir);
        char k[64];
        double v;
        while (fscanf(f, "%63s %lf", k, &v) == 2) m[k] = v;
        fclose(f);
    }
    vct_grid g{};
    g.n = (int)m["n"];
    g.levels = 1;
    g.dtype = VCT_F32;
    g.extent = 1.0f;
    const long long nt = (long long)m["n_tris"];
    const int surface = (int)m["surface"];
    vct_voxelize_params vp{};
    vp.n_lights = (int)m["n_lights"];
    vp.ambient = (float)m["ambient"];
    vp.diffuse = (float)m["diffuse"];
    auto lights = slurp(d + "/lights.bin", sizeof(float) * 9 * vp.n_lights);
    const float* L = reinterpret_cast<const float*>(lights.data());
    for (int l = 0; l < vp.n_lights; ++l)
        for (int i = 0; i < 3; ++i) {
            vp.light_pos[l][i] = L[l * 9 + i];
            vp.light_color[l][i] = L[l * 9 + 3 + i];
            vp.attenuation[l][i] = L[l * 9 + 6 + i];
        }
    const size_t nvox = (size_t)g.n * g.n * g.n;
    char* tris = buffer(sizeof(float) * 9 * nt, "tris");
    char* cols = buffer(sizeof(float) * 3 * nt, "colors");
    {
        auto t = slurp(d + "/tris.bin", sizeof(float) * 9 * nt);
        auto c = slurp(d + "/colors.bin", sizeof(float) * 3 * nt);
        memcpy(tris, t.data(), sizeof(float) * 9 * nt);
        memcpy(cols, c.data(), sizeof(float) * 3 * nt);
    }
    size_t ws_bytes = 0;
    if (vct_voxelize_workspace_bytes(&g, nt, surface, &ws_bytes) != VCT_OK) emu_fail("%s", vct_last_error());
    char* ws = buffer(ws_bytes, "voxelize workspace");
    char* base = buffer(nvox * 16, "base");
    char* nrm = surface ? buffer(nvox * 16, "normal grid") : nullptr;
    char* alb = surface ? buffer(nvox * 16, "albedo grid") : nullptr;
    if (vct_voxelize(&g, reinterpret_cast<float*>(tris), reinterpret_cast<float*>(cols), nt, &vp,
                     reinterpret_cast<float*>(base), reinterpret_cast<float*>(nrm), reinterpret_cast<float*>(alb), ws,
                     ws_bytes, nullptr) != VCT_OK)
        emu_fail("vct_voxelize: %s", vct_last_error());
    spill(d + "/vox_base.bin", base, nvox * 16);
    if (surface) {
        spill(d + "/vox_normal.bin", nrm, nvox * 16);
        spill(d + "/vox_albedo.bin", alb, nvox * 16);
    }
    emu_clear_allocations();
    for (char* p : {tris, cols, ws, base, nrm, alb}) free(p);
    return 0;
}
