"""GPU final shading (vct_shade: the thesis's cone variants and shading
equation) against the FP64 shading oracle.  Tolerance: per output channel,
max |gpu - oracle| / max |oracle| <= 5e-5 over non-ambiguous pixels (the
cone outputs carry the forward's 1e-5; the Phong power rdw^shininess turns the
~2e-7 float32 error of a unit-vector dot product into shininess x 2e-7 <= 1.3e-5
for shininess <= 64)."""
import numpy as np
import pytest
import torch

import oracle
import paper_2104_00618_amd as vct
from scenes import ConeParams, cone_set, random_gbuffer, random_grid, random_material, scene_lights
from tests.parity import fmt, range_errors, worst
from tests.workloads import sample_pixels, sub_gbuffer, workload

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
TOL = 5e-5


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def gpu_shade(base, n, pr, nr, cam, mat, params, sp, dtype="f32"):
    g = vct.Grid(n, dtype=dtype)
    pyr = vct.build_mips(dev(base), g)
    out = vct.shade(pyr, g, dev(pr), dev(nr), dev(cam), dev(mat), params, sp)
    torch.cuda.synchronize()
    return out.cpu().numpy(), pyr, g


def check(got, ref, amb, label):
    keep = ~np.asarray(amb).reshape(-1)
    e = range_errors(got, ref, keep)
    print(f"{label}: {fmt(e)} (ambiguous {int((~keep).sum())})", flush=True)
    assert worst(e)[0] <= TOL, (label, worst(e))


@pytest.mark.parametrize("flags", [{}, dict(diffuse_first_hit=False, occlusion_falloff=False, specular_brdf=False)],
                         ids=["variants", "unmodified"])
def test_shade_c0_full_frame(flags):
    w = workload("c0")
    mat = random_material(w.shape, seed=7)
    sp = scene_lights(2, **flags)
    got, _, _ = gpu_shade(w.base, w.n, w.pos_rough, w.normal, w.cam_pos, mat, w.params, sp)
    ref, info = oracle.shade(oracle.build_mips(w.base), w.pos_rough, w.normal, mat, w.cam_pos, w.params, sp,
                             return_info=True)
    check(got, ref, info["ambiguous"], f"shade c0 {flags or 'variants'}")
    assert np.all(got[w.normal[..., 3] == 0] == 0)


def test_shade_random_ragged_lights_and_no_light():
    n = 32
    base = random_grid(n, seed=31, alpha_max=0.3)
    pr, nr, cam = random_gbuffer(2, 37, 53, seed=32, n=n)
    mat = random_material(pr.shape[:3], seed=33)
    d, wt = cone_set("five")
    p = ConeParams(d, wt, alpha_thresh=0.95)
    mips = oracle.build_mips(base)
    for count, kw in ((3, dict(shadow_strength=2.0, shininess_falloff=4.0)), (0, {})):
        sp = scene_lights(count, **kw)
        got, _, _ = gpu_shade(base, n, pr, nr, cam, mat, p, sp)
        ref, info = oracle.shade(mips, pr, nr, mat, cam, p, sp, return_info=True)
        check(got, ref, info["ambiguous"], f"shade random 32^3 2x37x53, {count} lights")
    assert np.all(got[..., 3][nr[..., 3] != 0] == 1.0)


def test_shade_c1_full_launch_sampled_pixels():
    """Full 1920x1080 launch at 256^3 with 3 lights; 384 seeded pixels
    recomputed by the oracle."""
    w = workload("c1")
    mat = random_material(w.shape, seed=11)
    sp = scene_lights(3)
    got, _, _ = gpu_shade(w.base, w.n, w.pos_rough, w.normal, w.cam_pos, mat, w.params, sp)
    mips = oracle.build_mips(w.base)
    v, y, x = sample_pixels(w.shape, 384, seed=12)
    ref = np.zeros((len(v), 4))
    amb = np.zeros(len(v), dtype=bool)
    for sel, pr, nr, cam in sub_gbuffer(w.pos_rough, w.normal, w.cam_pos, v, y, x):
        m = mat[v[sel], y[sel], x[sel]][None, None]
        o, info = oracle.shade(mips, pr, nr, m, cam, w.params, sp, return_info=True)
        ref[sel] = o.reshape(-1, 4)
        amb[sel] = info["ambiguous"].reshape(-1)
    check(got[v, y, x], ref, amb, "shade c1 256^3 1080p sampled")


@pytest.mark.parametrize("dtype", ["f16", "bf16"])
def test_shade_f16_pyramid_uses_the_stored_values(dtype):
    w = workload("c0")
    mat = random_material(w.shape, seed=9)
    sp = scene_lights(2)
    got, pyr, g = gpu_shade(w.base, w.n, w.pos_rough, w.normal, w.cam_pos, mat, w.params, sp, dtype=dtype)
    decoded = [vct.unpack_level(pyr, g, l).cpu().numpy().astype(np.float64) for l in range(g.levels)]
    ref, info = oracle.shade(decoded, w.pos_rough, w.normal, mat, w.cam_pos, w.params, sp, return_info=True)
    check(got, ref, info["ambiguous"], f"shade c0 {dtype} pyramid")


def test_shade_empty_gbuffer():
    g = vct.Grid(16)
    pyr = vct.build_mips(torch.zeros((16, 16, 16, 4), device=DEV), g)
    z = torch.zeros((1, 0, 5, 4), device=DEV)
    out = vct.shade(pyr, g, z, z, torch.zeros((1, 3), device=DEV), z, workload("c0").params, scene_lights(1))
    assert out.shape == (1, 0, 5, 4)


@pytest.mark.parametrize("flags", [{}, dict(diffuse_first_hit=False, occlusion_falloff=False, specular_brdf=False)],
                         ids=["variants", "unmodified"])
def test_shade_sample_count_matches_oracle(flags):
    """vct_count_shade_samples counts the samples of every shading march
    exactly: pixels where the oracle sees a tie (termination, first hit) are
    dropped from the G-buffer on both sides, and the counts must then agree to
    the sample.  alpha_thresh 0.99, since with 1 a float32 alpha reaches 1.0
    one step before the float64 one."""
    w = workload("c0")
    p = w.params.replace(alpha_thresh=0.99)
    mat = random_material(w.shape, seed=8)
    sp = scene_lights(2, **flags)
    mips = oracle.build_mips(w.base)
    _, info = oracle.shade(mips, w.pos_rough, w.normal, mat, w.cam_pos, p, sp, return_info=True)
    nr = w.normal.copy()
    nr[info["ambiguous"], 3] = 0.0
    _, ref = oracle.shade(mips, w.pos_rough, nr, mat, w.cam_pos, p, sp, return_info=True)
    assert not ref["ambiguous"].any() and ref["samples"] > 0
    g = vct.Grid(w.n)
    pyr = vct.build_mips(dev(w.base), g)
    cnt = vct.count_shade_samples(pyr, g, dev(w.pos_rough), dev(nr), dev(w.cam_pos), dev(mat), p, sp)
    print(f"shade samples {flags or 'variants'}: gpu {cnt}, oracle {ref['samples']} "
          f"({int(info['ambiguous'].sum())} tie pixels dropped)", flush=True)
    assert cnt == ref["samples"]
    e = torch.zeros((1, 0, 3, 4), device=DEV)
    assert vct.count_shade_samples(pyr, g, e, e.clone(), dev(w.cam_pos), e.clone(), p, sp) == 0
