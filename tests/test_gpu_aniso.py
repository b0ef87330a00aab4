"""GPU anisotropic (six-direction) mips and the forward trace that samples
them, against the FP64 oracle: every directional level, the trace on random
and Cornell scenes with ragged tiles, float16 storage (path parity on the
decoded pyramid and storage error), sample counts, and sampled pixels of the
256^3 / 1080p launch."""
import numpy as np
import pytest
import torch

import oracle
from oracle import vct_aniso as va
import paper_2104_00618_amd as vct
from scenes import ConeParams, cone_set, random_gbuffer, random_grid
from tests.parity import fmt, range_errors, worst
from tests.workloads import sample_pixels, sub_gbuffer, workload

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
TOL = 1e-5


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def gpu_aniso(base, n, levels=None, dtype="f32"):
    g = vct.Grid(n, levels=levels, dtype=dtype, anisotropic=True)
    return vct.build_mips(dev(base), g), g


def decoded(pyr, g):
    """The GPU pyramid read back: [direction][level] float64."""
    return [[vct.unpack_level_dir(pyr, g, lv, d).cpu().numpy().astype(np.float64) for lv in range(g.levels)]
            for d in range(6)]


def check(gpu, ref, keep, tol, label):
    e = range_errors(gpu, ref, keep)
    print(f"{label}: {fmt(e)}; ambiguous excluded {int((~keep).sum())}", flush=True)
    assert worst(e)[0] <= tol, label


@pytest.mark.parametrize("n,levels", [(2, None), (4, None), (16, None), (64, None), (64, 3)])
def test_aniso_mips_f32_match_oracle(n, levels):
    base = random_grid(n, seed=200 + n, alpha_max=0.8)
    pyr, g = gpu_aniso(base, n, levels)
    ref = va.build_aniso_mips(base, g.levels)
    got = decoded(pyr, g)
    for d in range(6):
        np.testing.assert_array_equal(got[d][0], base)                   # level 0: the input, in every direction
        for lv in range(1, g.levels):
            err = np.abs(got[d][lv] - ref[d][lv]).max() / np.abs(ref[d][lv]).max()
            assert err <= 1e-6, (d, lv, err)
    # the directions differ (an isotropic build would make them equal)
    assert np.abs(got[0][1] - got[1][1]).max() > 1e-3


def test_aniso_mips_f16_within_storage_rounding():
    n = 32
    base = random_grid(n, seed=7, alpha_max=0.8)
    pyr, g = gpu_aniso(base, n, dtype="f16")
    ref = va.build_aniso_mips(base)
    got = decoded(pyr, g)
    for d in range(6):
        for lv in range(g.levels):
            # level l is rounded once per level on its way up: at most l + 1 half-ulps of float16, relative
            err = (np.abs(got[d][lv] - ref[d][lv]) / np.maximum(np.abs(ref[d][lv]), 2.0 ** -14)).max()
            assert err <= (lv + 1) * 2.0 ** -11 + 1e-7, (d, lv, err)


def test_aniso_trace_random_ragged():
    n = 32
    base = random_grid(n, seed=31, alpha_max=0.3)
    pr, nr, cam = random_gbuffer(2, 37, 53, seed=32, n=n)
    d, w = cone_set("six")
    p = ConeParams(d, w, alpha_thresh=0.99, light_pos=(0.3, 0.8, 0.6))
    pyr, g = gpu_aniso(base, n)
    out = vct.trace(pyr, g, dev(pr), dev(nr), dev(cam), p).cpu().numpy()
    ref, info = va.trace_aniso(va.build_aniso_mips(base), pr, nr, cam, p, return_info=True)
    check(out, ref, ~info["ambiguous"].reshape(-1), TOL, "aniso random 32^3 2x37x53")
    # sample counts are those of the oracle's march
    cnt = vct.count_samples(pyr, g, dev(pr), dev(nr), dev(cam), p)
    assert abs(cnt - info["samples"]) <= int(info["ambiguous"].sum()) * 64, (cnt, info["samples"])


def test_aniso_trace_cornell_and_partial_pyramid():
    w = workload("c0")
    n = w.n
    pr, nr, cam = w.pos_rough[:, ::3, ::3].copy(), w.normal[:, ::3, ::3].copy(), w.cam_pos
    for levels in (None, 4):
        pyr, g = gpu_aniso(w.base, n, levels)
        out = vct.trace(pyr, g, dev(pr), dev(nr), dev(cam), w.params).cpu().numpy()
        ref, info = va.trace_aniso(va.build_aniso_mips(w.base, g.levels), pr, nr, cam, w.params, return_info=True)
        check(out, ref, ~info["ambiguous"].reshape(-1), TOL, f"aniso c0 64^3 {pr.shape[1]}x{pr.shape[2]} levels {g.levels}")


def test_aniso_trace_f16_two_tiers():
    n = 32
    base = random_grid(n, seed=41, alpha_max=0.3)
    pr, nr, cam = random_gbuffer(1, 29, 31, seed=42, n=n)
    d, w = cone_set("five")
    p = ConeParams(d, w, alpha_thresh=0.99)
    pyr, g = gpu_aniso(base, n, dtype="f16")
    out = vct.trace(pyr, g, dev(pr), dev(nr), dev(cam), p).cpu().numpy()
    ref_dec, i_dec = va.trace_aniso(decoded(pyr, g), pr, nr, cam, p, return_info=True)
    check(out, ref_dec, ~i_dec["ambiguous"].reshape(-1), TOL, "aniso f16 path parity")
    ref, info = va.trace_aniso(va.build_aniso_mips(base), pr, nr, cam, p, return_info=True)
    check(out, ref, ~(info["ambiguous"] | i_dec["ambiguous"]).reshape(-1), 2e-3, "aniso f16 storage")


def test_aniso_trace_full_launch_sampled_pixels():
    """256^3 / 1920x1080 (the benchmark frame) with an anisotropic pyramid;
    512 seeded pixels recomputed by the oracle."""
    w = workload("c1")
    pyr, g = gpu_aniso(w.base, w.n)
    out = vct.trace(pyr, g, dev(w.pos_rough), dev(w.normal), dev(w.cam_pos), w.params).cpu().numpy()
    am = va.build_aniso_mips(w.base)
    v, y, x = sample_pixels(w.shape, 512, seed=5)
    ref = np.zeros((len(v), 8))
    amb = np.zeros(len(v), dtype=bool)
    for sel, pr, nr, cam in sub_gbuffer(w.pos_rough, w.normal, w.cam_pos, v, y, x):
        o, info = va.trace_aniso(am, pr, nr, cam, w.params, return_info=True)
        ref[sel] = o.reshape(-1, 8)
        amb[sel] = info["ambiguous"].reshape(-1)
    check(out[v, y, x], ref, ~amb, TOL, "aniso c1 256^3 1080p sampled")


def test_aniso_shade_matches_oracle():
    from oracle import vct_shade as vs
    from scenes import random_material, scene_lights
    w = workload("c0")
    pr, nr, cam = w.pos_rough[:, ::4, ::4].copy(), w.normal[:, ::4, ::4].copy(), w.cam_pos
    mat = random_material(pr.shape[:3], seed=9)
    for sp in (scene_lights(2), scene_lights(1, diffuse_first_hit=False, occlusion_falloff=False,
                                              specular_brdf=False)):
        pyr, g = gpu_aniso(w.base, w.n)
        out = vct.shade(pyr, g, dev(pr), dev(nr), dev(cam), dev(mat), w.params, sp).cpu().numpy()
        am = va.build_aniso_mips(w.base)
        ref, info = vs.shade(am[0], pr, nr, mat, cam, w.params, sp, return_info=True, sampler=va.aniso_sampler(am))
        check(out, ref, ~info["ambiguous"].reshape(-1), 5e-5, f"aniso shade c0 {pr.shape[1]}x{pr.shape[2]} "
              f"{sp.n_lights} lights first_hit={sp.diffuse_first_hit}")


def test_aniso_bounce_matches_oracle():
    from oracle import vct_bounce as vb
    from oracle import vct_voxelize as vx
    from scenes.mesh import cornell_mesh
    n = 32
    tris, cols = cornell_mesh(3)
    lights = [((0.5, 0.95, 0.5), (1.0, 1.0, 1.0), (1.0, 0.5, 0.25))]
    base, nrm, alb = (a.astype(np.float32) for a in vx.voxelize(tris, cols, n, lights, return_surface=True))
    d, w = cone_set("six")
    p = ConeParams(d, w, alpha_thresh=0.99)
    pyr, g = gpu_aniso(base, n)
    got = vct.bounce(pyr, g, dev(base), dev(nrm), dev(alb), p).cpu().numpy()
    am = va.build_aniso_mips(base)
    ref, info = vb.bounce(base, nrm, alb, p, mips=am[0], sampler=va.aniso_sampler(am), return_info=True)
    near = np.abs(np.linalg.norm(nrm[..., 0:3].astype(np.float64), axis=-1) - vb.MIN_NORMAL) < 1e-6
    keep = ~(info["ambiguous"] | near)
    inc_g = (got[..., 0:3] - base[..., 0:3]).reshape(-1, 3)
    inc_r = (ref[..., 0:3] - base[..., 0:3]).reshape(-1, 3)
    check(inc_g, inc_r, keep.reshape(-1), TOL, "aniso bounce 32^3 (added light)")
    same = (ref[..., 0:3] == base[..., 0:3]).all(-1) & keep
    assert np.array_equal(got[same].view(np.uint32), base[same].view(np.uint32))


def _aniso_grads(base, n, pr, nr, cam, p, gout, dtype="f32", repeats=6):
    pyr, g = gpu_aniso(base, n, dtype=dtype)
    t = [dev(x) for x in (pr, nr, cam)]
    go = dev(gout.astype(np.float32))
    rec = vct.trace_backward(pyr, g, *t, p, go).cpu().numpy()
    out, state = vct.trace_save(pyr, g, *t, p)
    sav = vct.trace_backward_saved(pyr, g, *t, p, state, go).cpu().numpy()
    # repeated calls: lanes of pixels with no surface hold no cone, and a
    # non-finite weight of one of them once poisoned a group's sum now and then
    again = [vct.trace_backward_saved(pyr, g, *t, p, state, go).cpu().numpy() for _ in range(repeats)]
    return rec, sav, again, out.cpu().numpy(), pyr, g


def _check_grad(got, ref, label, tmax=1e-4, trms=1e-5):
    scale = np.abs(ref).max()
    err = np.abs(got - ref).max() / scale
    rms = np.sqrt(np.mean((got - ref) ** 2)) / scale
    print(f"{label}: gradient max {err:.2e} rms {rms:.2e}", flush=True)
    assert err <= tmax and rms <= trms, label


@pytest.mark.parametrize("case", ["random", "cornell"])
def test_aniso_backward_matches_oracle(case):
    if case == "random":
        n = 16
        base = random_grid(n, seed=61, alpha_max=0.35)
        pr, nr, cam = random_gbuffer(2, 17, 19, seed=62, n=n)
        d, w = cone_set("six")
        p = ConeParams(d, w, alpha_thresh=0.99, light_pos=(0.4, 0.8, 0.6))
    else:
        wk = workload("c3fd")
        n, base, pr, nr, cam, p = wk.n, wk.base, wk.pos_rough, wk.normal, wk.cam_pos, wk.params
    am = va.build_aniso_mips(base)
    fwd, info = va.trace_aniso(am, pr, nr, cam, p, return_info=True)
    gout = np.random.default_rng(63).normal(size=fwd.shape)
    gout[info["ambiguous"]] = 0.0
    rec, sav, again, out, _, _ = _aniso_grads(base, n, pr, nr, cam, p, gout)
    check(out, fwd, ~info["ambiguous"].reshape(-1), TOL, f"aniso trace_save {case}")
    assert np.array_equal(rec.view(np.uint32), sav.view(np.uint32)), "saved path differs from the recompute path"
    for r in again:
        assert np.array_equal(sav.view(np.uint32), r.view(np.uint32)), "not reproducible"
    ref = va.trace_backward_aniso(am, pr, nr, cam, p, gout)
    _check_grad(sav, ref, f"aniso backward {case} {n}^3")


@pytest.mark.parametrize("dtype", ["f16", "bf16"])
def test_aniso_backward_f16_uses_stored_values(dtype):
    n = 16
    base = random_grid(n, seed=64, alpha_max=0.35)
    pr, nr, cam = random_gbuffer(1, 19, 21, seed=65, n=n)
    d, w = cone_set("five")
    p = ConeParams(d, w, alpha_thresh=0.99)
    gout = np.random.default_rng(66).normal(size=pr.shape[:3] + (8,))
    rec, sav, again, out, pyr, g = _aniso_grads(base, n, pr, nr, cam, p, gout, dtype=dtype)
    dec = decoded(pyr, g)
    _, info = va.trace_aniso(dec, pr, nr, cam, p, return_info=True)
    gout[info["ambiguous"]] = 0.0
    rec, sav, again, out, pyr, g = _aniso_grads(base, n, pr, nr, cam, p, gout, dtype=dtype)
    assert np.array_equal(rec.view(np.uint32), sav.view(np.uint32))
    for r in again:
        assert np.array_equal(sav.view(np.uint32), r.view(np.uint32)), "not reproducible"
    ref = va.trace_backward_aniso(dec, pr, nr, cam, p, gout)
    _check_grad(sav, ref, f"aniso backward {dtype} (oracle on the stored values)")


@pytest.mark.parametrize("n,levels", [(2, None), (4, None), (8, 2)])
def test_aniso_backward_tiny_and_partial_pyramids(n, levels):
    """Directional pyramids of a few texels (all levels in the workgroup LDS
    table) and a two-level pyramid (level 1 is the top)."""
    rng = np.random.default_rng(300 + n)
    a = rng.uniform(0, 0.3, size=(n, n, n, 1))
    base = np.concatenate([rng.uniform(0, 1, size=(n, n, n, 3)) * a, a], -1).astype(np.float32)
    pr, nr, cam = random_gbuffer(1, 9, 11, seed=400 + n, n=max(n, 8))   # (points inside the cube)
    d, w = cone_set("six")
    p = ConeParams(d, w, alpha_thresh=0.99)
    am = va.build_aniso_mips(base, levels)
    fwd, info = va.trace_aniso(am, pr, nr, cam, p, return_info=True)
    gout = rng.normal(size=fwd.shape)
    gout[info["ambiguous"]] = 0.0
    ref = va.trace_backward_aniso(am, pr, nr, cam, p, gout)
    pyr, g = gpu_aniso(base, n, levels=levels)
    t = [dev(x) for x in (pr, nr, cam)]
    go = dev(gout.astype(np.float32))
    rec = vct.trace_backward(pyr, g, *t, p, go).cpu().numpy()
    _, state = vct.trace_save(pyr, g, *t, p)
    sav = vct.trace_backward_saved(pyr, g, *t, p, state, go).cpu().numpy()
    assert np.array_equal(rec.view(np.uint32), sav.view(np.uint32))
    _check_grad(sav, ref, f"aniso backward tiny {n}^3 levels {levels}")


def test_aniso_training_step_full_launch_sparse_grad_out():
    """The training step the benchmark times, through an anisotropic pyramid:
    the 1920x1080 frame at 256^3 (trace_save + trace_backward_saved), with
    dL/d(out) nonzero on 64 seeded surface pixels only, so that the oracle can
    form the whole gradient from those pixels."""
    w = workload("c1")
    b, h, wd = w.shape
    rng = np.random.default_rng(91)
    surf = np.argwhere(w.normal[..., 3] != 0)
    pick = surf[rng.choice(len(surf), size=64, replace=False)]
    vv, yy, xx = pick[:, 0], pick[:, 1], pick[:, 2]
    am = va.build_aniso_mips(w.base)
    pr = w.pos_rough[vv, yy, xx][None, None]
    nr = w.normal[vv, yy, xx][None, None]
    fwd, info = va.trace_aniso(am, pr, nr, w.cam_pos[:1], w.params, return_info=True)
    go = rng.normal(size=fwd.shape)
    go[info["ambiguous"]] = 0.0              # (termination ties: no gradient through them)
    ref = va.trace_backward_aniso(am, pr, nr, w.cam_pos[:1], w.params, go)
    gout = np.zeros((b, h, wd, 8), np.float32)
    gout[vv, yy, xx] = go[0, 0]
    pyr, g = gpu_aniso(w.base, w.n)
    t = [dev(x) for x in (w.pos_rough, w.normal, w.cam_pos)]
    out, state = vct.trace_save(pyr, g, *t, w.params)
    got = vct.trace_backward_saved(pyr, g, *t, w.params, state, dev(gout)).cpu().numpy()
    check(out.cpu().numpy()[vv, yy, xx].reshape(1, 1, -1, 8), fwd, ~info["ambiguous"].reshape(-1), TOL,
          "aniso trace_save c1 1080p sampled")
    _check_grad(got, ref, "aniso training step c1 256^3 1920x1080, 64 pixels of gradient")
