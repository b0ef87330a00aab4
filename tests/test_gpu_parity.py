"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs.  Tolerance for float32 storage: per output channel,
max |gpu - oracle| / max |oracle| <= 1e-5 over pixels without a termination
tie (the oracle flags ties; they are counted, not compared)."""
import math

import numpy as np
import pytest
import torch

import oracle
import paper_2104_00618_amd as vct
from scenes import ConeParams, cone_set, random_gbuffer, random_grid
from tests.parity import fmt, range_errors, worst
from tests.workloads import oracle_at, sample_pixels, workload

pytestmark = pytest.mark.gpu

TOL = 1e-5
DEV = "cuda:0"


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def gpu_render(base, n, pr, nr, cam, params, dtype="f32", levels=None):
    g = vct.Grid(n, levels=levels, dtype=dtype)
    pyr = vct.build_mips(dev(base), g)
    out = vct.trace(pyr, g, dev(pr), dev(nr), dev(cam), params)
    torch.cuda.synchronize()
    return out.cpu().numpy(), pyr, g


def assert_parity(gpu, ref, keep, tol=TOL, label=""):
    errs = range_errors(gpu, ref, keep)
    mx, rms = worst(errs)
    print(f"{label}: {fmt(errs)}; ambiguous excluded {int((~keep).sum())}", flush=True)
    assert mx <= tol, f"{label}: worst range-normalised error {mx:.3e} > {tol:.0e}"


# ------------------------------------------------------------------ mips
@pytest.mark.parametrize("n,levels", [(1, None), (2, None), (4, None), (16, None), (64, None), (64, 3), (128, None)])
def test_mips_f32_match_oracle(n, levels):
    base = random_grid(n, seed=100 + n)
    g = vct.Grid(n, levels=levels)
    pyr = vct.build_mips(dev(base), g)
    ref = oracle.build_mips(base, g.levels)
    for l in range(g.levels):
        got = vct.unpack_level(pyr, g, l).cpu().numpy()
        np.testing.assert_allclose(got, ref[l], rtol=0, atol=2e-7, err_msg=f"level {l}")
    if n == 64 and levels is None:
        # level 0 is the input, bit for bit
        np.testing.assert_array_equal(vct.unpack_level(pyr, g, 0).cpu().numpy(), base)


def _round_to(x, dtype):
    t = torch.from_numpy(np.asarray(x, dtype=np.float32))
    return t.to(torch.float16 if dtype == "f16" else torch.bfloat16).to(torch.float32).numpy()


def _ulp(x, dtype):
    x = np.abs(np.asarray(x, dtype=np.float64))
    mant = 10 if dtype == "f16" else 7
    e = np.floor(np.log2(np.maximum(x, 2.0 ** -14)))
    return 2.0 ** (e - mant)


@pytest.mark.parametrize("dtype", ["f16", "bf16"])
def test_mips_reduced_precision_within_one_ulp(dtype):
    n = 64
    base = random_grid(n, seed=7)
    g = vct.Grid(n, dtype=dtype)
    pyr = vct.build_mips(dev(base), g)
    ref = oracle.build_mips(base)
    for l in range(g.levels):
        got = vct.unpack_level(pyr, g, l).cpu().numpy().astype(np.float64)
        exp = _round_to(ref[l], dtype).astype(np.float64)
        diff = np.abs(got - exp)
        assert np.all(diff <= _ulp(ref[l], dtype) * 1.0001), f"level {l}: {diff.max()}"
        if l == 0:
            np.testing.assert_array_equal(got, exp)       # the input, rounded once


# --------------------------------------------------------------- forward
def test_forward_c0_full_frame():
    w = workload("c0")
    out, _, _ = gpu_render(w.base, w.n, w.pos_rough, w.normal, w.cam_pos, w.params)
    ref, info = oracle.render(w.base, w.pos_rough, w.normal, w.cam_pos, w.params, return_info=True)
    keep = ~info["ambiguous"].reshape(-1)
    assert keep.mean() > 0.99
    assert_parity(out, ref, keep, label="c0 64^3 256x256")
    bg = w.normal[..., 3] == 0
    assert np.all(out[bg] == 0.0)


def test_forward_random_cones_ragged_tiles():
    """Random origins and normals over several 16x16 tiles with a ragged
    tail (37 x 53), two views, spec and occlusion on, alpha_thresh 0.99."""
    n = 32
    base = random_grid(n, seed=21, alpha_max=0.3)
    pr, nr, cam = random_gbuffer(2, 37, 53, seed=22, n=n)
    d, wt = cone_set("six")
    p = ConeParams(d, wt, alpha_thresh=0.99, light_pos=(0.3, 0.8, 0.6))
    out, _, _ = gpu_render(base, n, pr, nr, cam, p)
    ref, info = oracle.render(base, pr, nr, cam, p, return_info=True)
    keep = ~info["ambiguous"].reshape(-1)
    assert_parity(out, ref, keep, label="random 32^3 2x37x53")


def test_forward_c1_full_launch_sampled_pixels():
    """Full 1920x1080 launch at 256^3 (the benchmark configuration); 1536
    seeded pixels recomputed by the oracle one by one."""
    w = workload("c1")
    out, _, _ = gpu_render(w.base, w.n, w.pos_rough, w.normal, w.cam_pos, w.params)
    mips = oracle.build_mips(w.base)
    v, y, x = sample_pixels(w.shape, 1536, seed=1)
    ref, amb = oracle_at(mips, w, v, y, x)
    assert_parity(out[v, y, x], ref, ~amb, label="c1 256^3 1080p sampled")


def test_forward_partial_pyramid_and_tiny_grids():
    d, wt = cone_set("five")
    p = ConeParams(d, wt, alpha_thresh=0.99)
    for n, levels in ((1, 1), (2, 2), (8, 2), (16, 5)):
        base = random_grid(n, seed=n)
        pr, nr, cam = random_gbuffer(1, 9, 11, seed=n, n=max(n, 4))
        out, _, _ = gpu_render(base, n, pr, nr, cam, p, levels=levels)
        mips = oracle.build_mips(base, levels)
        ref, info = oracle.trace(mips, pr, nr, cam, p, return_info=True)
        assert_parity(out, ref, ~info["ambiguous"].reshape(-1), label=f"n={n} levels={levels}")


def test_p1_empty_grid_is_exactly_zero():
    w = workload("c0")
    out, _, _ = gpu_render(np.zeros_like(w.base), w.n, w.pos_rough, w.normal, w.cam_pos, w.params)
    assert np.all(out == 0.0)


def test_p2_uniform_grid_closed_form():
    n, a, L = 256, 0.1, 0.7
    base = np.zeros((n, n, n, 4), np.float32)
    base[...] = np.array([L * a, L * a, L * a, a], np.float32)
    p = ConeParams(np.array([[0, 0, 1.0]], np.float32), np.ones(1, np.float32), enable_spec=False,
                   enable_occ=False, alpha_thresh=1.0)
    pr, nr, cam = random_gbuffer(1, 16, 16, seed=3, n=n, invalid_frac=0.0)
    out, _, _ = gpu_render(base, n, pr, nr, cam, p)
    # 14 samples at N=256, 60 deg, beta 0.5, t0 0.001, t_max 1 (closed form)
    expect_a = 1 - (1 - np.float64(np.float32(a))) ** 14
    np.testing.assert_allclose(out[..., 3], expect_a, rtol=0, atol=2e-6)
    np.testing.assert_allclose(out[..., 0], np.float32(L * a) / np.float32(a) * expect_a, rtol=0, atol=2e-6)


def test_p3_zero_aperture_matches_oracle():
    n = 64
    base = random_grid(n, seed=31)
    p = ConeParams(np.array([[0, 0, 1.0]], np.float32), np.ones(1, np.float32), diffuse_aperture=0.0,
                   enable_spec=False, enable_occ=False, alpha_thresh=1.0, max_dist=0.4)
    pr, nr, cam = random_gbuffer(1, 16, 16, seed=32, n=n, invalid_frac=0.0)
    out, _, _ = gpu_render(base, n, pr, nr, cam, p)
    ref, info = oracle.render(base, pr, nr, cam, p, return_info=True)
    assert_parity(out, ref, ~info["ambiguous"].reshape(-1), label="zero aperture 64^3")


def test_count_samples_matches_oracle():
    w = workload("c0")
    g = vct.Grid(w.n)
    pyr = vct.build_mips(dev(w.base), g)
    cnt = vct.count_samples(pyr, g, dev(w.pos_rough), dev(w.normal), dev(w.cam_pos), w.params)
    mips = oracle.build_mips(w.base)
    lanes = oracle.cone_lanes(w.pos_rough, w.normal, w.cam_pos, w.params, w.n)
    res = oracle.march(mips, lanes, w.params)
    # Lanes with a termination tie, and (alpha_thresh = 1) lanes whose alpha gets
    # within float32 resolution of 1, may stop at a different step: float32 alpha
    # rounds to exactly 1.0 while the FP64 one is still 1 - 1e-9 (the extra
    # samples carry weight T < 1e-6).  Every other lane must agree exactly.
    loose = res["ambiguous"] | (res["alpha"] > 1 - 1e-6)
    strict = int(res["K"][~loose].sum())
    assert strict > 0.9 * res["K"].sum()
    assert cnt <= int(res["K"].sum()) + 2 * int(loose.sum())
    assert cnt >= strict
    print(f"count {cnt}, oracle {int(res['K'].sum())}, lanes near alpha 1: {int(loose.sum())}", flush=True)


def test_count_sample_levels_matches_oracle():
    """The samples of the march split by the levels they read: every sample
    counted once, and those with a fractional LOD (two levels blended) counted
    again, lane by lane as the oracle's march records them."""
    w = workload("c0")
    g = vct.Grid(w.n)
    pyr = vct.build_mips(dev(w.base), g)
    args = (pyr, g, dev(w.pos_rough), dev(w.normal), dev(w.cam_pos), w.params)
    n, n2 = vct.count_sample_levels(*args)
    assert n == vct.count_samples(*args)
    mips = oracle.build_mips(w.base)
    lanes = oracle.cone_lanes(w.pos_rough, w.normal, w.cam_pos, w.params, w.n)
    res = oracle.march(mips, lanes, w.params, record=True)
    two = np.zeros(len(res["K"]), dtype=np.int64)
    near = np.zeros(len(res["K"]), dtype=np.int64)
    for idx, _, _, lam, _, _ in res["steps"]:
        frac = lam - np.floor(lam)
        np.add.at(two, idx, (frac > 0).astype(np.int64))
        # a float32 LOD within rounding of an integer may land on either side
        np.add.at(near, idx, ((frac > 0) & (np.minimum(frac, 1 - frac) < 1e-5)).astype(np.int64))
    loose = res["ambiguous"] | (res["alpha"] > 1 - 1e-6) | (near > 0)
    strict2 = int(two[~loose].sum())
    print(f"two-level samples {n2} of {n}; oracle {int(two.sum())} ({strict2} on strict lanes, "
          f"{int(loose.sum())} loose lanes)", flush=True)
    assert 0 < n2 < n
    assert strict2 > 0.9 * two.sum()
    assert strict2 <= n2 <= int(two.sum()) + 2 * int(loose.sum()) + int(near.sum())


def test_empty_gbuffer_and_all_background():
    w = workload("c0")
    g = vct.Grid(w.n)
    pyr = vct.build_mips(dev(w.base), g)
    e = torch.zeros((1, 0, 5, 4), device=DEV)
    out = vct.trace(pyr, g, e, e.clone(), torch.zeros((1, 3), device=DEV), w.params)
    assert out.shape == (1, 0, 5, 8)
    assert vct.count_samples(pyr, g, e, e.clone(), torch.zeros((1, 3), device=DEV), w.params) == 0
    nr = w.normal.copy()
    nr[..., 3] = 0
    out = vct.trace(pyr, g, dev(w.pos_rough), dev(nr), dev(w.cam_pos), w.params)
    torch.cuda.synchronize()
    assert torch.all(out == 0)


# ------------------------------------------------------ reduced precision
@pytest.mark.parametrize("dtype,storage_tol", [("f16", 2e-3), ("bf16", 1.5e-2)])
def test_reduced_precision_two_tiers(dtype, storage_tol):
    """Tier 1 (path parity): GPU vs oracle run on the GPU's own decoded
    pyramid, 1e-5.  Tier 2 (storage error): GPU vs the FP64 oracle on the
    float32 grid: <= 2e-3 for float16; bfloat16 is reported (8-bit mantissa)."""
    w = workload("c1")
    out, pyr, g = gpu_render(w.base, w.n, w.pos_rough, w.normal, w.cam_pos, w.params, dtype=dtype)
    decoded = [vct.unpack_level(pyr, g, l).cpu().numpy().astype(np.float64) for l in range(g.levels)]
    v, y, x = sample_pixels(w.shape, 768, seed=2)
    ref_dec, amb_dec = oracle_at(decoded, w, v, y, x)
    assert_parity(out[v, y, x], ref_dec, ~amb_dec, label=f"{dtype} path parity")
    ref, amb = oracle_at(oracle.build_mips(w.base), w, v, y, x)
    keep = ~(amb | amb_dec)
    errs = range_errors(out[v, y, x], ref, keep)
    print(f"{dtype} storage error: {fmt(errs)}", flush=True)
    assert worst(errs)[0] <= storage_tol
