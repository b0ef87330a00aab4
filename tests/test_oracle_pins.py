"""Pins of the FP64 oracle against facts the paper and the mathematics fix
(closed forms, invariants, a library interpolator, brute force), not against
the oracle itself.  CPU only."""
import json
import math
import os

import numpy as np
import pytest
from scipy import ndimage

import oracle
from scenes import ConeParams, make_workload, random_grid, random_gbuffer
from scenes.configs import cone_set

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def single_cone_params(gamma, beta=0.5, t0=0.001, t_max=1.0, thresh=1.0, offset=1.0):
    """One front diffuse cone, no specular or occlusion cone."""
    return ConeParams(np.array([[0.0, 0.0, 1.0]], dtype=np.float32), np.ones(1, np.float32),
                      diffuse_aperture=gamma, enable_spec=False, enable_occ=False,
                      step_factor=beta, t0=t0, max_dist=t_max, alpha_thresh=thresh,
                      normal_offset=offset)


def one_pixel(x, nrm, rough=0.5, cam=(0.5, 0.5, 2.0)):
    pr = np.array([[[[x[0], x[1], x[2], rough]]]], dtype=np.float32)
    nr = np.array([[[[nrm[0], nrm[1], nrm[2], 1.0]]]], dtype=np.float32)
    return pr, nr, np.array([cam], dtype=np.float32)


def uniform_mips(n, value):
    levels = int(round(math.log2(n))) + 1
    return [np.broadcast_to(np.asarray(value, np.float64), (n >> l,) * 3 + (4,)) for l in range(levels)]


def closed_form_count(n, gamma, beta, t0, t_max):
    """Number of schedule points with t_k <= t_max, from the closed form of the
    schedule: linear steps of beta*v0 until 2 t tan(gamma/2) >= v0, geometric
    growth by (1 + 2 beta tan(gamma/2)) after."""
    v0 = 1.0 / n
    tan = math.tan(gamma / 2)
    if t_max < t0:
        return 0
    t_star = v0 / (2 * tan) if tan > 0 else math.inf
    k1 = max(0, math.ceil((t_star - t0) / (beta * v0))) if math.isfinite(t_star) else 10 ** 9
    t_k1 = t0 + k1 * beta * v0
    if t_max < t_k1:
        return math.floor((t_max - t0) / (beta * v0)) + 1
    r = 1 + 2 * beta * tan
    return k1 + math.floor(math.log(t_max / t_k1) / math.log(r)) + 1


# ---------------------------------------------------------------- P1 empty grid
def test_p1_empty_grid_gives_zero():
    w = make_workload("c0", h=24, w=24, n=32)
    out = oracle.render(np.zeros_like(w.base), w.pos_rough, w.normal, w.cam_pos, w.params)
    assert np.all(out == 0.0)


# ------------------------------------------------------- P2 uniform closed form
def _golden_cases():
    with open(os.path.join(GOLDEN, "uniform_grid_closed_form.json")) as f:
        return json.load(f)["cases"]


@pytest.mark.parametrize("case", _golden_cases())
def test_p2_uniform_grid_matches_closed_form(case):
    n, a, L = case["n_grid"], case["a"], case["L"]
    gamma = math.radians(case["gamma_deg"])
    p = single_cone_params(gamma, case["beta"], case["t0"], case["t_max"], case["alpha_thresh"])
    mips = uniform_mips(n, [L * a, L * a, L * a, a])
    pr, nr, cam = one_pixel((0.41, 0.37, 0.29), (0.3, 0.5, 0.81))
    out, info = oracle.trace(mips, pr, nr, cam, p, return_info=True)
    n_cf = closed_form_count(n, gamma, case["beta"], case["t0"], case["t_max"])
    n_cf = min(n_cf, math.ceil(math.log(1 - case["alpha_thresh"]) / math.log(1 - a))
               if case["alpha_thresh"] < 1 else n_cf)
    assert n_cf == case["n_samples"]
    assert int(info["K"][0]) == case["n_samples"]
    assert out[0, 0, 0, 3] == pytest.approx(case["alpha"], abs=1e-12)
    assert np.allclose(out[0, 0, 0, 0:3], L * case["alpha"], atol=1e-12)


@pytest.mark.parametrize("gamma_deg,t_max,n", [(60, 0.3, 128), (20, 0.9, 64), (5, 0.5, 32), (0, 0.2, 32)])
def test_p2_schedule_counts(gamma_deg, t_max, n):
    gamma = math.radians(gamma_deg)
    p = single_cone_params(gamma, 0.5, 0.001, t_max, 1.0)
    mips = uniform_mips(n, [0.0, 0.0, 0.0, 0.01])
    pr, nr, cam = one_pixel((0.5, 0.5, 0.5), (0.0, 1.0, 0.0))
    _, info = oracle.trace(mips, pr, nr, cam, p, return_info=True)
    assert int(info["K"][0]) == closed_form_count(n, gamma, 0.5, 0.001, t_max)


def test_p2_occlusion_and_specular_cones_use_their_own_extent_and_aperture():
    n, a = 64, 0.02
    mips = uniform_mips(n, [0.1 * a, 0.2 * a, 0.3 * a, a])
    d, wt = cone_set("six")
    p = ConeParams(d, wt, occ_aperture=math.radians(40), spec_aperture_scale=math.pi / 3,
                   light_pos=(0.5, 0.9, 0.5), max_dist=1.0, alpha_thresh=1.0)
    x, nrm = (0.5, 1.0 / 64, 0.5), (0.0, 1.0, 0.0)
    pr, nr, cam = one_pixel(x, nrm, rough=0.4)
    out, info = oracle.trace(mips, pr, nr, cam, p, return_info=True)
    o = np.array(x) + np.array(nrm) / 64
    dist = np.linalg.norm(np.array(p.light_pos) - o)
    k_occ = closed_form_count(n, math.radians(40), 0.5, 0.001, min(1.0, dist))
    k_spec = closed_form_count(n, 0.4 * math.pi / 3, 0.5, 0.001, 1.0)
    k_diff = closed_form_count(n, math.pi / 3, 0.5, 0.001, 1.0)
    assert list(info["K"]) == [k_diff] * 6 + [k_spec, k_occ]
    assert out[0, 0, 0, 7] == pytest.approx(1 - (1 - a) ** k_occ, abs=1e-12)
    assert np.allclose(out[0, 0, 0, 4:7], np.array([0.1, 0.2, 0.3]) * (1 - (1 - a) ** k_spec), atol=1e-12)
    wsum = float(np.sum(wt.astype(np.float64)))          # float32 weights 1/6 do not sum to 1 exactly
    assert out[0, 0, 0, 3] == pytest.approx(wsum * (1 - (1 - a) ** k_diff), abs=1e-12)


# ----------------------------------------- P3 zero aperture vs scipy trilinear
def _scipy_trilinear(grid, u):
    """scipy's linear interpolation at texel coordinates u (x, y, z order),
    replicating edge texels outside (clamp-to-edge)."""
    coords = np.stack([u[:, 2], u[:, 1], u[:, 0]])
    return np.stack([ndimage.map_coordinates(grid[..., c], coords, order=1, mode="nearest")
                     for c in range(4)], axis=1)


def test_p3_zero_aperture_march_samples_match_scipy():
    n = 32
    g = random_grid(n, seed=7).astype(np.float64)
    mips = oracle.build_mips(g)
    p = single_cone_params(0.0, beta=0.5, t0=0.003, t_max=0.7, thresh=2.0, offset=0.0)
    pr, nr, cam = random_gbuffer(1, 5, 7, seed=11, n=n, invalid_frac=0.0)
    lanes = oracle.cone_lanes(pr, nr, cam, p, n)
    res = oracle.march(mips, lanes, p, record=True)
    v0 = 1.0 / n
    checked = 0
    for k, (idx, ti, d, lam, a_prev, s) in enumerate(res["steps"]):
        # zero aperture: d is the voxel size, LOD 0, t_k = t0 + k beta v0
        assert np.all(d == v0) and np.all(lam == 0.0)
        assert np.allclose(ti, 0.003 + k * 0.5 * v0, rtol=0, atol=1e-12)
        pos = lanes["o"][idx] + ti[:, None] * lanes["w"][idx]
        ref = _scipy_trilinear(g, pos * n - 0.5)
        np.testing.assert_allclose(s, ref, rtol=0, atol=1e-12)
        checked += len(idx)
    assert checked == 35 * 45          # 5x7 lanes, t_k <= 0.7 for k < 45


def test_p3_positions_outside_grid_clamp_to_edge():
    n = 8
    g = random_grid(n, seed=3).astype(np.float64)
    mips = oracle.build_mips(g)
    rng = np.random.default_rng(0)
    pos = rng.uniform(-0.4, 1.4, size=(500, 3))
    s = oracle.sample(mips, pos, np.zeros(500))
    ref = _scipy_trilinear(g, pos * n - 0.5)
    np.testing.assert_allclose(s, ref, rtol=0, atol=1e-12)


# -------------------------------------------------- P4 mips vs block averages
@pytest.mark.parametrize("n", [4, 8, 16])
def test_p4_mips_are_block_means(n):
    g = random_grid(n, seed=n).astype(np.float64)
    mips = oracle.build_mips(g)
    assert len(mips) == int(math.log2(n)) + 1
    for l, m in enumerate(mips):
        b = 2 ** l
        k = n // b
        direct = g.reshape(k, b, k, b, k, b, 4).mean(axis=(1, 3, 5))
        np.testing.assert_allclose(m, direct, rtol=1e-14, atol=1e-15)


def test_p4_partial_pyramid_and_uniform_stays_uniform():
    g = np.full((16, 16, 16, 4), 0.3125)
    mips = oracle.build_mips(g, levels=3)
    assert len(mips) == 3
    for m in mips:
        assert np.all(m == 0.3125)


# ------------------------------------------ P5 texel centres at integer LOD
def test_p5_integer_lod_at_texel_centres_returns_texel():
    n = 16
    g = random_grid(n, seed=5).astype(np.float64)
    mips = oracle.build_mips(g)
    rng = np.random.default_rng(1)
    for l, m in enumerate(mips):
        nl = n >> l
        idx = rng.integers(0, nl, size=(64, 3))
        pos = (idx + 0.5) / nl
        s = oracle.sample(mips, pos, np.full(64, float(l)))
        np.testing.assert_array_equal(s, m[idx[:, 2], idx[:, 1], idx[:, 0]])


def test_lod_is_log2_of_diameter_over_voxel_size():
    """Checkerboard opacity: level 0 alternates 0/1, level 1 is uniformly 1/2.
    A cone whose first sample has diameter 1.5 voxels must blend the two
    levels with weight log2(1.5) on level 1 (reading R2)."""
    n = 64
    iz, iy, ix = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    alpha = ((ix + iy + iz) % 2).astype(np.float64)
    g = np.stack([0.25 * alpha, 0.5 * alpha, 0.75 * alpha, alpha], -1)
    t0, v0 = 1.0 / 128, 1.0 / n                      # exact in float32
    gamma = 2 * math.atan(0.75 * v0 / t0)          # 2 t0 tan(gamma/2) = 1.5 v0
    p = single_cone_params(gamma, t0=t0, t_max=t0 + 0.1 * v0, offset=0.0)   # one sample
    centre = (np.array([21, 40, 30]) + 0.5) / n      # texel with (x+y+z) odd -> alpha 1
    pr, nr, cam = one_pixel(centre - np.array([0.0, 0.0, t0]), (0.0, 0.0, 1.0))
    out = oracle.render(g, pr, nr, cam, p)
    f = math.log2(1.5)
    assert out[0, 0, 0, 3] == pytest.approx((1 - f) * 1.0 + f * 0.5, abs=1e-9)
    assert out[0, 0, 0, 1] == pytest.approx(0.5 * ((1 - f) * 1.0 + f * 0.5), abs=1e-9)


def test_lod_saturates_at_the_top_level():
    """A cone wider than the grid: once its diameter passes 2^(L-1) voxels the
    LOD stays at the top level L-1 (reading R5), whose single texel is the
    mean of the base grid, so every such sample equals that mean (to the
    rounding of its eight tap weights, which sum to 1)."""
    n = 8
    g = random_grid(n, seed=9).astype(np.float64)
    mips = oracle.build_mips(g)
    top = len(mips) - 1
    gamma = 2 * math.atan(2.0)                       # d = 4 t: t grows 3x a step once d > v0
    p = single_cone_params(gamma, beta=0.5, t0=0.01, t_max=8.0, offset=0.0)
    pr, nr, cam = one_pixel((0.4, 0.55, 0.2), (0.0, 0.0, 1.0))
    lanes = oracle.cone_lanes(pr, nr, cam, p, n)
    res = oracle.march(mips, lanes, p, record=True)
    v0 = 1.0 / n
    saturated = 0
    for idx, ti, d, lam, a_prev, s in res["steps"]:
        assert np.all(lam <= top)
        sat = d >= 2.0 ** top * v0
        assert np.all(lam[sat] == top)
        np.testing.assert_allclose(s[sat], np.broadcast_to(mips[top][0, 0, 0], s[sat].shape), rtol=1e-14)
        saturated += int(sat.sum())
    assert saturated >= 3
    np.testing.assert_allclose(mips[top][0, 0, 0], g.mean(axis=(0, 1, 2)), rtol=1e-14)


# ------------------------------------------------- P6 linearity of one sample
def test_p6_single_sample_march_is_linear_in_the_grid():
    n = 16
    g1 = random_grid(n, seed=1).astype(np.float64)
    g2 = random_grid(n, seed=2).astype(np.float64)
    p = single_cone_params(math.radians(50), t0=0.02, t_max=0.021, thresh=10.0)
    pr, nr, cam = random_gbuffer(1, 6, 6, seed=4, n=n, invalid_frac=0.0)
    f1 = oracle.render(g1, pr, nr, cam, p)
    f2 = oracle.render(g2, pr, nr, cam, p)
    f12 = oracle.render(g1 + g2, pr, nr, cam, p)
    np.testing.assert_allclose(f12, f1 + f2, rtol=0, atol=1e-13)
    assert np.abs(f1).max() > 0.05


# -------------------------------------------------- P8 rgb scaling separation
def test_p8_rgb_scale_scales_colour_only():
    w = make_workload("c0", h=16, w=16, n=32)
    g2 = w.base.astype(np.float64).copy()
    g2[..., 0:3] *= 3.0
    f1 = oracle.render(w.base, w.pos_rough, w.normal, w.cam_pos, w.params)
    f2 = oracle.render(g2, w.pos_rough, w.normal, w.cam_pos, w.params)
    np.testing.assert_allclose(f2[..., 0:3], 3 * f1[..., 0:3], rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(f2[..., 4:7], 3 * f1[..., 4:7], rtol=1e-13, atol=1e-15)
    np.testing.assert_array_equal(f2[..., 3], f1[..., 3])
    np.testing.assert_array_equal(f2[..., 7], f1[..., 7])


# ------------------------------------------------------------------ P9 bounds
def test_p9_alpha_in_unit_interval_and_colour_bounded_by_radiance():
    n = 32
    rng = np.random.default_rng(3)
    alpha = rng.uniform(0, 1, size=(n, n, n, 1))
    straight = rng.uniform(0, 0.8, size=(n, n, n, 3))
    g = np.concatenate([straight * alpha, alpha], -1)
    d, wt = cone_set("six")
    p = ConeParams(d, wt, alpha_thresh=0.99)
    pr, nr, cam = random_gbuffer(1, 8, 8, seed=9, n=n)
    mips = oracle.build_mips(g)
    lanes = oracle.cone_lanes(pr, nr, cam, p, n)
    res = oracle.march(mips, lanes, p)
    assert np.all(res["alpha"] >= 0) and np.all(res["alpha"] <= 1)
    assert np.all(res["c"] <= 0.8 * res["alpha"][:, None] + 1e-12)


# ---------------------------------------------------------- cone set geometry
def test_cone_axes_geometry():
    n = 32
    d, wt = cone_set("five")
    p = ConeParams(d, wt, light_pos=(0.5, 0.9, 0.5))
    pr, nr, cam = random_gbuffer(1, 4, 5, seed=2, n=n, invalid_frac=0.0)
    lanes = oracle.cone_lanes(pr, nr, cam, p, n)
    m = 20
    nn = nr.reshape(-1, 4)[:, 0:3].astype(np.float64)
    nn /= np.linalg.norm(nn, axis=1, keepdims=True)
    w = lanes["w"].reshape(7, m, 3)
    assert np.allclose(np.linalg.norm(w, axis=2), 1.0)
    assert np.allclose(np.sum(w[0] * nn, 1), 1.0)                       # front cone = normal
    for q in range(1, 5):                                                 # 45 deg from normal
        assert np.allclose(np.sum(w[q] * nn, 1), math.cos(math.radians(45)))
    for q in range(1, 5):                                                 # azimuths 90 deg apart
        nxt = 1 + q % 4
        pq = w[q] - np.sum(w[q] * nn, 1, keepdims=True) * nn
        pn = w[nxt] - np.sum(w[nxt] * nn, 1, keepdims=True) * nn
        assert np.allclose(np.sum(pq * pn, 1), 0.0, atol=1e-12)
    # specular: mirror of the view direction about the normal
    x = pr.reshape(-1, 4)[:, 0:3].astype(np.float64)
    v = x - cam.astype(np.float64)[0]
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    r = w[5]
    assert np.allclose(np.sum(r * nn, 1), -np.sum(v * nn, 1))
    assert np.allclose(np.cross(r - v, nn), 0.0, atol=1e-12)           # tangential parts agree
    # occlusion: toward the light from the offset origin
    o = x + nn / n
    lv = np.array(p.light_pos) - o
    assert np.allclose(w[6], lv / np.linalg.norm(lv, axis=1, keepdims=True))
    assert np.allclose(lanes["tmax"][6 * m:], np.minimum(1.0, np.linalg.norm(lv, axis=1)))


def test_tangent_frame_handedness_on_slab_scenes():
    """R10's frame, worked by hand: for n = +z, a = +y, t = a x n = +x and
    b = n x t = +y; for n = +y, a = +x, t = +z and b = +x.  A narrow cone along
    the tangent-space axis (0, 1, 0) must therefore reach an opaque slab
    placed on the world +y side (first case) or +x side (second case), and
    the cone along (0, -1, 0) must see nothing."""
    n = 16
    for nrm, axis in (((0.0, 0.0, 1.0), 1), ((0.0, 1.0, 0.0), 0)):
        base = np.zeros((n, n, n, 4))
        sl = [slice(None)] * 3
        sl[2 - axis] = slice(12, None)                     # world axis -> array axis ([z][y][x])
        base[tuple(sl)] = (1.0, 0.0, 0.0, 1.0)
        pr, nr, cam = one_pixel((0.5, 0.5, 0.5), nrm)
        for sign, lit in ((1.0, True), (-1.0, False)):
            p = ConeParams(np.array([[0.0, sign, 0.0]], np.float32), np.ones(1, np.float32),
                           diffuse_aperture=0.05, enable_spec=False, enable_occ=False, max_dist=0.45)
            d = oracle.render(base, pr, nr, cam, p)[0, 0, 0, 0]
            assert (d > 0.5) if lit else (d == 0.0), (nrm, sign, d)


def test_invalid_pixels_are_zero_and_valid_ones_not():
    w = make_workload("c0", h=16, w=16, n=32)
    nr = w.normal.copy()
    nr[0, ::2, :, 3] = 0.0
    out = oracle.render(w.base, w.pos_rough, nr, w.cam_pos, w.params)
    assert np.all(out[0, ::2] == 0.0)
    assert np.abs(out[0, 1::2]).max() > 0.0


# ------------------------------------------------------------- P7 gradients
def test_p7_mip_adjoint_is_the_transpose():
    n = 16
    rng = np.random.default_rng(0)
    v = rng.normal(size=(n, n, n, 4))
    mv = oracle.build_mips(v)
    u = [rng.normal(size=m.shape) for m in mv]
    lhs = sum(float(np.sum(a * b)) for a, b in zip(mv, u))
    rhs = float(np.sum(v * oracle.mip_adjoint(u)))
    assert lhs == pytest.approx(rhs, rel=1e-12)


@pytest.fixture(scope="module")
def fd_case():
    w = make_workload("c3fd")
    rng = np.random.default_rng(42)
    # a smoothed, partly transparent version of the scene so that gradients
    # reach many texels and alpha stays below the threshold for a while
    g = 0.6 * w.base.astype(np.float64) + 0.05 * rng.uniform(size=w.base.shape)
    gout = rng.normal(size=w.pos_rough.shape[:3] + (8,))
    return w, g, gout


def _loss_and_K(w, g, gout, levels=None):
    mips = oracle.build_mips(g)
    out, info = oracle.trace(mips, w.pos_rough, w.normal, w.cam_pos, w.params, return_info=True)
    return float(np.sum(out * gout)), info["K"]


def test_p7_gradient_matches_central_differences(fd_case):
    w, g, gout = fd_case
    mips = oracle.build_mips(g)
    grad = oracle.trace_backward(mips, w.pos_rough, w.normal, w.cam_pos, w.params, gout)
    _, K0 = _loss_and_K(w, g, gout)
    rng = np.random.default_rng(5)
    flat = np.abs(grad).reshape(-1)
    coords = list(np.argsort(flat)[-40:]) + list(rng.integers(0, flat.size, size=24))
    h = 1e-5
    gmax = flat.max()
    checked = 0
    for c in coords:
        gp = g.copy().reshape(-1)
        gp[c] += h
        gm = g.copy().reshape(-1)
        gm[c] -= h
        lp, Kp = _loss_and_K(w, gp.reshape(g.shape), gout)
        lm, Km = _loss_and_K(w, gm.reshape(g.shape), gout)
        if not (np.array_equal(Kp, K0) and np.array_equal(Km, K0)):
            continue                                            # termination changed (R12)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - flat[c] * np.sign(grad.reshape(-1)[c])) <= 1e-6 * gmax + 1e-9, c
        checked += 1
    assert checked >= 50


def test_p7_directional_derivative_over_all_coordinates(fd_case):
    w, g, gout = fd_case
    mips = oracle.build_mips(g)
    grad = oracle.trace_backward(mips, w.pos_rough, w.normal, w.cam_pos, w.params, gout)
    rng = np.random.default_rng(8)
    v = rng.normal(size=g.shape)
    h = 1e-6
    lp, Kp = _loss_and_K(w, g + h * v, gout)
    lm, Km = _loss_and_K(w, g - h * v, gout)
    _, K0 = _loss_and_K(w, g, gout)
    assert np.array_equal(Kp, K0) and np.array_equal(Km, K0)
    fd = (lp - lm) / (2 * h)
    an = float(np.sum(grad * v))
    assert fd == pytest.approx(an, rel=1e-6)
