"""Pins of the further-bounce oracle and of the voxelizer's surface attributes
against closed forms and counting facts (front-to-back compositing written
out along a grid row, a uniform medium's geometric series, exact averages of
known normals), not against the oracle's own formulas.  CPU only."""
import math

import numpy as np
import pytest

from oracle import vct_bounce as vb
from oracle import vct_voxelize as vx
from scenes.configs import ConeParams

N = 16
V0 = 1.0 / N


def _row_params(weight=0.75, steps=6):
    """One front cone, aperture so narrow that every sample is a level-0 texel
    centre: origin offset 1/2 voxel, t0 = v0 / 2, t += v0."""
    return ConeParams(np.array([[0.0, 0.0, 1.0]], np.float32), np.array([weight], np.float32),
                      diffuse_aperture=1e-4, step_factor=1.0, t0=0.5 * V0, normal_offset=0.5,
                      max_dist=(steps - 0.5) * V0, alpha_thresh=1.0)


def _composite_row(base, start, axis, sign, steps, thresh=1.0):
    """Front-to-back compositing of the texels met along +-axis from voxel
    `start` (z, y, x), clamped to the grid edge."""
    c = np.zeros(3)
    a = 0.0
    for k in range(steps):
        if not a < thresh:
            break
        idx = list(start)
        idx[2 - axis] = min(max(idx[2 - axis] + sign * (k + 1), 0), N - 1)
        s = base[tuple(idx)]
        c += (1.0 - a) * s[0:3]
        a += (1.0 - a) * s[3]
    return c


def _row_scene(seed):
    rng = np.random.default_rng(seed)
    alpha = rng.choice([0.0, 0.25, 0.5, 1.0], size=(N, N, N), p=[0.55, 0.2, 0.15, 0.1])
    base = np.zeros((N, N, N, 4))
    base[..., 0:3] = rng.uniform(0.0, 1.0, size=(N, N, N, 3)) * alpha[..., None]
    base[..., 3] = alpha
    normal = np.zeros((N, N, N, 4))
    albedo = np.zeros((N, N, N, 4))
    albedo[..., 0:3] = rng.uniform(0.1, 0.9, size=(N, N, N, 3))
    return rng, base, normal, albedo


def test_axis_normals_gather_the_composited_row():
    rng, base, normal, albedo = _row_scene(7)
    steps, w = 6, 0.75
    recv = []
    for axis in range(3):
        for sign in (1, -1):
            for _ in range(3):
                z, y, x = (int(v) for v in rng.integers(0, N, size=3))
                if any(r[0] == (z, y, x) for r in recv):
                    continue
                base[z, y, x] = (0.3, 0.2, 0.1, 0.5)
                nv = np.zeros(3)
                nv[axis] = sign * rng.uniform(0.5, 2.0)          # any length >= MIN_NORMAL
                normal[z, y, x, 0:3] = nv
                recv.append(((z, y, x), axis, sign))
    out = vb.bounce(base, normal, albedo, _row_params(w, steps))
    expect = base.copy()
    for (z, y, x), axis, sign in recv:
        c = _composite_row(base, (z, y, x), axis, sign, steps)
        expect[z, y, x, 0:3] += base[z, y, x, 3] * albedo[z, y, x, 0:3] * w * c
    np.testing.assert_allclose(out, expect, rtol=1e-12, atol=1e-15)
    # receivers really gathered something (the check is not vacuous)
    assert sum(np.any(out[r[0]] != base[r[0]]) for r in recv) >= len(recv) // 2


def test_zero_alpha_short_or_cancelled_normals_keep_their_value():
    _, base, normal, albedo = _row_scene(8)
    base[:] = 0.0
    base[2:6, 3:9, 4:12] = (0.2, 0.4, 0.6, 1.0)
    normal[..., 0:3] = (0.0, 1.0, 0.0)
    normal[3, 4, 5, 0:3] = (0.0, 0.5 * vb.MIN_NORMAL, 0.0)    # too short: no direction
    normal[3, 4, 6, 0:3] = 0.0                                # cancelled
    out, info = vb.bounce(base, normal, albedo, _row_params(), return_info=True)
    assert not info["surface"][3, 4, 5] and not info["surface"][3, 4, 6]
    np.testing.assert_array_equal(out[3, 4, 5], base[3, 4, 5])
    np.testing.assert_array_equal(out[3, 4, 6], base[3, 4, 6])
    np.testing.assert_array_equal(out[base[..., 3] == 0], base[base[..., 3] == 0])
    # an interior voxel looking at the opaque voxel above it gathers exactly that voxel
    np.testing.assert_allclose(out[3, 4, 7, 0:3], base[3, 4, 7, 0:3] + albedo[3, 4, 7, 0:3] * 0.75 * base[3, 5, 7, 0:3],
                               rtol=1e-12)


def test_zero_albedo_is_the_identity():
    _, base, normal, albedo = _row_scene(9)
    normal[..., 0:3] = (0.3, -0.4, 0.5)
    out = vb.bounce(base, normal, np.zeros_like(albedo), _row_params())
    np.testing.assert_array_equal(out, base)


def _uniform_samples(params):
    """Number of samples of every cone in a medium of one value (the t
    schedule of the march with d = max(2 t tan(gamma / 2), v0))."""
    t, k = params.t0, 0
    while t <= params.max_dist:
        d = max(2.0 * t * math.tan(params.diffuse_aperture / 2.0), V0)
        t += params.step_factor * d
        k += 1
    return k


@pytest.mark.parametrize("k", [0, 1, 2, 3])
def test_uniform_medium_follows_the_linear_recurrence(k):
    c = np.array([0.3, 0.15, 0.05])
    a, rho = 0.2, np.array([0.9, 0.5, 0.25])
    dirs = np.array([[0, 0, 1], [0.6, 0, 0.8], [0, -0.6, 0.8], [-0.48, 0.36, 0.8]], np.float32)
    wts = np.array([0.4, 0.3, 0.2, 0.1], np.float32)
    p = ConeParams(dirs, wts, diffuse_aperture=math.pi / 3, step_factor=0.5, t0=0.01, normal_offset=1.0,
                   max_dist=0.7, alpha_thresh=1.0)
    base = np.zeros((N, N, N, 4))
    base[..., 0:3] = c
    base[..., 3] = a
    normal = np.zeros((N, N, N, 4))
    normal[..., 0:3] = (0.0, 0.42, -0.56)
    albedo = np.zeros((N, N, N, 4))
    albedo[..., 0:3] = rho
    K = _uniform_samples(p)
    S = sum((1.0 - a) ** j for j in range(K))            # transmittance-weighted sample count
    W = float(np.sum(wts.astype(np.float64)))
    L = c.copy()
    for _ in range(k):
        L = c + a * rho * W * S * L
    out = vb.bounces(base, normal, albedo, p, k)
    np.testing.assert_allclose(out[..., 0:3], np.broadcast_to(L, (N, N, N, 3)), rtol=1e-12)
    np.testing.assert_array_equal(out[..., 3], a)


def test_bounce_traces_the_diffuse_cones_only():
    """In a uniform medium every cone takes the closed-form schedule length K,
    so the bounce's sample count is (surface voxels) x (diffuse cones) x K:
    no specular or occlusion cone is traced (B2)."""
    dirs = np.array([[0, 0, 1], [0.6, 0, 0.8], [0, -0.6, 0.8]], np.float32)
    p = ConeParams(dirs, np.array([0.5, 0.3, 0.2], np.float32), diffuse_aperture=math.pi / 3, step_factor=0.5,
                   t0=0.01, normal_offset=1.0, max_dist=0.5, alpha_thresh=1.0, enable_spec=True, enable_occ=True)
    base = np.zeros((N, N, N, 4))
    base[..., 0:3] = 0.1
    base[..., 3] = 0.05
    normal = np.zeros((N, N, N, 4))
    normal[2:5, 3:7, 4:9, 0:3] = (0.0, 0.0, 1.0)            # 3 x 4 x 5 surface voxels
    albedo = np.full((N, N, N, 4), 0.5)
    _, info = vb.bounce(base, normal, albedo, p, return_info=True)
    assert int(info["surface"].sum()) == 60
    assert info["samples"] == 60 * 3 * _uniform_samples(p)


def test_sampled_voxels_match_the_whole_grid():
    _, base, normal, albedo = _row_scene(10)
    normal[..., 0:3] = np.random.default_rng(0).normal(size=(N, N, N, 3))
    p = _row_params().replace(diffuse_aperture=0.8, step_factor=0.6, max_dist=0.5)
    full = vb.bounce(base, normal, albedo, p)
    vox = np.array([[1, 2, 3], [15, 0, 7], [8, 8, 8], [0, 15, 15]])
    part = vb.bounce(base, normal, albedo, p, voxels=vox)
    np.testing.assert_array_equal(part, full[vox[:, 0], vox[:, 1], vox[:, 2]])


# --- surface attributes of the voxelizer (reading V7) ------------------------

NV = 32
LIGHT = ((0.5, 0.5, 0.9), (1.0, 1.0, 1.0), (1.0, 0.0, 0.0))


def _quad_z(x0, x1, y0, y1, z, up=True):
    a, b, c, d = (x0, y0, z), (x1, y0, z), (x1, y1, z), (x0, y1, z)
    return [(a, b, c), (a, c, d)] if up else [(a, c, b), (a, d, c)]


def _quad_x(x, y0, y1, z0, z1):
    """Quad in the plane x, normal +x."""
    a, b, c, d = (x, y0, z0), (x, y1, z0), (x, y1, z1), (x, y0, z1)
    return [(a, b, c), (a, c, d)]


def test_flat_quad_normal_and_albedo_are_the_triangles():
    tris = np.array(_quad_z(0.1, 0.9, 0.2, 0.8, 0.45, up=False), np.float32)
    cols = np.array([[0.75, 0.5, 0.25]] * 2, np.float32)
    out, nrm, alb = vx.voxelize(tris, cols, NV, [LIGHT], return_surface=True)
    hit = out[..., 3] == 1.0
    assert hit.sum() > 300
    np.testing.assert_array_equal(nrm[hit], np.broadcast_to([0.0, 0.0, -1.0, 1.0], (hit.sum(), 4)))
    np.testing.assert_array_equal(alb[hit][:, 0:3], np.broadcast_to(cols[0].astype(np.float64), (hit.sum(), 3)))
    assert not nrm[~hit].any() and not alb[~hit].any()


def test_opposite_coincident_quads_cancel_and_average_colour():
    t = _quad_z(0.1, 0.9, 0.1, 0.9, 0.3)
    tris = np.array(t + _quad_z(0.1, 0.9, 0.1, 0.9, 0.3, up=False), np.float32)
    cols = np.array([[1, 0, 0]] * 2 + [[0, 0, 1]] * 2, np.float32)
    out, cnt, nrm, alb = vx.voxelize(tris, cols, NV, [LIGHT], return_counts=True, return_surface=True)
    hit = cnt > 0
    assert set(np.unique(cnt[hit])) == {2}
    assert not nrm[hit][:, 0:3].any()
    np.testing.assert_array_equal(alb[hit][:, 0:3], np.broadcast_to([0.5, 0.0, 0.5], (hit.sum(), 3)))
    # no direction: a bounce leaves these voxels alone
    assert not vb.surface_mask(out, nrm).any()


def test_crease_voxels_average_the_two_face_normals():
    # a +z quad at z = 0.5 over x < 0.62 and a +x quad at x = 0.605 over z in (0.45, 0.9):
    # the voxel column x = 19, z = 16 holds one fragment of each
    tris = np.array(_quad_z(0.1, 0.62, 0.2, 0.8, 0.5) + _quad_x(0.605, 0.2, 0.8, 0.45, 0.9), np.float32)
    out, cnt, nrm, _ = vx.voxelize(tris, np.ones((4, 3), np.float32), NV, [LIGHT], return_counts=True,
                                   return_surface=True)
    both = cnt[16, :, 19] == 2
    assert both.sum() >= 15
    np.testing.assert_array_equal(nrm[16, both, 19], np.broadcast_to([0.5, 0.0, 0.5, 1.0], (both.sum(), 4)))
    single = (cnt == 1)
    lens = np.linalg.norm(nrm[single][:, 0:3], axis=1)
    np.testing.assert_array_equal(lens, 1.0)
