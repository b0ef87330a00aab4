"""Pins of the anisotropic-mip oracle against closed forms (a uniform medium's
pre-integrated opacity, additive emission of transparent grids, a two-slab
block worked by hand) and against the pinned isotropic trace where the two
must agree (LOD below 1 never reaches a directional level).  CPU only."""
import math

import numpy as np
import pytest

import oracle
from oracle import vct_aniso as va
from scenes.configs import ConeParams


def test_uniform_medium_preintegrates_along_every_direction():
    n, c, a = 16, np.array([0.2, 0.1, 0.05]), 0.3
    base = np.zeros((n, n, n, 4))
    base[..., 0:3] = c
    base[..., 3] = a
    am = va.build_aniso_mips(base)
    assert len(am) == 6 and all(len(p) == 5 for p in am)
    for d in range(6):
        for lv in range(1, 5):
            k = 2 ** lv                                   # voxels crossed by a ray through a level-l texel
            t = (1.0 - a) ** k
            np.testing.assert_allclose(am[d][lv][..., 3], 1.0 - t, rtol=1e-13)
            np.testing.assert_allclose(am[d][lv][..., 0:3], np.broadcast_to(c * (1.0 - t) / a, am[d][lv][..., 0:3].shape),
                                       rtol=1e-13)
        assert am[d][0] is am[0][0] or np.array_equal(am[d][0], base)


def test_transparent_grid_adds_the_light_of_the_crossed_voxels():
    rng = np.random.default_rng(1)
    n = 16
    base = np.zeros((n, n, n, 4))
    base[..., 0:3] = rng.uniform(0, 1, size=(n, n, n, 3))     # alpha 0: emission only
    am = va.build_aniso_mips(base)
    for lv in range(1, 5):
        k = 2 ** lv
        m = n // k
        block_mean = base.reshape(m, k, m, k, m, k, 4).mean(axis=(1, 3, 5))
        for d in range(6):
            np.testing.assert_allclose(am[d][lv], k * block_mean, rtol=1e-12, atol=1e-14)


def test_two_slab_block_by_hand():
    base = np.zeros((2, 2, 2, 4))
    red = np.array([0.6, 0.0, 0.0, 0.6])      # premultiplied, the x = 0 slab
    blue = np.array([0.0, 0.0, 0.9, 0.9])     # the x = 1 slab
    base[:, :, 0] = red
    base[:, :, 1] = blue
    am = va.build_aniso_mips(base)
    top = [am[d][1][0, 0, 0] for d in range(6)]
    np.testing.assert_allclose(top[0], [0.6, 0.0, 0.4 * 0.9, 0.6 + 0.4 * 0.9], rtol=1e-14)    # +x: red in front
    np.testing.assert_allclose(top[1], [0.1 * 0.6, 0.0, 0.9, 0.9 + 0.1 * 0.6], rtol=1e-14)    # -x: blue in front
    along = 0.5 * np.array([0.6 + 0.4 * 0.6, 0.0, 0.9 + 0.1 * 0.9, 0.0])
    along[3] = 0.5 * ((0.6 + 0.4 * 0.6) + (0.9 + 0.1 * 0.9))
    for d in (2, 3, 4, 5):                      # along y or z each pair stays inside one slab
        np.testing.assert_allclose(top[d], along, rtol=1e-14)


def test_sample_weights_are_the_squared_axis_components():
    rng = np.random.default_rng(2)
    n = 8
    base = np.concatenate([rng.uniform(0, 1, size=(n, n, n, 3)) * 0.5, rng.uniform(0, 0.5, size=(n, n, n, 1))], -1)
    am = va.build_aniso_mips(base)
    # the centre of level-1 texel (k, j, i) sampled at LOD exactly 1 reads that texel alone
    i, j, k = 1, 2, 3
    p = np.array([[(i + 0.5) * 2 / n, (j + 0.5) * 2 / n, (k + 0.5) * 2 / n]] * 4)
    w = np.array([[1.0, 0.0, 0.0], [0.0, -1.0, 0.0], [0.6, -0.8, 0.0], [-0.48, 0.6, 0.64]])
    s = va.sample_aniso(am, p, np.ones(4), w)
    tex = [am[d][1][k, j, i] for d in range(6)]
    np.testing.assert_allclose(s[0], tex[0], rtol=1e-14)
    np.testing.assert_allclose(s[1], tex[3], rtol=1e-14)
    np.testing.assert_allclose(s[2], 0.36 * tex[0] + 0.64 * tex[3], rtol=1e-14)
    np.testing.assert_allclose(s[3], 0.2304 * tex[1] + 0.36 * tex[2] + 0.4096 * tex[4], rtol=1e-14)


def test_below_lod_one_the_trace_is_the_isotropic_trace():
    rng = np.random.default_rng(3)
    n = 16
    base = np.concatenate([rng.uniform(0, 1, size=(n, n, n, 3)) * 0.3, rng.uniform(0, 0.3, size=(n, n, n, 1))], -1)
    base[..., 0:3] *= base[..., 3:4]
    pr = np.concatenate([rng.uniform(0.2, 0.8, size=(1, 5, 7, 3)), np.full((1, 5, 7, 1), 0.01)], -1)
    nr = np.concatenate([rng.normal(size=(1, 5, 7, 3)), np.ones((1, 5, 7, 1))], -1)
    cam = np.array([[0.5, 0.5, 2.0]])
    dirs = np.array([[0, 0, 1], [0.6, 0, 0.8], [0, 0.6, 0.8]], np.float32)
    # apertures so narrow that d = v0 for every t <= max_dist: LOD 0 throughout
    p = ConeParams(dirs, np.full(3, 1 / 3, np.float32), diffuse_aperture=1e-3, spec_aperture_scale=1e-3,
                   occ_aperture=1e-3, light_pos=(0.5, 0.9, 0.5), max_dist=0.6, alpha_thresh=0.95)
    iso = oracle.trace(oracle.build_mips(base), pr, nr, cam, p)
    ani = va.trace_aniso(va.build_aniso_mips(base), pr, nr, cam, p)
    np.testing.assert_allclose(ani, iso, rtol=1e-13, atol=1e-15)
    # and with wide cones the directional levels do make a difference
    wide = p.replace(diffuse_aperture=math.pi / 3, spec_aperture_scale=math.pi / 3, occ_aperture=math.pi / 3)
    assert np.abs(va.trace_aniso(va.build_aniso_mips(base), pr, nr, cam, wide)
                  - oracle.trace(oracle.build_mips(base), pr, nr, cam, wide)).max() > 1e-3
