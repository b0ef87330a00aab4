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


def _uniform_cone(c, a, gamma, p, n, levels, mode="plain", strength=1.0):
    """(C, A) of one cone in a uniform medium through an anisotropic pyramid,
    by a scalar loop: the level-l texel holds the light and opacity of 2^l
    voxels, (c (1 - (1-a)^(2^l)) / a, 1 - (1-a)^(2^l)), in every direction.
    mode "first" returns the first sample's colour (every sample's alpha
    exceeds 1/100 here); "falloff" scales each alpha by the Hermite step of
    sqrt(t) * strength over [0, max_dist]."""
    v0 = 1.0 / n

    def level(lv):
        t = (1.0 - a) ** (2 ** lv)
        return np.append(c * (1.0 - t) / a, 1.0 - t)

    t, C, A = p.t0, np.zeros(3), 0.0
    while t <= p.max_dist and A < p.alpha_thresh:
        d = max(2.0 * t * math.tan(gamma / 2.0), v0)
        lam = min(max(math.log2(d / v0), 0.0), levels - 1)
        l0 = int(math.floor(lam))
        f = lam - l0
        s = (1.0 - f) * level(l0) + (f * level(min(l0 + 1, levels - 1)) if f > 0 else 0.0)
        if mode == "first":
            return s[0:3], s[3]
        if mode == "falloff":
            h = min(max(math.sqrt(t) * strength / p.max_dist, 0.0), 1.0)
            s = s.copy()
            s[3] *= h * h * (3.0 - 2.0 * h)
        C += (1.0 - A) * s[0:3]
        A += (1.0 - A) * s[3]
        t += p.step_factor * d
    return C, A


def _uniform_setup(n=16):
    c, a = np.array([0.12, 0.06, 0.03]), 0.15
    base = np.zeros((n, n, n, 4))
    base[..., 0:3] = c
    base[..., 3] = a
    rng = np.random.default_rng(4)
    pr = np.concatenate([rng.uniform(0.3, 0.7, size=(1, 3, 4, 3)), np.full((1, 3, 4, 1), 0.5)], -1)
    nr = np.concatenate([rng.normal(size=(1, 3, 4, 3)), np.ones((1, 3, 4, 1))], -1)
    dirs = np.array([[0, 0, 1], [0.6, 0, 0.8], [0, -0.6, 0.8]], np.float32)
    p = ConeParams(dirs, np.array([0.5, 0.3, 0.2], np.float32), diffuse_aperture=0.9, spec_aperture_scale=0.5,
                   occ_aperture=0.7, light_pos=(9.0, 9.0, 9.0), step_factor=0.6, t0=0.01, max_dist=0.6,
                   alpha_thresh=0.97)
    return n, c, a, base, pr, nr, p


def test_uniform_medium_trace_through_anisotropic_pyramids():
    n, c, a, base, pr, nr, p = _uniform_setup()
    am = va.build_aniso_mips(base)
    out = va.trace_aniso(am, pr, nr, np.array([[0.5, 0.5, 3.0]]), p)
    Cd, Ad = _uniform_cone(c, a, p.diffuse_aperture, p, n, 5)
    Cs, _ = _uniform_cone(c, a, 0.5 * p.spec_aperture_scale, p, n, 5)
    _, Ao = _uniform_cone(c, a, p.occ_aperture, p, n, 5)
    W = float(np.sum(p.diffuse_weights.astype(np.float64)))
    expect = np.concatenate([W * Cd, [W * Ad], Cs, [Ao]])
    np.testing.assert_allclose(out.reshape(-1, 8), np.broadcast_to(expect, (12, 8)), rtol=1e-12)
    # the isotropic pyramid of the same medium holds the 2x2x2 means (c, a) at every level: a different result
    assert np.abs(oracle.trace(oracle.build_mips(base), pr, nr, np.array([[0.5, 0.5, 3.0]]), p)
                  - out).max() > 1e-2


def test_uniform_medium_shading_and_bounce_through_the_sampler_hook():
    from oracle import vct_bounce as vb
    from oracle import vct_shade as vs
    from scenes.configs import ShadeParams
    n, c, a, base, pr, nr, p = _uniform_setup()
    am = va.build_aniso_mips(base)
    smp = va.aniso_sampler(am)
    # the oracles' own pyramid argument gets the isotropic pyramid, whose levels hold (c, a) unintegrated: a
    # march that bypassed the sampler hook would read it and miss the closed forms below
    iso = oracle.build_mips(base)
    Cd, _ = _uniform_cone(c, a, p.diffuse_aperture, p, n, 5)
    Cs, _ = _uniform_cone(c, a, 0.5 * p.spec_aperture_scale, p, n, 5)
    W = float(np.sum(p.diffuse_weights.astype(np.float64)))
    # no lights, unmodified cones: L = sum_q w_q C_q + C_spec
    sp = ShadeParams(np.zeros((0, 3), np.float32), np.zeros((0, 3), np.float32), np.zeros((0, 3), np.float32),
                     diffuse_first_hit=False, occlusion_falloff=False, specular_brdf=False)
    mat = np.concatenate([np.full((1, 3, 4, 3), 0.5), np.full((1, 3, 4, 1), 8.0)], -1)
    out = vs.shade(iso, pr, nr, mat, np.array([[0.5, 0.5, 3.0]]), p, sp, sampler=smp)
    np.testing.assert_allclose(out[..., 0:3].reshape(-1, 3), np.broadcast_to(W * Cd + Cs, (12, 3)), rtol=1e-12)
    # first-hit diffuse cones and one far, dark light with falloff occlusion: L = o_min (sum_q w_q s_0) + C_spec
    sp2 = ShadeParams(np.array([[9.0, 9.0, 9.0]], np.float32), np.zeros((1, 3), np.float32),
                      np.zeros((1, 3), np.float32), diffuse_first_hit=True, occlusion_falloff=True,
                      shadow_strength=2.0, specular_brdf=False)
    # (t0 = 0.2: the first sample lies between levels 1 and 2, where the directions are pre-integrated)
    p2 = p.replace(t0=0.2)
    out = vs.shade(iso, pr, nr, mat, np.array([[0.5, 0.5, 3.0]]), p2, sp2, sampler=smp)
    s0, _ = _uniform_cone(c, a, p2.diffuse_aperture, p2, n, 5, mode="first")
    _, Af = _uniform_cone(c, a, p2.occ_aperture, p2, n, 5, mode="falloff", strength=2.0)
    Cs2, _ = _uniform_cone(c, a, 0.5 * p2.spec_aperture_scale, p2, n, 5)
    np.testing.assert_allclose(out[..., 3].ravel(), 1.0 - Af, rtol=1e-12)
    np.testing.assert_allclose(out[..., 0:3].reshape(-1, 3), np.broadcast_to((1.0 - Af) * W * s0 + Cs2, (12, 3)),
                               rtol=1e-12)
    # one bounce in the same medium: c + a * rho * W * C_diffuse
    rho = np.array([0.9, 0.5, 0.2])
    nrm = np.zeros((n, n, n, 4))
    nrm[..., 0:3] = (0.3, 0.0, -0.4)
    alb = np.zeros((n, n, n, 4))
    alb[..., 0:3] = rho
    got = vb.bounce(base, nrm, alb, p, mips=iso, sampler=smp)
    np.testing.assert_allclose(got[..., 0:3], np.broadcast_to(c + a * rho * W * Cd, (n, n, n, 3)), rtol=1e-12)


def test_aniso_mip_adjoint_is_the_derivative_of_the_build():
    """<adjoint(G), delta> = d/de <G, build(base + e delta)> at e = 0 (central
    differences; the build is a polynomial in the base, so h = 1e-4 is exact to
    rounding)."""
    rng = np.random.default_rng(11)
    n = 8
    base = np.concatenate([rng.uniform(0, 0.6, size=(n, n, n, 3)), rng.uniform(0, 0.9, size=(n, n, n, 1))], -1)
    delta = rng.normal(size=base.shape)
    am = va.build_aniso_mips(base)
    G = [[rng.normal(size=m.shape) for m in pyr] for pyr in am]
    got = np.sum(va.aniso_mip_adjoint(am, G) * delta)

    def pairing(b):
        a = va.build_aniso_mips(b)
        # level 0 is shared: pair it once with the sum of the six level-0 gradients, as the adjoint does
        return (np.sum(sum(G[d][0] for d in range(6)) * a[0][0])
                + sum(np.sum(G[d][lv] * a[d][lv]) for d in range(6) for lv in range(1, len(a[d]))))

    h = 1e-4
    fd = (pairing(base + h * delta) - pairing(base - h * delta)) / (2 * h)
    np.testing.assert_allclose(got, fd, rtol=1e-9)


def test_aniso_trace_adjoint_matches_finite_differences():
    rng = np.random.default_rng(12)
    n = 8
    base = np.concatenate([rng.uniform(0, 0.5, size=(n, n, n, 3)), rng.uniform(0, 0.35, size=(n, n, n, 1))], -1)
    base[..., 0:3] *= base[..., 3:4]
    pr = np.concatenate([rng.uniform(0.3, 0.7, size=(1, 2, 3, 3)), np.full((1, 2, 3, 1), 0.6)], -1)
    nr = np.concatenate([rng.normal(size=(1, 2, 3, 3)), np.ones((1, 2, 3, 1))], -1)
    cam = np.array([[0.5, 0.5, 2.0]])
    dirs = np.array([[0, 0, 1], [0.6, 0, 0.8], [0, -0.6, 0.8]], np.float32)
    p = ConeParams(dirs, np.array([0.5, 0.3, 0.2], np.float32), diffuse_aperture=1.0, spec_aperture_scale=1.2,
                   occ_aperture=0.9, light_pos=(0.5, 0.9, 0.5), step_factor=0.7, t0=0.02, max_dist=0.7,
                   alpha_thresh=0.99)
    out, info = va.trace_aniso(va.build_aniso_mips(base), pr, nr, cam, p, return_info=True)
    gout = rng.normal(size=out.shape)
    gout[info["ambiguous"]] = 0.0
    grad = va.trace_backward_aniso(va.build_aniso_mips(base), pr, nr, cam, p, gout)

    def loss(b):
        return np.sum(gout * va.trace_aniso(va.build_aniso_mips(b), pr, nr, cam, p))

    idx = [tuple(int(v) for v in rng.integers(0, n, size=3)) + (int(rng.integers(0, 4)),) for _ in range(10)]
    big = np.unravel_index(np.argsort(-np.abs(grad).ravel())[:10], grad.shape)
    idx += list(zip(*[a.tolist() for a in big]))
    h = 1e-6
    for i in idx:
        bp, bm = base.copy(), base.copy()
        bp[i] += h
        bm[i] -= h
        fd = (loss(bp) - loss(bm)) / (2 * h)
        assert abs(fd - grad[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, grad[i])
    assert np.abs(grad).max() > 1e-2
