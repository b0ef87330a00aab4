"""Pins of the shading oracle (the thesis's cone variants and final shading
equation) against closed forms, textbook values, limits and the already
pinned cone trace; not against its own formulas.  CPU only."""
import math

import numpy as np
import pytest

import oracle
from scenes import ConeParams
from scenes.configs import ShadeParams, cone_set


def uniform_mips(n, value):
    levels = int(round(math.log2(n))) + 1
    return [np.broadcast_to(np.asarray(value, np.float64), (n >> l,) * 3 + (4,)) for l in range(levels)]


def one_pixel(x, nrm, cam, rough=0.5, albedo=(0.8, 0.6, 0.4), shininess=16.0):
    pr = np.array([[[[x[0], x[1], x[2], rough]]]], dtype=np.float32)
    nr = np.array([[[[nrm[0], nrm[1], nrm[2], 1.0]]]], dtype=np.float32)
    mat = np.array([[[[albedo[0], albedo[1], albedo[2], shininess]]]], dtype=np.float32)
    return pr, nr, mat, np.array([cam], dtype=np.float32)


def lights(*pos, idiff=(1.0, 1.0, 1.0), ispec=(0.5, 0.5, 0.5)):
    n = len(pos)
    return (np.array(pos, np.float32).reshape(n, 3), np.tile(np.array(idiff, np.float32), (n, 1)),
            np.tile(np.array(ispec, np.float32), (n, 1)))


def cone_params(**kw):
    d, w = cone_set("six")
    kw.setdefault("alpha_thresh", 0.99)
    return ConeParams(d, w, **kw)


# --- smoothstep and the BRDF --------------------------------------------------

def test_smoothstep_textbook_values():
    x = np.array([-1.0, 0.0, 0.25, 0.5, 0.75, 1.0, 3.0])
    np.testing.assert_allclose(oracle.smoothstep(0.0, 1.0, x), [0, 0, 0.15625, 0.5, 0.84375, 1, 1], atol=0)
    # symmetric about the midpoint, zero slope at both ends, range scaling
    u = np.linspace(0, 1, 11)
    np.testing.assert_allclose(oracle.smoothstep(0, 1, u) + oracle.smoothstep(0, 1, 1 - u), 1.0, atol=1e-15)
    eps = 1e-7
    assert oracle.smoothstep(0, 1, eps) < 1e-13 and 1 - oracle.smoothstep(0, 1, 1 - eps) < 1e-13
    np.testing.assert_allclose(oracle.smoothstep(0, 2, 2 * u), oracle.smoothstep(0, 1, u), atol=1e-15)


def test_fspec_closed_forms():
    sp = ShadeParams(*lights((0, 0, 0)), shininess_falloff=2.0)
    x = np.array([1.0, 0.0, 0.0])
    # perpendicular, no grace: (1 - (pi/2)/pi)^2 = 1/4
    assert oracle.f_spec(x, np.array([0.0, 1.0, 0.0]), 0.0, sp) == pytest.approx(0.25, abs=1e-15)
    # opposite, no grace: 0
    assert oracle.f_spec(x, -x, 0.0, sp) == pytest.approx(0.0, abs=1e-15)
    # inside the grace angle p = 0.008 pi * shininess: exactly 1
    g = 0.3
    ld = np.array([math.cos(g), math.sin(g), 0.0])
    assert oracle.f_spec(x, ld, 0.31 / (0.008 * math.pi), sp) == 1.0
    # outside it: (1 - (g - p)/pi)^q
    shin = 10.0
    p = 0.008 * math.pi * shin
    assert oracle.f_spec(x, ld, shin, sp) == pytest.approx((1 - max(0.0, g - p) / math.pi) ** 2, rel=1e-14)
    # q = 0 gives 1 everywhere
    assert oracle.f_spec(x, -x, 0.0, sp.replace(shininess_falloff=0.0)) == 1.0
    # accurate at tiny angles (the arc cosine of a dot product is not)
    tiny = 1e-7
    ld = np.array([math.cos(tiny), math.sin(tiny), 0.0])
    assert oracle.f_spec(x, ld, 0.0, sp) == pytest.approx((1 - tiny / math.pi) ** 2, rel=1e-15)


# --- direct term on an empty grid --------------------------------------------

@pytest.mark.parametrize("falloff,first_hit,brdf", [(True, True, True), (False, False, False)])
def test_empty_grid_gives_the_direct_phong_term(falloff, first_hit, brdf):
    """No voxels: every cone returns 0 and every visibility is 1, so L is the
    Lambert + Phong sum of the lights, known in closed form here."""
    n = 16
    mips = uniform_mips(n, (0.0, 0.0, 0.0, 0.0))
    # every input below is exact in float32, so the closed form holds to rounding
    x, nrm = (0.5, 0.25, 0.5), (0.0, 1.0, 0.0)
    s2 = math.sqrt(0.5)
    # light at 45 deg in the x-y plane; camera on its mirror direction, so R.w = 1
    lp = (0.75, 0.5, 0.5)
    cam = (0.25, 0.5, 0.5)
    pr, nr, mat, cm = one_pixel(x, nrm, cam, albedo=(0.75, 0.5, 0.25), shininess=32.0)
    sp = ShadeParams(*lights(lp, idiff=(1.0, 0.5, 0.25), ispec=(0.375, 0.375, 0.375)),
                     specular_color=(0.875, 0.875, 0.875),
                     occlusion_falloff=falloff, diffuse_first_hit=first_hit, specular_brdf=brdf)
    out = oracle.shade(mips, pr, nr, mat, cm, cone_params(), sp)[0, 0, 0]
    expect = np.array([0.75 * 1.0, 0.5 * 0.5, 0.25 * 0.25]) * s2 + 0.875 * 0.375 * 1.0
    np.testing.assert_allclose(out[0:3], expect, rtol=1e-12)
    assert out[3] == 1.0
    # camera along the normal instead: R.w = cos 45 deg, Phong falls to (1/sqrt 2)^32
    pr, nr, mat, cm = one_pixel(x, nrm, (0.5, 0.875, 0.5), albedo=(0.75, 0.5, 0.25), shininess=32.0)
    out = oracle.shade(mips, pr, nr, mat, cm, cone_params(), sp)[0, 0, 0]
    expect = np.array([0.75 * 1.0, 0.5 * 0.5, 0.25 * 0.25]) * s2 + 0.875 * 0.375 * s2 ** 32
    np.testing.assert_allclose(out[0:3], expect, rtol=1e-12)
    # light below the surface: no Lambert, no Phong
    pr, nr, mat, cm = one_pixel(x, nrm, cam)
    out = oracle.shade(mips, pr, nr, mat, cm, cone_params(), sp.replace(light_pos=np.array([[0.5, 0.125, 0.5]])))
    np.testing.assert_allclose(out[0, 0, 0, 0:3], 0.0, atol=1e-15)


def test_zero_shininess_makes_the_phong_factor_one():
    """(R.w)^0 = 1 for every view, 0^0 = 1 included (reading S5): with the
    camera where R.w = 0 the Phong factor is 0 at shininess 32 and 1 at 0."""
    n = 16
    mips = uniform_mips(n, (0.0, 0.0, 0.0, 0.0))
    x, nrm = (0.5, 0.25, 0.5), (0.0, 1.0, 0.0)
    s2 = math.sqrt(0.5)
    lp = (0.75, 0.5, 0.5)          # L = (1, 1, 0)/sqrt 2, R = (-1, 1, 0)/sqrt 2
    cam = (0.75, 0.5, 0.5)         # w = L, so R.w = 0
    sp = ShadeParams(*lights(lp, idiff=(1.0, 0.5, 0.25), ispec=(0.375, 0.375, 0.375)),
                     specular_color=(0.875, 0.875, 0.875))
    lambert = np.array([0.75 * 1.0, 0.5 * 0.5, 0.25 * 0.25]) * s2
    for shin, phong in ((32.0, 0.0), (0.0, 1.0)):
        pr, nr, mat, cm = one_pixel(x, nrm, cam, albedo=(0.75, 0.5, 0.25), shininess=shin)
        out = oracle.shade(mips, pr, nr, mat, cm, cone_params(), sp)[0, 0, 0]
        np.testing.assert_allclose(out[0:3], lambert + 0.875 * 0.375 * phong, rtol=1e-12, atol=1e-12)


def test_direct_term_is_scaled_by_the_light_visibility():
    """A uniform black absorber (rgb 0, alpha a): the cones gather no colour,
    so L is the direct term alone, and with one light it must be that
    light's visibility V = o_min times the empty-grid Lambert + Phong sum;
    V itself is (1 - a)^K over the K samples of the unmodified occlusion
    cone toward the light."""
    n = 16
    a = 0.05
    x, nrm, lp, cam = (0.5, 0.25, 0.5), (0.0, 1.0, 0.0), (0.75, 0.5, 0.5), (0.25, 0.5, 0.5)
    pr, nr, mat, cm = one_pixel(x, nrm, cam, albedo=(0.75, 0.5, 0.25), shininess=32.0)
    sp = ShadeParams(*lights(lp, idiff=(1.0, 0.5, 0.25), ispec=(0.375, 0.375, 0.375)),
                     specular_color=(0.875, 0.875, 0.875), occlusion_falloff=False)
    cp = cone_params(light_pos=lp, alpha_thresh=1.0)
    empty = oracle.shade(uniform_mips(n, (0.0, 0.0, 0.0, 0.0)), pr, nr, mat, cm, cp, sp)[0, 0, 0]
    mips = uniform_mips(n, (0.0, 0.0, 0.0, a))
    out = oracle.shade(mips, pr, nr, mat, cm, cp, sp)[0, 0, 0]
    lanes = oracle.cone_lanes(pr, nr, cm, cp.replace(diffuse_dirs=np.zeros((0, 3)), diffuse_weights=np.zeros(0),
                                                       enable_spec=False), n)
    k = int(oracle.march(mips, lanes, cp)["K"][0])
    assert k > 3
    assert out[3] == pytest.approx((1.0 - a) ** k, rel=1e-12)
    np.testing.assert_allclose(out[0:3], out[3] * empty[0:3], rtol=1e-12)


# --- first-hit diffuse cones --------------------------------------------------

def test_first_hit_on_uniform_grids():
    """On a uniform grid every sample equals the texel value: below the
    threshold no cone ever hits; above it every cone hits at its first sample
    and returns the premultiplied colour."""
    n = 16
    d, w = cone_set("six")
    cp = ConeParams(d, w, enable_spec=False, enable_occ=False, alpha_thresh=0.99)
    sp = ShadeParams(np.zeros((0, 3)), np.zeros((0, 3)), np.zeros((0, 3)), specular_brdf=False)
    pr, nr, mat, cm = one_pixel((0.5, 0.5, 0.5), (0.0, 0.0, 1.0), (0.5, 0.5, 3.0))
    # (the specular cone still runs: with no light its BRDF weight is 1, so
    # subtract the specular trace of the pinned forward)
    for a, hit in ((0.005, False), (0.02, True), (1.0, True)):
        c = np.array([0.3, 0.6, 0.9]) * a
        mips = uniform_mips(n, (c[0], c[1], c[2], a))
        out = oracle.shade(mips, pr, nr, mat, cm, cp, sp)[0, 0, 0]
        spec = oracle.trace(mips, pr, nr, cm, cp.replace(enable_spec=True))[0, 0, 0, 4:7]
        diffuse = out[0:3] - spec
        np.testing.assert_allclose(diffuse, c * float(np.sum(w, dtype=np.float64)) if hit else 0.0,
                                   rtol=1e-12, atol=1e-15)


# --- occlusion falloff --------------------------------------------------------

def test_falloff_occlusion_on_a_uniform_grid():
    """Uniform alpha a: V = prod_k (1 - a S(t_k)) with S the Hermite step of
    sqrt(t_k) * strength, over the sample distances t_k of the (pinned)
    unmodified occlusion march; strength 0 leaves V = 1 and a huge strength
    gives the unmodified cone."""
    n = 32
    a = 0.05
    mips = uniform_mips(n, (0.01, 0.02, 0.03, a))
    x, nrm = (0.3, 0.3, 0.3), (0.0, 1.0, 0.0)
    lp = (0.75, 0.875, 0.625)
    pr, nr, mat, cm = one_pixel(x, nrm, (0.5, 0.5, 2.0))
    cp = cone_params(light_pos=lp, alpha_thresh=1.0)
    # sample distances of the unmodified occlusion cone toward the light
    lanes = oracle.cone_lanes(pr, nr, cm, cp.replace(diffuse_dirs=np.zeros((0, 3)), diffuse_weights=np.zeros(0),
                                                       enable_spec=False), n)
    rec = oracle.march(mips, lanes, cp, record=True)
    tk = np.array([st[1][0] for st in rec["steps"]])
    base = ShadeParams(*lights(lp, idiff=(0, 0, 0), ispec=(0, 0, 0)), diffuse_first_hit=False, specular_brdf=False)
    for strength in (0.5, 2.0):
        sp = base.replace(shadow_strength=strength)
        vis = oracle.shade(mips, pr, nr, mat, cm, cp, sp)[0, 0, 0, 3]
        expect = np.prod(1.0 - a * oracle.smoothstep(0.0, 1.0, np.sqrt(tk) * strength))
        assert vis == pytest.approx(expect, rel=1e-13)
    assert oracle.shade(mips, pr, nr, mat, cm, cp, base.replace(shadow_strength=0.0))[0, 0, 0, 3] == 1.0
    huge = oracle.shade(mips, pr, nr, mat, cm, cp, base.replace(shadow_strength=1e9))[0, 0, 0, 3]
    assert huge == pytest.approx(1.0 - rec["alpha"][0], rel=1e-13)


# --- consistency with the pinned trace, and light-count invariants -------------

def test_flags_off_reduce_to_the_unmodified_cones():
    """With every variant off and dark lights, L = (1 - O) D.rgb + S.rgb, with
    D, S and O the outputs of the pinned forward trace for the same light."""
    from scenes import random_gbuffer, random_grid
    n = 16
    base = random_grid(n, seed=12, alpha_max=0.3)
    mips = oracle.build_mips(base)
    pr, nr, cam = random_gbuffer(1, 5, 7, seed=13, n=n)
    mat = np.random.default_rng(14).uniform(0, 1, size=pr.shape).astype(np.float32)
    lp = (0.25, 0.75, 0.625)      # exact in float32, as the shading lights are
    cp = cone_params(light_pos=lp)
    sp = ShadeParams(*lights(lp, idiff=(0, 0, 0), ispec=(0, 0, 0)), diffuse_first_hit=False,
                     occlusion_falloff=False, specular_brdf=False)
    out = oracle.shade(mips, pr, nr, mat, cam, cp, sp)
    ref = oracle.trace(mips, pr, nr, cam, cp)
    valid = nr[..., 3] != 0
    expect = (1.0 - ref[..., 7:8]) * ref[..., 0:3] + ref[..., 4:7]
    np.testing.assert_allclose(out[..., 0:3][valid], expect[valid], rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(out[..., 3][valid], 1.0 - ref[..., 7][valid], rtol=1e-12, atol=1e-15)
    assert np.all(out[~valid] == 0)


def test_duplicated_light_doubles_the_light_sums():
    from scenes import random_gbuffer, random_grid
    n = 16
    mips = oracle.build_mips(random_grid(n, seed=22, alpha_max=0.2))
    pr, nr, cam = random_gbuffer(1, 4, 5, seed=23, n=n, invalid_frac=0.0)
    mat = np.random.default_rng(24).uniform(0, 1, size=pr.shape).astype(np.float32)
    mat[..., 3] *= 50
    cp = cone_params()
    one = ShadeParams(*lights((0.4, 0.9, 0.5)))
    two = ShadeParams(*lights((0.4, 0.9, 0.5), (0.4, 0.9, 0.5)))
    none = ShadeParams(np.zeros((0, 3)), np.zeros((0, 3)), np.zeros((0, 3)))
    o1 = oracle.shade(mips, pr, nr, mat, cam, cp, one)
    o2 = oracle.shade(mips, pr, nr, mat, cam, cp, two)
    o0 = oracle.shade(mips, pr, nr, mat, cam, cp, none)
    np.testing.assert_allclose(o2[..., 3], o1[..., 3], rtol=0, atol=0)
    # no light: o_min = 1 and the BRDF sum is empty, so L is the diffuse sum alone
    assert np.all(o0[..., 3] == 1.0)
    diffuse = o0[..., 0:3]
    # L = o_min D + F C_spec + direct with F and direct doubling
    light_part1 = o1[..., 0:3] - o1[..., 3:4] * diffuse
    light_part2 = o2[..., 0:3] - o2[..., 3:4] * diffuse
    np.testing.assert_allclose(light_part2, 2 * light_part1, rtol=1e-12, atol=1e-15)


# --- sample count --------------------------------------------------------------

def _schedule_length(gamma, tmax, p, v0):
    """Samples of a cone of aperture gamma through an empty grid: the t
    recurrence t_0 = t0, d = max(2 t tan(gamma / 2), v0), t += beta d, one
    sample while t <= t_max (written out as a scalar loop)."""
    t, k = float(p.t0), 0
    while t <= tmax:
        d = max(2.0 * t * math.tan(gamma / 2.0), v0)
        t += float(p.step_factor) * d
        k += 1
    return k


@pytest.mark.parametrize("first_hit,falloff", [(True, True), (False, False)])
def test_sample_count_in_an_empty_grid_is_the_schedule_length(first_hit, falloff):
    """Nothing stops a cone early in an empty grid (no first hit, no opacity),
    so the shading pass takes exactly the schedule length of every cone: u
    diffuse, one specular, one occlusion cone per light with t_max = min(max_dist,
    distance to the light)."""
    n = 16
    v0 = 1.0 / n
    mips = uniform_mips(n, (0.0, 0.0, 0.0, 0.0))
    pr, nr, mat, cam = one_pixel((0.3, 0.4, 0.5), (0.0, 0.6, 0.8), (0.5, 0.5, 1.5), rough=0.3)
    p = cone_params(max_dist=0.6)
    sp = ShadeParams(*lights((0.5, 0.9, 0.5), (0.32, 0.45, 0.6)), diffuse_first_hit=first_hit,
                     occlusion_falloff=falloff)
    _, info = oracle.shade(mips, pr, nr, mat, cam, p, sp, return_info=True)
    lanes = oracle.cone_lanes(pr, nr, cam, p.replace(enable_occ=False), n)
    expect = sum(_schedule_length(g, tm, p, v0) for g, tm in zip(lanes["gamma"], lanes["tmax"]))
    o = lanes["o"][0]
    for light in sp.light_pos:
        dist = float(np.linalg.norm(np.asarray(light, np.float64) - o))
        expect += _schedule_length(p.occ_aperture, min(p.max_dist, dist), p, v0)
    assert len(lanes["gamma"]) == len(p.diffuse_dirs) + 1
    assert info["samples"] == expect and expect > 0
    assert not info["ambiguous"].any()
    # the near light cuts its occlusion cone short
    assert _schedule_length(p.occ_aperture, min(p.max_dist, float(np.linalg.norm(sp.light_pos[1] - o))), p, v0) < \
        _schedule_length(p.occ_aperture, p.max_dist, p, v0)


def test_opaque_grid_stops_every_cone_but_the_falloff_one_at_its_first_sample():
    """In a grid of alpha 1 a first-hit diffuse cone takes exactly one sample,
    and so do the accumulated diffuse, specular and plain occlusion cones (alpha
    reaches the threshold at once).  The occlusion cone with falloff scales each
    sample's alpha by a Hermite step of sqrt(t) * strength: with strength 0 the
    step is 0, nothing accumulates, and the cone takes its whole schedule even
    through the opaque grid; with strength 2 it takes more than one sample."""
    n = 16
    mips = uniform_mips(n, (0.2, 0.3, 0.4, 1.0))
    pr, nr, mat, cam = one_pixel((0.3, 0.4, 0.5), (0.0, 0.6, 0.8), (0.5, 0.5, 1.5))
    p = cone_params()
    sp = ShadeParams(*lights((0.5, 0.9, 0.5)), shadow_strength=2.0)
    u = len(p.diffuse_dirs)
    _, plain = oracle.shade(mips, pr, nr, mat, cam, p, sp.replace(occlusion_falloff=False), return_info=True)
    _, acc = oracle.shade(mips, pr, nr, mat, cam, p, sp.replace(diffuse_first_hit=False, occlusion_falloff=False),
                          return_info=True)
    _, fall = oracle.shade(mips, pr, nr, mat, cam, p, sp, return_info=True)
    _, zero = oracle.shade(mips, pr, nr, mat, cam, p, sp.replace(shadow_strength=0.0), return_info=True)
    assert plain["samples"] == u + 2 and acc["samples"] == u + 2
    lanes = oracle.cone_lanes(pr, nr, cam, p.replace(enable_occ=False), n)
    dist = float(np.linalg.norm(np.asarray(sp.light_pos[0], np.float64) - lanes["o"][0]))
    full = _schedule_length(p.occ_aperture, min(p.max_dist, dist), p, 1.0 / n)
    assert zero["samples"] == u + 1 + full
    assert u + 2 < fall["samples"] < u + 1 + full
