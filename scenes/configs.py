"""Seeded workload definitions (grid, views, cone set, march parameters).

Pure inputs: the diffuse cone directions here are a table of unit vectors in
the tangent frame (z = surface normal), given to the method as data, as the
thesis does with its front / intermediate / side cone sets (Section 5.4.4,
"Cone Configurations").  Nothing in this file samples, composites or mips.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from . import cornell


@dataclasses.dataclass
class ConeParams:
    """Cone-set and march parameters (the thesis's VoxSettings triple
    (t0, aperture, step factor) per cone class, Section 5.4.4)."""
    diffuse_dirs: np.ndarray            # float32[u, 3], tangent-frame unit vectors
    diffuse_weights: np.ndarray         # float32[u]
    diffuse_aperture: float = math.pi / 3
    enable_spec: bool = True
    enable_occ: bool = True
    spec_aperture_scale: float = math.pi / 3   # aperture = roughness * scale
    occ_aperture: float = math.pi / 3
    light_pos: tuple = cornell.LIGHT_POS
    step_factor: float = 0.5            # beta
    t0: float = 0.001
    normal_offset: float = 1.0          # origin offset along the normal, in voxels
    max_dist: float = 1.0
    alpha_thresh: float = 1.0

    @property
    def n_diffuse(self):
        return int(len(self.diffuse_dirs))

    def replace(self, **kw):
        return dataclasses.replace(self, **kw)


@dataclasses.dataclass
class ShadeParams:
    """Lights, specular colour and the cone-variant flags of the final shading
    pass (Section 5.4.4, "Cone Tracing"): occlusion falloff with a shadow
    strength, first-hit diffuse cones with their alpha threshold, and the
    angular-grace specular BRDF (grace = factor * shininess, exponent q)."""
    light_pos: np.ndarray                       # float32[n, 3]
    light_diffuse: np.ndarray                   # float32[n, 3]
    light_specular: np.ndarray                  # float32[n, 3]
    specular_color: tuple = (1.0, 1.0, 1.0)
    diffuse_first_hit: bool = True
    first_hit_alpha: float = 0.01
    occlusion_falloff: bool = True
    shadow_strength: float = 1.0
    specular_brdf: bool = True
    grace_per_shininess: float = 0.008 * math.pi
    shininess_falloff: float = 8.0

    @property
    def n_lights(self):
        return int(len(self.light_pos))

    def replace(self, **kw):
        return dataclasses.replace(self, **kw)


def scene_lights(count=2, **kw):
    """Shading parameters with `count` (<= 4) point lights: the scene light
    (white) first, then dimmer coloured lights inside the box."""
    pos = np.array([cornell.LIGHT_POS, (0.2, 0.6, 0.8), (0.8, 0.4, 0.3), (0.5, 0.3, 0.9)], np.float32)[:count]
    dif = np.array([(1.0, 1.0, 1.0), (0.5, 0.4, 0.3), (0.2, 0.3, 0.5), (0.3, 0.3, 0.3)], np.float32)[:count]
    spe = np.array([(0.5, 0.5, 0.5), (0.3, 0.3, 0.2), (0.2, 0.2, 0.3), (0.1, 0.1, 0.1)], np.float32)[:count]
    return ShadeParams(pos, dif, spe, **kw)


def random_material(shape, seed):
    """Per-pixel material [b, h, w, 4] = (albedo U[0.2, 0.9]^3, shininess U[1, 64])."""
    rng = np.random.default_rng(seed)
    alb = rng.uniform(0.2, 0.9, size=tuple(shape) + (3,))
    shin = rng.uniform(1.0, 64.0, size=tuple(shape) + (1,))
    return np.concatenate([alb, shin], -1).astype(np.float32)


def front_plus_ring(polar_deg, count, front=True):
    """Unit directions: optional front cone (the normal) plus ``count`` cones at
    ``polar_deg`` from the normal, evenly spaced in azimuth starting at 0."""
    dirs = []
    if front:
        dirs.append((0.0, 0.0, 1.0))
    p = math.radians(polar_deg)
    for k in range(count):
        a = 2 * math.pi * k / count
        dirs.append((math.sin(p) * math.cos(a), math.sin(p) * math.sin(a), math.cos(p)))
    return np.asarray(dirs, dtype=np.float32)


def cone_set(kind):
    """'six': front + 5 at 60 deg (tiles the hemisphere with 60 deg cones);
    'five': front + the thesis's 4 intermediate cones at 45 deg, 90 deg apart."""
    if kind == "six":
        d = front_plus_ring(60.0, 5)
    elif kind == "five":
        d = front_plus_ring(45.0, 4)
    else:
        raise ValueError(kind)
    w = np.full(len(d), 1.0 / len(d), dtype=np.float32)
    return d, w


@dataclasses.dataclass
class Workload:
    name: str
    n: int
    levels: int
    scene: object                       # cornell.Scene (base filled)
    pos_rough: np.ndarray               # float32[b, h, w, 4]
    normal: np.ndarray                  # float32[b, h, w, 4]
    cam_pos: np.ndarray                 # float32[b, 3]
    params: ConeParams
    dtype: str = "f32"

    @property
    def base(self):
        return self.scene.base

    @property
    def shape(self):
        return self.pos_rough.shape[:3]


def _views(sc, cams, h, w, device=None):
    pr, nr = [], []
    for eye, tgt in cams:
        a, b = cornell.render_gbuffer(sc, eye, tgt, h, w, device=device)
        pr.append(a)
        nr.append(b)
    cam = np.asarray([c[0] for c in cams], dtype=np.float32)
    return np.stack(pr), np.stack(nr), cam


C0_CAM = ((0.5, 0.5, 1.866), (0.5, 0.5, 0.0))


def make_workload(name, h=None, w=None, n=None, views=None, device=None):
    """Build one of the named workloads.  ``h``, ``w``, ``n`` and ``views``
    override the sizes (used by the small parity and finite-difference cases).
    ``device``: where the generator's torch operations run (default the CPU;
    a GPU gives the same bits, faster for the large workloads).

    c0     64^3 / 7 levels, 2 boxes, 1 x 256^2 fixed camera, 6+1+1 cones, alpha_thresh 1
    c1     256^3 / 9 levels, 4-8 boxes and spheres, 1 x 1920x1080 camera inside the box,
           5+1+1 cones, alpha_thresh 0.99
    c3gt   128^3 ground truth from the c1 generator, 8 x 512^2, 6+1+1 cones, 0.99
    c3fd   16^3 c0 generator, 2 x 32^2, 6+1+1, 0.99 (finite-difference gradient check)
    c4     512^3 / 10 levels, up to 16 boxes and spheres, 4 x 3840x2160, 5+1+1, 0.99
    """
    if name == "c0":
        n = n or 64
        sc = cornell.make_scene(n, seed=0, n_boxes=(2, 2), device=device)
        cams = [C0_CAM]
        h, w = h or 256, w or 256
        d, wt = cone_set("six")
        params = ConeParams(d, wt, alpha_thresh=1.0)
    elif name == "c1":
        n = n or 256
        cam = cornell.random_camera(101)
        sc = cornell.make_scene(n, seed=1, n_boxes=(2, 4), n_spheres=(2, 4), avoid=[cam[0]], device=device)
        cams = [cam]
        h, w = h or 1080, w or 1920
        d, wt = cone_set("five")
        params = ConeParams(d, wt, alpha_thresh=0.99)
    elif name == "c3gt":
        n = n or 128
        nv = views or 8
        cams = [cornell.random_camera(301 + i) for i in range(nv)]
        sc = cornell.make_scene(n, seed=3, n_boxes=(2, 4), n_spheres=(2, 4),
                                avoid=[c[0] for c in cams], device=device)
        h, w = h or 512, w or 512
        d, wt = cone_set("six")
        params = ConeParams(d, wt, alpha_thresh=0.99)
    elif name == "c3fd":
        n = n or 16
        nv = views or 2
        cams = [C0_CAM] + [cornell.random_camera(400 + i) for i in range(nv - 1)]
        sc = cornell.make_scene(n, seed=4, n_boxes=(2, 2), avoid=[c[0] for c in cams], device=device)
        h, w = h or 32, w or 32
        d, wt = cone_set("six")
        params = ConeParams(d, wt, alpha_thresh=0.99)
    elif name == "c4":
        n = n or 512
        nv = views or 4
        cams = [cornell.random_camera(501 + i) for i in range(nv)]
        sc = cornell.make_scene(n, seed=5, n_boxes=(4, 8), n_spheres=(4, 8),
                                avoid=[c[0] for c in cams], device=device)
        h, w = h or 2160, w or 3840
        d, wt = cone_set("five")
        params = ConeParams(d, wt, alpha_thresh=0.99)
    else:
        raise ValueError(name)
    pr, nr, cam = _views(sc, cams, h, w, device)
    levels = int(round(math.log2(n))) + 1
    return Workload(name, n, levels, sc, pr, nr, cam, params)


def random_grid(n, seed, alpha_max=1.0, rgb_max=1.0):
    """Uniform-random premultiplied RGBA grid (for sampler and gradient pins)."""
    rng = cornell._rng(seed)
    a = rng.uniform(0.0, alpha_max, size=(n, n, n, 1))
    c = rng.uniform(0.0, rgb_max, size=(n, n, n, 3)) * a
    return np.concatenate([c, a], axis=-1).astype(np.float32)


def random_gbuffer(b, h, w, seed, n, invalid_frac=0.1):
    """G-buffer of random interior points with random unit normals (no
    scene): exercises arbitrary cone origins and directions."""
    rng = cornell._rng(seed)
    v0 = 1.0 / n
    pos = rng.uniform(2 * v0, 1 - 2 * v0, size=(b, h, w, 3))
    nrm = rng.normal(size=(b, h, w, 3))
    nrm /= np.linalg.norm(nrm, axis=-1, keepdims=True)
    rough = rng.uniform(0.1, 0.9, size=(b, h, w, 1))
    valid = (rng.uniform(size=(b, h, w, 1)) >= invalid_frac).astype(np.float64)
    pr = np.concatenate([pos, rough], -1).astype(np.float32)
    nr = np.concatenate([nrm, valid], -1).astype(np.float32)
    cam = rng.uniform(0.2, 0.8, size=(b, 3)).astype(np.float32)
    return pr, nr, cam
