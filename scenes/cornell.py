"""Seeded procedural Cornell-box scenes and analytic G-buffers.

This module only manufactures inputs: a premultiplied RGBA voxel grid of
direct light and a deferred-shading G-buffer.  It contains none of the cone
tracing arithmetic (no mips, no sampling, no compositing), so the FP64 oracle
and the HIP path can both consume its output without sharing method code.

The thesis voxelizes triangle meshes by rasterization and stores the direct
(Lambert/Phong, one bounce) light of each surface voxel with opacity 1
(Chapter 4, "Voxelization Process" and "3D texture storage").  Its scenes and
Stanford meshes are not available, so a procedural stand-in is built here:

* scene cube [0, 1]^3; five walls are the outer voxel layer at x=0, x=1,
  y=0 (floor), y=1 (ceiling) and z=0 (back); the z=1 side is open;
* axis-aligned boxes (snapped to voxel faces) and spheres;
* opacity 1 where the voxel centre lies inside a solid, 0 elsewhere;
* radiance of a surface voxel = albedo * max(0, n.l) * S with one point light
  of unit intensity and no attenuation, S a hard shadow from a nearest-voxel
  march toward the light; interior voxels are (0, 0, 0, 1);
* RGBA stored premultiplied (rgb already multiplied by alpha).

The G-buffer is an analytic pinhole ray cast against the same solids, whose
box faces lie exactly on voxel faces.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

LIGHT_POS = (0.5, 0.95, 0.5)


@dataclasses.dataclass
class Box:
    lo: np.ndarray          # snapped lower corner (voxel face), float64[3]
    hi: np.ndarray          # snapped upper corner, float64[3]
    albedo: np.ndarray      # float64[3]
    roughness: float


@dataclasses.dataclass
class Sphere:
    centre: np.ndarray
    radius: float
    albedo: np.ndarray
    roughness: float


@dataclasses.dataclass
class Scene:
    n: int
    boxes: list
    spheres: list
    wall_albedo: dict       # name -> float64[3]
    wall_roughness: dict    # name -> float
    light: tuple
    base: np.ndarray | None = None   # float32[n, n, n, 4], [z][y][x][rgba]


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _snap_box(lo, hi, n):
    """Snap a box to the voxel faces enclosing exactly the voxels whose
    centres lie inside it (so voxelization and the ray cast agree)."""
    ilo = np.ceil(np.asarray(lo) * n - 0.5).astype(np.int64)
    ihi = np.floor(np.asarray(hi) * n - 0.5).astype(np.int64)
    ilo = np.clip(ilo, 1, n - 2)
    ihi = np.clip(ihi, ilo, n - 2)
    return ilo / n, (ihi + 1) / n


def make_scene(n, seed, n_boxes=(2, 2), n_spheres=(0, 0), box_edge=(0.15, 0.35),
               avoid=None, voxelize=True, device=None):
    """Draw a seeded scene.  ``n_boxes``/``n_spheres`` are inclusive count
    ranges.  ``avoid`` is a list of points (camera eyes) that no solid may
    contain."""
    rng = _rng(seed)
    rho_l, rho_r = rng.uniform(0.6, 0.9, size=2)
    walls = {
        "left": np.array([rho_l, 0.2, 0.2]),
        "right": np.array([0.2, rho_r, 0.2]),
        "floor": np.full(3, rng.uniform(0.2, 0.9)),
        "ceiling": np.full(3, rng.uniform(0.2, 0.9)),
        "back": np.full(3, rng.uniform(0.2, 0.9)),
    }
    wall_rough = {k: float(rng.uniform(0.1, 0.9)) for k in walls}
    avoid = [np.asarray(a, dtype=np.float64) for a in (avoid or [])]
    nb = int(rng.integers(n_boxes[0], n_boxes[1] + 1))
    ns = int(rng.integers(n_spheres[0], n_spheres[1] + 1))
    boxes, spheres = [], []
    v0 = 1.0 / n
    while len(boxes) < nb:
        edge = rng.uniform(box_edge[0], box_edge[1], size=3)
        lo = np.empty(3)
        lo[0] = rng.uniform(v0, 1 - v0 - edge[0])
        lo[1] = v0                       # resting on the floor
        lo[2] = rng.uniform(v0, 1 - v0 - edge[2])
        if rng.uniform() < 0.5:          # some float above the floor
            lo[1] = rng.uniform(v0, 1 - v0 - edge[1] - 0.15)
        slo, shi = _snap_box(lo, lo + edge, n)
        alb = rng.uniform(0.2, 0.9, size=3)
        rough = float(rng.uniform(0.1, 0.9))
        if any(np.all(a >= slo - 2 * v0) and np.all(a <= shi + 2 * v0) for a in avoid):
            continue
        boxes.append(Box(slo, shi, alb, rough))
    while len(spheres) < ns:
        r = rng.uniform(0.06, 0.15)
        c = rng.uniform(v0 + r, 1 - v0 - r, size=3)
        alb = rng.uniform(0.2, 0.9, size=3)
        rough = float(rng.uniform(0.1, 0.9))
        if any(np.linalg.norm(a - c) <= r + 2 * v0 for a in avoid):
            continue
        spheres.append(Sphere(c, float(r), alb, rough))
    sc = Scene(n, boxes, spheres, walls, wall_rough, LIGHT_POS)
    if voxelize:
        sc.base = voxelize_scene(sc, device)
    return sc


def _device(device):
    import torch

    return torch.device(device if device is not None else "cpu")


def _norm3(v):
    """Euclidean length of the rows of an [m, 3] float64 tensor as
    sqrt((x*x + y*y) + z*z): elementwise IEEE operations only, so the result
    is the same bits on any device."""
    import torch

    return torch.sqrt((v[:, 0] * v[:, 0] + v[:, 1] * v[:, 1]) + v[:, 2] * v[:, 2])


def _solid_and_albedo(sc, device=None):
    import torch

    dev = _device(device)
    n = sc.n
    c = (torch.arange(n, dtype=torch.float64, device=dev) + 0.5) / n
    solid = torch.zeros((n, n, n), dtype=torch.bool, device=dev)
    alb = torch.zeros((n, n, n, 3), dtype=torch.float32, device=dev)
    f32 = lambda v: torch.tensor(np.asarray(v, dtype=np.float64), dtype=torch.float64).to(torch.float32).to(dev)  # noqa: E731
    # walls: outer voxel layers (z=0 back, y=0 floor, y=n-1 ceiling, x=0 left, x=n-1 right)
    for name, sl in (("back", (0, slice(None), slice(None))),
                     ("floor", (slice(None), 0, slice(None))),
                     ("ceiling", (slice(None), n - 1, slice(None))),
                     ("left", (slice(None), slice(None), 0)),
                     ("right", (slice(None), slice(None), n - 1))):
        solid[sl] = True
        alb[sl] = f32(sc.wall_albedo[name])
    for b in sc.boxes:
        ilo = np.rint(b.lo * n).astype(int)
        ihi = np.rint(b.hi * n).astype(int)
        sl = (slice(ilo[2], ihi[2]), slice(ilo[1], ihi[1]), slice(ilo[0], ihi[0]))
        solid[sl] = True
        alb[sl] = f32(b.albedo)
    for s in sc.spheres:
        lo = np.maximum(np.floor((s.centre - s.radius) * n).astype(int) - 1, 0)
        hi = np.minimum(np.ceil((s.centre + s.radius) * n).astype(int) + 1, n)
        zz, yy, xx = torch.meshgrid(c[lo[2]:hi[2]], c[lo[1]:hi[1]], c[lo[0]:hi[0]], indexing="ij")
        dx, dy, dz = xx - float(s.centre[0]), yy - float(s.centre[1]), zz - float(s.centre[2])
        inside = (dx * dx + dy * dy) + dz * dz <= s.radius ** 2
        sub = (slice(lo[2], hi[2]), slice(lo[1], hi[1]), slice(lo[0], hi[0]))
        solid[sub] |= inside
        alb[sub] = torch.where(inside[..., None], f32(s.albedo), alb[sub])
    return solid, alb


def _shadow(solid, start, light, n):
    """Hard shadow: march from ``start`` toward the light in steps of half a
    voxel, looking up the nearest voxel; returns 1 where nothing solid is hit.
    Elementwise float64 torch operations on the tensors' device (the same
    bits on the CPU and a GPU)."""
    import torch

    dev = solid.device
    light = torch.tensor(np.asarray(light, dtype=np.float64), device=dev)
    st = start
    occ = solid.reshape(-1)
    delta = light[None, :] - st
    dist = _norm3(delta)
    dirn = delta / torch.clamp(dist, min=1e-12)[:, None]
    step = 0.5 / n
    vis = torch.ones(len(st), dtype=torch.bool, device=dev)
    idx = torch.arange(len(st), device=dev)
    t = torch.zeros(len(st), dtype=torch.float64, device=dev)
    while len(idx):
        p = st[idx] + t[idx, None] * dirn[idx]
        ijk = torch.clamp(torch.floor(p * n).to(torch.int64), 0, n - 1)
        hit = occ[(ijk[:, 2] * n + ijk[:, 1]) * n + ijk[:, 0]]
        vis[idx[hit]] = False
        t[idx] += step
        keep = (~hit) & (t[idx] < dist[idx])
        idx = idx[keep]
    return vis


def voxelize_scene(sc, device=None):
    """Premultiplied RGBA float32 grid [z][y][x][4] of one-bounce direct light
    (numpy).  ``device``: where the torch operations run (default the CPU);
    they are elementwise IEEE operations, so every device gives the same bits."""
    import torch

    n = sc.n
    solid, alb = _solid_and_albedo(sc, device)
    dev = solid.device
    pad = torch.ones((n + 2, n + 2, n + 2), dtype=torch.bool, device=dev)   # outside counts as solid
    pad[1:-1, 1:-1, 1:-1] = solid
    nrm = torch.zeros((n, n, n, 3), dtype=torch.float32, device=dev)
    surf = torch.zeros((n, n, n), dtype=torch.bool, device=dev)
    # (axis in [z,y,x] order, sign) -> unit vector in (x,y,z)
    for ax, comp in ((2, 0), (1, 1), (0, 2)):
        for sgn in (1, -1):
            sl = [slice(1, -1)] * 3
            sl[ax] = slice(1 + sgn, n + 1 + sgn)
            e = solid & ~pad[tuple(sl)]
            surf |= e
            nrm[..., comp] += e.to(torch.float32) * float(sgn)
    base = torch.zeros((n, n, n, 4), dtype=torch.float32, device=dev)
    base[..., 3] = solid.to(torch.float32)
    zi, yi, xi = torch.nonzero(surf, as_tuple=True)
    if len(zi):
        nv = nrm[zi, yi, xi].to(torch.float64)
        nl = _norm3(nv)
        ok = nl > 0
        nv = torch.where(ok[:, None], nv / torch.where(ok, nl, 1.0)[:, None], nv)
        centre = (torch.stack([xi, yi, zi], dim=1).to(torch.float64) + 0.5) / n
        light = torch.tensor(np.asarray(sc.light, dtype=np.float64), device=dev)
        ldir = light[None, :] - centre
        ldir = ldir / torch.clamp(_norm3(ldir), min=1e-12)[:, None]
        lam = torch.clamp((nv[:, 0] * ldir[:, 0] + nv[:, 1] * ldir[:, 1]) + nv[:, 2] * ldir[:, 2], min=0.0)
        lam = lam * ok.to(torch.float64)
        vis = _shadow(solid, centre + (1.5 / n) * nv, sc.light, n)
        rad = alb[zi, yi, xi].to(torch.float64) * (lam * vis.to(torch.float64))[:, None]
        base[zi, yi, xi, 0:3] = rad.to(torch.float32)
    return base.cpu().numpy()


# --------------------------------------------------------------------------
# G-buffer ray cast
# --------------------------------------------------------------------------

def camera_rays(eye, target, h, w, fov_deg=60.0):
    eye = np.asarray(eye, dtype=np.float64)
    fwd = np.asarray(target, dtype=np.float64) - eye
    fwd /= np.linalg.norm(fwd)
    up_w = np.array([0.0, 1.0, 0.0])
    right = np.cross(fwd, up_w)
    right /= np.linalg.norm(right)
    up = np.cross(right, fwd)
    th = math.tan(math.radians(fov_deg) / 2)
    aspect = w / h
    xs = (2 * (np.arange(w) + 0.5) / w - 1) * th * aspect
    ys = (1 - 2 * (np.arange(h) + 0.5) / h) * th
    d = (fwd[None, None, :] + xs[None, :, None] * right[None, None, :]
         + ys[:, None, None] * up[None, None, :])
    d /= np.linalg.norm(d, axis=2, keepdims=True)
    return eye, d.reshape(-1, 3)


def _planes(sc):
    """Inner wall faces and box faces as (axis, value, normal sign, rect lo, rect hi, albedo-free
    roughness).  Rect bounds are in full xyz with the plane axis ignored."""
    n = sc.n
    v0 = 1.0 / n
    out = []
    lo_in = np.array([v0, v0, v0])
    hi_in = np.array([1 - v0, 1 - v0, 1.0])
    for ax, val, sgn, name in ((0, v0, 1, "left"), (0, 1 - v0, -1, "right"),
                               (1, v0, 1, "floor"), (1, 1 - v0, -1, "ceiling"),
                               (2, v0, 1, "back")):
        out.append((ax, val, sgn, lo_in, hi_in, sc.wall_roughness[name]))
    for b in sc.boxes:
        for ax in range(3):
            out.append((ax, b.lo[ax], -1, b.lo, b.hi, b.roughness))
            out.append((ax, b.hi[ax], 1, b.lo, b.hi, b.roughness))
    return out


def render_gbuffer(sc, eye, target, h, w, fov_deg=60.0, device=None):
    """Analytic G-buffer: (pos_rough [h,w,4], normal [h,w,4]) float32 numpy.
    pos_rough = (x, y, z, roughness); normal = (nx, ny, nz, valid).
    Elementwise float64 torch operations on ``device`` (default the CPU); every
    device gives the same bits."""
    import torch

    dev = _device(device)
    o_np, d_np = camera_rays(eye, target, h, w, fov_deg)
    o = torch.tensor(o_np, dtype=torch.float64, device=dev)
    d = torch.from_numpy(d_np).to(dev)
    m = d.shape[0]
    best_t = torch.full((m,), float("inf"), dtype=torch.float64, device=dev)
    best_n = torch.zeros((m, 3), dtype=torch.float64, device=dev)
    best_r = torch.zeros(m, dtype=torch.float64, device=dev)
    best_plane = torch.zeros(m, dtype=torch.bool, device=dev)
    eps = 1e-9
    for ax, val, sgn, rlo, rhi, rough in _planes(sc):
        dd = d[:, ax]
        t = (float(val) - float(o_np[ax])) / dd
        facing = dd * sgn < 0
        inside = torch.ones(m, dtype=torch.bool, device=dev)
        for a2 in range(3):
            if a2 == ax:
                continue
            pa = float(o_np[a2]) + t * d[:, a2]
            inside &= (pa >= float(rlo[a2]) - eps) & (pa <= float(rhi[a2]) + eps)
        ok = facing & inside & (t > 1e-9) & (t < best_t)
        best_t = torch.where(ok, t, best_t)
        nv = torch.zeros(3, dtype=torch.float64, device=dev)
        nv[ax] = sgn
        best_n[ok] = nv
        best_r[ok] = float(rough)
        best_plane[ok] = True
    for s in sc.spheres:
        oc = o_np - np.asarray(s.centre, dtype=np.float64)
        c = torch.tensor(s.centre, dtype=torch.float64, device=dev)
        bq = (d[:, 0] * float(oc[0]) + d[:, 1] * float(oc[1])) + d[:, 2] * float(oc[2])
        cq = float((oc[0] * oc[0] + oc[1] * oc[1]) + oc[2] * oc[2]) - s.radius ** 2
        disc = bq * bq - cq
        t = -bq - torch.sqrt(torch.clamp(disc, min=0.0))
        ok = (disc >= 0) & (t > 1e-9) & (t < best_t)
        best_t = torch.where(ok, t, best_t)
        p = o[None, :] + t[ok, None] * d[ok]
        nv = (p - c[None, :]) / s.radius
        best_n[ok] = nv / _norm3(nv)[:, None]
        best_r[ok] = s.roughness
        best_plane[ok] = False
    valid = torch.isfinite(best_t)
    pos = torch.where(valid[:, None], o[None, :] + torch.where(valid, best_t, 0.0)[:, None] * d,
                      torch.zeros((), dtype=torch.float64, device=dev))
    pr = torch.zeros((m, 4), dtype=torch.float32, device=dev)
    nr = torch.zeros((m, 4), dtype=torch.float32, device=dev)
    pr[:, 0:3] = pos.to(torch.float32)
    pr[:, 3] = torch.where(valid, best_r, 0.0).to(torch.float32)
    nr[:, 0:3] = best_n.to(torch.float32)
    nr[:, 3] = valid.to(torch.float32)
    # plane hits lie exactly on their (voxel-face) plane: snap away the ray-cast rounding
    for ax in range(3):
        on_plane = valid & best_plane & (best_n[:, ax].abs() == 1.0)
        pr[on_plane, ax] = (torch.round(pos[on_plane, ax] * sc.n) / sc.n).to(torch.float32)
    return pr.cpu().numpy().reshape(h, w, 4), nr.cpu().numpy().reshape(h, w, 4)


def random_camera(seed):
    """Eye inside the box, looking toward the back wall (C1-style cameras)."""
    rng = _rng(seed)
    eye = np.array([rng.uniform(0.3, 0.7), rng.uniform(0.3, 0.7), rng.uniform(0.6, 0.9)])
    tgt = np.array([rng.uniform(0.4, 0.6), rng.uniform(0.4, 0.6), rng.uniform(0.1, 0.3)])
    return eye, tgt
