"""FP64 / exact-integer CPU oracle of GPU voxelization with direct-light
injection.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import or call this
module; only tests/ use it.  It shares no code with the HIP library.

What it computes (arXiv 2104.00618, Section 4.4 "Voxelization Process" and
Section 5.4.4 "Voxelization"): every triangle is rasterized once, along its
dominant axis (the largest component of its normal), by an orthographic
projection onto an N x N viewport; every fragment (a pixel centre inside the
projected triangle) is the voxel (pixel, floor(depth)) and receives the
direct light of the surface point (the Phong model without its glossy term,
with the triangle's own normal and distance attenuation), with alpha 1.
Voxels no fragment reaches stay (0, 0, 0, 0).

Readings (also listed in the repository's design notes):

V1  Rasterization: vertices are snapped to 1/256 of a voxel (8 subpixel
    bits) as round((p - origin) * (256 N / extent)) in float32 arithmetic;
    coverage is decided on the snapped vertices by exact integer edge
    functions at the pixel centres, a centre on an edge belonging to the
    triangle only when the edge (counter-clockwise orientation) runs upward,
    or horizontally leftward (so a shared edge is covered once); triangles of
    zero projected area produce nothing.
V2  Dominant axis: largest |n| component of the snapped normal, ties to x,
    then y, then z; the projection frame follows the thesis's swizzles
    (x-dominant (z, y | x), y-dominant (x, z | y), z-dominant (x, y | z)).
V3  Depth: the voxel layer is floor(w) of the depth w of the snapped plane at
    the pixel centre, computed exactly; fragments outside [0, N) are dropped.
V4  Several fragments in one voxel: their colours are averaged (the thesis's
    imageStore keeps an unspecified one; an average is deterministic).
V5  Direct light per fragment: colour * sum_l (ambient + diffuse max(0, N.L_l))
    light_l / (c_l + l_l d_l + q_l d_l^2), N the unit normal of the original
    (unsnapped) triangle as wound, L_l and d_l the unit direction and
    distance from the fragment to light l, the fragment being the pixel
    centre at depth w mapped back to world units.
V6  Triangles with a non-finite vertex, or a snapped coordinate beyond
    +-2^19 subpixel units, are skipped (the exact arithmetic's range).
V7  Surface attributes (for further bounces, which need a texture of surface
    normals): per voxel the average of its fragments' unit triangle normals
    (not renormalized) and of their triangle colours, with w = 1 where a
    fragment landed.
"""
from __future__ import annotations

import numpy as np

SUB = 256                # subpixels per voxel
COORD_LIMIT = 1 << 19    # |snapped coordinate| bound


def snap(tris, n, origin=(0.0, 0.0, 0.0), extent=1.0):
    """Snapped integer vertices [T, 3, 3] (float32 arithmetic, round half to
    even), and a validity mask [T] (V6)."""
    t = np.asarray(tris, dtype=np.float32)
    o = np.asarray(origin, dtype=np.float32)
    scale = np.float32(SUB * n / float(np.float32(extent)))
    finite = np.all(np.isfinite(t), axis=(1, 2))
    with np.errstate(invalid="ignore", over="ignore"):
        u = np.rint((t - o) * scale)
    ok = finite & np.all(np.abs(np.where(np.isfinite(u), u, 0)) <= COORD_LIMIT, axis=(1, 2))
    u = np.where(ok[:, None, None], u, 0).astype(np.int64)
    return u, ok


_SWIZZLE = {0: (2, 1, 0), 1: (0, 2, 1), 2: (0, 1, 2)}   # (X2, Y2, W) source axes per dominant axis


def _top_left(dx, dy):
    return (dy > 0) | ((dy == 0) & (dx < 0))


def fragments(tri_snapped, n):
    """Fragments of one snapped triangle: (vx, vy, vz, wnum, wden) arrays
    with voxel indices and the exact depth w = wnum / wden in subpixel
    units, plus the pixel centres (X2, Y2) and the swizzle."""
    A, B, C = (tri_snapped[i].astype(object) for i in range(3))   # exact Python integers
    nrm = np.cross((B - A).astype(np.int64), (C - A).astype(np.int64))
    dom = int(np.argmax(np.abs(nrm)))          # first maximal component: x, then y, then z
    sw = _SWIZZLE[dom]
    a = [int(A[i]) for i in sw]
    b = [int(B[i]) for i in sw]
    c = [int(C[i]) for i in sw]
    area = (b[0] - a[0]) * (c[1] - a[1]) - (b[1] - a[1]) * (c[0] - a[0])
    if area == 0:
        return None
    if area < 0:
        b, c = c, b
    xs = [a[0], b[0], c[0]]
    ys = [a[1], b[1], c[1]]
    h = SUB // 2
    i0 = max(0, -((h - min(xs)) // SUB))      # ceil((min - h) / SUB)
    i1 = min(n - 1, (max(xs) - h) // SUB)
    j0 = max(0, -((h - min(ys)) // SUB))
    j1 = min(n - 1, (max(ys) - h) // SUB)
    if i1 < i0 or j1 < j0:
        return None
    I, J = np.meshgrid(np.arange(i0, i1 + 1, dtype=np.int64), np.arange(j0, j1 + 1, dtype=np.int64), indexing="xy")
    PX = I.ravel() * SUB + h
    PY = J.ravel() * SUB + h
    inside = np.ones(PX.shape, dtype=bool)
    for (p, q) in ((a, b), (b, c), (c, a)):
        dx, dy = q[0] - p[0], q[1] - p[1]
        e = dx * (PY - p[1]) - dy * (PX - p[0])
        inside &= (e > 0) | ((e == 0) & _top_left(dx, dy))
    PX, PY = PX[inside], PY[inside]
    if PX.size == 0:
        return None
    # plane through the (swizzled) vertices: n' . (P - a) = 0, solved for W
    e1 = np.array([b[0] - a[0], b[1] - a[1], b[2] - a[2]], dtype=object)
    e2 = np.array([c[0] - a[0], c[1] - a[1], c[2] - a[2]], dtype=object)
    nx = e1[1] * e2[2] - e1[2] * e2[1]
    ny = e1[2] * e2[0] - e1[0] * e2[2]
    nw = e1[0] * e2[1] - e1[1] * e2[0]          # = area > 0
    wnum = [int(nw * a[2] - nx * (int(px) - a[0]) - ny * (int(py) - a[1])) for px, py in zip(PX, PY)]
    wnum = np.array(wnum, dtype=object)
    layer = np.array([w // (int(nw) * SUB) for w in wnum], dtype=np.int64)   # floor division (exact)
    keep = (layer >= 0) & (layer < n)
    X2 = (PX[keep] - h) // SUB
    Y2 = (PY[keep] - h) // SUB
    L = layer[keep]
    vox = [None, None, None]
    vox[sw[0]], vox[sw[1]], vox[sw[2]] = X2, Y2, L
    return {"vox": vox, "px": PX[keep], "py": PY[keep], "wnum": wnum[keep], "wden": int(nw), "swizzle": sw}


def voxelize(tris, colors, n, lights, ambient=0.1, diffuse=1.0, origin=(0.0, 0.0, 0.0), extent=1.0,
             return_counts=False, return_surface=False):
    """Base grid [N, N, N, 4] float64 ([z][y][x][rgba]) of the mesh; with
    return_surface also the normal and albedo grids (V7).

    lights: sequence of (position[3], colour[3], attenuation (c, l, q))."""
    snapped, ok = snap(tris, n, origin, extent)
    tris64 = np.asarray(tris, dtype=np.float32).astype(np.float64)
    cols = np.asarray(colors, dtype=np.float32).astype(np.float64)
    acc = np.zeros((n, n, n, 3))
    nacc = np.zeros((n, n, n, 3))
    cacc = np.zeros((n, n, n, 3))
    cnt = np.zeros((n, n, n), dtype=np.int64)
    o = np.asarray(origin, dtype=np.float32).astype(np.float64)
    v0 = float(np.float32(extent)) / n
    for t in np.nonzero(ok)[0]:
        fr = fragments(snapped[t], n)
        if fr is None:
            continue
        v = tris64[t]
        nn = np.cross(v[1] - v[0], v[2] - v[0])
        ln = np.linalg.norm(nn)
        nn = nn / ln if ln > 0 else nn
        # fragment positions in world units
        sub = np.zeros((len(fr["px"]), 3))
        sw = fr["swizzle"]
        sub[:, sw[0]] = fr["px"]
        sub[:, sw[1]] = fr["py"]
        sub[:, sw[2]] = np.array([float(w) for w in fr["wnum"]]) / fr["wden"]
        pos = o[None, :] + sub / SUB * v0
        col = np.zeros((len(pos), 3))
        for lp, lc, att in lights:
            d = np.asarray(lp, dtype=np.float64)[None, :] - pos
            dist = np.linalg.norm(d, axis=1)
            ldir = d / dist[:, None]
            lam = np.maximum(0.0, ldir @ nn)
            a = 1.0 / (att[0] + att[1] * dist + att[2] * dist * dist)
            col += (ambient + diffuse * lam)[:, None] * np.asarray(lc, dtype=np.float64)[None, :] * a[:, None]
        col *= cols[t][None, :]
        z, y, x = fr["vox"][2], fr["vox"][1], fr["vox"][0]
        np.add.at(acc, (z, y, x), col)
        np.add.at(nacc, (z, y, x), np.broadcast_to(nn, col.shape))
        np.add.at(cacc, (z, y, x), np.broadcast_to(cols[t], col.shape))
        np.add.at(cnt, (z, y, x), 1)
    out = np.zeros((n, n, n, 4))
    hit = cnt > 0
    out[hit, 0:3] = acc[hit] / cnt[hit][:, None]
    out[hit, 3] = 1.0
    res = [out]
    if return_counts:
        res.append(cnt)
    if return_surface:
        nrm = np.zeros((n, n, n, 4))
        alb = np.zeros((n, n, n, 4))
        nrm[hit, 0:3] = nacc[hit] / cnt[hit][:, None]
        alb[hit, 0:3] = cacc[hit] / cnt[hit][:, None]
        nrm[hit, 3] = alb[hit, 3] = 1.0
        res += [nrm, alb]
    return tuple(res) if len(res) > 1 else out
