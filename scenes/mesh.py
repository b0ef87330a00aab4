"""Seeded triangle meshes of the procedural Cornell box (input generator: no
voxelization or shading arithmetic).

The room is the cube [0, 1]^3 with five walls (x = 0 red, x = 1 green, floor,
ceiling and back wall grey; z = 1 open), each a quad of two triangles wound so
that its normal points into the room.  Objects are axis-aligned boxes (12
triangles) and UV spheres (2 * rings * segments triangles minus the pole
caps), wound counter-clockwise seen from outside.  Walls sit a small inset
inside the cube so that their fragments land inside the grid."""
from __future__ import annotations

import numpy as np

INSET = 1e-3


def _quad(a, b, c, d):
    """Two triangles (a, b, c) and (a, c, d) of the quad a-b-c-d."""
    return [(a, b, c), (a, c, d)]


def _walls(rng):
    lo, hi = INSET, 1.0 - INSET
    rho = rng.uniform(0.6, 0.9)
    grey = rng.uniform(0.2, 0.9, size=3)
    P = lambda x, y, z: (x, y, z)  # noqa: E731
    out = []
    # normals into the room: +x, -x, +y (floor), -y (ceiling), +z (back)
    out += [(t, (rho, 0.2, 0.2)) for t in _quad(P(lo, lo, lo), P(lo, hi, lo), P(lo, hi, hi), P(lo, lo, hi))]
    out += [(t, (0.2, rho, 0.2)) for t in _quad(P(hi, lo, lo), P(hi, lo, hi), P(hi, hi, hi), P(hi, hi, lo))]
    out += [(t, (grey[0],) * 3) for t in _quad(P(lo, lo, lo), P(lo, lo, hi), P(hi, lo, hi), P(hi, lo, lo))]
    out += [(t, (grey[1],) * 3) for t in _quad(P(lo, hi, lo), P(hi, hi, lo), P(hi, hi, hi), P(lo, hi, hi))]
    out += [(t, (grey[2],) * 3) for t in _quad(P(lo, lo, lo), P(hi, lo, lo), P(hi, hi, lo), P(lo, hi, lo))]
    return out


def box_triangles(lo, hi):
    """12 triangles of the box [lo, hi], outward normals."""
    x0, y0, z0 = lo
    x1, y1, z1 = hi
    v = [(x0, y0, z0), (x1, y0, z0), (x1, y1, z0), (x0, y1, z0),
         (x0, y0, z1), (x1, y0, z1), (x1, y1, z1), (x0, y1, z1)]
    faces = [(0, 3, 2, 1), (4, 5, 6, 7), (0, 1, 5, 4), (3, 7, 6, 2), (0, 4, 7, 3), (1, 2, 6, 5)]
    out = []
    for a, b, c, d in faces:
        out += _quad(v[a], v[b], v[c], v[d])
    return out


def sphere_triangles(center, radius, rings=12, segments=24):
    """UV sphere, outward normals."""
    cx, cy, cz = center
    th = np.linspace(0.0, np.pi, rings + 1)
    ph = np.linspace(0.0, 2.0 * np.pi, segments + 1)

    def p(i, j):
        return (cx + radius * np.sin(th[i]) * np.cos(ph[j]), cy + radius * np.cos(th[i]),
                cz + radius * np.sin(th[i]) * np.sin(ph[j]))
    out = []
    for i in range(rings):
        for j in range(segments):
            a, b, c, d = p(i, j), p(i + 1, j), p(i + 1, j + 1), p(i, j + 1)
            if i < rings - 1:          # (at the bottom ring b and c are both the pole)
                out.append((a, c, b))
            if i > 0:                  # (at the top ring a and d are both the pole)
                out.append((a, d, c))
    return out


def cornell_mesh(seed=0, n_boxes=3, n_spheres=2, rings=12, segments=24):
    """(triangles float32 [T, 3, 3] world, colours float32 [T, 3])."""
    rng = np.random.default_rng(seed)
    tris = _walls(rng)
    for _ in range(n_boxes):
        size = rng.uniform(0.1, 0.3, size=3)
        lo = rng.uniform(0.05, 0.95 - size)
        lo[1] = 0.0 + INSET
        col = tuple(rng.uniform(0.2, 0.9, size=3))
        tris += [(t, col) for t in box_triangles(tuple(lo), tuple(lo + size))]
    for _ in range(n_spheres):
        r = rng.uniform(0.06, 0.14)
        c = rng.uniform(0.1 + r, 0.9 - r, size=3)
        col = tuple(rng.uniform(0.2, 0.9, size=3))
        tris += [(t, col) for t in sphere_triangles(tuple(c), r, rings, segments)]
    t = np.array([np.array(tr, dtype=np.float64) for tr, _ in tris], dtype=np.float32)
    c = np.array([col for _, col in tris], dtype=np.float32)
    return t, c
