"""FP64 CPU oracle of anisotropic (six-direction) mip pyramids and of the
forward cone trace that samples them.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import or call this
module; only tests/ use it.  It shares no code with the HIP library; it builds
on the pinned sampler, cone lanes and march of vct_oracle.

What it computes (arXiv 2104.00618, Section 5.1.3 "Villegas": the mipmaps are
generated with anisotropic filtering, which is said to give cone traces more
precise results; the thesis gives no formula, so the usual directional
pre-integration of voxel cone tracing is taken):

* build_aniso_mips  six pyramids, one per axis direction (+x, -x, +y, -y, +z,
                    -z), sharing level 0 (the base grid).  A texel of level
                    l + 1 in direction d composites its two children along the
                    axis of d front to back as seen by a ray travelling along d
                    (c = c_f + (1 - a_f) c_b, a = a_f + (1 - a_f) a_b), and
                    averages the four such pairs of its 2 x 2 x 2 children.
* sample_aniso      for a cone with unit axis w: the sum over the three axes of
                    w_a^2 times the quadrilinear sample of the pyramid whose
                    direction is sign(w_a) along axis a.
* trace_aniso       the forward trace (readings R1-R12) with that sampler.

Readings (also listed in the repository's design notes):

A1  Directions are ordered +x, -x, +y, -y, +z, -z; "+x" is the pyramid read by
    cones travelling toward +x, whose front child is the one with the smaller
    x.  Level l + 1 of direction d is built from level l of the same
    direction (level 0 being the shared base grid).
A2  The directional weights are the squared axis components (they sum to 1 for
    a unit axis, so a sample stays a convex combination); a zero component
    takes the + pyramid with weight 0.
A3  The LOD, step schedule, clamp-to-edge taps and compositing are those of
    the isotropic trace; at level 0 every direction reads the same texels, so a
    sample below LOD 1 blends the base grid with the directional level 1.
"""
from __future__ import annotations

import numpy as np

from .vct_oracle import assemble, cone_lanes, march, sample

DIRECTIONS = ("+x", "-x", "+y", "-y", "+z", "-z")


def _pair_composite(m, axis, front_even):
    """Front-to-back composite of the two children along array axis `axis`."""
    ev = np.take(m, np.arange(0, m.shape[axis], 2), axis=axis)
    od = np.take(m, np.arange(1, m.shape[axis], 2), axis=axis)
    f, b = (ev, od) if front_even else (od, ev)
    out = np.empty_like(f)
    out[..., 0:3] = f[..., 0:3] + (1.0 - f[..., 3:4]) * b[..., 0:3]
    out[..., 3] = f[..., 3] + (1.0 - f[..., 3]) * b[..., 3]
    return out


def _pair_mean(m, axis):
    ev = np.take(m, np.arange(0, m.shape[axis], 2), axis=axis)
    od = np.take(m, np.arange(1, m.shape[axis], 2), axis=axis)
    return 0.5 * (ev + od)


def build_aniso_mips(base, levels=None):
    """[pyramid of direction d for d in DIRECTIONS], each a list of float64
    [N_l, N_l, N_l, 4] levels ([z][y][x][rgba]); level 0 is base in all six."""
    m0 = np.asarray(base, dtype=np.float64)
    n = m0.shape[0]
    lmax = int(round(np.log2(n))) + 1
    levels = lmax if levels is None else int(levels)
    assert 1 <= levels <= lmax
    out = []
    for d in range(6):
        axis = 2 - d // 2                  # x is array axis 2, y 1, z 0
        front_even = d % 2 == 0
        pyr = [m0]
        for _ in range(1, levels):
            m = _pair_composite(pyr[-1], axis, front_even)
            for other in (0, 1, 2):
                if other != axis:
                    m = _pair_mean(m, other)
            pyr.append(m)
        out.append(pyr)
    return out


def sample_aniso(amips, p, lam, w, origin=(0.0, 0.0, 0.0), extent=1.0):
    """Directionally weighted quadrilinear sample [m, 4] at positions p with
    LOD lam for cones with unit axes w [m, 3] (A2)."""
    w = np.asarray(w, dtype=np.float64)
    s = np.zeros((len(lam), 4))
    for a in range(3):
        wa = w[:, a]
        for d, sel in ((2 * a, wa >= 0), (2 * a + 1, wa < 0)):
            if sel.any():
                s[sel] += (wa[sel] ** 2)[:, None] * sample(amips[d], p[sel], lam[sel], origin, extent)
    return s


def aniso_sampler(amips, origin=(0.0, 0.0, 0.0), extent=1.0):
    """The sampler hook of the march, shading and bounce oracles for an
    anisotropic pyramid (pass amips[0] as their isotropic ``mips``: it gives
    the level count and N)."""
    return lambda p, lam, w: sample_aniso(amips, p, lam, w, origin, extent)


def trace_aniso(amips, pos_rough, normal, cam_pos, params, origin=(0.0, 0.0, 0.0), extent=1.0,
                return_info=False):
    """Forward trace [b, h, w, 8] float64 with anisotropic sampling (A3)."""
    n = amips[0][0].shape[0]
    shape = np.asarray(pos_rough).shape[:3]
    lanes = cone_lanes(pos_rough, normal, cam_pos, params, n, origin, extent)
    res = march(amips[0], lanes, params, origin, extent,
                sampler=lambda p, lam, w: sample_aniso(amips, p, lam, w, origin, extent))
    out = assemble(lanes, res, params, shape)
    if not return_info:
        return out
    amb_pix = np.zeros(int(np.prod(shape)), dtype=bool)
    np.logical_or.at(amb_pix, lanes["pix"], res["ambiguous"])
    return out, {"ambiguous": amb_pix.reshape(shape), "samples": int(res["K"].sum()), "K": res["K"]}
