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
* trace_backward_aniso
                    its adjoint with respect to the base grid (step counts
                    held fixed, R12): each sample's gradient goes to its taps
                    in the three pyramids it read, weighted by w_a^2 (to the
                    shared level 0 with the sum of the three), and each
                    direction's level gradients flow down through the
                    transpose of the linearised front-to-back composite into
                    the level below, ending in the shared level 0.

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

from .vct_oracle import assemble, cone_lanes, march, sample, taps, trace_backward

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


def _reduce_adjoint(G, child, axis, front_even):
    """Gradient of the level below from the gradient G [m, m, m, 4] of a
    directional level: parent = (1/4) sum over the four pairs of
    over(f, b) = f + (1 - f.a) b, so a front child receives
    (1/4)(G - e_a (G . b)) and a back child (1/4)(1 - f.a) G."""
    Gu = G
    for ax in range(3):
        if ax != axis:
            Gu = np.repeat(Gu, 2, axis=ax)
    ev = np.take(child, np.arange(0, child.shape[axis], 2), axis=axis)
    od = np.take(child, np.arange(1, child.shape[axis], 2), axis=axis)
    f, b = (ev, od) if front_even else (od, ev)
    gf = 0.25 * Gu
    gf[..., 3] -= 0.25 * np.sum(Gu * b, axis=-1)
    gb = 0.25 * Gu * (1.0 - f[..., 3:4])
    out = np.empty_like(child)
    even = [slice(None)] * 3
    odd = [slice(None)] * 3
    even[axis] = slice(0, None, 2)
    odd[axis] = slice(1, None, 2)
    out[tuple(even)] = gf if front_even else gb
    out[tuple(odd)] = gb if front_even else gf
    return out


def aniso_mip_adjoint(amips, level_grads):
    """dL/d(base) from per-direction level gradients level_grads[d][l] (level 0
    entries are the shared level's, summed over d), walking every direction
    from its top level down."""
    nlev = len(amips[0])
    G0 = sum(level_grads[d][0] for d in range(6))
    for d in range(6):
        axis = 2 - d // 2
        front_even = d % 2 == 0
        g = level_grads[d][nlev - 1].copy() if nlev > 1 else None
        for lv in range(nlev - 1, 0, -1):
            below = _reduce_adjoint(g, amips[d][lv - 1], axis, front_even)
            if lv - 1 == 0:
                G0 = G0 + below
            else:
                g = level_grads[d][lv - 1] + below
    return G0


def trace_backward_aniso(amips, pos_rough, normal, cam_pos, params, grad_out, origin=(0.0, 0.0, 0.0), extent=1.0):
    """Adjoint of trace_aniso with respect to the base grid: [N, N, N, 4] float64."""
    grads = [[np.zeros_like(m) for m in pyr] for pyr in amips]

    def scatter(p, lam, w, gs):
        w2 = w ** 2
        for lev, iz, iy, ix, wt in taps(amips[0], p, lam, origin, extent):
            for lv in np.unique(lev):
                sel = lev == lv
                for a in range(3):
                    if lv == 0:
                        # the three directions read the same level-0 texel
                        np.add.at(grads[0][0], (iz[sel], iy[sel], ix[sel]), (wt[sel] * w2[sel, a])[:, None] * gs[sel])
                        continue
                    for d, sd in ((2 * a, w[:, a] >= 0), (2 * a + 1, w[:, a] < 0)):
                        s2 = sel & sd
                        if s2.any():
                            np.add.at(grads[d][lv], (iz[s2], iy[s2], ix[s2]), (wt[s2] * w2[s2, a])[:, None] * gs[s2])

    return trace_backward(amips[0], pos_rough, normal, cam_pos, params, grad_out, origin, extent,
                          sampler=aniso_sampler(amips, origin, extent), scatter=scatter,
                          adjoint=lambda: aniso_mip_adjoint(amips, grads))
