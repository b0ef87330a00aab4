"""FP64 CPU oracle of a further light bounce inside the voxel grid.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import or call this
module; only tests/ (and the smoke check / cpu baseline legs) use it.  It
shares no code with the HIP library; it builds on the pinned mip pyramid, cone
lanes and march of vct_oracle.

What it computes (arXiv 2104.00618, Section 6.2.2 "Algorithm Limitations":
bounces beyond the first need a 3D texture of surface normals, with cones
traced again from the voxels that were hit, about their average surface
normal; Section 6.2.4 "Possibilities for Expansion" and Section 5.1.3
"Villegas": indirect light inserted into a further 3D texture, as deferred
voxel cone tracing does with albedo and normal textures from voxelization):

* bounce   from every surface voxel of the direct-light grid, the diffuse
           cones of the cone set are traced through the mip pyramid of that
           grid, about the voxel's average normal, and the voxel's radiance
           becomes its direct light plus its albedo times the gathered light.
* bounces  the same step repeated: each pass gathers from the pyramid of the
           previous pass's grid and adds to the direct light.

Readings (also listed in the repository's design notes):

B1  Surface voxels are those with alpha > 0 whose average normal (the normal
    grid of voxelization, reading V7) has length >= MIN_NORMAL; fragments of
    opposite orientation in one voxel cancel and leave it without a direction.
    Other voxels keep their value.
B2  Cone origin: the voxel centre, offset by normal_offset voxels along the
    unit average normal (reading R4); the tangent frame, cone axes, apertures,
    t0, max_dist, alpha_thresh and step factor are those of the forward trace
    (readings R1-R10); the specular and occlusion cones are not traced.
B3  bounced.rgb = base.rgb + base.a * albedo.rgb * sum_q w_q C_q (premultiplied
    storage: the added light is scaled by the voxel's opacity); alpha is kept.
B4  k bounces: L_0 = base, L_{j+1} = bounce(L_j) with the direct term of B3
    always taken from base (light is re-gathered, never double counted).
"""
from __future__ import annotations

import numpy as np

from .vct_oracle import build_mips, trace

MIN_NORMAL = 1e-2


def surface_mask(base, normal_grid):
    """Voxels that bounce light (B1): [N, N, N] bool."""
    base = np.asarray(base, dtype=np.float64)
    nrm = np.asarray(normal_grid, dtype=np.float64)[..., 0:3]
    return (base[..., 3] > 0) & (np.linalg.norm(nrm, axis=-1) >= MIN_NORMAL)


def voxel_gbuffer(mask, normal_grid, origin=(0.0, 0.0, 0.0), extent=1.0, voxels=None):
    """The surface voxels as a one-row G-buffer (B2): pos_rough [1, 1, M, 4]
    (voxel centre, roughness 0), normal [1, 1, M, 4] (average normal, valid 1)
    and the (z, y, x) index of every entry.  ``voxels`` (an [M, 3] array of
    (z, y, x)) restricts it to those voxels, in that order."""
    n = mask.shape[0]
    if voxels is None:
        z, y, x = np.nonzero(mask)
    else:
        v = np.asarray(voxels, dtype=np.int64).reshape(-1, 3)
        z, y, x = v[:, 0], v[:, 1], v[:, 2]
    o = np.asarray(origin, dtype=np.float32).astype(np.float64)
    v0 = float(np.float32(extent)) / n
    m = len(z)
    pr = np.zeros((1, 1, m, 4))
    pr[0, 0, :, 0] = o[0] + (x + 0.5) * v0
    pr[0, 0, :, 1] = o[1] + (y + 0.5) * v0
    pr[0, 0, :, 2] = o[2] + (z + 0.5) * v0
    nr = np.zeros((1, 1, m, 4))
    nr[0, 0, :, 0:3] = np.asarray(normal_grid, dtype=np.float64)[z, y, x, 0:3]
    nr[0, 0, :, 3] = 1.0
    return pr, nr, (z, y, x)


def bounce(base, normal_grid, albedo_grid, params, levels=None, origin=(0.0, 0.0, 0.0), extent=1.0,
           gather_from=None, mips=None, voxels=None, return_info=False, sampler=None):
    """One bounce (B1-B3): [N, N, N, 4] float64.

    gather_from: the grid whose pyramid the cones march through (default
    base; B4 passes the previous bounce); mips: that pyramid given directly
    (e.g. a decoded reduced-precision one); sampler: replaces the isotropic
    sample (an anisotropic pyramid's).  voxels: optional [M, 3] (z, y, x)
    list; then only those voxels are computed and the result is their [M, 4]
    values (for sampled checks of large grids)."""
    base = np.asarray(base, dtype=np.float64)
    if mips is None:
        src = base if gather_from is None else np.asarray(gather_from, dtype=np.float64)
        mips = build_mips(src, levels)
    mask = surface_mask(base, normal_grid)
    pr, nr, (z, y, x) = voxel_gbuffer(mask, normal_grid, origin, extent, voxels)
    # surface test of sampled voxels (all listed voxels are surface ones when voxels is None)
    live = mask[z, y, x]
    nr[0, 0, ~live, 3] = 0.0
    cone = params.replace(enable_spec=False, enable_occ=False)
    cam = np.zeros((1, 3))
    out, info = trace(mips, pr, nr, cam, cone, origin, extent, return_info=True, sampler=sampler)
    gathered = out[0, 0, :, 0:3]
    alb = np.asarray(albedo_grid, dtype=np.float64)[z, y, x, 0:3]
    vals = base[z, y, x].copy()
    vals[:, 0:3] += base[z, y, x, 3:4] * alb * gathered
    amb = info["ambiguous"][0, 0]
    if voxels is not None:
        return (vals, amb & live) if return_info else vals
    res = base.copy()
    res[z, y, x] = vals
    if not return_info:
        return res
    amb_grid = np.zeros(mask.shape, dtype=bool)
    amb_grid[z, y, x] = amb
    return res, {"surface": mask, "ambiguous": amb_grid, "samples": info["samples"]}


def bounces(base, normal_grid, albedo_grid, params, k, levels=None, origin=(0.0, 0.0, 0.0), extent=1.0):
    """k >= 0 bounces (B4)."""
    cur = np.asarray(base, dtype=np.float64)
    for _ in range(k):
        cur = bounce(base, normal_grid, albedo_grid, params, levels, origin, extent, gather_from=cur)
    return cur
