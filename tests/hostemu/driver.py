"""Write one case of the checked CPU build (tests/hostemu/harness.cpp) to a
directory, run the build on it and read its outputs back."""
import os
import subprocess

import numpy as np

DTYPES = {"f32": 0, "f16": 1, "bf16": 2}


def run_case(binary, d, base, pr, nr, cam, p, dtype="f32", levels=None, aniso=False, gout=None, backward=True,
             noalloc=False, n=None, block_origin=0, bounce=None, save_only=False,
             dump_levels=False, shade=None, material=None, origin=(0.0, 0.0, 0.0), extent=1.0, timeout=600):
    os.makedirs(d, exist_ok=True)
    # (block_origin w0: `base` is the corner block [w0, n)^3 of an n^3 grid that is zero elsewhere)
    n = n or base.shape[0]
    levels = levels or int(round(np.log2(n))) + 1
    b, h, w = pr.shape[:3]
    meta = dict(n=n, levels=levels, dtype=DTYPES[dtype], aniso=int(aniso), b=b, h=h, w=w,
                origin0=origin[0], origin1=origin[1], origin2=origin[2], extent=extent,
                n_diffuse=p.n_diffuse, diffuse_aperture=p.diffuse_aperture, enable_spec=int(p.enable_spec),
                enable_occ=int(p.enable_occ), spec_aperture_scale=p.spec_aperture_scale, occ_aperture=p.occ_aperture,
                light0=p.light_pos[0], light1=p.light_pos[1], light2=p.light_pos[2], step_factor=p.step_factor,
                t0=p.t0, normal_offset=p.normal_offset, max_dist=p.max_dist, alpha_thresh=p.alpha_thresh,
                backward=int(backward), noalloc=int(noalloc), dump_levels=int(dump_levels), block_origin=block_origin,
                shade=int(shade is not None), bounce=int(bounce is not None), save_only=int(save_only))
    np.ascontiguousarray(base, np.float32).tofile(f"{d}/base.bin")
    np.ascontiguousarray(pr, np.float32).tofile(f"{d}/pos_rough.bin")
    np.ascontiguousarray(nr, np.float32).tofile(f"{d}/normal.bin")
    np.ascontiguousarray(cam, np.float32).tofile(f"{d}/cam.bin")
    np.ascontiguousarray(p.diffuse_dirs, np.float32).tofile(f"{d}/dirs.bin")
    np.ascontiguousarray(p.diffuse_weights, np.float32).tofile(f"{d}/weights.bin")
    if backward and not save_only:
        np.ascontiguousarray(gout, np.float32).tofile(f"{d}/gout.bin")
    if bounce is not None:
        nrm_grid, alb_grid = bounce
        np.ascontiguousarray(nrm_grid, np.float32).tofile(f"{d}/normal_grid.bin")
        np.ascontiguousarray(alb_grid, np.float32).tofile(f"{d}/albedo_grid.bin")
    if shade is not None:
        sp = shade
        meta.update(n_lights=sp.n_lights, diffuse_first_hit=int(sp.diffuse_first_hit),
                    first_hit_alpha=sp.first_hit_alpha, occlusion_falloff=int(sp.occlusion_falloff),
                    shadow_strength=sp.shadow_strength, specular_brdf=int(sp.specular_brdf),
                    grace_per_shininess=sp.grace_per_shininess, shininess_falloff=sp.shininess_falloff)
        L = np.concatenate([sp.light_pos, sp.light_diffuse, sp.light_specular], axis=1)
        np.ascontiguousarray(L, np.float32).tofile(f"{d}/lights.bin")
        np.ascontiguousarray(material, np.float32).tofile(f"{d}/material.bin")
    with open(f"{d}/meta.txt", "w") as f:
        for k, v in meta.items():
            f.write(f"{k} {float(v)!r}\n")
    r = subprocess.run([binary, d], capture_output=True, text=True, timeout=timeout)
    if r.returncode != 0 or "EMU OK" not in r.stdout:
        raise RuntimeError(f"checked build failed ({r.returncode}):\n{r.stdout[-2000:]}\n{r.stderr[-4000:]}")
    res = {"trace": np.fromfile(f"{d}/trace.bin", np.float32).reshape(b, h, w, 8),
           "count": np.fromfile(f"{d}/count.bin", np.uint64), "log": r.stderr}
    if backward:
        res["save"] = np.fromfile(f"{d}/save.bin", np.float32).reshape(b, h, w, 8)
    if backward and not save_only:
        m = n - block_origin
        res["grad"] = np.fromfile(f"{d}/grad.bin", np.float32).reshape(m, m, m, 4)
        if block_origin:
            res["grad_outside_nonzero"] = int(np.fromfile(f"{d}/grad_outside_nonzero.bin", np.uint64)[0])
        if noalloc:
            res["grad_noalloc"] = np.fromfile(f"{d}/grad_noalloc.bin", np.float32).reshape(n, n, n, 4)
    if shade is not None:
        res["shade"] = np.fromfile(f"{d}/shade.bin", np.float32).reshape(b, h, w, 4)
    if bounce is not None:
        res["bounce"] = np.fromfile(f"{d}/bounce.bin", np.float32).reshape(n, n, n, 4)
    if dump_levels:
        res["levels"] = [[np.fromfile(f"{d}/level_{di}_{l}.bin", np.float32).reshape((n >> l,) * 3 + (4,))
                          for l in range(levels)] for di in range(6 if aniso else 1)]
    return res


def run_voxelize(binary, d, tris, colors, n, lights, ambient=0.1, diffuse=1.0, surface=True, timeout=600):
    """vct_voxelize through the checked build; returns base (and normal, albedo) as [n, n, n, 4]."""
    os.makedirs(d, exist_ok=True)
    tris = np.ascontiguousarray(tris, np.float32).reshape(-1, 3, 3)
    L = np.array([[*pos, *col, *att] for pos, col, att in lights], np.float32).reshape(-1, 9)
    tris.tofile(f"{d}/tris.bin")
    np.ascontiguousarray(colors, np.float32).tofile(f"{d}/colors.bin")
    L.tofile(f"{d}/lights.bin")
    with open(f"{d}/vmeta.txt", "w") as f:
        for k, v in dict(n=n, n_tris=len(tris), surface=int(surface), n_lights=len(L), ambient=ambient,
                         diffuse=diffuse).items():
            f.write(f"{k} {float(v)!r}\n")
    r = subprocess.run([binary, "--voxelize", d], capture_output=True, text=True, timeout=timeout)
    if r.returncode != 0 or "EMU OK" not in r.stdout:
        raise RuntimeError(f"checked build failed ({r.returncode}):\n{r.stdout[-2000:]}\n{r.stderr[-4000:]}")
    out = [np.fromfile(f"{d}/vox_base.bin", np.float32).reshape(n, n, n, 4)]
    if surface:
        out += [np.fromfile(f"{d}/vox_{k}.bin", np.float32).reshape(n, n, n, 4) for k in ("normal", "albedo")]
    return out
