"""FP64 CPU oracle for the thesis's cone variants and final shading equation.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import or call this
module; only tests/ (and the smoke check / cpu baseline legs) use it.  It
shares no code with the HIP library; it builds on the pinned cone lanes,
sampler and march of vct_oracle.

What it computes (arXiv 2104.00618, Section 5.4.4, "Cone Tracing": the
modified cone functions of the implementation and the shading equation that
combines them):

* occlusion falloff   each sampled alpha is scaled by a Hermite smoothstep
                      from 0 to max_dist of sqrt(distance travelled) times a
                      shadow strength before front-to-back accumulation.
* first-hit diffuse   the march stops at the first sample whose alpha exceeds
                      a threshold (1/100 in the thesis) and returns the colour
                      sampled there.
* specular BRDF       (1 - max(0, gamma - p) / pi)^q, gamma the angle between
                      the specular cone axis and the direction to a light,
                      p = 0.008 pi * shininess the angular grace, q the
                      shininess falloff.
* shade               L = o_min * sum_q w_q C_diff,q
                          + sum_s f_spec,s * C_spec
                          + sum_s V_s (c_d i_d,s (L_s . N) + c_s i_s,s (R_s . w)^shininess),
                      with one occlusion cone per light, V_s = 1 - its
                      accumulated alpha and o_min = min_s V_s.

Parameters are any object with the fields of scenes.configs.ShadeParams.

Readings (also listed in the repository's design notes):

S1  V_s = 1 - A_occ,s (the occlusion cone returns accumulated alpha; a smaller
    V is a stronger shadow, as the thesis states for the multiplied factor).
    With no light, o_min = 1.
S2  The first-hit diffuse cone returns the sampled (premultiplied) rgb of the
    first sample with alpha > threshold, or 0 if no sample qualifies before
    t_max; alpha_thresh does not stop it.  A sample within 1e-6 of the
    threshold marks the pixel ambiguous.
S3  "current_dist" of the falloff is the cone distance t of the sample.
S4  The diffuse sum keeps the configured cone weights w_q (the printed sum has
    none; w_q = 1 reproduces it).
S5  Lambert and Phong dot products are clamped at 0; R_s = reflect(-L_s, N);
    w is the unit direction from the surface point to the camera; L_s the unit
    direction from the surface point to light s; 0^0 = 1.
S6  gamma = atan2(|R x l|, R . l) (the arc cosine of the dot product, in a form
    that stays accurate near 0 and pi).
S7  The thesis traces one specular cone per light because f_spec depends on
    the light; all of them share axis and aperture, so one trace weighted by
    sum_s f_spec,s is the same value.
S8  Flags off give the unmodified cones of Section 4.3.2 (accumulated colour
    for diffuse, accumulated alpha for occlusion, f_spec = 1 once).
"""
from __future__ import annotations

import copy
import math
import numpy as np

from .vct_oracle import AMBIG_T_REL, cone_lanes, march, sample

AMBIG_HIT = 1e-6          # |s.a - first-hit threshold| below this marks a tie


def smoothstep(e0, e1, x):
    """Hermite interpolation: 0 below e0, 1 above e1, h^2 (3 - 2 h) between."""
    h = np.clip((np.asarray(x, dtype=np.float64) - e0) / (e1 - e0), 0.0, 1.0)
    return h * h * (3.0 - 2.0 * h)


def f_spec(axis, ldir, shininess, params):
    """Angular-grace specular BRDF (1 - max(0, gamma - p) / pi)^q (S6)."""
    axis = np.asarray(axis, dtype=np.float64)
    ldir = np.asarray(ldir, dtype=np.float64)
    cr = np.cross(axis, ldir)
    gamma = np.arctan2(np.linalg.norm(cr, axis=-1), np.sum(axis * ldir, axis=-1))
    p = params.grace_per_shininess * np.asarray(shininess, dtype=np.float64)
    return (1.0 - np.maximum(0.0, gamma - p) / math.pi) ** params.shininess_falloff


def _march_variant(mips, lanes, cone_params, mode, shade, origin=(0.0, 0.0, 0.0), extent=1.0, sampler=None):
    """The two modified marches: mode "first_hit" (S2) returns rgb [m,3];
    mode "falloff" returns accumulated alpha [m] with every sample's alpha
    scaled by smoothstep(0, max_dist, sqrt(t) * shadow_strength).  Also
    returns the ambiguity flag and the number of samples taken per lane."""
    n0 = mips[0].shape[0]
    nlev = len(mips)
    v0 = extent / n0
    x, w, gamma, tmax = lanes["o"], lanes["w"], lanes["gamma"], lanes["tmax"]
    beta = float(cone_params.step_factor)
    thresh = float(cone_params.alpha_thresh)
    m = len(gamma)
    t = np.full(m, float(cone_params.t0))
    rgb = np.zeros((m, 3))
    occ = np.zeros(m)
    taken = np.zeros(m, dtype=np.int64)
    amb = (np.abs(t - tmax) < AMBIG_T_REL * np.abs(tmax)) | lanes["tie"]
    active = t <= tmax
    if mode == "falloff":
        active &= occ < thresh
    cap = int(np.ceil(np.max(tmax, initial=0.0) / (beta * v0))) + 4
    it = 0
    while active.any():
        it += 1
        assert it <= cap, "march did not terminate"
        idx = np.nonzero(active)[0]
        ti = t[idx]
        d = np.maximum(2.0 * ti * np.tan(gamma[idx] / 2.0), v0)
        lam = np.clip(np.log2(d / v0), 0.0, nlev - 1)
        p = x[idx] + ti[:, None] * w[idx]
        s = sample(mips, p, lam, origin, extent) if sampler is None else sampler(p, lam, w[idx])
        taken[idx] += 1
        if mode == "first_hit":
            hit = s[:, 3] > shade.first_hit_alpha
            amb[idx] |= np.abs(s[:, 3] - shade.first_hit_alpha) < AMBIG_HIT
            rgb[idx[hit]] = s[hit, 0:3]
            t[idx] = ti + beta * d
            amb[idx] |= np.abs(t[idx] - tmax[idx]) < AMBIG_T_REL * np.abs(tmax[idx])
            active[idx] = (~hit) & (t[idx] <= tmax[idx])
        else:
            a_s = s[:, 3] * smoothstep(0.0, float(cone_params.max_dist), np.sqrt(ti) * shade.shadow_strength)
            occ[idx] = occ[idx] + (1.0 - occ[idx]) * a_s
            t[idx] = ti + beta * d
            if thresh < 1.0:
                amb[idx] |= np.abs(occ[idx] - thresh) < 1e-5
            amb[idx] |= np.abs(t[idx] - tmax[idx]) < AMBIG_T_REL * np.abs(tmax[idx])
            active[idx] = (t[idx] <= tmax[idx]) & (occ[idx] < thresh)
    return (rgb if mode == "first_hit" else occ), amb, taken


def _occlusion_lanes(pos_rough, normal, cone_params, light, n, origin, extent):
    """Occlusion lanes toward one light (the occlusion cone of cone_lanes with
    the light position replaced)."""
    p = copy.copy(cone_params)
    p.light_pos = tuple(float(v) for v in light)
    p.diffuse_dirs = np.zeros((0, 3))
    p.diffuse_weights = np.zeros(0)
    p.enable_spec = False
    p.enable_occ = True
    return cone_lanes(pos_rough, normal, np.zeros((1, 3)), p, n, origin, extent)


def shade(mips, pos_rough, normal, material, cam_pos, cone_params, shade, origin=(0.0, 0.0, 0.0), extent=1.0,
          return_info=False, sampler=None):
    """Shaded radiance and o_min per pixel: [b,h,w,4] float64 = (L.rgb, o_min).

    material [b,h,w,4] = (c_d.rgb, shininess); cone_params supplies the diffuse
    cone set, the specular aperture scale, the occlusion aperture and the march
    parameters (its light_pos and enable flags are not used: every light gets
    an occlusion cone and the specular cone is always traced)."""
    pr = np.asarray(pos_rough, dtype=np.float64)
    nr = np.asarray(normal, dtype=np.float64)
    mat = np.asarray(material, dtype=np.float64).reshape(-1, 4)
    shape = pr.shape[:3]
    b, h, w = shape
    n0 = mips[0].shape[0]
    npix = b * h * w
    flat_pr = pr.reshape(-1, 4)
    flat_nr = nr.reshape(-1, 4)
    valid = flat_nr[:, 3] != 0
    pix = np.nonzero(valid)[0]
    view = np.repeat(np.arange(b), h * w)
    amb = np.zeros(npix, dtype=bool)
    samples = 0                      # cone samples taken by every march (diffuse, specular, occlusion)

    # diffuse + specular lanes (Section 4.2 cone set)
    p = copy.copy(cone_params)
    p.enable_spec = True
    p.enable_occ = False
    lanes = cone_lanes(pos_rough, normal, cam_pos, p, n0, origin, extent)
    nd = len(cone_params.diffuse_dirs)
    wq = np.asarray(cone_params.diffuse_weights, dtype=np.float64)
    dsel = lanes["slot"] < nd
    ssel = lanes["slot"] == nd
    diffuse = np.zeros((npix, 3))
    if dsel.any():
        dl = {k: v[dsel] for k, v in lanes.items()}
        if shade.diffuse_first_hit:
            c, a, k = _march_variant(mips, dl, cone_params, "first_hit", shade, origin, extent, sampler)
        else:
            r = march(mips, dl, cone_params, origin, extent, sampler=sampler)
            c, a, k = r["c"], r["ambiguous"], r["K"]
        samples += int(np.sum(k))
        np.add.at(diffuse, dl["pix"], wq[dl["slot"]][:, None] * c)
        np.logical_or.at(amb, dl["pix"], a)
    sl = {k: v[ssel] for k, v in lanes.items()}
    rs = march(mips, sl, cone_params, origin, extent, sampler=sampler)
    samples += int(np.sum(rs["K"]))
    c_spec = np.zeros((npix, 3))
    c_spec[sl["pix"]] = rs["c"]
    np.logical_or.at(amb, sl["pix"], rs["ambiguous"])
    spec_axis = np.zeros((npix, 3))
    spec_axis[sl["pix"]] = sl["w"]

    # per-light occlusion cones, direct term, specular weights
    x = flat_pr[:, 0:3]
    nn = np.zeros((npix, 3))
    nn[pix] = flat_nr[pix, 0:3] / np.linalg.norm(flat_nr[pix, 0:3], axis=1, keepdims=True)
    cam = np.asarray(cam_pos, dtype=np.float64).reshape(-1, 3)[view]
    wv = cam - x
    wv[pix] /= np.linalg.norm(wv[pix], axis=1, keepdims=True)
    shin = mat[:, 3]
    c_d = mat[:, 0:3]
    c_s = np.asarray(shade.specular_color, dtype=np.float64)[None, :]
    o_min = np.ones(npix)
    direct = np.zeros((npix, 3))
    fsum = np.zeros(npix)
    for s in range(len(shade.light_pos)):
        light = np.asarray(shade.light_pos[s], dtype=np.float64)
        ol = _occlusion_lanes(pos_rough, normal, cone_params, light, n0, origin, extent)
        if shade.occlusion_falloff:
            occ, a, k = _march_variant(mips, ol, cone_params, "falloff", shade, origin, extent, sampler)
        else:
            r = march(mips, ol, cone_params, origin, extent, sampler=sampler)
            occ, a, k = r["alpha"], r["ambiguous"], r["K"]
        samples += int(np.sum(k))
        np.logical_or.at(amb, ol["pix"], a)
        vis = np.ones(npix)
        vis[ol["pix"]] = 1.0 - occ
        o_min = np.minimum(o_min, vis)
        ld = light[None, :] - x
        ld[pix] /= np.linalg.norm(ld[pix], axis=1, keepdims=True)
        ndl = np.sum(nn * ld, axis=1)
        refl = 2.0 * ndl[:, None] * nn - ld
        rdw = np.maximum(0.0, np.sum(refl * wv, axis=1))
        lam = np.maximum(0.0, ndl)
        phong = np.where(shin == 0.0, 1.0, rdw ** shin)
        term = (c_d * np.asarray(shade.light_diffuse[s], dtype=np.float64)[None, :] * lam[:, None]
                + c_s * np.asarray(shade.light_specular[s], dtype=np.float64)[None, :] * phong[:, None])
        direct += vis[:, None] * term
        if shade.specular_brdf:
            fsum += f_spec(spec_axis, ld, shin, shade)
    if not shade.specular_brdf:
        fsum = np.ones(npix)
    out = np.zeros((npix, 4))
    out[pix, 0:3] = (o_min[pix, None] * diffuse[pix] + fsum[pix, None] * c_spec[pix] + direct[pix])
    out[pix, 3] = o_min[pix]
    out = out.reshape(b, h, w, 4)
    if return_info:
        return out, {"ambiguous": amb.reshape(shape), "samples": samples}
    return out
