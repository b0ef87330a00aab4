"""FP64 CPU oracle for the voxel-cone-tracing hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import or call this
module; only tests/, the smoke check in __graft_entry__ and the cpu_baseline
leg of bench.py use it.  It shares no code with the HIP library.

What it computes (arXiv 2104.00618, "Real-Time Global Illumination Using
OpenGL And Voxel Cone Tracing"):

* build_mips      the mip pyramid of the voxel grid: each level halves every
                  side and is the mean of the 8 children ("Texture Filtering",
                  Section 4.3.3: bilinear minification at a ratio of exactly 2;
                  mips generated after voxelization, Section 4.5 summary and
                  Section 5.4.4 "Voxelization").
* sample          the volume sampler: texture lookup at position p with a LOD
                  from the cone diameter, trilinear inside a level and linear
                  between the two nearest levels (Section 4.3.3 and the colour
                  supersampler of Section 4.5).
* trace           per G-buffer pixel, u diffuse cones, one specular cone and
                  one occlusion cone (Section 4.2, component merging; Section
                  5.4.4, cone configurations), each a volume ray march with
                  front-to-back accumulation (Section 4.3.2, the cone-trace
                  function, with d = 2 t tan(gamma/2) and t += beta d).
* trace_backward  the exact adjoint of trace with the step count K of every
                  cone held fixed, into the base grid.

Readings where the paper is silent, garbled or inconsistent (each also listed
in the design notes of the repository):

R1  compositing is premultiplied front to back: c += (1 - alpha) c_s,
    alpha += (1 - alpha) alpha_s, where c_s is the (premultiplied) sampled
    colour.  The printed colour update rescales the accumulated colour by
    alpha and applies the sample alpha twice; it is read as the standard
    premultiplied form, whose alpha update matches the printed one.
R2  LOD lambda = log2(d / v0), v0 = extent / N the base voxel size (the printed
    log2(diameter / tex_size) mixes scene units with a texel count).
R3  d = max(2 t tan(gamma/2), v0): the LOD is clamped at 0 anyway, and the
    floor guarantees progress for narrow cones near the apex.
R4  cone origin o = x + n * normal_offset * v0; the march starts at t = t0.
R5  texel centres at (i + 1/2) v_l, lambda clamped to [0, L-1], clamp-to-edge
    addressing.
R6  L = log2 N + 1 levels by default (64^3 -> 7 levels, as in Section 5.4.4).
R7  a sample is taken at t_k iff t_k <= t_max and alpha_k < alpha_thresh.
R8  occlusion cone toward the light, t_max = min(max_dist, |light - o|),
    output O = accumulated alpha.
R9  specular axis = reflect(normalize(x - cam), n), aperture = roughness * scale.
R10 tangent frame a = (1,0,0) if |n_y| > 0.9 else (0,1,0); t = normalize(a x n);
    b = n x t; diffuse axis = normalize(t d_x + b d_y + n d_z); D is the
    weighted sum of the diffuse cones (weights given as input).
R11 pixels with normal.w == 0 produce 0 and receive no gradient.
R12 gradients hold every cone's sample count K fixed (the output is a
    polynomial in the grid between termination changes).
"""
from __future__ import annotations

import math

import numpy as np

AMBIG_ALPHA = 1e-5      # |alpha_k - alpha_thresh| below this marks a tie
AMBIG_T_REL = 1e-6      # |t_k - t_max| below this * t_max marks a tie
AMBIG_FRAME = 1e-6      # ||n_y| - 0.9| below this marks a tangent-frame tie (R10)


# ---------------------------------------------------------------------------
# mips (Section 4.3.3 "Texture Filtering"; Section 5.4.4 "Voxelization")
# ---------------------------------------------------------------------------

def build_mips(base, levels=None):
    """Return [M_0, ..., M_{L-1}] as float64 arrays [N_l, N_l, N_l, 4]
    ([z][y][x][rgba]).  M_{l+1} is the mean of the 2x2x2 children in M_l."""
    m0 = np.asarray(base, dtype=np.float64)
    n = m0.shape[0]
    lmax = int(round(math.log2(n))) + 1
    levels = lmax if levels is None else int(levels)
    assert 1 <= levels <= lmax
    mips = [m0]
    for _ in range(1, levels):
        m = mips[-1]
        children = [m[dz::2, dy::2, dx::2] for dz in (0, 1) for dy in (0, 1) for dx in (0, 1)]
        total = children[0].copy()
        for ch in children[1:]:
            total += ch
        mips.append(total / 8.0)
    return mips


def mip_adjoint(level_grads):
    """Transpose of build_mips: G_{L-1} = g_{L-1}; G_l = g_l + (each child
    receives 1/8 of its parent's G_{l+1}).  Returns G_0."""
    g = np.array(level_grads[-1], dtype=np.float64)
    for gl in reversed(level_grads[:-1]):
        up = np.repeat(np.repeat(np.repeat(g, 2, axis=0), 2, axis=1), 2, axis=2)
        g = np.asarray(gl, dtype=np.float64) + up / 8.0
    return g


# ---------------------------------------------------------------------------
# sampler (Section 4.3.3; colour supersampler of Section 4.5)
# ---------------------------------------------------------------------------

def taps(mips, p, lam, origin=(0.0, 0.0, 0.0), extent=1.0):
    """The 16 texel taps of a quadrilinear lookup at world positions p [m,3]
    with LOD lam [m].  Returns a list of (level[m], iz[m], iy[m], ix[m],
    weight[m]) whose weighted texel sum is the sample."""
    p = np.asarray(p, dtype=np.float64)
    lam = np.asarray(lam, dtype=np.float64)
    nlev = len(mips)
    n0 = mips[0].shape[0]
    l0 = np.floor(lam).astype(np.int64)
    l1 = np.minimum(l0 + 1, nlev - 1)
    f = lam - l0
    out = []
    for lev, lw in ((l0, 1.0 - f), (l1, f)):
        nl = (n0 >> lev).astype(np.float64)
        u = (p - np.asarray(origin, dtype=np.float64)[None, :]) / extent * nl[:, None] - 0.5
        i0 = np.floor(u).astype(np.int64)
        phi = u - i0
        for dz in (0, 1):
            for dy in (0, 1):
                for dx in (0, 1):
                    hi = (n0 >> lev) - 1
                    ix = np.clip(i0[:, 0] + dx, 0, hi)
                    iy = np.clip(i0[:, 1] + dy, 0, hi)
                    iz = np.clip(i0[:, 2] + dz, 0, hi)
                    w = ((phi[:, 0] if dx else 1.0 - phi[:, 0])
                         * (phi[:, 1] if dy else 1.0 - phi[:, 1])
                         * (phi[:, 2] if dz else 1.0 - phi[:, 2]))
                    out.append((lev, iz, iy, ix, lw * w))
    return out


def sample(mips, p, lam, origin=(0.0, 0.0, 0.0), extent=1.0):
    """Quadrilinear sample [m, 4] (premultiplied rgb, alpha)."""
    s = np.zeros((len(lam), 4))
    for lev, iz, iy, ix, w in taps(mips, p, lam, origin, extent):
        vals = np.empty((len(lev), 4))
        for l in np.unique(lev):
            sel = lev == l
            vals[sel] = mips[l][iz[sel], iy[sel], ix[sel]]
        s += w[:, None] * vals
    return s


# ---------------------------------------------------------------------------
# per-pixel cone set (Section 4.2; Section 5.4.4)
# ---------------------------------------------------------------------------

def _normalize(v):
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def cone_lanes(pos_rough, normal, cam_pos, params, n, origin=(0.0, 0.0, 0.0), extent=1.0):
    """Expand a G-buffer into one lane per (pixel, cone).

    Cones per pixel, in order: q = 0..u-1 diffuse, then specular (if enabled),
    then occlusion (if enabled).  Returns a dict of float64/int arrays over
    lanes of valid pixels, plus the pixel index and cone slot of each lane."""
    pr = np.asarray(pos_rough, dtype=np.float64)
    nr = np.asarray(normal, dtype=np.float64)
    b, h, w = pr.shape[:3]
    pr = pr.reshape(-1, 4)
    nr = nr.reshape(-1, 4)
    view = np.repeat(np.arange(b), h * w)
    valid = nr[:, 3] != 0
    pix = np.nonzero(valid)[0]
    x = pr[pix, 0:3]
    rough = pr[pix, 3]
    nn = _normalize(nr[pix, 0:3])
    v0 = extent / n
    o = x + nn * (params.normal_offset * v0)
    # tangent frame (R10)
    a = np.where((np.abs(nn[:, 1]) > 0.9)[:, None], np.array([1.0, 0.0, 0.0]), np.array([0.0, 1.0, 0.0]))
    tt = _normalize(np.cross(a, nn))
    bb = np.cross(nn, tt)
    lanes = {k: [] for k in ("pix", "slot", "o", "w", "gamma", "tmax", "tie")}
    frame_tie = np.abs(np.abs(nn[:, 1]) - 0.9) < AMBIG_FRAME
    dirs = np.asarray(params.diffuse_dirs, dtype=np.float64)
    m = len(pix)
    for q in range(len(dirs)):
        dq = dirs[q]
        wq = _normalize(tt * dq[0] + bb * dq[1] + nn * dq[2])
        lanes["pix"].append(pix)
        lanes["slot"].append(np.full(m, q))
        lanes["o"].append(o)
        lanes["w"].append(wq)
        lanes["gamma"].append(np.full(m, float(params.diffuse_aperture)))
        lanes["tmax"].append(np.full(m, float(params.max_dist)))
        lanes["tie"].append(frame_tie)
    slot = len(dirs)
    if params.enable_spec:
        cam = np.asarray(cam_pos, dtype=np.float64).reshape(-1, 3)[view[pix]]
        vdir = _normalize(x - cam)
        r = vdir - 2.0 * np.sum(vdir * nn, axis=1, keepdims=True) * nn
        lanes["pix"].append(pix)
        lanes["slot"].append(np.full(m, slot))
        lanes["o"].append(o)
        lanes["w"].append(_normalize(r))
        lanes["gamma"].append(rough * float(params.spec_aperture_scale))
        lanes["tmax"].append(np.full(m, float(params.max_dist)))
        lanes["tie"].append(np.zeros(m, dtype=bool))
    slot += 1
    if params.enable_occ:
        lvec = np.asarray(params.light_pos, dtype=np.float64)[None, :] - o
        dist = np.linalg.norm(lvec, axis=1)
        with np.errstate(invalid="ignore", divide="ignore"):
            wl = lvec / dist[:, None]
        wl[dist == 0] = 0.0
        lanes["pix"].append(pix)
        lanes["slot"].append(np.full(m, slot))
        lanes["o"].append(o)
        lanes["w"].append(wl)
        lanes["gamma"].append(np.full(m, float(params.occ_aperture)))
        lanes["tmax"].append(np.minimum(float(params.max_dist), dist))
        lanes["tie"].append(np.zeros(m, dtype=bool))
    out = {}
    for k, v in lanes.items():
        out[k] = np.concatenate(v) if v else np.zeros((0, 3) if k in ("o", "w") else (0,))
    out["pix"] = out["pix"].astype(np.int64)
    out["slot"] = out["slot"].astype(np.int64)
    out["tie"] = out["tie"].astype(bool)
    return out


# ---------------------------------------------------------------------------
# cone march (Section 4.3.2, cone-trace function)
# ---------------------------------------------------------------------------

def march(mips, lanes, params, origin=(0.0, 0.0, 0.0), extent=1.0, record=False, sampler=None):
    """Volume ray march of every lane.  Returns dict with c [m,3], alpha [m],
    K [m] (samples taken), ambiguous [m] (a termination decision within the
    tie band), and, if record, the per-step list of (lane idx, t, d, lam,
    alpha before, sample).  sampler(p, lam, w) replaces the isotropic
    quadrilinear sample when given (w: the lanes' unit axes)."""
    n0 = mips[0].shape[0]
    nlev = len(mips)
    v0 = extent / n0
    x = lanes["o"]
    w = lanes["w"]
    gamma = lanes["gamma"]
    tmax = lanes["tmax"]
    beta = float(params.step_factor)
    thresh = float(params.alpha_thresh)
    m = len(gamma)
    t = np.full(m, float(params.t0))
    c = np.zeros((m, 3))
    alpha = np.zeros(m)
    K = np.zeros(m, dtype=np.int64)
    amb = (np.abs(t - tmax) < AMBIG_T_REL * np.abs(tmax)) | lanes.get("tie", np.zeros(m, dtype=bool))
    active = (t <= tmax) & (alpha < thresh)
    steps = []
    cap = int(np.ceil(np.max(tmax, initial=0.0) / (beta * v0))) + 4
    it = 0
    while active.any():
        it += 1
        assert it <= cap, "march did not terminate"
        idx = np.nonzero(active)[0]
        ti = t[idx]
        d = np.maximum(2.0 * ti * np.tan(gamma[idx] / 2.0), v0)       # sampling diameter
        lam = np.clip(np.log2(d / v0), 0.0, nlev - 1)                  # LOD (R2)
        p = x[idx] + ti[:, None] * w[idx]                               # sampling position
        s = sample(mips, p, lam, origin, extent) if sampler is None else sampler(p, lam, w[idx])
        a_prev = alpha[idx]
        if record:
            steps.append((idx, ti, d, lam, a_prev.copy(), s))
        c[idx] += (1.0 - a_prev)[:, None] * s[:, 0:3]                   # colour accumulation (R1)
        alpha[idx] = a_prev + (1.0 - a_prev) * s[:, 3]                  # occlusion accumulation
        t[idx] = ti + beta * d
        K[idx] += 1
        if thresh < 1.0:
            amb[idx] |= np.abs(alpha[idx] - thresh) < AMBIG_ALPHA
        amb[idx] |= np.abs(t[idx] - tmax[idx]) < AMBIG_T_REL * np.abs(tmax[idx])
        active[idx] = (t[idx] <= tmax[idx]) & (alpha[idx] < thresh)
    res = {"c": c, "alpha": alpha, "K": K, "ambiguous": amb}
    if record:
        res["steps"] = steps
    return res


def _n_slots(params):
    return len(params.diffuse_dirs) + 2


def assemble(lanes, res, params, shape):
    """Per-pixel output [b,h,w,8] = (D.rgb, D.a, S.rgb, O) from lane results."""
    b, h, w = shape
    out = np.zeros((b * h * w, 8))
    nd = len(params.diffuse_dirs)
    wq = np.asarray(params.diffuse_weights, dtype=np.float64)
    pix, slot = lanes["pix"], lanes["slot"]
    for q in range(nd):
        sel = slot == q
        out[pix[sel], 0:3] += wq[q] * res["c"][sel]
        out[pix[sel], 3] += wq[q] * res["alpha"][sel]
    sel = slot == nd
    out[pix[sel], 4:7] = res["c"][sel]
    sel = slot == nd + 1
    out[pix[sel], 7] = res["alpha"][sel]
    return out.reshape(b, h, w, 8)


def trace(mips, pos_rough, normal, cam_pos, params, origin=(0.0, 0.0, 0.0), extent=1.0,
          return_info=False, sampler=None):
    """Forward: out [b,h,w,8] float64.  ``mips`` is the pyramid as returned by
    build_mips (or a decoded reduced-precision pyramid); ``sampler`` replaces
    the isotropic sample (see march)."""
    n = mips[0].shape[0]
    shape = np.asarray(pos_rough).shape[:3]
    lanes = cone_lanes(pos_rough, normal, cam_pos, params, n, origin, extent)
    res = march(mips, lanes, params, origin, extent, sampler=sampler)
    out = assemble(lanes, res, params, shape)
    if not return_info:
        return out
    amb_pix = np.zeros(int(np.prod(shape)), dtype=bool)
    np.logical_or.at(amb_pix, lanes["pix"], res["ambiguous"])
    info = {"lanes": lanes, "K": res["K"], "ambiguous_lane": res["ambiguous"],
            "ambiguous": amb_pix.reshape(shape), "samples": int(res["K"].sum())}
    return out, info


def lane_grads(lanes, params, grad_out):
    """dL/dC (3) and dL/dalpha of every lane from dL/d(out)."""
    g = np.asarray(grad_out, dtype=np.float64).reshape(-1, 8)
    nd = len(params.diffuse_dirs)
    wq = np.asarray(params.diffuse_weights, dtype=np.float64)
    pix, slot = lanes["pix"], lanes["slot"]
    gc = np.zeros((len(pix), 3))
    ga = np.zeros(len(pix))
    for q in range(nd):
        sel = slot == q
        gc[sel] = wq[q] * g[pix[sel], 0:3]
        ga[sel] = wq[q] * g[pix[sel], 3]
    sel = slot == nd
    gc[sel] = g[pix[sel], 4:7]
    sel = slot == nd + 1
    ga[sel] = g[pix[sel], 7]
    return gc, ga


def trace_backward(mips, pos_rough, normal, cam_pos, params, grad_out,
                   origin=(0.0, 0.0, 0.0), extent=1.0, return_levels=False, sampler=None, scatter=None,
                   adjoint=None):
    """Adjoint of trace (R12): dL/d(base grid) [N,N,N,4] float64.

    Every step of every lane is recorded; a reverse sweep then carries the
    suffix sums R_k = c_k + (1 - a_k) R_{k+1} and U_k = (1 - a_k) U_{k+1}
    (R_K = 0, U_K = 1), giving dL/dc_k = T_k dL/dC and
    dL/da_k = T_k (-dL/dC . R_{k+1} + dL/dA U_{k+1}), T_k = 1 - alpha_k.
    Each sample's gradient is scattered to its 16 taps with the tap weights,
    then carried through the mip reduction by its transpose.

    Hooks for other pyramids: sampler (see march); scatter(p, lam, w, gs)
    replaces the scatter into the isotropic level gradients and adjoint()
    the mip adjoint (then return_levels is not available)."""
    n = mips[0].shape[0]
    lanes = cone_lanes(pos_rough, normal, cam_pos, params, n, origin, extent)
    res = march(mips, lanes, params, origin, extent, record=True, sampler=sampler)
    gc, ga = lane_grads(lanes, params, grad_out)
    m = len(lanes["gamma"])
    R = np.zeros((m, 3))
    U = np.ones(m)
    level_grads = [np.zeros_like(ml) for ml in mips]
    for idx, ti, d, lam, a_prev, s in reversed(res["steps"]):
        T = 1.0 - a_prev
        g_c = T[:, None] * gc[idx]
        g_a = T * (-np.sum(gc[idx] * R[idx], axis=1) + ga[idx] * U[idx])
        R[idx] = s[:, 0:3] + (1.0 - s[:, 3])[:, None] * R[idx]
        U[idx] = (1.0 - s[:, 3]) * U[idx]
        gs = np.concatenate([g_c, g_a[:, None]], axis=1)
        p = lanes["o"][idx] + ti[:, None] * lanes["w"][idx]
        if scatter is not None:
            scatter(p, lam, lanes["w"][idx], gs)
            continue
        for lev, iz, iy, ix, wt in taps(mips, p, lam, origin, extent):
            for l in np.unique(lev):
                sel = lev == l
                np.add.at(level_grads[l], (iz[sel], iy[sel], ix[sel]), wt[sel, None] * gs[sel])
    if adjoint is not None:
        return adjoint()
    gb = mip_adjoint(level_grads)
    if return_levels:
        return gb, level_grads
    return gb


def render(base, pos_rough, normal, cam_pos, params, levels=None, origin=(0.0, 0.0, 0.0),
           extent=1.0, return_info=False):
    """build_mips followed by trace."""
    mips = build_mips(base, levels)
    return trace(mips, pos_rough, normal, cam_pos, params, origin, extent, return_info)
