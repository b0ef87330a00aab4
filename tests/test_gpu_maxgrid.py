"""Pyramids whose byte offsets pass 2^31 and 2^32, read through a corner
window.  The grid is zero except the corner block [W0, N)^3; G-buffer points
inside the block march short, narrow cones that stay inside it, so for every
level they reach the pyramid of the whole grid restricted to the block is the
pyramid of the block alone, and the FP64 oracle runs on that window (origin
W0/N, extent 1 - W0/N, the same voxel size) instead of on the whole grid.

* 1024^3 (every storage type): pyramids above 4 GiB, read with 64-bit
  addresses (float32 19.6 GB isotropic and 31 GB anisotropic, float16 and
  bfloat16 9.8 GB isotropic and 15.9 GB anisotropic).
* 512^3 float32: pyramids between 2 and 4 GiB read through the 32-bit
  buffer resources (2.45 GB isotropic, every level above 0 at a byte offset
  of 2^31 or more; 3.99 GB anisotropic).  Half of the G-buffer is a small
  planar patch, so that the lanes of a wave share footprints and the
  float32 march reads them with scalar loads at those offsets.

Reduced-precision pyramids are checked for path parity: the oracle runs on
the window of the GPU's own decoded levels."""
import numpy as np
import pytest
import torch

import oracle
from oracle import vct_aniso as va
import paper_2104_00618_amd as vct
from scenes import ConeParams, cone_set, random_grid
from tests.parity import fmt, range_errors, worst

pytestmark = pytest.mark.gpu
DEV = "cuda:0"

# (N, W0, positions of the G-buffer points, max_dist): the cones (20 degrees)
# reach LOD <= 3.9 (1024^3) and <= 4.2 (512^3); the points sit far enough
# inside the block that every tap of those levels lies in the window.
CASES = {1024: (768, (0.83, 0.92), 0.04), 512: (256, (0.65, 0.85), 0.1)}


def _inputs(n, seed=78):
    w0, (lo, hi), max_dist = CASES[n]
    rng = np.random.default_rng(seed)
    h, w = 16, 32
    pos = rng.uniform(lo, hi, size=(1, h, w, 3))
    rough = rng.uniform(0.05, 0.3, size=(1, h, w, 1))
    nrm = rng.normal(size=(1, h, w, 3))
    nrm /= np.linalg.norm(nrm, axis=-1, keepdims=True)
    # right tile: a planar patch, a quarter voxel between neighbouring pixels
    # (the lanes of each of its waves share most footprints on levels >= 2)
    c = np.array([0.5 * (lo + hi)] * 3)
    u = np.array([1.0, 0.0, 0.0])
    v = np.array([0.0, 0.8, 0.6])
    jj, ii = np.meshgrid(np.arange(16), np.arange(16), indexing="ij")
    pos[0, :, 16:] = c + (0.25 / n) * (ii[..., None] * u + jj[..., None] * v)
    nrm[0, :, 16:] = np.cross(u, v)
    rough[0, :, 16:] = 0.2
    pr = np.concatenate([pos, rough], -1).astype(np.float32)
    nr = np.concatenate([nrm, np.ones((1, h, w, 1))], -1).astype(np.float32)
    cam = np.array([[c[0], c[1], 0.5]], np.float32)
    d, wt = cone_set("six")
    ap = np.float32(0.349)
    p = ConeParams(d, wt, diffuse_aperture=float(ap), spec_aperture_scale=float(ap), occ_aperture=float(ap),
                   light_pos=(hi, 0.95, hi), max_dist=max_dist, alpha_thresh=0.99)
    return pr, nr, cam, p


def _window(n):
    w0 = CASES[n][0]
    return w0, (w0 / n,) * 3, (n - w0) / n


def _gpu_pyramid(n, block, dtype, aniso):
    w0 = CASES[n][0]
    base = torch.zeros((n, n, n, 4), dtype=torch.float32, device=DEV)
    base[w0:, w0:, w0:] = torch.from_numpy(block).to(DEV)
    g = vct.Grid(n, dtype=dtype, anisotropic=aniso)
    pyr = vct.build_mips(base, g)
    del base
    return g, pyr


def _window_mips(n, block, g, pyr, dtype, aniso):
    """The oracle's pyramid of the window: built from the block in FP64 for
    float32 storage, else the window of the GPU's decoded levels."""
    w0 = CASES[n][0]
    levels = int(round(np.log2(n - w0))) + 1
    if dtype == "f32":
        return va.build_aniso_mips(block) if aniso else oracle.build_mips(block)

    def cut(t, lv):
        o = w0 >> lv
        return t[o:, o:, o:].cpu().numpy().astype(np.float64)

    if aniso:
        return [[cut(vct.unpack_level_dir(pyr, g, lv, d), lv) for lv in range(levels)] for d in range(6)]
    return [cut(vct.unpack_level(pyr, g, lv), lv) for lv in range(levels)]


def _label(n, dtype, aniso, nbytes):
    return f"{n}^3 {dtype} {'anisotropic' if aniso else 'isotropic'} ({nbytes / 2**30:.2f} GiB pyramid)"


FORWARD = [(1024, "f32", False), (1024, "f32", True), (1024, "f16", False), (1024, "bf16", False),
           (1024, "f16", True), (512, "f32", False), (512, "f32", True)]


@pytest.mark.parametrize("n,dtype,aniso", FORWARD)
def test_far_texels_forward(n, dtype, aniso):
    block = random_grid(n - CASES[n][0], seed=77, alpha_max=0.25)
    g, pyr = _gpu_pyramid(n, block, dtype, aniso)
    nbytes = pyr.numel()
    if n == 512:
        assert 2 ** 31 < nbytes < 2 ** 32          # the narrow path above 2 GiB
    else:
        assert nbytes > 2 ** 32                    # the 64-bit path
    pr, nr, cam, p = _inputs(n)
    print(f"forward {_label(n, dtype, aniso, nbytes)}", flush=True)
    out = vct.trace(pyr, g, torch.from_numpy(pr).to(DEV), torch.from_numpy(nr).to(DEV),
                    torch.from_numpy(cam).to(DEV), p).cpu().numpy()
    mips = _window_mips(n, block, g, pyr, dtype, aniso)
    del pyr
    torch.cuda.empty_cache()
    _, origin, extent = _window(n)
    if aniso:
        ref, info = va.trace_aniso(mips, pr, nr, cam, p, origin, extent, return_info=True)
    else:
        ref, info = oracle.trace(mips, pr, nr, cam, p, origin, extent, return_info=True)
    keep = ~info["ambiguous"].reshape(-1)
    e = range_errors(out, ref, keep)
    print(f"{_label(n, dtype, aniso, nbytes)}: {fmt(e)}; ambiguous {int((~keep).sum())}", flush=True)
    assert worst(e)[0] <= 1e-5
    assert np.abs(ref).max() > 0.05          # the cones do see the block


BACKWARD = [(1024, "f32", False), (1024, "f32", True), (1024, "f16", False), (1024, "bf16", False),
            (512, "f32", False), (512, "f32", True)]


@pytest.mark.parametrize("n,dtype,aniso", BACKWARD)
def test_far_texels_backward_saved(n, dtype, aniso):
    """The training path (trace_save + trace_backward_saved) against the
    oracle's adjoint on the window; every voxel outside it gets exactly zero.
    The 1024^3 anisotropic accumulator (2.0e9 texels, 64 GB) is indexed far
    past 2^32 bytes."""
    w0, origin, extent = _window(n)
    block = random_grid(n - w0, seed=79, alpha_max=0.25)
    g, pyr = _gpu_pyramid(n, block, dtype, aniso)
    nbytes = pyr.numel()
    pr, nr, cam, p = _inputs(n)
    print(f"training path {_label(n, dtype, aniso, nbytes)}", flush=True)
    mips = _window_mips(n, block, g, pyr, dtype, aniso)
    fwd = va.trace_aniso if aniso else oracle.trace
    ref_out, info = fwd(mips, pr, nr, cam, p, origin, extent, return_info=True)
    # pixels with a termination tie may take another step count on either side: no gradient through them
    gout = np.random.default_rng(80).normal(size=pr.shape[:3] + (8,)).astype(np.float32)
    gout[info["ambiguous"]] = 0.0
    t = [torch.from_numpy(a).to(DEV) for a in (pr, nr, cam)]
    out, state = vct.trace_save(pyr, g, *t, p)
    grad = vct.trace_backward_saved(pyr, g, *t, p, state, torch.from_numpy(gout).to(DEV))
    del pyr, state
    inside = grad[w0:, w0:, w0:].cpu().numpy()
    grad[w0:, w0:, w0:] = 0
    outside_nonzero = int(torch.count_nonzero(grad).item())
    del grad
    torch.cuda.empty_cache()
    e = range_errors(out.cpu().numpy(), ref_out, ~info["ambiguous"].reshape(-1))
    bwd = va.trace_backward_aniso if aniso else oracle.trace_backward
    ref = bwd(mips, pr, nr, cam, p, gout, origin, extent)
    scale = np.abs(ref).max()
    err = np.abs(inside - ref).max() / scale
    rms = np.sqrt(np.mean((inside - ref) ** 2)) / scale
    print(f"{_label(n, dtype, aniso, nbytes)} training path: forward {fmt(e)}; gradient max {err:.2e} "
          f"rms {rms:.2e}; {outside_nonzero} nonzero outside the block; {int(info['ambiguous'].sum())} tie "
          f"pixels without gradient", flush=True)
    assert worst(e)[0] <= 1e-5 and err <= 1e-4 and rms <= 1e-5 and outside_nonzero == 0
