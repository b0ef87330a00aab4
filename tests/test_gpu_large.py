"""Largest workloads: the 512^3 / 4 x 3840x2160 float16-pyramid scene (forward
parity on sampled pixels at the full launch, backward properties at the full
launch) and the differentiation workload run as a fitting loop."""
import numpy as np
import pytest
import torch

import oracle
import paper_2104_00618_amd as vct
from tests.parity import fmt, range_errors, worst
from tests.workloads import oracle_at, sample_pixels, workload

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


@pytest.fixture(scope="module")
def c4():
    w = workload("c4", device=DEV)      # (the generator on the GPU: the same bits as on the CPU, faster)
    g = vct.Grid(w.n, dtype="f16")
    base = dev(w.base)
    pyr = vct.build_mips(base, g)
    t = (dev(w.pos_rough), dev(w.normal), dev(w.cam_pos))
    return w, g, base, pyr, t


def test_c4_forward_f16_sampled_pixels(c4):
    w, g, base, pyr, (pr, nr, cam) = c4
    out = vct.trace(pyr, g, pr, nr, cam, w.params)
    torch.cuda.synchronize()
    v, y, x = sample_pixels(w.shape, 384, seed=4)
    got = out[torch.from_numpy(v), torch.from_numpy(y), torch.from_numpy(x)].cpu().numpy()
    del out
    decoded = [vct.unpack_level(pyr, g, l).cpu().numpy().astype(np.float64) for l in range(g.levels)]
    ref_dec, amb_dec = oracle_at(decoded, w, v, y, x)
    del decoded
    e1 = range_errors(got, ref_dec, ~amb_dec)
    print(f"c4 f16 path parity: {fmt(e1)}", flush=True)
    assert worst(e1)[0] <= 1e-5
    ref, amb = oracle_at(oracle.build_mips(w.base), w, v, y, x)
    e2 = range_errors(got, ref, ~(amb | amb_dec))
    print(f"c4 f16 storage error: {fmt(e2)}", flush=True)
    assert worst(e2)[0] <= 2e-3


def test_c4_backward_full_launch_is_deterministic_and_exact_under_scaling(c4):
    w, g, base, pyr, (pr, nr, cam) = c4
    rng = np.random.default_rng(3)
    gout = dev((rng.normal(size=w.shape + (8,)) * 1e-3).astype(np.float32))
    ws = torch.empty(vct.backward_workspace_bytes(g, pr, nr, cam, w.params), dtype=torch.uint8, device=DEV)
    a = vct.trace_backward(pyr, g, pr, nr, cam, w.params, gout, ws)
    b = vct.trace_backward(pyr, g, pr, nr, cam, w.params, gout, ws)
    c = vct.trace_backward(pyr, g, pr, nr, cam, w.params, gout * 2, ws)
    torch.cuda.synchronize()
    assert torch.isfinite(a).all()
    assert torch.equal(a, b)
    assert torch.equal(c, a * 2)
    assert a.abs().max() > 0


def test_c4_training_step_sparse_grad_out_matches_oracle(c4):
    """The c4 training step at its full launch (512^3 float16 pyramid,
    4 x 3840x2160, trace_save + trace_backward_saved) with dL/d(out) nonzero
    on 64 seeded surface pixels spread over the four views, so that the oracle
    can form the whole gradient from those pixels.  Path parity: the oracle
    marches the GPU's decoded float16 levels, and the gradient is taken with
    respect to the float32 base with the storage rounding as the identity."""
    w, g, base, pyr, (pr, nr, cam) = c4
    b, h, wd = w.shape
    rng = np.random.default_rng(94)
    surf = np.argwhere(w.normal[..., 3] != 0)
    pick = surf[rng.choice(len(surf), size=64, replace=False)]
    vv, yy, xx = pick[:, 0], pick[:, 1], pick[:, 2]
    go = rng.normal(size=(64, 8))
    gout = torch.zeros((b, h, wd, 8), dtype=torch.float32, device=DEV)
    gout[torch.from_numpy(vv), torch.from_numpy(yy), torch.from_numpy(xx)] = torch.from_numpy(go).float().to(DEV)
    out, state = vct.trace_save(pyr, g, pr, nr, cam, w.params)
    got_out = out[torch.from_numpy(vv), torch.from_numpy(yy), torch.from_numpy(xx)].cpu().numpy()
    del out
    decoded = [vct.unpack_level(pyr, g, l).cpu().numpy().astype(np.float64) for l in range(g.levels)]
    # one oracle call over all views (each pixel keeps its camera): view v's
    # picked pixels in row v, padded with background pixels (no output, no gradient)
    m = max(int((vv == v).sum()) for v in range(b))
    prv = np.zeros((b, 1, m, 4), np.float32)
    nrv = np.zeros((b, 1, m, 4), np.float32)
    slot = np.zeros(64, dtype=int)
    for v in range(b):
        sel = np.nonzero(vv == v)[0]
        slot[sel] = np.arange(len(sel))
        prv[v, 0, :len(sel)] = w.pos_rough[v, yy[sel], xx[sel]]
        nrv[v, 0, :len(sel)] = w.normal[v, yy[sel], xx[sel]]
    o, info = oracle.trace(decoded, prv, nrv, w.cam_pos, w.params, return_info=True)
    ref_out = o[vv, 0, slot]
    amb = info["ambiguous"][vv, 0, slot]          # ties get no gradient on either side
    gv = np.zeros((b, 1, m, 8))
    gv[vv, 0, slot] = np.where(amb[:, None], 0.0, go)
    ref = oracle.trace_backward(decoded, prv, nrv, w.cam_pos, w.params, gv)
    del decoded
    go[amb] = 0.0
    gout[torch.from_numpy(vv), torch.from_numpy(yy), torch.from_numpy(xx)] = torch.from_numpy(go).float().to(DEV)
    got = vct.trace_backward_saved(pyr, g, pr, nr, cam, w.params, state, gout).cpu().numpy()
    del state
    e = range_errors(got_out, ref_out, ~amb)
    scale = np.abs(ref).max()
    err = np.abs(got - ref).max() / scale
    rms = np.sqrt(np.mean((got - ref) ** 2)) / scale
    print(f"c4 training step, 64 pixels of gradient ({int(amb.sum())} ties): forward {fmt(e)}; gradient max "
          f"{err:.2e} rms {rms:.2e}", flush=True)
    assert worst(e)[0] <= 1e-5
    assert err <= 1e-4 and rms <= 1e-5


def test_c3_fitting_loop_reduces_the_loss():
    """The differentiation workload: a learnable 128^3 grid initialised to
    opacity 0.1 and grey radiance 0.5 (stored premultiplied), fitted to 8
    512x512 target renders of the ground-truth scene by L2 on the indirect
    radiance (D.rgb and S.rgb); every step runs build_mips, trace and
    trace_backward in float32."""
    w = workload("c3gt")
    g = vct.Grid(w.n)
    pr, nr, cam = dev(w.pos_rough), dev(w.normal), dev(w.cam_pos)
    with torch.no_grad():
        target = vct.trace(vct.build_mips(dev(w.base), g), g, pr, nr, cam, w.params)
    grid = torch.empty((w.n,) * 3 + (4,), device=DEV)
    grid[...] = torch.tensor([0.05, 0.05, 0.05, 0.1], device=DEV)
    grid.requires_grad_(True)
    opt = torch.optim.Adam([grid], lr=0.01)
    valid = nr[..., 3:4] != 0
    n_valid = valid.sum() * 6
    losses = []
    for _ in range(25):
        opt.zero_grad()
        out = vct.render(grid, g, pr, nr, cam, w.params)
        diff = torch.cat([out[..., 0:3] - target[..., 0:3], out[..., 4:7] - target[..., 4:7]], -1) * valid
        loss = (diff ** 2).sum() / n_valid
        loss.backward()
        assert torch.isfinite(grid.grad).all()
        opt.step()
        losses.append(float(loss))
    print("fit losses", [f"{x:.3e}" for x in losses[::4]], flush=True)
    assert losses[-1] < 0.5 * losses[0]
