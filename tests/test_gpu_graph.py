"""The hot path captured in a HIP graph (torch.cuda.CUDAGraph around the
library's calls, which enqueue on the capturing stream) and replayed.  The
library clears its buffers with fill kernels, never a memset or a copy, and
synchronises with nothing, so a training step (build_mips + trace_save +
trace_backward_saved, and the forward trace), the same step through the
allocation-free backward, and a revoxelized bounce frame (voxelize with
surface attributes + build_mips + bounce) can be captured.
Every replay is compared bit for bit with the same calls made eagerly into
other buffers, with the inputs changed in place by eager work and the device
synchronised between replays."""
import numpy as np
import pytest
import torch

import paper_2104_00618_amd as vct
from scenes import ConeParams, cone_set, make_workload
from scenes.mesh import cornell_mesh

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
LIGHTS = [((0.5, 0.95, 0.5), (1.0, 1.0, 1.0), (1.0, 0.5, 0.25))]


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def same_bits(a, b):
    return torch.equal(a.contiguous().view(torch.int32), b.contiguous().view(torch.int32))


def capture(fn):
    """fn() once eagerly on a side stream (as torch requires before a capture), then captured."""
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        fn()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn()
    torch.cuda.synchronize()
    return g


@pytest.mark.parametrize("dtype", ["f32", "f16"])
def test_training_step_graph_replays_equal_eager_calls(dtype):
    w = make_workload("c0", h=96, w=160)
    base, pr, nr, cam = dev(w.base), dev(w.pos_rough), dev(w.normal), dev(w.cam_pos)
    grid = vct.Grid(w.n, dtype=dtype)
    gout = dev(np.random.default_rng(3).normal(size=w.shape + (8,)).astype(np.float32) * 1e-2)
    n_state = vct.lane_state_bytes(pr, nr, cam, w.params)
    n_ws = vct.backward_workspace_bytes(grid, pr, nr, cam, w.params) - n_state

    def buffers():
        return {"pyr": torch.empty(vct.pyramid_bytes(grid), dtype=torch.uint8, device=DEV),
                "out": torch.empty(w.shape + (8,), device=DEV), "fwd": torch.empty(w.shape + (8,), device=DEV),
                "st": torch.empty(n_state, dtype=torch.uint8, device=DEV),
                "ws": torch.empty(n_ws, dtype=torch.uint8, device=DEV),
                "gb": torch.empty((w.n,) * 3 + (4,), device=DEV)}

    def step(b):
        vct.build_mips(base, grid, b["pyr"])
        vct.trace_save(b["pyr"], grid, pr, nr, cam, w.params, b["out"], b["st"])
        vct.trace_backward_saved(b["pyr"], grid, pr, nr, cam, w.params, b["st"], gout, b["ws"], b["gb"])
        vct.trace(b["pyr"], grid, pr, nr, cam, w.params, b["fwd"])

    static, eager = buffers(), buffers()
    graph = capture(lambda: step(static))
    for r in range(4):
        if r:   # eager work on the inputs between replays
            base.mul_(0.8).add_(0.02 * r).clamp_(0.0, 1.0)
            gout.mul_(-1.25)
            torch.cuda.synchronize()
        graph.replay()
        step(eager)
        torch.cuda.synchronize()
        for k in ("out", "fwd", "gb"):
            assert same_bits(static[k], eager[k]), f"replay {r}: {k} differs from the eager call"
        assert static["gb"].abs().max().item() > 0
        print(f"{dtype} replay {r}: trace, training step and gradient equal to the eager calls", flush=True)


def test_allocation_free_backward_under_capture_equals_the_saved_backward():
    """The entry point for callers that cannot allocate, captured in a graph
    (its scratch is the library's per-GPU array, set up by an eager call
    before the capture): every replay equals the allocating saved backward
    called eagerly."""
    w = make_workload("c0", h=64, w=96)
    base, pr, nr, cam = dev(w.base), dev(w.pos_rough), dev(w.normal), dev(w.cam_pos)
    grid = vct.Grid(w.n)
    gout = dev(np.random.default_rng(5).normal(size=w.shape + (8,)).astype(np.float32) * 1e-2)
    pyr = torch.empty(vct.pyramid_bytes(grid), dtype=torch.uint8, device=DEV)
    out = torch.empty(w.shape + (8,), device=DEV)
    st = torch.empty(vct.lane_state_bytes(pr, nr, cam, w.params), dtype=torch.uint8, device=DEV)
    gb_graph = torch.empty((w.n,) * 3 + (4,), device=DEV)
    ws = torch.empty(vct.backward_workspace_bytes(grid, pr, nr, cam, w.params) - st.numel(), dtype=torch.uint8,
                     device=DEV)
    gb_eager = torch.empty_like(gb_graph)

    def step():
        vct.build_mips(base, grid, pyr)
        vct.trace_save(pyr, grid, pr, nr, cam, w.params, out, st)
        vct.trace_backward_saved_noalloc(pyr, grid, pr, nr, cam, w.params, st, gout, gb_graph)

    graph = capture(step)
    for r in range(3):
        if r:
            base.mul_(0.7).add_(0.03 * r).clamp_(0.0, 1.0)
            torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        vct.trace_backward_saved(pyr, grid, pr, nr, cam, w.params, st, gout, ws, gb_eager)
        torch.cuda.synchronize()
        assert same_bits(gb_graph, gb_eager), f"replay {r}: the captured allocation-free backward differs"
        assert gb_graph.abs().max().item() > 0


def test_revoxelized_bounce_frame_graph_replays_equal_eager_calls():
    n = 64
    tris, cols = cornell_mesh(1)
    t, c = dev(tris), dev(cols)
    grid = vct.Grid(n)
    d, wt = cone_set("five")
    params = ConeParams(d, wt, alpha_thresh=0.99)
    shape = (n, n, n, 4)

    def buffers():
        return {"vb": torch.empty(shape, device=DEV), "vn": torch.empty(shape, device=DEV),
                "va": torch.empty(shape, device=DEV), "out": torch.empty(shape, device=DEV),
                "vws": torch.empty(vct.voxelize_workspace_bytes(grid, t.shape[0], surface=True), dtype=torch.uint8,
                                   device=DEV),
                "pyr": torch.empty(vct.pyramid_bytes(grid), dtype=torch.uint8, device=DEV),
                "bws": torch.empty(vct.bounce_workspace_bytes(grid), dtype=torch.uint8, device=DEV)}

    def frame(b):
        vct.voxelize(t, c, grid, LIGHTS, base=b["vb"], workspace=b["vws"], surface=True, normal=b["vn"],
                     albedo=b["va"])
        vct.build_mips(b["vb"], grid, b["pyr"])
        vct.bounce(b["pyr"], grid, b["vb"], b["vn"], b["va"], params, out=b["out"], workspace=b["bws"])

    static, eager = buffers(), buffers()
    graph = capture(lambda: frame(static))
    for r in range(4):
        if r:   # move the mesh between replays (eager work on the graph's input)
            t.add_(torch.tensor([0.004, -0.003, 0.002], device=DEV))
            torch.cuda.synchronize()
        graph.replay()
        frame(eager)
        torch.cuda.synchronize()
        for k in ("vb", "vn", "va", "out"):
            assert same_bits(static[k], eager[k]), f"replay {r}: {k} differs from the eager call"
        occ = int((static["vb"][..., 3] > 0).sum().item())
        assert occ > 1000
        print(f"replay {r}: voxelize ({occ} voxels) + mips + bounce equal to the eager calls", flush=True)
