"""GPU voxelization with direct-light injection (vct_voxelize) against the
FP64 / exact-integer oracle: occupancy bit-exact, colours within 1e-5 of the
largest (range-normalised), determinism under any triangle order, and the
voxelized grid feeding build_mips + trace."""
import numpy as np
import pytest
import torch

import oracle
from oracle import vct_voxelize as vx
import paper_2104_00618_amd as vct
from scenes import ConeParams, cone_set, random_gbuffer
from scenes.mesh import cornell_mesh

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
LIGHTS = [((0.5, 0.95, 0.5), (1.0, 1.0, 1.0), (1.0, 0.5, 0.25)), ((0.2, 0.6, 0.8), (0.4, 0.3, 0.2), (1.0, 0.0, 0.0))]


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def mesh(seed, extra=40):
    tris, cols = cornell_mesh(seed)
    rng = np.random.default_rng(seed)
    t2 = rng.uniform(-0.2, 1.2, size=(extra, 3, 3)).astype(np.float32)      # random triangles, some leaving the grid
    return np.concatenate([tris, t2]), np.concatenate([cols, rng.uniform(0, 1, size=(extra, 3)).astype(np.float32)])


def gpu_voxelize(tris, cols, n, lights=LIGHTS, **kw):
    out = vct.voxelize(dev(tris), dev(cols), vct.Grid(n), lights, **kw)
    torch.cuda.synchronize()
    return tuple(o.cpu().numpy() for o in out) if isinstance(out, tuple) else out.cpu().numpy()


@pytest.mark.parametrize("n,seed", [(64, 1), (256, 2)])
def test_voxelize_matches_oracle(n, seed):
    tris, cols = mesh(seed)
    got = gpu_voxelize(tris, cols, n, ambient=0.15, diffuse=0.9)
    ref, cnt = vx.voxelize(tris, cols, n, LIGHTS, ambient=0.15, diffuse=0.9, return_counts=True)
    np.testing.assert_array_equal(got[..., 3], (cnt > 0).astype(np.float32))
    err = np.abs(got[..., :3] - ref[..., :3]).max() / np.abs(ref[..., :3]).max()
    print(f"voxelize {n}^3 {len(tris)} triangles: {int((cnt > 0).sum())} voxels, colour max rel {err:.2e}", flush=True)
    assert err <= 1e-5


def test_voxelize_dense_mesh_matches_oracle():
    """73,006 triangles, most of them smaller than a voxel at 64^3 (the spheres
    at 96 x 192): many triangles per wave of the pixel-space raster, triangles
    without pixels between them, and a multi-block offset scan."""
    tris, cols = cornell_mesh(2, rings=96, segments=192)
    got = gpu_voxelize(tris, cols, 64, surface=True)
    ref, cnt, rn, ra = vx.voxelize(tris, cols, 64, LIGHTS, return_counts=True, return_surface=True)
    base, nrm, alb = got
    np.testing.assert_array_equal(base[..., 3], (cnt > 0).astype(np.float32))
    err = np.abs(base[..., :3] - ref[..., :3]).max() / np.abs(ref[..., :3]).max()
    en = np.abs(nrm[..., :3] - rn[..., :3]).max()
    print(f"voxelize {len(tris)} triangles at 64^3: {int((cnt > 0).sum())} voxels, up to {int(cnt.max())} fragments "
          f"per voxel; colour max rel {err:.2e}, normal max abs {en:.2e}", flush=True)
    assert err <= 1e-5 and en <= 1e-6


def test_voxelize_is_deterministic_in_any_triangle_order():
    tris, cols = mesh(3, extra=200)
    a = gpu_voxelize(tris, cols, 64)
    b = gpu_voxelize(tris, cols, 64)
    perm = np.random.default_rng(4).permutation(len(tris))
    c = gpu_voxelize(tris[perm], cols[perm], 64)
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
    assert np.array_equal(a.view(np.uint32), c.view(np.uint32))


@pytest.mark.parametrize("n_tris", [4096, 4097])
def test_voxelize_offset_scan_either_side_of_one_workgroup(n_tris):
    """Up to 4,096 triangles the offset scan runs in one workgroup, above it in
    three phases: a mesh of either size (small random triangles, a tenth of
    them without pixels) matches the oracle."""
    rng = np.random.default_rng(n_tris)
    ctr = rng.uniform(0.0, 1.0, size=(n_tris, 1, 3))
    tris = (ctr + rng.uniform(-0.03, 0.03, size=(n_tris, 3, 3))).astype(np.float32)
    tris[::10, 1] = tris[::10, 0]                           # degenerate: no pixels
    cols = rng.uniform(0.1, 1.0, size=(n_tris, 3)).astype(np.float32)
    got = gpu_voxelize(tris, cols, 64, surface=True)
    ref, cnt, rn, ra = vx.voxelize(tris, cols, 64, LIGHTS, return_counts=True, return_surface=True)
    np.testing.assert_array_equal(got[0][..., 3], (cnt > 0).astype(np.float32))
    err = np.abs(got[0][..., :3] - ref[..., :3]).max() / np.abs(ref[..., :3]).max()
    en = np.abs(got[1][..., :3] - rn[..., :3]).max()
    ea = np.abs(got[2][..., :3] - ra[..., :3]).max()
    print(f"voxelize {n_tris} triangles at 64^3: {int((cnt > 0).sum())} voxels; colour max rel {err:.2e}, "
          f"normal {en:.2e}, albedo {ea:.2e}", flush=True)
    assert err <= 1e-5 and en <= 1e-6 and ea <= 1e-6


def test_voxelize_stacked_copies_contend_for_the_same_slots():
    """1,024 coincident copies of one quad, each copy with its own colour:
    every voxel the quad reaches is claimed by the fragments of all 1,024
    copies at once.  Occupancy, colours and normals match the oracle, the
    colour is that of one copy times the mean colour of the copies, and two
    runs agree bit for bit."""
    n, k = 32, 1024
    quad = np.array([[[0.1, 0.2, 0.45], [0.9, 0.2, 0.45], [0.9, 0.85, 0.55]],
                     [[0.1, 0.2, 0.45], [0.9, 0.85, 0.55], [0.1, 0.85, 0.55]]], np.float32)
    cols = np.random.default_rng(7).uniform(0.1, 1.0, size=(k, 3)).astype(np.float32)
    tris = np.tile(quad, (k, 1, 1))
    stacked_cols = np.repeat(cols, 2, axis=0)
    a = gpu_voxelize(tris, stacked_cols, n, surface=True)
    b = gpu_voxelize(tris, stacked_cols, n, surface=True)
    for x, y in zip(a, b):
        assert np.array_equal(x.view(np.uint32), y.view(np.uint32))
    ref, cnt, rn, ra = vx.voxelize(tris, stacked_cols, n, LIGHTS, return_counts=True, return_surface=True)
    one = vx.voxelize(quad, np.ones((2, 3), np.float32), n, LIGHTS)
    occ = cnt > 0
    assert occ.sum() > 200 and cnt[occ].min() >= k
    np.testing.assert_array_equal(a[0][..., 3], occ.astype(np.float32))
    mean = cols.astype(np.float64).mean(0)
    np.testing.assert_allclose(ref[occ, 0:3], one[occ, 0:3] * mean, rtol=1e-12)
    err = np.abs(a[0][..., 0:3] - ref[..., 0:3]).max() / np.abs(ref[..., 0:3]).max()
    en = np.abs(a[1][..., 0:3] - rn[..., 0:3]).max()
    ea = np.abs(a[2][..., 0:3] - ra[..., 0:3]).max()
    print(f"{k} stacked quads at {n}^3: {int(occ.sum())} voxels, {int(cnt.max())} fragments at most; colour max rel "
          f"{err:.2e}, normal {en:.2e}, albedo {ea:.2e}", flush=True)
    assert err <= 1e-5 and en <= 1e-6 and ea <= 1e-6


def test_voxelized_grid_feeds_mips_and_trace():
    """Mesh -> voxelize -> build_mips -> trace on the GPU against the same
    pipeline in the oracles."""
    n = 64
    tris, cols = cornell_mesh(5)
    base = gpu_voxelize(tris, cols, n)
    ref_base = vx.voxelize(tris, cols, n, LIGHTS)
    d, w = cone_set("six")
    p = ConeParams(d, w, alpha_thresh=0.99)
    pr, nr, cam = random_gbuffer(1, 24, 31, seed=6, n=n)
    g = vct.Grid(n)
    pyr = vct.build_mips(dev(base), g)
    out = vct.trace(pyr, g, dev(pr), dev(nr), dev(cam), p).cpu().numpy()
    ref, info = oracle.trace(oracle.build_mips(ref_base), pr, nr, cam, p, return_info=True)
    from tests.parity import fmt, range_errors, worst
    e = range_errors(out, ref, ~info["ambiguous"].reshape(-1))
    print(f"voxelize -> trace 64^3: {fmt(e)}", flush=True)
    assert worst(e)[0] <= 1e-5


@pytest.mark.parametrize("n,n_tris", [(16, 0), (16, 1), (64, 1)])
def test_voxelize_clears_every_output_grid_whatever_it_held(n, n_tris):
    """The three output grids start filled with garbage: the base grid is
    zero-filled before the raster pass, normal and albedo by workgroups of the
    raster launch (by the first fill when there are no triangles).  Every voxel
    no fragment reaches is zero in all three, and the reached ones match the
    oracle."""
    if n_tris:
        tris, cols = mesh(5)
    else:
        tris, cols = np.zeros((0, 3, 3), np.float32), np.zeros((0, 3), np.float32)
    grids = [torch.full((n, n, n, 4), v, dtype=torch.float32, device=DEV) for v in (5.0, float("nan"), -3.0)]
    vct.voxelize(dev(tris), dev(cols), vct.Grid(n), LIGHTS, base=grids[0], surface=True, normal=grids[1],
                 albedo=grids[2])
    torch.cuda.synchronize()
    got = [g.cpu().numpy() for g in grids]
    ref, cnt, rn, ra = vx.voxelize(tris, cols, n, LIGHTS, return_counts=True, return_surface=True)
    occ = cnt > 0
    assert (occ.sum() > 100) == bool(n_tris)
    for g in got:
        assert (g[~occ] == 0).all()
    np.testing.assert_array_equal(got[0][..., 3], occ.astype(np.float32))
    if n_tris:
        err = np.abs(got[0][..., :3] - ref[..., :3]).max() / np.abs(ref[..., :3]).max()
        en = np.abs(got[1][..., :3] - rn[..., :3]).max()
        ea = np.abs(got[2][..., :3] - ra[..., :3]).max()
        assert err <= 1e-5 and en <= 1e-6 and ea <= 1e-6


def test_voxelize_empty_and_nonfinite_inputs():
    empty = vct.voxelize(torch.zeros((0, 3, 3), device=DEV), torch.zeros((0, 3), device=DEV), vct.Grid(16), LIGHTS)
    assert not empty.any()
    bad = np.array([[[0.1, 0.1, np.nan], [0.5, 0.2, 0.3], [0.2, 0.5, 0.3]],
                    [[0.2, 0.2, 1e9], [0.5, 0.2, 0.3], [0.2, 0.5, 0.3]]], np.float32)
    assert not gpu_voxelize(bad, np.ones((2, 3), np.float32), 16).any()
