"""Pins of the voxelization oracle (triangle rasterization along the dominant
axis with direct-light injection) against closed forms and counting facts,
not against its own formulas.  CPU only."""
import math

import numpy as np
import pytest

from oracle import vct_voxelize as vx

N = 32
V0 = 1.0 / N
LIGHT = ((0.5, 0.5, 0.9), (1.0, 1.0, 1.0), (1.0, 0.0, 0.0))


def quad(x0, x1, y0, y1, z, up=True):
    """Two triangles covering [x0,x1] x [y0,y1] at height z, normal +z (up) or -z."""
    a, b, c, d = (x0, y0, z), (x1, y0, z), (x1, y1, z), (x0, y1, z)
    t = [(a, b, c), (a, c, d)] if up else [(a, c, b), (a, d, c)]
    return np.array(t, np.float32)


def test_axis_aligned_quad_fills_exactly_its_pixel_centres():
    # edges between pixel centres: the covered set is a closed-form rectangle
    x0, x1, y0, y1, z = 0.1, 0.62, 0.23, 0.77, 0.4
    out, cnt = vx.voxelize(quad(x0, x1, y0, y1, z), np.ones((2, 3), np.float32), N, [LIGHT], return_counts=True)
    centres = (np.arange(N) + 0.5) * V0
    xs = (centres > x0) & (centres < x1)
    ys = (centres > y0) & (centres < y1)
    layer = int(math.floor(z * N))
    expect = np.zeros((N, N, N), dtype=bool)
    expect[layer] = ys[:, None] & xs[None, :]
    np.testing.assert_array_equal(out[..., 3] == 1.0, expect)
    # the shared diagonal is covered once: every voxel holds exactly one fragment
    assert set(np.unique(cnt[expect])) == {1}


def test_quad_wider_than_the_grid_fills_its_whole_layer():
    """Every pixel centre of the N x N viewport lies inside, the last row and
    column included: one layer of N^2 voxels, one fragment each."""
    z = 0.4
    out, cnt = vx.voxelize(quad(-0.01, 1.01, -0.02, 1.03, z), np.ones((2, 3), np.float32), N, [LIGHT],
                           return_counts=True)
    layer = int(math.floor(z * N))
    expect = np.zeros((N, N, N), dtype=bool)
    expect[layer] = True
    np.testing.assert_array_equal(out[..., 3] == 1.0, expect)
    assert set(np.unique(cnt[expect])) == {1}


def test_edges_through_pixel_centres_are_covered_once():
    # corners on pixel centres: all four edges and the diagonal pass through centres
    c = lambda i: (i + 0.5) * V0  # noqa: E731
    tris = quad(c(3), c(20), c(5), c(22), 0.5)
    out, cnt = vx.voxelize(tris, np.ones((2, 3), np.float32), N, [LIGHT], return_counts=True)
    layer = int(math.floor(0.5 * N))
    covered = cnt[layer] > 0
    # top-left rule: of the square's 18 x 18 centres exactly 17 x 17 are in (two edges keep, two drop)
    assert covered.sum() == 17 * 17
    assert cnt.max() == 1
    # a neighbouring quad sharing the right edge takes exactly the dropped column
    out2, cnt2 = vx.voxelize(np.concatenate([tris, quad(c(20), c(25), c(5), c(22), 0.5)]),
                             np.ones((4, 3), np.float32), N, [LIGHT], return_counts=True)
    assert cnt2.max() == 1 and (cnt2[layer] > 0).sum() == 22 * 17


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_dominant_axis_puts_a_flat_triangle_in_one_layer(axis):
    tri = np.zeros((1, 3, 3), np.float32)
    # place the triangle in the plane coordinate[axis] = 0.6
    other = [k for k in range(3) if k != axis]
    tri[0, :, other[0]] = [0.2, 0.8, 0.5]
    tri[0, :, other[1]] = [0.3, 0.25, 0.85]
    tri[0, :, axis] = 0.6
    out, cnt = vx.voxelize(tri, np.ones((1, 3), np.float32), N, [LIGHT], return_counts=True)
    idx = np.argwhere(cnt > 0)                    # (z, y, x)
    assert len(idx) > 20
    assert np.all(idx[:, 2 - axis] == int(0.6 * N))


def test_tilted_triangle_rasterizes_along_its_largest_normal_component():
    # normal ~ (3, 2, 1): x-dominant, so every (y, z) column holds at most one fragment
    tri = np.array([[[0.5, 0.1, 0.1], [0.1, 0.7, 0.1], [0.3, 0.1, 0.7]]], np.float32)
    n = np.cross(tri[0, 1] - tri[0, 0], tri[0, 2] - tri[0, 0])
    assert np.argmax(np.abs(n)) == 0
    _, cnt = vx.voxelize(tri, np.ones((1, 3), np.float32), N, [LIGHT], return_counts=True)
    cols = cnt.sum(axis=2)                        # over x
    assert cols.max() == 1 and cols.sum() > 30


def test_direct_light_closed_form_and_attenuation():
    z = 0.5
    tris = quad(0.1, 0.9, 0.1, 0.9, z)
    col = np.array([[0.8, 0.5, 0.25]] * 2, np.float32)
    lp, h = (0.5, 0.5, 0.85), 0.35
    att = (1.5, 2.0, 3.0)
    amb, dif = 0.125, 0.75
    out = vx.voxelize(tris, col, N, [(lp, (1.0, 0.5, 0.25), att)], ambient=amb, diffuse=dif)
    layer = int(z * N)
    for j, i in ((5, 5), (16, 16), (9, 20)):
        p = np.array([(i + 0.5) * V0, (j + 0.5) * V0, z])
        d = np.linalg.norm(np.array(lp) - p)
        cos = (lp[2] - z) / d
        expect = np.array(col[0], np.float64) * (amb + dif * cos) * np.array([1.0, 0.5, 0.25]) / (1.5 + 2 * d + 3 * d * d)
        np.testing.assert_allclose(out[layer, j, i, 0:3], expect, rtol=1e-12)
        assert out[layer, j, i, 3] == 1.0
    # facing away from the light: ambient only
    out = vx.voxelize(quad(0.1, 0.9, 0.1, 0.9, z, up=False), col, N, [(lp, (1, 1, 1), (1, 0, 0))], ambient=amb,
                      diffuse=dif)
    np.testing.assert_allclose(out[layer, 16, 16, 0:3], col[0] * amb, rtol=1e-6)


def test_coincident_triangles_average():
    t = quad(0.1, 0.9, 0.1, 0.9, 0.3)
    tris = np.concatenate([t, t])
    cols = np.array([[1, 0, 0], [1, 0, 0], [0, 0, 1], [0, 0, 1]], np.float32)
    out, cnt = vx.voxelize(tris, cols, N, [LIGHT], return_counts=True)
    one = vx.voxelize(t, np.array([[1, 1, 1]] * 2, np.float32), N, [LIGHT])
    hit = cnt > 0
    assert set(np.unique(cnt[hit])) == {2}
    np.testing.assert_allclose(out[hit][:, 0], 0.5 * one[hit][:, 0], rtol=1e-12)
    np.testing.assert_allclose(out[hit][:, 2], 0.5 * one[hit][:, 2], rtol=1e-12)
    assert np.all(out[hit][:, 1] == 0)


def test_fragment_count_matches_projected_area():
    rng = np.random.default_rng(3)
    for _ in range(5):
        tri = rng.uniform(0.05, 0.95, size=(1, 3, 3)).astype(np.float32)
        n = np.cross(tri[0, 1] - tri[0, 0], tri[0, 2] - tri[0, 0]).astype(np.float64)
        dom = int(np.argmax(np.abs(n)))
        area = 0.5 * abs(n[dom]) / V0 ** 2          # projected area in pixels
        per = sum(np.linalg.norm(np.delete(tri[0, (k + 1) % 3] - tri[0, k], dom)) for k in range(3)) / V0
        _, cnt = vx.voxelize(tri, np.ones((1, 3), np.float32), N, [LIGHT], return_counts=True)
        # every covered pixel centre lies within half a pixel diagonal of the triangle
        assert abs(cnt.sum() - area) <= per * math.sqrt(0.5) + 1


def test_degenerate_outside_and_nonfinite_triangles_produce_nothing():
    tris = np.array([[[0.1, 0.1, 0.1], [0.5, 0.5, 0.5], [0.9, 0.9, 0.9]],       # collinear
                     [[2.0, 2.0, 2.0], [3.0, 2.0, 2.0], [2.0, 3.0, 2.0]],       # outside the grid
                     [[0.1, 0.1, np.nan], [0.5, 0.2, 0.3], [0.2, 0.5, 0.3]],    # non-finite
                     [[0.2, 0.2, 1e9], [0.5, 0.2, 0.3], [0.2, 0.5, 0.3]]],      # beyond the exact range
                    np.float32)
    out = vx.voxelize(tris, np.ones((4, 3), np.float32), N, [LIGHT])
    assert not out.any()


def test_snapping_rounds_to_the_nearest_subpixel_ties_to_even():
    """Reading V6 worked on exact float32 inputs at N = 16 (4096 subpixels per
    unit): k + 1/4 snaps down, k + 3/4 up, k + 1/2 to the even neighbour, on
    both sides of the origin."""
    n = 16
    frac = [(4.25, 4), (4.75, 5), (4.5, 4), (5.5, 6), (-4.75, -5), (-4.25, -4), (-5.5, -6), (0.5, 0)]
    coords = np.array([f for f, _ in frac], np.float64) / (vx.SUB * n)
    tris = np.zeros((len(frac), 3, 3), np.float32)
    tris[:, 0, 0] = coords
    u, ok = vx.snap(tris, n)
    assert ok.all()
    assert u[:, 0, 0].tolist() == [k for _, k in frac]
