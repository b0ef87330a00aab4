"""The checked CPU build: every library source compiled for the host, with
the gfx950 execution model emulated (tests/hostemu: 64-lane waves as
cooperative fibers, so the cross-lane reduction butterflies run as written;
range-checked buffer-resource loads; bounds hooks on every texel and
accumulator index), driven through the C ABI and compared with the FP64
oracle on edge shapes: a 1^3 grid, a 2-level 16^3 pyramid, ragged tiles,
float16 and bfloat16 storage, anisotropic 2^3 and 8^3 pyramids, shading,
the allocation-free backward, and a 512^3 float32 pyramid (2.3 GiB, every
coarse level past byte 2^31) with a sparse G-buffer.  A second build with
AddressSanitizer and UndefinedBehaviorSanitizer runs the small cases."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from oracle import vct_aniso as va
from oracle import vct_shade as vs
from scenes import ConeParams, cone_set, make_workload, random_gbuffer, random_grid, random_material, scene_lights
from tests.hostemu.driver import run_case, run_voxelize
from tests.parity import fmt, range_errors, worst

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2104_00618_amd", "csrc")
EMU = os.path.join(ROOT, "tests", "hostemu")
SOURCES = ["api.cpp", "mips.hip", "trace.hip", "backward.hip", "shade.hip", "voxelize.hip", "bounce.hip"]
CLANG = "/opt/rocm/llvm/bin/clang++"


def _build(out_dir, extra):
    """Compile the library sources, the emulator and the harness for the host."""
    if not os.path.exists(CLANG):
        pytest.skip("ROCm clang++ is not installed")
    os.makedirs(out_dir, exist_ok=True)
    flags = ["-std=c++17", "-D__HIP_PLATFORM_AMD__", "-DVCT_HOST_EMULATION", "-I/opt/rocm/include",
             f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}", f"-I{EMU}", "-Wno-unused-value",
             "-Wno-unused-function", *extra]
    jobs = []
    for src in SOURCES:
        jobs.append((src, [CLANG, *flags, "-x", "c++", "-include", "emu.h", "-c", os.path.join(CSRC, src), "-o",
                           os.path.join(out_dir, src + ".o")]))
    jobs.append(("emu.cpp", [CLANG, *flags, "-include", "emu.h", "-c", os.path.join(EMU, "emu.cpp"), "-o",
                             os.path.join(out_dir, "emu.o")]))
    for name in ("harness.cpp", "abi_checks.cpp", "voxelize_case.cpp"):
        jobs.append((name, [CLANG, *flags, "-c", os.path.join(EMU, name), "-o",
                            os.path.join(out_dir, name[:-4] + ".o")]))
    procs = [(name, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True))
             for name, cmd in jobs]
    for name, p in procs:
        out, _ = p.communicate()
        assert p.returncode == 0, f"{name}:\n{out[-4000:]}"
    exe = os.path.join(out_dir, "harness")
    objs = [os.path.join(out_dir, f) for f in os.listdir(out_dir) if f.endswith(".o")]
    r = subprocess.run([CLANG, *extra, *objs, "-o", exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    return exe


@pytest.fixture(scope="module")
def checked(tmp_path_factory):
    return _build(str(tmp_path_factory.mktemp("emu") / "plain"), ["-O2"])


@pytest.fixture(scope="module")
def sanitized(tmp_path_factory):
    return _build(str(tmp_path_factory.mktemp("emu") / "asan"),
                  ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                   "-fno-sanitize-recover=undefined"])


def _params(kind="six", **kw):
    d, w = cone_set(kind)
    return ConeParams(d, w, **{"alpha_thresh": 0.99, **kw})


def _check_forward(res, ref, amb, label, tol=1e-5):
    keep = ~amb.reshape(-1)
    for name in ("trace", "save"):
        if name in res:
            e = range_errors(res[name], ref, keep)
            print(f"{label} {name}: {fmt(e)}", flush=True)
            assert worst(e)[0] <= tol, (label, name)


def _check_grad(got, ref, label):
    scale = np.abs(ref).max()
    err = np.abs(got - ref).max() / scale
    rms = np.sqrt(np.mean((got - ref) ** 2)) / scale
    print(f"{label} gradient: max {err:.2e} rms {rms:.2e}", flush=True)
    assert err <= 1e-4 and rms <= 1e-5, label


def _case(binary, tmp, base, pr, nr, cam, p, label, levels=None, dtype="f32", seed=0, **kw):
    """One case through the checked build against the oracle: forward, saved
    backward, and the allocation-free backward bit for bit."""
    gout = np.random.default_rng(seed).normal(size=pr.shape[:3] + (8,)).astype(np.float32)
    if dtype == "f32":
        mips = oracle.build_mips(base, levels)
    else:   # path parity: the oracle marches the build's own decoded levels
        dec = run_case(binary, str(tmp), base, pr, nr, cam, p, dtype=dtype, levels=levels, backward=False,
                       dump_levels=True, **kw)
        mips = [lv.astype(np.float64) for lv in dec["levels"][0]]
    ref, info = oracle.trace(mips, pr, nr, cam, p, return_info=True)
    gout[info["ambiguous"]] = 0.0          # (termination ties: no gradient through them)
    res = run_case(binary, str(tmp), base, pr, nr, cam, p, dtype=dtype, levels=levels, gout=gout, noalloc=True,
                   **kw)
    _check_forward(res, ref, info["ambiguous"], label)
    assert np.array_equal(res["grad_noalloc"].view(np.uint32), res["grad"].view(np.uint32)), label
    _check_grad(res["grad"], oracle.trace_backward(mips, pr, nr, cam, p, gout), label)
    n_all, n_two = (int(c) for c in res["count"])
    assert 0 <= n_two <= n_all, label
    if not info["ambiguous"].any():
        assert n_all == info["samples"], label
    return res


def test_emulated_library_matches_oracle_c3fd(checked, tmp_path):
    w = make_workload("c3fd", h=16, w=16)
    rng = np.random.default_rng(0)
    base = (0.6 * w.base + 0.05 * rng.uniform(size=w.base.shape)).astype(np.float32)
    _case(checked, tmp_path, base, w.pos_rough, w.normal, w.cam_pos, w.params, "c3fd 16^3 2x16x16")


@pytest.mark.parametrize("dtype", ["f16", "bf16"])
def test_emulated_reduced_precision_path_parity(checked, tmp_path, dtype):
    n = 16
    base = random_grid(n, seed=5, alpha_max=0.3)
    pr, nr, cam = random_gbuffer(1, 13, 7, seed=6, n=n)     # ragged: one partial tile
    _case(checked, tmp_path, base, pr, nr, cam, _params("five"), f"16^3 {dtype} 1x13x7", dtype=dtype)


@pytest.mark.parametrize("n,levels,shape", [(1, None, (1, 9, 11)), (16, 2, (2, 13, 7)), (2, None, (1, 5, 3))])
def test_emulated_tiny_and_partial_pyramids(checked, tmp_path, n, levels, shape):
    base = random_grid(n, seed=10 + n, alpha_max=0.4)
    pr, nr, cam = random_gbuffer(*shape, seed=20 + n, n=max(n, 8))
    _case(checked, tmp_path, base, pr, nr, cam, _params(), f"{n}^3 levels {levels} {shape}", levels=levels)


@pytest.mark.parametrize("n,flat", [(2, False), (8, False), (8, True)])
def test_emulated_anisotropic_pyramids(checked, tmp_path, n, flat):
    """Anisotropic forward, saved forward, backward and the allocation-free
    backward.  flat: every pixel on one plane with one normal, so the diffuse
    cones of a wave share their axis and the scatter pass sums each group once
    for the three directions."""
    base = random_grid(n, seed=30 + n, alpha_max=0.35)
    pr, nr, cam = random_gbuffer(1, 8, 8, seed=40 + n, n=max(n, 8))
    if flat:
        g = np.linspace(0.2, 0.8, 8, dtype=np.float32)
        pr[0, :, :, 0], pr[0, :, :, 1] = np.meshgrid(g, g)
        pr[0, :, :, 2] = 0.3
        nr[0, :, :, 0:3] = (0.0, 0.0, 1.0)
        nr[0, :, :, 3] = 1.0
    p = _params()
    gout = np.random.default_rng(n).normal(size=(1, 8, 8, 8)).astype(np.float32)
    am = va.build_aniso_mips(base)
    ref, info = va.trace_aniso(am, pr, nr, cam, p, return_info=True)
    gout[info["ambiguous"]] = 0.0
    res = run_case(checked, str(tmp_path), base, pr, nr, cam, p, aniso=True, gout=gout, noalloc=True)
    label = f"anisotropic {n}^3{' flat' if flat else ''}"
    _check_forward(res, ref, info["ambiguous"], label)
    assert np.array_equal(res["grad_noalloc"].view(np.uint32), res["grad"].view(np.uint32))
    _check_grad(res["grad"], va.trace_backward_aniso(am, pr, nr, cam, p, gout), label)


def test_emulated_shading_matches_oracle(checked, tmp_path):
    w = make_workload("c3fd", h=12, w=12, views=1)
    mat = random_material(w.shape, seed=3)
    sp = scene_lights(2)
    res = run_case(checked, str(tmp_path), w.base, w.pos_rough, w.normal, w.cam_pos, w.params, backward=False,
                   shade=sp, material=mat)
    ref, info = vs.shade(oracle.build_mips(w.base), w.pos_rough, w.normal, mat, w.cam_pos, w.params, sp,
                         return_info=True)
    e = range_errors(res["shade"], ref, ~info["ambiguous"].reshape(-1))
    print(f"shade c3fd 1x12x12: {fmt(e)}", flush=True)
    assert worst(e)[0] <= 5e-5


@pytest.mark.parametrize("kind,aniso", [("one", True), ("five", False)])
def test_emulated_bounce_matches_oracle(checked, tmp_path, kind, aniso):
    """The further bounce through the checked build: flag, scan and list of the
    surface voxels, and the gather with one workgroup of 64 lanes per diffuse
    cone (a single cone: 64-thread workgroups) on a voxelized Cornell mesh."""
    from oracle import vct_bounce as vb
    from oracle import vct_voxelize as vx
    from scenes.mesh import cornell_mesh
    n = 16
    tris, cols = cornell_mesh(2)
    lights = [((0.5, 0.95, 0.5), (1.0, 1.0, 1.0), (1.0, 0.5, 0.25))]
    base, nrm, alb = (a.astype(np.float32) for a in vx.voxelize(tris, cols, n, lights, return_surface=True))
    if kind == "one":
        p = ConeParams(np.array([[0.0, 0.0, 1.0]], np.float32), np.array([1.0], np.float32), alpha_thresh=0.99)
    else:
        p = _params("five")
    e = np.zeros((1, 1, 1, 4), np.float32)
    res = run_case(checked, str(tmp_path), base, e, e, np.zeros((1, 3), np.float32), p, aniso=aniso,
                   backward=False, bounce=(nrm, alb))
    if aniso:
        am = va.build_aniso_mips(base)
        ref, info = vb.bounce(base, nrm, alb, p, mips=am[0], sampler=va.aniso_sampler(am), return_info=True)
    else:
        ref, info = vb.bounce(base, nrm, alb, p, return_info=True)
    near = np.abs(np.linalg.norm(nrm[..., 0:3].astype(np.float64), axis=-1) - vb.MIN_NORMAL) < 1e-6
    keep = ~(info["ambiguous"] | near)
    got = res["bounce"]
    inc_g = (got[..., 0:3] - base[..., 0:3]).reshape(-1, 3)
    inc_r = (ref[..., 0:3] - base[..., 0:3]).reshape(-1, 3)
    err = range_errors(inc_g, inc_r, keep.reshape(-1))
    print(f"bounce {n}^3 {kind} cone(s) {'anisotropic' if aniso else 'isotropic'}: {fmt(err)}", flush=True)
    assert worst(err)[0] <= 1e-5 and np.abs(inc_r).max() > 0
    same = (ref[..., 0:3] == base[..., 0:3]).all(-1) & keep
    assert np.array_equal(got[same].view(np.uint32), base[same].view(np.uint32))


@pytest.mark.parametrize("surface,small", [(True, 0), (False, 0), (True, 4200)])
def test_emulated_voxelization_matches_oracle(checked, sanitized, tmp_path, surface, small):
    """vct_voxelize through the checked build (setup, offset scan, the raster
    pass that claims one accumulator slot per reached voxel, the resolve of
    the used slots) and its AddressSanitizer build, on the Cornell mesh plus
    random triangles at 16^3: occupancy bit-exact, colours within 1e-5 of the
    largest, normals and albedo within 1e-6.  With 4,200 more small triangles
    the mesh passes the one-workgroup scan's 4,096 and takes the blocked one."""
    from oracle import vct_voxelize as vx
    from scenes.mesh import cornell_mesh
    n = 16
    tris, cols = cornell_mesh(2)
    rng = np.random.default_rng(11)
    tris = np.concatenate([tris, rng.uniform(-0.1, 1.1, size=(24, 3, 3)).astype(np.float32)])
    cols = np.concatenate([cols, rng.uniform(0, 1, size=(24, 3)).astype(np.float32)])
    if small:
        ctr = rng.uniform(0.0, 1.0, size=(small, 1, 3))
        tris = np.concatenate([tris, (ctr + rng.uniform(-0.06, 0.06, size=(small, 3, 3))).astype(np.float32)])
        cols = np.concatenate([cols, rng.uniform(0, 1, size=(small, 3)).astype(np.float32)])
        assert len(tris) > 4096
    lights = [((0.5, 0.95, 0.5), (1.0, 1.0, 1.0), (1.0, 0.5, 0.25)), ((0.2, 0.3, 0.8), (0.4, 0.3, 0.2), (1, 0, 0))]
    ref = vx.voxelize(tris, cols, n, lights, return_surface=True)
    for build in (checked, sanitized):
        got = run_voxelize(build, str(tmp_path / os.path.basename(os.path.dirname(build))), tris, cols, n, lights,
                           surface=surface)
        occ = ref[0][..., 3] > 0
        assert np.array_equal(got[0][..., 3], ref[0][..., 3].astype(np.float32))
        assert occ.sum() > 100 and (got[0][~occ] == 0).all()
        err = np.abs(got[0][..., 0:3] - ref[0][..., 0:3]).max() / np.abs(ref[0][..., 0:3]).max()
        msg = f"voxelize {n}^3 {len(tris)} triangles surface={surface}: colour {err:.2e}"
        assert err <= 1e-5
        if surface:
            for k, name in ((1, "normal"), (2, "albedo")):
                assert np.array_equal(got[k][..., 3], ref[k][..., 3].astype(np.float32))
                e = np.abs(got[k][..., 0:3] - ref[k][..., 0:3]).max()
                msg += f", {name} {e:.2e}"
                assert e <= 1e-6
        print(msg, flush=True)


def test_emulated_512_cubed_float32_pyramid_past_2_gib(checked, tmp_path):
    """A 512^3 float32 pyramid (2.3 GiB, every level above 0 at a byte offset
    of 2^31 or more) with a sparse G-buffer inside the corner block
    [256, 512)^3, whose pyramid restricted to the block is the pyramid of the
    block alone (the oracle runs on that window): the mip build, the forward
    and the forward that keeps lane states.  Every lane takes the scalar-load
    path here, so each of its offsets is checked against the 32-bit range and
    the allocation.  (The backward's 4.9 GB accumulator would take minutes of
    page faults here; the GPU tests run it at this size.)"""
    n, w0 = 512, 256
    block = random_grid(n - w0, seed=77, alpha_max=0.25)
    rng = np.random.default_rng(5)
    h, wd = 4, 8
    pos = rng.uniform(0.65, 0.85, size=(1, h, wd, 3))
    nrm = rng.normal(size=(1, h, wd, 3))
    nrm /= np.linalg.norm(nrm, axis=-1, keepdims=True)
    pr = np.concatenate([pos, rng.uniform(0.05, 0.3, size=(1, h, wd, 1))], -1).astype(np.float32)
    nr = np.concatenate([nrm, np.ones((1, h, wd, 1))], -1).astype(np.float32)
    cam = np.array([[0.75, 0.75, 0.5]], np.float32)
    ap = float(np.float32(0.349))
    p = _params(diffuse_aperture=ap, spec_aperture_scale=ap, occ_aperture=ap, light_pos=(0.85, 0.95, 0.85),
                max_dist=0.1)
    origin, extent = (w0 / n,) * 3, (n - w0) / n
    ref, info = oracle.trace(oracle.build_mips(block), pr, nr, cam, p, origin, extent, return_info=True)
    res = run_case(checked, str(tmp_path), block, pr, nr, cam, p, n=n, block_origin=w0, save_only=True,
                   timeout=1200)
    _check_forward(res, ref, info["ambiguous"], "512^3 f32 window")


def test_sanitized_build_runs_the_small_cases_clean(sanitized, tmp_path):
    """AddressSanitizer and UndefinedBehaviorSanitizer over the whole host
    build (the C ABI's validation and planning code included): a forward,
    saved and allocation-free backward and shading on small grids, isotropic
    and anisotropic.  Any report aborts the harness and fails the case."""
    w = make_workload("c3fd", h=8, w=8, views=1)
    _case(sanitized, tmp_path / "a", w.base, w.pos_rough, w.normal, w.cam_pos, w.params, "asan c3fd 1x8x8")
    base = random_grid(2, seed=3, alpha_max=0.4)
    pr, nr, cam = random_gbuffer(1, 5, 3, seed=4, n=8)
    run_case(sanitized, str(tmp_path / "b"), base, pr, nr, cam, _params(), aniso=True,
             gout=np.ones((1, 5, 3, 8), np.float32), noalloc=True)
    run_case(sanitized, str(tmp_path / "c"), w.base, w.pos_rough, w.normal, w.cam_pos, w.params, backward=False,
             shade=scene_lights(2), material=random_material(w.shape, seed=1))


def test_sanitized_build_rejects_bad_arguments_cleanly(sanitized):
    """The C ABI's validation under AddressSanitizer and
    UndefinedBehaviorSanitizer: null, negative, non-finite, oversized and
    overflowing arguments to every entry point give the documented code and
    a "function: message" error without touching a buffer (the pointers
    passed are not allocations), and valid size queries clear the error."""
    r = subprocess.run([sanitized, "--abi"], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    n = int(r.stdout.strip().rsplit(":", 1)[1])
    print(f"abi checks passed: {n}")
    assert n >= 90
