"""Benchmark of the voxel-cone-tracing hot path on one GPU.

A step is one pass of the whole hot path over the 256^3 / 1920x1080 scene, as
a training step runs it: vct_build_mips (float32 grid -> pyramid),
vct_trace_save (5 diffuse + specular + occlusion cones per pixel, keeping each
cone's end state) and vct_trace_backward_saved (gradient into the float32 base
grid for a seeded dL/d(out)).  Inputs are resident in HBM before timing.

    python bench.py [--steps K] [--warmup W] [--dtype f32|f16|bf16] [--no-cpu-baseline] [--no-configs]

Prints one JSON line.  value = forward cone samples per second of the whole
fwd+bwd step; the breakdown also gives the forward-only (vct_trace) rate, the
per-call and per-kernel times (HIP events on the stream the library launches
on), the step through vct_trace + vct_trace_backward (no saved state) and the
float16-storage forward for comparison.  `configs` times every configuration
of the workload family on its own (64^3 / 256^2; the 1080p scene at 64^3,
128^3 and 256^3; float16 and bfloat16 pyramids; the 128^3 fitting step; the
512^3 / 4 x 4K float16 scene), and `cpu_baseline` is the FP64 oracle on the
host's cores (at most 16 processes), timed before the GPU is used.
"""
import argparse
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("cone samples/s + ms/frame at 1080p (fwd, fwd+bwd), % HBM peak, FP16 vs FP32 storage")
HBM_PEAK_GBS = 8000.0
# MI355X's published FP32 vector peak (256 CUs at 2.4 GHz, counting packed
# FP32 instructions), and the ceiling without them: every kernel here is built
# with packed FP32 disabled, so its FMAs issue at 256 CUs x 4 SIMDs x 16 lanes
# x 2 flops x 2.4 GHz.
ALU_PEAK_TFLOPS = 157.3
ALU_NONPACKED_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
# Algorithmic FP32 operations (FMA = 2) of one cone sample, counted from the
# formulas.  Common to every sample: schedule 8, position 6, compositing 9,
# t update 2 (25); per level read: coordinates 6, floor/frac 6, 1 - phi 3,
# weights 12, 8 taps x 4 channels FMA 64 (91); the blend of two levels 13.
# A sample whose LOD is an integer reads one level (116), the others two (220).
# The scatter pass re-does the sample, forms its gradient (22) and the taps x
# channels weighted contributions with their accumulation (64 per level):
# 202 and 370.
FLOPS_FWD = {1: 116, 2: 220}
FLOPS_BWD_SCATTER = {1: 202, 2: 370}
BWD_KERNELS = ["clear accumulator", "bound from saved states", "scale", "pass 2 (re-march + scatter)", "mip adjoint"]
WORKLOAD = "c1"
WORKLOAD_DESC = ("procedural Cornell box 256^3 (9 levels, 4-8 boxes and spheres), 1 view 1920x1080, "
                 "5 diffuse cones (front + 4 at 45 deg, 60 deg aperture) + specular + occlusion, "
                 "beta 0.5, t0 0.001, max_dist 1, alpha_thresh 0.99")
# the thesis's frame times (whole OpenGL frame, GTX 1070; context only)
PAPER_FRAME_MS = {64: 16.66, 128: 31.3, 256: 127.4}


def flops(counts, model):
    """Algorithmic flops of a march with (samples, two-level samples)."""
    n, n2 = counts
    return (n - n2) * model[1] + n2 * model[2]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--dtype", default="f32", choices=["f32", "f16", "bf16"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true", help="skip the float16-storage forward comparison")
    ap.add_argument("--no-configs", action="store_true", help="skip the per-configuration rows")
    ap.add_argument("--cpu-workers", type=int, default=None,
                    help="host processes for the oracle baseline (default: the host's cores, at most 16)")
    return ap.parse_args()


# Sources that define each profiled kernel; HBM traffic measured by rocprofv3
# is reported only while their digest matches the one recorded with the counters.
KERNEL_SOURCES = {
    "k_bwd_pass2": ["backward.hip", "bwd_pixel.h", "march.h", "texel.h", "vct_internal.h"],
    "k_trace": ["trace.hip", "march.h", "texel.h", "vct_internal.h"],
}
PASS2_SOURCES = KERNEL_SOURCES["k_bwd_pass2"]
PROFILE = os.path.join(ROOT, "profiles", "cone_trace_256cubed_1080p_f32.md")


def code_text(text):
    """C++ source with comments removed and whitespace collapsed: the part of
    a file that can change a kernel."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_source_digest(csrc=None, kernel="k_bwd_pass2"):
    """Digest of the code (not the comments) of a kernel's sources."""
    import hashlib
    csrc = csrc or os.path.join(ROOT, "paper_2104_00618_amd", "csrc")
    files = PASS2_SOURCES if kernel == "k_bwd_pass2" else KERNEL_SOURCES[kernel]
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(csrc, f)) as fh:
            h.update(code_text(fh.read()).encode())
        h.update(b"\0")
    return h.hexdigest()[:16]


def _traffic_line(kernel):
    """The committed profile's traffic line of a kernel (a regex match), or (None, reason)."""
    try:
        text = open(PROFILE).read()
    except OSError:
        return None, "no profile"
    m = re.search(r"traffic " + kernel + r": fetch_bytes=(\d+) write_bytes=(\d+)(?: l2_hit=([0-9.]+))? "
                  r"sources=([0-9a-f]+)", text)
    if not m:
        return None, "no traffic line in the profile"
    if m.group(4) != kernel_source_digest(kernel=kernel):
        return None, "kernel sources changed since the counters were taken"
    return m, None


def measured_traffic(kernel="k_bwd_pass2"):
    """(bytes per launch, note) of a kernel from the committed profile, or (None, reason)."""
    m, why = _traffic_line(kernel)
    if m is None:
        return None, why
    return int(m.group(1)) + int(m.group(2)), f"FETCH_SIZE + WRITE_SIZE (calibrated) from {os.path.basename(PROFILE)}"


def measured_l2_hit(kernel="k_bwd_pass2"):
    """L2 hit rate TCC_HIT / (TCC_HIT + TCC_MISS) of a kernel from the committed profile, or None."""
    m, _ = _traffic_line(kernel)
    return float(m.group(3)) if (m is not None and m.group(3)) else None


def measured_pass2_traffic():
    return measured_traffic("k_bwd_pass2")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# inputs of the oracle baseline's worker processes (set before they are forked)
_CPU = {}


def _cpu_chunk(i):
    """Worker: the oracle's forward and adjoint of pixel chunk i (one thread)."""
    import oracle
    from threadpoolctl import threadpool_limits

    c = _CPU
    sl = slice(i * c["per"], (i + 1) * c["per"])
    pr, nr, go = c["pr"][:, :, sl], c["nr"][:, :, sl], c["gout"][:, :, sl]
    w = c["w"]
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        _, info = oracle.trace(c["mips"], pr, nr, w.cam_pos, w.params, return_info=True)
        t1 = time.perf_counter()
        g = oracle.trace_backward(c["mips"], pr, nr, w.cam_pos, w.params, go)
        t2 = time.perf_counter()
    return info["samples"], t1 - t0, t2 - t1, float(np.abs(g).sum())


def cpu_workers(requested=None):
    """Host processes for the oracle baseline: the host's cores, at most 16 (a
    one-GPU machine's share)."""
    return max(1, int(requested) if requested else min(16, os.cpu_count() or 1))


def cpu_baseline(w, workers=1, per_worker=4096, seed=0):
    """The FP64 oracle as it stands doing the step on a seeded pixel sample of
    the same frame, on `workers` host processes: build_mips of the full grid
    (one thread), then the forward of all cones of per_worker pixels and its
    adjoint (seeded dL/d(out)) in each process, each on one thread.  Every
    process runs the oracle's whole adjoint of its chunk, mip adjoint included.
    The processes are forked here, so call this before the GPU is touched.
    Returns the baseline and the timed parts (for the per-row table)."""
    import multiprocessing as mp

    import oracle
    from threadpoolctl import threadpool_limits
    from tests.workloads import sample_pixels

    n_pix = workers * per_worker
    v, y, x = sample_pixels(w.shape, n_pix, seed)
    t0 = time.perf_counter()
    with threadpool_limits(limits=1):
        mips = oracle.build_mips(w.base)
    t1 = time.perf_counter()
    _CPU.update(w=w, mips=mips, per=per_worker, pr=w.pos_rough[v, y, x][None, None],
                nr=w.normal[v, y, x][None, None],
                gout=np.random.default_rng(seed).normal(size=(1, 1, n_pix, 8)) * 1e-3)
    if workers == 1:
        res = [_cpu_chunk(0)]
        t2 = time.perf_counter()
    else:
        with mp.get_context("fork").Pool(workers) as pool:
            t1 = time.perf_counter()
            res = pool.map(_cpu_chunk, range(workers), chunksize=1)
            t2 = time.perf_counter()
    _CPU.clear()
    n = sum(r[0] for r in res)
    fwd_cpu, bwd_cpu = sum(r[1] for r in res), sum(r[2] for r in res)
    parts = {"mips_s": t1 - t0, "parallel_s": t2 - t1, "samples": n, "pixels": n_pix, "workers": workers,
             # (per-core rates times the cores: the two phases ran interleaved across processes)
             "forward_samples_per_s": n / fwd_cpu * workers, "backward_samples_per_s": n / bwd_cpu * workers}
    ncones = w.params.n_diffuse + int(w.params.enable_spec) + int(w.params.enable_occ)
    base = {"value": n / ((t1 - t0) + (t2 - t1)), "unit": "cone samples/s", "cores": workers, "kind": "oracle",
            "sample": f"build_mips of the {w.n}^3 grid (one thread, {t1 - t0:.1f} s), then the forward and adjoint "
                      f"of all {ncones} cones of {n_pix} seeded pixels of the {w.shape[2]}x{w.shape[1]} frame "
                      f"({n} samples) in {workers} processes of one thread each, {per_worker} pixels apiece, each "
                      f"with its own mip adjoint ({t2 - t1:.1f} s wall); NumPy FP64"}
    return base, parts


def cpu_rows(w, vox_mesh, vlights, seed=1):
    """The oracle on bounded samples of the other rows' workloads (seconds each)."""
    import oracle
    from oracle import vct_aniso, vct_bounce, vct_shade, vct_voxelize
    from scenes import random_material, scene_lights
    from tests.workloads import sample_pixels

    out = {}
    mips = oracle.build_mips(w.base)
    v, y, x = sample_pixels(w.shape, 2048, seed)
    pr, nr = w.pos_rough[v, y, x][None, None], w.normal[v, y, x][None, None]
    mat = random_material(pr.shape[:3], seed)
    t = time.perf_counter()
    vct_shade.shade(mips, pr, nr, mat, w.cam_pos, w.params, scene_lights(3))
    dt = time.perf_counter() - t
    out["f1_shade"] = {"value": 2048 / dt, "unit": "pixels/s", "cores": 1, "kind": "oracle",
                       "sample": f"2048 seeded pixels of the 1080p frame, 3 lights, pyramid given ({dt:.1f} s)"}
    tris, cols = vox_mesh
    t = time.perf_counter()
    vb, vn, va_ = vct_voxelize.voxelize(tris, cols, w.n, vlights, return_surface=True)
    dt = time.perf_counter() - t
    out["f2_voxelize"] = {"value": len(tris) / dt, "unit": "triangles/s", "cores": 1, "kind": "oracle",
                          "sample": f"the whole {len(tris)}-triangle Cornell mesh at {w.n}^3 with surface grids "
                                    f"({dt:.1f} s)"}
    surf = np.argwhere(vct_bounce.surface_mask(vb, vn))
    pick = surf[np.random.default_rng(seed).choice(len(surf), size=min(2000, len(surf)), replace=False)]
    t = time.perf_counter()
    vct_bounce.bounce(vb, vn, va_, w.params, voxels=pick)
    dt = time.perf_counter() - t
    out["f3_bounce"] = {"value": len(pick) / dt, "unit": "surface voxels/s", "cores": 1, "kind": "oracle",
                        "sample": f"{len(pick)} seeded surface voxels of the {w.n}^3 mesh grid, pyramid built "
                                  f"({dt:.1f} s)"}
    t = time.perf_counter()
    am = vct_aniso.build_aniso_mips(w.base)
    _, info = vct_aniso.trace_aniso(am, pr[:, :, :1024], nr[:, :, :1024], w.cam_pos, w.params, return_info=True)
    dt = time.perf_counter() - t
    out["f4_anisotropic"] = {"value": info["samples"] / dt, "unit": "cone samples/s", "cores": 1, "kind": "oracle",
                             "sample": f"anisotropic pyramids of the {w.n}^3 grid + all 7 cones of 1024 seeded "
                                       f"pixels ({info['samples']} samples, {dt:.1f} s)"}
    return out


BOUNCE_KERNELS = ["flag + copy", "scan", "list", "gather"]


def bench_bounce(vct, torch, grid, vt, vc, vlights, params, timed, steps):
    """One further bounce at the grid of the step: voxelize the Cornell mesh
    with surface normal and albedo grids, build the direct-light pyramid,
    bounce (surface voxels re-gather through it), and build the pyramid of the
    bounced grid for the final gather."""
    dev = vt.device
    n = grid.n
    shape = (n, n, n, 4)
    vbase, vnrm, valb, bout = (torch.empty(shape, dtype=torch.float32, device=dev) for _ in range(4))
    vws = torch.empty(vct.voxelize_workspace_bytes(grid, vt.shape[0], surface=True), dtype=torch.uint8, device=dev)
    vox_ms = timed(lambda: vct.voxelize(vt, vc, grid, vlights, base=vbase, workspace=vws, surface=True,
                                        normal=vnrm, albedo=valb), steps)
    del vws
    vpyr = vct.build_mips(vbase, grid)
    bws = torch.empty(vct.bounce_workspace_bytes(grid), dtype=torch.uint8, device=dev)
    bounce_ms = timed(lambda: vct.bounce(vpyr, grid, vbase, vnrm, valb, params, out=bout, workspace=bws), steps)
    kev = [vct.KernelEvents(len(BOUNCE_KERNELS) + 1) for _ in range(steps)]
    for k in kev:
        k.arm()
        vct.bounce(vpyr, grid, vbase, vnrm, valb, params, out=bout, workspace=bws)
    torch.cuda.synchronize()
    kms = np.mean([k.times() for k in kev], axis=0)
    remip_ms = timed(lambda: vct.build_mips(bout, grid, vpyr), steps)
    # cone samples of the bounce: the surface voxels as a one-row G-buffer (centres (i + 1/2) / N are exact
    # in float32 for this power-of-two grid over the unit cube, so the march and its count are the bounce's)
    a = vbase[..., 3] > 0
    nn = vnrm[..., 0:3]
    live = a & ((nn * nn).sum(-1) >= 1e-4)
    idx = torch.nonzero(live)                      # (z, y, x)
    m = int(idx.shape[0])
    rows = (m + 1023) // 1024                      # 1024-wide rows, the tail padded with background pixels
    pr = torch.zeros((rows * 1024, 4), device=dev)
    nr = torch.zeros((rows * 1024, 4), device=dev)
    pr[:m, 0:3] = (idx.flip(1).to(torch.float32) + 0.5) / n
    nr[:m, 0:3] = vnrm[live][:, 0:3]
    nr[:m, 3] = 1.0
    pr, nr = pr.reshape(1, rows, 1024, 4), nr.reshape(1, rows, 1024, 4)
    cam = torch.zeros((1, 3), device=dev)
    vct.build_mips(vbase, grid, vpyr)              # the direct-light pyramid the bounce marched through
    samples = vct.count_samples(vpyr, grid, pr, nr, cam, params.replace(enable_spec=False, enable_occ=False))
    flag_bytes = n ** 3 * 16 * 2                   # base read + copy written (out is not base here)
    res = {"surface_voxels": m, "cones_per_voxel": params.n_diffuse, "samples": samples,
           "voxelize_with_surface_ms": vox_ms, "bounce_ms": bounce_ms,
           "bounce_kernels_ms": {k: float(t) for k, t in zip(BOUNCE_KERNELS, kms)},
           "remip_ms": remip_ms, "voxelize_mips_bounce_mips_ms": vox_ms + 2 * remip_ms + bounce_ms,
           "gather_samples_per_s": samples / (kms[3] * 1e-3),
           "gather_frac_of_alu_peak": FLOPS_FWD[2] * samples / (kms[3] * 1e-3) / 1e12 / ALU_PEAK_TFLOPS,
           "flag_GBps": flag_bytes / (kms[0] * 1e-3) / 1e9,
           "flag_frac_of_hbm_peak": flag_bytes / (kms[0] * 1e-3) / 1e9 / HBM_PEAK_GBS}
    log(f"bounce: {m} surface voxels, {samples} samples; voxelize+surface {vox_ms:.3f} ms, bounce {bounce_ms:.3f} ms "
        f"({', '.join(f'{k} {t:.3f}' for k, t in zip(BOUNCE_KERNELS, kms))}), re-mip {remip_ms:.3f} ms")
    return res


def time_ms(torch, fn, reps, warm=1):
    """Mean ms per call of fn over reps calls (CUDA events on the current stream)."""
    for _ in range(warm):
        fn()
    e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    e[0].record()
    for _ in range(reps):
        fn()
    e[1].record()
    torch.cuda.synchronize()
    return e[0].elapsed_time(e[1]) / reps


def bench_config(vct, torch, w, dtype, reps, label, backward=True):
    """One configuration: forward (build_mips + trace) and training step
    (build_mips + trace_save + trace_backward_saved) per frame, cone samples
    and the rates.  Inputs resident in HBM; HIP events on the current stream."""
    dev = torch.device("cuda:0")
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
    base, pr, nr, cam = T(w.base), T(w.pos_rough), T(w.normal), T(w.cam_pos)
    g = vct.Grid(w.n, dtype=dtype)
    pyr = vct.build_mips(base, g)
    out = torch.empty(w.shape + (8,), dtype=torch.float32, device=dev)
    counts = vct.count_sample_levels(pyr, g, pr, nr, cam, w.params)
    npix = int(np.prod(w.shape))
    mips_ms = time_ms(torch, lambda: vct.build_mips(base, g, pyr), reps)
    trace_ms = time_ms(torch, lambda: vct.trace(pyr, g, pr, nr, cam, w.params, out), reps)
    r = {"grid": w.n, "levels": w.levels, "views": w.shape[0], "height": w.shape[1], "width": w.shape[2],
         "cones_per_pixel": w.params.n_diffuse + 2, "storage": dtype, "pyramid_bytes": int(pyr.numel()),
         "samples_per_frame": counts[0], "two_level_samples": counts[1], "samples_per_pixel": counts[0] / npix,
         "build_mips_ms": mips_ms, "trace_ms": trace_ms, "fwd_ms_per_frame": mips_ms + trace_ms,
         "fwd_samples_per_s": counts[0] / ((mips_ms + trace_ms) * 1e-3),
         "trace_frac_of_alu_peak": flops(counts, FLOPS_FWD) / (trace_ms * 1e-3) / 1e12 / ALU_PEAK_TFLOPS}
    if backward:
        st = torch.empty(vct.lane_state_bytes(pr, nr, cam, w.params), dtype=torch.uint8, device=dev)
        ws = torch.empty(vct.backward_workspace_bytes(g, pr, nr, cam, w.params) - st.numel(), dtype=torch.uint8,
                         device=dev)
        gout = T((np.random.default_rng(0).normal(size=w.shape + (8,)) * 1e-3).astype(np.float32))
        gb = torch.empty_like(base)
        save_ms = time_ms(torch, lambda: vct.trace_save(pyr, g, pr, nr, cam, w.params, out, st), reps)
        bwd_ms = time_ms(torch, lambda: vct.trace_backward_saved(pyr, g, pr, nr, cam, w.params, st, gout, ws, gb),
                         reps)
        r.update(trace_save_ms=save_ms, trace_backward_saved_ms=bwd_ms, fwd_bwd_ms_per_frame=mips_ms + save_ms + bwd_ms,
                 fwd_bwd_samples_per_s=counts[0] / ((mips_ms + save_ms + bwd_ms) * 1e-3))
        del st, ws, gb, gout
    log(f"{label}: {w.n}^3 {dtype}, {w.shape[0]}x{w.shape[2]}x{w.shape[1]}, {counts[0]} samples; fwd "
        f"{r['fwd_ms_per_frame']:.3f} ms" + (f", fwd+bwd {r['fwd_bwd_ms_per_frame']:.3f} ms" if backward else ""))
    del pyr, out, base
    torch.cuda.empty_cache()
    return r


def bench_configs(vct, torch, make_workload):
    """The configurations of the workload family, each timed on its own:
    64^3 / 256^2 (6+1+1 cones, alpha_thresh 1), the 1080p scene at 64^3,
    128^3 and 256^3 (the thesis's frame-time table sweeps the grid size),
    float16 and bfloat16 pyramids of the 256^3 scene, the 128^3 / 8 x 512^2
    fitting step and the 512^3 / 4 x 3840x2160 scene with float16 and float32
    pyramids."""
    dev = "cuda:0"
    cfg = {}
    cfg["c0_64cubed_256sq_f32"] = bench_config(vct, torch, make_workload("c0", device=dev), "f32", 20, "c0")
    sweep = {}
    for n in (64, 128, 256):
        wn = make_workload("c1", n=n, device=dev)
        r = bench_config(vct, torch, wn, "f32", 10, f"1080p sweep {n}^3")
        r["thesis_frame_ms_gtx1070"] = PAPER_FRAME_MS[n]
        sweep[f"{n}cubed"] = r
    cfg["c1_1080p_grid_sweep_f32"] = sweep
    w1 = make_workload("c1", device=dev)
    for dt in ("f16", "bf16"):
        r = bench_config(vct, torch, w1, dt, 10, f"c2 {dt}")
        r["trace_speedup_vs_f32"] = sweep["256cubed"]["trace_ms"] / r["trace_ms"]
        r["fwd_speedup_vs_f32"] = sweep["256cubed"]["fwd_ms_per_frame"] / r["fwd_ms_per_frame"]
        r["fwd_bwd_speedup_vs_f32"] = sweep["256cubed"]["fwd_bwd_ms_per_frame"] / r["fwd_bwd_ms_per_frame"]
        cfg[f"c2_256cubed_1080p_{dt}"] = r
    del w1
    cfg["c3_fit_step_128cubed_8x512sq_f32"] = bench_config(vct, torch, make_workload("c3gt", device=dev), "f32", 10,
                                                           "c3 fit step")
    t0 = time.perf_counter()
    w4 = make_workload("c4", device=dev)
    log(f"c4 workload generated on the GPU in {time.perf_counter() - t0:.1f} s")
    c4 = bench_config(vct, torch, w4, "f16", 3, "c4")
    # the same frame through a float32 pyramid (2.45 GB): where the pyramid no
    # longer sits in the caches, what the float16 storage buys
    c4f = bench_config(vct, torch, w4, "f32", 3, "c4 f32")
    for k in ("trace", "fwd", "fwd_bwd"):
        key = "trace_ms" if k == "trace" else f"{k}_ms_per_frame"
        c4[f"{k}_speedup_vs_f32"] = c4f[key] / c4[key]
    cfg["c4_512cubed_4x4k_f16"] = c4
    cfg["c4_512cubed_4x4k_f32"] = c4f
    del w4
    return cfg


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the library has no multi-GPU "
              f"implementation", file=sys.stderr)
        sys.exit(2)
    from scenes import make_workload

    t0 = time.perf_counter()
    w = make_workload(WORKLOAD)
    log(f"workload generated in {time.perf_counter() - t0:.1f} s")
    cpu_base = cpu_parts = None
    if not args.no_cpu_baseline:
        # first, before anything touches the GPU: the worker processes are forked
        nw = cpu_workers(args.cpu_workers)
        log(f"timing the oracle on {nw} host processes")
        cpu_base, cpu_parts = cpu_baseline(w, workers=nw)
        log(f"oracle: {cpu_base['value']:.3g} samples/s on {nw} cores")

    import torch

    import paper_2104_00618_amd as vct

    dev = torch.device("cuda:0")
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
    base, pr, nr, cam = T(w.base), T(w.pos_rough), T(w.normal), T(w.cam_pos)
    rng = np.random.default_rng(0)
    gout = T(rng.normal(size=w.shape + (8,)).astype(np.float32) * 1e-3)
    grid = vct.Grid(w.n, dtype=args.dtype)
    pyr = torch.empty(vct.pyramid_bytes(grid), dtype=torch.uint8, device=dev)
    out = torch.empty(w.shape + (8,), dtype=torch.float32, device=dev)
    ws_full = vct.backward_workspace_bytes(grid, pr, nr, cam, w.params)
    st_bytes = vct.lane_state_bytes(pr, nr, cam, w.params)
    ws = torch.empty(ws_full, dtype=torch.uint8, device=dev)
    state = torch.empty(st_bytes, dtype=torch.uint8, device=dev)
    ws_saved = ws[:ws_full - st_bytes]
    gbase = torch.empty_like(base)
    vct.build_mips(base, grid, pyr)
    counts = vct.count_sample_levels(pyr, grid, pr, nr, cam, w.params)
    samples = counts[0]
    npix = int(np.prod(w.shape))
    log(f"{samples} cone samples per frame ({samples / npix:.1f} per pixel, {counts[1] / samples:.3f} read two "
        f"levels), workspace {ws.numel() / 2**30:.2f} GiB, lane states {st_bytes / 2**30:.2f} GiB")

    # a plain copy of known size (256 MiB read + 256 MiB written): its
    # FETCH_SIZE / WRITE_SIZE counters calibrate the byte counters of the
    # profiled kernels
    cal_src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
    cal_dst = torch.empty_like(cal_src)
    cal_dst.copy_(cal_src)
    torch.cuda.synchronize()
    del cal_src, cal_dst

    def step(ev=None, kev=None):
        if ev is not None:
            ev[0].record()
        vct.build_mips(base, grid, pyr)
        if ev is not None:
            ev[1].record()
        vct.trace_save(pyr, grid, pr, nr, cam, w.params, out, state)
        if ev is not None:
            ev[2].record()
        if kev is not None:
            kev.arm()
        vct.trace_backward_saved(pyr, grid, pr, nr, cam, w.params, state, gout, ws_saved, gbase)
        if ev is not None:
            ev[3].record()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    kevs = [vct.KernelEvents(len(BWD_KERNELS) + 1) for _ in range(args.steps)]
    log(f"timing {args.steps} steps")
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.steps):
        step(evs[i], kevs[i])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    mips_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in evs]))
    save_ms = float(np.mean([e[1].elapsed_time(e[2]) for e in evs]))
    bwd_ms = float(np.mean([e[2].elapsed_time(e[3]) for e in evs]))
    bwd_k = np.mean([k.times() for k in kevs], axis=0)
    ms_step = wall * 1e3 / args.steps
    log(f"step {ms_step:.3f} ms: mips {mips_ms:.3f}, trace_save {save_ms:.3f}, backward {bwd_ms:.3f} "
        f"({', '.join(f'{n} {t:.3f}' for n, t in zip(BWD_KERNELS, bwd_k))})")

    # outside the timed steps: the forward alone (inference) and the step
    # through the entry points that keep no state
    def timed(fn, k):
        return time_ms(torch, fn, k)

    fwd_ms = timed(lambda: vct.trace(pyr, grid, pr, nr, cam, w.params, out), args.steps)
    # final shading with the thesis's cone variants (first-hit diffuse, occlusion
    # falloff, angular-grace specular), one and three lights
    from scenes import random_material, scene_lights
    mat = T(random_material(w.shape, seed=11))
    shade_out = torch.empty(w.shape + (4,), dtype=torch.float32, device=dev)
    shade_ms = {f"{nl}_lights": timed(lambda nl=nl: vct.shade(pyr, grid, pr, nr, cam, mat, w.params, scene_lights(nl),
                                                                shade_out), args.steps) for nl in (1, 3)}
    shade_samples = vct.count_shade_samples(pyr, grid, pr, nr, cam, mat, w.params, scene_lights(3))
    recompute_bwd_ms = timed(lambda: vct.trace_backward(pyr, grid, pr, nr, cam, w.params, gout, ws, gbase),
                             max(args.steps // 2, 1))
    # per-frame revoxelization: voxelize the Cornell mesh (direct-light injection) into the 256^3 base grid
    from scenes.mesh import cornell_mesh
    vt, vc = cornell_mesh(1)
    vox_mesh = (vt, vc)
    vox_tris = int(vt.shape[0])
    vt, vc = T(vt), T(vc)
    vws = torch.empty(vct.voxelize_workspace_bytes(grid, vox_tris), dtype=torch.uint8, device=dev)
    vbase = torch.empty_like(base)
    vlights = [((0.5, 0.95, 0.5), (1.0, 1.0, 1.0), (1.0, 0.5, 0.25))]
    vox_ms = timed(lambda: vct.voxelize(vt, vc, grid, vlights, base=vbase, workspace=vws), args.steps)
    del vws
    # the same room with 256 x 512 spheres: 522,286 triangles, most smaller than a voxel
    bt, bc = cornell_mesh(1, rings=256, segments=512)
    big_tris = int(bt.shape[0])
    bt, bc = T(bt), T(bc)
    vws = torch.empty(vct.voxelize_workspace_bytes(grid, big_tris), dtype=torch.uint8, device=dev)
    vox_big_ms = timed(lambda: vct.voxelize(bt, bc, grid, vlights, base=vbase, workspace=vws), args.steps)
    del vws, bt, bc
    log(f"trace alone {fwd_ms:.3f} ms; recompute path step {mips_ms + fwd_ms + recompute_bwd_ms:.3f} ms; "
        f"shade {', '.join(f'{k} {v:.3f} ms' for k, v in shade_ms.items())}; voxelize {vox_ms:.3f} ms "
        f"({vox_tris} triangles), {vox_big_ms:.3f} ms ({big_tris} triangles)")
    bounce = bench_bounce(vct, torch, grid, vt, vc, vlights, w.params, timed, args.steps)
    # the same frame through an anisotropic (six-direction) pyramid
    ga = vct.Grid(w.n, dtype=args.dtype, anisotropic=True)
    pa = torch.empty(vct.pyramid_bytes(ga), dtype=torch.uint8, device=dev)
    amips_ms = timed(lambda: vct.build_mips(base, ga, pa), args.steps)
    atrace_ms = timed(lambda: vct.trace(pa, ga, pr, nr, cam, w.params, out), args.steps)
    asamples = vct.count_samples(pa, ga, pr, nr, cam, w.params)
    # training through it: forward with saved states, then the adjoint (directional
    # scatter + the per-level mip adjoint)
    aws = torch.empty(vct.backward_workspace_bytes(ga, pr, nr, cam, w.params) - st_bytes, dtype=torch.uint8,
                      device=dev)
    asave_ms = timed(lambda: vct.trace_save(pa, ga, pr, nr, cam, w.params, out, state), args.steps)
    abwd_ms = timed(lambda: vct.trace_backward_saved(pa, ga, pr, nr, cam, w.params, state, gout, aws, gbase),
                    args.steps)
    aniso = {"pyramid_bytes": int(pa.numel()), "isotropic_pyramid_bytes": int(pyr.numel()),
             "build_mips_ms": amips_ms, "trace_ms": atrace_ms, "samples_per_frame": asamples,
             "trace_samples_per_s": asamples / (atrace_ms * 1e-3), "fwd_ms_per_frame": amips_ms + atrace_ms,
             "trace_slowdown_vs_isotropic": atrace_ms / fwd_ms,
             "trace_save_ms": asave_ms, "trace_backward_saved_ms": abwd_ms,
             "fwd_bwd_ms_per_frame": amips_ms + asave_ms + abwd_ms,
             "backward_slowdown_vs_isotropic": abwd_ms / bwd_ms}
    del pa
    log(f"anisotropic: mips {amips_ms:.3f} ms, trace {atrace_ms:.3f} ms ({asamples} samples, "
        f"{atrace_ms / fwd_ms:.2f}x the isotropic trace); trace_save {asave_ms:.3f} ms, "
        f"backward {abwd_ms:.3f} ms ({abwd_ms / bwd_ms:.2f}x the isotropic backward)")
    if args.dtype == "f32" and not args.no_compare:
        # the same anisotropic frame with float16 storage (1.6x the isotropic
        # bytes, three directions read per level above 0)
        gh = vct.Grid(w.n, dtype="f16", anisotropic=True)
        ph = torch.empty(vct.pyramid_bytes(gh), dtype=torch.uint8, device=dev)
        hmips_ms = timed(lambda: vct.build_mips(base, gh, ph), args.steps)
        htrace_ms = timed(lambda: vct.trace(ph, gh, pr, nr, cam, w.params, out), args.steps)
        hsave_ms = timed(lambda: vct.trace_save(ph, gh, pr, nr, cam, w.params, out, state), args.steps)
        hbwd_ms = timed(lambda: vct.trace_backward_saved(ph, gh, pr, nr, cam, w.params, state, gout, aws, gbase),
                        args.steps)
        aniso["f16_storage"] = {
            "pyramid_bytes": int(ph.numel()), "build_mips_ms": hmips_ms, "trace_ms": htrace_ms,
            "fwd_ms_per_frame": hmips_ms + htrace_ms, "trace_save_ms": hsave_ms,
            "trace_backward_saved_ms": hbwd_ms, "fwd_bwd_ms_per_frame": hmips_ms + hsave_ms + hbwd_ms,
            "trace_speedup_vs_f32": atrace_ms / htrace_ms,
            "fwd_speedup_vs_f32": (amips_ms + atrace_ms) / (hmips_ms + htrace_ms),
            "fwd_bwd_speedup_vs_f32": (amips_ms + asave_ms + abwd_ms) / (hmips_ms + hsave_ms + hbwd_ms)}
        del ph
        log(f"anisotropic f16 storage: mips {hmips_ms:.3f} ms, trace {htrace_ms:.3f} ms "
            f"({atrace_ms / htrace_ms:.2f}x the f32 trace); training step {hmips_ms + hsave_ms + hbwd_ms:.3f} ms "
            f"({aniso['f16_storage']['fwd_bwd_speedup_vs_f32']:.2f}x)")
    del aws

    texel_bytes = 16 if args.dtype == "f32" else 8
    trace_bytes = samples * 16 * texel_bytes + npix * 64
    trace_gbs = trace_bytes / (fwd_ms * 1e-3) / 1e9
    tr_traffic, tr_note = measured_traffic("k_trace") if (args.dtype == "f32" and WORKLOAD == "c1") else (
        None, "counters were taken on the float32 1080p workload only")
    fwd_flops = flops(counts, FLOPS_FWD)
    breakdown = {
        "build_mips_ms": mips_ms, "trace_save_ms": save_ms, "trace_backward_saved_ms": bwd_ms,
        "trace_backward_saved_kernels_ms": {n: float(t) for n, t in zip(BWD_KERNELS, bwd_k)},
        "trace_ms": fwd_ms, "fwd_ms_per_frame": mips_ms + fwd_ms,
        "shade_ms": shade_ms,
        "revoxelize": {"triangles": vox_tris, "voxelize_ms": vox_ms, "voxelize_plus_mips_ms": vox_ms + mips_ms,
                       "dense_mesh": {"triangles": big_tris, "voxelize_ms": vox_big_ms,
                                      "triangles_per_s": big_tris / (vox_big_ms * 1e-3)}},
        "bounce": bounce,
        "anisotropic": aniso,
        "fwd_bwd_ms_per_frame": mips_ms + save_ms + bwd_ms,
        "recompute_path": {"trace_backward_ms": recompute_bwd_ms,
                           "fwd_bwd_ms_per_frame": mips_ms + fwd_ms + recompute_bwd_ms},
        "samples_per_frame": samples, "two_level_samples_per_frame": counts[1],
        "samples_per_pixel": samples / npix,
        "fwd_samples_per_s": samples / ((mips_ms + fwd_ms) * 1e-3),
        "trace_kernel_samples_per_s": samples / (fwd_ms * 1e-3),
        "trace_kernel": {
            "alu_TFLOPs": fwd_flops / (fwd_ms * 1e-3) / 1e12,
            "frac_of_alu_peak": fwd_flops / (fwd_ms * 1e-3) / 1e12 / ALU_PEAK_TFLOPS,
            "frac_of_nonpacked_alu_ceiling": fwd_flops / (fwd_ms * 1e-3) / 1e12 / ALU_NONPACKED_TFLOPS,
            # the logical taps (16 texels a sample) are served from L1, L2 and the
            # scalar cache: a cache-traffic figure, not a fraction of HBM bandwidth
            "logical_tap_GBps": trace_gbs, "logical_tap_bytes_over_hbm_peak_cache_served": trace_gbs / HBM_PEAK_GBS,
            "hbm_bytes_per_launch": tr_traffic, "hbm_bytes_note": tr_note,
            "hbm_GBps": None if tr_traffic is None else tr_traffic / (fwd_ms * 1e-3) / 1e9,
            "hbm_frac_of_peak": None if tr_traffic is None else tr_traffic / (fwd_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "l2_hit_rate": measured_l2_hit("k_trace") if tr_traffic is not None else None},
    }

    if not args.no_compare and args.dtype == "f32":
        g16 = vct.Grid(w.n, dtype="f16")
        p16 = vct.build_mips(base, g16)
        o16 = torch.empty_like(out)
        s16 = vct.count_samples(p16, g16, pr, nr, cam, w.params)
        for _ in range(2):
            vct.trace(p16, g16, pr, nr, cam, w.params, o16)
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        e[0].record()
        for _ in range(args.steps):
            vct.build_mips(base, g16, p16)
        e[1].record()
        for _ in range(args.steps):
            vct.trace(p16, g16, pr, nr, cam, w.params, o16)
        e[2].record()
        torch.cuda.synchronize()
        m16 = e[0].elapsed_time(e[1]) / args.steps
        f16 = e[1].elapsed_time(e[2]) / args.steps
        # the training step on the float16 pyramid (same lane-state buffer and gradient)
        ws16 = torch.empty(vct.backward_workspace_bytes(g16, pr, nr, cam, w.params) - st_bytes, dtype=torch.uint8,
                           device=dev)
        save16 = timed(lambda: vct.trace_save(p16, g16, pr, nr, cam, w.params, o16, state), args.steps)
        bwd16 = timed(lambda: vct.trace_backward_saved(p16, g16, pr, nr, cam, w.params, state, gout, ws16, gbase),
                      args.steps)
        step16 = m16 + save16 + bwd16
        breakdown["f16_storage"] = {
            "build_mips_ms": m16, "trace_ms": f16, "samples_per_frame": s16,
            "trace_speedup_vs_f32": fwd_ms / f16, "fwd_speedup_vs_f32": (mips_ms + fwd_ms) / (m16 + f16),
            "trace_logical_GBps": (s16 * 128 + npix * 64) / (f16 * 1e-3) / 1e9,
            "trace_save_ms": save16, "trace_backward_saved_ms": bwd16, "fwd_bwd_ms_per_frame": step16,
            "fwd_bwd_speedup_vs_f32": breakdown["fwd_bwd_ms_per_frame"] / step16}
        log(f"f16 storage: mips {m16:.3f} ms, trace {f16:.3f} ms ({fwd_ms / f16:.2f}x vs f32); training step "
            f"{step16:.3f} ms ({breakdown['fwd_bwd_ms_per_frame'] / step16:.2f}x vs f32)")
        del p16, o16, ws16

    # dominant kernel of the step: the backward scatter pass (VALU work plus
    # integer atomics; its HBM traffic is a fraction of the bandwidth)
    p2_ms = float(bwd_k[3])
    p2_flops = flops(counts, FLOPS_BWD_SCATTER)
    p2_tflops = p2_flops / (p2_ms * 1e-3) / 1e12
    p2_traffic, p2_traffic_note = measured_traffic("k_bwd_pass2") if (args.dtype == "f32" and WORKLOAD == "c1") else (
        None, "counters were taken on the float32 1080p workload only")
    roofline = {"kernel": "k_bwd_pass2 (re-march + deterministic tap-gradient scatter), one launch per step",
                "bound": "alu", "achieved": p2_tflops, "peak": ALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": p2_tflops / ALU_PEAK_TFLOPS, "traffic": p2_traffic, "traffic_note": p2_traffic_note,
                "peak_note": "MI355X published FP32 vector peak (counts packed FP32, which these kernels are "
                             "built without)",
                "peak_nonpacked": ALU_NONPACKED_TFLOPS, "frac_nonpacked": p2_tflops / ALU_NONPACKED_TFLOPS,
                "traffic_frac_of_hbm_peak": None if p2_traffic is None else
                p2_traffic / (p2_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                "traffic_GBps": None if p2_traffic is None else p2_traffic / (p2_ms * 1e-3) / 1e9,
                "l2_hit_rate": measured_l2_hit("k_bwd_pass2") if p2_traffic is not None else None,
                "launch_ms": p2_ms, "flops_per_launch": p2_flops,
                "flops_model": f"{FLOPS_BWD_SCATTER[2]} FP32 ops per two-level sample x {counts[1]} + "
                               f"{FLOPS_BWD_SCATTER[1]} per one-level sample x {samples - counts[1]} "
                               f"(vct_count_sample_levels)"}
    res = {
        "metric": METRIC,
        "value": samples / (ms_step * 1e-3),
        "unit": "cone samples/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.dtype, "data": "synthetic (seeded procedural scene and G-buffer; random dL/dout)",
        "config": {"workload": WORKLOAD_DESC, "grid": w.n, "levels": w.levels, "views": w.shape[0],
                   "height": w.shape[1], "width": w.shape[2], "cones_per_pixel": w.params.n_diffuse + 2,
                   "step": "build_mips + trace_save + trace_backward_saved"},
        "breakdown": breakdown,
        "roofline": roofline,
    }
    mip_bytes = w.n ** 3 * 16 + int(pyr.numel()) - 2 * ((w.n // 16) ** 3) * 16   # base read + levels written
    vox_bytes = w.n ** 3 * 16                     # the light grid, written once
    alu_row = lambda fl, ms: {"bound": "alu", "achieved": fl / (ms * 1e-3) / 1e12, "peak": ALU_PEAK_TFLOPS,  # noqa: E731
                              "unit": "TFLOP/s", "frac": fl / (ms * 1e-3) / 1e12 / ALU_PEAK_TFLOPS,
                              "frac_nonpacked": fl / (ms * 1e-3) / 1e12 / ALU_NONPACKED_TFLOPS}
    rows = {
        "a1_build_mips": {"kernel": "k_mip_block", "ms": mips_ms, "bound": "hbm",
                          "achieved": mip_bytes / (mips_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": mip_bytes / (mips_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                          "model": f"float32 base read once + every level written ({mip_bytes} bytes)"},
        "a2_a6_trace": dict(alu_row(fwd_flops, fwd_ms), kernel="k_trace", ms=fwd_ms,
                            model=f"{FLOPS_FWD[2]} FP32 ops per two-level sample x {counts[1]} + {FLOPS_FWD[1]} per "
                                  f"one-level sample x {samples - counts[1]}",
                            logical_tap_GBps=trace_gbs),
        "a7_backward": dict(roofline, ms=bwd_ms),
        "f1_shade": dict(alu_row(FLOPS_FWD[2] * shade_samples, shade_ms["3_lights"]), kernel="k_shade",
                         ms=shade_ms["3_lights"], pixels_per_s=npix / (shade_ms["3_lights"] * 1e-3),
                         samples=shade_samples, samples_per_s=shade_samples / (shade_ms["3_lights"] * 1e-3),
                         model=f"{FLOPS_FWD[2]} FP32 ops per cone sample (every sample counted as two-level; the "
                               f"per-light terms are left out) x {shade_samples} samples (vct_count_shade_samples, "
                               f"3 lights, the thesis's variants)"),
        "f2_voxelize": {"kernel": "k_clear + k_tri_setup + offset scan + k_clear_slots + k_raster + k_resolve",
                        "ms": vox_ms, "bound": "hbm", "achieved": vox_bytes / (vox_ms * 1e-3) / 1e9,
                        "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": vox_bytes / (vox_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                        "model": f"16 B per voxel: the light grid written once ({vox_bytes} bytes); accumulators "
                                 f"exist only for the voxels the mesh reaches, so the raster pass's atomics, not "
                                 f"HBM, set the rest of the time"},
        "f3_bounce": dict(alu_row(FLOPS_FWD[2] * bounce["samples"], bounce["bounce_kernels_ms"]["gather"]),
                          kernel="k_gather (k_flag: hbm)", ms=bounce["bounce_ms"],
                          model=f"{FLOPS_FWD[2]} FP32 ops per cone sample x {bounce['samples']} samples",
                          flag_frac_of_hbm_peak=bounce["flag_frac_of_hbm_peak"]),
        "f4_anisotropic": dict(alu_row(FLOPS_FWD[2] * aniso["samples_per_frame"], aniso["trace_ms"]),
                               kernel="k_trace<ANISO>", ms=aniso["trace_ms"],
                               model=f"{FLOPS_FWD[2]} FP32 ops per cone sample (the isotropic count: a lower bound, "
                                     f"samples above level 0 read up to three directions)",
                               backward_ms=aniso["trace_backward_saved_ms"],
                               fwd_bwd_ms_per_frame=aniso["fwd_bwd_ms_per_frame"]),
    }
    res["rows"] = rows
    if not args.no_configs:
        del ws, state, ws_saved
        torch.cuda.empty_cache()
        res["configs"] = bench_configs(vct, torch, make_workload)
    # whether float16 storage gives the faster forward, frame by frame
    f16_faster = {}
    if "f16_storage" in breakdown:
        f16_faster["isotropic_256cubed_1080p"] = breakdown["f16_storage"]["fwd_speedup_vs_f32"] > 1.0
    if "f16_storage" in aniso:
        f16_faster["anisotropic_256cubed_1080p"] = aniso["f16_storage"]["fwd_speedup_vs_f32"] > 1.0
    if "configs" in res:
        f16_faster["isotropic_512cubed_4x4k"] = res["configs"]["c4_512cubed_4x4k_f16"]["fwd_speedup_vs_f32"] > 1.0
    if f16_faster:
        res["fp16_forward_faster_than_fp32"] = dict(
            f16_faster, met_everywhere=all(f16_faster.values()),
            note="speedups of the float16-storage forward over float32 are in breakdown.f16_storage, "
                 "breakdown.anisotropic.f16_storage and configs.c4_512cubed_4x4k_f16")
    if cpu_base is not None:
        res["cpu_baseline"] = cpu_base
        nw = cpu_parts["workers"]
        rows["a1_build_mips"]["cpu_baseline"] = {"value": w.n ** 3 / cpu_parts["mips_s"], "unit": "base texels/s",
                                                 "cores": 1, "kind": "oracle", "sample": f"the whole {w.n}^3 grid"}
        rows["a2_a6_trace"]["cpu_baseline"] = {
            "value": cpu_parts["forward_samples_per_s"], "unit": "cone samples/s", "cores": nw, "kind": "oracle",
            "sample": f"all 7 cones of {cpu_parts['pixels']} seeded pixels in {nw} processes (per-core rate x cores)"}
        rows["a7_backward"]["cpu_baseline"] = {
            "value": cpu_parts["backward_samples_per_s"], "unit": "cone samples/s", "cores": nw, "kind": "oracle",
            "sample": f"adjoint of all 7 cones of {cpu_parts['pixels']} seeded pixels in {nw} processes, each with "
                      f"its own mip adjoint (per-core rate x cores)"}
        log("timing the oracle on bounded samples of the other rows (one thread)")
        # one host thread for every library NumPy may call, so "cores": 1 is what ran
        from threadpoolctl import threadpool_limits
        with threadpool_limits(limits=1):
            other_rows = cpu_rows(w, vox_mesh, vlights)
        for k, v in other_rows.items():
            rows[k]["cpu_baseline"] = v
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
