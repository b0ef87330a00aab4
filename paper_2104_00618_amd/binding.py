"""Thin ctypes binding of libvct (argument marshalling only).

Every computation runs in the HIP library; torch supplies device memory and
the current stream.  If libvct.so is missing the import of any entry point
raises: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import math
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvct.so")

VCT_F32, VCT_F16, VCT_BF16 = 0, 1, 2
DTYPES = {"f32": VCT_F32, "f16": VCT_F16, "bf16": VCT_BF16}
MAX_DIFFUSE = 16


class VctError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class CGrid(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("levels", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("origin", ctypes.c_float * 3), ("extent", ctypes.c_float), ("anisotropic", ctypes.c_int32)]


class CGBuffer(ctypes.Structure):
    _fields_ = [("b", ctypes.c_int32), ("h", ctypes.c_int32), ("w", ctypes.c_int32),
                ("pos_rough", ctypes.c_void_p), ("normal", ctypes.c_void_p), ("cam_pos", ctypes.c_void_p)]


class CConeParams(ctypes.Structure):
    _fields_ = [("n_diffuse", ctypes.c_int32),
                ("diffuse_dir", (ctypes.c_float * 3) * MAX_DIFFUSE),
                ("diffuse_weight", ctypes.c_float * MAX_DIFFUSE),
                ("diffuse_aperture", ctypes.c_float),
                ("enable_spec", ctypes.c_int32), ("enable_occ", ctypes.c_int32),
                ("spec_aperture_scale", ctypes.c_float), ("occ_aperture", ctypes.c_float),
                ("light_pos", ctypes.c_float * 3),
                ("step_factor", ctypes.c_float), ("t0", ctypes.c_float), ("normal_offset", ctypes.c_float),
                ("max_dist", ctypes.c_float), ("alpha_thresh", ctypes.c_float)]


_lib = None


def lib():
    """Load libvct.so (built in-tree by paper_2104_00618_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_2104_00618_amd.build.build() (no fallback exists)")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    vp, sz = ctypes.c_void_p, ctypes.c_size_t
    sig = {
        "vct_pyramid_bytes": [P(CGrid), P(sz)],
        "vct_build_mips": [P(CGrid), vp, vp, sz, vp],
        "vct_unpack_level": [P(CGrid), vp, ctypes.c_int32, vp, vp],
        "vct_unpack_level_dir": [P(CGrid), vp, ctypes.c_int32, ctypes.c_int32, vp, vp],
        "vct_trace": [P(CGrid), vp, P(CGBuffer), P(CConeParams), vp, vp],
        "vct_count_samples": [P(CGrid), vp, P(CGBuffer), P(CConeParams), vp, vp],
        "vct_count_sample_levels": [P(CGrid), vp, P(CGBuffer), P(CConeParams), vp, vp],
        "vct_shade": [P(CGrid), vp, P(CGBuffer), vp, P(CConeParams), P(CShadeParams), vp, vp],
        "vct_count_shade_samples": [P(CGrid), vp, P(CGBuffer), vp, P(CConeParams), P(CShadeParams), vp, vp],
        "vct_voxelize_workspace_bytes": [P(CGrid), ctypes.c_int64, ctypes.c_int32, P(sz)],
        "vct_voxelize": [P(CGrid), vp, vp, ctypes.c_int64, P(CVoxelizeParams), vp, vp, vp, vp, sz, vp],
        "vct_bounce_workspace_bytes": [P(CGrid), P(sz)],
        "vct_bounce": [P(CGrid), vp, vp, vp, vp, P(CConeParams), vp, vp, sz, vp],
        "vct_backward_workspace_bytes": [P(CGrid), P(CGBuffer), P(CConeParams), P(sz)],
        "vct_trace_backward": [P(CGrid), vp, P(CGBuffer), P(CConeParams), vp, vp, vp, sz, vp],
        "vct_lane_state_bytes": [P(CGBuffer), P(CConeParams), P(sz)],
        "vct_trace_save": [P(CGrid), vp, P(CGBuffer), P(CConeParams), vp, vp, sz, vp],
        "vct_trace_backward_saved": [P(CGrid), vp, P(CGBuffer), P(CConeParams), vp, sz, vp, vp, vp, sz, vp],
        "vct_trace_backward_saved_noalloc": [P(CGrid), vp, P(CGBuffer), P(CConeParams), vp, sz, vp, vp, vp],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    L.vct_record_kernel_events.argtypes = [ctypes.c_void_p, ctypes.c_int32]
    L.vct_record_kernel_events.restype = ctypes.c_int
    L.vct_last_error.argtypes = []
    L.vct_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


_hip = None


def _hiprt():
    global _hip
    if _hip is None:
        h = ctypes.CDLL("libamdhip64.so")
        h.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        h.hipEventDestroy.argtypes = [ctypes.c_void_p]
        h.hipEventSynchronize.argtypes = [ctypes.c_void_p]
        h.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p, ctypes.c_void_p]
        _hip = h
    return _hip


class KernelEvents:
    """Per-kernel timing of the next library call on this thread
    (vct_record_kernel_events): arm() before the call, times() afterwards
    gives the duration of each of its first n - 1 kernels in ms."""

    def __init__(self, n):
        h = _hiprt()
        self.n = n
        self.ev = (ctypes.c_void_p * n)()
        for i in range(n):
            e = ctypes.c_void_p()
            if h.hipEventCreate(ctypes.byref(e)) != 0:
                raise RuntimeError("hipEventCreate failed")
            self.ev[i] = e.value

    def arm(self):
        _check(lib().vct_record_kernel_events(ctypes.cast(self.ev, ctypes.c_void_p), self.n))

    def times(self):
        h = _hiprt()
        h.hipEventSynchronize(self.ev[self.n - 1])
        out = []
        for i in range(self.n - 1):
            ms = ctypes.c_float()
            if h.hipEventElapsedTime(ctypes.byref(ms), self.ev[i], self.ev[i + 1]) != 0:
                raise RuntimeError("hipEventElapsedTime failed")
            out.append(ms.value)
        return out

    def __del__(self):
        try:
            for i in range(self.n):
                _hiprt().hipEventDestroy(self.ev[i])
        except Exception:
            pass


def _check(rc):
    if rc != 0:
        raise VctError(rc, lib().vct_last_error().decode())


# ---------------------------------------------------------------------------
# argument structs
# ---------------------------------------------------------------------------

class Grid:
    """Grid descriptor: N^3 base texels over [origin, origin + extent]^3."""

    def __init__(self, n, levels=None, dtype="f32", origin=(0.0, 0.0, 0.0), extent=1.0, anisotropic=False):
        self.n = int(n)
        self.levels = int(levels) if levels is not None else int(round(math.log2(max(self.n, 1)))) + 1
        self.dtype = dtype
        self.origin = tuple(float(v) for v in origin)
        self.extent = float(extent)
        self.anisotropic = bool(anisotropic)

    def c(self):
        g = CGrid()
        g.n = self.n
        g.levels = self.levels
        g.dtype = DTYPES[self.dtype] if isinstance(self.dtype, str) else int(self.dtype)
        for i in range(3):
            g.origin[i] = self.origin[i]
        g.extent = self.extent
        g.anisotropic = 1 if self.anisotropic else 0
        return g


MAX_LIGHTS = 8


class CShadeParams(ctypes.Structure):
    _fields_ = [("n_lights", ctypes.c_int32),
                ("light_pos", (ctypes.c_float * 3) * MAX_LIGHTS),
                ("light_diffuse", (ctypes.c_float * 3) * MAX_LIGHTS),
                ("light_specular", (ctypes.c_float * 3) * MAX_LIGHTS),
                ("specular_color", ctypes.c_float * 3),
                ("diffuse_first_hit", ctypes.c_int32), ("first_hit_alpha", ctypes.c_float),
                ("occlusion_falloff", ctypes.c_int32), ("shadow_strength", ctypes.c_float),
                ("specular_brdf", ctypes.c_int32), ("grace_per_shininess", ctypes.c_float),
                ("shininess_falloff", ctypes.c_float)]


def shade_params(p):
    """C struct from any object with the fields of scenes.configs.ShadeParams."""
    c = CShadeParams()
    pos = [tuple(map(float, v)) for v in p.light_pos]
    if len(pos) > MAX_LIGHTS or len(p.light_diffuse) != len(pos) or len(p.light_specular) != len(pos):
        raise ValueError("light_pos / light_diffuse / light_specular: at most 8 lights, one row per light")
    c.n_lights = len(pos)
    for l in range(len(pos)):
        for i in range(3):
            c.light_pos[l][i] = pos[l][i]
            c.light_diffuse[l][i] = float(p.light_diffuse[l][i])
            c.light_specular[l][i] = float(p.light_specular[l][i])
    for i in range(3):
        c.specular_color[i] = float(p.specular_color[i])
    c.diffuse_first_hit = int(bool(p.diffuse_first_hit))
    c.first_hit_alpha = float(p.first_hit_alpha)
    c.occlusion_falloff = int(bool(p.occlusion_falloff))
    c.shadow_strength = float(p.shadow_strength)
    c.specular_brdf = int(bool(p.specular_brdf))
    c.grace_per_shininess = float(p.grace_per_shininess)
    c.shininess_falloff = float(p.shininess_falloff)
    return c


class CVoxelizeParams(ctypes.Structure):
    _fields_ = [("n_lights", ctypes.c_int32),
                ("light_pos", (ctypes.c_float * 3) * MAX_LIGHTS),
                ("light_color", (ctypes.c_float * 3) * MAX_LIGHTS),
                ("attenuation", (ctypes.c_float * 3) * MAX_LIGHTS),
                ("ambient", ctypes.c_float), ("diffuse", ctypes.c_float)]


def voxelize_params(lights, ambient=0.1, diffuse=1.0):
    """C struct from a sequence of (position[3], colour[3], attenuation (c, l, q))."""
    c = CVoxelizeParams()
    if len(lights) > MAX_LIGHTS:
        raise ValueError("at most 8 lights")
    c.n_lights = len(lights)
    for l, (pos, col, att) in enumerate(lights):
        for i in range(3):
            c.light_pos[l][i] = float(pos[i])
            c.light_color[l][i] = float(col[i])
            c.attenuation[l][i] = float(att[i])
    c.ambient = float(ambient)
    c.diffuse = float(diffuse)
    return c


def cone_params(p):
    """C struct from any object with the cone-set attributes (n_diffuse taken
    from len(diffuse_dirs))."""
    c = CConeParams()
    dirs = [tuple(map(float, d)) for d in p.diffuse_dirs]
    wts = [float(w) for w in p.diffuse_weights]
    if len(dirs) > MAX_DIFFUSE or len(wts) != len(dirs):
        raise ValueError("diffuse_dirs / diffuse_weights: at most 16 cones, one weight per direction")
    c.n_diffuse = len(dirs)
    for q, d in enumerate(dirs):
        for i in range(3):
            c.diffuse_dir[q][i] = d[i]
        c.diffuse_weight[q] = wts[q]
    c.diffuse_aperture = float(p.diffuse_aperture)
    c.enable_spec = int(bool(p.enable_spec))
    c.enable_occ = int(bool(p.enable_occ))
    c.spec_aperture_scale = float(p.spec_aperture_scale)
    c.occ_aperture = float(p.occ_aperture)
    for i in range(3):
        c.light_pos[i] = float(p.light_pos[i])
    c.step_factor = float(p.step_factor)
    c.t0 = float(p.t0)
    c.normal_offset = float(p.normal_offset)
    c.max_dist = float(p.max_dist)
    c.alpha_thresh = float(p.alpha_thresh)
    return c


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream(dev):
    return ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


def _need(t, name, dtype, shape=None, device=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if device is not None and t.device != device:
        raise ValueError(f"{name} is on {t.device}, expected {device}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


def _gbuf(pos_rough, normal, cam_pos):
    dev = pos_rough.device
    b, h, w = pos_rough.shape[:3]
    _need(pos_rough, "pos_rough", torch.float32, (b, h, w, 4))
    _need(normal, "normal", torch.float32, (b, h, w, 4), dev)
    _need(cam_pos, "cam_pos", torch.float32, (b, 3), dev)
    g = CGBuffer()
    g.b, g.h, g.w = b, h, w
    g.pos_rough = pos_rough.data_ptr()
    g.normal = normal.data_ptr()
    g.cam_pos = cam_pos.data_ptr()
    return g


# ---------------------------------------------------------------------------
# entry points
# ---------------------------------------------------------------------------

def pyramid_bytes(grid):
    n = ctypes.c_size_t()
    _check(lib().vct_pyramid_bytes(ctypes.byref(grid.c()), ctypes.byref(n)))
    return n.value


def build_mips(base, grid, pyramid=None):
    """Pack `base` (float32 [N,N,N,4] premultiplied RGBA, on the GPU) and build
    its mip pyramid.  Returns the opaque pyramid buffer (uint8 tensor)."""
    _need(base, "base", torch.float32, (grid.n, grid.n, grid.n, 4))
    nb = pyramid_bytes(grid)
    if pyramid is None:
        pyramid = torch.empty(nb, dtype=torch.uint8, device=base.device)
    _need(pyramid, "pyramid", torch.uint8, None, base.device)
    with torch.cuda.device(base.device):
        _check(lib().vct_build_mips(ctypes.byref(grid.c()), _ptr(base), _ptr(pyramid), pyramid.numel(),
                                    _stream(base.device)))
    return pyramid


def unpack_level(pyramid, grid, level):
    nl = grid.n >> level
    out = torch.empty((nl, nl, nl, 4), dtype=torch.float32, device=pyramid.device)
    with torch.cuda.device(pyramid.device):
        _check(lib().vct_unpack_level(ctypes.byref(grid.c()), _ptr(pyramid), int(level), _ptr(out),
                                      _stream(pyramid.device)))
    return out


def unpack_level_dir(pyramid, grid, level, direction):
    """Level `level` of direction `direction` (0..5 = +x, -x, +y, -y, +z, -z)
    of an anisotropic pyramid as float32 [N_l, N_l, N_l, 4]."""
    nl = grid.n >> level
    out = torch.empty((nl, nl, nl, 4), dtype=torch.float32, device=pyramid.device)
    with torch.cuda.device(pyramid.device):
        _check(lib().vct_unpack_level_dir(ctypes.byref(grid.c()), _ptr(pyramid), int(level), int(direction),
                                          _ptr(out), _stream(pyramid.device)))
    return out


def trace(pyramid, grid, pos_rough, normal, cam_pos, params, out=None):
    """Forward cone trace.  Returns float32 [b,h,w,8] = (D.rgb, D.a, S.rgb, O)."""
    gb = _gbuf(pos_rough, normal, cam_pos)
    _need(pyramid, "pyramid", torch.uint8, None, pos_rough.device)
    if out is None:
        out = torch.empty(tuple(pos_rough.shape[:3]) + (8,), dtype=torch.float32, device=pos_rough.device)
    _need(out, "out", torch.float32, tuple(pos_rough.shape[:3]) + (8,), pos_rough.device)
    with torch.cuda.device(pos_rough.device):
        _check(lib().vct_trace(ctypes.byref(grid.c()), _ptr(pyramid), ctypes.byref(gb),
                               ctypes.byref(cone_params(params)), _ptr(out), _stream(pos_rough.device)))
    return out


def shade(pyramid, grid, pos_rough, normal, cam_pos, material, params, sparams, out=None):
    """Final shading with the thesis's cone variants.  Returns float32
    [b,h,w,4] = (L.rgb, o_min)."""
    gb = _gbuf(pos_rough, normal, cam_pos)
    dev = pos_rough.device
    _need(pyramid, "pyramid", torch.uint8, None, dev)
    _need(material, "material", torch.float32, tuple(pos_rough.shape), dev)
    if out is None:
        out = torch.empty(tuple(pos_rough.shape[:3]) + (4,), dtype=torch.float32, device=dev)
    _need(out, "out", torch.float32, tuple(pos_rough.shape[:3]) + (4,), dev)
    with torch.cuda.device(dev):
        _check(lib().vct_shade(ctypes.byref(grid.c()), _ptr(pyramid), ctypes.byref(gb), _ptr(material),
                               ctypes.byref(cone_params(params)), ctypes.byref(shade_params(sparams)), _ptr(out),
                               _stream(dev)))
    return out



def count_shade_samples(pyramid, grid, pos_rough, normal, cam_pos, material, params, sparams):
    """Total cone samples the marches of shade() take (integer, exact)."""
    gb = _gbuf(pos_rough, normal, cam_pos)
    dev = pos_rough.device
    _need(pyramid, "pyramid", torch.uint8, None, dev)
    _need(material, "material", torch.float32, tuple(pos_rough.shape), dev)
    cnt = torch.zeros(1, dtype=torch.int64, device=dev)
    with torch.cuda.device(dev):
        _check(lib().vct_count_shade_samples(ctypes.byref(grid.c()), _ptr(pyramid), ctypes.byref(gb), _ptr(material),
                                             ctypes.byref(cone_params(params)), ctypes.byref(shade_params(sparams)),
                                             _ptr(cnt), _stream(dev)))
    return int(cnt.item())

def voxelize_workspace_bytes(grid, n_tris, surface=False):
    n = ctypes.c_size_t()
    _check(lib().vct_voxelize_workspace_bytes(ctypes.byref(grid.c()), int(n_tris), int(bool(surface)),
                                              ctypes.byref(n)))
    return n.value


def voxelize(tris, colors, grid, lights, ambient=0.1, diffuse=1.0, base=None, workspace=None, surface=False,
             normal=None, albedo=None):
    """Voxelize a triangle mesh (float32 [T, 3, 3] world positions, float32
    [T, 3] colours) with direct-light injection into a float32 base grid
    [N, N, N, 4] (premultiplied RGBA).  With surface=True also the average
    normal and colour grids; returns (base, normal, albedo) then."""
    dev = tris.device
    shape = (grid.n, grid.n, grid.n, 4)
    _need(tris, "tris", torch.float32, (tris.shape[0], 3, 3), dev)
    _need(colors, "colors", torch.float32, (tris.shape[0], 3), dev)
    if base is None:
        base = torch.empty(shape, dtype=torch.float32, device=dev)
    _need(base, "base", torch.float32, shape, dev)
    if surface:
        normal = torch.empty(shape, dtype=torch.float32, device=dev) if normal is None else normal
        albedo = torch.empty(shape, dtype=torch.float32, device=dev) if albedo is None else albedo
        _need(normal, "normal", torch.float32, shape, dev)
        _need(albedo, "albedo", torch.float32, shape, dev)
    else:
        normal = albedo = None
    if workspace is None:
        workspace = torch.empty(voxelize_workspace_bytes(grid, tris.shape[0], surface), dtype=torch.uint8,
                                device=dev)
    _need(workspace, "workspace", torch.uint8, None, dev)
    with torch.cuda.device(dev):
        _check(lib().vct_voxelize(ctypes.byref(grid.c()), _ptr(tris), _ptr(colors), int(tris.shape[0]),
                                  ctypes.byref(voxelize_params(lights, ambient, diffuse)), _ptr(base),
                                  _ptr(normal), _ptr(albedo), _ptr(workspace), workspace.numel(), _stream(dev)))
    return (base, normal, albedo) if surface else base


def bounce_workspace_bytes(grid):
    n = ctypes.c_size_t()
    _check(lib().vct_bounce_workspace_bytes(ctypes.byref(grid.c()), ctypes.byref(n)))
    return n.value


def bounce(pyramid, grid, base, normal, albedo, params, out=None, workspace=None):
    """One further bounce: from every surface voxel of `base` the diffuse
    cones of `params` march through `pyramid`; returns float32 [N, N, N, 4]
    = base + base.a * albedo * gathered light (other voxels: base).  `out`
    may be `base` (in place)."""
    dev = base.device
    shape = (grid.n, grid.n, grid.n, 4)
    _need(pyramid, "pyramid", torch.uint8, None, dev)
    for t, nm in ((base, "base"), (normal, "normal"), (albedo, "albedo")):
        _need(t, nm, torch.float32, shape, dev)
    if out is None:
        out = torch.empty(shape, dtype=torch.float32, device=dev)
    _need(out, "out", torch.float32, shape, dev)
    if workspace is None:
        workspace = torch.empty(bounce_workspace_bytes(grid), dtype=torch.uint8, device=dev)
    _need(workspace, "workspace", torch.uint8, None, dev)
    with torch.cuda.device(dev):
        _check(lib().vct_bounce(ctypes.byref(grid.c()), _ptr(pyramid), _ptr(base), _ptr(normal), _ptr(albedo),
                                ctypes.byref(cone_params(params)), _ptr(out), _ptr(workspace), workspace.numel(),
                                _stream(dev)))
    return out


def count_samples(pyramid, grid, pos_rough, normal, cam_pos, params):
    """Total cone samples the forward march takes (integer, exact)."""
    gb = _gbuf(pos_rough, normal, cam_pos)
    cnt = torch.zeros(1, dtype=torch.int64, device=pos_rough.device)
    with torch.cuda.device(pos_rough.device):
        _check(lib().vct_count_samples(ctypes.byref(grid.c()), _ptr(pyramid), ctypes.byref(gb),
                                       ctypes.byref(cone_params(params)), _ptr(cnt), _stream(pos_rough.device)))
    return int(cnt.item())


def count_sample_levels(pyramid, grid, pos_rough, normal, cam_pos, params):
    """(all cone samples, samples that read two levels) of the forward march."""
    gb = _gbuf(pos_rough, normal, cam_pos)
    cnt = torch.zeros(2, dtype=torch.int64, device=pos_rough.device)
    with torch.cuda.device(pos_rough.device):
        _check(lib().vct_count_sample_levels(ctypes.byref(grid.c()), _ptr(pyramid), ctypes.byref(gb),
                                             ctypes.byref(cone_params(params)), _ptr(cnt),
                                             _stream(pos_rough.device)))
    c = cnt.cpu().tolist()
    return int(c[0]), int(c[1])


def backward_workspace_bytes(grid, pos_rough, normal, cam_pos, params):
    gb = _gbuf(pos_rough, normal, cam_pos)
    n = ctypes.c_size_t()
    _check(lib().vct_backward_workspace_bytes(ctypes.byref(grid.c()), ctypes.byref(gb),
                                              ctypes.byref(cone_params(params)), ctypes.byref(n)))
    return n.value


def trace_backward(pyramid, grid, pos_rough, normal, cam_pos, params, grad_out, workspace=None, grad_base=None):
    """dL/d(base) float32 [N,N,N,4] for dL/d(out) = grad_out."""
    gb = _gbuf(pos_rough, normal, cam_pos)
    dev = pos_rough.device
    _need(grad_out, "grad_out", torch.float32, tuple(pos_rough.shape[:3]) + (8,), dev)
    nbytes = backward_workspace_bytes(grid, pos_rough, normal, cam_pos, params)
    if workspace is None:
        workspace = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    _need(workspace, "workspace", torch.uint8, None, dev)
    if grad_base is None:
        grad_base = torch.empty((grid.n, grid.n, grid.n, 4), dtype=torch.float32, device=dev)
    _need(grad_base, "grad_base", torch.float32, (grid.n, grid.n, grid.n, 4), dev)
    with torch.cuda.device(dev):
        _check(lib().vct_trace_backward(ctypes.byref(grid.c()), _ptr(pyramid), ctypes.byref(gb),
                                        ctypes.byref(cone_params(params)), _ptr(grad_out), _ptr(grad_base),
                                        _ptr(workspace), workspace.numel(), _stream(dev)))
    return grad_base


def lane_state_bytes(pos_rough, normal, cam_pos, params):
    gb = _gbuf(pos_rough, normal, cam_pos)
    n = ctypes.c_size_t()
    _check(lib().vct_lane_state_bytes(ctypes.byref(gb), ctypes.byref(cone_params(params)), ctypes.byref(n)))
    return n.value


def trace_save(pyramid, grid, pos_rough, normal, cam_pos, params, out=None, lane_state=None):
    """Forward that also returns the cones' end states for trace_backward_saved."""
    gb = _gbuf(pos_rough, normal, cam_pos)
    dev = pos_rough.device
    if out is None:
        out = torch.empty(tuple(pos_rough.shape[:3]) + (8,), dtype=torch.float32, device=dev)
    _need(out, "out", torch.float32, tuple(pos_rough.shape[:3]) + (8,), dev)
    if lane_state is None:
        lane_state = torch.empty(lane_state_bytes(pos_rough, normal, cam_pos, params), dtype=torch.uint8, device=dev)
    _need(lane_state, "lane_state", torch.uint8, None, dev)
    with torch.cuda.device(dev):
        _check(lib().vct_trace_save(ctypes.byref(grid.c()), _ptr(pyramid), ctypes.byref(gb),
                                    ctypes.byref(cone_params(params)), _ptr(out), _ptr(lane_state),
                                    lane_state.numel(), _stream(dev)))
    return out, lane_state


def trace_backward_saved(pyramid, grid, pos_rough, normal, cam_pos, params, lane_state, grad_out, workspace=None,
                         grad_base=None):
    """trace_backward given the lane states of trace_save (bitwise equal result)."""
    gb = _gbuf(pos_rough, normal, cam_pos)
    dev = pos_rough.device
    _need(grad_out, "grad_out", torch.float32, tuple(pos_rough.shape[:3]) + (8,), dev)
    _need(lane_state, "lane_state", torch.uint8, None, dev)
    nbytes = backward_workspace_bytes(grid, pos_rough, normal, cam_pos, params) - lane_state_bytes(
        pos_rough, normal, cam_pos, params)
    if workspace is None:
        workspace = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    _need(workspace, "workspace", torch.uint8, None, dev)
    if grad_base is None:
        grad_base = torch.empty((grid.n, grid.n, grid.n, 4), dtype=torch.float32, device=dev)
    _need(grad_base, "grad_base", torch.float32, (grid.n, grid.n, grid.n, 4), dev)
    with torch.cuda.device(dev):
        _check(lib().vct_trace_backward_saved(ctypes.byref(grid.c()), _ptr(pyramid), ctypes.byref(gb),
                                              ctypes.byref(cone_params(params)), _ptr(lane_state), lane_state.numel(),
                                              _ptr(grad_out), _ptr(grad_base), _ptr(workspace), workspace.numel(),
                                              _stream(dev)))
    return grad_base


NOALLOC_SCRATCH_BYTES = 128 << 20


def trace_backward_saved_noalloc(pyramid, grid, pos_rough, normal, cam_pos, params, lane_state, grad_out,
                                 grad_base):
    """trace_backward_saved through the entry point that allocates nothing (its
    scratch is the library's per-GPU array; grad_base is the caller's output)."""
    gb = _gbuf(pos_rough, normal, cam_pos)
    dev = pos_rough.device
    _need(grad_out, "grad_out", torch.float32, tuple(pos_rough.shape[:3]) + (8,), dev)
    _need(lane_state, "lane_state", torch.uint8, None, dev)
    _need(grad_base, "grad_base", torch.float32, (grid.n, grid.n, grid.n, 4), dev)
    with torch.cuda.device(dev):
        _check(lib().vct_trace_backward_saved_noalloc(ctypes.byref(grid.c()), _ptr(pyramid), ctypes.byref(gb),
                                                      ctypes.byref(cone_params(params)), _ptr(lane_state),
                                                      lane_state.numel(), _ptr(grad_out), _ptr(grad_base),
                                                      _stream(dev)))
    return grad_base


class VCTTrace(torch.autograd.Function):
    """out = trace(build_mips(base)); backward gives dL/d(base) through the
    hand-written adjoint (deterministic).  The forward keeps every cone's end
    state (trace_save) so the backward skips one re-march."""

    @staticmethod
    def forward(ctx, base, pos_rough, normal, cam_pos, grid, params):
        pyr = build_mips(base.contiguous(), grid)
        out, state = trace_save(pyr, grid, pos_rough, normal, cam_pos, params)
        ctx.save_for_backward(pos_rough, normal, cam_pos)
        ctx.pyr = pyr
        ctx.state = state
        ctx.grid = grid
        ctx.params = params
        return out

    @staticmethod
    def backward(ctx, grad_out):
        pos_rough, normal, cam_pos = ctx.saved_tensors
        g = trace_backward_saved(ctx.pyr, ctx.grid, pos_rough, normal, cam_pos, ctx.params, ctx.state,
                                 grad_out.contiguous())
        return g, None, None, None, None, None


def render(base, grid, pos_rough, normal, cam_pos, params):
    """Differentiable forward: build_mips + trace."""
    return VCTTrace.apply(base, pos_rough, normal, cam_pos, grid, params)
