"""Cached seeded workloads and oracle helpers for the GPU tests."""
import functools

import numpy as np

from scenes import make_workload


@functools.lru_cache(maxsize=None)
def workload(name, **kw):
    return make_workload(name, **kw)


def sample_pixels(shape, m, seed):
    """m distinct seeded pixel indices (view, y, x) of a [b, h, w] G-buffer."""
    b, h, w = shape
    rng = np.random.default_rng(seed)
    flat = rng.choice(b * h * w, size=min(m, b * h * w), replace=False)
    v = flat // (h * w)
    y = (flat // w) % h
    x = flat % w
    return v, y, x


def sub_gbuffer(pos_rough, normal, cam_pos, v, y, x):
    """A G-buffer holding only the chosen pixels, one view per source view so
    that every pixel keeps its camera: returned as per-view lists."""
    out = []
    for vv in np.unique(v):
        sel = v == vv
        pr = pos_rough[vv, y[sel], x[sel]][None, None]
        nr = normal[vv, y[sel], x[sel]][None, None]
        out.append((sel, pr, nr, cam_pos[vv:vv + 1]))
    return out


def oracle_at(mips, w, v, y, x, params=None):
    """Oracle output [m, 8] and ambiguity [m] at the chosen pixels."""
    import oracle
    params = params or w.params
    m = len(v)
    out = np.zeros((m, 8))
    amb = np.zeros(m, dtype=bool)
    for sel, pr, nr, cam in sub_gbuffer(w.pos_rough, w.normal, w.cam_pos, v, y, x):
        o, info = oracle.trace(mips, pr, nr, cam, params, return_info=True)
        out[sel] = o.reshape(-1, 8)
        amb[sel] = info["ambiguous"].reshape(-1)
    return out, amb
