"""Error metrics for GPU-vs-oracle parity (shared by the GPU tests and bench)."""
import numpy as np

CHANNELS = ("D.r", "D.g", "D.b", "D.a", "S.r", "S.g", "S.b", "O")


def range_errors(gpu, ref, keep=None):
    """Per output channel: max |gpu - ref| / max |ref| and RMS / max |ref|,
    over pixels where ``keep`` is true (non-ambiguous, by default all)."""
    gpu = np.asarray(gpu, dtype=np.float64).reshape(-1, gpu.shape[-1])
    ref = np.asarray(ref, dtype=np.float64).reshape(-1, ref.shape[-1])
    if keep is None:
        keep = np.ones(len(ref), dtype=bool)
    keep = np.asarray(keep).reshape(-1)
    out = {}
    for c in range(ref.shape[1]):
        scale = np.abs(ref[:, c]).max()
        d = np.abs(gpu[keep, c] - ref[keep, c])
        if scale == 0:
            out[c] = (float(d.max(initial=0.0)), float(np.sqrt(np.mean(d ** 2))) if d.size else 0.0)
        else:
            out[c] = (float(d.max(initial=0.0) / scale), float(np.sqrt(np.mean(d ** 2)) / scale) if d.size else 0.0)
    return out


def worst(errs):
    return max(v[0] for v in errs.values()), max(v[1] for v in errs.values())


def fmt(errs):
    names = CHANNELS if len(errs) == 8 else [str(i) for i in range(len(errs))]
    return ", ".join(f"{names[c]} max {m:.2e} rms {r:.2e}" for c, (m, r) in errs.items())
