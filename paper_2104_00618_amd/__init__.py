"""MI355X-native voxel cone tracing hot path (arXiv 2104.00618).

The computation lives in libvct.so (hand-written HIP for gfx950 behind the C
ABI of include/vct.h); this package only marshals torch tensors into it."""
from .binding import (Grid, KernelEvents, VctError, VCTTrace, backward_workspace_bytes, build_mips, count_samples,  # noqa: F401
                      count_sample_levels,
                      count_shade_samples,
                      cone_params, lane_state_bytes, lib, pyramid_bytes, render, shade, shade_params, trace, trace_backward,
                      trace_backward_saved, trace_backward_saved_noalloc, trace_save, unpack_level,
                      unpack_level_dir, voxelize,
                      voxelize_params, voxelize_workspace_bytes, bounce, bounce_workspace_bytes)
