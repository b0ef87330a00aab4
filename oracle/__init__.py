"""FP64 CPU oracle for the voxel cone tracing hot path.

Test infrastructure only: imported by tests/, the smoke check and the
cpu_baseline leg of bench.py, never by the library or its binding."""
from .vct_oracle import (build_mips, mip_adjoint, taps, sample, cone_lanes, march,  # noqa: F401
                         assemble, trace, trace_backward, lane_grads, render)
from .vct_shade import f_spec, shade, smoothstep  # noqa: F401
from .vct_bounce import MIN_NORMAL, bounce, bounces, surface_mask  # noqa: F401
from .vct_aniso import (aniso_mip_adjoint, aniso_sampler, build_aniso_mips, sample_aniso, trace_aniso,  # noqa: F401
                        trace_backward_aniso)
