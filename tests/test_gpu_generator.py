"""The seeded input generator run on the GPU (as the large workloads are, in
the tests and the bench) gives the same bits as on the CPU: its torch
operations are elementwise IEEE float64 operations, which round the same on
every device."""
import numpy as np
import pytest

from scenes import make_workload

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name,kw", [("c1", {}), ("c3gt", {"views": 2})])
def test_generator_on_gpu_gives_the_cpu_bits(name, kw):
    cpu = make_workload(name, **kw)
    gpu = make_workload(name, device="cuda:0", **kw)
    for field in ("base", "pos_rough", "normal", "cam_pos"):
        a, b = getattr(cpu, field), getattr(gpu, field)
        assert a.shape == b.shape and a.dtype == b.dtype, field
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), f"{name} {field}"
