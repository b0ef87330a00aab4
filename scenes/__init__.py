"""Seeded synthetic inputs (procedural Cornell-box grids, analytic G-buffers,
cone-set tables).  Shared by the oracle tests and the HIP path; holds no cone
tracing arithmetic."""
from . import cornell, configs  # noqa: F401
from .configs import (ConeParams, ShadeParams, Workload, make_workload, cone_set, random_grid,  # noqa: F401
                      random_gbuffer, random_material, scene_lights)
