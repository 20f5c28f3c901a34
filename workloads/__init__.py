"""Seeded synthetic inputs shared by the oracle and the GPU library (no method arithmetic)."""
from .rng import SplitMix64, stream_seed  # noqa: F401
from .meshes import (FLUID, SOLID, LOAD_POINT_FORCE, LOAD_SKIN_PRESSURE,  # noqa: F401
                     LOAD_VOLUME_VELOCITY, Load, Material, Mesh, fluid_nodes, solid_nodes)
from .configs import (Workload, batched_variants, box, fuselage_variants, fuselage_workload,  # noqa: F401
                      plate_cavity_workload, small_plate_cavity)
