"""Seeded synthetic workloads: periodic mixed-element meshes and initial-state inputs.

This package holds no arithmetic of the DG method itself. It builds mesh tables
(element types, corner vertex ids, corner coordinates, centroids), the analytic
initial field and the seeded noise, and is shared by the oracle, the tests and
the benchmark.
"""
from .meshgen import (  # noqa: F401
    HEX, PRISM, PYR, TET, TYPE_NAMES, Mesh, make_mesh, deformed, motion, cell_kinds_config,
    config_mesh, tgv_primitive, density_wave_primitive, node_noise, time_step,
    CONFIGS, config_params, batched_configs, stored_dofs, coefficient_state,
)
