"""Seeded synthetic SPD problems for the hierarchical solver.

This package only builds inputs (matrices, grids, right-hand sides); it
holds none of the solver's arithmetic.  Both the CPU oracle and the HIP
path take their inputs from here.
"""
from .problems import (  # noqa: F401
    Problem,
    laplace2d,
    slab_scalar,
    slab_vector,
    slab_icesheet,
    layer_mesh,
    extruded_mesh,
    lognormal_field,
    rhs,
    batch_params,
    batch_system,
    batch_rhs,
    config,
    config_variant,
    CONFIG_NAMES,
)
