"""Seeded synthetic inputs for the FE^2 hot path.

This package builds problem descriptions (macro meshes, boundary data and
RVE microstructures) as plain NumPy arrays.  It holds none of the method's
arithmetic: no element routine, no constitutive law, no solver.  Both the
FP64 oracle and the GPU library read the same descriptions, which is why it
lives on its own.
"""
from .generators import (  # noqa: F401
    Problem,
    config,
    config_names,
    macro_q4_grid,
    macro_q9_grid,
    macro_hex8_grid,
    macro_q4_cook,
    lame_from_young,
    phases_laminate,
    phases_circle,
    phases_sphere,
    phases_cross,
    subset_problem,
    element_basis,
    oned_problem,
    OneDProblem,
    mlp_init,
    cfg5_material_points,
    surrogate_samples,
    SURROGATE_BOX,
)
