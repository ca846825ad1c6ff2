"""Seeded synthetic inputs for the BEM hot path.

This package only produces inputs: triangle meshes with body tags, body
tables, evaluation points, field-line start points and load cases.  It holds
none of the method's arithmetic (no kernels, no quadrature, no assembly), so
that the oracle and the GPU path can both consume the same inputs while
sharing no computation.
"""

from .meshes import (  # noqa: F401
    Problem,
    icosphere,
    sphere_problem,
    coated_sphere_problem,
    floating_shell_problem,
    coax_problem,
    coax_problem_for_size,
    coax_conductors_problem,
    coax_conductors_for_vertices,
    sphere_sheet_problem,
    bushing_problem,
    union_problem,
)
from .seeds import (  # noqa: F401
    sphere_eval_points,
    gap_eval_points,
    electrode_line_starts,
    rod_load_cases,
    vertex_perturbations,
)
