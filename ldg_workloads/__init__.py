"""Seeded synthetic inputs (meshes, initial and boundary data) for line-DG.

Shared by the CPU oracle, the tests and the benchmark; holds none of the
discretisation's arithmetic.
"""
from .mesh import (Mesh, gll_points, quad_mesh, hex_mesh, reorient_elements, random_rotations, line_end_node,  # noqa: F401
                   with_boundary_kinds, BC_DIRICHLET, BC_NEUMANN, BC_SLIP)
from . import fields, configs  # noqa: F401
