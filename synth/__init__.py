"""Seeded synthetic inputs: tetrahedral meshes, boundary sets and material tables.

This package is shared by the CPU oracle and the GPU path.  It builds inputs
only: lattice meshes split into tetrahedra, boundary-node masks, loaded
boundary triangles with their traction vectors, fibre directions and material
records.  It performs none of the finite-element arithmetic of the method
(no stresses, no element integrals, no nodal loads).
"""
from .meshes import (  # noqa: F401
    Problem,
    cube_mesh,
    tube_mesh,
    boundary_faces,
    cube_problem,
    tube_problem,
    uniaxial_problem,
    random_state,
    config_problem,
    FsiModel,
    fsi_duct,
    fsi_tube,
    lumen_mesh,
)
