"""Seeded synthetic AMR inputs (block geometry + FP64 cell densities).

This package only *describes inputs*: block-structured octree AMR meshes in the
PARAMESH style (8x8x8-cell blocks, each refined block split into 8 children)
and the density carried by their leaf cells.  It holds none of the potential
method's arithmetic, so both the CPU oracle and the GPU library may consume
what it produces.
"""
from .grids import (  # noqa: F401
    AMRGrid,
    build_grid,
    uniform_sphere,
    maclaurin_spheroid,
    cloud_core,
    plummer_mix,
    plummer_sphere,
    random_amr,
    single_block,
    maclaurin_axes,
)
