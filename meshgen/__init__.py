"""Seeded synthetic inputs for the Newton-Stokes operator: column meshes, fields, states.

This package produces *inputs only*: mesh topology (hexahedral columns with
one level of isotropic 2:1 refinement, Sec. 3.1 "Meshing"), node placement at
tensor Gauss-Lobatto positions, seeded random fields (the Fourier construction
of eq. (randfield) in Sec. 4.3), dome thickness profiles and seeded states.
It contains none of the finite-element arithmetic (no quadrature, no basis
derivatives, no hanging-node weights); both the CPU oracle and the GPU engine
consume what it produces and compute everything else on their own.
"""
from .columns import ColumnMesh, column_mesh, GLL_CLOSED_FORM
from .configs import make_config, CONFIGS

__all__ = ["ColumnMesh", "column_mesh", "GLL_CLOSED_FORM", "make_config", "CONFIGS"]
