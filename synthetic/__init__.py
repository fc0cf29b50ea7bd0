"""Seeded synthetic inputs shared by the tests, the bench and the oracle.

This package produces *inputs only*: triangulated surfaces (vertex and
triangle arrays) and seeded random vectors.  It contains none of the
H-matrix method's arithmetic (no quadrature, no kernel, no clustering), so
that the CPU oracle and the HIP path can both consume the same inputs
without sharing any computation.
"""
from .meshes import icosphere, mesh_sha256, perturbed_sphere, with_near_duplicates
from .vectors import normal_columns, sample_rows

__all__ = ["icosphere", "perturbed_sphere", "with_near_duplicates", "mesh_sha256",
           "normal_columns", "sample_rows"]
