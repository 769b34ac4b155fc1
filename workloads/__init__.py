"""Seeded synthetic inputs shared by the tests, the bench and the smoke check.

This package only *generates inputs*: unstructured simplex meshes of the unit
square / cube, element-wise diffusion coefficients and analytic source
functions.  It contains none of the discretisation or solver arithmetic; the
oracle and the GPU library each implement those on their own.
"""
from .meshes import Mesh, mesh2d_jittered_delaunay, mesh2d_square_neumann_sides, mesh3d_kuhn, quad_grid  # noqa: F401
from .fields import kappa_grf, kappa_spheres, source_sine, exact_sine  # noqa: F401
from .configs import CONFIGS, config_mesh  # noqa: F401
