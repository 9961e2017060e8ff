"""Seeded synthetic inputs shared by the oracle and the HIP path.

This package only *generates* data: simplicial meshes (interior nodes numbered
first), nodal coefficient fields and right-hand sides.  It contains none of the
method's arithmetic (no kernel, quadrature, tree or assembly), so that the
oracle and the GPU path can both read the same inputs without sharing code.
"""
from .meshes import Mesh, interval_mesh, square_mesh, disk_mesh  # noqa: F401
from . import configs  # noqa: F401
