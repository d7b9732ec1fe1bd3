"""Seeded synthetic inputs shared by the oracle and the HIP path.

This package only generates inputs (meshes, bathymetry fields, initial
conditions, friction fields, gauges).  It contains none of the method's
arithmetic and imports neither the oracle nor the library.
"""
from .gen import (  # noqa: F401
    Raster, fractal_raster, workload, WORKLOADS, uniform_mesh_desc, quadtree_desc,
)
