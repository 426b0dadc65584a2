"""Seeded synthetic inputs for the regularized single-layer sum.

Surfaces (six-patch POU discretizations with trapezoid-POU weights), smooth
force densities and request streams. This package holds no single-layer
arithmetic; the oracle tests and the GPU path both draw their inputs from it.
"""
from .surfaces import (ELLIPSOID_PAPER, ELLIPSOID_SERVING, RBC, SPHERE, Shape, Surface,
                       make_surface, pou, bump, chart, patch_centre, fine_grid, fine_pou,
                       fine_positions)
from .forces import sh_force, uniform_force, real_sph_harm
from . import workloads

__all__ = ["Shape", "Surface", "make_surface", "pou", "bump", "chart", "patch_centre",
           "fine_grid", "fine_pou", "fine_positions",
           "sh_force", "uniform_force", "real_sph_harm", "workloads",
           "SPHERE", "RBC", "ELLIPSOID_SERVING", "ELLIPSOID_PAPER"]
