"""Seeded synthetic inputs for the Hadamard-Babich (HB) integrator.

This package builds the *inputs* of the HB volume integrator: the cell grid,
the medium (slowness n(r) at the cell centres), the tabulated HB ingredients
tau^2, v0, v1 at Chebyshev node pairs, and right-hand sides.  It is shared by
the CPU oracle and the GPU path and deliberately contains none of the
integrator's own arithmetic (no Lagrange interpolation, no Hankel terms, no
self terms, no compression): only the media, their tabulation at fixed node
pairs, and random numbers.

In the paper the tables come from Lax-Friedrichs WENO eikonal/transport solves
with point sources at the Chebyshev nodes (Sec. 4.1, eq. chebinterp and the
tabulation paragraph after it); that solver is outside this project.  Here the
tables are filled from closed forms where the medium has one (homogeneous and
constant-gradient media, Sec. 5.1) and from a smooth straight-ray stand-in
otherwise.
"""
from .media import (Homogeneous, ConstantGradient, GaussianBump, Sinusoid3D, Sinusoid2D,
                    n2_taylor, medium_grid, taylor_at)
from .tables import cheb_unit_nodes, node_coords, tabulate
from .problem import HBProblem, make_problem
from .rhs import complex_normal, gaussian_sources, point_sources
from .curves import Curve, circle, open_square
from . import configs

__all__ = [
    "Homogeneous", "ConstantGradient", "GaussianBump", "Sinusoid3D", "Sinusoid2D", "n2_taylor",
    "medium_grid", "taylor_at",
    "cheb_unit_nodes", "node_coords", "tabulate", "HBProblem", "make_problem",
    "complex_normal", "gaussian_sources", "point_sources", "Curve", "circle", "open_square", "configs",
]
