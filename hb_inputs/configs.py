"""The five workloads the integrator is measured on, as seeded synthetic
inputs.  ``c1``..``c5`` accept a reduced size for tests; the defaults are the
full sizes.  Wavelength counts are at n = 1 (lambda = 2 pi / omega).

  c1  2D homogeneous n = 1, 64^2 cells, 8 cells per wavelength, closed-form
      tables (nI = 3, one box), 1 complex128 RHS.
  c2  2D Gaussian bump n = 1 + 0.3 exp(-|r - (1/2,1/2)|^2 / (2 * 0.1^2)),
      1024^2 cells, 128 wavelengths, piecewise tables 8x8 boxes x 8x8 nodes,
      1 RHS.
  c3  64 constant-gradient problems c(y) = 1 + g y, g ~ U[0.2, 1],
      N_side in {128, 256, 512}, omega = 2 pi N_side / 8, global nI = 13,
      1..256 complex64 Gaussian RHS each.
  c4  c2's medium on 256^2 cells, omega = 64 pi, 512 receivers, 20 point
      sources.
  c5  3D n = 1 + 0.2 sin(2 pi x) sin(2 pi y) sin(2 pi z), 64^3 cells,
      omega = 16 pi, global nI = 9, 32 complex64 RHS.
"""
from __future__ import annotations

import math

import numpy as np

from .media import Homogeneous, GaussianBump, ConstantGradient, Sinusoid3D
from .problem import make_problem

CFG_SEED = {"c1": 1, "c2": 2, "c3": 3, "c4": 4, "c5": 5}


def c1(n_side=64, nterms=2):
    omega = 2.0 * math.pi * n_side / 8.0
    return make_problem(Homogeneous(1.0), 2, (n_side, n_side), omega, nI=3,
                        nterms=nterms, name=f"c1-homogeneous-2d-{n_side}")


def bump_problem(n_side, omega, nbox=8, nI=8, name="bump"):
    return make_problem(GaussianBump(), 2, (n_side, n_side), omega, nI=nI,
                        nbox=(nbox, nbox), name=name)


def c2(n_side=1024, nbox=8):
    omega = 2.0 * math.pi * n_side / 8.0
    return bump_problem(n_side, omega, nbox=nbox,
                        name=f"c2-gaussian-bump-2d-{n_side}")


def c3(nprob=64, sides=(128, 256, 512), max_rhs=256, seed=None):
    """Returns a list of (problem, nrhs, rhs_seed)."""
    g = np.random.default_rng([CFG_SEED["c3"], 0] if seed is None else seed)
    out = []
    for p in range(nprob):
        side = int(g.choice(sides))
        grad = float(g.uniform(0.2, 1.0))
        nrhs = int(g.integers(1, max_rhs + 1))
        omega = 2.0 * math.pi * side / 8.0
        prob = make_problem(ConstantGradient(1.0, (0.0, grad)), 2, (side, side),
                            omega, nI=13, name=f"c3-p{p}-cg-{side}-g{grad:.3f}")
        out.append((prob, nrhs, [CFG_SEED["c3"], 1, p]))
    return out


def c4(n_side=256):
    omega = 2.0 * math.pi * n_side / 8.0
    return bump_problem(n_side, omega, nbox=8, name=f"c4-gaussian-bump-2d-{n_side}")


def c5(n_side=64, nI=9):
    omega = 2.0 * math.pi * n_side / 8.0
    return make_problem(Sinusoid3D(), 3, (n_side,) * 3, omega, nI=nI,
                        name=f"c5-sinusoid-3d-{n_side}")
