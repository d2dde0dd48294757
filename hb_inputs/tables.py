"""Tabulation of tau^2, v0, v1 at Chebyshev node pairs (Sec. 4.1).

Layout (shared by every consumer of the tables):
  * the table region is ``nbox[0] x nbox[1] (x nbox[2])`` cubic boxes of side
    ``box_size`` starting at ``box_origin``; box index
    b = bx + nbox0 * (by + nbox1 * bz);
  * each box carries nI first-kind Chebyshev nodes per axis at
    lo + box_size * (1 + cos((2k+1) pi / (2 nI))) / 2, k = 0..nI-1;
    node multi-index a = k1 + nI * (k2 + nI * k3);
  * global node index A = b * nI^d + a; NT = nboxes * nI^d;
  * a table F is NT x NT, row-major, F[A, B] = f(node A (observation),
    node B (source)).
With one box this is the paper's global table; several boxes give a
piecewise table (one Chebyshev expansion per pair of boxes).
"""
from __future__ import annotations

import math

import numpy as np


def cheb_unit_nodes(nI: int) -> np.ndarray:
    """First-kind Chebyshev nodes mapped to [0, 1]."""
    k = np.arange(nI, dtype=np.float64)
    return 0.5 * (1.0 + np.cos((2.0 * k + 1.0) * math.pi / (2.0 * nI)))


def node_coords(dim, nI, nbox, box_origin, box_size) -> np.ndarray:
    """Coordinates of all NT table nodes, shape (NT, dim), in table order."""
    u = cheb_unit_nodes(nI)
    nbox = tuple(int(b) for b in nbox[:dim])
    nb = int(np.prod(nbox))
    nloc = nI ** dim
    P = np.empty((nb * nloc, dim))
    for b in range(nb):
        bidx = []
        rem = b
        for ax in range(dim):
            bidx.append(rem % nbox[ax])
            rem //= nbox[ax]
        for a in range(nloc):
            rem = a
            for ax in range(dim):
                k = rem % nI
                rem //= nI
                P[b * nloc + a, ax] = box_origin[ax] + (bidx[ax] + u[k]) * box_size
    return P


def tabulate(medium, dim, nI, nbox, box_origin, box_size, chunk_rows=256):
    """Return (tau2, v0, v1) tables, each (NT, NT) float64, symmetrised.

    The media used here are reciprocal, so the exact tables are symmetric;
    the explicit (F + F^T)/2 removes rounding asymmetry so that the
    discretised operator is exactly reciprocal when the table is.
    """
    P = node_coords(dim, nI, nbox, box_origin, box_size)
    NT = P.shape[0]
    tau2 = np.empty((NT, NT))
    v0 = np.empty((NT, NT))
    v1 = np.empty((NT, NT))
    for a0 in range(0, NT, chunk_rows):
        a1 = min(NT, a0 + chunk_rows)
        R = np.broadcast_to(P[a0:a1, None, :], (a1 - a0, NT, dim))
        R0 = np.broadcast_to(P[None, :, :], (a1 - a0, NT, dim))
        t, p, q = medium.ingredients(R, R0, dim)
        tau2[a0:a1] = t
        v0[a0:a1] = p
        v1[a0:a1] = q
    for F in (tau2, v0, v1):
        F += F.T.copy()
        F *= 0.5
    return tau2, v0, v1
