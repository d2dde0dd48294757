"""Seeded right-hand sides.  Seeds are numpy ``default_rng`` seed sequences
(lists of ints), so the same (config, stream) pair gives the same numbers on
every machine."""
from __future__ import annotations

import numpy as np


def rng(seed):
    return np.random.default_rng(seed)


def complex_normal(shape, seed, dtype=np.complex128):
    """Re and Im i.i.d. N(0, 1)."""
    g = rng(seed)
    re = g.standard_normal(shape)
    im = g.standard_normal(shape)
    return (re + 1j * im).astype(dtype)


def gaussian_sources(prob, nrhs, seed, width_cells=2.0, dtype=np.complex64):
    """Column k = exp(i phi_k) exp(-|r - c_k|^2 / (2 (width_cells h)^2)) with
    c_k ~ U[0.1, 0.9]^d (in units of the domain) and phi_k ~ U[0, 2 pi)."""
    g = rng(seed)
    P = prob.centres()
    lo = np.asarray(prob.origin)
    ext = np.asarray(prob.ncell[: prob.dim]) * prob.h
    out = np.empty((prob.Nv, nrhs), dtype=np.complex128)
    sig = width_cells * prob.h
    for k in range(nrhs):
        c = lo + ext * g.uniform(0.1, 0.9, size=prob.dim)
        phi = g.uniform(0.0, 2.0 * np.pi)
        r2 = np.sum((P - c) ** 2, axis=1)
        out[:, k] = np.exp(1j * phi) * np.exp(-r2 / (2.0 * sig * sig))
    return np.asfortranarray(out.astype(dtype))


def point_sources(prob, count, seed):
    """``count`` distinct cells with complex N(0,1) amplitudes a_j; returns
    (cells, s) with s = sum_j a_j delta_j / h^d, i.e. I = h^d s has the
    amplitudes at the chosen cells (point sources, Sec. 3.1)."""
    g = rng(seed)
    cells = np.sort(g.choice(prob.Nv, size=count, replace=False))
    amp = g.standard_normal(count) + 1j * g.standard_normal(count)
    s = np.zeros(prob.Nv, dtype=np.complex128)
    s[cells] = amp / prob.h ** prob.dim
    return cells, s
