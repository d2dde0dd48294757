"""Dense FP64 oracle of the HB integrator with a curve inclusion
(Sec. 3.2, domain with a sound-hard inclusion; test infrastructure only).

    U = (K^{v2v} + K^{s2v} (K^{s2s})^{-1} K^{v2s}) I,   I = h^d s
                                                    (eq. m_v2v_inclu)
with, for segment centres r^s_i of lengths w_i and cell centres r_j,
    K^{v2s}_ij = g(r^s_i, r_j)                          (eq. m_v2s)
    K^{s2v}_ij = g(r_i, r^s_j) w_j                      (eq. m_s2v)
                 (for a segment centre inside cell j, g is that cell's self
                 term: the cell average of the leading HB term, App. A)
    K^{s2s}_ij = -g(r^s_i, r^s_j) w_j,  i != j          (eq. s2s)
    K^{s2s}_ii = minus the integral of the leading HB term over segment i
                 in its small-segment closed form
                 -(i w_i / 4) [1 + (2i/pi)(log(e^gamma omega n_i w_i / 4) - 1)]
where g is the HB ansatz evaluated from the tables (eq. babich, N = 1).
The printed diagonal of eq. s2s lacks the factor i of the leading term
(i/4) H0 and writes the Euler constant where e^gamma belongs; the reading
above is the exact integral's small-argument expansion, pinned against
quadrature in the tests.  The system K^{s2s} P = K^{v2s} I (eq. m_sie)
enforces u^inc + u^sca = 0 at the segment centres.

Pins (tests/test_inclusion_pins.py): the diagonal against quadrature of the
segment integral; the whole operator, in a homogeneous medium where the
ansatz is the exact Green's function, against the series solution of
scattering by a disc with zero boundary values, converging as N_s grows;
K^{s2v} against the transpose of K^{v2s} (symmetric tables).
"""
from __future__ import annotations

import math

import numpy as np

from .hb_oracle import apply as v2v_apply
from .hb_oracle import apply_adjoint as v2v_apply_adjoint
from .hb_oracle import hb_terms, interpolate, self_term


def point_kernel(prob, Pr, Pc, skip_diagonal=False):
    """g(r, r0) of the HB ansatz from the tables for observation points Pr
    and source points Pc, complex128 (len(Pr), len(Pc)); with skip_diagonal
    (Pr and Pc the same points) the diagonal is left 0."""
    Pr = np.atleast_2d(np.asarray(Pr, np.float64))
    Pc = np.atleast_2d(np.asarray(Pc, np.float64))
    tau = np.sqrt(np.maximum(interpolate(prob, prob.tau2, Pr, Pc), 0.0))
    if skip_diagonal:
        np.fill_diagonal(tau, 1.0)
    f0, f1 = hb_terms(prob.dim, prob.omega, tau)
    K = interpolate(prob, prob.v0, Pr, Pc) * f0
    if prob.nterms == 2:
        K = K + interpolate(prob, prob.v1, Pr, Pc) * f1
    if skip_diagonal:
        np.fill_diagonal(K, 0.0)
    return K


def segment_self(prob, w, n):
    """K^{s2s}_ii for a segment of length w where the slowness is n."""
    w = np.asarray(w, np.float64)
    L = np.euler_gamma + np.log(prob.omega * np.asarray(n, np.float64) * w / 4.0)
    return -(1j * w / 4.0) * (1.0 + (2j / math.pi) * (L - 1.0))


def containing_cell(prob, P):
    """Natural index of the cell floor((x - origin)/h) (clamped) holding
    each point."""
    P = np.atleast_2d(np.asarray(P, np.float64))
    nat = np.zeros(P.shape[0], np.int64)
    stride = 1
    for ax in range(prob.dim):
        k = np.floor((P[:, ax] - prob.origin[ax]) / prob.h).astype(np.int64)
        nat += np.clip(k, 0, prob.ncell[ax] - 1) * stride
        stride *= prob.ncell[ax]
    return nat


def _segment_cell_kernel(prob, curve, cells):
    """g between every segment centre and the cells `cells`
    ((N_s, len(cells))).  A segment centre lying in a cell is paired with
    that cell through the cell's self term (the cell average of the leading
    HB term, App. A): the point value of the log-singular kernel at
    sub-cell distances is not resolved by the tables (the paper is silent;
    this is the reading)."""
    with np.errstate(invalid="ignore", divide="ignore"):
        G = point_kernel(prob, curve.centres, prob.centres(cells))
    own = containing_cell(prob, curve.centres)
    pos = {int(c): k for k, c in enumerate(cells)}
    for i, c in enumerate(own):
        if int(c) in pos:
            G[i, pos[int(c)]] = self_term(prob, prob.slowness[c])
    return G


def v2s(prob, curve, cols=None):
    """K^{v2s}[:, cols] (N_s x len(cols)); cols in natural cell order."""
    cols = np.arange(prob.Nv) if cols is None else np.asarray(cols, np.int64)
    return _segment_cell_kernel(prob, curve, cols)


def s2v(prob, curve, rows=None):
    """K^{s2v}[rows] (len(rows) x N_s): g(r_j, r^s_i) w_i, with the same
    pairing of a segment centre and its cell as K^{v2s} (g is reciprocal for
    symmetric tables)."""
    rows = np.arange(prob.Nv) if rows is None else np.asarray(rows, np.int64)
    with np.errstate(invalid="ignore", divide="ignore"):
        G = point_kernel(prob, prob.centres(rows), curve.centres)
    own = containing_cell(prob, curve.centres)
    pos = {int(r): k for k, r in enumerate(rows)}
    for i, c in enumerate(own):
        if int(c) in pos:
            G[pos[int(c)], i] = self_term(prob, prob.slowness[c])
    return G * curve.w[None, :]


def s2s(prob, curve):
    """K^{s2s} (N_s x N_s)."""
    ns = curve.Ns
    G = point_kernel(prob, curve.centres, curve.centres, skip_diagonal=True)
    K = -G * curve.w[None, :]
    K[np.arange(ns), np.arange(ns)] = segment_self(prob, curve.w, curve.slowness)
    return K


def apply(prob, curve, s, rows=None, chunk_entries=1 << 22):
    """U[rows] of eq. m_v2v_inclu for sources s ((N_v,) or (N_v, nrhs))."""
    s = np.asarray(s, np.complex128)
    I = s * prob.h ** prob.dim
    Uinc = np.zeros((curve.Ns,) + s.shape[1:], np.complex128)     # eq. m_v2s
    step = max(1, chunk_entries // curve.Ns)
    for a in range(0, prob.Nv, step):
        cols = np.arange(a, min(prob.Nv, a + step))
        Uinc += v2s(prob, curve, cols) @ I[cols]
    P = np.linalg.solve(s2s(prob, curve), Uinc)                    # eq. m_sie
    return v2v_apply(prob, s, rows) + s2v(prob, curve, rows) @ P   # eq. m_s2v


def apply_adjoint(prob, curve, s, cols=None):
    """(T^H s)[cols] for the total operator T = (K^{v2v} + K^{s2v}
    (K^{s2s})^{-1} K^{v2s}) h^d of eq. m_v2v_inclu."""
    s = np.asarray(s, np.complex128)
    Q = np.linalg.solve(s2s(prob, curve).conj().T, s2v(prob, curve).conj().T @ s)
    return v2v_apply_adjoint(prob, s, cols) + \
        prob.h ** prob.dim * (v2s(prob, curve, cols).conj().T @ Q)
