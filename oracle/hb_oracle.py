"""Dense FP64 oracle of the HB integrator (test infrastructure only).

Parity pins: every function here is checked in ``tests/test_oracle_pins.py``
against something independent of this file (closed-form Green's functions,
mpmath Hankel functions, brute-force cell quadratures, exact polynomial
interpolation, explicit double loops).  No function is "parity unpinned".
"""
from __future__ import annotations

import math
from functools import lru_cache

import numpy as np
from scipy import integrate, special

SQRT_PI = math.sqrt(math.pi)


# ---------------------------------------------------------------------------
# Chebyshev interpolation (Sec. 4.1, eq. chebinterp, eq. chebinterpblock)
# ---------------------------------------------------------------------------
def cheb_nodes(nI):
    """First-kind Chebyshev nodes of one box, as fractions of the box side:
    (1 + cos((2k+1) pi / (2 nI))) / 2, k = 0..nI-1."""
    k = np.arange(nI, dtype=np.float64)
    return 0.5 * (1.0 + np.cos((2.0 * k + 1.0) * math.pi / (2.0 * nI)))


def lagrange_1d(x, nodes):
    """Lagrange basis by the product formula of Sec. 4.1:
    l_i(x) = prod_{k != i} (x - x_k) / (x_i - x_k).  Returns (len(x), nI)."""
    x = np.asarray(x, np.float64)
    nI = len(nodes)
    out = np.ones((x.size, nI))
    for i in range(nI):
        for k in range(nI):
            if k != i:
                out[:, i] *= (x - nodes[k]) / (nodes[i] - nodes[k])
    return out


def interp_weights(prob, P):
    """Box index of each point and its tensor Lagrange weights
    T_a(r) = prod_s l_{a_s}(r_s) over the nodes of that box; a point on a
    box face belongs to the box floor((x - origin)/size), clamped to the
    table region.  Returns (box (m,), T (m, nI^d))."""
    P = np.atleast_2d(np.asarray(P, np.float64))
    d, nI = prob.dim, prob.nI
    nodes = cheb_nodes(nI)
    box = np.zeros(P.shape[0], dtype=np.int64)
    stride = 1
    W = None
    for ax in range(d):
        rel = (P[:, ax] - prob.box_origin[ax]) / prob.box_size
        b = np.clip(np.floor(rel).astype(np.int64), 0, prob.nbox[ax] - 1)
        box += b * stride
        stride *= prob.nbox[ax]
        l = lagrange_1d(rel - b, nodes)            # (m, nI) for this axis
        # multi-index a = k1 + nI*(k2 + nI*k3): earlier axes vary fastest
        W = l if W is None else (l[:, :, None] * W[:, None, :]).reshape(P.shape[0], -1)
    return box, W


def interpolate(prob, F, Prow, Pcol):
    """F(r_i, r_j) ~ T^o F^c T^s for observation points Prow and source
    points Pcol (eq. chebinterpblock), evaluated per pair of table boxes."""
    bo, To = interp_weights(prob, Prow)
    bs, Ts = interp_weights(prob, Pcol)
    nloc = prob.nI ** prob.dim
    out = np.empty((To.shape[0], Ts.shape[0]))
    for a in np.unique(bo):
        ri = np.nonzero(bo == a)[0]
        Fa = F[a * nloc:(a + 1) * nloc]
        for b in np.unique(bs):
            ci = np.nonzero(bs == b)[0]
            Fab = Fa[:, b * nloc:(b + 1) * nloc]
            out[np.ix_(ri, ci)] = To[ri] @ Fab @ Ts[ci].T
    return out


# ---------------------------------------------------------------------------
# HB terms (Sec. 2, eq. termf) and self terms (Appendix A)
# ---------------------------------------------------------------------------
def hb_terms(d, omega, tau):
    """(f_{-(d-2)/2}, f_{1-(d-2)/2})(omega, tau) of eq. termf,
    f_q = i (sqrt(pi)/2) e^{i q pi} (2 tau/omega)^q H^(1)_q(omega tau).
    2D: q = 0, 1 with H^(1)_q = J_q + i Y_q.
    3D: q = -1/2, 1/2, where the half-order Hankel functions are elementary:
        f_{-1/2} = e^{i omega tau} / (2 tau),  f_{1/2} = (i/omega) e^{i omega tau}.
    """
    tau = np.asarray(tau, np.float64)
    x = omega * tau
    if d == 2:
        h0 = special.j0(x) + 1j * special.y0(x)
        h1 = special.j1(x) + 1j * special.y1(x)
        f0 = 1j * (SQRT_PI / 2.0) * h0
        f1 = -1j * SQRT_PI * (tau / omega) * h1
        return f0, f1
    if d == 3:
        e = np.exp(1j * x)
        return e / (2.0 * tau), (1j / omega) * e
    raise ValueError("dimension must be 2 or 3")


@lru_cache(maxsize=65536)
def _self_term_cached(d, h, n, omega):
    if d == 2:
        # Lemma (eq. HankelIntegral2dlemma): integral of H0(omega n |r-r0|)
        # over the cell = (n omega)^-2 [8 int_0^{pi/4} X H1(X) dtheta + 4i],
        # X = h n omega / (2 cos theta); times v0(r,r) i sqrt(pi)/2 = i/4.
        a = h * n * omega / 2.0

        def re(t):
            X = a / math.cos(t)
            return X * special.j1(X)

        def im(t):
            X = a / math.cos(t)
            return X * special.y1(X)

        kw = dict(epsabs=0.0, epsrel=1e-12, limit=200)
        s = integrate.quad(re, 0.0, math.pi / 4.0, **kw)[0] + \
            1j * integrate.quad(im, 0.0, math.pi / 4.0, **kw)[0]
        I = (8.0 * s + 4.0j) / (n * omega) ** 2
        return (1j / 4.0) * I / h ** 2
    if d == 3:
        # Q_s of eq. e312 with f of eq. e313 and r_1 of eq. e314; the cell
        # integral is i Q_s / (4 pi omega^2 n^2).
        def f(rp, phi, part):
            c = math.cos(phi)
            rho = rp / c
            r1 = omega * n * (h / 2.0) * math.sqrt(1.0 + rho * rho)
            val = (np.exp(1j * r1) * (1.0 - 1j * r1) - 1.0) * rho / \
                (1.0 + rho * rho) ** 1.5 / c
            return val.real if part == 0 else val.imag

        kw = dict(epsabs=0.0, epsrel=1e-12)
        re = integrate.dblquad(lambda rp, phi: f(rp, phi, 0), 0.0, math.pi / 4.0,
                               0.0, 1.0, **kw)[0]
        im = integrate.dblquad(lambda rp, phi: f(rp, phi, 1), 0.0, math.pi / 4.0,
                               0.0, 1.0, **kw)[0]
        Qs = -48j * (re + 1j * im)
        I = 1j * Qs / (4.0 * math.pi * omega ** 2 * n ** 2)
        return I / h ** 3
    raise ValueError("dimension must be 2 or 3")


def self_term(prob, n_i):
    """K_ii for a cell of slowness n_i (Appendix A; leading HB term with v0
    at its source value, integrated over the cell, divided by h^d)."""
    return complex(_self_term_cached(prob.dim, float(prob.h), float(n_i),
                                     float(prob.omega)))


# ---------------------------------------------------------------------------
# Entries and products (Sec. 3.1, eq. m_v2v)
# ---------------------------------------------------------------------------
def entries(prob, rows, cols):
    """K[rows][:, cols] in natural cell order, complex128."""
    rows = np.asarray(rows, np.int64)
    cols = np.asarray(cols, np.int64)
    Pr = prob.centres(rows)
    Pc = prob.centres(cols)
    tau2 = interpolate(prob, prob.tau2, Pr, Pc)
    v0 = interpolate(prob, prob.v0, Pr, Pc)
    tau = np.sqrt(np.maximum(tau2, 0.0))
    same = rows[:, None] == cols[None, :]
    tau_safe = np.where(same, 1.0, tau)
    f0, f1 = hb_terms(prob.dim, prob.omega, tau_safe)
    K = v0 * f0
    if prob.nterms == 2:
        v1 = interpolate(prob, prob.v1, Pr, Pc)
        K = K + v1 * f1
    ii, jj = np.nonzero(same)
    for a, b in zip(ii, jj):
        K[a, b] = self_term(prob, prob.slowness[rows[a]])
    return K


def _chunk(n, size):
    for a in range(0, n, size):
        yield a, min(n, a + size)


def apply(prob, s, rows=None, chunk_entries=1 << 22):
    """u[rows] = (K (h^d s))[rows]; s is (N_v,) or (N_v, nrhs)."""
    s = np.asarray(s, np.complex128)
    rows = np.arange(prob.Nv) if rows is None else np.asarray(rows, np.int64)
    I = s * prob.h ** prob.dim
    cols = np.arange(prob.Nv)
    out = np.empty((rows.size,) + s.shape[1:], np.complex128)
    step = max(1, chunk_entries // prob.Nv)
    for a, b in _chunk(rows.size, step):
        out[a:b] = entries(prob, rows[a:b], cols) @ I
    return out


def apply_adjoint(prob, s, cols=None, chunk_entries=1 << 22):
    """(h^d K^H s)[cols]: the conjugate transpose of the discretised
    integrator, applied to s."""
    s = np.asarray(s, np.complex128)
    cols = np.arange(prob.Nv) if cols is None else np.asarray(cols, np.int64)
    rows = np.arange(prob.Nv)
    out = np.empty((cols.size,) + s.shape[1:], np.complex128)
    step = max(1, chunk_entries // prob.Nv)
    for a, b in _chunk(cols.size, step):
        Kc = entries(prob, rows, cols[a:b])
        out[a:b] = Kc.conj().T @ s
    return out * prob.h ** prob.dim


def dense(prob):
    """The full N_v x N_v matrix K (small problems only)."""
    idx = np.arange(prob.Nv)
    return entries(prob, idx, idx)
