"""HB tables from the eikonal and transport solves (test infrastructure only).

The paper tabulates tau^2, v0, v1 at pairs of Chebyshev nodes (Sec. 4.1,
eq. chebinterp): for every source node it solves the eikonal and transport
equations on a grid of spacing h0 aligned with the source and interpolates
the grid values to the other nodes with local cubics (Fig. table-compute).
The solves (Sec. 2.3) use the factored eikonal (eq. faceik) and the
transport recurrence (eq. equVs) by Lax-Friedrichs WENO sweeping, with the
unknowns held at their Taylor expansions about the source (Sec. 2.2:
eq. expansionT / recursiveT, eq. expansionV0 / recursiveB, eq. expansionV1 /
C0, C1, recursiveC; truncation P_T = 6, P_B = P_S = 4, P_C = 2) in a square
of half-width P - 1 cells around it.

This module is plain and slow: the recursions are written term by term on
dense polynomial coefficient arrays, the sweeps are the C loops of
oracle/sweep.c (gcc, called through ctypes), one source at a time.  It
shares no code with the library; it reads the medium (slowness on the grid,
Taylor coefficients of n^2 at the source) from ``hb_inputs``.

Readings (2D only):
  * tt = n0 |r - r0| (the paper's first choice of the factor), n0 = n(r0);
  * fixed neighbourhoods: |i - i0| <= P - 1 and |j - j0| <= P - 1 grid
    points ("a neighbourhood of size 2(P - 1) h0 centred at the source");
  * the LxF sweep and WENO5 details are those stated in oracle/sweep.c
    (WENO epsilon h0^2, the O(h^2) choice of the WENO accuracy analyses:
    with the customary 1e-6 the v1 sweeps of the sinusoidal medium end in
    a limit cycle of updates near 1e-5 instead of converging; viscosities the largest |dH/dp|, |dH/dq| bounds over the
    grid: tt for the eikonal, |b_x|, |b_y| for the transport; first-order
    one-sided differences in
    the three outer grid layers where the WENO stencil does not fit,
    relaxation 1 for the eikonal and 1/2 for the transport sweeps);
  * grad tau^2, Laplacians: sixth-order central differences on the grid,
    second order in the three outer layers;
  * the grid covers the table region plus `margin` cells on every side;
    values at the nodes come from the 4 x 4 Lagrange cubic around each node.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

from .hb_oracle import cheb_nodes

HERE = os.path.dirname(os.path.abspath(__file__))
PT, PS, PB, PC = 6, 4, 4, 2
DEG = 8          # polynomial arrays hold degrees <= DEG


# ---------------------------------------------------------------------------
# Taylor expansions about the source (Sec. 2.2)
# ---------------------------------------------------------------------------
def _hom(A, k):
    """Homogeneous part of degree k of a coefficient array A[i, j] (x^i y^j)."""
    B = np.zeros_like(A)
    for i in range(k + 1):
        if i < A.shape[0] and k - i < A.shape[1]:
            B[i, k - i] = A[i, k - i]
    return B


def _mul(A, B):
    C = np.zeros((DEG + 1, DEG + 1))
    for i in range(DEG + 1):
        for j in range(DEG + 1 - i):
            if A[i, j] == 0.0:
                continue
            for k in range(DEG + 1 - i - j):
                for l in range(DEG + 1 - i - j - k):
                    C[i + k, j + l] += A[i, j] * B[k, l]
    return C


def _dx(A):
    C = np.zeros_like(A)
    for i in range(1, DEG + 1):
        C[i - 1, :] = i * A[i, :]
    return C


def _dy(A):
    C = np.zeros_like(A)
    for j in range(1, DEG + 1):
        C[:, j - 1] = j * A[:, j]
    return C


def _lap(A):
    return _dx(_dx(A)) + _dy(_dy(A))


def _gdot(A, B):
    return _mul(_dx(A), _dx(B)) + _mul(_dy(A), _dy(B))


def poly_eval(A, x, y):
    """Value of the coefficient array A at (x, y) (arrays broadcast)."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    out = np.zeros(np.broadcast(x, y).shape)
    for i in range(A.shape[0]):
        for j in range(A.shape[1] - i):
            if A[i, j] != 0.0:
                out = out + A[i, j] * x ** i * y ** j
    return out


def taylor(S, d=2):
    """Homogeneous parts T_k (k <= P_T), B_k (k <= P_B), C_k (k <= P_C) of
    tau^2, v0 and v1 about the source from the Taylor coefficients S[i, j]
    of n^2 (i + j <= P_S), by the recursions of Sec. 2.2."""
    Sfull = np.zeros((DEG + 1, DEG + 1))
    Sfull[: S.shape[0], : S.shape[1]] = S
    Sk = [_hom(Sfull, k) for k in range(PS + 1)]
    S0 = Sk[0][0, 0]
    Z = lambda: np.zeros((DEG + 1, DEG + 1))
    # eq. recursiveT: T_0 = T_1 = 0, T_2 = S_0 |r|^2,
    # (P-1) S_0 T_P = sum_{k=1}^{P-2} S_k T_{P-k} - 1/4 sum_{k=2}^{P-2} grad T_{k+1} . grad T_{P-k+1}
    T = [Z() for _ in range(PT + 1)]
    T[2][2, 0] = T[2][0, 2] = S0
    for P in range(3, PT + 1):
        acc = Z()
        for k in range(1, P - 1):
            if k <= PS:
                acc += _mul(Sk[k], T[P - k])
        for k in range(2, P - 1):
            acc -= 0.25 * _gdot(T[k + 1], T[P - k + 1])
        T[P] = _hom(acc, P) / ((P - 1) * S0)
    # eq. recursiveB (with B_1 its P = 1 case): B_0 = n0^(d-2) / (2 pi^((d-1)/2)),
    # 2 P S_0 B_P = -sum_{k=1}^{P-1} grad B_k . grad T_{P+2-k}
    #               - 1/2 sum_{k=0}^{P-1} B_k lap T_{P+2-k} + d sum_{k=0}^{P-1} B_k S_{P-k}
    B = [Z() for _ in range(PB + 1)]
    B[0][0, 0] = math.sqrt(S0) ** (d - 2) / (2.0 * math.pi ** ((d - 1) / 2.0))
    for P in range(1, PB + 1):
        acc = Z()
        for k in range(1, P):
            acc -= _gdot(B[k], T[P + 2 - k])
        for k in range(0, P):
            acc -= 0.5 * _mul(B[k], _lap(T[P + 2 - k]))
            acc += d * _mul(B[k], Sk[P - k])
        B[P] = _hom(acc, P) / (2 * P * S0)
    # eq. C0, C1, recursiveC: 2 (P+1) S_0 C_P = 1/2 lap B_{P+2}
    #   - sum_{k=1}^{P-1} grad C_k . grad T_{P+2-k} - 1/2 sum_{k=0}^{P-1} C_k lap T_{P+2-k}
    #   - (2-d) sum_{k=0}^{P-1} C_k S_{P-k}
    C = [Z() for _ in range(PC + 1)]
    for P in range(0, PC + 1):
        acc = 0.5 * _lap(B[P + 2])
        for k in range(1, P):
            acc -= _gdot(C[k], T[P + 2 - k])
        for k in range(0, P):
            acc -= 0.5 * _mul(C[k], _lap(T[P + 2 - k]))
            acc -= (2 - d) * _mul(C[k], Sk[P - k])
        C[P] = _hom(acc, P) / (2 * (P + 1) * S0)
    return T, B, C


# ---------------------------------------------------------------------------
# LxF-WENO sweeps (oracle/sweep.c)
# ---------------------------------------------------------------------------
_LIB = None


def sweep_library():
    """Compile oracle/sweep.c with gcc (when missing or older than the
    source) and load it."""
    global _LIB
    if _LIB is not None:
        return _LIB
    src = os.path.join(HERE, "sweep.c")
    so = os.path.join(HERE, "libsweep.so")
    if not os.path.exists(so) or os.path.getmtime(so) < os.path.getmtime(src):
        tmp = so + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-o", tmp, src, "-lm"])
        os.replace(tmp, so)
    lib = ctypes.CDLL(so)
    D = ctypes.POINTER(ctypes.c_double)
    lib.hb_sweep.restype = ctypes.c_int
    lib.hb_sweep.argtypes = [ctypes.c_int, D, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                             ctypes.c_double, D, D, D, D, D, D, ctypes.POINTER(ctypes.c_ubyte), ctypes.c_double,
                             ctypes.c_double, ctypes.c_int, D]
    _LIB = lib
    return lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def viscosity(bound):
    """The Lax-Friedrichs viscosity of a sweep: the largest value of the
    pointwise bound over the whole grid (the global choice; bounds taken
    point by point, or over small neighbourhoods, let the sweeps diverge for
    sources near the edge of the table region)."""
    return np.full_like(np.asarray(bound, np.float64), float(np.max(bound)))


def _sweep(kind, u, h, c, visc, fixed, omega, tol=1e-13, maxrounds=4000):
    nx, ny = u.shape
    U = np.asfortranarray(u, dtype=np.float64).copy(order="F")
    cs = [np.asfortranarray(a, dtype=np.float64) for a in tuple(c) + tuple(visc)]
    fx = np.asfortranarray(fixed, dtype=np.uint8)
    last = ctypes.c_double()
    rounds = sweep_library().hb_sweep(kind, _dp(U), nx, ny, h, h * h, *[_dp(a) for a in cs],
                                      fx.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte)),
                                      omega, tol, maxrounds, ctypes.byref(last))
    if not last.value < tol:
        raise RuntimeError(f"sweeps did not converge: {rounds} rounds, last update {last.value}")
    return np.array(U), rounds


def _d1(u, h, axis):
    """First derivative along `axis`: sixth-order central differences where
    the seven points lie in the grid, second-order central next to the
    edges, second-order one-sided on them."""
    u = np.moveaxis(np.asarray(u, np.float64), axis, 0)
    n = u.shape[0]
    d = np.empty_like(u)
    c = (-1 / 60, 3 / 20, -3 / 4, 0.0, 3 / 4, -3 / 20, 1 / 60)
    d[3:n - 3] = sum(c[k] * u[k:n - 6 + k] for k in range(7)) / h
    for i in (1, 2, n - 3, n - 2):
        d[i] = (u[i + 1] - u[i - 1]) / (2 * h)
    d[0] = (-3 * u[0] + 4 * u[1] - u[2]) / (2 * h)
    d[n - 1] = (3 * u[n - 1] - 4 * u[n - 2] + u[n - 3]) / (2 * h)
    return np.moveaxis(d, 0, axis)


def _d2(u, h, axis):
    """Second derivative along `axis`, with the same order reduction."""
    u = np.moveaxis(np.asarray(u, np.float64), axis, 0)
    n = u.shape[0]
    d = np.empty_like(u)
    c = (1 / 90, -3 / 20, 3 / 2, -49 / 18, 3 / 2, -3 / 20, 1 / 90)
    d[3:n - 3] = sum(c[k] * u[k:n - 6 + k] for k in range(7)) / (h * h)
    for i in (1, 2, n - 3, n - 2):
        d[i] = (u[i + 1] - 2 * u[i] + u[i - 1]) / (h * h)
    d[0] = (2 * u[0] - 5 * u[1] + 4 * u[2] - u[3]) / (h * h)
    d[n - 1] = (2 * u[n - 1] - 5 * u[n - 2] + 4 * u[n - 3] - u[n - 4]) / (h * h)
    return np.moveaxis(d, 0, axis)


def fd6(u, h):
    """(d/dx, d/dy, Laplacian) of grid values u (_d1, _d2)."""
    return _d1(u, h, 0), _d1(u, h, 1), _d2(u, h, 0) + _d2(u, h, 1)


def source_grid(r0, lo, hi, h0, margin):
    """Index range of the grid aligned with r0 (point r0 + (i, j) h0) that
    covers [lo - margin h0, hi + margin h0] per axis; returns (i_lo, n) per
    axis, the source at index -i_lo."""
    out = []
    for ax in range(2):
        a = int(math.floor((lo[ax] - r0[ax]) / h0)) - margin
        b = int(math.ceil((hi[ax] - r0[ax]) / h0)) + margin
        out.append((a, b - a + 1))
    return out


def solve_source(medium_n, S, r0, lo, hi, h0, margin=8):
    """tau^2, v0, v1 on the grid aligned with the source r0 (2D).  medium_n:
    callable giving n at points (..., 2); S: Taylor coefficients of n^2 at
    r0 (S[i, j], i + j <= 4).  Returns (x0 of index 0, y0 of index 0, tau2,
    v0, v1, rounds)."""
    (ia, nx), (ja, ny) = source_grid(r0, lo, hi, h0, margin)
    I = np.arange(ia, ia + nx)[:, None] * np.ones((1, ny))
    J = np.ones((nx, 1)) * np.arange(ja, ja + ny)[None, :]
    X = r0[0] + I * h0
    Y = r0[1] + J * h0
    n = medium_n(np.stack([X, Y], axis=-1))
    T, B, C = taylor(S)
    n0 = math.sqrt(S[0, 0])
    dx, dy = X - r0[0], Y - r0[1]
    rho = np.hypot(dx, dy)
    tt = n0 * rho
    with np.errstate(invalid="ignore", divide="ignore"):
        ttx = np.where(rho > 0, n0 * dx / rho, 0.0)
        tty = np.where(rho > 0, n0 * dy / rho, 0.0)
    near = lambda P: (np.abs(I) <= P - 1) & (np.abs(J) <= P - 1)
    # factored eikonal: tau = tt * tb, tb held at sqrt(sum T_k) / tt near the source
    fixT = near(PT)
    t2tay = poly_eval(sum(T), dx, dy)
    with np.errstate(invalid="ignore", divide="ignore"):
        tbf = np.where(rho > 0, np.sqrt(np.maximum(t2tay, 0.0)) / np.where(rho > 0, tt, 1.0), 1.0)
    tb = np.where(fixT, tbf, 1.0)
    # |dH/dp|, |dH/dq| <= tt
    vt = viscosity(tt)
    tb, r1 = _sweep(0, tb, h0, (n, tt, ttx, tty), (vt, vt), fixT, 1.0)
    tau2 = (tb * tt) ** 2
    gx, gy, lt = fd6(tau2, h0)
    ax, ay = 2.0 * gx, 2.0 * gy
    # v0 (eq. equVs with s = -1): 2 grad tau^2 . grad v0 + v0 (lap tau^2 - 2 d n^2) = 0
    fixB = near(PB)
    v0 = np.where(fixB, poly_eval(sum(B), dx, dy), B[0][0, 0])
    vx, vy = viscosity(np.abs(ax)), viscosity(np.abs(ay))
    v0, r2 = _sweep(1, v0, h0, (ax, ay, lt - 4.0 * n * n, np.zeros_like(n)), (vx, vy), fixB, 0.5)
    # v1 (s = 0): 2 grad tau^2 . grad v1 + v1 (lap tau^2 + 2 n^2 (2 - d)) = lap v0
    _, _, lv0 = fd6(v0, h0)
    fixC = near(PC)
    v1 = np.where(fixC, poly_eval(sum(C), dx, dy), 0.0)
    v1, r3 = _sweep(1, v1, h0, (ax, ay, lt, lv0), (vx, vy), fixC, 0.5)
    return X[0, 0], Y[0, 0], tau2, v0, v1, (r1, r2, r3)


def cubic_at(F, x0, y0, h0, P):
    """Values of the grid function F (F[i, j] at (x0 + i h0, y0 + j h0)) at
    the points P (m, 2) by the tensor Lagrange cubic on the 4 x 4 grid
    points around each point."""
    P = np.atleast_2d(P)
    out = np.empty(P.shape[0])
    for m, (x, y) in enumerate(P):
        fx, fy = (x - x0) / h0, (y - y0) / h0
        i, j = int(math.floor(fx)), int(math.floor(fy))
        tx, ty = fx - i, fy - j
        wx = [-tx * (tx - 1) * (tx - 2) / 6, (tx + 1) * (tx - 1) * (tx - 2) / 2,
              -(tx + 1) * tx * (tx - 2) / 2, (tx + 1) * tx * (tx - 1) / 6]
        wy = [-ty * (ty - 1) * (ty - 2) / 6, (ty + 1) * (ty - 1) * (ty - 2) / 2,
              -(ty + 1) * ty * (ty - 2) / 2, (ty + 1) * ty * (ty - 1) / 6]
        acc = 0.0
        for a in range(4):
            for b in range(4):
                acc += wx[a] * wy[b] * F[i - 1 + a, j - 1 + b]
        out[m] = acc
    return out


def node_coords(nI, nbox, box_origin, box_size):
    """Table nodes in table order (2D), as in the tables' layout."""
    u = cheb_nodes(nI)
    P = []
    for b in range(nbox[0] * nbox[1]):
        bx, by = b % nbox[0], b // nbox[0]
        for a in range(nI * nI):
            k1, k2 = a % nI, a // nI
            P.append((box_origin[0] + (bx + u[k1]) * box_size,
                      box_origin[1] + (by + u[k2]) * box_size))
    return np.array(P)


def tables(medium_n, taylor_at, nI, nbox, box_origin, box_size, h0, margin=8):
    """(tau2, v0, v1) tables, NT x NT with F[A, B] = f(node A, source node B),
    symmetrised; taylor_at(r0) gives the n^2 Taylor coefficients at r0."""
    P = node_coords(nI, nbox, box_origin, box_size)
    NT = P.shape[0]
    lo = (box_origin[0], box_origin[1])
    hi = (box_origin[0] + nbox[0] * box_size, box_origin[1] + nbox[1] * box_size)
    out = [np.empty((NT, NT)) for _ in range(3)]
    for b in range(NT):
        x0, y0, t2, a0, a1, _ = solve_source(medium_n, taylor_at(P[b]), P[b], lo, hi, h0, margin)
        for F, g in zip(out, (t2, a0, a1)):
            F[:, b] = cubic_at(g, x0, y0, h0, P)
    for F in out:
        F += F.T.copy()
        F *= 0.5
    return tuple(out)
