"""Media: slowness n(r) and the HB ingredients tau^2, v0, v1 for a source r0.

Every medium exposes
  * ``slowness(P)``            n at points P (shape (..., d)),
  * ``ingredients(R, R0, d)``  (tau^2, v0, v1) for paired observation points R
                               and source points R0 (same leading shape).

The HB coefficients follow the normalisation of the paper's ansatz (eq. hb
with the source value of v0 in eq. initialv0): v0(r0, r0) = n0^(d-2) /
(2 pi^((d-1)/2)).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import mpmath
import numpy as np

_GL16_T, _GL16_W = np.polynomial.legendre.leggauss(16)
_GL16_T = 0.5 * (_GL16_T + 1.0)      # nodes on [0, 1]
_GL16_W = 0.5 * _GL16_W


def _v0_source(n0, d):
    """Source value of v0 (eq. initialv0)."""
    return n0 ** (d - 2) / (2.0 * math.pi ** ((d - 1) / 2.0))


@dataclass(frozen=True)
class Homogeneous:
    """Constant slowness n0: tau = n0 |r - r0|, v0 = source value, v1 = 0
    (Sec. 5.1, constant media: the HB ansatz is then the exact Green's
    function)."""
    n0: float = 1.0
    name: str = "homogeneous"

    def slowness(self, P):
        P = np.asarray(P, dtype=np.float64)
        return np.full(P.shape[:-1], self.n0)

    def slowness_mp(self, x, y):
        return mpmath.mpf(self.n0)

    def ingredients(self, R, R0, d):
        R = np.asarray(R, np.float64)
        R0 = np.asarray(R0, np.float64)
        r2 = np.sum((R - R0) ** 2, axis=-1)
        tau2 = self.n0 ** 2 * r2
        v0 = np.full_like(tau2, _v0_source(self.n0, d))
        v1 = np.zeros_like(tau2)
        return tau2, v0, v1


def _acosh1p(x):
    """arccosh(1 + x) without cancellation for small x >= 0."""
    return np.log1p(x + np.sqrt(x * (x + 2.0)))


def _sigma_over_sinh(s):
    s = np.asarray(s, np.float64)
    out = np.ones_like(s)
    big = s > 1e-4
    out[big] = s[big] / np.sinh(s[big])
    sm = ~big
    out[sm] = 1.0 - s[sm] ** 2 / 6.0 + 7.0 * s[sm] ** 4 / 360.0
    return out


# Taylor coefficients (in s^2) of q(s) = p' + p^2 + coth(s) p with
# p = (1/s - coth s)/2, valid for |s| < pi; used below 0.3.
_Q_SERIES = (-1.0 / 3.0, 1.0 / 60.0, -1.0 / 378.0, 1.0 / 2700.0,
             -1.0 / 20790.0, 691.0 / 116093250.0)


def _q_radial(s):
    """q(s) = (phi'' + coth(s) phi') / phi for phi = sqrt(s / sinh s).

    With p = (ln phi)' = (1/s - coth s)/2 one has phi'/phi = p and
    phi''/phi = p' + p^2.
    """
    s = np.asarray(s, np.float64)
    out = np.empty_like(s)
    sm = s < 0.3
    s2 = s[sm] ** 2
    acc = np.zeros_like(s2)
    for c in reversed(_Q_SERIES):
        acc = acc * s2 + c
    out[sm] = acc
    b = s[~sm]
    coth = 1.0 / np.tanh(b)
    p = 0.5 * (1.0 / b - coth)
    dp = 0.5 * (-1.0 / b ** 2 + 1.0 / np.sinh(b) ** 2)
    out[~sm] = dp + p * p + coth * p
    return out


_GL32_T, _GL32_W = np.polynomial.legendre.leggauss(32)
_GL32_T = 0.5 * (_GL32_T + 1.0)
_GL32_W = 0.5 * _GL32_W


@dataclass(frozen=True)
class ConstantGradient:
    """Velocity c(r) = c0 + G.r (slowness n = 1/c), the constant-gradient
    medium of Sec. 5.1 (2D) and Sec. 5.1.2 (3D).

    tau has the closed form (1/|G|) arccosh(1 + |G|^2 R^2 / (2 c(r) c(r0))).
    The HB coefficients are functions of sigma = |G| tau:
      2D: v0 = (1/(2 sqrt(pi))) sqrt(sigma / sinh sigma),
          v1 = v0 * (|G|^2/4) (1/sigma) int_0^sigma q(s) ds,
      3D: v0 = sqrt(n n0)/(2 pi) * sigma / sinh sigma,  v1 = -(|G|^2/16) v0.
    These solve the transport recurrence (eq. equVs) with the source value of
    eq. initialv0; the tests check both by finite differences.
    """
    c0: float
    G: tuple
    name: str = "constant-gradient"

    def velocity(self, P):
        P = np.asarray(P, np.float64)
        G = np.asarray(self.G, np.float64)[: P.shape[-1]]
        return self.c0 + P @ G

    def slowness(self, P):
        return 1.0 / self.velocity(P)

    def slowness_mp(self, x, y):
        return 1 / (self.c0 + self.G[0] * x + self.G[1] * y)

    def tau(self, R, R0):
        R = np.asarray(R, np.float64)
        R0 = np.asarray(R0, np.float64)
        g = float(np.linalg.norm(self.G))
        r2 = np.sum((R - R0) ** 2, axis=-1)
        x = 0.5 * g * g * r2 / (self.velocity(R) * self.velocity(R0))
        return _acosh1p(x) / g

    def ingredients(self, R, R0, d):
        g = float(np.linalg.norm(self.G))
        tau = self.tau(R, R0)
        sigma = g * tau
        if d == 2:
            v0 = _v0_source(1.0, 2) * np.sqrt(_sigma_over_sinh(sigma))
            # (1/sigma) int_0^sigma q = int_0^1 q(sigma t) dt
            qs = _q_radial(sigma[..., None] * _GL32_T)
            w = (g * g / 4.0) * np.sum(qs * _GL32_W, axis=-1)
            v1 = v0 * w
        elif d == 3:
            n = self.slowness(R)
            n0 = self.slowness(R0)
            v0 = np.sqrt(n * n0) / (2.0 * math.pi) * _sigma_over_sinh(sigma)
            v1 = -(g * g / 16.0) * v0
        else:
            raise ValueError("dimension must be 2 or 3")
        return tau * tau, v0, v1


class _StraightRay:
    """Smooth reciprocal stand-in for media without a closed form:
    tau = |r - r0| * mean of n along the segment (16-point Gauss-Legendre),
    v0 = sqrt(n n0)^(d-2)/(2 pi^((d-1)/2)) (the source value, made
    reciprocal), v1 = 0.  It is symmetric in r <-> r0 and smooth, but it is
    not a solution of the eikonal/transport equations."""

    def ingredients(self, R, R0, d):
        R = np.asarray(R, np.float64)
        R0 = np.asarray(R0, np.float64)
        D = R - R0
        dist = np.sqrt(np.sum(D * D, axis=-1))
        acc = np.zeros(dist.shape)
        for t, w in zip(_GL16_T, _GL16_W):
            acc += w * self.slowness(R0 + t * D)
        tau = dist * acc
        if d == 2:
            v0 = np.full_like(tau, _v0_source(1.0, 2))
        else:
            v0 = np.sqrt(self.slowness(R) * self.slowness(R0)) / (2.0 * math.pi)
        return tau * tau, v0, np.zeros_like(tau)


@dataclass(frozen=True)
class GaussianBump(_StraightRay):
    """n(r) = 1 + amp * exp(-|r - centre|^2 / (2 width^2)) (2D)."""
    amp: float = 0.3
    centre: tuple = (0.5, 0.5)
    width: float = 0.1
    name: str = "gaussian-bump"

    def slowness(self, P):
        P = np.asarray(P, np.float64)
        c = np.asarray(self.centre, np.float64)
        r2 = np.sum((P - c) ** 2, axis=-1)
        return 1.0 + self.amp * np.exp(-r2 / (2.0 * self.width ** 2))

    def slowness_mp(self, x, y):
        r2 = (x - self.centre[0]) ** 2 + (y - self.centre[1]) ** 2
        return 1 + self.amp * mpmath.exp(-r2 / (2 * mpmath.mpf(self.width) ** 2))


@dataclass(frozen=True)
class Sinusoid2D(_StraightRay):
    """n(x, y) = 1 / (1 + amp sin(pi (x + 0.05)) sin(pi y / 2)): the 2D
    sinusoidal medium of the paper's numerical results (Sec. 5.1.1), whose
    phase and HB coefficients have no closed form; its tables come from the
    eikonal and transport solves (hbi_tabulate), the straight-ray stand-in
    serving only as a placeholder."""
    amp: float = 0.2
    name: str = "sinusoid-2d"

    def slowness(self, P):
        P = np.asarray(P, np.float64)
        return 1.0 / (1.0 + self.amp * np.sin(math.pi * (P[..., 0] + 0.05)) *
                      np.sin(0.5 * math.pi * P[..., 1]))

    def slowness_mp(self, x, y):
        return 1 / (1 + self.amp * mpmath.sin(mpmath.pi * (x + mpmath.mpf("0.05"))) *
                    mpmath.sin(mpmath.pi * y / 2))


def n2_taylor(medium, r0, order=4, dps=40):
    """Taylor coefficients of n(r)^2 about r0 (2D): S[i, j] is the coefficient
    of (x - x0)^i (y - y0)^j, i + j <= order, from the medium's own
    high-precision form (mpmath differentiation)."""
    mpmath.mp.dps = dps
    x0, y0 = (mpmath.mpf(float(c)) for c in r0[:2])
    f = lambda x, y: medium.slowness_mp(x, y) ** 2
    S = np.zeros((order + 1, order + 1))
    for i in range(order + 1):
        for j in range(order + 1 - i):
            v = mpmath.diff(f, (x0, y0), (i, j))
            S[i, j] = float(v) / (math.factorial(i) * math.factorial(j))
    return S


@dataclass(frozen=True)
class Sinusoid3D(_StraightRay):
    """n(r) = 1 + amp * sin(2 pi x) sin(2 pi y) sin(2 pi z) (3D)."""
    amp: float = 0.2
    name: str = "sinusoid-3d"

    def slowness(self, P):
        P = np.asarray(P, np.float64)
        s = np.sin(2.0 * math.pi * P)
        return 1.0 + self.amp * s[..., 0] * s[..., 1] * s[..., 2]


def medium_grid(medium, lo, hi, spacing, pad=4):
    """n^2 of a 2D medium on a regular grid covering [lo - pad spacing,
    hi + pad spacing] per axis: returns (n2[i, j], origin, spacing)."""
    nx = int(math.ceil((hi[0] - lo[0]) / spacing)) + 2 * pad + 1
    ny = int(math.ceil((hi[1] - lo[1]) / spacing)) + 2 * pad + 1
    origin = (lo[0] - pad * spacing, lo[1] - pad * spacing)
    X = origin[0] + spacing * np.arange(nx)[:, None] + 0.0 * np.arange(ny)[None, :]
    Y = origin[1] + spacing * np.arange(ny)[None, :] + 0.0 * np.arange(nx)[:, None]
    n = medium.slowness(np.stack([X, Y], axis=-1))
    return n * n, origin, spacing


def taylor_at(medium, P, order=4):
    """(len(P), order + 1, order + 1) Taylor coefficients of n^2 about the
    points P (n2_taylor at each)."""
    return np.stack([n2_taylor(medium, p, order) for p in np.atleast_2d(P)])
