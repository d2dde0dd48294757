"""CPU pins of the inclusion oracle (oracle.inclusion), Sec. 3.2 domain with
inclusion, eq. m_v2v_inclu.

* The self entry of K^{s2s} against adaptive quadrature of minus the segment
  integral of the leading HB term (i/4) H0(omega n |t|).
* The whole operator in a homogeneous medium (where the HB ansatz is the
  exact Green's function) against the series solution of a point source
  scattered by a disc with zero boundary values (Bessel/Hankel expansion
  about the disc centre), converging as the number of segments grows; the
  self entry as printed (without the leading term's factor i) misses it by
  an order of magnitude more.
* K^{s2v} equals the transpose of K^{v2s} times the segment lengths
  (reciprocity of symmetric tables).
* The adjoint against the conjugate transpose of the dense total operator
  assembled column by column on a tiny grid.
"""
import math

import numpy as np
import pytest
from scipy import integrate, special

import hb_inputs
import oracle

inc = oracle.inclusion


@pytest.mark.parametrize("kw", [0.01, 0.05, 0.2])
def test_segment_self_matches_quadrature(kw):
    prob = hb_inputs.configs.c1(16)
    n = 1.3
    w = kw / (prob.omega * n)
    k = prob.omega * n
    opts = dict(limit=400, epsabs=0.0, epsrel=1e-13)
    ij0 = integrate.quad(lambda t: special.j0(k * t), 0.0, w / 2, **opts)[0]
    iy0 = integrate.quad(lambda t: special.y0(k * t), 0.0, w / 2, **opts)[0]
    # -int_{-w/2}^{w/2} (i/4)(J0 + i Y0) dt
    exact = -2.0 * ((1j / 4.0) * ij0 - 0.25 * iy0)
    got = complex(inc.segment_self(prob, np.array([w]), np.array([n]))[0])
    # the closed form drops O((kw)^2 log kw) of the small-argument expansion
    assert abs(got - exact) <= 0.2 * kw ** 2 * abs(exact), (kw, got, exact)


def _disc_case():
    prob = hb_inputs.configs.c1()            # homogeneous, 64^2 cells, omega = 16 pi
    centre, R = np.array([0.5, 0.5]), 0.15
    cell = lambda x, y: int(x / prob.h) + prob.ncell[0] * int(y / prob.h)
    j0 = cell(0.2, 0.25)
    rows = np.array([cell(0.8, 0.7), cell(0.5, 0.85), cell(0.15, 0.6),
                     cell(0.85, 0.3), cell(0.6, 0.12)])
    k = prob.omega
    P0 = prob.centres([j0])[0]
    rho0 = np.linalg.norm(P0 - centre)
    ph0 = math.atan2(P0[1] - centre[1], P0[0] - centre[0])
    ref = []
    for r in prob.centres(rows):
        rho = np.linalg.norm(r - centre)
        ph = math.atan2(r[1] - centre[1], r[0] - centre[0])
        m = np.arange(-int(k * R + 40), int(k * R + 41))
        c = -(1j / 4) * special.jv(m, k * R) * special.hankel1(m, k * rho0) / special.hankel1(m, k * R)
        sca = np.sum(c * special.hankel1(m, k * rho) * np.exp(1j * m * (ph - ph0)))
        ref.append((1j / 4) * special.hankel1(0, k * np.linalg.norm(r - P0)) + sca)
    s = np.zeros(prob.Nv, complex)
    s[j0] = 1.0 / prob.h ** 2                 # I = e_j0: a unit point source
    return prob, centre, R, rows, s, np.array(ref)


def test_disc_scattering_series(monkeypatch):
    prob, centre, R, rows, s, ref = _disc_case()
    err = {}
    for ns in (512, 1024):
        u = inc.apply(prob, hb_inputs.circle(prob, centre, R, ns), s, rows)
        err[ns] = np.abs(u - ref).max() / np.abs(ref).max()
    assert err[512] < 2e-3 and err[1024] < 1e-3, err
    assert err[1024] < 0.7 * err[512], err
    # the self entry as printed, without the factor i of (i/4) H0
    printed = lambda p, w, n, f=inc.segment_self: f(p, w, n) / 1j
    monkeypatch.setattr(inc, "segment_self", printed)
    u = inc.apply(prob, hb_inputs.circle(prob, centre, R, 512), s, rows)
    assert np.abs(u - ref).max() / np.abs(ref).max() > 10 * err[512]


def test_s2v_is_weighted_transpose_of_v2s():
    prob = hb_inputs.configs.c2(32, nbox=2)
    cv = hb_inputs.circle(prob, (0.4, 0.55), 0.12, 40)
    rows = np.arange(0, prob.Nv, 7)
    A = inc.s2v(prob, cv, rows)
    B = inc.v2s(prob, cv, rows).T * cv.w[None, :]
    assert np.abs(A - B).max() <= 1e-12 * np.abs(B).max()


def test_adjoint_is_conjugate_transpose():
    prob = hb_inputs.configs.c2(16, nbox=2)
    cv = hb_inputs.circle(prob, (0.45, 0.5), 0.2, 24)
    E = np.eye(prob.Nv)
    T = inc.apply(prob, cv, E)                # columns T e_j
    TH = inc.apply_adjoint(prob, cv, E)
    assert np.abs(TH - T.conj().T).max() <= 1e-12 * np.abs(T).max()
