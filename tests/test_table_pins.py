"""CPU pins of the table oracle (oracle.hb_tables): the eikonal and transport
solves of Sec. 2.2-2.3 and the tabulation of Sec. 4.1, checked against what
the mathematics fixes independently of the code:
  * the Taylor recursions against the closed-form constant-gradient tau^2,
    v0, v1 (hb_inputs.media, derived from eq. eikonal / eq. equVs and pinned
    by their own residual tests): the truncation errors fall like r^7, r^5,
    r^3 (P_T = 6, P_B = 4, P_C = 2);
  * a homogeneous medium is an exact fixed point of the discrete sweeps
    (tau = n |r - r0|, v0 = 1/(2 sqrt(pi)), v1 = 0 to rounding);
  * constant gradient: the grid solutions converge to the closed forms at
    the orders the paper asks of them (fifth for tau, third for v0, first
    for v1, Sec. 2.3), measured on the interior over h0 = 1/16, 1/32, 1/64;
  * the local cubic interpolation is exact for cubic polynomials;
  * a whole table (nI = 5) matches the closed-form table within the grid
    error (tighter on the interior nodes), and is symmetric.
"""
import math

import numpy as np
import pytest

import hb_inputs
from oracle import hb_tables as ht

CG = hb_inputs.ConstantGradient(1.0, (0.0, 0.7))


def test_taylor_recursions_match_constant_gradient_closed_form():
    r0 = np.array([0.37, 0.41])
    T, B, C = ht.taylor(hb_inputs.n2_taylor(CG, r0))
    errs = {"tau2": [], "v0": [], "v1": []}
    for rr in (0.01, 0.02):
        x, y = rr * 0.6, rr * 0.8
        t2, a0, a1 = CG.ingredients(r0 + [x, y], r0, 2)
        errs["tau2"].append(abs(ht.poly_eval(sum(T), x, y) - t2))
        errs["v0"].append(abs(ht.poly_eval(sum(B), x, y) - a0))
        errs["v1"].append(abs(ht.poly_eval(sum(C), x, y) - a1))
    for key, order in (("tau2", 7), ("v0", 5), ("v1", 3)):
        e1, e2 = errs[key]
        assert e2 < 1e-6, (key, e2)
        slope = math.log2(e2 / e1)
        assert abs(slope - order) < 0.6, (key, slope)
    # leading terms: T_2 = n0^2 |r|^2, B_0 = 1 / (2 sqrt(pi))
    n0 = float(CG.slowness(r0))
    assert abs(T[2][2, 0] - n0 * n0) < 1e-12 and abs(T[2][0, 2] - n0 * n0) < 1e-12
    assert abs(B[0][0, 0] - 1 / (2 * math.sqrt(math.pi))) < 1e-15


def _solve(med, r0, h0):
    x0, y0, t2, v0, v1, rounds = ht.solve_source(med.slowness, hb_inputs.n2_taylor(med, r0), r0,
                                                 (0.0, 0.0), (1.0, 1.0), h0)
    nx, ny = t2.shape
    X = x0 + h0 * np.arange(nx)[:, None] + 0.0 * np.arange(ny)[None, :]
    Y = y0 + h0 * np.arange(ny)[None, :] + 0.0 * np.arange(nx)[:, None]
    inside = (X > -1e-12) & (X < 1 + 1e-12) & (Y > -1e-12) & (Y < 1 + 1e-12)
    return X, Y, inside, t2, v0, v1


def test_homogeneous_medium_is_an_exact_fixed_point():
    med = hb_inputs.Homogeneous(1.3)
    r0 = (0.4, 0.55)
    X, Y, inside, t2, v0, v1 = _solve(med, r0, 1 / 16)
    exact = 1.3 ** 2 * ((X - r0[0]) ** 2 + (Y - r0[1]) ** 2)
    assert np.abs(t2 - exact)[inside].max() < 1e-12
    assert np.abs(v0 - 1 / (2 * math.sqrt(math.pi))).max() < 1e-13
    assert np.abs(v1).max() < 1e-12


def test_constant_gradient_solves_converge_at_the_stated_orders():
    """Orders measured on the interior square [1/8, 7/8]^2 over h0 = 1/16,
    1/32, 1/64: near the edge of the table region the first-order closure of
    the outer grid layers (three layers, eight cells from the region's edge)
    caps the accuracy of v0 and v1, so edge errors do not fall at these
    orders."""
    r0 = (0.5, 0.5)
    errs = []
    for h0 in (1 / 16, 1 / 32, 1 / 64):
        X, Y, inside, t2, v0, v1 = _solve(CG, r0, h0)
        core = inside & (np.abs(X - 0.5) <= 0.375 + 1e-12) & (np.abs(Y - 0.5) <= 0.375 + 1e-12)
        e2, e0, e1 = CG.ingredients(np.stack([X, Y], -1), np.array(r0), 2)
        errs.append([np.abs(t2 - e2)[core].max(), np.abs(v0 - e0)[core].max(),
                     np.abs(v1 - e1)[core].max()])
        if h0 == 1 / 32:
            assert np.abs(t2 - e2)[inside].max() < 2e-6, errs
            assert np.abs(v0 - e0)[inside].max() < 3e-5, errs
            assert np.abs(v1 - e1)[inside].max() < 3e-3, errs
    for (a2, a0, a1), (b2, b0, b1) in zip(errs, errs[1:]):
        assert math.log2(a2 / b2) > 5.0, errs       # tau (tau^2) fifth order or better
        assert math.log2(a0 / b0) > 3.0, errs       # v0 third order or better
        assert math.log2(a1 / b1) > 1.0, errs       # v1 first order or better


def test_cubic_interpolation_is_exact_for_cubics():
    h0, x0, y0 = 0.1, -0.3, -0.2
    I, J = np.meshgrid(np.arange(20), np.arange(20), indexing="ij")
    f = lambda x, y: 1.5 * x ** 3 - 0.7 * x * x * y + 2 * y ** 3 + x * y - 0.3
    F = f(x0 + I * h0, y0 + J * h0)
    P = np.random.default_rng(3).uniform(0.0, 1.2, size=(40, 2))
    assert np.abs(ht.cubic_at(F, x0, y0, h0, P) - f(P[:, 0], P[:, 1])).max() < 1e-12


def test_table_matches_closed_form_table():
    """Every entry within the grid error of the closed form; on the pairs of
    nodes in the interior square [1/8, 7/8]^2 (away from the first-order
    closure of the outer grid layers) to the interior accuracy of the
    solves, v1 within 5% of its largest value."""
    nI = 5
    t2, v0, v1 = ht.tables(CG.slowness, lambda r: hb_inputs.n2_taylor(CG, r), nI, (1, 1),
                           (0.0, 0.0), 1.0, 1 / 32)
    e2, e0, e1 = hb_inputs.tabulate(CG, 2, nI, (1, 1), (0.0, 0.0), 1.0)
    for F in (t2, v0, v1):
        assert np.array_equal(F, F.T)
    assert np.abs(t2 - e2).max() < 2e-5
    assert np.abs(v0 - e0).max() < 1e-3
    assert np.abs(v1 - e1).max() < 3e-2
    P = ht.node_coords(nI, (1, 1), (0.0, 0.0), 1.0)
    core = np.flatnonzero((np.abs(P[:, 0] - 0.5) <= 0.375) & (np.abs(P[:, 1] - 0.5) <= 0.375))
    assert core.size == 9
    sub = np.ix_(core, core)
    assert np.abs(t2 - e2)[sub].max() < 1e-6
    assert np.abs(v0 - e0)[sub].max() < 1e-5
    assert np.abs(v1 - e1)[sub].max() < 0.05 * np.abs(e1[sub]).max()
    assert np.abs(e1[sub]).max() > 5e-3
