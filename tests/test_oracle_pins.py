"""Pins of the FP64 oracle against things that do not come from it:
closed-form Green's functions, mpmath Hankel functions, exact polynomial
interpolation, independent brute-force cell quadratures and explicit loops.
Each pin is chosen so a plausible slip in the oracle (dropped term, wrong
sign, wrong index, transposed operand, wrong h^d scaling) fails it."""
import json
import math
import os

import mpmath
import numpy as np
import pytest
from scipy import integrate, special
from scipy.interpolate import BarycentricInterpolator

import hb_inputs
import oracle
from hb_inputs.media import ConstantGradient, Homogeneous
from hb_inputs.problem import HBProblem, make_problem

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                     "paper_media.json")))


def f_general(q, omega, tau):
    """eq. termf evaluated with mpmath (arbitrary order, own Hankel)."""
    tau = mpmath.mpf(tau)
    return complex(1j * mpmath.sqrt(mpmath.pi) / 2 * mpmath.exp(1j * q * mpmath.pi)
                   * (2 * tau / omega) ** q * mpmath.hankel1(q, omega * tau))


@pytest.mark.parametrize("d,qs", [(2, (0, 1)), (3, (-0.5, 0.5))])
@pytest.mark.parametrize("omega,tau", [(50.0, 0.37), (16 * math.pi, 1.0 / 64),
                                       (804.2, 1.8), (3.0, 0.2)])
def test_hb_terms_match_general_formula(d, qs, omega, tau):
    fa, fb = oracle.hb_terms(d, omega, np.array([tau]))
    for got, q in zip((fa[0], fb[0]), qs):
        ref = f_general(mpmath.mpf(q), omega, tau)
        assert abs(got - ref) <= 1e-13 * abs(ref)


def test_c1_entries_are_free_space_green_function():
    """Homogeneous n=1: K_ij = (i/4) H0(omega |r_i - r_j|) (Sec. 5.1.1); the
    nI = 3 table reproduces tau^2 = |r - r0|^2 exactly."""
    p = hb_inputs.configs.c1()
    rng = np.random.default_rng(7)
    rows = rng.choice(p.Nv, 40, replace=False)
    cols = rng.choice(p.Nv, 50, replace=False)
    K = oracle.entries(p, rows, cols)
    P, Q = p.centres(rows), p.centres(cols)
    for a in range(0, 40, 3):
        for b in range(0, 50, 7):
            if rows[a] == cols[b]:
                continue
            r = float(np.linalg.norm(P[a] - Q[b]))
            ref = complex(0.25j * mpmath.hankel1(0, p.omega * r))
            assert abs(K[a, b] - ref) <= 1e-12 * abs(ref)


def test_3d_homogeneous_entries():
    """3D constant media: g = exp(i omega n0 R) / (4 pi R) (Sec. 5.1.2)."""
    n0 = 1.5
    p = make_problem(Homogeneous(n0), 3, (6, 6, 6), 9.0, nI=3)
    rows = np.arange(0, p.Nv, 5)
    cols = np.arange(1, p.Nv, 7)
    K = oracle.entries(p, rows, cols)
    R = np.linalg.norm(p.centres(rows)[:, None] - p.centres(cols)[None], axis=-1)
    off = rows[:, None] != cols[None, :]
    ref = np.exp(1j * p.omega * n0 * R) / (4 * math.pi * np.where(off, R, 1.0))
    assert np.max(np.abs(K - ref)[off] / np.abs(ref)[off]) < 1e-12


def _poly_problem(dim, nI, nbox, rng):
    """Tables filled with a non-symmetric polynomial of degree < nI per
    coordinate in each argument; interpolation must reproduce it."""
    cx = rng.standard_normal((dim, nI))
    cy = rng.standard_normal((dim, nI))

    def poly(R, R0):
        out = np.ones(R.shape[:-1])
        for ax in range(dim):
            out = out * np.polynomial.polynomial.polyval(R[..., ax], cx[ax]) \
                * np.polynomial.polynomial.polyval(R0[..., ax], cy[ax] + 0.1 * ax)
        return out

    box_size = 1.0 / max(nbox)
    P = hb_inputs.node_coords(dim, nI, nbox, (0.0,) * dim, box_size)
    F = poly(P[:, None, :], P[None, :, :])
    ncell = (8,) * dim
    prob = HBProblem(dim=dim, ncell=ncell, origin=(0.0,) * dim, h=1 / 8,
                     omega=1.0, nterms=2, nI=nI, nbox=nbox,
                     box_origin=(0.0,) * dim, box_size=box_size, tau2=F,
                     v0=F, v1=F, slowness=np.ones(8 ** dim))
    return prob, poly


@pytest.mark.parametrize("dim,nI,nbox", [(2, 5, (1, 1)), (2, 4, (2, 3)),
                                         (3, 3, (1, 1, 1)), (3, 3, (2, 1, 2))])
def test_interpolation_exact_for_polynomials(dim, nI, nbox):
    rng = np.random.default_rng(dim * 100 + nI)
    prob, poly = _poly_problem(dim, nI, nbox, rng)
    ext = np.array(nbox[:dim]) / max(nbox)
    Pr = rng.uniform(0, 1, (30, dim)) * ext
    Pc = rng.uniform(0, 1, (25, dim)) * ext
    got = oracle.interpolate(prob, prob.tau2, Pr, Pc)
    ref = poly(Pr[:, None, :], Pc[None, :, :])
    assert np.max(np.abs(got - ref)) <= 1e-10 * np.max(np.abs(ref))


def _brute_self_2d(h, n, omega):
    """(1/h^2) int_cell (i/4) H0(omega n |r0|) dr0 over 4 triangles with apex
    at the centre, coordinates x in [0,h/2], y = u x: dA = x dx du."""
    def inner(u, part):
        s = math.sqrt(1.0 + u * u)
        fn = special.j0 if part == 0 else special.y0
        return integrate.quad(lambda x: fn(omega * n * x * s) * x, 0.0, h / 2,
                              epsabs=0, epsrel=1e-13, limit=200)[0]
    re = integrate.quad(lambda u: inner(u, 0), -1, 1, epsabs=0, epsrel=1e-13)[0]
    im = integrate.quad(lambda u: inner(u, 1), -1, 1, epsabs=0, epsrel=1e-13)[0]
    return 0.25j * 4.0 * (re + 1j * im) / h ** 2


def _brute_self_3d(h, n, omega, m=24):
    """(1/h^3) int_cube exp(i omega n R)/(4 pi R): 6 pyramids with apex at
    the centre, z in [0,h/2], x = u z, y = v z, dV = z^2 dz du dv; the
    integrand z exp(i omega n z s)/(4 pi s) is smooth, so tensor
    Gauss-Legendre converges fast."""
    t, w = np.polynomial.legendre.leggauss(m)
    z = (t + 1) * h / 4
    wz = w * h / 4
    U, V, Z = np.meshgrid(t, t, z, indexing="ij")
    W = w[:, None, None] * w[None, :, None] * wz[None, None, :]
    s = np.sqrt(1 + U ** 2 + V ** 2)
    val = np.sum(W * Z * np.exp(1j * omega * n * Z * s) / (4 * math.pi * s))
    return 6.0 * val / h ** 3


@pytest.mark.parametrize("h,n,omega", [(1 / 64, 1.0, 16 * math.pi),
                                       (1 / 1024, 1.3, 256 * math.pi),
                                       (0.05, 2.0, 30.0)])
def test_self_term_2d_matches_bruteforce(h, n, omega):
    p = make_problem(Homogeneous(n), 2, (4, 4), omega, nI=3)
    p.h = h
    got = oracle.self_term(p, n)
    ref = _brute_self_2d(h, n, omega)
    assert abs(got - ref) <= 1e-10 * abs(ref)


@pytest.mark.parametrize("h,n,omega", [(1 / 64, 1.0, 16 * math.pi),
                                       (0.1, 1.2, 40.0)])
def test_self_term_3d_matches_bruteforce(h, n, omega):
    p = make_problem(Homogeneous(n), 3, (2, 2, 2), omega, nI=3)
    p.h = h
    got = oracle.self_term(p, n)
    ref = _brute_self_3d(h, n, omega)
    assert abs(got - ref) <= 1e-10 * abs(ref)


def test_apply_point_source_gives_column():
    """s = delta_j / h^d (Sec. 3.1, point source) => u = K[:, j]."""
    p = hb_inputs.configs.c1(16)
    j = 37
    s = np.zeros(p.Nv, complex)
    s[j] = 1.0 / p.h ** 2
    u = oracle.apply(p, s)
    P = p.centres()
    for i in range(0, p.Nv, 5):
        if i == j:
            ref = _brute_self_2d(p.h, 1.0, p.omega)
        else:
            r = float(np.linalg.norm(P[i] - P[j]))
            ref = complex(0.25j * mpmath.hankel1(0, p.omega * r))
        assert abs(u[i] - ref) <= 1e-11 * abs(ref)


def test_apply_matches_explicit_loops_constant_gradient():
    """Tiny 2D constant-gradient problem (non-trivial v0, v1, n): explicit
    double loops over eq. chebinterp with scipy's barycentric Lagrange basis,
    mpmath Hankel functions in eq. termf, the brute-force self term and
    u_i = sum_j K_ij h^2 s_j."""
    cg = GOLDEN["constant_gradient_2d"]
    med = ConstantGradient(cg["c0"], tuple(cg["G0"]))
    p = make_problem(med, 2, (4, 4), 23.0, nI=4)
    rng = np.random.default_rng(3)
    s = rng.standard_normal(p.Nv) + 1j * rng.standard_normal(p.Nv)
    nodes = 0.5 * (1 + np.cos((2 * np.arange(p.nI) + 1) * math.pi / (2 * p.nI)))
    basis = [BarycentricInterpolator(nodes, np.eye(p.nI)[k]) for k in range(p.nI)]
    P = p.centres()

    def T(r):
        lx = [float(b(r[0])) for b in basis]
        ly = [float(b(r[1])) for b in basis]
        return [lx[k1] * ly[k2] for k2 in range(p.nI) for k1 in range(p.nI)]

    Ts = [T(P[i]) for i in range(p.Nv)]
    u_ref = []
    for i in range(p.Nv):
        acc = 0j
        for j in range(p.Nv):
            if i == j:
                kij = _brute_self_2d(p.h, p.slowness[i], p.omega)
            else:
                vals = []
                for F in (p.tau2, p.v0, p.v1):
                    v = 0.0
                    for a in range(p.NT):
                        for b in range(p.NT):
                            v += Ts[i][a] * F[a, b] * Ts[j][b]
                    vals.append(v)
                tau = math.sqrt(max(vals[0], 0.0))
                kij = vals[1] * f_general(0, p.omega, tau) + vals[2] * f_general(1, p.omega, tau)
            acc += kij * p.h ** 2 * s[j]
        u_ref.append(acc)
    u = oracle.apply(p, s)
    u_ref = np.array(u_ref)
    assert np.linalg.norm(u - u_ref) <= 1e-11 * np.linalg.norm(u_ref)


def test_reciprocity_symmetric_tables():
    """Symmetric tables => K = K^T (eq. m_v2v with g(r,r0) = g(r0,r))."""
    p = hb_inputs.configs.c2(16, nbox=2)
    K = oracle.dense(p)
    assert np.max(np.abs(K - K.T)) <= 1e-12 * np.max(np.abs(K))


def test_adjoint_dot_product():
    cg = GOLDEN["constant_gradient_2d"]
    p = make_problem(ConstantGradient(cg["c0"], tuple(cg["G0"])), 2, (12, 12), 40.0, nI=5)
    x = hb_inputs.complex_normal(p.Nv, [9, 1])
    y = hb_inputs.complex_normal(p.Nv, [9, 2])
    lhs = np.vdot(y, oracle.apply(p, x))
    rhs = np.vdot(oracle.apply_adjoint(p, y), x)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_3d_constant_gradient_against_holford_exact():
    """Two-term HB with the tabulated v0, v1 against Holford's exact Green's
    function (Sec. 5.1.2): the one-term error falls like 1/omega and the
    two-term error like 1/omega^2 (eq. inferror, d = 3)."""
    cg = GOLDEN["constant_gradient_3d"]
    a, c = cg["holford_a"], cg["holford_c"]
    med = ConstantGradient(cg["c0"], tuple(cg["G0"]))
    rng = np.random.default_rng(11)
    R = rng.uniform(0, 0.52, (150, 3))
    r0 = np.array([0.26, 0.21, 0.3])
    errs = {}
    for omega in (16 * math.pi, 64 * math.pi):
        t2, v0, v1 = med.ingredients(R, r0[None], 3)
        f0, f1 = oracle.hb_terms(3, omega, np.sqrt(t2))
        Rr = np.linalg.norm(R - r0, axis=1)
        Rp = np.sqrt((R[:, 0] - r0[0]) ** 2 + (R[:, 1] + r0[1] - 2 * c) ** 2 + (R[:, 2] - r0[2]) ** 2)
        ex = np.sqrt(np.abs(R[:, 1] - c) * abs(r0[1] - c)) / (2 * math.pi * Rr * Rp) * \
            np.exp(2j * np.sqrt(a * a * omega ** 2 - 0.25) * np.arctanh(Rr / Rp))
        e1 = np.max(np.abs(v0 * f0 - ex) / np.abs(ex))
        e2 = np.max(np.abs(v0 * f0 + v1 * f1 - ex) / np.abs(ex))
        errs[omega] = (e1, e2)
    (a1, a2), (b1, b2) = errs[16 * math.pi], errs[64 * math.pi]
    assert a2 < 1e-2 * a1 and b2 < 1e-3 * b1
    assert 3.0 < a1 / b1 < 5.0          # ~ omega^-1
    assert 12.0 < a2 / b2 < 20.0        # ~ omega^-2
