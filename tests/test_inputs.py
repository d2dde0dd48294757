"""Pins of the seeded input generators: the closed-form media satisfy the
eikonal equation (eq. eikonal) and the transport recurrence (eq. equVs) by
finite differences, the source value of v0 is eq. initialv0, and the table
layout is the documented one."""
import json
import math
import os

import numpy as np
import pytest

import hb_inputs
from hb_inputs.media import ConstantGradient, GaussianBump, Homogeneous, Sinusoid3D

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                     "paper_media.json")))


def _fd(fun, r, d, hh=1e-3):
    """4th-order central differences: (value, gradient, laplacian)."""
    f0 = fun(r)
    g = np.zeros(d)
    lap = 0.0
    for ax in range(d):
        e = np.zeros(d)
        e[ax] = hh
        fp, fm, fpp, fmm = fun(r + e), fun(r - e), fun(r + 2 * e), fun(r - 2 * e)
        g[ax] = (8 * (fp - fm) - (fpp - fmm)) / (12 * hh)
        lap += (-fpp + 16 * fp - 30 * f0 + 16 * fm - fmm) / (12 * hh * hh)
    return f0, g, lap


@pytest.mark.parametrize("key", ["constant_gradient_2d", "constant_gradient_3d"])
def test_constant_gradient_solves_eikonal_and_transport(key):
    cg = GOLDEN[key]
    d = len(cg["G0"])
    med = ConstantGradient(cg["c0"], tuple(cg["G0"]))
    rng = np.random.default_rng(5)
    lo, hi = cg["domain"][0]
    for _ in range(4):
        r0 = rng.uniform(lo + 0.1, hi - 0.1, d)
        r = rng.uniform(lo + 0.05, hi - 0.05, d)
        if np.linalg.norm(r - r0) < 0.1:
            continue
        comp = lambda k: (lambda x: med.ingredients(x[None], r0[None], d)[k][0])
        t2, gt2, lt2 = _fd(comp(0), r, d)
        v0, gv0, lv0 = _fd(comp(1), r, d)
        v1, gv1, lv1 = _fd(comp(2), r, d)
        n = med.slowness(r[None])[0]
        # eq. eikonal: |grad tau^2|^2 = 4 tau^2 n^2
        assert abs(gt2 @ gt2 - 4 * t2 * n * n) <= 1e-8 * (4 * t2 * n * n)
        # eq. equVs with 4 tau n^2 d/dtau = 2 grad(tau^2) . grad
        res0 = 2 * gt2 @ gv0 + v0 * (lt2 - 2 * d * n * n)
        assert abs(res0) <= 1e-8 * abs(v0 * lt2)
        res1 = 2 * gt2 @ gv1 + v1 * (lt2 + 2 * n * n * (2 - d)) - lv0
        assert abs(res1) <= 1e-6 * abs(lv0)


@pytest.mark.parametrize("d,n0", [(2, 1.0), (2, 1.7), (3, 1.0), (3, 2.0)])
def test_v0_source_value(d, n0):
    """v0(r0, r0) = n0^(d-2) / (2 pi^((d-1)/2)) (eq. initialv0)."""
    r0 = np.full((1, d), 0.3)
    for med in (Homogeneous(n0), ConstantGradient(1.0 / n0, (0.0, 0.4, 0.0)[:d] if d == 3 else (0.0, 0.4))):
        ns = med.slowness(r0)[0]
        ref = {2: 1 / (2 * math.sqrt(math.pi)), 3: ns / (2 * math.pi)}[d]
        _, v0, _ = med.ingredients(r0, r0, d)
        assert abs(v0[0] - ref) < 1e-14


def test_stand_in_is_reciprocal_and_smooth():
    rng = np.random.default_rng(1)
    for med, d in ((GaussianBump(), 2), (Sinusoid3D(), 3)):
        R, R0 = rng.uniform(0, 1, (50, d)), rng.uniform(0, 1, (50, d))
        a = med.ingredients(R, R0, d)
        b = med.ingredients(R0, R, d)
        for x, y in zip(a, b):
            assert np.max(np.abs(x - y)) <= 1e-14 * max(1.0, np.max(np.abs(x)))


def test_table_layout_and_symmetry():
    p = hb_inputs.configs.c2(32, nbox=2)
    assert p.NT == 4 * 64 and p.tau2.shape == (256, 256)
    P = hb_inputs.node_coords(2, 8, (2, 2), (0.0, 0.0), 0.5)
    # node 0 of box 1 (bx=1, by=0) sits in [0.5, 1] x [0, 0.5]
    assert 0.5 < P[64, 0] < 1.0 and 0.0 < P[64, 1] < 0.5
    # a = k1 + nI*k2: node 1 differs from node 0 in x only
    assert P[1, 1] == P[0, 1] and P[1, 0] < P[0, 0]
    for F in (p.tau2, p.v0, p.v1):
        assert np.array_equal(F, F.T)
    i = 5
    assert p.tau2[i, i] == 0.0


def test_configs_shapes():
    p1 = hb_inputs.configs.c1()
    assert p1.Nv == 4096 and p1.NT == 9 and abs(p1.omega - 16 * math.pi) < 1e-12
    p5 = hb_inputs.configs.c5(8, nI=3)
    assert p5.Nv == 512 and p5.dim == 3
    probs = hb_inputs.configs.c3(nprob=3, sides=(16, 32), max_rhs=4)
    assert len(probs) == 3 and all(1 <= n <= 4 for _, n, _ in probs)
