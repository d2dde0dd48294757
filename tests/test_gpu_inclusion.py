"""GPU parity of the curve inclusion (Sec. 3.2, eq. m_v2v_inclu) against the
FP64 oracle (oracle.inclusion), through the C ABI.

G[j, i] = g(r_j, r^s_i), which gives K^{v2s} = G^T and K^{s2v} = G W, is a
single butterfly over the cell tree and a tree of the segments (Sec. 4.2,
L = min(L_v, L_s) levels), compressed at a hundredth of the build tolerance;
HBI_INCLUSION_DENSE=1 keeps it dense for comparison.

Tolerances: dense, the inclusion term differs from the oracle by rounding in
the entries (~1e-13), amplified by the condition number of K^{s2s} (40-60
here) in the inverse: 1e-10 relative in FP64, 2e-5 in FP32.  As a butterfly
at 1e-9 (FP64) the compression error, amplified the same way, stays below
1e-8; in FP32 (1e-7) the rounding of the factors dominates as in the dense
case.  The total operator adds the volume factors' tolerance (1e-6 at tol
1e-7, FP64; 1e-4 at 1e-5, FP32).
"""
import dataclasses
import math

import numpy as np
import pytest

import hb_inputs
import oracle
from _hbi_util import ensure_built, requires_gpu

pytestmark = [pytest.mark.gpu, requires_gpu]
inc = oracle.inclusion


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


@pytest.fixture(scope="module")
def torch_mod():
    ensure_built()
    import torch
    return torch


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


CASES = {
    "homogeneous-64": lambda: (hb_inputs.configs.c1(), (0.5, 0.5), 0.15, 256),
    "bump-64": lambda: (hb_inputs.configs.c2(64, nbox=4), (0.35, 0.6), 0.12, 200),
}


def _inclusion_term(prob, curve, S):
    I = S * prob.h ** 2
    return inc.s2v(prob, curve) @ np.linalg.solve(inc.s2s(prob, curve), inc.v2s(prob, curve) @ I)


@pytest.mark.parametrize("mode", ["butterfly", "dense"])
@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("prec,tol,b_inc,b_tot", [("f64", 1e-7, 1e-10, 1e-6),
                                                  ("f32", 1e-5, 2e-5, 1e-4)])
def test_inclusion_matches_oracle(torch_mod, monkeypatch, mode, name, prec, tol, b_inc, b_tot):
    torch = torch_mod
    import paper_2210_02698_amd as hbi
    if mode == "dense":
        monkeypatch.setenv("HBI_INCLUSION_DENSE", "1")
    elif prec == "f64":
        b_inc = 1e-8
    prob, centre, R, ns = CASES[name]()
    curve = hb_inputs.circle(prob, centre, R, ns)
    say(f"inclusion {name} {prec} {mode} ns={ns}")
    dt = torch.complex128 if prec == "f64" else torch.complex64
    s_h = hb_inputs.complex_normal((prob.Nv, 2), [31, ns])
    S = torch.from_numpy(np.asfortranarray(s_h)).to("cuda:0").to(dt)
    plain = hbi.Operator(prob, device=0).build(tol=tol, prec=prec)
    op = hbi.Operator(prob, device=0).set_inclusion(curve).build(tol=tol, prec=prec)
    info = op.info()
    assert info["inclusion_ns"] == ns
    # 2^L segment leaves of at most 8 segments, L <= L_v
    assert info["inclusion_bf_levels"] == (-1 if mode == "dense" else
                                           min(info["L_v"], math.ceil(math.log2(ns / 8))))
    u = op.apply(S[:, 0].contiguous()).cpu().numpy().astype(np.complex128)
    u0 = plain.apply(S[:, 0].contiguous()).cpu().numpy().astype(np.complex128)
    ref_inc = _inclusion_term(prob, curve, s_h[:, 0])
    e_inc = rel(u - u0, ref_inc)
    ref = oracle.apply(prob, s_h[:, 0]) + ref_inc
    e_tot = rel(u, ref)
    say(f"  inclusion term {e_inc:.2e}, total {e_tot:.2e}")
    assert e_inc < b_inc, e_inc
    assert e_tot < b_tot, e_tot
    # two right-hand sides in one call: each column as alone (the volume part
    # runs on the MFMA tiles, the inclusion term per column)
    U = op.apply(S).cpu().numpy().astype(np.complex128)
    assert rel(U[:, 0], u) < (1e-12 if prec == "f64" else 2e-5)
    U0 = plain.apply(S).cpu().numpy().astype(np.complex128)
    assert rel(U[:, 1] - U0[:, 1], _inclusion_term(prob, curve, s_h[:, 1])) < b_inc
    plain.close()
    op.close()


def test_inclusion_adjoint(torch_mod):
    """The conjugate transpose: its inclusion term against the oracle's, and
    the dot-product identity of the total operator."""
    torch = torch_mod
    import paper_2210_02698_amd as hbi
    prob, centre, R, ns = CASES["bump-64"]()
    curve = hb_inputs.circle(prob, centre, R, ns)
    say("inclusion adjoint bump-64 f64")
    plain = hbi.Operator(prob, device=0).build(tol=1e-7)
    op = hbi.Operator(prob, device=0).set_inclusion(curve).build(tol=1e-7)
    x = hb_inputs.complex_normal(prob.Nv, [32, 0])
    y = hb_inputs.complex_normal(prob.Nv, [32, 1])
    X = torch.from_numpy(x).to("cuda:0")
    Y = torch.from_numpy(y).to("cuda:0")
    g = op.apply_adjoint(Y).cpu().numpy()
    g0 = plain.apply_adjoint(Y).cpu().numpy()
    Q = np.linalg.solve(inc.s2s(prob, curve).conj().T, inc.s2v(prob, curve).conj().T @ y)
    ref_inc = prob.h ** 2 * (inc.v2s(prob, curve).conj().T @ Q)
    assert rel(g - g0, ref_inc) < 1e-8
    Tx = op.apply(X).cpu().numpy()
    lhs, rhs = np.vdot(y, Tx), np.vdot(g, x)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    plain.close()
    op.close()


def test_inclusion_removed_and_swept(torch_mod):
    """set_inclusion(None) gives back the volume operator bit for bit; a
    frequency copy carries the inclusion and matches the oracle there."""
    torch = torch_mod
    import paper_2210_02698_amd as hbi
    prob, centre, R, ns = CASES["homogeneous-64"]()
    curve = hb_inputs.circle(prob, centre, R, ns)
    s_h = hb_inputs.complex_normal(prob.Nv, [33, 0])
    s = torch.from_numpy(s_h).to("cuda:0")
    say("inclusion removed / swept")
    plain = hbi.Operator(prob, device=0).build(tol=1e-7)
    op = hbi.Operator(prob, device=0).set_inclusion(curve).build(tol=1e-7)
    w2 = 12 * math.pi
    op2 = hbi.Operator.at_omega(op, w2).build(tol=1e-7)
    assert op2.info()["inclusion_ns"] == ns
    p2 = dataclasses.replace(prob, omega=w2)
    c2 = hb_inputs.circle(p2, centre, R, ns)
    u2 = op2.apply(s).cpu().numpy()
    ref2 = oracle.apply(p2, s_h) + _inclusion_term(p2, c2, s_h)
    assert rel(u2, ref2) < 1e-6
    op.set_inclusion(None).build(tol=1e-7)
    assert op.info()["inclusion_ns"] == 0
    assert torch.equal(op.apply(s), plain.apply(s))
    for o in (plain, op, op2):
        o.close()


def test_inclusion_rejected_calls(torch_mod):
    import ctypes
    torch = torch_mod
    import paper_2210_02698_amd as hbi
    from paper_2210_02698_amd import _lib
    lib = _lib.load()
    prob, centre, R, ns = CASES["homogeneous-64"]()
    curve = hb_inputs.circle(prob, centre, R, 16)
    op = hbi.Operator(prob, device=0)
    xy = np.ascontiguousarray(curve.centres)
    w = np.ascontiguousarray(curve.w)
    n = np.ascontiguousarray(curve.slowness)
    P = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    assert lib.hbi_set_inclusion(op._ctx, 16, None, P(w), P(n)) == _lib.HBI_ERR_ARG
    bad = w.copy(); bad[3] = 0.0
    assert lib.hbi_set_inclusion(op._ctx, 16, P(xy), P(bad), P(n)) == _lib.HBI_ERR_ARG
    far = xy.copy(); far[5, 0] = 7.0
    assert lib.hbi_set_inclusion(op._ctx, 16, P(far), P(w), P(n)) == _lib.HBI_ERR_ARG
    assert lib.hbi_set_inclusion(op._ctx, 40000, P(xy), P(w), P(n)) == _lib.HBI_ERR_ARG
    ctx2 = ctypes.c_void_p()
    assert lib.hbi_create(0, None, ctypes.byref(ctx2)) == _lib.HBI_OK
    assert lib.hbi_set_inclusion(ctx2, 16, P(xy), P(w), P(n)) == _lib.HBI_ERR_STATE
    assert lib.hbi_destroy(ctx2) == _lib.HBI_OK
    p3 = hb_inputs.configs.c5(8, nI=5)
    op3 = hbi.Operator(p3, device=0)
    assert lib.hbi_set_inclusion(op3._ctx, 16, P(xy), P(w), P(n)) == _lib.HBI_ERR_ARG
    op.set_inclusion(curve).build(tol=1e-5, prec="f32")
    s = torch.zeros((prob.Nv, 1), dtype=torch.complex64, device="cuda:0")
    with pytest.raises(hbi.HBIError):
        hbi.apply_batched([op], [s])
    # still usable
    u = op.apply(s[:, 0].contiguous())
    assert torch.count_nonzero(u).item() == 0
    op3.close()
    op.close()


def test_inclusion_butterfly_storage_and_accuracy(torch_mod):
    """The open square of side 0.8 (20 segments per shortest wavelength) in
    the Gaussian-bump medium at 128^2 and 256^2 cells (omega = 32 pi,
    64 pi; 1,000 and 2,000 segments), FP32 at tol 1e-5: the butterfly's
    entries grow like N_v (x4 here, under x5), not like N_v N_s (x8), and are
    a small fraction of the dense G; the total field matches the oracle on
    sampled rows at 128^2."""
    torch = torch_mod
    import paper_2210_02698_amd as hbi
    ent = {}
    for n in (128, 256):
        prob = hb_inputs.configs.c4(n)
        curve = hb_inputs.open_square(prob, (0.5, 0.5), 0.8, 20)
        say(f"inclusion butterfly {n}^2 open square ns={curve.Ns} f32")
        op = hbi.Operator(prob, device=0).set_inclusion(curve).build(tol=1e-5, prec="f32")
        info = op.info()
        ent[n] = info["inclusion_bf_entries"]
        say(f"  L={info['inclusion_bf_levels']} entries {ent[n]} "
            f"({ent[n] / (prob.Nv * curve.Ns):.3f} of dense G) rank max "
            f"{info['inclusion_bf_rank_max']}")
        assert ent[n] < 0.1 * prob.Nv * curve.Ns
        if n == 128:
            s_h = hb_inputs.complex_normal(prob.Nv, [34, 0])
            u = op.apply(torch.from_numpy(s_h).to("cuda:0").to(torch.complex64))
            rows = np.sort(np.random.default_rng([34, 1]).choice(prob.Nv, 64, replace=False))
            ref = inc.apply(prob, curve, s_h, rows)
            e = rel(u.cpu().numpy().astype(np.complex128)[rows], ref)
            say(f"  total field rel err {e:.2e}")
            assert e < 1e-4
        op.close()
    assert ent[256] < 5 * ent[128], ent


@pytest.mark.parametrize("ns,levels", [(5, 0), (16, 1), (40, 3)])
def test_inclusion_butterfly_few_segments(torch_mod, ns, levels):
    """Degenerate butterflies of G: 5 segments give L = 0 (one
    interpolative decomposition of all cells against the leaf, then K^L over
    every cell), 16 segments L = 1 (one transfer level), 40 segments L = 3;
    the inclusion term and its adjoint match the oracle in FP64."""
    torch = torch_mod
    import paper_2210_02698_amd as hbi
    prob = hb_inputs.configs.c1()
    curve = hb_inputs.circle(prob, (0.45, 0.55), 0.1, ns)
    say(f"inclusion butterfly ns={ns}")
    plain = hbi.Operator(prob, device=0).build(tol=1e-7)
    op = hbi.Operator(prob, device=0).set_inclusion(curve).build(tol=1e-7)
    assert op.info()["inclusion_bf_levels"] == levels
    s_h = hb_inputs.complex_normal(prob.Nv, [35, ns])
    s = torch.from_numpy(s_h).to("cuda:0")
    u = op.apply(s).cpu().numpy() - plain.apply(s).cpu().numpy()
    assert rel(u, _inclusion_term(prob, curve, s_h)) < 1e-8
    g = op.apply_adjoint(s).cpu().numpy() - plain.apply_adjoint(s).cpu().numpy()
    Q = np.linalg.solve(inc.s2s(prob, curve).conj().T, inc.s2v(prob, curve).conj().T @ s_h)
    assert rel(g, prob.h ** 2 * (inc.v2s(prob, curve).conj().T @ Q)) < 1e-8
    plain.close()
    op.close()


def test_blocked_and_column_inverse_agree(torch_mod, monkeypatch):
    """The inverse of K^{s2s} by 32-column panels (an MFMA update of the rest
    per panel, the default) and column by column give the same operator to
    rounding: 200 segments, 7 panels, the last one partial; FP64."""
    torch = torch_mod
    import paper_2210_02698_amd as hbi
    prob, centre, R, ns = CASES["bump-64"]()
    curve = hb_inputs.circle(prob, centre, R, ns)
    s = torch.from_numpy(hb_inputs.complex_normal(prob.Nv, [36, 0])).to("cuda:0")
    u = {}
    for mode in ("panels", "columns"):
        if mode == "columns":
            monkeypatch.setenv("HBI_S2S_INVERSE", "columns")
        say(f"K^s2s inverse by {mode}")
        op = hbi.Operator(prob, device=0).set_inclusion(curve).build(tol=1e-7)
        u[mode] = op.apply(s).cpu().numpy()
        op.close()
    d = rel(u["panels"], u["columns"])
    say(f"panels vs columns {d:.2e}")
    assert d < 1e-12, d
