"""GPU parity of the HIP path (through the C ABI) against the FP64 oracle.

Tolerances:
  * hb_entry (FP64): entries agree to 1e-12 relative to the block maximum;
    the only differences are rounding order in the interpolation and the
    two independent Hankel evaluations (both ~1e-15).
  * bf_apply FP64 at tol: the compressed operator differs from K by about
    tol per ID level (eq. ID); the stated target is rel. L2 error <= 1e-6 at
    tol = 1e-7, and <= 1e-4 for FP32 factors built at 1e-6.
  * adjoint: the dot-product identity <K x, y> = <x, K^H y> holds for the
    compressed operator to rounding (1e-12 FP64).
"""
import math

import numpy as np
import pytest

import hb_inputs
import oracle
from _hbi_util import ensure_built, requires_gpu
from _parity import check
from hb_inputs.media import ConstantGradient

pytestmark = [pytest.mark.gpu, requires_gpu]


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


@pytest.fixture(scope="module")
def torch_mod():
    ensure_built()
    import torch
    return torch


def make_op(prob, tol=1e-7, prec="f64", **kw):
    import paper_2210_02698_amd as hbi
    op = hbi.Operator(prob, device=0)
    op.build(tol=tol, prec=prec, **kw)
    return op


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def to_dev(torch, x, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")
    return t if dtype is None else t.to(dtype)


# ---------------------------------------------------------------- hb_entry
ENTRY_CASES = {
    "c1-homogeneous-2d": lambda: hb_inputs.configs.c1(32),
    "bump-piecewise-2d": lambda: hb_inputs.configs.c2(32, nbox=4),
    "constant-gradient-2d-nI13": lambda: hb_inputs.make_problem(
        ConstantGradient(1.0, (0.0, 0.7)), 2, (24, 24), 2 * math.pi * 3, nI=13),
    "sinusoid-3d": lambda: hb_inputs.configs.c5(8, nI=5),
    "constant-gradient-3d": lambda: hb_inputs.make_problem(
        ConstantGradient(0.708, (0.0, -0.8, 0.0)), 3, (8, 8, 8), 20.0, nI=6, extent=0.52),
}


@pytest.mark.parametrize("name", list(ENTRY_CASES))
def test_entries_match_oracle(torch_mod, name):
    torch = torch_mod
    prob = ENTRY_CASES[name]()
    say(f"entries {name} Nv={prob.Nv}")
    import paper_2210_02698_amd as hbi
    op = hbi.Operator(prob, device=0)
    rng = np.random.default_rng(1)
    rows = rng.choice(prob.Nv, min(prob.Nv, 70), replace=False)
    cols = np.concatenate([rng.choice(prob.Nv, min(prob.Nv, 300), replace=False), rows[:5]])
    got = op.entries(rows, cols).cpu().numpy()
    ref = oracle.entries(prob, rows, cols)
    scale = np.abs(ref)
    err = np.abs(got - ref) / np.maximum(scale, 1e-3 * scale.max())
    assert err.max() < 1e-12, (name, err.max())
    op.close()


# ---------------------------------------------------------------- bf_apply
@pytest.fixture(scope="module")
def c1_case(torch_mod):
    prob = hb_inputs.configs.c1()
    K = oracle.dense(prob)
    return prob, K


def test_bruteforce_tiny_full_matrix(torch_mod):
    """Applying the compressed operator to identity columns reproduces the
    dense matrix h^d K entry by entry (N_v = 256, L_v = 2)."""
    torch = torch_mod
    prob = hb_inputs.configs.c2(16, nbox=2)
    say(f"bruteforce tiny Nv={prob.Nv}")
    op = make_op(prob, tol=1e-10)
    I = torch.eye(prob.Nv, dtype=torch.complex128, device="cuda:0")
    M = op.apply(I).cpu().numpy()
    ref = oracle.dense(prob) * prob.h ** 2
    err = np.abs(M - ref).max() / np.abs(ref).max()
    assert err < 1e-8, err
    MA = op.apply_adjoint(I).cpu().numpy()
    assert np.abs(MA - ref.conj().T).max() / np.abs(ref).max() < 1e-8
    op.close()


def test_c1_apply_fp64(torch_mod, c1_case):
    torch = torch_mod
    prob, K = c1_case
    say("c1 apply fp64 tol 1e-7")
    op = make_op(prob, tol=1e-7)
    s = hb_inputs.complex_normal(prob.Nv, [hb_inputs.configs.CFG_SEED["c1"], 0])
    u = op.apply(to_dev(torch, s)).cpu().numpy()
    ref = K @ (s * prob.h ** 2)
    check(u, ref, 1e-6, "c1 fp64")
    say(f"c1 info {op.info()}")
    # determinism: bitwise identical repeat
    u2 = op.apply(to_dev(torch, s)).cpu().numpy()
    assert np.array_equal(u, u2)
    # adjoint against the oracle's conjugate transpose
    ua = op.apply_adjoint(to_dev(torch, s)).cpu().numpy()
    refa = K.conj().T @ s * prob.h ** 2
    check(ua, refa, 1e-6, "c1 fp64 adjoint")
    op.close()


def test_adjoint_dot_product(torch_mod):
    torch = torch_mod
    prob = hb_inputs.configs.c2(64, nbox=4)
    say(f"adjoint dot product Nv={prob.Nv}")
    op = make_op(prob, tol=1e-7)
    x = hb_inputs.complex_normal(prob.Nv, [5, 1])
    y = hb_inputs.complex_normal(prob.Nv, [5, 2])
    Kx = op.apply(to_dev(torch, x)).cpu().numpy()
    KHy = op.apply_adjoint(to_dev(torch, y)).cpu().numpy()
    lhs, rhs = np.vdot(y, Kx), np.vdot(KHy, x)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    op.close()


@pytest.mark.parametrize("prec,nrhs", [("f64", 3), ("f64", 37), ("f32", 37), ("f32", 130)])
def test_multi_rhs_matches_single(torch_mod, prec, nrhs):
    """nrhs >= 2 runs the MFMA tile path; each column must equal the
    single-RHS apply up to rounding (different summation order)."""
    torch = torch_mod
    prob = hb_inputs.configs.c2(48, nbox=2)
    say(f"multi rhs {prec} nrhs={nrhs}")
    op = make_op(prob, tol=1e-7 if prec == "f64" else 1e-6, prec=prec)
    dt = torch.complex128 if prec == "f64" else torch.complex64
    S = hb_inputs.complex_normal((nrhs, prob.Nv), [7, nrhs])
    U = op.apply(to_dev(torch, S, dt).t()).cpu().numpy()
    tol = 1e-12 if prec == "f64" else 2e-5
    for r in range(0, nrhs, max(1, nrhs // 7)):
        u = op.apply(to_dev(torch, S[r], dt)).cpu().numpy()
        assert rel(U[:, r], u) < tol, (r, rel(U[:, r], u))
    # and against the FP64 oracle on seeded rows, every RHS
    rows = np.sort(np.random.default_rng([7, nrhs]).choice(prob.Nv, 64, replace=False))
    ref = oracle.apply(prob, S.T.astype(np.complex128), rows)
    check(U[rows], ref, 1e-6 if prec == "f64" else 1e-4, f"multi rhs {prec} {nrhs} vs oracle")
    # replay of the captured graph gives identical results
    U2 = op.apply(to_dev(torch, S, dt).t()).cpu().numpy()
    assert np.array_equal(U, U2)
    # the adjoint with several RHS (MFMA tiles of the conjugate-transposed
    # factors) against the single-RHS adjoint, the oracle and the forward
    # product (dot-product identity, all columns at once)
    UA = op.apply_adjoint(to_dev(torch, S, dt).t()).cpu().numpy()
    for r in range(0, nrhs, max(1, nrhs // 7)):
        ua = op.apply_adjoint(to_dev(torch, S[r], dt)).cpu().numpy()
        assert rel(UA[:, r], ua) < tol, (r, rel(UA[:, r], ua))
    refa = oracle.apply_adjoint(prob, S.T.astype(np.complex128), rows)
    check(UA[rows], refa, 1e-6 if prec == "f64" else 1e-4, f"multi rhs {prec} {nrhs} adjoint")
    Y = hb_inputs.complex_normal((nrhs, prob.Nv), [7, nrhs, 1])
    KX = U.astype(np.complex128)
    KHY = op.apply_adjoint(to_dev(torch, Y, dt).t()).cpu().numpy().astype(np.complex128)
    npdt = np.complex64 if prec == "f32" else np.complex128   # the values the GPU saw
    Xr = S.T.astype(npdt).astype(np.complex128)
    Yr = Y.T.astype(npdt).astype(np.complex128)
    lhs, rhs_ = np.vdot(Yr, KX), np.vdot(KHY, Xr)
    assert abs(lhs - rhs_) <= (1e-12 if prec == "f64" else 1e-5) * abs(lhs), (lhs, rhs_)
    op.close()


def _batched(torch, ops, S, dt):
    import ctypes
    from paper_2210_02698_amd import _lib
    lib = _lib.load()
    n = len(ops)
    S = [s.t().contiguous().t() for s in S]      # column-major N_v x nrhs
    assert all(s.stride(0) == 1 for s in S)
    ctxs = (ctypes.c_void_p * n)(*[o._ctx.value for o in ops])
    Ut = [torch.empty((s.shape[1], s.shape[0]), dtype=dt, device="cuda:0").t() for s in S]
    sp = (ctypes.c_void_p * n)(*[s.data_ptr() for s in S])
    up = (ctypes.c_void_p * n)(*[u.data_ptr() for u in Ut])
    nr = (ctypes.c_int32 * n)(*[s.shape[1] for s in S])
    ld = (ctypes.c_int64 * n)(*[s.shape[0] for s in S])
    ops[0].set_stream()
    _lib.check(lib.hbi_apply_batched(ctxs, n, sp, up, nr, ld), ops[0]._ctx)
    torch.cuda.synchronize()
    return [u.cpu().numpy() for u in Ut]


@pytest.mark.parametrize("budget", [None, 24 << 20])
def test_apply_batched_uneven_problems(torch_mod, budget, monkeypatch):
    """Several constant-gradient problems of uneven size and RHS count in one
    call; matches per-problem single-RHS applies.  A small workspace budget
    forces right-hand-side chunking and several passes in the graph."""
    torch = torch_mod
    if budget:
        monkeypatch.setenv("HBI_MULTI_BYTES", str(budget))
    specs = [(32, 0.3, 1), (48, 0.7, 21), (40, 0.5, 40), (64, 0.9, 17)]
    ops, S, probs = [], [], []
    for side, g, nr in specs:
        prob = hb_inputs.make_problem(ConstantGradient(1.0, (0.0, g)), 2, (side, side),
                                      2 * math.pi * side / 8, nI=7)
        probs.append(prob)
        ops.append(make_op(prob, tol=1e-6, prec="f32"))
        S.append(to_dev(torch, hb_inputs.gaussian_sources(prob, nr, [3, side]), torch.complex64))
    say(f"batched {len(ops)} problems budget={budget}")
    U = _batched(torch, ops, S, torch.complex64)
    for op, s, u in zip(ops, S, U):
        for r in range(s.shape[1]):
            ref = op.apply(s[:, r].contiguous()).cpu().numpy()
            assert rel(u[:, r], ref) < 2e-5
    # replay with fresh output buffers (pointer patch of the captured graph)
    U2 = _batched(torch, ops, S, torch.complex64)
    for a, b in zip(U, U2):
        assert np.array_equal(a, b)
    # parity of one problem against the FP64 oracle
    for p in range(len(probs)):
        rows = np.arange(p, probs[p].Nv, 37)
        ref = oracle.apply(probs[p], S[p].cpu().numpy().astype(np.complex128), rows)
        check(U[p][rows], ref, 1e-4, f"batched member {p} vs oracle")
    for op in ops:
        op.close()


def test_apply_batched_after_a_member_is_rebuilt(torch_mod):
    """The captured graph of a batched call is keyed on the builds of all of
    its problems: after the second problem is rebuilt (new factor memory),
    the same call with the same RHS counts captures again and matches
    per-problem applies of the new factors."""
    torch = torch_mod
    ops, S = [], []
    for side, g, nr in [(32, 0.3, 3), (40, 0.6, 5)]:
        prob = hb_inputs.make_problem(ConstantGradient(1.0, (0.0, g)), 2, (side, side),
                                      2 * math.pi * side / 8, nI=7)
        ops.append(make_op(prob, tol=1e-6, prec="f32"))
        S.append(to_dev(torch, hb_inputs.gaussian_sources(prob, nr, [4, side]), torch.complex64))
    say("batched before and after rebuilding problem 1")
    U = _batched(torch, ops, S, torch.complex64)
    ops[1].build(tol=1e-4, prec="f32")
    U2 = _batched(torch, ops, S, torch.complex64)
    for p, (op, s) in enumerate(zip(ops, S)):
        for r in range(s.shape[1]):
            ref = op.apply(s[:, r].contiguous()).cpu().numpy()
            assert rel(U2[p][:, r], ref) < 2e-5
    assert np.array_equal(U[0], U2[0])
    assert not np.array_equal(U[1], U2[1])   # other factors, other result
    for op in ops:
        op.close()


@pytest.mark.parametrize("ncell", [(37, 29), (5, 7), (64, 1), (40, 40)])
def test_ragged_and_degenerate_grids(torch_mod, ncell):
    """Uneven clusters (N_v not a power of two), a single leaf (N_v <= 64,
    no butterflies) and a 1-cell-high strip."""
    torch = torch_mod
    nx, ny = ncell
    prob = hb_inputs.make_problem(ConstantGradient(1.0, (0.0, 0.5)), 2, (nx, ny),
                                  2 * math.pi * max(nx, ny) / 8, nI=6, extent=1.0)
    say(f"ragged {ncell} Nv={prob.Nv}")
    op = make_op(prob, tol=1e-8)
    s = hb_inputs.complex_normal(prob.Nv, [8, nx, ny])
    u = op.apply(to_dev(torch, s)).cpu().numpy()
    ref = oracle.apply(prob, s)
    check(u, ref, 1e-6, f"ragged {ncell}")
    op.close()


def test_fp32_factors(torch_mod, c1_case):
    torch = torch_mod
    prob, K = c1_case
    say("c1 fp32")
    op = make_op(prob, tol=1e-6, prec="f32")
    s = hb_inputs.complex_normal(prob.Nv, [1, 3])
    u = op.apply(to_dev(torch, s, torch.complex64)).cpu().numpy()
    ref = K @ (s * prob.h ** 2)
    check(u, ref, 1e-4, "c1 fp32")
    op.close()


def test_3d_apply_sampled_rows(torch_mod):
    torch = torch_mod
    prob = hb_inputs.configs.c5(16, nI=6)
    say(f"3d apply Nv={prob.Nv}")
    op = make_op(prob, tol=1e-7)
    s = hb_inputs.complex_normal(prob.Nv, [5, 9])
    u = op.apply(to_dev(torch, s)).cpu().numpy()
    rows = np.random.default_rng(2).choice(prob.Nv, 256, replace=False)
    ref = oracle.apply(prob, s, rows)
    check(u[rows], ref, 1e-6, "3d fp64 1 RHS")
    op.close()


@pytest.mark.parametrize("prec,tol,bound", [("f64", 1e-7, 1e-6), ("f32", 1e-5, 1e-4)])
def test_id_kernels_agree(torch_mod, monkeypatch, prec, tol, bound):
    """By default blocks of at most 64 candidate columns are decomposed on
    chip (pivoted QR of the triangular factor of the block) and wider ones,
    at tol >= 1e-7 and with at least as many rows as columns, through their
    Gram matrix (pivoted Cholesky), the rest by the global-memory pivoted
    QR; HBI_ID_KERNEL=cpqr sends every wide block to the global-memory
    pivoted QR, =global every block, and =blocked every block to its panel
    (deferred-update) form.  The last two builds also turn the per-cell
    column-side cache off (HBI_HC_CACHE_BYTES=0), so entries come from the
    per-block column side.  All four operators agree with the oracle and
    with each other to the compression tolerance, with nearly the same
    ranks."""
    torch = torch_mod
    prob = hb_inputs.configs.c2(128)
    dt = torch.complex128 if prec == "f64" else torch.complex64
    s = hb_inputs.complex_normal(prob.Nv, [11, 4])
    rows = np.random.default_rng(6).choice(prob.Nv, 64, replace=False)
    ref = oracle.apply(prob, s, rows)
    out = {}
    for kind in ("auto", "cpqr", "global", "blocked"):
        if kind != "auto":
            monkeypatch.setenv("HBI_ID_KERNEL", kind)
        if kind in ("global", "blocked"):
            monkeypatch.setenv("HBI_HC_CACHE_BYTES", "0")
        say(f"id kernel {kind} {prec} tol {tol}")
        op = make_op(prob, tol=tol, prec=prec)
        u = op.apply(to_dev(torch, s, dt)).cpu().numpy().astype(np.complex128)
        out[kind] = (u, op.info())
        check(u[rows], ref, bound, f"id kernel {kind}")
        say(f"{kind} rank mean {out[kind][1]['rank_mean']:.3f}")
        op.close()
    info = out["auto"][1]
    say(f"auto paths: on chip {info['n_id_onchip']}, Gram {info['n_id_gram']}, "
        f"global {info['n_id_global']}")
    assert info["n_id_onchip"] > 0, info
    assert info["n_id_gram"] > 0, info
    assert out["cpqr"][1]["n_id_gram"] == 0 and out["cpqr"][1]["n_id_global"] > 0
    assert out["global"][1]["n_id_onchip"] == 0
    for kind in ("cpqr", "global", "blocked"):
        d = rel(out["auto"][0], out[kind][0])
        say(f"auto vs {kind} {d:.3e}")
        assert d < bound, (kind, d)
        r1, r2 = out["auto"][1]["rank_mean"], out[kind][1]["rank_mean"]
        assert abs(r1 - r2) <= 0.02 * r2, (kind, r1, r2)


def test_gram_id_in_3d(torch_mod, monkeypatch):
    """The 3D sinusoid at 32^3 cells, FP32 at tol 1e-6: the wide blocks go
    through their Gram matrix; the operator matches the oracle on sampled
    rows and the one built with the pivoted QR of every wide block to the
    tolerance, with ranks within 3 %."""
    torch = torch_mod
    prob = hb_inputs.configs.c5(32, nI=9)
    s = hb_inputs.complex_normal(prob.Nv, [13, 0])
    rows = np.sort(np.random.default_rng(13).choice(prob.Nv, 48, replace=False))
    ref = oracle.apply(prob, s, rows)
    out = {}
    for kind in ("auto", "cpqr"):
        if kind == "cpqr":
            monkeypatch.setenv("HBI_ID_KERNEL", "cpqr")
        say(f"3d id path {kind}")
        op = make_op(prob, tol=1e-6, prec="f32")
        u = op.apply(to_dev(torch, s, torch.complex64)).cpu().numpy().astype(np.complex128)
        out[kind] = (u, op.info())
        check(u[rows], ref, 1e-4, f"3d {kind}")
        op.close()
    ia, ic = out["auto"][1], out["cpqr"][1]
    say(f"Gram IDs {ia['n_id_gram']}, rank mean {ia['rank_mean']:.2f} vs {ic['rank_mean']:.2f}, "
        f"build {ia['build_s']:.2f} s vs {ic['build_s']:.2f} s")
    assert ia["n_id_gram"] > 0 and ic["n_id_gram"] == 0
    assert abs(ia["rank_mean"] - ic["rank_mean"]) <= 0.03 * ic["rank_mean"]
    assert rel(out["auto"][0], out["cpqr"][0]) < 1e-4


def test_small_build_workspace_many_batches(torch_mod):
    """A 4 MiB build workspace splits every level into many batches (sibling
    pairs kept together); the operator is the same as with the default
    workspace, block for block."""
    torch = torch_mod
    prob = hb_inputs.configs.c2(96)
    s = to_dev(torch, hb_inputs.complex_normal(prob.Nv, [12, 1]))
    say("build workspace 4 MiB vs default")
    u = {}
    for ws in (None, 4 << 20):
        op = make_op(prob, tol=1e-7, workspace_bytes=ws)
        u[ws] = op.apply(s).cpu().numpy()
        info = op.info()
        op.close()
    d = rel(u[4 << 20], u[None])
    say(f"small vs default workspace {d:.3e}, nnz {info['nnz_total']}")
    assert d < 1e-13, d


def test_autograd_gradient(torch_mod):
    """Loss ||P K h^d s - d||^2: gradient from HBApply.backward equals the
    dense adjoint and central finite differences (the loss is quadratic, so
    the differences are exact up to rounding)."""
    torch = torch_mod
    import paper_2210_02698_amd as hbi
    prob = hb_inputs.configs.c4(32)
    say(f"autograd Nv={prob.Nv}")
    op = make_op(prob, tol=1e-9)
    g = np.random.default_rng(4)
    P = np.sort(g.choice(prob.Nv, 64, replace=False))
    cells, s_true = hb_inputs.point_sources(prob, 5, [4, 2])
    d = oracle.apply(prob, s_true, P)
    s0 = hb_inputs.complex_normal(prob.Nv, [4, 3])
    s = to_dev(torch, s0).requires_grad_(True)
    Pd = torch.from_numpy(P).to("cuda:0")
    dd = to_dev(torch, d)
    u = hbi.HBApply.apply(op, s)
    loss = (u[Pd] - dd).abs().pow(2).sum()
    loss.backward()
    grad = s.grad.cpu().numpy()
    K = oracle.dense(prob)
    hd = prob.h ** 2
    r = K[P] @ (s0 * hd) - d
    ref = 2 * hd * (K[P].conj().T @ r)     # torch convention: dL/d(conj s) * 2
    assert rel(grad, ref) < 1e-6

    def L(x):
        return float(np.sum(np.abs(K[P] @ (x * hd) - d) ** 2))

    for j in g.choice(prob.Nv, 6, replace=False):
        for unit in (1.0, 1j):
            e = np.zeros(prob.Nv, complex)
            e[j] = unit * 1e-3
            fd = (L(s0 + e) - L(s0 - e)) / 2e-3
            an = (np.conj(unit) * grad[j]).real
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd))
    op.close()


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_inverse_source_gradient_bump256(torch_mod, prec):
    """Differentiation workload: Gaussian bump on 256^2 cells, P = 512 seeded
    receivers, d = P K s_true from 20 seeded point sources (FP64 oracle),
    loss ||P K h^d s - d||^2 at a seeded complex64 s.  The gradient through
    HBApply (hand-written adjoint) matches the dense FP64 adjoint
    2 h^d K[P]^H (K[P] h^d s - d) and central finite differences (step 1e-3)
    of the dense FP64 loss, which is exactly quadratic, in 64 seeded
    coordinates (real and imaginary directions)."""
    torch = torch_mod
    import paper_2210_02698_amd as hbi
    prob = hb_inputs.configs.c4()
    say(f"gradient bump256 {prec}")
    op = make_op(prob, tol=1e-7 if prec == "f64" else 1e-6, prec=prec)
    seed = hb_inputs.configs.CFG_SEED["c4"]
    g = np.random.default_rng([seed, 0])
    P = np.sort(g.choice(prob.Nv, 512, replace=False))
    cells, s_true = hb_inputs.point_sources(prob, 20, [seed, 1])
    KP = oracle.entries(prob, P, np.arange(prob.Nv))          # dense FP64 rows
    hd = prob.h ** 2
    d = KP @ (s_true * hd)
    s0 = hb_inputs.complex_normal(prob.Nv, [seed, 2], dtype=np.complex64).astype(np.complex128)
    dt = torch.complex64 if prec == "f32" else torch.complex128
    s = to_dev(torch, s0, dt).requires_grad_(True)
    Pd = torch.from_numpy(P).to("cuda:0")
    dd = to_dev(torch, d, dt)
    u = hbi.HBApply.apply(op, s)
    loss = (u[Pd] - dd).abs().pow(2).sum()
    loss.backward()
    grad = s.grad.cpu().numpy().astype(np.complex128)
    r = KP @ (s0 * hd) - d
    ref = 2 * hd * (KP.conj().T @ r)
    e = rel(grad, ref)
    say(f"gradient rel err vs dense adjoint {e:.2e}")
    assert e < (1e-4 if prec == "f32" else 1e-6), e

    # the dense FP64 loss at s0 + delta e_j, formed from the residual r:
    # K[P] (s0 + delta e_j) h^d - d = r + delta h^d K[P][:, j]
    def L(j, delta):
        return float(np.sum(np.abs(r + KP[:, j] * (delta * hd)) ** 2))

    scale = np.linalg.norm(ref) / np.sqrt(prob.Nv)
    for j in g.choice(prob.Nv, 64, replace=False):
        for unit in (1.0, 1j):
            fd = (L(j, unit * 1e-3) - L(j, -unit * 1e-3)) / 2e-3
            an = (np.conj(unit) * grad[j]).real
            assert abs(fd - an) <= 1e-3 * scale + 1e-4 * abs(fd), (j, unit, fd, an)
    op.close()


@pytest.mark.parametrize("prec,tol,bound", [("f64", 1e-7, 1e-6), ("f32", 1e-5, 1e-4)])
def test_transfer_stage_branches(torch_mod, monkeypatch, prec, tol, bound):
    """The forward transfer stage has three kinds of work item: 64-row
    windows whose inputs and column orders are staged in the wave's LDS
    slice, the same with the inputs gathered from global memory (units
    wider than the slice, HBI_WSTAGE_LDS_CAP entries), and
    16-row windows with four lanes a row for units of more than
    HBI_WSTAGE_WIDE_C columns.  Thresholds taken from the unit widths of the
    default build make all of them occur on a 128^2 bump; the build
    statistics count the items of each kind, and the product matches the
    oracle and the default plan."""
    torch = torch_mod
    prob = hb_inputs.configs.c2(128, nbox=4)
    dt = torch.complex128 if prec == "f64" else torch.complex64
    s = hb_inputs.complex_normal(prob.Nv, [13, 5])
    rows = np.sort(np.random.default_rng([13, 6]).choice(prob.Nv, 96, replace=False))
    ref = oracle.apply(prob, s, rows)
    say(f"transfer branches {prec} default plan")
    op = make_op(prob, tol=tol, prec=prec)
    info0 = op.info()
    u0 = op.apply(to_dev(torch, s, dt)).cpu().numpy()
    op.close()
    assert info0["wstage_items_lds"] > 0 and info0["wstage_items_global"] == 0, info0
    check(u0[rows], ref, bound, f"default plan {prec}")
    # the median width goes to the global gathers, the widest quarter to
    # 16-row windows
    cq = info0["wstage_c_quantiles"]
    esz = 16 if prec == "f64" else 8
    per_c = 1 + 4.0 / esz     # slice entries per column: input and two orders
    cap = int(per_c * cq[2]) - 1
    wide = cq[3] - 1
    monkeypatch.setenv("HBI_WSTAGE_LDS_CAP", str(cap))
    monkeypatch.setenv("HBI_WSTAGE_WIDE_C", str(wide))
    say(f"transfer branches {prec}: widths {cq}, cap {cap}, wide above {wide}")
    op = make_op(prob, tol=tol, prec=prec)
    info = op.info()
    say(f"items: lds {info['wstage_items_lds']} global {info['wstage_items_global']} "
        f"wide {info['wstage_items_wide']}")
    assert info["wstage_cap_lds"] == cap
    for kind in ("lds", "global", "wide"):
        assert info[f"wstage_items_{kind}"] > 0, kind
    assert info["nnz_total"] == info0["nnz_total"]
    u = op.apply(to_dev(torch, s, dt)).cpu().numpy()
    check(u[rows], ref, bound, f"forced branches {prec}")
    # same factors, other work items: equal up to the order of the sums
    assert rel(u, u0) < (1e-13 if prec == "f64" else 1e-5)
    # the adjoint is untouched by the forward plan
    y = hb_inputs.complex_normal(prob.Nv, [13, 7])
    Kx = op.apply(to_dev(torch, s, dt)).cpu().numpy().astype(np.complex128)
    KHy = op.apply_adjoint(to_dev(torch, y, dt)).cpu().numpy().astype(np.complex128)
    lhs, rhs = np.vdot(y, Kx), np.vdot(KHy, s)
    assert abs(lhs - rhs) <= (1e-12 if prec == "f64" else 1e-5) * abs(lhs)
    op.close()


def test_autograd_several_rhs(torch_mod):
    """HBApply on an N_v x 3 block: the backward pass runs the MFMA adjoint
    (several right-hand sides) and equals the dense adjoint column by
    column."""
    torch = torch_mod
    import paper_2210_02698_amd as hbi
    prob = hb_inputs.configs.c4(32)
    say(f"autograd 3 RHS Nv={prob.Nv}")
    op = make_op(prob, tol=1e-9)
    S0 = np.asfortranarray(hb_inputs.complex_normal((prob.Nv, 3), [4, 9]))
    D = hb_inputs.complex_normal((prob.Nv, 3), [4, 10])
    s = torch.from_numpy(S0).to("cuda:0").requires_grad_(True)
    u = hbi.HBApply.apply(op, s)
    loss = (u - torch.from_numpy(D).to("cuda:0")).abs().pow(2).sum()
    loss.backward()
    grad = s.grad.cpu().numpy()
    K = oracle.dense(prob)
    hd = prob.h ** 2
    ref = 2 * hd * (K.conj().T @ (K @ (S0 * hd) - D))
    check(grad, ref, 1e-6, "autograd 3 RHS")
    op.close()
