"""GPU parity of the many-right-hand-side (MFMA tile) path against the FP64
oracle, at the shapes of the measured workloads.

  * 3D sinusoid (n = 1 + 0.2 sin 2pi x sin 2pi y sin 2pi z, global nI = 9)
    on 32^3 cells with 32 RHS: FP32 factors at tol 1e-6 (bound 1e-4) and
    FP64 at tol 1e-7 (bound 1e-6), on 256 seeded rows x all RHS.
  * The batched constant-gradient workload's shapes (c(y) = 1 + g y,
    nI = 13, Gaussian sources of width 2h): a 256^2 problem with 256 RHS, a
    128^2 problem with 1 RHS and a 128^2 problem with 300 RHS (more than one
    job of at most 256 columns) in one hbi_apply_batched call, FP32 at tol
    1e-5 (bound 1e-4), every problem on seeded rows x all RHS.
Each bound is on the relative L2 error and, 20 times larger, on the worst
row relative to the rms of the reference (tests/_parity.py).
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


@pytest.mark.parametrize("prec,tol,bound", [("f32", 1e-6, 1e-4), ("f64", 1e-7, 1e-6)])
def test_3d_many_rhs_matches_oracle(torch_mod, prec, tol, bound):
    torch = torch_mod
    import paper_2210_02698_amd as hbi
    prob = hb_inputs.configs.c5(32, nI=9)
    nrhs = 32
    say(f"3d many rhs {prec} Nv={prob.Nv} nrhs={nrhs} tol={tol}")
    op = hbi.Operator(prob, device=0).build(tol=tol, prec=prec)
    dt = torch.complex64 if prec == "f32" else torch.complex128
    npdt = np.complex64 if prec == "f32" else np.complex128
    S = np.asfortranarray(hb_inputs.complex_normal((prob.Nv, nrhs), [5, 32, 1]).astype(npdt))
    U = op.apply(torch.from_numpy(S).to("cuda:0")).cpu().numpy()
    rows = np.sort(np.random.default_rng([5, 32, 2]).choice(prob.Nv, 256, replace=False))
    ref = oracle.apply(prob, S.astype(np.complex128), rows)
    check(U[rows], ref, bound, f"3d {prec} 32 RHS")
    # the adjoint with several RHS against the oracle's h^d K^H on the same rows
    UA = op.apply_adjoint(torch.from_numpy(S[:, :4].copy(order="F")).to("cuda:0")).cpu().numpy()
    refa = oracle.apply_adjoint(prob, S[:, :4].astype(np.complex128), rows)
    check(UA[rows], refa, bound, f"3d {prec} adjoint 4 RHS")
    op.close()


def _cg_problem(side, g):
    return hb_inputs.make_problem(ConstantGradient(1.0, (0.0, g)), 2, (side, side),
                                  2 * math.pi * side / 8, nI=13,
                                  name=f"cg-{side}-g{g:.2f}")


def test_batched_workload_shapes_match_oracle(torch_mod):
    torch = torch_mod
    import paper_2210_02698_amd as hbi
    specs = [(256, 0.6, 256), (128, 0.3, 1), (128, 0.9, 300)]
    ops, S, probs = [], [], []
    for p, (side, g, nr) in enumerate(specs):
        prob = _cg_problem(side, g)
        probs.append(prob)
        ops.append(hbi.Operator(prob, device=0).build(tol=1e-5, prec="f32"))
        S.append(torch.from_numpy(hb_inputs.gaussian_sources(prob, nr, [3, 7, p])).to("cuda:0"))
        say(f"batched member {p}: {prob.name} Nv={prob.Nv} nrhs={nr} "
            f"nnz={ops[-1].info()['nnz_total']}")
    U = [u.cpu().numpy() for u in hbi.apply_batched(ops, S)]
    for p, prob in enumerate(probs):
        rows = np.sort(np.random.default_rng([3, 7, 10 + p]).choice(prob.Nv, 48, replace=False))
        ref = oracle.apply(prob, S[p].cpu().numpy().astype(np.complex128), rows)
        check(U[p][rows], ref, 1e-4, f"batched member {p} ({specs[p][2]} RHS)")
    # a replay (captured graph, same pointers) gives the same numbers
    U2 = [u.cpu().numpy() for u in hbi.apply_batched(ops, S)]
    for a, b in zip(U, U2):
        assert np.array_equal(a, b)
    for op in ops:
        op.close()

