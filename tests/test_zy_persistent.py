"""The batched product as one persistent cooperative launch
(HBI_BATCHED_PERSISTENT=1) against the HIP-graph path and the FP64 oracle.
Collected after the other GPU tests (before the allocation-free entry
point's): a box that cannot launch cooperatively fails here without
hiding them."""
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


@pytest.mark.parametrize("prec,tol,bound", [("f32", 1e-5, 1e-4), ("f64", 1e-7, 1e-6)])
def test_batched_persistent_launch(torch_mod, monkeypatch, prec, tol, bound):
    """The batched product as one persistent cooperative launch (every pass's
    gather, stages and scatter as phases of one kernel, grid-wide barriers
    between them) gives the graph's numbers bit for bit, over several passes
    (a small workspace budget), replays identically, matches the FP64 oracle
    on sampled rows, and the many-RHS adjoint does the same."""
    torch = torch_mod
    import paper_2210_02698_amd as hbi
    dt = torch.complex64 if prec == "f32" else torch.complex128
    monkeypatch.setenv("HBI_MULTI_BYTES", str(24 << 20))
    specs = [(64, 0.6, 40), (32, 0.3, 1), (48, 0.9, 17)]
    ops, S, probs = [], [], []
    for p, (side, g, nr) in enumerate(specs):
        prob = hb_inputs.make_problem(ConstantGradient(1.0, (0.0, g)), 2, (side, side),
                                      2 * math.pi * side / 8, nI=7, name=f"cg-{side}")
        probs.append(prob)
        ops.append(hbi.Operator(prob, device=0).build(tol=tol, prec=prec))
        S.append(torch.from_numpy(hb_inputs.gaussian_sources(prob, nr, [4, 9, p])).to("cuda:0").to(dt))
    say(f"persistent batched {prec}: {len(ops)} problems, RHS {[s.shape[1] for s in S]}")
    monkeypatch.setenv("HBI_BATCHED_PERSISTENT", "0")
    Ug = [u.cpu().numpy() for u in hbi.apply_batched(ops, S)]
    Ag = ops[0].apply_adjoint(S[0]).cpu().numpy()
    monkeypatch.setenv("HBI_BATCHED_PERSISTENT", "1")
    n0 = ops[0].info()["batched_persistent_launches"]
    Up = [u.cpu().numpy() for u in hbi.apply_batched(ops, S)]
    Up2 = [u.cpu().numpy() for u in hbi.apply_batched(ops, S)]
    Ap = ops[0].apply_adjoint(S[0]).cpu().numpy()
    torch.cuda.synchronize()
    # three persistent launches went through the first problem's context:
    # two batched products and the adjoint
    assert ops[0].info()["batched_persistent_launches"] - n0 == 3
    for p in range(len(ops)):
        assert np.array_equal(Up[p], Ug[p]), f"member {p}"
        assert np.array_equal(Up2[p], Ug[p]), f"member {p} replay"
        rows = np.sort(np.random.default_rng([4, 9, 20 + p]).choice(probs[p].Nv, 48, replace=False))
        ref = oracle.apply(probs[p], S[p].cpu().numpy().astype(np.complex128), rows)
        check(Up[p][rows], ref, bound, f"persistent member {p}")
    assert np.array_equal(Ap, Ag)
    cols = np.sort(np.random.default_rng([4, 9, 30]).choice(probs[0].Nv, 32, replace=False))
    ref = oracle.apply_adjoint(probs[0], S[0].cpu().numpy().astype(np.complex128), cols)
    check(Ap[cols], ref, bound, "persistent adjoint")
    for op in ops:
        op.close()
