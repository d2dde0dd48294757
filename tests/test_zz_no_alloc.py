"""hbi_apply_noalloc: the single-RHS product with its per-level vectors in
the library's fixed per-device scratch array (nothing allocated).  Checked
through the C ABI against hbi_apply on the same operator and input, on two
calls in a row where the second has the smaller input (a smaller problem on
the same device, so the array holds the first call's larger contents), with
several right-hand sides, and for the documented rejections."""
import numpy as np
import pytest

import hb_inputs
from _hbi_util import ensure_built, requires_gpu
from _parity import rel_l2

pytestmark = [pytest.mark.gpu, requires_gpu]

LIMIT = 128 << 20   # HBI_NOALLOC_SCRATCH_BYTES


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


@pytest.fixture(scope="module")
def torch_mod():
    ensure_built()
    import torch
    return torch


def _pair(torch, op, S):
    """(hbi_apply, hbi_apply_noalloc) of S on op, as host arrays."""
    ref = op.apply(S).cpu().numpy()
    out = torch.empty_like(S)
    got = op.apply_noalloc(S, out).cpu().numpy()
    return ref, got


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_noalloc_matches_apply_on_two_calls_larger_then_smaller(torch_mod, prec):
    torch = torch_mod
    import paper_2210_02698_amd as hbi
    tol, bound = (1e-7, 1e-12) if prec == "f64" else (1e-5, 1e-6)
    dt = torch.complex128 if prec == "f64" else torch.complex64
    big = hb_inputs.configs.c2(128, nbox=4)
    small = hb_inputs.configs.c1(32)
    ops = [hbi.Operator(p, device=0).build(tol=tol, prec=prec) for p in (big, small)]
    for p, op in zip((big, small), ops):
        need = op.info()["apply_scratch_bytes"]
        say(f"noalloc {prec} {p.name} Nv={p.Nv} scratch {need} bytes")
        assert 0 < need <= LIMIT
    # first call: the larger problem, then the smaller one on the same array
    for k, (p, op) in enumerate(zip((big, small), ops)):
        s = torch.from_numpy(hb_inputs.complex_normal(p.Nv, [61, k])).to("cuda:0").to(dt)
        ref, got = _pair(torch, op, s)
        e = rel_l2(got, ref)
        say(f"call {k}: noalloc vs apply rel diff {e:.2e}")
        assert e <= bound, (k, e)
    # several right-hand sides (column-major N_v x 3) on the smaller problem
    S = torch.from_numpy(np.asfortranarray(hb_inputs.complex_normal((small.Nv, 3), [61, 9])))
    S = S.to("cuda:0").to(dt)
    out = torch.empty((3, small.Nv), dtype=dt, device="cuda:0").t()
    got = ops[1].apply_noalloc(S, out).cpu().numpy()
    for r in range(3):
        ref = ops[1].apply(S[:, r].contiguous()).cpu().numpy()
        assert rel_l2(got[:, r], ref) <= bound, r
    for op in ops:
        op.close()


def test_noalloc_rejects_what_does_not_fit(torch_mod):
    torch = torch_mod
    import paper_2210_02698_amd as hbi
    # a product whose vectors exceed the fixed array: a clear argument error
    p = hb_inputs.configs.c2(640, nbox=8)
    op = hbi.Operator(p, device=0).build(tol=1e-7, prec="f64")
    need = op.info()["apply_scratch_bytes"]
    say(f"noalloc too large: Nv={p.Nv} needs {need} bytes")
    assert need > LIMIT
    s = torch.zeros(p.Nv, dtype=torch.complex128, device="cuda:0")
    with pytest.raises(hbi.HBIError) as ei:
        op.apply_noalloc(s, torch.empty_like(s))
    assert "scratch" in str(ei.value)
    op.close()
    # a context with a curve inclusion
    q = hb_inputs.configs.c4(64)
    op = hbi.Operator(q, device=0).set_inclusion(hb_inputs.open_square(q, (0.5, 0.5), 0.8, 4))
    op.build(tol=1e-5, prec="f32")
    s = torch.zeros(q.Nv, dtype=torch.complex64, device="cuda:0")
    with pytest.raises(hbi.HBIError) as ei:
        op.apply_noalloc(s, torch.empty_like(s))
    assert "inclusion" in str(ei.value)
    op.close()
