"""Error paths of the C ABI on a live context: every rejected call returns
its status code and leaves the context usable (checked by a correct apply
afterwards)."""
import ctypes

import numpy as np
import pytest

import hb_inputs
from _hbi_util import ensure_built, requires_gpu

pytestmark = [pytest.mark.gpu, requires_gpu]


def test_rejected_calls_leave_context_usable():
    ensure_built()
    import torch
    import paper_2210_02698_amd as hbi
    from paper_2210_02698_amd import _lib
    lib = _lib.load()
    prob = hb_inputs.configs.c1(16)
    op = hbi.Operator(prob, device=0)
    ctx = op._ctx
    s = torch.zeros(prob.Nv, dtype=torch.complex128, device="cuda:0")
    u = torch.zeros_like(s)
    vp = lambda t: ctypes.c_void_p(t.data_ptr())
    # apply before build
    assert lib.hbi_apply(ctx, vp(s), vp(u), 1, prob.Nv) == _lib.HBI_ERR_STATE
    assert b"before build" in lib.hbi_last_error(ctx)
    # bad build arguments
    assert lib.hbi_build(ctx, 0.0, 0) == _lib.HBI_ERR_ARG
    assert lib.hbi_build(ctx, 1e-7, 7) == _lib.HBI_ERR_ARG
    # a fresh context has no tables
    ctx2 = ctypes.c_void_p()
    assert lib.hbi_create(0, None, ctypes.byref(ctx2)) == _lib.HBI_OK
    assert lib.hbi_build(ctx2, 1e-7, 0) == _lib.HBI_ERR_STATE
    # frequency sweep: a source without tables, a bad frequency, no source
    assert lib.hbi_load_tables_from(ctx, ctx2, 1.0) == _lib.HBI_ERR_STATE
    assert b"no tables" in lib.hbi_last_error(ctx)
    assert lib.hbi_load_tables_from(ctx2, ctx, -1.0) == _lib.HBI_ERR_ARG
    assert lib.hbi_load_tables_from(ctx2, ctx, float("nan")) == _lib.HBI_ERR_ARG
    assert lib.hbi_load_tables_from(ctx2, None, 1.0) == _lib.HBI_ERR_ARG
    assert lib.hbi_destroy(ctx2) == _lib.HBI_OK
    # bad tables
    t = _lib.hbi_tables()
    t.dim = 4
    assert lib.hbi_load_tables(ctx, ctypes.byref(t)) == _lib.HBI_ERR_ARG
    # entries: index out of range
    rows = np.array([0, prob.Nv], dtype=np.int32)
    cols = np.array([0], dtype=np.int32)
    out = torch.empty(2, dtype=torch.complex128, device="cuda:0")
    assert lib.hbi_entries(ctx, rows.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), 2,
                           cols.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), 1,
                           vp(out)) == _lib.HBI_ERR_ARG
    op.build(tol=1e-7, prec="f64")
    # bad apply arguments
    assert lib.hbi_apply(ctx, vp(s), vp(u), 0, prob.Nv) == _lib.HBI_ERR_ARG
    assert lib.hbi_apply(ctx, vp(s), vp(u), 1, prob.Nv - 1) == _lib.HBI_ERR_ARG
    assert lib.hbi_apply(ctx, vp(s), vp(s), 1, prob.Nv) == _lib.HBI_ERR_ARG   # aliasing
    # precision mismatch in a batched call
    op32 = hbi.Operator(prob, device=0).build(tol=1e-6, prec="f32")
    ctxs = (ctypes.c_void_p * 2)(ctx.value, op32._ctx.value)
    ptrs = (ctypes.c_void_p * 2)(s.data_ptr(), s.data_ptr())
    outs = (ctypes.c_void_p * 2)(u.data_ptr(), u.data_ptr())
    nr = (ctypes.c_int32 * 2)(1, 1)
    ld = (ctypes.c_int64 * 2)(prob.Nv, prob.Nv)
    assert lib.hbi_apply_batched(ctxs, 2, ptrs, outs, nr, ld) == _lib.HBI_ERR_ARG
    # still usable: the apply of a point source gives a column of K (eq. m_v2v)
    j = 37
    s[j] = 1.0 / prob.h ** 2
    col = op.apply(s).cpu().numpy()
    ref = op.entries(np.arange(prob.Nv), [j]).cpu().numpy()[:, 0]
    assert np.linalg.norm(col - ref) / np.linalg.norm(ref) < 1e-6
    op32.close()
    op.close()


def test_out_of_memory_is_reported_and_recovered(monkeypatch):
    """Allocation failures, forced on the host (HBI_FAIL_ALLOC_BYTES: every
    device allocation of at least that many bytes fails before any kernel of
    the call is launched), come back as HBI_ERR_OOM with the failing call in
    the message, for a build and for a batched apply; the context keeps its
    tables, refuses to apply, and builds and applies normally once memory is
    available again."""
    ensure_built()
    import torch
    import paper_2210_02698_amd as hbi
    from paper_2210_02698_amd import _lib
    prob = hb_inputs.configs.c2(64, nbox=4)
    s = torch.from_numpy(hb_inputs.complex_normal(prob.Nv, [71, 0])).to("cuda:0")
    ref = hbi.Operator(prob, device=0).build(tol=1e-7)
    u_ref = ref.apply(s).cpu().numpy()
    op = hbi.Operator(prob, device=0)
    print("[gpu-case] forced out of memory: build", flush=True)
    monkeypatch.setenv("HBI_FAIL_ALLOC_BYTES", str(1 << 20))
    with pytest.raises(hbi.HBIError) as ei:
        op.build(tol=1e-7)
    assert ei.value.status == _lib.HBI_ERR_OOM, ei.value
    assert op.info()["state"] == 1
    monkeypatch.delenv("HBI_FAIL_ALLOC_BYTES")
    with pytest.raises(hbi.HBIError):
        op.apply(s)               # no factors: the binding refuses
    op.build(tol=1e-7)
    assert np.array_equal(op.apply(s).cpu().numpy(), u_ref)
    # a batched apply whose workspace cannot be allocated
    print("[gpu-case] forced out of memory: batched apply", flush=True)
    S = [s.reshape(-1, 1).repeat(1, 3).t().contiguous().t(), s.reshape(-1, 1)]
    monkeypatch.setenv("HBI_FAIL_ALLOC_BYTES", str(1 << 16))
    with pytest.raises(hbi.HBIError) as ei:
        hbi.apply_batched([op, ref], S)
    assert ei.value.status == _lib.HBI_ERR_OOM, ei.value
    monkeypatch.delenv("HBI_FAIL_ALLOC_BYTES")
    U = hbi.apply_batched([op, ref], S)
    torch.cuda.synchronize()
    assert np.allclose(U[1].cpu().numpy()[:, 0], u_ref, rtol=0, atol=1e-12 * np.abs(u_ref).max())
    op.close()
    ref.close()
