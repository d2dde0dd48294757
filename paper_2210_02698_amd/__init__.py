"""MI355X-native butterfly-compressed Hadamard-Babich (HB) integrator.

Python face of libhbi.so (include/hbi.h).  PyTorch provides device memory and
streams; every step of entry evaluation, compression and application runs in
the library's HIP kernels.

    op = Operator(problem, device=0)          # problem statement + tables
    op.build(tol=1e-7, prec="f64")            # HODBF factors (Sec. 4.2)
    u = op.apply(s)                           # u = K (h^d s)    (eq. m_v2v)
    g = op.apply_adjoint(r)                   # g = h^d K^H r
    u = HBApply.apply(op, s)                  # differentiable in s

``problem`` is any object with the attributes dim, ncell, origin, h, omega,
nterms, nI, nbox, box_origin, box_size, tau2, v0, v1, slowness (see
hbi_tables in include/hbi.h for their meaning and layout).
"""
from __future__ import annotations

import ctypes
import json

import numpy as np

from . import _lib
from ._lib import HBIError, HBI_F32, HBI_F64

__all__ = ["Operator", "HBApply", "HBIError", "load_library", "apply_batched", "tabulate"]


def load_library():
    return _lib.load()


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class Operator:
    def __init__(self, problem, device: int = 0, stream=None):
        import torch
        self._lib = _lib.load()
        self.device = torch.device("cuda", device)
        self.dim = int(problem.dim)
        self.ncell = tuple(int(c) for c in problem.ncell[: self.dim])
        self.Nv = int(np.prod(self.ncell))
        self.h = float(problem.h)
        self.prec = None
        ctx = ctypes.c_void_p()
        st = stream if stream is not None else torch.cuda.current_stream(self.device).cuda_stream
        _lib.check(self._lib.hbi_create(device, ctypes.c_void_p(st), ctypes.byref(ctx)))
        self._ctx = ctx
        self._keep = []
        self.load(problem)

    @classmethod
    def at_omega(cls, src: "Operator", omega: float, stream=None) -> "Operator":
        """A new operator with the tables and cells of ``src`` at angular
        frequency ``omega`` (the HB ingredients do not depend on it; copied
        on the device, only the self terms are evaluated again).  Build it
        before applying."""
        import torch
        self = cls.__new__(cls)
        self._lib = src._lib
        self.device = src.device
        self.dim, self.ncell, self.Nv, self.h = src.dim, src.ncell, src.Nv, src.h
        self.prec = None
        ctx = ctypes.c_void_p()
        st = stream if stream is not None else torch.cuda.current_stream(self.device).cuda_stream
        _lib.check(self._lib.hbi_create(self.device.index, ctypes.c_void_p(st), ctypes.byref(ctx)))
        self._ctx = ctx
        self._keep = []
        self._check(self._lib.hbi_load_tables_from(self._ctx, src._ctx, float(omega)))
        return self

    def set_omega(self, omega: float):
        """Same tables and cells at angular frequency ``omega``; drops the
        factors (build again before applying)."""
        self._check(self._lib.hbi_load_tables_from(self._ctx, self._ctx, float(omega)))
        self.prec = None
        return self

    # -- marshalling helpers -------------------------------------------------
    def _check(self, status):
        _lib.check(status, self._ctx)

    def load(self, p):
        t = _lib.hbi_tables()
        t.dim = self.dim
        for a in range(3):
            t.ncell[a] = int(p.ncell[a]) if a < self.dim else 1
            t.origin[a] = float(p.origin[a]) if a < self.dim else 0.0
            t.nbox[a] = int(p.nbox[a]) if a < self.dim else 1
            t.box_origin[a] = float(p.box_origin[a]) if a < self.dim else 0.0
        t.h = float(p.h)
        t.omega = float(p.omega)
        t.nterms = int(p.nterms)
        t.nI = int(p.nI)
        t.box_size = float(p.box_size)
        arrs = [np.ascontiguousarray(p.tau2, dtype=np.float64),
                np.ascontiguousarray(p.v0, dtype=np.float64),
                None if p.v1 is None else np.ascontiguousarray(p.v1, dtype=np.float64),
                np.ascontiguousarray(p.slowness, dtype=np.float64)]
        # the library reads NT x NT doubles per table and N_v slowness
        # values through these pointers: check the sizes here
        nbox = int(np.prod([t.nbox[a] for a in range(self.dim)]))
        NT = nbox * int(p.nI) ** self.dim
        for name, a in zip(("tau2", "v0", "v1"), arrs[:3]):
            if a is None:
                if name != "v1" or int(p.nterms) != 1:
                    raise ValueError(f"{name} is required")
            elif a.size != NT * NT:
                raise ValueError(f"{name} must hold NT x NT = {NT} x {NT} entries, got {a.shape}")
        if arrs[3].size != self.Nv:
            raise ValueError(f"slowness must hold N_v = {self.Nv} entries, got {arrs[3].size}")
        t.tau2 = _dptr(arrs[0])
        t.v0 = _dptr(arrs[1])
        t.v1 = _dptr(arrs[2]) if arrs[2] is not None else ctypes.POINTER(ctypes.c_double)()
        t.slowness = _dptr(arrs[3])
        self._check(self._lib.hbi_load_tables(self._ctx, ctypes.byref(t)))
        self.prec = None

    def set_inclusion(self, curve=None):
        """A curve inclusion (Sec. 3.2): ``curve`` has ``centres`` (N_s, 2),
        ``w`` (N_s,) and ``slowness`` (N_s,); None removes it.  Drops the
        factors; after the next build, apply / apply_adjoint use the total
        operator (K^{v2v} + K^{s2v} (K^{s2s})^{-1} K^{v2s}) h^d."""
        if curve is None:
            self._check(self._lib.hbi_set_inclusion(self._ctx, 0, None, None, None))
        else:
            xy = np.ascontiguousarray(curve.centres, dtype=np.float64)
            w = np.ascontiguousarray(curve.w, dtype=np.float64)
            n = np.ascontiguousarray(curve.slowness, dtype=np.float64)
            if xy.shape != (w.size, 2) or n.shape != w.shape:
                raise ValueError("curve: centres (N_s, 2), w and slowness (N_s,)")
            self._check(self._lib.hbi_set_inclusion(self._ctx, int(w.size), _dptr(xy), _dptr(w),
                                                    _dptr(n)))
        self.prec = None
        return self

    def set_stream(self, stream=None):
        import torch
        st = stream if stream is not None else torch.cuda.current_stream(self.device).cuda_stream
        self._check(self._lib.hbi_set_stream(self._ctx, ctypes.c_void_p(st)))

    def build(self, tol: float = 1e-7, prec: str = "f64", chi=None, leaf_size=None,
              neighbor_radius=None, band_width=None, workspace_bytes=None):
        o = _lib.hbi_build_opts()
        o.chi = float(chi or 0.0)
        o.leaf_size = int(leaf_size or 0)
        o.neighbor_radius = float(neighbor_radius or 0.0)
        o.band_width = int(band_width or 0)
        o.workspace_bytes = int(workspace_bytes or 0)
        self._check(self._lib.hbi_set_build_opts(self._ctx, ctypes.byref(o)))
        p = {"f64": HBI_F64, "f32": HBI_F32}[prec]
        self.set_stream()
        self._check(self._lib.hbi_build(self._ctx, float(tol), p))
        self.prec = prec
        return self

    @property
    def dtype(self):
        import torch
        return torch.complex128 if self.prec == "f64" else torch.complex64

    def _prep(self, s):
        import torch
        if self.prec is None:
            raise HBIError(_lib.HBI_ERR_STATE, "apply before build")
        if s.device != self.device:
            raise ValueError(f"input on {s.device}, operator on {self.device}")
        if s.dtype != self.dtype:
            raise TypeError(f"expected {self.dtype}, got {s.dtype}")
        vec = s.dim() == 1
        S = s.reshape(self.Nv, -1) if vec else s
        if S.shape[0] != self.Nv:
            raise ValueError(f"expected {self.Nv} rows, got {S.shape[0]}")
        # column-major N_v x nrhs: a row-major (nrhs, N_v) buffer transposed
        if not (S.stride(0) == 1 and (S.shape[1] == 1 or S.stride(1) == self.Nv)):
            S = S.t().contiguous().t()
        return S, vec

    def _run(self, fn, s, out=None):
        import torch
        S, vec = self._prep(s)
        nrhs = S.shape[1]
        ld = S.stride(1) if nrhs > 1 else self.Nv
        U = torch.empty((nrhs, self.Nv), dtype=self.dtype, device=self.device).t() \
            if out is None else _out_view(out, self.Nv, nrhs, ld, self.dtype, self.device, S)
        self.set_stream()
        self._check(fn(self._ctx, ctypes.c_void_p(S.data_ptr()), ctypes.c_void_p(U.data_ptr()),
                       nrhs, ld))
        return U.reshape(-1) if vec else U

    def apply(self, s, out=None):
        """u = K (h^d s) (eq. m_v2v)."""
        return self._run(self._lib.hbi_apply, s, out)

    def apply_adjoint(self, s, out=None):
        """u = h^d K^H s."""
        return self._run(self._lib.hbi_apply_adjoint, s, out)

    def apply_noalloc(self, s, out):
        """u = K (h^d s) through hbi_apply_noalloc: the library allocates
        nothing (its per-level vectors live in a fixed per-device scratch
        array), so the caller gives the output buffer."""
        return self._run(self._lib.hbi_apply_noalloc, s, out)

    def entries(self, rows, cols):
        """K[rows][:, cols] (natural indices) as a complex128 device tensor."""
        import torch
        r = np.ascontiguousarray(rows, dtype=np.int32)
        c = np.ascontiguousarray(cols, dtype=np.int32)
        out = torch.empty((c.size, r.size), dtype=torch.complex128, device=self.device)
        self.set_stream()
        self._check(self._lib.hbi_entries(
            self._ctx, r.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), r.size,
            c.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), c.size,
            ctypes.c_void_p(out.data_ptr())))
        return out.t()

    def info(self) -> dict:
        buf = ctypes.create_string_buffer(16384)
        self._check(self._lib.hbi_get_info(self._ctx, buf, len(buf)))
        return json.loads(buf.value.decode())

    def profile(self, enable: bool):
        """Turn per-kernel event timing of applies on (returns None) or off
        (returns the recorded {"kernels": {name: {launches, ms, bytes}}})."""
        if enable:
            self._check(self._lib.hbi_set_profiling(self._ctx, 1))
            return None
        buf = ctypes.create_string_buffer(1 << 16)
        self._check(self._lib.hbi_get_profile(self._ctx, buf, len(buf)))
        self._check(self._lib.hbi_set_profiling(self._ctx, 0))
        return json.loads(buf.value.decode())

    def close(self):
        if getattr(self, "_ctx", None):
            self._lib.hbi_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _out_view(u, nv, nrhs, ld, dtype, device, s=None):
    """The caller's output buffer `u` as the nv x nrhs column-major view
    (leading dimension ld) that the library writes, or an error: a buffer of
    another type, size or layout would be written outside its bounds or
    scrambled, and a reshaped copy would silently receive the result."""
    if u.dtype != dtype or u.device != device:
        raise ValueError(f"out must be {dtype} on {device}, got {u.dtype} on {u.device}")
    if u.dim() == 1:
        if nrhs != 1 or u.shape[0] != nv or u.stride(0) != 1:
            raise ValueError(f"a 1-D out must hold {nv} contiguous entries for one RHS")
        U = u.view(nv, 1)
    elif u.dim() == 2:
        if tuple(u.shape) != (nv, nrhs):
            raise ValueError(f"out must be {nv} x {nrhs}, got {tuple(u.shape)}")
        if u.stride(0) != 1 or (nrhs > 1 and u.stride(1) != ld):
            raise ValueError(f"out must be column-major with leading dimension {ld}")
        U = u
    else:
        raise ValueError("out must be 1-D or 2-D")
    if s is not None:
        esz = U.element_size()
        a0, a1 = U.data_ptr(), U.data_ptr() + esz * (ld * (nrhs - 1) + nv)
        b0 = s.data_ptr()
        b1 = b0 + esz * ((s.stride(1) if s.dim() == 2 else nv) * (nrhs - 1) + nv)
        if a0 < b1 and b0 < a1:
            raise ValueError("out overlaps the input")
    return U


def _span(t):
    """[first byte, last byte + 1) of a 2-D column-major device view."""
    esz = t.element_size()
    ld = t.stride(1) if t.shape[1] > 1 else t.shape[0]
    return t.data_ptr(), t.data_ptr() + esz * (ld * (t.shape[1] - 1) + t.shape[0])


def _overlaps(a, b):
    return a[0] < b[1] and b[0] < a[1]


def apply_batched(ops, S, out=None):
    """u_p = K_p (h^d s_p) for every operator in `ops` in one library call
    (hbi_apply_batched): all problems' stages share launches and the call is
    replayed from a captured HIP graph.  S[p] is an (N_v,p x nrhs_p) device
    tensor of the operator's dtype; returns column-major outputs."""
    import torch
    lib = _lib.load()
    n = len(ops)
    if n == 0:
        return []
    Sc = [s.reshape(s.shape[0], -1) for s in S]
    Sc = [s if (s.stride(0) == 1 and (s.shape[1] == 1 or s.stride(1) == s.shape[0]))
          else s.t().contiguous().t() for s in Sc]
    for op, s in zip(ops, Sc):
        if s.dtype != op.dtype or s.shape[0] != op.Nv or s.device != op.device:
            raise ValueError("right-hand side does not match its operator")
    if out is not None:
        if len(out) != n:
            raise ValueError(f"out must hold {n} buffers")
        U = [_out_view(u, s.shape[0], s.shape[1], s.shape[0], s.dtype, s.device, s)
             for u, s in zip(out, Sc)]
        # an output may overlap no other problem's input or output either:
        # passes of a large batch run problems at different times
        spans = [_span(x) for x in U]
        ins = [_span(x) for x in Sc]
        for p in range(n):
            for q in range(n):
                if q != p and (_overlaps(spans[p], ins[q]) or _overlaps(spans[p], spans[q])):
                    raise ValueError(f"out[{p}] overlaps the input or output of problem {q}")
    else:
        U = [torch.empty((s.shape[1], s.shape[0]), dtype=s.dtype, device=s.device).t()
             for s in Sc]
    ctxs = (ctypes.c_void_p * n)(*[o._ctx.value for o in ops])
    sp = (ctypes.c_void_p * n)(*[s.data_ptr() for s in Sc])
    up = (ctypes.c_void_p * n)(*[u.data_ptr() for u in U])
    nr = (ctypes.c_int32 * n)(*[s.shape[1] for s in Sc])
    ld = (ctypes.c_int64 * n)(*[s.shape[0] for s in Sc])
    ops[0].set_stream()
    _lib.check(lib.hbi_apply_batched(ctxs, n, sp, up, nr, ld), ops[0]._ctx)
    return U


def tabulate(n2, origin, spacing, taylor, nI, nbox, box_origin, box_size, h0, margin=8,
             device=0, info=False):
    """Tables tau^2, v0, v1 (NT x NT each, the layout of hbi_tables) from the
    eikonal and transport solves on the GPU (hbi_tabulate, 2D).  n2: the
    medium's n^2 on a regular grid, array (nx, ny) indexed [i, j] at
    origin + (i, j) spacing; taylor: (NT, 5, 5) Taylor coefficients of n^2
    about every table node (entry [A, i, j] multiplies (x - x_A)^i
    (y - y_A)^j).  With info=True the solve counters of hbi_get_info
    (tab_sources, tab_rounds_max, tab_point_updates, tab_s) come back as a
    fourth value."""
    import torch
    lib = _lib.load()
    n2 = np.asarray(n2, dtype=np.float64)
    if n2.ndim != 2:
        raise ValueError("n2 must be a 2D grid")
    NT = int(nbox[0]) * int(nbox[1]) * int(nI) ** 2
    tay = np.ascontiguousarray(taylor, dtype=np.float64)
    if tay.shape != (NT, 5, 5):
        raise ValueError(f"taylor must be ({NT}, 5, 5)")
    grid = np.ascontiguousarray(n2.T)          # x fastest
    m = _lib.hbi_medium2d()
    m.n[0], m.n[1] = n2.shape
    m.origin[0], m.origin[1] = float(origin[0]), float(origin[1])
    m.spacing = float(spacing)
    m.n2 = _dptr(grid)
    m.taylor = _dptr(tay)
    out = [np.empty((NT, NT)) for _ in range(3)]
    nb = (ctypes.c_int32 * 2)(int(nbox[0]), int(nbox[1]))
    bo = (ctypes.c_double * 2)(float(box_origin[0]), float(box_origin[1]))
    ctx = ctypes.c_void_p()
    st = torch.cuda.current_stream(torch.device("cuda", device)).cuda_stream
    _lib.check(lib.hbi_create(device, ctypes.c_void_p(st), ctypes.byref(ctx)))
    try:
        _lib.check(lib.hbi_tabulate(ctx, ctypes.byref(m), int(nI), nb, bo, float(box_size),
                                    float(h0), int(margin), *[_dptr(F) for F in out]), ctx)
        if info:
            buf = ctypes.create_string_buffer(1 << 14)
            _lib.check(lib.hbi_get_info(ctx, buf, len(buf)), ctx)
            d = json.loads(buf.value.decode())
            stats = {k: d[k] for k in ("tab_sources", "tab_rounds_max", "tab_point_updates",
                                       "tab_s")}
    finally:
        lib.hbi_destroy(ctx)
    return (*out, stats) if info else tuple(out)


def _autograd_function():
    import torch

    class HBApply(torch.autograd.Function):
        """u = K (h^d s), differentiable in s; backward is the hand-written
        conjugate-transpose apply (grad_s = h^d K^H grad_u)."""

        @staticmethod
        def forward(ctx, op, s):
            ctx.op = op
            return op.apply(s)

        @staticmethod
        def backward(ctx, grad_u):
            return None, ctx.op.apply_adjoint(grad_u.contiguous() if grad_u.dim() == 1 else grad_u)

    return HBApply


class _LazyHBApply:
    _cls = None

    def __getattr__(self, name):
        if _LazyHBApply._cls is None:
            _LazyHBApply._cls = _autograd_function()
        return getattr(_LazyHBApply._cls, name)


HBApply = _LazyHBApply()
