"""Checks of the Python binding that need no GPU: the caller's output
buffers are accepted only as the column-major views the library writes."""
import pytest
import torch

from paper_2210_02698_amd import _out_view

CPU = torch.device("cpu")
NV, NR = 10, 3


def colmajor(nv, nr, dtype=torch.complex64):
    return torch.empty((nr, nv), dtype=dtype).t()


def test_column_major_buffer_is_used_in_place():
    u = colmajor(NV, NR)
    v = _out_view(u, NV, NR, NV, torch.complex64, CPU)
    assert v.data_ptr() == u.data_ptr() and v.stride() == (1, NV)
    one = torch.empty(NV, dtype=torch.complex64)
    w = _out_view(one, NV, 1, NV, torch.complex64, CPU)
    assert w.shape == (NV, 1) and w.data_ptr() == one.data_ptr()


@pytest.mark.parametrize("bad", [
    lambda: torch.empty((NV, NR), dtype=torch.complex64),          # row-major
    lambda: colmajor(NV, NR - 1),                                  # too few columns
    lambda: colmajor(NV - 1, NR),                                  # too few rows
    lambda: colmajor(NV, NR, torch.complex128),                    # other type
    lambda: torch.empty(NV * NR, dtype=torch.complex64),           # 1-D, several RHS
    lambda: colmajor(NV + 2, NR)[:NV],                             # leading dim NV + 2
    lambda: torch.empty((2, NV, NR), dtype=torch.complex64),       # 3-D
])
def test_other_buffers_are_rejected(bad):
    with pytest.raises(ValueError):
        _out_view(bad(), NV, NR, NV, torch.complex64, CPU)


def test_strided_vector_is_rejected():
    u = torch.empty(2 * NV, dtype=torch.complex64)[::2]
    with pytest.raises(ValueError):
        _out_view(u, NV, 1, NV, torch.complex64, CPU)


def test_overlap_with_the_input_is_rejected():
    s = colmajor(NV, NR)
    with pytest.raises(ValueError, match="overlaps"):
        _out_view(s, NV, NR, NV, torch.complex64, CPU, s)
    big = torch.empty((2 * NR, NV), dtype=torch.complex64)
    s2, u2 = big[:NR].t(), big[NR:].t()        # adjacent, disjoint
    assert _out_view(u2, NV, NR, NV, torch.complex64, CPU, s2).data_ptr() == u2.data_ptr()
    with pytest.raises(ValueError, match="overlaps"):
        _out_view(big[NR - 1:2 * NR - 1].t(), NV, NR, NV, torch.complex64, CPU, s2)


class _FakeOp:
    """Stands in for an Operator in the checks that run before any library
    call (no device needed)."""

    def __init__(self, nv, dtype=torch.complex64):
        self.Nv, self.dtype, self.device = nv, dtype, CPU


def test_batched_output_overlapping_another_problem_is_rejected():
    import paper_2210_02698_amd as hbi
    ops = [_FakeOp(NV), _FakeOp(NV)]
    buf = torch.empty((4 * NR, NV), dtype=torch.complex64)
    s0, s1 = buf[0:NR].t(), buf[NR:2 * NR].t()
    u0, u1 = buf[2 * NR:3 * NR].t(), buf[3 * NR:].t()
    with pytest.raises(ValueError, match="overlaps the input or output of problem 1"):
        hbi.apply_batched(ops, [s0, s1], out=[s1, u1])       # out[0] is problem 1's input
    with pytest.raises(ValueError, match=r"out\[0\] overlaps the input or output of problem 1"):
        hbi.apply_batched(ops, [s0, s1], out=[u0, u0])       # two outputs share memory


def _table_problem(nI=3, nbox=(1, 1), ncell=(4, 4), nterms=2, bad=None):
    import types
    import numpy as np
    NT = int(np.prod(nbox)) * nI ** 2
    p = types.SimpleNamespace(dim=2, ncell=ncell, origin=(0.0, 0.0), h=0.25, omega=1.0,
                              nterms=nterms, nI=nI, nbox=nbox, box_origin=(0.0, 0.0),
                              box_size=1.0, tau2=np.zeros((NT, NT)), v0=np.zeros((NT, NT)),
                              v1=np.zeros((NT, NT)), slowness=np.ones(ncell[0] * ncell[1]))
    if bad == "tau2":
        p.tau2 = np.zeros((NT, NT - 1))
    elif bad == "v1":
        p.v1 = None
    elif bad == "slowness":
        p.slowness = np.ones(ncell[0] * ncell[1] - 1)
    return p


@pytest.mark.parametrize("bad", ["tau2", "v1", "slowness"])
def test_missized_tables_are_rejected_before_the_library_reads_them(bad):
    from paper_2210_02698_amd import Operator
    op = Operator.__new__(Operator)        # no device context: the check comes first
    op.dim, op.Nv = 2, 16
    op._lib = None
    with pytest.raises(ValueError):
        op.load(_table_problem(bad=bad))
