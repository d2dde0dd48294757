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
