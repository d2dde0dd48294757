"""Error measures shared by the GPU parity tests.

rel_l2(got, ref)     ||got - ref||_2 / ||ref||_2 over all rows and RHS.
row_max(got, ref)    max_i |got_i - ref_i| / rms(ref), per RHS column, the
                     largest over columns: an error confined to a few rows
                     (one unit of one transfer stage, say) is diluted in the
                     L2 figure of a long vector but not here.
ROW_FACTOR           how much larger than the L2 bound the row figure may be
                     (the largest of N Gaussian-like residuals is about
                     sqrt(2 ln N) ~ 4-5 times their rms at the sizes used).
"""
import numpy as np

ROW_FACTOR = 20.0


def rel_l2(got, ref):
    got = np.asarray(got, np.complex128)
    ref = np.asarray(ref, np.complex128)
    return float(np.linalg.norm(got - ref) / np.linalg.norm(ref))


def row_max(got, ref):
    got = np.asarray(got, np.complex128)
    ref = np.asarray(ref, np.complex128)
    if ref.ndim == 1:
        got, ref = got[:, None], ref[:, None]
    rms = np.sqrt(np.mean(np.abs(ref) ** 2, axis=0))
    return float(np.max(np.abs(got - ref).max(axis=0) / rms))


def check(got, ref, bound, what=""):
    """Assert the L2 bound and the per-row bound; returns both figures."""
    e, m = rel_l2(got, ref), row_max(got, ref)
    print(f"[gpu-case] {what} rel L2 {e:.3e} row max {m:.3e} (bound {bound:.1e})", flush=True)
    assert e < bound, (what, e)
    assert m < ROW_FACTOR * bound, (what, m)
    return e, m
