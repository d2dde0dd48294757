"""Storage of the HODBF factors against the paper's complexity statement
(Sec. 4.2: storage and apply cost O(N_v log^2 N_v) at a fixed number of
cells per wavelength).

The 2D Gaussian-bump medium at 8 cells per wavelength (omega = 2 pi
N_side / 8) on 64^2 .. 512^2 cells, FP64 factors at tol 1e-7.  Checked:
  * nnz / (N_v log2^2 N_v) stays within a factor 1.6 of its geometric mean
    over the sizes (a dense or N_v^{3/2} store would grow by 4-8x per step);
  * nnz / N_v grows from one size to the next by no more than twice the
    log^2 ratio (log2 N_2 / log2 N_1)^2 (at most 1.7 for 4x the cells);
  * the reported per-cell figures are nnz_total / N_v.
"""
import math

import numpy as np
import pytest

import hb_inputs
from _hbi_util import ensure_built, requires_gpu

pytestmark = [pytest.mark.gpu, requires_gpu]


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


def test_storage_grows_like_n_log2_n():
    ensure_built()
    import paper_2210_02698_amd as hbi
    rows = []
    for side in (64, 128, 256, 512):
        prob = hb_inputs.configs.c2(side, nbox=min(8, side // 16))
        op = hbi.Operator(prob, device=0).build(tol=1e-7, prec="f64")
        info = op.info()
        op.close()
        n, nnz = prob.Nv, info["nnz_total"]
        assert abs(info["nnz_per_cell"] - nnz / n) <= 1e-3 * nnz / n
        norm = nnz / n / math.log2(n) ** 2
        assert abs(info["nnz_per_cell_over_log2sq"] - norm) <= 1e-4 * norm
        q = info["wstage_c_quantiles"]
        assert all(a <= b for a, b in zip(q, q[1:])) and 0 < q[0] and q[-1] <= 4096, q
        say(f"{side}^2: nnz/N_v {nnz / n:.1f}, /log2^2 {norm:.3f}, build {info['build_s']:.2f}s")
        rows.append((n, nnz / n, norm))
    norms = np.array([r[2] for r in rows])
    gm = math.exp(np.mean(np.log(norms)))
    assert norms.max() / gm < 1.6 and gm / norms.min() < 1.6, norms
    for (n1, p1, _), (n2, p2, _) in zip(rows, rows[1:]):
        assert p2 / p1 <= 2.0 * (math.log2(n2) / math.log2(n1)) ** 2, (n1, n2, p1, p2)
