"""GPU tables from the eikonal and transport solves (hbi_tabulate) against the
table oracle (oracle.hb_tables), and the integrator built on them.

  * homogeneous medium: the sweeps' exact fixed point, so the tables equal
    n^2 |r - r0|^2, 1/(2 sqrt(pi)) and 0 to rounding;
  * constant gradient, nI = 5, h0 = 1/32: every entry of the three tables
    agrees with the oracle's (same discrete equations, Gauss-Seidel in
    another order, n^2 interpolated from a grid of spacing h0/4) to 1e-8 of
    the table's largest entry, and with the closed-form table within the
    grid error;
  * the paper's 2D sinusoidal medium (Sec. 5.1.1), nI = 6, h0 = 1/32: the
    same comparison with the oracle, then tables -> hbi_load_tables -> build
    -> apply, against the FP64 oracle product on the same tables.
"""
import math

import numpy as np
import pytest

import hb_inputs
import oracle
from oracle import hb_tables as ht
from _hbi_util import ensure_built, requires_gpu
from _parity import check

pytestmark = [pytest.mark.gpu, requires_gpu]


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


def gpu_tables(med, nI, nbox, box_origin, box_size, h0, margin=8):
    ensure_built()
    import paper_2210_02698_amd as hbi
    lo = box_origin
    hi = (box_origin[0] + nbox[0] * box_size, box_origin[1] + nbox[1] * box_size)
    n2, org, sp = hb_inputs.medium_grid(med, lo, hi, h0 / 4, pad=4 * (margin + 4))
    P = hb_inputs.node_coords(2, nI, nbox, box_origin, box_size)
    return hbi.tabulate(n2, org, sp, hb_inputs.taylor_at(med, P), nI, nbox, box_origin,
                        box_size, h0, margin)


def oracle_tables(med, nI, nbox, box_origin, box_size, h0, margin=8):
    return ht.tables(med.slowness, lambda r: hb_inputs.n2_taylor(med, r), nI, nbox, box_origin,
                     box_size, h0, margin)


def test_homogeneous_tables_are_exact():
    med = hb_inputs.Homogeneous(1.2)
    say("tabulate homogeneous nI=4")
    t2, a0, a1 = gpu_tables(med, 4, (1, 1), (0.0, 0.0), 1.0, 1 / 16)
    e2, e0, e1 = hb_inputs.tabulate(med, 2, 4, (1, 1), (0.0, 0.0), 1.0)
    assert np.abs(t2 - e2).max() < 1e-12
    assert np.abs(a0 - e0).max() < 1e-13
    assert np.abs(a1).max() < 1e-12


@pytest.mark.parametrize("name", ["constant-gradient", "sinusoid-2d"])
def test_tables_match_oracle(name):
    med = (hb_inputs.ConstantGradient(1.0, (0.0, 0.7)) if name == "constant-gradient"
           else hb_inputs.Sinusoid2D())
    nI = 5 if name == "constant-gradient" else 6
    say(f"tabulate {name} nI={nI} h0=1/32")
    got = gpu_tables(med, nI, (1, 1), (0.0, 0.0), 1.0, 1 / 32)
    ref = oracle_tables(med, nI, (1, 1), (0.0, 0.0), 1.0, 1 / 32)
    for label, g, r in zip(("tau2", "v0", "v1"), got, ref):
        e = np.abs(g - r).max() / np.abs(r).max()
        say(f"{name} {label}: max |gpu - oracle| / max|oracle| = {e:.2e}")
        assert e < 1e-8, (label, e)
        assert np.array_equal(g, g.T)
    if name == "constant-gradient":
        e2, e0, e1 = hb_inputs.tabulate(med, 2, nI, (1, 1), (0.0, 0.0), 1.0)
        assert np.abs(got[0] - e2).max() < 2e-5 and np.abs(got[1] - e0).max() < 1e-3
        assert np.abs(got[2] - e1).max() < 3e-2


def test_integrator_on_solved_tables():
    """Tables of the sinusoidal medium from hbi_tabulate, loaded into an
    operator on 64^2 cells (omega = 16 pi), built and applied: the product
    matches the FP64 oracle on the same tables."""
    torch = pytest.importorskip("torch")
    import paper_2210_02698_amd as hbi
    med = hb_inputs.Sinusoid2D()
    nI = 6
    t2, a0, a1 = gpu_tables(med, nI, (1, 1), (0.0, 0.0), 1.0, 1 / 32)
    prob = hb_inputs.make_problem(med, 2, (64, 64), 2 * math.pi * 8, nI=nI,
                                  name="sinusoid-2d-solved-tables")
    prob.tau2, prob.v0, prob.v1 = t2, a0, a1
    say(f"integrator on solved tables Nv={prob.Nv}")
    op = hbi.Operator(prob, device=0).build(tol=1e-7, prec="f64")
    s = hb_inputs.complex_normal(prob.Nv, [91, 0])
    u = op.apply(torch.from_numpy(s).to("cuda:0")).cpu().numpy()
    rows = np.sort(np.random.default_rng([91, 1]).choice(prob.Nv, 128, replace=False))
    check(u[rows], oracle.apply(prob, s, rows), 1e-6, "product on solved tables")
    op.close()


def test_tables_of_several_boxes_match_oracle():
    """Piecewise tables: 2 x 1 boxes of nI = 4 nodes on [0, 2] x [0, 1]
    (constant gradient, h0 = 1/16); every source's grid covers both boxes,
    and the table layout (box-major, node k1 + nI k2) matches the oracle's."""
    med = hb_inputs.ConstantGradient(1.0, (0.0, 0.7))
    say("tabulate constant-gradient 2x1 boxes nI=4 h0=1/16")
    got = gpu_tables(med, 4, (2, 1), (0.0, 0.0), 1.0, 1 / 16)
    ref = oracle_tables(med, 4, (2, 1), (0.0, 0.0), 1.0, 1 / 16)
    for label, g, r in zip(("tau2", "v0", "v1"), got, ref):
        assert g.shape == (32, 32)
        e = np.abs(g - r).max() / np.abs(r).max()
        say(f"2x1 boxes {label}: max |gpu - oracle| / max|oracle| = {e:.2e}")
        assert e < 1e-8, (label, e)


def test_tabulate_rejects_bad_arguments():
    """Argument errors come back as HBI_ERR_ARG before any solve: a node
    count outside 2..16, a margin below 4, a medium grid that does not cover
    the source grids, and n^2 <= 0 at a node."""
    import paper_2210_02698_amd as hbi
    ensure_built()
    med = hb_inputs.Homogeneous(1.0)
    n2, org, sp = hb_inputs.medium_grid(med, (0.0, 0.0), (1.0, 1.0), 1 / 64, pad=4 * 12)
    P = hb_inputs.node_coords(2, 3, (1, 1), (0.0, 0.0), 1.0)
    tay = hb_inputs.taylor_at(med, P)

    def run(nI=3, taylor=tay, n2=n2, margin=8, h0=1 / 16):
        return hbi.tabulate(n2, org, sp, taylor, nI, (1, 1), (0.0, 0.0), 1.0, h0, margin)

    run()   # the valid call
    with pytest.raises(hbi.HBIError, match="nI must be in 2..16"):
        run(nI=1, taylor=tay[:1])
    with pytest.raises(hbi.HBIError, match="bad nbox, box_size, h0 or margin"):
        run(margin=3)
    with pytest.raises(hbi.HBIError, match="does not cover the source grids"):
        run(n2=n2[40:-40, 40:-40])
    bad = tay.copy()
    bad[4, 0, 0] = -1.0
    with pytest.raises(hbi.HBIError, match="n\\^2 must be positive"):
        run(taylor=bad)
