"""Benchmark of the HB integrator apply on one MI355X.

Workload (default): 2D Gaussian-bump medium n = 1 + 0.3 exp(-|r-(1/2,1/2)|^2
/ (2 * 0.1^2)) on the unit square, 1024 x 1024 cells (128 wavelengths at
n = 1, omega = 256 pi), piecewise Chebyshev tables (8 x 8 boxes x 8 x 8
nodes), one seeded complex N(0,1) right-hand side.

Per run:
  1. FP64 build at tol 1e-7 and FP32 build (FP64 QR/ID, factors rounded to
     complex64) at tol 1e-5, the loosest power of ten whose measured error
     stays an order of magnitude inside the metric's 1e-4 bound; build
     seconds are wall time of hbi_build.
  2. Parity: relative L2 error of each apply against the FP64 CPU oracle on
     seeded sampled rows.
  3. Timed applies u = K (h^d s) with the input resident in HBM: W warm-up
     steps, then K timed steps between device synchronisations.  `value`
     is the FP32 apply throughput in Gcell*RHS/s (the metric's rel. error
     bound is 1e-4); the FP64 figures are reported beside it.
  4. Roofline: per-kernel HIP-event durations recorded by the library on
     its stream over a second pass of the same number of applies, right
     after the timed steps (which carry no per-kernel events); algorithmic
     bytes from the factor layout; counted HBM traffic from the committed
     counter record while the kernel source is the one it was taken with.
  5. CPU baseline: the oracle (as is) on a bounded sample of rows on the
     host, scaled to Gcell*RHS/s.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "HB butterfly apply Gcell·RHS/s at rel err ≤1e-4; build s; % HBM/MFMA peak"


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, or None when the kernel source changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "k_wstage_f32_bump1024_traffic.json")
    src = os.path.join(ROOT, "paper_2210_02698_amd", "csrc", "hbi_apply.hip")
    try:
        rec = json.load(open(path))
        cur = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except (OSError, ValueError):
        return None
    if rec.get("kernels_source_sha256") != cur or not rec.get("kernel", "").startswith(kernel):
        return None
    return rec.get("traffic_bytes_per_launch")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n-side", type=int, default=1024)
    ap.add_argument("--tol64", type=float, default=1e-7)
    ap.add_argument("--tol32", type=float, default=None,
                    help="FP32 build tolerance [1e-5 for the 2D workloads, 1e-6 for 3D]")
    ap.add_argument("--chi", type=float, default=0.0, help="proxy oversampling (0 = library default)")
    ap.add_argument("--oracle-rows", type=int, default=24)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--workload", choices=["bump", "batched", "3d", "sweep", "inclusion"],
                    default="bump",
                    help="bump: the headline 1024^2 single-RHS apply; batched: 64 "
                         "constant-gradient problems with 1-256 RHS each; 3d: 64^3 sinusoid "
                         "with 32 RHS; sweep: four frequencies from one table set, 16 RHS "
                         "each; inclusion: 256^2 bump with an open-square curve inclusion")
    ap.add_argument("--nprob", type=int, default=64)
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="run one device copy of this many MiB first (HBM counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "one GPU only: the multi-GPU sharding is designed, not built; run with --gpus 1"}))
        sys.exit(2)
    if args.tol32 is None:
        args.tol32 = 1e-6 if args.workload == "3d" else 1e-5
    if args.workload == "inclusion":
        return run_inclusion(args)
    if args.workload != "bump":
        return run_multi(args)

    import numpy as np
    import torch

    import hb_inputs
    import paper_2210_02698_amd as hbi

    if not os.path.exists(os.path.join(ROOT, "paper_2210_02698_amd", "libhbi.so")):
        from paper_2210_02698_amd import build as _b
        _b.build()

    dev = torch.device("cuda:0")
    if args.calib_copy_mb:
        n = args.calib_copy_mb << 20
        a = torch.empty(n, dtype=torch.uint8, device=dev).fill_(1)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"calibration copy of {n} bytes done")
        del a, b
    t0 = time.time()
    prob = hb_inputs.configs.c2(args.n_side)
    log(f"problem {prob.name}: N_v={prob.Nv} NT={prob.NT} tables {time.time() - t0:.1f}s")
    s_h = hb_inputs.complex_normal(prob.Nv, [hb_inputs.configs.CFG_SEED["c2"], 0])
    rows = np.sort(np.random.default_rng([2, 7]).choice(prob.Nv, args.oracle_rows, replace=False))

    # oracle on the sampled rows: parity reference and CPU baseline
    cpu = None
    ref = None
    if not args.no_cpu:
        import oracle
        try:
            from threadpoolctl import threadpool_limits
            limiter = threadpool_limits(1)
        except Exception:
            limiter = None
        t0 = time.perf_counter()
        ref = oracle.apply(prob, s_h, rows)
        t_or = time.perf_counter() - t0
        if limiter is not None:
            limiter.restore_original_limits()
        cpu = {"value": args.oracle_rows / t_or / 1e9, "unit": "Gcell·RHS/s", "cores": 1,
               "kind": "oracle",
               "sample": f"{args.oracle_rows} seeded rows of the dense FP64 oracle u = K h^d s "
                         f"(each row: {prob.Nv} HB entries from the tables), single thread, "
                         f"{t_or:.1f} s; full-apply time extrapolates to "
                         f"{t_or * prob.Nv / args.oracle_rows / 3600:.1f} h"}
        log(f"oracle {args.oracle_rows} rows in {t_or:.1f}s")

    def timed(op, s):
        for _ in range(args.warmup):
            op.apply(s)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            op.apply(s)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        # per-kernel HIP event timings: the same applies launched kernel by
        # kernel with events between them (the timed loop replays a graph)
        op.profile(True)
        for _ in range(args.steps):
            op.apply(s)
        torch.cuda.synchronize()
        prof = op.profile(False)
        return dt, prof

    results = {}
    for prec, tol in (("f64", args.tol64), ("f32", args.tol32)):
        if prec == "f64" and args.no_fp64:
            continue
        op = hbi.Operator(prob, device=0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        op.build(tol=tol, prec=prec, chi=args.chi or None)
        torch.cuda.synchronize()
        build_s = time.perf_counter() - t0
        info = op.info()
        log(f"{prec} build {build_s:.2f}s info {info}")
        dt = torch.complex128 if prec == "f64" else torch.complex64
        s = torch.from_numpy(s_h).to(dev).to(dt)
        u = op.apply(s)
        torch.cuda.synchronize()
        err = None
        if ref is not None:
            ug = u.cpu().numpy().astype(np.complex128)[rows]
            err = float(np.linalg.norm(ug - ref) / np.linalg.norm(ref))
        t_apply, prof = timed(op, s)
        esz = 16 if prec == "f64" else 8
        # factor entries, and the transfer units' column orders the forward
        # product gathers its inputs through (half of the index store)
        fbytes = info["nnz_total"] * esz + info["index_bytes"] // 2
        vec_bytes = (2 * prob.Nv + 2 * info["z_entries"]) * esz
        results[prec] = dict(build_s=build_s, err=err, ms=t_apply * 1e3, info=info, prof=prof,
                             gcells=prob.Nv / t_apply / 1e9,
                             apply_gbs=(fbytes + vec_bytes) / t_apply / 1e9,
                             factor_bytes=fbytes)
        log(f"{prec} apply {t_apply * 1e3:.3f} ms  err {err}  prof {prof}")
        op.close()
        del op
        torch.cuda.empty_cache()

    head = results["f32"]
    # dominant kernel roofline from the library's per-kernel event timings
    prof = head["prof"]
    dom = max(prof["kernels"], key=lambda k: prof["kernels"][k]["ms"])
    kd = prof["kernels"][dom]
    achieved = kd["bytes"] / (kd["ms"] / kd["launches"] * 1e-3) / kd["launches"] / 1e9
    line = {
        "metric": METRIC,
        "value": round(head["gcells"], 6),
        "unit": "Gcell·RHS/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64 (fp32 factors and accumulation; fp64 phase, weights and QR in the build)",
        "data": "synthetic (seeded inputs; straight-ray stand-in tables)",
        "config": {"workload": f"2D Gaussian-bump medium, {args.n_side}x{args.n_side} cells, "
                               f"omega={2 * args.n_side / 8:.0f}pi, 1 RHS",
                   "N_v": prob.Nv, "nrhs": 1, "tol_fp32_build": args.tol32,
                   "tol_fp64_build": args.tol64, "parallelism": "single GPU"},
        "rel_err_vs_oracle": head["err"],
        "build_s": round(head["build_s"], 3),
        "apply_achieved_GBs": round(head["apply_gbs"], 1),
        "apply_hbm_frac": round(head["apply_gbs"] / HBM_PEAK_GBS, 4),
        "factor_bytes": head["factor_bytes"],
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(dom) if args.n_side == 1024 else None,
                     "algorithmic_bytes_per_launch": round(kd["bytes"] / kd["launches"])},
        "cpu_baseline": cpu,
    }
    if "f64" in results:
        r = results["f64"]
        line["fp64"] = {"value": round(r["gcells"], 6), "ms_per_step": round(r["ms"], 4),
                        "rel_err_vs_oracle": r["err"], "build_s": round(r["build_s"], 3),
                        "apply_achieved_GBs": round(r["apply_gbs"], 1),
                        "factor_bytes": r["factor_bytes"]}
        line["fp32_speedup_over_fp64"] = round(r["ms"] / head["ms"], 3)
    print(json.dumps(line), flush=True)


MFMA_F32_PEAK_TFLOPS = 157.3


def run_multi(args):
    """Many right-hand sides: the batched constant-gradient workload (FP32
    factors at tol 1e-5) or the 3D sinusoid (tol 1e-6), hbi_apply_batched
    under its graph."""
    import numpy as np
    import torch

    import hb_inputs
    import paper_2210_02698_amd as hbi

    dev = torch.device("cuda:0")
    src, t_load, t_copy = None, 0.0, 0.0
    if args.workload == "batched":
        cases = hb_inputs.configs.c3(nprob=args.nprob)
        workload = (f"{len(cases)} 2D constant-gradient problems c(y)=1+g y, N_v in "
                    "{128^2, 256^2, 512^2}, 1-256 Gaussian-source RHS each, nI=13")
    elif args.workload == "sweep":
        # one table set (the HB ingredients do not depend on omega), operators
        # at four frequencies built from it
        import dataclasses
        base = hb_inputs.configs.c4()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        src = hbi.Operator(base, device=0)
        torch.cuda.synchronize()
        t_load = time.perf_counter() - t0
        cases = [(dataclasses.replace(base, omega=base.omega * f), 16,
                  [hb_inputs.configs.CFG_SEED["c4"], 5, i])
                 for i, f in enumerate((0.25, 0.5, 0.75, 1.0))]
        workload = ("frequency sweep from one table set: 2D Gaussian-bump medium, 256x256 cells, "
                    "tables 8x8 boxes x 8x8 nodes, omega = 16pi, 32pi, 48pi, 64pi, 16 RHS each")
    else:
        prob = hb_inputs.configs.c5()
        cases = [(prob, 32, [hb_inputs.configs.CFG_SEED["c5"], 0])]
        workload = "3D sinusoid n=1+0.2 sin2pi x sin2pi y sin2pi z, 64^3 cells, 32 RHS, nI=9"
    ops, S, t_build = [], [], 0.0
    for p, (prob, nrhs, seed) in enumerate(cases):
        if src is not None:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            op = hbi.Operator.at_omega(src, prob.omega)
            torch.cuda.synchronize()
            t_copy += time.perf_counter() - t0
        else:
            op = hbi.Operator(prob, device=0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        op.build(tol=args.tol32, prec="f32")
        torch.cuda.synchronize()
        t_build += time.perf_counter() - t0
        if args.workload == "batched":
            sh = hb_inputs.gaussian_sources(prob, nrhs, seed)
        else:
            sh = np.asfortranarray(hb_inputs.complex_normal((prob.Nv, nrhs), seed).astype(np.complex64))
        ops.append(op)
        S.append(torch.from_numpy(sh).to(dev))
        log(f"problem {p}: {prob.name} N_v={prob.Nv} nrhs={nrhs} build total {t_build:.1f}s "
            f"nnz={op.info()['nnz_total']}")
    U = hbi.apply_batched(ops, S)          # autotune + graph capture
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        hbi.apply_batched(ops, S, out=U)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        hbi.apply_batched(ops, S, out=U)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / args.steps
    cells = sum(c[0].Nv * c[1] for c in cases)
    flops = sum(8.0 * op.info()["nnz_total"] * c[1] for op, c in zip(ops, cases))
    # CPU baseline: the oracle on sampled rows of a few problems, also the
    # parity reference of those rows
    errs, cpu = [], None
    if not args.no_cpu:
        import oracle
        pick = ([0] if len(cases) == 1 else list(range(len(cases))) if src is not None
                else sorted({0, len(cases) // 2, len(cases) - 1}))
        t_or, rows_done = 0.0, 0
        for p in pick:
            prob = cases[p][0]
            rows = np.sort(np.random.default_rng([9, p]).choice(prob.Nv, 8, replace=False))
            sh = S[p].cpu().numpy().astype(np.complex128)
            t1 = time.perf_counter()
            ref = oracle.apply(prob, sh, rows)
            t_or += time.perf_counter() - t1
            rows_done += len(rows) * sh.shape[1]
            got = U[p].cpu().numpy().astype(np.complex128)[rows]
            errs.append(float(np.linalg.norm(got - ref) / np.linalg.norm(ref)))
        cpu = {"value": rows_done / t_or / 1e9, "unit": "Gcell·RHS/s", "cores": 1,
               "kind": "oracle",
               "sample": f"{rows_done} (row, RHS) outputs of the FP64 oracle on "
                         f"problems {pick}, {t_or:.1f} s"}
    achieved = flops / t / 1e12
    line = {
        "metric": METRIC, "value": round(cells / t / 1e9, 6), "unit": "Gcell·RHS/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(t * 1e3, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64 (fp32 factors, MFMA fp32 accumulation; fp64 build)",
        "data": "synthetic (seeded inputs)",
        "config": {"workload": workload, "problems": len(cases),
                   "cell_rhs_total": cells, "tol_fp32_build": args.tol32,
                   "parallelism": "single GPU"},
        "rel_err_vs_oracle_max": max(errs) if errs else None,
        "build_s_total": round(t_build, 2),
        "roofline": {"bound": "mfma", "kernel": "k_wstage_mr/k_vstage_mr/k_final_mr",
                     "achieved": round(achieved, 2), "peak": MFMA_F32_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(achieved / MFMA_F32_PEAK_TFLOPS, 4),
                     "traffic": None},
        "cpu_baseline": cpu,
    }
    if src is not None:
        line["sweep"] = {"omegas_over_pi": [round(c[0].omega / np.pi, 3) for c in cases],
                         "table_load_s": round(t_load, 3),
                         "table_copy_s_mean": round(t_copy / len(cases), 3),
                         "rel_err_vs_oracle_per_omega": errs or None}
        src.close()
    print(json.dumps(line), flush=True)


def run_inclusion(args):
    """Total field with a curve inclusion (eq. m_v2v_inclu): 2D Gaussian bump
    256^2 at omega = 64 pi, an open square of side 0.8 centred in the domain
    (20 segments per shortest wavelength), FP32, one Gaussian source."""
    import numpy as np
    import torch

    import hb_inputs
    import paper_2210_02698_amd as hbi

    dev = torch.device("cuda:0")
    prob = hb_inputs.configs.c4()
    curve = hb_inputs.open_square(prob, (0.5, 0.5), 0.8, 20)
    P = prob.centres()
    r2 = np.sum((P - np.array([0.5, 0.5])) ** 2, axis=1)
    s_h = np.exp(-r2 / (2.0 * (2.0 * prob.h) ** 2)).astype(np.complex128)
    op = hbi.Operator(prob, device=0).set_inclusion(curve)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    op.build(tol=args.tol32, prec="f32")
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    info = op.info()
    log(f"inclusion build {build_s:.2f}s info {info}")
    s = torch.from_numpy(s_h).to(dev).to(torch.complex64)
    u = op.apply(s)
    for _ in range(args.warmup):
        op.apply(s)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        op.apply(s)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / args.steps
    # algorithmic bytes: the volume factors once, G twice (gather and
    # scatter), the K^{s2s} inverse once, the vectors
    vol = info["nnz_total"] * 8 + (2 * prob.Nv + 2 * info["z_entries"]) * 8
    incb = 2 * prob.Nv * curve.Ns * 8 + curve.Ns ** 2 * 8 + 2 * prob.Nv * 8
    achieved = (vol + incb) / t / 1e9
    err, cpu = None, None
    if not args.no_cpu:
        import oracle
        rows = np.sort(np.random.default_rng([11, 1]).choice(prob.Nv, 16, replace=False))
        t1 = time.perf_counter()
        ref = oracle.inclusion.apply(prob, curve, s_h, rows)
        t_or = time.perf_counter() - t1
        got = u.cpu().numpy().astype(np.complex128)[rows]
        err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        cpu = {"value": len(rows) / t_or / 1e9, "unit": "Gcell·RHS/s", "cores": 1,
               "kind": "oracle",
               "sample": f"{len(rows)} rows of the FP64 oracle (volume rows, the full "
                         f"K^{{v2s}} product and the dense K^{{s2s}} solve), {t_or:.1f} s"}
    line = {
        "metric": METRIC, "value": round(prob.Nv / t / 1e9, 6), "unit": "Gcell·RHS/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(t * 1e3, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64 (fp32 factors and dense inclusion operators; fp64 build and inverse)",
        "data": "synthetic (seeded inputs; straight-ray stand-in tables)",
        "config": {"workload": "2D Gaussian-bump medium 256x256, omega=64pi, open-square "
                               f"inclusion side 0.8 ({curve.Ns} segments), 1 RHS",
                   "N_v": prob.Nv, "N_s": curve.Ns, "tol_fp32_build": args.tol32,
                   "parallelism": "single GPU"},
        "rel_err_vs_oracle": err, "build_s": round(build_s, 3),
        "build_inclusion_s": info["build_inclusion_s"],
        "inclusion_bytes": info["inclusion_bytes"],
        "roofline": {"bound": "hbm", "kernel": "whole apply (volume factors + dense inclusion)",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    op.close()


if __name__ == "__main__":
    main()
