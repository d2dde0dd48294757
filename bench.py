"""Benchmark of the HB integrator apply on one MI355X.

Default run (`python bench.py`), one JSON line:
  * headline: 2D Gaussian-bump medium n = 1 + 0.3 exp(-|r-(1/2,1/2)|^2 /
    (2 * 0.1^2)) on the unit square, 1024 x 1024 cells (128 wavelengths at
    n = 1, omega = 256 pi), piecewise Chebyshev tables (8 x 8 boxes x 8 x 8
    nodes), one seeded complex N(0,1) right-hand side.  FP64 factors at tol
    1e-7 and FP32 factors (FP64 build, rounded) at tol 1e-5; `value` is the
    FP32 apply in Gcell*RHS/s, the FP64 figures are reported beside it, and
    the conjugate-transpose product (hbi_apply_adjoint) of both is timed the
    same way and checked against the oracle's h^d K^H s on 128 columns.
  * "batched": 64 constant-gradient problems c(y) = 1 + g y of 128^2, 256^2
    or 512^2 cells with 1-256 Gaussian-source RHS each, FP32, one batched
    call (MFMA tiles, replayed HIP graph).
  * "3d": 3D sinusoid n = 1 + 0.2 sin 2pi x sin 2pi y sin 2pi z on 64^3
    cells, 32 RHS, FP32 factors at tol 1e-6, MFMA tiles.
  * "gradient": inverse-source gradient steps on the 256^2 bump (512
    receivers; forward apply, loss, backward through hbi_apply_adjoint),
    FP32 and FP64, each gradient against the dense FP64 oracle's.
  * "tables": the tau^2, v0, v1 tables of the paper's 2D sinusoidal medium
    (13 x 13 Chebyshev nodes, h0 = 0.01) from the eikonal and transport
    solves (hbi_tabulate), in source nodes per second.

Each workload: build seconds (wall time of hbi_build), the relative L2
error against the FP64 CPU oracle on seeded rows (and the worst row), W
warm-up and K timed applies with the inputs resident in HBM between device
synchronisations, and a roofline of the dominant kernel (HBM bytes for the
single-RHS apply, MFMA flops for the many-RHS ones).

CPU baseline: the oracle, as it is, on the host's cores before any GPU work
(a forked process pool, one BLAS thread per worker, at most 16 workers);
the rows it computes are the parity references.  Also the C1 workload
(2D homogeneous, 64^2 cells) as a full dense oracle apply and as a
stored-dense K @ s product on all workers' cores.

--workload picks one workload alone (bump, batched, 3d, tables, sweep, inclusion), or
the complexity sweep (storage and build time over sizes).
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
MFMA_F32_PEAK_TFLOPS = 157.3
METRIC = "HB butterfly apply Gcell·RHS/s at rel err ≤1e-4; build s; % HBM/MFMA peak"
MAX_WORKERS = 16


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


# ---------------------------------------------------------------------------
# CPU phase: the oracle on a process pool (fork, before any GPU work)
# ---------------------------------------------------------------------------
_JOBS = {}   # key -> (problem, rhs matrix); inherited by the forked workers


def _worker_init():
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except Exception:
        pass


def _oracle_task(args):
    key, rows = args
    import oracle
    prob, S = _JOBS[key]
    return key, rows, oracle.apply(prob, S, rows)


def _oracle_adj_task(args):
    key, rows = args
    import oracle
    prob, S = _JOBS[key]
    return key, rows, oracle.apply_adjoint(prob, S, rows)


def _table_task(args):
    key, rows = args
    import numpy as np
    import hb_inputs
    from oracle import hb_tables as ht
    med, P, h0, lo, hi = _JOBS[key]
    out = []
    for b in rows:
        r = ht.solve_source(med.slowness, hb_inputs.n2_taylor(med, P[b]), P[b], lo, hi, h0)
        out.append(float(sum(r[5])))
    return key, rows, np.array(out)


def _dense_task(args):
    key, rows = args
    import numpy as np
    import oracle
    prob, _ = _JOBS[key]
    return key, rows, oracle.entries(prob, rows, np.arange(prob.Nv))


def cpu_info():
    n_aff = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "affinity": n_aff, "model": model,
            "workers": max(1, min(MAX_WORKERS, n_aff or 1))}


def run_pool(tasks, fn, workers):
    """tasks: list of (key, rows); returns {key: (rows, result)} concatenated
    in task order, and the wall time."""
    import multiprocessing as mp
    import numpy as np
    out = {}
    t0 = time.perf_counter()
    ctx = mp.get_context("fork")
    with ctx.Pool(workers, initializer=_worker_init) as pool:
        for key, rows, res in pool.imap(fn, tasks):
            out.setdefault(key, []).append((rows, res))
    dt = time.perf_counter() - t0
    merged = {}
    for key, parts in out.items():
        merged[key] = (np.concatenate([p[0] for p in parts]),
                       np.concatenate([p[1] for p in parts]))
    return merged, dt


def split_rows(key, rows, per):
    return [(key, rows[a:a + per]) for a in range(0, len(rows), per)]


# ---------------------------------------------------------------------------
# GPU helpers
# ---------------------------------------------------------------------------
def rel_err(got, ref):
    import numpy as np
    got = np.asarray(got, np.complex128)
    ref = np.asarray(ref, np.complex128)
    e = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    g2 = got if got.ndim == 2 else got[:, None]
    r2 = ref if ref.ndim == 2 else ref[:, None]
    rms = np.sqrt(np.mean(np.abs(r2) ** 2, axis=0))
    row = float(np.max(np.abs(g2 - r2).max(axis=0) / rms))
    return e, row


def ensure_lib():
    if not os.path.exists(os.path.join(ROOT, "paper_2210_02698_amd", "libhbi.so")):
        from paper_2210_02698_amd import build as _b
        _b.build()


def timed_single(op, s, steps, warmup):
    import torch
    for _ in range(warmup):
        op.apply(s)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        op.apply(s)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    # per-kernel HIP event timings: a second pass of the same applies with
    # the library's events around every kernel (the timed steps carry none)
    op.profile(True)
    for _ in range(steps):
        op.apply(s)
    torch.cuda.synchronize()
    return dt, op.profile(False)


def timed_batched(ops, S, steps, warmup):
    import torch
    import paper_2210_02698_amd as hbi
    U = hbi.apply_batched(ops, S)          # autotune + graph capture
    torch.cuda.synchronize()
    for _ in range(warmup):
        hbi.apply_batched(ops, S, out=U)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        hbi.apply_batched(ops, S, out=U)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps, U


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------
def prepare_bump(args):
    import numpy as np
    import hb_inputs
    t0 = time.time()
    prob = hb_inputs.configs.c2(args.n_side)
    log(f"bump: N_v={prob.Nv} NT={prob.NT} tables {time.time() - t0:.1f}s")
    s_h = hb_inputs.complex_normal(prob.Nv, [hb_inputs.configs.CFG_SEED["c2"], 0])
    rows = np.sort(np.random.default_rng([2, 7]).choice(prob.Nv, args.bump_rows, replace=False))
    _JOBS["bump"] = (prob, s_h)
    return dict(prob=prob, s=s_h, rows=rows)


def prepare_batched(args):
    import numpy as np
    import hb_inputs
    t0 = time.time()
    cases = hb_inputs.configs.c3(nprob=args.nprob)
    S, rows = [], []
    for p, (prob, nrhs, seed) in enumerate(cases):
        sh = hb_inputs.gaussian_sources(prob, nrhs, seed)
        S.append(sh)
        rows.append(np.sort(np.random.default_rng([9, p]).choice(prob.Nv, args.batched_rows,
                                                                 replace=False)))
        _JOBS[f"batched{p}"] = (prob, sh.astype(np.complex128))
    log(f"batched: {len(cases)} problems, tables and RHS {time.time() - t0:.1f}s")
    return dict(cases=cases, S=S, rows=rows)


def prepare_3d(args):
    import numpy as np
    import hb_inputs
    t0 = time.time()
    prob = hb_inputs.configs.c5(args.n_side_3d)
    nrhs = 32
    sh = np.asfortranarray(hb_inputs.complex_normal(
        (prob.Nv, nrhs), [hb_inputs.configs.CFG_SEED["c5"], 0]).astype(np.complex64))
    rows = np.sort(np.random.default_rng([5, 7]).choice(prob.Nv, args.rows_3d, replace=False))
    _JOBS["3d"] = (prob, sh.astype(np.complex128))
    log(f"3d: N_v={prob.Nv} tables {time.time() - t0:.1f}s")
    return dict(prob=prob, S=sh, rows=rows, nrhs=nrhs)


def prepare_c1():
    import hb_inputs
    prob = hb_inputs.configs.c1()
    s_h = hb_inputs.complex_normal(prob.Nv, [hb_inputs.configs.CFG_SEED["c1"], 0])
    _JOBS["c1"] = (prob, s_h)
    return dict(prob=prob, s=s_h)


def cpu_phase(work, args):
    """Oracle rows of every workload on the pool; C1 dense baselines."""
    import numpy as np
    info = cpu_info()
    W = info["workers"]
    refs = {}
    base = {}
    if "bump" in work:
        w = work["bump"]
        res, dt = run_pool(split_rows("bump", w["rows"], 4), _oracle_task, W)
        refs["bump"] = res["bump"][1]
        n = len(w["rows"])
        base["bump"] = {"value": n / dt / 1e9, "unit": "Gcell·RHS/s", "cores": W,
                        "kind": "oracle",
                        "sample": f"{n} seeded rows of the dense FP64 oracle u = K h^d s "
                                  f"(each row: {w['prob'].Nv} HB entries from the tables), "
                                  f"{W} worker processes, {dt:.1f} s wall; the full apply "
                                  f"extrapolates to {dt * w['prob'].Nv / n / 3600:.2f} h",
                        "cpu": info}
        log(f"cpu: bump {n} rows on {W} workers in {dt:.1f}s")
        ra = w["rows"][::4]
        res, dta = run_pool(split_rows("bump", ra, 4), _oracle_adj_task, W)
        refs["bump_adj"] = res["bump"][1]
        log(f"cpu: bump adjoint {len(ra)} columns in {dta:.1f}s")
    if "batched" in work:
        w = work["batched"]
        tasks = []
        for p, r in enumerate(w["rows"]):
            tasks += split_rows(f"batched{p}", r, len(r))
        res, dt = run_pool(tasks, _oracle_task, W)
        refs["batched"] = [res[f"batched{p}"][1] for p in range(len(w["rows"]))]
        outs = sum(len(r) * c[1] for r, c in zip(w["rows"], w["cases"]))
        base["batched"] = {"value": outs / dt / 1e9, "unit": "Gcell·RHS/s", "cores": W,
                           "kind": "oracle",
                           "sample": f"{args.batched_rows} seeded rows x all RHS of each of the "
                                     f"{len(w['rows'])} problems ({outs} outputs), {W} worker "
                                     f"processes, {dt:.1f} s wall", "cpu": info}
        log(f"cpu: batched {outs} outputs in {dt:.1f}s")
    if "3d" in work:
        w = work["3d"]
        res, dt = run_pool(split_rows("3d", w["rows"], 8), _oracle_task, W)
        refs["3d"] = res["3d"][1]
        outs = len(w["rows"]) * w["nrhs"]
        base["3d"] = {"value": outs / dt / 1e9, "unit": "Gcell·RHS/s", "cores": W,
                      "kind": "oracle",
                      "sample": f"{len(w['rows'])} seeded rows x {w['nrhs']} RHS of the dense "
                                f"FP64 oracle, {W} worker processes, {dt:.1f} s wall",
                      "cpu": info}
        log(f"cpu: 3d {outs} outputs in {dt:.1f}s")
    if "grad" in work:
        w = work["grad"]
        prob = w["prob"]
        hd = prob.h ** prob.dim
        t0 = time.perf_counter()
        res, _ = run_pool(split_rows("grad", w["P"], 32), _dense_task, W)
        KP = res["grad"][1]
        d = KP @ (w["s_true"] * hd)
        r = KP @ (w["s0"] * hd) - d
        g = 2 * hd * (KP.conj().T @ r)
        dt = time.perf_counter() - t0
        refs["grad"] = {"d": d, "grad": g}
        base["grad"] = {"value": prob.Nv / dt / 1e9, "unit": "Gcell/s (gradient steps)",
                        "cores": W, "kind": "oracle",
                        "sample": f"one full gradient: the {len(w['P'])} receiver rows of K by "
                                  f"the dense FP64 oracle on {W} worker processes, then "
                                  f"K[P] h^d s - d and 2 h^d K[P]^H r, {dt:.1f} s wall",
                        "cpu": info}
        log(f"cpu: gradient in {dt:.1f}s")
    if "tables" in work:
        w = work["tables"]
        res, dt = run_pool(split_rows("tables", w["sample"], 1), _table_task, W)
        n = len(w["sample"])
        base["tables"] = {"value": n / dt, "unit": "sources/s", "cores": min(W, n),
                          "kind": "oracle",
                          "sample": f"{n} seeded source nodes of the 169, each solved by the "
                                    f"table oracle (C sweeps, one thread per source), "
                                    f"{min(W, n)} worker processes, {dt:.1f} s wall",
                          "cpu": info}
        log(f"cpu: tables {n} sources in {dt:.1f}s")
    if "c1" in work:
        w = work["c1"]
        prob = w["prob"]
        allr = np.arange(prob.Nv)
        res, dt = run_pool(split_rows("c1", allr, 256), _oracle_task, W)
        # stored dense: K assembled once (untimed), then K @ (h^d s) on the
        # BLAS threads of this process
        resK, dtK = run_pool(split_rows("c1", allr, 256), _dense_task, W)
        K = resK["c1"][1]
        hd = prob.h ** prob.dim
        try:
            from threadpoolctl import threadpool_limits
            lim = threadpool_limits(W)
        except Exception:
            lim = None
        reps = 20
        t0 = time.perf_counter()
        for _ in range(reps):
            u = K @ (w["s"] * hd)
        dtm = (time.perf_counter() - t0) / reps
        if lim is not None:
            lim.restore_original_limits()
        err = float(np.linalg.norm(u - res["c1"][1]) / np.linalg.norm(res["c1"][1]))
        base["c1"] = {"oracle_full_apply": {"value": prob.Nv / dt / 1e9, "unit": "Gcell·RHS/s",
                                            "seconds": round(dt, 3), "cores": W},
                      "stored_dense_matvec": {"value": prob.Nv / dtm / 1e9,
                                              "unit": "Gcell·RHS/s",
                                              "seconds": dtm, "threads": W,
                                              "assembly_s": round(dtK, 3),
                                              "rel_diff_vs_oracle": err},
                      "workload": "2D homogeneous n=1, 64x64 cells, omega=16pi, nI=3, 1 RHS",
                      "cpu": info}
        refs["c1"] = res["c1"][1]
        log(f"cpu: c1 full oracle {dt:.2f}s, stored dense K@s {dtm * 1e3:.3f} ms")
    return refs, base


def gpu_bump(args, w, ref, cpu, ref_adj=None):
    import numpy as np
    import torch
    import paper_2210_02698_amd as hbi
    dev = torch.device("cuda:0")
    prob, rows = w["prob"], w["rows"]
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
        log(f"bump {prec} build {build_s:.2f}s info {info}")
        dt = torch.complex128 if prec == "f64" else torch.complex64
        s = torch.from_numpy(w["s"]).to(dev).to(dt)
        u = op.apply(s)
        torch.cuda.synchronize()
        err = row = None
        if ref is not None:
            err, row = rel_err(u.cpu().numpy()[rows], ref)
        t_apply, prof = timed_single(op, s, args.steps, args.warmup)
        # the conjugate-transpose product (bf_adjoint): same factors, same
        # bytes, gathers only; checked against the oracle's h^d K^H s
        ua = op.apply_adjoint(s)
        torch.cuda.synchronize()
        aerr = arow = None
        if ref_adj is not None:
            aerr, arow = rel_err(ua.cpu().numpy()[rows[::4]], ref_adj)
        for _ in range(args.warmup):
            op.apply_adjoint(s)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            op.apply_adjoint(s)
        torch.cuda.synchronize()
        t_adj = (time.perf_counter() - t0) / args.steps
        log(f"bump {prec} adjoint {t_adj * 1e3:.3f} ms err {aerr} row {arow}")
        esz = 16 if prec == "f64" else 8
        # algorithmic bytes of one product (from the factor layout): factor
        # entries, vectors read and written, index lists and descriptors
        results[prec] = dict(build_s=build_s, err=err, row=row, ms=t_apply * 1e3, info=info,
                             prof=prof, gcells=prob.Nv / t_apply / 1e9,
                             apply_gbs=info["apply_bytes"] / t_apply / 1e9,
                             factor_bytes=info["nnz_total"] * esz,
                             adj={"value": round(prob.Nv / t_adj / 1e9, 6),
                                  "ms_per_step": round(t_adj * 1e3, 4),
                                  "apply_achieved_GBs": round(info["apply_bytes"] / t_adj / 1e9, 1),
                                  "rel_err_vs_oracle": aerr, "row_max_err_vs_oracle": arow})
        log(f"bump {prec} apply {t_apply * 1e3:.3f} ms err {err} row {row} prof {prof}")
        op.close()
        del op
        torch.cuda.empty_cache()
    head = results["f32"]
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
                   "tol_fp64_build": args.tol64, "oracle_rows": len(rows),
                   "parallelism": "single GPU"},
        "rel_err_vs_oracle": head["err"],
        "row_max_err_vs_oracle": head["row"],
        "build_s": round(head["build_s"], 3),
        "apply_achieved_GBs": round(head["apply_gbs"], 1),
        "apply_hbm_frac": round(head["apply_gbs"] / HBM_PEAK_GBS, 4),
        "factor_bytes": head["factor_bytes"],
        "kernels_ms_per_apply": {k: round(v["ms"] / v["launches"] * (
            v["launches"] / args.steps), 4) for k, v in prof["kernels"].items()},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(dom) if args.n_side == 1024 else None,
                     "algorithmic_bytes_per_launch": round(kd["bytes"] / kd["launches"])},
        "cpu_baseline": cpu,
        "adjoint": dict(head["adj"], oracle_columns=len(rows[::4])),
    }
    if "f64" in results:
        r = results["f64"]
        line["fp64"] = {"value": round(r["gcells"], 6), "ms_per_step": round(r["ms"], 4),
                        "rel_err_vs_oracle": r["err"], "row_max_err_vs_oracle": r["row"],
                        "build_s": round(r["build_s"], 3),
                        "apply_achieved_GBs": round(r["apply_gbs"], 1),
                        "factor_bytes": r["factor_bytes"], "adjoint": r["adj"]}
        line["fp32_speedup_over_fp64"] = round(r["ms"] / head["ms"], 3)
    return line


def gpu_many(args, kind, w, refs, cpu, tol):
    """The batched workload or the 3D one: build, one batched call, timing."""
    import numpy as np
    import torch
    import paper_2210_02698_amd as hbi
    dev = torch.device("cuda:0")
    if kind == "batched":
        cases = [(p, n) for p, n, _ in w["cases"]]
        S_h = w["S"]
        rows = w["rows"]
        workload = (f"{len(cases)} 2D constant-gradient problems c(y)=1+g y, N_v in "
                    "{128^2, 256^2, 512^2}, 1-256 Gaussian-source RHS each, nI=13")
    else:
        cases = [(w["prob"], w["nrhs"])]
        S_h = [w["S"]]
        rows = [w["rows"]]
        refs = [refs] if refs is not None else None
        workload = (f"3D sinusoid n=1+0.2 sin2pi x sin2pi y sin2pi z, {args.n_side_3d}^3 cells, "
                    "32 RHS, nI=9")
    ops, S, t_build = [], [], 0.0
    for p, (prob, nrhs) in enumerate(cases):
        op = hbi.Operator(prob, device=0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        op.build(tol=tol, prec="f32")
        torch.cuda.synchronize()
        t_build += time.perf_counter() - t0
        ops.append(op)
        S.append(torch.from_numpy(S_h[p]).to(dev))
        if p % 16 == 0 or p == len(cases) - 1:
            log(f"{kind}: problem {p} N_v={prob.Nv} nrhs={nrhs} build total {t_build:.1f}s")
    t, U = timed_batched(ops, S, args.steps, args.warmup)
    info0 = ops[0].info()
    tile = {"nb": info0.get("batched_tile_nb"), "ku": info0.get("batched_tile_ku")}
    log(f"{kind}: tuned tile {tile}")
    # the same batch as one persistent cooperative launch per call (the
    # library's opt-in mode) beside the graph replay timed above
    tp = p_same = None
    if not args.no_persistent:
        prev = os.environ.get("HBI_BATCHED_PERSISTENT")
        os.environ["HBI_BATCHED_PERSISTENT"] = "1"
        try:
            tp, Up = timed_batched(ops, S, args.steps, args.warmup)
            p_same = all(bool(torch.equal(a, b)) for a, b in zip(U, Up))
        finally:
            if prev is None:
                os.environ.pop("HBI_BATCHED_PERSISTENT")
            else:
                os.environ["HBI_BATCHED_PERSISTENT"] = prev
        del Up
        log(f"{kind}: persistent launch {tp * 1e3:.3f} ms per step, graph {t * 1e3:.3f}, "
            f"bitwise equal {p_same}")
    cells = sum(c[0].Nv * c[1] for c in cases)
    nnz = [op.info()["nnz_total"] for op in ops]
    flops = sum(8.0 * n * c[1] for n, c in zip(nnz, cases))
    errs, rowm = [], []
    if refs is not None:
        for p in range(len(cases)):
            got = U[p].cpu().numpy()[rows[p]]
            e, r = rel_err(got, refs[p])
            errs.append(e)
            rowm.append(r)
    achieved = flops / t / 1e12
    out = {"value": round(cells / t / 1e9, 6), "unit": "Gcell·RHS/s",
           "ms_per_step": round(t * 1e3, 4), "steps": args.steps, "warmup": args.warmup,
           "dtype": "c64 (fp32 factors, MFMA fp32 accumulation; fp64 build)",
           "config": {"workload": workload, "problems": len(cases), "cell_rhs_total": cells,
                      "tol_fp32_build": tol},
           "rel_err_vs_oracle_max": max(errs) if errs else None,
           "row_max_err_vs_oracle": max(rowm) if rowm else None,
           "build_s_total": round(t_build, 2),
           "factor_entries_total": int(sum(nnz)),
           "roofline": {"bound": "mfma", "kernel": "k_wstage_mr/k_vstage_mr/k_final_mr",
                        "achieved": round(achieved, 2), "peak": MFMA_F32_PEAK_TFLOPS,
                        "unit": "TFLOP/s", "frac": round(achieved / MFMA_F32_PEAK_TFLOPS, 4),
                        "flops_per_step": flops, "traffic": None},
           "tuned_tile": tile,
           "persistent_launch": None if tp is None else {
               "ms_per_step": round(tp * 1e3, 4), "value": round(cells / tp / 1e9, 6),
               "bitwise_equal_to_graph": p_same},
           "cpu_baseline": cpu}
    log(f"{kind}: {out['value']} Gcell*RHS/s {out['ms_per_step']} ms err {out['rel_err_vs_oracle_max']}")
    for op in ops:
        op.close()
    del ops, S, U
    torch.cuda.empty_cache()
    return out


def run_sweep(args):
    """Four frequencies from one table set (the HB ingredients do not depend
    on omega), 16 RHS each, one batched call."""
    import dataclasses
    import numpy as np
    import torch
    import hb_inputs
    import oracle
    import paper_2210_02698_amd as hbi
    ensure_lib()
    dev = torch.device("cuda:0")
    base = hb_inputs.configs.c4()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    src = hbi.Operator(base, device=0)
    torch.cuda.synchronize()
    t_load = time.perf_counter() - t0
    cases = [(dataclasses.replace(base, omega=base.omega * f), 16,
              [hb_inputs.configs.CFG_SEED["c4"], 5, i])
             for i, f in enumerate((0.25, 0.5, 0.75, 1.0))]
    ops, S, t_build, t_copy = [], [], 0.0, 0.0
    for prob, nrhs, seed in cases:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        op = hbi.Operator.at_omega(src, prob.omega)
        torch.cuda.synchronize()
        t_copy += time.perf_counter() - t0
        t0 = time.perf_counter()
        op.build(tol=args.tol32, prec="f32")
        torch.cuda.synchronize()
        t_build += time.perf_counter() - t0
        sh = np.asfortranarray(hb_inputs.complex_normal((prob.Nv, nrhs), seed).astype(np.complex64))
        ops.append(op)
        S.append(torch.from_numpy(sh).to(dev))
    t, U = timed_batched(ops, S, args.steps, args.warmup)
    cells = sum(c[0].Nv * c[1] for c in cases)
    flops = sum(8.0 * op.info()["nnz_total"] * c[1] for op, c in zip(ops, cases))
    errs = []
    if not args.no_cpu:
        for p, (prob, nrhs, seed) in enumerate(cases):
            rows = np.sort(np.random.default_rng([9, p]).choice(prob.Nv, 8, replace=False))
            ref = oracle.apply(prob, S[p].cpu().numpy().astype(np.complex128), rows)
            errs.append(rel_err(U[p].cpu().numpy()[rows], ref)[0])
    achieved = flops / t / 1e12
    line = {"metric": METRIC, "value": round(cells / t / 1e9, 6), "unit": "Gcell·RHS/s",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": round(t * 1e3, 4), "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "c64 (fp32 factors, MFMA fp32 accumulation; fp64 build)",
            "data": "synthetic (seeded inputs; straight-ray stand-in tables)",
            "config": {"workload": "frequency sweep from one table set: 2D Gaussian-bump medium, "
                                   "256x256 cells, tables 8x8 boxes x 8x8 nodes, omega = 16pi, "
                                   "32pi, 48pi, 64pi, 16 RHS each",
                       "problems": len(cases), "cell_rhs_total": cells,
                       "tol_fp32_build": args.tol32, "parallelism": "single GPU"},
            "build_s_total": round(t_build, 2),
            "roofline": {"bound": "mfma", "kernel": "k_wstage_mr/k_vstage_mr/k_final_mr",
                         "achieved": round(achieved, 2), "peak": MFMA_F32_PEAK_TFLOPS,
                         "unit": "TFLOP/s", "frac": round(achieved / MFMA_F32_PEAK_TFLOPS, 4),
                         "traffic": None},
            "cpu_baseline": None,
            "sweep": {"omegas_over_pi": [round(c[0].omega / np.pi, 3) for c in cases],
                      "table_load_s": round(t_load, 3),
                      "table_copy_s_mean": round(t_copy / len(cases), 3),
                      "rel_err_vs_oracle_per_omega": errs or None}}
    src.close()
    print(json.dumps(line), flush=True)


def prepare_gradient(args):
    """The differentiation workload: Gaussian bump on 256^2 cells (omega =
    64 pi), P = 512 seeded receiver cells, data d = P K h^d s_true from 20
    seeded point sources, loss ||P K h^d s - d||^2 at a seeded complex
    N(0,1) s; its gradient is 2 h^d K[P]^H (K[P] h^d s - d)."""
    import numpy as np
    import hb_inputs
    prob = hb_inputs.configs.c4()
    seed = hb_inputs.configs.CFG_SEED["c4"]
    g = np.random.default_rng([seed, 0])
    P = np.sort(g.choice(prob.Nv, 512, replace=False))
    _, s_true = hb_inputs.point_sources(prob, 20, [seed, 1])
    s0 = hb_inputs.complex_normal(prob.Nv, [seed, 2], dtype=np.complex64).astype(np.complex128)
    _JOBS["grad"] = (prob, None)
    return dict(prob=prob, P=P, s_true=s_true, s0=s0)


def gpu_gradient(args, w, ref, cpu):
    """Gradient steps through HBApply (forward apply, loss on the receivers,
    backward = hbi_apply_adjoint), FP32 (tol 1e-5) and FP64 (tol 1e-7)
    factors; each step's gradient against the dense FP64 oracle's."""
    import numpy as np
    import torch
    import paper_2210_02698_amd as hbi
    prob, P = w["prob"], w["P"]
    hd = prob.h ** prob.dim
    dev = torch.device("cuda:0")
    out = {}
    for prec, tol in (("f32", args.tol32), ("f64", args.tol64)):
        dt = torch.complex64 if prec == "f32" else torch.complex128
        op = hbi.Operator(prob, device=0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        op.build(tol=tol, prec=prec)
        torch.cuda.synchronize()
        build_s = time.perf_counter() - t0
        Pd = torch.from_numpy(P).to(dev)
        dd = torch.from_numpy(ref["d"]).to(dev).to(dt)
        s0 = torch.from_numpy(w["s0"]).to(dev).to(dt)

        def step():
            s = s0.detach().clone().requires_grad_(True)
            u = hbi.HBApply.apply(op, s)
            loss = (u[Pd] - dd).abs().pow(2).sum()
            loss.backward()
            return s.grad

        grad = step()
        torch.cuda.synchronize()
        g_h = grad.cpu().numpy().astype(np.complex128)
        err = float(np.linalg.norm(g_h - ref["grad"]) / np.linalg.norm(ref["grad"]))
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / args.steps
        log(f"gradient {prec}: {t * 1e3:.3f} ms per step, rel err {err:.2e}")
        out[prec] = {"value": round(prob.Nv / t / 1e9, 6), "ms_per_step": round(t * 1e3, 4),
                     "rel_err_vs_oracle": err, "build_s": round(build_s, 3), "tol": tol}
        op.close()
    head = out["f32"]
    return {"value": head["value"], "unit": "Gcell/s (gradient steps)",
            "ms_per_step": head["ms_per_step"], "steps": args.steps, "warmup": args.warmup,
            "dtype": "c64 (fp32 factors; fp64 build)",
            "config": {"workload": "inverse-source gradient: 2D Gaussian bump 256x256, omega=64pi, "
                                   "512 receivers, loss ||P K h^d s - d||^2, gradient by the "
                                   "adjoint apply",
                       "N_v": prob.Nv, "receivers": len(P)},
            "rel_err_vs_oracle": head["rel_err_vs_oracle"], "build_s": head["build_s"],
            "fp64": out["f64"], "cpu_baseline": cpu}


TAB_FLOPS_PER_UPDATE = 290   # FP64 operations of one sweep point update (two WENO5
                             # one-sided derivatives per axis, the numerical Hamiltonian)
FP64_VALU_PEAK_TFLOPS = 78.6


def prepare_tables(args):
    """Inputs of the table generation: the paper's 2D sinusoidal medium
    (Sec. 5.1) with its table sizes, nI = 13 nodes per axis on the unit square
    and h0 = 0.01; n^2 on a grid of spacing h0/4 and its Taylor coefficients
    at the 169 nodes."""
    import numpy as np
    import hb_inputs
    from oracle import hb_tables as ht
    med = hb_inputs.Sinusoid2D()
    nI, h0, margin = 13, 0.01, 8
    lo, hi = (0.0, 0.0), (1.0, 1.0)
    t0 = time.time()
    P = hb_inputs.node_coords(2, nI, (1, 1), lo, 1.0)
    taylor = hb_inputs.taylor_at(med, P)
    n2, org, sp = hb_inputs.medium_grid(med, lo, hi, h0 / 4, pad=4 * (margin + 4))
    log(f"tables: inputs {time.time() - t0:.1f}s")
    _JOBS["tables"] = (med, ht.node_coords(nI, (1, 1), lo, 1.0), h0, lo, hi)
    sample = np.sort(np.random.default_rng([13, 1]).choice(P.shape[0], 16, replace=False))
    return dict(med=med, nI=nI, h0=h0, margin=margin, n2=n2, org=org, sp=sp, taylor=taylor,
                NT=P.shape[0], sample=sample)


def gpu_tables(args, w, cpu):
    """hbi_tabulate on the prepared inputs: wall time per call (inputs host to
    device, the 169 sources' solves, tables back), the solves' kernel time
    and point updates from hbi_get_info."""
    import torch
    import paper_2210_02698_amd as hbi
    run = lambda: hbi.tabulate(w["n2"], w["org"], w["sp"], w["taylor"], w["nI"], (1, 1),
                               (0.0, 0.0), 1.0, w["h0"], w["margin"], info=True)
    run()                                   # warm-up
    steps = max(1, min(args.steps, 3))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        *_, st = run()
    t = (time.perf_counter() - t0) / steps
    achieved = st["tab_point_updates"] * TAB_FLOPS_PER_UPDATE / st["tab_s"] / 1e12
    return {"value": round(w["NT"] / t, 3), "unit": "sources/s", "ms_per_step": round(t * 1e3, 2),
            "steps": steps, "dtype": "f64",
            "config": {"workload": "2D sinusoidal medium n = 1/(1 + 0.2 sin(pi(x+0.05)) "
                                   "sin(pi y/2)), 13x13 Chebyshev source nodes, h0 = 0.01 "
                                   "(117^2-point grids), tau^2 / v0 / v1 tables",
                       "NT": w["NT"], "h0": w["h0"], "margin": w["margin"]},
            "solve_s": round(st["tab_s"], 4), "rounds_max": st["tab_rounds_max"],
            "point_updates": st["tab_point_updates"],
            "roofline": {"bound": "alu", "kernel": "k_tab_source",
                         "achieved": round(achieved, 4), "peak": FP64_VALU_PEAK_TFLOPS,
                         "unit": "TFLOP/s", "frac": round(achieved / FP64_VALU_PEAK_TFLOPS, 5),
                         "flops_per_point_update": TAB_FLOPS_PER_UPDATE, "traffic": None},
            "parity": "tests/test_gpu_tabulate.py (tables against the oracle to 1e-8)",
            "cpu_baseline": cpu}


def run_inclusion(args):
    """Total field with a curve inclusion (eq. m_v2v_inclu): the 2D Gaussian
    bump at n^2 cells (default 1024^2, omega = 2 pi n / 8), an open square
    of side 0.8 centred in the domain (20 segments per shortest wavelength:
    7,989 segments at 1024^2), FP32, one Gaussian source.  G (cells x
    segments) is a single butterfly; a dense G would take N_v N_s entries
    (64 GB at 1024^2).  The source is cut to exact zeros below 1e-13 of its
    peak, so the oracle's K^{v2s} product needs only the cells where it is
    non-zero."""
    import numpy as np
    import torch
    import hb_inputs
    import paper_2210_02698_amd as hbi
    ensure_lib()
    dev = torch.device("cuda:0")
    n = args.n_side_inc
    prob = hb_inputs.configs.c2(n)
    curve = hb_inputs.open_square(prob, (0.5, 0.5), 0.8, 20)
    P = prob.centres()
    r2 = np.sum((P - np.array([0.5, 0.5])) ** 2, axis=1)
    s_h = np.exp(-r2 / (2.0 * (2.0 * prob.h) ** 2)).astype(np.complex128)
    s_h[np.abs(s_h) < 1e-13] = 0.0
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
    # algorithmic bytes: the volume factors once, the inclusion operators'
    # stored entries once per product, the vectors
    vol = info["nnz_total"] * 8 + (2 * prob.Nv + 2 * info["z_entries"]) * 8
    incb = info["inclusion_apply_bytes"]
    achieved = (vol + incb) / t / 1e9
    err, cpu = None, None
    if not args.no_cpu:
        import oracle
        from oracle import inclusion as oinc
        rows = np.sort(np.random.default_rng([11, 1]).choice(prob.Nv, 16, replace=False))
        t1 = time.perf_counter()
        sup = np.flatnonzero(s_h)
        uinc = oinc.v2s(prob, curve, sup) @ (s_h[sup] * prob.h ** prob.dim)   # eq. m_v2s
        pq = np.linalg.solve(oinc.s2s(prob, curve), uinc)                     # eq. m_sie
        ref = oracle.apply(prob, s_h, rows) + oinc.s2v(prob, curve, rows) @ pq
        t_or = time.perf_counter() - t1
        got = u.cpu().numpy().astype(np.complex128)[rows]
        err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        try:
            from threadpoolctl import threadpool_info
            blas = max([d.get("num_threads", 1) for d in threadpool_info()
                        if d.get("user_api") == "blas"] or [1])
        except Exception:
            blas = 1
        cpu = {"value": len(rows) / t_or / 1e9, "unit": "Gcell·RHS/s", "cores": blas,
               "kind": "oracle",
               "sample": f"{len(rows)} rows of the FP64 oracle: the volume rows, K^{{v2s}} "
                         f"over the source's {len(sup)} non-zero cells, the dense K^{{s2s}} "
                         f"solve ({blas} BLAS threads, the rest one thread), {t_or:.1f} s"}
    line = {
        "metric": METRIC, "value": round(prob.Nv / t / 1e9, 6), "unit": "Gcell·RHS/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(t * 1e3, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64 (fp32 factors and inclusion operators; fp64 build and inverse)",
        "data": "synthetic (seeded inputs; straight-ray stand-in tables)",
        "config": {"workload": f"2D Gaussian-bump medium {n}x{n}, omega={n // 4}pi, open-square "
                               f"inclusion side 0.8 ({curve.Ns} segments), 1 RHS",
                   "N_v": prob.Nv, "N_s": curve.Ns, "tol_fp32_build": args.tol32,
                   "parallelism": "single GPU"},
        "rel_err_vs_oracle": err, "build_s": round(build_s, 3),
        "build_inclusion_s": info["build_inclusion_s"],
        "inclusion_bytes": info["inclusion_bytes"],
        "inclusion_bf_levels": info["inclusion_bf_levels"],
        "inclusion_bf_entries": info["inclusion_bf_entries"],
        "dense_G_bytes": prob.Nv * curve.Ns * 8,
        "roofline": {"bound": "hbm", "kernel": "whole apply (volume factors + inclusion)",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    op.close()


def run_complexity(args):
    """Storage and build time across sizes at 8 cells per wavelength: the 2D
    Gaussian bump on 128^2 .. 1024^2 cells (FP64, tol 1e-7) and the 3D
    sinusoid on 16^3 .. 64^3 cells (FP32, tol 1e-6), against the
    O(N_v log^2 N_v) storage of the paper's complexity statement; and the
    single butterfly of the open-square inclusion (20 segments per
    wavelength, FP32 at tol 1e-5) on the same 2D sizes, against the O(N_v)
    storage stated for K^{s2v} (Sec. 4.2)."""
    import torch
    import hb_inputs
    import paper_2210_02698_amd as hbi
    ensure_lib()
    out = {"workload": "complexity sweep: storage and build time against N_v log2^2 N_v; "
                       "the inclusion butterfly's storage against N_v",
           "2d": [], "3d": [], "inclusion": []}
    cases = [("2d", s, hb_inputs.configs.c2(s), "f64", 1e-7) for s in (128, 256, 512, 1024)]
    cases += [("3d", s, hb_inputs.configs.c5(s), "f32", 1e-6) for s in (16, 32, 48, 64)]
    cases += [("inclusion", s, hb_inputs.configs.c2(s), "f32", 1e-5) for s in (128, 256, 512, 1024)]
    for kind, side, prob, prec, tol in cases:
        op = hbi.Operator(prob, device=0)
        curve = None
        if kind == "inclusion":
            curve = hb_inputs.open_square(prob, (0.5, 0.5), 0.8, 20)
            op.set_inclusion(curve)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        op.build(tol=tol, prec=prec)
        torch.cuda.synchronize()
        bs = time.perf_counter() - t0
        info = op.info()
        op.close()
        n = prob.Nv
        l2 = math.log2(n) ** 2
        if kind == "inclusion":
            ent = info["inclusion_bf_entries"]
            rec = {"side": side, "N_v": n, "N_s": curve.Ns, "prec": prec, "tol": tol,
                   "levels": info["inclusion_bf_levels"], "bf_entries": ent,
                   "bf_entries_per_cell": round(ent / n, 2),
                   "dense_G_entries": n * curve.Ns, "rank_max": info["inclusion_bf_rank_max"],
                   "build_inclusion_s": round(info["build_inclusion_s"], 3)}
        else:
            rec = {"side": side, "N_v": n, "prec": prec, "tol": tol,
                   "nnz_total": info["nnz_total"],
                   "nnz_per_cell": round(info["nnz_total"] / n, 2),
                   "nnz_per_cell_over_log2sq": round(info["nnz_total"] / n / l2, 4),
                   "build_s": round(bs, 3),
                   "build_us_per_cell_over_log2sq": round(bs / n / l2 * 1e6, 5),
                   "rank_max": info["rank_max"], "rank_mean": info["rank_mean"]}
        out[kind].append(rec)
        log(f"complexity {kind} {side}: {rec}")
        torch.cuda.empty_cache()
    r = out["inclusion"]
    a, b = r[0], r[-1]
    out["inclusion_fit"] = {
        "bf_entries_exponent": round(math.log(b["bf_entries"] / a["bf_entries"]) /
                                     math.log(b["N_v"] / a["N_v"]), 4),
        "dense_G_exponent": round(math.log(b["dense_G_entries"] / a["dense_G_entries"]) /
                                  math.log(b["N_v"] / a["N_v"]), 4)}
    for kind in ("2d", "3d"):
        r = out[kind]
        # growth exponents between the smallest and largest size
        a, b = r[0], r[-1]
        out[kind + "_fit"] = {
            "nnz_exponent": round(math.log(b["nnz_total"] / a["nnz_total"]) /
                                  math.log(b["N_v"] / a["N_v"]), 4),
            "build_exponent": round(math.log(b["build_s"] / a["build_s"]) /
                                    math.log(b["N_v"] / a["N_v"]), 4),
            "n_log2sq_exponent": round(math.log(b["N_v"] * math.log2(b["N_v"]) ** 2 /
                                                (a["N_v"] * math.log2(a["N_v"]) ** 2)) /
                                       math.log(b["N_v"] / a["N_v"]), 4)}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n-side", type=int, default=1024)
    ap.add_argument("--n-side-3d", type=int, default=64)
    ap.add_argument("--n-side-inc", type=int, default=1024,
                    help="cells per side of the inclusion workload")
    ap.add_argument("--tol64", type=float, default=1e-7)
    ap.add_argument("--tol32", type=float, default=1e-5,
                    help="FP32 build tolerance of the 2D workloads")
    ap.add_argument("--tol32-3d", type=float, default=1e-6)
    ap.add_argument("--chi", type=float, default=0.0, help="proxy oversampling (0 = library default)")
    ap.add_argument("--bump-rows", type=int, default=512)
    ap.add_argument("--batched-rows", type=int, default=8)
    ap.add_argument("--rows-3d", type=int, default=512)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-persistent", action="store_true",
                    help="skip the persistent-launch timing of the batched and 3d "
                         "workloads (profiled runs: rocprofv3 can crash at exit "
                         "after a cooperative launch)")
    ap.add_argument("--workload", choices=["all", "bump", "batched", "3d", "grad", "tables",
                                           "sweep", "inclusion", "complexity"],
                    default="all",
                    help="all: the headline bump line with the batched and 3d workloads beside "
                         "it; bump: the 1024^2 single-RHS apply alone; batched: 64 "
                         "constant-gradient problems with 1-256 RHS each; 3d: 64^3 sinusoid "
                         "with 32 RHS; grad: inverse-source gradient steps on the 256^2 bump; "
                         "tables: the tau^2/v0/v1 tables of the 2D sinusoidal "
                         "medium from the eikonal and transport solves; sweep: four "
                         "frequencies from one table set, 16 RHS "
                         "each; inclusion: 1024^2 bump with an open-square curve inclusion; "
                         "complexity: storage and build time over sizes")
    ap.add_argument("--nprob", type=int, default=64)
    ap.add_argument("--calib-copy-mb", type=str, default="",
                    help="run device copies of these many MiB first, comma-separated (HBM "
                         "counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "one GPU only: the multi-GPU sharding is designed, not "
                                   "built; run with --gpus 1"}))
        sys.exit(2)
    if args.workload == "inclusion":
        return run_inclusion(args)
    if args.workload == "sweep":
        return run_sweep(args)
    if args.workload == "complexity":
        return run_complexity(args)

    # CPU phase (no GPU touched yet): inputs, then the oracle on the pool
    want = {"all": ("bump", "batched", "3d", "grad", "tables", "c1")}.get(args.workload,
                                                                   (args.workload,))
    work = {}
    if "bump" in want:
        work["bump"] = prepare_bump(args)
    if "batched" in want:
        work["batched"] = prepare_batched(args)
    if "3d" in want:
        work["3d"] = prepare_3d(args)
    if "grad" in want:
        work["grad"] = prepare_gradient(args)
    if "tables" in want:
        work["tables"] = prepare_tables(args)
    if "c1" in want and not args.no_cpu:
        work["c1"] = prepare_c1()
    refs, base = ({}, {}) if args.no_cpu else cpu_phase(work, args)
    _JOBS.clear()

    # GPU phase
    import torch
    ensure_lib()
    for mb in [int(x) for x in args.calib_copy_mb.split(",") if x.strip()]:
        n = mb << 20
        a = torch.empty(n, dtype=torch.uint8, device="cuda:0").fill_(1)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"calibration copy of {n} bytes done")
        del a, b
    line = None
    if "bump" in work:
        line = gpu_bump(args, work["bump"], refs.get("bump"), base.get("bump"),
                        refs.get("bump_adj"))
    for kind in ("batched", "3d"):
        if kind not in work:
            continue
        tol = args.tol32_3d if kind == "3d" else args.tol32
        obj = gpu_many(args, kind, work[kind], refs.get(kind), base.get(kind), tol)
        if line is None:
            line = {"metric": METRIC, "value": obj["value"], "unit": obj["unit"], "n_gpus": 1,
                    "steps": args.steps, "warmup": args.warmup,
                    "ms_per_step": obj["ms_per_step"], "higher_is_better": True,
                    "scaling": "weak", "vs_baseline": None, "dtype": obj["dtype"],
                    "data": "synthetic (seeded inputs)",
                    "config": dict(obj["config"], parallelism="single GPU"),
                    "rel_err_vs_oracle_max": obj["rel_err_vs_oracle_max"],
                    "row_max_err_vs_oracle": obj["row_max_err_vs_oracle"],
                    "build_s_total": obj["build_s_total"], "roofline": obj["roofline"],
                    "cpu_baseline": obj["cpu_baseline"]}
        else:
            line[kind] = obj
            if "fp64" in line:
                # the FP32 many-RHS apply against the FP64 single-RHS apply
                obj["speedup_over_fp64_single_rhs"] = round(obj["value"] / line["fp64"]["value"], 2)
    if "grad" in work and "grad" in refs:
        obj = gpu_gradient(args, work["grad"], refs["grad"], base.get("grad"))
        if line is None:
            line = {"metric": "inverse-source gradient steps (Gcell/s)", "value": obj["value"],
                    "unit": obj["unit"], "n_gpus": 1, "steps": obj["steps"],
                    "warmup": obj["warmup"], "ms_per_step": obj["ms_per_step"],
                    "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
                    "dtype": obj["dtype"], "data": "synthetic (seeded inputs; stand-in tables)",
                    "config": dict(obj["config"], parallelism="single GPU"),
                    "rel_err_vs_oracle": obj["rel_err_vs_oracle"], "fp64": obj["fp64"],
                    "roofline": None, "cpu_baseline": obj["cpu_baseline"]}
        else:
            line["gradient"] = obj
    if "tables" in work:
        obj = gpu_tables(args, work["tables"], base.get("tables"))
        if line is None:
            line = {"metric": "HB table generation sources/s (eikonal and transport solves)",
                    "value": obj["value"], "unit": obj["unit"], "n_gpus": 1,
                    "steps": obj["steps"], "warmup": 1, "ms_per_step": obj["ms_per_step"],
                    "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
                    "dtype": obj["dtype"], "data": "synthetic (the paper's medium in closed form)",
                    "config": dict(obj["config"], parallelism="single GPU"),
                    "solve_s": obj["solve_s"], "rounds_max": obj["rounds_max"],
                    "point_updates": obj["point_updates"], "parity": obj["parity"],
                    "roofline": obj["roofline"], "cpu_baseline": obj["cpu_baseline"]}
        else:
            line["tables"] = obj
    if "c1" in base:
        line["cpu_dense_c1"] = base["c1"]
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
