#!/usr/bin/env python3
"""DD factor + solve benchmark on one MI355X.

One step = the whole hot path on one batch of synthetic input: numeric
factorisation of every domain (batched multifrontal LDL^T, interface-block
inverses), assembly and block LDL^T of the auxiliary matrix, and the
multi-RHS solve (plus FP64 refinement in the mixed form).  The inputs (domain
matrices, right-hand sides) are resident in HBM before timing starts.

Prints one JSON line.  `value` is the effective TFLOP/s of the FP32+refine
path, (factor flops + nrhs * solve flops) / (factor + solve seconds), with the
flop count of the plain FP64 algorithm, so refinement iterations count as time
only; the FP64 path is measured on the same inputs and reported beside it.
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

METRIC = "DD factor+solve sec & eff. TFLOP/s, FP32+refine vs FP64 at rel. resid 1e-9"
PEAK = {"fp64": 78.6, "fp32_refine": 157.3}        # dense MFMA TFLOP/s (MI355X)
WORKLOADS = {
    "cube48": "48^3 Nedelec-hex curl-curl (318,096 unknowns), 4^3 domains of 12^3, eps_r U[1,4] tan-delta 0.02, "
              "k0 ~10 elements/wavelength, 8 complex-normal RHS",
    "cube24": "24^3 Nedelec-hex curl-curl, 3^3 domains of 8^3, 8 RHS (small check case)",
    "cube64j": "64^3 Nedelec-hex curl-curl, nodes jittered +/-0.2h (762,048 unknowns), 216 domains from random "
               "axis cuts of 6..14 elements, eps_r U[1,8] tan-delta 0.02, 64 complex-normal RHS",
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def torn_residual(case, u, lam):
    """Per-column ||[f - K u - B^T lam ; -B u]|| / ||f|| on the host (FP64)."""
    import numpy as np
    f = case.torn_rhs()
    r2 = np.zeros(f.shape[1])
    rl = np.zeros((case.n_mult, f.shape[1]), complex)
    off = 0
    for i, d in enumerate(case.domains):
        Bi = case.B(i)
        ui = u[off:off + d.n]
        r = case.f_torn[i] - d.K @ ui - Bi.T @ lam
        r2 += (np.abs(r) ** 2).sum(axis=0)
        rl -= Bi @ ui
        off += d.n
    r2 += (np.abs(rl) ** 2).sum(axis=0)
    return np.sqrt(r2) / np.linalg.norm(f, axis=0)


def run_path(case, vals, f, prec, steps, warmup, graph, tune, tiles=None, timed_events=False):
    import torch
    from paper_2002_05019_amd.binding import Solver
    nrhs = f.shape[1]
    s = Solver.from_case(case, precision=prec, max_rhs=max(8, nrhs), use_graph=graph,
                         schur_tile=tiles).bind("cuda:0")
    tiles = s.tune() if tune and tiles is None else tiles
    if tiles:
        log(f"[bench] {prec}: tuned Schur-update tiles per front-size bucket {tiles}")
    for _ in range(warmup):
        s.factor(vals)
        s.solve(f)
    torch.cuda.synchronize()
    times, tf, ts = [], [], []
    if timed_events:
        # HIP events around every Schur-update launch of the timed steps (the
        # factorisation then runs as plain launches)
        s.kernel_timer_start("schur_update")
    for _ in range(steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.factor(vals)
        u = s.solve(f)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        inf = s.info()
        tf.append(inf["t_factor"])
        ts.append(inf["t_solve"])
        log(f"[bench] {prec} step {len(times)}: {times[-1] * 1e3:.1f} ms "
            f"(factor {tf[-1] * 1e3:.1f} ms, solve {ts[-1] * 1e3:.1f} ms)")
    kt = None
    if timed_events:
        kt = s.kernel_timer_read()
        kt["factorizations"] = steps
        s.kernel_timer_start(None)
    info = s.info()
    sub = None
    if prec == "fp64":
        # recovery of one eighth of the domains (the condensation and the
        # auxiliary solve still involve all of them)
        pick = list(range(0, case.n_dom, 8))
        ts_sub = []
        for _ in range(3):
            s.solve_subset(f, pick)
            ts_sub.append(s.info()["t_solve"])
        sub = {"domains": len(pick), "of": case.n_dom, "solve_ms": round(min(ts_sub) * 1e3, 3)}
    u, lam = s.solve(f, return_lam=True)
    torch.cuda.synchronize()
    out = dict(solver=s, times=times, t_factor=tf, t_solve=ts, info=info, kt=kt, tiles=tiles,
               u=u.cpu().numpy(), lam=lam.cpu().numpy(), status=s.last_status, subset=sub)
    return out


def kernel_timing(solver, vals, kernel="schur_update"):
    import torch
    solver.kernel_timer_start(kernel)
    solver.factor(vals)
    torch.cuda.synchronize()
    kt = solver.kernel_timer_read()
    kt["factorizations"] = 1
    solver.kernel_timer_start(None)
    return kt


def recorded_traffic(workload, tiles, launches, path=None):
    """HBM bytes per Schur-update launch from the committed rocprofv3 counter
    record (FETCH_SIZE / WRITE_SIZE scaled by a copy-kernel calibration), or
    None when the kernels, the workload, the tile policy or the number of
    launches per factorisation differ from the measured ones."""
    import hashlib
    path = path or os.path.join(ROOT, "profiles", f"schur_update_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    with open(os.path.join(ROOT, "paper_2002_05019_amd", "csrc", "kernels.hip"), "rb") as fh:
        h = hashlib.sha256(fh.read()).hexdigest()
    if h != rec["kernels_hip_sha256"] or list(tiles or []) != rec["schur_tile_by_front_size"]:
        return None
    if launches != rec["launches"]:
        return None
    return rec["bytes_per_launch"]


def record_traffic(calib_f, calib_w, syrk_f, syrk_w, calib_mib, workload, tiles):
    """Writes the per-launch HBM traffic record of the Schur update from four
    rocprofv3 --pmc output folders (FETCH_SIZE then WRITE_SIZE of a device
    copy of calib_mib MiB, and of a run with the given workload and tiles)."""
    import csv
    import hashlib

    def rows(d):
        with open(os.path.join(d, "run_counter_collection.csv")) as fh:
            return list(csv.DictReader(fh))

    def copy_kib(d, counter):
        v = [float(r["Counter_Value"]) for r in rows(d)
             if r["Counter_Name"] == counter and "copyBuffer" in r["Kernel_Name"]]
        if not v:
            raise SystemExit(f"no copy kernel with {counter} in {d}")
        return sum(v)

    def syrk_kib(d, counter):
        v = [float(r["Counter_Value"]) for r in rows(d)
             if r["Counter_Name"] == counter
             and r["Kernel_Name"].replace("void ", "", 1).startswith("dd::k_syrk<float, dd::Tile<64, 64, 2, 2, 16>")]
        if not v:
            raise SystemExit(f"no Schur-update launch with {counter} in {d}")
        return sum(v) / len(v), len(v)

    true_kib = calib_mib * 1024.0
    sf, sw = true_kib / copy_kib(calib_f, "FETCH_SIZE"), true_kib / copy_kib(calib_w, "WRITE_SIZE")
    (fk, n), (wk, _) = syrk_kib(syrk_f, "FETCH_SIZE"), syrk_kib(syrk_w, "WRITE_SIZE")
    with open(os.path.join(ROOT, "paper_2002_05019_amd", "csrc", "kernels.hip"), "rb") as fh:
        h = hashlib.sha256(fh.read()).hexdigest()
    rec = {"kernel": "k_syrk<float, Tile<64,64,2,2,16>> (trailing Schur update, FP32+refine path)", "workload": workload,
           "schur_tile_by_front_size": tiles, "launches": n,
           "fetch_kib_per_launch": round(fk, 1), "write_kib_per_launch": round(wk, 1),
           "fetch_scale": round(sf, 4), "write_scale": round(sw, 4),
           "bytes_per_launch": int(round((fk * sf + wk * sw) * 1024)), "kernels_hip_sha256": h}
    path = os.path.join(ROOT, "profiles", f"schur_update_{workload}_traffic.json")
    with open(path, "w") as fh:
        json.dump(rec, fh, indent=1)
    log(f"[bench] wrote {path}: {rec['bytes_per_launch'] / 1e6:.1f} MB per launch over {n} launches")


def cpu_baseline(case, solver, budget_s=30.0):
    """The oracle's per-domain elimination (SuperLU factorisation + interface
    inverse) on interior domains, timed on the host; scaled to TFLOP/s with the
    same algorithmic flop count the GPU path is credited with."""
    import oracle
    # interior domains carry the largest interface; take the first ones
    order = sorted(range(case.n_dom), key=lambda i: -len(case.gamma(i)))
    t_tot, fl_tot, done = 0.0, 0.0, []
    for i in order:
        t0 = time.perf_counter()
        oracle.interface_inverse(case.domains[i].K, case.gamma(i))
        dt = time.perf_counter() - t0
        t_tot += dt
        fl_tot += solver.domain_flops(i)
        done.append(i)
        log(f"[bench] cpu oracle domain {i}: {dt:.1f} s")
        if t_tot > budget_s * 0.5:
            break
    return {"value": fl_tot / t_tot / 1e12, "unit": "TFLOP/s", "cores": 1, "kind": "oracle",
            "sample": f"SuperLU factorisation + interface inverse of {len(done)} interior 12^3 domain(s) "
                      f"of {case.n_dom} ({t_tot:.1f} s, single-threaded SuperLU)",
            "seconds": round(t_tot, 2)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cube48", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison path")
    ap.add_argument("--graph", type=int, default=1, help="replay factor/solve from hipGraphs (1) or launch (0)")
    ap.add_argument("--tune", type=int, default=1, help="autotune the Schur-update tiles before timing (1) or not (0)")
    ap.add_argument("--tiles", default=None,
                    help="Schur-update tile edge per front-size bucket, e.g. 64,64,64,64,128 (implies --tune 0)")
    ap.add_argument("--kernel-events", choices=["timed", "extra"], default="timed",
                    help="time the Schur-update launches with HIP events inside the timed steps, or in one "
                         "extra factorisation after them (then the timed steps replay graphs)")
    ap.add_argument("--copy-calib-mib", type=int, default=0,
                    help="only copy a buffer of this many MiB on the device and exit (counter calibration)")
    ap.add_argument("--record-traffic", nargs=4, metavar=("CALIB_F", "CALIB_W", "PMC_F", "PMC_W"),
                    help="write the Schur-update traffic record from four rocprofv3 --pmc folders (no GPU "
                         "work): FETCH_SIZE / WRITE_SIZE of a --copy-calib-mib run, then of a run with "
                         "--workload and --tiles")
    args = ap.parse_args()
    if args.record_traffic:
        record_traffic(*args.record_traffic, calib_mib=args.copy_calib_mib or 1024, workload=args.workload,
                       tiles=[int(t) for t in (args.tiles or "64,64,64,64,64").split(",")])
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (the solver is single-GPU); got --gpus {args.gpus}",
              file=sys.stderr)
        sys.exit(2)
    if args.copy_calib_mib:
        import torch
        src = torch.ones(args.copy_calib_mib << 18, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] copied {args.copy_calib_mib} MiB")
        return
    tiles = [int(t) for t in args.tiles.split(",")] if args.tiles else None
    import numpy as np
    import torch
    from paper_2002_05019_amd.problem import make_case

    t0 = time.perf_counter()
    case = make_case(args.workload)
    log(f"[bench] workload {args.workload}: {case.n_global} unknowns, {case.n_dom} domains, "
        f"{case.n_mult} multipliers, generated in {time.perf_counter() - t0:.1f} s")
    vals = torch.from_numpy(np.concatenate([d.K.data for d in case.domains])).to("cuda:0")
    f = torch.from_numpy(case.torn_rhs()).to("cuda:0")
    nrhs = f.shape[1]

    res = {}
    paths = ["fp32_refine"] if args.no_fp64 else ["fp64", "fp32_refine"]
    for prec in paths:
        res[prec] = run_path(case, vals, f, prec, args.steps, args.warmup, bool(args.graph), bool(args.tune), tiles,
                             timed_events=(prec == "fp32_refine" and args.kernel_events == "timed"))
        if prec == "fp32_refine" and args.kernel_events == "extra":
            # kernel-level event timing of the Schur update in one extra
            # (untimed, plain-launch) factorisation of the same path
            res[prec]["kt"] = kernel_timing(res[prec]["solver"], vals)
        r = res[prec]
        r["resid"] = torn_residual(case, r["u"], r["lam"])
        log(f"[bench] {prec}: host-checked torn residual max {r['resid'].max():.2e}")

    mx = res["fp32_refine"]
    info = mx["info"]
    flops = info["flops_factor"] + nrhs * info["flops_solve"]
    ms = float(np.mean(mx["times"])) * 1e3
    value = flops / (ms * 1e-3) / 1e12
    kt = mx["kt"]
    achieved = kt["flops"] / kt["seconds"] / 1e12 if kt and kt["seconds"] > 0 else None
    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "TFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "complex64 fronts + fp64 refinement", "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload], "name": args.workload, "domains": case.n_dom,
                   "unknowns": case.n_global, "multipliers": case.n_mult, "nrhs": nrhs,
                   "precision": "fp32_refine", "refine_tol": 1e-9, "hipgraph": bool(args.graph),
                   "schur_tile_by_front_size": mx["tiles"]},
        "mixed": {"factor_ms": round(float(np.mean(mx["t_factor"])) * 1e3, 3),
                  "solve_ms": round(float(np.mean(mx["t_solve"])) * 1e3, 3),
                  "refine_iters": info["refine_iters"], "rel_resid": info["rel_resid"],
                  "host_resid_max": float(mx["resid"].max()), "status": mx["status"],
                  "n_perturbed": info["n_perturbed"]},
        "flops_per_step": flops,
        "roofline": None if achieved is None else {
            "kernel": "schur_update (complex FP32 MFMA trailing update, 64/128 tiles)", "bound": "mfma",
            "achieved": round(achieved, 3), "peak": PEAK["fp32_refine"], "unit": "TFLOP/s",
            "frac": round(achieved / PEAK["fp32_refine"], 4),
            "traffic": recorded_traffic(args.workload, mx["tiles"], kt["launches"] // kt["factorizations"]),
            "launches": kt["launches"], "avg_launch_us": round(kt["seconds"] / kt["launches"] * 1e6, 2)},
    }
    if "fp64" in res:
        d = res["fp64"]
        ms64 = float(np.mean(d["times"])) * 1e3
        out["fp64"] = {"ms_per_step": round(ms64, 3), "tflops": round(flops / (ms64 * 1e-3) / 1e12, 3),
                       "factor_ms": round(float(np.mean(d["t_factor"])) * 1e3, 3),
                       "solve_ms": round(float(np.mean(d["t_solve"])) * 1e3, 3),
                       "host_resid_max": float(d["resid"].max()), "n_perturbed": d["info"]["n_perturbed"],
                       "subset_recovery": d["subset"]}
        err = np.linalg.norm(mx["u"] - d["u"], axis=0) / np.linalg.norm(d["u"], axis=0)
        out["mixed"]["err_vs_fp64"] = float(err.max())
        out["mixed"]["speedup_vs_fp64"] = round(ms64 / ms, 3)
    out["memory"] = {"workspace_gb_mixed": round(info["workspace_bytes"] / 1e9, 3),
                     "factor_gb_mixed": round(info["bytes_factor"] / 1e9, 3)}
    if "fp64" in res:
        out["memory"]["workspace_gb_fp64"] = round(res["fp64"]["info"]["workspace_bytes"] / 1e9, 3)
        out["memory"]["factor_gb_fp64"] = round(res["fp64"]["info"]["bytes_factor"] / 1e9, 3)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(case, mx["solver"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
