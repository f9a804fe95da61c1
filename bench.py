#!/usr/bin/env python3
"""DD factor + solve benchmark on one MI355X.

One step = the whole hot path on one batch of synthetic input: numeric
factorisation of every domain (batched multifrontal LDL^T, interface-block
inverses), assembly and block LDL^T of the auxiliary matrix, and the
multi-RHS solve (plus FP64 refinement in the mixed form).  The inputs (domain
matrices, right-hand sides) are resident in HBM before timing starts, and the
timed steps replay the factorisation and the solve from hipGraphs.

Prints one JSON line.  `value` is the effective TFLOP/s of the FP32+refine
path on the 48^3 workload, (factor flops + nrhs * solve flops) / (factor +
solve seconds), with the flop count of the plain FP64 algorithm, so
refinement iterations count as time only; the FP64 path is measured on the
same inputs and reported beside it.  The 216-domain uneven workload (64^3,
64 RHS) is measured the same way in `uneven_batching`.  `roofline` is the
trailing Schur update of the mixed path, timed with HIP events around every
launch of one extra (plain-launch) factorisation; `solve_roofline` the FP64
solve against HBM bandwidth; `memory` the workspace beside the global FP64
sparse direct factor of the same mesh (nested-dissection model).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DD factor+solve sec & eff. TFLOP/s, FP32+refine vs FP64 at rel. resid 1e-9"
PEAK = {"fp64": 78.6, "fp32_refine": 157.3}        # dense MFMA TFLOP/s (MI355X)
HBM_GBS = 8000.0                                   # HBM3E GB/s (MI355X)
WORKLOADS = {
    "cube48": "48^3 Nedelec-hex curl-curl (318,096 unknowns), 4^3 domains of 12^3, eps_r U[1,4] tan-delta 0.02, "
              "k0 ~10 elements/wavelength, 8 complex-normal RHS",
    "cube24": "24^3 Nedelec-hex curl-curl, 3^3 domains of 8^3, 8 RHS (small check case)",
    "cube64j": "64^3 Nedelec-hex curl-curl, nodes jittered +/-0.2h (762,048 unknowns), 216 domains from random "
               "axis cuts of 6..14 elements, eps_r U[1,8] tan-delta 0.02, 64 complex-normal RHS",
    "cube96j": "96^3 Nedelec-hex curl-curl, nodes jittered +/-0.2h (2,599,200 unknowns), 8^3 domains of 12^3, "
               "eps_r U[1,4] tan-delta 0.01, 256 complex-normal RHS (FP32 fronts + FP64 refinement)",
    "tet40s": "Whitney-tet curl-curl on a jittered 40^3 Kuhn mesh carved to a ball (223,907 unknowns), dielectric "
              "sphere eps_r 4 in eps_r 1, tan-delta 0.02, 64 domains from the graph partitioner, 8 complex-normal RHS",
}
MESH_N = {"cube48": 48, "cube24": 24, "cube64j": 64, "cube96j": 96}   # cube meshes (global direct model)


def make_workload(name):
    if name.startswith("tet"):
        from paper_2002_05019_amd.tetmesh import make_tet_case
        return make_tet_case(name)
    from paper_2002_05019_amd.problem import make_case
    return make_case(name)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def global_direct_model(n, leaf=2):
    """Nested-dissection model of an undecomposed sparse LDL^T of the n^3 PEC
    cube's edge-element matrix, the comparison the paper draws (section III):
    recursively bisect the element box along its longest side at the
    midpoint (leaves of at most `leaf` elements per side); a box's front
    eliminates the edges strictly inside its cut section (a leaf: the edges
    strictly inside the box) and carries as update rows the non-PEC edges on
    the box surface.  Returns the factor's nonzeros (lower triangle with
    diagonal), its complex FMAs ((s+R)^3 - R^3)/6 per front, and the number
    of eliminated unknowns (every non-PEC edge exactly once)."""
    def span(lo, hi):           # node indices in [lo, hi] strictly inside (0, n)
        return max(0, min(hi, n - 1) - max(lo, 1) + 1)

    def perim(l1, h1, l2, h2):  # non-PEC nodes on the boundary of a rectangle
        return span(l1, h1) * span(l2, h2) - max(0, h1 - l1 - 1) * max(0, h2 - l2 - 1)

    tot = {"eliminated": 0, "nnz": 0, "fma": 0.0}

    def rec(b):
        x0, x1, y0, y1, z0, z1 = b
        a, bb, c = x1 - x0, y1 - y0, z1 - z0
        # update rows: edges along each axis over the non-PEC perimeter nodes
        R = a * perim(y0, y1, z0, z1) + bb * perim(x0, x1, z0, z1) + c * perim(x0, x1, y0, y1)
        if max(a, bb, c) <= leaf:
            s = a * (bb - 1) * (c - 1) + bb * (a - 1) * (c - 1) + c * (a - 1) * (bb - 1)
        else:
            d = max(range(3), key=lambda k: (a, bb, c)[k])
            m = b[2 * d] + (b[2 * d + 1] - b[2 * d]) // 2
            o = [(b[2], b[3], b[4], b[5]), (b[0], b[1], b[4], b[5]), (b[0], b[1], b[2], b[3])][d]
            p, q = o[1] - o[0], o[3] - o[2]
            s = p * (q - 1) + q * (p - 1)          # edges strictly inside the cut section
            left, right = list(b), list(b)
            left[2 * d + 1] = m
            right[2 * d] = m
            rec(tuple(left))
            rec(tuple(right))
        tot["eliminated"] += s
        tot["nnz"] += s * (s + 1) // 2 + s * R
        tot["fma"] += ((s + R) ** 3 - R ** 3) / 6.0

    rec((0, n, 0, n, 0, n))
    return tot


def host_residuals(case, u, lam):
    """Per column, on the host (FP64): the torn residual
    ||[f - K u - B^T lam ; -B u]|| / ||f|| and the residual of the undecomposed
    system ||f - A u|| / ||f|| with u the owner copies."""
    import numpy as np
    nr = u.shape[1]
    r2 = np.zeros(nr)
    rl = np.zeros((case.n_mult, nr), complex)
    off = 0
    t0 = time.perf_counter()
    for i, d in enumerate(case.domains):
        Bi = case.B(i)
        ui = u[off:off + d.n]
        r = case.f_torn[i] - d.K @ ui - Bi.T @ lam
        r2 += (np.abs(r) ** 2).sum(axis=0)
        rl -= Bi @ ui
        off += d.n
        if (i + 1) % 64 == 0:
            log(f"[bench] host torn residual: {i + 1} of {case.n_dom} domains ({time.perf_counter() - t0:.0f} s)")
    r2 += (np.abs(rl) ** 2).sum(axis=0)
    fn = np.sqrt(sum((np.abs(x) ** 2).sum(axis=0) for x in case.f_torn))
    torn = np.sqrt(r2) / fn
    ug = case.owner_copy(u)
    A = case.A
    glob = np.zeros(nr)
    for j0 in range(0, nr, 32):
        g = case.f[:, j0:j0 + 32] - A @ ug[:, j0:j0 + 32]
        glob[j0:j0 + 32] = np.linalg.norm(g, axis=0) / np.linalg.norm(case.f[:, j0:j0 + 32], axis=0)
        if nr > 32:
            log(f"[bench] host global residual: columns {j0}..{min(nr, j0 + 32)} ({time.perf_counter() - t0:.0f} s)")
    return torn, glob


def run_path(case, vals, f, prec, steps, warmup, graph, tune, tiles=None, max_rhs=None):
    """Times `steps` factor + solve steps (after `warmup`), replayed from
    hipGraphs when `graph`; returns the solver, the times and the last
    solution."""
    import torch
    from paper_2002_05019_amd.binding import Solver
    nrhs = f.shape[1]
    mr = max_rhs or max(8, min(nrhs, 64))
    s = Solver.from_case(case, precision=prec, max_rhs=mr, use_graph={0: False, 1: True, 2: "solve"}[graph],
                         schur_tile=tiles).bind("cuda:0")
    tiles = s.tune() if tune and tiles is None else tiles
    if tiles:
        log(f"[bench] {prec}: tuned Schur-update tiles per front-size bucket {tiles}")
    for _ in range(warmup):
        s.factor(vals)
        s.solve(f)
    torch.cuda.synchronize()
    times, tf, ts = [], [], []
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
    info = s.info()
    u, lam = s.solve(f, return_lam=True)
    torch.cuda.synchronize()
    return dict(solver=s, times=times, t_factor=tf, t_solve=ts, info=info, tiles=tiles,
                u=u.cpu().numpy(), lam=lam.cpu().numpy(), status=s.last_status)


def subset_timing(s, f, n_dom):
    """FP64 recovery of one eighth of the domains (the condensation and the
    auxiliary solve still involve all of them)."""
    pick = list(range(0, n_dom, 8))
    ts = []
    for _ in range(3):
        s.solve_subset(f, pick)
        ts.append(s.info()["t_solve"])
    return {"domains": len(pick), "of": n_dom, "solve_ms": round(min(ts) * 1e3, 3)}


def kernel_timing(solver, vals, kernel="schur_update"):
    """HIP events around every launch of one factorisation kernel, in one
    extra factorisation with plain launches (on the launch stream)."""
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
    if launches != rec.get("launches_per_factorization"):
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

    # the counter run (--steps 1 --warmup 0) factors twice: the timed step and
    # the extra plain-launch factorisation timed per launch
    true_kib = calib_mib * 1024.0
    sf, sw = true_kib / copy_kib(calib_f, "FETCH_SIZE"), true_kib / copy_kib(calib_w, "WRITE_SIZE")
    (fk, n), (wk, _) = syrk_kib(syrk_f, "FETCH_SIZE"), syrk_kib(syrk_w, "WRITE_SIZE")
    with open(os.path.join(ROOT, "paper_2002_05019_amd", "csrc", "kernels.hip"), "rb") as fh:
        h = hashlib.sha256(fh.read()).hexdigest()
    rec = {"kernel": "k_syrk<float, Tile<64,64,2,2,16>> (trailing Schur update, FP32+refine path)", "workload": workload,
           "schur_tile_by_front_size": tiles, "launches": n, "launches_per_factorization": n // 2,
           "fetch_kib_per_launch": round(fk, 1), "write_kib_per_launch": round(wk, 1),
           "fetch_scale": round(sf, 4), "write_scale": round(sw, 4),
           "bytes_per_launch": int(round((fk * sf + wk * sw) * 1024)), "kernels_hip_sha256": h}
    path = os.path.join(ROOT, "profiles", f"schur_update_{workload}_traffic.json")
    with open(path, "w") as fh:
        json.dump(rec, fh, indent=1)
    log(f"[bench] wrote {path}: {rec['bytes_per_launch'] / 1e6:.1f} MB per launch over {n} launches")


def _oracle_domain(args):
    """One domain's elimination by the oracle (worker process)."""
    import oracle
    K, gamma = args
    t0 = time.perf_counter()
    oracle.interface_inverse(K, gamma)
    return time.perf_counter() - t0


def cpu_baseline(case, dom_flops, step_flops, workers=None):
    """The oracle's elimination of every domain (SuperLU factorisation and
    interface inverse: steps a1 + a2 of the step), spread over the host's
    cores with worker processes (started before the GPU is touched), timed
    wall-clock and scaled to TFLOP/s with the algorithmic flops the GPU path
    is credited with for those domains."""
    import multiprocessing as mp
    nproc = os.cpu_count() or 1
    workers = workers or max(1, min(16, nproc))
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    # fresh single-threaded worker processes (one core each)
    for v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[v] = "1"
    jobs = [(case.domains[i].K, case.gamma(i)) for i in range(case.n_dom)]
    with mp.get_context("spawn").Pool(workers) as pool:
        pool.map(_oracle_domain, jobs[:workers], chunksize=1)   # start-up and imports, untimed
        t0 = time.perf_counter()
        per = pool.map(_oracle_domain, jobs, chunksize=1)
        wall = time.perf_counter() - t0
    fl = float(sum(dom_flops))
    log(f"[bench] cpu oracle: {case.n_dom} domains on {workers} processes in {wall:.1f} s "
        f"(sum of per-domain times {sum(per):.1f} s)")
    return {"value": fl / wall / 1e12, "unit": "TFLOP/s", "cores": workers, "kind": "oracle",
            "sample": f"SuperLU factorisation + interface inverse of all {case.n_dom} domains (steps a1+a2, "
                      f"{100.0 * fl / step_flops:.0f}% of the step's flops), one domain per task on {workers} "
                      f"worker processes, {wall:.1f} s wall",
            "seconds": round(wall, 2), "nproc": nproc, "cpu_model": model,
            "share_of_step_flops": round(fl / step_flops, 4)}


def measure(case, vals, f, args, tiles, paths, kernel_events=True):
    """Both paths on one workload: timings, host residuals, rooflines."""
    import numpy as np
    res = {}
    mr = 64 if MESH_N.get(case.spec.name, 0) >= 96 else None
    for prec in paths:
        r = run_path(case, vals, f, prec, args.steps, args.warmup, args.graph, bool(args.tune), tiles,
                     max_rhs=mr)
        if prec == "fp32_refine" and kernel_events:
            r["kt"] = kernel_timing(r["solver"], vals)
        if prec == "fp64":
            r["subset"] = subset_timing(r["solver"], f, case.n_dom)
        r["torn"], r["glob"] = host_residuals(case, r["u"], r["lam"])
        log(f"[bench] {case.spec.name} {prec}: host residuals max torn {r['torn'].max():.2e} "
            f"global {r['glob'].max():.2e}")
        res[prec] = r
        if prec == "fp64" and len(paths) > 1:
            # keep only what the report needs before the next path binds its workspace
            r["solver"].close()
            r["solver"] = None
            import gc
            import torch
            gc.collect()
            torch.cuda.empty_cache()
    return res


def path_record(r, flops):
    import numpy as np
    ms = float(np.mean(r["times"])) * 1e3
    info = r["info"]
    out = {"ms_per_step": round(ms, 3), "tflops": round(flops / (ms * 1e-3) / 1e12, 3),
           "factor_ms": round(float(np.mean(r["t_factor"])) * 1e3, 3),
           "solve_ms": round(float(np.mean(r["t_solve"])) * 1e3, 3),
           "host_resid_global_max": float(r["glob"].max()), "host_resid_torn_max": float(r["torn"].max()),
           "status": r["status"], "n_perturbed": info["n_perturbed"],
           "n_pivot_2x2": info["n_pivot_2x2"], "n_interchanges": info["n_interchanges"],
           "workspace_gb": round(info["workspace_bytes"] / 1e9, 3),
           "factor_gb": round(info["bytes_factor"] / 1e9, 3)}
    if info["refine_iters"] or info["rel_resid"]:
        out["refine_iters"] = info["refine_iters"]
        out["rel_resid"] = info["rel_resid"]
    if r.get("subset"):
        out["subset_recovery"] = r["subset"]
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cube48", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison path")
    ap.add_argument("--no-uneven", action="store_true", help="skip the 216-domain uneven-batching record")
    ap.add_argument("--graph", type=int, default=2, choices=[0, 1, 2],
                    help="replay factor and solve from hipGraphs (1), the solve only (2), or launch (0)")
    ap.add_argument("--tune", type=int, default=1, help="autotune the Schur-update tiles before timing (1) or not (0)")
    ap.add_argument("--tiles", default=None,
                    help="Schur-update tile edge per front-size bucket, e.g. 64,64,64,64,128 (implies --tune 0)")
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
    from paper_2002_05019_amd.binding import Solver

    t0 = time.perf_counter()
    case = make_workload(args.workload)
    log(f"[bench] workload {args.workload}: {case.n_global} unknowns, {case.n_dom} domains, "
        f"{case.n_mult} multipliers, generated in {time.perf_counter() - t0:.1f} s")
    nrhs = case.spec.nrhs
    big = MESH_N.get(args.workload, 0) >= 96
    paths = ["fp32_refine"] if (args.no_fp64 or big) else ["fp64", "fp32_refine"]
    # host-only symbolic phase: flop counts (and the CPU baseline, which runs
    # before anything touches the GPU)
    host = Solver.from_case(case, precision="fp64", max_rhs=8)
    dom_flops = [host.domain_flops(i) for i in range(case.n_dom)]
    hi = host.info()
    host.close()
    cpu = None if args.no_cpu else cpu_baseline(case, dom_flops, hi["flops_factor"] + nrhs * hi["flops_solve"])
    import torch
    vals = torch.from_numpy(np.concatenate([d.K.data for d in case.domains])).to("cuda:0")
    f = torch.from_numpy(case.torn_rhs()).to("cuda:0")

    res = measure(case, vals, f, args, tiles, paths)
    mx = res["fp32_refine"]
    info = mx["info"]
    flops = info["flops_factor"] + nrhs * info["flops_solve"]
    ms = float(np.mean(mx["times"])) * 1e3
    value = flops / (ms * 1e-3) / 1e12
    kt = mx.get("kt")
    achieved = kt["flops"] / kt["seconds"] / 1e12 if kt and kt["seconds"] > 0 else None
    dm = global_direct_model(MESH_N[args.workload]) if args.workload in MESH_N else None
    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "TFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "complex64 fronts + fp64 refinement", "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload], "name": args.workload, "domains": case.n_dom,
                   "unknowns": case.n_global, "multipliers": case.n_mult, "nrhs": nrhs,
                   "precision": "fp32_refine", "refine_tol": 1e-9,
                   "hipgraph": {0: "none", 1: "factorisation and solve", 2: "solve"}[args.graph],
                   "schur_tile_by_front_size": mx["tiles"]},
        "mixed": path_record(mx, flops),
        "flops_per_step": flops,
        "roofline": None if achieved is None else {
            "kernel": "schur_update (complex FP32 MFMA trailing update, 64/128 tiles)", "bound": "mfma",
            "achieved": round(achieved, 3), "peak": PEAK["fp32_refine"], "unit": "TFLOP/s",
            "frac": round(achieved / PEAK["fp32_refine"], 4),
            "traffic": recorded_traffic(args.workload, mx["tiles"], kt["launches"] // kt["factorizations"]),
            "launches": kt["launches"], "avg_launch_us": round(kt["seconds"] / kt["launches"] * 1e6, 2),
            "timed": "HIP events around every launch of one extra plain-launch factorisation"},
    }
    if "fp64" in res:
        d = res["fp64"]
        out["fp64"] = path_record(d, flops)
        err = np.linalg.norm(mx["u"] - d["u"], axis=0) / np.linalg.norm(d["u"], axis=0)
        out["mixed"]["err_vs_fp64"] = float(err.max())
        out["mixed"]["speedup_vs_fp64"] = round(out["fp64"]["ms_per_step"] / ms, 3)
        bs = d["info"]["bytes_solve"]
        ts = out["fp64"]["solve_ms"] * 1e-3
        out["solve_roofline"] = {"kernel": "FP64 multi-RHS solve (all sweeps)", "bound": "hbm",
                                 "achieved": round(bs / ts / 1e9, 1), "peak": HBM_GBS, "unit": "GB/s",
                                 "frac": round(bs / ts / 1e9 / HBM_GBS, 4), "bytes_per_solve": bs}
    out["memory"] = {"workspace_gb_mixed": out["mixed"]["workspace_gb"],
                     "factor_gb_mixed": out["mixed"]["factor_gb"]}
    if dm is not None:
        out["memory"].update({"global_direct_fp64_gb": round(dm["nnz"] * 16 / 1e9, 3),
                              "global_direct_fp64_flops": dm["fma"] * 8,
                              "global_direct_note": "undecomposed sparse LDL^T of the same mesh, geometric nested "
                                                    "dissection model, complex FP64 (16 B per factor entry)"})
    if "fp64" in res:
        out["memory"]["workspace_gb_fp64"] = out["fp64"]["workspace_gb"]
        out["memory"]["factor_gb_fp64"] = out["fp64"]["factor_gb"]
    if not args.no_uneven and args.workload == "cube48":
        out["uneven_batching"] = uneven_record(args, tiles)
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


def uneven_record(args, tiles):
    """The 216-domain uneven workload (64^3 jittered, random axis cuts, 64
    RHS), both paths, tuned tiles and graph replay."""
    import gc

    import numpy as np
    import torch
    from paper_2002_05019_amd.problem import make_case
    t0 = time.perf_counter()
    case = make_case("cube64j")
    log(f"[bench] cube64j generated in {time.perf_counter() - t0:.1f} s")
    vals = torch.from_numpy(np.concatenate([d.K.data for d in case.domains])).to("cuda:0")
    f = torch.from_numpy(case.torn_rhs()).to("cuda:0")
    res = measure(case, vals, f, args, tiles, ["fp64", "fp32_refine"], kernel_events=False)
    mx, d = res["fp32_refine"], res["fp64"]
    flops = mx["info"]["flops_factor"] + case.spec.nrhs * mx["info"]["flops_solve"]
    out = {"workload": WORKLOADS["cube64j"], "domains": case.n_dom, "unknowns": case.n_global, "nrhs": case.spec.nrhs,
           "flops_per_step": flops, "mixed": path_record(mx, flops), "fp64": path_record(d, flops),
           "global_direct_fp64_gb": round(global_direct_model(64)["nnz"] * 16 / 1e9, 3)}
    err = np.linalg.norm(mx["u"] - d["u"], axis=0) / np.linalg.norm(d["u"], axis=0)
    out["mixed"]["err_vs_fp64"] = float(err.max())
    out["mixed"]["speedup_vs_fp64"] = round(out["fp64"]["ms_per_step"] / out["mixed"]["ms_per_step"], 3)
    mx["solver"].close()
    del res, mx, d, vals, f
    gc.collect()
    torch.cuda.empty_cache()
    return out


if __name__ == "__main__":
    main()
