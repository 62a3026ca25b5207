"""Benchmark: coupled Stokes-Darcy solves/s on one MI355X.

Workload C2 (default, the headline configuration): 1024 x 512 cells in each
subdomain (N = 2,097,152 unknowns), lognormal permeability
ln K ~ N(ln 1e-4, 1) with an 8-cell Gaussian correlation (seed 2), viscosity
1e-3, parabolic inflow of peak 1e-2, zero-traction outflow;
block-Gauss-Seidel preconditioned FGMRES(60) with one smoothed-aggregation
V-cycle per velocity and Darcy block and the viscosity-scaled pressure-mass
Schur block, to relative residual 1e-8.  One step = one complete solve from
x = 0 with the matrix and the AMG hierarchy resident in HBM.  Mixed
precision is the headline ("mixed": FP32 preconditioner, FP64 Arnoldi
product, orthogonalisation and outer residual); FP64 and "mixed32" (the
Arnoldi product in FP32 too) are reported beside it, and the same solvers on
the 512 x 256 workload (C1, seed 1) under "c1".  --config C1: that workload
as the headline (FP64).  --config T1: the C1 channel as a transient flow
started from rest, 20 backward-Euler steps of dt = 0.1 with the hierarchies
set up once and every step warm-started from the previous state
(Cahouet-Chabard middle block); one step = one time step.  --config C4: the
same on a 3-D channel of 96 x 48 x 96 cells per subdomain (N = 2,207,232).
--config P1: the setup of the paper's experiments replayed with the solvers
built here.  Inputs are synthetic and seeded.  The CPU leg times the oracle
(its FGMRES with the same preconditioner, one thread and all threads, median
of three; SuperLU on the 512 x 256 system) and provides an FP64 reference
solution (its FGMRES to relative residual 1e-12) against which the
per-block errors of every GPU solution are reported, beside their
differences from the oracle's own iterate at the same tolerance.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--config C1|C2|T1|C4|P1] [--no-cpu]
       python bench.py --partitioned [--config C4 --march] | --variants | --serving N | --counter-run
       python bench.py --summarize-counters FETCH_DIR WRITE_DIR --counter-out RUN_JSON
                       --traffic-out OUT_JSON   (no GPU: counter CSVs -> traffic JSON)
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
WORKLOAD = ("512x256 free-flow + 512x256 porous cells (N=524288), lognormal K seed 1, "
            "BGS(SA-AMG V-cycle, mu*Mp^-1, SA-AMG V-cycle) + FGMRES(m), rel. residual 1e-8")
ROOFLINE_KERNEL = {"fp64": "k_arn_project<double, double>",
                   "mixed": "k_arn_project<double, float>",
                   "mixed32": "k_arn_project<float, float>"}
WORKLOAD_C2 = ("1024x512 free-flow + 1024x512 porous cells (N=2097152), lognormal K seed 2, "
               "BGS(SA-AMG V-cycle, mu*Mp^-1, SA-AMG V-cycle) + FGMRES(m), rel. residual 1e-8")


def traffic_file(config):
    return os.path.join(ROOT, "profiles", f"traffic_arnoldi_project_{config.lower()}.json")


def kernels_sha():
    import hashlib
    src = os.path.join(ROOT, "paper_2108_13229_amd", "csrc", "kernels.hip")
    return hashlib.sha256(open(src, "rb").read()).hexdigest()


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="C2", choices=["C1", "C2", "T1", "C4", "P1"])
    ap.add_argument("--paper-n", type=int, default=128,
                    help="P1: cells per unit length of the paper's geometry")
    ap.add_argument("--dn-sub-tol", type=float, default=1e-13,
                    help="P1 and --partitioned: relative residual of the coupling's subdomain solves")
    ap.add_argument("--no-cpu", action="store_true",
                    help="skip the CPU oracle leg (baseline timing and reference solution)")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--precision", default=None, choices=["fp64", "mixed", "mixed32"],
                    help="headline precision (default: fp64 for C1, mixed for C2)")
    ap.add_argument("--restart", type=int, default=60)
    ap.add_argument("--roofline-solves", type=int, default=3)
    ap.add_argument("--serving", type=int, default=0,
                    help="serving mode: replay a seeded trace of this many requests")
    ap.add_argument("--slots", type=int, default=8)
    ap.add_argument("--partitioned", action="store_true",
                    help="the Dirichlet-Neumann coupling (Aitken, IQN-ILS) beside the "
                         "monolithic solve on the chosen 2-D workload")
    ap.add_argument("--march", action="store_true",
                    help="--partitioned on T1/C4: march --steps backward-Euler steps with the "
                         "coupling (Aitken, IQN-ILS) beside the monolithic march")
    ap.add_argument("--variants", action="store_true",
                    help="the monolithic preconditioner variants of the paper's Table 2 "
                         "(pv-BJ/BGS with AMG, td-BJ/BGS with Uzawa and AMG) on the workload")
    ap.add_argument("--counter-run", action="store_true",
                    help="one solve (headline precision) with plain (non-graph) launches plus "
                         "a 512 MiB device copy, for hardware-counter passes")
    ap.add_argument("--counter-out", default=None,
                    help="--counter-run: where to write the run's launches and algorithmic "
                         "bytes (JSON); --summarize-counters: where to read them")
    ap.add_argument("--summarize-counters", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="turn two rocprofv3 --pmc passes (FETCH_SIZE, WRITE_SIZE) of "
                         "--counter-run into the dominant kernel's HBM traffic (no GPU)")
    ap.add_argument("--traffic-out", default=None)
    ap.add_argument("--cpu-repeats", type=int, default=3)
    ap.add_argument("--no-stencil", action="store_true",
                    help="headline solvers read every column index (stencil_slices = 0); "
                         "the results are the same, the time is not")
    ap.add_argument("--no-c1", action="store_true",
                    help="C2: leave out the 512 x 256 solves reported beside the headline")
    return ap.parse_args()


def run_solves(S, steps, warmup):
    import torch
    lat = []
    its = []
    for k in range(warmup + steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, st, rc = S.solve()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        if rc != 0:
            raise RuntimeError(f"solve did not converge (status {rc})")
        if k >= warmup:
            lat.append(dt)
            its.append(st["iters"])
    return np.array(lat), its, st, x.cpu().numpy()


def block_errors(x, ref, off):
    """Relative error per block: velocity (u, v), free-flow and porous pressure."""
    out = []
    for lo, hi in ((off[0], off[2]), (off[2], off[3]), (off[3], off[4])):
        out.append(float(np.linalg.norm(x[lo:hi] - ref[lo:hi]) / np.linalg.norm(ref[lo:hi])))
    return out


def roofline(S, n_solves, precision, config):
    """Dominant kernel (w = A z_j fused with the projection pass of the
    Gram-Schmidt step over the basis): its launches are bracketed by HIP
    events on the solver's stream during n_solves solves of the same
    workload; achieved = algorithmic bytes of those launches / their summed
    durations.  traffic = HBM bytes per launch from the committed counter
    passes (FETCH_SIZE + WRITE_SIZE, copy-calibrated), when they were taken
    on this kernel source, workload and precision."""
    S.profile("arnoldi_spmv")
    for _ in range(n_solves):
        S.solve()
    r = S.profile_read()
    S.profile("off")
    return roofline_from(r, precision, config)


def roofline_from(r, precision, config):
    """The roofline object from a profile read (launches, seconds, bytes of
    the dominant kernel)."""
    achieved = r["bytes"] / r["seconds"] / 1e9
    traffic = None
    try:
        with open(traffic_file(config)) as f:
            t = json.load(f)
        if (t.get("kernels_hip_sha256") == kernels_sha()
                and t.get("kernel") == ROOFLINE_KERNEL[precision]):
            traffic = t["hbm_bytes_per_launch"]
    except (OSError, ValueError, KeyError):
        traffic = None
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "kernel": ROOFLINE_KERNEL[precision], "launches": r["launches"],
            "avg_launch_us": 1e6 * r["seconds"] / r["launches"],
            "alg_bytes_per_launch": r["bytes"] / r["launches"]}


def paper_setting(sd, P, args):
    """The paper's own solver setting on a workload (Sec. 5, Table 2):
    PD-GMRES (m_init = m_min = 3, m_step = 5) with P^pv_BGS(AMG, AMG) and the
    identity middle block, non-smoothed aggregation AMG (MIS(1) roots), one
    V-cycle with two damped-Jacobi sweeps on each side (the parallel stand-in
    for the paper's Gauss-Seidel); FP64, relative residual 1e-8; one warm-up
    and three timed solves."""
    S = sd.Solver(P, krylov="pdgmres", precond="BGS", schur="identity", amg="plain", mis=1,
                  tol=1e-8, restart=args.restart, maxit=20000)
    lat, its, st, _ = run_solves(S, 3, 1)
    S.close()
    return {"solver": "PD-GMRES(3,3,5) + P^pv_BGS(plain-aggregation AMG, identity, "
                      "plain-aggregation AMG), FP64",
            "solves_per_s": float(len(lat) / lat.sum()), "ms_per_solve": float(1e3 * lat.mean()),
            "iters": int(np.median(its)), "restarts": st["restarts"]}


def precond_roofline(S, n_solves):
    """One whole preconditioner application (V-cycles and block sweep, every
    kernel of it): HIP events around each application during n_solves solves
    (launched one by one), against its algorithmic bytes (summed over its
    kernels; each matrix value and index, padding excluded, and each vector
    entry read or written once)."""
    S.profile("precond")
    for _ in range(n_solves):
        S.solve()
    r = S.profile_read()
    S.profile("off")
    b, launches = S.precond_cost()
    t = r["seconds"] / max(1, r["launches"])
    return {"alg_bytes_per_application": b, "launches_per_application": launches,
            "applications": r["launches"], "avg_application_us": 1e6 * t,
            "achieved": b / t / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": b / t / 1e9 / HBM_PEAK_GBS}


def counter_run(sd, p, restart, precision, config, out_path):
    """Kernels launched one by one (no graph replay) so that per-dispatch
    counters attach to each kernel; then a plain 512 MiB device-to-device copy
    whose FETCH_SIZE / WRITE_SIZE calibrate the counters (64 Mi doubles).  The
    solve's launches of the dominant kernel and their algorithmic bytes go to
    out_path for --summarize-counters."""
    import torch
    P = sd.Problem(p, device=True)
    S = sd.Solver(P, precond="BGS", schur="mass", tol=1e-8, restart=restart,
                  precision=precision)
    S.profile("arnoldi_spmv")
    x, st, rc = S.solve()
    torch.cuda.synchronize()
    r = S.profile_read()
    a = torch.ones(64 * 1024 * 1024, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    rec = {"counter_run": True, "config": config, "precision": precision,
           "kernel": ROOFLINE_KERNEL[precision], "iters": st["iters"],
           "launches": r["launches"], "alg_bytes_per_launch": r["bytes"] / r["launches"],
           "copy_bytes": a.numel() * 8, "kernels_hip_sha256": kernels_sha()}
    if out_path:
        with open(out_path, "w") as f:
            json.dump(rec, f, indent=1)
    print(json.dumps(rec))


def _counter_grid_rows(d, counter):
    """(kernel name, grid size, value) per dispatch from a rocprofv3 --pmc CSV
    tree, in dispatch order."""
    import csv
    import glob
    rows = []
    for fn in sorted(glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)):
        with open(fn) as f:
            for rec in csv.DictReader(f):
                if rec.get("Counter_Name") == counter:
                    rows.append((int(rec.get("Dispatch_Id") or 0), rec["Kernel_Name"],
                                 int(rec.get("Grid_Size") or rec.get("Grid_Size_X") or 0),
                                 float(rec["Counter_Value"])))
    return [(n, g, v) for _, n, g, v in sorted(rows, key=lambda t: t[0])]


def _counter_rows(d, counter):
    """(kernel name, value) per dispatch from a rocprofv3 --pmc CSV tree."""
    import csv
    import glob
    files = sorted(glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True))
    if not files:
        raise SystemExit(f"no *counter_collection.csv under {d}")
    rows = []
    for fn in files:
        with open(fn) as f:
            for rec in csv.DictReader(f):
                if rec.get("Counter_Name") == counter:
                    rows.append((int(rec.get("Dispatch_Id") or 0), rec["Kernel_Name"],
                                 float(rec["Counter_Value"])))
    return [(n, v) for _, n, v in sorted(rows, key=lambda t: t[0])]


def summarize_counters(fetch_dir, write_dir, run_json, out_json):
    """HBM traffic per launch of the dominant kernel from two counter passes
    of --counter-run (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch), each
    scaled by the reading of the 512 MiB copy that ends the run.  Launches
    that returned at once (enqueued ahead of the cycle's end: a reading below
    1 % of the median) are left out, and of the others the first as many as
    the run timed (columns j = 0 .. k-1 of the cycle; the launch that closes
    the last column is not in the algorithmic bytes either)."""
    with open(run_json) as f:
        run = json.load(f)
    kern = run["kernel"]
    out = {"kernel": kern, "workload": f"{run['config']} {run['precision']} restart 60, "
                                       f"one solve ({run['launches']} launches)"}
    for counter, d, key in (("FETCH_SIZE", fetch_dir, "fetch"), ("WRITE_SIZE", write_dir,
                                                                  "write")):
        rows = _counter_rows(d, counter)
        copy = [v for n, v in rows if "copyBuffer" in n]
        vals = np.array([v for n, v in rows if kern in n])
        if not copy or vals.size == 0:
            raise SystemExit(f"{counter}: copy kernel or {kern} not found in {d}")
        keep = vals[vals >= 0.01 * np.median(vals)][:run["launches"]]
        scale = run["copy_bytes"] / (max(copy) * 1024.0)
        out[f"{key}_size_kib_per_launch_raw"] = float(keep.mean())
        out[f"{key}_launches_counted"] = int(keep.size)
        out[f"{key}_scale"] = scale
        out[f"{key}_copy_kib"] = max(copy)
        out[f"{key}_bytes_per_launch"] = float(keep.mean()) * 1024.0 * scale
    out["copy_bytes"] = run["copy_bytes"]
    out["hbm_bytes_per_launch"] = out["fetch_bytes_per_launch"] + out["write_bytes_per_launch"]
    out["alg_bytes_per_launch"] = run["alg_bytes_per_launch"]
    out["traffic_over_algorithmic"] = out["hbm_bytes_per_launch"] / run["alg_bytes_per_launch"]
    # every kernel of the run by launch shape: mean HBM bytes per dispatch
    # (both counters scaled as above), launches that did work only
    per = {}
    for counter, d, key in (("FETCH_SIZE", fetch_dir, "fetch"), ("WRITE_SIZE", write_dir,
                                                                  "write")):
        scale = out[f"{key}_scale"]
        for name, grid, v in _counter_grid_rows(d, counter):
            short = name.replace("sd::(anonymous namespace)::", "").replace("void ", "")
            short = short.split("(")[0]
            per.setdefault((short, grid), {"fetch": [], "write": []})[key].append(
                v * 1024.0 * scale)
    out["all_kernels"] = []
    for (name, grid), d in sorted(per.items(), key=lambda kv: -sum(kv[1]["fetch"])):
        f = np.array(d["fetch"])
        w = np.array(d["write"]) if d["write"] else np.zeros(1)
        keep = f >= 0.01 * np.median(f) if f.size else f
        out["all_kernels"].append({"kernel": name, "grid": grid, "dispatches": int(f.size),
                                   "hbm_bytes_per_dispatch": float(f[keep].mean() + w.mean())
                                   if f.size else 0.0})
    out["kernels_hip_sha256"] = run["kernels_hip_sha256"]
    if out["kernels_hip_sha256"] != kernels_sha():
        print("warning: kernels.hip changed since the counter run", file=sys.stderr)
    with open(out_json, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


def replay(sd, probs, arrivals, slots, **opts):
    """Submit each request at its arrival time (seconds after start); returns
    per-request latency (done - arrival) and the makespan."""
    S = sd.Server(max_slots=slots)
    t0 = time.perf_counter()
    tickets = []
    for p, ta in zip(probs, arrivals):
        dt = ta - (time.perf_counter() - t0)
        if dt > 0:
            time.sleep(dt)
        tickets.append((S.submit(p, **opts), time.perf_counter() - t0))
    lat, iters = [], []
    t_end = 0.0
    for (t, t_sub), ta in zip(tickets, arrivals):
        r = S.wait(t, timeout=600, with_x=False)
        if r["status"] != 0:
            raise RuntimeError(f"request failed: {r['status']}")
        # server clock and wall clock share the start within milliseconds;
        # latency = completion - arrival on the server clock
        lat.append(r["t_done"] - (r["t_submit"] - (t_sub - ta)))
        iters.append(r["stats"]["iters"])
        t_end = max(t_end, r["t_done"])
        S.release(t)
    stats = S.batch_stats()
    S.close()
    return np.array(lat), time.perf_counter() - t0, iters, stats


def serving(sd, args):
    """Seeded request stream (grid uniform over 64x32 ... 512x256 per
    subdomain, lognormal K with sigma ~ U[0.5, 2], inflow ~ U[1e-3, 1e-1]):
    saturated throughput with all requests queued at t = 0, then Poisson
    arrivals at 0.9x that rate; baseline: one request at a time in FP64."""
    import torch
    from sdinputs import serving_trace, trace_problem
    n = args.serving
    trace0 = serving_trace(n, rate_per_s=0.0, seed=7)
    probs = [trace_problem(t) for t in trace0]
    # serving pays one AMG setup per solve and is bound by the host CPU time
    # of the preparation: a dense coarse level of at most 512 rows (its
    # inverse costs O(n^3) on the host) gives +17 % saturated throughput for
    # 5 % more iterations than 1024 rows (2048 is the single-solve default),
    # and separate pre-smoothing and restriction passes spare the host the
    # product G = R (I - A M2) (+15-20 %, a few more launches)
    opts = dict(tol=1e-8, restart=args.restart, precision="mixed", coarse_max=512,
                fused_restriction=0)
    lat_sat, span_sat, _, bst_sat = replay(sd, probs, [0.0] * n, args.slots, **opts)
    rate = 0.9 * n / span_sat
    trace = serving_trace(n, rate_per_s=rate, seed=7)
    arr = [t["t_arrival"] for t in trace]
    lat, span, iters, bst = replay(sd, probs, arr, args.slots, **opts)
    # FP64 one request at a time (assembly, setup, solve), same arrivals
    t0 = time.perf_counter()
    lat1 = []
    for p, ta in zip(probs, arr):
        dt = ta - (time.perf_counter() - t0)
        if dt > 0:
            time.sleep(dt)
        P = sd.Problem(p)
        Sv = sd.Solver(P, tol=1e-8, restart=args.restart, coarse_max=512, fused_restriction=0)
        x, st, rc = Sv.solve()
        torch.cuda.synchronize()
        lat1.append(time.perf_counter() - t0 - ta)
        Sv.close()
        P.close()
    span1 = time.perf_counter() - t0
    out = {
        "metric": "Stokes-Darcy serving: solves/s and p50/p99 latency (mixed, continuous batching)",
        "value": n / span, "unit": "solves/s", "n_gpus": 1, "higher_is_better": True,
        "requests": n, "slots": args.slots, "arrival_rate_per_s": rate,
        "saturated_solves_per_s": n / span_sat,
        "p50_ms": 1e3 * float(np.percentile(lat, 50)),
        "p99_ms": 1e3 * float(np.percentile(lat, 99)),
        "median_iters": float(np.median(iters)),
        # shared launches: graph replays, each an Arnoldi column for every
        # active member of a group of same-shape requests
        "shared_launches": {"saturated": dict(bst_sat, columns_per_replay=bst_sat[
                                "member_columns"] / max(1, bst_sat["replays"])),
                            "at_rate": dict(bst, columns_per_replay=bst["member_columns"] /
                                            max(1, bst["replays"]))},
        "fp64_one_at_a_time": {"solves_per_s": n / span1,
                               "p50_ms": 1e3 * float(np.percentile(lat1, 50)),
                               "p99_ms": 1e3 * float(np.percentile(lat1, 99))},
        "data": "synthetic", "dtype": "f32+f64",
        "config": {"workload": "Poisson request stream, grids 64x32..512x256 per subdomain, "
                               "lognormal K sigma U[0.5,2], inflow U[1e-3,1e-1], seed 7",
                   "restart": args.restart, "coarse_max": 512, "fused_restriction": 0},
    }
    # dominant kernel on the largest request of the trace (mixed, as served)
    big = max(probs, key=lambda q: q.nx * q.ny)
    P = sd.Problem(big)
    S = sd.Solver(P, **opts)
    if args.roofline_solves > 0:
        out["roofline"] = roofline(S, args.roofline_solves, "mixed", "serving")
        out["roofline"]["request"] = f"{big.nx}x{big.ny} per subdomain (N={P.N})"
    S.close()
    P.close()
    if not args.no_cpu:
        out["cpu_baseline"] = serving_cpu_baseline(probs, args.restart)
    print(json.dumps(out))


def serving_cpu_baseline(probs, restart, budget_s=20.0):
    """The oracle serving the trace one request at a time on one thread:
    assembly, AMG set-up (coarse levels up to 1024 rows, as served) and the
    FP64 FGMRES solve of each request, in trace order, until budget_s has
    been spent."""
    from threadpoolctl import threadpool_limits
    from oracle import amg, krylov, precond
    from oracle.assemble import assemble
    done = 0
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        for p in probs:
            a = assemble(p)
            M = precond.build(p, a, "BGS", opts=amg.AMGOptions(coarse_max=1024))
            krylov.fgmres(a.A, a.b, M, tol=1e-8, m=restart)
            done += 1
            if time.perf_counter() - t0 > budget_s:
                break
        span = time.perf_counter() - t0
    return dict(value=done / span, unit="solves/s", cores=1, kind="oracle",
                sample=f"the first {done} requests of the trace, each assembled, set up and "
                       f"solved by the oracle one at a time ({span:.1f} s), 1 thread")


WORKLOAD_T1 = ("512x256 free-flow + 512x256 porous cells (N=524288), lognormal K seed 1, "
               "flow from rest, backward Euler dt=0.1, hierarchies set up once; "
               "BGS(SA-AMG V-cycle, Cahouet-Chabard mu*Mp^-1 + SA-AMG(B^T D^-1 B), SA-AMG "
               "V-cycle) + FGMRES(m) warm-started, rel. residual 1e-8 per step")


WORKLOAD_C4 = ("3-D 96x48x96 free-flow + 96x48x96 porous cells (N=2207232), lognormal K "
               "(6-cell correlation, seed 4), flow from rest, backward Euler dt=0.1, hierarchies "
               "set up once; BGS(SA-AMG V-cycle, Cahouet-Chabard mu*Mp^-1 + SA-AMG(B^T D^-1 B), "
               "SA-AMG V-cycle) + FGMRES(m) warm-started, rel. residual 1e-8 per step")


def transient(sd, args, p):
    """Backward-Euler time stepping (T1: the 2-D C1 grid; C4: the 3-D box):
    args.steps steps (default 20) from rest on the step matrix, timed as one
    sd_advance call after an untimed warm-up run of args.warmup steps."""
    import torch
    n_steps = args.steps
    t0 = time.perf_counter()
    P = sd.Problem(p, device=True)
    t_asm = time.perf_counter() - t0
    res = {}
    roof = None
    for prec in ["fp64"] if args.no_mixed else ["fp64", "mixed"]:
        t0 = time.perf_counter()
        S = sd.Solver(P, precond="BGS", schur="cc", tol=1e-8, restart=args.restart,
                      precision=prec)
        t_setup = time.perf_counter() - t0
        if args.warmup > 0:
            xw = torch.zeros(P.N, dtype=torch.float64, device="cuda")
            S.advance(xw, args.warmup)
        x = torch.zeros(P.N, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stats, done, rc = S.advance(x, n_steps)
        torch.cuda.synchronize()
        span = time.perf_counter() - t0
        if rc != 0:
            raise RuntimeError(f"time step {done + 1} failed (status {rc})")
        res[prec] = dict(steps_per_s=n_steps / span, ms_per_step=1e3 * span / n_steps,
                         iters_per_step=[s["iters"] for s in stats],
                         max_rel_res=max(s["rel_res"] for s in stats), setup_s=t_setup)
        if prec == "fp64" and args.roofline_solves > 0:
            roof = roofline(S, args.roofline_solves, prec, args.config)
        S.close()
    # the viscous Schur block alone on the same step system (first step)
    S = sd.Solver(P, precond="BGS", schur="mass", tol=1e-8, restart=args.restart, maxit=300)
    x0, st, rc = S.solve()
    S.close()
    head = res["fp64"]
    out = {
        "metric": "backward-Euler time steps/s to rel. residual 1e-8 per step",
        "value": head["steps_per_s"], "unit": "steps/s", "n_gpus": 1,
        "steps": n_steps, "warmup": args.warmup, "ms_per_step": head["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": WORKLOAD_T1 if args.config == "T1" else WORKLOAD_C4,
                   "N": P.N, "nnz": P.nnz, "dt": p.dt,
                   "assembly_s": t_asm, "precision": "fp64"},
        "restart": args.restart, "fp64": res.get("fp64"), "mixed": res.get("mixed"),
        "viscous_schur_only_step1": {"iters": st["iters"], "status": rc,
                                     "rel_res": st["rel_res"], "maxit": 300},
        "roofline": roof,
    }
    if args.config == "C4":
        out["cpu_baseline"] = None
        out["cpu_baseline_note"] = ("not measured at this size: the oracle's AMG setup alone "
                                    "exceeds the bounded CPU sample")
    elif not args.no_cpu:
        from threadpoolctl import threadpool_limits
        from oracle import krylov, precond
        from oracle.assemble import assemble
        with threadpool_limits(limits=1):
            a = assemble(p)
            M = precond.build(p, a, "BGS", schur=precond.SCHUR_CC)
            t0 = time.perf_counter()
            r = krylov.fgmres(a.A, a.b, M, tol=1e-8, m=args.restart)
            t1 = time.perf_counter() - t0
        out["cpu_baseline"] = dict(
            value=1.0 / t1, unit="steps/s", cores=1, kind="oracle",
            sample=f"the first time step (from rest) of the same workload: oracle FGMRES with "
                   f"the same preconditioner, {r.iters} iterations, {t1:.1f} s; assembly and "
                   f"AMG setup not included; 1 thread")
    print(json.dumps(out))


def partitioned(sd, args, p):
    """Partitioned coupling (Sec. 3) against the monolithic solve on the same
    workload, in FP64 and in mixed precision: solves/s of the
    Dirichlet-Neumann iteration with Aitken and with IQN-ILS (sub-solves to
    --dn-sub-tol, interface tolerance 1e-8, at most 1000 coupling
    iterations), and of the monolithic FGMRES to 1e-8; per-block differences
    of the partitioned solutions from the monolithic one.  A backward-Euler
    workload (C4: the first step of the 3-D box) uses the Cahouet-Chabard
    middle block in the monolithic solve and in the free-flow sub-solve."""
    import torch
    P = sd.Problem(p, device=True)
    schur = "cc" if p.dt > 0 else "mass"
    res = {}
    roof = None
    for prec in ("fp64", "mixed"):
        S = sd.Solver(P, precond="BGS", schur=schur, tol=1e-8, restart=args.restart,
                      precision=prec)
        lat, its, st, xm = run_solves(S, max(1, args.steps // 4), 1)
        r = {"monolithic": dict(solves_per_s=float(len(lat) / lat.sum()),
                                ms_per_solve=float(1e3 * lat.mean()), iters=int(np.median(its)))}
        if prec == "fp64" and args.roofline_solves:
            roof = roofline(S, args.roofline_solves, "fp64", args.config)
        S.close()
        D = sd.Partitioned(P, tol=args.dn_sub_tol, restart=args.restart, precision=prec,
                           schur=schur)
        for accel in ("aitken", "iqn-ils"):
            D.solve(accel=accel, eps=1e-8, maxit=1000)           # warm-up
            ts = []
            for _ in range(max(1, args.steps // 10)):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                x, st, rc = D.solve(accel=accel, eps=1e-8, maxit=1000)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
            r[accel.replace("-", "_")] = dict(
                solves_per_s=1.0 / float(np.mean(ts)), ms_per_solve=1e3 * float(np.mean(ts)),
                coupling_iters=st["iters"], converged=st["converged"],
                ff_fgmres_iters=st["ff_iters"], pm_fgmres_iters=st["pm_iters"],
                diff_vs_monolithic=block_errors(x.cpu().numpy(), xm, P.block_off))
        D.close()
        res[prec] = r
    workload = {"C1": WORKLOAD, "C2": WORKLOAD_C2, "C4": WORKLOAD_C4}.get(args.config, args.config)
    out = {"metric": "Stokes-Darcy solves/s: partitioned Dirichlet-Neumann vs monolithic",
           "value": res["fp64"]["iqn_ils"]["solves_per_s"], "unit": "solves/s", "n_gpus": 1,
           "higher_is_better": True, "dtype": "f64", "data": "synthetic",
           "config": {"workload": workload, "N": P.N, "sub_tol": args.dn_sub_tol, "eps": 1e-8,
                      "maxit": 1000, "schur": schur},
           "monolithic": res["fp64"]["monolithic"], "aitken": res["fp64"]["aitken"],
           "iqn_ils": res["fp64"]["iqn_ils"], "mixed": res["mixed"], "roofline": roof}
    if roof is not None:
        roof["note"] = ("the monolithic solve's dominant kernel; the coupling's subdomain "
                        "solves run the same kernels on the subdomain systems")
    if not args.no_cpu and p.nz == 0:
        out["cpu_baseline"] = dn_cpu_baseline(p, res["fp64"]["iqn_ils"]["coupling_iters"])
    elif not args.no_cpu:
        out["cpu_baseline"] = None
        out["cpu_baseline_note"] = "the oracle's coupling is 2-D only"
    print(json.dumps(out))


def partitioned_march(sd, args, p):
    """A backward-Euler workload (T1, C4) marched args.steps steps from rest
    by the monolithic solver (Cahouet-Chabard middle block, sd_advance) and
    by the partitioned Dirichlet-Neumann coupling (Sec. 3) with Aitken
    relaxation and with IQN-ILS (sub-solves to --dn-sub-tol, interface
    tolerance 1e-8, at most 1000 coupling iterations per step), in FP64 and
    in mixed precision.  Each march sets up once and starts from x = 0; the
    coupling's step right-hand side comes from sd_step_rhs.  Reported: steps/s,
    iterations per step, steps that missed their tolerance and the per-block
    difference of each final state from the monolithic one."""
    import torch
    n_steps = args.steps
    P = sd.Problem(p, device=True)
    res = {}
    roof = None
    for prec in ("fp64", "mixed"):
        r = {}
        S = sd.Solver(P, precond="BGS", schur="cc", tol=1e-8, restart=args.restart,
                      precision=prec)
        xw = torch.zeros(P.N, dtype=torch.float64, device="cuda")
        S.advance(xw, 1)                       # captures the graphs
        x = torch.zeros(P.N, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stats, done, rc = S.advance(x, n_steps)
        torch.cuda.synchronize()
        span = time.perf_counter() - t0
        xm = x.cpu().numpy()
        r["monolithic"] = dict(steps_per_s=n_steps / span, ms_per_step=1e3 * span / n_steps,
                               iters_per_step=[s["iters"] for s in stats], status=rc)
        if prec == "fp64" and args.roofline_solves > 0:
            roof = roofline(S, args.roofline_solves, prec, args.config)
        D = sd.Partitioned(P, tol=args.dn_sub_tol, restart=args.restart, precision=prec,
                           schur="cc")
        for accel in ("aitken", "iqn-ils"):
            x = torch.zeros(P.N, dtype=torch.float64, device="cuda")
            rhs = torch.empty_like(x)
            its, missed = [], []
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for k in range(n_steps):
                S.step_rhs(x, out=rhs)
                x, st, rc = D.solve(accel=accel, eps=1e-8, maxit=1000, b=rhs, x=x)
                its.append(st["iters"])
                if rc != 0:
                    missed.append(k + 1)
                print(f"{prec} {accel} step {k + 1}: {st['iters']} coupling iterations",
                      file=sys.stderr, flush=True)
            torch.cuda.synchronize()
            span = time.perf_counter() - t0
            r[accel.replace("-", "_")] = dict(
                steps_per_s=n_steps / span, ms_per_step=1e3 * span / n_steps,
                coupling_iters_per_step=its, steps_not_converged=missed,
                diff_vs_monolithic=block_errors(x.cpu().numpy(), xm, P.block_off))
            print(f"{prec} {accel}: {span:.1f} s, coupling iterations {its}", file=sys.stderr,
                  flush=True)
        D.close()
        S.close()
        res[prec] = r
    workload = {"T1": WORKLOAD_T1, "C4": WORKLOAD_C4}[args.config]
    out = {"metric": "backward-Euler time steps/s: partitioned Dirichlet-Neumann vs monolithic",
           "value": res["mixed"]["monolithic"]["steps_per_s"], "unit": "steps/s", "n_gpus": 1,
           "steps": n_steps, "higher_is_better": True, "dtype": "f32+f64", "data": "synthetic",
           "config": {"workload": workload, "N": P.N, "nnz": P.nnz, "dt": p.dt,
                      "sub_tol": args.dn_sub_tol, "eps": 1e-8, "maxit": 1000},
           "fp64": res["fp64"], "mixed": res["mixed"], "roofline": roof,
           "cpu_baseline": None,
           "cpu_baseline_note": "the oracle's coupling is 2-D only and its AMG set-up alone "
                                "exceeds a bounded CPU sample at this size"}
    print(json.dumps(out))


def dn_cpu_baseline(p, gpu_iters, sample_iters=20):
    """The oracle's Dirichlet-Neumann iteration with IQN-ILS (exact sparse-LU
    subdomain solves), one thread: the factorisation and sample_iters
    coupling iterations are timed, the remaining iterations up to the count
    the GPU solve needed are extrapolated at the measured rate."""
    from threadpoolctl import threadpool_limits
    from oracle import dn
    from oracle.assemble import assemble
    with threadpool_limits(limits=1):
        a = assemble(p)
        t0 = time.perf_counter()
        subs = dn.subsolvers(p, a)
        t_factor = time.perf_counter() - t0
        t0 = time.perf_counter()
        r = dn.solve_dn(p, a, eps=1e-8, maxit=sample_iters, accel="iqn-ils", subs=subs)
        per_iter = (time.perf_counter() - t0) / len(r.history)
    t_solve = t_factor + gpu_iters * per_iter
    return dict(value=1.0 / t_solve, unit="solves/s", cores=1, kind="oracle",
                sample=f"oracle DN + IQN-ILS with sparse-LU subdomain solves: factorisation "
                       f"{t_factor:.1f} s and {len(r.history)} coupling iterations "
                       f"({per_iter:.3f} s each) timed, extrapolated to the {gpu_iters} "
                       f"iterations of the GPU solve; 1 thread")


def variants(sd, args, p):
    """The iterative monolithic rows of the paper's Table 2 with FGMRES(m):
    P^pv_BJ(AMG, AMG) and P^pv_BGS(AMG, AMG) with the paper's identity middle
    block, P^td_BJ(Uzawa, AMG), P^td_BGS(Uzawa, AMG), P^td_BJ(Uzawa, ILU(0))
    and P^td_BGS(Uzawa, ILU(0)), beside this library's default (pv-BGS with
    mu M_p^-1); FP64, tolerance 1e-8.  The AMG rows run again with the
    paper's outer solver, PD-GMRES (m_init = m_min = 3, m_step = 5, cycles
    capped at the restart length)."""
    P = sd.Problem(p, device=True)
    amg_rows = [("pv-BJ(AMG,AMG), identity", dict(precond="BJ", schur="identity")),
                ("pv-BGS(AMG,AMG), identity", dict(precond="BGS", schur="identity")),
                ("td-BJ(Uzawa,AMG)", dict(precond="TD_BJ")),
                ("td-BGS(Uzawa,AMG)", dict(precond="TD_BGS"))]
    rows = amg_rows + [
        ("td-BJ(Uzawa,ILU(0))", dict(precond="TD_BJ", darcy="ilu0")),
        ("td-BGS(Uzawa,ILU(0))", dict(precond="TD_BGS", darcy="ilu0"))]
    rows += [("PD-GMRES " + n, dict(o, krylov="pdgmres")) for n, o in amg_rows]
    rows += [("PD-GMRES pv-BGS(AMG,AMG), mu*Mp^-1", dict(precond="BGS", schur="mass",
                                                          krylov="pdgmres")),
             ("pv-BGS(AMG,AMG), mu*Mp^-1 (default)", dict(precond="BGS", schur="mass"))]
    out = {"metric": "Stokes-Darcy solves/s per preconditioner variant (FGMRES, FP64, tol 1e-8)",
           "unit": "solves/s", "n_gpus": 1, "dtype": "f64", "data": "synthetic",
           "config": {"workload": WORKLOAD if args.config == "C1" else WORKLOAD_C2,
                      "N": P.N, "restart": args.restart}, "variants": {}}
    roof = None
    for name, o in rows:
        if o.get("darcy") == "ilu0":
            # thousands of iterations at this size: one timed solve, recorded
            # also when it stops at maxit
            import torch
            S = sd.Solver(P, tol=1e-8, restart=args.restart, maxit=20000, **o)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            x, st, rc = S.solve()
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            out["variants"][name] = dict(solves_per_s=float(1.0 / dt), ms_per_solve=1e3 * dt,
                                         iters=st["iters"], converged=rc == 0,
                                         rel_res=st["rel_res"], middle_scale=S.middle_scale())
        else:
            import torch
            S = sd.Solver(P, tol=1e-8, restart=args.restart, maxit=20000, **o)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            x, st, rc = S.solve()
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            if rc != 0 or dt > 2.0:
                # not converged, or too slow to repeat: the one solve is the row
                out["variants"][name] = dict(solves_per_s=float(1.0 / dt), ms_per_solve=1e3 * dt,
                                             iters=st["iters"], restarts=st["restarts"],
                                             converged=rc == 0, rel_res=st["rel_res"],
                                             middle_scale=S.middle_scale())
                S.close()
                continue
            lat, its, st, x = run_solves(S, max(2, args.steps // 4), 0)
            out["variants"][name] = dict(solves_per_s=float(len(lat) / lat.sum()),
                                         ms_per_solve=float(1e3 * lat.mean()),
                                         iters=int(np.median(its)), restarts=st["restarts"],
                                         middle_scale=S.middle_scale())
            if name.endswith("(default)") and args.roofline_solves > 0:
                roof = roofline(S, args.roofline_solves, "fp64", args.config)
        S.close()
    out["value"] = out["variants"]["pv-BGS(AMG,AMG), mu*Mp^-1 (default)"]["solves_per_s"]
    out["roofline"] = roof
    if roof is not None:
        roof["row"] = "pv-BGS(AMG,AMG), mu*Mp^-1 (default)"
    if not args.no_cpu:
        base, _, _, _ = cpu_baseline(p, args.restart, timed=True, reference=False,
                                     repeats=args.cpu_repeats)
        base["row"] = "pv-BGS(AMG,AMG), mu*Mp^-1 (default)"
        out["cpu_baseline"] = base
    print(json.dumps(out))


def paper_replay(sd, args):
    """The setup of the paper's experiments (Sec. 5): a 3 x 1 channel over a
    1 x 1 porous block under its middle third, n x n cells per unit square,
    K = 1e-6, alpha_BJ = 1, viscosity 1e-3, p = 0 under the block, the
    channel driven by a half-cosine pressure difference rising to 1e-9 over
    t_end = 5e6 s, 25 backward-Euler steps of 2e5 s.  Each solver of the
    paper's comparison that is built here marches the 25 steps with its
    set-up done once: monolithic FGMRES with P^pv_BGS (mu M_p^-1 middle
    block) and with P^td_BGS(Uzawa, AMG), and the partitioned
    Dirichlet-Neumann coupling with IQN-ILS (sub-solves to --dn-sub-tol,
    interface tolerance 1e-6: with K = 1e-6 the interface velocity is the
    small difference q_top - sigma of two pressures, resolved only as far as
    the sub-solves are accurate).  Reported: seconds
    for the 25 steps, iterations, steps whose solve did not meet its
    tolerance, and the largest difference of each final state from the first
    solver's."""
    import torch
    from sdinputs import paper_inflow_pressure, paper_setup_problem
    n = args.paper_n
    dt, steps = 2e5, 25
    P0 = sd.Problem(paper_setup_problem(n, 0.0, dt=dt), device=True)
    P1 = sd.Problem(paper_setup_problem(n, 1.0, dt=dt), device=True)
    b0 = torch.from_numpy(np.array(P0.csr()[3])).cuda()
    db = torch.from_numpy(np.array(P1.csr()[3]) - np.array(P0.csr()[3])).cuda()
    out = {"metric": "paper-setup replay: seconds for 25 backward-Euler steps",
           "unit": "s", "n_gpus": 1, "higher_is_better": False, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": f"3x1 channel over 1x1 block, {n} cells per unit length "
                                  f"(N={P0.N}), K=1e-6, half-cosine dp <= 1e-9, 25 steps of 2e5 s",
                      "N": P0.N, "nnz": P0.nnz}, "solvers": {}}
    finals = {}
    runs = [("monolithic FGMRES + P^pv_BGS(AMG, mu Mp^-1, AMG)", "mono", dict(precond="BGS")),
            ("monolithic FGMRES + P^td_BGS(Uzawa, AMG)", "mono", dict(precond="TD_BGS")),
            ("partitioned DN + IQN-ILS", "dn", {})]
    for name, kind, o in runs:
        t0 = time.perf_counter()
        if kind == "mono":
            S = sd.Solver(P0, tol=1e-8, restart=args.restart, maxit=5000, **o)
        else:
            S = sd.Partitioned(P0, tol=args.dn_sub_tol, restart=args.restart)
        torch.cuda.synchronize()
        t_setup = time.perf_counter() - t0
        helper = sd.Solver(P0, tol=1e-8, restart=1) if kind == "dn" else S
        # the march runs twice: the first pass captures the solver's graphs,
        # the second is timed
        for timed in (False, True):
            failed = []
            x = torch.zeros(P0.N, dtype=torch.float64, device="cuda")
            rhs = torch.empty_like(x)
            its = []
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for k in range(1, steps + 1):
                bk = b0 + paper_inflow_pressure(k * dt) * db
                helper.step_rhs(x, b_data=bk, out=rhs)
                if kind == "mono":
                    x, st, rc = S.solve(b=rhs, x=x, use_x0=True)
                else:
                    x, st, rc = S.solve(accel="iqn-ils", eps=1e-6, maxit=500, b=rhs, x=x)
                its.append(st["iters"])
                if rc != 0:
                    failed.append(k)
            torch.cuda.synchronize()
            span = time.perf_counter() - t0
        finals[name] = x.cpu().numpy()
        out["solvers"][name] = dict(seconds=span, ms_per_step=1e3 * span / steps,
                                    setup_s=t_setup, iters_per_step=its,
                                    steps_not_converged=failed)
        S.close()
        if kind == "dn":
            helper.close()
    ref = finals[runs[0][0]]
    for name, x in finals.items():
        out["solvers"][name]["max_diff_vs_first"] = float(np.abs(x - ref).max() / np.abs(ref).max())
    out["value"] = out["solvers"][runs[0][0]]["seconds"]
    # dominant kernel of the first solver: one more (untimed) march with the
    # launches of k_arn_project bracketed by HIP events
    S = sd.Solver(P0, tol=1e-8, restart=args.restart, maxit=5000, precond="BGS")
    S.profile("arnoldi_spmv")
    x = torch.zeros(P0.N, dtype=torch.float64, device="cuda")
    rhs = torch.empty_like(x)
    for k in range(1, steps + 1):
        S.step_rhs(x, b_data=b0 + paper_inflow_pressure(k * dt) * db, out=rhs)
        x, st, rc = S.solve(b=rhs, x=x, use_x0=True)
    out["roofline"] = roofline_from(S.profile_read(), "fp64", "P1")
    S.profile("off")
    S.close()
    if not args.no_cpu:
        out["cpu_baseline"] = p1_cpu_baseline(n, dt, steps, args.restart)
    print(json.dumps(out))


def p1_cpu_baseline(n, dt, steps, restart):
    """The oracle marching the same 25 steps with FGMRES and the same
    pv-BGS preconditioner (set-up once, each step warm-started), one
    thread; seconds for the march, set-up excluded."""
    from threadpoolctl import threadpool_limits
    from oracle import krylov, precond
    from oracle.assemble import assemble
    from oracle.transient import step_rhs
    from sdinputs import paper_inflow_pressure, paper_setup_problem
    with threadpool_limits(limits=1):
        p0 = paper_setup_problem(n, 0.0, dt=dt)
        a0 = assemble(p0)
        db = assemble(paper_setup_problem(n, 1.0, dt=dt)).b - a0.b
        M = precond.build(p0, a0, "BGS")
        x = np.zeros(a0.N)
        t0 = time.perf_counter()
        for k in range(1, steps + 1):
            rhs = step_rhs(a0, a0.b + paper_inflow_pressure(k * dt) * db, x)
            x = krylov.fgmres(a0.A, rhs, M, tol=1e-8, m=restart, x0=x).x
        span = time.perf_counter() - t0
    return dict(value=span, unit="s", cores=1, kind="oracle",
                sample=f"the whole {steps}-step march of the first solver (oracle FGMRES, "
                       f"same preconditioner, set-up excluded), 1 thread")


def host_info():
    """CPU model, logical CPUs and the CPUs this process may run on."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        affinity = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        affinity = None
    return {"cpu_model": model, "nproc": os.cpu_count(), "cpus_available": affinity}


def _blas_threads():
    from threadpoolctl import threadpool_info
    n = [i.get("num_threads", 1) for i in threadpool_info()]
    return max(n) if n else 1


def cpu_baseline(p, restart, timed=True, reference=True, repeats=3):
    """The oracle's FP64 FGMRES with the same preconditioner: set-up once on
    one thread (assembly + AMG, timed separately), then `repeats` full solves
    on one thread (median: the value) and `repeats` with every thread the
    host allows (the oracle's sparse products are single-threaded in SciPy;
    only its dense steps use more).  Also returns the oracle's iterate at the
    same tolerance and, with reference, its FGMRES to relative residual 1e-12
    for the per-block errors of the GPU solutions."""
    from threadpoolctl import threadpool_limits
    from oracle import krylov, precond
    from oracle.assemble import assemble
    base, x_same = None, None
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        a = assemble(p)
        M = precond.build(p, a, "BGS")
        t_setup = time.perf_counter() - t0
        if timed:
            ts = []
            for _ in range(max(1, repeats)):
                t0 = time.perf_counter()
                r = krylov.fgmres(a.A, a.b, M, tol=1e-8, m=restart)
                ts.append(time.perf_counter() - t0)
            x_same = r.x
            t1 = float(np.median(ts))
            base = dict(value=1.0 / t1, unit="solves/s", cores=1, kind="oracle",
                        sample=f"{len(ts)} full FP64 solves of the same workload (oracle FGMRES, "
                               f"same preconditioner, {r.iters} iterations; median "
                               f"{t1:.2f} s, all {', '.join(f'{t:.2f}' for t in ts)} s; "
                               f"assembly + AMG setup {t_setup:.1f} s not included), 1 thread",
                        median_s=t1, runs_s=ts, setup_s=t_setup, iters=r.iters, **host_info())
    if timed:
        ts = []
        for _ in range(max(1, repeats)):
            t0 = time.perf_counter()
            krylov.fgmres(a.A, a.b, M, tol=1e-8, m=restart)
            ts.append(time.perf_counter() - t0)
        base["all_threads"] = dict(value=1.0 / float(np.median(ts)), unit="solves/s",
                                   threads=_blas_threads(), median_s=float(np.median(ts)),
                                   runs_s=ts)
    if not reference:
        return base, None, None, x_same
    ref = krylov.fgmres(a.A, a.b, M, tol=1e-12, m=restart, maxit=5000)
    rel = float(np.linalg.norm(a.b - a.A @ ref.x) / np.linalg.norm(a.b))
    return (base, ref.x,
            f"oracle FP64 FGMRES to relative residual {rel:.1e} ({ref.iters} iterations)",
            x_same)


def direct_baseline(config="C1"):
    """SciPy's SuperLU (sparse LU with COLAMD ordering; the analogue of the
    paper's UMFPACK direct solver) on a workload, one factorisation and one
    solve, on the threads the host allows."""
    import scipy.sparse.linalg as spla
    from oracle.assemble import assemble
    from sdinputs import config_problem
    a = assemble(config_problem(config))
    A = a.A.tocsc()
    t0 = time.perf_counter()
    lu = spla.splu(A)
    t1 = time.perf_counter()
    x = lu.solve(a.b)
    t2 = time.perf_counter()
    rel = float(np.linalg.norm(a.b - a.A @ x) / np.linalg.norm(a.b))
    return dict(kind="SciPy SuperLU", workload=config, N=int(a.N), nnz=int(A.nnz),
                factor_s=t1 - t0, solve_s=t2 - t1, solves_per_s=1.0 / (t2 - t0),
                nnz_LU=int(lu.L.nnz + lu.U.nnz), rel_res=rel)


def headline_solves(sd, P, precs, args, roof_prec, config):
    """args.warmup + args.steps solves per precision on one problem; the
    dominant kernel's roofline for roof_prec."""
    res, xs, roof = {}, {}, None
    for prec in precs:
        t0 = time.perf_counter()
        S = sd.Solver(P, precond="BGS", schur="mass", tol=1e-8, restart=args.restart,
                      precision=prec, stencil_slices=0 if args.no_stencil else 1)
        t_setup = time.perf_counter() - t0
        lat, its, st, x = run_solves(S, args.steps, args.warmup)
        xs[prec] = x
        res[prec] = dict(solves_per_s=float(len(lat) / lat.sum()),
                         ms_per_solve=float(1e3 * lat.mean()),
                         p50_ms=float(1e3 * np.percentile(lat, 50)),
                         p99_ms=float(1e3 * np.percentile(lat, 99)),
                         iters=int(np.median(its)), restarts=st["restarts"],
                         rel_res=st["rel_res"], setup_s=t_setup)
        if prec == roof_prec and args.roofline_solves > 0:
            roof = roofline(S, args.roofline_solves, prec, config)
            res[prec]["preconditioner"] = precond_roofline(S, args.roofline_solves)
        S.close()
    return res, xs, roof


def main():
    args = parse()
    if args.summarize_counters:
        summarize_counters(*args.summarize_counters, args.counter_out, args.traffic_out)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "the solver has no multi-GPU path", file=sys.stderr)
        sys.exit(2)
    import torch
    from sdinputs import config_problem
    from paper_2108_13229_amd import sd

    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(1)
    if args.serving:
        serving(sd, args)
        return
    if args.config == "P1":
        paper_replay(sd, args)
        return
    p = config_problem(args.config)
    if args.partitioned:
        if p.dt > 0 and args.march:
            partitioned_march(sd, args, p)
        else:
            partitioned(sd, args, p)
        return
    if args.config in ("T1", "C4"):
        transient(sd, args, p)
        return
    if args.variants:
        variants(sd, args, p)
        return
    headline = args.precision or ("fp64" if args.config == "C1" else "mixed")
    if args.counter_run:
        counter_run(sd, p, args.restart, headline, args.config, args.counter_out)
        return
    t0 = time.perf_counter()
    P = sd.Problem(p, device=True)
    t_asm = time.perf_counter() - t0
    precs = ["fp64"] if args.no_mixed else ["fp64", "mixed", "mixed32"]
    if headline not in precs:
        precs.append(headline)
    res, xs, roof = headline_solves(sd, P, precs, args, headline, args.config)
    head = res[headline]
    out = {
        "metric": "Stokes-Darcy solves/s to rel. residual 1e-8 (mixed vs FP64), p50/p99 latency",
        "value": head["solves_per_s"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_solve"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if headline == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": WORKLOAD if args.config == "C1" else WORKLOAD_C2,
                   "N": P.N, "nnz": P.nnz, "assembly_s": t_asm, "precision": headline,
                   "stencil_slices": 0 if args.no_stencil else 1},
        "p50_ms": head["p50_ms"],
        "p99_ms": head["p99_ms"],
        "restart": args.restart,
        "fp64": res.get("fp64"),
        "mixed": res.get("mixed"),
        "mixed32": res.get("mixed32"),
        "roofline": roof,
    }
    if args.config == "C2" and not args.no_c1:
        # the 512 x 256 workload with the same solvers, beside the headline
        from sdinputs import config_problem as cp
        P1 = sd.Problem(cp("C1"), device=True)
        r1, _, roof1 = headline_solves(sd, P1, ["fp64", "mixed"], args, "fp64", "C1")
        out["c1"] = {"workload": WORKLOAD, "N": P1.N, "nnz": P1.nnz, **r1, "roofline": roof1}
        out["c1"]["paper_setting"] = paper_setting(sd, P1, args)
        P1.close()
    if not args.no_cpu:
        base, ref, ref_kind, x_same = cpu_baseline(p, args.restart,
                                                   timed=args.config in ("C1", "C2"),
                                                   repeats=args.cpu_repeats)
        if base is not None:
            if args.config == "C2":
                base["direct"] = direct_baseline("C1")
            out["cpu_baseline"] = base
        off = P.block_off
        acc = {"reference": ref_kind, "blocks": ["velocity", "free-flow pressure",
                                                 "porous pressure"]}
        for prec, x in xs.items():
            acc[prec] = block_errors(x, ref, off)
        acc["mixed_vs_fp64"] = block_errors(xs.get("mixed", xs[headline]), xs["fp64"], off)
        if x_same is not None:
            # parity: each GPU iterate against the oracle's own FGMRES iterate at
            # the same tolerance and restart
            acc["vs_oracle_iterate_same_tol"] = {prec: block_errors(x, x_same, off)
                                                 for prec, x in xs.items()}
        # tolerance at which the FP64 solve's error is <= 1e-8 in every block
        need = None
        for tol in (1e-9, 1e-10, 1e-11):
            S = sd.Solver(P, precond="BGS", schur="mass", tol=tol, restart=args.restart)
            x, st, rc = S.solve()
            e = block_errors(x.cpu().numpy(), ref, off)
            S.close()
            if max(e) <= 1e-8:
                need = {"tol": tol, "iters": st["iters"], "errors": e}
                break
        acc["fp64_tol_for_1e-8_error"] = need
        out["accuracy"] = acc
    print(json.dumps(out))


if __name__ == "__main__":
    main()
