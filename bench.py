#!/usr/bin/env python3
"""Benchmark of the subspace-accelerated Poisson sequence on one MI355X.

    python bench.py [--gpus 1] [--steps 20] [--warmup 5] [--workload periodic_16385x33]

A step is one LSERK45 time step of the synthetic simulation: five sequential mixed-stage
Poisson solves (one per Runge-Kutta stage), each from the EWMA-subspace initial guess
(Alg. 2 with the sketch of Alg. 4), GMRES to relative residual 1e-8 with the still-water
V-cycle preconditioner, FP64. The default workload is the large single simulation
(periodic 16385 x 33, n = 557 056, GMRES(40), rank 16). Inputs (surfaces at the stage times,
manufactured right-hand sides b = A p* formed by the library's own operator) are resident in
HBM before the timed region starts. The same steps are then solved from the previous
solution (the paper's baseline) and from a cold start (the plain path). Extra legs: the bar,
FP32 refinement, ILU(0), and the closed loop (Alg. 1: right-hand sides from the velocity field
of an Airy wave on the same grid, every guess mode). Prints one JSON line; progress goes to
stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
RANGE_WINDOW = 20  # K of the range-finder comparison (Alg. 3; the paper's bar runs use K = 20)
# kernel sources whose hash keys the committed counter summaries
KERNEL_SOURCES = ("paper_2511_18071_amd/csrc/device.h", "paper_2511_18071_amd/csrc/solve64.hip",
                  "paper_2511_18071_amd/csrc/internal.h", "paper_2511_18071_amd/csrc/api.hip")


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def counters_path(workload: str) -> str:
    return os.path.join(ROOT, "profiles", f"sa_solve_kernel_{workload}_counters.md")


def read_fields(path: str) -> dict:
    fields = {}
    try:
        text = open(path).read()
    except OSError:
        return fields
    for line in text.splitlines():
        if line.startswith("- ") and ": " in line:
            k, v = line[2:].split(": ", 1)
            fields[k.strip("` ")] = v.strip("` ")
    return fields


def measured_traffic(workload: str, steps: int, warmup: int, cluster: int):
    """HBM bytes per EWMA launch of the solve kernel from the committed counter summary of the
    workload, or None when it was taken on other kernel sources or another run configuration."""
    f = read_fields(counters_path(workload))
    try:
        same = (f["kernel-source-sha256"] == kernel_hash() and f["workload"] == workload
                and int(f["steps"]) == steps and int(f["warmup"]) == warmup and int(f["cluster"]) == cluster)
        return float(f["hbm-bytes-per-launch"]) if same else None
    except (KeyError, ValueError):
        return None


def parse(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="periodic_16385x33")
    ap.add_argument("--cluster", type=int, default=0, help="workgroups per solve (0 = size rule)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extra", action="store_true",
                    help="only the EWMA run (no previous/cold comparison, phases or bar leg)")
    ap.add_argument("--serve-sims", type=int, default=256, help="serving: simulations")
    ap.add_argument("--serve-systems", type=int, default=10, help="serving: systems per simulation")
    ap.add_argument("--serve-rate", type=float, default=None,
                    help="serving: offered solves/s of the open loop (default: 0.7 x the measured saturation rate)")
    ap.add_argument("--serve-inflight", type=int, default=8,
                    help="serving: ticks in flight (the process is given as many hardware queues)")
    ap.add_argument("--serve-upw", type=int, default=10000,
                    help="serving: unknowns per workgroup when the server sizes the clusters")
    ap.add_argument("--serve-precision", default="fp32_ir", choices=["fp32_ir", "fp64"],
                    help="serving: precision of the batched solves (the configuration's FP32 inner GMRES with FP64 "
                         "refinement, or FP64 throughout)")
    ap.add_argument("--serve-baseline-stride", type=int, default=8,
                    help="serving: the one-at-a-time FP64 baseline solves every k-th simulation")
    ap.add_argument("--operator-probe", default="", metavar="WORKLOAD",
                    help="only apply the operator of WORKLOAD's first system 50 times and print its rate")
    ap.add_argument("--operator3d-probe", default="", metavar="GRID",
                    help="time only the three-dimensional operator kernel on a wave field, e.g. 513x513x17_p_p")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES bytes five times (the "
                         "reference kernel that scales HBM counter readings)")
    return ap.parse_args(argv)


def default_cluster(w) -> int:
    # the library's own default: one workgroup per 32-column tile of the finest level, at most 256
    return int(min(256, max(1, (w.ncol + 31) // 32)))


def traffic_bytes(w, infos, pcv, k) -> float:
    """Algorithmic HBM bytes of the solves in `infos`, in vectors of n FP64 values.

    guess            3k + 3   read Y_old and x, write Y_new, read b (block operator + Gram),
                              read Y_new, write x0
    r0 = b - A x0    3        read x0 and b, write r0
    cycle start      pcv + 1  V-cycle of r and its norm (once per cycle; the first one also
                              sets the check trigger)
    Arnoldi step j   2 + pcv + 3j + 8
                              operator (read v_j, write t), V-cycle, CGS2 in three passes over
                              V_0..V_j and w: dots (j+2), update + dots (j+3), update + norm (j+3)
    check / cycle end  j + 6  x + V y (read j+1 basis vectors and x, write) and b - A x (3)
    """
    vb = 8.0 * w.n
    m = w.restart
    total = 0.0
    for inf in infos:
        v = (3 * k + 3) + 3
        if inf.iters > 0:
            cycles = inf.restarts + 1
            v += cycles * (pcv + 1)
            for step in range(inf.iters):
                j = step % m
                v += 2 + pcv + 3 * j + 8
            jbar = min(inf.iters, m) / 2.0
            v += (inf.checks + cycles) * (jbar + 6)
        total += v * vb
    return total


def precond_vectors(w) -> float:
    """Vectors moved by one V(1, nu2) cycle of the still-water preconditioner: per level the
    down pass reads f and writes u and the coarse f (2.5), the first up pass reads u, f and
    the coarse correction and writes the output (3.5), every further post-sweep reads its
    input and f and writes its output (3); levels halve in size, so the hierarchy moves
    (6 + 3 (nu2 - 1)) x (1 + 1/2 + 1/4 + ...) fine-grid vectors: 12 for V(1,1), 18 for V(1,2)."""
    return 2.0 * (6.0 + 3.0 * (getattr(w, "nu2", 1) - 1))


def stage_inputs(B, w, nsys, G):
    """Surfaces, manufactured solutions p* and right-hand sides b = A p* of the first nsys
    systems, resident on the device."""
    import torch
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    etas = torch.empty((nsys, 2, w.nphys), dtype=torch.float64, device=dev)
    bs = torch.empty((nsys, w.n), dtype=torch.float64, device=dev)
    ps = torch.empty((nsys, w.n), dtype=torch.float64, device=dev)
    with B.Problem.from_workload(w, stream=stream, cluster=G, precond="none", guess="cold") as gen:
        for s in range(nsys):
            ep, ec, pst = w.system(s)
            etas[s, 0].copy_(torch.from_numpy(ep))
            etas[s, 1].copy_(torch.from_numpy(ec))
            ps[s].copy_(torch.from_numpy(pst))
            torch.cuda.synchronize()
            gen.set_surface(etas[s, 0], etas[s, 1])
            gen.apply_operator(ps[s], bs[s])
    torch.cuda.synchronize()
    return etas, bs, ps


def run_sequence(B, w, etas, bs, ps, mode, warmup_steps, steps, G, xs=None, **opts):
    """One guess mode over the staged systems: 5 * warmup_steps untimed solves, then 5 * steps
    timed ones. Every solve kernel launch is bracketed by events on the problem's stream (the
    warm-up launches too, so the mean launch time covers the same launches as a kernel trace of
    the process). Returns wall time of the timed solves, reports, event latencies and the
    per-solve errors against p*."""
    import torch
    stream = torch.cuda.current_stream()
    nw, nt = 5 * warmup_steps, 5 * steps
    p = B.Problem.from_workload(w, stream=stream, cluster=G, guess=mode, **opts)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * (nw + nt))]
    if xs is None:
        xs = torch.empty((nw + nt, w.n), dtype=torch.float64, device="cuda:0")
    for s in range(nw):
        p.set_surface(etas[s, 0], etas[s, 1])
        p.push_rhs(bs[s])
        ev[2 * s].record(stream)
        p.solve(sync=False)
        ev[2 * s + 1].record(stream)
        p.solution_async(xs[s])
    warm_infos = p.read_log()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(nw, nw + nt):
        p.set_surface(etas[s, 0], etas[s, 1])
        p.push_rhs(bs[s])
        ev[2 * s].record(stream)
        p.solve(sync=False)
        ev[2 * s + 1].record(stream)
        p.solution_async(xs[s])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    infos = p.read_log()
    p.close()
    lat = np.array([ev[2 * i].elapsed_time(ev[2 * i + 1]) for i in range(nw + nt)])
    # forward error against the manufactured solution, per solve (after the timed region)
    err = ((xs[: nw + nt] - ps[: nw + nt]).norm(dim=1) / ps[: nw + nt].norm(dim=1)).cpu().numpy()
    all_infos = warm_infos + infos
    bad = [i for i in infos if i.status != 0 or i.relres > opts.get("rtol", w.rtol)]
    return dict(wall=wall, infos=infos, all_infos=all_infos, lat=lat[nw:], all_lat=lat, failed=len(bad),
                err=err, nw=nw, xs=xs)


def summary(w, r, nsol):
    its = np.array([i.iters for i in r["infos"]])
    nw = r["nw"]
    rel = np.array([i.relres for i in r["infos"]])
    return {"value": round(nsol / r["wall"], 3), "iters_per_solve": round(float(its.mean()), 3),
            "p50_solve_ms": round(float(np.percentile(r["lat"], 50)), 4),
            "p99_solve_ms": round(float(np.percentile(r["lat"], 99)), 4),
            "max_relres": float(rel.max()), "failed_solves": r["failed"],
            "err_vs_pstar_max": float(r["err"][nw:].max()), "err_vs_pstar_median": float(np.median(r["err"][nw:]))}


def closed_loop_leg(B, w, G, rtol, warmup_steps=2, steps=10, steepness=0.05):
    """The closed loop (Alg. 1) on the workload's periodic grid: LSERK45 steps of size w.dtau
    from an Airy wave of the carrier wavenumber (height steepness x wavelength), each stage's
    pressure right-hand side built on the device from the velocity field and solved with the
    guess mode under test, to relative residual rtol. Reports solves/s over the timed steps
    (right-hand-side kernels and the per-stage report included), Arnoldi steps per solve, and
    how far the final states of the modes lie apart."""
    import torch
    from paper_2511_18071_amd import workload as W
    eta0, u0, w0 = W.airy_state(w, steepness)
    out, finals = {}, {}
    for mode in ("ewma", "previous", "cold"):
        p = B.Problem.from_workload(w, stream=torch.cuda.current_stream(), cluster=G, guess=mode, rtol=rtol)
        loop = B.ClosedLoop(p, w.dtau)
        loop.set_state(eta0, u0, w0)
        for _ in range(warmup_steps):
            loop.step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        infos, step_ms = [], []
        for _ in range(steps):
            t1 = time.perf_counter()
            infos += loop.step()
            step_ms.append(1e3 * (time.perf_counter() - t1))
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        finals[mode] = loop.state()
        loop.close()
        p.close()
        its = np.array([i.iters for i in infos])
        out[mode] = {"value": round(len(infos) / wall, 3), "iters_per_solve": round(float(its.mean()), 3),
                     "ms_per_step": round(float(np.mean(step_ms)), 4),
                     "max_relres": float(max(i.relres for i in infos)),
                     "failed_solves": int(sum(1 for i in infos if i.status != 0 or i.relres > rtol))}
        say(f"  closed loop rtol {rtol:g} {mode}: {out[mode]['value']:.2f} solves/s, {out[mode]['iters_per_solve']} steps/solve")
    e_ref, u_ref, _ = finals["cold"]
    diff = {m: float(max(np.abs(finals[m][0] - e_ref).max() / np.abs(e_ref).max(),
                         np.abs(finals[m][1] - u_ref).max() / np.abs(u_ref).max())) for m in ("ewma", "previous")}
    mass = abs(float(finals["ewma"][0].mean()) - float(eta0.mean())) / float(np.abs(eta0).max())
    return dict(out, speedup_vs_previous=round(out["ewma"]["value"] / out["previous"]["value"], 3),
                speedup_vs_plain=round(out["ewma"]["value"] / out["cold"]["value"], 3),
                state_diff_vs_cold=diff, mean_surface_drift_rel=mass,
                rtol=rtol, initial="Airy wave, carrier wavenumber, H/L = %g" % steepness, dtau=w.dtau,
                steps=steps, warmup=warmup_steps, cluster_workgroups=G)


def phase_breakdown(B, w, etas, bs, G, nsys=10):
    """Device time per phase of the first nsys EWMA solves (profile mode: the first workgroup
    reads the clock at each phase boundary)."""
    import torch
    stream = torch.cuda.current_stream()
    p = B.Problem.from_workload(w, stream=stream, cluster=G, profile=1)
    for s in range(nsys):
        p.set_surface(etas[s, 0], etas[s, 1])
        p.push_rhs(bs[s])
        p.solve(sync=False)
    infos = p.read_log()
    t, det = p.phase_times(detail=True)
    p.close()
    total = t["total"]
    nlev = int(np.count_nonzero(det[1:49:2] > 0)) + 1
    return {"solves": nsys, "iters": int(sum(i.iters for i in infos)), "total_ms": round(total, 3),
            "share": {k: round(v / total, 4) for k, v in t.items() if k != "total"},
            "precond_ms": {"coarsest": round(float(det[0]), 3),
                           "down": [round(float(det[1 + 2 * l]), 3) for l in range(nlev)],
                           "up": [round(float(det[2 + 2 * l]), 3) for l in range(nlev)],
                           "tail_wait": round(float(det[48]), 3)}}


def cpu_baseline(w, gpu_x0, gpu_info0):
    """The FP64 oracle on the host cores, on a bounded sample of the same workload: the first
    system of the sequence (the history is empty there, so the first solve of every guess mode
    starts cold), timed with BLAS limited to one thread and with all threads. Its solution is
    also the reference for the GPU's first solve (decisions and solution difference)."""
    from threadpoolctl import threadpool_info, threadpool_limits

    from oracle.sequence import Simulation

    ep, ec, pst = w.system(0)
    legs = {}
    ref = None
    for label, limit in (("one_thread", 1), ("all_threads", None)):
        with threadpool_limits(limits=limit):
            threads = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
            sim = Simulation.from_workload(w)
            b = sim.operator(ep, ec) @ pst
            t0 = time.perf_counter()
            res = sim.solve(ep, ec, b)  # assembles the system's operator, guesses, runs GMRES
            dt = time.perf_counter() - t0
        legs[label] = dict(seconds=round(dt, 3), threads=int(threads if limit is None else 1), iters=res.info.iters)
        say(f"  cpu baseline {label}: {dt:.1f} s, {res.info.iters} iterations")
        ref = res
    one = legs["one_thread"]
    allc = legs["all_threads"]
    dx = float(np.linalg.norm(gpu_x0 - ref.x) / np.linalg.norm(ref.x))
    same = (gpu_info0.iters, gpu_info0.restarts, gpu_info0.checks) == (ref.info.iters, ref.info.restarts, ref.info.checks)
    nproc = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return {
        "value": round(1.0 / one["seconds"], 5), "unit": "solves/s", "cores": 1, "kind": "oracle",
        "sample": (f"system 0 of {w.name} (empty history, so a cold solve: {one['iters']} GMRES({w.restart}) "
                   f"iterations; the oracle assembles the system's operator, applies the still-water V-cycle, "
                   f"CGS2 and true-residual checks in FP64 NumPy/SciPy), one BLAS thread"),
        "ms_per_iteration": round(1e3 * one["seconds"] / max(1, one["iters"]), 3),
        "all_cores": {"value": round(1.0 / allc["seconds"], 5), "cores": allc["threads"], "nproc": nproc,
                      "ms_per_iteration": round(1e3 * allc["seconds"] / max(1, allc["iters"]), 3)},
        "gpu_vs_oracle_system0": {"same_decisions": bool(same), "gpu_iters": gpu_info0.iters,
                                  "oracle_iters": ref.info.iters, "solution_rel_diff": dx,
                                  "oracle_relres": float(ref.info.relres), "gpu_relres": float(gpu_info0.relres)},
    }


def run_main(args):
    import torch
    from paper_2511_18071_amd import binding as B
    from paper_2511_18071_amd import workload as W

    w = W.get(args.workload)
    G = args.cluster or default_cluster(w)
    nsys = 5 * (args.warmup + args.steps)
    nsol = 5 * args.steps
    say(f"bench: {w.name} n={w.n}, {nsys} systems, cluster {G}")
    t0 = time.perf_counter()
    etas, bs, ps = stage_inputs(B, w, nsys, G)
    say(f"  inputs staged ({time.perf_counter() - t0:.1f} s)")
    xs = torch.empty((nsys, w.n), dtype=torch.float64, device="cuda:0")
    ewma = run_sequence(B, w, etas, bs, ps, "ewma", args.warmup, args.steps, G, xs)
    x0 = xs[0].cpu().numpy()
    info0 = ewma["all_infos"][0]
    say(f"  ewma: {nsol / ewma['wall']:.2f} solves/s")
    out_modes = {}
    if not args.no_extra:
        if w.r != 0.9:  # the same systems with the forgetting factor of the other configurations
            r9 = run_sequence(B, w, etas, bs, ps, "ewma", args.warmup, args.steps, G, xs, r=0.9)
            out_modes["ewma_r0.9"] = r9
            say(f"  ewma r=0.9: {nsol / r9['wall']:.2f} solves/s")
        for mode in ("previous", "cold", "range", "range_q"):
            extra = dict(window=RANGE_WINDOW) if mode.startswith("range") else {}
            if mode == "range_q":
                extra["orthonormalize"] = 1
            r = run_sequence(B, w, etas, bs, ps, mode.split("_")[0], args.warmup, args.steps, G, xs, **extra)
            out_modes[mode] = r
            say(f"  {mode}: {nsol / r['wall']:.2f} solves/s")
    value = nsol / ewma["wall"]
    kernel_ms = float(ewma["all_lat"].mean())
    pcv = precond_vectors(w)
    bytes_per = traffic_bytes(w, ewma["all_infos"], pcv, w.k) / len(ewma["all_infos"])
    achieved = bytes_per / (kernel_ms * 1e-3) / 1e9
    traffic = measured_traffic(w.name, args.steps, args.warmup, G)
    s = summary(w, ewma, nsol)
    out = {
        "metric": "solves/s @relres 1e-8 (subspace vs plain), iters/solve, p99 solve latency",
        "value": round(value, 3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * ewma["wall"] / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "nx": w.nx, "nz": w.nz, "bc": w.bc, "unknowns": w.n,
                   "systems_per_step": 5, "restart": w.restart, "rtol": w.rtol, "precond": f"still-water V(1,{w.nu2})",
                   "guess": f"EWMA rank {w.k}, r={w.r}, column drop {w.tau_drop:g}", "cluster_workgroups": G},
        "iters_per_solve": s["iters_per_solve"],
        "p50_solve_ms": s["p50_solve_ms"],
        "p99_solve_ms": s["p99_solve_ms"],
        "failed_solves": s["failed_solves"],
        "errors": {"max_relres": s["max_relres"], "err_vs_pstar_max": s["err_vs_pstar_max"],
                   "err_vs_pstar_median": s["err_vs_pstar_median"],
                   "per_solve_relres": [float("%.3e" % i.relres) for i in ewma["infos"]],
                   "per_solve_err_vs_pstar": [float("%.3e" % e) for e in ewma["err"][ewma["nw"]:]]},
    }
    if out_modes:
        sp = summary(w, out_modes["previous"], nsol)
        sc = summary(w, out_modes["cold"], nsol)
        out["previous"] = dict(sp, guess="previous solution (the paper's baseline)")
        out["plain"] = dict(sc, guess="cold (x0 = 0)")
        out["range_finder"] = dict(summary(w, out_modes["range"], nsol),
                                   guess=f"Alg. 3 range finder, V = X Omega, window K = {RANGE_WINDOW}, k = {w.k}")
        out["range_finder_q"] = dict(summary(w, out_modes["range_q"], nsol),
                                     guess=f"Alg. 3 range finder, V = Q (orthonormalised), window K = {RANGE_WINDOW}, k = {w.k}")
        out["speedup_vs_plain"] = round(out_modes["cold"]["wall"] / ewma["wall"], 3)
        if "ewma_r0.9" in out_modes:
            out["ewma_r0.9"] = dict(summary(w, out_modes["ewma_r0.9"], nsol), guess=f"EWMA rank {w.k}, r=0.9")
        out["speedup_vs_previous"] = round(out_modes["previous"]["wall"] / ewma["wall"], 3)
    out["roofline"] = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": round(achieved / HBM_PEAK_GBS, 5),
                       "traffic": round(traffic) if traffic else None,
                       "traffic_frac": round(traffic / (kernel_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 5) if traffic else None,
                       "kernel_source_sha256": kernel_hash(),
                       "kernel": "sa_solve_kernel", "kernel_ms": round(kernel_ms, 4),
                       "launches": len(ewma["all_infos"]),
                       "algorithmic_bytes_per_launch": round(bytes_per)}
    if not args.no_extra:
        out["phases"] = phase_breakdown(B, w, etas, bs, G)
        out["mfma_share"] = 0.0
        say("  phases done")
    del etas, bs, ps
    torch.cuda.empty_cache()
    if not args.no_extra and w.bc == "periodic" and w.kind == "stream":
        # at the benchmark's tolerance and at the paper's (1e-4, Sec. 5.2)
        leg = {}
        for rt in (w.rtol, 1e-4):
            try:
                leg[f"rtol_{rt:g}"] = closed_loop_leg(B, w, G, rt)
            except B.SawaveError as err:  # a stage that did not converge ends the leg, not the line
                leg[f"rtol_{rt:g}"] = {"error": str(err)}
                say(f"  closed loop rtol {rt:g}: {err}")
        out[f"closed_loop_{w.name}"] = leg
        say("  closed-loop leg done")
    if not args.no_extra and w.name != "bar_513x17":
        wb = W.get("bar_513x17")
        Gb = default_cluster(wb)
        e2, b2, p2 = stage_inputs(B, wb, 5 * 25, Gb)
        rb = run_sequence(B, wb, e2, b2, p2, "ewma", 5, 20, Gb)
        rc = run_sequence(B, wb, e2, b2, p2, "cold", 5, 20, Gb)
        rp = run_sequence(B, wb, e2, b2, p2, "previous", 5, 20, Gb)
        rr = run_sequence(B, wb, e2, b2, p2, "range", 5, 20, Gb, window=RANGE_WINDOW)
        rq = run_sequence(B, wb, e2, b2, p2, "range", 5, 20, Gb, window=RANGE_WINDOW, orthonormalize=1)
        its = lambda r: round(float(np.mean([i.iters for i in r["infos"]])), 3)
        out["bar_513x17"] = dict(summary(wb, rb, 100), plain_value=round(100 / rc["wall"], 3),
                                 plain_iters_per_solve=its(rc),
                                 previous_value=round(100 / rp["wall"], 3), previous_iters_per_solve=its(rp),
                                 range_finder_value=round(100 / rr["wall"], 3), range_finder_iters_per_solve=its(rr),
                                 range_finder_q_value=round(100 / rq["wall"], 3), range_finder_q_iters_per_solve=its(rq),
                                 steps=20, warmup=5, cluster_workgroups=Gb, guess=f"EWMA rank {wb.k}, r={wb.r}")
        # the forgetting factors the bar's configuration names
        sweep = {}
        for rr in (0.8, 0.9, 0.95):
            r_ = rb if rr == wb.r else run_sequence(B, wb, e2, b2, p2, "ewma", 5, 20, Gb, r=rr)
            sweep[f"r_{rr:g}"] = {"value": round(100 / r_["wall"], 3), "iters_per_solve": its(r_),
                                  "failed_solves": r_["failed"]}
        out["bar_513x17"]["forgetting_sweep"] = sweep
        say("  bar leg done")
        # the precision variant of the bar: FP32 inner GMRES with FP64 refinement against the
        # all-FP64 path, both to relative residual 1e-10 on the FP64 residual, same systems
        tight = 1e-10
        r64 = run_sequence(B, wb, e2, b2, p2, "ewma", 5, 20, Gb, rtol=tight)
        r32 = run_sequence(B, wb, e2, b2, p2, "ewma", 5, 20, Gb, rtol=tight, precision="fp32_ir")
        nw = r64["nw"]
        dx = ((r32["xs"] - r64["xs"]).norm(dim=1) / r64["xs"].norm(dim=1)).cpu().numpy()[nw:]

        def prec_summary(r):
            rel = np.array([i.relres for i in r["infos"]])
            return {"value": round(100 / r["wall"], 3),
                    "iters_per_solve": round(float(np.mean([i.iters for i in r["infos"]])), 3),
                    "refinements_per_solve": round(float(np.mean([i.refinements for i in r["infos"]])), 3),
                    "max_relres": float(rel.max()),
                    "failed_solves": int(sum(1 for i in r["infos"] if i.status != 0 or i.relres > tight)),
                    "err_vs_pstar_max": float(r["err"][nw:].max())}
        out["precision_bar_513x17"] = {
            "rtol": tight, "fp64": prec_summary(r64), "fp32_inner_fp64_refinement": prec_summary(r32),
            "time_to_accuracy_fp64_over_fp32": round(r64["wall"] / r32["wall"], 3),
            "solution_diff_fp32_vs_fp64_max": float(dx.max()), "solution_diff_fp32_vs_fp64_median": float(np.median(dx)),
            "steps": 20, "warmup": 5, "cluster_workgroups": Gb}
        say("  precision leg done")
        # the paper's preconditioner: ILU(0) of the sixth-order operator at still water (one
        # workgroup, level-scheduled substitutions) against the V-cycle, same systems, at the
        # benchmark's rtol 1e-8 and at the paper's bar tolerance 1e-4
        ilu = {}
        for rt in (w.rtol if w.name == "bar_513x17" else 1e-8, 1e-4):
            row = {}
            for pc in ("ilu0", "mg"):
                for mode in ("ewma", "previous"):
                    r = run_sequence(B, wb, e2, b2, p2, mode, 5, 20, Gb, precond=pc, rtol=rt)
                    row[f"{pc}_{mode}"] = {"value": round(100 / r["wall"], 3), "iters_per_solve": its(r),
                                           "failed_solves": r["failed"]}
            ilu[f"rtol_{rt:g}"] = row
        out["ilu0_bar_513x17"] = dict(ilu, steps=20, warmup=5, cluster_workgroups_ilu0=1,
                                      cluster_workgroups_mg=Gb)
        say("  ILU(0) leg done")
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w, x0, info0)
    print(json.dumps(out), flush=True)


def run_serving(args):
    """Continuous batching of the serving mix (independent simulations of different sizes).

    Inputs (surfaces and b = A p* of every system) are formed by the library's operator and
    resident in HBM first. Four runs on fresh simulations: saturation (every request queued
    at t = 0, FIFO per simulation), open loop (Poisson arrivals at --serve-rate, by default 70 %
    of the saturation rate just measured, and again at the configuration's 200 solves/s;
    round robin over the simulations), all three FP32-inner refinement with the EWMA guess
    through the server; and the one-at-a-time FP64 cold-start path (sa_solve, no sketch) on
    every k-th simulation. All at relative residual 1e-8 checked on the FP64 residual.
    Latency is measured from each request's scheduled arrival time (not from when the host
    loop got round to submitting it), on the server's clock.
    """
    import torch
    from paper_2511_18071_amd import binding as B
    from paper_2511_18071_amd import workload as W

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    sims = W.serving_mix(args.serve_sims, seed=5, nsys=args.serve_systems)
    nsys = args.serve_systems
    t_setup = time.perf_counter()
    say(f"serving: {len(sims)} simulations x {nsys} systems, {sum(w.n for w in sims)} unknowns")
    inputs = []
    with B.Server(stream=stream) as gen:
        for i, w in enumerate(sims):
            if i % 32 == 0:
                say(f"  inputs of simulation {i} ({time.perf_counter() - t_setup:.0f} s)")
            sid = gen.open(w, precond="none", guess="cold", cluster=1)
            eta = torch.empty((nsys, 2, w.nphys), dtype=torch.float64, device=dev)
            bs = torch.empty((nsys, w.n), dtype=torch.float64, device=dev)
            for s in range(nsys):
                ep, ec, ps = w.system(s)
                eta[s, 0].copy_(torch.from_numpy(ep))
                eta[s, 1].copy_(torch.from_numpy(ec))
                torch.cuda.synchronize()
                gen.apply_operator(sid, eta[s, 0], eta[s, 1], torch.from_numpy(ps).to(dev), bs[s])
            gen.close_sim(sid)
            inputs.append((eta, bs))
    torch.cuda.synchronize()
    total_unknowns = sum(w.n for w in sims)
    nreq = len(sims) * nsys
    # request j: simulation j mod nsims, its (j // nsims)-th system (round robin, FIFO per sim)
    order = [(j % len(sims), j // len(sims)) for j in range(nreq)]

    def serve(arrivals, label):
        say(f"  {label}: opening {len(sims)} simulations ({time.perf_counter() - t_setup:.0f} s)")
        sopts = dict(unknowns_per_workgroup=args.serve_upw)
        if args.serve_inflight:
            sopts["max_inflight"] = args.serve_inflight
        srv = B.Server(stream=stream, **sopts)
        ids = [srv.open(w, precision=args.serve_precision) for w in sims]
        if any(i is None for i in ids):
            raise RuntimeError("serving mix does not fit the HBM budget")
        torch.cuda.synchronize()
        lat, infos, who = [], [], []
        arrival_of, req_of = {}, {}
        k = 0
        say(f"  {label}: serving {nreq} requests")
        t0 = time.perf_counter()
        # server clock (ms since the server was created) at the host time t0
        base_ms = srv.clock_ms()
        t_say = t0
        while k < nreq or srv.outstanding > 0:
            if time.perf_counter() - t_say > 10.0:
                t_say = time.perf_counter()
                say(f"    {len(lat)} of {nreq} done, {t_say - t0:.0f} s")
            now = time.perf_counter() - t0
            while k < nreq and arrivals[k] <= now:
                i, s = order[k]
                eta, bs = inputs[i]
                t = srv.submit(ids[i], eta[s, 0], eta[s, 1], bs[s])
                arrival_of[t] = base_ms + 1e3 * arrivals[k]
                req_of[t] = (i, s)
                k += 1
            # block only until the next arrival falls due, so that no arrival waits on the host
            timeout = None if k >= nreq else max(0.0, arrivals[k] - (time.perf_counter() - t0))
            for c in srv.poll(wait=srv.outstanding > 0, timeout_s=timeout):
                lat.append(c.t_done_ms - arrival_of.pop(c.ticket))
                infos.append(c.info)
                who.append(req_of.pop(c.ticket))
        wall = time.perf_counter() - t0
        bytes_used = srv.bytes_used
        ticks = srv.stats()
        srv.close()
        return dict(wall=wall, lat=np.array(lat), infos=infos, who=who, bytes=bytes_used, ticks=ticks)

    sat = serve(np.zeros(nreq), "saturation")
    rate = args.serve_rate if args.serve_rate else 0.7 * nreq / sat["wall"]
    rng = np.random.default_rng(5)
    arr = np.cumsum(rng.exponential(1.0 / rate, nreq))
    ol = serve(arr, "open loop")
    # the arrival rate the serving configuration names (Poisson, 200 solves/s)
    arr200 = np.cumsum(np.random.default_rng(7).exponential(1.0 / 200.0, nreq))
    ol200 = serve(arr200, "open loop at 200/s")
    say(f"  baseline: one-at-a-time FP64 cold start ({time.perf_counter() - t_setup:.0f} s)")
    base_lat, base_its, base_bad = [], [], 0
    for i in range(0, len(sims), args.serve_baseline_stride):
        w = sims[i]
        eta, bs = inputs[i]
        p = B.Problem.from_workload(w, stream=stream, cluster=default_cluster(w), guess="cold")
        for s in range(nsys):
            p.set_surface(eta[s, 0], eta[s, 1])
            p.push_rhs(bs[s])
            torch.cuda.synchronize()
            t = time.perf_counter()
            info = p.solve()
            base_lat.append(1e3 * (time.perf_counter() - t))
            base_its.append(info.iters)
            base_bad += info.status != 0 or info.relres > w.rtol
        p.close()
    base_rate = len(base_lat) / (1e-3 * sum(base_lat))

    def stats(r):
        its = np.array([i.iters for i in r["infos"]])
        bad = [(w, i) for w, i in zip(r["who"], r["infos"]) if i.status != 0 or i.relres > 1e-8]
        t = r["ticks"]
        nt = max(1, t["ticks"])
        return dict(solves_per_s=round(nreq / r["wall"], 2), wall_s=round(r["wall"], 3),
                    ticks=t["ticks"], solves_per_tick=round(t["solves"] / nt, 2),
                    host_ms_per_tick_launch=round(t["launch_host_ms"] / nt, 4),
                    ms_per_tick_enqueue_to_done=round(t["tick_ms"] / nt, 3),
                    p50_ms=round(float(np.percentile(r["lat"], 50)), 3),
                    p99_ms=round(float(np.percentile(r["lat"], 99)), 3),
                    iters_per_solve=round(float(its.mean()), 3),
                    refinements_per_solve=round(float(np.mean([i.refinements for i in r["infos"]])), 3),
                    max_relres=float(max(i.relres for i in r["infos"])), failed_solves=len(bad),
                    device_failed=t["device_failed"],
                    failures=[dict(sim=w[0], system=w[1], status=i.status, iters=i.iters, restarts=i.restarts,
                                   refinements=i.refinements, relres0=float("%.3e" % i.relres0),
                                   relres=float("%.3e" % i.relres)) for w, i in bad[:16]])

    s_sat, s_ol = stats(sat), stats(ol)
    out = {
        "metric": "serving solves/s at saturation @relres 1e-8, p50/p99 solve latency (open loop)",
        "value": s_sat["solves_per_s"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": nreq,
        "warmup": 0,
        "ms_per_step": round(1e3 * sat["wall"] / nreq, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if args.serve_precision == "fp32_ir" else "f64",
        "data": "synthetic",
        "config": {"workload": f"serving_mix({len(sims)} simulations x {nsys} systems, seed 5)",
                   "unknowns_total": total_unknowns,
                   "precision": "fp32 inner GMRES, fp64 refinement" if args.serve_precision == "fp32_ir" else "fp64",
                   "guess": "EWMA", "hbm_bytes_resident": sat["bytes"],
                   "unknowns_per_workgroup": args.serve_upw, "ticks_in_flight": args.serve_inflight,
                   "coresident_workgroups": sat["ticks"]["capacity"],
                   "workgroups_per_tick": sat["ticks"]["tick_budget"],
                   "hw_queues": int(os.environ.get("GPU_MAX_HW_QUEUES", "4"))},
        "saturation": s_sat,
        "open_loop": dict(offered_solves_per_s=round(rate, 2), **s_ol),
        "open_loop_200": dict(offered_solves_per_s=200.0, **stats(ol200)),
        "baseline_one_at_a_time_fp64_cold": {
            "solves_per_s": round(base_rate, 2), "solves": len(base_lat),
            "sample": f"every {args.serve_baseline_stride}th simulation, all its systems",
            "p50_ms": round(float(np.percentile(base_lat, 50)), 3),
            "p99_ms": round(float(np.percentile(base_lat, 99)), 3),
            "iters_per_solve": round(float(np.mean(base_its)), 3), "failed_solves": base_bad},
        "speedup_vs_baseline": round(s_sat["solves_per_s"] / base_rate, 2),
        "setup_s": round(time.perf_counter() - t_setup, 1),
    }
    print(json.dumps(out), flush=True)


def copy_probe(nbytes: int):
    """Five launches of a plain device copy of nbytes: FETCH_SIZE and WRITE_SIZE of these
    dispatches against nbytes give the factor that turns the counters into bytes."""
    import torch
    n = nbytes // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": n * 8, "launches": 5}), flush=True)


def operator_probe(name: str, reps: int = 50):
    """The standalone operator kernel on the first system of a workload: x and y in HBM, one
    launch per application (plus the geometry kernel), synchronised each time."""
    import torch
    from paper_2511_18071_amd import binding as B
    from paper_2511_18071_amd import workload as W
    w = W.get(name)
    ep, ec, ps = w.system(0)
    e0, e1 = torch.from_numpy(ep).cuda(), torch.from_numpy(ec).cuda()
    x = torch.from_numpy(ps).cuda()
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    p = B.Problem.from_workload(w, stream=torch.cuda.current_stream(), precond="none", guess="cold")
    p.set_surface(e0, e1)
    for _ in range(5):
        p.apply_operator(x, y)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        p.apply_operator(x, y)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    p.close()
    print(json.dumps({"operator_probe": name, "unknowns": w.n, "launches": reps + 5,
                      "ms_per_application": round(1e3 * dt, 4)}), flush=True)


def operator3d_probe(name: str, reps: int = 50) -> dict:
    """The three-dimensional operator kernel on a wave field: x and y resident in HBM, one
    launch per application on the current stream, bracketed by HIP events (the geometry
    kernel runs once, at set_surface). Algorithmic bytes per application: read x, write y."""
    import torch
    from paper_2511_18071_amd import binding as B
    from paper_2511_18071_amd import workload as W
    w = W.wave3d(name)
    ep, ec, ps = w.system(0)
    st = torch.cuda.current_stream()
    x = torch.from_numpy(ps).cuda()
    y = torch.empty_like(x)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * reps)]
    with B.Operator3D(w.nx, w.ny, w.nz, w.bc_x, w.bc_y, w.length_x, w.length_y, w.depth(), stream=st) as op:
        op.set_surface(ep, ec)
        for _ in range(5):
            op.apply(x, y)
        op.sync()
        for i in range(reps):
            ev[2 * i].record(st)
            op.apply(x, y)
            ev[2 * i + 1].record(st)
        op.sync()
        wg = op.workgroups
    ms = float(np.mean([ev[2 * i].elapsed_time(ev[2 * i + 1]) for i in range(reps)]))
    nbytes = 16.0 * w.n
    gbs = nbytes / (ms * 1e-3) / 1e9
    return {"workload": name, "unknowns": w.n, "workgroups": wg, "launches": reps + 5,
            "ms_per_application": round(ms, 5), "algorithmic_bytes": int(nbytes),
            "achieved_gbs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
            "gflops": round(170.0 * w.n / (ms * 1e-3) / 1e9, 1)}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: it measures the one-GPU path (asked for {args.gpus}).",
              file=sys.stderr)
        sys.exit(2)
    if args.operator3d_probe:
        print(json.dumps({"operator3d_probe": operator3d_probe(args.operator3d_probe)}), flush=True)
    elif args.operator_probe:
        operator_probe(args.operator_probe)
    elif args.copy_probe:
        copy_probe(args.copy_probe)
    elif args.workload == "serving":
        # one hardware queue per tick stream (read when the HIP runtime starts, which has not
        # happened yet): ticks that share a queue run one after the other
        if int(os.environ.get("GPU_MAX_HW_QUEUES", "4")) < args.serve_inflight:
            os.environ["GPU_MAX_HW_QUEUES"] = str(args.serve_inflight)
        run_serving(args)
    else:
        run_main(args)
    # release every device resource before the interpreter's own teardown
    try:
        import torch
        if torch.cuda.is_available():
            torch.cuda.synchronize()
    except Exception:
        pass


if __name__ == "__main__":
    main()
