#!/usr/bin/env python3
"""Benchmark of the subspace-accelerated Poisson sequence on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload bar_513x17]

A step is one LSERK45 time step of the synthetic simulation: five sequential mixed-stage
Poisson solves (one per Runge-Kutta stage), each from the EWMA-subspace initial guess,
GMRES to relative residual 1e-8 with the still-water V-cycle preconditioner, FP64.
Inputs (surfaces at the stage times, manufactured right-hand sides b = A p* formed by the
library's own operator) are resident in HBM before the timed region starts. The same K
steps are then solved by the plain path (cold start x0 = 0, same GMRES) for the
subspace-vs-plain comparison. Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# counters of the solve kernel taken on this workload (FETCH_SIZE and WRITE_SIZE runs) and the
# hash of the kernel sources they were taken with: the traffic is reported only while the
# sources are unchanged
COUNTERS = os.path.join(ROOT, "profiles", "sa_solve_kernel_bar_513x17_counters.md")
KERNEL_SOURCES = ("paper_2511_18071_amd/csrc/device.h", "paper_2511_18071_amd/csrc/solve64.hip",
                  "paper_2511_18071_amd/csrc/internal.h", "paper_2511_18071_amd/csrc/api.hip")


def kernel_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(workload: str, steps: int, warmup: int, cluster: int):
    """HBM bytes per EWMA launch of the solve kernel from the committed counter summary, or
    None when it was taken on other kernel sources or another run configuration."""
    try:
        text = open(COUNTERS).read()
    except OSError:
        return None
    fields = {}
    for line in text.splitlines():
        if line.startswith("- ") and ": " in line:
            k, v = line[2:].split(": ", 1)
            fields[k.strip("` ")] = v.strip("` ")
    try:
        same = (fields["kernel-source-sha256"] == kernel_hash() and fields["workload"] == workload
                and int(fields["steps"]) == steps and int(fields["warmup"]) == warmup
                and int(fields["cluster"]) == cluster)
        return float(fields["hbm-bytes-per-launch"]) if same else None
    except (KeyError, ValueError):
        return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=4)
    ap.add_argument("--workload", default="bar_513x17")
    ap.add_argument("--cluster", type=int, default=0, help="workgroups per solve (0 = size rule)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-solves", type=int, default=30)
    ap.add_argument("--serve-sims", type=int, default=256, help="serving: simulations")
    ap.add_argument("--serve-systems", type=int, default=10, help="serving: systems per simulation")
    ap.add_argument("--serve-rate", type=float, default=None,
                    help="serving: offered solves/s of the open loop (default: 0.7 x the measured saturation rate)")
    ap.add_argument("--serve-inflight", type=int, default=16,
                    help="serving: ticks in flight (the process is given as many hardware queues)")
    ap.add_argument("--serve-upw", type=int, default=20000,
                    help="serving: unknowns per workgroup when the server sizes the clusters")
    ap.add_argument("--serve-baseline-stride", type=int, default=8,
                    help="serving: the one-at-a-time FP64 baseline solves every k-th simulation")
    ap.add_argument("--operator-probe", default="", metavar="WORKLOAD",
                    help="only apply the operator of WORKLOAD's first system 50 times (standalone "
                         "kernel: one workgroup per 64-column tile) and print its rate")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES bytes five times (the "
                         "reference kernel that scales HBM counter readings)")
    return ap.parse_args()


def default_cluster(w) -> int:
    # the library's own default: one workgroup per 32-column tile of the finest level, at most 128
    return int(min(128, max(1, (w.ncol + 31) // 32)))


def traffic_bytes(w, infos, pcv, k) -> float:
    """Algorithmic HBM bytes of the solves in `infos`, in vectors of n FP64 values.

    guess            3k + 3   read Y_old and x, write Y_new, read b (block operator + Gram),
                              read Y_new, write x0
    r0 = b - A x0    3        read x0 and b, write r0
    trigger M^-1 b   pcv + 1  one V-cycle and the norm of its output
    cycle start      pcv + 1  V-cycle of r and its norm (once per cycle)
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
            v += pcv + 1
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
    """Vectors moved by one V(1,1) cycle of the still-water preconditioner: per level the
    down pass reads f and writes u and the coarse f (2.5), the up pass reads u, f and the
    coarse correction and writes the output (3.5); levels halve in size, so the hierarchy
    moves 6 x (1 + 1/2 + 1/4 + ...) ~ 12 fine-grid vectors."""
    return 12.0


def run_gpu(args, w):
    import torch
    from paper_2511_18071_amd import binding as B

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    nsys = 5 * (args.warmup + args.steps)
    G = args.cluster or default_cluster(w)
    # ---- stage the inputs: surfaces at the stage times and b = A p*
    etas = torch.empty((nsys, 2, w.nphys), dtype=torch.float64, device=dev)
    bs = torch.empty((nsys, w.n), dtype=torch.float64, device=dev)
    with B.Problem.from_workload(w, stream=stream, cluster=G) as gen:
        for s in range(nsys):
            ep, ec, ps = w.system(s)
            etas[s, 0].copy_(torch.from_numpy(ep))
            etas[s, 1].copy_(torch.from_numpy(ec))
            pst = torch.from_numpy(ps).to(dev)
            gen.set_surface(etas[s, 0], etas[s, 1])
            gen.apply_operator(pst, bs[s])
    torch.cuda.synchronize()

    def run(mode):
        # every launch of the solve kernel is bracketed by events on the problem's stream, the
        # warm-up launches too, so the mean kernel time covers the same launches as a kernel
        # trace of this process
        p = B.Problem.from_workload(w, stream=stream, cluster=G, guess=mode)
        nw = 5 * args.warmup
        evw = [torch.cuda.Event(enable_timing=True) for _ in range(2 * nw)]
        for s in range(nw):
            p.set_surface(etas[s, 0], etas[s, 1])
            p.push_rhs(bs[s])
            evw[2 * s].record(stream)
            p.solve(sync=False)
            evw[2 * s + 1].record(stream)
        warm_infos = p.read_log()
        torch.cuda.synchronize()
        warm_lat = [evw[2 * i].elapsed_time(evw[2 * i + 1]) for i in range(nw)]
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * 5 * args.steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i, s in enumerate(range(nw, nsys)):
            p.set_surface(etas[s, 0], etas[s, 1])
            p.push_rhs(bs[s])
            ev[2 * i].record(stream)
            p.solve(sync=False)
            ev[2 * i + 1].record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        infos = p.read_log()
        lat = np.array([ev[2 * i].elapsed_time(ev[2 * i + 1]) for i in range(5 * args.steps)])
        x = p.solution()
        p.close()
        bad = [i for i in infos if i.status != 0 or i.relres > w.rtol]
        return dict(wall=wall, infos=infos, lat=lat, failed=len(bad), x=x,
                    all_infos=warm_infos + infos, all_lat=np.concatenate([warm_lat, lat]))

    ewma = run("ewma")
    plain = run("cold")
    return ewma, plain, G


def cpu_baseline(w, nsolves):
    from threadpoolctl import threadpool_limits

    from oracle.sequence import Simulation

    with threadpool_limits(limits=1):
        sim = Simulation.from_workload(w)
        systems = []
        for s in range(nsolves):
            ep, ec, ps = w.system(s)
            systems.append((ep, ec, sim.operator(ep, ec) @ ps))
        t0 = time.perf_counter()
        its = []
        for ep, ec, b in systems:
            its.append(sim.solve(ep, ec, b).info.iters)
        dt = time.perf_counter() - t0
    return dict(value=nsolves / dt, unit="solves/s", cores=1, kind="oracle",
                sample=f"first {nsolves} systems of {w.name} (FP64 oracle: assembled CSR operator, "
                       f"V-cycle, GMRES(30), EWMA rank {w.k} guess by Householder QR), "
                       f"{np.mean(its):.2f} iterations/solve, one thread")


def run_serving(args):
    """Continuous batching of the serving mix (independent simulations of different sizes).

    Inputs (surfaces and b = A p* of every system) are formed by the library's operator and
    resident in HBM first. Four runs on fresh simulations: saturation (every request queued
    at t = 0, FIFO per simulation), open loop (Poisson arrivals at --serve-rate, by default 70 %
    of the saturation rate just measured, so that latency is that of a sustainable load, and
    again at the configuration's 200 solves/s, above saturation on one GPU; round robin
    over the simulations), all three FP32-inner refinement with the EWMA guess through the server;
    and the one-at-a-time FP64 cold-start path (sa_solve, no sketch) on every k-th simulation.
    All at relative residual 1e-8 checked on the FP64 residual.
    """
    import torch
    from paper_2511_18071_amd import binding as B
    from paper_2511_18071_amd import workload as W

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    sims = W.serving_mix(args.serve_sims, seed=5, nsys=args.serve_systems)
    nsys = args.serve_systems
    t_setup = time.perf_counter()
    say = lambda *a: print(*a, file=sys.stderr, flush=True)  # progress (the JSON line goes to stdout)
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
        ids = [srv.open(w, precision="fp32_ir") for w in sims]
        if any(i is None for i in ids):
            raise RuntimeError("serving mix does not fit the HBM budget")
        torch.cuda.synchronize()
        lat, infos = [], []
        k = 0
        say(f"  {label}: serving {nreq} requests")
        t0 = time.perf_counter()
        t_say = t0
        while k < nreq or srv.outstanding > 0:
            if time.perf_counter() - t_say > 10.0:
                t_say = time.perf_counter()
                say(f"    {len(lat)} of {nreq} done, {t_say - t0:.0f} s")
            now = time.perf_counter() - t0
            while k < nreq and arrivals[k] <= now:
                i, s = order[k]
                eta, bs = inputs[i]
                srv.submit(ids[i], eta[s, 0], eta[s, 1], bs[s])
                k += 1
            wait = k >= nreq or (arrivals[k] - (time.perf_counter() - t0)) > 0.002
            for c in srv.poll(wait=wait and srv.outstanding > 0):
                lat.append(c.t_done_ms - c.t_submit_ms)
                infos.append(c.info)
        wall = time.perf_counter() - t0
        bytes_used = srv.bytes_used
        srv.close()
        return dict(wall=wall, lat=np.array(lat), infos=infos, bytes=bytes_used)

    sat = serve(np.zeros(nreq), "saturation")
    rate = args.serve_rate if args.serve_rate else 0.7 * nreq / sat["wall"]
    rng = np.random.default_rng(5)
    arr = np.cumsum(rng.exponential(1.0 / rate, nreq))
    ol = serve(arr, "open loop")
    # the arrival rate the serving configuration names (Poisson, 200 solves/s): above the
    # saturation rate on one GPU, so its latencies are those of a growing queue
    arr200 = np.cumsum(np.random.default_rng(7).exponential(1.0 / 200.0, nreq))
    ol200 = serve(arr200, "open loop at 200/s")
    say(f"  baseline: one-at-a-time FP64 cold start ({time.perf_counter() - t_setup:.0f} s)")
    # one-at-a-time FP64 cold start (sa_solve) on every k-th simulation
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
        bad = sum(1 for i in r["infos"] if i.status != 0 or i.relres > 1e-8)
        return dict(solves_per_s=round(nreq / r["wall"], 2), wall_s=round(r["wall"], 3),
                    p50_ms=round(float(np.percentile(r["lat"], 50)), 3),
                    p99_ms=round(float(np.percentile(r["lat"], 99)), 3),
                    iters_per_solve=round(float(its.mean()), 3),
                    refinements_per_solve=round(float(np.mean([i.refinements for i in r["infos"]])), 3),
                    max_relres=float(max(i.relres for i in r["infos"])), failed_solves=bad)

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
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"serving_mix({len(sims)} simulations x {nsys} systems, seed 5)",
                   "unknowns_total": total_unknowns, "precision": "fp32 inner GMRES, fp64 refinement",
                   "guess": "EWMA", "hbm_bytes_resident": sat["bytes"],
                   "unknowns_per_workgroup": args.serve_upw, "ticks_in_flight": args.serve_inflight,
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


def main():
    args = parse()
    if args.operator_probe:
        operator_probe(args.operator_probe)
        return
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: this build measures the one-GPU path (asked for {args.gpus}).",
              file=sys.stderr)
        sys.exit(2)
    from paper_2511_18071_amd import workload as W

    if args.workload == "serving":
        # one hardware queue per tick stream (read when the HIP runtime starts, which has not
        # happened yet): ticks that share a queue run one after the other
        if int(os.environ.get("GPU_MAX_HW_QUEUES", "4")) < args.serve_inflight:
            os.environ["GPU_MAX_HW_QUEUES"] = str(args.serve_inflight)
        run_serving(args)
        return
    w = W.get(args.workload)
    ewma, plain, G = run_gpu(args, w)
    nsol = 5 * args.steps
    value = nsol / ewma["wall"]
    its = np.array([i.iters for i in ewma["infos"]])
    its_plain = np.array([i.iters for i in plain["infos"]])
    # roofline of the solve kernel over all its launches (warm-up included)
    kernel_ms = float(ewma["all_lat"].mean())
    pcv = precond_vectors(w)
    bytes_per = traffic_bytes(w, ewma["all_infos"], pcv, w.k) / len(ewma["all_infos"])
    achieved = bytes_per / (kernel_ms * 1e-3) / 1e9
    out = {
        "metric": "solves/s @relres 1e-8 (subspace vs plain), iters/solve, p99 solve latency",
        "value": round(value, 2),
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
                   "systems_per_step": 5, "restart": w.restart, "rtol": w.rtol, "precond": "still-water V(1,1)",
                   "guess": f"EWMA rank {w.k}, r={w.r}", "cluster_workgroups": G},
        "iters_per_solve": round(float(its.mean()), 3),
        "p50_solve_ms": round(float(np.percentile(ewma["lat"], 50)), 4),
        "p99_solve_ms": round(float(np.percentile(ewma["lat"], 99)), 4),
        "failed_solves": ewma["failed"],
        "plain": {"value": round(nsol / plain["wall"], 2), "iters_per_solve": round(float(its_plain.mean()), 3),
                  "p99_solve_ms": round(float(np.percentile(plain["lat"], 99)), 4), "guess": "cold (x0 = 0)",
                  "failed_solves": plain["failed"]},
        "speedup_vs_plain": round(plain["wall"] / ewma["wall"], 3),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 5),
                     "traffic": measured_traffic(w.name, args.steps, args.warmup, G),
                     "kernel_source_sha256": kernel_hash(),
                     "kernel": "sa_solve_kernel", "kernel_ms": round(kernel_ms, 4),
                     "launches": len(ewma["all_infos"]),
                     "algorithmic_bytes_per_launch": round(bytes_per)},
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_solves)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
