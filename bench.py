#!/usr/bin/env python3
"""Benchmark of the NR99 linear MHS multigrid path on one MI355X.

One step = the whole path for one equilibrium: the lower-boundary solve of
equation (11), the interior solve of equation (8) and the recovery of B, p,
rho.  The workload is the 257^3 unit box, cycling over the six runs
alpha in {0, 0.5, 1} x a in {0, 0.5} (xi = a exp(-z/0.2)), each with six
seeded Gaussian bipoles.  Both solves stop at relative residual 1e-10, which
brings every field to relative error <= 1e-8 against the exact discrete
solution (measured by the GPU parity tests).  The headline value is the
FP32-in-FP64 refinement path, as whole-job throughput with several requests
in flight at once (continuous batching, --batch); the plain FP64 path and
one-request-at-a-time figures of both are reported beside it.  Prints one
JSON line.  Inputs are resident in HBM before timing starts.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "V-cycle GB/s & solves/s at 257^3 to 1e-8 (FP64 vs mixed); p50/p99 latency"
HBM_PEAK_GBPS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "smooth_l0_traffic_mhs257.txt")
# the kernel source and what sets its launch shape and ring depth
KERNEL_SRCS = [os.path.join(ROOT, "paper_1307_6720_amd", "csrc", f) for f in ("kernels.hip", "internal.h", "api.cpp")]


def kernels_digest():
    h = hashlib.sha256()
    for f in KERNEL_SRCS:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=18)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="mhs-257")
    ap.add_argument("--rtol", type=float, default=1e-10)
    ap.add_argument("--inner-cycles", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-run", type=int, default=3)
    ap.add_argument("--serve-requests", type=int, default=512,
                    help="requests of the serving stream (0 skips the serving leg)")
    ap.add_argument("--serve-rate", type=float, default=0.0,
                    help="Poisson arrival rate in requests/s (0: 0.5x and 0.9x of the capacity measured "
                         "with every request queued at once)")
    ap.add_argument("--serve-slots", type=int, default=16)
    ap.add_argument("--batch", type=int, default=6,
                    help="concurrent requests in the batched pass over the workload (0: single stream only)")
    ap.add_argument("--serve-budget-gb", type=float, default=64.0)
    ap.add_argument("--counter-probe", action="store_true",
                    help="run only the workload of the rocprofv3 FETCH_SIZE/WRITE_SIZE runs")
    ap.add_argument("--summarize-counters", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="print the traffic summary from the two counter runs' counter_collection.csv")
    ap.add_argument("--summarize-trace", nargs=2, metavar=("STATS_CSV", "TRACE_CSV"),
                    help="print the kernel summary of a --kernel-trace --stats run")
    return ap.parse_args()


def percentile(xs, q):
    s = sorted(xs)
    if not s:
        return None
    k = (len(s) - 1) * q
    lo, hi = int(k), min(int(k) + 1, len(s) - 1)
    return s[lo] + (s[hi] - s[lo]) * (k - lo)


def recorded_traffic():
    """Per-launch HBM traffic of the level-0 smoother measured with rocprofv3
    counters, valid only for the kernel source it was measured on."""
    try:
        meta = {}
        with open(TRAFFIC_FILE) as fh:
            for line in fh:
                if ":" in line:
                    k, v = line.split(":", 1)
                    meta[k.strip()] = v.strip()
        if meta.get("kernels_sha256") != kernels_digest():
            return None
        return float(meta["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


# ---------------------------------------------------------------------------
# rocprofv3 helpers: the workload of the counter runs and the summaries kept
# under profiles/ (the counter-derived traffic is read back by recorded_traffic)
# ---------------------------------------------------------------------------
def _short_kernel(name):
    n = re.sub(r"\(mhs::[^)]*\)", "", name)
    n = n.replace("void mhs::(anonymous namespace)::", "").replace("mhs::(anonymous namespace)::", "")
    return re.sub(r"\(.*\)$", "", n)


# level-0 FP32 smoother variants of one refinement step and their compulsory
# bytes per fine node: the zero-guess sweep (read f, write u), two sweeps with
# f (read u, f; write u) and the prolongation sweep (+ coarse correction, N/8
# floats)
SMOOTH_L0_MIX = {"k_sweep3<float, 3>": (1, 8.0), "k_sweep3<float, 1>": (2, 12.0), "k_sweep3<float, 9>": (1, 12.5)}
COPY_BYTES = 1 << 30


def counter_probe():
    """Workload of the FETCH_SIZE / WRITE_SIZE runs: a device copy of
    COPY_BYTES (the calibration kernel: it reads and writes exactly that
    many bytes), then two mixed-path equilibria of the 257^3 workload."""
    import torch

    import synth
    from paper_1307_6720_amd import PREC_FP64, PREC_MIXED
    from paper_1307_6720_amd.solver import Plan, make_opts

    src = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    w = synth.workload("mhs-257", run=3)
    plan = Plan(w.grid, PREC_FP64 | PREC_MIXED, device="cuda:0")
    bz = torch.from_numpy(w.bz0).to("cuda:0")
    P = torch.zeros(w.grid.shape, dtype=torch.float64, device="cuda:0")
    for _ in range(2):
        plan.solve_boundary(bz, P, make_opts(rtol=1e-10))
        plan.solve_interior(w.model, P, make_opts(PREC_MIXED, rtol=1e-10))
    torch.cuda.synchronize()
    plan.close()
    print("counter probe done", flush=True)


def summarize_counters(fetch_csv, write_csv):
    """Per-launch HBM traffic of the level-0 FP32 smoother from the two
    counter runs of counter_probe, each counter scaled by what it reads for
    the calibration copy.  Prints the summary kept under profiles/."""
    import collections
    import csv
    import statistics

    def load(path, counter):
        agg = collections.OrderedDict()
        with open(path) as fh:
            for r in csv.DictReader(fh):
                if r["Counter_Name"] != counter:
                    continue
                k = r["Dispatch_Id"]
                if k not in agg:
                    agg[k] = [r["Kernel_Name"], 0.0]
                agg[k][1] += float(r["Counter_Value"]) * 1024.0  # KiB per dispatch
        return list(agg.values())

    fetch, write = load(fetch_csv, "FETCH_SIZE"), load(write_csv, "WRITE_SIZE")

    def calib(rows):
        # the largest copy kernel is the calibration copy
        return max(v for n, v in rows if "copyBuffer" in n or "copy" in _short_kernel(n).lower()) / COPY_BYTES

    cf, cw = calib(fetch), calib(write)
    N = 257 ** 3
    per = {}
    for k in SMOOTH_L0_MIX:
        fv = [v for n, v in fetch if _short_kernel(n) == k]
        wv = [v for n, v in write if _short_kernel(n) == k]
        # level-0 launches carry 8x the traffic of level 1; launches issued
        # after convergence exit at once and carry none
        f0 = [x for x in fv if x > max(fv) / 3]
        w0 = [x for x in wv if x > max(wv) / 3]
        per[k] = (len(f0), statistics.mean(f0) / cf, statistics.mean(w0) / cw)
    print(f"calibration: a device copy of {COPY_BYTES} B reads FETCH_SIZE = {cf:.4f} x bytes read, "
          f"WRITE_SIZE = {cw:.4f} x bytes written; counts below are divided by these factors")
    for k, (n, fb, wb) in per.items():
        print(f"{k:22s} level-0 launches {n:3d}  read {fb / 1e6:8.1f} MB ({fb / N:5.2f} B/node, "
              f"compulsory {SMOOTH_L0_MIX[k][1] - 4:.2f})  write {wb / 1e6:8.1f} MB ({wb / N:5.2f} B/node, compulsory 4.00)")
    tot = sum(c for c, _ in SMOOTH_L0_MIX.values())
    avg = sum(c * (per[k][1] + per[k][2]) for k, (c, _) in SMOOTH_L0_MIX.items()) / tot
    alg = sum(c * b for c, b in SMOOTH_L0_MIX.values()) * N / tot
    print(f"class average per launch (1 zero-guess : 2 with f : 1 prolongation): traffic {avg / 1e6:.1f} MB, "
          f"compulsory {alg / 1e6:.1f} MB, ratio {avg / alg:.3f}")
    print(f"kernels_sha256: {kernels_digest()}")
    print(f"traffic_bytes_per_launch: {avg:.0f}")


def summarize_trace(stats_csv, trace_csv, one_groups=1024, top=24):
    """Kernel-time summary of a rocprofv3 --kernel-trace --stats run of
    bench.py: the stats table, the launches that ran (> 5 us; launches
    issued after a solve converged exit at once) by kernel and workgroup
    count, and the average duration of the level-0 FP32 smoother launches
    (the kernel bench.py's roofline times with HIP events)."""
    import collections
    import csv
    import statistics

    with open(stats_csv) as fh:
        rows = list(csv.DictReader(fh))
    print(f"## kernel stats (top {top}, as written by rocprofv3 --stats)")
    print(f"{'kernel':58s} {'calls':>6s} {'total_ms':>9s} {'avg_us':>8s} {'pct':>6s}")
    for r in rows[:top]:
        print(f"{_short_kernel(r['Name'])[:58]:58s} {int(r['Calls']):6d} {int(r['TotalDurationNs']) / 1e6:9.3f} "
              f"{float(r['AverageNs']) / 1e3:8.2f} {float(r['Percentage']):6.2f}")
    with open(trace_csv) as fh:
        rows = list(csv.DictReader(fh))
    agg = collections.defaultdict(list)
    l0 = collections.defaultdict(list)
    for r in rows:
        k = _short_kernel(r["Kernel_Name"])
        g = int(r["Grid_Size_X"]) // max(1, int(r["Workgroup_Size_X"]))
        d = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
        agg[(k, g)].append(d)
        if k in SMOOTH_L0_MIX and d > 25.0:
            l0[(k, g)].append(d)
    print()
    print("## launches that ran (> 5 us), by kernel and workgroup count")
    print(f"{'kernel':40s} {'groups':>7s} {'ran':>5s} {'avg_us':>8s} {'med_us':>8s} {'skip':>5s} {'ran_ms':>8s}")
    out = []
    for (k, g), v in agg.items():
        ran = sorted(d for d in v if d > 5.0)
        if ran:
            out.append((sum(ran), k, g, len(ran), sum(ran) / len(ran), ran[len(ran) // 2], len(v) - len(ran)))
    for s, k, g, n, avg, med, sk in sorted(out, reverse=True)[:32]:
        print(f"{k[:40]:40s} {g:7d} {n:5d} {avg:8.2f} {med:8.2f} {sk:5d} {s / 1e3:8.3f}")
    print()
    print("## launches (> 25 us) of the mixed path's level-0 smoother; one request's level-0 launch has "
          f"{one_groups} workgroups, merged launches of several requests have more")
    tot = cnt = 0
    for (k, g), v in sorted(l0.items()):
        print(f"{k:22s} groups {g:5d} launches {len(v):4d} avg_us {statistics.mean(v):8.2f} "
              f"median_us {statistics.median(v):8.2f}")
        if g == one_groups:
            tot += sum(v)
            cnt += len(v)
    if cnt:
        print(f"one-request level-0 launches: {cnt}, average {tot / cnt:.2f} us")


def cpu_baseline(run):
    """The oracle (plain C multigrid + numpy field recovery), single thread,
    on one equilibrium of the same workload."""
    import numpy as np

    import synth
    from oracle import fields as ofields
    from oracle import ref

    w = synth.workload("mhs-257", run=run)
    m = w.model
    t0 = time.perf_counter()
    P, st, info = ref.solve(w.bz0, m.xi, m.alpha, w.grid.shape, rtol2=1e-10, rtol3=1e-10)
    ofields.fields(P, m.alpha, m.xi, m.dxi, m.pb, m.rhob, m.mu0, m.g)
    dt = time.perf_counter() - t0
    assert st == ref.OK and np.isfinite(P).all()
    return {"value": 1.0 / dt, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": f"one full solve of {w.name} run {run} ({w.grid.nx}^3): 2D+3D V(2,2) to rtol 1e-10 "
                      f"({info['cycles2d']}+{info['cycles3d']} cycles) plus fields, {dt:.2f} s"}


def serve_leg(a, torch, dev):
    """The serving stream: requests over {65^3, 129^3, 129^2 x 65, 257^3}
    with random alpha, xi, magnetograms; first each solved alone with the
    plain FP64 path (plans pooled by shape), then served by the batching
    server (mixed precision) with Poisson arrivals."""
    import synth
    from paper_1307_6720_amd import PREC_FP64, PREC_MIXED
    from paper_1307_6720_amd.serve import DeviceBackend, Request, Server
    from paper_1307_6720_amd.solver import Plan, solve

    specs = synth.serving_requests(n=a.serve_requests)
    works = [synth.request_workload(r) for r in specs]
    bzs = [torch.from_numpy(w.bz0).to(dev) for w in works]

    # FP64 single-request path, one after another
    plans = {}
    for w in works:
        if w.grid.shape not in plans:
            plans[w.grid.shape] = Plan(w.grid, PREC_FP64 | PREC_MIXED, device=dev)
    outs = {sh: (torch.empty(sh, dtype=torch.float64, device=dev),) +
            tuple(torch.empty(sh, dtype=torch.float64, device=dev) for _ in range(5)) for sh in plans}
    for w, bz in list(zip(works, bzs))[:4]:  # warm every shape's path
        solve(plans[w.grid.shape], bz, w.model, precision=PREC_FP64, rtol=a.rtol, out=outs[w.grid.shape])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for w, bz in zip(works, bzs):
        solve(plans[w.grid.shape], bz, w.model, precision=PREC_FP64, rtol=a.rtol, out=outs[w.grid.shape])
    torch.cuda.synchronize()
    single = len(works) / (time.perf_counter() - t0)
    for p in plans.values():
        p.close()
    del outs

    be = DeviceBackend(max_slots=a.serve_slots, device=dev)
    srv = Server(be, int(a.serve_budget_gb * (1 << 30)))

    def stream(arrivals):
        reqs = [Request(id=i, dims=(w.grid.nx, w.grid.ny, w.grid.nz), model=w.model, bz0=bz,
                        precision=PREC_MIXED, rtol=a.rtol, arrival=t)
                for i, (t, w, bz) in enumerate(zip(arrivals, works, bzs))]
        srv.ticks = srv.peak_active = srv.peak_queue = 0
        return srv.run(reqs)[1]

    stream([0.0] * min(8, len(works)))  # warm the batch path and the resident pool
    sat = stream([0.0] * len(works))  # everything queued at once: capacity
    loads = [a.serve_rate] if a.serve_rate > 0 else [0.5 * sat["solves_per_s"], 0.9 * sat["solves_per_s"]]
    poisson = []
    for rate in loads:  # Poisson arrivals at a fraction of capacity: latency
        st = stream([r["arrival_unit"] / rate for r in specs])
        poisson.append({"offered_rate": rate, "solves_per_s": st["solves_per_s"], "p50_ms": st["p50_ms"],
                        "p99_ms": st["p99_ms"], "ok": st["ok"], "peak_active": st["peak_active"],
                        "peak_queue": st["peak_queue"]})
    be.close()
    shapes = {}
    for w in works:
        k = "x".join(map(str, (w.grid.nx, w.grid.ny, w.grid.nz)))
        shapes[k] = shapes.get(k, 0) + 1
    return {"requests": len(works), "shapes": shapes, "precision": "mixed", "rtol": a.rtol,
            "max_slots": a.serve_slots,
            "saturated": {"solves_per_s": sat["solves_per_s"], "ok": sat["ok"], "ticks": sat["ticks"],
                          "peak_active": sat["peak_active"], "p50_ms": sat["p50_ms"], "p99_ms": sat["p99_ms"]},
            "poisson": poisson,
            "peak_resident_gb": srv.peak_bytes / 2**30,
            "fp64_single_solves_per_s": single,
            "speedup_vs_fp64_single": sat["solves_per_s"] / single}


def batched_leg(a, runs, bz, prec, steps, warm=True):
    """The same equilibria served by the batching server with `a.batch`
    requests in flight (all queued at once): whole-job throughput and
    per-request latency."""
    from paper_1307_6720_amd.serve import DeviceBackend, Request, Server

    be = DeviceBackend(max_slots=a.batch, device=bz[0].device)
    srv = Server(be, 64 << 30)

    def reqs(n):
        return [Request(id=k, dims=(runs[k % len(runs)].grid.nx, runs[k % len(runs)].grid.ny,
                                    runs[k % len(runs)].grid.nz),
                        model=runs[k % len(runs)].model, bz0=bz[k % len(runs)], precision=prec, rtol=a.rtol,
                        arrival=0.0) for k in range(n)]

    if warm:
        srv.run(reqs(a.batch))
    srv.ticks = srv.peak_active = 0
    done, st = srv.run(reqs(steps))
    be.close()
    assert st["ok"] == steps, st
    cyc = [r.info3d["cycles"] for r in done]
    return {"solves_per_s": st["solves_per_s"], "ms_per_solve": 1e3 / st["solves_per_s"], "p50_ms": st["p50_ms"],
            "p99_ms": st["p99_ms"], "requests": steps, "in_flight": a.batch, "ticks": st["ticks"],
            "cycles": sum(cyc) / len(cyc)}


def main():
    a = parse()
    if a.summarize_counters:
        summarize_counters(*a.summarize_counters)
        return
    if a.summarize_trace:
        summarize_trace(*a.summarize_trace)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if a.gpus != 1 or world != 1:
        print("bench.py: this build measures one GPU only (the path has no multi-GPU sharding); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    if a.counter_probe:
        counter_probe()
        return

    import numpy as np
    import torch

    import synth
    from paper_1307_6720_amd import PREC_FP64, PREC_MIXED, _lib
    from paper_1307_6720_amd.solver import Plan, make_opts

    dev = torch.device("cuda:0")
    runs = [synth.workload(a.workload, run=r) for r in range(synth.nruns(a.workload))]
    grid = runs[0].grid
    N = grid.npoints
    plan = Plan(grid, PREC_FP64 | PREC_MIXED, device=dev)
    bz = [torch.from_numpy(w.bz0).to(dev) for w in runs]
    P = torch.zeros(grid.shape, dtype=torch.float64, device=dev)
    F = tuple(torch.empty_like(P) for _ in range(5))
    torch.cuda.synchronize()

    def step(k, prec):
        w = runs[k % len(runs)]
        i2 = plan.solve_boundary(bz[k % len(runs)], P, make_opts(PREC_FP64, a.rtol))
        i3 = plan.solve_interior(w.model, P, make_opts(prec, a.rtol, inner_cycles=a.inner_cycles))
        plan.fields(w.model, P, F)
        return i2, i3

    def timed(prec, steps, classes=None):
        """Run `steps` equilibria; with `classes`, time those kernel
        classes with HIP events (a separate pass: events add queue packets
        between kernels, so the throughput figures come from unprofiled
        passes)."""
        lat, cyc, t3 = [], [], []
        if classes is not None:
            plan.profile(True, classes)
            plan.profile_read(reset=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(steps):
            ts = time.perf_counter()
            i2, i3 = step(k, prec)
            torch.cuda.synchronize()
            lat.append(time.perf_counter() - ts)
            cyc.append(i3.cycles)
            t3.append(i3.seconds)
        torch.cuda.synchronize()
        total = time.perf_counter() - t0
        prof = None
        if classes is not None:
            prof = plan.profile_read(reset=True)
            plan.profile(False)
        return total, lat, cyc, t3, prof

    for prec in (PREC_MIXED, PREC_FP64):
        for k in range(a.warmup):
            step(k, prec)
    torch.cuda.synchronize()

    mix_total, mix_lat, mix_cyc, mix_t3, _ = timed(PREC_MIXED, a.steps)
    f64_total, f64_lat, f64_cyc, f64_t3, _ = timed(PREC_FP64, a.steps)
    # kernel breakdown (every class timed) and the dominant kernel alone
    _, _, _, _, mix_prof = timed(PREC_MIXED, a.steps, classes=list(_lib.PROF_NAMES))
    _, _, _, _, f64_prof = timed(PREC_FP64, a.steps, classes=list(_lib.PROF_NAMES))
    _, _, _, _, dom_prof = timed(PREC_MIXED, a.steps, classes=["smooth_l0"])

    # unfused compulsory-traffic model of the method (bytes per fine node):
    # FP64 V(2,2) 108.57; one refinement step with m FP32 V(2,2) 32 + 74.29 m
    m = a.inner_cycles
    f64_cycle_bytes = 108.57 * N
    mix_step_bytes = (32.0 + 74.29 * m) * N
    f64_vc_gbps = sum(f64_cyc) * f64_cycle_bytes / sum(f64_t3) / 1e9
    mix_vc_gbps = sum(mix_cyc) * mix_step_bytes / sum(mix_t3) / 1e9

    def kernels(prof):
        out = {}
        for name, (ms, n, b) in prof.items():
            if n:
                out[name] = {"launches": n, "avg_us": 1e3 * ms / n, "ms": ms,
                             "gbps": b / (ms * 1e-3) / 1e9 if ms > 0 else None}
        return out

    kmix = kernels(mix_prof)
    dom = "smooth_l0"
    ms, n, b = dom_prof[dom]
    achieved = b / (ms * 1e-3) / 1e9
    traffic = recorded_traffic()
    roofline = {"bound": "hbm", "kernel": "level-0 FP32 red-black smoother k_sweep3<float, 3|1|9> (zero guess, with f, with prolongation)",
                "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBPS, "traffic": traffic,
                "algorithmic_bytes_per_launch": b / n, "avg_launch_us": 1e3 * ms / n, "launches": n}

    batched = batched_fp64 = None
    if a.batch > 0:
        batched = batched_leg(a, runs, bz, PREC_MIXED, a.steps)
        batched_fp64 = batched_leg(a, runs, bz, PREC_FP64, a.steps)

    serving = None
    if a.serve_requests > 0:
        serving = serve_leg(a, torch, dev)

    single_mixed = a.steps / mix_total
    if batched is not None:
        value, ms_step = batched["solves_per_s"], batched["ms_per_solve"]
        p50, p99 = batched["p50_ms"], batched["p99_ms"]
        path = f"mixed (FP32 V(2,2) in FP64 refinement), {a.batch} requests in flight (continuous batching)"
    else:
        value, ms_step = single_mixed, 1e3 * mix_total / a.steps
        p50, p99 = 1e3 * percentile(mix_lat, 0.5), 1e3 * percentile(mix_lat, 0.99)
        path = "mixed (FP32 V(2,2) in FP64 refinement), one request at a time"
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32",
        "data": "synthetic",
        "config": {"workload": a.workload, "grid": f"{grid.nx}x{grid.ny}x{grid.nz}",
                   "runs": len(runs), "path": path, "batch": a.batch,
                   "rtol": a.rtol, "inner_cycles": m, "error_target": 1e-8},
        "p50_ms": p50,
        "p99_ms": p99,
        "refinement_steps": sum(mix_cyc) / len(mix_cyc),
        "ir_step_model_gbps": mix_vc_gbps,
        "single_stream": {"mixed": {"solves_per_s": single_mixed, "ms_per_solve": 1e3 * mix_total / a.steps,
                                    "p50_ms": 1e3 * percentile(mix_lat, 0.5),
                                    "p99_ms": 1e3 * percentile(mix_lat, 0.99)},
                          "fp64": {"solves_per_s": a.steps / f64_total, "ms_per_solve": 1e3 * f64_total / a.steps,
                                   "p50_ms": 1e3 * percentile(f64_lat, 0.5),
                                   "p99_ms": 1e3 * percentile(f64_lat, 0.99)}},
        "batched": {"mixed": batched, "fp64": batched_fp64},
        "fp64": {"value": a.steps / f64_total, "unit": "solves/s", "ms_per_step": 1e3 * f64_total / a.steps,
                 "p50_ms": 1e3 * percentile(f64_lat, 0.5), "p99_ms": 1e3 * percentile(f64_lat, 0.99),
                 "vcycles": sum(f64_cyc) / len(f64_cyc), "vcycle_model_gbps": f64_vc_gbps,
                 "kernels": kernels(f64_prof)},
        "kernels": kmix,
        "kernels_note": "per-class HIP-event timings from a separate pass with every class timed",
        "roofline": roofline,
        "serving": serving,
        "context": {"paper_speedup": "x30 GPU vs serial (x32.4 at 128^3, x29.6 at 256^3); hardware unstated"},
    }
    if not a.no_cpu:
        cb = cpu_baseline(a.cpu_run)
        line["cpu_baseline"] = cb
        line["speedup_vs_cpu_baseline"] = line["value"] / cb["value"]
    plan.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
