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
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if a.gpus != 1 or world != 1:
        print("bench.py: this build measures one GPU only (the path has no multi-GPU sharding); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

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
