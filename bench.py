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
import gc
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
    ap.add_argument("--steps", type=int, default=36)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="mhs-257")
    ap.add_argument("--rtol", type=float, default=1e-10)
    ap.add_argument("--inner-cycles", type=int, default=3,
                    help="FP32 V-cycles per refinement step of the mixed path")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-run", type=int, default=3)
    ap.add_argument("--serve-requests", type=int, default=512,
                    help="requests of the serving stream (0 skips the serving leg)")
    ap.add_argument("--serve-rate", type=float, default=0.0,
                    help="Poisson arrival rate in requests/s (0: 0.5x and 0.9x of the capacity measured "
                         "with every request queued at once)")
    ap.add_argument("--serve-slots", type=int, default=32,
                    help="slots of the serving batch (requests in flight)")
    ap.add_argument("--batch", type=int, default=12,
                    help="concurrent requests in the batched pass over the workload (0: single stream only)")
    ap.add_argument("--serve-budget-gb", type=float, default=64.0)
    ap.add_argument("--large-workload", default="mhs-513x513x257",
                    help="the large single equilibrium reported beside the headline ('' skips it)")
    ap.add_argument("--large-rtol", type=float, default=1e-12,
                    help="stopping rtol of the large equilibrium (calibrated for 1e-8 error in every field)")
    ap.add_argument("--no-general", dest="general", action="store_false",
                    help="skip the general-operator leg (a lap u + b u = c at 257^3)")
    ap.add_argument("--large-only", action="store_true",
                    help="run only the large-equilibrium leg (the workload of its rocprofv3 summary)")
    ap.add_argument("--counter-probe", action="store_true",
                    help="run only the workload of the rocprofv3 FETCH_SIZE/WRITE_SIZE runs")
    ap.add_argument("--summarize-counters", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="print the traffic summary from the two counter runs' counter_collection.csv")
    ap.add_argument("--summarize-trace", nargs="+", metavar="CSV",
                    help="print the kernel summary of a --kernel-trace --stats [--marker-trace] run: "
                         "STATS_CSV TRACE_CSV [MARKER_CSV]")
    return ap.parse_args()


def percentile(xs, q):
    s = sorted(xs)
    if not s:
        return None
    k = (len(s) - 1) * q
    lo, hi = int(k), min(int(k) + 1, len(s) - 1)
    return s[lo] + (s[hi] - s[lo]) * (k - lo)


def recorded_traffic():
    """HBM traffic of the level-0 smoother measured with rocprofv3 counters
    (bytes per one-request launch, and traffic / compulsory bytes of merged
    launches), valid only for the kernel source it was measured on."""
    try:
        meta = {}
        with open(TRAFFIC_FILE) as fh:
            for line in fh:
                if ":" in line:
                    k, v = line.split(":", 1)
                    meta[k.strip()] = v.strip()
        if meta.get("kernels_sha256") != kernels_digest():
            return None
        return {"single_ratio": float(meta["single_traffic_ratio"]),
                "merged_ratio": float(meta["merged_traffic_ratio"])}
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


# level-0 FP32 smoother variants and their compulsory bytes per fine node:
# the zero-guess sweep (read f, write u; the first sweep of a refinement
# step), sweeps with f (read u, f; write u) and the prolongation sweep
# (+ coarse correction, N/8 floats); per FP32 V(2,2) cycle one prolongation
# sweep and two or three with f
SMOOTH_L0_MIX = {"k_sweep3<float, 3>": 8.0, "k_sweep3<float, 1>": 12.0, "k_sweep3<float, 9>": 12.5}
COPY_BYTES = 1 << 30
# workgroups of a one-request level-0 smoother launch at 257^3: 4 x 16 tiles
# of 64 x 16 nodes per plane, 8 chunks of 32 planes
SMOOTH_L0_GROUPS_257 = 512


def counter_probe(batch=12, requests=24):
    """Workload of the FETCH_SIZE / WRITE_SIZE runs: a device copy of
    COPY_BYTES (the calibration kernel: it reads and writes exactly that
    many bytes), two mixed-path equilibria of the 257^3 workload one at a
    time, then `requests` of its equilibria served with `batch` in flight
    (the merged launches of the batched pass)."""
    import torch

    import synth
    from paper_1307_6720_amd import PREC_FP64, PREC_MIXED
    from paper_1307_6720_amd.serve import DeviceBackend, Request, Server
    from paper_1307_6720_amd.solver import Plan, make_opts

    dev = "cuda:0"
    src = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    runs = [synth.workload("mhs-257", run=r) for r in range(synth.nruns("mhs-257"))]
    w = runs[3]
    plan = Plan(w.grid, PREC_FP64 | PREC_MIXED, device=dev)
    bz = torch.from_numpy(w.bz0).to(dev)
    P = torch.zeros(w.grid.shape, dtype=torch.float64, device=dev)
    for _ in range(2):
        plan.solve_boundary(bz, P, make_opts(rtol=1e-10))
        plan.solve_interior(w.model, P, make_opts(PREC_MIXED, rtol=1e-10))
    torch.cuda.synchronize()
    plan.close()
    bzs = [torch.from_numpy(r.bz0).to(dev) for r in runs]
    be = DeviceBackend(max_slots=batch, device=dev)
    srv = Server(be, 64 << 30)
    reqs = [Request(id=k, dims=(runs[0].grid.nx, runs[0].grid.ny, runs[0].grid.nz), model=runs[k % len(runs)].model,
                    bz0=bzs[k % len(runs)], precision=PREC_MIXED, rtol=1e-10) for k in range(requests)]
    done, st = srv.run(reqs)
    torch.cuda.synchronize()
    be.close()
    assert st["ok"] == requests, st
    print("counter probe done", flush=True)


def summarize_counters(fetch_csv, write_csv, one_groups=SMOOTH_L0_GROUPS_257):
    """HBM traffic of the level-0 FP32 smoother from the two counter runs of
    counter_probe, each counter scaled by what it reads for the calibration
    copy.  A launch of the smoother covering k requests of the 257^3
    workload has k * one_groups workgroups; level-0 launches read about
    8x what level-1 launches of the same k read, and launches issued after
    a solve converged read nothing.  Prints the summary kept under
    profiles/: the ratio of measured to compulsory bytes over the
    one-request (k = 1) and over the merged (k > 1) launches, weighted by
    their launch counts (bench.py scales its own compulsory bytes per launch
    by them)."""
    import collections
    import csv

    def load(path, counter):
        agg = collections.OrderedDict()
        with open(path) as fh:
            for r in csv.DictReader(fh):
                if r["Counter_Name"] != counter:
                    continue
                d = r["Dispatch_Id"]
                if d not in agg:
                    agg[d] = [r["Kernel_Name"], int(r["Grid_Size"]) // max(1, int(r["Workgroup_Size"])), 0.0]
                agg[d][2] += float(r["Counter_Value"]) * 1024.0  # KiB per dispatch
        return list(agg.values())

    fetch, write = load(fetch_csv, "FETCH_SIZE"), load(write_csv, "WRITE_SIZE")

    def calib(rows):
        # the largest copy kernel is the calibration copy
        return max(v for n, g, v in rows if "copy" in n.lower()) / COPY_BYTES

    cf, cw = calib(fetch), calib(write)
    N = 257 ** 3

    def level0(rows, scale, min_bytes_per_req):
        out = collections.defaultdict(list)  # (kernel, k) -> bytes
        for n, g, v in rows:
            kn = _short_kernel(n)
            if kn not in SMOOTH_L0_MIX or g % one_groups:
                continue
            k = g // one_groups
            if v / scale > k * min_bytes_per_req:
                out[(kn, k)].append(v / scale)
        return out

    # level 0 reads >= 4 B/node (>= 67 MB) and writes 3.94 B/node per request;
    # level 1 an eighth of that
    F = level0(fetch, cf, 30e6)
    W = level0(write, cw, 30e6)
    print(f"calibration: a device copy of {COPY_BYTES} B reads FETCH_SIZE = {cf:.4f} x bytes read, "
          f"WRITE_SIZE = {cw:.4f} x bytes written; counts below are divided by these factors")
    print("level-0 launches by variant and requests per launch (k): bytes per request, over the launches in "
          "which every request ran (within 10 % of the median; in the tick where a request stops, its items "
          "exit at once)")

    def full(xs, k):
        med = sorted(xs)[len(xs) // 2] / k
        return [x for x in xs if x / k >= 0.9 * med]

    meas = alg = meas1 = alg1 = 0.0
    for key in sorted(set(F) & set(W)):
        kn, k = key
        fk, wk = full(F[key], k), full(W[key], k)
        fb, wb = sum(fk) / len(fk) / k, sum(wk) / len(wk) / k
        c = SMOOTH_L0_MIX[kn]
        print(f"  {kn:22s} k={k:2d}  launches {len(fk):3d} of {len(F[key]):3d}  read {fb / N:5.2f} B/node "
              f"(compulsory {c - 4:.2f})  write {wb / N:5.2f} B/node (compulsory 4.00)")
        if k > 1:
            meas += (fb + wb) * k * len(fk)
            alg += k * c * N * len(fk)
        else:
            meas1 += (fb + wb) * len(fk)
            alg1 += c * N * len(fk)
    print(f"one-request launches (k = 1): traffic / compulsory = {meas1 / alg1:.3f}")
    print(f"merged launches (k > 1): traffic / compulsory = {meas / alg:.3f}")
    print(f"kernels_sha256: {kernels_digest()}")
    print(f"single_traffic_ratio: {meas1 / alg1:.4f}")
    print(f"merged_traffic_ratio: {meas / alg:.4f}")


def _level0_split(launches, one_groups):
    """Pick the level-0 launches among launches of the smoother: (start,
    end, kernel, groups) tuples.  Within one kernel variant and workgroup
    count (equal requests per launch), level-0 launches take several times
    longer than level-1 launches and launches whose items all exited at once
    take a few microseconds (about 1 us per 1024 workgroups): the level-0
    launches are those above the largest duration ratio between neighbours
    among the launches longer than 3 us per 1024 workgroups (at least 5 us).
    Where the durations form one cluster (merged launches, whose level-1
    launches have other workgroup counts), the cluster is level 0 if its
    median takes at least 15 us per request (a level-0 FP32 sweep of one
    257^3 request takes 25-55 us, a level-1 sweep under 10 us)."""
    import collections

    by = collections.defaultdict(list)
    for x in launches:
        by[(x[2], x[3])].append(x)
    out = []
    for (_, g), v in by.items():
        floor = max(5000.0, 3000.0 * g / 1024)
        v = sorted((x for x in v if (x[1] - x[0]) > floor), key=lambda x: x[1] - x[0])
        if not v:
            continue
        d = [x[1] - x[0] for x in v]
        gaps = [d[i + 1] / d[i] for i in range(len(d) - 1)]
        if not gaps or max(gaps) < 1.8:
            # one cluster: no level-0 / level-1 split to make
            if d[len(d) // 2] >= 15000.0 * max(1, g // one_groups):
                out.extend(v)
            continue
        cut = gaps.index(max(gaps)) + 1
        out.extend(v[cut:])
    return sorted(out)


def summarize_trace(stats_csv, trace_csv, marker_csv=None, one_groups=SMOOTH_L0_GROUPS_257, top=24):
    """Kernel-time summary of a rocprofv3 --kernel-trace --stats (and
    --marker-trace) run of bench.py: the stats table; the launches that ran
    (> 5 us; launches issued after a solve converged exit at once) by
    kernel and workgroup count; and the level-0 FP32 smoother launches (a
    launch covering k requests of the 257^3 workload has k * one_groups
    workgroups) with their average duration, over the run and inside each
    ROCTx range of bench.py (the passes whose HIP-event timings give the
    roofline)."""
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
    sm = []  # (start, end, kernel, groups) of the FP32 smoother variants
    for r in rows:
        kn = _short_kernel(r["Kernel_Name"])
        g = int(r["Grid_Size_X"]) // max(1, int(r["Workgroup_Size_X"]))
        t0, t1 = int(r["Start_Timestamp"]), int(r["End_Timestamp"])
        agg[(kn, g)].append((t1 - t0) / 1e3)
        if kn in SMOOTH_L0_MIX and g % one_groups == 0:
            sm.append((t0, t1, kn, g))
    print()
    print("## launches that ran (> 5 us), by kernel and workgroup count")
    print(f"{'kernel':40s} {'groups':>7s} {'ran':>5s} {'avg_us':>8s} {'med_us':>8s} {'skip':>5s} {'ran_ms':>8s}")
    out = []
    for (kn, g), v in agg.items():
        ran = sorted(d for d in v if d > 5.0)
        if ran:
            out.append((sum(ran), kn, g, len(ran), sum(ran) / len(ran), ran[len(ran) // 2], len(v) - len(ran)))
    for tot, kn, g, n, avg, med, sk in sorted(out, reverse=True)[:32]:
        print(f"{kn[:40]:40s} {g:7d} {n:5d} {avg:8.2f} {med:8.2f} {sk:5d} {tot / 1e3:8.3f}")

    def table(sel, title):
        print()
        print(title)
        l0 = _level0_split(sel, one_groups)
        by = collections.defaultdict(list)
        for t0, t1, kn, g in l0:
            by[(kn, g // one_groups)].append((t1 - t0) / 1e3)
        for (kn, k), v in sorted(by.items()):
            print(f"  {kn:22s} k={k}  launches {len(v):4d}  avg_us {statistics.mean(v):8.2f}  "
                  f"median_us {statistics.median(v):8.2f}")
        ds = [(t1 - t0) / 1e3 for t0, t1, _, _ in l0]
        if ds:
            print(f"  all: {len(ds)} launches, average {statistics.mean(ds):.2f} us")

    if not marker_csv:
        table(sm, "## level-0 FP32 smoother launches over the whole run, by requests per launch k")
    else:
        with open(marker_csv) as fh:
            marks = list(csv.DictReader(fh))
        for m in marks:
            name = next((v for v in m.values() if v in ("roofline_pass", "roofline_single_request_pass")), None)
            if name is None:
                continue
            a, b = int(m["Start_Timestamp"]), int(m["End_Timestamp"])
            table([x for x in sm if a <= x[0] and x[1] <= b],
                  f"## the same inside the ROCTx range {name} (bench.py times these launches with HIP events)")


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def field_errors_vs_exact(run, results):
    """Per-field relative max-norm errors of GPU results of one equilibrium
    of the workload against the exact discrete solution and its field
    recovery (the oracle's): P, Bx, By, Bz, p - p_b, rho - rho_b.  `results`
    maps a label to host arrays (P, Bx, By, Bz, p, rho).  Part of the CPU
    baseline leg, outside every timed region."""
    import numpy as np

    import synth
    from oracle import exact
    from oracle import fields as ofields

    w = synth.workload("mhs-257", run=run)
    m = w.model
    want_P = exact.solve(w.bz0, w.grid.nz, m.xi, m.alpha)
    want = ofields.fields(want_P, m.alpha, m.xi, m.dxi, m.pb, m.rhob, m.mu0, m.g)
    pb, rb = m.pb[:, None, None], m.rhob[:, None, None]
    ref_ = [want_P, want[0], want[1], want[2], want[3] - pb, want[4] - rb]

    def rel(a, b):
        d = np.abs(b).max()
        return float(np.abs(a - b).max() / (d if d > 0 else 1.0))

    out = {}
    for label, got in results.items():
        got = list(got)
        got[4] = got[4] - pb
        got[5] = got[5] - rb
        out[label] = {n: rel(g, r) for n, g, r in zip(("P", "Bx", "By", "Bz", "dp", "drho"), got, ref_)}
    return out


def cpu_baseline(run, reps=3):
    """The oracle (plain C multigrid + numpy field recovery) on one
    equilibrium of the same workload, timed with one thread and with the
    host's CPU share (OpenMP over the node loops of the C multigrid; the
    numpy field recovery is single-threaded either way); median of `reps`
    runs each.  The 2D + 3D solve and the fields are timed separately."""
    import os

    import numpy as np

    import synth
    from oracle import fields as ofields
    from oracle import ref

    w = synth.workload("mhs-257", run=run)
    m = w.model
    share = len(os.sched_getaffinity(0))
    want = int(os.environ.get("OMP_NUM_THREADS") or share)
    legs = {}
    for label, th in (("single_thread", 1), ("all_cores", want)):
        used = ref.set_threads(th)
        solve_s, fields_s = [], []
        for _ in range(reps):
            t0 = time.perf_counter()
            P, st, info = ref.solve(w.bz0, m.xi, m.alpha, w.grid.shape, rtol2=1e-10, rtol3=1e-10)
            t1 = time.perf_counter()
            ofields.fields(P, m.alpha, m.xi, m.dxi, m.pb, m.rhob, m.mu0, m.g)
            t2 = time.perf_counter()
            assert st == ref.OK and np.isfinite(P).all()
            solve_s.append(t1 - t0)
            fields_s.append(t2 - t1)
        tot = float(np.median(np.add(solve_s, fields_s)))
        legs[label] = {"value": 1.0 / tot, "unit": "solves/s", "cores": used,
                       "solve_s_median": float(np.median(solve_s)), "fields_s_median": float(np.median(fields_s)),
                       "runs_s": [round(a + b, 3) for a, b in zip(solve_s, fields_s)]}
    ref.set_threads(want)
    best = legs["all_cores"]
    return {"value": best["value"], "unit": "solves/s", "cores": best["cores"], "kind": "oracle",
            "sample": f"one full solve of {w.name} run {run} ({w.grid.nx}^3): 2D+3D V(2,2) to rtol 1e-10 "
                      f"({info['cycles2d']}+{info['cycles3d']} cycles) plus fields, median of {reps}; "
                      f"C multigrid (gcc -O2, OpenMP over node loops) with {best['cores']} threads, "
                      f"numpy fields on one",
            "cpu_model": _cpu_model(), "nproc": os.cpu_count(), "cpu_share": share,
            "single_thread": legs["single_thread"], "all_cores": legs["all_cores"]}


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

    budget = int(a.serve_budget_gb * (1 << 30))
    be = DeviceBackend(max_slots=a.serve_slots, device=dev, hbm_budget=budget)
    srv = Server(be, budget)

    def stream(arrivals):
        reqs = [Request(id=i, dims=(w.grid.nx, w.grid.ny, w.grid.nz), model=w.model, bz0=bz,
                        precision=PREC_MIXED, rtol=a.rtol, inner_cycles=a.inner_cycles, arrival=t)
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


class _Roctx:
    """ROCTx ranges around the passes of this benchmark (rocprofv3
    --marker-trace records them; the trace summary uses them to pick the
    launches of the pass the roofline is computed from).  No-op when the
    library is absent."""

    def __init__(self):
        import ctypes

        self.lib = None
        for name in ("librocprofiler-sdk-roctx.so", "/opt/rocm/lib/librocprofiler-sdk-roctx.so", "libroctx64.so"):
            try:
                self.lib = ctypes.CDLL(name)
                self.lib.roctxRangePushA.argtypes = [ctypes.c_char_p]
                break
            except OSError:
                continue

    def push(self, name):
        if self.lib is not None:
            self.lib.roctxRangePushA(name.encode())

    def pop(self):
        if self.lib is not None:
            self.lib.roctxRangePop()


ROCTX = _Roctx()
ROOFLINE_RANGE = "roofline_pass"


def large_leg(a, torch, dev, reps=5):
    """The large anisotropic equilibrium (513 x 513 x 257, dz = 2 dx, xi(0) =
    1): per path, the solve time, the refinement steps or V-cycles and the
    traffic model's rate of the 3D part, plus the level shapes (the first
    step halves x and y only).  Solves to the calibrated rtol (1e-12: at
    1e-10 the noisy magnetogram leaves B, p, rho up to 2e-7 off the exact
    solution, at 1e-12 within 6e-9)."""
    import synth
    from paper_1307_6720_amd import PREC_FP64, PREC_MIXED
    from paper_1307_6720_amd.solver import Plan, make_opts, solve

    w = synth.workload(a.large_workload)
    g = w.grid
    N = g.npoints
    plan = Plan(g, PREC_FP64 | PREC_MIXED, device=dev)
    bz = torch.from_numpy(w.bz0).to(dev)
    arrays = tuple(torch.empty(g.shape, dtype=torch.float64, device=dev) for _ in range(6))
    out = {"workload": a.large_workload, "grid": f"{g.nx}x{g.ny}x{g.nz}", "rtol": a.large_rtol,
           "rtol_note": "the rtol at which every field is within 1e-8 of the exact solution on this grid"}
    for prec, name, per_cycle in ((PREC_MIXED, "mixed", (32.0 + 74.29 * a.inner_cycles) * N),
                                  (PREC_FP64, "fp64", 108.57 * N)):
        for _ in range(2):
            solve(plan, bz, w.model, precision=prec, rtol=a.large_rtol, inner_cycles=a.inner_cycles, out=arrays)
        torch.cuda.synchronize()
        ts, res = [], None
        for _ in range(reps):
            t0 = time.perf_counter()
            res = solve(plan, bz, w.model, precision=prec, rtol=a.large_rtol, inner_cycles=a.inner_cycles, out=arrays)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        # per-class HIP-event timings and compulsory-byte rates of one more
        # pass, the three steps as three calls (every launch of the recovery
        # timed; the interior's own time for the traffic model)
        plan.profile(True)
        plan.profile_read(reset=True)
        P, F = arrays[0], arrays[1:]
        plan.solve_boundary(bz, P, make_opts(PREC_FP64, a.large_rtol))
        i3 = plan.solve_interior(w.model, P, make_opts(prec, a.large_rtol, inner_cycles=a.inner_cycles)).as_dict()
        plan.fields(w.model, P, F)
        torch.cuda.synchronize()
        kern = {k: {"launches": n, "avg_us": 1e3 * ms / n, "gbps": b / (ms * 1e-3) / 1e9}
                for k, (ms, n, b) in plan.profile_read(reset=True).items() if n and ms > 0}
        plan.profile(False)
        out[name] = {"ms_per_solve": 1e3 * sum(ts) / reps, "cycles_3d": i3["cycles"],
                     "cycles_2d": res.info2d["cycles"], "rel_residual": i3["rel_residual"],
                     "model_gbps_3d": i3["cycles"] * per_cycle / i3["seconds"] / 1e9, "kernels": kern}
    out["levels"] = [list(plan.level_shape(3, l)) for l in range(plan.levels(3))]
    plan.close()
    del arrays
    return out


def general_leg(torch, dev, n=257, reps=3, rtol=1e-10):
    """The general problem a lap u + b u = c (per-node coefficients, the
    synth.general_problem recipe) on an n^3 unit box: time per solve to
    rtol, V-cycles, and the HIP-event rate of its kernels (algorithmic bytes:
    a sweep reads u, b/a, c/a and writes u, 32 B per node)."""
    import synth
    from paper_1307_6720_amd import PLAN_GENERAL, PREC_FP64
    from paper_1307_6720_amd.solver import Plan, make_opts

    g = synth.make_grid(n, n, n)
    a, b, c, u = synth.general_problem(g.shape, (g.lx, g.ly, g.lz), 41)
    a, b, c, u0 = (torch.from_numpy(x).to(dev) for x in (a, b, c, u))
    plan = Plan(g, PREC_FP64 | PLAN_GENERAL, device=dev)
    u = u0.clone()
    opts = make_opts(PREC_FP64, rtol)
    plan.solve_general(a, b, c, u, opts)
    ts, info = [], None
    for _ in range(reps):
        u.copy_(u0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = plan.solve_general(a, b, c, u, opts)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    u.copy_(u0)
    plan.profile(True, ["general"])
    plan.profile_read(reset=True)
    plan.solve_general(a, b, c, u, opts)
    torch.cuda.synchronize()
    ms, nl, by = plan.profile_read(reset=True)["general"]
    plan.profile(False)
    plan.close()
    return {"grid": f"{n}^3", "rtol": rtol, "ms_per_solve": 1e3 * sum(ts) / reps, "cycles": info.cycles,
            "rel_residual": info.rel_residual, "kernel_ms": ms, "launches": nl,
            "kernel_gbps": by / (ms * 1e-3) / 1e9 if ms > 0 else None,
            "note": "FP64 V(2,2); one-thread-per-node kernels; GB/s from algorithmic bytes (sweep 32 B/node, "
                    "residual 32, restriction 8 + 8/8, prolongation 16 + 8/8) over summed HIP-event durations"}


def level0_kz(grid):
    """Planes per workgroup of the level-0 smoother: the library's rule
    (about 1024 groups of 64 x 8 node units per request, at most 32 planes)."""
    units = -(-(grid.nx - 2) // 64) * -(-(grid.ny - 2) // 8)
    return max(1, min(32, -(-(grid.nz - 2) * units // 1024)))


def pattern_reference(torch, dev, grid, nreq):
    """Rates of mhs_probe_smoother_pattern: the level-0 smoother's memory
    traffic (12 B per interior node) in its own order with no LDS, barrier
    or arithmetic, for one request and for `nreq` requests per launch as in
    the merged launches; with the smoother's tile and z-chunk, and with a
    row-wide 256 x 8 tile (the headroom of another tiling).  HIP events on
    the stream of the launches, median of 9."""
    import ctypes as C

    from paper_1307_6720_amd import _lib

    L = _lib.lib()
    n = grid.nx * grid.ny * grid.nz
    interior = (grid.nx - 2) * (grid.ny - 2) * (grid.nz - 2)
    kz = level0_kz(grid)
    out = {}
    for label, k in (("single", 1), ("merged", nreq)):
        u = torch.zeros(k * n, dtype=torch.float32, device=dev)
        f = torch.zeros_like(u)
        o = torch.zeros_like(u)
        stream = C.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
        rates = {}
        for name, tile, tkz in (("pattern_reference_gbps", 0, kz), ("pattern_wide_tile_gbps", 1, 8)):
            def launch():
                _lib.check(L.mhs_probe_smoother_pattern(C.c_void_p(u.data_ptr()), C.c_void_p(f.data_ptr()),
                                                        C.c_void_p(o.data_ptr()), grid.nx, grid.ny, grid.nz, k,
                                                        tile, tkz, stream))
            for _ in range(3):
                launch()
            ts = []
            for _ in range(9):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                launch()
                e1.record()
                torch.cuda.synchronize()
                ts.append(e0.elapsed_time(e1))
            ms = sorted(ts)[len(ts) // 2]
            rates[name] = 12.0 * interior * k / (ms * 1e-3) / 1e9
        rates["pattern_note"] = (f"mhs_probe_smoother_pattern, {k} request(s) of {grid.nx}x{grid.ny}x{grid.nz} "
                                 f"per launch; smoother tile 64x16, {kz} planes per group; wide tile 256x8, 8 planes")
        out[label] = rates
        del u, f, o
    return out


def batched_leg(a, runs, bz, prec, steps, warm=True, profile=False):
    """The same equilibria served by the batching server with `a.batch`
    requests in flight (all queued at once): whole-job throughput and
    per-request latency.  With `profile`, two more passes over the same
    requests time the merged launches with HIP events: every class, then
    the level-0 smoother alone (inside the ROCTx range ROOFLINE_RANGE)."""
    import torch

    from paper_1307_6720_amd.serve import DeviceBackend, Request, Server

    be = DeviceBackend(max_slots=a.batch, device=bz[0].device)
    srv = Server(be, 64 << 30)

    def reqs(n):
        return [Request(id=k, dims=(runs[k % len(runs)].grid.nx, runs[k % len(runs)].grid.ny,
                                    runs[k % len(runs)].grid.nz),
                        model=runs[k % len(runs)].model, bz0=bz[k % len(runs)], precision=prec, rtol=a.rtol,
                        inner_cycles=a.inner_cycles, arrival=0.0) for k in range(n)]

    if warm:
        srv.run(reqs(a.batch))
    srv.ticks = srv.peak_active = 0
    done, st = srv.run(reqs(steps))
    assert st["ok"] == steps, st
    cyc = [r.info3d["cycles"] for r in done]
    out = {"solves_per_s": st["solves_per_s"], "ms_per_solve": 1e3 / st["solves_per_s"], "p50_ms": st["p50_ms"],
           "p99_ms": st["p99_ms"], "requests": steps, "in_flight": a.batch, "ticks": st["ticks"],
           "cycles": sum(cyc) / len(cyc)}
    if profile:
        b = be.batch
        for key, classes in (("prof_all", None), ("prof_smooth_l0", ["smooth_l0"])):
            b.profile(True, classes)
            b.profile_read(reset=True)
            torch.cuda.synchronize()
            if key == "prof_smooth_l0":
                ROCTX.push(ROOFLINE_RANGE)
            srv.run(reqs(steps))
            torch.cuda.synchronize()
            if key == "prof_smooth_l0":
                ROCTX.pop()
            out[key] = b.profile_read(reset=True)
            b.profile(False)
    be.close()
    return out


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
        print("bench.py: measures one GPU only (the path has no multi-GPU sharding); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    if a.counter_probe:
        counter_probe()
        return
    if a.large_only:
        import torch

        print(json.dumps({"large_case": large_leg(a, torch, torch.device("cuda:0"))}), flush=True)
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

    def step(k, prec, split=False):
        """One equilibrium: one library call (mhs_solve_equilibrium), or
        with `split` its three steps as three calls (the profiled passes:
        the combined call does not time the recovery it enqueues behind its
        batches)."""
        w = runs[k % len(runs)]
        o2 = make_opts(PREC_FP64, a.rtol)
        o3 = make_opts(prec, a.rtol, inner_cycles=a.inner_cycles)
        if not split:
            return plan.solve_equilibrium(bz[k % len(runs)], w.model, P, F, o2, o3)
        i2 = plan.solve_boundary(bz[k % len(runs)], P, o2)
        i3 = plan.solve_interior(w.model, P, o3)
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
            i2, i3 = step(k, prec, split=classes is not None)
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

    # Python's full garbage collections traverse every live object (torch and
    # numpy bring ~170k); one in a timed pass stalls the host ~40-60 ms between
    # two library calls.  Long-lived objects move to the permanent generation.
    gc.collect()
    gc.freeze()
    for prec in (PREC_MIXED, PREC_FP64):
        for k in range(a.warmup):
            step(k, prec)
    torch.cuda.synchronize()

    mix_total, mix_lat, mix_cyc, mix_t3, _ = timed(PREC_MIXED, a.steps)
    f64_total, f64_lat, f64_cyc, f64_t3, _ = timed(PREC_FP64, a.steps)
    # kernel breakdown (every class timed) and the dominant kernel alone
    _, _, _, _, mix_prof = timed(PREC_MIXED, a.steps, classes=list(_lib.PROF_NAMES))
    _, _, _, _, f64_prof = timed(PREC_FP64, a.steps, classes=list(_lib.PROF_NAMES))
    ROCTX.push("roofline_single_request_pass")
    _, _, _, _, dom_prof = timed(PREC_MIXED, a.steps, classes=["smooth_l0"])
    ROCTX.pop()

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
    traffic = recorded_traffic()

    def roofline_of(prof, where):
        ms, n, b = prof["smooth_l0"]
        achieved = b / (ms * 1e-3) / 1e9
        return {"bound": "hbm",
                "kernel": "level-0 FP32 red-black smoother k_sweep3<float, 3|1|9> (zero guess, with f, with prolongation)",
                "launches_timed": where,
                "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBPS, "traffic": None,
                "algorithmic_bytes_per_launch": b / n, "avg_launch_us": 1e3 * ms / n, "launches": n}

    roof_single = roofline_of(dom_prof, "one request per launch (single-stream pass)")
    roof_single["traffic"] = (None if traffic is None else
                              traffic["single_ratio"] * roof_single["algorithmic_bytes_per_launch"])

    batched = batched_fp64 = None
    if a.batch > 0:
        batched = batched_leg(a, runs, bz, PREC_MIXED, a.steps, profile=True)
        batched_fp64 = batched_leg(a, runs, bz, PREC_FP64, a.steps)
        roofline = roofline_of(batched.pop("prof_smooth_l0"),
                               f"merged launches of the batched pass ({a.batch} requests in flight)")
        # counters taken on merged launches of the same pass: measured bytes
        # per compulsory byte, times this pass's compulsory bytes per launch
        roofline["traffic"] = (None if traffic is None else
                               traffic["merged_ratio"] * roofline["algorithmic_bytes_per_launch"])
        batched["kernels"] = kernels(batched.pop("prof_all"))
    else:
        roofline = roof_single

    def copy_reference(nbytes):
        """A plain device copy (torch copy_ of float32) moving the same bytes
        as one launch of the dominant kernel: half read, half written."""
        n = max(1, int(nbytes // 8))
        x = torch.ones(n, dtype=torch.float32, device=dev)
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0.record()
        for _ in range(10):
            y.copy_(x)
        t1.record()
        torch.cuda.synchronize()
        gbps = 8.0 * n / (t0.elapsed_time(t1) / 10 * 1e-3) / 1e9
        del x, y
        return gbps

    for r in (roofline, roof_single):
        if "copy_reference_gbps" not in r:
            r["copy_reference_gbps"] = copy_reference(r["algorithmic_bytes_per_launch"])
            r["frac_of_copy_reference"] = r["achieved"] / r["copy_reference_gbps"]
    pattern = pattern_reference(torch, dev, grid, a.batch if batched is not None else 1)
    roofline.update(pattern["merged" if batched is not None else "single"])
    roofline["frac_of_pattern_reference"] = roofline["achieved"] / roofline["pattern_reference_gbps"]
    roof_single.update(pattern["single"])
    roof_single["frac_of_pattern_reference"] = roof_single["achieved"] / roof_single["pattern_reference_gbps"]

    # diagnostics of (1)-(3) on the last equilibrium's fields (off the
    # solve's path): j, |force residual|, div B; 80 B per node (read 5, write 5)
    D = tuple(torch.empty_like(P) for _ in range(5))
    w = runs[(a.steps - 1) % len(runs)]
    for _ in range(3):
        plan.diagnostics(w.model, *F, out=D)
    plan.profile(True, ["diag"])
    plan.profile_read(reset=True)
    for _ in range(10):
        plan.diagnostics(w.model, *F, out=D)
    torch.cuda.synchronize()
    dms, dn, dbytes = plan.profile_read(reset=True)["diag"]
    plan.profile(False)
    diag_gbps = dbytes / (dms * 1e-3) / 1e9
    jx, jy, jz = D[0], D[1], D[2]
    lor = torch.sqrt((jy * F[2] - jz * F[1]) ** 2 + (jz * F[0] - jx * F[2]) ** 2 + (jx * F[1] - jy * F[0]) ** 2)
    diagnostics = {"kernel": "k_diag", "avg_us": 1e3 * dms / dn, "launches": dn, "bytes_per_node": 80,
                   "achieved_gbps": diag_gbps, "frac_of_hbm_peak": diag_gbps / HBM_PEAK_GBPS,
                   "force_residual_over_lorentz": float(D[3].max() / lor.max())}
    del D, lor

    # field lines of the same equilibrium from 16384 seeds on the base
    # (RK4, ds = half a node spacing, at most 1024 steps): one thread per line
    gx = torch.linspace(0.02, 0.98, 128, dtype=torch.float64, device=dev)
    seeds = torch.stack([gx.repeat(128) * grid.lx, gx.repeat_interleave(128) * grid.ly,
                         torch.zeros(128 * 128, dtype=torch.float64, device=dev)], dim=1).contiguous()
    ds = 0.5 * grid.lx / (grid.nx - 1)
    L_out = (torch.empty((1025, seeds.shape[0], 3), dtype=torch.float64, device=dev),
             torch.empty(seeds.shape[0], dtype=torch.int32, device=dev),
             torch.empty(seeds.shape[0], dtype=torch.int32, device=dev))
    plan.trace_field_lines(*F[:3], seeds, ds, 1024, 1e-8, out=L_out)
    plan.profile(True, ["trace"])
    plan.profile_read(reset=True)
    for _ in range(3):
        plan.trace_field_lines(*F[:3], seeds, ds, 1024, 1e-8, out=L_out)
    torch.cuda.synchronize()
    tms, tn, _ = plan.profile_read(reset=True)["trace"]
    plan.profile(False)
    cnt, st = L_out[1].cpu(), L_out[2].cpu()
    steps = int((cnt - 1).sum())
    field_lines = {"kernel": "k_trace", "lines": int(seeds.shape[0]), "ds": ds, "max_steps": 1024,
                   "steps_taken": steps, "avg_ms": tms / tn, "steps_per_s": steps / (tms / tn * 1e-3),
                   "ended": {"left_box": int((st == 1).sum()), "null": int((st == 2).sum()),
                             "step_cap": int((st == 0).sum())}}
    del L_out

    serving = None
    if a.serve_requests > 0:
        serving = serve_leg(a, torch, dev)
    large = large_leg(a, torch, dev) if a.large_workload else None
    general = general_leg(torch, dev) if a.general else None

    single_mixed = a.steps / mix_total
    if batched is not None:
        value, ms_step = batched["solves_per_s"], batched["ms_per_solve"]
        p50, p99 = batched["p50_ms"], batched["p99_ms"]
        path = f"mixed ({m} FP32 V(2,2) per FP64 refinement step), {a.batch} requests in flight (continuous batching)"
    else:
        value, ms_step = single_mixed, 1e3 * mix_total / a.steps
        p50, p99 = 1e3 * percentile(mix_lat, 0.5), 1e3 * percentile(mix_lat, 0.99)
        path = f"mixed ({m} FP32 V(2,2) per FP64 refinement step), one request at a time"
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
                                    "p99_ms": 1e3 * percentile(mix_lat, 0.99),
                                    "solves_per_s_at_p50": 1.0 / percentile(mix_lat, 0.5)},
                          "fp64": {"solves_per_s": a.steps / f64_total, "ms_per_solve": 1e3 * f64_total / a.steps,
                                   "p50_ms": 1e3 * percentile(f64_lat, 0.5),
                                   "p99_ms": 1e3 * percentile(f64_lat, 0.99),
                                   "solves_per_s_at_p50": 1.0 / percentile(f64_lat, 0.5)}},
        "batched": {"mixed": batched, "fp64": batched_fp64},
        "fp64": {"value": a.steps / f64_total, "unit": "solves/s", "ms_per_step": 1e3 * f64_total / a.steps,
                 "p50_ms": 1e3 * percentile(f64_lat, 0.5), "p99_ms": 1e3 * percentile(f64_lat, 0.99),
                 "vcycles": sum(f64_cyc) / len(f64_cyc), "vcycle_model_gbps": f64_vc_gbps,
                 "kernels": kernels(f64_prof)},
        "kernels": kmix,
        "kernels_note": "per-class HIP-event timings from a separate pass with every class timed",
        "roofline": roofline,
        "roofline_single_request": roof_single,
        "diagnostics": diagnostics,
        "field_lines": field_lines,
        "serving": serving,
        "large_case": large,
        "general": general,
        "context": {"paper_speedup": "x30 GPU vs serial (x32.4 at 128^3, x29.6 at 256^3); hardware unstated"},
    }
    if not a.no_cpu:
        # per-field errors of one equilibrium (the CPU leg's run) on both
        # paths, against the exact discrete solution (untimed)
        w = runs[a.cpu_run % len(runs)]
        bzk = bz[a.cpu_run % len(runs)]
        results = {}
        for label, prec, rt in (("mixed_rtol%g" % a.rtol, PREC_MIXED, a.rtol),
                                ("fp64_rtol%g" % a.rtol, PREC_FP64, a.rtol), ("fp64_rtol1e-12", PREC_FP64, 1e-12)):
            plan.solve_boundary(bzk, P, make_opts(PREC_FP64, rt))
            plan.solve_interior(w.model, P, make_opts(prec, rt, inner_cycles=a.inner_cycles))
            plan.fields(w.model, P, F)
            torch.cuda.synchronize()
            results[label] = [t.cpu().numpy() for t in (P,) + F]
        line["errors"] = {"workload": f"{a.workload} run {a.cpu_run}",
                          "metric": "max|x - x_exact| / max|x_exact| per field; p, rho as p - p_b, rho - rho_b",
                          "gates": {"mixed": 1e-8, "fp64": 1e-10},
                          **field_errors_vs_exact(a.cpu_run, results)}
        del results
        cb = cpu_baseline(a.cpu_run)
        line["cpu_baseline"] = cb
        line["speedup_vs_cpu_baseline"] = line["value"] / cb["value"]
        line["speedup_vs_cpu_single_thread"] = line["value"] / cb["single_thread"]["value"]
    plan.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
