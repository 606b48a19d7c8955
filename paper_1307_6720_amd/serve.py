"""Continuous-batching server for NR99 equilibria on one device.

Requests (grid, alpha, xi tables, magnetogram, precision, tolerance) arrive
over time.  The server keeps multigrid plans and output buffers resident in
a pool keyed by grid shape, admits queued requests in arrival order while a
batch slot is free and the device memory in use stays within the HBM
budget, and drives the batch: every tick advances each admitted request by
one V-cycle or refinement step, with equal stages of all requests merged
into single descriptor-driven launches (the mhs_batch_* entry points).
Requests that finish retire and their resources return to the pool.

The scheduling policy is plain Python and device-independent: it talks to a
backend (``DeviceBackend`` here; tests substitute a host-only simulation).
"""

from __future__ import annotations

import ctypes as C
import time
from collections import OrderedDict, deque
from dataclasses import dataclass, field

import numpy as np

from . import _lib
from ._lib import PREC_FP64, PREC_MIXED, check


@dataclass
class Request:
    """One equilibrium to compute.  ``bz0`` is (ny, nx) float64 (host numpy
    or a device tensor); ``model`` carries alpha and the per-z tables xi,
    dxi, pb, rhob (length nz) and mu0, g."""

    id: int
    dims: tuple  # (nx, ny, nz)
    model: object
    bz0: object
    precision: int = PREC_MIXED
    rtol: float = 1e-10
    inner_cycles: int | None = None  # FP32 V-cycles per refinement step (mixed); None: the library's default
    lengths: tuple = (1.0, 1.0, 1.0)
    arrival: float = 0.0  # seconds after the start of the run
    # filled by the server
    admitted: float | None = None
    finished: float | None = None
    status: int | None = None
    info2d: dict = field(default_factory=dict)
    info3d: dict = field(default_factory=dict)

    @property
    def latency(self):
        return None if self.finished is None else self.finished - self.arrival


def percentile(xs, q):
    s = sorted(xs)
    if not s:
        return None
    k = (len(s) - 1) * q
    lo, hi = int(k), min(int(k) + 1, len(s) - 1)
    return s[lo] + (s[hi] - s[lo]) * (k - lo)


class Server:
    """Admission, pooling and the tick loop.

    backend: object with ``footprint(key)``, ``acquire(key)``, ``free(res)``,
    ``admit(res, req)``, ``step()``, ``poll(slot)``, ``release(slot)`` and
    ``max_slots`` (see DeviceBackend).
    hbm_budget: bytes of device memory the pool may hold (resident plans and
    buffers, in use or idle).
    on_finish(req, resident): optional; called before a finished request's
    resources return to the pool (e.g. to copy its outputs).

    The tick loop runs in Python: a full garbage collection during it (tens
    of ms with torch loaded) delays every request in flight.  Latency-bound
    callers can call ``gc.collect(); gc.freeze()`` once after setting up.
    """

    def __init__(self, backend, hbm_budget, on_finish=None):
        self.backend = backend
        self.budget = int(hbm_budget)
        self.on_finish = on_finish
        self.queue = deque()
        self.idle = OrderedDict()  # key -> list of idle residents (LRU order of keys)
        self.resident_bytes = 0
        self.active = {}  # slot -> (request, resident)
        self.peak_bytes = 0
        self.peak_active = 0
        self.peak_queue = 0
        self.ticks = 0
        self._retired = []

    @staticmethod
    def key(req):
        return (tuple(req.dims), tuple(req.lengths))

    def submit(self, req):
        self.queue.append(req)
        self.peak_queue = max(self.peak_queue, len(self.queue))

    def _evict_idle(self, need):
        """Free idle residents (least recently used shapes first) until
        `need` more bytes fit the budget.  Returns True on success."""
        while self.resident_bytes + need > self.budget:
            victim = None
            for k, lst in self.idle.items():
                if lst:
                    victim = k
                    break
            if victim is None:
                return False
            res = self.idle[victim].pop()
            if not self.idle[victim]:
                del self.idle[victim]
            self.resident_bytes -= res.nbytes
            self.backend.free(res)
        return True

    def _take_resident(self, req):
        k = self.key(req)
        lst = self.idle.get(k)
        if lst:
            res = lst.pop()
            if not lst:
                del self.idle[k]
            return res
        need = self.backend.footprint(k)
        if need > self.budget:
            raise ValueError(f"request {req.id}: footprint {need} B exceeds the HBM budget {self.budget} B")
        if not self._evict_idle(need):
            return None
        res = self.backend.acquire(k)
        self.resident_bytes += res.nbytes
        self.peak_bytes = max(self.peak_bytes, self.resident_bytes)
        return res

    def _return_resident(self, res):
        self.idle.setdefault(res.key, []).append(res)
        self.idle.move_to_end(res.key)

    def admit_ready(self, now):
        """Admit queued requests in arrival order while a slot and memory
        are available.  Returns the number admitted."""
        n = 0
        while self.queue and len(self.active) < self.backend.max_slots:
            req = self.queue[0]
            if req.arrival > now:
                break
            res = self._take_resident(req)
            if res is None:
                break  # head of line waits for memory
            self.queue.popleft()
            try:
                slot = self.backend.admit(res, req)
            except _lib.MHSError as e:
                # rejected at admission (e.g. not elliptic): retire at once
                req.status = e.code
                req.admitted = req.finished = now
                self._return_resident(res)
                self._retired.append(req)
                continue
            req.admitted = now
            self.active[slot] = (req, res)
            n += 1
        self.peak_active = max(self.peak_active, len(self.active))
        return n

    def tick(self, now_fn):
        """One batch step; retires finished requests.  Returns them."""
        done = []
        if self.active:
            self.backend.step()
            self.ticks += 1
            t = now_fn()
            for slot in list(self.active):
                fin, info2, info3 = self.backend.poll(slot)
                if not fin:
                    continue
                req, res = self.active.pop(slot)
                req.finished = t
                req.info2d, req.info3d = info2, info3
                req.status = info3.get("status") if info2.get("status", 0) == 0 else info2.get("status")
                if self.on_finish is not None:
                    self.on_finish(req, res)
                self.backend.release(slot)
                self._return_resident(res)
                done.append(req)
        return done

    def run(self, requests, clock=time.perf_counter, idle_sleep=0.0):
        """Serve `requests` (sorted by arrival, seconds from the start).
        Returns (finished requests, stats)."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        pending = deque(reqs)
        finished = []
        self._retired = finished
        t0 = clock()
        now = lambda: clock() - t0  # noqa: E731
        while pending or self.queue or self.active:
            t = now()
            while pending and pending[0].arrival <= t:
                self.submit(pending.popleft())
            self.admit_ready(t)
            if self.active:
                finished.extend(self.tick(now))
            elif pending and not self.queue:
                # nothing to do until the next arrival
                wait = pending[0].arrival - now()
                if wait > 0 and idle_sleep:
                    time.sleep(min(wait, idle_sleep))
            elif self.queue:
                # with nothing running every resident is idle and can be
                # evicted, so the head of the queue always fits
                raise RuntimeError("admission made no progress")
        wall = now()
        lat = [r.latency for r in finished if r.status == 0]
        stats = {
            "requests": len(finished),
            "ok": sum(1 for r in finished if r.status == 0),
            "wall_s": wall,
            "solves_per_s": (len(lat) / wall) if wall > 0 else None,
            "p50_ms": 1e3 * percentile(lat, 0.5) if lat else None,
            "p99_ms": 1e3 * percentile(lat, 0.99) if lat else None,
            "ticks": self.ticks,
            "peak_active": self.peak_active,
            "peak_queue": self.peak_queue,
            "peak_resident_bytes": self.peak_bytes,
        }
        return finished, stats


# ---------------------------------------------------------------------------
# device backend: plans, buffers and the mhs_batch_* entry points
# ---------------------------------------------------------------------------
class Batch:
    """Binding of mhs_batch (workspace from torch)."""

    def __init__(self, max_slots, device="cuda:0", hbm_budget=0):
        """hbm_budget: bytes the admitted requests may hold together
        (mhs_request_bytes each; 0 = no limit): admission past it raises
        MHSError with code MHS_ERR_BUDGET."""
        import torch

        self.torch = torch
        self.device = torch.device(device)
        L = _lib.lib()
        n = C.c_size_t()
        check(L.mhs_batch_workspace_bytes(max_slots, C.byref(n)))
        self.max_slots = max_slots
        with torch.cuda.device(self.device):
            self.ws = torch.empty(n.value, dtype=torch.uint8, device=self.device)
            h = C.c_void_p()
            check(L.mhs_batch_create(max_slots, int(hbm_budget), C.c_void_p(self.ws.data_ptr()), n.value,
                                     C.byref(h)))
        self.h = h

    def bytes_in_use(self):
        n = C.c_size_t()
        check(_lib.lib().mhs_batch_bytes_in_use(self.h, C.byref(n)))
        return n.value

    def close(self):
        if getattr(self, "h", None):
            _lib.lib().mhs_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def admit(self, plan, model, bz0, P, F, opts):
        from .solver import _ModelArgs, _ptr

        m = _ModelArgs.of(model)
        slot = C.c_int32()
        with self.torch.cuda.device(self.device):
            check(_lib.lib().mhs_batch_admit(self.h, plan.h, C.byref(m.c), _ptr(bz0), _ptr(P),
                                             *[_ptr(t) for t in F], C.byref(opts), C.byref(slot)))
        return slot.value

    def step(self):
        n = C.c_int32()
        with self.torch.cuda.device(self.device):
            s = C.c_void_p(self.torch.cuda.current_stream(self.device).cuda_stream)
            check(_lib.lib().mhs_batch_step(self.h, s, C.byref(n)))
        return n.value

    def poll(self, slot):
        done = C.c_int32()
        i2, i3 = _lib.Info(), _lib.Info()
        check(_lib.lib().mhs_batch_poll(self.h, slot, C.byref(done), C.byref(i2), C.byref(i3)))
        return bool(done.value), i2.as_dict(), i3.as_dict()

    def release(self, slot):
        check(_lib.lib().mhs_batch_release(self.h, slot))

    def profile(self, enable=True, classes=None):
        """Time merged launches of the given classes (names from
        PROF_NAMES; all by default); enable=False turns profiling off."""
        mask = 0
        if enable:
            for n in (_lib.PROF_NAMES if classes is None else classes):
                mask |= 1 << _lib.PROF_NAMES.index(n)
        check(_lib.lib().mhs_batch_profile_enable(self.h, mask))

    def profile_read(self, reset=False):
        """{class: (total_ms, launches, compulsory_bytes)} since the last reset."""
        out = {}
        for k, name in enumerate(_lib.PROF_NAMES):
            ms, n, b = C.c_double(), C.c_int64(), C.c_double()
            check(_lib.lib().mhs_batch_profile_read(self.h, k, C.byref(ms), C.byref(n), C.byref(b), 0))
            out[name] = (ms.value, n.value, b.value)
        if reset:
            check(_lib.lib().mhs_batch_profile_read(self.h, 0, None, None, None, 1))
        return out


@dataclass
class Resident:
    """A plan with its output buffers, resident on the device."""

    key: tuple
    plan: object
    bz0: object
    P: object
    F: tuple
    nbytes: int


class DeviceBackend:
    """Plans and buffers from torch, requests through a Batch.  hbm_budget
    is also handed to the batch (mhs_batch_create), which then refuses an
    admission past it; the Server's pool budget, which counts idle
    residents too, keeps admissions within it first."""

    def __init__(self, max_slots=32, device="cuda:0", precisions=PREC_FP64 | PREC_MIXED, hbm_budget=0):
        import torch

        self.torch = torch
        self.device = torch.device(device)
        self.precisions = precisions
        self.max_slots = max_slots
        self.batch = Batch(max_slots, device, hbm_budget)

    def footprint(self, key):
        from .solver import GridSpec, request_bytes

        (nx, ny, nz), (lx, ly, lz) = key
        return request_bytes(GridSpec(nx, ny, nz, lx, ly, lz), self.precisions)

    def acquire(self, key):
        from .solver import GridSpec, Plan

        torch = self.torch
        (nx, ny, nz), (lx, ly, lz) = key
        plan = Plan(GridSpec(nx, ny, nz, lx, ly, lz), self.precisions, device=self.device)
        shape = (nz, ny, nx)
        P = torch.zeros(shape, dtype=torch.float64, device=self.device)
        F = tuple(torch.empty(shape, dtype=torch.float64, device=self.device) for _ in range(5))
        bz0 = torch.empty((ny, nx), dtype=torch.float64, device=self.device)
        return Resident(key, plan, bz0, P, F, self.footprint(key))

    def free(self, res):
        res.plan.close()

    def admit(self, res, req):
        from .solver import make_opts

        torch = self.torch
        b = req.bz0
        if isinstance(b, np.ndarray):
            b = torch.from_numpy(np.ascontiguousarray(b, dtype=np.float64))
        res.bz0.copy_(b, non_blocking=False)
        opts = make_opts(req.precision, req.rtol, inner_cycles=req.inner_cycles)
        return self.batch.admit(res.plan, req.model, res.bz0, res.P, res.F, opts)

    def step(self):
        return self.batch.step()

    def poll(self, slot):
        return self.batch.poll(slot)

    def release(self, slot):
        self.batch.release(slot)

    def close(self):
        self.batch.close()
