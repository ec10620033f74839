"""Continuous-batching request loop for voxelization and gradient requests.

Requests arrive over time (a mesh, a grid, and optionally a loss target when the
caller wants d(loss)/d(vertices)).  The loop

  * admits arrivals in order while a slot is free and the request's device footprint
    fits in the HBM budget (a request larger than the whole budget is rejected);
  * keeps each admitted request's mesh, grid outputs and gradient buffers resident
    on the device until it completes;
  * every scheduler step gives each request still in its forward phase a fair share
    of a bounded amount of work (a slice of its voxels) and runs all slices in ONE
    batched persistent launch, so requests that arrive while others are on the GPU
    join the next step and their work overlaps;
  * when a request's last slice has been launched, its loss and adjoint are queued on
    a second stream (overlapping with later forward steps);
  * completion times come from device events, so latency = completion - arrival is
    not delayed by host polling.

A voxel's winding number does not depend on which slice or batch computed it, so each
result is bit-identical alone and in any mix.  The scheduling logic talks to the GPU
only through an executor object; tests drive it with a simulated executor on the CPU.
"""
from __future__ import annotations

import collections
import math
import time
from dataclasses import dataclass, field

import numpy as np

POINT_QUANTUM = 2048  # slice sizes are multiples of this many voxels
SHARE_POLICY = "age"  # "fair": equal shares; "age": shares grow with time since arrival
AGE_TAU = 0.25        # seconds of waiting that double a request's share under "age"


@dataclass
class ServeRequest:
    rid: int
    V: np.ndarray               # float [nV, 3]
    F: np.ndarray               # int [nF, 3]
    grid: object                # anything with lo, hi, n
    arrival: float = 0.0        # seconds after the start of the run
    occupancy: str = "threshold"
    target: np.ndarray | None = None   # float32 [P]: present for gradient requests
    tau: float = 0.5
    k: float = 50.0

    @property
    def points(self) -> int:
        return int(self.grid.n[0]) * int(self.grid.n[1]) * int(self.grid.n[2])

    @property
    def wants_grad(self) -> bool:
        return self.target is not None

    @property
    def pairs(self) -> int:
        return self.points * len(self.F) * (2 if self.wants_grad else 1)


@dataclass
class ServeResult:
    rid: int
    arrival: float
    admitted: float = math.nan
    done: float = math.nan
    rejected: bool = False
    error: str = ""
    W: object = None
    occ: object = None
    loss: object = None
    dLdV: object = None

    @property
    def latency(self) -> float:
        return self.done - self.arrival


@dataclass
class _Active:
    req: ServeRequest
    res: ServeResult
    footprint: int
    state: object = None        # executor-owned per-request state
    next_point: int = 0
    launched_all: bool = False


def footprint_bytes(req: ServeRequest, slice_points: int) -> int:
    """Device bytes a request holds while admitted: mesh, outputs, gradient buffers,
    and its share of the batched workspace (face records and chunk partials)."""
    nV, nF, P = len(req.V), len(req.F), req.points
    b = 12 * nV + 12 * nF + 4 * P + (4 if req.occupancy == "sigmoid" else 1) * P
    chunks = max(1, -(-nF // 4096))
    b += 48 * nF + (4 * chunks * min(P, slice_points) if chunks > 1 else 0)
    if req.wants_grad:
        # target, dL/dW, dL/dV, and the adjoint's workspace: face records, per-split corner
        # partials (about 8192 wave64s of faces), corner sums, sort buffers, vertex bounds
        splits = min(512, max(1, -(-8192 // max(1, -(-nF // 64)))))
        b += 8 * P + 12 * nV + 48 * nF + 36 * nF * splits + 36 * nF + 64 * nF + 8 * nV + (1 << 20)
    return int(b)


class Server:
    """The scheduler.  ``executor`` performs device work; ``clock`` returns seconds."""

    def __init__(self, executor, hbm_budget: int = 64 << 30, slots: int = 16,
                 quantum_pairs: float = 2.0e10, max_inflight: int = 2, clock=time.perf_counter):
        self.ex = executor
        self.budget = int(hbm_budget)
        self.slots = int(slots)
        self.quantum = float(quantum_pairs)
        self.max_inflight = int(max_inflight)
        self.clock = clock
        self.pending = collections.deque()   # arrived, not yet admitted
        self.active: list[_Active] = []
        self.in_use = 0
        self.results: dict[int, ServeResult] = {}
        self.steps = 0
        self.peak_in_use = 0
        self.peak_active = 0
        self.t0 = 0.0
        self.step_log = []   # (number of requests, voxels) per launched step

    # ---------------------------------------------------------------- intake
    def submit(self, req: ServeRequest) -> ServeResult:
        res = ServeResult(req.rid, req.arrival)
        self.results[req.rid] = res
        max_slice = self._max_slice_points(req)
        fp = footprint_bytes(req, max_slice)
        if fp > self.budget:
            res.rejected = True
            res.error = f"footprint {fp} B exceeds the HBM budget {self.budget} B"
            return res
        self.pending.append(_Active(req, res, fp))
        return res

    def _max_slice_points(self, req: ServeRequest) -> int:
        per = self.quantum / max(1, len(req.F))
        pts = max(POINT_QUANTUM, int(per) // POINT_QUANTUM * POINT_QUANTUM)
        return min(pts, req.points)

    def _admit(self, now: float):
        while self.pending and len(self.active) < self.slots:
            a = self.pending[0]
            if self.in_use + a.footprint > self.budget:
                break  # in order: wait for memory to free up
            self.pending.popleft()
            a.res.admitted = now
            a.state = self.ex.admit(a.req)
            self.active.append(a)
            self.in_use += a.footprint
            self.peak_in_use = max(self.peak_in_use, self.in_use)
            self.peak_active = max(self.peak_active, len(self.active))

    # ------------------------------------------------------------------ step
    def _plan_slices(self):
        fwd = [a for a in self.active if not a.launched_all]
        if not fwd:
            return []
        if SHARE_POLICY == "age":
            now = self.clock() - self.t0
            w = [1.0 + max(0.0, now - a.req.arrival) / AGE_TAU for a in fwd]
        else:
            w = [1.0] * len(fwd)
        wsum = sum(w)
        slices = []
        for a, wi_ in zip(fwd, w):
            share = self.quantum * wi_ / wsum
            nF = max(1, len(a.req.F))
            pts = max(POINT_QUANTUM, int(share / nF) // POINT_QUANTUM * POINT_QUANTUM)
            pts = min(pts, self._max_slice_points(a.req), a.req.points - a.next_point)
            slices.append((a, a.next_point, pts))
            a.next_point += pts
            if a.next_point >= a.req.points:
                a.launched_all = True
        return slices

    def step(self) -> bool:
        """Admit, launch one batched forward step, queue finished requests' gradients,
        retire completed requests.  Returns False when there is nothing left to do."""
        self._admit(self.clock() - self.t0)
        slices = self._plan_slices()
        if slices:
            self.ex.wait_inflight(self.max_inflight - 1)
            self.ex.launch_forward([(a.state, a.req, p0, n) for a, p0, n in slices])
            self.steps += 1
            self.step_log.append((len(slices), sum(n for _, _, n in slices)))
            for a, _, _ in slices:
                if a.launched_all:
                    self.ex.finish(a.state, a.req)
        self._retire()
        return bool(self.active or self.pending)

    def _retire(self):
        keep = []
        for a in self.active:
            t = self.ex.done_time(a.state) if a.launched_all else None
            if t is None:
                keep.append(a)
                continue
            a.res.done = t
            self.ex.collect(a.state, a.res)
            self.in_use -= a.footprint
        self.active = keep

    def drain(self, idle_sleep: float = 2e-4):
        while self.step():
            if not any(not a.launched_all for a in self.active):
                self.ex.idle(idle_sleep)

    # ------------------------------------------------------------ trace driver
    def run_trace(self, requests, idle_sleep: float = 2e-4):
        """Replay ``requests`` (sorted by arrival, seconds from now) in real time."""
        reqs = sorted(requests, key=lambda r: (r.arrival, r.rid))
        t0 = self.clock()
        self.t0 = t0
        self.ex.start(t0)
        i = 0
        while i < len(reqs) or self.active or self.pending:
            now = self.clock() - t0
            while i < len(reqs) and reqs[i].arrival <= now:
                self.submit(reqs[i])
                i += 1
            busy = self.step()
            if not busy and i < len(reqs):
                self.ex.idle(min(idle_sleep, max(0.0, reqs[i].arrival - (self.clock() - t0))))
            elif busy and not any(not a.launched_all for a in self.active):
                self.ex.idle(idle_sleep)
        self.ex.sync()
        return [self.results[r.rid] for r in reqs]


def latency_stats(results) -> dict:
    lat = np.array([r.latency for r in results if not r.rejected and np.isfinite(r.done)])
    if len(lat) == 0:
        return {"count": 0}
    return {
        "count": int(len(lat)),
        "p50_ms": float(np.percentile(lat, 50) * 1e3),
        "p99_ms": float(np.percentile(lat, 99) * 1e3),
        "mean_ms": float(lat.mean() * 1e3),
        "max_ms": float(lat.max() * 1e3),
        "rejected": int(sum(r.rejected for r in results)),
    }


# ============================================================== GPU executor

class GpuExecutor:
    """Device side of the server: uploads, batched forward steps on one stream, loss
    and adjoint on a second stream, completion times from timing events."""

    def __init__(self, device="cuda", graph: bool = True, strips: bool = True):
        import torch
        self.torch = torch
        self.strips = strips
        self.dev = torch.device(device)
        self.fwd = torch.cuda.Stream(self.dev)
        self.aux = torch.cuda.Stream(self.dev)
        self.graph = graph
        self.inflight = collections.deque()
        self.ref = None
        self.t_ref = 0.0

    def start(self, t0: float):
        torch = self.torch
        torch.cuda.synchronize(self.dev)
        self.ref = torch.cuda.Event(enable_timing=True)
        self.ref.record(self.fwd)
        self.ref.synchronize()
        self.t_ref = time.perf_counter() - t0

    def admit(self, req: ServeRequest):
        import paper_2407_11272_amd as wn
        torch = self.torch
        st = {}
        with torch.cuda.stream(self.fwd):
            V = torch.from_numpy(np.ascontiguousarray(req.V, dtype=np.float32)).pin_memory()
            F = torch.from_numpy(np.ascontiguousarray(req.F, dtype=np.int32)).pin_memory()
            st["V"] = V.to(self.dev, non_blocking=True)
            st["F"] = F.to(self.dev, non_blocking=True)
            st["hold"] = (V, F)
            R = None
            if self.strips and len(req.F):
                Rh = torch.from_numpy(wn.wn_build_strips(req.F, len(req.V))).pin_memory()
                R = Rh.to(self.dev, non_blocking=True)
                st["hold_strips"] = Rh
            job = wn.MeshJob(st["V"], st["F"], wn.Grid.of(req.grid), req.occupancy, req.tau, req.k, strips=R)
            job.prepare()
            st["job"] = job
            if req.wants_grad:
                T = torch.from_numpy(np.ascontiguousarray(req.target, dtype=np.float32)).pin_memory()
                st["target"] = T.to(self.dev, non_blocking=True)
                st["hold"] = (V, F, T)
        return st

    def wait_inflight(self, keep: int):
        while len(self.inflight) > max(0, keep):
            self.inflight.popleft().synchronize()

    def launch_forward(self, slices):
        import paper_2407_11272_amd as wn
        torch = self.torch
        jobs = []
        for st, req, p0, n in slices:
            base = st["job"]
            jobs.append(wn.MeshJob(base.V, base.F, base.grid, base.occupancy, base.tau, base.k, base.W, base.occ,
                                   point_begin=p0, point_count=n, strips=base.strips))
        with torch.cuda.stream(self.fwd):
            wn.wn_voxelize_batched(jobs, graph=self.graph)
            ev = torch.cuda.Event()
            ev.record(self.fwd)
        self.inflight.append(ev)

    def finish(self, st, req: ServeRequest):
        import paper_2407_11272_amd as wn
        torch = self.torch
        fwd_done = torch.cuda.Event(enable_timing=True)
        fwd_done.record(self.fwd)
        if not req.wants_grad:
            st["done"] = fwd_done
            return
        with torch.cuda.stream(self.aux):
            self.aux.wait_event(fwd_done)
            job = st["job"]
            W = job.W.reshape(-1)
            st["loss"], dLdW = wn.wn_sigmoid_mse(W, st["target"], req.tau, req.k)
            st["dLdV"] = wn.wn_backward(job.V, job.F, dLdW, grid=job.grid)
            done = torch.cuda.Event(enable_timing=True)
            done.record(self.aux)
        st["done"] = done

    def done_time(self, st):
        ev = st.get("done")
        if ev is None or not ev.query():
            return None
        return self.t_ref + self.ref.elapsed_time(ev) / 1e3

    def collect(self, st, res: ServeResult):
        job = st["job"]
        res.W, res.occ = job.W, job.occ
        res.loss, res.dLdV = st.get("loss"), st.get("dLdV")
        st.clear()

    def idle(self, seconds: float):
        if seconds > 0:
            time.sleep(seconds)

    def sync(self):
        self.torch.cuda.synchronize(self.dev)


def run_plain_fifo(requests, device="cuda", keep_results: bool = False, strips: bool = True):
    """Baseline: the same trace, FIFO, one mesh per launch (the same forward kernel on
    the same strip order, then the loss and wn_backward for gradient requests), on one
    stream; completion from events."""
    import torch
    import paper_2407_11272_amd as wn
    dev = torch.device(device)
    s = torch.cuda.Stream(dev)
    reqs = sorted(requests, key=lambda r: (r.arrival, r.rid))
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    ref = torch.cuda.Event(enable_timing=True)
    ref.record(s)
    ref.synchronize()
    t_ref = time.perf_counter() - t0
    out = []
    pend = []
    with torch.cuda.stream(s):
        for r in reqs:
            while time.perf_counter() - t0 < r.arrival:
                time.sleep(2e-4)
            V = torch.from_numpy(np.ascontiguousarray(r.V, dtype=np.float32)).pin_memory().to(dev, non_blocking=True)
            F = torch.from_numpy(np.ascontiguousarray(r.F, dtype=np.int32)).pin_memory().to(dev, non_blocking=True)
            if strips and len(r.F):
                R = torch.from_numpy(wn.wn_build_strips(r.F, len(r.V))).pin_memory().to(dev, non_blocking=True)
                W, occ = wn.wn_voxelize_strips(V, F, R, grid=wn.Grid.of(r.grid), occupancy=r.occupancy, tau=r.tau,
                                               k=r.k)
            else:
                W, occ = wn.wn_voxelize(V, F, grid=wn.Grid.of(r.grid), occupancy=r.occupancy, tau=r.tau, k=r.k)
            res = ServeResult(r.rid, r.arrival, admitted=r.arrival)
            if r.wants_grad:
                T = torch.from_numpy(np.ascontiguousarray(r.target, dtype=np.float32)).pin_memory().to(
                    dev, non_blocking=True)
                res.loss, dLdW = wn.wn_sigmoid_mse(W.reshape(-1), T, r.tau, r.k)
                res.dLdV = wn.wn_backward(V, F, dLdW, grid=wn.Grid.of(r.grid))
            ev = torch.cuda.Event(enable_timing=True)
            ev.record(s)
            if keep_results:
                res.W, res.occ = W, occ
            pend.append((res, ev))
            out.append(res)
            # bound the host's lead over the device, as the server does
            while len(pend) > 2:
                rr, e = pend.pop(0)
                e.synchronize()
                rr.done = t_ref + ref.elapsed_time(e) / 1e3
    torch.cuda.synchronize(dev)
    for rr, e in pend:
        rr.done = t_ref + ref.elapsed_time(e) / 1e3
    return out
