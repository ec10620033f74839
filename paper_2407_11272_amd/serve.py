"""Continuous-batching request loop for voxelization and gradient requests.

Requests arrive over time (a mesh, a grid, and optionally a loss target when the
caller wants d(loss)/d(vertices)).  The loop

  * admits arrivals in order while a slot is free (a slot is held until the request's
    work is all launched) and the request's device footprint fits in the HBM budget (a
    request larger than the whole budget is rejected);
  * keeps each admitted request's mesh, grid outputs and gradient buffers resident
    on the device until it completes;
  * cuts every request into units of work: slices of its voxels for the forward pass
    and, for gradient requests, consecutive point ranges of the adjoint (each a whole
    number of rounds over the adjoint's splits, whose running sums stay in the request's
    workspace and are added in split order at the end);
  * every scheduler step spends a bounded amount of work.  Under the default
    earliest-deadline policy each request gets a deadline at admission (its arrival
    plus a slack proportional to its estimated service time, capped) and the step's
    budget goes to requests in deadline order, so short requests overtake long ones
    while a long request, once its deadline is the earliest, is not starved.  The cap
    bounds how long the longest requests can be overtaken: requests arriving more than
    the cap after one of them queue behind it, as they would in arrival order, which
    keeps the tail of the latency distribution from growing past plain FIFO's.  Under the share
    policies every request gets a slice in proportion to a weight (equal, or growing
    with its age).  All forward slices of a step run in ONE batched persistent launch;
    the step's losses and adjoint units follow it on a second stream, overlapping with
    the next step's forward;
  * completion times come from device events, so latency = completion - arrival is
    not delayed by host polling.

A voxel's winding number does not depend on which slice or batch computed it, and a
request's adjoint splits depend only on its own size and its ranges run in order, so
each result is bit-identical alone and in any mix.  The scheduling logic talks to the GPU only through
an executor object; tests drive it with a simulated executor on the CPU.
"""
from __future__ import annotations

import collections
import math
import time
from dataclasses import dataclass

import numpy as np

POINT_QUANTUM = 2048      # forward slices are multiples of this many voxels
STEP_PAIRS = 4.0e10       # point-face pairs of work per scheduler step (adjoint pairs weighted)
POLICY = "edf"            # "edf": earliest deadline first; "fair": equal shares; "age": shares grow with age
AGE_TAU = 0.25            # seconds of waiting that double a request's share under "age"
ADJOINT_COST = 2.8        # cost of one adjoint (point, face) pair in forward pairs
RATE_PAIRS = 1.4e12       # forward pairs per second, for the deadline estimate
DEADLINE_SLACK = 2.0      # deadline = arrival + min(DEADLINE_SLACK * estimated service, DEADLINE_CAP) + DEADLINE_BASE
DEADLINE_BASE = 0.05      # seconds
DEADLINE_CAP = 1.5        # seconds: past this, a long request is no longer overtaken by later arrivals


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
    dLdT: object = None

    @property
    def latency(self) -> float:
        return self.done - self.arrival


@dataclass
class _Active:
    req: ServeRequest
    res: ServeResult
    footprint: int
    adj_unit: int = 0           # adjoint: points per unit granule (one round over its splits)
    deadline: float = 0.0
    state: object = None        # executor-owned per-request state
    next_point: int = 0         # forward: next voxel to launch
    launched_all: bool = False  # forward: every slice launched
    adj_next: int = 0           # adjoint: next point to launch
    adj_ended: bool = False     # adjoint: the last unit (with the final sum) launched

    @property
    def all_launched(self) -> bool:
        return self.launched_all and (self.adj_ended or not self.req.wants_grad)


def _lib():
    from . import _lib as L
    return L.load()


def adjoint_unit(nF: int, P: int) -> int:
    """Points per adjoint unit granule of a served gradient request: one round of 256-point
    tiles over the adjoint's splits, so that every unit keeps all of its splits busy.
    Depends only on the request."""
    from . import _lib as L
    S = int(_lib().wn_backward_splits(max(0, nF), max(0, P)))
    if S < 1:
        raise ValueError("sizes out of range for the adjoint")
    return S * L.WN_BWD_TILE


def footprint_bytes(req: ServeRequest, slice_points: int) -> int:
    """Device bytes a request holds while admitted: mesh, outputs, gradient buffers,
    and its share of the batched workspace (face records and chunk partials)."""
    nV, nF, P = len(req.V), len(req.F), req.points
    b = 12 * nV + 12 * nF + 4 * P + (4 if req.occupancy == "sigmoid" else 1) * P
    chunks = max(1, -(-nF // 4096))
    b += 48 * nF + (4 * chunks * min(P, slice_points) if chunks > 1 else 0)
    if req.wants_grad:
        # target, dL/dW, dL/dV, the face-pair list (at most 2 int32 per face), and the
        # adjoint's own workspace (face or pair records, the splits' running corner sums,
        # corner sort buffers, vertex bounds)
        from . import _lib as L
        ws = _lib().wn_workspace_size(L.WN_OP_BACKWARD, nV, nF, P)
        if ws == 0:
            raise ValueError("sizes out of range for the adjoint")
        b += 8 * P + 12 * nV + 8 * nF + int(ws) + 512
    return int(b)


class Server:
    """The scheduler.  ``executor`` performs device work; ``clock`` returns seconds."""

    def __init__(self, executor, hbm_budget: int = 64 << 30, slots: int = 16,
                 quantum_pairs: float = STEP_PAIRS, max_inflight: int = 2, clock=time.perf_counter,
                 policy: str | None = None, adjoint_cost: float = ADJOINT_COST, rate_pairs: float = RATE_PAIRS,
                 deadline_slack: float = DEADLINE_SLACK, deadline_base: float = DEADLINE_BASE,
                 deadline_cap: float = DEADLINE_CAP, admit_ms: float = 4.0):
        self.ex = executor
        self.budget = int(hbm_budget)
        self.slots = int(slots)
        self.quantum = float(quantum_pairs)
        self.max_inflight = int(max_inflight)
        self.clock = clock
        self.policy = policy or POLICY
        if self.policy not in ("edf", "fair", "age"):
            raise ValueError("policy must be 'edf', 'fair' or 'age'")
        self.adj_cost = float(adjoint_cost)
        self.rate = float(rate_pairs)
        self.slack = float(deadline_slack)
        self.base = float(deadline_base)
        self.cap = float(deadline_cap)
        # host time per step for admissions (at least one is admitted): each uploads a mesh
        # (and a gradient request its target), so a burst of large arrivals is spread over
        # steps while the GPU works on those already admitted, and small ones still enter
        # many at a time
        self.admit_s = max(0.0, float(admit_ms)) / 1e3
        self.pending = collections.deque()   # arrived, not yet admitted
        self.active: list[_Active] = []
        self.in_use = 0
        self.results: dict[int, ServeResult] = {}
        self.steps = 0
        self.peak_in_use = 0
        self.peak_active = 0
        self.t0 = 0.0
        self.step_log = []   # (number of requests, forward voxels, adjoint points) per step

    # ---------------------------------------------------------------- intake
    def submit(self, req: ServeRequest) -> ServeResult:
        res = ServeResult(req.rid, req.arrival)
        self.results[req.rid] = res
        max_slice = self._max_slice_points(req)
        try:
            fp = footprint_bytes(req, max_slice)
        except ValueError as err:
            res.rejected = True
            res.error = str(err)
            return res
        if fp > self.budget:
            res.rejected = True
            res.error = f"footprint {fp} B exceeds the HBM budget {self.budget} B"
            return res
        a = _Active(req, res, fp)
        nF, P = len(req.F), req.points
        work = P * nF
        if req.wants_grad:
            a.adj_unit = adjoint_unit(nF, P)
            work += self.adj_cost * P * nF
        a.deadline = req.arrival + min(self.slack * work / self.rate, self.cap) + self.base
        prep = getattr(self.ex, "prepare", None)
        if prep is not None:
            prep(req)   # host-side work that can start before admission (strip order)
        self.pending.append(a)
        return res

    def _max_slice_points(self, req: ServeRequest) -> int:
        per = self.quantum / max(1, len(req.F))
        pts = max(POINT_QUANTUM, int(per) // POINT_QUANTUM * POINT_QUANTUM)
        return min(pts, req.points)

    def _working(self) -> int:
        """Admitted requests with work still to launch.  A request whose work is all
        launched gives its slot back at once (its memory stays counted until it
        completes), so the next one is admitted while its last steps run and the GPU
        does not drain between them."""
        return sum(1 for a in self.active if not a.all_launched)

    def _admit(self, now: float):
        t_start = self.clock()
        admitted = 0
        while self.pending and self._working() < self.slots:
            if admitted and self.clock() - t_start >= self.admit_s:
                break
            a = self.pending[0]
            if self.in_use + a.footprint > self.budget:
                break  # in order: wait for memory to free up
            self.pending.popleft()
            admitted += 1
            a.res.admitted = now
            a.state = self.ex.admit(a.req)
            self.active.append(a)
            self.in_use += a.footprint
            self.peak_in_use = max(self.peak_in_use, self.in_use)
            self.peak_active = max(self.peak_active, self._working())

    # ------------------------------------------------------------------ step
    def _plan(self):
        """Units of work for one step: forward slices [(a, p0, n)], requests whose
        forward completes [a], adjoint units [(a, p0, n, last)]."""
        todo = [a for a in self.active if not a.all_launched]
        if not todo:
            return [], [], []
        if self.policy == "edf":
            order = sorted(todo, key=lambda a: (a.deadline, a.req.rid))
            budgets = None
        else:
            order = todo
            if self.policy == "age":
                now = self.clock() - self.t0
                w = [1.0 + max(0.0, now - a.req.arrival) / AGE_TAU for a in todo]
            else:
                w = [1.0] * len(todo)
            wsum = sum(w)
            budgets = [self.quantum * wi_ / wsum for wi_ in w]
        left = self.quantum
        fwd, fdone, adj = [], [], []
        for i, a in enumerate(order):
            b = left if budgets is None else budgets[i]
            if budgets is None and b <= 0:
                break
            must = budgets is not None or i == 0   # the head (or every share) always progresses
            nF, P = max(1, len(a.req.F)), a.req.points
            spent = 0.0
            if not a.launched_all:
                pts = int(b / nF) // POINT_QUANTUM * POINT_QUANTUM
                if pts < POINT_QUANTUM and must:
                    pts = POINT_QUANTUM
                pts = min(pts, self._max_slice_points(a.req), P - a.next_point)
                if pts > 0:
                    fwd.append((a, a.next_point, pts))
                    a.next_point += pts
                    spent += pts * nF
                if a.next_point >= P:
                    a.launched_all = True
                    fdone.append(a)
            if a.launched_all and a.req.wants_grad and not a.adj_ended:
                unit = a.adj_unit * nF * self.adj_cost
                k = int((b - spent) // unit)
                if k < 1 and must and spent == 0:
                    k = 1
                if k > 0 or P == 0:
                    n = min(k * a.adj_unit, P - a.adj_next)
                    last = a.adj_next + n >= P
                    adj.append((a, a.adj_next, n, last))
                    a.adj_next += n
                    a.adj_ended = last
                    spent += n * nF * self.adj_cost
            if budgets is None:
                left -= spent
        return fwd, fdone, adj

    def step(self, intake=None) -> bool:
        """Admit, launch one step (a batched forward launch and adjoint units), retire
        completed requests.  Returns False when there is nothing left to do.

        When there is work to launch, the host first waits until fewer than
        ``max_inflight`` steps are queued on the device, then calls ``intake`` (which
        submits the requests that arrived meanwhile), admits and plans: the plan sees
        every arrival up to the moment it is launched, so a short request that arrives
        while a long one runs waits for at most the steps already queued."""
        if self.pending or any(not a.all_launched for a in self.active):
            self.ex.wait_inflight(self.max_inflight - 1)
        if intake is not None:
            intake()
        self._admit(self.clock() - self.t0)
        fwd, fdone, adj = self._plan()
        if fwd or fdone or adj:
            self.ex.launch_step([(a.state, a.req, p0, n) for a, p0, n in fwd],
                                [(a.state, a.req) for a in fdone],
                                [(a.state, a.req, p0, n, last) for a, p0, n, last in adj])
            self.steps += 1
            reqs = {id(a) for a, _, _ in fwd} | {id(a) for a, _, _, _ in adj}
            self.step_log.append((len(reqs), sum(n for _, _, n in fwd), sum(n for _, _, n, _ in adj)))
        self._retire()
        return bool(self.active or self.pending)

    def _retire(self):
        keep = []
        for a in self.active:
            t = self.ex.done_time(a.state) if a.all_launched else None
            if t is None:
                keep.append(a)
                continue
            a.res.done = t
            self.ex.collect(a.state, a.res)
            self.in_use -= a.footprint
        self.active = keep

    def drain(self, idle_sleep: float = 2e-4):
        while self.step():
            if all(a.all_launched for a in self.active):
                self.ex.idle(idle_sleep)

    # ------------------------------------------------------------ trace driver
    def run_trace(self, requests, idle_sleep: float = 2e-4, progress=None):
        """Replay ``requests`` (sorted by arrival, seconds from now) in real time.
        ``progress(submitted, total)``, if given, is called once per loop pass."""
        reqs = sorted(requests, key=lambda r: (r.arrival, r.rid))
        t0 = self.clock()
        self.t0 = t0
        self.ex.start(t0)
        i = 0

        def intake():
            nonlocal i
            now = self.clock() - t0
            while i < len(reqs) and reqs[i].arrival <= now:
                self.submit(reqs[i])
                i += 1

        while i < len(reqs) or self.active or self.pending:
            intake()
            busy = self.step(intake)
            if progress is not None:
                progress(i, len(reqs))
            if not busy and i < len(reqs):
                self.ex.idle(min(idle_sleep, max(0.0, reqs[i].arrival - (self.clock() - t0))))
            elif busy and all(a.all_launched for a in self.active):
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
    """Device side of the server: uploads, then per step one batched forward launch on
    the forward stream, and the loss of requests whose forward completed and adjoint
    units on a second stream after that forward; completion times from timing events."""

    def __init__(self, device="cuda", graph: bool = True, strips: bool = True, keep_dLdT: bool = False,
                 face_pairs: bool = True):
        import concurrent.futures
        import torch
        self.torch = torch
        self.strips = strips
        self.keep_dLdT = keep_dLdT   # also return per-corner dL/dT of gradient requests
        self.face_pairs = face_pairs  # gradient requests' adjoint with two faces per lane
        self.dev = torch.device(device)
        self.fwd = torch.cuda.Stream(self.dev)
        self.aux = torch.cuda.Stream(self.dev)   # losses and adjoint units (default priority)
        self.graph = graph
        self.inflight = collections.deque()
        self.ref = None
        self.t_ref = 0.0
        # strip orders are built on host threads from submission on (the builder is a C
        # call that releases the interpreter lock), off the loop that keeps the GPU fed
        self.pool = concurrent.futures.ThreadPoolExecutor(max_workers=2)
        self.strip_jobs = {}
        self.pair_jobs = {}

    def prepare(self, req: ServeRequest):
        import paper_2407_11272_amd as wn
        if self.strips and len(req.F):
            self.strip_jobs[req.rid] = self.pool.submit(wn.wn_build_strips, req.F, len(req.V))
        if self.face_pairs and req.wants_grad and len(req.F):
            self.pair_jobs[req.rid] = self.pool.submit(wn.wn_build_face_pairs, req.F, len(req.V))

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
                job = self.strip_jobs.pop(req.rid, None)
                rec = job.result() if job is not None else wn.wn_build_strips(req.F, len(req.V))
                Rh = torch.from_numpy(rec).pin_memory()
                R = Rh.to(self.dev, non_blocking=True)
                st["hold_strips"] = Rh
            job = wn.MeshJob(st["V"], st["F"], wn.Grid.of(req.grid), req.occupancy, req.tau, req.k, strips=R)
            job.prepare()
            st["job"] = job
            if req.wants_grad:
                T = torch.from_numpy(np.ascontiguousarray(req.target, dtype=np.float32)).pin_memory()
                st["target"] = T.to(self.dev, non_blocking=True)
                st["hold"] = (V, F, T)
                st["dLdW"] = torch.empty(req.points, dtype=torch.float32, device=self.dev)
                pairs = None
                if self.face_pairs and len(req.F):
                    pj = self.pair_jobs.pop(req.rid, None)
                    ph = pj.result() if pj is not None else wn.wn_build_face_pairs(req.F, len(req.V))
                    Ph = torch.from_numpy(ph).pin_memory()
                    pairs = Ph.to(self.dev, non_blocking=True)
                    st["hold_pairs"] = Ph
                st["adj"] = wn.SlicedBackward(st["V"], st["F"], grid=job.grid, pairs=pairs,
                                              vertex_sums=not self.keep_dLdT)
                if self.keep_dLdT:
                    st["dLdT"] = torch.empty((len(req.F), 3, 3), dtype=torch.float32, device=self.dev)
        return st

    def wait_inflight(self, keep: int):
        while len(self.inflight) > max(0, keep):
            self.inflight.popleft().synchronize()

    def _done_event(self, st, stream):
        ev = self.torch.cuda.Event(enable_timing=True)
        ev.record(stream)
        st["done"] = ev

    def launch_step(self, fwd, fdone, adj):
        """The step's batched forward on the forward stream; its losses and adjoint units
        on the second stream after that forward, so that they overlap with the next
        step's forward and each launch's last, partly filled round is filled by the
        other stream's work."""
        import paper_2407_11272_amd as wn
        torch = self.torch
        with torch.cuda.stream(self.fwd):
            if fwd:
                jobs = []
                for st, req, p0, n in fwd:
                    base = st["job"]
                    jobs.append(wn.MeshJob(base.V, base.F, base.grid, base.occupancy, base.tau, base.k, base.W,
                                           base.occ, point_begin=p0, point_count=n, strips=base.strips))
                wn.wn_voxelize_batched(jobs, graph=self.graph)
            for st, req in fdone:
                if not req.wants_grad:
                    self._done_event(st, self.fwd)
            fev = torch.cuda.Event()
            fev.record(self.fwd)
        grads = [(st, req) for st, req in fdone if req.wants_grad]
        if not grads and not adj:
            self.inflight.append(fev)
            return
        self.aux.wait_event(fev)
        with torch.cuda.stream(self.aux):
            for st, req in grads:
                W = st["job"].W.reshape(-1)
                st["loss"], _ = wn.wn_sigmoid_mse(W, st["target"], req.tau, req.k, dLdW=st["dLdW"])
                st["adj"].begin()
            for st, req, p0, n, last in adj:
                if n > 0:
                    st["adj"].points(p0, n, st["dLdW"])
                if last:
                    st["dLdV"] = st["adj"].end(dLdT=st.get("dLdT"))
                    self._done_event(st, self.aux)
            ev = torch.cuda.Event()
            ev.record(self.aux)
        self.inflight.append(ev)

    def done_time(self, st):
        ev = st.get("done")
        if ev is None or not ev.query():
            return None
        return self.t_ref + self.ref.elapsed_time(ev) / 1e3

    def collect(self, st, res: ServeResult):
        job = st["job"]
        res.W, res.occ = job.W, job.occ
        res.loss, res.dLdV, res.dLdT = st.get("loss"), st.get("dLdV"), st.get("dLdT")
        st.clear()

    def idle(self, seconds: float):
        if seconds > 0:
            time.sleep(seconds)

    def sync(self):
        self.torch.cuda.synchronize(self.dev)


def run_plain_fifo(requests, device="cuda", keep_results: bool = False, strips: bool = True, progress=None):
    """Baseline: the same trace, FIFO, one mesh per launch (the same forward kernel on
    the same strip order, then the loss and wn_backward for gradient requests), on one
    stream; completion from events.  ``progress(submitted, total)`` as in run_trace."""
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
        for n, r in enumerate(reqs):
            while time.perf_counter() - t0 < r.arrival:
                time.sleep(2e-4)
                if progress is not None:
                    progress(n, len(reqs))
            if progress is not None:
                progress(n + 1, len(reqs))
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
