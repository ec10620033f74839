"""CPU tests of the continuous-batching scheduler against a simulated executor.

The simulated executor runs on a virtual clock: a forward step takes (pairs / rate)
seconds of device time, gradients run on a second virtual stream after the request's
forward finishes.  No GPU and no winding numbers are involved; these tests check
admission by footprint, slot limits, in-order admission, slice coverage, that steps
mix several requests, and that small requests are not stuck behind large ones.
"""
import numpy as np
import pytest

from paper_2407_11272_amd.serve import Server, ServeRequest, footprint_bytes, latency_stats
from wn_inputs import Grid


class VClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class FakeExecutor:
    def __init__(self, clock: VClock, rate: float = 5e11, step_overhead: float = 1e-4):
        self.clock = clock
        self.rate = rate
        self.overhead = step_overhead
        self.fwd_free = 0.0
        self.aux_free = 0.0
        self.inflight = []
        self.slices = {}
        self.steps = []

    def start(self, t0):
        pass

    def admit(self, req):
        self.slices[req.rid] = []
        return {"rid": req.rid}

    def wait_inflight(self, keep):
        while len(self.inflight) > max(0, keep):
            t = self.inflight.pop(0)
            self.clock.t = max(self.clock.t, t)

    def launch_forward(self, slices):
        pairs = sum(n * len(req.F) for _, req, _, n in slices)
        start = max(self.fwd_free, self.clock.t)
        self.fwd_free = start + self.overhead + pairs / self.rate
        self.inflight.append(self.fwd_free)
        self.steps.append([req.rid for _, req, _, _ in slices])
        for st, req, p0, n in slices:
            self.slices[req.rid].append((p0, n))

    def finish(self, st, req):
        done = self.fwd_free
        if req.wants_grad:
            start = max(self.aux_free, done)
            self.aux_free = start + req.points * len(req.F) / self.rate
            done = self.aux_free
        st["done"] = done

    def done_time(self, st):
        d = st.get("done")
        return d if d is not None and d <= self.clock.t else None

    def collect(self, st, res):
        pass

    def idle(self, seconds):
        self.clock.t += max(seconds, 1e-4)

    def sync(self):
        self.clock.t = max(self.clock.t, self.fwd_free, self.aux_free)


def _req(rid, faces, res, arrival, grad=False):
    V = np.zeros((faces // 2 + 2, 3), np.float32)
    F = np.zeros((faces, 3), np.int32)
    g = Grid.cube(res)
    target = np.zeros(g.size, np.float32) if grad else None
    return ServeRequest(rid, V, F, g, arrival, "sigmoid" if grad else "threshold", target)


def _run(reqs, **kw):
    clock = VClock()
    ex = FakeExecutor(clock)
    srv = Server(ex, clock=clock, **kw)
    out = srv.run_trace(reqs, idle_sleep=1e-3)
    return srv, ex, out


def test_every_request_completes_and_slices_partition_the_grid():
    rng = np.random.default_rng(0)
    reqs = [_req(i, int(rng.integers(1000, 60000)), int(rng.choice([32, 64, 128])), float(i) * 0.01,
                 grad=bool(i % 3 == 0)) for i in range(40)]
    srv, ex, out = _run(reqs, slots=8, quantum_pairs=5e9)
    assert all(np.isfinite(r.done) and not r.rejected for r in out)
    for r in reqs:
        sl = sorted(ex.slices[r.rid])
        pos = 0
        for p0, n in sl:
            assert p0 == pos and n > 0
            pos += n
        assert pos == r.points
        # slices are whole quanta of 2048 voxels except the last
        assert all(n % 2048 == 0 for _, n in sl[:-1])
    for r in out:
        assert r.done >= r.arrival and r.admitted >= r.arrival - 1e-12
    st = latency_stats(out)
    assert st["count"] == 40 and st["p99_ms"] >= st["p50_ms"] > 0


def test_footprint_admission_and_rejection():
    big = _req(0, 100000, 256, 0.0, grad=True)
    small = [_req(i, 2000, 64, 0.001 * i) for i in range(1, 6)]
    budget = footprint_bytes(small[0], 10 ** 9) * 2 + 1000
    srv, ex, out = _run([big] + small, hbm_budget=budget, slots=16)
    res = {r.rid: r for r in out}
    assert res[0].rejected and "budget" in res[0].error
    assert all(np.isfinite(res[i].done) for i in range(1, 6))
    assert srv.peak_in_use <= budget
    assert srv.peak_active <= 2  # only two small requests fit at once


def test_slot_limit_and_in_order_admission():
    reqs = [_req(i, 5000, 64, 0.0) for i in range(12)]
    srv, ex, out = _run(reqs, slots=3, quantum_pairs=1e9)
    assert srv.peak_active == 3
    adm = [r.admitted for r in sorted(out, key=lambda r: r.rid)]
    assert adm == sorted(adm)
    assert all(np.isfinite(r.done) for r in out)


def test_steps_mix_requests_and_small_ones_overtake_large():
    """A small request arriving during a large one shares the next steps with it and
    finishes long before it (with FIFO it would wait for the whole large one)."""
    large = _req(0, 100000, 256, 0.0)
    smalls = [_req(i, 2000, 64, 0.05 + 0.01 * i) for i in range(1, 4)]
    srv, ex, out = _run([large] + smalls, slots=8, quantum_pairs=1e10)
    res = {r.rid: r for r in out}
    assert any(len(set(s)) > 1 for s in ex.steps), "no step combined requests"
    service_large = large.points * len(large.F) / ex.rate
    for i in range(1, 4):
        assert res[i].latency < 0.2 * service_large
        assert res[i].done < res[0].done


def test_gradient_requests_finish_after_their_forward():
    reqs = [_req(0, 8000, 64, 0.0, grad=True), _req(1, 8000, 64, 0.0)]
    srv, ex, out = _run(reqs, slots=4)
    res = {r.rid: r for r in out}
    assert res[0].done > res[1].done


def test_idle_server_returns():
    srv, ex, out = _run([], slots=2)
    assert out == [] and srv.steps == 0
