"""CPU tests of the continuous-batching scheduler against a simulated executor.

The simulated executor runs on a virtual clock: a step takes (forward pairs +
adjoint cost x adjoint pairs) / rate seconds of device time.  No GPU and no winding
numbers are involved (the library is loaded only for its host-side size functions);
these tests check admission by footprint, slot limits, in-order admission, that the
forward slices and adjoint units of every request partition its points and come in the
right order, that steps mix several requests, that short requests overtake long ones
under every policy, and that a long request is not starved by a stream of short ones.
"""
import numpy as np
import pytest

from paper_2407_11272_amd.serve import (ADJOINT_COST, Server, ServeRequest, adjoint_unit, footprint_bytes,
                                        latency_stats)
from wn_inputs import Grid


class VClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class FakeExecutor:
    def __init__(self, clock: VClock, rate: float = 5e11, step_overhead: float = 1e-4,
                 adjoint_cost: float = ADJOINT_COST, upload_s: float = 0.0):
        self.clock = clock
        self.upload_s = upload_s
        self.rate = rate
        self.overhead = step_overhead
        self.adj_cost = adjoint_cost
        self.busy_until = 0.0
        self.inflight = []
        self.slices = {}
        self.adj = {}
        self.fwd_done_step = {}
        self.steps = []

    def start(self, t0):
        pass

    def admit(self, req):
        self.clock.t += self.upload_s   # host time of the upload
        self.slices[req.rid] = []
        self.adj[req.rid] = []
        return {"rid": req.rid}

    def wait_inflight(self, keep):
        while len(self.inflight) > max(0, keep):
            t = self.inflight.pop(0)
            self.clock.t = max(self.clock.t, t)

    def launch_step(self, fwd, fdone, adj):
        pairs = sum(n * len(req.F) for _, req, _, n in fwd)
        pairs += self.adj_cost * sum(n * len(req.F) for _, req, _, n, _ in adj)
        start = max(self.busy_until, self.clock.t)
        end = start + self.overhead + pairs / self.rate
        self.busy_until = end
        self.inflight.append(end)
        k = len(self.steps)
        self.steps.append([req.rid for _, req, _, _ in fwd] + [req.rid for _, req, _, _, _ in adj])
        for st, req, p0, n in fwd:
            self.slices[req.rid].append((p0, n, k))
        for st, req in fdone:
            self.fwd_done_step[req.rid] = k
            if not req.wants_grad:
                st["done"] = end
        for st, req, p0, n, last in adj:
            self.adj[req.rid].append((p0, n, last, k))
            if last:
                st["done"] = end

    def done_time(self, st):
        d = st.get("done")
        return d if d is not None and d <= self.clock.t else None

    def collect(self, st, res):
        pass

    def idle(self, seconds):
        self.clock.t += max(seconds, 1e-4)

    def sync(self):
        self.clock.t = max(self.clock.t, self.busy_until)


def _req(rid, faces, res, arrival, grad=False):
    V = np.zeros((faces // 2 + 2, 3), np.float32)
    F = np.zeros((faces, 3), np.int32)
    g = Grid.cube(res)
    target = np.zeros(g.size, np.float32) if grad else None
    return ServeRequest(rid, V, F, g, arrival, "sigmoid" if grad else "threshold", target)


def _run(reqs, upload_s=0.0, **kw):
    clock = VClock()
    ex = FakeExecutor(clock, upload_s=upload_s)
    srv = Server(ex, clock=clock, **kw)
    out = srv.run_trace(reqs, idle_sleep=1e-3)
    return srv, ex, out


@pytest.mark.parametrize("policy", ["edf", "fair", "age"])
def test_every_request_completes_and_units_partition_the_grid(policy):
    rng = np.random.default_rng(0)
    reqs = [_req(i, int(rng.integers(1000, 60000)), int(rng.choice([32, 64, 128])), float(i) * 0.01,
                 grad=bool(i % 3 == 0)) for i in range(40)]
    srv, ex, out = _run(reqs, slots=8, quantum_pairs=5e9, policy=policy)
    assert all(np.isfinite(r.done) and not r.rejected for r in out)
    for r in reqs:
        sl = sorted(ex.slices[r.rid])
        pos = 0
        for p0, n, _ in sl:
            assert p0 == pos and n > 0
            pos += n
        assert pos == r.points
        # slices are whole quanta of 2048 voxels except the last
        assert all(n % 2048 == 0 for _, n, _ in sl[:-1])
        last_fwd_step = max(k for _, _, k in sl)
        assert ex.fwd_done_step[r.rid] == last_fwd_step
        units = ex.adj[r.rid]
        if not r.wants_grad:
            assert units == []
            continue
        # adjoint units: consecutive whole rounds over the adjoint's splits, in order,
        # after the forward, the last one flagged
        unit = adjoint_unit(len(r.F), r.points)
        pos = 0
        for i, (p0, n, last, k) in enumerate(units):
            assert p0 == pos and n > 0 and k >= last_fwd_step
            assert last == (i == len(units) - 1)
            assert n % unit == 0 or p0 + n == r.points
            pos += n
        assert pos == r.points
    for r in out:
        assert r.done >= r.arrival and r.admitted >= r.arrival - 1e-12
    st = latency_stats(out)
    assert st["count"] == 40 and st["p99_ms"] >= st["p50_ms"] > 0


def test_adjoint_unit_depends_only_on_the_request():
    # one round of 256-point tiles over the adjoint's splits: many splits for few faces
    # (to fill the GPU alone), few for many faces (their running sums stay within 256 MiB)
    from paper_2407_11272_amd import _lib as L
    lib = L.load()
    assert adjoint_unit(5000, 64 ** 3) == adjoint_unit(5000, 64 ** 3)
    assert adjoint_unit(1000, 64 ** 3) == 256 * lib.wn_backward_splits(1000, 64 ** 3)
    big = lib.wn_backward_splits(100000, 256 ** 3)
    assert 1 <= big and big * 72 * 100000 <= 256 << 20
    assert lib.wn_backward_splits(1000, 64 ** 3) > big
    # the largest served gradient request's adjoint workspace stays well under 1 GB
    assert lib.wn_workspace_size(L.WN_OP_BACKWARD, 60000, 100000, 256 ** 3) < 400 << 20


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


def test_gradient_footprint_counts_the_adjoint_splits():
    from paper_2407_11272_amd import _lib as L
    r = _req(0, 100000, 256, 0.0, grad=True)
    splits = L.load().wn_backward_splits(len(r.F), r.points)
    assert footprint_bytes(r, 10 ** 9) > 72 * len(r.F) * splits
    assert footprint_bytes(r, 10 ** 9) > footprint_bytes(_req(0, 100000, 256, 0.0), 10 ** 9)


def test_slot_limit_and_in_order_admission():
    reqs = [_req(i, 5000, 64, 0.0) for i in range(12)]
    srv, ex, out = _run(reqs, slots=3, quantum_pairs=1e9)
    assert srv.peak_active == 3
    adm = [r.admitted for r in sorted(out, key=lambda r: r.rid)]
    assert adm == sorted(adm)
    assert all(np.isfinite(r.done) for r in out)


@pytest.mark.parametrize("admit_ms,upload_ms,per_step", [(4.0, 0.0, 12), (4.0, 3.0, 2), (4.0, 1.5, 3),
                                                           (0.0, 1.0, 1), (10.0, 20.0, 1)])
def test_admissions_per_step_follow_the_host_time_budget(admit_ms, upload_ms, per_step):
    """Each step admits arrivals in order until their uploads have used `admit_ms` of host
    time (at least one per step); every request still completes."""
    reqs = [_req(i, 5000, 64, 0.0) for i in range(12)]
    srv, ex, out = _run(reqs, upload_s=upload_ms / 1e3, slots=16, quantum_pairs=1e12, admit_ms=admit_ms)
    first_step = {}
    for k, rids in enumerate(ex.steps):
        for rid in rids:
            first_step.setdefault(rid, k)
    per = np.bincount(list(first_step.values()))
    assert per[0] == per_step and per.max() <= per_step
    order = [rid for rid, _ in sorted(first_step.items(), key=lambda kv: (kv[1], kv[0]))]
    assert order == sorted(order)
    assert all(np.isfinite(r.done) for r in out)


@pytest.mark.parametrize("policy", ["edf", "fair", "age"])
def test_steps_mix_requests_and_small_ones_overtake_large(policy):
    """A small request arriving during a large one shares the next steps with it and
    finishes long before it (with FIFO it would wait for the whole large one)."""
    large = _req(0, 100000, 256, 0.0)
    smalls = [_req(i, 2000, 64, 0.05 + 0.01 * i) for i in range(1, 4)]
    srv, ex, out = _run([large] + smalls, slots=8, quantum_pairs=1e10, policy=policy)
    res = {r.rid: r for r in out}
    assert any(len(set(s)) > 1 for s in ex.steps), "no step combined requests"
    service_large = large.points * len(large.F) / ex.rate
    for i in range(1, 4):
        assert res[i].latency < 0.2 * service_large
        assert res[i].done < res[0].done


def test_gradient_requests_finish_after_their_forward():
    reqs = [_req(0, 8000, 64, 0.0, grad=True), _req(1, 8000, 64, 0.0)]
    srv, ex, out = _run(reqs, slots=4, quantum_pairs=5e8)
    res = {r.rid: r for r in out}
    assert res[0].done > res[1].done
    assert ex.adj[0][0][3] >= ex.fwd_done_step[0]


def test_edf_large_gradient_request_is_not_starved():
    """A large gradient request under a steady stream of short requests: under the
    deadline policy it finishes within a few times its own service time, while every
    short request still finishes long before it would behind the large one."""
    big = _req(0, 50000, 128, 0.0, grad=True)
    service = big.points * len(big.F) * (1 + ADJOINT_COST) / 5e11
    smalls = [_req(i, 3000, 64, 0.004 * i) for i in range(1, int(3 * service / 0.004))]
    srv, ex, out = _run([big] + smalls, slots=16, quantum_pairs=2e9, policy="edf")
    res = {r.rid: r for r in out}
    assert res[0].latency < 3.0 * service
    lat_small = np.array([res[i].latency for i in range(1, len(smalls) + 1)])
    assert np.percentile(lat_small, 50) < 0.2 * service
    # the adjoint ran in several units, and short requests ran between the large one's
    # forward and its last adjoint unit
    assert len(ex.adj[0]) > 1
    k0, k1 = min(k for _, _, k in ex.slices[0]), ex.adj[0][-1][3]
    assert any(set(s) - {0} for s in ex.steps[k0:k1 + 1])


def test_edf_deadline_cap_stops_overtaking_of_a_long_request():
    """Under the deadline policy a long request's slack is capped: a short request that
    arrives early in its run overtakes it, one that arrives after the cap has passed
    queues behind it (as it would in arrival order)."""
    big = _req(0, 102400, 256, 0.0)   # about 3.4 s of device time at the simulated rate
    early = _req(1, 2000, 64, 0.2)
    late = _req(2, 2000, 64, 1.0)
    q = 48 * 2048 * 102400            # a step is exactly one slice of the long request
    srv, ex, out = _run([big, early, late], slots=8, quantum_pairs=q, policy="edf",
                        deadline_slack=2.0, deadline_cap=0.5, deadline_base=0.0)
    res = {r.rid: r for r in out}
    assert res[1].done < res[0].done
    assert res[2].done >= res[0].done   # (it may share the long one's last step)
    # without the cap both overtake
    srv, ex, out = _run([big, early, late], slots=8, quantum_pairs=q, policy="edf",
                        deadline_slack=2.0, deadline_cap=float("inf"), deadline_base=0.0)
    res = {r.rid: r for r in out}
    assert res[1].done < res[0].done and res[2].done < res[0].done


def test_plan_sees_arrivals_made_while_the_host_waited():
    """The host waits for a queued step before it plans the next one, and takes in the
    requests that arrived during that wait: a short request arriving while a long one
    runs is in the first step launched after its arrival."""
    big = _req(0, 100000, 256, 0.0)
    small = _req(1, 2000, 64, 0.105)
    srv, ex, out = _run([big, small], slots=8, quantum_pairs=1e10, policy="edf", max_inflight=2)
    step_time = 1e10 / ex.rate + ex.overhead
    first = min(k for _, _, k in ex.slices[1])
    # the step running when it arrived and the one queued behind it, then its own
    res = {r.rid: r for r in out}
    assert res[1].latency < 3 * step_time
    assert first <= int(0.105 / step_time) + 2


def test_idle_server_returns():
    srv, ex, out = _run([], slots=2)
    assert out == [] and srv.steps == 0


def test_unknown_policy_is_rejected():
    with pytest.raises(ValueError):
        Server(FakeExecutor(VClock()), policy="lifo")


@pytest.mark.parametrize("policy", ["edf", "fair", "age"])
def test_degenerate_requests_complete(policy):
    """No faces, an empty grid, and a one-voxel grid, with and without gradients."""
    def req(rid, faces, n, grad):
        V = np.zeros((max(3, faces // 2 + 2), 3), np.float32)
        F = np.zeros((faces, 3), np.int32)
        g = Grid((-0.5,) * 3, (0.5,) * 3, (n, n, n))
        return ServeRequest(rid, V, F, g, 0.001 * rid, "sigmoid" if grad else "threshold",
                            np.zeros(g.size, np.float32) if grad else None)
    reqs = [req(0, 0, 16, False), req(1, 0, 16, True), req(2, 500, 0, False), req(3, 500, 0, True),
            req(4, 500, 1, True), req(5, 2000, 32, True)]
    srv, ex, out = _run(reqs, slots=4, quantum_pairs=1e8, policy=policy)
    assert all(np.isfinite(r.done) and not r.rejected for r in out)
    for r in reqs:
        assert sum(n for _, n, _ in ex.slices[r.rid]) == r.points
        if r.wants_grad:
            units = ex.adj[r.rid]
            assert units and units[-1][2] and sum(n for _, n, _, _ in units) == r.points


def test_adjoint_unit_of_a_huge_grid():
    # a huge grid: the split count is bounded (at most 4096, at most 256 MiB of running
    # sums), so a unit granule stays a few thousand tiles at most
    P = 1024 ** 3
    u = adjoint_unit(100000, P)
    assert u % 256 == 0 and 256 <= u <= 4096 * 256
