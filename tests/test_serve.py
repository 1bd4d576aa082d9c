"""Scheduling logic of the serving loop, on the CPU with a fake backend and a
virtual clock: admission by memory budget (FIFO), overlap of arrivals with
ticks, latency statistics and failure handling."""
import numpy as np
import pytest

from paper_2107_14790_amd.serve import Request, Server, latency_stats, poisson_arrivals


class G:
    def __init__(self, n, halo=0):
        self.n = n
        self.halo = halo
        self.origin = (0.0, 0.0, 0.0)
        self.h = 1.0


class VClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-6)


class FakeBackend:
    """Service time proportional to the voxels advanced; output = a
    deterministic function of the block and the iterations it received."""

    def __init__(self, clock, per_voxel_iter=1e-9, fail_on_tick=None):
        self.clock = clock
        self.c = per_voxel_iter
        self.active = 0
        self.max_active = 0
        self.fail_on_tick = fail_on_tick
        self.ticks = 0
        self.order = []

    def nbytes(self, grid):
        n = int(np.prod(grid.n))
        if n <= 0:
            raise ValueError("empty block")
        return 100 * n

    def prepare(self, req):
        self.active += 1
        self.max_active = max(self.max_active, self.active)
        self.order.append(req.rid)
        return {"rid": req.rid, "n": int(np.prod(req.grid.n)), "done": 0}

    def step(self, handles, k):
        self.ticks += 1
        if self.fail_on_tick is not None and self.ticks == self.fail_on_tick:
            raise RuntimeError("device error")
        for h in handles:
            h["done"] += k
        self.clock.t += self.c * k * sum(h["n"] for h in handles)

    def mark(self):
        return None  # the work is done when step returns

    def done(self, token):
        return True

    def finish(self, h):
        return (h["rid"], h["n"], h["done"])

    def release(self, h):
        self.active -= 1


def reqs(count, rate=100.0, iters=500, seed=0, edge=(32, 64)):
    t = poisson_arrivals(rate, count, seed)
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        e = int(rng.integers(edge[0], edge[1] + 1))
        out.append(Request(i, G((e, e, e), 2), float(t[i]), iters))
    return out


def run(requests, budget=10 ** 12, tick=50, **kw):
    clk = VClock()
    be = FakeBackend(clk, **kw)
    srv = Server(be, budget, tick_iters=tick, clock=clk, sleep=clk.sleep)
    return srv.run(requests), be, srv


def test_all_blocks_complete_with_their_iterations():
    rq = reqs(40)
    res, be, srv = run(rq)
    assert all(r.ok for r in res)
    for r, q in zip(res, sorted(rq, key=lambda x: x.arrival)):
        assert r.output == (q.rid, int(np.prod(q.grid.n)), 500)
        assert r.finished >= r.admitted >= r.arrival
    assert be.active == 0 and srv.used == 0
    st = latency_stats(res)
    assert st["n_ok"] == 40 and st["p99_s"] >= st["p50_s"] > 0


def test_budget_limits_resident_blocks_and_admission_is_fifo():
    rq = [Request(i, G((40, 40, 40)), 0.001 * i, 200) for i in range(12)]
    budget = 100 * 40 ** 3 * 3  # three blocks fit
    res, be, srv = run(rq, budget=budget)
    assert all(r.ok for r in res)
    assert be.max_active == 3 and srv.peak_used <= budget
    assert be.order == list(range(12))
    adm = [r.admitted for r in res]
    assert adm == sorted(adm)


def test_continuous_batching_overlaps_blocks():
    rq = reqs(30, rate=1e4)  # everything arrives at once
    res, be, srv = run(rq)
    assert srv.max_active_seen > 10
    assert srv.ticks <= 12  # 500 iterations in ticks of 50, blocks advancing together (late ones join)


def test_late_arrivals_join_running_batch():
    rq = [Request(0, G((64, 64, 64)), 0.0, 500), Request(1, G((32, 32, 32)), 1e-4, 500)]
    res, be, srv = run(rq, per_voxel_iter=1e-8)
    assert res[1].admitted < res[0].finished  # joined while block 0 was still running
    assert res[0].output[2] == 500 and res[1].output[2] == 500


def test_over_budget_and_invalid_blocks_fail_alone():
    rq = reqs(10)
    rq.append(Request(100, G((400, 400, 400)), 0.01, 500))   # over budget
    rq.append(Request(101, G((0, 10, 10)), 0.02, 500))       # empty block
    res, be, srv = run(rq, budget=100 * 80 ** 3 * 4)
    by = {r.rid: r for r in res}
    assert not by[100].ok and "budget" in by[100].error
    assert not by[101].ok and "invalid" in by[101].error
    assert all(by[i].ok for i in range(10))


def test_cancellation_of_pending_and_active_requests():
    rq = [Request(i, G((40, 40, 40)), 0.0, 500) for i in range(4)]
    rq[3].cancelled = True
    clk = VClock()
    be = FakeBackend(clk)
    srv = Server(be, 100 * 40 ** 3 * 2, tick_iters=50, clock=clk, sleep=clk.sleep)
    orig = be.step

    def step(handles, k):
        orig(handles, k)
        if be.ticks == 2:
            rq[0].cancelled = True  # cancel an active block mid-solve
    be.step = step
    res = srv.run(rq)
    by = {r.rid: r for r in res}
    assert not by[0].ok and by[0].error == "cancelled"
    assert not by[3].ok and by[3].error == "cancelled"
    assert by[1].ok and by[2].ok
    assert be.active == 0 and srv.used == 0


def test_failed_tick_fails_its_blocks_and_server_continues():
    rq = reqs(6, rate=1e4) + [Request(50, G((32, 32, 32)), 10.0, 100)]
    res, be, srv = run(rq, fail_on_tick=3)
    by = {r.rid: r for r in res}
    failed = [r for r in res if not r.ok]
    assert failed and all("step failed" in r.error for r in failed)
    assert by[50].ok and by[50].output[2] == 100
    assert srv.used == 0


class AsyncFakeBackend(FakeBackend):
    """A device that runs queued ticks one after another while the host goes
    on: step costs the host `host_cost` and queues the tick's service time on
    the device; a token is the device time at which the work queued so far
    ends."""

    def __init__(self, clock, host_cost=1e-3, **kw):
        super().__init__(clock, **kw)
        self.host_cost = host_cost
        self.dev_t = 0.0
        self.busy = 0.0
        self.first_start = None
        self.queued = []  # device end times of queued ticks

    def step(self, handles, k):
        self.ticks += 1
        self.clock.t += self.host_cost
        svc = self.c * k * sum(h["n"] for h in handles)
        start = max(self.dev_t, self.clock.t)
        if self.first_start is None:
            self.first_start = start
        self.dev_t = start + svc
        self.busy += svc
        for h in handles:
            h["done"] += k
        self.queued = [t for t in self.queued if t > self.clock.t] + [self.dev_t]
        self.max_queued = max(getattr(self, "max_queued", 0), len(self.queued))

    def mark(self):
        return self.dev_t

    def done(self, token):
        return self.clock.t >= token


@pytest.mark.parametrize("depth", [1, 2, 3])
def test_ticks_are_queued_ahead_of_the_device(depth):
    rq = [Request(i, G((48, 48, 48)), 0.0, 500) for i in range(8)]
    clk = VClock()
    be = AsyncFakeBackend(clk, host_cost=2e-3, per_voxel_iter=1e-9)
    srv = Server(be, 10 ** 12, tick_iters=50, clock=clk, sleep=clk.sleep, depth=depth, poll_s=1e-5)
    res = srv.run(rq)
    assert all(r.ok and r.output[2] == 500 for r in res)
    assert be.max_queued <= depth
    idle = (be.dev_t - be.first_start) - be.busy
    if depth == 1:
        # the device waits for the host between ticks
        assert idle >= 0.9 * (srv.ticks - 1) * be.host_cost
    else:
        # the next tick is already queued when one ends
        assert idle <= 1e-9
    # a block counts as done only once its last tick has ended on the device
    assert all(r.finished >= be.first_start + 500 * 48 ** 3 * 8 * 1e-9 - 1e-9 for r in res)
    assert be.active == 0 and srv.used == 0
