"""Serving scheduler logic on the CPU with a fake pool (deterministic service times):
admission by footprint and slots, joining a running batch, retirement, latency percentiles."""
import numpy as np

from paper_1506_00907_amd.dgrtm import DgrtmError
from paper_1506_00907_amd.serving import Request, make_requests, serve_batched, serve_sequential


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-3)


class FakeShot:
    def __init__(self, total):
        self.left = total


class FakePool:
    """Each global step of a batched launch costs `cost` seconds of fake time regardless of
    how many shots share it (the point of batching small launches).  Device work completes as it
    is queued, so every event is ready at once."""

    def __init__(self, clock, total_steps=40, fp=100, cost=0.01, fail_steps=(), fail_new=()):
        self.clock, self.total, self.fp, self.cost = clock, total_steps, fp, cost
        self.running = []
        self.inflight = []
        self.launch_sizes = []
        self.n_step_calls = 0
        self.n_new_calls = 0
        self.fail_steps = set(fail_steps)    # step calls (0-based) that raise, as a failed library call
        self.fail_new = set(fail_new)        # new_shot calls (0-based) that raise
        self.marks = 0

    def footprint(self, req):
        return self.fp(req) if callable(self.fp) else self.fp

    def new_shot(self, req):
        i = self.n_new_calls
        self.n_new_calls += 1
        if i in self.fail_new:
            raise DgrtmError("dgrtm_shot_create failed (-5): injected")
        return FakeShot(self.total)

    def step(self, shots, n):
        i = self.n_step_calls
        self.n_step_calls += 1
        if i in self.fail_steps:
            raise DgrtmError("dgrtm_step_shots failed (-5): injected")
        self.launch_sizes.append(len(shots))
        for s in shots:
            s.left = max(0, s.left - n)
        self.clock.t += self.cost * n

    def mark(self):
        self.marks += 1
        return self.marks

    def ready(self, mark):
        return True

    def wait(self, mark):
        pass

    def sync(self):
        pass

    def is_done(self, s):
        return s.left == 0

    def collect_start(self, s):
        return self.mark(), (lambda: s.left)

    def run_alone(self, req):
        self.clock.t += self.cost * self.total
        return 0


def test_requests_are_seeded_and_poisson():
    a = make_requests(64, 2.0, ["m0", "m1", "m2"], 1.0, seed=7)
    b = make_requests(64, 2.0, ["m0", "m1", "m2"], 1.0, seed=7)
    assert [r.arrival for r in a] == [r.arrival for r in b]
    gaps = np.diff([0.0] + [r.arrival for r in a])
    assert abs(gaps.mean() - 0.5) < 0.2 and all(g >= 0 for g in gaps)
    assert {r.mesh for r in a} == {"m0", "m1", "m2"}
    assert all(10 <= r.f_peak <= 20 and 0.2 <= r.src_xy[0] <= 1.8 for r in a)


def test_batched_serving_admits_joins_and_retires():
    clk = FakeClock()
    pool = FakePool(clk, total_steps=40)
    reqs = [Request(i, "m", (1, 1), 15.0, arrival=0.05 * i, t_final=1.0) for i in range(6)]
    res = serve_batched({"m": pool}, reqs, hbm_budget=350, max_slots=8, steps_per_tick=4, clock=clk,
                        sleep=clk.sleep)
    assert all(r.done > r.arrival >= 0 for r in reqs)
    # memory admits at most 3 at a time (3 x 100 <= 350)
    assert max(pool.launch_sizes) == 3
    # later requests join while earlier ones run: more than one shot per launch happens
    assert sum(1 for n in pool.launch_sizes if n > 1) > 0
    s = res.summary()
    lat = sorted(r.latency for r in reqs)
    assert s["latency_p50_s"] == round(float(np.percentile(lat, 50)), 3)
    assert s["shots"] == 6


def test_batching_beats_sequential_on_fake_costs():
    reqs1 = [Request(i, "m", (1, 1), 15.0, arrival=0.0, t_final=1.0) for i in range(8)]
    reqs2 = [Request(i, "m", (1, 1), 15.0, arrival=0.0, t_final=1.0) for i in range(8)]
    c1, c2 = FakeClock(), FakeClock()
    rb = serve_batched({"m": FakePool(c1)}, reqs1, hbm_budget=10 ** 9, steps_per_tick=4, clock=c1, sleep=c1.sleep)
    rs = serve_sequential({"m": FakePool(c2)}, reqs2, clock=c2, sleep=c2.sleep)
    assert rb.makespan < rs.makespan / 4


def test_per_mesh_slot_limits():
    """A dict of slot limits: one shot at a time on the expensive mesh, several on the cheap one;
    a mesh missing from the dict runs one shot at a time."""
    clk = FakeClock()
    big, small, other = FakePool(clk, total_steps=40), FakePool(clk, total_steps=8), FakePool(clk, total_steps=8)
    reqs = [Request(i, ("big", "small", "other")[i % 3], (1, 1), 15.0, arrival=0.0, t_final=1.0)
            for i in range(12)]
    serve_batched({"big": big, "small": small, "other": other}, reqs, hbm_budget=10 ** 9,
                  max_slots={"big": 1, "small": 4}, steps_per_tick=4, clock=clk, sleep=clk.sleep)
    assert all(r.done > r.arrival for r in reqs)
    assert max(big.launch_sizes) == 1 and max(other.launch_sizes) == 1
    assert max(small.launch_sizes) == 4
    # shots on one mesh finish in arrival order when they run one at a time
    done_big = [r.done for r in reqs if r.mesh == "big"]
    assert done_big == sorted(done_big)


def test_oversized_request_is_rejected_and_the_rest_served():
    clk = FakeClock()
    pool = FakePool(clk, total_steps=20, fp=lambda r: 10 ** 6 if r.rid == 2 else 100)
    reqs = [Request(i, "m", (1, 1), 15.0, arrival=0.01 * i, t_final=1.0) for i in range(5)]
    res = serve_batched({"m": pool}, reqs, hbm_budget=1000, steps_per_tick=4, clock=clk, sleep=clk.sleep)
    assert [r.status for r in reqs] == ["done", "done", "rejected", "done", "done"]
    s = res.summary()
    assert s["shots"] == 4 and s["rejected"] == 1 and s["failed"] == 0


def test_failed_step_releases_the_slots_and_reruns_the_shots():
    clk = FakeClock()
    # the third launch fails: both shots in it give their slots and memory back and run again
    pool = FakePool(clk, total_steps=12, fail_steps={2})
    reqs = [Request(i, "m", (1, 1), 15.0, arrival=0.0, t_final=1.0) for i in range(3)]
    got = {}
    res = serve_batched({"m": pool}, reqs, hbm_budget=200, steps_per_tick=4, clock=clk, sleep=clk.sleep,
                        results=got)
    assert all(r.status == "done" for r in reqs)
    assert [r.retries for r in reqs] == [1, 1, 0]
    assert set(got) == {0, 1, 2} and all(v == 0 for v in got.values())
    assert res.summary()["retries"] == 2
    # memory is never over-committed: two shots of 100 bytes at most share a launch
    assert max(pool.launch_sizes) == 2


def test_failed_admission_is_retried_then_given_up():
    clk = FakeClock()
    # the first shot creation fails once: the request goes back to the front and runs
    pool = FakePool(clk, total_steps=8, fail_new={0})
    reqs = [Request(i, "m", (1, 1), 15.0, arrival=0.0, t_final=1.0) for i in range(2)]
    serve_batched({"m": pool}, reqs, hbm_budget=10 ** 6, steps_per_tick=4, clock=clk, sleep=clk.sleep)
    assert [r.status for r in reqs] == ["done", "done"] and [r.retries for r in reqs] == [1, 0]
    # creation fails three times in a row: with two retries allowed the request is given up
    clk = FakeClock()
    pool = FakePool(clk, total_steps=8, fail_new={0, 1, 2})
    reqs = [Request(0, "m", (1, 1), 15.0, arrival=0.0, t_final=1.0),
            Request(1, "m", (1, 1), 15.0, arrival=5.0, t_final=1.0)]
    res = serve_batched({"m": pool}, reqs, hbm_budget=10 ** 6, steps_per_tick=4, clock=clk, sleep=clk.sleep,
                        max_retries=2)
    assert reqs[0].status == "failed" and reqs[0].retries == 3
    assert reqs[1].status == "done"
    s = res.summary()
    assert s["failed"] == 1 and s["shots"] == 1


def test_a_pool_that_always_fails_ends_the_loop():
    clk = FakeClock()
    pool = FakePool(clk, total_steps=8, fail_steps=set(range(100)))
    reqs = [Request(i, "m", (1, 1), 15.0, arrival=0.0, t_final=1.0) for i in range(2)]
    res = serve_batched({"m": pool}, reqs, hbm_budget=10 ** 6, steps_per_tick=4, clock=clk, sleep=clk.sleep,
                        max_retries=1)
    assert all(r.status == "failed" for r in reqs)
    assert res.summary()["failed"] == 2
