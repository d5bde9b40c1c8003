"""Serving scheduler logic on the CPU with a fake pool (deterministic service times):
admission by footprint and slots, joining a running batch, retirement, latency percentiles."""
import numpy as np

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
    how many shots share it (the point of batching small launches)."""

    def __init__(self, clock, total_steps=40, fp=100, cost=0.01):
        self.clock, self.total, self.fp, self.cost = clock, total_steps, fp, cost
        self.running = []
        self.launch_sizes = []

    def footprint(self, req):
        return self.fp

    def new_shot(self, req):
        return FakeShot(self.total)

    def step(self, shots, n):
        self.launch_sizes.append(len(shots))
        for s in shots:
            s.left = max(0, s.left - n)
        self.clock.t += self.cost * n

    def sync(self):
        pass

    def is_done(self, s):
        return s.left == 0

    def collect(self, s):
        return s.left

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
