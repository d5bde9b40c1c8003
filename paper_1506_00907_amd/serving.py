"""Continuous-batching RTM shot server on one GPU.

Requests (a mesh, a source position, a Ricker frequency) arrive over time.  The server
keeps every admitted shot's wavefields, checkpoints and image resident in HBM, admits a
waiting request as soon as a slot and memory are free (admission by the shot's exact
workspace footprint and a per-mesh slot limit), and advances all running shots of a mesh
together: shots of one mesh at the same step mode share each kernel launch
(dgrtm_step_shots).  Each mesh has its own stream, so shots on different meshes overlap on
the device.  A request that arrives while
others run joins at the next tick, at a global-step boundary.

The baseline it is compared with is the plain one-shot-at-a-time FP32 solve: requests are
served in arrival order, each with a full forward + adjoint run, one after the other.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np

from . import dgrtm
from . import inputs as I


@dataclass
class Request:
    rid: int
    mesh: str
    src_xy: tuple
    f_peak: float
    arrival: float                 # seconds after the start of the stream
    t_final: float
    admitted: float = -1.0
    done: float = -1.0
    status: str = "queued"         # queued, done, rejected or failed
    retries: int = 0

    @property
    def latency(self) -> float:
        return self.done - self.arrival


def make_requests(n: int, rate: float, meshes: list[str], t_final: float, seed: int = 7,
                  burst: bool = False) -> list[Request]:
    """Seeded request stream: Poisson arrivals (or all at t = 0), mesh uniform, source (x, y)
    uniform in [0.2, 1.8]^2 km, Ricker peak frequency uniform in [10, 20] Hz."""
    rng = np.random.default_rng(seed + 1)
    arr = np.zeros(n) if burst else I.poisson_arrivals(n, rate, seed)
    out = []
    for i in range(n):
        out.append(Request(i, meshes[int(rng.integers(len(meshes)))],
                           (float(rng.uniform(0.2, 1.8)), float(rng.uniform(0.2, 1.8))),
                           float(rng.uniform(10.0, 20.0)), float(arr[i]), t_final))
    return out


class MeshSlotPool:
    """A bound mesh, its stream, and the shots running on it.

    Everything a pool queues runs on its own stream: with that stream current the binding adds no
    wait against any other stream, so the ticks of different meshes overlap on the device.  The
    host never waits for a pool inside the serving loop: it records an event after each tick
    (`mark`), polls events (`ready`), and copies results to pinned host memory asynchronously
    (`collect_start`)."""

    def __init__(self, name: str, n_levels: int = 3, n_rec: int = 100):
        import torch
        mm, rho, c, N = I.config_mesh(name)
        self.name = name
        self.stream = torch.cuda.Stream()          # default priority
        self.mesh = dgrtm.Mesh(N, mm.verts, mm.etov, bc_default=dgrtm.BC_TRANSPARENT)
        self.mesh.set_model(rho, c, n_levels).bind("cuda", stream=self.stream)
        self.box = mm.box
        self.n_rec = n_rec
        self.running: list = []            # Running entries (see serve_batched)
        self.inflight: list = []           # events of queued ticks, oldest first

    def spec(self, req: Request) -> dgrtm.ShotSpec:
        sh = I.rtm_shot(box=self.box, src_xy=req.src_xy, f_peak=req.f_peak, n_rec=self.n_rec, t_final=req.t_final)
        return dgrtm.ShotSpec(t_final=sh.t_final, src=sh.src, f_peak=sh.f_peak, t_peak=sh.t_peak, rec=sh.rec)

    def footprint(self, req: Request) -> int:
        import ctypes as C
        spec = self.spec(req)
        a = dgrtm.ShotArgs()
        a.struct_size = C.sizeof(dgrtm.ShotArgs)
        a.has_source = 1
        rec = np.ascontiguousarray(spec.rec, dtype=np.float64)
        a.n_rec = rec.shape[0]
        a.rec_xyz = rec.ctypes.data
        a.t_final = spec.t_final
        nb = C.c_size_t()
        dgrtm._check(dgrtm._lib.dgrtm_shot_bytes(self.mesh.h, C.byref(a), C.byref(nb)), "dgrtm_shot_bytes")
        return int(nb.value)

    # -- the operations the scheduler needs (a fake pool implements the same for CPU tests)
    def new_shot(self, req: Request):
        import torch
        with torch.cuda.stream(self.stream):
            shot = dgrtm.Shot(self.mesh, self.spec(req))
            shot.begin(None, dgrtm.IMAGE_CHARACTERISTIC, (0.0, 0.0, 1.0), 0)
        return shot

    def step(self, shots, n_global: int):
        import torch
        with torch.cuda.stream(self.stream):
            dgrtm.step_shots(shots, n_global)

    def mark(self):
        import torch
        ev = torch.cuda.Event()
        ev.record(self.stream)
        return ev

    @staticmethod
    def ready(mark) -> bool:
        return mark.query()

    @staticmethod
    def wait(mark):
        mark.synchronize()

    def sync(self):
        self.stream.synchronize()

    @staticmethod
    def is_done(shot) -> bool:
        return shot.state()[0] == dgrtm.PHASE_DONE

    def collect_start(self, shot):
        """Queue the copies of the shot's traces and image to pinned host memory on the pool's
        stream; returns (event, result function)."""
        import torch
        with torch.cuda.stream(self.stream):
            tr, img = shot.traces(), shot.image()
            tr_h = torch.empty(tr.shape, dtype=tr.dtype, pin_memory=True)
            img_h = torch.empty(img.shape, dtype=img.dtype, pin_memory=True)
            tr_h.copy_(tr, non_blocking=True)
            img_h.copy_(img, non_blocking=True)
            ev = self.mark()
        held = [tr, img]            # the device copies stay alive until the event has passed

        def result():
            held.clear()
            return tr_h.numpy(), img_h.numpy()
        return ev, result

    def collect(self, shot):
        ev, result = self.collect_start(shot)
        ev.synchronize()
        return result()

    def run_alone(self, req: Request):
        import torch
        with torch.cuda.stream(self.stream):
            shot = dgrtm.Shot(self.mesh, self.spec(req))
            tr = shot.forward()
            shot.adjoint(tr, dgrtm.IMAGE_CHARACTERISTIC, (0.0, 0.0, 1.0), 0)
            img = shot.image()
        self.sync()
        return tr.cpu().numpy(), img.cpu().numpy()


@dataclass
class ServeResult:
    requests: list
    makespan: float
    batched_launch_slots: list = field(default_factory=list)

    def summary(self) -> dict:
        done = [r for r in self.requests if r.status == "done"]
        lat = np.array([r.latency for r in done]) if done else np.zeros(1)
        return {"shots": len(done), "makespan_s": round(self.makespan, 3),
                "shots_per_hour": round(3600.0 * len(done) / max(self.makespan, 1e-9), 2),
                "latency_p50_s": round(float(np.percentile(lat, 50)), 3),
                "latency_p99_s": round(float(np.percentile(lat, 99)), 3),
                "rejected": sum(r.status == "rejected" for r in self.requests),
                "failed": sum(r.status == "failed" for r in self.requests),
                "retries": sum(r.retries for r in self.requests)}


@dataclass
class Running:
    req: Request
    shot: object
    fp: int
    finish: object = None          # event after the tick in which the shot's last step was queued
    collecting: object = None      # (event, result) of the result copies


def serve_batched(pools: dict, requests: list[Request], hbm_budget: int, max_slots=8,
                  steps_per_tick: int = 16, results: dict | None = None, clock=time.perf_counter,
                  sleep=time.sleep, log=None, queue_depth: int = 2, max_retries: int = 2) -> ServeResult:
    """Continuous batching: admit as slots/memory free up; advance every running shot each tick.

    `max_slots`: shots running at once on one mesh (an int, or a dict mesh -> int; a mesh missing
    from the dict runs one shot at a time).  Each pool keeps up to `queue_depth` ticks of
    `steps_per_tick` global steps queued on its stream; a shot retires once the event after its
    last step has passed and its results have reached the host.

    A request whose footprint exceeds `hbm_budget` is marked "rejected" and the others are
    served.  When a library call fails (DgrtmError) while admitting or advancing shots, the
    shots concerned release their slots and memory and their requests go back to the front of
    the queue, to be run again from the start (a shot's pipeline state after a failed call is
    not trusted); a request that fails more than `max_retries` times is marked "failed".
    `log(msg)`, if given, is called when a request completes, is rejected or fails."""
    pending = sorted(requests, key=lambda r: r.arrival)
    waiting: list[Request] = []
    used = 0
    t0 = clock()
    finished = 0
    ticks = []
    order = []                     # (pool, event) of queued ticks, in issue order

    def say(msg):
        if log is not None:
            log(msg)

    def release(p, entries, err):
        """Free the entries' slots and memory; return the requests to run again."""
        nonlocal used, finished
        back = []
        for e in entries:
            if e in p.running:
                p.running.remove(e)
            used -= e.fp
            e.req.retries += 1
            if e.req.retries > max_retries:
                e.req.status = "failed"
                e.req.done = clock() - t0
                finished += 1
                say(f"request {e.req.rid} ({e.req.mesh}) failed: {err}")
            else:
                say(f"request {e.req.rid} ({e.req.mesh}) re-queued after: {err}")
                back.append(e.req)
        return back

    while finished < len(requests):
        now = clock() - t0
        while pending and pending[0].arrival <= now:
            waiting.append(pending.pop(0))
        # admission in arrival order, by footprint and free slots
        still, again = [], []
        progressed = False
        for req in waiting:
            pool = pools[req.mesh]
            fp = pool.footprint(req)
            if fp > hbm_budget:
                req.status = "rejected"
                req.done = clock() - t0
                finished += 1
                progressed = True
                say(f"request {req.rid} ({req.mesh}) rejected: needs {fp} bytes, the budget is {hbm_budget}")
                continue
            limit = max_slots.get(req.mesh, 1) if isinstance(max_slots, dict) else max_slots
            if len(pool.running) < limit and used + fp <= hbm_budget:
                used += fp
                progressed = True
                try:
                    shot = pool.new_shot(req)
                except dgrtm.DgrtmError as err:
                    again += release(pool, [Running(req, None, fp)], err)
                    continue
                req.admitted = clock() - t0
                pool.running.append(Running(req, shot, fp))
            else:
                still.append(req)
        waiting = again + still
        # queue ticks: every pool keeps up to queue_depth ticks in flight
        for p in pools.values():
            while len(p.inflight) < queue_depth:
                live = [e for e in p.running if e.finish is None]
                if not live:
                    break
                try:
                    p.step([e.shot for e in live], steps_per_tick)
                except dgrtm.DgrtmError as err:
                    waiting[:0] = release(p, live, err)
                    progressed = True
                    break
                ev = p.mark()
                p.inflight.append(ev)
                order.append((p, ev))
                ticks.append(len(live))
                for e in live:
                    if p.is_done(e.shot):
                        e.finish = ev
                progressed = True
        # retire: ticks that have passed, then results that have reached the host
        for p in pools.values():
            while p.inflight and p.ready(p.inflight[0]):
                p.inflight.pop(0)
            for e in list(p.running):
                if e.finish is not None and e.collecting is None and e.finish not in p.inflight:
                    e.collecting = p.collect_start(e.shot)
                    progressed = True
                if e.collecting is not None and p.ready(e.collecting[0]):
                    out = e.collecting[1]()
                    e.req.done = clock() - t0
                    e.req.status = "done"
                    if results is not None:
                        results[e.req.rid] = out
                    p.running.remove(e)
                    used -= e.fp
                    finished += 1
                    progressed = True
                    say(f"request {e.req.rid} ({e.req.mesh}) done at {e.req.done:.3f} s")
        order = [(p, ev) for p, ev in order if ev in p.inflight]
        if progressed:
            continue
        # nothing to do until the device or the clock moves on
        collecting = [(p, e) for p in pools.values() for e in p.running if e.collecting is not None]
        if order:
            order[0][0].wait(order[0][1])
        elif collecting:
            collecting[0][0].wait(collecting[0][1].collecting[0])
        elif pending:
            sleep(max(0.0, min(0.01, pending[0].arrival - (clock() - t0))))
        elif waiting:
            raise RuntimeError(f"requests {[r.rid for r in waiting]} can never be admitted (slot limits)")
    return ServeResult(requests, clock() - t0, ticks)


def serve_sequential(pools: dict, requests: list[Request], results: dict | None = None, clock=time.perf_counter,
                     sleep=time.sleep, log=None) -> ServeResult:
    """Baseline: one shot at a time in arrival order, full forward + adjoint each."""
    t0 = clock()
    for req in sorted(requests, key=lambda r: r.arrival):
        now = clock() - t0
        if req.arrival > now:
            sleep(req.arrival - now)
        pool = pools[req.mesh]
        req.admitted = clock() - t0
        out = pool.run_alone(req)
        req.done = clock() - t0
        req.status = "done"
        if results is not None:
            results[req.rid] = out
        if log is not None:
            log(f"request {req.rid} ({req.mesh}) done at {req.done:.3f} s")
    return ServeResult(requests, clock() - t0)
