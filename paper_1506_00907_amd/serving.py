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
    """A bound mesh, its stream, and the shots running on it."""

    def __init__(self, name: str, n_levels: int = 3, n_rec: int = 100):
        import torch
        mm, rho, c, N = I.config_mesh(name)
        self.name = name
        self.stream = torch.cuda.Stream()          # default priority
        self.mesh = dgrtm.Mesh(N, mm.verts, mm.etov, bc_default=dgrtm.BC_TRANSPARENT)
        self.mesh.set_model(rho, c, n_levels).bind("cuda", stream=self.stream)
        self.box = mm.box
        self.n_rec = n_rec
        self.running: list[tuple[Request, dgrtm.Shot, int]] = []    # request, shot, footprint

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
        dgrtm.step_shots(shots, n_global)

    def sync(self):
        self.stream.synchronize()

    @staticmethod
    def is_done(shot) -> bool:
        return shot.state()[0] == dgrtm.PHASE_DONE

    @staticmethod
    def collect(shot):
        return shot.traces().cpu().numpy(), shot.image().cpu().numpy()

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
        lat = np.array([r.latency for r in self.requests])
        return {"shots": len(self.requests), "makespan_s": round(self.makespan, 3),
                "shots_per_hour": round(3600.0 * len(self.requests) / self.makespan, 2),
                "latency_p50_s": round(float(np.percentile(lat, 50)), 3),
                "latency_p99_s": round(float(np.percentile(lat, 99)), 3)}


def serve_batched(pools: dict, requests: list[Request], hbm_budget: int, max_slots=8,
                  steps_per_tick: int = 16, results: dict | None = None, clock=time.perf_counter,
                  sleep=time.sleep, log=None) -> ServeResult:
    """Continuous batching: admit as slots/memory free up; advance every running shot each tick.
    `max_slots`: shots running at once on one mesh (an int, or a dict mesh -> int; a mesh
    missing from the dict runs one shot at a time).
    `log(msg)`, if given, is called when a request completes."""
    pending = sorted(requests, key=lambda r: r.arrival)
    waiting: list[Request] = []
    used = 0
    t0 = clock()
    done_count = 0
    ticks = []
    while done_count < len(requests):
        now = clock() - t0
        while pending and pending[0].arrival <= now:
            waiting.append(pending.pop(0))
        # admission in arrival order, by footprint and free slots
        still = []
        for req in waiting:
            pool = pools[req.mesh]
            fp = pool.footprint(req)
            if fp > hbm_budget:
                raise ValueError(f"request {req.rid} needs {fp} bytes, more than the budget")
            limit = max_slots.get(req.mesh, 1) if isinstance(max_slots, dict) else max_slots
            if len(pool.running) < limit and used + fp <= hbm_budget:
                shot = pool.new_shot(req)
                used += fp
                req.admitted = clock() - t0
                pool.running.append((req, shot, fp))
            else:
                still.append(req)
        waiting = still
        busy = [p for p in pools.values() if p.running]
        if not busy:
            if pending:
                sleep(max(0.0, min(0.01, pending[0].arrival - now)))
            continue
        for p in busy:   # one tick of every mesh: their streams overlap on the device
            p.step([s for _, s, _ in p.running], steps_per_tick)
            ticks.append(len(p.running))
        for p in busy:
            p.sync()
            t_now = clock() - t0
            keep = []
            for req, shot, fp in p.running:
                if p.is_done(shot):
                    req.done = t_now
                    if results is not None:
                        results[req.rid] = p.collect(shot)
                    used -= fp
                    done_count += 1
                    if log is not None:
                        log(f"request {req.rid} ({req.mesh}) done at {t_now:.3f} s")
                else:
                    keep.append((req, shot, fp))
            p.running = keep
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
        if results is not None:
            results[req.rid] = out
        if log is not None:
            log(f"request {req.rid} ({req.mesh}) done at {req.done:.3f} s")
    return ServeResult(requests, clock() - t0)
