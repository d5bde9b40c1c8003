"""Benchmark: one RTM shot per step on one MI355X, FP32 path.

A step is one pass of the whole hot path over one shot: forward source run from rest
(multi-rate AB3, source checkpoints in HBM, receiver recording), then the backward pass
(segment-wise recompute of the source wavefield from the checkpoints, backward receiver run
with the recorded traces re-injected, characteristic imaging condition accumulated in FP64),
then the image export.  Inputs (mesh, model, shot geometry) are seeded synthetic stand-ins
for the paper's workloads and are resident in HBM before the timed region starts.

Workload "big_4m" (the default: the largest shot that fits one GPU): 10 x 10 x 4 km box,
4 147 200 jittered tetrahedra, the top 0.5 km refined 4x, N = 4, smooth random velocity
1.5-4.5 km/s (seeded Gaussian-filtered noise) with a 4.5 km/s ellipsoidal inclusion, 4 LTS
levels, 15 Hz Ricker source 8 m deep at the centre, 256 x 256 receivers 10 m deep, transparent
boundaries, t_final = 0.04 s by default (checkpointing holds the source wavefield in HBM, which
bounds the simulated time of a shot on this mesh).

Workload "rtm_200k" (also reported, as a secondary block, after the main one): 2 x 2 x 1 km
box, dipping two-layer model 1.5 / 3.0 km/s, 201 600 jittered tetrahedra refined 2x at the
interface, N = 4, 3 levels, 100 x 100 receivers, t_final = 1 s for its own run.

After the timed shots: the split-BF16 form against FP32 on a shorter shot of the same mesh, the
rtm_200k block, a serving section (a seeded Poisson stream over three meshes, continuous
batching against one shot at a time) and the FP64 oracle timed on the host.

Prints one JSON line (rank 0, N = 1 only).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def bytes_per_element_step(Np: int, Nfp: int, mode: int) -> int:
    """Algorithmic HBM bytes of one element-step of the fused step kernel (FP32 state).

    plain: q read + write (8 Np), rhs ring 2 reads + 1 write (12 Np), neighbour traces in and
    own traces out (2 x 2 x 4 Nfp), geometry/material (20), neighbour ids and codes (8), flags (1).
    record: + q-_S and r-_S written (2 Np).  image: + q-_S and 3 r-_S read (4 Np) and the FP64
    image read and written (4 Np in float units).  replay (mode 4, the source field backward with
    recorded boundary traces): as record; a boundary face reads its recorded run where an interior
    face reads its neighbour's.
    """
    words = 20 * Np + 16 * Nfp + 29
    if mode in (1, 4):
        words += 2 * Np
    if mode == 2:
        words += 8 * Np
    return 4 * words


def flops_per_element_step(Np: int, Nfp: int) -> int:
    # volume 6 Np^2 MACs, surface 2 x 4 Nfp Np MACs (LIFT on the p and the scalar v penalty)
    return 2 * (6 * Np * Np + 8 * Nfp * Np)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_1506_00907_amd", "csrc", "kernels.hip"), "rb") as f:
        h.update(f.read())
    return h.hexdigest()[:16]


def load_traffic(workload: str, mode_name: str, profiles_dir: str = os.path.join(ROOT, "profiles")):
    """HBM bytes per launch from committed rocprofv3 PMC runs, if taken on the current kernel."""
    p = os.path.join(profiles_dir, f"step_kernel_{workload}_traffic.json")
    if not os.path.exists(p):
        return None
    d = json.load(open(p))
    if d.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    m = d.get("modes", {}).get(mode_name)
    return None if m is None else round(m["bytes_per_launch"], 1)


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def column_elements(mesh_in, width_cells: int = 8) -> "np.ndarray":
    """Elements of a vertical column of width_cells x width_cells cells at the centre of a Kuhn box
    (all layers, so that every multi-rate level of the mesh is in it); element id = 6 cell + perm,
    cells x fastest, then y, then z."""
    import numpy as np
    nx, ny, nz = mesh_in.meta["nx"], mesh_in.meta["ny"], mesh_in.meta["nz"]
    i0, j0 = (nx - width_cells) // 2, (ny - width_cells) // 2
    ii, jj, mm_ = np.meshgrid(np.arange(i0, i0 + width_cells), np.arange(j0, j0 + width_cells), np.arange(nz),
                              indexing="ij")
    cells = (ii + nx * (jj + ny * mm_)).ravel()
    return np.sort((6 * cells[:, None] + np.arange(6)[None]).ravel())


def cpu_baseline(mesh_in, rho, c, N, n_levels, seconds_target=15.0, max_elements=40000):
    """The FP64 oracle's multi-rate forward stepping, timed on a bounded sample of the workload.

    Meshes larger than max_elements are sampled by a vertical column of cells through the whole
    depth (the oracle's set-up of the whole 4.1M-element mesh alone would take the better part of
    an hour): the oracle runs on that sub-mesh, with levels assigned on it by the same rule."""
    import numpy as np

    from oracle.dg import Operator
    from oracle.mesh import BC_TRANSPARENT, OMesh, local_dt, lts_levels
    from oracle.refelem import get_ref
    from oracle.timestep import MRAB

    verts, etov, rho_s, c_s, what = mesh_in.verts, mesh_in.etov, rho, c, f"the same {mesh_in.K}-element mesh"
    if mesh_in.K > max_elements:
        w = 8
        while True:
            el = column_elements(mesh_in, w)
            if el.size <= max_elements or w == 1:
                break
            w -= 1
        used = np.unique(etov[el])
        remap = np.full(verts.shape[0], -1, dtype=np.int64)
        remap[used] = np.arange(used.size)
        verts, etov, rho_s, c_s = verts[used], remap[etov[el]], rho[el], c[el]
        what = (f"a {w} x {w}-cell column through the whole depth of the {mesh_in.K}-element mesh "
                f"({el.size} elements)")
    om = OMesh(get_ref(N), verts, etov, bc_default=BC_TRANSPARENT)
    op = Operator(om, rho_s, c_s)
    lev, L, dtl = lts_levels(local_dt(om.verts, om.etov, c_s, N), om.EToE, n_levels)
    rng = np.random.default_rng(0)
    st = MRAB(op, lev, L, dtl)
    st.set_state(rng.standard_normal((om.K, 4, op.ref.Np)) * 1e-3)
    stride = 2 ** (L - lev)
    t0 = time.perf_counter()
    esteps = 0
    while time.perf_counter() - t0 < seconds_target:
        n = st.n
        esteps += int(np.count_nonzero(n % stride == 0))
        st.local_step()
    dt = time.perf_counter() - t0
    return {"value": esteps * 4 * op.ref.Np / dt / 1e9, "unit": "GDOF-steps/s", "cores": _threads(),
            "kind": "oracle", "cpu_model": _cpu_model(),
            "sample": f"{st.n} local steps ({esteps} element-steps, {L} levels "
                      f"{[int(x) for x in np.bincount(lev, minlength=L + 1)[1:]]}) of the FP64 multi-rate "
                      f"forward run on {what}, {dt:.1f} s"}


def serving_bench(n_requests=12, t_final=0.05, meshes=("srv_50k", "srv_200k", "srv_800k"), seed=7,
                  hbm_budget=200 * 2 ** 30):
    """Continuous batching vs the one-shot-at-a-time FP32 solve on the same seeded Poisson stream."""
    import copy
    import numpy as np
    from paper_1506_00907_amd import serving as S
    pools = {}
    for m in meshes:
        ts = time.perf_counter()
        pools[m] = S.MeshSlotPool(m)
        log(f"serving: mesh {m} bound in {time.perf_counter() - ts:.1f} s")
    # capacity of the sequential solver: one warm-up shot per mesh
    svc = []
    for m in meshes:
        req = S.Request(-1, m, (1.0, 1.0), 15.0, 0.0, t_final)
        pools[m].run_alone(req)                      # compile / first-touch
        t0 = time.perf_counter()
        pools[m].run_alone(req)
        svc.append(time.perf_counter() - t0)
        log(f"serving: one {m} shot alone takes {svc[-1]:.3f} s")
    capacity = 1.0 / float(np.mean(svc))
    rate = 1.2 * capacity
    # shots of the most expensive mesh(es) run one at a time per mesh: their launches fill the GPU
    # on their own, and a second long shot in the same launches would only stretch both; cheaper
    # meshes batch up to 8 shots per launch
    slots = {m: (1 if t >= 0.5 * max(svc) else 8) for m, t in zip(meshes, svc)}
    reqs = S.make_requests(n_requests, rate, list(meshes), t_final, seed=seed)
    seq_res, bat_res = {}, {}
    rs = S.serve_sequential(pools, copy.deepcopy(reqs), results=seq_res, log=log)
    log(f"serving: one-at-a-time done in {rs.makespan:.2f} s")
    rb = S.serve_batched(pools, copy.deepcopy(reqs), hbm_budget, max_slots=slots, results=bat_res, log=log)
    log(f"serving: continuous batching done in {rb.makespan:.2f} s")
    worst_img, worst_tr = 0.0, 0.0
    for rid in seq_res:
        (ta, ia), (tb, ib) = seq_res[rid], bat_res[rid]
        worst_tr = max(worst_tr, float(np.abs(ta - tb).max() / max(np.abs(ta).max(), 1e-30)))
        worst_img = max(worst_img, float(np.linalg.norm(ia - ib) / max(np.linalg.norm(ia), 1e-30)))
    return {"requests": n_requests, "t_final_s": t_final, "meshes": list(meshes),
            "arrival_rate_per_s": round(rate, 4), "sequential_capacity_per_s": round(capacity, 4),
            "shot_alone_s": {m: round(t, 3) for m, t in zip(meshes, svc)}, "slots_per_mesh": slots,
            "batched": rb.summary(), "sequential": rs.summary(),
            "mix_vs_alone_max_rel_image_diff": worst_img, "mix_vs_alone_max_rel_trace_diff": worst_tr}


# LTS levels (at most), receiver grid (n x n), source position, default simulated time and
# default simulated time of the split-BF16 comparison shot of each benchmark shot
SHOT_SHAPES = {
    # the 200k-tet two-layer shot
    "default": {"levels": 3, "n_rec": 100, "t_final": 1.0, "bf16_t_final": 0.25},
    # the ~4M-tet 10 x 10 x 4 km shot: 190 global steps; its checkpointed workspace is ~170 GB
    "big_4m": {"levels": 4, "n_rec": 256, "src_xy": (5.0, 5.0), "t_final": 0.04, "bf16_t_final": 0.01},
}


def precision_compare(dgrtm, I, mesh, box, src_xy, n_rec, t_final, esteps_global, dof):
    """One shot of the same workload (shorter simulated time) in both forms: throughput of each and
    the split-BF16 result's relative L2 difference from the FP32 result on the same shot."""
    import numpy as np
    import torch
    spec = I.rtm_shot(box=box, src_xy=src_xy, n_rec=n_rec, t_final=t_final)
    res = {}
    for prec in (dgrtm.FP32, dgrtm.SPLIT_BF16):
        sh = dgrtm.Shot(mesh, dgrtm.ShotSpec(t_final=spec.t_final, src=spec.src, f_peak=spec.f_peak,
                                             t_peak=spec.t_peak, rec=spec.rec, precision=prec))
        torch.cuda.synchronize()
        ts = time.perf_counter()
        tr = sh.forward()
        sh.adjoint(tr, condition=dgrtm.IMAGE_CHARACTERISTIC, up=(0.0, 0.0, 1.0), g_image_start=0)
        im = sh.image()
        torch.cuda.synchronize()
        res[prec] = (time.perf_counter() - ts, tr.cpu().numpy(), im.cpu().numpy(), sh.n_global)
        log(f"{'split-BF16' if prec else 'FP32'} comparison shot: {res[prec][0]:.2f} s")
        del sh
    ng = res[dgrtm.FP32][3]
    gdof = 3 * ng * esteps_global * dof / 1e9

    def rel(a, b):
        return float(np.linalg.norm(a - b) / max(float(np.linalg.norm(b)), 1e-300))

    f, b = res[dgrtm.FP32], res[dgrtm.SPLIT_BF16]
    return {"value": round(gdof / b[0], 3), "unit": "GDOF-steps/s",
            "dtype": "split-bf16 operator products (hi*hi + hi*lo + lo*hi), fp32 accumulation and state",
            "t_final_s": t_final, "global_steps": int(ng), "ms_per_shot": round(1e3 * b[0], 1),
            "fp32_same_shot": {"value": round(gdof / f[0], 3), "ms_per_shot": round(1e3 * f[0], 1)},
            "rel_l2_vs_fp32_same_shot": {"traces": rel(b[1], f[1]), "image": rel(b[2], f[2])}}


def log(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def traffic_from_pmc(workload: str, fetch_dir: str, write_dir: str, copy_fetch_dir: str, copy_write_dir: str,
                     command: str, profiles_dir: str = os.path.join(ROOT, "profiles")) -> str:
    """HBM bytes per step-kernel launch from two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE, KiB per
    dispatch), each scaled by what the same counter reads for a device copy of known size, averaged
    over the launches of each step mode like the roofline's achieved figure.  Writes the JSON that
    the roofline's traffic field reads."""
    import csv
    import glob

    def rows(d):
        f = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
        if not f:
            raise FileNotFoundError(f"no counter_collection.csv under {d}")
        return list(csv.DictReader(open(f[0])))

    def copy_scale(d):
        # the largest rocclr copy dispatch of the calibration run moved 2^30 bytes each way
        r = [x for x in rows(d) if "copyBuffer" in x["Kernel_Name"]]
        kib = max(float(x["Counter_Value"]) for x in r)
        return (2 ** 30) / (kib * 1024.0), kib

    sf, kf = copy_scale(copy_fetch_dir)
    sw, kw = copy_scale(copy_write_dir)
    names = {0: "forward_step", 1: "recompute_step", 2: "image_step", 4: "replay_step"}
    per = {}
    for d, scale, key in ((fetch_dir, sf, "fetch"), (write_dir, sw, "write")):
        for r in rows(d):
            n = r["Kernel_Name"]
            if "step_kernel" not in n:
                continue
            # template arguments: step_kernel_dma<N, MODE, PREC>, step_kernel_lowreg<N, MODE, OPS_LDS, PREC>
            targs = [t.strip() for t in n.split("<")[1].split(">")[0].split(",")]
            if targs[-1] not in ("0", "false"):
                continue   # the split-BF16 form's launches (same bytes; the roofline line is FP32)
            mode = int(targs[1])
            per.setdefault(names.get(mode, str(mode)), {"fetch": [], "write": []})[key].append(
                float(r["Counter_Value"]) * 1024.0 * scale)
    modes = {m: {"fetch_bytes_per_launch": sum(v["fetch"]) / len(v["fetch"]),
                 "write_bytes_per_launch": sum(v["write"]) / len(v["write"]),
                 "bytes_per_launch": sum(v["fetch"]) / len(v["fetch"]) + sum(v["write"]) / len(v["write"]),
                 "launches": len(v["fetch"])} for m, v in per.items() if v["fetch"] and v["write"]}
    out = {"workload": workload, "kernel_source_sha256_16": kernel_source_hash(),
           "copy_calibration": {"bytes": 2 ** 30, "FETCH_SIZE_KiB": kf, "WRITE_SIZE_KiB": kw,
                                "fetch_scale": sf, "write_scale": sw},
           "command": command, "modes": modes}
    path = os.path.join(profiles_dir, f"step_kernel_{workload}_traffic.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    return path


def mfma_from_pmc(pmc_dir: str, trace_dir: str) -> str:
    """Matrix-core use of the FP32 step kernels from one rocprofv3 --pmc run of SQ_VALU_MFMA_BUSY_CYCLES,
    SQ_BUSY_CU_CYCLES, SQ_INSTS_VALU_MFMA_MOPS_F32 and GRBM_GUI_ACTIVE (per-dispatch averages), with
    the kernel durations from a --kernel-trace run of the same command.  One MOPS is 512 FLOP; the
    FP32 matrix peak is 157.3 TFLOP/s; GRBM_GUI_ACTIVE is summed over the 8 XCDs."""
    import csv
    import glob

    def rows(d, pat):
        f = glob.glob(os.path.join(d, "**", pat), recursive=True)
        if not f:
            raise FileNotFoundError(f"no {pat} under {d}")
        out = []
        for path in f:
            out += list(csv.DictReader(open(path)))
        return out

    dur = {}
    for r in rows(trace_dir, "*kernel_trace.csv"):
        dur.setdefault(r["Kernel_Name"], []).append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3)
    cnt = {}
    for r in rows(pmc_dir, "*counter_collection.csv"):
        n = r["Kernel_Name"]
        if "step_kernel" not in n:
            continue
        targs = [t.strip() for t in n.split("<")[1].split(">")[0].split(",")]
        if targs[-1] not in ("0", "false"):
            continue
        cnt.setdefault(n, {}).setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    lines = [f"{'kernel':<44} {'disp':>5} {'dur_us':>8} {'MFMA_TFLOP/s':>12} {'of_peak':>8} {'MFMA_busy/SIMD':>15} "
             f"{'CU_busy':>8}"]
    for n, c in sorted(cnt.items()):
        avg = {k: sum(v) / len(v) for k, v in c.items()}
        d = dur.get(n)
        if not d:
            continue
        du = sum(d) / len(d)
        tf = avg["SQ_INSTS_VALU_MFMA_MOPS_F32"] * 512.0 / (du * 1e-6) / 1e12
        act = avg["GRBM_GUI_ACTIVE"] / 8.0
        lines.append(f"{n.split('(')[0].replace('void ', ''):<44} {len(c['GRBM_GUI_ACTIVE']):>5} {du:>8.1f} {tf:>12.1f} "
                     f"{tf / 157.3:>8.3f} {avg['SQ_VALU_MFMA_BUSY_CYCLES'] / (1024 * act):>15.3f} "
                     f"{avg['SQ_BUSY_CU_CYCLES'] / (256 * act):>8.3f}")
    return "\n".join(lines)


def kernel_trace_summary(trace_dir: str, levels: int) -> str:
    """Per-kernel calls and durations from a rocprofv3 --kernel-trace CSV, and the step-kernel
    launches split by active prefix: launch i of a step kernel (in dispatch order) is local step
    i mod 2^(levels-1) of its global step, whose active levels are the finest 1 + (trailing zeros
    of i, at most levels - 1)."""
    import csv
    import glob
    f = glob.glob(os.path.join(trace_dir, "**", "*kernel_trace.csv"), recursive=True)
    if not f:
        raise FileNotFoundError(f"no kernel_trace.csv under {trace_dir}")
    rows = []
    for path in f:
        rows += list(csv.DictReader(open(path)))
    rows.sort(key=lambda r: int(r["Dispatch_Id"]))
    per = {}
    for r in rows:
        per.setdefault(r["Kernel_Name"], []).append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3)
    total = sum(sum(v) for v in per.values())
    lines = [f"{'kernel':<72} {'calls':>7} {'avg_us':>9} {'total_ms':>9} {'%':>6}"]
    for name, d in sorted(per.items(), key=lambda kv: -sum(kv[1])):
        lines.append(f"{name[:72]:<72} {len(d):>7} {sum(d) / len(d):>9.2f} {sum(d) * 1e-3:>9.2f} "
                     f"{100 * sum(d) / total:>6.2f}")
    nl = 2 ** (levels - 1)

    def active(i):
        n = i % nl
        if n == 0:
            return levels
        k = 0
        while n % 2 == 0:
            n //= 2
            k += 1
        return min(levels, k + 1)

    lines.append("")
    lines.append(f"step kernel launches by active prefix (levels active, finest first; {levels} = every level), "
                 "mean microseconds:")
    for name, d in sorted(per.items()):
        if "step_kernel" not in name:
            continue
        by = {}
        for i, x in enumerate(d):
            by.setdefault(active(i), []).append(x)
        parts = " ".join(f"{a}:{sum(v) / len(v):.1f}" for a, v in sorted(by.items()))
        lines.append(f"  {name.split('(')[0]} mean {sum(d) / len(d):.1f}  {parts}")
    return "\n".join(lines)


def _threads() -> int:
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        if os.environ.get(k):
            return int(os.environ[k])
    return os.cpu_count() or 1


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="big_4m")
    ap.add_argument("--t-final", type=float, default=None, help="simulated time of a shot (default per workload)")
    ap.add_argument("--sample-every", type=int, default=7, help="time every n-th step-kernel launch")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--bf16-t-final", type=float, default=-1.0,
                    help="simulated time of the split-BF16 vs FP32 comparison shot (0 = skip, <0 = per workload)")
    ap.add_argument("--secondary", default="rtm_200k", help="second workload reported after the main one ('' = skip)")
    ap.add_argument("--secondary-t-final", type=float, default=0.25)
    ap.add_argument("--storage", choices=["checkpoints", "boundary"], default="checkpoints",
                    help="how the main workload's shots keep the source wavefield for the backward run")
    ap.add_argument("--no-replay-compare", action="store_true",
                    help="skip the boundary-replay vs checkpoint comparison on the secondary workload")
    ap.add_argument("--serving", type=int, default=64, help="requests in the serving section (0 = skip)")
    ap.add_argument("--serving-t-final", type=float, default=0.01)
    ap.add_argument("--traffic-from-pmc", nargs=4, metavar=("FETCH_DIR", "WRITE_DIR", "COPY_FETCH_DIR", "COPY_WRITE_DIR"),
                    help="write profiles/step_kernel_<workload>_traffic.json from rocprofv3 --pmc output and exit")
    ap.add_argument("--pmc-command", default="", help="the profiling command, recorded in the traffic JSON")
    ap.add_argument("--kernel-trace-summary", metavar="TRACE_DIR",
                    help="print the per-kernel summary of a rocprofv3 --kernel-trace CSV run and exit")
    ap.add_argument("--levels", type=int, default=0, help="LTS levels of the traced workload (with --kernel-trace-summary)")
    ap.add_argument("--mfma-from-pmc", nargs=2, metavar=("PMC_DIR", "TRACE_DIR"),
                    help="print the matrix-core use of the FP32 step kernels from rocprofv3 runs and exit")
    args = ap.parse_args()
    if args.mfma_from_pmc:
        print(mfma_from_pmc(*args.mfma_from_pmc))
        return
    if args.kernel_trace_summary:
        lv = args.levels or SHOT_SHAPES.get(args.workload, SHOT_SHAPES["default"])["levels"]
        print(kernel_trace_summary(args.kernel_trace_summary, lv))
        return
    if args.traffic_from_pmc:
        print(traffic_from_pmc(args.workload, *args.traffic_from_pmc, command=args.pmc_command))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the whole mesh and shot live on one MI355X "
              "(sharding a shot or a survey over several GPUs is not implemented)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1506_00907_amd import dgrtm, inputs as I

    out, ctx = run_workload(dgrtm, I, args.workload, args.t_final, args.steps, args.warmup, args.sample_every,
                            storage=1 if args.storage == "boundary" else 0)
    mesh, mm, rho, c, N, shape, esteps_global, dof = ctx
    if args.bf16_t_final != 0:
        bt = shape["bf16_t_final"] if args.bf16_t_final < 0 else args.bf16_t_final
        log(f"split-BF16 vs FP32 comparison shots (t_f = {bt} s) ...")
        out["split_bf16"] = precision_compare(dgrtm, I, mesh, mm.box, shape.get("src_xy", (0.7797, 1.0)),
                                              shape["n_rec"], bt, esteps_global, dof)
    del mesh, ctx
    torch.cuda.empty_cache()
    if args.secondary and args.secondary != args.workload:
        log(f"secondary block: {args.secondary} ...")
        keep = ("value", "unit", "ms_per_step", "steps", "warmup", "config", "images_per_hour",
                "single_rate_equivalent_GDOF_steps_s", "roofline")
        imgs = []
        sec, sctx = run_workload(dgrtm, I, args.secondary, args.secondary_t_final, 2, 1, args.sample_every,
                                 keep_image=imgs)
        out["secondary"] = {k: sec[k] for k in keep}
        del sctx
        torch.cuda.empty_cache()
        if not args.no_replay_compare:
            log(f"secondary block with boundary-trace replay: {args.secondary} ...")
            rep_, rctx = run_workload(dgrtm, I, args.secondary, args.secondary_t_final, 2, 1, args.sample_every,
                                      storage=1, keep_image=imgs)
            blk = {k: rep_[k] for k in keep}
            # both images approximate the same integral; they differ by the re-simulated source
            # field's departure from the forward one (the backward run cannot undo the upwind
            # dissipation of the forward run)
            blk["image_rel_l2_vs_checkpointed"] = float(np.linalg.norm(imgs[1] - imgs[0]) / np.linalg.norm(imgs[0]))
            out["secondary_boundary_replay"] = blk
            del rctx
            torch.cuda.empty_cache()
    if args.serving > 0:
        log(f"serving: {args.serving} requests ...")
        out["serving"] = serving_bench(args.serving, args.serving_t_final)
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        log("oracle CPU baseline sample ...")
        out["cpu_baseline"] = cpu_baseline(mm, rho, c, N, shape["levels"])
    print(json.dumps(out), flush=True)


def run_workload(dgrtm, I, workload, t_final, steps, warmup, sample_every, storage=0, keep_image=None):
    """Set up one workload's mesh and shot, run warmup + timed shots, and return the result
    dict (metric line fields) and the context the later sections reuse."""
    import numpy as np
    import torch

    shape = SHOT_SHAPES.get(workload, SHOT_SHAPES["default"])
    if t_final is None:
        t_final = shape["t_final"]
    log(f"building the {workload} mesh ...")
    ts = time.perf_counter()
    mm, rho, c, N = I.config_mesh(workload)
    log(f"mesh generated: {mm.K} elements in {time.perf_counter() - ts:.1f} s; host set-up and upload ...")
    n_levels = shape["levels"]
    mesh = dgrtm.Mesh(N, mm.verts, mm.etov, bc_default=dgrtm.BC_TRANSPARENT).set_model(rho, c, n_levels).bind("cuda")
    src_xy = shape.get("src_xy", (0.7797, 1.0))
    spec = I.rtm_shot(box=mm.box, src_xy=src_xy, n_rec=shape["n_rec"], t_final=t_final)
    shot = dgrtm.Shot(mesh, dgrtm.ShotSpec(t_final=spec.t_final, src=spec.src, f_peak=spec.f_peak,
                                           t_peak=spec.t_peak, rec=spec.rec, storage=storage))
    lev = mesh.export_setup()["level"].astype(np.int64)
    L = mesh.L
    hist = np.bincount(lev, minlength=L + 1)[1:]
    esteps_global = int(sum(hist[l - 1] * 2 ** (l - 1) for l in range(1, L + 1)))
    ng = shot.n_global
    dof = 4 * mesh.Np
    traces = torch.empty((shot.n_rec, ng + 1), dtype=torch.float32, device="cuda")
    img = torch.zeros((mesh.K, mesh.Np), dtype=torch.float64, device="cuda")

    def one_shot():
        shot.forward(traces)
        shot.adjoint(traces, condition=dgrtm.IMAGE_CHARACTERISTIC, up=(0.0, 0.0, 1.0), g_image_start=0)
        shot.image(img)

    log(f"mesh {workload}: {mesh.K} elements, N={N}, {L} levels {list(map(int, hist))}, "
        f"{ng} global steps per shot, shot workspace {shot.bytes / 1e9:.1f} GB")
    for i in range(warmup):
        ts = time.perf_counter()
        one_shot()
        torch.cuda.synchronize()
        log(f"warm-up shot {i}: {time.perf_counter() - ts:.2f} s")
    torch.cuda.synchronize()
    shot.profile_start(sample_every)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat = []
    for _ in range(steps):
        ts = time.perf_counter()
        one_shot()
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - ts)
        log(f"timed shot {len(lat) - 1}: {lat[-1]:.2f} s")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = {m: shot.profile_read(m) for m in (0, 1, 2, 4)}
    # element-steps per shot: forward + recompute + backward, each over every global step
    es_shot = 3 * ng * esteps_global
    value = es_shot * steps * dof / wall / 1e9
    sr_equiv = 3 * ng * mesh.K * 2 ** (L - 1) * steps * dof / wall / 1e9
    mode_names = {0: "forward_step", 1: "recompute_step", 2: "image_step", 4: "replay_step"}
    rl = {}
    for m, p in prof.items():
        if p["launches"] == 0:
            continue
        b = p["element_steps"] * bytes_per_element_step(mesh.Np, mesh.Nfp, m)
        rl[mode_names[m]] = {"avg_launch_us": 1e3 * p["kernel_ms"] / p["launches"],
                             "achieved_GBs": b / (p["kernel_ms"] * 1e-3) / 1e9,
                             "kernel_ms_sampled": p["kernel_ms"], "launches_sampled": p["launches"],
                             "algo_bytes_per_launch": b / p["launches"]}
    dom = max(rl, key=lambda k: prof[{v: k2 for k2, v in mode_names.items()}[k]]["kernel_ms"])
    tr = load_traffic(workload, dom)
    out = {
        "metric": "GDOF-steps/s FP32 vs split-BF16 at stated error; shots/h + p50/p99 shot latency",
        "value": round(value, 3),
        "unit": "GDOF-steps/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": round(1e3 * wall / steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32",
        "data": "synthetic (seeded mesh, model and shot; no dataset)",
        "config": {"workload": workload, "elements": int(mesh.K), "order_N": int(N), "levels": int(L),
                   "level_histogram_coarse_to_fine": [int(x) for x in hist], "global_steps": int(ng),
                   "t_final_s": round(ng * mesh.dt_local * 2 ** (L - 1), 6), "receivers": int(shot.n_rec),
                   "image": "characteristic", "parallelism": "single GPU",
                   "storage": "boundary traces (source re-simulated backward)" if storage else "checkpoints",
                   "shot_workspace_GB": round(shot.bytes / 1e9, 2)},
        "images_per_hour": round(3600.0 * steps / wall, 2),
        "shot_latency_s": {"p50": round(float(np.percentile(lat, 50)), 3),
                           "p99": round(float(np.percentile(lat, 99)), 3),
                           "note": "identical shots back to back; the serving section has a request stream"},
        "single_rate_equivalent_GDOF_steps_s": round(sr_equiv, 3),
        "roofline": {"bound": "hbm", "kernel": f"step_kernel ({dom})",
                     "achieved": round(rl[dom]["achieved_GBs"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(rl[dom]["achieved_GBs"] / HBM_PEAK_GBS, 4),
                     "traffic": tr, "per_mode": rl},
    }
    # the timed shot's workspace (checkpoints and segment records) is released before the other
    # sections allocate theirs: on the largest meshes one shot's workspace is most of the HBM
    if keep_image is not None:
        keep_image.append(img.cpu().numpy())
    del shot, traces, img
    return out, (mesh, mm, rho, c, N, shape, esteps_global, dof)


if __name__ == "__main__":
    main()
