"""Python binding of libdgrtm (include/dgrtm.h): argument marshalling only.

Every numerical step runs inside the HIP library; PyTorch only provides device memory
(workspaces and outputs) and the HIP stream.  If the library has not been built, importing
this module raises immediately: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from contextlib import contextmanager
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdgrtm.so")

BC_RIGID, BC_TRANSPARENT, BC_FREE = 1, 2, 3
IMAGE_PRESSURE, IMAGE_CHARACTERISTIC = 0, 1
IMAGE_TRAPEZOID = 0x100
FP32, SPLIT_BF16 = 0, 1
STORE_CHECKPOINTS, STORE_BOUNDARY = 0, 1
SOURCE_FIELD, RECEIVER_FIELD = 0, 1
PHASE_IDLE, PHASE_FORWARD, PHASE_RECOMPUTE, PHASE_BACKWARD, PHASE_DONE = 0, 1, 2, 3, 4

_SYMBOLS = {
    "dgrtm_last_error": (C.c_char_p, []),
    "dgrtm_mesh_create": (C.c_int32, [C.c_int, C.c_int64, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_int,
                                      C.POINTER(C.c_void_p)]),
    "dgrtm_set_model": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_double,
                                    C.POINTER(C.c_double), C.POINTER(C.c_int)]),
    "dgrtm_mesh_bytes": (C.c_int32, [C.c_void_p, C.POINTER(C.c_size_t)]),
    "dgrtm_mesh_bind": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "dgrtm_mesh_set_launch_cap": (C.c_int32, [C.c_void_p, C.c_int64]),
    "dgrtm_export_setup": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "dgrtm_export_operators": (C.c_int32, [C.c_void_p] + [C.c_void_p] * 5),
    "dgrtm_locate": (C.c_int32, [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]),
    "dgrtm_mesh_info": (C.c_int32, [C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int),
                                    C.POINTER(C.c_int64), C.POINTER(C.c_int), C.POINTER(C.c_double)]),
    "dgrtm_mesh_destroy": (None, [C.c_void_p]),
    "dgrtm_shot_steps": (C.c_int32, [C.c_void_p, C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int32)]),
    "dgrtm_shot_bytes": (C.c_int32, [C.c_void_p, C.c_void_p, C.POINTER(C.c_size_t)]),
    "dgrtm_shot_create": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.POINTER(C.c_void_p)]),
    "dgrtm_forward": (C.c_int32, [C.c_void_p, C.c_void_p]),
    "dgrtm_adjoint": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_int64]),
    "dgrtm_image": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_int]),
    "dgrtm_residual": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.POINTER(C.c_double)]),
    "dgrtm_residual_noalloc": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]),
    "dgrtm_apply_rhs": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int]),
    "dgrtm_set_state": (C.c_int32, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]),
    "dgrtm_get_state": (C.c_int32, [C.c_void_p, C.c_int, C.c_void_p]),
    "dgrtm_run": (C.c_int32, [C.c_void_p, C.c_int, C.c_int64, C.c_int, C.c_int]),
    "dgrtm_shot_begin": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_int64]),
    "dgrtm_step_shots": (C.c_int32, [C.c_void_p, C.c_int, C.c_int64]),
    "dgrtm_shot_traces": (C.c_int32, [C.c_void_p, C.c_void_p]),
    "dgrtm_shot_state": (C.c_int32, [C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "dgrtm_profile_start": (C.c_int32, [C.c_void_p, C.c_int]),
    "dgrtm_profile_read": (C.c_int32, [C.c_void_p, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_int64),
                                       C.POINTER(C.c_int64)]),
    "dgrtm_shot_destroy": (None, [C.c_void_p]),
}


class ShotArgs(C.Structure):
    _fields_ = [("struct_size", C.c_int32), ("has_source", C.c_int32), ("src_xyz", C.c_double * 3),
                ("f_peak", C.c_double), ("t_peak", C.c_double), ("amp", C.c_double),
                ("wavelet", C.c_void_p), ("n_rec", C.c_int64), ("rec_xyz", C.c_void_p),
                ("t_final", C.c_double), ("ckpt_interval", C.c_int64), ("precision", C.c_int32),
                ("storage", C.c_int32)]


def load_library(path: str = LIB_PATH) -> C.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"libdgrtm.so not built at {path}: run __graft_entry__.build() "
                          "or python paper_1506_00907_amd/build.py")
    lib = C.CDLL(path)
    for name, (res, args) in _SYMBOLS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


# PyTorch provides the device memory and streams; its HIP runtime is brought in before the
# library, so that one runtime serves both whatever order a caller imports them in.
try:
    import torch as _torch_first  # noqa: F401
except ImportError:
    pass

_lib = load_library()


class DgrtmError(RuntimeError):
    pass


def _check(status: int, what: str):
    if status != 0:
        raise DgrtmError(f"{what} failed ({status}): {_lib.dgrtm_last_error().decode()}")


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def _torch():
    import torch
    return torch


@contextmanager
def _ordered(mesh, *inputs):
    """Run library calls on the mesh's stream, ordered against the caller's current stream.

    On entry the mesh stream waits for the work already queued on the caller's stream (the
    producers of `inputs` and of freshly allocated outputs); on exit the caller's stream waits
    for the mesh stream, so a tensor handed back (or written in place) is complete for any
    later use or free on the caller's stream.  `inputs` that the library keeps reading after
    the call are marked as used on the mesh stream."""
    torch = _torch()
    cur = torch.cuda.current_stream(mesh.device)
    other = cur != mesh.stream
    if other:
        mesh.stream.wait_stream(cur)
        for t in inputs:
            if t is not None:
                t.record_stream(mesh.stream)
    yield
    if other:
        cur.wait_stream(mesh.stream)


class Mesh:
    """A tetrahedral mesh with its DG operators (host set-up, then bound to a device workspace)."""

    def __init__(self, N: int, verts: np.ndarray, etov: np.ndarray, bc_default: int = BC_TRANSPARENT,
                 face_bc: np.ndarray | None = None):
        self.verts = np.ascontiguousarray(verts, dtype=np.float64)
        self.etov = np.ascontiguousarray(etov, dtype=np.int64)
        fb = None if face_bc is None else np.ascontiguousarray(face_bc, dtype=np.int8)
        h = C.c_void_p()
        _check(_lib.dgrtm_mesh_create(int(N), self.verts.shape[0], _ptr(self.verts), self.etov.shape[0],
                                      _ptr(self.etov), None if fb is None else _ptr(fb), int(bc_default),
                                      C.byref(h)), "dgrtm_mesh_create")
        self.h = h
        self.K = int(self.etov.shape[0])
        self.ws = None
        self._info()

    def _info(self):
        N, Np, Nfp, L = C.c_int(), C.c_int(), C.c_int(), C.c_int()
        K, dtl = C.c_int64(), C.c_double()
        _check(_lib.dgrtm_mesh_info(self.h, C.byref(N), C.byref(Np), C.byref(Nfp), C.byref(K), C.byref(L),
                                    C.byref(dtl)), "dgrtm_mesh_info")
        self.N, self.Np, self.Nfp, self.L, self.dt_local = N.value, Np.value, Nfp.value, L.value, dtl.value

    def set_model(self, rho, c, n_levels_max: int = 3, cfl: float = 0.15):
        self.rho = np.ascontiguousarray(rho, dtype=np.float64)
        self.c = np.ascontiguousarray(c, dtype=np.float64)
        dtl, L = C.c_double(), C.c_int()
        _check(_lib.dgrtm_set_model(self.h, _ptr(self.rho), _ptr(self.c), int(n_levels_max), float(cfl),
                                    C.byref(dtl), C.byref(L)), "dgrtm_set_model")
        self._info()
        return self

    def bind(self, device="cuda", stream=None):
        torch = _torch()
        nb = C.c_size_t()
        _check(_lib.dgrtm_mesh_bytes(self.h, C.byref(nb)), "dgrtm_mesh_bytes")
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        with torch.cuda.stream(self.stream):
            self.ws = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
        with _ordered(self):
            _check(_lib.dgrtm_mesh_bind(self.h, self.ws.data_ptr(), nb.value, C.c_void_p(self.stream.cuda_stream)),
                   "dgrtm_mesh_bind")
        return self

    def set_launch_cap(self, max_groups: int):
        """Test hook: cap the work-groups of the step launches (0 = default grid)."""
        _check(_lib.dgrtm_mesh_set_launch_cap(self.h, int(max_groups)), "dgrtm_mesh_set_launch_cap")
        return self

    def export_setup(self):
        K, Nfp = self.K, self.Nfp
        EToE = np.zeros((K, 4), np.int32)
        EToF = np.zeros((K, 4), np.int8)
        vmapP = np.zeros((K, 4, Nfp), np.int32)
        level = np.zeros(K, np.int8)
        pos = np.zeros(K, np.int64)
        has_model = hasattr(self, "rho")
        _check(_lib.dgrtm_export_setup(self.h, _ptr(EToE), _ptr(EToF), _ptr(vmapP),
                                       _ptr(level) if has_model else None, _ptr(pos) if has_model else None),
               "dgrtm_export_setup")
        out = {"EToE": EToE, "EToF": EToF, "vmapP": vmapP}
        if has_model:
            out["level"], out["sorted_pos"] = level, pos
        return out

    def locate(self, xyz):
        """Element (user order) holding each point, -1 outside the mesh (host work)."""
        xyz = np.ascontiguousarray(np.atleast_2d(xyz), dtype=np.float64)
        elem = np.zeros(xyz.shape[0], np.int64)
        _check(_lib.dgrtm_locate(self.h, xyz.shape[0], _ptr(xyz), _ptr(elem)), "dgrtm_locate")
        return elem

    def export_operators(self):
        Np, F = self.Np, 4 * self.Nfp
        Dr, Ds, Dt = (np.zeros((Np, Np)) for _ in range(3))
        L = np.zeros((Np, F))
        rst = np.zeros((Np, 3))
        _check(_lib.dgrtm_export_operators(self.h, _ptr(Dr), _ptr(Ds), _ptr(Dt), _ptr(L), _ptr(rst)),
               "dgrtm_export_operators")
        return {"Dr": Dr, "Ds": Ds, "Dt": Dt, "LIFT": L, "rst": rst}

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.dgrtm_mesh_destroy(self.h)
            self.h = None


@dataclass
class ShotSpec:
    t_final: float
    src: np.ndarray | None = None
    f_peak: float = 15.0
    t_peak: float = 0.1127
    amp: float = 1.0
    rec: np.ndarray | None = None
    wavelet: np.ndarray | None = None
    ckpt_interval: int = 0
    precision: int = 0
    storage: int = 0


class Shot:
    """One RTM shot living in its own device workspace."""

    def __init__(self, mesh: Mesh, spec: ShotSpec):
        if mesh.ws is None:
            raise DgrtmError("bind the mesh before creating a shot")
        torch = _torch()
        self.mesh = mesh
        self.spec = spec
        a = ShotArgs()
        a.struct_size = C.sizeof(ShotArgs)
        a.has_source = 0 if spec.src is None else 1
        if spec.src is not None:
            for i in range(3):
                a.src_xyz[i] = float(spec.src[i])
        a.f_peak, a.t_peak, a.amp = spec.f_peak, spec.t_peak, spec.amp
        self._rec = None if spec.rec is None else np.ascontiguousarray(spec.rec, dtype=np.float64)
        self._wav = None if spec.wavelet is None else np.ascontiguousarray(spec.wavelet, dtype=np.float32)
        a.wavelet = None if self._wav is None else _ptr(self._wav)
        a.n_rec = 0 if self._rec is None else self._rec.shape[0]
        a.rec_xyz = None if self._rec is None else _ptr(self._rec)
        a.t_final = float(spec.t_final)
        a.ckpt_interval = int(spec.ckpt_interval)
        a.precision = int(spec.precision)
        a.storage = int(spec.storage)
        self.args = a
        ng, nl = C.c_int64(), C.c_int32()
        _check(_lib.dgrtm_shot_steps(mesh.h, C.byref(a), C.byref(ng), C.byref(nl)), "dgrtm_shot_steps")
        self.n_global, self.n_local = ng.value, nl.value
        nb = C.c_size_t()
        _check(_lib.dgrtm_shot_bytes(mesh.h, C.byref(a), C.byref(nb)), "dgrtm_shot_bytes")
        self.bytes = nb.value
        with torch.cuda.stream(mesh.stream):
            self.ws = torch.empty(nb.value, dtype=torch.uint8, device=mesh.device)
        h = C.c_void_p()
        with _ordered(mesh):
            _check(_lib.dgrtm_shot_create(mesh.h, C.byref(a), self.ws.data_ptr(), nb.value, C.byref(h)),
                   "dgrtm_shot_create")
        self.h = h
        self.n_rec = int(a.n_rec)

    # ---- RTM
    def forward(self, traces=None):
        torch = _torch()
        if traces is None and self.n_rec:
            traces = torch.empty((self.n_rec, self.n_global + 1), dtype=torch.float32, device=self.mesh.device)
        with _ordered(self.mesh):
            _check(_lib.dgrtm_forward(self.h, None if traces is None else traces.data_ptr()), "dgrtm_forward")
        return traces

    def adjoint(self, data, condition: int = IMAGE_CHARACTERISTIC, up=(0.0, 0.0, 1.0), g_image_start: int = 0):
        u = np.ascontiguousarray(up, dtype=np.float64)
        with _ordered(self.mesh):
            _check(_lib.dgrtm_adjoint(self.h, None if data is None else data.data_ptr(), int(condition), _ptr(u),
                                      int(g_image_start)), "dgrtm_adjoint")

    def image(self, out=None, accumulate: bool = False):
        torch = _torch()
        if out is None:
            out = torch.zeros((self.mesh.K, self.mesh.Np), dtype=torch.float64, device=self.mesh.device)
        with _ordered(self.mesh):
            _check(_lib.dgrtm_image(self.h, out.data_ptr(), int(accumulate)), "dgrtm_image")
        return out

    def residual(self, a, b) -> float:
        r = C.c_double()
        with _ordered(self.mesh):
            _check(_lib.dgrtm_residual(self.h, a.data_ptr(), b.data_ptr(), a.numel(), C.byref(r)),
                   "dgrtm_residual")
        return r.value

    # ---- test hooks
    def apply_rhs(self, q, reversed_time: bool = False):
        torch = _torch()
        out = torch.empty_like(q)
        with _ordered(self.mesh):
            _check(_lib.dgrtm_apply_rhs(self.h, q.data_ptr(), out.data_ptr(), int(reversed_time)),
                   "dgrtm_apply_rhs")
        return out

    def set_state(self, which: int, q, h1=None, h2=None):
        with _ordered(self.mesh):
            _check(_lib.dgrtm_set_state(self.h, int(which), None if q is None else q.data_ptr(),
                                        None if h1 is None else h1.data_ptr(),
                                        None if h2 is None else h2.data_ptr()), "dgrtm_set_state")

    def get_state(self, which: int):
        torch = _torch()
        out = torch.empty((self.mesh.K, 4, self.mesh.Np), dtype=torch.float32, device=self.mesh.device)
        with _ordered(self.mesh):
            _check(_lib.dgrtm_get_state(self.h, int(which), out.data_ptr()), "dgrtm_get_state")
        return out

    def run(self, which: int, n_global: int, reversed_time: bool = False, with_source: bool = False):
        with _ordered(self.mesh):
            _check(_lib.dgrtm_run(self.h, int(which), int(n_global), int(reversed_time), int(with_source)),
                   "dgrtm_run")

    # ---- pipeline (continuous batching)
    def begin(self, data=None, condition: int = IMAGE_CHARACTERISTIC, up=(0.0, 0.0, 1.0), g_image_start: int = 0):
        self._up = np.ascontiguousarray(up, dtype=np.float64)
        self._data = data
        with _ordered(self.mesh, data):
            _check(_lib.dgrtm_shot_begin(self.h, None if data is None else data.data_ptr(), int(condition),
                                         _ptr(self._up), int(g_image_start)), "dgrtm_shot_begin")

    def state(self):
        ph, done, total = C.c_int(), C.c_int64(), C.c_int64()
        _check(_lib.dgrtm_shot_state(self.h, C.byref(ph), C.byref(done), C.byref(total)), "dgrtm_shot_state")
        return ph.value, done.value, total.value

    def traces(self):
        """The shot's own recorded traces (device copy)."""
        torch = _torch()
        out = torch.empty((self.n_rec, self.n_global + 1), dtype=torch.float32, device=self.mesh.device)
        with _ordered(self.mesh):
            _check(_lib.dgrtm_shot_traces(self.h, out.data_ptr()), "dgrtm_shot_traces")
        return out

    # ---- measurement
    def profile_start(self, sample_every: int):
        _check(_lib.dgrtm_profile_start(self.h, int(sample_every)), "dgrtm_profile_start")

    def profile_read(self, mode: int):
        ms, n, es = C.c_double(), C.c_int64(), C.c_int64()
        _check(_lib.dgrtm_profile_read(self.h, int(mode), C.byref(ms), C.byref(n), C.byref(es)),
               "dgrtm_profile_read")
        return {"kernel_ms": ms.value, "launches": n.value, "element_steps": es.value}

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.dgrtm_shot_destroy(self.h)
            self.h = None


def step_shots(shots, n_global: int = 1):
    """Advance several shots of one mesh by n_global global steps of their pipelines, batched."""
    arr = (C.c_void_p * len(shots))(*[s.h for s in shots])
    if not shots:
        return
    with _ordered(shots[0].mesh):
        _check(_lib.dgrtm_step_shots(arr, len(shots), int(n_global)), "dgrtm_step_shots")


def residual_noalloc(a, b, out=None, stream=None):
    """FP64 sum of (a - b)^2 over two device float tensors, computed by the library without any
    device allocation of its own (its partial sums live in a static device array).  The result
    is written into `out` (a device float64 tensor of one element, allocated here if not given)
    on `stream` (default: the current stream of a's device); the call does not wait for it."""
    torch = _torch()
    if a.dtype != torch.float32 or b.dtype != torch.float32 or a.numel() != b.numel():
        raise DgrtmError("residual_noalloc: a and b must be float32 tensors of equal size")
    if not (a.is_contiguous() and b.is_contiguous()):
        raise DgrtmError("residual_noalloc: a and b must be contiguous")
    if out is None:
        out = torch.empty(1, dtype=torch.float64, device=a.device)
    st = stream if stream is not None else torch.cuda.current_stream(a.device)
    _check(_lib.dgrtm_residual_noalloc(a.data_ptr(), b.data_ptr(), a.numel(), out.data_ptr(),
                                       C.c_void_p(st.cuda_stream)), "dgrtm_residual_noalloc")
    return out
