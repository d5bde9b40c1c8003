"""The host driver's schedule on the CPU, against a recording fake device.

csrc/api.cpp and csrc/setup.cpp are built with the host compiler and linked against
tests/sched/fake_device.cpp, which stands in for the kernels and the HIP runtime: device memory
is host memory, and every launch is logged instead of run.  The log of a shot (forward, then the
adjoint with the image) is checked against the oracle's own stepping:

* every step launch updates exactly the elements the oracle's multi-rate AB3 (Alg. 1) evaluates
  at that local step, in the same order of local steps, in the right time direction;
* the receiver field's data are taken at the physical local step the oracle uses;
* every image evaluation of the oracle finds its source step inside the segment the driver has
  recomputed (checkpointed runs: the source step paired by the imaging section's formula;
  boundary-trace replay: the same own step, both fields running backward);
* checkpoints, segment restores, receiver records and boundary-trace records come where the
  RTM procedure needs them;
* shots stepped together (batched launches) see the same schedule as each shot alone.
"""
import ctypes as C
import os
import shutil
import subprocess

import numpy as np
import pytest

from tests.oracle_cases import case, oracle_shot
from paper_1506_00907_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CXX = shutil.which("g++")

R_STEP, R_RECORD, R_COPY, R_TRACE_INIT, R_SEG_INIT, R_FILL, R_BND, R_REPLAY_HIST = 1, 2, 3, 4, 5, 6, 7, 8
M_PLAIN, M_RECORD_SEG, M_IMAGE, M_RHS_ONLY, M_REPLAY_SEG, M_RHS_REPLAY = 0, 1, 2, 3, 4, 5
D2D = 3   # hipMemcpyDeviceToDevice
MESH = "two_layer_small:4:4:3:2"   # 288 tets, N = 2, 3 levels


@pytest.fixture(scope="module")
def fake(tmp_path_factory):
    if CXX is None:
        pytest.skip("no host C++ compiler")
    out = str(tmp_path_factory.mktemp("fake") / "libdgrtm_fake.so")
    srcs = [os.path.join(ROOT, "tests", "sched", "fake_device.cpp"),
            os.path.join(ROOT, "paper_1506_00907_amd", "csrc", "api.cpp"),
            os.path.join(ROOT, "paper_1506_00907_amd", "csrc", "setup.cpp")]
    cmd = [CXX, "-std=c++17", "-O1", "-fPIC", "-shared", "-ffp-contract=off", "-D__HIP_PLATFORM_AMD__",
           "-I/opt/rocm/include"] + srcs + ["-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr
    from paper_1506_00907_amd import dgrtm
    lib = C.CDLL(out)
    for name, (res, args) in dgrtm._SYMBOLS.items():
        if hasattr(lib, name):
            fn = getattr(lib, name)
            fn.restype, fn.argtypes = res, args
    lib.fake_log_size.restype = C.c_int64
    lib.fake_log_words.restype = C.c_int
    lib.fake_log_read.argtypes = [C.c_void_p]
    return lib, dgrtm


def _ok(lib, status):
    assert status == 0, lib.dgrtm_last_error().decode()


def _aligned(nbytes):
    buf = np.zeros(nbytes + 512, np.uint8)
    off = (-buf.ctypes.data) % 256
    return buf, buf.ctypes.data + off


class FakeMesh:
    def __init__(self, fake, name=MESH, n_levels=3):
        lib, dg = fake
        self.lib, self.dg = lib, dg
        mm, rho, c, N = I.config_mesh(name)
        self.mm = mm
        self.verts = np.ascontiguousarray(mm.verts, np.float64)
        self.etov = np.ascontiguousarray(mm.etov, np.int64)
        h = C.c_void_p()
        _ok(lib, lib.dgrtm_mesh_create(N, self.verts.shape[0], self.verts.ctypes.data, self.etov.shape[0],
                                       self.etov.ctypes.data, None, dg.BC_TRANSPARENT, C.byref(h)))
        self.h = h
        self.rho, self.c = np.ascontiguousarray(rho, np.float64), np.ascontiguousarray(c, np.float64)
        dtl, L = C.c_double(), C.c_int()
        _ok(lib, lib.dgrtm_set_model(h, self.rho.ctypes.data, self.c.ctypes.data, n_levels, 0.15, C.byref(dtl),
                                     C.byref(L)))
        self.L, self.dt_local = L.value, dtl.value
        nb = C.c_size_t()
        _ok(lib, lib.dgrtm_mesh_bytes(h, C.byref(nb)))
        self.ws, p = _aligned(nb.value)
        _ok(lib, lib.dgrtm_mesh_bind(h, p, nb.value, None))
        K = self.etov.shape[0]
        Nfp = (N + 1) * (N + 2) // 2
        self.level = np.zeros(K, np.int8)
        self.pos = np.zeros(K, np.int64)
        EToE, EToF, vmapP = np.zeros((K, 4), np.int32), np.zeros((K, 4), np.int8), np.zeros((K, 4, Nfp), np.int32)
        _ok(lib, lib.dgrtm_export_setup(h, EToE.ctypes.data, EToF.ctypes.data, vmapP.ctypes.data,
                                        self.level.ctypes.data, self.pos.ctypes.data))
        self.K = K

    def active(self, k_end):
        """User elements in the active prefix [0, k_end) of the sorted order."""
        return np.flatnonzero(self.pos < k_end)


class FakeShot:
    def __init__(self, mesh: FakeMesh, t_final, ckpt_interval=0, storage=0, n_rec=4, seed=0):
        lib, dg = mesh.lib, mesh.dg
        self.mesh, self.lib, self.dg = mesh, lib, dg
        self.spec = I.rtm_shot(box=mesh.mm.box, src_xy=(0.61, 0.83), n_rec=n_rec, t_final=t_final)
        a = dg.ShotArgs()
        a.struct_size = C.sizeof(dg.ShotArgs)
        a.has_source = 1
        for i in range(3):
            a.src_xyz[i] = float(self.spec.src[i])
        a.f_peak, a.t_peak, a.amp = self.spec.f_peak, self.spec.t_peak, 1.0
        self._rec = np.ascontiguousarray(self.spec.rec, np.float64)
        a.wavelet = None
        a.n_rec = self._rec.shape[0]
        a.rec_xyz = self._rec.ctypes.data
        a.t_final = float(t_final)
        a.ckpt_interval = int(ckpt_interval)
        a.precision = 0
        a.storage = int(storage)
        self.args = a
        ng, nl = C.c_int64(), C.c_int32()
        _ok(lib, lib.dgrtm_shot_steps(mesh.h, C.byref(a), C.byref(ng), C.byref(nl)))
        self.NG, self.nl = ng.value, nl.value
        nb = C.c_size_t()
        _ok(lib, lib.dgrtm_shot_bytes(mesh.h, C.byref(a), C.byref(nb)))
        self.ws, p = _aligned(nb.value)
        self.ws_base, self.ws_end = p, p + nb.value
        h = C.c_void_p()
        _ok(lib, lib.dgrtm_shot_create(mesh.h, C.byref(a), p, nb.value, C.byref(h)))
        self.h = h
        self.traces = np.zeros((a.n_rec, self.NG + 1), np.float32)

    def forward(self):
        _ok(self.lib, self.lib.dgrtm_forward(self.h, self.traces.ctypes.data))

    def adjoint(self, condition=1, g_image_start=0):
        up = np.array([0.0, 0.0, 1.0])
        _ok(self.lib, self.lib.dgrtm_adjoint(self.h, self.traces.ctypes.data, condition, up.ctypes.data,
                                             int(g_image_start)))

    def owns(self, ptr):
        return self.ws_base <= ptr < self.ws_end


def read_log(lib):
    n, w = lib.fake_log_size(), lib.fake_log_words()
    out = np.zeros((n, w), np.int64)
    if n:
        lib.fake_log_read(out.ctypes.data)
    lib.fake_log_clear()
    return out


def steps(log, mode=None):
    s = log[log[:, 0] == R_STEP]
    return s if mode is None else s[s[:, 1] == mode]


# ------------------------------------------------------------------ the oracle's schedule

def oracle_ev_sequence(lev, L, n_steps):
    """Elements the oracle's MRAB evaluates at each local step (its local_step, run on a mesh whose
    operator is never needed: the hook records and the rhs is not looked at)."""
    from oracle.timestep import MRAB
    _, op, _, _, _ = case(MESH)
    seen = []
    st = MRAB(op, lev, L, 1.0, on_eval=lambda ev, m, q, h: seen.append(np.array(ev)))
    for _ in range(n_steps):
        st.local_step()
    return seen


def oracle_image_pairs(sh: FakeShot, lev, L, dtl, g_image_start=0):
    """(receiver local step n, elements, paired source own steps) of every image evaluation of the
    oracle's checkpoint-free adjoint: which source step each receiver step correlates with."""
    import oracle.rtm as R
    _, op, _, _, _ = case(MESH)
    osh = oracle_shot(op, lev, L, dtl, sh.NG, sh.spec)
    cur = {"n": -1}
    pairs = []

    class Tracking(R.MRAB):
        def local_step(self):
            cur["n"] = self.n
            super().local_step()

    class QS:
        def __init__(self, a):
            self.a = a

        def __getitem__(self, idx):
            mS, ev = idx
            pairs.append((cur["n"], np.array(ev), np.array(mS)))
            return self.a[idx]

    orig = R.MRAB
    R.MRAB = Tracking
    try:
        tr = osh.forward()
        osh.qS = QS(osh.qS)
        osh.adjoint(tr, g_image_start=g_image_start)
    finally:
        R.MRAB = orig
    return pairs


# ------------------------------------------------------------------ tests

@pytest.fixture(scope="module")
def mesh(fake):
    m = FakeMesh(fake)
    _, _, lev, L, _ = case(MESH)
    assert m.L == L and np.array_equal(m.level, lev), "levels as the oracle assigns them"
    return m


def _lev_user(mesh):
    return mesh.level.astype(np.int64)


def test_forward_schedule_matches_alg1(fake, mesh):
    lib, _ = fake
    read_log(lib)
    sh = FakeShot(mesh, t_final=10.5 * mesh.dt_local * 4, ckpt_interval=3)
    read_log(lib)
    sh.forward()
    log = read_log(lib)
    L, nl, NG = mesh.L, sh.nl, sh.NG
    assert nl == 2 ** (L - 1) and NG == 11
    plain = steps(log, M_PLAIN)
    assert len(plain) == NG * nl and np.all(plain[:, 5] == 1)
    assert np.array_equal(plain[:, 6], np.arange(NG * nl)), "local steps in order"
    assert np.all(plain[:, 3] == 0) and np.all(plain[:, 13] == 0) and np.all(plain[:, 12] == 0)
    ev = oracle_ev_sequence(_lev_user(mesh), L, NG * nl)
    for n, row in enumerate(plain):
        assert np.array_equal(mesh.active(row[2]), np.sort(ev[n])), f"local step {n}"
    # receiver records: the state at rest, then after every global step, at successive columns
    idx = np.flatnonzero((log[:, 0] == R_STEP) | (log[:, 0] == R_RECORD))
    kinds = log[idx, 0]
    rec = log[log[:, 0] == R_RECORD]
    assert len(rec) == NG + 1
    assert np.all(np.diff(rec[:, 2]) == 4) and np.all(rec[:, 4] == NG + 1)
    expect = [R_RECORD] + ([R_STEP] * nl + [R_RECORD]) * NG
    assert kinds.tolist() == expect
    # checkpoints: a block of device copies (state and the two newest rhs of every level) before
    # global steps 0, C, 2C, ...
    nonempty = len(np.unique(mesh.level))
    first_of_global = {int(np.flatnonzero((log[:, 0] == R_STEP) & (log[:, 6] == g * nl))[0]): g for g in range(NG)}
    copies_before = {}
    i = 0
    for j, r in enumerate(log):
        if j in first_of_global:
            copies_before[first_of_global[j]] = i
            i = 0
        if r[0] == R_COPY and r[1] == D2D:
            i += 1
        elif r[0] in (R_STEP, R_RECORD):
            i = 0
    for g in range(NG):
        assert copies_before[g] == (1 + 2 * nonempty if g % 3 == 0 else 0), f"global step {g}"


@pytest.mark.parametrize("g_image_start", [0, 4])
def test_adjoint_segments_and_image_pairing(fake, mesh, g_image_start):
    lib, _ = fake
    read_log(lib)
    sh = FakeShot(mesh, t_final=10.5 * mesh.dt_local * 4, ckpt_interval=3)
    sh.forward()
    read_log(lib)
    sh.adjoint(g_image_start=g_image_start)
    log = read_log(lib)
    L, nl, NG, Cc = mesh.L, sh.nl, sh.NG, 3
    lev = _lev_user(mesh)
    img = steps(log, M_IMAGE)
    seg = steps(log, M_RECORD_SEG)
    # segments: c from the last down to the one holding g_image_start, each recomputed forward
    # (restore, traces, segment history) and then imaged backward over its window
    cs = list(range((NG - 1) // Cc, g_image_start // Cc - 1, -1))
    inits = log[log[:, 0] == R_SEG_INIT]
    assert len(inits) == len(cs)
    for r, c in zip(inits, cs):
        assert r[1] == 0 and r[2] == L
        assert [int(r[3 + l]) for l in range(L)] == [(c * Cc) << l for l in range(L)]
    want_seg = np.concatenate([np.arange(c * Cc * nl, min(NG, c * Cc + Cc) * nl) for c in cs])
    assert np.array_equal(seg[:, 6], want_seg)
    assert np.all(seg[:, 3] == 0)
    n_img = (NG - g_image_start) * nl
    assert np.array_equal(img[:, 6], np.arange(n_img)), "receiver local steps in order"
    assert np.all(img[:, 3] == 1) and np.all(img[:, 13] == 1) and np.all(img[:, 12] == 1)
    assert np.all(img[:, 7] == NG * nl - img[:, 6]), "data at the physical local step"
    assert np.all(img[:, 10] == g_image_start * nl) and np.all(img[:, 11] == 0)
    # each image launch follows the recompute of its own segment and precedes the next one's
    order = [(r[1], r[6], r[8]) for r in log[log[:, 0] == R_STEP]]
    for c in cs:
        g0, g1 = c * Cc, min(NG, c * Cc + Cc)
        sel = [i for i, o in enumerate(order) if o[0] == M_IMAGE and o[2] == g0]
        rec = [i for i, o in enumerate(order) if o[0] == M_RECORD_SEG and g0 * nl <= o[1] < g1 * nl]
        assert sel and rec and max(rec) < min(sel)
        assert [order[i][1] for i in sel] == list(range((NG - g1) * nl, (NG - max(g0, g_image_start)) * nl))
    # each segment starts from its checkpoint: the state and the two newest rhs of every level
    # come back by device copies, then its traces and its segment history, before its first
    # recompute launch
    steps_at = np.flatnonzero(log[:, 0] == R_STEP)
    nonempty = len(np.unique(mesh.level))
    prev = -1
    for c in cs:
        first = next(i for i in steps_at if log[i, 1] == M_RECORD_SEG and log[i, 6] == c * Cc * nl)
        blk = log[prev + 1:first]
        kinds = blk[:, 0]
        assert np.sum((kinds == R_COPY) & (blk[:, 1] == D2D)) == 1 + 2 * nonempty, f"segment {c}"
        assert np.sum(kinds == R_TRACE_INIT) == 1 and np.sum(kinds == R_SEG_INIT) == 1
        ti = blk[kinds == R_TRACE_INIT][0]
        assert ti[2] == c * Cc * nl, "traces of the restored state at the segment's first local step"
        prev = max(i for i in steps_at if log[i, 1] == M_IMAGE and log[i, 8] == c * Cc) if c != cs[-1] else first
    # active sets of the backward run are the oracle's
    ev = oracle_ev_sequence(lev, L, n_img)
    for n, row in enumerate(img):
        assert np.array_equal(mesh.active(row[2]), np.sort(ev[n]))
    # every image evaluation of the oracle finds its source step in the recomputed segment
    pairs = oracle_image_pairs(sh, lev, L, mesh.dt_local, g_image_start)
    assert len(pairs) > 0
    for n, evs, mS in pairs:
        row = img[n]
        g0, g1 = row[8], row[9]
        lv = lev[evs]
        assert np.all(mS >= (g0 << (lv - 1))) and np.all(mS < (g1 << (lv - 1))), f"receiver local step {n}"
    # the oracle images every element-step of the receiver run over [t_i, t_f]
    n_pairs = sum(e.size for _, e, _ in pairs)
    stride = 2 ** (L - lev)
    assert n_pairs == sum(int(((NG - g_image_start) * nl) // s) for s in stride)


def test_boundary_replay_schedule(fake, mesh):
    lib, dg = fake
    read_log(lib)
    sh = FakeShot(mesh, t_final=6.5 * mesh.dt_local * 4, storage=dg.STORE_BOUNDARY)
    sh.forward()
    flog = read_log(lib)
    L, nl, NG = mesh.L, sh.nl, sh.NG
    lev = _lev_user(mesh)
    _, op, _, _, _ = case(MESH)
    nbf = np.array([op.m.is_bdry[lev == l].sum() for l in range(1, L + 1)])
    # after every forward launch, the boundary traces of the levels it updated
    seq = flog[np.isin(flog[:, 0], (R_STEP, R_BND))]
    assert len(seq) == 2 * NG * nl
    for i in range(NG * nl):
        s, b = seq[2 * i], seq[2 * i + 1]
        assert s[0] == R_STEP and b[0] == R_BND and s[6] == i and b[1] == i
        act = np.unique(lev[mesh.active(s[2])])
        assert b[2] == nbf[act - 1].sum()
    sh.adjoint()
    log = read_log(lib)
    st = log[log[:, 0] == R_STEP]
    # start: the reversed-time rhs at t_f, t_f - dt_g, t_f - 2 dt_g, then the extrapolated history
    start = st[:3]
    assert np.all(start[:, 1] == M_RHS_REPLAY) and np.all(start[:, 3] == 1)
    assert start[:, 7].tolist() == [NG * nl, (NG - 1) * nl, (NG - 2) * nl]
    assert np.all(start[:, 2] > mesh.pos.max()), "every element"
    hist_i = np.flatnonzero(log[:, 0] == R_REPLAY_HIST)
    assert len(hist_i) == 1 and hist_i[0] > np.flatnonzero(log[:, 0] == R_STEP)[2]
    # then per backward global step: the source field's local steps, then the receiver field's,
    # over the same window, both backward
    rest = st[3:]
    ev = oracle_ev_sequence(lev, L, NG * nl)
    assert len(rest) == 2 * NG * nl
    for gb in range(NG):
        blk = rest[2 * gb * nl:2 * (gb + 1) * nl]
        S, R = blk[:nl], blk[nl:]
        assert np.all(S[:, 1] == M_REPLAY_SEG) and np.all(R[:, 1] == M_IMAGE)
        for part in (S, R):
            assert part[:, 6].tolist() == list(range(gb * nl, (gb + 1) * nl))
            assert np.all(part[:, 3] == 1) and np.all(part[:, 13] == 1)
            assert np.all(part[:, 7] == NG * nl - part[:, 6])
            assert np.all(part[:, 8] == gb) and np.all(part[:, 9] == gb + 1)
        assert np.all(R[:, 11] & 1) and np.all(R[:, 10] == 0) and np.all(S[:, 12] == 2)
        for j in range(nl):
            n = gb * nl + j
            act = mesh.active(S[j, 2])
            assert np.array_equal(act, np.sort(ev[n])) and np.array_equal(mesh.active(R[j, 2]), act)
            # the pairing: the same own step of both fields, inside the window
            lv = lev[act]
            m = n // 2 ** (L - lv)
            assert np.all(m >= (gb << (lv - 1))) and np.all(m < ((gb + 1) << (lv - 1)))
    # the first segment's history rows come from the extrapolated start history; every later
    # segment's are the previous segment's last two rows, moved to the front by two device copies
    # per level before the segment's first source-field launch
    inits = log[log[:, 0] == R_SEG_INIT]
    assert len(inits) == 1 and inits[0, 1] == 1 and [int(inits[0, 3 + l]) for l in range(L)] == [0] * L
    rows = np.flatnonzero(log[:, 0] == R_STEP)
    nonempty = len(np.unique(mesh.level))
    for gb in range(1, NG):
        first_S = rows[3 + 2 * gb * nl]
        last_R = rows[3 + 2 * gb * nl - 1]
        between = log[last_R + 1:first_S]
        assert log[first_S, 1] == M_REPLAY_SEG and log[last_R, 1] == M_IMAGE
        assert np.sum((between[:, 0] == R_COPY) & (between[:, 1] == D2D)) == 2 * nonempty
        assert not np.any(between[:, 0] == R_SEG_INIT)


def test_batched_shots_see_their_solo_schedule(fake, mesh):
    lib, dg = fake
    up = np.array([0.0, 0.0, 1.0])
    solo = {}
    shots = []
    for i, (tf, cint) in enumerate([(5.5, 2), (4.5, 3), (5.5, 2)]):
        read_log(lib)
        s = FakeShot(mesh, t_final=tf * mesh.dt_local * 4, ckpt_interval=cint)
        read_log(lib)
        _ok(lib, lib.dgrtm_shot_begin(s.h, s.traces.ctypes.data, 1, up.ctypes.data, 0))
        hs = (C.c_void_p * 1)(s.h)
        while True:
            ph = C.c_int()
            _ok(lib, lib.dgrtm_shot_state(s.h, C.byref(ph), None, None))
            if ph.value == dg.PHASE_DONE:
                break
            _ok(lib, lib.dgrtm_step_shots(hs, 1, 1))
        lg = steps(read_log(lib))
        solo[i] = [tuple(r[[1, 3, 6, 7, 8, 9]]) for r in lg]
        shots.append(s)
    # the same shots, restarted and stepped together; the third joins two global steps late
    read_log(lib)
    for s in shots[:2]:
        _ok(lib, lib.dgrtm_shot_begin(s.h, s.traces.ctypes.data, 1, up.ctypes.data, 0))
    hs = (C.c_void_p * 3)(*[s.h for s in shots])
    _ok(lib, lib.dgrtm_step_shots(hs, 2, 2))
    _ok(lib, lib.dgrtm_shot_begin(shots[2].h, shots[2].traces.ctypes.data, 1, up.ctypes.data, 0))
    for _ in range(40):
        _ok(lib, lib.dgrtm_step_shots(hs, 3, 1))
    lg = steps(read_log(lib))
    got = {i: [] for i in range(3)}
    shared = 0
    for r in lg:
        owner = [i for i, s in enumerate(shots) if s.owns(int(r[15]))]
        assert len(owner) == 1
        got[owner[0]].append(tuple(r[[1, 3, 6, 7, 8, 9]]))
        shared += r[5] > 1
    for i in range(3):
        assert got[i] == solo[i], f"shot {i}"
    assert shared > 0, "shots in the same mode share launches"
    # within one launch every slot is in the launch's mode and time direction
    for k in np.unique(np.flatnonzero(lg[:, 4] == 0)):
        blk = lg[k:k + lg[k, 5]]
        assert np.all(blk[:, 1] == blk[0, 1]) and np.all(blk[:, 3] == blk[0, 3]) and np.all(blk[:, 2] == blk[0, 2])
