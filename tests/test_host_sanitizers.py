"""The library's host set-up (csrc/setup.cpp: reference element, connectivity, levels, face-node
maps, point location) built with AddressSanitizer and UndefinedBehaviorSanitizer by the host
compiler and run on several meshes; its integer results must also equal the oracle's."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import source as OS
from oracle.mesh import BC_TRANSPARENT, OMesh, local_dt, lts_levels
from oracle.refelem import get_ref
from paper_1506_00907_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CXX = shutil.which("g++")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if CXX is None:
        pytest.skip("no host C++ compiler")
    out = str(tmp_path_factory.mktemp("asan") / "host_setup_driver")
    flags = ["-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
             "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
    srcs = [os.path.join(ROOT, "tests", "host_setup_driver.cpp"),
            os.path.join(ROOT, "paper_1506_00907_amd", "csrc", "setup.cpp")]
    r = subprocess.run([CXX] + flags + srcs + ["-o", out], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr
    return out


def _one_tet():
    # one tetrahedron given with negative orientation: every face a boundary, padded to a tile
    v = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]])
    return v, np.array([[0, 2, 1, 3]]), np.ones(1), np.ones(1)


CASES = [("two_layer_small:5:4:3:4", 3), ("two_layer_small:3:3:2:6", 3), ("eigen_cube", 1), ("one_tet:5", 1)]


@pytest.mark.parametrize("name,nl", CASES)
def test_host_setup_is_clean_under_sanitizers(driver, tmp_path, name, nl):
    if name.startswith("one_tet"):
        verts, etov, rho, c = _one_tet()
        N = int(name.split(":")[1])
    else:
        mm, rho, c, N = I.config_mesh(name)
        verts, etov = mm.verts, mm.etov
    rng = np.random.default_rng(1)
    lo, hi = verts.min(0), verts.max(0)
    pts = np.vstack([verts[etov[::7]].mean(axis=1), lo + rng.uniform(0, 1, (20, 3)) * (hi - lo), verts[:10],
                     [hi + 1.0]])
    for fn, a in (("verts.f64", verts.astype(np.float64)), ("etov.i64", etov.astype(np.int64)),
                  ("rho.f64", rho.astype(np.float64)), ("c.f64", c.astype(np.float64)),
                  ("pts.f64", pts.astype(np.float64))):
        a.tofile(str(tmp_path / fn))
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    env.pop("LD_PRELOAD", None)
    r = subprocess.run([driver, str(tmp_path), str(N), str(nl)], capture_output=True, text=True, env=env,
                       timeout=600)
    assert r.returncode == 0 and "runtime error" not in r.stderr and "Sanitizer" not in r.stderr, r.stderr[-4000:]
    K = etov.shape[0]
    om = OMesh(get_ref(N), verts, etov, bc_default=BC_TRANSPARENT)
    assert np.array_equal(np.fromfile(str(tmp_path / "EToE.i32"), np.int32).reshape(K, 4), om.EToE)
    assert np.array_equal(np.fromfile(str(tmp_path / "EToF.i8"), np.int8).reshape(K, 4), om.EToF)
    assert np.array_equal(np.fromfile(str(tmp_path / "vmapP.i32"), np.int32).reshape(K, 4, -1), om.vmapP)
    lev, L, dtl = lts_levels(local_dt(om.verts, om.etov, c, N), om.EToE, nl)
    assert np.array_equal(np.fromfile(str(tmp_path / "level.i8"), np.int8), lev)
    elem = np.fromfile(str(tmp_path / "elem.i64"), np.int64)
    want = []
    for x in pts:
        try:
            want.append(int(OS.locate(om, x[None])[0]))
        except ValueError:       # outside the mesh
            want.append(-1)
    assert want[-1] == -1
    assert np.array_equal(elem, np.array(want))
