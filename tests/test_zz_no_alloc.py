"""The allocation-free entry point dgrtm_residual_noalloc against dgrtm_residual, through the C ABI."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _shot():
    from paper_1506_00907_amd import dgrtm, inputs as I
    mm, rho, c, N = I.config_mesh("two_layer_small:3:3:2:2")
    lm = dgrtm.Mesh(N, mm.verts, mm.etov, bc_default=dgrtm.BC_TRANSPARENT).set_model(rho, c, 3).bind("cuda:0")
    spec = I.rtm_shot(n_rec=2)
    return dgrtm.Shot(lm, dgrtm.ShotSpec(t_final=4 * lm.dt_local * 2 ** (lm.L - 1), src=spec.src, rec=spec.rec))


def test_noalloc_residual_matches_workspace_residual():
    import torch
    from paper_1506_00907_amd import dgrtm
    shot = _shot()
    rng = np.random.default_rng(11)
    out = torch.full((1,), -1.0, dtype=torch.float64, device="cuda:0")
    # two calls in a row, the second smaller (the static partial sums keep the first call's values):
    # 300 chunks of 16384 values plus a ragged tail, then one chunk and a tail
    for n in (300 * 16384 + 4321, 16384 + 77):
        a = torch.from_numpy(rng.standard_normal(n).astype(np.float32)).to("cuda:0")
        b = torch.from_numpy(rng.standard_normal(n).astype(np.float32)).to("cuda:0")
        ref = shot.residual(a, b)
        got = dgrtm.residual_noalloc(a, b, out=out)
        torch.cuda.synchronize()
        val = float(got.item())
        # the plain definition, summed on the host in FP64
        d = a.cpu().numpy().astype(np.float64) - b.cpu().numpy().astype(np.float64)
        exact = float(np.dot(d, d))
        print(f"n={n}: noalloc {val!r} workspace {ref!r} host {exact!r}", flush=True)
        assert abs(val - ref) <= 1e-12 * ref
        assert abs(val - exact) <= 1e-12 * exact
        # fixed summation order: a second call gives the same bits
        again = float(dgrtm.residual_noalloc(a, b).item())
        assert again == val


def test_noalloc_residual_empty_and_too_large():
    import torch
    from paper_1506_00907_amd import dgrtm
    out = torch.full((1,), -1.0, dtype=torch.float64, device="cuda:0")
    a = torch.zeros(0, dtype=torch.float32, device="cuda:0")
    dgrtm.residual_noalloc(a, a, out=out)
    assert float(out.item()) == 0.0
    # a size beyond the static scratch is refused on the host before anything is launched
    lib = dgrtm._lib
    x = torch.zeros(4, dtype=torch.float32, device="cuda:0")
    st = torch.cuda.current_stream().cuda_stream
    rc = lib.dgrtm_residual_noalloc(x.data_ptr(), x.data_ptr(), (1 << 30) + 1, out.data_ptr(), ctypes.c_void_p(st))
    assert rc == -1
    assert b"exceeds the maximum" in lib.dgrtm_last_error()
    assert float(out.item()) == 0.0
