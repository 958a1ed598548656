"""r1_envelope_stress_noalloc (fixed per-device workspace, nothing allocated)
against r1_envelope_stress, through the C-ABI: the same kernels run on the same
inputs, so W, P, tree and flags must agree bit for bit.  Two calls in a row on
one handle, the second with fewer points (and at depth 2 fewer outer
directions), so the second reads a workspace that still holds the first call's
data; both precisions, depths 1 and 2."""
import ctypes

import numpy as np
import pytest

from paper_2211_14318_amd import workloads as WL

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2211_14318_amd import r1
    h = r1.Handle(0)
    yield r1, h, torch
    h.close()


def _call(r1, h, torch, fn, mat, spec, F, bn):
    n = F.shape[1]
    d = mat.dim
    W = torch.full((n,), -7.0, dtype=F.dtype, device="cuda")
    P = torch.full((d * d, n), -7.0, dtype=F.dtype, device="cuda")
    T = torch.full((n, 3, 4), -7, dtype=torch.int32, device="cuda")
    fl = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    st = fn(h.h, ctypes.byref(mat), ctypes.byref(spec.c), n, h._dtype_code(F),
            ctypes.c_void_p(F.data_ptr()), ctypes.c_void_p(bn.data_ptr()), ctypes.c_void_p(W.data_ptr()),
            ctypes.c_void_p(P.data_ptr()), ctypes.c_void_p(T.data_ptr()), ctypes.c_void_p(fl.data_ptr()),
            ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 0, (st, r1.lib().r1_last_error(h.h))
    torch.cuda.synchronize()
    return W, P, T, fl


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("depth", [1, 2])
def test_noalloc_matches_envelope_stress(lib, dtype, depth):
    r1, h, torch = lib
    tdt = torch.float64 if dtype == "f64" else torch.float32
    mat = r1.material()
    if depth == 1:
        cases = [WL.small_random(2, 300, (4, 4), 201, tau=1.0, seed_tag=950),
                 WL.small_random(2, 70, (4, 2), 65, tau=1.2, seed_tag=951)]
    else:
        cases = [WL.small_random(2, 96, (4, 4), 33, tau=1.5, depth=2, inner=(4, 2, 65), seed_tag=952),
                 WL.small_random(2, 40, (2, 2), 17, tau=1.5, depth=2, inner=(4, 2, 33), seed_tag=953)]
    lib_ = r1.lib()
    for k, cfg in enumerate(cases):
        spec = r1.LaminationSpec(cfg["levels"])
        F = torch.tensor(cfg["F"], dtype=tdt, device="cuda").contiguous()
        bn = torch.tensor(cfg["beta_n"], dtype=tdt, device="cuda").contiguous()
        ref = _call(r1, h, torch, lib_.r1_envelope_stress, mat, spec, F, bn)
        got = _call(r1, h, torch, lib_.r1_envelope_stress_noalloc, mat, spec, F, bn)
        for name, a, b in zip(("W", "P", "tree", "flags"), ref, got):
            assert torch.equal(a, b), (dtype, depth, k, name)
        assert bool(torch.isfinite(got[0]).all())


def test_noalloc_rejects_requests_beyond_the_workspace(lib):
    r1, h, torch = lib
    mat = r1.material()
    n = 70000          # 70000 points x 64 outer directions x 16 B > 64 MiB
    a, b = WL.angle_directions(8, 8)
    ai, bi = WL.angle_directions(4, 2)
    spec = r1.LaminationSpec([WL.level(a, b, 33, 1.0), WL.level(ai, bi, 17, 1.0)])
    F = torch.zeros((4, n), dtype=torch.float32, device="cuda")
    bn = torch.zeros(n, dtype=torch.float32, device="cuda")
    W = torch.zeros(n, dtype=torch.float32, device="cuda")
    st = r1.lib().r1_envelope_stress_noalloc(h.h, ctypes.byref(mat), ctypes.byref(spec.c), n, r1.R1_F32,
                                             ctypes.c_void_p(F.data_ptr()), ctypes.c_void_p(bn.data_ptr()),
                                             ctypes.c_void_p(W.data_ptr()), None, None, None,
                                             ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == -1
    msg = r1.lib().r1_last_error(h.h).decode()
    assert "workspace" in msg and "67108864" in msg, msg
    assert float(W.abs().max()) == 0.0          # nothing launched
