"""Learned surrogate: GPU BF16-MFMA gradients against the FP64 network oracle,
fused inference against the oracle forward, training, error-gate calibration,
routing and fallback, persistence, and the gain over plain lamination."""
import os
import tempfile
import time

import numpy as np
import pytest

from oracle import oracle as O
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


def bf16_round(a):
    """Round FP32 values to BF16 (round to nearest even), as the matrix cores see them."""
    a = np.ascontiguousarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)


def hidden_blocks(d_in, width, n_hidden, d_out):
    """(start, end) of the width x width weight blocks in the flat layout."""
    out, o = [], width * d_in + width
    for _ in range(1, n_hidden):
        out.append((o, o + width * width))
        o += width * width + width
    return out


@pytest.mark.parametrize("dim,width", [(2, 32), (2, 128), (3, 256)])
def test_gradients_match_fp64_oracle(lib, dim, width):
    r1, h, torch = lib
    d = dim * dim + 1
    s = r1.Surrogate(h, dim=dim, n_hidden=4, width=width, seed=3)
    shape = (d, width, 4, d)
    rng = np.random.default_rng(9)
    params = s.get_params().astype(np.float64)
    # the matrix-core layers use BF16 weights: give the oracle the same weights
    p_bf = params.copy()
    for a, b in hidden_blocks(*shape):
        p_bf[a:b] = bf16_round(params[a:b])
    B = 128
    Xn = rng.normal(size=(B, d)).astype(np.float32)
    Yn = rng.normal(size=(B, d)).astype(np.float32)
    loss_g, g_g = s.loss_grad(torch.tensor(Xn, device="cuda"), torch.tensor(Yn, device="cuda"))
    g_g = g_g.cpu().numpy().astype(np.float64)
    loss_c, g_c = O.mlp_loss_grad(shape, p_bf, Xn.astype(np.float64), Yn.astype(np.float64))
    rel = np.linalg.norm(g_g - g_c) / np.linalg.norm(g_c)
    print("dim %d width %d: loss gpu %.6f cpu %.6f, gradient rel err %.3e" % (dim, width, loss_g, loss_c, rel))
    assert abs(loss_g - loss_c) <= 1e-2 * abs(loss_c)
    assert rel < 2e-2
    # every layer's gradient points the same way
    offs = [0]
    for l in range(5):
        n_in = d if l == 0 else width
        n_out = d if l == 4 else width
        offs.append(offs[-1] + n_out * n_in + n_out)
    for l in range(5):
        a, b = offs[l], offs[l + 1]
        cos = g_g[a:b] @ g_c[a:b] / (np.linalg.norm(g_g[a:b]) * np.linalg.norm(g_c[a:b]))
        assert cos > 0.999, (l, cos)
    s.close()


def laminate(lib, F, bn, levels, dt):
    r1, h, torch = lib
    mat = r1.material()
    spec = r1.LaminationSpec(levels)
    Ft = torch.tensor(F, dtype=dt, device="cuda").contiguous()
    bt = torch.tensor(bn, dtype=dt, device="cuda").contiguous()
    out = h.envelope(mat, spec, Ft, bt, stress=True)
    torch.cuda.synchronize()
    return Ft, bt, out


@pytest.fixture(scope="module")
def trained(lib):
    """A 2D network trained on 131,072 rows of config-1-style lamination data."""
    r1, h, torch = lib
    cfg = WL.config4_training(n=131072, seed_tag=60)
    Ft, bt, out = laminate(lib, cfg["F"], cfg["beta_n"], cfg["levels"], torch.float32)
    s = r1.Surrogate(h, dim=2, n_hidden=4, width=128, seed=1)
    X, Y = s.pack(Ft, bt, out["W"], out["P"])
    mat = r1.material()
    rep1 = s.train(mat, X, Y, epochs=1, batch=4096, lr=2e-3, seed=1)
    rep = s.train(mat, X, Y, epochs=150, batch=4096, lr=2e-3, seed=2)
    print("training: 1 epoch loss %.4e / val %.4e; +150 epochs loss %.4e / val %.4e (%d steps, %.0f ms)" % (
        rep1["train_loss"], rep1["val_loss"], rep["train_loss"], rep["val_loss"], rep["steps"], rep["ms"]))
    cal = WL.config4_training(n=65536, seed_tag=61)
    Fc, bc, oc = laminate(lib, cal["F"], cal["beta_n"], cal["levels"], torch.float32)
    Xc, Yc = s.pack(Fc, bc, oc["W"], oc["P"])
    allowed = s.calibrate(mat, Xc, Yc, tol=1e-3, quantile=0.99)
    print("calibration: %d of %d gate cells with a threshold" % (allowed, 16 * 8))
    yield s, rep1, rep, allowed, cfg["levels"]
    s.close()


def test_training_reduces_loss(trained):
    s, rep1, rep, allowed, _ = trained
    assert rep["val_loss"] < 0.5 * rep1["val_loss"]
    assert rep["train_loss"] < 0.5 * rep1["train_loss"]
    assert allowed > 0


def test_inference_matches_oracle_forward(lib, trained):
    """Points the gates accept: the fused BF16 inference equals the FP64 network oracle's
    forward on the same (standardized) inputs, mapped back through W(F) and P0(F)."""
    r1, h, torch = lib
    s, _, _, _, levels = trained
    cfg = WL.config4_training(n=4096, seed_tag=62)
    F, bn = cfg["F"], cfg["beta_n"]
    Ft = torch.tensor(F, dtype=torch.float32, device="cuda").contiguous()
    bt = torch.tensor(bn, dtype=torch.float32, device="cuda").contiguous()
    out = s.infer(r1.material(), r1.LaminationSpec(levels), Ft, bt)
    torch.cuda.synchronize()
    fl = out["flags"].cpu().numpy()
    ok = np.nonzero((fl & r1.PT_FALLBACK) == 0)[0][:256]
    assert len(ok) > 50
    nm = s.norm()
    params = s.get_params().astype(np.float64)
    Fi, bi = Ft.double().cpu().numpy(), bt.double().cpu().numpy()
    x = np.concatenate([Fi[:, ok].T, bi[ok, None]], axis=1)
    xn = (x.astype(np.float32) - nm["x_mean"]) / nm["x_std"]
    y, _ = O.mlp_forward((5, 128, 4, 5), params, xn.astype(np.float64))
    y = y * nm["y_std"] + nm["y_mean"]
    om = O.material(dim=2)
    lam = y[:, 0] > 0                  # a non-positive gap means no lamination: W(F), P0(F)
    W_ref = np.array([O.energy(om, Fi[:, p].reshape(2, 2), bi[p]) for p in ok]) - np.where(lam, y[:, 0], 0)
    P_ref = np.array([O.stress0(om, Fi[:, p].reshape(2, 2), bi[p]).ravel() for p in ok]) - \
        np.where(lam[:, None], y[:, 1:], 0)
    Wg = out["W"].cpu().numpy()[ok]
    Pg = out["P"].cpu().numpy()[:, ok].T
    # BF16 activations/weights: errors of a few BF16 ulps of the standardized outputs;
    # points near the no-lamination switch may fall on either side of it
    near = np.abs(y[:, 0]) < 0.02 * nm["y_std"][0]
    far = ~near
    assert far.sum() > 40
    assert np.max(np.abs(Wg - W_ref)[far]) < 0.02 * nm["y_std"][0] + 1e-6
    assert np.max(np.abs(Pg - P_ref)[far]) < 0.02 * np.max(nm["y_std"][1:]) + 1e-6


def test_routing_fallback_and_accuracy(lib, trained):
    """Inference points from the inference distribution (beta_n up to 1.1, a wider F
    spread): out-of-box points fall back and equal plain lamination exactly; accepted
    points are within the calibrated 1e-3 relative energy error of plain lamination."""
    r1, h, torch = lib
    s, _, _, _, levels = trained
    cfg = WL.config4_inference(n=32768, seed_tag=63)
    Ft, bt, plain = laminate(lib, cfg["F"], cfg["beta_n"], levels, torch.float32)
    out = s.infer(r1.material(), r1.LaminationSpec(levels), Ft, bt)
    torch.cuda.synchronize()
    fl = out["flags"].cpu().numpy()
    fb = (fl & r1.PT_FALLBACK) != 0
    assert out["n_fallback"] == int(fb.sum())
    Wp, Pp = plain["W"].cpu().numpy(), plain["P"].cpu().numpy()
    Wg, Pg = out["W"].cpu().numpy(), out["P"].cpu().numpy()
    assert np.array_equal(Wg[fb], Wp[fb]) and np.array_equal(Pg[:, fb], Pp[:, fb])
    bi = bt.cpu().numpy()
    assert np.all(fb[bi > 1.0])                     # beta_n outside the training range
    acc = ~fb
    err = np.abs(Wg[acc] - Wp[acc]) / np.maximum(np.abs(Wp[acc]), 1e-2)
    print("fallback %.1f%%, accepted: max rel err %.2e, p99 %.2e, frac > 1e-3: %.4f" % (
        100 * fb.mean(), err.max(), np.percentile(err, 99), np.mean(err > 1e-3)))
    assert acc.sum() > 0.2 * len(fl)
    assert np.mean(err > 1e-3) < 0.01
    assert np.all(Wg[acc] <= (Wp[acc] + 1e-2 * np.maximum(np.abs(Wp[acc]), 1e-2)) + 1.0)  # finite, sane


def test_save_load_roundtrip(lib, trained):
    r1, h, torch = lib
    s, _, _, _, levels = trained
    cfg = WL.config4_inference(n=2048, seed_tag=64)
    Ft = torch.tensor(cfg["F"], dtype=torch.float32, device="cuda").contiguous()
    bt = torch.tensor(cfg["beta_n"], dtype=torch.float32, device="cuda").contiguous()
    a = s.infer(r1.material(), r1.LaminationSpec(levels), Ft, bt)
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "s.r1s")
        s.save(path)
        s2 = r1.Surrogate.load(h, path)
        b = s2.infer(r1.material(), r1.LaminationSpec(levels), Ft, bt)
        torch.cuda.synchronize()
        s2.close()
    assert torch.equal(a["W"], b["W"]) and torch.equal(a["P"], b["P"]) and torch.equal(a["flags"], b["flags"])


def test_surrogate_gain_over_plain_lamination(lib, trained):
    """The trained network with routing answers the same points faster than plain
    lamination of the same configuration on the same GPU."""
    r1, h, torch = lib
    s, _, _, _, levels = trained
    cfg = WL.config4_inference(n=262144, seed_tag=65)
    Ft = torch.tensor(cfg["F"], dtype=torch.float32, device="cuda").contiguous()
    bt = torch.tensor(cfg["beta_n"], dtype=torch.float32, device="cuda").contiguous()
    mat = r1.material()
    spec = r1.LaminationSpec(levels)
    n = Ft.shape[1]
    W = torch.empty(n, device="cuda")
    P = torch.empty((4, n), device="cuda")
    out = s.infer(mat, spec, Ft, bt)
    h.envelope_into(mat, spec, Ft, bt, W, P)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        h.envelope_into(mat, spec, Ft, bt, W, P)
    torch.cuda.synchronize()
    t_plain = (time.perf_counter() - t0) / 3
    t0 = time.perf_counter()
    for _ in range(3):
        out = s.infer(mat, spec, Ft, bt, out=out)
    torch.cuda.synchronize()
    t_sur = (time.perf_counter() - t0) / 3
    print("plain %.3f ms, surrogate %.3f ms (fallback %.1f%%): speedup %.2fx" % (
        1e3 * t_plain, 1e3 * t_sur, 100 * out["n_fallback"] / n, t_plain / t_sur))
    assert t_sur < t_plain


@pytest.mark.parametrize("width", [128, 256])
def test_3d_inference_matches_oracle_forward(lib, width):
    """3D network (inputs: 9 F entries and beta_n): after a short training on 3D
    lamination data, uncalibrated inference (box gate only) equals the FP64 network
    oracle's forward mapped through W(F) and P0(F).  Width 128 runs the kernel with
    LDS-resident weights, width 256 the one that reads them from L2."""
    r1, h, torch = lib
    cfg = WL.config5(n=16384)
    lv = cfg["levels"][0]
    lv = dict(lv, a=lv["a"][:64], b=lv["b"][:64], n_t=129)
    mat = r1.material(dim=3)
    spec = r1.LaminationSpec([lv])
    Ft = torch.tensor(cfg["F"], dtype=torch.float32, device="cuda").contiguous()
    bt = torch.tensor(cfg["beta_n"], dtype=torch.float32, device="cuda").contiguous()
    out = h.envelope(mat, spec, Ft, bt, stress=True)
    s = r1.Surrogate(h, dim=3, n_hidden=4, width=width, seed=5)
    X, Y = s.pack(Ft, bt, out["W"], out["P"])
    rep = s.train(mat, X, Y, epochs=4, batch=1024, lr=1e-3, seed=1)
    assert np.isfinite(rep["val_loss"])
    inf = WL.config5(n=2048)
    Fi = torch.tensor(inf["F"], dtype=torch.float32, device="cuda").contiguous()
    bi = torch.tensor(inf["beta_n"], dtype=torch.float32, device="cuda").contiguous()
    res = s.infer(mat, spec, Fi, bi)
    torch.cuda.synchronize()
    fl = res["flags"].cpu().numpy()
    ok = np.nonzero((fl & r1.PT_FALLBACK) == 0)[0][:256]
    assert len(ok) > 100
    nm = s.norm()
    params = s.get_params().astype(np.float64)
    Fn, bn = Fi.double().cpu().numpy(), bi.double().cpu().numpy()
    x = np.concatenate([Fn[:, ok].T, bn[ok, None]], axis=1)
    xn = (x.astype(np.float32) - nm["x_mean"]) / nm["x_std"]
    y, _ = O.mlp_forward((10, width, 4, 10), params, xn.astype(np.float64))
    y = y * nm["y_std"] + nm["y_mean"]
    om = O.material(dim=3)
    lam = y[:, 0] > 0
    W_ref = np.array([O.energy(om, Fn[:, p].reshape(3, 3), bn[p]) for p in ok]) - np.where(lam, y[:, 0], 0)
    P_ref = np.array([O.stress0(om, Fn[:, p].reshape(3, 3), bn[p]).ravel() for p in ok]) - \
        np.where(lam[:, None], y[:, 1:], 0)
    Wg = res["W"].cpu().numpy()[ok]
    Pg = res["P"].cpu().numpy()[:, ok].T
    near = np.abs(y[:, 0]) < 0.02 * nm["y_std"][0]
    far = ~near
    err_w = np.max(np.abs(Wg - W_ref)[far])
    err_p = np.max(np.abs(Pg - P_ref)[far])
    print("3d width %d: %d accepted points, max |dW| %.2e, max |dP| %.2e (y_std %.2e)" % (
        width, far.sum(), err_w, err_p, nm["y_std"][0]))
    assert far.sum() > 80
    assert err_w < 0.02 * nm["y_std"][0] + 1e-6
    assert err_p < 0.02 * np.max(nm["y_std"][1:]) + 1e-6
    s.close()
