"""The depth-2 workload at its full size (4096 points, 2D; outer level 64 directions
x 1025 points, inner level 32 x 257, tau 1.5), in the launch that bench.py times
(r1_envelope_stress with stress, tree and flags), against the FP64 oracle through a
transfer standard:
  - GPU FP64 against the oracle's stored values (tests/golden/config2_oracle_f64.json,
    written by make_oracle_golden.py from the oracle alone) at 64 seeded points:
    energy to 1e-12, the same tree and stress to 1e-10 where the oracle's laminate
    is unambiguous, the GPU's tree evaluated by the oracle at ties;
  - GPU FP32 against GPU FP64 at every point: energy to 1e-5; the same tree, or
    else a tree whose oracle energy (Algorithm 3) is within 1e-5 of the FP64 W
    (an optimal laminate to FP32 accuracy) and whose oracle stress is the FP32 P;
  - GPU FP32 against the oracle's stored values at 32 of those points, FP32-rounded
    inputs (config2_oracle_f32in.json);
  - every point: Algorithm 3 on the FP32 tree gives the FP32 W, P (1e-5 / 2e-5) and
    the tangent moduli of that tree, and W <= W(F).
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2211_14318_amd import workloads as WL
from tests import parity as PA

pytestmark = pytest.mark.gpu


def _run(r1, h, torch, cfg, dt, tangent=False):
    n = cfg["n"]
    mat = r1.material_from(cfg["material"], 2)
    spec = r1.LaminationSpec(cfg["levels"])
    F = torch.tensor(cfg["F"], dtype=dt, device="cuda").contiguous()
    bn = torch.tensor(cfg["beta_n"], dtype=dt, device="cuda").contiguous()
    W = torch.empty(n, dtype=dt, device="cuda")
    P = torch.empty((4, n), dtype=dt, device="cuda")
    T = torch.empty((n, 3, 4), dtype=torch.int32, device="cuda")
    fl = torch.empty(n, dtype=torch.int32, device="cuda")
    h.envelope_into(mat, spec, F, bn, W, P, T, fl)
    A = h.laminate_tangent(mat, spec, F, bn, W, T) if tangent else None
    torch.cuda.synchronize()
    return dict(W=W.double().cpu().numpy(), P=P.double().cpu().numpy(), tree=T.cpu().numpy(),
                flags=fl.cpu().numpy(), A=A.double().cpu().numpy() if tangent else None,
                F=F.double().cpu().numpy(), bn=bn.double().cpu().numpy())


@pytest.fixture(scope="module")
def runs():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2211_14318_amd import r1
    h = r1.Handle(0)
    cfg = WL.config2()
    g32 = _run(r1, h, torch, cfg, torch.float32, tangent=True)
    g64 = _run(r1, h, torch, cfg, torch.float64)
    yield cfg, g32, g64
    h.close()


def _nodes(tree_row):
    return [tuple(int(x) for x in tree_row[k, :3]) for k in range(3)]


def test_full_size_fp64_against_stored_oracle(runs):
    cfg, _, g = runs
    hdr, pts = PA.load_oracle_golden("config2_oracle_f64.json")
    assert hdr["workload"] == cfg["name"] and len(pts) == 64
    sel = np.array([q["p"] for q in pts])
    F, bn, W, P, trees = PA.golden_arrays(pts)
    assert np.array_equal(F, cfg["F"][:, sel]) and np.array_equal(bn, cfg["beta_n"][sel])
    err = PA.energy_errors(g["W"][sel], W, "f64")
    print("FP64 at 64 stored oracle points: max energy error %.2e" % err.max())
    assert err.max() <= PA.RTOL["f64"]
    om, ospec = PA.orc_material(cfg["material"], 2), PA.orc_spec(cfg["levels"])
    st = {}
    ne, nt = PA.check_stress(om, ospec, 2, F, bn, W, P, trees, g["P"][:, sel], g["tree"][sel], "f64", st)
    print("   stress: %d exact, %d tie-checked (tree energy within %.2e)" % (ne, nt, st.get("tie_w", 0.0)))
    assert ne >= 60


def test_full_size_fp32_against_fp64_every_point(runs):
    """The transfer standard: FP32 against the GPU's FP64 result at all 4096 points."""
    cfg, g32, g64 = runs
    n = cfg["n"]
    assert np.all(np.isfinite(g64["W"])) and np.all((g64["flags"] & 3) == 0)
    err = PA.energy_errors(g32["W"], g64["W"], "f32")
    print("FP32 vs FP64, %d points: max energy error %.2e, p99 %.2e" % (n, err.max(), np.percentile(err, 99)))
    assert err.max() <= PA.RTOL["f32"]
    om, ospec = PA.orc_material(cfg["material"], 2), PA.orc_spec(cfg["levels"])
    same = np.all(g32["tree"][:, :, :3] == g64["tree"][:, :, :3], axis=(1, 2))
    worst_p = 0.0
    for p in np.nonzero(same)[0]:
        sc = max(np.max(np.abs(g64["P"][:, p])), 1.0)
        worst_p = max(worst_p, np.max(np.abs(g32["P"][:, p] - g64["P"][:, p])) / sc)
    assert worst_p <= PA.PTOL["f32"], worst_p
    n_other = 0
    for p in np.nonzero(~same)[0]:
        n_other += 1
        Fp = g32["F"][:, p].reshape(2, 2)
        We, Pe = O.eval_tree(om, ospec, Fp, g32["bn"][p], _nodes(g32["tree"][p]))
        scale = max(abs(g64["W"][p]), PA.W_FLOOR["f32"])
        assert abs(We - g64["W"][p]) <= PA.RTOL["f32"] * scale, (p, We, g64["W"][p])
        sc = max(np.max(np.abs(Pe)), 1.0)
        assert np.max(np.abs(Pe.ravel() - g32["P"][:, p])) <= PA.PTOL["f32"] * sc, (p, Pe, g32["P"][:, p])
    print("   same tree at %d points (stress within %.2e), another optimal laminate at %d"
          % (int(same.sum()), worst_p, n_other))



def test_full_size_fp32_against_stored_oracle(runs):
    cfg, g, _ = runs
    hdr, pts = PA.load_oracle_golden("config2_oracle_f32in.json")
    assert hdr["workload"] == cfg["name"] and len(pts) == 32
    sel = np.array([q["p"] for q in pts])
    F, bn, W, P, trees = PA.golden_arrays(pts)
    assert np.array_equal(F, g["F"][:, sel]) and np.array_equal(bn, g["bn"][sel])
    err = PA.energy_errors(g["W"][sel], W, "f32")
    print("FP32 at 32 stored oracle points: max energy error %.2e" % err.max())
    assert err.max() <= PA.RTOL["f32"]
    om, ospec = PA.orc_material(cfg["material"], 2), PA.orc_spec(cfg["levels"])
    st = {}
    ne, nt = PA.check_stress(om, ospec, 2, F, bn, W, P, trees, g["P"][:, sel], g["tree"][sel], "f32", st)
    print("   stress: %d exact, %d tie-checked (tree energy within %.2e)" % (ne, nt, st.get("tie_w", 0.0)))
    assert ne + nt == len(pts)


def test_full_size_tree_consistency(runs):
    """Every point: the FP32 W, P and tangent moduli are Algorithm 3 on the FP32 tree."""
    cfg, g, _ = runs
    om, ospec = PA.orc_material(cfg["material"], 2), PA.orc_spec(cfg["levels"])
    n = cfg["n"]
    assert np.all(np.isfinite(g["W"])) and np.all((g["flags"] & 3) == 0)
    worst_w = worst_p = worst_a = 0.0
    for p in range(n):
        Fp = g["F"][:, p].reshape(2, 2)
        We, Pe, Ae = O.eval_tree_tangent(om, ospec, Fp, g["bn"][p], _nodes(g["tree"][p]))
        w0 = O.energy(om, Fp, g["bn"][p])
        scale = max(abs(We), PA.W_FLOOR["f32"])
        assert g["W"][p] <= w0 + PA.RTOL["f32"] * max(abs(w0), PA.W_FLOOR["f32"]), (p, g["W"][p], w0)
        ew = abs(g["W"][p] - We) / scale
        ep = np.max(np.abs(g["P"][:, p] - Pe.ravel())) / max(np.max(np.abs(Pe)), 1.0)
        ea = np.max(np.abs(g["A"][:, p] - Ae.ravel())) / max(np.max(np.abs(Ae)), 1.0)
        worst_w, worst_p, worst_a = max(worst_w, ew), max(worst_p, ep), max(worst_a, ea)
        assert ew <= PA.RTOL["f32"], (p, g["W"][p], We)
        assert ep <= PA.PTOL["f32"], (p, g["P"][:, p], Pe)
        assert ea <= 1e-6, (p, g["A"][:, p], Ae)
    print("tree consistency over %d points: W %.2e, P %.2e, A %.2e (relative)" % (n, worst_w, worst_p, worst_a))
