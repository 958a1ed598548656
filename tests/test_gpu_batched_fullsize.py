"""The uneven batch at its full size (65,536 2D points; per point n_t in {257, 513,
1025, 2049}, 32/64/128 directions, depth 1 or 2 with an inner level of 32 x 257),
FP32, through the plan and the autotuned layouts that bench.py times:
  - 2 stored oracle points of every one of the 24 table entries
    (tests/golden/config3_oracle_f32in.json, written by make_oracle_golden.py from
    the oracle alone, at the FP32-rounded inputs the GPU reads): energy to 1e-5, the
    same tree and stress where the oracle's laminate is unambiguous, the GPU's tree
    evaluated by the oracle at ties;
  - every point: Algorithm 3 on the GPU's tree gives the GPU's W and P, and
    W <= W(F).
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2211_14318_amd import workloads as WL
from tests import parity as PA

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def batch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2211_14318_amd import r1
    h = r1.Handle(0)
    cfg = WL.config3()
    mat = r1.material()
    specs = [r1.LaminationSpec(t) for t in cfg["table"]]
    F = torch.tensor(cfg["F"], dtype=torch.float32, device="cuda")
    bn = torch.tensor(cfg["beta_n"], dtype=torch.float32, device="cuda")
    idx = torch.tensor(cfg["lam_idx"], dtype=torch.int32, device="cuda")
    plan = h.batched_plan(mat, specs, idx, torch.float32)
    o = plan.outputs(stress=True, tree=True)
    plan.execute(F, bn, o["W"], o["P"], o["tree"], o["flags"])
    torch.cuda.synchronize()
    lanes = {nt: (h.segment_width(nt, r1.R1_F32, 2), h.inner_segment_width(nt, r1.R1_F32, 2))
             for nt in WL.BATCH_NT}
    g = dict(W=o["W"].double().cpu().numpy(), P=o["P"].double().cpu().numpy(), tree=o["tree"].cpu().numpy(),
             flags=o["flags"].cpu().numpy(), F=F.double().cpu().numpy(), bn=bn.double().cpu().numpy())
    plan.close()
    print("tuned lanes per line (one-level, inner) by grid size:", lanes)
    yield cfg, g
    h.close()


def test_batched_full_size_against_stored_oracle(batch):
    cfg, g = batch
    hdr, pts = PA.load_oracle_golden("config3_oracle_f32in.json")
    assert hdr["workload"] == cfg["name"]
    entries = np.array([q["entry"] for q in pts])
    assert sorted(set(entries.tolist())) == list(range(len(cfg["table"])))
    assert np.all(np.bincount(entries) >= 2)
    om = PA.orc_material(cfg["material"], 2)
    worst = 0.0
    n_exact = n_tie = 0
    st = {}
    for k, lv in enumerate(cfg["table"]):
        sub = [q for q in pts if q["entry"] == k]
        sel = np.array([q["p"] for q in sub])
        assert np.all(cfg["lam_idx"][sel] == k)
        F, bn, W, P, trees = PA.golden_arrays(sub)
        assert np.array_equal(F, g["F"][:, sel]) and np.array_equal(bn, g["bn"][sel])
        err = PA.energy_errors(g["W"][sel], W, "f32")
        worst = max(worst, err.max())
        assert err.max() <= PA.RTOL["f32"], (k, err)
        ne, nt = PA.check_stress(om, PA.orc_spec(lv), len(lv), F, bn, W, P, trees, g["P"][:, sel],
                                 g["tree"][sel], "f32", st)
        n_exact += ne
        n_tie += nt
    print("uneven batch, %d stored points over %d entries: max energy error %.2e; stress %d exact, %d tie-checked"
          " (tree energy within %.2e)" % (len(pts), len(cfg["table"]), worst, n_exact, n_tie, st.get("tie_w", 0.0)))
    assert n_exact + n_tie == len(pts)


def test_batched_full_size_tree_consistency(batch):
    cfg, g = batch
    om = PA.orc_material(cfg["material"], 2)
    specs = [PA.orc_spec(lv) for lv in cfg["table"]]
    assert np.all(np.isfinite(g["W"])) and np.all((g["flags"] & 3) == 0)
    worst_w = worst_p = 0.0
    for p in range(cfg["n"]):
        k = int(cfg["lam_idx"][p])
        depth = len(cfg["table"][k])
        Fp = g["F"][:, p].reshape(2, 2)
        nodes = [tuple(int(x) for x in g["tree"][p, j, :3]) for j in range(3 if depth == 2 else 1)]
        nodes += [(0, 0, 0)] * (3 - len(nodes))
        We, Pe = O.eval_tree(om, specs[k], Fp, g["bn"][p], nodes)
        w0 = O.energy(om, Fp, g["bn"][p])
        scale = max(abs(We), PA.W_FLOOR["f32"])
        assert g["W"][p] <= w0 + PA.RTOL["f32"] * max(abs(w0), PA.W_FLOOR["f32"]), (p, g["W"][p], w0)
        ew = abs(g["W"][p] - We) / scale
        ep = np.max(np.abs(g["P"][:, p] - Pe.ravel())) / max(np.max(np.abs(Pe)), 1.0)
        worst_w, worst_p = max(worst_w, ew), max(worst_p, ep)
        assert ew <= PA.RTOL["f32"], (p, k, g["W"][p], We)
        assert ep <= PA.PTOL["f32"], (p, k, g["P"][:, p], Pe)
    print("tree consistency over %d points: W %.2e, P %.2e (relative)" % (cfg["n"], worst_w, worst_p))
