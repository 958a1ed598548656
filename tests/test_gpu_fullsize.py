"""The headline workload at its full size (4096 points, 2D, FP32; outer level 64
directions x 1025 points, inner level 32 x 257, depth 2), in the launch that
bench.py times (r1_envelope_stress with stress, tree and flags), against the FP64
oracle:
  - every point: the oracle's Algorithm 3 on the GPU's tree gives the GPU's W (so
    W is the energy of a laminate on the grid: an upper bound of W^2 that the
    grid attains) and its stress P, and W <= W(F);
  - every point: the tangent moduli of that tree (r1_laminate_tangent) equal the
    oracle's Algorithm 3 moduli on the same tree;
  - sampled points: the oracle's full two-level envelope (about a minute of CPU per
    point, run in a process pool): W within the FP32 bar, and where the laminate
    is unambiguous the same tree and stress.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2211_14318_amd import workloads as WL
from tests import parity as PA

pytestmark = pytest.mark.gpu

N_SAMPLED = 6


@pytest.fixture(scope="module")
def headline():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2211_14318_amd import r1
    h = r1.Handle(0)
    cfg = WL.config2()
    n = cfg["n"]
    dt = torch.float32
    mat = r1.material_from(cfg["material"], 2)
    spec = r1.LaminationSpec(cfg["levels"])
    F = torch.tensor(cfg["F"], dtype=dt, device="cuda").contiguous()
    bn = torch.tensor(cfg["beta_n"], dtype=dt, device="cuda").contiguous()
    W = torch.empty(n, dtype=dt, device="cuda")
    P = torch.empty((4, n), dtype=dt, device="cuda")
    T = torch.empty((n, 3, 4), dtype=torch.int32, device="cuda")
    fl = torch.empty(n, dtype=torch.int32, device="cuda")
    h.envelope_into(mat, spec, F, bn, W, P, T, fl)
    A = h.laminate_tangent(mat, spec, F, bn, W, T)
    torch.cuda.synchronize()
    g = dict(W=W.double().cpu().numpy(), P=P.double().cpu().numpy(), tree=T.cpu().numpy(),
             flags=fl.cpu().numpy(), A=A.double().cpu().numpy(),
             F=F.double().cpu().numpy(), bn=bn.double().cpu().numpy())
    yield cfg, g
    h.close()


def test_full_size_tree_consistency(headline):
    cfg, g = headline
    om, ospec = PA.orc_material(cfg["material"], 2), PA.orc_spec(cfg["levels"])
    n = cfg["n"]
    assert np.all(np.isfinite(g["W"])) and np.all((g["flags"] & 3) == 0)
    worst_w = worst_p = worst_a = 0.0
    for p in range(n):
        Fp = g["F"][:, p].reshape(2, 2)
        nodes = [tuple(int(x) for x in g["tree"][p, k, :3]) for k in range(3)]
        We, Pe, Ae = O.eval_tree_tangent(om, ospec, Fp, g["bn"][p], nodes)
        w0 = O.energy(om, Fp, g["bn"][p])
        scale = max(abs(We), PA.W_FLOOR["f32"])
        assert g["W"][p] <= w0 + PA.RTOL["f32"] * max(abs(w0), PA.W_FLOOR["f32"]), (p, g["W"][p], w0)
        ew = abs(g["W"][p] - We) / scale
        ep = np.max(np.abs(g["P"][:, p] - Pe.ravel())) / max(np.max(np.abs(Pe)), 1.0)
        ea = np.max(np.abs(g["A"][:, p] - Ae.ravel())) / max(np.max(np.abs(Ae)), 1.0)
        worst_w, worst_p, worst_a = max(worst_w, ew), max(worst_p, ep), max(worst_a, ea)
        assert ew <= 10 * PA.RTOL["f32"], (p, g["W"][p], We)
        assert ep <= PA.PTOL["f32"], (p, g["P"][:, p], Pe)
        assert ea <= 1e-6, (p, g["A"][:, p], Ae)
    print("tree consistency over %d points: W %.2e, P %.2e, A %.2e (relative)" % (n, worst_w, worst_p, worst_a))


@pytest.mark.timeout(900)
def test_full_size_sampled_oracle(headline):
    cfg, g = headline
    rng = np.random.default_rng(20221128)
    sel = np.sort(rng.choice(cfg["n"], N_SAMPLED, replace=False))
    W, P, trees = PA.oracle_pool_map(cfg["material"], 2, cfg["levels"], g["F"][:, sel].copy(),
                                     g["bn"][sel].copy(), workers=N_SAMPLED)
    err = PA.energy_errors(g["W"][sel], W, "f32")
    print("sampled points %s: W rel err %s" % (sel.tolist(), np.array2string(err, precision=2)))
    assert err.max() <= PA.RTOL["f32"]
    om, ospec = PA.orc_material(cfg["material"], 2), PA.orc_spec(cfg["levels"])
    ne, nt = PA.check_stress(om, ospec, 2, g["F"][:, sel], g["bn"][sel], W, P, trees,
                             g["P"][:, sel], g["tree"][sel], "f32")
    print("   stress: %d exact, %d tie-checked" % (ne, nt))
