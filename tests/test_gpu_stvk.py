"""St. Venant-Kirchhoff damage model (eq. 2.2 in eq. 2.9) on the GPU against the FP64
oracle, through the C-ABI: plain lamination at depth 1 and 2 in 2D and 3D, points
with det F <= 0 (admissible for this energy), tangent moduli, the uneven batch and
the surrogate's exact-energy epilogue.  Material: Table 6.3's STVK row."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2211_14318_amd import workloads as WL
from tests import parity as PA
from tests import test_gpu_parity as GP
from tests import test_gpu_tangent as GT

pytestmark = pytest.mark.gpu

STVK = 2
MAT = dict(mu=1.0, lam=0.5, D_inf=0.9, D0=0.3)


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2211_14318_amd import r1
    h = r1.Handle(0)
    yield r1, h, torch
    h.close()


def stvk_cfg(**kw):
    cfg = WL.small_random(**kw)
    cfg["material"] = MAT
    return cfg


@pytest.mark.parametrize("kind", ["f64", "f32"])
def test_stvk_depth1_2d(lib, kind):
    cfg = stvk_cfg(dim=2, n=64, n_dir_ab=(4, 4), n_t=201, tau=1.0, seed_tag=600)
    g, W = GP.check_case(lib, cfg, kind, model=STVK, min_exact=40)
    assert np.all(np.isfinite(g["W"])) and np.all(g["flags"] & 3 == 0)


@pytest.mark.parametrize("kind", ["f64", "f32"])
def test_stvk_depth1_3d(lib, kind):
    cfg = stvk_cfg(dim=3, n=19, n_dir_ab=(4, 4), n_t=65, tau=1.0, seed_tag=601, sigma=0.2, det_min=0.2)
    GP.check_case(lib, cfg, kind, model=STVK, min_exact=8)


@pytest.mark.parametrize("kind", ["f64", "f32"])
def test_stvk_depth2_2d(lib, kind):
    cfg = stvk_cfg(dim=2, n=24, n_dir_ab=(4, 4), n_t=65, tau=1.5, depth=2, inner=(4, 2, 33), seed_tag=602)
    GP.check_case(lib, cfg, kind, model=STVK, min_exact=10)


def test_stvk_depth2_3d(lib):
    cfg = stvk_cfg(dim=3, n=6, n_dir_ab=(2, 2), n_t=17, tau=1.0, depth=2, inner=(2, 2, 9), seed_tag=603,
                   sigma=0.2, det_min=0.2)
    GP.check_case(lib, cfg, "f64", model=STVK, min_exact=2)


@pytest.mark.parametrize("depth", [1, 2])
def test_stvk_det_le_0_points(lib, depth):
    """det F <= 0 is admissible for St. Venant-Kirchhoff: W, P and the tree are those of
    the oracle, no point is flagged, and lines through such points cross det = 0."""
    r1 = lib[0]
    F = np.array([[1.0, 0.0, 0.0, -0.5], [0.0, 0.0, 0.0, 0.0], [-1.1, 0.2, 0.1, 0.9],
                  [0.3, 0.8, 0.8, 0.3], [1.2, 0.1, 0.0, 0.95]]).T.copy()
    a, b = WL.angle_directions(4, 4)
    levels = [WL.level(a, b, 41, 1.5)]
    if depth == 2:
        ai, bi = WL.angle_directions(4, 2)
        levels.append(WL.level(ai, bi, 21, 1.5))
    cfg = dict(name="stvk-det", dim=2, material=MAT, F=F, beta_n=np.array([0.0, 0.05, 0.1, 0.2, 0.0]),
               levels=levels)
    assert np.sum(np.linalg.det(F.T.reshape(-1, 2, 2)) <= 0) == 4
    g, W = GP.check_case(lib, cfg, "f64", model=STVK, min_exact=3)
    assert np.all(np.isfinite(g["W"])) and np.all(g["flags"] & (r1.PT_DETLE0 | r1.PT_NONFINITE) == 0)


@pytest.mark.parametrize("kind,dim,depth", [("f64", 2, 1), ("f32", 2, 2), ("f64", 3, 1)])
def test_stvk_tangent(lib, kind, dim, depth):
    if dim == 2:
        cfg = stvk_cfg(dim=2, n=32, n_dir_ab=(4, 4), n_t=65, tau=1.5, depth=depth, inner=(4, 2, 33),
                       seed_tag=604 + depth)
    else:
        cfg = stvk_cfg(dim=3, n=12, n_dir_ab=(3, 3), n_t=33, tau=1.0, seed_tag=606, sigma=0.2, det_min=0.2)
    GT.check_tangent_case(lib, cfg, kind, model=STVK, min_exact=5)


@pytest.mark.parametrize("kind", ["f64", "f32"])
def test_stvk_batched_against_oracle(lib, kind):
    """The uneven persistent batch with St. Venant-Kirchhoff kernels: per-point oracle parity
    over depth-1 and depth-2 table entries."""
    r1, h, torch = lib
    table = []
    for nt in (33, 65):
        for na, nb in ((4, 2), (5, 3)):
            a, b = WL.angle_directions(na, nb)
            table.append([WL.level(a, b, nt, 1.0)])
    ai, bi = WL.angle_directions(4, 2)
    a, b = WL.angle_directions(4, 4)
    table.append([WL.level(a, b, 17, 1.2), WL.level(ai, bi, 17, 1.2)])
    rng = np.random.default_rng(607)
    cfg = WL.small_random(2, 60, (1, 1), 3, seed_tag=607)
    idx = rng.integers(0, len(table), size=60).astype(np.int32)
    dt = torch.float64 if kind == "f64" else torch.float32
    mat = r1.material_from(MAT, 2, STVK)
    Ft = torch.tensor(cfg["F"], dtype=dt, device="cuda").contiguous()
    bt = torch.tensor(cfg["beta_n"], dtype=dt, device="cuda").contiguous()
    out = h.envelope_batched(mat, [r1.LaminationSpec(t) for t in table], torch.tensor(idx, device="cuda"),
                             Ft, bt, stress=True, tree=True)
    torch.cuda.synchronize()
    g = {k: (v.cpu().numpy() if v is not None else None) for k, v in out.items()}
    Fin, bin_ = Ft.double().cpu().numpy(), bt.double().cpu().numpy()
    om = PA.orc_material(MAT, 2, STVK)
    n_exact = 0
    for k, lv in enumerate(table):
        sel = np.nonzero(idx == k)[0]
        if len(sel) == 0:
            continue
        spec = PA.orc_spec(lv)
        W, P, trees = O.envelope_batch(om, spec, Fin[:, sel], bin_[sel], want_stress=True, want_tree=True)
        assert PA.energy_errors(g["W"][sel], W, kind).max() <= PA.RTOL[kind], k
        ne, _ = PA.check_stress(om, spec, len(lv), Fin[:, sel], bin_[sel], W, P, trees, g["P"][:, sel],
                                g["tree"][sel], kind)
        n_exact += ne
    assert n_exact >= 30


def test_stvk_surrogate_epilogue(lib):
    """A network trained on St. Venant-Kirchhoff lamination data: where it serves a point,
    inference returns W(F) - max(g, 0) and P0(F) - dP with the St. Venant-Kirchhoff W and P0
    (oracle), g and dP the FP64 network oracle's forward; fallback points equal plain
    lamination."""
    r1, h, torch = lib
    cfg = WL.config4_training(n=32768, seed_tag=608)
    levels = cfg["levels"]
    mat = r1.material_from(MAT, 2, STVK)
    spec = r1.LaminationSpec(levels)
    Ft = torch.tensor(cfg["F"], dtype=torch.float32, device="cuda").contiguous()
    bt = torch.tensor(cfg["beta_n"], dtype=torch.float32, device="cuda").contiguous()
    plain = h.envelope(mat, spec, Ft, bt, stress=True, flags=False)
    s = r1.Surrogate(h, dim=2, n_hidden=2, width=32, seed=3)
    X, Y = s.pack(Ft, bt, plain["W"], plain["P"])
    s.train(mat, X, Y, epochs=5, batch=1024, lr=2e-3, seed=4)
    test = WL.config4_training(n=2048, seed_tag=609)
    Fq = torch.tensor(test["F"], dtype=torch.float32, device="cuda").contiguous()
    bq = torch.tensor(test["beta_n"], dtype=torch.float32, device="cuda").contiguous()
    out = s.infer(mat, spec, Fq, bq)
    ref = h.envelope(mat, spec, Fq, bq, stress=True, flags=False)
    torch.cuda.synchronize()
    fl = out["flags"].cpu().numpy()
    fb = (fl & r1.PT_FALLBACK) != 0
    Wg, Pg = out["W"].cpu().numpy(), out["P"].cpu().numpy()
    assert np.array_equal(Wg[fb], ref["W"].cpu().numpy()[fb])
    assert np.array_equal(Pg[:, fb], ref["P"].cpu().numpy()[:, fb])
    ok = np.nonzero(~fb)[0][:256]
    assert len(ok) > 50
    nm = s.norm()
    params = s.get_params().astype(np.float64)
    Fi, bi = Fq.double().cpu().numpy(), bq.double().cpu().numpy()
    x = np.concatenate([Fi[:, ok].T, bi[ok, None]], axis=1)
    xn = (x.astype(np.float32) - nm["x_mean"]) / nm["x_std"]
    y, _ = O.mlp_forward((5, 32, 2, 5), params, xn.astype(np.float64))
    y = y * nm["y_std"] + nm["y_mean"]
    om = PA.orc_material(MAT, 2, STVK)
    lam = y[:, 0] > 0
    W_ref = np.array([O.energy(om, Fi[:, p].reshape(2, 2), bi[p]) for p in ok]) - np.where(lam, y[:, 0], 0)
    P_ref = np.array([O.stress0(om, Fi[:, p].reshape(2, 2), bi[p]).ravel() for p in ok]) - \
        np.where(lam[:, None], y[:, 1:], 0)
    far = np.abs(y[:, 0]) >= 0.02 * nm["y_std"][0]
    assert far.sum() > 40
    assert np.max(np.abs(Wg[ok] - W_ref)[far]) < 0.02 * nm["y_std"][0] + 1e-6
    assert np.max(np.abs(Pg[:, ok].T - P_ref)[far]) < 0.02 * np.max(nm["y_std"][1:]) + 1e-6
    s.close()
