"""Global lamination on a deformation-gradient mesh (r1_grid_*) against the FP64 oracle,
through the C-ABI.  The line kernel uses the oracle's monotone-chain orientation test and
hull formula, so FP64 iterates agree to rounding of the inputs (W^0 differs from the
oracle's by ~1e-16 relative, as every W evaluation does); FP32 to the FP32 energy bar."""
import numpy as np
import pytest

from oracle import oracle as O
from tests import parity as PA

pytestmark = pytest.mark.gpu

NH = dict(mu=1.0, lam=0.5, D_inf=0.9, D0=0.3)          # Table 6.1 material (both rows)
BETA_STVK = 0.07986236557499998                        # history the printed STVK curves carry


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2211_14318_amd import r1
    h = r1.Handle(0)
    yield r1, h, torch
    h.close()


def meshes(dim):
    if dim == 2:
        return (4, 5, 5, 6), (0.6, -0.4, -0.4, 0.5), 0.2
    return (3, 2, 2, 2, 4, 2, 2, 2, 3), (0.8, -0.1, -0.1, -0.1, 0.7, -0.1, -0.1, -0.1, 0.8), 0.2


def lam_meshes(dim):
    """Small meshes on which both energies laminate over several iterations."""
    if dim == 2:
        return meshes(2)
    return (6, 2, 2, 2, 6, 2, 2, 2, 6), (0.1, -0.175, -0.175, -0.175, 0.1, -0.175, -0.175, -0.175, 0.1), 0.35


def both_grids(r1, dim, n, lo, delta):
    return r1.grid(dim, n, lo, delta), O.grid(dim, n, lo, delta)


def _line_through(n, steps_r, p):
    """Node indices of the mesh line through node p with integer step steps_r (component
    0 slowest, as the nodes are numbered), in order of l, and p's position on it."""
    n = np.asarray(n)
    I = np.array(np.unravel_index(p, tuple(n)))
    s = np.asarray(steps_r)
    lo, hi = -10 ** 6, 10 ** 6
    for c in range(len(n)):
        if s[c] > 0:
            lo, hi = max(lo, -(I[c] // s[c])), min(hi, (n[c] - 1 - I[c]) // s[c])
        elif s[c] < 0:
            lo, hi = max(lo, -((n[c] - 1 - I[c]) // -s[c])), min(hi, I[c] // -s[c])
    ls = np.arange(lo, hi + 1)
    J = I[None, :] + ls[:, None] * s[None, :]
    return np.ravel_multi_index(tuple(J.T), tuple(n)), -lo


def check_laminate_validity(n, steps, W_prev, C_prev, W_new, C_new, nodes, eps, ctol):
    """Eq. 5.2 (first case) as a validity check, independent of how ties are broken: at
    each given node the new value is the minimum over its own value and every
    direction's hull value (Algorithm 1 on the node's mesh line through the previous
    iterate, orc_hull_at_centre) to within 16 eps max(|W|, 1e-3), and the carried
    quantities C_new (stresses, moduli) are those of one laminate attaining that
    minimum to within the same margin: the node's own C_prev if no lowering is needed,
    else the hull segment's endpoints' C_prev with the weights of the value."""
    for p in nodes:
        cands = [(W_prev[p], None)]
        for r in range(len(steps)):
            line, c = _line_through(n, steps[r], p)
            v, im, ip, _ = O.hull_at_centre(W_prev[line], c)
            if im != ip:
                xi = (c - im) / (ip - im)
                cands.append((v, xi * C_prev[:, line[ip]] + (1 - xi) * C_prev[:, line[im]]))
        m = min(v for v, _ in cands)
        margin = 16 * eps * max(abs(m), 1e-3)
        assert abs(W_new[p] - m) <= margin, (p, W_new[p], m)
        sc = max(np.max(np.abs(C_new[:, p])), 1.0)
        ok = [v <= m + margin and np.max(np.abs((C_prev[:, p] if c is None else c) - C_new[:, p])) <= ctol * sc
              for v, c in cands]
        assert any(ok), (p, W_new[p], [v for v, _ in cands])


@pytest.mark.parametrize("kind", ["f64", "f32"])
@pytest.mark.parametrize("model", [0, 2])
@pytest.mark.parametrize("dim", [2, 3])
def test_grid_energy_matches_oracle(lib, kind, model, dim):
    r1, h, torch = lib
    dt = torch.float64 if kind == "f64" else torch.float32
    n, lo, delta = meshes(dim)
    # shifted off-diagonal ranges give nodes with det F < 0 (none within 4e-3 of det F = 0,
    # where the sign of a rounded determinant would decide finiteness)
    lo = [v - 0.53 if i % (dim + 1) else v for i, v in enumerate(lo)]
    g, og = both_grids(r1, dim, n, lo, delta)
    W = h.grid_energy(r1.material_from(NH, dim, model), g, 0.05, dt)
    torch.cuda.synchronize()
    Wo = O.grid_energy(PA.orc_material(NH, dim, model), og, 0.05)
    err = PA.energy_errors(W.double().cpu().numpy(), Wo, kind)
    # the parity bar holds where W is well conditioned; near det F = 0 the neo-Hooke log
    # term amplifies the rounding of det F (computed by different formulas on each side)
    det = np.array([np.linalg.det(O.grid_node(og, p)) for p in range(O.grid_size(og))])
    good = (np.abs(det) >= 0.05) | (model != 0)
    assert err[good].max() <= PA.RTOL[kind], err[good].max()
    assert err.max() <= max(PA.RTOL[kind], 1e-9), err.max()
    if model == 0:
        assert np.any(~np.isfinite(Wo)) and np.sum(good) > len(good) // 2


@pytest.mark.parametrize("kind", ["f64", "f32"])
@pytest.mark.parametrize("dim", [2, 3])
def test_grid_one_iteration_on_random_values(lib, kind, dim):
    """One iteration from seeded random node values with +inf holes: the same lines, hulls
    and minima as the oracle (FP64 to the last bit of its formula; FP32 to its rounding)."""
    r1, h, torch = lib
    dt = torch.float64 if kind == "f64" else torch.float32
    n, lo, delta = meshes(dim)
    g, og = both_grids(r1, dim, n, lo, delta)
    rng = np.random.default_rng(70 + dim)
    W0 = rng.normal(size=O.grid_size(og))
    W0[rng.random(W0.size) < 0.1] = np.inf
    W = torch.tensor(W0, dtype=dt, device="cuda")
    hist = h.grid_laminate(g, r1.grid_r11(dim), W, k_max=1, tol=0.0)
    torch.cuda.synchronize()
    Wi = torch.tensor(W0, dtype=dt).double().numpy()        # the values the GPU was given
    ref, md = O.grid_sweep(og, O.grid_r11(dim), Wi)
    Wg = W.double().cpu().numpy()
    fin = np.isfinite(ref)
    assert np.array_equal(np.isfinite(Wg), fin)
    tol = 1e-15 if kind == "f64" else 2e-6
    assert np.max(np.abs(Wg[fin] - ref[fin])) <= tol
    assert len(hist) == 1 and abs(hist[0] - md) <= tol
    assert np.sum(Wg[fin] < Wi[fin]) > W0.size // 10


@pytest.mark.parametrize("kind", ["f64", "f32"])
@pytest.mark.parametrize("n", [(150, 1, 3, 40), (150, 4, 4, 3)])
def test_grid_every_hull_path_on_random_values(lib, kind, n):
    """Lines of 150 nodes (read in place: a column of them exceeds the LDS budget), 40, 4,
    3 and 1 node, a component with a single node; the first mesh runs the sparse mode
    (lines of 3+ nodes cover 43% of the direction-node pairs), the second the dense one.
    One iteration with random node stresses carried equals the oracle's sweep."""
    r1, h, torch = lib
    dt = torch.float64 if kind == "f64" else torch.float32
    g, og = both_grids(r1, 2, n, (0.5, -0.2, -0.3, 0.7), 0.05)
    N = O.grid_size(og)
    rng = np.random.default_rng(sum(n))
    W0 = rng.normal(size=N)
    W0[rng.random(N) < 0.05] = np.inf
    P0 = rng.normal(size=(4, N))
    W = torch.tensor(W0, dtype=dt, device="cuda")
    P = torch.tensor(P0, dtype=dt, device="cuda")
    hist = h.grid_laminate(g, r1.grid_r11(2), W, k_max=1, tol=0.0, P=P)
    torch.cuda.synchronize()
    Wi = torch.tensor(W0, dtype=dt).double().numpy()
    Pi = torch.tensor(P0, dtype=dt).double().numpy()
    ref, md, Pref = O.grid_sweep(og, O.grid_r11(2), Wi, Pi)
    Wg, Pg = W.double().cpu().numpy(), P.double().cpu().numpy()
    fin = np.isfinite(ref)
    assert np.array_equal(np.isfinite(Wg), fin)
    tol = 1e-15 if kind == "f64" else 2e-6
    assert np.max(np.abs(Wg[fin] - ref[fin])) <= tol
    assert len(hist) == 1 and abs(hist[0] - md) <= tol
    lowered = fin & (ref < Wi)
    assert lowered.sum() > N // 20
    # the stress of a node is its laminate's: equal to the oracle's, or (where the
    # directions tie to rounding) that of another laminate attaining the minimum
    ctol = 1e-14 if kind == "f64" else 2e-6
    differ = np.nonzero(fin & np.any(np.abs(Pg - Pref) > ctol * np.maximum(np.abs(Pref).max(axis=0), 1.0), axis=0))[0]
    eps = 2.0 ** -52 if kind == "f64" else 2.0 ** -23
    check_laminate_validity(n, O.grid_r11(2), Wi, Pi, Wg, Pg, differ, eps, ctol)
    print("%s: %d of %d nodes lowered, %d with another laminate than the oracle's" % (kind, lowered.sum(), N,
                                                                                       len(differ)))


@pytest.mark.parametrize("model,dim", [(0, 2), (2, 2), (2, 3), (0, 3)])
def test_grid_iterations_match_oracle(lib, model, dim):
    """The whole iteration to the stopping rule on small meshes (FP64)."""
    r1, h, torch = lib
    n, lo, delta = lam_meshes(dim)
    g, og = both_grids(r1, dim, n, lo, delta)
    W = h.grid_energy(r1.material_from(NH, dim, model), g, 0.04, torch.float64)
    hist = h.grid_laminate(g, r1.grid_r11(dim), W, k_max=20, tol=1e-6)
    torch.cuda.synchronize()
    Wo, ho = O.grid_laminate(og, O.grid_r11(dim), O.grid_energy(PA.orc_material(NH, dim, model), og, 0.04),
                             k_max=20, tol=1e-6)
    print("model %d %dD: %d iterations, decreases %s" % (model, dim, len(hist), np.array2string(hist, precision=3)))
    assert len(hist) == len(ho) and len(hist) >= 2
    assert np.allclose(hist, ho, rtol=1e-9, atol=1e-13)
    Wg = W.cpu().numpy()
    fin = np.isfinite(Wo)
    assert np.array_equal(np.isfinite(Wg), fin)
    assert np.max(np.abs(Wg[fin] - Wo[fin]) / np.maximum(np.abs(Wo[fin]), 1e-3)) <= 1e-12


def test_grid_stvk_paper_mesh_full_size(lib):
    """The 672,400-node mesh of Table 6.1 (STVK) with R^1_1 in FP64: the GPU's sequence of
    maximal decreases equals the oracle's, its final iterate the oracle's, and (as the
    oracle's does) it reproduces the printed convergence table with the readings of the
    oracle pin."""
    r1, h, torch = lib
    n, lo = (20, 41, 41, 20), (0.1, -2.0, -2.0, 0.1)
    g, og = both_grids(r1, 2, n, lo, 0.1)
    W = h.grid_energy(r1.material_from(NH, 2, 2), g, BETA_STVK, torch.float64)
    hist = h.grid_laminate(g, r1.grid_r11(2), W, k_max=20, tol=1e-4)
    torch.cuda.synchronize()
    Wo, ho = O.grid_laminate(og, O.grid_r11(2), O.grid_energy(PA.orc_material(NH, 2, 2), og, BETA_STVK),
                             k_max=20, tol=1e-4)
    assert len(hist) == len(ho) == 11
    assert np.allclose(hist, ho, rtol=1e-9, atol=1e-14)
    Wg = W.cpu().numpy()
    assert np.max(np.abs(Wg - Wo) / np.maximum(np.abs(Wo), 1e-3)) <= 1e-12
    printed = np.array([0.18478, 0.07939, 0.01625, 0.00237, 0.00132, 0.00075, 0.00045, 0.00037, 0.00014])
    assert abs(hist[1] - printed[0]) / printed[0] < 1e-4
    assert np.all(np.abs(hist[1:10] - printed) <= 0.13 * printed + 5e-6)


def test_grid_3d_paper_mesh_sampled(lib):
    """The 5,832,000-node 3D STVK mesh of Table 6.3 with the 169 steps of R^1_1 (FP64): the
    first iteration at 64 sampled nodes against the oracle's single-node update on the
    oracle's own W^0."""
    r1, h, torch = lib
    n = (20, 3, 3, 3, 20, 3, 3, 3, 20)
    lo = (0.1, -0.1, -0.1, -0.1, 0.1, -0.1, -0.1, -0.1, 0.1)
    g, og = both_grids(r1, 3, n, lo, 0.1)
    assert O.grid_size(og) == 5832000
    W = h.grid_energy(r1.material_from(NH, 3, 2), g, BETA_STVK, torch.float64)
    hist = h.grid_laminate(g, r1.grid_r11(3), W, k_max=1, tol=0.0)
    torch.cuda.synchronize()
    W0 = O.grid_energy(PA.orc_material(NH, 3, 2), og, BETA_STVK)
    steps = O.grid_r11(3)
    rng = np.random.default_rng(75)
    Wg = W.cpu().numpy()
    lowered = np.flatnonzero(Wg < W0 - 1e-12)
    assert len(lowered) > 1000
    sel = np.concatenate([rng.choice(lowered, 48, replace=False), rng.choice(Wg.size, 16, replace=False)])
    for p in sel:
        v = O.grid_update_node(og, steps, W0, int(p))
        assert abs(Wg[p] - v) <= 1e-12 * max(abs(v), 1e-3), (p, Wg[p], v)
    print("3D mesh: first decrease %.6f, %d nodes lowered" % (hist[0], len(lowered)))


@pytest.mark.parametrize("kind", ["f64", "f32"])
@pytest.mark.parametrize("dim", [2, 3])
def test_grid_interpolation_matches_oracle(lib, kind, dim):
    r1, h, torch = lib
    dt = torch.float64 if kind == "f64" else torch.float32
    n, lo, delta = meshes(dim)
    g, og = both_grids(r1, dim, n, lo, delta)
    rng = np.random.default_rng(80 + dim)
    W0 = rng.normal(size=O.grid_size(og))
    hi = np.array(lo) + delta * (np.array(n) - 1)
    P = rng.uniform(np.array(lo) - 0.05, hi + 0.05, size=(200, dim * dim))
    Wt = torch.tensor(W0, dtype=dt, device="cuda")
    Ft = torch.tensor(P.T.copy(), dtype=dt, device="cuda").contiguous()
    out = h.grid_interpolate(g, Wt, Ft)
    torch.cuda.synchronize()
    Wi = Wt.double().cpu().numpy()
    Fi = Ft.double().cpu().numpy()
    ref = np.array([O.grid_interpolate(og, Wi, Fi[:, k]) for k in range(Fi.shape[1])])
    got = out.double().cpu().numpy()
    assert np.array_equal(np.isnan(got), np.isnan(ref)) and np.any(np.isnan(ref)) and np.any(~np.isnan(ref))
    ok = ~np.isnan(ref)
    tol = 1e-13 if kind == "f64" else 1e-5
    assert np.max(np.abs(got[ok] - ref[ok])) <= tol


def test_grid_invalid_arguments(lib):
    r1, h, torch = lib
    g = r1.grid(2, (3, 3, 3, 3), (0, 0, 0, 0), 0.5)
    W = torch.zeros(81, dtype=torch.float64, device="cuda")
    with pytest.raises(r1.R1Error):
        h.grid_laminate(g, np.zeros((1, 4), dtype=np.int32), W)             # zero step
    with pytest.raises(r1.R1Error):                                          # a component beyond 512 nodes
        h.grid_laminate(r1.grid(2, (3, 3, 3, 600), (0, 0, 0, 0), 0.5), r1.grid_r11(2),
                        torch.zeros(3 * 3 * 3 * 600, dtype=torch.float64, device="cuda"))
    with pytest.raises(r1.R1Error):
        h.grid_energy(r1.material_from(NH, 3, 0), g, 0.0, torch.float64)    # dimension mismatch
    with pytest.raises(r1.R1Error):
        h.grid_laminate(r1.grid(2, (3, 3, 3, 3), (0, 0, 0, 0), 0.0), r1.grid_r11(2), W)


def _iterate_with_validity(h, r1, torch, g, og, dim, n, W, P, A, k_max, tol):
    """Runs the GPU iteration one step at a time (same stopping rule); after each step the
    carried stresses (and moduli) must equal the oracle sweep's from the same previous
    state, or else be those of another laminate attaining the minimum
    (check_laminate_validity).  Returns the decreases and the count of such nodes."""
    steps = O.grid_r11(dim)
    hist, n_other = [], 0
    dd = dim * dim
    for _ in range(k_max):
        Wp = W.cpu().numpy().copy()
        Cp = np.concatenate([P.cpu().numpy()] + ([A.cpu().numpy()] if A is not None else []))
        d = h.grid_laminate(g, r1.grid_r11(dim), W, k_max=1, tol=0.0, P=P, A=A)
        torch.cuda.synchronize()
        hist.append(d[0])
        Wn = W.cpu().numpy()
        Cn = np.concatenate([P.cpu().numpy()] + ([A.cpu().numpy()] if A is not None else []))
        Wr, md, Cr = O.grid_sweep(og, steps, Wp, Cp)
        fin = np.isfinite(Wr)
        assert np.max(np.abs(Wn[fin] - Wr[fin]) / np.maximum(np.abs(Wr[fin]), 1e-3)) <= 1e-14
        assert abs(d[0] - md) <= 1e-14 * max(abs(md), 1e-3)
        sc = np.maximum(np.abs(Cr).max(axis=0), 1.0)
        differ = np.nonzero(fin & np.any(np.abs(Cn - Cr) > 1e-11 * sc, axis=0))[0]
        check_laminate_validity(n, steps, Wp, Cp, Wn, Cn, differ, 2.0 ** -52, 1e-11)
        n_other += len(differ)
        assert np.all(np.isnan(Cn[:dd, ~fin]))
        if d[0] <= tol:
            break
    return hist, n_other


@pytest.mark.parametrize("model,dim", [(0, 2), (2, 2), (2, 3), (0, 3)])
def test_grid_stress_matches_oracle(lib, model, dim):
    """Node stresses carried through the iterations (eq. 5.2, first case): after every
    iteration each node's stress is its laminate's (the oracle's, or another laminate
    attaining the minimum), and their interpolation off the mesh is the oracle's
    interpolation of them (second case)."""
    r1, h, torch = lib
    n, lo, delta = lam_meshes(dim)
    g, og = both_grids(r1, dim, n, lo, delta)
    W, P = h.grid_energy(r1.material_from(NH, dim, model), g, 0.04, torch.float64, stress=True)
    W0, P0 = O.grid_energy(PA.orc_material(NH, dim, model), og, 0.04, stress=True)
    Wo, ho, Po = O.grid_laminate(og, O.grid_r11(dim), W0.copy(), k_max=20, tol=1e-6, P=P0.copy())
    hist, n_other = _iterate_with_validity(h, r1, torch, g, og, dim, n, W, P, None, k_max=20, tol=1e-6)
    assert len(hist) == len(ho)
    Pg = P.cpu().numpy()
    fin = np.isfinite(Wo)
    scale = max(np.max(np.abs(Po[:, fin])), 1.0)
    assert np.max(np.abs(W.cpu().numpy()[fin] - Wo[fin]) / np.maximum(np.abs(Wo[fin]), 1e-3)) <= 1e-12
    assert np.all(np.isnan(Pg[:, ~fin])) and np.all(np.isnan(Po[:, ~fin]))
    changed = np.sum(np.any(np.abs(Po - P0) > 1e-12, axis=0) & fin)
    assert changed > 10
    print("   %d node laminates other than the oracle's, each valid" % n_other)
    # off-mesh: interpolate each stress component at points inside cells of finite nodes
    rng = np.random.default_rng(90 + dim)
    hi = np.array(lo) + delta * (np.array(n) - 1)
    pts = rng.uniform(lo, hi, size=(64, dim * dim))
    Ft = torch.tensor(pts.T.copy(), dtype=torch.float64, device="cuda").contiguous()
    for c in range(dim * dim):
        got = h.grid_interpolate(g, P[c].contiguous(), Ft).cpu().numpy()
        ref = np.array([O.grid_interpolate(og, Pg[c], pts[k]) for k in range(len(pts))])
        ok = np.isfinite(ref)
        assert np.array_equal(np.isfinite(got), ok)
        assert np.max(np.abs(got[ok] - ref[ok]), initial=0.0) <= 1e-11 * scale
    print("model %d %dD: %d iterations, %d node stresses changed" % (model, dim, len(hist), changed))


def test_grid_double_well_stress_on_gpu(lib):
    """The double-well envelope's gradient at every node, carried by the GPU iteration."""
    r1, h, torch = lib
    g, og = both_grids(r1, 2, (9, 3, 3, 5), (-2.0, -0.5, -0.5, 0.0), 0.5)
    W, P = h.grid_energy(r1.material(model=r1.R1_TEST_DOUBLEWELL), g, 0.0, torch.float64, stress=True)
    h.grid_laminate(g, r1.grid_r11(2), W, k_max=5, tol=0.0, P=P)
    torch.cuda.synchronize()
    Pg = P.cpu().numpy()
    for p in range(O.grid_size(og)):
        F = O.grid_node(og, p)
        ref = 2.0 * (F - np.eye(2))
        ref[0, 0] = 4.0 * F[0, 0] * (F[0, 0] ** 2 - 1.0) if abs(F[0, 0]) > 1.0 else 0.0
        assert np.max(np.abs(Pg[:, p] - ref.ravel())) < 1e-13


@pytest.mark.parametrize("model,dim", [(0, 2), (2, 2), (2, 3), (0, 3)])
def test_grid_tangent_matches_oracle(lib, model, dim):
    """Moduli carried through the iterations with the stresses (Algorithm 3's tangent on the
    mesh): A^0 equals the oracle's node by node, and after every iteration each node's
    stress and moduli are those of its laminate (the oracle's, or another laminate
    attaining the minimum)."""
    r1, h, torch = lib
    n, lo, delta = lam_meshes(dim)
    g, og = both_grids(r1, dim, n, lo, delta)
    W, P, A = h.grid_energy(r1.material_from(NH, dim, model), g, 0.04, torch.float64, stress=True, tangent=True)
    W0g, A0g = W.cpu().numpy(), A.cpu().numpy()
    hist, n_other = _iterate_with_validity(h, r1, torch, g, og, dim, n, W, P, A, k_max=20, tol=1e-6)
    W0, P0, A0 = O.grid_energy(PA.orc_material(NH, dim, model), og, 0.04, stress=True, tangent=True)
    fin0 = np.isfinite(W0)
    sc0 = max(np.max(np.abs(A0[:, fin0])), 1.0)
    assert np.max(np.abs(A0g[:, fin0] - A0[:, fin0])) <= 1e-12 * sc0
    assert np.all(np.isnan(A0g[:, ~fin0])) and np.all(np.isnan(A0[:, ~fin0]))
    Wo, ho, Co = O.grid_laminate(og, O.grid_r11(dim), W0, k_max=20, tol=1e-6, P=np.concatenate([P0, A0]))
    dd = dim * dim
    Po, Ao = Co[:dd], Co[dd:]
    assert len(hist) == len(ho)
    fin = np.isfinite(Wo)
    Pg, Ag = P.cpu().numpy(), A.cpu().numpy()
    scale = max(np.max(np.abs(Ao[:, fin])), 1.0)
    assert np.all(np.isnan(Ag[:, ~fin]))
    print("   %d node laminates other than the oracle's, each valid" % n_other)
    changed = np.sum(np.any(np.abs(Ao - A0) > 1e-12, axis=0) & fin)
    assert changed > 10
    # the carried moduli stay symmetric (each leaf's d^2W is)
    Asq = Ag[:, fin].reshape(dd, dd, -1)
    assert np.max(np.abs(Asq - Asq.transpose(1, 0, 2))) <= 1e-11 * scale
    print("model %d %dD: %d iterations, %d node moduli changed" % (model, dim, len(hist), changed))


def test_grid_double_well_tangent_on_gpu(lib):
    """Double-well moduli on the mesh: laminated nodes (|F11| < 1) hold the leaves' 8 at
    (11, 11), the others 12 F11^2 - 4; 2 elsewhere on the diagonal (FP32 and FP64)."""
    r1, h, torch = lib
    g, og = both_grids(r1, 2, (9, 3, 3, 5), (-2.0, -0.5, -0.5, 0.0), 0.5)
    for dt, tol in ((torch.float64, 1e-13), (torch.float32, 1e-5)):
        W, A = h.grid_energy(r1.material(model=r1.R1_TEST_DOUBLEWELL), g, 0.0, dt, tangent=True)
        h.grid_laminate(g, r1.grid_r11(2), W, k_max=5, tol=0.0, A=A)
        torch.cuda.synchronize()
        Ag = A.double().cpu().numpy()
        for p in range(O.grid_size(og)):
            F11 = O.grid_node(og, p)[0, 0]
            ref = np.diag([8.0 if abs(F11) < 1.0 else 12.0 * F11 ** 2 - 4.0, 2.0, 2.0, 2.0]).ravel()
            assert np.max(np.abs(Ag[:, p] - ref)) < tol * 50, (dt, F11)
