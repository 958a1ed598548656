"""Helpers comparing the GPU path with the FP64 oracle (test infrastructure).

Tolerances:
  energy  |W_gpu - W_orc| <= RTOL * max(|W_orc|, W_FLOOR)
          RTOL = 1e-12 (FP64 path) / 1e-5 (FP32 path).  W is a difference of
          O(1) terms (mu/2 |F|^2, mu ln J, lambda/2 ln^2 J, D_inf D0 e^...), so
          its rounding error is absolute, a few ulp of 1: ~1e-7 in FP32, ~1e-15
          in FP64.  W_FLOOR is the |W| below which that absolute error exceeds
          RTOL * |W|: 1e-2 for FP32 (1e-7 / 1e-5), 1e-3 for FP64 (1e-15 / 1e-12).
  stress  compared where the oracle's laminate is unambiguous: the runner-up
          direction and the nearest other sample to the chosen hull segment
          are further than TIE * max(|W|, W_FLOOR).  Elsewhere several
          laminates are correct; there the GPU's tree is evaluated by the
          oracle (Algorithm 3 on that tree) and must give the oracle's energy
          and the GPU's stress.
"""
import numpy as np

from oracle import oracle as O

W_FLOOR = {"f64": 1e-3, "f32": 1e-2}
RTOL = {"f64": 1e-12, "f32": 1e-5}
TIE = {"f64": 1e-9, "f32": 1e-4}
PTOL = {"f64": 1e-10, "f32": 2e-5}


def orc_spec(levels):
    return O.LaminationSpec([(l["a"], l["b"], l["n_t"], l["tau"]) for l in levels])


def orc_material(mat_dict, dim, model=O.MODEL_NH_DAMAGE):
    return O.material(dim=dim, model=model, mu=mat_dict["mu"], lam=mat_dict["lam"],
                      D_inf=mat_dict["D_inf"], D0=mat_dict["D0"])


def energy_errors(w_gpu, w_orc, kind):
    w_gpu = np.asarray(w_gpu, dtype=np.float64)
    w_orc = np.asarray(w_orc, dtype=np.float64)
    fin = np.isfinite(w_orc)
    assert np.array_equal(np.isfinite(w_gpu), fin), "finite pattern differs"
    err = np.zeros_like(w_orc)
    err[fin] = np.abs(w_gpu[fin] - w_orc[fin]) / np.maximum(np.abs(w_orc[fin]), W_FLOOR[kind])
    return err


def paper_erel(w_gpu, w_orc, gamma=1e-8):
    """E_rel = |a - b| / (gamma + |b|), the relative error of Section 6.2 (gamma = 1e-8)."""
    fin = np.isfinite(w_orc)
    return np.abs(w_gpu[fin] - w_orc[fin]) / (gamma + np.abs(w_orc[fin]))


def is_tie(tree, depth, W, kind):
    scale = max(abs(W), W_FLOOR[kind])
    nodes = tree[:1] if depth == 1 else tree[:3]
    for nd in nodes:
        if nd["dir_gap"] < TIE[kind] * scale or nd["bridge_gap"] < TIE[kind] * scale:
            return True
    return False


TIE_FLAG = {"f64": 1e-10, "f32": 1e-5}   # the library's tie margin (flag R1_PT_TIE)
PT_TIE = 16


def check_tie_flags(trees_orc, depth, W_orc, flags_gpu, kind):
    """The GPU's R1_PT_TIE flag against the oracle's runner-up gaps: every node of the
    tree whose winning direction laminates (oracle dir_gap finite) counts; a gap below a
    tenth of the margin must be flagged, a gap above ten times the margin must not.
    Returns (n_flagged, n_between)."""
    n_flag = n_mid = 0
    for p in range(len(W_orc)):
        if not np.isfinite(W_orc[p]):
            continue
        nodes = trees_orc[p][:1] if depth == 1 else trees_orc[p][:3]
        g = min(nd["dir_gap"] / (TIE_FLAG[kind] * max(abs(nd["value"]), W_FLOOR[kind])) for nd in nodes)
        flagged = bool(flags_gpu[p] & PT_TIE)
        if g < 0.1:
            assert flagged, (p, g)
        elif g > 10.0:
            assert not flagged, (p, g)
        else:
            n_mid += 1
        n_flag += flagged
    return n_flag, n_mid


def check_stress(mat, spec, depth, F_soa, beta_n, W_orc, P_orc, trees_orc, P_gpu, tree_gpu, kind, stats=None):
    """Returns (n_checked_exact, n_ties).  tree_gpu: (n, 3, 4) int32 array.  stats
    (nullable dict) receives under "tie_w" the largest relative energy difference
    between the GPU's tree (evaluated by the oracle) and the oracle's W at ties.

    At fine FP32 grids most points count as ties: the samples beside a bridge's
    tangent point lie within a few 1e-5 of the bridge line, so either may be the
    laminate's endpoint.  There the GPU's tree must be a laminate whose exact energy
    is within 10x the energy bar of the minimum, and the GPU's stress that tree's."""
    d = mat.dim
    n = F_soa.shape[1]
    n_exact = n_ties = 0
    lv = spec.levels
    for p in range(n):
        if not np.isfinite(W_orc[p]):
            assert np.all(np.isnan(P_gpu[:, p]))
            continue
        scale = max(np.abs(P_orc[:, p]).max(), 1.0)
        g_nodes = [(int(tree_gpu[p, k, 0]), int(tree_gpu[p, k, 1]), int(tree_gpu[p, k, 2]))
                   for k in range(3)]
        o_nodes = [(t["dir"], t["i_minus"], t["i_plus"]) for t in trees_orc[p]]
        nn = 1 if depth == 1 else 3
        if is_tie(trees_orc[p], depth, W_orc[p], kind):
            n_ties += 1
            F = F_soa[:, p].reshape(d, d)
            We, Pe = O.eval_tree(mat, spec, F, beta_n[p], g_nodes)
            dev = abs(We - W_orc[p]) / max(abs(W_orc[p]), W_FLOOR[kind])
            if stats is not None:
                stats["tie_w"] = max(stats.get("tie_w", 0.0), dev)
            assert dev <= RTOL[kind] * 10, (p, We, W_orc[p])
            assert np.max(np.abs(Pe.ravel() - P_gpu[:, p])) <= PTOL[kind] * scale, (p, Pe, P_gpu[:, p])
        else:
            n_exact += 1
            assert g_nodes[:nn] == o_nodes[:nn], (p, g_nodes, o_nodes)
            assert np.max(np.abs(P_gpu[:, p] - P_orc[:, p])) <= PTOL[kind] * scale, (p, P_gpu[:, p], P_orc[:, p])
    return n_exact, n_ties


def oracle_envelope_points(mat_dict, dim, levels, F_soa, beta_n, model=0):
    """Process-pool worker (picklable arguments only): the oracle's envelope, stress and
    tree at the given points."""
    mat = orc_material(mat_dict, dim, model)
    spec = orc_spec(levels)
    return O.envelope_batch(mat, spec, F_soa, beta_n, want_stress=True, want_tree=True)


def oracle_pool_map(mat_dict, dim, levels, F_soa, beta_n, workers):
    """The oracle at each column of F_soa, one point per task on `workers` fresh
    interpreters (spawned: the parent may hold a GPU context).  Returns W, P, trees."""
    import concurrent.futures as cf
    import multiprocessing as mp
    n = F_soa.shape[1]
    with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
        futs = [ex.submit(oracle_envelope_points, mat_dict, dim, levels, F_soa[:, p:p + 1].copy(),
                          beta_n[p:p + 1].copy()) for p in range(n)]
        res = [f.result() for f in futs]
    W = np.concatenate([r[0] for r in res])
    P = np.concatenate([r[1] for r in res], axis=1)
    trees = [r[2][0] for r in res]
    return W, P, trees


def load_oracle_golden(name):
    """Stored oracle values written by tests/golden/make_oracle_golden.py (which calls
    only the oracle): the header dict and the points, each with p, F, beta_n, W, P,
    tree (per node [dir, i_minus, i_plus]), dir_gap and bridge_gap."""
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", name)
    with open(path) as f:
        d = json.load(f)

    def num(v):
        if isinstance(v, str):
            return float(v)
        if isinstance(v, list):
            return [num(x) for x in v]
        return v

    pts = []
    for q in d["points"]:
        q = {k: num(v) for k, v in q.items()}
        q["nodes"] = [dict(dir=t[0], i_minus=t[1], i_plus=t[2], dir_gap=g, bridge_gap=b)
                      for t, g, b in zip(q["tree"], q["dir_gap"], q["bridge_gap"])]
        pts.append(q)
    hdr = {k: v for k, v in d.items() if k != "points"}
    return hdr, pts


def golden_arrays(pts, dim=2):
    """F (d*d, m), beta_n (m,), W (m,), P (d*d, m) and the tree dicts of stored points."""
    F = np.array([q["F"] for q in pts], dtype=np.float64).T.copy()
    bn = np.array([q["beta_n"] for q in pts], dtype=np.float64)
    W = np.array([q["W"] for q in pts], dtype=np.float64)
    P = np.array([q["P"] for q in pts], dtype=np.float64).T.copy()
    return F, bn, W, P, [q["nodes"] for q in pts]
