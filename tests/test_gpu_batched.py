"""Uneven batch in one persistent, graph-captured launch (r1_envelope_batched):
against the FP64 oracle per point, and every graph replay against the eager
(non-graph) result of the same points."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2211_14318_amd import workloads as WL
from tests import parity as PA

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


def small_table():
    """Depth 1 and 2 entries with different grids and direction counts (ragged sizes)."""
    t = []
    for nt in (33, 65, 129):
        for na, nb in ((4, 2), (4, 4), (5, 3)):
            a, b = WL.angle_directions(na, nb)
            t.append([WL.level(a, b, nt, 1.0)])
    ai, bi = WL.angle_directions(4, 2)
    for nt in (17, 33):
        a, b = WL.angle_directions(4, 4)
        t.append([WL.level(a, b, nt, 1.2), WL.level(ai, bi, 17, 1.2)])
    return t


def make_batch(n, seed, table):
    rng = np.random.default_rng(seed)
    cfg = WL.small_random(2, n, (1, 1), 3, seed_tag=seed)
    idx = rng.integers(0, len(table), size=n).astype(np.int32)
    return cfg["F"], cfg["beta_n"], idx


def run_batched(lib, table, F, bn, idx, kind, stress=True):
    r1, h, torch = lib
    dt = torch.float64 if kind == "f64" else torch.float32
    mat = r1.material()
    specs = [r1.LaminationSpec(t) for t in table]
    Ft = torch.tensor(F, dtype=dt, device="cuda").contiguous()
    bt = torch.tensor(bn, dtype=dt, device="cuda").contiguous()
    it = torch.tensor(idx, dtype=torch.int32, device="cuda")
    out = h.envelope_batched(mat, specs, it, Ft, bt, stress=stress, tree=True)
    torch.cuda.synchronize()
    return {k: (v.cpu().numpy() if v is not None else None) for k, v in out.items()}, Ft, bt


@pytest.mark.parametrize("kind", ["f64", "f32"])
def test_batched_against_oracle(lib, kind):
    table = small_table()
    F, bn, idx = make_batch(70, 700, table)
    # a point with det F <= 0 and one depth-2 point of it
    F[:, 3] = [1.0, 0.0, 0.0, -0.3]
    idx[3] = len(table) - 1
    g, Ft, bt = run_batched(lib, table, F, bn, idx, kind)
    Fin = Ft.double().cpu().numpy()
    bin_ = bt.double().cpu().numpy()
    mat = PA.orc_material(WL.MATERIAL, 2)
    n_exact = n_tie = 0
    for k, lv in enumerate(table):
        sel = np.nonzero(idx == k)[0]
        if len(sel) == 0:
            continue
        spec = PA.orc_spec(lv)
        W, P, trees = O.envelope_batch(mat, spec, Fin[:, sel], bin_[sel], want_stress=True, want_tree=True)
        err = PA.energy_errors(g["W"][sel], W, kind)
        assert err.max() <= PA.RTOL[kind], (k, err.max())
        ne, nt = PA.check_stress(mat, spec, len(lv), Fin[:, sel], bin_[sel], W, P, trees,
                                 g["P"][:, sel], g["tree"][sel], kind)
        n_exact += ne
        n_tie += nt
    print("batched %s: %d exact, %d tie-checked" % (kind, n_exact, n_tie))
    assert n_exact >= 40
    assert g["W"][3] == np.inf and g["flags"][3] & 1


def test_graph_replays_match_eager_results(lib):
    """Replay the captured launch several times with eager work and synchronisation in
    between (and new input values in the same buffers); each replay must equal the
    eager per-entry launches on the same inputs."""
    r1, h, torch = lib
    table = small_table()
    F, bn, idx = make_batch(48, 701, table)
    mat = r1.material()
    specs = [r1.LaminationSpec(t) for t in table]
    Ft = torch.tensor(F, dtype=torch.float32, device="cuda").contiguous()
    bt = torch.tensor(bn, dtype=torch.float32, device="cuda").contiguous()
    it = torch.tensor(idx, dtype=torch.int32, device="cuda")
    n = F.shape[1]
    W = torch.empty(n, dtype=torch.float32, device="cuda")
    P = torch.empty((4, n), dtype=torch.float32, device="cuda")
    T = torch.empty((n, 3, 4), dtype=torch.int32, device="cuda")
    fl = torch.empty(n, dtype=torch.int32, device="cuda")
    import ctypes
    arr = (r1.Lamination * len(specs))(*[s.c for s in specs])
    for rep in range(4):
        if rep == 2:     # new values in the same buffers: the graph must read them
            Ft.mul_(1.01)
        W.fill_(-7.0)
        P.fill_(-7.0)
        st = r1.lib().r1_envelope_batched(h.h, ctypes.byref(mat), arr, len(specs), n,
                                          ctypes.c_void_p(it.data_ptr()), r1.R1_F32,
                                          ctypes.c_void_p(Ft.data_ptr()), ctypes.c_void_p(bt.data_ptr()),
                                          ctypes.c_void_p(W.data_ptr()), ctypes.c_void_p(P.data_ptr()),
                                          ctypes.c_void_p(T.data_ptr()), ctypes.c_void_p(fl.data_ptr()),
                                          ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
        assert st == 0
        torch.cuda.synchronize()
        # eager: one plain launch per table entry on its points
        for k, s in enumerate(specs):
            sel = torch.nonzero(it == k).flatten()
            if sel.numel() == 0:
                continue
            out = h.envelope(mat, s, Ft[:, sel].contiguous(), bt[sel].contiguous(), stress=True, tree=True)
            torch.cuda.synchronize()
            assert torch.equal(out["W"], W[sel]), (rep, k)
            assert torch.equal(out["P"], P[:, sel]), (rep, k)
            assert torch.equal(out["tree"], T[sel]), (rep, k)


def test_batched_rejects_bad_table_index(lib):
    r1, h, torch = lib
    table = small_table()
    F, bn, idx = make_batch(8, 702, table)
    idx[5] = len(table)
    with pytest.raises(r1.R1Error) as e:
        run_batched(lib, table, F, bn, idx, "f64")
    assert e.value.status == -1


def test_autotuner_returns_admissible_width(lib):
    """One-level lines and inner levels of depth 2 are tuned separately (the inner
    level on the depth-2 path); each query returns its own role's choice."""
    r1, h, torch = lib
    mat = r1.material()
    for nt in (257, 1025):
        lanes = h.autotune(mat, nt, r1.R1_F32)
        assert lanes in (8, 16, 32, 64)
        assert h.segment_width(nt, r1.R1_F32, 2) == lanes
        inner = h.autotune_inner(mat, nt, r1.R1_F32)
        print("n_t %d: one-level lanes %d, inner lanes %d" % (nt, lanes, inner))
        assert inner in (8, 16, 32, 64)
        assert h.inner_segment_width(nt, r1.R1_F32, 2) == inner
        assert h.segment_width(nt, r1.R1_F32, 2) == lanes


def test_tuning_records_round_trip(lib):
    """The tuned widths leave a handle as records and enter a fresh one unchanged, so
    a caller can keep the autotuner's results between runs; a bad record (even n_t,
    unknown role, unsupported width, a width too narrow for the grid) is refused and
    installs nothing."""
    r1, h, torch = lib
    mat = r1.material()
    h.autotune(mat, 129, r1.R1_F32)
    h.autotune_inner(mat, 129, r1.R1_F32)
    rec = h.tuning()
    assert rec.shape[1] == 5 and len(rec) >= 2
    assert {(129, r1.R1_F32, 2, 0), (129, r1.R1_F32, 2, 1)} <= {tuple(r[:4]) for r in rec}
    h2 = r1.Handle(0)
    try:
        assert len(h2.tuning()) == 0
        h2.set_tuning(rec)
        assert np.array_equal(h2.tuning(), rec)
        assert h2.segment_width(129, r1.R1_F32, 2) == h.segment_width(129, r1.R1_F32, 2)
        assert h2.inner_segment_width(129, r1.R1_F32, 2) == h.inner_segment_width(129, r1.R1_F32, 2)
        for bad in ([128, 0, 2, 0, 16], [129, 0, 2, 2, 16], [129, 0, 2, 0, 12], [2049, 0, 2, 0, 8]):
            with pytest.raises(r1.R1Error):
                h2.set_tuning(np.array([[257, 0, 2, 0, 16], bad]))
            assert np.array_equal(h2.tuning(), rec)
    finally:
        h2.close()


def _eager(lib, table, Ft, bt, it):
    """One plain launch per table entry on its points (torch tensors)."""
    r1, h, torch = lib
    mat = r1.material()
    n = Ft.shape[1]
    W = torch.empty(n, dtype=Ft.dtype, device="cuda")
    P = torch.empty((4, n), dtype=Ft.dtype, device="cuda")
    T = torch.empty((n, 3, 4), dtype=torch.int32, device="cuda")
    for k, lv in enumerate(table):
        sel = torch.nonzero(it == k).flatten()
        if sel.numel() == 0:
            continue
        out = h.envelope(mat, r1.LaminationSpec(lv), Ft[:, sel].contiguous(), bt[sel].contiguous(),
                         stress=True, tree=True)
        W[sel], P[:, sel], T[sel] = out["W"], out["P"], out["tree"]
    torch.cuda.synchronize()
    return W, P, T


def test_batched_follows_new_indices_in_the_same_buffer(lib):
    """r1_envelope_batched plans by the contents of lam_idx: new indices written
    into the same device buffer give the results of the new indices."""
    r1, h, torch = lib
    table = small_table()
    F, bn, idx = make_batch(64, 703, table)
    Ft = torch.tensor(F, dtype=torch.float32, device="cuda").contiguous()
    bt = torch.tensor(bn, dtype=torch.float32, device="cuda").contiguous()
    it = torch.tensor(idx, dtype=torch.int32, device="cuda")
    mat = r1.material()
    specs = [r1.LaminationSpec(t) for t in table]
    rng = np.random.default_rng(704)
    for rep in range(3):
        out = h.envelope_batched(mat, specs, it, Ft, bt, stress=True, tree=True)
        torch.cuda.synchronize()
        W, P, T = _eager(lib, table, Ft, bt, it)
        assert torch.equal(out["W"], W) and torch.equal(out["P"], P) and torch.equal(out["tree"], T), rep
        # depth-1 points become depth-2 points and back, in place
        it.copy_(torch.tensor(rng.integers(0, len(table), size=64).astype(np.int32), device="cuda"))


def test_plan_keeps_its_own_indices_and_directions(lib):
    """A plan built from lam_idx is not affected by later writes to lam_idx, nor by
    the handle's direction cache evicting (600 plain calls with distinct
    directions pass its 512-entry limit) between replays."""
    r1, h, torch = lib
    table = small_table()
    F, bn, idx = make_batch(56, 705, table)
    Ft = torch.tensor(F, dtype=torch.float64, device="cuda").contiguous()
    bt = torch.tensor(bn, dtype=torch.float64, device="cuda").contiguous()
    it = torch.tensor(idx, dtype=torch.int32, device="cuda")
    mat = r1.material()
    plan = h.batched_plan(mat, [r1.LaminationSpec(t) for t in table], it, torch.float64)
    o = plan.outputs(stress=True, tree=True)
    plan.execute(Ft, bt, o["W"], o["P"], o["tree"], o["flags"])
    torch.cuda.synchronize()
    W0, P0, T0 = o["W"].clone(), o["P"].clone(), o["tree"].clone()
    We, Pe, Te = _eager(lib, table, Ft, bt, it)
    assert torch.equal(W0, We) and torch.equal(P0, Pe) and torch.equal(T0, Te)
    it.fill_(0)                                  # the plan keeps its own copy
    Fs = torch.tensor(WL.small_random(2, 4, (1, 1), 3, seed_tag=706)["F"], dtype=torch.float64, device="cuda")
    bs = torch.zeros(4, dtype=torch.float64, device="cuda")
    for k in range(600):                         # distinct directions: new cache entries
        th = 0.001 * (k + 1)
        a = np.array([[np.cos(th), np.sin(th)]])
        lv = [WL.level(a, a.copy(), 9, 0.5)]
        if k % 7 == 0:                           # depth 2 while the cache is full
            lv.append(WL.level(a[:, ::-1].copy(), a.copy(), 9, 0.5))
        h.envelope(mat, r1.LaminationSpec(lv), Fs, bs, stress=False)
    torch.cuda.synchronize()
    for rep in range(2):
        o["W"].fill_(-7.0)
        plan.execute(Ft, bt, o["W"], o["P"], o["tree"], o["flags"])
        torch.cuda.synchronize()
        assert torch.equal(o["W"], W0) and torch.equal(o["P"], P0) and torch.equal(o["tree"], T0), rep
    # other output buffers: a second captured graph of the same plan
    o2 = plan.outputs(stress=False, tree=False, flags=False)
    plan.execute(Ft, bt, o2["W"])
    torch.cuda.synchronize()
    assert torch.equal(o2["W"], W0)
    plan.close()


def test_depth2_after_cache_eviction_matches_oracle(lib):
    """A depth-2 call whose two levels are both new while the direction cache is
    full: both levels are resolved before anything is evicted."""
    r1, h, torch = lib
    mat = r1.material()
    Fs = torch.tensor(WL.small_random(2, 4, (1, 1), 3, seed_tag=707)["F"], dtype=torch.float64, device="cuda")
    bs = torch.zeros(4, dtype=torch.float64, device="cuda")
    for k in range(520):
        th = 0.002 * (k + 1)
        a = np.array([[np.cos(th), np.sin(th)]])
        h.envelope(mat, r1.LaminationSpec([WL.level(a, a.copy(), 9, 0.5)]), Fs, bs, stress=False)
    cfg = WL.small_random(2, 24, (2, 2), 17, tau=1.2, depth=2, inner=(2, 2, 17), seed_tag=708)
    out = h.envelope(mat, r1.LaminationSpec(cfg["levels"]), torch.tensor(cfg["F"], device="cuda"),
                     torch.tensor(cfg["beta_n"], device="cuda"), stress=True)
    torch.cuda.synchronize()
    om = PA.orc_material(WL.MATERIAL, 2)
    W, _, _ = O.envelope_batch(om, PA.orc_spec(cfg["levels"]), cfg["F"], cfg["beta_n"], want_stress=True)
    assert PA.energy_errors(out["W"].cpu().numpy(), W, "f64").max() <= PA.RTOL["f64"]
