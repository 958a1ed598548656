"""Benchmark: quadrature-point envelope evaluations per second on one MI355X.

Headline workload (one step): rank-one lamination of 4,096 2D quadrature
points to depth 2 -- outer level 64 directions x 1,025 points (tau 1.5), inner
level 32 directions x 257 points -- energy, laminate stress and lamination
tree, in FP32 (FP64 with --dtype f64).  Inputs are seeded synthetic gradients
F = I + 0.3 N(0,1) (det F > 0.1) and beta_n ~ U[0, 0.5], resident in HBM.

Prints one JSON line.  `roofline` prices the dominant kernel (the outer-line
kernel, which evaluates every inner envelope) by its algorithmic flops
(18 per W sample) against the FP32 (FP64) vector peak, timed with HIP events
on its launch stream.  `cpu_baseline` times the FP64 oracle on a bounded
sample of the same workload on the host's cores; the same oracle results give
`error`, the GPU's error on those points.  Secondary legs (skip with --quick):
`surrogate` (train the MLP on 2M lamination rows, then 1M-point inference
with routing against plain lamination of the same configuration), `batched`
(65,536 points with uneven grids/directions/depths in one graph replay),
`plain_3d` (262,144 3D points, 256 directions x 513 points),
`surrogate_3d` (a 4 x 256 network on the same 3D workload), `stvk` (the
headline shapes with the St. Venant-Kirchhoff damage model, 15 flops per
sample), `tangent` (Algorithm 3's tangent moduli of 1M depth-1 laminates,
priced by its algorithmic bytes against HBM) and `grid` (the paper's own grid
variant of the method on its 2D and 3D meshes, to the stopping rule).
"""
import argparse
import json
import multiprocessing as mp
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FLOPS_PER_W = 18           # algorithmic flops per W sample (FMA = 2), transcendentals not counted
PEAK = {"f32": 157.3, "f64": 78.6}   # MI355X vector peak, TFLOP/s
PEAK_NONPACKED = {"f32": 78.6, "f64": 78.6}   # without packed FP32 (the library is compiled without it)
GAMMA = 1e-8               # relative error E_rel = |a - b| / (gamma + |b|)


def w_samples_outer_kernel(cfg):
    """Distinct W evaluations of one outer-kernel launch: every outer line's
    non-centre samples are inner envelopes, each n_dir_i*(n_t_i - 1) + 1 samples."""
    lo, li = cfg["levels"]
    inner = len(li["a"]) * (li["n_t"] - 1) + 1
    return cfg["n"] * len(lo["a"]) * (lo["n_t"] - 1) * inner


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_outer_depth2_n4096_64x1025_32x257_f32_hbm.txt")
TRAFFIC_SOURCES = ["paper_2211_14318_amd/csrc/r1_device.hpp", "paper_2211_14318_amd/csrc/r1_kernels.hpp"]


def measured_traffic():
    """HBM bytes per k_outer launch from the committed counter summary, or None when the
    kernel sources have changed since the counters were taken (or the file is absent)."""
    import hashlib
    try:
        kv = {}
        for line in open(TRAFFIC_FILE):
            if "=" in line and not line.startswith("#"):
                k, v = line.split("=", 1)
                kv[k.strip()] = v.strip()
        h = hashlib.sha256(b"".join(open(os.path.join(ROOT, f), "rb").read() for f in TRAFFIC_SOURCES))
        if h.hexdigest()[:16] != kv.get("source_fingerprint"):
            return None
        return int(float(kv["bytes_per_launch"]))
    except (OSError, KeyError, ValueError):
        return None


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def erel_stats(a, b, floor=0.0):
    import numpy as np
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    e = np.abs(a - b) / (GAMMA + np.maximum(np.abs(b), floor))
    return dict(max=float(e.max()), p99=float(np.percentile(e, 99)), n=int(e.size))


# ---------------------------------------------------------------- CPU baseline (oracle)

def _oracle_worker(idx):
    from oracle import oracle as O
    from paper_2211_14318_amd import workloads as WL
    cfg = WL.config2()
    m = cfg["material"]
    mat = O.material(dim=2, mu=m["mu"], lam=m["lam"], D_inf=m["D_inf"], D0=m["D0"])
    spec = O.LaminationSpec([(l["a"], l["b"], l["n_t"], l["tau"]) for l in cfg["levels"]])
    F = cfg["F"][:, idx].reshape(2, 2)
    t0 = time.time()
    W, P, _ = O.envelope(mat, spec, F, cfg["beta_n"][idx], want_tree=True)
    return idx, time.time() - t0, W, P.ravel().tolist()


def cpu_baseline(workers):
    from oracle import oracle as O
    O.build(force=False)
    t0 = time.time()
    with mp.get_context("spawn").Pool(workers) as pool:
        res = pool.map(_oracle_worker, list(range(workers)))
    wall = time.time() - t0
    per = [r[1] for r in res]
    w_per_point = w_samples_outer_kernel(_cfg2_shape()) / 4096.0
    base = dict(value=workers / wall, unit="QP/s", cores=workers, nproc=os.cpu_count(), kind="oracle",
                sample="first %d points of the workload, one point per process (energy, stress and "
                       "tree, FP64 serial oracle), %.1f s wall, %.1f s per point" %
                       (workers, wall, sum(per) / len(per)),
                single_core_qps=len(per) / sum(per),
                w_evals_per_s=workers / wall * w_per_point,
                single_core_w_evals_per_s=len(per) / sum(per) * w_per_point,
                cpu_model=_cpu_model())
    return base, {r[0]: (r[2], r[3]) for r in res}


def _cfg2_shape():
    from paper_2211_14318_amd import workloads as WL
    return WL.config2(n=4096)


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


# ---------------------------------------------------------------- secondary legs

def timed(fn, reps, torch):
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def served_stats(w_served, w_ref, served, floor=1e-2):
    """Relative energy error of the points the network served, |W|-floored at 1e-2."""
    import numpy as np
    e = np.abs(w_served[served] - w_ref[served]) / np.maximum(np.abs(w_ref[served]), floor)
    if e.size == 0:
        return {"n": 0}
    return {"n": int(e.size), "max": float(e.max()), "p999": float(np.percentile(e, 99.9)),
            "p99": float(np.percentile(e, 99)), "frac_gt_1e-3": float(np.mean(e > 1e-3))}


# Surrogate gate settings: per-cell thresholds on the predicted gap admit a cell's
# calibration rows only while every one of them is within GATE_TOL (quantile 1),
# and the a-posteriori check sends a served point to the fallback when a chord of
# subset samples passes CHECK_EPS below its value.
GATE_TOL, GATE_QUANTILE, CHECK_EPS = 2.5e-4, 1.0, 5e-4


def leg_surrogate(h, r1, WL, torch, np, n_train=2_000_000, n_cal=2_000_000, n_inf=1_000_000, epochs=20):
    """Config 4: MLP 5 -> 4x128 SiLU -> 5 trained on config-1-style lamination rows."""
    mat = r1.material()
    tr = WL.config4_training(n=n_train)
    spec = r1.LaminationSpec(tr["levels"])
    F = torch.tensor(tr["F"], dtype=torch.float32, device="cuda")
    bn = torch.tensor(tr["beta_n"], dtype=torch.float32, device="cuda")
    t0 = time.perf_counter()
    out = h.envelope(mat, spec, F, bn, stress=True, flags=False)
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    s = r1.Surrogate(h, dim=2, n_hidden=4, width=128, seed=2211)
    X, Y = s.pack(F, bn, out["W"], out["P"])
    del F, bn, out
    rep = s.train(mat, X, Y, epochs=epochs, batch=4096, lr=2e-3, seed=1)
    del X, Y
    cal = WL.config4_training(n=n_cal, seed_tag=42)
    Fc = torch.tensor(cal["F"], dtype=torch.float32, device="cuda")
    bc = torch.tensor(cal["beta_n"], dtype=torch.float32, device="cuda")
    oc = h.envelope(mat, spec, Fc, bc, stress=True, flags=False)
    Xc, Yc = s.pack(Fc, bc, oc["W"], oc["P"])
    cells = s.calibrate(mat, Xc, Yc, tol=GATE_TOL, quantile=GATE_QUANTILE)
    del Fc, bc, oc, Xc, Yc
    inf = WL.config4_inference(n=n_inf)
    Fi = torch.tensor(inf["F"], dtype=torch.float32, device="cuda")
    bi = torch.tensor(inf["beta_n"], dtype=torch.float32, device="cuda")
    W = torch.empty(n_inf, device="cuda")
    P = torch.empty((4, n_inf), device="cuda")
    t_plain = timed(lambda: h.envelope_into(mat, spec, Fi, bi, W, P), 5, torch)
    o64 = h.envelope(mat, spec, Fi.double(), bi.double(), stress=False, flags=False)
    W64 = o64["W"].cpu().numpy()
    del o64
    # the gate alone, then with the a-posteriori check (the reported path)
    s.set_check(0.0)
    so = s.infer(mat, spec, Fi, bi)
    gate_only = served_stats(so["W"].cpu().numpy(), W64, (so["flags"].cpu().numpy() & r1.PT_FALLBACK) == 0)
    t_gate = timed(lambda: s.infer(mat, spec, Fi, bi, out=so), 5, torch)
    s.set_check(CHECK_EPS)
    so = s.infer(mat, spec, Fi, bi)
    t_sur = timed(lambda: s.infer(mat, spec, Fi, bi, out=so), 5, torch)
    fb = (so["flags"].cpu().numpy() & r1.PT_FALLBACK) != 0
    acc = ~fb
    Wp = W.cpu().numpy()
    Ws = so["W"].cpu().numpy()
    # stored FP64 oracle values at the first inference points
    Wo, sel = golden_energies("config4_infer_oracle_f32in.json", inf)
    n_o = len(sel)
    eo = np.abs(Ws[sel] - Wo) / np.maximum(np.abs(Wo), 1e-2)
    acc_o = acc[sel]
    s.close()
    return {
        "workload": "surrogate-2d: train 2M rows (16 dirs x 201 pts, k=1), infer 1M points",
        "plain_qps": round(n_inf / t_plain, 1), "surrogate_qps": round(n_inf / t_sur, 1),
        "speedup": round(t_plain / t_sur, 3), "fallback_frac": round(float(fb.mean()), 4),
        "gate": {"cells_allowed": cells, "tol": GATE_TOL, "quantile": GATE_QUANTILE, "calibration_rows": n_cal,
                 "check_eps": CHECK_EPS},
        "erel_floor": 1e-2,
        "accepted_erel_vs_fp32_plain": served_stats(Ws, Wp.astype(np.float64), acc),
        "accepted_erel_vs_fp64_plain": served_stats(Ws, W64, acc),
        "without_check": {"speedup": round(t_plain / t_gate, 3), "accepted_erel_vs_fp64_plain": gate_only},
        "erel_vs_oracle_first_%d" % n_o: {"served": int(acc_o.sum()), "served_max": float(eo[acc_o].max()),
                                          "served_p99": float(np.percentile(eo[acc_o], 99)),
                                          "served_frac_gt_1e-3": float(np.mean(eo[acc_o] > 1e-3)),
                                          "fallback_max": float(eo[~acc_o].max())},
        "train": {"rows": n_train, "epochs": epochs, "steps": rep["steps"], "ms": round(rep["ms"], 1),
                  "val_loss": rep["val_loss"], "data_gen_ms": round(1e3 * t_data, 1)},
        "mlp": "5 -> 4 x 128 SiLU -> 5, BF16 MFMA / FP32 accumulate",
    }


def leg_surrogate_3d(h, r1, WL, torch, np, n_train=1_000_000, n_cal=1_000_000, epochs=8):
    """3D: MLP 10 -> 4x256 SiLU -> 10 trained on 3D lamination rows (256 directions
    x 513 points), against plain lamination of the 262,144-point 3D workload."""
    mat = r1.material(dim=3)
    tr = WL.config5(n=n_train, seed_tag=50)
    spec = r1.LaminationSpec(tr["levels"])
    F = torch.tensor(tr["F"], dtype=torch.float32, device="cuda")
    bn = torch.tensor(tr["beta_n"], dtype=torch.float32, device="cuda")
    out = h.envelope(mat, spec, F, bn, stress=True, flags=False)
    s = r1.Surrogate(h, dim=3, n_hidden=4, width=256, seed=2211)
    X, Y = s.pack(F, bn, out["W"], out["P"])
    del F, bn, out
    rep = s.train(mat, X, Y, epochs=epochs, batch=4096, lr=1e-3, seed=1)
    del X, Y
    cal = WL.config5(n=n_cal, seed_tag=51)
    Fc = torch.tensor(cal["F"], dtype=torch.float32, device="cuda")
    bc = torch.tensor(cal["beta_n"], dtype=torch.float32, device="cuda")
    oc = h.envelope(mat, spec, Fc, bc, stress=True, flags=False)
    Xc, Yc = s.pack(Fc, bc, oc["W"], oc["P"])
    cells = s.calibrate(mat, Xc, Yc, tol=GATE_TOL, quantile=GATE_QUANTILE)
    del Fc, bc, oc, Xc, Yc
    inf = WL.config5()
    n = inf["n"]
    Fi = torch.tensor(inf["F"], dtype=torch.float32, device="cuda")
    bi = torch.tensor(inf["beta_n"], dtype=torch.float32, device="cuda")
    W = torch.empty(n, device="cuda")
    P = torch.empty((9, n), device="cuda")
    t_plain = timed(lambda: h.envelope_into(mat, spec, Fi, bi, W, P), 3, torch)
    o64 = h.envelope(mat, spec, Fi.double(), bi.double(), stress=False, flags=False)
    W64 = o64["W"].cpu().numpy()
    del o64
    s.set_check(CHECK_EPS)
    so = s.infer(mat, spec, Fi, bi)
    t_sur = timed(lambda: s.infer(mat, spec, Fi, bi, out=so), 3, torch)
    fb = (so["flags"].cpu().numpy() & r1.PT_FALLBACK) != 0
    Wp, Ws = W.cpu().numpy(), so["W"].cpu().numpy()
    acc = ~fb
    s.close()
    return {
        "workload": "surrogate-3d: train 1M rows (256 dirs x 513 pts, k=1), infer " + inf["name"],
        "plain_qps": round(n / t_plain, 1), "surrogate_qps": round(n / t_sur, 1),
        "speedup": round(t_plain / t_sur, 3), "fallback_frac": round(float(fb.mean()), 4),
        "gate": {"cells_allowed": cells, "tol": GATE_TOL, "quantile": GATE_QUANTILE, "calibration_rows": n_cal,
                 "check_eps": CHECK_EPS},
        "erel_floor": 1e-2,
        "accepted_erel_vs_fp32_plain": served_stats(Ws, Wp.astype(np.float64), acc),
        "accepted_erel_vs_fp64_plain": served_stats(Ws, W64, acc),
        "train": {"rows": n_train, "epochs": epochs, "steps": rep["steps"], "ms": round(rep["ms"], 1),
                  "val_loss": rep["val_loss"]},
        "mlp": "10 -> 4 x 256 SiLU -> 10, BF16 MFMA / FP32 accumulate",
    }


def load_golden(name):
    """Stored FP64 oracle values (tests/golden/, written by make_oracle_golden.py from the
    oracle alone): the points with p, F, beta_n, W, P and tree."""
    with open(os.path.join(ROOT, "tests", "golden", name)) as f:
        d = json.load(f)
    return d["points"]


def golden_error(W_gpu, tree_gpu, pts, floor):
    """Energy error of GPU results at stored oracle points, relative with |W| floored, and
    how many of the points have the oracle's tree."""
    import numpy as np
    sel = np.array([q["p"] for q in pts])
    Wo = np.array([float(q["W"]) for q in pts])
    e = np.abs(W_gpu[sel] - Wo) / np.maximum(np.abs(Wo), floor)
    same = sum(all(list(tree_gpu[q["p"], k, :3]) == q["tree"][k] for k in range(len(q["tree"]))) for q in pts)
    return {"n": int(len(pts)), "energy_max": float(e.max()), "energy_p50": float(np.median(e)),
            "erel_floor": floor, "same_tree": int(same)}


def golden_energies(name, cfg):
    """Stored oracle energies W[p] for the points p of a workload (FP32-rounded inputs), after
    checking that the workload generator still draws the inputs they were computed at."""
    import hashlib
    import numpy as np
    with open(os.path.join(ROOT, "tests", "golden", name)) as f:
        d = json.load(f)
    sel = np.array([q["p"] for q in d["points"]])
    fp = hashlib.sha256(np.float32(cfg["F"][:, sel]).tobytes() +
                        np.float32(cfg["beta_n"][sel]).tobytes()).hexdigest()[:16]
    if fp != d["inputs_sha256_16"]:
        raise RuntimeError("%s was computed for other inputs than the workload generator draws" % name)
    return np.array([float(q["W"]) for q in d["points"]]), sel


def w_samples_depth1(n, lv):
    return n * (len(lv["a"]) * (lv["n_t"] - 1) + 1)


def leg_plain_2d(h, r1, WL, torch, np, reps=10):
    """Depth 1, 16 directions x 201 points (the surrogate's fallback lamination), on the
    1M inference points of the surrogate workload, with stress: one-level kernel alone."""
    cfg = WL.config4_inference(n=1_000_000)
    mat = r1.material()
    spec = r1.LaminationSpec(cfg["levels"])
    n = cfg["n"]
    F = torch.tensor(cfg["F"], dtype=torch.float32, device="cuda").contiguous()
    bn = torch.tensor(cfg["beta_n"], dtype=torch.float32, device="cuda").contiguous()
    W = torch.empty(n, device="cuda")
    P = torch.empty((4, n), device="cuda")
    h.envelope_into(mat, spec, F, bn, W, P)
    torch.cuda.synchronize()
    h.timing(True)
    h.timing_reset()
    t = timed(lambda: h.envelope_into(mat, spec, F, bn, W, P), reps, torch)
    ms, cnt = h.timing_query("depth1")
    h.timing(False)
    avg_s = ms / max(cnt, 1) / 1e3
    ws = w_samples_depth1(n, cfg["levels"][0])
    ach = FLOPS_PER_W * ws / avg_s / 1e12
    return {"workload": "plain-2d-n%d-16x201-k1 (stress on)" % n, "qps": round(n / t, 1), "ms": round(1e3 * t, 3),
            "roofline": dict(bound="alu", kernel="k_depth1", avg_ms=round(1e3 * avg_s, 4), achieved=round(ach, 2),
                             unit="TFLOP/s", peak=PEAK["f32"], frac=round(ach / PEAK["f32"], 4),
                             peak_nonpacked=PEAK_NONPACKED["f32"], frac_nonpacked=round(ach / PEAK_NONPACKED["f32"], 4),
                             w_samples_per_launch=ws, flops_per_w=FLOPS_PER_W),
            "all_finite": bool(torch.isfinite(W).all().item())}


def leg_headline_f64(h, r1, WL, torch, np):
    """The depth-2 workload in FP64, once, against the 64 stored FP64 oracle points."""
    cfg = WL.config2()
    n = cfg["n"]
    mat = r1.material_from(cfg["material"], 2)
    spec = r1.LaminationSpec(cfg["levels"])
    dt = torch.float64
    F = torch.tensor(cfg["F"], dtype=dt, device="cuda").contiguous()
    bn = torch.tensor(cfg["beta_n"], dtype=dt, device="cuda").contiguous()
    W = torch.empty(n, dtype=dt, device="cuda")
    P = torch.empty((4, n), dtype=dt, device="cuda")
    T = torch.empty((n, 3, 4), dtype=torch.int32, device="cuda")
    h.timing(True)
    h.timing_reset()
    t0 = time.perf_counter()
    h.envelope_into(mat, spec, F, bn, W, P, T)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    ms, cnt = h.timing_query("outer")
    h.timing(False)
    avg_s = ms / max(cnt, 1) / 1e3
    ach = FLOPS_PER_W * w_samples_outer_kernel(cfg) / avg_s / 1e12
    err = golden_error(W.cpu().numpy(), T.cpu().numpy(), load_golden("config2_oracle_f64.json"), 1e-3)
    return {"workload": cfg["name"] + " in FP64", "qps": round(n / t, 2), "ms": round(1e3 * t, 1),
            "roofline": dict(bound="alu", kernel="k_outer", avg_ms=round(1e3 * avg_s, 2), achieved=round(ach, 3),
                             unit="TFLOP/s", peak=PEAK["f64"], frac=round(ach / PEAK["f64"], 4),
                             flops_per_w=FLOPS_PER_W),
            "error_vs_fp64_oracle": err}


def leg_batched(h, r1, WL, torch, np):
    """Config 3: 65,536 points, per point n_t in {257..2049}, 32/64/128 directions, depth 1 or 2."""
    cfg = WL.config3()
    mat = r1.material()
    specs = [r1.LaminationSpec(t) for t in cfg["table"]]
    F = torch.tensor(cfg["F"], dtype=torch.float32, device="cuda")
    bn = torch.tensor(cfg["beta_n"], dtype=torch.float32, device="cuda")
    idx = torch.tensor(cfg["lam_idx"], dtype=torch.int32, device="cuda")
    t0 = time.perf_counter()
    plan = h.batched_plan(mat, specs, idx, torch.float32)              # plan, autotune
    out = plan.outputs(stress=True, tree=True)
    run = lambda: plan.execute(F, bn, out["W"], out["P"], out["tree"], out["flags"])
    run()                                                              # capture, first replay
    torch.cuda.synchronize()
    t_first = time.perf_counter() - t0
    t = timed(run, 1, torch)
    table, li = cfg["table"], cfg["lam_idx"]
    wsum = 0
    for k, lv in enumerate(table):
        cnt = int(np.sum(li == k))
        if len(lv) == 1:
            wsum += cnt * len(lv[0]["a"]) * (lv[0]["n_t"] - 1)
        else:
            wsum += cnt * len(lv[0]["a"]) * (lv[0]["n_t"] - 1) * (len(lv[1]["a"]) * (lv[1]["n_t"] - 1) + 1)
    W = out["W"].cpu().numpy()
    # the graph replay, timed by the host clock between synchronizations (10 s of
    # device work against microseconds of host work)
    ach = FLOPS_PER_W * wsum / t / 1e12
    plan.close()
    return {"workload": cfg["name"] + " (uneven n_t/n_dir/depth, one persistent graph launch)",
            "qps": round(cfg["n"] / t, 1), "ms": round(1e3 * t, 1), "w_samples": int(wsum),
            "w_samples_per_s": float(wsum / t), "first_call_ms": round(1e3 * t_first, 1),
            "roofline": dict(bound="alu", kernel="graph (k_bpoint, k_bouter, k_bfinal)", avg_ms=round(1e3 * t, 1),
                             achieved=round(ach, 2), unit="TFLOP/s", peak=PEAK["f32"], frac=round(ach / PEAK["f32"], 4),
                             peak_nonpacked=PEAK_NONPACKED["f32"],
                             frac_nonpacked=round(ach / PEAK_NONPACKED["f32"], 4), flops_per_w=FLOPS_PER_W),
            "error_vs_fp64_oracle": golden_error(W.astype(np.float64), out["tree"].cpu().numpy(),
                                                 load_golden("config3_oracle_f32in.json"), 1e-2),
            "all_finite": bool(np.isfinite(W).all())}


def leg_3d(h, r1, WL, torch, np):
    """Config 5: 262,144 3D points, 256 directions (Fibonacci x Fibonacci), 513 points."""
    cfg = WL.config5()
    mat = r1.material(dim=3)
    spec = r1.LaminationSpec(cfg["levels"])
    F = torch.tensor(cfg["F"], dtype=torch.float32, device="cuda")
    bn = torch.tensor(cfg["beta_n"], dtype=torch.float32, device="cuda")
    n = cfg["n"]
    W = torch.empty(n, device="cuda")
    P = torch.empty((9, n), device="cuda")
    lv = cfg["levels"][0]
    lanes = h.autotune(mat, lv["n_t"], r1.R1_F32)              # untimed, as a caller would once
    h.envelope_into(mat, spec, F, bn, W, P)
    torch.cuda.synchronize()
    h.timing(True)
    h.timing_reset()
    t = timed(lambda: h.envelope_into(mat, spec, F, bn, W, P), 3, torch)
    ms, cnt = h.timing_query("depth1")
    h.timing(False)
    avg_s = ms / max(cnt, 1) / 1e3
    ws = w_samples_depth1(n, lv)
    ach = FLOPS_PER_W * ws / avg_s / 1e12
    Wo, sel = golden_energies("config5_oracle_f32in.json", cfg)
    return {"workload": cfg["name"], "qps": round(n / t, 1), "ms": round(1e3 * t, 2), "lanes_per_line": lanes,
            "w_samples_per_s": float(ws / t),
            "roofline": dict(bound="alu", kernel="k_depth1", avg_ms=round(1e3 * avg_s, 3), achieved=round(ach, 2),
                             unit="TFLOP/s", peak=PEAK["f32"], frac=round(ach / PEAK["f32"], 4),
                             peak_nonpacked=PEAK_NONPACKED["f32"], frac_nonpacked=round(ach / PEAK_NONPACKED["f32"], 4),
                             w_samples_per_launch=ws, flops_per_w=FLOPS_PER_W),
            "erel_vs_oracle": erel_stats(W.cpu().numpy()[sel], Wo, floor=1e-2)}


FLOPS_PER_W_STVK = 15      # St. Venant-Kirchhoff sample: 7 FMA + 1 min, the exponential not counted
STVK_MATERIAL = dict(mu=1.0, lam=0.5, D_inf=0.9, D0=0.3)   # Table 6.3, STVK row


def leg_stvk(h, r1, WL, torch, np, steps=2):
    """The headline depth-2 shapes (4096 points, outer 64 x 1025, inner 32 x 257, FP32) with the
    St. Venant-Kirchhoff damage model: energy, laminate stress and tree."""
    cfg = WL.config2()
    mat = r1.material_from(STVK_MATERIAL, 2, r1.R1_STVK_DAMAGE)
    spec = r1.LaminationSpec(cfg["levels"])
    n = cfg["n"]
    F = torch.tensor(cfg["F"], dtype=torch.float32, device="cuda").contiguous()
    bn = torch.tensor(cfg["beta_n"], dtype=torch.float32, device="cuda").contiguous()
    W = torch.empty(n, device="cuda")
    P = torch.empty((4, n), device="cuda")
    T = torch.empty((n, 3, 4), dtype=torch.int32, device="cuda")
    h.envelope_into(mat, spec, F, bn, W, P, T)
    torch.cuda.synchronize()
    h.timing(True)
    h.timing_reset()
    t = timed(lambda: h.envelope_into(mat, spec, F, bn, W, P, T), steps, torch)
    outer_ms, outer_n = h.timing_query("outer")
    h.timing(False)
    avg_s = outer_ms / max(outer_n, 1) / 1e3
    flops = FLOPS_PER_W_STVK * w_samples_outer_kernel(cfg)
    achieved = flops / avg_s / 1e12
    return {"workload": cfg["name"].replace("plain-", "stvk-"), "material": STVK_MATERIAL,
            "qps": round(n / t, 1), "ms": round(1e3 * t, 1),
            "roofline": dict(bound="alu", kernel="k_outer", avg_ms=round(1e3 * avg_s, 3),
                             achieved=round(achieved, 3), unit="TFLOP/s", peak=PEAK["f32"],
                             frac=round(achieved / PEAK["f32"], 4), peak_nonpacked=PEAK_NONPACKED["f32"],
                             frac_nonpacked=round(achieved / PEAK_NONPACKED["f32"], 4),
                             flops_per_w=FLOPS_PER_W_STVK),
            "all_finite": bool(np.isfinite(W.cpu().numpy()).all())}


def tangent_bytes(d, depth, elem):
    """Algorithmic bytes per point of the tangent post-pass: F, beta_n and W read, the tree
    nodes it names read (16 B each), d^4 moduli written."""
    return elem * (d * d + 2) + 16 * (1 if depth == 1 else 3) + elem * d ** 4


def leg_tangent(h, r1, WL, torch, np, reps=20):
    """Tangent moduli (Algorithm 3) of 1M depth-1 laminates (16 directions x 201 points, FP32),
    from the trees of a plain lamination call: the post-pass kernel alone."""
    cfg = WL.config4_inference(n=1_000_000)
    mat = r1.material()
    spec = r1.LaminationSpec(cfg["levels"])
    F = torch.tensor(cfg["F"], dtype=torch.float32, device="cuda").contiguous()
    bn = torch.tensor(cfg["beta_n"], dtype=torch.float32, device="cuda").contiguous()
    out = h.envelope(mat, spec, F, bn, stress=False, tree=True, flags=False)
    A = h.laminate_tangent(mat, spec, F, bn, out["W"], out["tree"])            # warm-up
    torch.cuda.synchronize()
    h.timing(True)
    h.timing_reset()
    # One more lamination call (milliseconds of GPU work) ahead of the launches keeps the
    # stream busy while the host issues them, so they run back to back and each launch's
    # events bracket the kernel, not the host's time between calls.
    h.envelope(mat, spec, F, bn, stress=False, tree=True, flags=False)
    for _ in range(reps):
        A = h.laminate_tangent(mat, spec, F, bn, out["W"], out["tree"])
    ms, cnt = h.timing_query("tangent")
    h.timing(False)
    n = cfg["n"]
    avg_s = ms / max(cnt, 1) / 1e3
    per = tangent_bytes(2, 1, 4)
    gbs = per * n / avg_s / 1e9
    return {"workload": "tangent-2d-n%d-16x201-k1" % n, "n": n, "avg_ms": round(1e3 * avg_s, 4),
            "roofline": dict(bound="hbm", kernel="k_tangent", achieved=round(gbs, 1), unit="GB/s", peak=8000.0,
                             frac=round(gbs / 8000.0, 4), bytes_per_point=per),
            "all_finite": bool(torch.isfinite(A).all().item())}


def grid_lines_at_least(n, s, m):
    """Lines of step s with at least m nodes on a mesh of n[c] nodes per component: the
    nodes whose m-1 steps ahead stay inside, minus those whose one step back does too
    (each set a box, the product of per-component interval lengths)."""
    ahead = back = 1
    for nc, v in zip(n, s):
        lo, hi = max(0, -(m - 1) * v), min(nc, nc - (m - 1) * v)
        ahead *= max(hi - lo, 0)
        back *= max(min(hi, nc + v) - max(lo, v), 0)
    return ahead - back


def grid_line_nodes(n, steps):
    """Direction-node pairs on lines of at least 3 nodes (only those can lower a node)."""
    import numpy as np
    total = 0
    for s in np.asarray(steps).reshape(len(steps), -1):
        s = [int(v) for v in s]
        m = 3
        while True:
            c = grid_lines_at_least(n, s, m)
            if c == 0:
                break
            total += c * (3 if m == 3 else 1)
            m += 1
    return total


def grid_bytes(n_nodes, line_nodes, elem):
    """Algorithmic HBM bytes of one mesh iteration: every node of every line that can
    lower a node (at least 3 nodes) read once per direction, the previous iterate read
    and the next one written once."""
    return elem * (line_nodes + 2 * n_nodes)


def leg_grid(h, r1, WL, torch, np):
    """Global lamination on the paper's meshes (FP64, reduced direction set R^1_1):
    Table 6.1's 2D STVK and NH meshes run to the stopping rule (max decrease <= 1e-4,
    at most 20 iterations), and Table 6.3's 3D STVK mesh for 3 iterations; the 2D STVK
    mesh once more carrying the node stresses and tangent moduli (eq. 5.2, Algorithm 3)."""
    mat_t = dict(mu=1.0, lam=0.5, D_inf=0.9, D0=0.3)
    stvk2 = ((20, 41, 41, 20), (0.1, -2.0, -2.0, 0.1), 0.1, 0.07986236557499998, 20)
    cases = [("stvk-2d-672400", 2, r1.R1_STVK_DAMAGE) + stvk2 + (False,),
             ("nh-2d-648025", 2, r1.R1_NEOHOOKE_DAMAGE, (23, 35, 35, 23), (0.1, -2.55, -2.55, 0.1), 0.15, 0.06, 20,
              False),
             ("stvk-3d-5832000", 3, r1.R1_STVK_DAMAGE, (20, 3, 3, 3, 20, 3, 3, 3, 20),
              (0.1, -0.1, -0.1, -0.1, 0.1, -0.1, -0.1, -0.1, 0.1), 0.1, 0.07986236557499998, 3, False),
             ("stvk-2d-672400+stress+tangent", 2, r1.R1_STVK_DAMAGE) + stvk2 + (True,)]
    out = []
    for name, dim, model, n, lo, delta, beta, k_max, carry in cases:
        g = r1.grid(dim, n, lo, delta)
        steps = r1.grid_r11(dim)
        mat = r1.material_from(mat_t, dim, model)
        P = A = None
        if carry:
            W, P, A = h.grid_energy(mat, g, beta, torch.float64, stress=True, tangent=True)
        else:
            W = h.grid_energy(mat, g, beta, torch.float64)
        W0 = W.clone()
        # one untimed iteration first: it sizes the handle's workspace for this mesh
        Wc = W0.clone()
        h.grid_laminate(g, steps, Wc, k_max=1, tol=0.0, P=None if P is None else P.clone(),
                        A=None if A is None else A.clone())
        del Wc
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        hist = h.grid_laminate(g, steps, W, k_max=k_max, tol=1e-4, P=P, A=A)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        # per-launch kernel time from HIP events, in a second run (the events add gaps
        # between the launches, so the whole-run time above is taken without them)
        if not carry:
            W.copy_(W0)
            torch.cuda.synchronize()
            h.timing(True)
            h.timing_reset()
            h.grid_laminate(g, steps, W, k_max=k_max, tol=1e-4)
            torch.cuda.synchronize()
            ms, cnt = h.timing_query("grid_lines")
            h.timing(False)
        else:
            ms, cnt = 0.0, 0
        nodes = r1.grid_size(g)
        per_it = t / len(hist)
        line_nodes = grid_line_nodes(n, steps)
        gbs = grid_bytes(nodes, line_nodes, 8) / per_it / 1e9
        out.append({"mesh": name, "nodes": nodes, "directions": len(steps), "iterations": len(hist),
                    "decrease": [float("%.6g" % v) for v in hist], "ms_total": round(1e3 * t, 2),
                    "ms_per_iteration": round(1e3 * per_it, 3),
                    "node_updates_per_s": float(nodes * len(hist) / t),
                    "lines_kernel_ms_per_launch": round(ms / cnt, 4) if cnt else None})
        if not carry:
            out[-1]["roofline"] = dict(bound="hbm", kernel="k_grid_hulls + k_grid_pick", achieved=round(gbs, 1),
                                       unit="GB/s", peak=8000.0, frac=round(gbs / 8000.0, 4),
                                       bytes_per_iteration=grid_bytes(nodes, line_nodes, 8),
                                       line_nodes_per_iteration=line_nodes)
        del W, W0, P, A
    return {"workload": "global lamination on the paper's meshes (Tables 6.1, 6.3), FP64, R^1_1", "meshes": out}


# ---------------------------------------------------------------- main

def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--dtype", choices=["f32", "f64"], default="f32")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--quick", action="store_true", help="headline workload only")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (HBM counter calibration)")
    ap.add_argument("--leg", choices=["surrogate", "batched", "plain_3d", "plain_2d", "headline_f64", "surrogate_3d",
                                      "stvk", "tangent", "grid"],
                    help="only run this secondary leg and print its result (a profiling aid)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this benchmark runs on one GPU only (quadrature points are independent, so "
              "several GPUs would each take a cost-balanced share of them); got --gpus %d" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2211_14318_amd import r1, workloads as WL

    if args.copy_probe:
        x = torch.empty(args.copy_probe * (1 << 18), dtype=torch.float32, device="cuda").fill_(1.0)
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": x.numel() * 4}))
        return

    if args.leg:
        legs = dict(surrogate=leg_surrogate, batched=leg_batched, plain_3d=leg_3d, plain_2d=leg_plain_2d,
                    headline_f64=leg_headline_f64, surrogate_3d=leg_surrogate_3d, stvk=leg_stvk,
                    tangent=leg_tangent, grid=leg_grid)
        h = r1.Handle(0)
        res = legs[args.leg](h, r1, WL, torch, np)
        print(json.dumps({"leg": args.leg, **res}))
        h.close()
        return

    cfg = WL.config2()
    dt = torch.float32 if args.dtype == "f32" else torch.float64
    h = r1.Handle(0)
    mat = r1.material_from(cfg["material"], 2)
    spec = r1.LaminationSpec(cfg["levels"])
    n = cfg["n"]
    F = torch.tensor(cfg["F"], dtype=dt, device="cuda").contiguous()
    bn = torch.tensor(cfg["beta_n"], dtype=dt, device="cuda").contiguous()
    W = torch.empty(n, dtype=dt, device="cuda")
    P = torch.empty((4, n), dtype=dt, device="cuda")
    T = torch.empty((n, 3, 4), dtype=torch.int32, device="cuda")
    fl = torch.empty(n, dtype=torch.int32, device="cuda")

    def step():
        h.envelope_into(mat, spec, F, bn, W, P, T, fl)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    h.timing(True)
    h.timing_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    outer_ms, outer_n = h.timing_query("outer")
    h.timing(False)
    ms_per_step = 1e3 * elapsed / args.steps
    Wn = W.double().cpu().numpy()
    Pn = P.double().cpu().numpy()
    assert np.isfinite(Wn).all(), "non-finite envelope values"
    value = n / (elapsed / args.steps)

    flops = FLOPS_PER_W * w_samples_outer_kernel(cfg)
    avg_s = outer_ms / max(outer_n, 1) / 1e3
    achieved = flops / avg_s / 1e12
    roof = dict(bound="alu", achieved=round(achieved, 3), peak=PEAK[args.dtype], unit="TFLOP/s",
                frac=round(achieved / PEAK[args.dtype], 4),
                traffic=measured_traffic() if args.dtype == "f32" else None,
                peak_nonpacked=PEAK_NONPACKED[args.dtype],
                frac_nonpacked=round(achieved / PEAK_NONPACKED[args.dtype], 4),
                kernel="k_outer", avg_ms=round(outer_ms / max(outer_n, 1), 3),
                w_samples_per_launch=w_samples_outer_kernel(cfg), flops_per_w=FLOPS_PER_W)
    out = {
        "metric": "QP envelope evals/sec (plain lamination, depth 2, energy + laminate stress)",
        "value": round(value, 2),
        "unit": "QP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {"workload": cfg["name"], "n_qp": n, "depth": 2,
                   "outer": "64 directions x 1025 points, tau 1.5",
                   "inner": "32 directions x 257 points, tau 1.5",
                   "w_evals_per_step": w_samples_outer_kernel(cfg)},
        "roofline": roof,
    }
    log("headline: %.1f QP/s, k_outer %.3f ms (%.1f%% of peak)" % (value, roof["avg_ms"], 100 * roof["frac"]))
    if args.dtype == "f32":
        out["error_vs_stored_oracle"] = golden_error(Wn, T.cpu().numpy(), load_golden("config2_oracle_f32in.json"),
                                                     1e-2)
    if not args.quick:
        out["headline_f64"] = leg_headline_f64(h, r1, WL, torch, np)
        log("headline in FP64: %.1f QP/s, k_outer %.3f%% of peak" % (out["headline_f64"]["qps"],
                                                                     100 * out["headline_f64"]["roofline"]["frac"]))
        out["plain_2d"] = leg_plain_2d(h, r1, WL, torch, np)
        log("plain 2d depth-1 leg: %.1f QP/s" % out["plain_2d"]["qps"])
        out["surrogate"] = leg_surrogate(h, r1, WL, torch, np)
        log("surrogate leg: speedup %.3f, fallback %.3f" % (out["surrogate"]["speedup"],
                                                         out["surrogate"]["fallback_frac"]))
        out["batched"] = leg_batched(h, r1, WL, torch, np)
        log("batched leg: %.1f QP/s" % out["batched"]["qps"])
        out["plain_3d"] = leg_3d(h, r1, WL, torch, np)
        log("3d leg: %.1f QP/s" % out["plain_3d"]["qps"])
        out["stvk"] = leg_stvk(h, r1, WL, torch, np)
        log("stvk leg: %.1f QP/s, k_outer %.1f ms" % (out["stvk"]["qps"], out["stvk"]["roofline"]["avg_ms"]))
        out["tangent"] = leg_tangent(h, r1, WL, torch, np)
        log("tangent leg: %.4f ms per 1M points" % out["tangent"]["avg_ms"])
        out["grid"] = leg_grid(h, r1, WL, torch, np)
        log("grid leg: " + ", ".join("%s %d it %.1f ms" % (m["mesh"], m["iterations"], m["ms_total"])
                                     for m in out["grid"]["meshes"]))
        out["surrogate_3d"] = leg_surrogate_3d(h, r1, WL, torch, np)
        log("3d surrogate leg: speedup %.3f, fallback %.3f" % (out["surrogate_3d"]["speedup"],
                                                            out["surrogate_3d"]["fallback_frac"]))
    h.close()
    if not args.no_cpu_baseline:
        workers = os.cpu_count() or 1          # every host core: one oracle point per process
        log("cpu baseline: %d oracle processes" % workers)
        base, ref = cpu_baseline(workers)
        out["cpu_baseline"] = base
        idx = sorted(ref)
        out["error"] = {"vs": "FP64 oracle on the cpu_baseline points",
                        "energy_erel": erel_stats(Wn[idx], [ref[i][0] for i in idx]),
                        "energy_erel_floor_1e-2": erel_stats(Wn[idx], [ref[i][0] for i in idx], 1e-2),
                        "stress_max_abs": float(np.max(np.abs(Pn[:, idx].T - np.array([ref[i][1] for i in idx]))))}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
