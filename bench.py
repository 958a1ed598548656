"""Benchmark: quadrature-point envelope evaluations per second on one MI355X.

Workload (one step): rank-one lamination of 4,096 2D quadrature points to
depth 2 -- outer level 64 directions x 1,025 points (tau 1.5), inner level 32
directions x 257 points -- energy, laminate stress and lamination tree, in
FP32 (or FP64 with --dtype f64).  Inputs are seeded synthetic gradients
F = I + 0.3 N(0,1) (det F > 0.1) and beta_n ~ U[0, 0.5], resident in HBM.

Prints one JSON line.  `roofline` prices the dominant kernel (the outer-line
kernel, which evaluates every inner envelope) by its algorithmic flops
(18 per W sample) against the FP32 (FP64) vector peak, timed with HIP events
on its launch stream.  `cpu_baseline` times the FP64 oracle on a bounded
sample of the same workload on the host's cores.
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


def w_samples_outer_kernel(cfg):
    """Distinct W evaluations of one outer-kernel launch: every outer line's
    non-centre samples are inner envelopes, each n_dir_i*(n_t_i - 1) + 1 samples."""
    lo, li = cfg["levels"]
    inner = len(li["a"]) * (li["n_t"] - 1) + 1
    return cfg["n"] * len(lo["a"]) * (lo["n_t"] - 1) * inner


def _oracle_worker(args):
    idx, dtype = args
    from oracle import oracle as O
    from paper_2211_14318_amd import workloads as WL
    cfg = WL.config2()
    m = cfg["material"]
    mat = O.material(dim=2, mu=m["mu"], lam=m["lam"], D_inf=m["D_inf"], D0=m["D0"])
    spec = O.LaminationSpec([(l["a"], l["b"], l["n_t"], l["tau"]) for l in cfg["levels"]])
    F = cfg["F"][:, idx].reshape(2, 2)
    t0 = time.time()
    O.envelope(mat, spec, F, cfg["beta_n"][idx], want_tree=True)
    return time.time() - t0


def cpu_baseline(workers):
    from oracle import oracle as O
    O.build(force=False)
    t0 = time.time()
    with mp.get_context("spawn").Pool(workers) as pool:
        per = pool.map(_oracle_worker, [(i, "f64") for i in range(workers)])
    wall = time.time() - t0
    return dict(value=workers / wall, unit="QP/s", cores=workers, kind="oracle",
                sample="first %d points of the workload, one point per process (energy, stress and "
                       "tree, FP64 serial oracle), %.1f s wall, %.1f s per point" %
                       (workers, wall, sum(per) / len(per)))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--dtype", choices=["f32", "f64"], default="f32")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this benchmark runs on one GPU only (quadrature points are independent; "
              "the multi-GPU split is described in DESIGN.md); got --gpus %d" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2211_14318_amd import r1, workloads as WL

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
    assert torch.isfinite(W).all().item(), "non-finite envelope values"
    value = n / (elapsed / args.steps)

    flops = FLOPS_PER_W * w_samples_outer_kernel(cfg)
    avg_s = outer_ms / max(outer_n, 1) / 1e3
    achieved = flops / avg_s / 1e12
    roof = dict(bound="alu", achieved=round(achieved, 3), peak=PEAK[args.dtype], unit="TFLOP/s",
                frac=round(achieved / PEAK[args.dtype], 4), traffic=None,
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
    h.close()
    if not args.no_cpu_baseline:
        workers = min(16, os.cpu_count() or 1)
        out["cpu_baseline"] = cpu_baseline(workers)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
