"""Writes the stored oracle values that the full-size GPU parity tests and the
bench's error figures compare against.  It calls only the FP64 oracle (oracle/)
and the seeded input generators (paper_2211_14318_amd/workloads.py), never the
GPU library.  Run from the repository root:

    python tests/golden/make_oracle_golden.py [--workers N]

Outputs (JSON; floats written with repr, so they read back exactly):
  config2_oracle_f64.json   64 seeded points of the depth-2 workload
                            (4096 points, outer 64 x 1025, inner 32 x 257, tau 1.5)
                            at their FP64 inputs: W^2, P^2, the tree and its gaps
  config2_oracle_f32in.json the first 32 of those points at FP32-rounded inputs
                            (the inputs the FP32 path reads)
  config3_oracle_f32in.json the uneven batch (65,536 points, 24 table entries):
                            the first 2 points of every entry at FP32-rounded inputs
  config4_infer_oracle_f32in.json  W^1 at the first 2000 of the surrogate's 1M inference
                            points (16 directions x 201 points, depth 1), FP32-rounded inputs
  config5_oracle_f32in.json W^1 at 64 evenly spaced points of the 3D workload (262,144
                            points, 256 directions x 513 points), FP32-rounded inputs
Each point takes the oracle's full two-level recursion (about 40 s of one core for
the depth-2 workload), so the script runs a process pool.
"""
import argparse
import concurrent.futures as cf
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import oracle as O                      # noqa: E402
from paper_2211_14318_amd import workloads as WL     # noqa: E402

CONFIG2_SEED = 20221128
CONFIG2_N64 = 64
CONFIG2_N32 = 32
CONFIG3_PER_ENTRY = 2
CONFIG4_N = 2000
CONFIG5_N = 64


def _energy(args):
    dim, mat_d, levels, F, bn = args
    mat = O.material(dim=dim, mu=mat_d["mu"], lam=mat_d["lam"], D_inf=mat_d["D_inf"], D0=mat_d["D0"])
    spec = O.LaminationSpec([(l["a"], l["b"], l["n_t"], l["tau"]) for l in levels])
    W, _, _ = O.envelope(mat, spec, np.asarray(F, dtype=np.float64).reshape(dim, dim), float(bn))
    return W


def inputs_fingerprint(F, bn):
    """sha256 (16 hex digits) of the FP32-rounded inputs, to detect a changed generator."""
    import hashlib
    return hashlib.sha256(np.float32(F).tobytes() + np.float32(bn).tobytes()).hexdigest()[:16]


def _point(args):
    mat_d, levels, F, bn = args
    mat = O.material(dim=2, mu=mat_d["mu"], lam=mat_d["lam"], D_inf=mat_d["D_inf"], D0=mat_d["D0"])
    spec = O.LaminationSpec([(l["a"], l["b"], l["n_t"], l["tau"]) for l in levels])
    W, P, tree = O.envelope(mat, spec, np.asarray(F, dtype=np.float64).reshape(2, 2), float(bn), want_tree=True)
    return dict(W=W, P=[float(v) for v in np.asarray(P).ravel()],
                tree=[[t["dir"], t["i_minus"], t["i_plus"]] for t in tree[:len(levels) * 2 - 1]],
                dir_gap=[t["dir_gap"] for t in tree[:len(levels) * 2 - 1]],
                bridge_gap=[t["bridge_gap"] for t in tree[:len(levels) * 2 - 1]])


def _f32(x):
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def _dump(path, header, points):
    def enc(v):
        if isinstance(v, float) and not np.isfinite(v):
            return "inf" if v > 0 else ("-inf" if v < 0 else "nan")
        return v

    def walk(o):
        if isinstance(o, dict):
            return {k: walk(v) for k, v in o.items()}
        if isinstance(o, list):
            return [walk(v) for v in o]
        return enc(o)

    with open(path, "w") as f:
        json.dump(dict(header, points=walk(points)), f, indent=0)
        f.write("\n")


def config2_sample():
    """The 64 sampled point indices of the depth-2 workload (sorted)."""
    rng = np.random.default_rng(CONFIG2_SEED)
    return np.sort(rng.choice(4096, CONFIG2_N64, replace=False))


def config3_sample(cfg):
    """The first CONFIG3_PER_ENTRY points of every table entry, entry by entry."""
    out = []
    for k in range(len(cfg["table"])):
        out.extend(int(p) for p in np.nonzero(cfg["lam_idx"] == k)[0][:CONFIG3_PER_ENTRY])
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workers", type=int, default=os.cpu_count() or 8)
    ap.add_argument("--only", choices=["config2", "config3", "config4", "config5"], default=None)
    args = ap.parse_args()
    cmd = "python tests/golden/make_oracle_golden.py"
    cite = ("FP64 oracle (oracle/*.c): successive lamination of eq. 3.3 along the discrete lines of "
            "Section 4.1, Algorithm 1 for each line, stress by eq. 5.2 / Algorithm 3; arXiv 2211.14318")
    t0 = time.time()
    with cf.ProcessPoolExecutor(args.workers) as ex:
        if args.only in (None, "config2"):
            cfg = WL.config2()
            sel = config2_sample()
            jobs = [(cfg["material"], cfg["levels"], cfg["F"][:, p], cfg["beta_n"][p]) for p in sel]
            jobs += [(cfg["material"], cfg["levels"], _f32(cfg["F"][:, p]), _f32(cfg["beta_n"][p]))
                     for p in sel[:CONFIG2_N32]]
            res = list(ex.map(_point, jobs))
            pts64 = [dict(p=int(p), F=[float(v) for v in cfg["F"][:, p]], beta_n=float(cfg["beta_n"][p]), **r)
                     for p, r in zip(sel, res[:CONFIG2_N64])]
            pts32 = [dict(p=int(p), F=[float(v) for v in _f32(cfg["F"][:, p])],
                          beta_n=float(_f32(cfg["beta_n"][p])), **r)
                     for p, r in zip(sel[:CONFIG2_N32], res[CONFIG2_N64:])]
            hdr = dict(workload=cfg["name"], source=cite, command=cmd, seed=CONFIG2_SEED)
            _dump(os.path.join(HERE, "config2_oracle_f64.json"), dict(hdr, inputs="FP64"), pts64)
            _dump(os.path.join(HERE, "config2_oracle_f32in.json"), dict(hdr, inputs="FP32-rounded"), pts32)
            print("config2: %d + %d points, %.0f s" % (len(pts64), len(pts32), time.time() - t0), flush=True)
        if args.only in (None, "config3"):
            cfg = WL.config3()
            sel = config3_sample(cfg)
            jobs = [(cfg["material"], cfg["table"][int(cfg["lam_idx"][p])], _f32(cfg["F"][:, p]),
                     _f32(cfg["beta_n"][p])) for p in sel]
            res = list(ex.map(_point, jobs))
            pts = [dict(p=p, entry=int(cfg["lam_idx"][p]), F=[float(v) for v in _f32(cfg["F"][:, p])],
                        beta_n=float(_f32(cfg["beta_n"][p])), **r) for p, r in zip(sel, res)]
            hdr = dict(workload=cfg["name"], source=cite, command=cmd, inputs="FP32-rounded",
                       per_entry=CONFIG3_PER_ENTRY)
            _dump(os.path.join(HERE, "config3_oracle_f32in.json"), hdr, pts)
            print("config3: %d points, %.0f s" % (len(pts), time.time() - t0), flush=True)
        for tag in ("config4", "config5"):
            if args.only not in (None, tag):
                continue
            if tag == "config4":
                cfg = WL.config4_inference(n=1_000_000)
                sel = np.arange(CONFIG4_N)
            else:
                cfg = WL.config5()
                sel = np.linspace(0, cfg["n"] - 1, CONFIG5_N).astype(int)
            dim = cfg["dim"]
            Fs, bs = cfg["F"][:, sel], cfg["beta_n"][sel]
            jobs = [(dim, cfg["material"], cfg["levels"], _f32(Fs[:, k]), _f32(bs[k])) for k in range(len(sel))]
            W = list(ex.map(_energy, jobs, chunksize=16))
            hdr = dict(workload=cfg["name"], source=cite, command=cmd, inputs="FP32-rounded",
                       inputs_sha256_16=inputs_fingerprint(Fs, bs))
            _dump(os.path.join(HERE, "%s_oracle_f32in.json" % ("config4_infer" if tag == "config4" else tag)), hdr,
                  [dict(p=int(p), W=float(w)) for p, w in zip(sel, W)])
            print("%s: %d points, %.0f s" % (tag, len(sel), time.time() - t0), flush=True)


if __name__ == "__main__":
    main()
