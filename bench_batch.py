"""Benchmark of the batched workload: 64 matrices of uneven size, each with
its own number of right-hand sides, in one persistent launch replayed from a
HIP graph, against 64 separate launches.

    python bench_batch.py [--count 64] [--steps K] [--warmup W]
                          [--layouts colmajor,rowmajor]

Matrices: grid side U{16..96}, stencil drawn from {7, 19, 27} points, one
drop probability U[0, 0.3], values N(0,1), diagonal 1.1*|row sum|, k ~
U{1..16} right-hand sides; matrix i uses seed 4000 + i.  The autotuner
(mhdc_autotune) picks n_b and the launch shape per matrix from timed runs;
mhdc_batch_tune picks the batch's workgroup size.  A step is one product of
all matrices with all their right-hand sides, inputs resident in HBM.
Right-hand sides are column-major (k_i rows of n_i) or stored row by row
(n_i rows of k_i, the row-major batch kernel); both are timed.

Prints one JSON line; value = GFLOP/s = sum_i 2*nnz_i*k_i / (time per step).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def timed(fn, steps, warmup, stream):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3 / steps


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--count", type=int, default=64)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--theta", type=float, default=0.6)
    ap.add_argument("--layouts", default="colmajor,rowmajor")
    ap.add_argument("--fixed-only", action="store_true",
                    help="skip the autotuner: only the n_b = 256 handles (for counter runs)")
    args = ap.parse_args()
    layouts = args.layouts.split(",")

    import numpy as np
    import torch

    from paper_2105_04937_amd import mhdc, synth

    mhdc.lib()
    stream = torch.cuda.current_stream()
    cands = (32, 64, 128, 256, 512)
    tuned, fixed, Xs, meta = [], [], [], []
    t_tune = 0.0
    for i in range(args.count):
        m, k = synth.batch_member(i)
        d = mhdc.to_device(m)
        fixed.append(mhdc.MHDCMatrix.from_csr(*d, 256, args.theta))
        if args.fixed_only:
            res = dict(n_b=256, launch=None)
        else:
            t0 = time.perf_counter()
            h, res = mhdc.autotune(*d, args.theta, nrhs=k, nb_candidates=cands)
            t_tune += time.perf_counter() - t0
            tuned.append(h)
        X = np.random.default_rng([4000 + i, 2]).uniform(-1, 1, size=(k, m.n))
        Xs.append(torch.from_numpy(np.ascontiguousarray(X)).cuda())
        meta.append(dict(n=m.n, nnz=m.nnz, k=k, points=m.meta["points"], n_b=res["n_b"],
                         launch=res["launch"]))
        del d
        if i % 8 == 7:
            log("prepared %d matrices" % (i + 1))

    Xs_rm = [X.t().contiguous() for X in Xs] if "rowmajor" in layouts else []

    def separate(mats, Xl, Ys, rowmajor):
        def f():
            for h, X, Y in zip(mats, Xl, Ys):
                if rowmajor:
                    h.spmm_rowmajor(X, Y, stream)
                else:
                    h.spmm(X, Y, stream)
        return f

    res = {}
    runs = [(lab, mats, lay) for lay in layouts
            for lab, mats in (("autotuned", tuned), ("n_b256", fixed)) if mats]
    for label, mats, lay in runs:
        rowmajor = lay == "rowmajor"
        Xl = Xs_rm if rowmajor else Xs
        label = label if not rowmajor else label + "_rowmajor"
        b = mhdc.Batch(mats, Xl, layout=lay)
        wg, _ = b.tune(stream)
        info = b.info()
        t_graph = timed(lambda: b.graph_launch(stream), args.steps, args.warmup, stream)
        t_run = timed(lambda: b.run(stream), args.steps, args.warmup, stream)
        Ys_sep = [torch.empty_like(X) for X in Xl]
        t_sep = timed(separate(mats, Xl, Ys_sep, rowmajor), args.steps, args.warmup, stream)
        b.run(stream)
        torch.cuda.synchronize()
        same = all(torch.equal(a.view(torch.int64), c.view(torch.int64))
                   for a, c in zip(b.Ys, Ys_sep))
        res[label] = dict(wg=wg, grid=info["grid"], tiles=info["total_tiles"],
                          graph_us=round(t_graph * 1e6, 1), run_us=round(t_run * 1e6, 1),
                          separate_us=round(t_sep * 1e6, 1),
                          gflops_graph=round(info["flops"] / t_graph / 1e9, 1),
                          gb_per_s_graph=round(info["bytes_alg"] / t_graph / 1e9, 1),
                          gflops_separate=round(info["flops"] / t_sep / 1e9, 1),
                          speedup_vs_separate=round(t_sep / t_graph, 3),
                          bit_identical_to_separate=bool(same),
                          bytes_alg=info["bytes_alg"], flops=info["flops"])
        log("%-9s graph %.1f us  run %.1f us  separate %.1f us  %.1f GFLOP/s  %.0f GB/s" % (
            label, t_graph * 1e6, t_run * 1e6, t_sep * 1e6, info["flops"] / t_graph / 1e9,
            info["bytes_alg"] / t_graph / 1e9))
        b.close()

    best = res[("autotuned" if tuned else "n_b256") +
               ("" if "colmajor" in layouts else "_rowmajor")]
    rec = {
        "metric": "batched M-HDC SpMM GFLOP/s (one persistent hipGraph launch), FP64, 1xMI355X",
        "value": best["gflops_graph"], "unit": "GFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(best["graph_us"] / 1e3, 4), "higher_is_better": True,
        "dtype": "f64", "data": "synthetic (seeded stencil matrices, X ~ U[-1,1])",
        "config": {"workload": "%d matrices, side U{16..96}, 7/19/27-point, drop U[0,0.3], "
                               "k U{1..16}" % args.count,
                   "rows": sum(d["n"] for d in meta), "nnz": sum(d["nnz"] for d in meta),
                   "rhs_total": sum(d["k"] for d in meta)},
        "roofline": {"bound": "hbm", "achieved": best["gb_per_s_graph"], "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": round(best["gb_per_s_graph"] / PEAK_HBM_GBS, 4)},
        "autotune_s": round(t_tune, 2),
        "n_b_chosen": {str(nb): sum(1 for d in meta if d["n_b"] == nb) for nb in cands},
        "variants": res,
    }
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
