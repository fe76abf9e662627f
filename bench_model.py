"""Accuracy of the paper's performance model on MI355X (Secs. 5.2 and 6.4):
for partially diagonal matrices, the measured relative performance of
M-HDC over CSR, RP_exe = t(CSR) / t(M-HDC), against the estimate RP_est =
V(CSR) / V(M-HDC) from the byte volumes (Eq. 28 with v_x = 1, as each
handle reports it), over theta in {0.5 .. 0.9} and n_b in {32 .. 1024};
relative error RE = (RP_est - RP_exe) / RP_exe (the measure of Figs. 29-30).

    python bench_model.py [--steps 50]

Matrices: 27-point 192^3 with the octant drop probabilities (the
partially diagonal benchmark case), 27-point 160^3 with one global drop
probability 0.2 / 0.4, 19-point 160^3 with drop 0.3 and one random column
per row; values N(0,1), diagonal 1.1 |row sum|.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def timed(fn, steps, warmup, stream):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(3):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1) / 1e3 / steps)
    return best


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    args = ap.parse_args()

    import numpy as np
    import torch

    from paper_2105_04937_amd import mhdc, synth
    mhdc.lib()
    s = torch.cuda.current_stream()
    cases = (("27-point 192^3, octant drops", 192, 27, list(synth.OCTANT_DROP), 2, 3),
             ("27-point 160^3, drop 0.2", 160, 27, 0.2, 0, 11),
             ("27-point 160^3, drop 0.4", 160, 27, 0.4, 0, 12),
             ("19-point 160^3, drop 0.3, +1 random/row", 160, 19, 0.3, 1, 13))
    thetas = (0.5, 0.6, 0.7, 0.8, 0.9)
    nbs = (32, 64, 128, 256, 512, 1024)
    rows = []
    for name, N, pts, drop, extra, seed in cases:
        rp, ci, v = synth.stencil_matrix_gpu(N, seed, points=pts, drop=drop, extra_per_row=extra)
        n = rp.numel() - 1
        g = torch.Generator(device="cuda")
        g.manual_seed(seed)
        x = torch.rand(n, generator=g, device="cuda", dtype=torch.float64) * 2 - 1
        y = torch.empty_like(x)
        csr = mhdc.CSRMatrix.from_csr(rp, ci, v)
        t_csr = timed(lambda: csr.spmv(x, y, s), args.steps, args.warmup, s)
        csr.close()
        for th in thetas:
            for nb in nbs:
                h = mhdc.MHDCMatrix.from_csr(rp, ci, v, nb, th)
                inf = h.info()
                t = timed(lambda: h.spmv(x, y, s), args.steps, args.warmup, s)
                h.close()
                rp_exe = t_csr / t
                rows.append(dict(matrix=name, theta=th, n_b=nb, alpha=round(inf["alpha"], 4),
                                 beta=round(inf["beta"], 4), rp_est=round(inf["rp_est"], 4),
                                 rp_exe=round(rp_exe, 4),
                                 re=round((inf["rp_est"] - rp_exe) / rp_exe, 4),
                                 us=round(t * 1e6, 2), csr_us=round(t_csr * 1e6, 2)))
        best = max((r for r in rows if r["matrix"] == name), key=lambda r: r["rp_exe"])
        log("%-40s CSR %.1f us; best M-HDC %.1f us at theta %.1f n_b %d (RP_exe %.3f, RP_est %.3f)"
            % (name, t_csr * 1e6, best["us"], best["theta"], best["n_b"], best["rp_exe"],
               best["rp_est"]))
        del rp, ci, v, x, y
        torch.cuda.empty_cache()
    re = np.array([r["re"] for r in rows])
    by_nb = {str(nb): round(float(np.mean(np.abs([r["re"] for r in rows if r["n_b"] == nb]))), 4)
             for nb in nbs}
    summary = dict(points=len(rows), mean_abs_re=round(float(np.mean(np.abs(re))), 4),
                   share_abs_re_le_0_05=round(float(np.mean(np.abs(re) <= 0.05)), 3),
                   mean_abs_re_by_n_b=by_nb)
    log(json.dumps(summary))
    print(json.dumps({"metric": "performance-model accuracy (RE of RP_est vs measured), "
                                "FP64, 1xMI355X", "value": summary["mean_abs_re"],
                      "unit": "|RE|", "higher_is_better": False, "summary": summary,
                      "rows": rows}))


if __name__ == "__main__":
    main()
