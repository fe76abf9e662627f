"""Stencil study of Sec. 6.3 on one MI355X: the CSR, DIA (unblocked, Fig. 5)
and B-DIA (blocked) kernels on the paper's banded 1D-3point, 2D-5point and
3D-7point matrices for n in [1e4, 5e7], the relative performance at
n = 5e7 next to the byte-model estimates of Eqs. 9, 16 and 19, and the
B-DIA tile size sweep at n = 1e7 (the GPU counterpart of Fig. 24's bl).

    python bench_stencil.py [--max-n 5e7] [--n-loops 5]

Matrices: a_ij != 0 for j - i in {0, +-1} / {0, +-1, +-n_x} (n_x = floor
sqrt n) / {0, +-1, +-n_x, +-n_x^2} (n_x = floor cbrt n), 0 <= j < n;
off-diagonals U[-1, -0.5], diagonal 1.01 |row sum|; x ~ U[-1, 1].  DIA and
B-DIA run on one HDC handle with theta = 0 (all band diagonals, empty CSR
part): hdc_spmv_unblocked is Fig. 5's kernel (one pass over y per
diagonal), hdc_spmv the blocked tile kernel.  Timing per Fig. 18: best of
n_loops of the mean over n_ites back-to-back calls (n_ites scaled with n).
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

B_RATIO = 0.5  # b = b_int / b_fp for INT32 indices and FP64 values
GAMMA_PAPER = {3: 1.0 / 3.0, 5: 1.0 / 5.0, 7: 3.0 / 7.0}  # Sec. 6.3's choices


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def model_ratios(nd, gamma, b=B_RATIO):
    """P(DIA)/P(CSR) = V(CSR)/V(DIA) from Eq. 9, P(B-DIA)/P(CSR) from
    Eq. 16, P(B-DIA)/P(DIA) from Eq. 19 (Sec. 5.1)."""
    dia_csr = 1.0 + (b * (nd + 1) - (3.0 - gamma) * nd) / (4.0 * nd + 1.0)
    bdia_csr = 1.0 + b * (nd + 1) / ((1.0 + gamma) * nd + 1.0)
    bdia_dia = 1.0 + (3.0 - gamma) * nd / ((1.0 + gamma) * nd + 1.0)
    return dict(dia_over_csr=dia_csr, bdia_over_csr=bdia_csr, bdia_over_dia=bdia_dia)


def paper_time(fn, n_ites, n_loops, stream):
    import torch
    fn()
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(n_loops):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(n_ites):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1) / 1e3 / n_ites)
    return best


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--max-n", type=float, default=5e7)
    ap.add_argument("--n-loops", type=int, default=5)
    ap.add_argument("--bl-n", type=float, default=1e7)
    args = ap.parse_args()

    import torch

    from paper_2105_04937_amd import mhdc, synth
    mhdc.lib()
    dev = torch.device("cuda:0")
    s = torch.cuda.current_stream(dev)
    sizes = [n for n in (1e4, 3e4, 1e5, 3e5, 1e6, 3e6, 1e7, 5e7) if n <= args.max_n]
    rows, comparison, bl_sweep = [], {}, {}
    for points in (3, 5, 7):
        nd = points
        for nf in sizes:
            n = int(nf)
            rp, ci, v = synth.banded_stencil_gpu(n, points, 6, device=dev)
            nnz = ci.numel()
            g = torch.Generator(device=dev)
            g.manual_seed(n)
            x = torch.rand(n, generator=g, device=dev, dtype=torch.float64) * 2 - 1
            y = torch.empty_like(x)
            n_ites = max(10, min(1000, (1 << 27) // max(n * nd, 1)))
            csr = mhdc.CSRMatrix.from_csr(rp, ci, v)
            hdc = mhdc.HDCMatrix.from_csr(rp, ci, v, 0.0)
            assert hdc.info()["R"] == 0 and hdc.info()["K"] == len(synth.banded_offsets(n, points))
            t_csr = paper_time(lambda: csr.spmv(x, y, s), n_ites, args.n_loops, s)
            t_dia = paper_time(lambda: hdc.spmv_unblocked(x, y, s), n_ites, args.n_loops, s)
            t_bdia = paper_time(lambda: hdc.spmv(x, y, s), n_ites, args.n_loops, s)
            rec = dict(points=points, n=n, nnz=nnz, n_ites=n_ites,
                       csr_gflops=round(2 * nnz / t_csr / 1e9, 1),
                       dia_gflops=round(2 * nnz / t_dia / 1e9, 1),
                       bdia_gflops=round(2 * nnz / t_bdia / 1e9, 1),
                       csr_us=round(t_csr * 1e6, 2), dia_us=round(t_dia * 1e6, 2),
                       bdia_us=round(t_bdia * 1e6, 2))
            rows.append(rec)
            log("%d-point n=%-9d CSR %8.1f  DIA %8.1f  B-DIA %8.1f GFLOP/s" % (
                points, n, rec["csr_gflops"], rec["dia_gflops"], rec["bdia_gflops"]))
            if nf == sizes[-1]:
                comparison["%dpt" % points] = dict(
                    n=n, measured=dict(dia_over_csr=round(t_csr / t_dia, 3),
                                       bdia_over_csr=round(t_csr / t_bdia, 3),
                                       bdia_over_dia=round(t_dia / t_bdia, 3)),
                    model_paper_gamma={k: round(v_, 3) for k, v_ in
                                       model_ratios(nd, GAMMA_PAPER[points]).items()},
                    model_gamma_1_over_nd={k: round(v_, 3) for k, v_ in
                                           model_ratios(nd, 1.0 / nd).items()})
            if nf == args.bl_n:
                sweep = {}
                for vr, wg in ((1, 64), (2, 64), (4, 64), (1, 256), (2, 256), (4, 256)):
                    hdc.set_launch(vr, wg, 16 if wg * vr == 256 else 0)
                    t = paper_time(lambda: hdc.spmv(x, y, s), n_ites, args.n_loops, s)
                    sweep[str(vr * wg)] = round(2 * nnz / t / 1e9, 1)
                bl_sweep["%dpt" % points] = dict(n=n, tile_rows_to_gflops=sweep,
                                                 dia_gflops=rec["dia_gflops"])
                log("  tile sweep %s" % sweep)
            csr.close()
            hdc.close()
            del rp, ci, v, x, y
            torch.cuda.empty_cache()
    print(json.dumps({"metric": "stencil study (Sec. 6.3): CSR / DIA / B-DIA GFLOP/s, FP64, "
                                "1xMI355X", "unit": "GFLOP/s", "higher_is_better": True,
                      "dtype": "f64", "data": "synthetic banded stencils",
                      "n_loops": args.n_loops, "rows": rows, "comparison": comparison,
                      "tile_sweep": bl_sweep}))


if __name__ == "__main__":
    main()
