"""Context benchmark: rocSPARSE's CSR SpMV (rocsparse_dcsrmv, plain and
after rocsparse_dcsrmv_analysis) on the same matrices as bench.py, next to
this library's CSR and M-HDC kernels.  The vendor library is a point of
reference for the GPU CSR baseline, not part of the path.

    python bench_vendor.py [--steps K] [--warmup W]

Matrices: heptadiagonal 7-point 256^3 (M-HDC n_b = 256) and partially
diagonal 27-point 192^3 (M-HDC n_b = 128), theta = 0.6, x ~ U[-1,1].  The
vendor results are checked against the CPU oracle by
tests/test_gpu_vendor.py; here each is only compared with this library's CSR
product row by row (|y - y_ref| <= 1e-13 (|A||x|)) as a sanity check of the
run.  Prints one JSON line.
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
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3 / steps


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    args = ap.parse_args()

    import numpy as np
    import torch

    from paper_2105_04937_amd import mhdc, synth
    mhdc.lib()
    dev = torch.device("cuda:0")
    s = torch.cuda.current_stream(dev)
    from paper_2105_04937_amd import vendor
    rs = vendor.RocSparse(s)
    rows = []
    for name, gen, nb, seed in (("heptadiagonal 7-point 256^3", lambda: synth.heptadiagonal(256, 2),
                                 256, 2),
                                ("partially diagonal 27-point 192^3",
                                 lambda: synth.partially_diagonal(192, 3), 128, 3)):
        log("generating %s" % name)
        m = gen()
        rp, ci, v = mhdc.to_device(m, dev)
        x = torch.from_numpy(synth.vector(m.n, seed)).to(dev)
        y = torch.empty_like(x)
        absa = torch.from_numpy(np.abs(m.val)).to(dev)
        bound = None
        rec = {"matrix": name, "n": m.n, "nnz": m.nnz}
        csr = mhdc.CSRMatrix.from_csr(rp, ci, v)
        bytes_csr = csr.info()["bytes_alg"]
        y_ref = torch.empty_like(x)
        csr.spmv(x, y_ref, s)
        # |A||x| through the library's own CSR kernel on |values|, |x|
        acsr = mhdc.CSRMatrix.from_csr(rp, ci, absa)
        bound = torch.empty_like(x)
        acsr.spmv(x.abs(), bound, s)
        acsr.close()
        t = timed(lambda: csr.spmv(x, y, s), args.steps, args.warmup, s)
        rec["library_csr_us"] = round(t * 1e6, 2)
        csr.close()
        h = mhdc.MHDCMatrix.from_csr(rp, ci, v, nb, 0.6)
        t = timed(lambda: h.spmv(x, y, s), args.steps, args.warmup, s)
        rec["library_mhdc_us"] = round(t * 1e6, 2)
        rec["mhdc_n_b"] = nb
        h.close()
        for label, info in (("rocsparse_plain", None), ("rocsparse_analysis", "x")):
            inf = rs.analysis(m.n, m.nnz, rp, ci, v) if info else None
            rs.csrmv(m.n, m.nnz, rp, ci, v, inf, x, y)
            torch.cuda.synchronize()
            ok = bool(((y - y_ref).abs() <= 1e-13 * bound).all().item())
            t = timed(lambda: rs.csrmv(m.n, m.nnz, rp, ci, v, inf, x, y), args.steps,
                      args.warmup, s)
            rec[label + "_us"] = round(t * 1e6, 2)
            rec[label + "_gb_per_s"] = round(bytes_csr / t / 1e9, 1)
            rec[label + "_within_1e-13"] = ok
            if info:
                rs.free_info(inf)
            log("%-36s %-20s %9.1f us  (%s)" % (name, label, t * 1e6, "ok" if ok else "MISMATCH"))
        log("%-36s library CSR %.1f us, M-HDC %.1f us" % (name, rec["library_csr_us"],
                                                          rec["library_mhdc_us"]))
        rows.append(rec)
        del rp, ci, v, x, y, y_ref, bound, absa
        torch.cuda.empty_cache()
    print(json.dumps({"metric": "rocSPARSE dcsrmv vs library CSR and M-HDC (context), FP64, 1xMI355X",
                      "unit": "us", "higher_is_better": False, "steps": args.steps,
                      "warmup": args.warmup, "data": "synthetic", "rows": rows}))


if __name__ == "__main__":
    main()
