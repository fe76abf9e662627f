"""Multi-right-hand-side products Y = A X (k = 1, 2, 4, 8, 16) on the
heptadiagonal 7-point 256^3 matrix (M-HDC n_b = 256, theta = 0.6, and CSR)
and on the partially diagonal 27-point 192^3 matrix (M-HDC n_b = 128, CSR).
X and Y are column-major (n x k, leading dimension n): `colmajor` runs the
column-major kernel (spmm), `colmajor_ws` the workspace entry (spmm_ws,
route 0: the library's choice, printed as route 1 = column-major kernel or
2 = transposed through the row-major kernel); `rowmajor` stores them row
by row (element (i, r) at X[i*k + r]).  A is read once per product, so
algorithmic bytes = A + 16 n k (the transpositions of route 2 are extra).  Each handle runs its default
launch shape; a step is one spmm with inputs resident in HBM, timed with
HIP events on the launch stream.

    python bench_spmm.py [--steps K] [--warmup W] [--matrix all|hepta|partial]
                         [--ks 1,2,4,8,16] [--formats mhdc,csr]
                         [--layouts colmajor,colmajor_ws,rowmajor]

Prints one JSON line; value = GFLOP/s of M-HDC at k = 16 on the 256^3 case.
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
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--matrix", choices=("all", "hepta", "partial"), default="all")
    ap.add_argument("--ks", default="1,2,4,8,16", help="right-hand side counts, comma-separated")
    ap.add_argument("--formats", default="mhdc,csr", help="subset of mhdc,csr")
    ap.add_argument("--layouts", default="colmajor,colmajor_ws,rowmajor",
                    help="subset of colmajor,colmajor_ws,rowmajor")
    args = ap.parse_args()
    ks = [int(t) for t in args.ks.split(",")]
    formats = args.formats.split(",")
    layouts = args.layouts.split(",")

    import torch

    from paper_2105_04937_amd import mhdc, synth
    mhdc.lib()
    dev = torch.device("cuda:0")
    s = torch.cuda.current_stream(dev)
    rows = []
    cases = (("heptadiagonal 7-point 256^3", lambda: synth.heptadiagonal(256, 2), 256),
             ("partially diagonal 27-point 192^3", lambda: synth.partially_diagonal(192, 3), 128))
    cases = [c for c in cases if args.matrix == "all" or c[0].startswith(
        {"hepta": "heptadiagonal", "partial": "partially"}[args.matrix])]
    for name, gen, nb in cases:
        log("generating %s" % name)
        m = gen()
        d = mhdc.to_device(m, dev)
        n = m.n
        for label, fmt, make in (("M-HDC n_b=%d" % nb, "mhdc",
                                  lambda: mhdc.MHDCMatrix.from_csr(*d, nb, 0.6)),
                                 ("CSR", "csr", lambda: mhdc.CSRMatrix.from_csr(*d))):
            if fmt not in formats:
                continue
            h = make()
            inf = h.info()
            a_bytes = inf["bytes_alg"] - 16.0 * n
            for k in ks:
                for lay in layouts:
                    route = None
                    if lay == "rowmajor":
                        X = torch.rand((n, k), dtype=torch.float64, device=dev)
                        fn = lambda: h.spmm_rowmajor(X, Y, s)  # noqa: E731
                    elif lay == "colmajor_ws":
                        X = torch.rand((k, n), dtype=torch.float64, device=dev)
                        ws = torch.empty(h.workspace_bytes(k), dtype=torch.uint8, device=dev)
                        route = h.ws_route(k)
                        fn = lambda: h.spmm_ws(X, Y, 0, ws, s)  # noqa: E731
                    else:
                        X = torch.rand((k, n), dtype=torch.float64, device=dev)
                        fn = lambda: h.spmm(X, Y, s)  # noqa: E731
                    Y = torch.empty_like(X)
                    t = timed(fn, args.steps, args.warmup, s)
                    gbs = (a_bytes + 16.0 * n * k) / t / 1e9
                    gfl = 2.0 * m.nnz * k / t / 1e9
                    log("%-34s %-12s %-11s k=%2d %9.1f us %7.1f GB/s %7.1f GFLOP/s%s" % (
                        name, label, lay, k, t * 1e6, gbs, gfl,
                        "" if route is None else "  route %d" % route))
                    rows.append(dict(matrix=name, format=label, layout=lay, k=k,
                                     us=round(t * 1e6, 2), gb_per_s=round(gbs, 1),
                                     gflops=round(gfl, 1), bytes_alg=a_bytes + 16.0 * n * k))
                    if route is not None:
                        rows[-1]["route"] = route
                        del ws
                    del X, Y
            h.close()
        del d, m
        torch.cuda.empty_cache()
    top = ([r for r in rows if r["k"] == max(ks) and r["format"].startswith("M-HDC")
            and r["layout"] == layouts[-1]] or rows)[0]
    print(json.dumps({"metric": "multi-RHS M-HDC SpMM GFLOP/s, FP64, 1xMI355X",
                      "value": top["gflops"], "unit": "GFLOP/s", "higher_is_better": True,
                      "dtype": "f64", "data": "synthetic (seeded stencil matrices, X ~ U[0,1))",
                      "steps": args.steps, "warmup": args.warmup, "rows": rows}))


if __name__ == "__main__":
    main()
