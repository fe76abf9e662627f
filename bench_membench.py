"""Memory benchmark sweep of Sec. 6.2 on one MI355X: the direct kernel
C[i] += A[i]*B[i] and the indirect kernel C[i] += A[i]*B[I[i]] (I[i] = i)
over array sizes N, effective bandwidth M*N/t with M = 32 and 36 bytes per
element.  Timing per Fig. 18: best over n_loops of the mean over n_ites
back-to-back calls (HIP events on the launch stream).

    python bench_membench.py [--max-log2 28]

Prints one JSON line; value = the direct kernel's bandwidth at the largest N.
"""
from __future__ import annotations

import argparse
import json
import os
import sys

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--min-log2", type=int, default=12)
    ap.add_argument("--max-log2", type=int, default=28)
    ap.add_argument("--n-loops", type=int, default=5)
    args = ap.parse_args()

    import torch

    from paper_2105_04937_amd import mhdc
    mhdc.lib()
    s = torch.cuda.current_stream()
    rows = []
    for lg in range(args.min_log2, args.max_log2 + 1, 2):
        N = 1 << lg
        A = torch.rand(N, dtype=torch.float64, device="cuda")
        B = torch.rand(N, dtype=torch.float64, device="cuda")
        C = torch.rand(N, dtype=torch.float64, device="cuda")
        I = torch.arange(N, dtype=torch.int32, device="cuda")
        n_ites = max(5, min(1000, (1 << 26) // N))
        for kind, M, fn in (("direct", 32, lambda: mhdc.stream_direct(A, B, C, s)),
                            ("indirect", 36, lambda: mhdc.stream_indirect(A, B, I, C, s))):
            fn()
            torch.cuda.synchronize()
            best = float("inf")
            for _ in range(args.n_loops):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(s)
                for _ in range(n_ites):
                    fn()
                e1.record(s)
                torch.cuda.synchronize()
                best = min(best, e0.elapsed_time(e1) / 1e3 / n_ites)
            gbs = M * N / best / 1e9
            rows.append(dict(kind=kind, log2N=lg, N=N, us=round(best * 1e6, 3),
                             gb_per_s=round(gbs, 1), n_ites=n_ites))
            print("%-8s N=2^%-2d %10.2f us %8.1f GB/s" % (kind, lg, best * 1e6, gbs),
                  file=sys.stderr, flush=True)
        del A, B, C, I
    top = [r for r in rows if r["kind"] == "direct"][-1]
    print(json.dumps({"metric": "memory benchmark (Sec. 6.2) effective bandwidth, 1xMI355X",
                      "value": top["gb_per_s"], "unit": "GB/s", "higher_is_better": True,
                      "dtype": "f64", "data": "synthetic", "rows": rows}))


if __name__ == "__main__":
    main()
