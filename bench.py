"""Benchmark: FP64 M-HDC SpMV on one MI355X against the GPU CSR and HDC
baselines, plus the CPU oracle on the host cores.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-partial]

Workload (the headline case): 7-point heptadiagonal matrix on a 256^3 grid
(16,777,216 rows, 117,047,296 nonzeros, off-diagonals U[-1,-0.5], diagonal
1.01*|row sum|), x ~ U[-1,1], M-HDC with n_b = 256 and theta = 0.6.  A step is
one y = A x with the matrix already converted and resident in HBM; W untimed
steps, then exactly K timed steps between device synchronisations, timed with
HIP events on the stream the kernels are launched on.

Prints ONE JSON line.  value = GFLOP/s = 2*nnz / (time per step) (Eq. 1 of the
paper); roofline.achieved = algorithmic bytes per launch / time per launch.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_mhdc_spmv_hepta256.json")
SPMV_SRC = [os.path.join(ROOT, "paper_2105_04937_amd", "csrc", f)
            for f in ("spmv.hip", "spmv_tile.h")]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def time_steps(fn, steps, warmup, stream):
    """W untimed calls, then K timed calls bracketed by device syncs and HIP
    events recorded on `stream`.  Returns seconds per call."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3 / steps


def interleaved(fns, rounds, steps, warmup, stream):
    """Median seconds per call of each function, timed in `rounds` rounds
    that take the functions in turn (steps calls each), so that drifts of
    clock or temperature fall on all of them alike."""
    import statistics

    import torch
    for fn in fns.values():
        for _ in range(warmup):
            fn()
    torch.cuda.synchronize()
    ts = {k: [] for k in fns}
    for _ in range(rounds):
        for k, fn in fns.items():
            ts[k].append(time_steps(fn, steps, 0, stream))
    return {k: statistics.median(v) for k, v in ts.items()}


def rocsparse_csrmv(m, d, x, stream):
    """rocSPARSE's analysed CSR SpMV on the same device arrays as a
    callable y = A x (the vendor's GPU CSR kernel, a point of reference for
    the CSR baseline), or None without librocsparse.so."""
    import torch
    from paper_2105_04937_amd import vendor
    if not vendor.available():
        return None, None
    rs = vendor.RocSparse(stream)
    rp, ci, v = d
    info = rs.analysis(m.n, m.nnz, rp, ci, v)
    y = torch.empty_like(x)
    fn = lambda: rs.csrmv(m.n, m.nnz, rp, ci, v, info, x, y)  # noqa: E731

    def close():
        torch.cuda.synchronize()
        rs.free_info(info)
        rs.close()
    return fn, close


def paper_protocol(fn, n_ites, n_loops, stream):
    """Sec. 6.1.3 / Fig. 18: best over n_loops of the mean over n_ites calls."""
    import torch
    best = float("inf")
    for _ in range(n_loops):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(n_ites):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1) / 1e3 / n_ites)
    return best


def kernel_source_sha256():
    """Hash of the SpMV kernel sources (launcher + tile routine)."""
    h = hashlib.sha256()
    for p in SPMV_SRC:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def kernel_traffic(launch):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when absent or taken on a different version of the kernel source or
    another launch shape."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
        if rec.get("spmv_source_sha256") != kernel_source_sha256():
            return None
        if list(rec.get("launch", [])) != list(launch):
            return None
        return rec.get("bytes_per_launch")
    except (OSError, ValueError):
        return None


def cpu_baseline(m, x, nnz):
    """The oracle's CSR SpMV (plain C, FP64, one OpenMP thread per host core)
    on the same matrix, with the paper's protocol (best over n_loops = 5 of
    the mean over n_ites = 20 calls); plus one single-thread loop."""
    os.environ.setdefault("OMP_PROC_BIND", "close")  # the paper's compact placement
    import oracle
    cores = len(os.sched_getaffinity(0))
    oracle.csr_spmv(m.rowptr, m.colind, m.val, x, cores)  # warm-up
    best = float("inf")
    t_all = time.perf_counter()
    for _ in range(5):
        t0 = time.perf_counter()
        for _ in range(20):
            oracle.csr_spmv(m.rowptr, m.colind, m.val, x, cores)
        best = min(best, (time.perf_counter() - t0) / 20)
    wall = time.perf_counter() - t_all
    t0 = time.perf_counter()
    for _ in range(3):
        oracle.csr_spmv(m.rowptr, m.colind, m.val, x, 1)
    t1 = (time.perf_counter() - t0) / 3
    return {"value": round(2.0 * nnz / best / 1e9, 3), "unit": "GFLOP/s", "cores": cores,
            "kind": "oracle",
            "sample": "full 256^3 heptadiagonal matrix: 100 oracle CSR SpMV calls on %d threads "
                      "(best of 5 loops x mean of 20, %.1f s wall, ~%.0f core-s) + 3 calls on 1 "
                      "thread" % (cores, wall, wall * cores),
            "ms_per_call": round(best * 1e3, 3),
            "single_thread_gflops": round(2.0 * nnz / t1 / 1e9, 3)}


def run_format(make, x, steps, warmup, stream, label):
    import torch
    t0 = time.perf_counter()
    mat = make()
    torch.cuda.synchronize()
    conv = time.perf_counter() - t0
    y = torch.empty_like(x)
    fn = lambda: mat.spmv(x, y, stream)  # noqa: E731
    t = time_steps(fn, steps, warmup, stream)
    inf = mat.info()
    log("%-6s %8.3f us/step  %8.1f GFLOP/s  %7.1f GB/s  (convert %.2f s)" % (
        label, t * 1e6, 2 * inf["nnz"] / t / 1e9, inf["bytes_alg"] / t / 1e9, conv))
    return mat, y, t, conv, inf


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n-b", type=int, default=256)
    ap.add_argument("--theta", type=float, default=0.6)
    ap.add_argument("--grid", type=int, default=256)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-partial", action="store_true")
    ap.add_argument("--only-mhdc", action="store_true", help="time the M-HDC kernel only")
    ap.add_argument("--pp-ites", type=int, default=1000,
                    help="paper protocol: calls per loop (n_ites of Fig. 18)")
    ap.add_argument("--pp-loops", type=int, default=20,
                    help="paper protocol: loops, best taken (n_loops of Fig. 18)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2105_04937_amd import mhdc, synth

    mhdc.lib()  # fail loudly before any work if the HIP library is missing
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)

    N = args.grid
    log("generating heptadiagonal %d^3" % N)
    m = synth.heptadiagonal(N, 2)
    x_np = synth.vector(m.n, 2)
    rp, ci, v = mhdc.to_device(m, dev)
    x = torch.from_numpy(x_np).to(dev)

    h, y, t_mhdc, conv_mhdc, inf = run_format(
        lambda: mhdc.MHDCMatrix.from_csr(rp, ci, v, args.n_b, args.theta), x, args.steps,
        args.warmup, stream, "M-HDC")
    t_pp = paper_protocol(lambda: h.spmv(x, y, stream), args.pp_ites, args.pp_loops, stream)
    launch = [inf[f] for f in ("rows_per_lane", "wg_size", "xcd_remap", "csr_mode", "rhs_group")]
    out = {}
    if not args.only_mhdc:
        hd, _, t_hdc, conv_hdc, inf_h = run_format(
            lambda: mhdc.HDCMatrix.from_csr(rp, ci, v, args.theta), x, args.steps, args.warmup,
            stream, "HDC")
        hd.close()
        cs, _, t_csr, conv_csr, inf_c = run_format(
            lambda: mhdc.CSRMatrix.from_csr(rp, ci, v), x, args.steps, args.warmup, stream, "CSR")
        cs.close()
        out["csr"] = {"gflops": round(2 * inf_c["nnz"] / t_csr / 1e9, 2),
                      "gb_per_s": round(inf_c["bytes_alg"] / t_csr / 1e9, 1),
                      "us_per_step": round(t_csr * 1e6, 2), "bytes_alg": inf_c["bytes_alg"],
                      "roofline_frac": round(inf_c["bytes_alg"] / t_csr / 1e9 / PEAK_HBM_GBS, 4)}
        # the vendor's analysed csrmv on the same arrays: the speed-up is
        # quoted against the faster of the two GPU CSR kernels
        t_best_csr = t_csr
        vfn, vclose = rocsparse_csrmv(m, (rp, ci, v), x, stream)
        if vfn:
            t_vs = time_steps(vfn, args.steps, args.warmup, stream)
            vclose()
            log("rocSPARSE csrmv (analysed) %8.3f us/step  %7.1f GB/s" % (
                t_vs * 1e6, inf_c["bytes_alg"] / t_vs / 1e9))
            out["csr"]["rocsparse_analysed_us"] = round(t_vs * 1e6, 2)
            out["csr"]["rocsparse_roofline_frac"] = round(
                inf_c["bytes_alg"] / t_vs / 1e9 / PEAK_HBM_GBS, 4)
            t_best_csr = min(t_csr, t_vs)
        out["hdc"] = {"gflops": round(2 * inf_h["nnz"] / t_hdc / 1e9, 2),
                      "gb_per_s": round(inf_h["bytes_alg"] / t_hdc / 1e9, 1),
                      "us_per_step": round(t_hdc * 1e6, 2), "K": inf_h["K"]}
        out["speedup_vs_csr"] = round(t_best_csr / t_mhdc, 4)
        out["speedup_vs_library_csr"] = round(t_csr / t_mhdc, 4)
        out["speedup_vs_csr_model"] = round(inf["rp_est"], 4)
        out["mhdc_roofline_frac"] = round(inf["bytes_alg"] / t_mhdc / 1e9 / PEAK_HBM_GBS, 4)
        # block size sweep on the same matrix (default launch of each handle)
        sweep = {str(args.n_b): {"us": round(t_mhdc * 1e6, 2),
                                 "gb_per_s": round(inf["bytes_alg"] / t_mhdc / 1e9, 1),
                                 "K": inf["K"], "launch": launch}}
        for nb in (128, 512, 1024, 2048, 4096):
            if str(nb) in sweep:
                continue
            hs, _, ts, _, i_s = run_format(
                lambda: mhdc.MHDCMatrix.from_csr(rp, ci, v, nb, args.theta), x,
                max(args.steps // 4, 1), args.warmup, stream, "n_b=%d" % nb)
            hs.close()
            sweep[str(nb)] = {"us": round(ts * 1e6, 2),
                              "gb_per_s": round(i_s["bytes_alg"] / ts / 1e9, 1), "K": i_s["K"],
                              "launch": [i_s[f] for f in ("rows_per_lane", "wg_size", "xcd_remap",
                                                          "csr_mode", "rhs_group")]}
        out["n_b_sweep"] = dict(sorted(sweep.items(), key=lambda kv: int(kv[0])))

    # memory benchmark (Sec. 6.2, direct kernel): achievable HBM rate
    Ns = 1 << 27
    A = torch.rand(Ns, dtype=torch.float64, device=dev)
    B = torch.rand(Ns, dtype=torch.float64, device=dev)
    C = torch.rand(Ns, dtype=torch.float64, device=dev)
    t_st = time_steps(lambda: mhdc.stream_direct(A, B, C, stream), 20, 3, stream)
    del A, B, C
    stream_gbs = 32.0 * Ns / t_st / 1e9
    log("stream direct: %.1f GB/s" % stream_gbs)

    partial = None
    if not args.no_partial:
        log("generating partially diagonal 27-point 192^3")
        m3 = synth.partially_diagonal(192, 3)
        d3 = mhdc.to_device(m3, dev)
        x3 = torch.from_numpy(synth.vector(m3.n, 3)).to(dev)
        res = {}
        for nb in (32, 96, 128):
            h3, _, t3, _, i3 = run_format(lambda: mhdc.MHDCMatrix.from_csr(*d3, nb, 0.6), x3,
                                          args.steps // 2, args.warmup, stream, "M%d" % nb)
            res["mhdc_nb%d" % nb] = {"gflops": round(2 * i3["nnz"] / t3 / 1e9, 2),
                                     "gb_per_s": round(i3["bytes_alg"] / t3 / 1e9, 1),
                                     "us": round(t3 * 1e6, 2), "alpha": round(i3["alpha"], 4),
                                     "beta": round(i3["beta"], 4),
                                     "rp_est": round(i3["rp_est"], 4)}
            h3.close()
        c3, _, tc3, _, ic3 = run_format(lambda: mhdc.CSRMatrix.from_csr(*d3), x3,
                                        args.steps // 2, args.warmup, stream, "CSR")
        hd3, _, th3, _, ih3 = run_format(lambda: mhdc.HDCMatrix.from_csr(*d3, 0.6), x3,
                                         args.steps // 2, args.warmup, stream, "HDC")
        hd3.close()
        res["csr"] = {"gflops": round(2 * ic3["nnz"] / tc3 / 1e9, 2),
                      "gb_per_s": round(ic3["bytes_alg"] / tc3 / 1e9, 1), "us": round(tc3 * 1e6, 2)}
        res["hdc"] = {"gflops": round(2 * ih3["nnz"] / th3 / 1e9, 2), "us": round(th3 * 1e6, 2),
                      "alpha": round(ih3["alpha"], 4)}
        # the learned selector's choice for this matrix (network + byte-model judge)
        from paper_2105_04937_amd import learned
        hsel, dec = mhdc.select(*d3, model=learned.load_network(),
                                tolerance=learned.JUDGE_TOLERANCE)
        res["mhdc_selected"] = {"theta": dec["theta"], "n_b": dec["n_b"],
                                "used_rule": bool(dec["used_rule"])}
        # the same choice refined by timing its grid neighbours on the device
        href, dref = mhdc.select_refine(*d3, model=learned.load_network(),
                                        tolerance=learned.JUDGE_TOLERANCE, stream=stream)
        res["mhdc_refined"] = {"theta": dref["theta"], "n_b": dref["n_b"],
                               "used_rule": bool(dref["used_rule"])}
        # M-HDC against GPU CSR: the pre-declared configuration (n_b = 128,
        # theta = 0.6) and the selector's choices, timed in interleaved
        # rounds with the library's CSR and rocSPARSE's analysed csrmv
        h128 = mhdc.MHDCMatrix.from_csr(*d3, 128, 0.6)
        ya, yb, yc, yd = (torch.empty_like(x3) for _ in range(4))
        fns = {"mhdc_nb128": lambda: h128.spmv(x3, ya, stream),
               "selected": lambda: hsel.spmv(x3, yb, stream),
               "refined": lambda: href.spmv(x3, yc, stream),
               "csr": lambda: c3.spmv(x3, yd, stream)}
        vfn, vclose = rocsparse_csrmv(m3, d3, x3, stream)
        if vfn:
            fns["rocsparse"] = vfn
        ti = interleaved(fns, 5, max(args.steps // 10, 1), args.warmup, stream)
        if vclose:
            vclose()
        t_best_csr = min(ti["csr"], ti.get("rocsparse", float("inf")))
        res["interleaved_us"] = {k: round(v_ * 1e6, 2) for k, v_ in ti.items()}
        res["mhdc_selected"]["us"] = res["interleaved_us"]["selected"]
        res["mhdc_refined"]["us"] = res["interleaved_us"]["refined"]
        res["speedup_mhdc_nb128_vs_csr"] = round(t_best_csr / ti["mhdc_nb128"], 4)
        res["speedup_selected_vs_csr"] = round(t_best_csr / ti["selected"], 4)
        res["speedup_refined_vs_csr"] = round(t_best_csr / ti["refined"], 4)
        log("interleaved: %s" % res["interleaved_us"])
        for hh in (h128, hsel, href, c3):
            hh.close()
        res["workload"] = "27-point 192^3, octant drops {0,.05,.1,.2,.3,.5,.7,.9}, +2 random/row"
        res["nnz"] = m3.nnz
        partial = res
        del d3, x3, m3

    cpu = None
    if not args.no_cpu:
        log("timing the CPU oracle")
        cpu = cpu_baseline(m, x_np, m.nnz)

    gflops = 2.0 * inf["nnz"] / t_mhdc / 1e9
    achieved = inf["bytes_alg"] / t_mhdc / 1e9
    traffic = kernel_traffic(launch)
    rec = {
        "metric": "M-HDC SpMV GFLOP/s + HBM GB/s vs GPU CSR, FP64, 1xMI355X",
        "value": round(gflops, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t_mhdc * 1e3, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded heptadiagonal stencil, x ~ U[-1,1])",
        "config": {"workload": "heptadiagonal 7-point 256^3 (n=%d, nnz=%d), M-HDC n_b=%d "
                               "theta=%.2f" % (m.n, m.nnz, args.n_b, args.theta),
                   "n": m.n, "nnz": m.nnz, "n_b": args.n_b, "theta": args.theta,
                   "launch": launch},
        "hbm_gb_per_s": round(achieved, 1),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
                     "traffic": traffic},
        "bytes_alg_per_launch": inf["bytes_alg"],
        "bytes_paper_model": inf["bytes_paper"],
        # counted HBM bytes against the algorithmic bytes and the paper's V
        "traffic_vs_alg": round(traffic / inf["bytes_alg"], 4) if traffic else None,
        "traffic_vs_paper_model": round(traffic / inf["bytes_paper"], 4) if traffic else None,
        "paper_protocol_us": round(t_pp * 1e6, 2),
        "paper_protocol": {"n_ites": args.pp_ites, "n_loops": args.pp_loops},
        "convert_s": round(conv_mhdc, 3),
        "stream_direct_gb_per_s": round(stream_gbs, 1),
        "cpu_baseline": cpu,
    }
    rec.update(out)
    if partial:
        rec["partially_diagonal_192"] = partial
    h.close()
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
