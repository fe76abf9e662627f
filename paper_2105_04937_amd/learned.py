"""Learned (theta, n_b) selector: data collection, training, evaluation.

The paper proposes a policy for M-HDC's two parameters (50 <~ bl <~ 500,
theta = 0.6; Sec. 6.4.3) and leaves their choice open (Sec. 7).  Here:

* collect: draw matrices of the stencil families (7/19/27-point grids with
  per-octant or global coupling drops and random extra columns, grid side
  U{48..144}, or U{145..208} for the *_large splits), compute the 66 census features (mhdc_features), and time the
  M-HDC SpMV for every (theta, n_b) of the grid theta in {0.5 .. 0.9}
  (Sec. 6.4.1's values) x n_b in {32 .. 4096} (mhdc_from_csr +
  mhdc_time_spmv).  One JSON line per matrix.
* train: the network is trained with the library's own kernels: a short
  warm-up on the squared error to each matrix's measured arg-min over the
  grid, near-ties broken towards the best fixed grid point of the training
  set (target(); mhdc_mlp_train), then on the grid loss, which scores the
  network's output by the matrix's measured time ratio interpolated
  between the grid points (grid_of(); mhdc_mlp_train_grid).  Regressing on
  the arg-min alone averages between distant near-best points; the grid
  loss lets each matrix pull the output towards wherever its time is low.
* train --scorer: the 40-output scorer (one estimate of the log time ratio
  per grid point; mhdc_mlp_create_scorer) is trained on the same grids with
  its weighted squared error (mhdc_mlp_train_grid), on inputs standardised
  with the training set's feature means and deviations; the standardisation
  is then folded into the first layer (W1 / sd, b1 - (W1 / sd) mu), so the
  stored network reads the library's raw features.  Its decision is the
  grid point of the smallest estimate: unlike a single (theta, log2 n_b)
  output it can keep apart several distant near-best regions.
* evaluate: the network's decisions (mhdc_mlp_decide) are looked up in the
  measured grid of held-out matrices, after the byte-model judge that
  mhdc_select applies, and compared with the exhaustive best and the policy.

Everything that computes on matrices or the network runs in the library's
kernels; this module draws random inputs, keeps records and forms targets.

    python -m paper_2105_04937_amd.learned collect --split train --start 0 --count 1000 --out F
    python -m paper_2105_04937_amd.learned train --data A B ... --test T --out-dir D
"""
from __future__ import annotations

import argparse
import gzip
import json
import math
import os
import sys
import time

import numpy as np

THETAS = (0.5, 0.6, 0.7, 0.8, 0.9)
NBS = (32, 64, 128, 256, 512, 1024, 2048, 4096)
RULE = (0.6, 256)
SEED_BASE = {"train": 5000, "test": 9000, "train_large": 7000, "test_large": 9500}
SIDES = {"": (48, 144), "_large": (145, 208)}  # grid side range per split family
LOSS_W = (25.0, 0.25)       # 1/0.2^2 for theta, 1/2^2 for log2 n_b
HERE = os.path.dirname(os.path.abspath(__file__))
DATA_DIR = os.path.join(HERE, "selector_data")


JUDGE_TOLERANCE = 0.25      # mhdc_select keeps a proposal up to 1.25 x the policy's V
WEIGHTS = os.path.join(DATA_DIR, "weights.npy")  # the 40-output scorer (the default)
# the 66 -> 128 -> 128 -> 2 network with output (theta, log2 n_b), trained with
# the grid loss; its held-out report is eval_report_theta_nb.json
WEIGHTS_THETA_NB = os.path.join(DATA_DIR, "weights_theta_nb.npy")


def key(theta, nb):
    return "%.1f/%d" % (theta, nb)


def load_network(path=WEIGHTS):
    """A trained selector network (parameters stored as float32 .npy; the
    kind, scorer or 2-output, follows from the parameter count)."""
    from paper_2105_04937_amd import mhdc
    return mhdc.MLP(np.load(path, allow_pickle=False))


def draw_family(rng, large=False):
    """Matrix parameters of one sample (drawn from its own seed); the large
    splits draw grid sides 145..208 (3M to 9M rows, beyond the Infinity
    Cache), the others 48..144."""
    lo, hi = SIDES["_large" if large else ""]
    N = int(rng.integers(lo, hi + 1))
    if rng.random() < 0.15:
        return dict(N=N, points=7, drop=0.0, extra=0, family="hepta")
    points = int(rng.choice([7, 19, 27]))
    if rng.random() < 0.5:
        drop = [float(a) for a in rng.uniform(0.0, 0.95, size=8)]
        fam = "octant"
    else:
        drop = float(rng.uniform(0.0, 0.6))
        fam = "global"
    extra = int(rng.choice([0, 0, 1, 2, 4]))
    return dict(N=N, points=points, drop=drop, extra=extra, family=fam)


def collect(split, start, count, out_path):
    import torch

    from paper_2105_04937_amd import mhdc, synth
    mhdc.lib()
    with open(out_path, "a") as out:
        for i in range(start, start + count):
            t0 = time.time()
            seed = SEED_BASE[split] + i
            fam = draw_family(np.random.default_rng(seed), large=split.endswith("_large"))
            rp, ci, v = synth.stencil_matrix_gpu(fam["N"], seed, points=fam["points"],
                                                 drop=fam["drop"], extra_per_row=fam["extra"])
            n, nnz = rp.numel() - 1, ci.numel()
            feat = mhdc.features(rp, ci, v).cpu().numpy()
            g = torch.Generator(device="cuda")
            g.manual_seed(seed)
            x = torch.rand(n, generator=g, device="cuda", dtype=torch.float64) * 2 - 1
            y = torch.empty_like(x)
            us, vb = {}, {}
            for th in THETAS:
                for nb in NBS:
                    h = mhdc.MHDCMatrix.from_csr(rp, ci, v, nb, th)
                    vb[key(th, nb)] = h.info()["bytes_paper"]
                    us[key(th, nb)] = round(h.time_spmv(x, y), 3)
                    h.close()
            rec = dict(id=i, split=split, seed=seed, family=fam, n=n, nnz=nnz,
                       features=[float(f) for f in feat], us=us, bytes_paper=vb)
            out.write(json.dumps(rec) + "\n")
            out.flush()
            best = min(us, key=us.get)
            print("%s %d n=%d nnz=%d best=%s %.1fus rule=%.1fus (%.1fs)" % (
                split, i, n, nnz, best, us[best], us[key(*RULE)], time.time() - t0), flush=True)
            del rp, ci, v, x, y


def load(paths):
    recs = []
    for p in paths:
        op = gzip.open if p.endswith(".gz") else open
        with op(p, "rt") as f:
            recs.extend(json.loads(l) for l in f if l.strip())
    return recs


def grid_coords(ks):
    th = np.array([float(k.split("/")[0]) for k in ks])
    lb = np.array([math.log2(int(k.split("/")[1])) for k in ks])
    return th, lb


def prior_point(recs):
    """The grid point with the lowest mean time ratio t / t_best over the
    training matrices (the best single fixed choice)."""
    ks = list(recs[0]["us"])
    R = np.array([[r["us"][k] / min(r["us"].values()) for k in ks] for r in recs])
    return ks[int(np.argmin(R.mean(axis=0)))]


def target(rec, prior, eps=0.02):
    """Training target: the grid point minimising t/t_min + eps * (grid steps
    from the prior point), i.e. the measured arg-min with near-ties (the
    landscape is flat within timing noise and has several distant minima)
    broken towards the best fixed choice.  Averaging near-best points
    instead (a soft arg-min) regresses between distant minima."""
    ks = list(rec["us"])
    t = np.array([rec["us"][k] for k in ks])
    th, lb = grid_coords(ks)
    pth, plb = grid_coords([prior])
    score = t / t.min() + eps * (np.abs(lb - plb[0]) + np.abs(th - pth[0]) / 0.1)
    i = int(np.argmin(score))
    return np.array([th[i], lb[i]], np.float32)


def init_params(seed, n_out=2, scale=math.sqrt(6.0)):
    """Uniform weights in +-scale / sqrt(fan_in) (He-uniform by default),
    zero biases (the order of the C-ABI parameter vector: W1 128x66, b1, W2
    128x128, b2, W3 n_out x 128, b3)."""
    rng = np.random.default_rng(seed)
    parts = []
    for shape in ((128, 66), (128,), (128, 128), (128,), (n_out, 128), (n_out,)):
        if len(shape) == 2:
            lim = scale / math.sqrt(shape[1])
            parts.append(rng.uniform(-lim, lim, size=shape).ravel())
        else:
            parts.append(np.zeros(shape))
    return np.concatenate(parts).astype(np.float32)


def grid_of(rec):
    """The matrix's grid-loss values: log(t / t_best) at the 40 grid points,
    theta outer (theta = 0.5 + 0.1 i, n_b = 2^(5+j), at 8 i + j)."""
    t = np.array([[rec["us"][key(th, nb)] for nb in NBS] for th in THETAS], np.float64)
    return np.log(t / t.min()).ravel().astype(np.float32)


def train(recs, steps=8000, B=128, lr=1e-3, seed=0, warm=500):
    """Adam on the library's kernels: `warm` steps on the squared error to
    the arg-min targets, then the grid loss; lr for the first 3/4 of all
    steps, lr/3 for the rest (the optimizer state carries over)."""
    import torch

    from paper_2105_04937_amd import mhdc
    prior = prior_point(recs)
    X = np.array([r["features"] for r in recs], np.float32)
    T = np.stack([target(r, prior) for r in recs]).astype(np.float32)
    G = np.stack([grid_of(r) for r in recs]).astype(np.float32)
    rng = np.random.default_rng(seed)
    per = []
    while sum(len(p) for p in per) < steps * B:
        per.append(rng.permutation(len(recs)))
    order = np.concatenate(per)[:steps * B].astype(np.int32)
    net = mhdc.MLP(init_params(seed))
    Xd, Td, Gd = (torch.from_numpy(a).cuda() for a in (X, T, G))
    s1 = (3 * steps) // 4
    od = lambda a, b: torch.from_numpy(order[a * B:b * B]).cuda()  # noqa: E731
    h0 = net.train(Xd, Td, od(0, warm), warm, B, lr, w=LOSS_W)
    h1 = net.train_grid(Xd, Gd, od(warm, s1), s1 - warm, B, lr)
    h2 = net.train_grid(Xd, Gd, od(s1, steps), steps - s1, B, lr / 3)
    return net, np.concatenate([h.cpu().numpy() for h in (h0, h1, h2)]), prior


def fold_standardisation(params, mu, sd):
    """Parameters of the network that, on raw features x, computes what
    `params` computes on (x - mu) / sd: W1' = W1 / sd (per input column),
    b1' = b1 - W1' mu; the other layers unchanged.  FP64, stored as FP32."""
    p = np.asarray(params, np.float64).copy()
    W1 = p[:128 * 66].reshape(128, 66) / np.asarray(sd, np.float64)[None, :]
    b1 = p[128 * 66:128 * 66 + 128] - W1 @ np.asarray(mu, np.float64)
    p[:128 * 66] = W1.ravel()
    p[128 * 66:128 * 66 + 128] = b1
    return p.astype(np.float32)


def train_scorer(recs, steps=8000, B=128, lr=1e-3, seed=0):
    """The 40-output scorer on the library's kernels: weights uniform in
    +-1/sqrt(fan_in), Adam with the scorer loss (mhdc_mlp_train_grid) on
    standardised features, lr for the first 3/4 of the steps and lr/3 for
    the rest, then the standardisation folded into the first layer.  Returns
    (network on raw features, loss history, (mu, sd)).  The loss weights
    (exp(-g / 0.1) + 0.05), this initialisation and the step count were
    chosen on a validation split of the training matrices (400 of them,
    trained on the other 2,000), not on the held-out files."""
    import torch

    from paper_2105_04937_amd import mhdc
    X = np.array([r["features"] for r in recs], np.float32)
    mu = X.mean(axis=0, dtype=np.float64)
    sd = X.std(axis=0, dtype=np.float64) + 1e-6
    Xs = ((X - mu) / sd).astype(np.float32)
    G = np.stack([grid_of(r) for r in recs]).astype(np.float32)
    rng = np.random.default_rng(seed)
    per = []
    while sum(len(p) for p in per) < steps * B:
        per.append(rng.permutation(len(recs)))
    order = np.concatenate(per)[:steps * B].astype(np.int32)
    net = mhdc.MLP(init_params(seed, mhdc.GRID_POINTS, scale=1.0))
    Xd, Gd = (torch.from_numpy(a).cuda() for a in (Xs, G))
    s1 = (3 * steps) // 4
    od = lambda a, b: torch.from_numpy(order[a * B:b * B]).cuda()  # noqa: E731
    h1 = net.train_grid(Xd, Gd, od(0, s1), s1, B, lr)
    h2 = net.train_grid(Xd, Gd, od(s1, steps), steps - s1, B, lr / 3)
    folded = mhdc.MLP(fold_standardisation(net.params(), mu, sd))
    net.close()
    return folded, np.concatenate([h.cpu().numpy() for h in (h1, h2)]), (mu, sd)


def evaluate(net, recs, tolerance=JUDGE_TOLERANCE):
    """Per held-out matrix: time of the judged network choice, of the policy
    and of the exhaustive best, all from the measured grid.  The judge and
    the refinement candidates are the library's own (mhdc_judge_keep,
    mhdc_refine_candidates), so this evaluates exactly what mhdc_select and
    mhdc_select_refine decide."""
    import torch

    from paper_2105_04937_amd import mhdc
    X = torch.from_numpy(np.array([r["features"] for r in recs], np.float32)).cuda()
    th, nb, ok = (t.cpu().numpy() for t in net.decide(X))
    rows = []
    for r, t_, b_, o_ in zip(recs, th, nb, ok):
        us = r["us"]
        kb = min(us, key=us.get)
        kr = key(*RULE)
        kn = key(float(t_), int(b_))
        use_net = bool(o_) and mhdc.judge_keep(r["bytes_paper"][kn], r["bytes_paper"][kr],
                                               tolerance)
        ks = kn if use_net else kr
        # mhdc_select_refine: the choice and its candidates, the fastest by
        # the measured grid
        th_s, nb_s = (float(t_), int(b_)) if use_net else RULE
        cands = {ks} | {key(a, b) for a, b in mhdc.refine_candidates(th_s, nb_s)}
        kf = min(cands, key=us.get)
        # the byte model's verdict on the selection against plain CSR
        v_csr = 12.0 * r["nnz"] + 20.0 * r["n"]
        rows.append(dict(id=r["id"], best=kb, net=kn, used_net=use_net, refined=kf,
                         t_best=us[kb], t_sel=us[ks], t_rule=us[kr], t_net=us[kn],
                         t_refined=us[kf], csr_cheaper=v_csr < r["bytes_paper"][ks]))
    t_best = np.array([x["t_best"] for x in rows])
    t_sel = np.array([x["t_sel"] for x in rows])
    t_rule = np.array([x["t_rule"] for x in rows])
    t_net = np.array([x["t_net"] for x in rows])
    t_ref = np.array([x["t_refined"] for x in rows])
    rep = dict(
        matrices=len(rows),
        within_5pct_selected=float(np.mean(t_sel <= 1.05 * t_best)),
        within_5pct_refined=float(np.mean(t_ref <= 1.05 * t_best)),
        mean_ratio_refined=float(np.mean(t_ref / t_best)),
        within_5pct_rule=float(np.mean(t_rule <= 1.05 * t_best)),
        mean_ratio_selected=float(np.mean(t_sel / t_best)),
        mean_ratio_rule=float(np.mean(t_rule / t_best)),
        mean_ratio_network_unjudged=float(np.mean(t_net / t_best)),
        geomean_speedup_over_rule=float(np.exp(np.mean(np.log(t_rule / t_sel)))),
        total_time_selected_us=float(t_sel.sum()), total_time_rule_us=float(t_rule.sum()),
        total_time_best_us=float(t_best.sum()),
        used_network=float(np.mean([x["used_net"] for x in rows])),
        judge_override_rate=float(np.mean([not x["used_net"] for x in rows])),
        within_5pct_network_unjudged=float(np.mean(t_net <= 1.05 * t_best)),
        byte_model_prefers_csr=float(np.mean([x["csr_cheaper"] for x in rows])),
    )
    return rep, rows


def report(net, recs, test, test_paths, train_meta):
    """Held-out evaluation of a trained network, the training-set figures
    beside it, the judge's tolerance sweep on both sets (the tolerance is
    chosen on the training set) and the best fixed grid point."""
    rep, _ = evaluate(net, test)
    rep_train, _ = evaluate(net, recs)
    judge, judge_train = {}, {}
    for tol in (0.0, 0.05, 0.10, 0.25, 1e9):
        for dst, rs in ((judge, test), (judge_train, recs)):
            r_, _ = evaluate(net, rs, tolerance=tol)
            dst["%g" % tol] = {k: r_[k] for k in ("within_5pct_selected", "mean_ratio_selected",
                                                  "used_network", "judge_override_rate")}
    prior = prior_point(recs)
    ks = list(test[0]["us"])
    R = np.array([[r["us"][k] / min(r["us"].values()) for k in ks] for r in test])
    rep.update(judge_tolerance=JUDGE_TOLERANCE, train_matrices=len(recs), prior=prior,
               prior_fixed_on_test=dict(mean_ratio=float(R[:, ks.index(prior)].mean()),
                                        within_5pct=float(np.mean(R[:, ks.index(prior)] <= 1.05))),
               judge_tolerance_sweep=judge, judge_tolerance_sweep_train=judge_train,
               train_set=rep_train, **train_meta)
    if len(test_paths) > 1:  # one summary per held-out file as well
        rep["per_test_file"] = {os.path.basename(t): evaluate(net, load([t]))[0]
                                for t in test_paths}
    return rep


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    c = sub.add_parser("collect")
    c.add_argument("--split", choices=tuple(SEED_BASE), required=True)
    c.add_argument("--start", type=int, default=0)
    c.add_argument("--count", type=int, default=100)
    c.add_argument("--out", required=True)
    t = sub.add_parser("train")
    t.add_argument("--data", nargs="+", required=True)
    t.add_argument("--test", nargs="+", required=True)
    t.add_argument("--steps", type=int, default=8000)
    t.add_argument("--lr", type=float, default=1e-3)
    t.add_argument("--scorer", action="store_true",
                   help="train the 40-output scorer instead of the 2-output network")
    t.add_argument("--out-dir", required=True)
    e = sub.add_parser("evaluate", help="re-evaluate stored weights (no training)")
    e.add_argument("--data", nargs="+", required=True)
    e.add_argument("--test", nargs="+", required=True)
    e.add_argument("--weights", default=WEIGHTS)
    e.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    sys.path.insert(0, os.path.dirname(HERE))
    if a.cmd == "collect":
        collect(a.split, a.start, a.count, a.out)
        return
    recs = load(a.data)
    test = load(a.test)
    if a.cmd == "evaluate":
        meta = {}
        if os.path.exists(a.out):  # keep the training record of the weights
            with open(a.out) as f:
                old = json.load(f)
            meta = {k: old[k] for k in ("train_steps", "train_seconds", "loss_first",
                                         "loss_last", "network", "train_loss",
                                         "train_warm_steps") if k in old}
        rep = report(load_network(a.weights), recs, test, a.test, meta)
        with open(a.out, "w") as f:
            json.dump(rep, f, indent=1)
        print(json.dumps(rep))
        return
    t0 = time.time()
    if a.scorer:
        net, hist, _ = train_scorer(recs, steps=a.steps, lr=a.lr)
        meta = dict(network="scorer: 66 -> 128 -> 128 -> 40, one estimate of log(t / t_best) "
                            "per grid point, decision = the point of the smallest estimate; "
                            "weights uniform in +-1/sqrt(fan_in) at the start",
                    train_loss="scorer loss (weighted squared error per grid point, weight "
                               "exp(-g / 0.1) + 0.05) on standardised features, "
                               "standardisation folded into the first layer")
    else:
        net, hist, _ = train(recs, steps=a.steps, lr=a.lr)
        meta = dict(network="66 -> 128 -> 128 -> 2, output (theta, log2 n_b)",
                    train_warm_steps=500,
                    train_loss="squared error to the arg-min for the warm-up steps, then "
                               "the grid loss")
    dt = time.time() - t0
    os.makedirs(a.out_dir, exist_ok=True)
    np.save(os.path.join(a.out_dir, "weights.npy"), net.params())
    rep = report(net, recs, test, a.test,
                 dict(train_steps=a.steps, train_seconds=round(dt, 2),
                      loss_first=float(hist[:20].mean()), loss_last=float(hist[-20:].mean()),
                      **meta))
    with open(os.path.join(a.out_dir, "eval_report.json"), "w") as f:
        json.dump(rep, f, indent=1)
    print(json.dumps(rep))


if __name__ == "__main__":
    main()
