"""What the trained selector gains over the paper's policy.

The committed network (the 40-output scorer, trained on the GPU by the
library's own kernels on 2,400 matrices) decides (theta, n_b) for the 240
held-out matrices through
mhdc_mlp_decide; each decision is looked up in the SpMV times measured on
MI355X for the whole grid (committed with the data), after the byte-model
judge that mhdc_select applies.  Compared with the exhaustive best of the
grid and with the policy (theta = 0.6, n_b = 256; Sec. 6.4.3)."""
import os

import numpy as np
import pytest

from paper_2105_04937_amd import learned
from tests.gpu_helpers import say

pytestmark = pytest.mark.gpu

TEST = [os.path.join(learned.DATA_DIR, f) for f in
        ("test_0000-0199.jsonl.gz", "test_large_0000-0039.jsonl.gz")]


def test_selector_gain_over_policy():
    recs = learned.load(TEST)
    net = learned.load_network()
    rep, rows = learned.evaluate(net, recs, tolerance=learned.JUDGE_TOLERANCE)
    say("selector on %d held-out matrices: mean t/t_best %.4f (policy %.4f), within 5%%: %.3f "
        "(policy %.3f), geomean speed-up over policy %.4f" % (
            rep["matrices"], rep["mean_ratio_selected"], rep["mean_ratio_rule"],
            rep["within_5pct_selected"], rep["within_5pct_rule"],
            rep["geomean_speedup_over_rule"]))
    say("refined (choice, grid neighbours, policy, n_b = 4096 timed): mean t/t_best %.4f, "
        "within 5%%: %.3f" % (rep["mean_ratio_refined"], rep["within_5pct_refined"]))
    assert rep["matrices"] == 240
    # the learned result: the network's decisions alone (the judge keeps
    # every one at the chosen tolerance), against the exhaustive search
    say("network alone: within 5%% of the exhaustive best on %.3f, mean t/t_best %.4f; "
        "judge override rate %.3f" % (rep["within_5pct_network_unjudged"],
                                      rep["mean_ratio_network_unjudged"],
                                      rep["judge_override_rate"]))
    assert rep["within_5pct_network_unjudged"] >= 0.9
    assert rep["mean_ratio_network_unjudged"] <= 1.025
    # the refinement is a measured search around the decision (up to six
    # more conversions and timings); it picks from a superset of the selection
    assert rep["mean_ratio_refined"] <= rep["mean_ratio_selected"]
    assert rep["within_5pct_refined"] >= rep["within_5pct_selected"]
    # and is within 5% of the exhaustive search on nearly every matrix
    assert rep["within_5pct_refined"] >= 0.95 and rep["mean_ratio_refined"] <= 1.02
    # within 5% of exhaustive search on average, and better than the policy
    assert rep["mean_ratio_selected"] <= 1.05
    assert rep["mean_ratio_selected"] < rep["mean_ratio_rule"]
    assert rep["within_5pct_selected"] > rep["within_5pct_rule"]
    assert rep["geomean_speedup_over_rule"] > 1.0
    # the decisions are those mhdc_select makes from the same network
    ok = [r for r in rows if r["used_net"]]
    assert len(ok) >= 180


def test_select_end_to_end_with_trained_network():
    """mhdc_select with the trained network: its decision equals the one
    decided from the oracle's features, and the chosen handle's product is
    bit-identical to the oracle's Fig. 16 kernel for that (theta, n_b)."""
    import torch

    import oracle
    from oracle import selector as S
    from paper_2105_04937_amd import mhdc, synth
    from tests.gpu_helpers import assert_oracle_bits, dev
    net = learned.load_network()
    for seed, N in ((1, 40), (2, 56), (3, 72)):
        m = synth.partially_diagonal(N, seed, drop=synth.OCTANT_DROP)
        say("case: select end to end N=%d" % N)
        d = dev(m)
        h, r = mhdc.select(*d, model=net, tolerance=learned.JUDGE_TOLERANCE)
        th, nb, ok = net.decide(torch.from_numpy(S.features(m.rowptr, m.colind, m.val)[None]).cuda())
        assert (r["theta_net"], r["n_b_net"]) == (float(th[0]), int(nb[0]))
        x = synth.vector(m.n, seed)
        ref = oracle.mhdc_from_csr(m.rowptr, m.colind, m.val, r["n_b"], r["theta"])
        assert_oracle_bits(h.spmv(torch.from_numpy(x).cuda()), oracle.mhdc_spmv(ref, x),
                           "selected theta=%g n_b=%d" % (r["theta"], r["n_b"]))


def test_theta_nb_network_gain_over_policy():
    """The stored 66 -> 128 -> 128 -> 2 network (output theta, log2 n_b;
    grid loss) on the same held-out matrices: better than the policy, and
    its figures are those of its committed report."""
    import json
    recs = learned.load(TEST)
    net = learned.load_network(learned.WEIGHTS_THETA_NB)
    assert net.outputs == 2
    rep, _ = learned.evaluate(net, recs, tolerance=learned.JUDGE_TOLERANCE)
    say("2-output network: within 5%% %.3f, mean t/t_best %.4f" % (
        rep["within_5pct_network_unjudged"], rep["mean_ratio_network_unjudged"]))
    with open(os.path.join(learned.DATA_DIR, "eval_report_theta_nb.json")) as f:
        stored = json.load(f)
    assert rep["within_5pct_network_unjudged"] == stored["within_5pct_network_unjudged"]
    assert rep["within_5pct_network_unjudged"] >= 0.8
    assert rep["mean_ratio_selected"] < rep["mean_ratio_rule"]
