"""GPU side of the learned selector through the C-ABI: the census features
against the oracle bit for bit, the network's forward pass and gradient
against the FP64 oracle, Adam training against the oracle's Adam, training
determinism, and mhdc_select's judge and fallback."""
import numpy as np
import pytest
import torch

import oracle
from oracle import selector as S
from paper_2105_04937_amd import mhdc, synth
from tests.gpu_helpers import assert_oracle_bits, dev, say

pytestmark = pytest.mark.gpu


def _feature_cases():
    return [
        synth.random_csr(300, 1, density=0.02, bands=[0, 1, -7, 40], zero_frac=0.1),
        synth.random_csr(600, 2, density=0.1, bands=[0, 3]),  # > 8192 entries per block
        synth.laplacian7(16),
        synth.partially_diagonal(20, 4),
        synth.heptadiagonal(24, 5),
        synth.random_csr(1, 3, density=1.0),
    ]


@pytest.mark.parametrize("m", _feature_cases(), ids=lambda m: "n%d" % m.n)
def test_features_match_oracle(m):
    say("case: features n=%d nnz=%d" % (m.n, m.nnz))
    f = mhdc.features(*dev(m)).cpu().numpy()
    want = S.features(m.rowptr, m.colind, m.val)
    assert np.array_equal(f[:64].view(np.int32), want[:64].view(np.int32))
    # log2 terms: one float32 ulp at most
    assert np.all(np.abs(f[64:].view(np.int32) - want[64:].view(np.int32)) <= 1)


def _params(seed, noise=0.05):
    rng = np.random.default_rng(seed)
    p = S.init_params(seed)
    return (p + rng.normal(0, noise, p.size)).astype(np.float32)


def test_forward_and_gradient_match_oracle():
    say("case: mlp forward / gradient")
    rng = np.random.default_rng(0)
    p = _params(1)
    net = mhdc.MLP(p)
    for B in (1, 37, 128):
        X = rng.uniform(0, 1, size=(B, 66)).astype(np.float32)
        T = rng.normal(size=(B, 2)).astype(np.float32)
        Xd, Td = torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()
        out = net.forward(Xd).cpu().numpy()
        ref, _ = S.forward(p, X)
        assert np.allclose(out, ref, rtol=1e-5, atol=1e-5)
        loss, g = net.loss_grad(Xd, Td, w=(25.0, 0.1))
        L, gref = S.loss_and_grad(p, X, T, w=(25.0, 0.1))
        assert abs(loss.item() - L) <= 1e-5 * max(1.0, abs(L))
        g = g.cpu().numpy()
        assert np.allclose(g, gref, rtol=1e-3, atol=1e-5 * np.abs(gref).max())
    net.close()


def test_training_matches_oracle_adam_and_is_deterministic():
    say("case: mlp training")
    rng = np.random.default_rng(5)
    N, B, steps, lr = 300, 32, 6, 1e-3
    X = rng.uniform(0, 1, size=(N, 66)).astype(np.float32)
    T = np.stack([0.5 + 0.4 * X[:, 3], 5 + 7 * X[:, 10]], axis=1).astype(np.float32)
    order = np.concatenate([rng.permutation(N)[:B] for _ in range(steps)]).astype(np.int32)
    p0 = _params(7, noise=0.0)
    Xd, Td, od = (torch.from_numpy(a).cuda() for a in (X, T, order))
    net = mhdc.MLP(p0)
    hist = net.train(Xd, Td, od, steps, B, lr, w=(25.0, 0.1)).cpu().numpy()
    p_gpu = net.params()
    # oracle: the same minibatches, FP64 backprop and Adam
    p = p0.astype(np.float64)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    for t in range(steps):
        idx = order[t * B:(t + 1) * B]
        L, g = S.loss_and_grad(p, X[idx], T[idx], w=(25.0, 0.1))
        assert abs(hist[t] - L) <= 1e-4 * max(1.0, L)
        p, m, v = S.adam(p, g, m, v, t + 1, lr)
    d = np.abs(p_gpu - p)
    assert d.max() <= 2 * steps * lr          # an Adam step moves a weight by at most ~lr
    assert np.quantile(d, 0.99) <= 1e-5       # and nearly all agree to FP32 accuracy
    # determinism: the same start and order give the same bits
    net2 = mhdc.MLP(p0)
    net2.train(Xd, Td, od, steps, B, lr, w=(25.0, 0.1))
    assert np.array_equal(net2.params().view(np.int32), p_gpu.view(np.int32))
    # a row index outside [0, N) is rejected before any step runs
    for badval in (N, -1):
        bad = od.clone()
        bad[B + 3] = badval
        net3 = mhdc.MLP(p0)
        with pytest.raises(mhdc.MhdcError) as ei:
            net3.train(Xd, Td, bad, steps, B, lr, w=(25.0, 0.1))
        assert ei.value.name == "MHDC_ERR_INVALID_ARG"
        assert np.array_equal(net3.params().view(np.int32), p0.view(np.int32))


def _inside_params(X, seed):
    """Parameters whose outputs on X fall inside the sweep grid's cells."""
    p = _params(seed, noise=0.0).astype(np.float64) * 0.5
    out, _ = S.forward(p, X)
    p[-2] += 0.645 - out[:, 0].mean()
    p[-1] += 8.45 - out[:, 1].mean()
    return p.astype(np.float32)


def test_grid_loss_gradient_matches_oracle():
    """The grid loss of the measured-time landscape and its gradient by
    backpropagation against the FP64 oracle, for outputs inside the grid and
    outside it (where only the distance penalty acts on that output)."""
    say("case: mlp grid loss / gradient")
    rng = np.random.default_rng(8)
    for B, shift in ((5, (0.0, 0.0)), (37, (0.0, 0.0)), (64, (0.6, -4.0)), (16, (-0.4, 6.0))):
        X = rng.uniform(0, 1, size=(B, 66)).astype(np.float32)
        p = _inside_params(X, 3 + B)
        p[-2] += shift[0]
        p[-1] += shift[1]
        G = rng.uniform(0.0, 0.4, size=(B, 40)).astype(np.float32)
        net = mhdc.MLP(p)
        loss, g = net.grid_loss_grad(torch.from_numpy(X).cuda(), torch.from_numpy(G).cuda())
        L, gref = S.grid_loss_and_grad(p.astype(np.float64), X, G)
        assert abs(loss.item() - L) <= 1e-5 * max(1.0, abs(L)), (loss.item(), L)
        g = g.cpu().numpy()
        assert np.allclose(g, gref, rtol=1e-3, atol=1e-5 * np.abs(gref).max())
        net.close()


def test_grid_training_matches_oracle_adam_and_is_deterministic():
    say("case: mlp training with the grid loss")
    rng = np.random.default_rng(9)
    N, B, steps, lr = 200, 32, 5, 1e-3
    X = rng.uniform(0, 1, size=(N, 66)).astype(np.float32)
    G = rng.uniform(0.0, 0.4, size=(N, 40)).astype(np.float32)
    order = np.concatenate([rng.permutation(N)[:B] for _ in range(steps)]).astype(np.int32)
    p0 = _inside_params(X, 11)
    Xd, Gd, od = (torch.from_numpy(a).cuda() for a in (X, G, order))
    net = mhdc.MLP(p0)
    hist = net.train_grid(Xd, Gd, od, steps, B, lr).cpu().numpy()
    p_gpu = net.params()
    p = p0.astype(np.float64)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    for t in range(steps):
        idx = order[t * B:(t + 1) * B]
        L, g = S.grid_loss_and_grad(p, X[idx], G[idx])
        assert abs(hist[t] - L) <= 1e-4 * max(1.0, L)
        p, m, v = S.adam(p, g, m, v, t + 1, lr)
    d = np.abs(p_gpu - p)
    assert d.max() <= 2 * steps * lr
    assert np.quantile(d, 0.99) <= 1e-5
    net2 = mhdc.MLP(p0)
    net2.train_grid(Xd, Gd, od, steps, B, lr)
    assert np.array_equal(net2.params().view(np.int32), p_gpu.view(np.int32))
    bad = od.clone()
    bad[7] = N
    net3 = mhdc.MLP(p0)
    with pytest.raises(mhdc.MhdcError) as ei:
        net3.train_grid(Xd, Gd, bad, steps, B, lr)
    assert ei.value.name == "MHDC_ERR_INVALID_ARG"


def test_training_reduces_loss():
    say("case: mlp training reduces loss")
    rng = np.random.default_rng(9)
    N, B, steps = 1024, 128, 400
    X = rng.uniform(0, 1, size=(N, 66)).astype(np.float32)
    T = np.stack([0.5 + 0.4 * X[:, 0] * X[:, 1], 5 + 7 * X[:, 40]], axis=1).astype(np.float32)
    order = np.concatenate([rng.permutation(N)[:B] for _ in range(steps)]).astype(np.int32)
    net = mhdc.MLP(S.init_params(3))
    hist = net.train(*(torch.from_numpy(a).cuda() for a in (X, T, order)), steps, B, 3e-3,
                     w=(25.0, 0.1)).cpu().numpy()
    assert hist[-20:].mean() < 0.1 * hist[:5].mean()


def _fixed_net(theta, log2nb):
    p = np.zeros(S.N_PARAMS, np.float32)
    p[-2], p[-1] = theta, log2nb   # b3: constant output
    return mhdc.MLP(p)


def test_select_policy_network_and_judge():
    m = synth.partially_diagonal(24, 12)
    say("case: select n=%d" % m.n)
    d = dev(m)
    x = synth.vector(m.n, 1)
    xd = torch.from_numpy(x).cuda()
    h, r = mhdc.select(*d, model=None)
    assert (r["theta"], r["n_b"], r["used_rule"]) == (0.6, 256, 1)
    ref = oracle.mhdc_from_csr(m.rowptr, m.colind, m.val, 256, 0.6)
    assert_oracle_bits(h.spmv(xd), oracle.mhdc_spmv(ref, x), "policy")
    # a network that always proposes (0.7, 128): kept when the model allows it
    net = _fixed_net(0.68, 7.2)
    h, r = mhdc.select(*d, model=net, tolerance=1e9)
    assert (r["theta_net"], r["n_b_net"], r["net_ok"]) == (0.7, 128, 1)
    assert (r["theta"], r["n_b"], r["used_rule"]) == (0.7, 128, 0)
    inf = h.info()
    assert (inf["n_b"], inf["theta"]) == (128, 0.7)
    ref = oracle.mhdc_from_csr(m.rowptr, m.colind, m.val, 128, 0.7)
    assert_oracle_bits(h.spmv(xd), oracle.mhdc_spmv(ref, x), "network choice")
    # the judge: a proposal the byte model rates worse than the policy is refused
    bad = _fixed_net(0.9, 12.0)
    h, r = mhdc.select(*d, model=bad, tolerance=0.0)
    if r["bytes_net"] > r["bytes_rule"]:
        assert r["used_rule"] == 1 and (r["theta"], r["n_b"]) == (0.6, 256)
    else:
        assert r["used_rule"] == 0
    # non-finite output: fallback
    p = np.zeros(S.N_PARAMS, np.float32)
    p[-2] = np.nan
    h, r = mhdc.select(*d, model=mhdc.MLP(p))
    assert r["net_ok"] == 0 and r["used_rule"] == 1


@pytest.mark.parametrize("theta", [0.0, 0.5, 0.9])
def test_select_reports_the_csr_verdict(theta):
    """The byte model's verdict on the chosen layout against plain CSR
    (Sec. 5.3): rp_est = V_CSR / V of the chosen handle, its alpha and beta,
    and csr_cheaper exactly when V_CSR < V, i.e. alpha < 2/3 (Eqs. 31-32),
    the oracle model evaluated on the oracle converter's layout."""
    from oracle import model
    m = synth.random_csr(400, 21, density=0.01, bands=[0, 1, -1, 5, -9, 40], band_fill=0.62)
    say("case: select verdict theta=%.1f" % theta)
    d = dev(m)
    net = _fixed_net(theta, 6.0)   # proposes (clip(theta, 0.5, 0.9), 64)
    h, r = mhdc.select(*d, model=net, tolerance=1e9)
    ref = oracle.mhdc_from_csr(m.rowptr, m.colind, m.val, r["n_b"], r["theta"])
    S_, R_ = ref.dia_val.size, ref.R
    v = model.v_hdc_blocked(m.n, R_, S_)
    v_csr = model.v_csr_general(m.n, m.nnz)
    assert r["rp_est"] == v_csr / v
    assert (r["alpha"], r["beta"]) == model.alpha_beta(m.nnz, R_, S_)
    assert r["csr_cheaper"] == int(v_csr < v)
    assert r["csr_cheaper"] == int(S_ > 0 and r["alpha"] < 2.0 / 3.0)
    h.close()


def test_select_refine_returns_a_timed_neighbour():
    """mhdc_select_refine returns mhdc_select's choice, one of its grid
    neighbours (n_b halved / doubled, theta -+ 0.1), the policy or the
    choice's theta at n_b = 4096, and the handle is exactly the oracle's
    conversion of that (theta, n_b)."""
    m = synth.partially_diagonal(24, 12)
    say("case: select refine n=%d" % m.n)
    d = dev(m)
    x = synth.vector(m.n, 2)
    xd = torch.from_numpy(x).cuda()
    for model in (None, _fixed_net(0.68, 7.2), _fixed_net(0.9, 12.0)):
        _, r0 = mhdc.select(*d, model=model, tolerance=1e9)
        h, r = mhdc.select_refine(*d, model=model, tolerance=1e9)
        allowed = {(round(r0["theta"], 1), r0["n_b"]), (0.6, 256), (round(r0["theta"], 1), 4096)}
        for th, nb in ((r0["theta"], r0["n_b"] // 2), (r0["theta"], r0["n_b"] * 2),
                       (r0["theta"] - 0.1, r0["n_b"]), (r0["theta"] + 0.1, r0["n_b"])):
            th = round(th, 1)
            if 0.5 <= th <= 0.9 and 32 <= nb <= 4096:
                allowed.add((th, nb))
        got = (round(r["theta"], 1), r["n_b"])
        assert got in allowed, (got, allowed)
        assert r["used_rule"] == (got == (0.6, 256))
        inf = h.info()
        assert (round(inf["theta"], 1), inf["n_b"]) == got
        ref = oracle.mhdc_from_csr(m.rowptr, m.colind, m.val, got[1], r["theta"])
        assert_oracle_bits(h.spmv(xd), oracle.mhdc_spmv(ref, x), "refined %s" % (got,))
        h.close()


def test_select_refine_tiny_matrices():
    """One-row and empty-band matrices go through the refinement as well."""
    for m in (synth.random_csr(1, 3, density=1.0), synth.random_csr(50, 4, density=0.0),
              synth.random_csr(70, 5, density=0.1, bands=[0, 1])):
        say("case: select refine n=%d nnz=%d" % (m.n, m.nnz))
        d = dev(m)
        h, r = mhdc.select_refine(*d, model=_fixed_net(0.68, 7.2))
        x = synth.vector(m.n, 3)
        ref = oracle.mhdc_from_csr(m.rowptr, m.colind, m.val, r["n_b"], r["theta"])
        assert_oracle_bits(h.spmv(torch.from_numpy(x).cuda()), oracle.mhdc_spmv(ref, x),
                           "tiny refined")
        h.close()


# ------------------------------------------------------------------ scorer
def _scorer_params(seed, noise=0.05):
    rng = np.random.default_rng(seed)
    p = S.init_params(seed, S.N_SCORES)
    return (p + rng.normal(0, noise, p.size)).astype(np.float32)


def test_scorer_forward_loss_gradient_match_oracle():
    """The 40-output scorer through the C-ABI: forward pass, scorer loss and
    gradient against the FP64 oracle; the squared error to 2 targets is not
    offered for it."""
    say("case: scorer forward / loss / gradient")
    rng = np.random.default_rng(12)
    p = _scorer_params(2)
    net = mhdc.MLP(p)
    assert net.outputs == 40 and net.params().size == S.N_PARAMS_SCORER
    assert np.array_equal(net.params().view(np.int32), p.view(np.int32))
    for B in (1, 37, 128):
        X = rng.uniform(0, 1, size=(B, 66)).astype(np.float32)
        G = rng.uniform(0.0, 0.5, size=(B, 40)).astype(np.float32)
        G[:, 3] = 0.0
        Xd, Gd = torch.from_numpy(X).cuda(), torch.from_numpy(G).cuda()
        out = net.forward(Xd).cpu().numpy()
        ref, _ = S.forward(p, X)
        assert out.shape == (B, 40) and np.allclose(out, ref, rtol=1e-5, atol=1e-5)
        loss, g = net.grid_loss_grad(Xd, Gd)
        L, gref = S.score_loss_and_grad(p.astype(np.float64), X, G)
        assert abs(loss.item() - L) <= 1e-5 * max(1.0, abs(L)), (loss.item(), L)
        g = g.cpu().numpy()
        assert g.size == S.N_PARAMS_SCORER
        assert np.allclose(g, gref, rtol=1e-3, atol=1e-5 * np.abs(gref).max())
        o2 = torch.empty((B, 40), dtype=torch.float32, device="cuda")
        net.forward_noalloc(Xd, o2)
        assert np.array_equal(o2.cpu().numpy().view(np.int32), out.view(np.int32))
    with pytest.raises(mhdc.MhdcError) as ei:
        net.loss_grad(Xd, torch.zeros((B, 2), dtype=torch.float32, device="cuda"))
    assert ei.value.name == "MHDC_ERR_NOT_SUPPORTED"
    net.close()


def test_scorer_training_matches_oracle_adam_and_is_deterministic():
    say("case: scorer training")
    rng = np.random.default_rng(13)
    N, B, steps, lr = 200, 32, 5, 1e-3
    X = rng.uniform(0, 1, size=(N, 66)).astype(np.float32)
    G = rng.uniform(0.0, 0.4, size=(N, 40)).astype(np.float32)
    order = np.concatenate([rng.permutation(N)[:B] for _ in range(steps)]).astype(np.int32)
    p0 = _scorer_params(14)
    Xd, Gd, od = (torch.from_numpy(a).cuda() for a in (X, G, order))
    net = mhdc.MLP(p0)
    hist = net.train_grid(Xd, Gd, od, steps, B, lr).cpu().numpy()
    p_gpu = net.params()
    p = p0.astype(np.float64)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    for t in range(steps):
        idx = order[t * B:(t + 1) * B]
        L, g = S.score_loss_and_grad(p, X[idx], G[idx])
        assert abs(hist[t] - L) <= 1e-4 * max(1.0, L)
        p, m, v = S.adam(p, g, m, v, t + 1, lr)
    d = np.abs(p_gpu - p)
    assert d.max() <= 2 * steps * lr
    assert np.quantile(d, 0.99) <= 1e-5
    net2 = mhdc.MLP(p0)
    net2.train_grid(Xd, Gd, od, steps, B, lr)
    assert np.array_equal(net2.params().view(np.int32), p_gpu.view(np.int32))
    with pytest.raises(mhdc.MhdcError) as ei:
        net2.train(Xd, torch.zeros((N, 2), dtype=torch.float32, device="cuda"), od, steps, B, lr)
    assert ei.value.name == "MHDC_ERR_NOT_SUPPORTED"


def test_scorer_decide_and_select():
    """decide takes the grid point of the smallest output, as the oracle's
    decode_scores does on the oracle's forward pass; mhdc_select builds the
    handle of a constant scorer's point (judge permitting)."""
    say("case: scorer decide / select")
    rng = np.random.default_rng(15)
    p = _scorer_params(16, noise=0.2)
    net = mhdc.MLP(p)
    X = rng.uniform(0, 1, size=(300, 66)).astype(np.float32)
    th, nb, ok = (t.cpu().numpy() for t in net.decide(torch.from_numpy(X).cuda()))
    out = net.forward(torch.from_numpy(X).cuda()).cpu().numpy()
    wth, wnb, wok = S.decode_scores(out)   # decode of the GPU's own outputs: exact
    assert np.array_equal(th, wth) and np.array_equal(nb, wnb) and np.array_equal(ok, wok)
    rth, rnb, _ = S.decode_scores(S.forward(p, X)[0])
    assert np.mean((rth == th) & (rnb == nb)) >= 0.99   # FP32 vs FP64 near-ties aside
    net.close()
    # a constant scorer (b3 only) whose smallest output is (0.7, 128)
    c = np.ones(40, np.float32)
    c[8 * 2 + 2] = -1.0
    q = np.zeros(S.N_PARAMS_SCORER, np.float32)
    q[-40:] = c
    const = mhdc.MLP(q)
    m = synth.partially_diagonal(24, 7)
    h, res = mhdc.select(*dev(m), model=const, tolerance=1e9)
    assert (res["theta_net"], res["n_b_net"], res["net_ok"]) == (0.7, 128, 1)
    assert (res["theta"], res["n_b"], res["used_rule"]) == (0.7, 128, 0)
    assert h.info()["n_b"] == 128 and abs(h.info()["theta"] - 0.7) < 1e-12
    h.close()
    const.close()
