"""Pins of the selector oracle: the census features against a brute-force
count over dense diagonals and closed forms, backpropagation against
central finite differences in FP64, Adam against its first-step closed form."""
import numpy as np
import pytest

from oracle import selector as S
from paper_2105_04937_amd import synth


def test_param_count():
    assert S.N_PARAMS == 66 * 128 + 128 + 128 * 128 + 128 + 128 * 2 + 2 == 25_346


def test_offset_bins():
    d = np.array([0, 1, 2, 3, 4, 7, 8, -1, -2, -3, -4, 2**30, -(2**30), 2**31 - 1, 5, -6])
    want = [32, 33, 34, 34, 35, 35, 36, 31, 30, 30, 29, 63, 1, 63, 35, 29]
    assert list(S.offset_bin(d)) == want
    a = np.array([1, 2, 3, 4, 2**20 - 1, 2**20, 2**30 + 5])
    assert list(S.floor_log2(a)) == [0, 1, 1, 2, 19, 20, 30]


def _brute(A, nb):
    n = A.shape[0]
    nnz_stored = None
    f = np.zeros(S.N_IN)
    n_blk = (n + nb - 1) // nb
    for ib in range(n_blk):
        r0, r1 = ib * nb, min(n, ib * nb + nb)
        for d in range(-(n - 1), n):
            cnt = sum(1 for i in range(r0, r1) if 0 <= i + d < n and A[i, i + d] != 0)
            if cnt:
                if d == 0:
                    b = 32
                else:
                    k = abs(d).bit_length() - 1
                    b = 33 + min(k, 30) if d > 0 else 31 - min(k, 31)
                f[b] += cnt * cnt / (r1 - r0)
    return f, nnz_stored


@pytest.mark.parametrize("n,nb", [(40, 8), (33, 7), (64, 64), (20, 256)])
def test_features_brute_force(n, nb):
    m = synth.random_csr(n, n + nb, density=0.1, bands=[0, 1, -3, 9], zero_frac=0.1)
    A = synth.dense_of(m)
    f = S.features(m.rowptr, m.colind, m.val, probe_nb=nb)
    raw, _ = _brute(A, nb)
    assert np.allclose(f[:64], (raw[:64] / m.nnz).astype(np.float32), rtol=1e-6, atol=0)
    assert f[64] == np.float32(np.log2(n) / 32)
    assert f[65] == np.float32(np.log2(m.nnz) / 32)


def test_features_closed_forms():
    # identity: one full diagonal per block -> f[32] = 1
    n = 700
    rp = np.arange(n + 1, dtype=np.int32)
    ci = np.arange(n, dtype=np.int32)
    f = S.features(rp, ci, np.ones(n))
    assert f[32] == 1.0 and f[:64].sum() == 1.0
    # 7-point grid with bl = N = 256: the bins of +-1, +-256, +-65536 and 0
    # hold full (or one-short) partial diagonals; their total is close to 1
    m = synth.laplacian7(16)
    f = S.features(m.rowptr, m.colind, m.val, probe_nb=256)
    assert 0.9 < f[:64].sum() <= 1.0
    want = {int(S.offset_bin(d)) for d in (0, 1, -1, 16, -16, 256, -256)}
    assert set(int(b) for b in np.nonzero(f[:64])[0]) == want


def test_backprop_matches_finite_differences():
    rng = np.random.default_rng(0)
    p = S.init_params(1).astype(np.float64) + rng.normal(0, 0.01, S.N_PARAMS)
    X = rng.uniform(0, 1, size=(7, S.N_IN))
    T = rng.normal(size=(7, 2))
    L, g = S.loss_and_grad(p, X, T, w=(1.0, 0.25))
    idx = rng.choice(S.N_PARAMS, size=300, replace=False)
    idx = np.concatenate([idx, [S.N_PARAMS - 1, S.N_PARAMS - 2, S.N_PARAMS - 130, 0]])
    h = 1e-6
    for i in idx:
        e = np.zeros(S.N_PARAMS)
        e[i] = h
        Lp, _ = S.loss_and_grad(p + e, X, T, w=(1.0, 0.25))
        Lm, _ = S.loss_and_grad(p - e, X, T, w=(1.0, 0.25))
        fd = (Lp - Lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(2)
    p = rng.normal(size=50)
    g = rng.normal(size=50)
    p1, m, v = S.adam(p, g, np.zeros(50), np.zeros(50), 1, lr=0.01, eps=0.0)
    assert np.allclose(p1, p - 0.01 * np.sign(g), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_decode():
    th, nb = S.decode([[0.3, 4.2], [0.72, 7.6], [1.5, 20.0], [0.649, 8.5]])
    assert list(th) == [0.5, 0.7, 0.9, 0.6] and list(nb) == [32, 256, 4096, 256]


# ------------------------------------------------------------ grid loss
def _grid(rng, B):
    return rng.uniform(0.0, 0.5, size=(B, S.GRID_TH, S.GRID_NB))


def test_grid_value_at_nodes_and_outside():
    """At a grid point the value is that point's entry; outside the box it
    is the clamped point's value plus the distance in output units, with
    slope -1 / +1 pointing back into the box."""
    rng = np.random.default_rng(3)
    G = _grid(rng, 1)
    for i in range(S.GRID_TH):
        for j in range(S.GRID_NB):
            v, _ = S.grid_value(G, [[0.5 + 0.1 * i, 5.0 + j]])
            assert abs(v[0] - G[0, i, j]) <= 1e-12
    v, d = S.grid_value(G, [[0.3, 13.5]])
    assert abs(v[0] - (G[0, 0, 7] + 0.2 + 1.5)) <= 1e-12
    assert list(d[0]) == [-1.0, 1.0]
    v, d = S.grid_value(G, [[1.2, 2.0]])
    assert abs(v[0] - (G[0, 4, 0] + 0.3 + 3.0)) <= 1e-12
    assert list(d[0]) == [1.0, -1.0]


def test_grid_value_affine_closed_form():
    """On an affine grid G[i][j] = a i + b j + c the bilinear value is
    exactly affine: a u + b v + c with u = (theta - 0.5)/0.1, v = log2 n_b
    - 5, and the output gradient is (a / 0.1, b)."""
    rng = np.random.default_rng(4)
    a, b, c = 0.07, -0.03, 0.2
    ii, jj = np.meshgrid(np.arange(S.GRID_TH), np.arange(S.GRID_NB), indexing="ij")
    G = np.broadcast_to(a * ii + b * jj + c, (9, S.GRID_TH, S.GRID_NB))
    o = np.stack([rng.uniform(0.51, 0.89, 9), rng.uniform(5.1, 11.9, 9)], axis=1)
    v, d = S.grid_value(G, o)
    want = a * (o[:, 0] - 0.5) / 0.1 + b * (o[:, 1] - 5.0) + c
    assert np.allclose(v, want, rtol=0, atol=1e-12)
    assert np.allclose(d, [[a / 0.1, b]] * 9, rtol=0, atol=1e-12)


def test_grid_backprop_matches_finite_differences():
    """dL/dp of the grid loss against central differences in FP64, at
    parameters whose outputs lie inside grid cells (away from the kinks on
    the grid lines, where the loss has no derivative)."""
    rng = np.random.default_rng(5)
    p = S.init_params(6).astype(np.float64) * 0.5
    X = rng.uniform(0, 1, size=(6, S.N_IN))
    # place the outputs inside cells through the output bias
    out, _ = S.forward(p, X)
    p[-2] += 0.645 - out[:, 0].mean()
    p[-1] += 8.45 - out[:, 1].mean()
    out, _ = S.forward(p, X)
    u, v = (out[:, 0] - 0.5) / 0.1, out[:, 1] - 5.0
    assert np.all(np.abs(u - np.round(u)) > 1e-3) and np.all(np.abs(v - np.round(v)) > 1e-3)
    assert np.all((out[:, 0] > 0.5) & (out[:, 0] < 0.9) & (out[:, 1] > 5) & (out[:, 1] < 12))
    G = _grid(rng, 6)
    L, g = S.grid_loss_and_grad(p, X, G)
    idx = np.concatenate([rng.choice(S.N_PARAMS, size=200, replace=False),
                          [S.N_PARAMS - 1, S.N_PARAMS - 2, S.N_PARAMS - 130, 0]])
    h = 1e-7
    for i in idx:
        e = np.zeros(S.N_PARAMS)
        e[i] = h
        Lp, _ = S.grid_loss_and_grad(p + e, X, G)
        Lm, _ = S.grid_loss_and_grad(p - e, X, G)
        fd = (Lp - Lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-5 * max(1.0, abs(fd)), (i, fd, g[i])


# ---------------------------------------------------------------- scorer
def test_scorer_param_count_and_layout():
    """66 -> 128 -> 128 -> 40: 66*128 + 128 + 128*128 + 128 + 40*128 + 40
    parameters; the output count is read back from a vector's length."""
    assert S.N_PARAMS_SCORER == 66 * 128 + 128 + 128 * 128 + 128 + 40 * 128 + 40 == 30248
    assert S.n_outputs(S.init_params(0, S.N_SCORES)) == 40
    assert S.n_outputs(S.init_params(0)) == 2
    assert S.forward(S.init_params(3, 40), np.ones((2, S.N_IN)))[0].shape == (2, 40)


def _constant_scorer(c):
    """Scorer parameters whose output is the constant vector c for every
    input (all weights zero, b3 = c)."""
    p = np.zeros(S.N_PARAMS_SCORER)
    p[-S.N_SCORES:] = c
    return p


def test_scorer_loss_closed_forms():
    """Zero at out = G; out = G + delta e_k costs w_k delta^2 / 40 with
    w_k = exp(-G_k / T) + F: a near-best point (G_k = 0) weighs 1 + F, a
    point twice as slow (G_k = log 2) exp(-log 2 / T) + F."""
    rng = np.random.default_rng(5)
    G = rng.uniform(0.0, 0.6, size=S.N_SCORES)
    G[7] = 0.0
    G[30] = np.log(2.0)
    X = rng.uniform(0, 1, size=(1, S.N_IN))
    L, g = S.score_loss_and_grad(_constant_scorer(G), X, G[None])
    assert L == 0.0 and not np.any(g)
    for k, wk in ((7, 1.0 + S.SCORE_FLOOR), (30, 2.0 ** (-1.0 / S.SCORE_TEMP) + S.SCORE_FLOOR)):
        c = G.copy()
        c[k] += 0.3
        L, g = S.score_loss_and_grad(_constant_scorer(c), X, G[None])
        assert abs(L - wk * 0.09 / 40) <= 1e-15
        # only b3[k] and W3 row k (zero hidden activations) see the error
        gb3 = g[-S.N_SCORES:]
        assert abs(gb3[k] - 2 * wk * 0.3 / 40) <= 1e-15 and np.count_nonzero(gb3) == 1


def test_scorer_backprop_matches_finite_differences():
    rng = np.random.default_rng(6)
    p = S.init_params(2, S.N_SCORES).astype(np.float64) + rng.normal(0, 0.01, S.N_PARAMS_SCORER)
    X = rng.uniform(0, 1, size=(5, S.N_IN))
    G = rng.uniform(0.0, 0.5, size=(5, S.N_SCORES))
    L, g = S.score_loss_and_grad(p, X, G)
    idx = rng.choice(S.N_PARAMS_SCORER, size=300, replace=False)
    idx = np.concatenate([idx, [S.N_PARAMS_SCORER - 1, S.N_PARAMS_SCORER - 41, 0]])
    h = 1e-6
    for i in idx:
        e = np.zeros(S.N_PARAMS_SCORER)
        e[i] = h
        fd = (S.score_loss_and_grad(p + e, X, G)[0] - S.score_loss_and_grad(p - e, X, G)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_decode_scores():
    """Grid point k = 8 i + j (theta outer, the order of the training grids)
    -> theta 0.5 + 0.1 i, n_b 2^(5 + j); the first of equal minima; a
    non-finite row falls back to the policy point with ok = 0."""
    out = np.ones((5, S.N_SCORES))
    out[0, 0] = 0.0            # (0.5, 32)
    out[1, 39] = -1.0          # (0.9, 4096)
    out[2, 9] = out[2, 20] = -2.0   # tie: index 9 = (0.6, 64)
    out[3, 12] = np.nan
    out[4, 8 * 2 + 3] = 0.5    # (0.7, 256)
    th, nb, ok = S.decode_scores(out)
    assert list(th) == [0.5, 0.9, 0.6, 0.6, 0.7]
    assert list(nb) == [32, 4096, 64, 256, 256]
    assert list(ok) == [1, 1, 1, 0, 1]
