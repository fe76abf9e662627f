"""CPU oracle for the learned (theta, n_b) selector -- TEST INFRASTRUCTURE.

The paper leaves open how to decide the M-HDC parameters for a given matrix
(Sec. 7: whether and how to use M-HDC) and proposes a policy instead:
50 <~ bl <~ 500 and theta = 0.6, with the CSR rate as the informative
quantity (Sec. 6.4.3).  The selector replaces the policy by a small network
read off a census of the matrix; this module is the plain FP64 definition of
everything the GPU side computes for it:

* features: a census of partial diagonals at probe block size 256 (the same
  count N~(d, ib) as Sec. 4.3) summarised per offset bin;
* a 66 -> 128 -> 128 -> 2 multilayer perceptron with ReLU hidden layers
  (or 40 outputs, the scorer below), its squared-error loss, the gradient
  by backpropagation, and Adam;
* the grid loss: the network's output read as a point of the (theta,
  log2 n_b) grid on which the paper sweeps its parameters (Sec. 6.4.1),
  scored by the measured time there, interpolated bilinearly between the
  grid points;
* the scorer: the same network with one output per point of that grid
  (66 -> 128 -> 128 -> 40), each output an estimate of the point's log time
  ratio, trained by a weighted squared error and read by taking the grid
  point of the smallest estimate.

Only tests import this module.
"""
from __future__ import annotations

import numpy as np

N_BINS = 64
N_IN = N_BINS + 2
HIDDEN = 128
N_OUT = 2
PROBE_NB = 256


def shapes(n_out: int = N_OUT):
    """Parameter blocks of the 66 -> 128 -> 128 -> n_out network."""
    return [(HIDDEN, N_IN), (HIDDEN,), (HIDDEN, HIDDEN), (HIDDEN,), (n_out, HIDDEN), (n_out,)]


SHAPES = shapes(N_OUT)
N_PARAMS = sum(int(np.prod(s)) for s in SHAPES)  # 25,346


# ----------------------------------------------------------------- features
def floor_log2(a: np.ndarray) -> np.ndarray:
    """floor(log2(a)) for integers a >= 1, exactly."""
    a = np.asarray(a, dtype=np.int64)
    k = np.floor(np.log2(a.astype(np.float64))).astype(np.int64)
    k = np.where((np.int64(1) << (k + 1)) <= a, k + 1, k)
    k = np.where((np.int64(1) << k) > a, k - 1, k)
    return k


def offset_bin(d) -> np.ndarray:
    """Bin of offset d: 32 for d = 0; 33 + min(floor(log2 d), 30) for d > 0;
    31 - min(floor(log2 -d), 31) for d < 0."""
    d = np.asarray(d, dtype=np.int64)
    k = floor_log2(np.maximum(np.abs(d), 1))
    return np.where(d == 0, 32, np.where(d > 0, 33 + np.minimum(k, 30), 31 - np.minimum(k, 31)))


def features(rowptr, colind, val, probe_nb: int = PROBE_NB) -> np.ndarray:
    """66 selector inputs (float32):
    f[b] = (sum over (ib, d) in bin b of N~(d,ib)^2 / rows_ib) / nnz, b < 64,
    with N~ counted at block size probe_nb over entries with val != 0 and
    nnz the number of stored entries; f[64] = log2(n)/32, f[65] = log2(nnz)/32
    (0 for nnz = 0).  The integer sums are split into full blocks and the
    last block so the division happens once per part, in FP64."""
    rowptr = np.asarray(rowptr, np.int64)
    colind = np.asarray(colind, np.int64)
    val = np.asarray(val, np.float64)
    n = rowptr.size - 1
    nnz = int(rowptr[-1])
    f = np.zeros(N_IN, np.float64)
    if n == 0:
        return f.astype(np.float32)
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(rowptr))
    keep = val != 0.0
    r, c = rows[keep], colind[keep]
    ib = r // probe_nb
    d = c - r
    n_blk = (n + probe_nb - 1) // probe_nb
    rows_last = n - (n_blk - 1) * probe_nb
    key = ib * (2 * n) + (d + n)             # one integer per (block, offset)
    uk, cnt = np.unique(key, return_counts=True)
    ub = uk // (2 * n)
    ud = uk % (2 * n) - n
    bins = offset_bin(ud)
    sq = cnt.astype(np.int64) ** 2
    last = ub == n_blk - 1
    s_full = np.bincount(bins[~last], weights=sq[~last], minlength=N_BINS)
    s_last = np.bincount(bins[last], weights=sq[last], minlength=N_BINS)
    if nnz > 0:
        f[:N_BINS] = (s_full / float(probe_nb) + s_last / float(rows_last)) / float(nnz)
        f[N_BINS + 1] = np.log2(float(nnz)) / 32.0
    f[N_BINS] = np.log2(float(n)) / 32.0
    return f.astype(np.float32)


# ----------------------------------------------------------------- network
def init_params(seed: int, n_out: int = N_OUT) -> np.ndarray:
    """He-uniform weights, zero biases, as one float32 vector in the order
    W1 (128x66), b1, W2 (128x128), b2, W3 (n_out x 128), b3 (row-major)."""
    rng = np.random.default_rng(seed)
    parts = []
    for s in shapes(n_out):
        if len(s) == 2:
            lim = np.sqrt(6.0 / s[1])
            parts.append(rng.uniform(-lim, lim, size=s).ravel())
        else:
            parts.append(np.zeros(s))
    return np.concatenate(parts).astype(np.float32)


def n_outputs(p) -> int:
    """Outputs of the network whose parameter vector is p (2 or 40)."""
    rest = len(p) - (HIDDEN * N_IN + HIDDEN + HIDDEN * HIDDEN + HIDDEN)
    assert rest % (HIDDEN + 1) == 0, "not a parameter vector of this network"
    return rest // (HIDDEN + 1)


def unpack(p):
    out, o = [], 0
    for s in shapes(n_outputs(p)):
        k = int(np.prod(s))
        out.append(np.asarray(p[o:o + k], np.float64).reshape(s))
        o += k
    return out


def pack(parts) -> np.ndarray:
    return np.concatenate([np.asarray(a, np.float64).ravel() for a in parts])


def forward(p, X):
    """h1 = relu(X W1^T + b1), h2 = relu(h1 W2^T + b2), out = h2 W3^T + b3."""
    W1, b1, W2, b2, W3, b3 = unpack(p)
    X = np.asarray(X, np.float64)
    a1 = X @ W1.T + b1
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ W2.T + b2
    h2 = np.maximum(a2, 0.0)
    out = h2 @ W3.T + b3
    return out, (X, a1, h1, a2, h2)


def loss_and_grad(p, X, T, w=(1.0, 1.0)):
    """L = sum_b sum_o w_o (out_bo - T_bo)^2 / B and dL/dp by backpropagation."""
    out, cache = forward(p, X)
    B = cache[0].shape[0]
    w = np.asarray(w, np.float64)
    diff = out - np.asarray(T, np.float64)
    L = float(np.sum(w * diff * diff) / B)
    d_out = 2.0 * w * diff / B
    return L, backward(p, cache, d_out)


# the grid of Sec. 6.4.1: theta in 0.5 .. 0.9 (step 0.1), n_b = 2^5 .. 2^12
GRID_TH, GRID_NB = 5, 8


def grid_value(G, o):
    """Loss of outputs o[B][2] = (theta, log2 n_b) on grids G[B][5][8]
    (G[r][i][j]: the measured log time ratio of matrix r at theta = 0.5 +
    0.1 i, n_b = 2^(5+j)).  Inside the grid's box the value is the bilinear
    interpolation of the four surrounding points; the cell of a point on an
    inner grid line is the one above it (i = min(floor(u), 3),
    j = min(floor(v), 6)).  Outside, the value at the clamped point plus the
    distance to the box in output units (|theta - clamp| + |log2 n_b -
    clamp|).  Returns (value[B], d value / d o [B][2])."""
    G = np.asarray(G, np.float64).reshape(-1, GRID_TH, GRID_NB)
    o = np.asarray(o, np.float64)
    t = np.clip(o[:, 0], 0.5, 0.9)
    l = np.clip(o[:, 1], 5.0, 12.0)
    u = (t - 0.5) / 0.1
    v = l - 5.0
    i = np.minimum(np.floor(u), GRID_TH - 2).astype(np.int64)
    j = np.minimum(np.floor(v), GRID_NB - 2).astype(np.int64)
    fu, fv = u - i, v - j
    r = np.arange(o.shape[0])
    g00, g10 = G[r, i, j], G[r, i + 1, j]
    g01, g11 = G[r, i, j + 1], G[r, i + 1, j + 1]
    val = ((1 - fu) * (1 - fv) * g00 + fu * (1 - fv) * g10 + (1 - fu) * fv * g01
           + fu * fv * g11)
    du = (1 - fv) * (g10 - g00) + fv * (g11 - g01)
    dv = (1 - fu) * (g01 - g00) + fu * (g11 - g10)
    inside_t = (o[:, 0] >= 0.5) & (o[:, 0] <= 0.9)
    inside_l = (o[:, 1] >= 5.0) & (o[:, 1] <= 12.0)
    d0 = np.where(inside_t, du / 0.1, np.where(o[:, 0] < 0.5, -1.0, 1.0))
    d1 = np.where(inside_l, dv, np.where(o[:, 1] < 5.0, -1.0, 1.0))
    val = val + np.abs(o[:, 0] - t) + np.abs(o[:, 1] - l)
    return val, np.stack([d0, d1], axis=1)


def grid_loss_and_grad(p, X, G):
    """L = sum_b grid_value(G_b, out_b) / B and dL/dp by backpropagation."""
    out, cache = forward(p, X)
    B = cache[0].shape[0]
    val, d = grid_value(G, out)
    return float(np.sum(val) / B), backward(p, cache, d / B)


def backward(p, cache, d_out):
    """dL/dp for dL/d(out) = d_out through the network of forward()."""
    W1, b1, W2, b2, W3, b3 = unpack(p)
    X, a1, h1, a2, h2 = cache
    gW3 = d_out.T @ h2
    gb3 = d_out.sum(axis=0)
    d_h2 = d_out @ W3
    d_a2 = d_h2 * (a2 > 0)
    gW2 = d_a2.T @ h1
    gb2 = d_a2.sum(axis=0)
    d_h1 = d_a2 @ W2
    d_a1 = d_h1 * (a1 > 0)
    gW1 = d_a1.T @ X
    gb1 = d_a1.sum(axis=0)
    return pack([gW1, gb1, gW2, gb2, gW3, gb3])


def adam(p, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba) at step t >= 1; returns (p, m, v)."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** t)
    vh = v / (1 - beta2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def decode(out):
    """Network output -> (theta, n_b): theta = round(10 clip(o0, 0.5, 0.9))/10
    (the theta grid of Sec. 6.4.1), n_b = 2 ** clip(round(o1), 5, 12);
    rounding half to even on both."""
    out = np.atleast_2d(np.asarray(out, np.float64))
    theta = np.round(np.clip(out[:, 0], 0.5, 0.9) * 10.0) / 10.0
    nb = 2 ** np.clip(np.round(out[:, 1]), 5, 12).astype(np.int64)
    return theta, nb


# ------------------------------------------------------------------ scorer
N_SCORES = GRID_TH * GRID_NB          # one output per grid point, theta outer
N_PARAMS_SCORER = sum(int(np.prod(s)) for s in shapes(N_SCORES))  # 30,248
SCORE_TEMP, SCORE_FLOOR = 0.1, 0.05   # loss weight exp(-g / SCORE_TEMP) + SCORE_FLOOR


def score_loss_and_grad(p, X, G):
    """Scorer loss on grids G[B][40] (the log time ratios, theta outer):
    L = sum_b sum_k w_bk (out_bk - G_bk)^2 / (40 B) with w = exp(-G / T) + F
    (T = SCORE_TEMP, F = SCORE_FLOOR: the near-best points weigh most, the
    rest enough to keep their order), and dL/dp by backpropagation."""
    out, cache = forward(p, X)
    B = cache[0].shape[0]
    G = np.asarray(G, np.float64).reshape(B, N_SCORES)
    w = np.exp(-G / SCORE_TEMP) + SCORE_FLOOR
    diff = out - G
    L = float(np.sum(w * diff * diff) / (N_SCORES * B))
    return L, backward(p, cache, 2.0 * w * diff / (N_SCORES * B))


def decode_scores(out):
    """Scorer outputs [B][40] -> (theta, n_b, ok): the grid point k of the
    smallest output (the first on ties), theta = 0.5 + 0.1 (k // 8), n_b =
    2^(5 + k % 8); rows with a non-finite output give ok = 0 and the policy
    point (0.6, 256)."""
    out = np.atleast_2d(np.asarray(out, np.float64))
    theta = np.full(out.shape[0], 0.6)
    nb = np.full(out.shape[0], 256, np.int64)
    ok = np.zeros(out.shape[0], np.int64)
    for r, row in enumerate(out):
        if not np.all(np.isfinite(row)):
            continue
        k = int(np.argmin(row))
        theta[r] = round(0.5 + 0.1 * (k // GRID_NB), 1)
        nb[r] = 2 ** (5 + k % GRID_NB)
        ok[r] = 1
    return theta, nb, ok
