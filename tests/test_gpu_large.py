"""Largest-size case: more than 2^31 DIA value slots (S = K * n_b), so every
slot index in the converter, the SpMV kernel and the unblocked HDC kernel
must be 64-bit.  The matrix is built on the device: tridiagonal (2 on the
diagonal, -1 beside it) on n = 2^28 rows, plus 8 far diagonals that hold a
single 1 per row block of n_b = 2^16 rows; with theta = 0 every block keeps
all 11 partial diagonals (Sec. 4.3), so S = 11 n > 2^31 while nnz stays
below 2^31.  With x_i = (i mod 7) - 3 every product and sum is a small
integer, so the exact y is a closed form: y_i = 2 x_i - x_(i-1) - x_(i+1)
(missing terms at the ends) plus x_(i+d) on the rows that carry a far
entry of offset d.  The check compares sampled rows (and whole first and
last blocks) bit for bit."""
import numpy as np
import pytest
import torch

from paper_2105_04937_amd import mhdc
from tests.gpu_helpers import say

pytestmark = pytest.mark.gpu

N = 1 << 28
NB = 1 << 16
FAR = (-30011, -20011, -5003, -1009, 1013, 5009, 20021, 30029)


def _far_row(ib, j):
    return ib * NB + (j * 997 + 13) % NB


def _build(dev):
    n_blk = N // NB
    i = torch.arange(N, dtype=torch.int64, device=dev)
    rows, cols, vals = [], [], []
    for off, v in ((-1, -1.0), (0, 2.0), (1, -1.0)):
        keep = (i + off >= 0) & (i + off < N)
        r = i[keep]
        rows.append(r)
        cols.append(r + off)
        vals.append(torch.full((r.numel(),), v, dtype=torch.float64, device=dev))
    ib = torch.arange(n_blk, dtype=torch.int64, device=dev)
    for j, d in enumerate(FAR):
        r = ib * NB + (j * 997 + 13) % NB
        keep = (r + d >= 0) & (r + d < N)
        rows.append(r[keep])
        cols.append(r[keep] + d)
        vals.append(torch.ones(int(keep.sum()), dtype=torch.float64, device=dev))
    del i
    row = torch.cat(rows)
    col = torch.cat(cols)
    val = torch.cat(vals)
    del rows, cols, vals
    key = row * N + col
    del row
    order = torch.argsort(key)
    key = key[order]
    val = val[order]
    del order, col
    r_sorted = key // N
    colind = (key - r_sorted * N).to(torch.int32)
    del key
    counts = torch.bincount(r_sorted, minlength=N)
    del r_sorted
    rowptr = torch.zeros(N + 1, dtype=torch.int64, device=dev)
    rowptr[1:] = torch.cumsum(counts, 0)
    del counts
    return rowptr.to(torch.int32), colind, val


def _expected(rows, xh):
    """Closed form of y on the given rows (x_i = (i mod 7) - 3)."""
    def x(i):
        return float(i % 7 - 3)
    out = np.empty(len(rows))
    far_of = {}
    for j, d in enumerate(FAR):
        far_of[j] = d
    for t, i in enumerate(rows):
        s = 2.0 * x(i)
        if i > 0:
            s -= x(i - 1)
        if i + 1 < N:
            s -= x(i + 1)
        ib = i // NB
        for j, d in far_of.items():
            if _far_row(ib, j) == i and 0 <= i + d < N:
                s += x(i + d)
        out[t] = s
    return out


def _sample_rows():
    rng = np.random.default_rng(1)
    return np.unique(np.concatenate([
        np.arange(0, NB + 5), np.arange(N - NB - 5, N),
        rng.integers(0, N, 20000),
        np.array([_far_row(ib, j) for ib in rng.integers(0, N // NB, 64) for j in range(8)])]))


def _check(y, sample, want, name):
    got = y[torch.from_numpy(sample).to(y.device)].cpu().numpy()
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, "%s rows %s: got %s want %s" % (name, sample[bad[:5]], got[bad[:5]],
                                                          want[bad[:5]])


def test_more_than_2_31_dia_slots():
    dev = torch.device("cuda")
    say("case: large n=%d n_b=%d (S > 2^31)" % (N, NB))
    rp, ci, v = _build(dev)
    nnz = ci.numel()
    assert nnz < 2**31 - 1
    x = (torch.arange(N, dtype=torch.int64, device=dev) % 7 - 3).to(torch.float64)
    sample = _sample_rows()
    want = _expected(sample.tolist(), None)
    h = mhdc.MHDCMatrix.from_csr(rp, ci, v, NB, 0.0)
    inf = h.info()
    say("large M-HDC: K=%d S=%d R=%d nnz=%d" % (inf["K"], inf["S"], inf["R"], nnz))
    assert inf["R"] == 0 and inf["S"] == inf["K"] * NB and inf["S"] > 2**31
    _check(h.spmv(x), sample, want, "M-HDC")
    h.close()
    torch.cuda.empty_cache()
    say("case: large HDC theta=0 (global DIA, S > 2^31)")
    hd = mhdc.HDCMatrix.from_csr(rp, ci, v, 0.0)
    inf = hd.info()
    assert inf["K"] == 11 and inf["R"] == 0 and inf["S"] == 11 * N
    _check(hd.spmv(x), sample, want, "HDC blocked")
    _check(hd.spmv_unblocked(x), sample, want, "HDC unblocked")
    hd.close()
    del rp, ci, v, x
    torch.cuda.empty_cache()
