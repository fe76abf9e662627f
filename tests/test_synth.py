"""Structure of the seeded synthetic inputs (no method arithmetic involved)."""
import numpy as np
import pytest

from paper_2105_04937_amd import synth


def _check_csr(m):
    assert m.rowptr[0] == 0 and m.rowptr[-1] == m.nnz
    assert np.all(np.diff(m.rowptr) >= 0)
    assert m.colind.min() >= 0 and m.colind.max() < m.n
    for i in range(0, m.n, max(1, m.n // 200)):
        c = m.colind[m.rowptr[i]:m.rowptr[i + 1]]
        assert np.all(np.diff(c) > 0)


def test_laplacian7_counts():
    N = 32
    m = synth.laplacian7(N)
    _check_csr(m)
    assert m.n == 32768 and m.nnz == 7 * N**3 - 6 * N**2 == 223_232


def test_heptadiagonal_values():
    m = synth.heptadiagonal(10, 2)
    _check_csr(m)
    rows = np.repeat(np.arange(m.n), np.diff(m.rowptr))
    diag = rows == m.colind
    off = m.val[~diag]
    assert np.all((off >= -1.0) & (off <= -0.5))
    rs = np.bincount(rows[~diag], weights=np.abs(off), minlength=m.n)
    assert np.allclose(m.val[diag], 1.01 * rs, rtol=1e-15)
    m2 = synth.heptadiagonal(10, 2)
    assert np.array_equal(m.val, m2.val)


def test_partially_diagonal_structure():
    N = 24
    m = synth.partially_diagonal(N, 3)
    _check_csr(m)
    rows = np.repeat(np.arange(m.n), np.diff(m.rowptr))
    # every row keeps its diagonal
    assert np.sum(rows == m.colind) == m.n
    # octant 0 drops nothing: interior rows of octant 0 hold 27 + 2 entries
    r = np.arange(m.n)
    ix, iy, iz = r % N, (r // N) % N, r // (N * N)
    inner0 = (ix > 0) & (ix < N // 2) & (iy > 0) & (iy < N // 2) & (iz > 0) & (iz < N // 2)
    assert np.all(np.diff(m.rowptr)[inner0] == 29)
    # octant 7 drops 90%: far fewer entries
    inner7 = (ix >= N // 2) & (ix < N - 1) & (iy >= N // 2) & (iy < N - 1) & (iz >= N // 2) & (iz < N - 1)
    assert np.diff(m.rowptr)[inner7].mean() < 1 + 2 + 26 * 0.2
    diag = rows == m.colind
    rs = np.abs(np.bincount(rows[~diag], weights=m.val[~diag], minlength=m.n))
    assert np.allclose(m.val[diag], 1.1 * rs, rtol=1e-14, atol=0)


def test_batch_member_ranges():
    for i in range(6):
        m, k = synth.batch_member(i)
        _check_csr(m)
        assert 16 <= m.meta["side"] <= 96 and m.meta["points"] in (7, 19, 27)
        assert 0.0 <= m.meta["p"] <= 0.3 and 1 <= k <= 16


def test_vector():
    x = synth.vector(1000, 1)
    assert x.shape == (1000,) and x.min() >= -1 and x.max() <= 1
    X = synth.vector(100, 1, k=4)
    assert X.shape == (100, 4) and X.flags.f_contiguous


def test_banded_offsets():
    """Sec. 6.3: n_x = floor(sqrt(n)) for 5 points, floor(cbrt(n)) for 7."""
    assert synth.banded_offsets(100, 3) == [-1, 0, 1]
    assert synth.banded_offsets(99, 5) == [-9, -1, 0, 1, 9]
    assert synth.banded_offsets(100, 5) == [-10, -1, 0, 1, 10]
    assert synth.banded_offsets(999, 7) == [-81, -9, -1, 0, 1, 9, 81]
    assert synth.banded_offsets(1000, 7) == [-100, -10, -1, 0, 1, 10, 100]
    assert synth.banded_offsets(50_000_000, 7)[-1] == 368 * 368
    assert synth.banded_offsets(3, 5) == [-1, 0, 1]  # n_x = 1 merges with +-1


@pytest.mark.parametrize("n,points", [(1, 3), (7, 7), (64, 5), (1000, 7), (1001, 3)])
def test_banded_stencil_structure(n, points):
    m = synth.banded_stencil(n, points, 5)
    offs = synth.banded_offsets(n, points)
    for i in range(n):
        cols = m.colind[m.rowptr[i]:m.rowptr[i + 1]]
        assert list(cols) == [i + o for o in offs if 0 <= i + o < n]
        v = m.val[m.rowptr[i]:m.rowptr[i + 1]]
        off = v[cols != i]
        assert np.all((off >= -1.0) & (off < -0.5))
        assert v[cols == i][0] == 1.01 * abs(off.sum())
    # the device generator builds the same structure
    import torch
    rp, ci, _ = synth.banded_stencil_gpu(n, points, 5, device="cpu")
    assert np.array_equal(rp.numpy(), m.rowptr) and np.array_equal(ci.numpy(), m.colind)
