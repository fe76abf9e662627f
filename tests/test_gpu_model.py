"""The byte model across the boundary: every handle kind reports the
algorithmic bytes, the paper's volume V (Eqs. 24/34), alpha and beta (Eqs.
23/33) and the estimated relative performance over CSR (Eq. 28) that the
oracle's model computes from the oracle converter's layout of the same
matrix -- on the Example matrix, on random matrices whose remainder sits in
a few row groups or in all of them, and on ragged and empty cases.  The
full-size cases are in test_gpu_full."""
import numpy as np
import pytest

import oracle
from paper_2105_04937_amd import mhdc, synth
from tests.gpu_helpers import check_byte_model, dev, say
from tests.test_gpu_small import _example_csr

pytestmark = pytest.mark.gpu


def _sparse_remainder(n, rows, seed):
    """A banded matrix (offsets 0, +-1, +-7) plus one random entry in each of
    the given rows: the remainder touches only a few 64-row groups."""
    rng = np.random.default_rng(seed)
    A = {}
    for i in range(n):
        for d in (-7, -1, 0, 1, 7):
            if 0 <= i + d < n:
                A[(i, i + d)] = float(rng.integers(1, 9))
    for i in rows:
        j = int(rng.integers(0, n))
        while (i, j) in A:
            j = int(rng.integers(0, n))
        A[(i, j)] = 3.0
    keys = sorted(A)
    r = np.array([k[0] for k in keys], np.int64)
    rp = np.zeros(n + 1, np.int32)
    np.cumsum(np.bincount(r, minlength=n), out=rp[1:])
    return synth.CSRMatrix(n, rp, np.array([k[1] for k in keys], np.int32),
                           np.array([A[k] for k in keys]), meta=dict(seed=seed))


def _model_cases():
    return [
        _example_csr(),
        _sparse_remainder(5000, [3, 2000, 4999], 11),
        synth.random_csr(3000, 12, density=0.002, bands=[0, 1, -1, 40], band_fill=0.9),
        synth.random_csr(257, 13, density=0.05, bands=[0, 2, -5], zero_frac=0.2),
        synth.random_csr(1, 14, density=1.0),
        synth.random_csr(10, 15, density=0.0),
    ]


@pytest.mark.parametrize("m", _model_cases(), ids=lambda m: "n%d_s%d" % (m.n, m.meta["seed"]))
def test_byte_model_matches_oracle(m):
    say("case: byte model n=%d seed=%d nnz=%d" % (m.n, m.meta["seed"], m.nnz))
    d = dev(m)
    for bl in (1, 4, 64, 100, 4096):
        for theta in (0.0, 0.5, 0.6, 1.0):
            h = mhdc.MHDCMatrix.from_csr(*d, bl, theta)
            check_byte_model(h, m, oracle.mhdc_from_csr(m.rowptr, m.colind, m.val, bl, theta))
            h.close()
    for theta in (0.0, 0.6, 1.0):
        hd = mhdc.HDCMatrix.from_csr(*d, theta)
        check_byte_model(hd, m, oracle.hdc_from_csr(m.rowptr, m.colind, m.val, theta))
        hd.close()
    cs = mhdc.CSRMatrix.from_csr(*d)
    inf = check_byte_model(cs, m)
    assert inf["rp_est"] == 1.0
    cs.close()


def test_byte_model_example_values():
    """Fig. 15 / Fig. 7 / Fig. 2 layouts of the Example matrix, counted by
    hand: B_alg 392 / 384 / 404 bytes, V 356 / 372 / 400 bytes."""
    m = _example_csr()
    d = dev(m)
    h = mhdc.MHDCMatrix.from_csr(*d, 4, 0.6)
    hd = mhdc.HDCMatrix.from_csr(*d, 0.6)
    cs = mhdc.CSRMatrix.from_csr(*d)
    got = [(x.info()["bytes_alg"], x.info()["bytes_paper"]) for x in (h, hd, cs)]
    assert got == [(392.0, 356.0), (384.0, 372.0), (404.0, 400.0)]
    for x in (h, hd, cs):
        x.close()
