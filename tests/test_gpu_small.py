"""GPU parity on small inputs: the paper's worked example, brute-force random
matrices with ragged blocks, degenerate shapes, every launch shape, several
right-hand sides, error paths.  Every call goes through the C-ABI."""
import numpy as np
import pytest
import torch

import oracle
from paper_2105_04937_amd import mhdc, synth
from tests.conftest import load_golden
from tests.gpu_helpers import (assert_oracle_bits, assert_same_bits, assert_spmv_close,
                               check_hdc_arrays, check_mhdc_arrays, check_round_trip, dev, say)

pytestmark = pytest.mark.gpu

THETAS = [0.0, 0.5, 0.6, 2.0 / 3.0, 0.75, 1.0]
SHAPES = [(1, 64, 0), (1, 64, 1), (2, 64, 1), (4, 64, 1), (1, 256, 1), (2, 256, 0),
          (2, 256, 1), (4, 256, 1), (1, 256, 0, 2), (2, 256, 0, 2), (1, 64, 0, 2, 0),
          (2, 256, 0, 1, 0), (1, 64, 4), (2, 64, 2), (1, 64, 16), (1, 256, 8, 2, 0),
          (1, 64, 3), (1, 64, 9)]


def _example_csr():
    rows = np.array(load_golden("example_matrix.txt")["row"], dtype=np.float64)
    m = synth.CSRMatrix(8, *(lambda r, c: (
        np.concatenate([[0], np.cumsum(np.bincount(r, minlength=8))]).astype(np.int32),
        c.astype(np.int32), rows[r, c]))(*np.nonzero(rows)), meta=dict(seed=0))
    return m


def test_example_matrix_mhdc_hdc_csr():
    say("case: Example matrix, bl=4 theta=0.6")
    m = _example_csr()
    rp, ci, v = dev(m)
    g = load_golden("example_products.txt")
    h = mhdc.MHDCMatrix.from_csr(rp, ci, v, 4, 0.6)
    check_mhdc_arrays(h, oracle.mhdc_from_csr(m.rowptr, m.colind, m.val, 4, 0.6))
    f15 = load_golden("example_mhdc_bl4_theta0.6.txt")
    t = h.export()
    assert t["dia_off"].cpu().tolist() == [int(a) for a in f15["dia_col_offset"][0]]
    hd = mhdc.HDCMatrix.from_csr(rp, ci, v, 0.6)
    check_hdc_arrays(hd, oracle.hdc_from_csr(m.rowptr, m.colind, m.val, 0.6))
    cs = mhdc.CSRMatrix.from_csr(rp, ci, v)
    for x, y in zip(g["x"], g["y"]):
        xd = torch.tensor(x, dtype=torch.float64, device="cuda")
        for mat in (h, hd, cs):
            got = mat.spmv(xd).cpu().numpy()
            assert np.array_equal(got, np.array(y)), (mat, got)
    check_round_trip(h, m)


def _cases():
    out = []
    for s, n in enumerate([1, 2, 5, 8, 17, 33, 64, 100, 257]):
        bands = [0, 1, -1, 3, -(n // 2)] if n > 2 else [0]
        out.append(synth.random_csr(n, 100 + s, density=min(0.08, 8.0 / n), bands=bands,
                                    int_values=True))
        out.append(synth.random_csr(n, 200 + s, density=min(0.3, 16.0 / n)))
    out.append(synth.random_csr(40, 300, density=0.05, bands=[0, 2, -5], zero_frac=0.2,
                                int_values=True))
    out.append(synth.random_csr(10, 301, density=0.0))  # no stored entries
    out.append(synth.random_csr(700, 302, density=0.004, bands=[0, 1, -1, 30, -30, 300],
                                band_fill=0.8))
    return out


@pytest.mark.parametrize("m", _cases(), ids=lambda m: "n%d_s%d" % (m.n, m.meta["seed"]))
def test_random_conversion_and_spmv(m):
    say("case: random n=%d seed=%d nnz=%d" % (m.n, m.meta["seed"], m.nnz))
    rp, ci, v = dev(m)
    x = synth.vector(m.n, 3)
    xd = torch.from_numpy(x).cuda()
    yref = oracle.csr_spmv(m.rowptr, m.colind, m.val, x)
    for bl in (1, 3, 4, 32, 64, 128, 1000):
        for theta in THETAS:
            ref = oracle.mhdc_from_csr(m.rowptr, m.colind, m.val, bl, theta)
            h = mhdc.MHDCMatrix.from_csr(rp, ci, v, bl, theta)
            check_mhdc_arrays(h, ref)
            check_round_trip(h, m)
            y = h.spmv(xd)
            assert_spmv_close(y, m, x, Y_ref=yref)
            assert_oracle_bits(y, oracle.mhdc_spmv(ref, x), "mhdc bl=%d theta=%g" % (bl, theta))
            h.close()
    for theta in THETAS:
        ref = oracle.hdc_from_csr(m.rowptr, m.colind, m.val, theta)
        hd = mhdc.HDCMatrix.from_csr(rp, ci, v, theta)
        check_hdc_arrays(hd, ref)
        y = hd.spmv(xd)
        assert_spmv_close(y, m, x, Y_ref=yref)
        assert_oracle_bits(y, oracle.hdc_spmv(ref, x), "hdc theta=%g" % theta)
    cs = mhdc.CSRMatrix.from_csr(rp, ci, v)
    y = cs.spmv(xd)
    assert_oracle_bits(y, yref, "csr")
    if np.all(m.val == np.round(m.val)):
        xi = np.arange(m.n, dtype=np.float64) - 5.0
        want = oracle.csr_spmv(m.rowptr, m.colind, m.val, xi)
        xid = torch.from_numpy(xi).cuda()
        for mat in (mhdc.MHDCMatrix.from_csr(rp, ci, v, 4, 0.5), cs,
                    mhdc.HDCMatrix.from_csr(rp, ci, v, 0.5)):
            assert np.array_equal(mat.spmv(xid).cpu().numpy(), want)
    del y


def test_launch_shapes_give_identical_bits():
    """Each row sums its remainder entries in column order and then its
    diagonals in offset order whatever the launch shape, so every shape
    returns the same bits."""
    m = synth.partially_diagonal(20, 11, drop=synth.OCTANT_DROP)
    say("case: launch shapes, n=%d nnz=%d" % (m.n, m.nnz))
    rp, ci, v = dev(m)
    x = synth.vector(m.n, 4)
    xd = torch.from_numpy(x).cuda()
    for bl, theta in ((20, 0.6), (64, 0.6), (128, 0.5), (256, 0.9), (48, 0.6)):
        h = mhdc.MHDCMatrix.from_csr(rp, ci, v, bl, theta)
        want = oracle.mhdc_spmv(oracle.mhdc_from_csr(m.rowptr, m.colind, m.val, bl, theta), x)
        first = None
        for shp in SHAPES:
            h.set_launch(*shp)
            y = h.spmv(xd).cpu().numpy()
            if first is None:
                first = y
                assert_spmv_close(y, m, x)
            assert_same_bits(y, first, "shape %s bl %d" % (shp, bl))
            assert_oracle_bits(y, want, "shape %s bl %d" % (shp, bl))
            assert_same_bits(h.spmv(xd).cpu().numpy(), first, "repeat")
    cs = mhdc.CSRMatrix.from_csr(rp, ci, v)
    first = None
    for shp in SHAPES:
        cs.set_launch(*shp)
        y = cs.spmv(xd).cpu().numpy()
        first = y if first is None else first
        assert_same_bits(y, first, "csr shape %s" % (shp,))


def test_hdc_unblocked_matches_blocked():
    """The unblocked HDC kernel (Fig. 8; Fig. 5 for a pure DIA matrix) adds
    the same rounded products in the same order per row as the blocked
    kernel: bit-identical to hdc_spmv and to the oracle's Fig. 8 kernel, on
    random matrices with a CSR part and on the banded stencils of Sec. 6.3
    (with ragged sizes and n_x = 1)."""
    cases = [(synth.random_csr(300, 5, density=0.05, bands=(-7, 0, 3), zero_frac=0.05), t)
             for t in (0.0, 0.5, 0.9)]
    cases += [(synth.banded_stencil(n, p, 2), 0.0) for n, p in
              ((1, 3), (5, 5), (7, 7), (1000, 3), (4097, 5), (100_001, 7))]
    cases.append((synth.partially_diagonal(14, 4, drop=0.3), 0.6))
    for m, theta in cases:
        say("case: unblocked HDC n=%d theta=%g" % (m.n, theta))
        rp, ci, v = dev(m)
        x = synth.vector(m.n, 9)
        xd = torch.from_numpy(x).cuda()
        h = mhdc.HDCMatrix.from_csr(rp, ci, v, theta)
        want = oracle.hdc_spmv(oracle.hdc_from_csr(m.rowptr, m.colind, m.val, theta), x)
        for shp in ((1, 64, 0), (2, 256, 1), (1, 256, 0, 2)):
            h.set_launch(*shp)
            yb = h.spmv(xd).cpu().numpy()
            yu = h.spmv_unblocked(xd).cpu().numpy()
            assert_same_bits(yu, yb, "unblocked vs blocked n=%d shape %s" % (m.n, shp))
            assert_oracle_bits(yu, want, "unblocked vs oracle n=%d" % m.n)
        h.close()
    assert mhdc.lib().hdc_spmv_unblocked(None, None, None, None) == -1  # MHDC_ERR_INVALID_ARG


@pytest.mark.parametrize("k", [1, 2, 3, 5, 8, 11, 16])
def test_multi_rhs(k):
    m = synth.partially_diagonal(14, 21, drop=0.2)
    say("case: spmm k=%d n=%d" % (k, m.n))
    rp, ci, v = dev(m)
    X = np.ascontiguousarray(np.random.default_rng(k).uniform(-1, 1, size=(k, m.n)))
    Xd = torch.from_numpy(X).cuda()
    Yref = oracle.csr_spmm(m.rowptr, m.colind, m.val, np.asfortranarray(X.T))
    mats = [mhdc.MHDCMatrix.from_csr(rp, ci, v, 64, 0.6), mhdc.MHDCMatrix.from_csr(rp, ci, v, 14, 0.6),
            mhdc.HDCMatrix.from_csr(rp, ci, v, 0.6), mhdc.CSRMatrix.from_csr(rp, ci, v)]
    refs = [oracle.mhdc_from_csr(m.rowptr, m.colind, m.val, 64, 0.6),
            oracle.mhdc_from_csr(m.rowptr, m.colind, m.val, 14, 0.6),
            oracle.hdc_from_csr(m.rowptr, m.colind, m.val, 0.6), None]
    for mat, ref in zip(mats, refs):
        for shp in ((1, 64, 1), (2, 256, 1), (4, 256, 0), (1, 256, 0, 1, 0), (1, 256, 0, 2, 0),
                    (1, 256, 0, 0, 4), (2, 256, 0, 2, 2), (1, 64, 0, 1, 1)):
            mat.set_launch(*shp)
            Y = mat.spmm(Xd).cpu().numpy()
            for r in range(k):
                assert_spmv_close(Y[r], m, X[r], Y_ref=Yref[:, r])
                # one right-hand side alone gives the same bits
                y1 = mat.spmv(Xd[r].contiguous()).cpu().numpy()
                assert_same_bits(Y[r], y1, "rhs %d" % r)
                if ref is None:
                    want = Yref[:, r]
                elif ref.n_blk == 1 and ref.bl == m.n and isinstance(mat, mhdc.HDCMatrix):
                    want = oracle.hdc_spmv(ref, X[r])
                else:
                    want = oracle.mhdc_spmv(ref, X[r])
                assert_oracle_bits(Y[r], want, "rhs %d" % r)


def test_spmm_padded_leading_dimensions():
    """mhdc_spmm / hdc_spmm / csr_spmm with ldx, ldy > n through the C-ABI:
    every column equals its own spmv bit for bit, the padding rows of Y
    keep their sentinel, and ldx < n is refused."""
    m = synth.partially_diagonal(12, 8, drop=0.1)
    rp, ci, v = dev(m)
    n, k = m.n, 5
    ldx, ldy = n + 5, n + 3
    X = torch.from_numpy(np.random.default_rng(3).uniform(-1, 1, size=(k, ldx))).cuda()
    L = mhdc.lib()
    s = torch.cuda.current_stream()
    for make, fn in ((lambda: mhdc.MHDCMatrix.from_csr(rp, ci, v, 32, 0.6), L.mhdc_spmm),
                     (lambda: mhdc.HDCMatrix.from_csr(rp, ci, v, 0.6), L.hdc_spmm),
                     (lambda: mhdc.CSRMatrix.from_csr(rp, ci, v), L.csr_spmm)):
        h = make()
        say("case: padded ld %s" % type(h).__name__)
        Y = torch.full((k, ldy), 7.25, dtype=torch.float64, device="cuda")
        assert fn(h._h, X.data_ptr(), ldx, Y.data_ptr(), ldy, k, s.cuda_stream) == 0
        torch.cuda.synchronize()
        Yh = Y.cpu().numpy()
        for r in range(k):
            y1 = h.spmv(X[r, :n].contiguous()).cpu().numpy()
            assert_same_bits(Yh[r, :n], y1, "column %d" % r)
            assert np.all(Yh[r, n:] == 7.25)
        assert mhdc.ERRORS[fn(h._h, X.data_ptr(), n - 1, Y.data_ptr(), ldy, k,
                              s.cuda_stream)] == "MHDC_ERR_INVALID_ARG"
        h.close()


def test_degenerate_shapes():
    say("case: degenerate shapes")
    # n = 0
    rp = torch.zeros(1, dtype=torch.int32, device="cuda")
    ci = torch.zeros(0, dtype=torch.int32, device="cuda")
    v = torch.zeros(0, dtype=torch.float64, device="cuda")
    for mat in (mhdc.MHDCMatrix.from_csr(rp, ci, v, 4, 0.6), mhdc.HDCMatrix.from_csr(rp, ci, v, 0.6),
                mhdc.CSRMatrix.from_csr(rp, ci, v)):
        y = mat.spmv(torch.zeros(0, dtype=torch.float64, device="cuda"))
        assert y.numel() == 0
    # n = 1 with one entry; a matrix of empty rows; n_b = 1 and n_b >= n
    for m in (synth.random_csr(1, 5, density=1.0), synth.random_csr(50, 6, density=0.0),
              synth.random_csr(3, 7, density=1.0)):
        rp, ci, v = dev(m)
        x = synth.vector(m.n, 1)
        xd = torch.from_numpy(x).cuda()
        for bl in (1, 2, m.n, 10 * m.n + 3):
            h = mhdc.MHDCMatrix.from_csr(rp, ci, v, bl, 0.6)
            check_mhdc_arrays(h, oracle.mhdc_from_csr(m.rowptr, m.colind, m.val, bl, 0.6))
            assert_spmv_close(h.spmv(xd), m, x)


def test_signed_zero_nan_round_trip():
    m = synth.random_csr(90, 8, density=0.02, bands=[0, 1, -2, 7], band_fill=1.0)
    v = m.val.copy()
    v[::7] = -0.0
    v[3] = np.inf
    v[5] = -np.inf
    v[11] = np.nan
    m = synth.CSRMatrix(m.n, m.rowptr, m.colind, v, m.meta)
    say("case: signed zero / NaN round trip")
    rp, ci, vd = dev(m)
    for bl in (4, 32, 90):
        h = mhdc.MHDCMatrix.from_csr(rp, ci, vd, bl, 0.5)
        check_mhdc_arrays(h, oracle.mhdc_from_csr(m.rowptr, m.colind, m.val, bl, 0.5))
        check_round_trip(h, m)


def test_error_paths():
    say("case: error paths")
    m = synth.random_csr(20, 9, density=0.2, bands=[0])
    rp, ci, v = dev(m)
    with pytest.raises(mhdc.MhdcError) as e:
        mhdc.MHDCMatrix.from_csr(rp, ci, v, 0, 0.6)
    assert e.value.name == "MHDC_ERR_INVALID_ARG"
    for th in (float("nan"), -0.1, 1.5):
        with pytest.raises(mhdc.MhdcError) as e:
            mhdc.MHDCMatrix.from_csr(rp, ci, v, 4, th)
        assert e.value.name == "MHDC_ERR_INVALID_ARG"
    # unsorted / duplicate / out-of-range columns, broken rowptr
    bad = []
    c2 = m.colind.copy()
    r = int(np.argmax(np.diff(m.rowptr) >= 2))
    a = m.rowptr[r]
    c2[a], c2[a + 1] = c2[a + 1], c2[a]
    bad.append((m.rowptr, c2))
    c3 = m.colind.copy()
    c3[a + 1] = c3[a]
    bad.append((m.rowptr, c3))
    c4 = m.colind.copy()
    c4[0] = m.n
    bad.append((m.rowptr, c4))
    p5 = m.rowptr.copy()
    p5[3] = p5[4] + 1
    bad.append((p5, m.colind))
    p6 = m.rowptr.copy()
    p6[0] = 1
    bad.append((p6, m.colind))
    for p, c in bad:
        pd, cd = torch.from_numpy(p).cuda(), torch.from_numpy(c).cuda()
        for make in (lambda: mhdc.MHDCMatrix.from_csr(pd, cd, v, 4, 0.6),
                     lambda: mhdc.HDCMatrix.from_csr(pd, cd, v, 0.6),
                     lambda: mhdc.CSRMatrix.from_csr(pd, cd, v)):
            with pytest.raises(mhdc.MhdcError) as e:
                make()
            assert e.value.name == "MHDC_ERR_BAD_CSR"
    # nnz above 2^31 - 4097 is refused from rowptr[n] alone, before any
    # kernel reads colind or val
    for make in (lambda p: mhdc.MHDCMatrix.from_csr(p, ci, v, 4, 0.6),
                 lambda p: mhdc.HDCMatrix.from_csr(p, ci, v, 0.6),
                 lambda p: mhdc.CSRMatrix.from_csr(p, ci, v)):
        for last in (2**31 - 4096, 2**31 - 1):
            pbig = torch.tensor([0, 0, last], dtype=torch.int32, device="cuda")
            with pytest.raises(mhdc.MhdcError) as e:
                make(pbig)
            assert e.value.name == "MHDC_ERR_SIZE"
    h = mhdc.MHDCMatrix.from_csr(rp, ci, v, 4, 0.6)
    buf = torch.zeros(2 * m.n, dtype=torch.float64, device="cuda")
    with pytest.raises(mhdc.MhdcError) as e:
        h.spmv(buf[:m.n], buf[m.n // 2: m.n // 2 + m.n])  # overlapping x and y
    assert e.value.name == "MHDC_ERR_INVALID_ARG"
    X = torch.zeros((17, m.n), dtype=torch.float64, device="cuda")
    with pytest.raises(mhdc.MhdcError):
        h.spmm(X)
    with pytest.raises(mhdc.MhdcError) as e:
        h.set_launch(3, 256, 1)
    assert e.value.name == "MHDC_ERR_NOT_SUPPORTED"
    for remap in (65, 128, -1):
        with pytest.raises(mhdc.MhdcError) as e:
            h.set_launch(1, 256, remap)
        assert e.value.name == "MHDC_ERR_NOT_SUPPORTED"
    # outputs of the wrong size are refused by the binding before any launch
    x = torch.zeros(m.n, dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        h.spmv(x, torch.zeros(m.n - 1, dtype=torch.float64, device="cuda"))
    with pytest.raises(ValueError):
        h.spmm(torch.zeros((2, m.n), dtype=torch.float64, device="cuda"),
               torch.zeros((2, m.n - 1), dtype=torch.float64, device="cuda"))
    with pytest.raises(ValueError):
        mhdc.stream_direct(x, x[:-1], torch.zeros_like(x))


def _row_repeat(ptr, col):
    """Share of the nonempty rows whose column offsets repeat the previous
    row's, counted row by row on the host."""
    ptr = np.asarray(ptr, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    nonempty = rep = 0
    for i in range(len(ptr) - 1):
        a, b = ptr[i], ptr[i + 1]
        if a == b:
            continue
        nonempty += 1
        if i > 0:
            p = ptr[i - 1]
            if a - p == b - a and np.array_equal(col[a:b] - i, col[p:a] - (i - 1)):
                rep += 1
    return rep / nonempty if nonempty else 0.0


def test_row_repeat_picks_csr_mode():
    """row_repeat of the CSR part equals the host count, and the default
    launch of a handle without DIA part stages values and columns
    (csr_mode 2) exactly when at least half the nonempty rows repeat;
    results are the same bits either way."""
    cases = [("7-point 12^3", synth.heptadiagonal(12, 1), True),
             ("27-point 10^3 octant drops", synth.partially_diagonal(10, 2, drop=synth.OCTANT_DROP),
              False),
             ("random 300", synth.random_csr(300, 5, density=0.02), False),
             ("banded 3-point", synth.banded_stencil(4000, 3, 1), True)]
    for name, m, regular in cases:
        say("case: row repeat %s" % name)
        rp, ci, v = dev(m)
        want = _row_repeat(m.rowptr, m.colind)
        assert (want >= 0.5) == regular, (name, want)
        cs = mhdc.CSRMatrix.from_csr(rp, ci, v)
        inf = cs.info()
        assert inf["row_repeat"] == want, (name, inf["row_repeat"], want)
        assert inf["csr_mode"] == (2 if inf["rows_per_lane"] == 1 and regular else 0)
        x = synth.vector(m.n, 7)
        xd = torch.from_numpy(x).cuda()
        y_def = cs.spmv(xd).cpu().numpy()
        cs.set_launch(inf["rows_per_lane"], inf["wg_size"], inf["xcd_remap"], 1, 0)
        assert_same_bits(cs.spmv(xd).cpu().numpy(), y_def, name)
        cs.close()
        h = mhdc.MHDCMatrix.from_csr(rp, ci, v, 64, 0.6)
        t = h.export()
        want_r = _row_repeat(t["rem_ptr"].cpu().numpy(), t["rem_col"].cpu().numpy())
        inf = h.info()
        assert inf["row_repeat"] == want_r, (name, inf["row_repeat"], want_r)
        if inf["R"] == 0:
            assert inf["row_repeat"] == 0.0
        # next to a DIA part the remainder keeps the staged products
        assert inf["csr_mode"] == (2 if inf["rows_per_lane"] == 1 and want_r >= 0.5
                                   and inf["K"] == 0 else 0)
        h.close()


def _xcd_run_share(D, T, c):
    """Share of the x rows a T-row tile reads through a diagonal D rows away
    that lie in tiles on the tile's own XCD, with runs of c tiles per XCD
    (tile u on XCD (u // c) % 8), over one round of 8c tiles: brute force."""
    same = 0
    for t in range(8 * c):
        for row in range(t * T, t * T + T):
            same += (row + D) // T // c % 8 == t // c % 8
    return same / (8 * c * T)


def test_default_xcd_runs_follow_the_farthest_diagonal():
    """The default launch of a large handle takes the run length in [8, 16]
    whose XCD keeps the most of the x rows its farthest kept diagonal reads
    (ties to the longer run; 16 without a DIA part).  7-point 128^3: the
    +-N^2 diagonals are 64 tiles away, one round of runs of 8.  The default
    launch gives the oracle's bits."""
    m = synth.heptadiagonal(128, 5)
    say("case: XCD runs, 7-point 128^3 n=%d" % m.n)
    shares = {c: _xcd_run_share(128 * 128, 256, c) for c in range(8, 17)}
    want = max(range(16, 7, -1), key=lambda c: (shares[c], c))
    assert want == 8 and shares[8] == 1.0 and shares[16] == 0.0
    rp, ci, v = dev(m)
    x = synth.vector(m.n, 9)
    xd = torch.from_numpy(x).cuda()
    h = mhdc.MHDCMatrix.from_csr(rp, ci, v, 256, 0.6)
    assert h.info()["xcd_remap"] == want
    ref = oracle.mhdc_from_csr(m.rowptr, m.colind, m.val, 256, 0.6)
    assert_oracle_bits(h.spmv(xd), oracle.mhdc_spmv(ref, x), "M-HDC, runs of 8")
    hd = mhdc.HDCMatrix.from_csr(rp, ci, v, 0.6)
    assert hd.info()["xcd_remap"] == want
    cs = mhdc.CSRMatrix.from_csr(rp, ci, v)
    assert cs.info()["xcd_remap"] == 16  # no DIA part
    for mat in (h, hd, cs):
        mat.close()


def test_conversion_and_spmv_are_deterministic():
    """Two conversions of the same matrix give the same arrays byte for byte,
    and two products the same bits, whatever order the census atomics took:
    blocks small enough for the LDS hash (n_b = 32) and large enough for the
    global table (n_b = 4096, ~90k entries per block), HDC and CSR."""
    m = synth.partially_diagonal(24, 5, drop=synth.OCTANT_DROP)
    rp, ci, v = dev(m)
    x = torch.from_numpy(synth.vector(m.n, 5)).cuda()
    for nb in (32, 4096):
        say("case: determinism n_b=%d" % nb)
        runs = []
        for _ in range(2):
            h = mhdc.MHDCMatrix.from_csr(rp, ci, v, nb, 0.6)
            t = {k: a.cpu().numpy() for k, a in h.export().items()}
            t["y"] = h.spmv(x).cpu().numpy()
            h.close()
            runs.append(t)
        for k in runs[0]:
            assert_same_bits(runs[1][k], runs[0][k], "n_b=%d %s" % (nb, k))
    for make in (lambda: mhdc.HDCMatrix.from_csr(rp, ci, v, 0.6),
                 lambda: mhdc.CSRMatrix.from_csr(rp, ci, v)):
        ys = []
        for _ in range(2):
            h = make()
            ys.append(h.spmv(x).cpu().numpy())
            h.close()
        assert_same_bits(ys[1], ys[0], "HDC/CSR product")


def test_census_table_overflow_to_global():
    """Blocks whose distinct offsets do not fit the 8192-slot LDS table
    (4096-row blocks of a matrix with 40 random columns per row; HDC chunks
    of 10k entries) are counted again in their global table region: the
    arrays still equal the oracle's byte for byte, and so do blocks of the
    same matrix that fit (n_b = 64)."""
    m = synth.random_csr(20000, 77, density=0.002, bands=[0, 1, -1])
    say("case: census overflow n=%d nnz=%d" % (m.n, m.nnz))
    rp, ci, v = dev(m)
    for nb, th in ((4096, 0.005), (64, 0.05)):
        h = mhdc.MHDCMatrix.from_csr(rp, ci, v, nb, th)
        check_mhdc_arrays(h, oracle.mhdc_from_csr(m.rowptr, m.colind, m.val, nb, th))
        h.close()
    hd = mhdc.HDCMatrix.from_csr(rp, ci, v, 0.01)
    check_hdc_arrays(hd, oracle.hdc_from_csr(m.rowptr, m.colind, m.val, 0.01))
    x = synth.vector(m.n, 4)
    assert_spmv_close(hd.spmv(torch.from_numpy(x).cuda()).cpu().numpy(), m, x)
    hd.close()


def test_concurrent_streams_share_a_handle():
    """A handle is read-only after conversion: products on two streams at
    once (default priority, different x and y) give the bits of the same
    products run one after the other."""
    m = synth.partially_diagonal(20, 6, drop=synth.OCTANT_DROP)
    rp, ci, v = dev(m)
    say("case: two streams, one handle n=%d" % m.n)
    h = mhdc.MHDCMatrix.from_csr(rp, ci, v, 64, 0.6)
    xs = [torch.from_numpy(synth.vector(m.n, 30 + i)).cuda() for i in range(2)]
    want = [h.spmv(x).cpu().numpy() for x in xs]
    ys = [torch.empty(m.n, dtype=torch.float64, device="cuda") for _ in range(2)]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    torch.cuda.synchronize()
    for _ in range(20):
        for x, y, st in zip(xs, ys, streams):
            h.spmv(x, y, stream=st)
    torch.cuda.synchronize()
    for i in range(2):
        assert_same_bits(ys[i].cpu().numpy(), want[i], "stream %d" % i)
    h.close()


def test_allocation_failure_leaks_nothing():
    """Fail the k-th device allocation of a conversion, a batch (both
    layouts) and a selection for every k: each attempt reports MHDC_ERR_OOM
    and returns all memory it took."""
    m = synth.partially_diagonal(12, 13)
    say("case: injected allocation failures")
    rp, ci, v = dev(m)
    L = mhdc.lib()
    h0 = mhdc.MHDCMatrix.from_csr(rp, ci, v, 32, 0.6)
    Xc = [torch.rand((3, m.n), dtype=torch.float64, device="cuda") for _ in range(2)]
    Yc = [torch.empty_like(X) for X in Xc]
    Xr = torch.rand((m.n, 3), dtype=torch.float64, device="cuda")
    Yr = torch.empty_like(Xr)
    from oracle import selector as S
    net = mhdc.MLP(S.init_params(1))
    makers = (lambda: mhdc.MHDCMatrix.from_csr(rp, ci, v, 32, 0.6),
              lambda: mhdc.HDCMatrix.from_csr(rp, ci, v, 0.6),
              lambda: mhdc.CSRMatrix.from_csr(rp, ci, v),
              lambda: mhdc.Batch([h0, h0], Xc, Ys=Yc),
              lambda: mhdc.Batch([h0], [Xr], Ys=[Yr], layout="rowmajor"),
              lambda: mhdc.select(rp, ci, v, model=net)[0])
    # one successful run of each first: the runtime loads a kernel's code
    # object on its first launch and keeps it, which is no leak
    for make in makers:
        make().close()
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for make in makers:
        k = 1
        while True:
            L.mhdc_debug_fail_alloc(k)
            try:
                h = make()
            except mhdc.MhdcError as e:
                assert e.name == "MHDC_ERR_OOM"
                k += 1
                continue
            finally:
                L.mhdc_debug_fail_alloc(0)
            h.close()
            break
        assert k >= 2
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] >= free0 - (4 << 20)
    net.close()
    h0.close()


@pytest.mark.parametrize("N,shift", [(100_003, 0), (100_000, 0), (1, 0), (2, 0), (4097, 1)])
def test_memory_benchmark_kernels(N, shift):
    """Sec. 6.2 kernels, bit-exact against the sequential loops; odd N and a
    view shifted by one element (8-byte aligned only) take the scalar path."""
    say("case: memory benchmark kernels N=%d shift=%d" % (N, shift))
    rng = np.random.default_rng(N)
    A, B, C = (rng.random(N + shift) for _ in range(3))
    I = rng.permutation(N + shift).astype(np.int32)
    I[I >= N] = 0
    Ad, Bd, Id = (torch.from_numpy(t).cuda()[shift:] for t in (A, B, I))
    Cd = torch.from_numpy(C).cuda()[shift:]
    mhdc.stream_direct(Ad.contiguous() if shift == 0 else Ad, Bd, Cd)
    want = oracle.stream_direct(A[shift:], B[shift:], C[shift:])
    assert np.array_equal(Cd.cpu().numpy(), want)
    Cd2 = torch.from_numpy(C).cuda()[shift:]
    Ii = I[shift:].copy()
    Ii[Ii >= N] = 0
    mhdc.stream_indirect(Ad, Bd, torch.from_numpy(Ii).cuda(), Cd2)
    assert np.array_equal(Cd2.cpu().numpy(), oracle.stream_indirect(A[shift:], B[shift:], Ii,
                                                                    C[shift:]))
