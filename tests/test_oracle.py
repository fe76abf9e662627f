"""Pins of the CPU oracle against what the paper and the mathematics fix.

Every check here is independent of the oracle's own code path: the paper's
printed encodings of its Example matrix (Figs. 2, 4, 7, 15), products worked
by hand, dense brute force, a closed form of the 7-point Laplacian, and the
invariants the paper states (alpha >= theta, HDC == M-HDC with bl = n).
"""
import numpy as np
import pytest

import oracle
from oracle import model
from paper_2105_04937_amd import synth
from tests.conftest import load_golden

THETAS = [0.0, 0.5, 0.6, 2.0 / 3.0, 0.75, 1.0]


def _arr(rows, dt):
    return np.array(rows[0], dtype=dt)


# ---------------------------------------------------------------- worked example
def test_example_csr_is_fig2(example):
    g = load_golden("example_csr.txt")
    assert np.array_equal(example["rowptr"], _arr(g["row_ptr"], np.int32))
    assert np.array_equal(example["colind"], _arr(g["col_ind"], np.int32))
    assert np.array_equal(example["val"], _arr(g["val"], np.float64))


def test_example_products(example):
    g = load_golden("example_products.txt")
    for x, y in zip(g["x"], g["y"]):
        x = np.array(x)
        got = oracle.csr_spmv(example["rowptr"], example["colind"], example["val"], x)
        assert np.array_equal(got, np.array(y))
        assert np.array_equal(oracle.dense_matvec(example["A"], x), np.array(y))


def test_example_dia_is_fig4(example):
    """The DIA format keeps every nonzero diagonal line: HDC with theta = 0."""
    g = load_golden("example_dia.txt")
    m = oracle.hdc_from_csr(example["rowptr"], example["colind"], example["val"], 0.0)
    assert np.array_equal(m.dia_off, _arr(g["offset"], np.int32))
    assert np.array_equal(m.dia_val.reshape(m.K, 8), np.array(g["val"]))
    assert m.R == 0


def test_example_hdc_is_fig7(example):
    g = load_golden("example_hdc_theta0.6.txt")
    m = oracle.hdc_from_csr(example["rowptr"], example["colind"], example["val"], 0.6)
    assert np.array_equal(m.dia_off, _arr(g["dia_offset"], np.int32))
    assert np.array_equal(m.dia_val.reshape(m.K, 8), np.array(g["dia_val"]))
    assert np.array_equal(m.rem_val, _arr(g["csr_val"], np.float64))
    assert np.array_equal(m.rem_col, _arr(g["csr_col_ind"], np.int32))
    assert np.array_equal(m.rem_ptr, _arr(g["csr_row_ptr"], np.int32))


@pytest.mark.parametrize("theta", [0.6, 0.75])
def test_example_mhdc_is_fig15(example, theta):
    """theta = 0.75 is the tie case: offsets 2 and 5 of block 0 and -4 of
    block 1 have exactly 3 of 4 rows, so ">=" keeps them (the formula of
    Sec. 4.3) and the arrays are those of Fig. 15."""
    g = load_golden("example_mhdc_bl4_theta0.6.txt")
    m = oracle.mhdc_from_csr(example["rowptr"], example["colind"], example["val"], 4, theta)
    assert np.array_equal(m.dia_off, _arr(g["dia_col_offset"], np.int32))
    assert np.array_equal(m.dia_ptr, _arr(g["dia_ptr"], np.int32))
    assert np.array_equal(m.dia_val.reshape(m.K, 4), np.array(g["dia_val"]))
    assert np.array_equal(m.rem_val, _arr(g["csr_val"], np.float64))
    assert np.array_equal(m.rem_col, _arr(g["csr_col_ind"], np.int32))
    assert np.array_equal(m.rem_ptr, _arr(g["csr_row_ptr"], np.int32))


def test_example_mhdc_above_tie(example):
    """Just above 3/4 the three 3-of-4 partial diagonals leave the DIA part."""
    m = oracle.mhdc_from_csr(example["rowptr"], example["colind"], example["val"], 4, 0.76)
    assert list(m.dia_off) == [0, 0]
    assert list(m.dia_ptr) == [0, 1, 2]
    assert m.R == 20 - 8


def test_example_kernels_exact(example):
    g = load_golden("example_products.txt")
    a = (example["rowptr"], example["colind"], example["val"])
    mh = oracle.mhdc_from_csr(*a, 4, 0.6)
    hd = oracle.hdc_from_csr(*a, 0.6)
    for x, y in zip(g["x"], g["y"]):
        assert np.array_equal(oracle.mhdc_spmv(mh, np.array(x)), np.array(y))
        assert np.array_equal(oracle.hdc_spmv(hd, np.array(x)), np.array(y))


# ---------------------------------------------------------------- brute force
def _small_cases():
    cases = []
    for s, n in enumerate([1, 2, 5, 8, 17, 33, 64]):
        bands = [0, 1, -1, 3, -(n // 2)] if n > 2 else [0]
        cases.append(synth.random_csr(n, 100 + s, density=0.08, bands=bands, int_values=True))
        cases.append(synth.random_csr(n, 200 + s, density=0.3, bands=(), int_values=False))
    cases.append(synth.random_csr(40, 300, density=0.05, bands=[0, 2, -5], zero_frac=0.2,
                                  int_values=True))
    cases.append(synth.random_csr(10, 301, density=0.0, bands=()))  # empty matrix
    return cases


def _bound(m, x):
    """2 * gamma_mmax * (|A||x|): the worst-case gap between two summation
    orders of rows with at most mmax terms (u = 2^-53)."""
    mmax = int(np.max(np.diff(m.rowptr))) if m.n else 0
    u = 2.0 ** -53
    g = mmax * u / (1 - mmax * u)
    return 2 * g * oracle.csr_absmv(m.rowptr, m.colind, m.val, x)


@pytest.mark.parametrize("m", _small_cases(), ids=lambda m: "n%d_s%d" % (m.n, m.meta["seed"]))
def test_csr_vs_dense(m):
    A = synth.dense_of(m)
    x = synth.vector(m.n, 7)
    y = oracle.csr_spmv(m.rowptr, m.colind, m.val, x)
    # ascending-column dense sum only adds exact zeros in between
    assert np.array_equal(y, oracle.dense_matvec(A, x))
    # an independent summation order (BLAS) within the rounding bound
    assert np.all(np.abs(y - A @ x) <= _bound(m, x))
    if m.n:
        xi = np.arange(m.n, dtype=np.float64) - 3.0
        if np.all(m.val == np.round(m.val)):
            assert np.array_equal(oracle.csr_spmv(m.rowptr, m.colind, m.val, xi), A @ xi)


def test_csr_spmm_vs_dense():
    m = synth.random_csr(30, 11, density=0.1, bands=[0, 1], int_values=True)
    X = np.asfortranarray(np.random.default_rng(3).integers(-4, 5, size=(30, 5)).astype(float))
    Y = oracle.csr_spmm(m.rowptr, m.colind, m.val, X)
    assert np.array_equal(Y, synth.dense_of(m) @ X)


def _brute_selection(A, bl, theta):
    """Kept (block, offset) pairs counted straight from the dense matrix."""
    n = A.shape[0]
    keep = []
    for ib in range(0 if n == 0 else (n + bl - 1) // bl):
        r0, r1 = ib * bl, min(n, ib * bl + bl)
        rows = r1 - r0
        for d in range(-(n - 1), n):
            cnt = sum(1 for i in range(r0, r1) if 0 <= i + d < n and A[i, i + d] != 0.0)
            if cnt >= 1 and cnt / rows >= theta:
                keep.append((ib, d))
    return keep


@pytest.mark.parametrize("m", _small_cases()[:8] + _small_cases()[-2:],
                         ids=lambda m: "n%d_s%d" % (m.n, m.meta["seed"]))
@pytest.mark.parametrize("bl", [1, 3, 4, 7, 16, 1000])
def test_mhdc_convert_brute_force(m, bl):
    A = synth.dense_of(m)
    x = synth.vector(m.n, 9)
    nnz = m.nnz
    for theta in THETAS:
        mh = oracle.mhdc_from_csr(m.rowptr, m.colind, m.val, bl, theta)
        got = [(ib, int(d)) for ib in range(mh.n_blk)
               for d in mh.dia_off[mh.dia_ptr[ib]:mh.dia_ptr[ib + 1]]]
        assert got == _brute_selection(A, bl, theta)
        # segment values are the matrix entries (R6), padding is +0.0
        for ib in range(mh.n_blk):
            r0 = ib * bl
            for k in range(mh.dia_ptr[ib], mh.dia_ptr[ib + 1]):
                seg = mh.dia_val[k * bl:(k + 1) * bl]
                for t in range(bl):
                    i, j = r0 + t, r0 + t + int(mh.dia_off[k])
                    inside = i < m.n and 0 <= j < m.n
                    want = A[i, j] if inside and A[i, j] != 0.0 else 0.0
                    assert seg[t] == want
                    if want == 0.0:
                        assert not np.signbit(seg[t])
        # conservation: nonzero DIA slots + remainder = stored entries
        assert np.count_nonzero(mh.dia_val) + mh.R == nnz
        # round trip CSR -> M-HDC -> CSR is the identity on bit patterns
        p, c, v = oracle.mhdc_to_csr(mh)
        assert np.array_equal(p, m.rowptr) and np.array_equal(c, m.colind)
        assert np.array_equal(v.view(np.int64), m.val.view(np.int64))
        # the Fig. 16 kernel reproduces CSR SpMV
        y = oracle.mhdc_spmv(mh, x)
        yref = oracle.csr_spmv(m.rowptr, m.colind, m.val, x)
        assert np.all(np.abs(y - yref) <= _bound(m, x))
        if np.all(m.val == np.round(m.val)):
            xi = np.arange(m.n, dtype=np.float64) - 2.0
            assert np.array_equal(oracle.mhdc_spmv(mh, xi),
                                  oracle.csr_spmv(m.rowptr, m.colind, m.val, xi))


@pytest.mark.parametrize("m", _small_cases(), ids=lambda m: "n%d_s%d" % (m.n, m.meta["seed"]))
def test_hdc_is_mhdc_with_one_block(m):
    """B-HDC equals M-HDC with bl = n in its selection (Sec. 6.4.2): the HDC
    converter and the M-HDC converter with one block give the same arrays."""
    for theta in THETAS:
        h = oracle.hdc_from_csr(m.rowptr, m.colind, m.val, theta)
        mh = oracle.mhdc_from_csr(m.rowptr, m.colind, m.val, max(m.n, 1), theta)
        for f in ("dia_ptr", "dia_off", "dia_val", "rem_ptr", "rem_col", "rem_val"):
            assert np.array_equal(getattr(h, f), getattr(mh, f)), f
        x = synth.vector(m.n, 5)
        assert np.all(np.abs(oracle.hdc_spmv(h, x) - oracle.csr_spmv(m.rowptr, m.colind, m.val, x))
                      <= _bound(m, x))


def test_selection_invariants():
    """alpha~ >= theta per partial diagonal (Sec. 6.4.2), R non-decreasing in
    theta, and theta = 0 leaves only the stored zeros in the remainder."""
    m = synth.random_csr(60, 42, density=0.05, bands=[0, 1, -1, 7, -20], band_fill=0.7,
                         int_values=True, zero_frac=0.1)
    nzeros = int(np.sum(m.val == 0.0))
    for bl in (5, 8, 13, 60):
        prevR = -1
        for theta in THETAS:
            mh = oracle.mhdc_from_csr(m.rowptr, m.colind, m.val, bl, theta)
            for ib in range(mh.n_blk):
                rows = min(m.n, (ib + 1) * bl) - ib * bl
                for k in range(mh.dia_ptr[ib], mh.dia_ptr[ib + 1]):
                    filled = np.count_nonzero(mh.dia_val[k * bl:(k + 1) * bl])
                    assert filled / rows >= theta and filled >= 1
            assert mh.R >= prevR
            prevR = mh.R
            if theta == 0.0:
                assert mh.R == nzeros


def test_signed_zero_nan_inf_round_trip():
    m = synth.random_csr(24, 77, density=0.05, bands=[0, 1, -2], band_fill=1.0)
    v = m.val.copy()
    v[::7] = -0.0
    v[3] = np.inf
    v[5] = -np.inf
    v[11] = np.nan
    for bl in (4, 24):
        mh = oracle.mhdc_from_csr(m.rowptr, m.colind, v, bl, 0.5)
        p, c, vv = oracle.mhdc_to_csr(mh)
        assert np.array_equal(p, m.rowptr) and np.array_equal(c, m.colind)
        assert np.array_equal(vv.view(np.int64), v.view(np.int64))


# ---------------------------------------------------------------- closed forms
def test_laplacian_linear_field_closed_form():
    """For x linear on the grid, (L x)_p = sum over the missing neighbours e
    of x_lin(p + e): zero inside, nonzero only on the faces."""
    N = 9
    m = synth.laplacian7(N)
    a, b, c, d = 3.0, -2.0, 5.0, 7.0
    r = np.arange(m.n)
    ix, iy, iz = r % N, (r // N) % N, r // (N * N)
    x = a * ix + b * iy + c * iz + d
    want = np.zeros(m.n)
    for (dx, dy, dz) in [(-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)]:
        out = ((ix + dx < 0) | (ix + dx >= N) | (iy + dy < 0) | (iy + dy >= N)
               | (iz + dz < 0) | (iz + dz >= N))
        want += np.where(out, a * (ix + dx) + b * (iy + dy) + c * (iz + dz) + d, 0.0)
    y = oracle.csr_spmv(m.rowptr, m.colind, m.val, x)
    assert np.array_equal(y, want)
    interior = (ix > 0) & (ix < N - 1) & (iy > 0) & (iy < N - 1) & (iz > 0) & (iz < N - 1)
    assert np.all(y[interior] == 0.0)
    for bl in (N, 2 * N, 50):
        mh = oracle.mhdc_from_csr(m.rowptr, m.colind, m.val, bl, 0.6)
        assert np.array_equal(oracle.mhdc_spmv(mh, x), want)
    # constant field: c times the number of missing neighbours
    y1 = oracle.csr_spmv(m.rowptr, m.colind, m.val, np.full(m.n, 2.0))
    missing = 7 - np.diff(m.rowptr)
    assert np.array_equal(y1, 2.0 * missing)


def test_heptadiagonal_block_count_formula():
    """With bl = N every block is one grid line: offsets 0 and +-1 are always
    kept, +-N unless the line lies on a y face, +-N^2 unless on a z face, so
    K = 3 N^2 + 4 N (N - 1) and every slot count is K * N."""
    N = 12
    m = synth.heptadiagonal(N, 2)
    mh = oracle.mhdc_from_csr(m.rowptr, m.colind, m.val, N, 0.6)
    assert mh.K == 3 * N * N + 4 * N * (N - 1)
    assert mh.R == 0
    assert mh.dia_val.size == mh.K * N
    # the 256^3 headline case by the same formula
    N = 256
    K = 3 * N * N + 4 * N * (N - 1)
    S = K * N
    assert (K, S) == (457_728, 117_178_368)


# ---------------------------------------------------------------- byte model
def test_model_stencil_closed_forms():
    n = 1.0
    for nd, gam in [(3, 1 / 3), (5, 1 / 5), (7, 3 / 7), (7, 1 / 7), (4, 0.5)]:
        vc = model.v_csr_stencil(n, nd, gam)
        vd = model.v_dia_stencil(n, nd)
        vb = model.v_bdia_stencil(n, nd, gam)
        assert (vc - vd) / vd == pytest.approx(model.eq9_dia_over_csr(nd, gam), rel=1e-14)
        assert (vc - vb) / vb == pytest.approx(model.eq16_bdia_over_csr(nd, gam), rel=1e-14)
        assert (vd - vb) / vb == pytest.approx(model.eq19_bdia_over_dia(nd, gam), rel=1e-14)
        # bounds of Eqs. 10-21 (b = 1/2)
        assert vc / vd <= 1.0 + 1e-12
        assert 1 + model.B / 2 - 1e-12 <= vc / vb <= 1 + model.B + 1e-12
        assert 5 / 3 - 1e-12 <= vd / vb <= 4 + 1e-12
    assert model.v_csr_stencil(1, 7, 1 / 7) / model.v_bdia_stencil(1, 7, 1 / 7) == pytest.approx(13 / 9)
    assert model.v_csr_stencil(1, 7, 3 / 7) / model.v_bdia_stencil(1, 7, 3 / 7) == pytest.approx(15 / 11)


def test_model_eq28_matches_volumes():
    n, c = 1000.0, 20.0
    nnz = c * n
    for alpha in (2 / 3, 0.8, 1.0):
        for beta in (0.0, 0.25, 0.5, 1.0):
            R = beta * nnz
            slots = (1 - beta) * nnz / alpha
            vc = model.v_csr_general(n, nnz)
            vm = model.v_hdc_blocked(n, R, slots)
            assert (vc - vm) / vm == pytest.approx(model.eq28_speedup_minus_one(alpha, beta, c), rel=1e-12)
            a2, b2 = model.alpha_beta(nnz, R, slots)
            assert b2 == pytest.approx(beta)
            if slots > 0:
                assert a2 == pytest.approx(alpha)
    # break-even fill alpha = 1/(b+1) = 2/3 (Eq. 32); upper bound 1 + b (Eq. 30)
    assert model.eq28_speedup_minus_one(2 / 3, 0.3, 30) == pytest.approx(0.0, abs=1e-15)
    assert model.rp_est(1.0, 0.0, 1e9) == pytest.approx(1.5, rel=1e-6)


def test_b_alg_example_by_hand(example):
    """Algorithmic bytes of the Example matrix counted by hand from the
    printed layouts: Fig. 15 (bl = 4, theta = 0.6: dia_ptr 3, offsets 5,
    20 slots, remainder row_ptr 9, 3 entries), Fig. 7 (theta = 0.6: 2
    offsets, 16 slots, 7 entries), Fig. 2 (20 entries); x and y 8 each."""
    n, nnz = example["n"], example["val"].size
    assert model.b_alg_blocked(n, 5, 20, 2, 3) == 4 * 3 + 4 * 5 + 8 * 20 + 4 * 9 + 12 * 3 + 16 * 8
    assert model.b_alg_hdc(n, 2, 7) == 4 * 2 + 8 * 16 + 4 * 9 + 12 * 7 + 16 * 8
    assert model.b_alg_csr(n, nnz) == 4 * 9 + 12 * 20 + 16 * 8
    # paper volumes (Eqs. 24/34, v_x = 1): no block pointer, no offsets
    assert model.v_hdc_blocked(n, 3, 20) == 12 * 3 + 4 * 8 + 8 * 20 + 8 * 8 + 8 * 8
    assert model.v_csr_general(n, nnz) == 12 * 20 + 4 * 8 + 16 * 8


@pytest.mark.parametrize("m", _small_cases()[:6], ids=lambda m: "n%d_s%d" % (m.n, m.meta["seed"]))
@pytest.mark.parametrize("bl", [1, 4, 7, 1000])
def test_b_alg_is_the_stored_layout(m, bl):
    """B_alg equals the bytes of the arrays the oracle's converters actually
    store (a remainder row pointer only when the remainder has entries),
    plus x read once and y written once, k columns each."""
    for theta in (0.0, 0.6, 1.0):
        mh = oracle.mhdc_from_csr(m.rowptr, m.colind, m.val, bl, theta)
        stored = (mh.dia_ptr.nbytes + mh.dia_off.nbytes + mh.dia_val.nbytes + mh.rem_col.nbytes
                  + mh.rem_val.nbytes + (mh.rem_ptr.nbytes if mh.R > 0 else 0))
        for k in (1, 3):
            xy = 2 * 8 * m.n * k
            assert model.b_alg_blocked(m.n, mh.K, mh.dia_val.size, mh.n_blk, mh.R, k) == stored + xy
        hd = oracle.hdc_from_csr(m.rowptr, m.colind, m.val, theta)
        stored = (hd.dia_off.nbytes + hd.dia_val.nbytes + hd.rem_col.nbytes + hd.rem_val.nbytes
                  + (hd.rem_ptr.nbytes if hd.R > 0 else 0))
        assert model.b_alg_hdc(m.n, hd.K, hd.R) == stored + 16 * m.n
    assert model.b_alg_csr(m.n, m.nnz, 2) == (m.rowptr.nbytes + m.colind.nbytes + m.val.nbytes
                                             + 2 * 8 * m.n * 2)


def test_b_alg_heptadiagonal_closed_form():
    """7-point grid of side N with bl = N (one grid line per block): every
    block keeps offsets 0 and +-1, and +-N, +-N^2 unless its line lies on
    the matching face, so K = 3N^2 + 4N(N-1), n_blk = N^2, R = 0 and
    B_alg = 4(N^2+1) + 4K + 8KN + 16N^3 (1,207,955,460 bytes at N = 256)."""
    for N in (5, 8, 12):
        m = synth.heptadiagonal(N, 2)
        mh = oracle.mhdc_from_csr(m.rowptr, m.colind, m.val, N, 0.6)
        K = 3 * N * N + 4 * N * (N - 1)
        assert (mh.K, mh.R, mh.n_blk) == (K, 0, N * N)
        want = 4 * (N * N + 1) + 4 * K + 8 * K * N + 16 * N ** 3
        assert model.b_alg_blocked(m.n, mh.K, mh.dia_val.size, mh.n_blk, mh.R) == want
    N, K = 256, 3 * 256 ** 2 + 4 * 256 * 255
    assert model.b_alg_blocked(N ** 3, K, K * N, N * N, 0) == 1_207_955_460


def test_stream_kernels():
    """Sec. 6.2 kernels on integer-valued arrays, where every result is
    exact: C[i] = 1 + i * (3 + i) for the direct kernel; the indirect kernel
    with the reversed index reads B[n-1-i]; with the identity index it
    equals the direct kernel; an index outside [0, n) leaves C[i] as is."""
    n = 100
    i = np.arange(n, dtype=np.float64)
    A, B, C = i.copy(), 3.0 + i, np.ones(n)
    assert np.array_equal(oracle.stream_direct(A, B, C), 1.0 + i * (3.0 + i))
    rev = np.arange(n - 1, -1, -1, dtype=np.int32)
    assert np.array_equal(oracle.stream_indirect(A, B, rev, C), 1.0 + i * (3.0 + (n - 1 - i)))
    rng = np.random.default_rng(0)
    A, B, C = rng.random(n), rng.random(n), rng.random(n)
    I = np.arange(n, dtype=np.int32)
    assert np.array_equal(oracle.stream_indirect(A, B, I, C), oracle.stream_direct(A, B, C))
    I[[3, 50]] = [-1, n]
    got = oracle.stream_indirect(A, B, I, C)
    assert got[3] == C[3] and got[50] == C[50]


@pytest.mark.parametrize("n,points", [(1000, 3), (1024, 5), (1000, 7), (999, 7)])
def test_banded_stencil_dia_closed_forms(n, points):
    """Sec. 6.3 banded stencils are pure DIA: HDC at theta = 0 keeps exactly
    the band offsets with an empty remainder and S = n per diagonal; with
    integer values every product and sum is exact, so the HDC kernel (Fig. 8)
    equals the CSR definition bit for bit; the per-block selection of M-HDC
    at theta = 1 keeps an offset in a block iff all its rows have it."""
    from paper_2105_04937_amd import synth
    m = synth.banded_stencil(n, points, 3)
    offs = synth.banded_offsets(n, points)
    h = oracle.hdc_from_csr(m.rowptr, m.colind, m.val, 0.0)
    assert list(h.dia_off) == offs and h.R == 0 and h.dia_val.size == len(offs) * n
    vi = np.round(m.val * 4.0)  # small integers: exact arithmetic
    vi[vi == 0] = 1.0
    x = np.arange(n, dtype=np.float64) % 7 - 3
    hi = oracle.hdc_from_csr(m.rowptr, m.colind, vi, 0.0)
    assert np.array_equal(oracle.hdc_spmv(hi, x), oracle.csr_spmv(m.rowptr, m.colind, vi, x))
    bl = 64
    mb = oracle.mhdc_from_csr(m.rowptr, m.colind, m.val, bl, 1.0)
    for ib in range(mb.n_blk):
        r0, r1 = ib * bl, min(n, ib * bl + bl)
        want = [o for o in offs if all(0 <= i + o < n for i in range(r0, r1))]
        assert list(mb.dia_off[mb.dia_ptr[ib]:mb.dia_ptr[ib + 1]]) == want


@pytest.mark.parametrize("m", _small_cases()[:6], ids=lambda m: "n%d_s%d" % (m.n, m.meta["seed"]))
def test_absmv_and_threads(m):
    """|A||x| (the scale of the parity bound) equals numpy's |A| @ |x| exactly
    on small-integer data; the row-parallel CSR loop gives the same bits as
    the sequential one (each row is still summed in column order)."""
    A = synth.dense_of(m)
    xi = (np.arange(m.n, dtype=np.float64) % 5) - 2.0
    vi = np.round(m.val * 3.0)
    Ai = np.zeros_like(A)
    for i in range(m.n):
        for k in range(m.rowptr[i], m.rowptr[i + 1]):
            Ai[i, m.colind[k]] = vi[k]
    assert np.array_equal(oracle.csr_absmv(m.rowptr, m.colind, vi, xi), np.abs(Ai) @ np.abs(xi))
    x = synth.vector(m.n, 3)
    assert np.array_equal(oracle.csr_spmv(m.rowptr, m.colind, m.val, x, 4),
                          oracle.csr_spmv(m.rowptr, m.colind, m.val, x, 1))
