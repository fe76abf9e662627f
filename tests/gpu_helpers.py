"""Shared helpers of the GPU parity tests: device copies, the oracle
comparisons and the tolerance of the parity contract."""
import sys

import numpy as np
import torch

import oracle
from paper_2105_04937_amd import mhdc

REL_TOL = 1e-13  # |y - y_ref|_i <= REL_TOL * (|A||x|)_i


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(m):
    return mhdc.to_device(m)


def bits(a):
    a = np.ascontiguousarray(a)
    return a.view(np.int64) if a.dtype == np.float64 else a


def assert_same_bits(got, want, name):
    got = np.asarray(got)
    want = np.asarray(want)
    assert got.shape == want.shape, "%s: shape %s != %s" % (name, got.shape, want.shape)
    assert np.array_equal(bits(got), bits(want)), "%s differs at %s" % (
        name, np.nonzero(bits(got) != bits(want))[0][:10])


def assert_spmv_close(y_gpu, m, x, Y_ref=None, absAx=None, tol=REL_TOL):
    """Element-wise parity: |y - y_ref| <= tol * |A||x| (exact where |A||x| = 0)."""
    y = y_gpu.detach().cpu().numpy() if isinstance(y_gpu, torch.Tensor) else y_gpu
    yref = oracle.csr_spmv(m.rowptr, m.colind, m.val, x, 0) if Y_ref is None else Y_ref
    scale = oracle.csr_absmv(m.rowptr, m.colind, m.val, x) if absAx is None else absAx
    err = np.abs(y - yref)
    bad = ~(err <= tol * scale)
    assert not bad.any(), "rows %s: got %s want %s scale %s" % (
        np.nonzero(bad)[0][:5], y[bad][:5], yref[bad][:5], scale[bad][:5])
    return y


def check_mhdc_arrays(h, ref):
    """Every array of an M-HDC handle equals the oracle's, bit for bit."""
    t = h.export()
    torch.cuda.synchronize()
    assert_same_bits(t["dia_ptr"].cpu().numpy(), ref.dia_ptr, "dia_ptr")
    assert_same_bits(t["dia_off"].cpu().numpy(), ref.dia_off, "dia_off")
    assert_same_bits(t["dia_val"].cpu().numpy(), ref.dia_val, "dia_val")
    assert_same_bits(t["rem_ptr"].cpu().numpy(), ref.rem_ptr, "rem_ptr")
    assert_same_bits(t["rem_col"].cpu().numpy(), ref.rem_col, "rem_col")
    assert_same_bits(t["rem_val"].cpu().numpy(), ref.rem_val, "rem_val")


def check_hdc_arrays(h, ref):
    t = h.export()
    torch.cuda.synchronize()
    assert_same_bits(t["dia_off"].cpu().numpy(), ref.dia_off, "dia_off")
    assert_same_bits(t["dia_val"].cpu().numpy(), ref.dia_val, "dia_val")
    assert_same_bits(t["rem_ptr"].cpu().numpy(), ref.rem_ptr, "rem_ptr")
    assert_same_bits(t["rem_col"].cpu().numpy(), ref.rem_col, "rem_col")
    assert_same_bits(t["rem_val"].cpu().numpy(), ref.rem_val, "rem_val")


def check_round_trip(h, m):
    rp, ci, v = h.to_csr()
    torch.cuda.synchronize()
    assert_same_bits(rp.cpu().numpy(), m.rowptr, "rowptr")
    assert_same_bits(ci.cpu().numpy(), m.colind, "colind")
    assert_same_bits(v.cpu().numpy(), m.val, "val")


def assert_oracle_bits(y_gpu, y_oracle, name):
    """The GPU kernel reproduces the paper's sequential kernel bit for bit."""
    y = y_gpu.detach().cpu().numpy() if isinstance(y_gpu, torch.Tensor) else y_gpu
    assert_same_bits(y, y_oracle, name)


def check_byte_model(mat, m, ref=None):
    """The byte-model figures a handle reports (mhdc_info) equal the oracle
    model's (Sec. 5.3, Eqs. 23-36) computed from the oracle converter's own
    layout `ref` (None for a CSR handle): the integer byte counts and the
    alpha/beta divisions exactly, rp_est exactly as V_CSR / V and within
    1e-12 of the closed form of Eq. 28."""
    from oracle import model
    inf = mat.info()
    n, nnz = m.n, m.nnz
    if ref is None:
        K, S, R, n_blk = 0, 0, nnz, inf["n_blk"]
        want_alg = model.b_alg_csr(n, nnz)
        want_v = model.v_csr_general(n, nnz)
    else:
        K, S, R, n_blk = ref.K, ref.dia_val.size, ref.R, ref.n_blk
        if inf["kind"] == 1:
            assert S == K * n
            want_alg = model.b_alg_hdc(n, K, R)
        else:
            want_alg = model.b_alg_blocked(n, K, S, n_blk, R)
        want_v = model.v_hdc_blocked(n, R, S)
    got = tuple(inf[f] for f in ("nnz", "K", "S", "R", "n_blk"))
    assert got == (nnz, K, S, R, n_blk), (got, (nnz, K, S, R, n_blk))
    assert inf["bytes_alg"] == want_alg, (inf["bytes_alg"], want_alg)
    assert inf["bytes_paper"] == want_v, (inf["bytes_paper"], want_v)
    alpha, beta = model.alpha_beta(nnz, R, S)
    assert (inf["alpha"], inf["beta"]) == (alpha, beta)
    v_csr = model.v_csr_general(n, nnz)
    assert inf["rp_est"] == (v_csr / want_v if want_v > 0 else 1.0)
    if n > 0 and nnz > 0:
        eq28 = model.rp_est(alpha, beta, nnz / n)
        assert abs(inf["rp_est"] - eq28) <= 1e-12 * eq28, (inf["rp_est"], eq28)
    return inf
