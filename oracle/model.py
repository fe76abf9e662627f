"""Performance model of Sec. 5 written out as plain formulas -- TEST INFRASTRUCTURE.

Byte counts V = V_A + V_x + V_y (Eq. 4) for the CSR, DIA, B-DIA, B-HDC and
M-HDC kernels, with b_fp = 8 and b_int = 4 (FP64 values, INT32 indices), and
the speed-up expressions the paper derives from them (Eqs. 3, 9, 16, 19, 28).
Only the tests read this module.
"""
from __future__ import annotations

B_FP = 8.0
B_INT = 4.0
B = B_INT / B_FP  # b, Eq. 6


# -- stencil matrices, Sec. 5.2 (N_nz ~= n_diag * n, Eq. 5) -----------------
def v_csr_stencil(n, ndiag, gamma):
    """V^(CSR) for a stencil: val + col_ind + row_ptr, x with cache factor
    gamma, y written once (Sec. 5.2.1)."""
    va = B_FP * (ndiag + B * ndiag + B) * n
    vx = B_FP * gamma * ndiag * n
    vy = B_FP * n
    return va + vx + vy


def v_dia_stencil(n, ndiag):
    """V^(DIA): every x and y access goes to memory; y is zeroed once and
    read+written per diagonal (Sec. 5.2.2)."""
    return B_FP * ndiag * n + B_FP * ndiag * n + B_FP * (1 + 2 * ndiag) * n


def v_bdia_stencil(n, ndiag, gamma):
    """V^(B-DIA): y stays in cache, x with cache factor gamma (Sec. 5.2.3)."""
    return B_FP * ndiag * n + B_FP * gamma * ndiag * n + B_FP * n


def eq9_dia_over_csr(ndiag, gamma):
    """(V^CSR - V^DIA) / V^DIA in the closed form of Eq. 9."""
    return (B * (ndiag + 1) - (3 - gamma) * ndiag) / (4 * ndiag + 1)


def eq16_bdia_over_csr(ndiag, gamma):
    """(V^CSR - V^B-DIA) / V^B-DIA with gamma^CSR = gamma^B-DIA (Eq. 16)."""
    return B * (ndiag + 1) / ((1 + gamma) * ndiag + 1)


def eq19_bdia_over_dia(ndiag, gamma):
    """(V^DIA - V^B-DIA) / V^B-DIA (Eq. 19)."""
    return (3 - gamma) * ndiag / ((1 + gamma) * ndiag + 1)


# -- general matrices, Sec. 5.3 ----------------------------------------------
def v_csr_general(n, nnz, vx=1.0):
    """V^(CSR) = (b_fp + b_int) nnz + b_int n + b_fp v_x n + b_fp n."""
    return (B_FP + B_INT) * nnz + B_INT * n + B_FP * vx * n + B_FP * n


def v_hdc_blocked(n, R, slots, vx=1.0):
    """V^(B-HDC) / V^(M-HDC) (Eqs. 24, 34): CSR part val+col of the R
    remainder entries, its row_ptr, the stored DIA slots, x and y.
    `slots` is n_diag * n for B-HDC and sum_ib n_diag^(ib) * bl for M-HDC."""
    return (B_FP + B_INT) * R + B_INT * n + B_FP * slots + B_FP * vx * n + B_FP * n


def alpha_beta(nnz, R, slots):
    """Filling rate alpha = (1 - beta) nnz / slots and CSR rate beta (Eqs. 23, 33)."""
    beta = R / nnz if nnz else 0.0
    alpha = (nnz - R) / slots if slots else 1.0
    return alpha, beta


def eq28_speedup_minus_one(alpha, beta, c, vx=1.0):
    """(V^CSR - V^B-HDC) / V^B-HDC in the closed form of Eq. 28 (Delta v_x = 0)."""
    num = B * (1 - beta) * c - (1 - beta) * (1.0 / alpha - 1.0) * c
    den = beta * (c + B * c) + B + (1 - beta) * c / alpha + vx + 1
    return num / den


def rp_est(alpha, beta, c, vx=1.0):
    """Estimated relative performance P^(M-HDC)/P^(CSR) = 1 + Eq. 28 (Eq. 3)."""
    return 1.0 + eq28_speedup_minus_one(alpha, beta, c, vx)


def relative_error(rp_estimate, rp_executed):
    """RE = (RP_est - RP_exe) / RP_exe (Sec. 6.4.3)."""
    return (rp_estimate - rp_executed) / rp_executed


# -- algorithmic bytes of one product with the stored layouts ---------------
# The least a product y = A X (k right-hand sides) must move with a given
# layout: every stored array element read once, every x element read once,
# every y element written once (the paper's V with v_x = 1, but counting the
# stored layout exactly: block pointer, offsets, padding slots).  A CSR part
# with no entries needs no row pointer (nothing of it is read).
def b_alg_blocked(n, K, S, n_blk, R, k=1):
    """M-HDC (Sec. 4.3, Fig. 15): dia_ptr[n_blk+1], dia_offset[K],
    dia_val[S], the remainder's row_ptr[n+1] (if R > 0), col_ind[R], val[R],
    x and y."""
    rp = B_INT * (n + 1) if R > 0 else 0.0
    return (B_INT * (n_blk + 1) + B_INT * K + B_FP * S + rp + (B_INT + B_FP) * R
            + 2 * B_FP * n * k)


def b_alg_hdc(n, K, R, k=1):
    """HDC (Sec. 3.4, Fig. 7): offset[K], val[K][n], the CSR part's
    row_ptr[n+1] (if R > 0), col_ind[R], val[R], x and y; no block pointer."""
    rp = B_INT * (n + 1) if R > 0 else 0.0
    return B_INT * K + B_FP * K * n + rp + (B_INT + B_FP) * R + 2 * B_FP * n * k


def b_alg_csr(n, nnz, k=1):
    """CSR (Sec. 3.2, Fig. 2): row_ptr[n+1], col_ind[nnz], val[nnz], x, y."""
    return B_INT * (n + 1) + (B_INT + B_FP) * nnz + 2 * B_FP * n * k
