"""Seeded synthetic inputs for M-HDC SpMV: grid stencil matrices and vectors.

This module draws inputs only; it holds none of the method's arithmetic (no
conversion, no selection, no SpMV).  Both the CPU oracle's tests and the GPU
path take their inputs from here.  Every generator is a pure function of its
seed (numpy PCG64 via ``default_rng``).

Matrices are returned as zero-based CSR (``rowptr`` int32 [n+1], ``colind``
int32 [nnz] strictly increasing per row, ``val`` float64 [nnz]).

Grid numbering: point (ix, iy, iz) of an N^3 grid is row
r = ix + N*(iy + N*iz); a coupling to a neighbour outside the grid is dropped
("truncated" boundary), so rows on faces have fewer entries.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class CSRMatrix:
    n: int
    rowptr: np.ndarray
    colind: np.ndarray
    val: np.ndarray
    meta: dict

    @property
    def nnz(self) -> int:
        return int(self.colind.size)


def stencil_points(points: int):
    """Neighbour displacements (dx, dy, dz) of a 7-, 19- or 27-point stencil,
    ordered by (dz, dy, dx) so that columns ascend for N >= 3.  The 19-point
    stencil is the set |dx|+|dy|+|dz| <= 2."""
    pts = []
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                m = abs(dx) + abs(dy) + abs(dz)
                if points == 7 and m <= 1:
                    pts.append((dx, dy, dz))
                elif points == 19 and m <= 2:
                    pts.append((dx, dy, dz))
                elif points == 27:
                    pts.append((dx, dy, dz))
    if points not in (7, 19, 27):
        raise ValueError("stencil must have 7, 19 or 27 points")
    return pts


def _grid_structure(N: int, points: int):
    """Columns and in-grid mask of every stencil coupling, shape (n, S)."""
    n = N * N * N
    r = np.arange(n, dtype=np.int64)
    ix = r % N
    iy = (r // N) % N
    iz = r // (N * N)
    pts = stencil_points(points)
    S = len(pts)
    cols = np.empty((n, S), dtype=np.int32)
    inside = np.empty((n, S), dtype=bool)
    diag_s = pts.index((0, 0, 0))
    for s, (dx, dy, dz) in enumerate(pts):
        cols[:, s] = (r + dx + N * dy + N * N * dz).astype(np.int32)
        inside[:, s] = ((ix + dx >= 0) & (ix + dx < N) & (iy + dy >= 0) & (iy + dy < N)
                        & (iz + dz >= 0) & (iz + dz < N))
    return n, ix, iy, iz, cols, inside, diag_s


def _finish(n, cols, keep, diag_mask):
    """Flatten the kept couplings row by row into CSR structure."""
    counts = keep.sum(axis=1)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    if rowptr[-1] >= 2**31:
        raise ValueError("nnz does not fit INT32 indices")
    colind = cols[keep]
    is_diag = diag_mask[keep]
    return rowptr.astype(np.int32), colind.astype(np.int32, copy=False), is_diag


def _set_diagonal(rowptr, colind, val, is_diag, factor):
    """Diagonal = factor * |sum of the row's off-diagonal values|."""
    n = rowptr.size - 1
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(rowptr))
    off = np.where(is_diag, 0.0, val)
    rs = np.bincount(rows, weights=off, minlength=n)
    val[is_diag] = factor * np.abs(rs[rows[is_diag]])
    return val


def laplacian7(N: int) -> CSRMatrix:
    """7-point Laplacian on an N^3 grid: diagonal 6, neighbours -1, couplings
    across the grid faces dropped (the 32^3 parity case)."""
    n, _, _, _, cols, inside, diag_s = _grid_structure(N, 7)
    diag_mask = np.zeros_like(inside)
    diag_mask[:, diag_s] = True
    rowptr, colind, is_diag = _finish(n, cols, inside, diag_mask)
    val = np.where(is_diag, 6.0, -1.0).astype(np.float64)
    return CSRMatrix(n, rowptr, colind, val, dict(kind="laplacian7", N=N))


def heptadiagonal(N: int, seed: int) -> CSRMatrix:
    """7-point stencil on an N^3 grid, off-diagonal values U[-1, -0.5],
    diagonal = 1.01 * |row sum of the off-diagonals| (the 256^3 case)."""
    rng = np.random.default_rng(seed)
    n, _, _, _, cols, inside, diag_s = _grid_structure(N, 7)
    diag_mask = np.zeros_like(inside)
    diag_mask[:, diag_s] = True
    rowptr, colind, is_diag = _finish(n, cols, inside, diag_mask)
    del cols, inside, diag_mask
    val = rng.uniform(-1.0, -0.5, size=colind.size)
    val = _set_diagonal(rowptr, colind, val, is_diag, 1.01)
    return CSRMatrix(n, rowptr, colind, val, dict(kind="hepta", N=N, seed=seed))


OCTANT_DROP = (0.0, 0.05, 0.1, 0.2, 0.3, 0.5, 0.7, 0.9)


def partially_diagonal(N: int, seed: int, points: int = 27,
                       drop=OCTANT_DROP, extra_per_row: int = 2,
                       diag_factor: float = 1.1) -> CSRMatrix:
    """Partially diagonal stencil matrix (the 192^3 case by default).

    * stencil couplings of `points` points on an N^3 grid, truncated at faces;
    * `drop` is either one probability or eight, one per octant: the octant of
      a row's grid point is o = 4*[iz >= N/2] + 2*[iy >= N/2] + [ix >= N/2];
      each off-diagonal coupling of the row is dropped independently with that
      probability (the diagonal is never dropped);
    * `extra_per_row` further columns per row drawn uniformly from [0, n) and
      redrawn while they hit a column already in the row;
    * values N(0, 1); diagonal = diag_factor * |sum of the off-diagonals|.
    Draw order: drop uniforms, extra columns (and redraws), values.
    """
    rng = np.random.default_rng(seed)
    n, ix, iy, iz, cols, inside, diag_s = _grid_structure(N, points)
    S = cols.shape[1]
    diag_mask = np.zeros_like(inside)
    diag_mask[:, diag_s] = True
    if np.ndim(drop) == 0:
        p_row = np.full(n, float(drop))
    else:
        h = N // 2
        octant = 4 * (iz >= h) + 2 * (iy >= h) + (ix >= h)
        p_row = np.asarray(drop, dtype=np.float64)[octant]
    del ix, iy, iz
    keep = inside.copy()
    if np.any(p_row > 0):
        u = rng.random((n, S))
        dropped = (u < p_row[:, None]) & ~diag_mask
        keep &= ~dropped
        del u, dropped
    if extra_per_row > 0:
        present = np.where(keep, cols, -1)
        extra = rng.integers(0, n, size=(n, extra_per_row), dtype=np.int64).astype(np.int32)
        while True:
            clash = np.zeros((n, extra_per_row), dtype=bool)
            for e in range(extra_per_row):
                ce = extra[:, e:e + 1]
                clash[:, e] = (present == ce).any(axis=1)
                for f in range(e):
                    clash[:, e] |= extra[:, f] == extra[:, e]
            nb = int(clash.sum())
            if nb == 0:
                break
            extra[clash] = rng.integers(0, n, size=nb, dtype=np.int64).astype(np.int32)
        del present
        big = np.iinfo(np.int32).max
        allc = np.concatenate([np.where(keep, cols, big), extra], axis=1)
        alld = np.concatenate([diag_mask, np.zeros((n, extra_per_row), bool)], axis=1)
        del cols
        order = np.argsort(allc, axis=1, kind="stable")
        allc = np.take_along_axis(allc, order, axis=1)
        alld = np.take_along_axis(alld, order, axis=1)
        del order
        keepall = allc != big
        rowptr, colind, is_diag = _finish(n, allc, keepall, alld)
    else:
        rowptr, colind, is_diag = _finish(n, cols, keep, diag_mask)
    val = rng.standard_normal(size=colind.size)
    val = _set_diagonal(rowptr, colind, val, is_diag, diag_factor)
    return CSRMatrix(n, rowptr, colind, val,
                     dict(kind="partial", N=N, seed=seed, points=points,
                          drop=list(np.atleast_1d(drop)), extra=extra_per_row))


def batch_member(index: int, base_seed: int = 4000):
    """One matrix of the batched workload: grid side U{16..96}, stencil drawn
    from {7, 19, 27} points, one drop probability U[0, 0.3], values N(0,1),
    diagonal 1.1 * |row sum|, no random extra columns; plus its number of
    right-hand sides k ~ U{1..16}.  Returns (matrix, k)."""
    rng = np.random.default_rng(base_seed + index)
    side = int(rng.integers(16, 97))
    points = int(rng.choice([7, 19, 27]))
    p = float(rng.uniform(0.0, 0.3))
    k = int(rng.integers(1, 17))
    mseed = int(rng.integers(0, 2**31 - 1))
    m = partially_diagonal(side, mseed, points=points, drop=p, extra_per_row=0)
    m.meta.update(dict(index=index, side=side, points=points, p=p, k=k))
    return m, k


def stencil_matrix_gpu(N: int, seed: int, points: int = 27, drop=0.0, extra_per_row: int = 0,
                       diag_factor: float = 1.1, device="cuda"):
    """Device-side generator of the same family as partially_diagonal()
    (stencil couplings truncated at faces, per-octant or global drop
    probability, extra uniform columns redrawn on collision, N(0,1) values,
    diagonal = diag_factor * |row sum of off-diagonals|), drawn with a
    torch generator seeded by `seed` on `device`.  Used where thousands of
    matrices are needed (the selector's training and test sets); its stream
    of random numbers differs from the numpy generator's.  Returns
    (rowptr, colind, val) device tensors (int32, int32, float64)."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    n = N * N * N
    r = torch.arange(n, device=device, dtype=torch.int64)
    ix, iy, iz = r % N, (r // N) % N, r // (N * N)
    pts = stencil_points(points)
    S = len(pts)
    cols = torch.empty((n, S), dtype=torch.int64, device=device)
    keep = torch.empty((n, S), dtype=torch.bool, device=device)
    dpos = pts.index((0, 0, 0))
    for s, (dx, dy, dz) in enumerate(pts):
        cols[:, s] = r + dx + N * dy + N * N * dz
        keep[:, s] = ((ix + dx >= 0) & (ix + dx < N) & (iy + dy >= 0) & (iy + dy < N)
                      & (iz + dz >= 0) & (iz + dz < N))
    if np.ndim(drop) == 0:
        p_row = torch.full((n,), float(drop), device=device, dtype=torch.float64)
    else:
        h = N // 2
        octant = 4 * (iz >= h).long() + 2 * (iy >= h).long() + (ix >= h).long()
        p_row = torch.as_tensor(np.asarray(drop, np.float64), device=device)[octant]
    del ix, iy, iz
    u = torch.rand((n, S), generator=g, device=device, dtype=torch.float64)
    dropped = u < p_row[:, None]
    dropped[:, dpos] = False
    keep &= ~dropped
    del u, dropped
    big = np.iinfo(np.int64).max
    allc = torch.where(keep, cols, torch.full_like(cols, big))
    del cols
    if extra_per_row > 0:
        extra = torch.randint(0, n, (n, extra_per_row), generator=g, device=device,
                              dtype=torch.int64)
        while True:
            clash = torch.zeros((n, extra_per_row), dtype=torch.bool, device=device)
            for e in range(extra_per_row):
                clash[:, e] = (allc == extra[:, e:e + 1]).any(dim=1)
                for f in range(e):
                    clash[:, e] |= extra[:, f] == extra[:, e]
            nb = int(clash.sum())
            if nb == 0:
                break
            extra[clash] = torch.randint(0, n, (nb,), generator=g, device=device,
                                         dtype=torch.int64)
        allc = torch.cat([allc, extra], dim=1)
        del extra
    allc, _ = torch.sort(allc, dim=1)
    valid = allc != big
    counts = valid.sum(dim=1)
    rowptr = torch.zeros(n + 1, dtype=torch.int64, device=device)
    rowptr[1:] = torch.cumsum(counts, 0)
    colind = allc[valid]
    rows = torch.repeat_interleave(torch.arange(n, device=device), counts)
    del allc, valid
    val = torch.randn(colind.numel(), generator=g, device=device, dtype=torch.float64)
    is_diag = colind == rows
    off = torch.where(is_diag, torch.zeros_like(val), val)
    rs = torch.zeros(n, dtype=torch.float64, device=device).index_add_(0, rows, off)
    val = torch.where(is_diag, diag_factor * rs.abs()[rows], val)
    return rowptr.to(torch.int32), colind.to(torch.int32), val


def banded_offsets(n: int, points: int):
    """Offsets of the paper's banded stencil matrices (Sec. 6.3): 3 points
    {0, +-1}; 5 points adds +-n_x with n_x = floor(sqrt(n)); 7 points adds
    +-n_x and +-n_x^2 with n_x = floor(cbrt(n)).  Ascending."""
    if points == 3:
        offs = [0, 1]
    elif points == 5:
        nx = int(np.floor(np.sqrt(n)))
        while (nx + 1) * (nx + 1) <= n:
            nx += 1
        while nx * nx > n:
            nx -= 1
        offs = [0, 1, nx]
    elif points == 7:
        nx = int(round(n ** (1.0 / 3.0)))
        while (nx + 1) ** 3 <= n:
            nx += 1
        while nx ** 3 > n:
            nx -= 1
        offs = [0, 1, nx, nx * nx]
    else:
        raise ValueError("points must be 3, 5 or 7")
    return sorted(set([-o for o in offs] + offs))


def banded_stencil(n: int, points: int, seed: int) -> CSRMatrix:
    """Banded stencil matrix of Sec. 6.3: a_ij != 0 exactly for j - i in
    banded_offsets(n, points) and 0 <= j < n (no truncation at grid faces);
    off-diagonals U[-1, -0.5] in CSR order, diagonal 1.01 * |row sum|."""
    rng = np.random.default_rng(seed)
    offs = np.asarray(banded_offsets(n, points), dtype=np.int64)
    i = np.arange(n, dtype=np.int64)
    cols = i[:, None] + offs[None, :]
    keep = (cols >= 0) & (cols < n)
    counts = keep.sum(axis=1)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    rowptr[1:] = np.cumsum(counts)
    colind = cols[keep]
    rows = np.repeat(i, counts)
    val = rng.uniform(-1.0, -0.5, size=colind.size)
    is_diag = colind == rows
    val[is_diag] = 0.0
    rs = np.zeros(n)
    np.add.at(rs, rows, val)
    val[is_diag] = 1.01 * np.abs(rs)
    return CSRMatrix(n, rowptr.astype(np.int32), colind.astype(np.int32), val,
                     dict(kind="banded", points=points, offsets=[int(o) for o in offs]))


def banded_stencil_gpu(n: int, points: int, seed: int, device="cuda"):
    """Device-side banded_stencil() (same structure and value rule, torch
    generator, different random stream) for sizes up to 5e7 rows.  Returns
    (rowptr, colind, val) device tensors (int32, int32, float64)."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    offs = torch.as_tensor(banded_offsets(n, points), dtype=torch.int64, device=device)
    i = torch.arange(n, dtype=torch.int64, device=device)
    cols = i[:, None] + offs[None, :]
    keep = (cols >= 0) & (cols < n)
    counts = keep.sum(dim=1)
    rowptr = torch.zeros(n + 1, dtype=torch.int64, device=device)
    rowptr[1:] = torch.cumsum(counts, 0)
    colind = cols[keep]
    del cols, keep
    rows = torch.repeat_interleave(i, counts)
    val = torch.rand(colind.numel(), generator=g, device=device, dtype=torch.float64) * 0.5 - 1.0
    is_diag = colind == rows
    val = torch.where(is_diag, torch.zeros_like(val), val)
    rs = torch.zeros(n, dtype=torch.float64, device=device).index_add_(0, rows, val)
    val = torch.where(is_diag, 1.01 * rs.abs()[rows], val)
    return rowptr.to(torch.int32), colind.to(torch.int32), val


def vector(n: int, seed: int, k: int = 1) -> np.ndarray:
    """x ~ U[-1, 1]; shape (n,) for k == 1, else (n, k) column-major."""
    rng = np.random.default_rng([seed, 1])
    if k == 1:
        return rng.uniform(-1.0, 1.0, size=n)
    return np.asfortranarray(rng.uniform(-1.0, 1.0, size=(k, n)).T)


def random_csr(n: int, seed: int, density: float = 0.1, bands=(),
               band_fill: float = 0.9, int_values: bool = False,
               zero_frac: float = 0.0) -> CSRMatrix:
    """Small random test matrix: background entries with probability
    `density`, plus each offset in `bands` filled with probability
    `band_fill`.  With int_values the values are small nonzero integers (so
    every sum is exact in FP64).  zero_frac of the stored entries are set to
    explicit zeros (alternating +0.0 / -0.0)."""
    rng = np.random.default_rng(seed)
    mask = rng.random((n, n)) < density
    i = np.arange(n)
    for d in bands:
        j = i + d
        ok = (j >= 0) & (j < n)
        fill = rng.random(n) < band_fill
        mask[i[ok & fill], j[ok & fill]] = True
    rows, cols = np.nonzero(mask)
    nnz = rows.size
    if int_values:
        v = rng.integers(1, 10, size=nnz).astype(np.float64) * rng.choice([-1.0, 1.0], size=nnz)
    else:
        v = rng.standard_normal(nnz)
    if zero_frac > 0 and nnz:
        z = rng.random(nnz) < zero_frac
        zi = np.nonzero(z)[0]
        v[zi] = np.where(np.arange(zi.size) % 2 == 0, 0.0, -0.0)
    rowptr = np.zeros(n + 1, np.int32)
    np.cumsum(np.bincount(rows, minlength=n), out=rowptr[1:])
    return CSRMatrix(n, rowptr, cols.astype(np.int32), v,
                     dict(kind="random", seed=seed, density=density, bands=list(bands)))


def dense_of(m: CSRMatrix) -> np.ndarray:
    """Dense copy of a small CSR matrix (for brute-force checks)."""
    A = np.zeros((m.n, m.n), np.float64)
    rows = np.repeat(np.arange(m.n), np.diff(m.rowptr))
    A[rows, m.colind] = m.val
    return A
