"""Column-major products given a workspace (mhdc_spmm_ws and its HDC / CSR
twins): on either route (the column-major kernel, or transposition into the
workspace and the row-major kernel storing Y by column) every column
equals the oracle's sequential kernel bit for bit; the lone-entry count
that picks the route equals a host brute force; bad workspaces are
refused."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from paper_2105_04937_amd import mhdc, synth
from tests.gpu_helpers import assert_oracle_bits, dev, say

pytestmark = pytest.mark.gpu

KS = (1, 3, 4, 9, 16)


def _matrices():
    """(name, matrix, [(kind, handle factory, oracle kernel)])."""
    out = []
    for name, m in (("7-point 12^3", synth.heptadiagonal(12, 1)),
                    ("27-point 11^3 octant drops", synth.partially_diagonal(11, 4)),
                    ("random 300", synth.random_csr(300, 5, density=0.02))):
        ref_b = oracle.mhdc_from_csr(m.rowptr, m.colind, m.val, 64, 0.6)
        ref_h = oracle.hdc_from_csr(m.rowptr, m.colind, m.val, 0.6)
        out.append((name, m, [
            ("M-HDC", lambda d: mhdc.MHDCMatrix.from_csr(*d, 64, 0.6),
             lambda x, r=ref_b: oracle.mhdc_spmv(r, x)),
            ("HDC", lambda d: mhdc.HDCMatrix.from_csr(*d, 0.6),
             lambda x, r=ref_h: oracle.hdc_spmv(r, x)),
            ("CSR", lambda d: mhdc.CSRMatrix.from_csr(*d),
             lambda x, m=m: oracle.csr_spmv(m.rowptr, m.colind, m.val, x, 0)),
        ]))
    return out


def test_spmm_ws_matches_oracle():
    """Routes 0, 1 and 2 for k in KS on matrices whose row counts leave a
    ragged last tile of the transposition (1331 rows: 5 x 256 + 51):
    every column is the oracle kernel's, bit for bit."""
    for name, m, kinds in _matrices():
        d = dev(m)
        for kind, make, want_fn in kinds:
            h = make(d)
            for k in KS:
                Xn = synth.vector(m.n, 40 + k, k) if k > 1 else synth.vector(m.n, 40)[:, None]
                X = torch.from_numpy(np.ascontiguousarray(Xn.T)).cuda()
                want = [want_fn(np.ascontiguousarray(Xn[:, r])) for r in range(k)]
                ws = torch.empty(h.workspace_bytes(k), dtype=torch.uint8, device="cuda")
                for route in (0, 1, 2):
                    say("case: spmm_ws %s %s k=%d route %d" % (name, kind, k, route))
                    Y = torch.full((k, m.n), float("nan"), dtype=torch.float64, device="cuda")
                    h.spmm_ws(X, Y, route=route, ws=ws)
                    for r in range(k):
                        assert_oracle_bits(Y[r], want[r], "%s %s k=%d route %d column %d" % (
                            name, kind, k, route, r))
            h.close()


def _lone_per_row(ptr, col):
    """Entries per row with no column within 16 in either of the two
    previous rows (rows before the first hold none): brute force."""
    ptr = np.asarray(ptr, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    n = len(ptr) - 1
    lone = 0
    for i in range(n):
        near = np.concatenate([col[ptr[i - 1]:ptr[i]] if i >= 1 else col[:0],
                               col[ptr[i - 2]:ptr[i - 1]] if i >= 2 else col[:0]])
        for j in col[ptr[i]:ptr[i + 1]]:
            if near.size == 0 or not np.any(np.abs(near - j) <= 16):
                lone += 1
    return lone / n if n else 0.0


def test_lone_count_and_route_rule():
    """lone_per_row of the CSR part equals the host brute force exactly;
    the default route is 2 exactly when k >= 2 and k * lone_per_row >= 2."""
    cases = [("7-point 12^3", synth.heptadiagonal(12, 1)),
             ("27-point 10^3 octant drops", synth.partially_diagonal(10, 2)),
             ("27-point 10^3 one random column", synth.partially_diagonal(
                 10, 3, drop=0.0, extra_per_row=1)),
             ("random 300", synth.random_csr(300, 5, density=0.02)),
             ("banded 3-point", synth.banded_stencil(4000, 3, 1))]
    seen = set()
    for name, m in cases:
        d = dev(m)
        for kind, h in (("CSR", mhdc.CSRMatrix.from_csr(*d)),
                        ("M-HDC", mhdc.MHDCMatrix.from_csr(*d, 64, 0.6))):
            say("case: lone count %s %s" % (name, kind))
            inf = h.info()
            if kind == "CSR":
                want = _lone_per_row(m.rowptr, m.colind)
            else:
                t = h.export()
                want = _lone_per_row(t["rem_ptr"].cpu().numpy(), t["rem_col"].cpu().numpy())
            assert inf["lone_per_row"] == want, (name, kind, inf["lone_per_row"], want)
            for k in range(1, 17):
                route = 2 if (k >= 2 and inf["R"] > 0 and want * k >= 2.0) else 1
                assert h.ws_route(k) == route, (name, kind, k)
                seen.add(route)
            h.close()
    assert seen == {1, 2}


def test_spmm_ws_strides_and_errors():
    """Leading dimensions above n on route 2 (same bits as mhdc_spmm), and
    the refusals: workspace too small, misaligned or overlapping X or Y, a
    route outside 0..2; route 1 needs no workspace."""
    m = synth.partially_diagonal(9, 6, drop=0.0, extra_per_row=2)
    d = dev(m)
    h = mhdc.MHDCMatrix.from_csr(*d, 32, 0.6)
    n, k, ldx, ldy = m.n, 5, m.n + 37, m.n + 3
    lib = mhdc.lib()
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    Xb = torch.rand((k, ldx), dtype=torch.float64, device="cuda")
    Yb = torch.full((k, ldy), -7.0, dtype=torch.float64, device="cuda")
    need = h.workspace_bytes(k)
    assert need == n * 6 * 8
    ws = torch.empty(need + 512, dtype=torch.uint8, device="cuda")
    assert ws.data_ptr() % 256 == 0
    vp = lambda t, off=0: ctypes.c_void_p(t.data_ptr() + off)

    say("case: spmm_ws strided route 2")
    rc = lib.mhdc_spmm_ws(h._h, vp(Xb), ldx, vp(Yb), ldy, k, 2, vp(ws), need, s)
    assert rc == 0, mhdc.lib().mhdc_last_error_message()
    Xc = Xb[:, :n].contiguous()
    Yc = h.spmm(Xc)
    assert torch.equal(Yb[:, :n].contiguous().view(torch.int64), Yc.view(torch.int64))
    assert bool((Yb[:, n:] == -7.0).all()), "padding of Y written"

    say("case: spmm_ws refusals")
    bad = [("too small", (vp(Xb), ldx, vp(Yb), ldy, k, 2, vp(ws), need - 1)),
           ("NULL", (vp(Xb), ldx, vp(Yb), ldy, k, 2, None, need)),
           ("misaligned", (vp(Xb), ldx, vp(Yb), ldy, k, 2, vp(ws, 16), need)),
           ("route 3", (vp(Xb), ldx, vp(Yb), ldy, k, 3, vp(ws), need)),
           ("route -1", (vp(Xb), ldx, vp(Yb), ldy, k, -1, vp(ws), need)),
           ("k 17", (vp(Xb), ldx, vp(Yb), ldy, 17, 2, vp(ws), need)),
           ("ldx < n", (vp(Xb), n - 1, vp(Yb), ldy, k, 2, vp(ws), need))]
    big = torch.empty(need + k * ldx * 8 + 256, dtype=torch.uint8, device="cuda")
    Xin = big[:k * ldx * 8].view(torch.float64).view(k, ldx)
    Xin.copy_(Xb)
    off = (k * ldx * 8 + 255) // 256 * 256  # first aligned byte past X
    bad.append(("ws overlaps X", (vp(Xin), ldx, vp(Yb), ldy, k, 2, vp(big), need)))
    bad.append(("ws overlaps Y", (vp(Xin), ldx, vp(Yb), ldy, k, 2, vp(Yb), need)))
    for what, args in bad:
        rc = lib.mhdc_spmm_ws(h._h, *args, s)
        assert rc == -1, (what, rc)
    rc = lib.mhdc_spmm_ws(h._h, vp(Xin), ldx, vp(Yb), ldy, k, 2, vp(big, off), need, s)
    assert rc == 0, "workspace right after X"
    Yb.fill_(0.0)
    rc = lib.mhdc_spmm_ws(h._h, vp(Xb), ldx, vp(Yb), ldy, k, 1, None, 0, s)
    assert rc == 0, "route 1 without workspace"
    assert torch.equal(Yb[:, :n].contiguous().view(torch.int64), Yc.view(torch.int64))
    torch.cuda.synchronize()
    h.close()


def test_spmm_ws_empty_and_tiny():
    """n = 0 and n = 1 on route 2 (one partial transposition tile)."""
    e = mhdc.CSRMatrix.from_csr(torch.zeros(1, dtype=torch.int32, device="cuda"),
                                torch.zeros(0, dtype=torch.int32, device="cuda"),
                                torch.zeros(0, dtype=torch.float64, device="cuda"))
    assert e.workspace_bytes(4) == 0
    X = torch.zeros((4, 0), dtype=torch.float64, device="cuda")
    e.spmm_ws(X, torch.zeros_like(X), route=2, ws=torch.empty(0, dtype=torch.uint8,
                                                              device="cuda"))
    e.close()
    rp = torch.tensor([0, 1], dtype=torch.int32, device="cuda")
    ci = torch.tensor([0], dtype=torch.int32, device="cuda")
    v = torch.tensor([3.0], dtype=torch.float64, device="cuda")
    for h in (mhdc.CSRMatrix.from_csr(rp, ci, v), mhdc.MHDCMatrix.from_csr(rp, ci, v, 1, 1.0)):
        X = torch.tensor([[1.5], [-2.0], [0.25], [8.0], [1e-300]], dtype=torch.float64,
                         device="cuda")
        Y = h.spmm_ws(X, route=2)
        assert torch.equal(Y, 3.0 * X)
        h.close()


def _random_case(seed):
    """One seeded case: a matrix of a random family and size, a format, k
    and padded leading dimensions."""
    rng = np.random.default_rng(seed)
    fam = int(rng.integers(0, 3))
    if fam == 0:
        n = int(rng.integers(1, 1500))
        m = synth.random_csr(n, seed, density=float(rng.uniform(0.001, 0.02)),
                             bands=tuple(int(b) for b in rng.integers(-40, 40, size=3)))
    elif fam == 1:
        m = synth.partially_diagonal(int(rng.integers(3, 13)), seed,
                                     drop=float(rng.uniform(0, 0.6)),
                                     extra_per_row=int(rng.integers(0, 3)))
    else:
        m = synth.banded_stencil(int(rng.integers(1, 5000)), int(rng.choice([3, 5, 7])), seed)
    fmt = ("M-HDC", "HDC", "CSR")[int(rng.integers(0, 3))]
    n_b = int(rng.choice([1, 7, 32, 64, 256]))
    theta = float(rng.choice([0.3, 0.6, 0.9]))
    k = int(rng.integers(1, 17))
    ldx = m.n + int(rng.integers(0, 40))
    ldy = m.n + int(rng.integers(0, 40))
    return m, fmt, n_b, theta, k, ldx, ldy


@pytest.mark.parametrize("seed", range(24))
def test_spmm_ws_random_shapes(seed):
    """Seeded random matrices, formats, k and leading dimensions: routes
    0, 1 and 2 equal mhdc_spmm bit for bit (the padding of Y untouched), and
    the last column equals the oracle's sequential kernel."""
    m, fmt, n_b, theta, k, ldx, ldy = _random_case(seed)
    say("case: spmm_ws random seed %d: %s n=%d nnz=%d n_b=%d theta=%.1f k=%d ldx=%d ldy=%d" % (
        seed, fmt, m.n, m.nnz, n_b, theta, k, ldx, ldy))
    d = dev(m)
    if fmt == "M-HDC":
        h = mhdc.MHDCMatrix.from_csr(*d, n_b, theta)
        want_last = lambda x: oracle.mhdc_spmv(  # noqa: E731
            oracle.mhdc_from_csr(m.rowptr, m.colind, m.val, n_b, theta), x)
    elif fmt == "HDC":
        h = mhdc.HDCMatrix.from_csr(*d, theta)
        want_last = lambda x: oracle.hdc_spmv(  # noqa: E731
            oracle.hdc_from_csr(m.rowptr, m.colind, m.val, theta), x)
    else:
        h = mhdc.CSRMatrix.from_csr(*d)
        want_last = lambda x: oracle.csr_spmv(m.rowptr, m.colind, m.val, x, 0)  # noqa: E731
    lib = mhdc.lib()
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    Xb = torch.rand((k, ldx), dtype=torch.float64, device="cuda", generator=g) - 0.5
    Xc = Xb[:, :m.n].contiguous()
    ref = h.spmm(Xc)
    ws = torch.empty(h.workspace_bytes(k) + 256, dtype=torch.uint8, device="cuda")
    for route in (0, 1, 2):
        Yb = torch.full((k, ldy), -3.0, dtype=torch.float64, device="cuda")
        rc = lib.mhdc_spmm_ws if fmt == "M-HDC" else (
            lib.hdc_spmm_ws if fmt == "HDC" else lib.csr_spmm_ws)
        r = rc(h._h, ctypes.c_void_p(Xb.data_ptr()), ldx, ctypes.c_void_p(Yb.data_ptr()), ldy,
               k, route, ctypes.c_void_p(ws.data_ptr()), ws.numel(), s)
        assert r == 0, mhdc.lib().mhdc_last_error_message()
        assert torch.equal(Yb[:, :m.n].contiguous().view(torch.int64), ref.view(torch.int64)), route
        assert bool((Yb[:, m.n:] == -3.0).all()), route
    if m.n > 0:
        x_last = Xc[k - 1].cpu().numpy()
        assert_oracle_bits(ref[k - 1], want_last(x_last), "last column")
    h.close()


def test_spmm_ws_graph_replay():
    """Route 2 captured in a graph (it allocates nothing and records no
    memset): four replays on fresh inputs, with eager work and
    synchronisations between them, each equal to the eager column-major
    product bit for bit."""
    m = synth.partially_diagonal(11, 4)
    h = mhdc.MHDCMatrix.from_csr(*dev(m), 64, 0.6)
    assert h.info()["R"] > 0
    k = 8
    g = torch.Generator(device="cuda")
    g.manual_seed(11)
    X = torch.rand((k, m.n), dtype=torch.float64, device="cuda", generator=g)
    Y = torch.empty_like(X)
    ws = torch.empty(h.workspace_bytes(k), dtype=torch.uint8, device="cuda")
    h.spmm_ws(X, Y, route=2, ws=ws)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    say("case: spmm_ws graph capture")
    with torch.cuda.graph(graph):
        h.spmm_ws(X, Y, route=2, ws=ws)
    for rep in range(4):
        say("case: spmm_ws graph replay %d" % rep)
        X.copy_(torch.rand((k, m.n), dtype=torch.float64, device="cuda", generator=g))
        want = h.spmm(X)
        Y.fill_(float("nan"))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(Y.view(torch.int64), want.view(torch.int64)), rep
    del graph
    h.close()


@pytest.fixture(scope="module")
def full_matrices():
    """The two full-size matrices, generated once for the module."""
    say("generating partially diagonal 27-point 192^3 and heptadiagonal 256^3")
    return {"partial192": synth.partially_diagonal(192, 3), "hepta256": synth.heptadiagonal(256, 2)}


@pytest.mark.slow
@pytest.mark.parametrize("case", ["partial192 M-HDC", "partial192 HDC", "partial192 CSR",
                                  "hepta256 M-HDC"])
def test_spmm_ws_full_size_16(case, full_matrices):
    """16 right-hand sides at full size: on the partially diagonal 192^3
    matrix (n_b = 128) every handle's default route is the row-major one; on
    the heptadiagonal 256^3 matrix (n_b = 256, no CSR part) route 2 is
    forced, which stores Y by column straight from the lanes.  Every column
    equals the column-major kernel's bits (itself pinned to the oracle at
    these sizes), and column 0 the oracle's sequential kernel of the
    handle's format (Figs. 3, 8, 16)."""
    name, fmt = case.split()
    say("case: spmm_ws full size %s" % case)
    m = full_matrices[name]
    d = dev(m)
    nb = 128 if name == "partial192" else 256
    if fmt == "M-HDC":
        h = mhdc.MHDCMatrix.from_csr(*d, nb, 0.6)
    elif fmt == "HDC":
        h = mhdc.HDCMatrix.from_csr(*d, 0.6)
    else:
        h = mhdc.CSRMatrix.from_csr(*d)
    del d
    k = 16
    route = 0 if name == "partial192" else 2
    if route == 0:
        assert h.ws_route(k) == 2
    X = torch.empty((k, m.n), dtype=torch.float64, device="cuda")
    x0 = synth.vector(m.n, 3)
    X[0] = torch.from_numpy(x0).cuda()
    for r in range(1, k):
        X[r] = torch.from_numpy(synth.vector(m.n, 100 + r)).cuda()
    Yd = h.spmm(X)
    Y = h.spmm_ws(X, route=route)
    assert torch.equal(Y.view(torch.int64), Yd.view(torch.int64))
    del Yd
    if fmt == "M-HDC":
        want = oracle.mhdc_spmv(oracle.mhdc_from_csr(m.rowptr, m.colind, m.val, nb, 0.6), x0)
    elif fmt == "HDC":
        want = oracle.hdc_spmv(oracle.hdc_from_csr(m.rowptr, m.colind, m.val, 0.6), x0)
    else:
        want = oracle.csr_spmv(m.rowptr, m.colind, m.val, x0, 0)
    assert_oracle_bits(Y[0], want, "column 0")
    h.close()
