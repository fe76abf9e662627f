"""Batched persistent launch, HIP-graph replay and the autotuner, through the
C-ABI.  Every item of a batch must equal its single-matrix launch bit for bit
and the oracle's sequential M-HDC kernel (Fig. 16) bit for bit."""
import numpy as np
import pytest
import torch

import oracle
from paper_2105_04937_amd import mhdc, synth
from tests.gpu_helpers import assert_oracle_bits, assert_same_bits, assert_spmv_close, dev, say

pytestmark = pytest.mark.gpu


def _items():
    """Mixed workload: batch members (7/19/27-point, drops, k = 1..16), a
    matrix without remainder, one with only a remainder, a tiny one, one
    with a ragged last block."""
    out = []
    for i in (0, 1, 2, 3, 5, 8):
        m, k = synth.batch_member(i)
        out.append((m, k, [64, 128, 32, 256, 64, 48][len(out) % 6]))
    out.append((synth.laplacian7(20), 3, 400))            # R = 0
    out.append((synth.random_csr(300, 5, density=0.02), 2, 64))  # mostly remainder
    out.append((synth.random_csr(5, 6, density=0.5, bands=[0]), 16, 4))
    out.append((synth.partially_diagonal(13, 7), 9, 100))  # 2197 rows, ragged last block
    return out


@pytest.fixture(scope="module")
def batch_case():
    items = _items()
    say("batch: %d items, rows %s" % (len(items), [m.n for m, _, _ in items]))
    mats, Xs, refs, devs = [], [], [], []
    for j, (m, k, nb) in enumerate(items):
        d = dev(m)
        devs.append(d)
        mats.append(mhdc.MHDCMatrix.from_csr(*d, nb, 0.6))
        X = np.ascontiguousarray(np.random.default_rng(100 + j).uniform(-1, 1, size=(k, m.n)))
        Xs.append(torch.from_numpy(X).cuda())
        refs.append(oracle.mhdc_from_csr(m.rowptr, m.colind, m.val, nb, 0.6))
    return items, mats, Xs, refs, devs


def _check_items(items, mats, Xs, Ys, refs):
    torch.cuda.synchronize()
    for (m, k, nb), mat, X, Y, ref in zip(items, mats, Xs, Ys, refs):
        Xh = X.cpu().numpy()
        Yh = Y.cpu().numpy()
        single = mat.spmm(X).cpu().numpy()
        assert_same_bits(Yh, single, "batch item n=%d vs single launch" % m.n)
        for r in range(k):
            assert_oracle_bits(Yh[r], oracle.mhdc_spmv(ref, Xh[r]), "item n=%d rhs %d" % (m.n, r))
            assert_spmv_close(Yh[r], m, Xh[r])


def test_batch_run_matches_items(batch_case):
    items, mats, Xs, refs, _ = batch_case
    for wg in (256, 64):
        say("case: batch run wg=%d" % wg)
        b = mhdc.Batch(mats, Xs, wg_size=wg)
        inf = b.info()
        assert inf["count"] == len(items) and inf["grid"] >= 1
        assert inf["total_tiles"] == sum((m.n + wg - 1) // wg for m, _, _ in items)
        b.run()
        _check_items(items, mats, Xs, b.Ys, refs)
        b.close()


def test_batch_rowmajor_matches_items(batch_case):
    """Right-hand sides stored row by row: every item equals its own
    mhdc_spmm_rowmajor launch and the oracle's Fig. 16 kernel bit for bit,
    in a plain run and in a graph replay, for both workgroup sizes."""
    items, mats, Xs, refs, _ = batch_case
    Xr = [X.t().contiguous() for X in Xs]   # (n_i, k_i), row-major
    for wg in (256, 64):
        say("case: row-major batch wg=%d" % wg)
        b = mhdc.Batch(mats, Xr, wg_size=wg, layout="rowmajor")
        b.run()
        torch.cuda.synchronize()
        for (m, k, nb), mat, X, Y, ref in zip(items, mats, Xr, b.Ys, refs):
            single = mat.spmm_rowmajor(X)
            assert_same_bits(Y.cpu().numpy(), single.cpu().numpy(),
                             "row-major item n=%d vs single launch" % m.n)
            Xh, Yh = X.cpu().numpy(), Y.cpu().numpy()
            for r in range(k):
                assert_oracle_bits(np.ascontiguousarray(Yh[:, r]),
                                   oracle.mhdc_spmv(ref, np.ascontiguousarray(Xh[:, r])),
                                   "row-major item n=%d rhs %d" % (m.n, r))
        got = [Y.clone() for Y in b.Ys]
        for Y in b.Ys:
            Y.fill_(float("nan"))
        stream = torch.cuda.Stream()
        b.graph_launch(stream)
        stream.synchronize()
        for g, Y in zip(got, b.Ys):
            assert_same_bits(g.cpu().numpy(), Y.cpu().numpy(), "row-major graph replay")
        b.close()
    with pytest.raises(ValueError):
        mhdc.Batch(mats, Xs, layout="rowmajor")   # column-major shapes


def test_batch_graph_replays(batch_case):
    """Replay the captured graph several times with eager work in between;
    every replay must equal the eager batch result for the current X."""
    items, mats, Xs0, refs, _ = batch_case
    say("case: batch graph replays")
    Xs = [X.clone() for X in Xs0]
    b = mhdc.Batch(mats, Xs)
    stream = torch.cuda.Stream()
    for rep in range(4):
        with torch.cuda.stream(stream):
            for X in Xs:
                X.mul_(-1.25).add_(0.125)  # eager work on the same stream
            b.graph_launch(stream)
        stream.synchronize()
        got = [Y.clone() for Y in b.Ys]
        b.run()
        torch.cuda.synchronize()
        for g, Y in zip(got, b.Ys):
            assert_same_bits(g.cpu().numpy(), Y.cpu().numpy(), "replay %d" % rep)
    _check_items(items, mats, Xs, b.Ys, refs)
    # rebind to fresh tensors: the graph reads the new table
    Xs2 = [torch.flip(X, dims=[1]).contiguous() for X in Xs]
    Ys2 = [torch.empty_like(X) for X in Xs2]
    b.bind(Xs2, Ys2)
    b.graph_launch()
    _check_items(items, mats, Xs2, Ys2, refs)
    b.close()


def test_batch_tune_and_errors(batch_case):
    items, mats, Xs, refs, _ = batch_case
    say("case: batch tune + errors")
    b = mhdc.Batch(mats, Xs)
    wg, us = b.tune()
    assert wg in (64, 256) and us > 0
    b.run()
    _check_items(items, mats, Xs, b.Ys, refs)
    b.close()
    bad = [torch.zeros((17, mats[0].n), dtype=torch.float64, device="cuda")] + Xs[1:]
    with pytest.raises(ValueError):
        mhdc.Batch(mats, bad[:1] + Xs[1:], Ys=[torch.zeros(1, device="cuda")] + Xs[1:])
    with pytest.raises(mhdc.MhdcError) as e:
        mhdc.Batch(mats, bad)
    assert e.value.name == "MHDC_ERR_INVALID_ARG"
    with pytest.raises(mhdc.MhdcError) as e:   # Y_i aliases X_i
        mhdc.Batch(mats, Xs, Ys=Xs)
    assert e.value.name == "MHDC_ERR_INVALID_ARG"
    # a refused rebinding leaves the batch with its previous binding: it
    # still runs, and a later workgroup-size change rebuilds from it
    b = mhdc.Batch(mats, Xs)
    with pytest.raises(mhdc.MhdcError) as e:
        b.bind(Xs, Xs)
    assert e.value.name == "MHDC_ERR_INVALID_ARG"
    b.run()
    _check_items(items, mats, Xs, b.Ys, refs)
    b.set_wg(64)
    assert b.info()["wg_size"] == 64
    for Y in b.Ys:
        Y.fill_(float("nan"))
    b.run()
    _check_items(items, mats, Xs, b.Ys, refs)
    b.close()


def test_batch_schedule_small_counts_and_rebuild(batch_case):
    """Batches of fewer members than XCDs (the XCDs without members take
    others' tiles from the start) and one of more: every tile is taken
    exactly once (outputs start as NaN) and every member equals its single
    launch and the oracle.  A workgroup-size change replaces the schedule:
    graph replays before and after it, and back, give the same results."""
    items, mats, Xs, refs, _ = batch_case
    for sel in ([0], [6, 8, 9], list(range(9))):
        say("case: batch schedule, members %s" % sel)
        its = [items[i] for i in sel]
        Ys = [torch.full_like(Xs[i], float("nan")) for i in sel]
        b = mhdc.Batch([mats[i] for i in sel], [Xs[i] for i in sel], Ys=Ys)
        b.run()
        _check_items(its, [mats[i] for i in sel], [Xs[i] for i in sel], Ys, [refs[i] for i in sel])
        b.close()
    say("case: batch schedule rebuilt by set_wg under graph replay")
    Ys = [torch.full_like(X, float("nan")) for X in Xs]
    b = mhdc.Batch(mats, Xs, Ys=Ys)
    b.graph_launch()
    _check_items(items, mats, Xs, Ys, refs)
    for wg in (64, 256):
        b.set_wg(wg)
        for Y in Ys:
            Y.fill_(float("nan"))
        b.graph_launch()
        b.graph_launch()
        _check_items(items, mats, Xs, Ys, refs)
    b.close()


@pytest.mark.parametrize("k", [1, 4])
def test_autotune(k):
    m = synth.partially_diagonal(40, 17, drop=0.15)
    say("case: autotune n=%d k=%d" % (m.n, k))
    d = dev(m)
    cands = (32, 64, 128, 256)
    h, res = mhdc.autotune(*d, 0.6, nrhs=k, nb_candidates=cands)
    assert res["n_b"] in cands and res["tried"] >= len(cands) * 3 and res["us"] > 0
    inf = h.info()
    assert inf["n_b"] == res["n_b"]
    assert (inf["rows_per_lane"], inf["wg_size"], inf["xcd_remap"], inf["csr_mode"],
            inf["rhs_group"]) == res["launch"]
    ref = oracle.mhdc_from_csr(m.rowptr, m.colind, m.val, res["n_b"], 0.6)
    X = np.ascontiguousarray(np.random.default_rng(k).uniform(-1, 1, size=(k, m.n)))
    Y = h.spmm(torch.from_numpy(X).cuda()).cpu().numpy()
    for r in range(k):
        assert_oracle_bits(Y[r], oracle.mhdc_spmv(ref, X[r]), "autotuned rhs %d" % r)


def test_full_batch_configuration():
    """The benchmarked batch at its full size: 64 members (grid side
    U{16..96}, 7/19/27 points, drop U[0, 0.3], k = U{1..16}; matrix i from
    seed 4000 + i), n_b = 256, theta = 0.6.  One graph replay equals the 64
    single launches bit for bit, and for every eighth member each column
    equals the oracle's sequential M-HDC kernel (Fig. 16) bit for bit."""
    say("case: full 64-member batch")
    mats, Xs, members = [], [], []
    for i in range(64):
        m, k = synth.batch_member(i)
        mats.append(mhdc.MHDCMatrix.from_csr(*dev(m), 256, 0.6))
        X = np.random.default_rng([4000 + i, 2]).uniform(-1, 1, size=(k, m.n))
        Xs.append(torch.from_numpy(np.ascontiguousarray(X)).cuda())
        members.append((m, k))
    b = mhdc.Batch(mats, Xs)
    stream = torch.cuda.Stream()
    b.graph_launch(stream)
    stream.synchronize()
    for j, ((m, k), mat, X, Y) in enumerate(zip(members, mats, Xs, b.Ys)):
        single = mat.spmm(X)
        assert_same_bits(Y.cpu().numpy(), single.cpu().numpy(), "member %d vs single" % j)
        if j % 8 == 0:
            ref = oracle.mhdc_from_csr(m.rowptr, m.colind, m.val, 256, 0.6)
            Xh, Yh = X.cpu().numpy(), Y.cpu().numpy()
            for r in range(k):
                assert_oracle_bits(Yh[r], oracle.mhdc_spmv(ref, Xh[r]), "member %d rhs %d" % (j, r))
    b.close()
    for mat in mats:
        mat.close()
