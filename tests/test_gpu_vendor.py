"""rocSPARSE's CSR SpMV (the vendor GPU kernel that stands beside this
library's CSR baseline, as the paper's Intel MKL comparison does in
Sec. 6.4.4) checked against the CPU oracle element by element on the two
full-size workloads: |y - y_ref|_i <= 1e-13 (|A||x|)_i, plain and after
analysis.  Skipped where librocsparse.so is not installed."""
import numpy as np
import pytest
import torch

import oracle
from paper_2105_04937_amd import mhdc, synth, vendor
from tests.gpu_helpers import assert_spmv_close, say

pytestmark = [pytest.mark.gpu, pytest.mark.slow,
              pytest.mark.skipif(not vendor.available(),
                                 reason="librocsparse.so is not installed under ROCM_PATH")]


@pytest.mark.parametrize("name", ["hepta256", "partial192"])
def test_rocsparse_matches_oracle(name):
    say("case: rocSPARSE csrmv vs oracle, %s" % name)
    if name == "hepta256":
        m, seed = synth.heptadiagonal(256, 2), 2
    else:
        m, seed = synth.partially_diagonal(192, 3), 3
    x = synth.vector(m.n, seed)
    yref = oracle.csr_spmv(m.rowptr, m.colind, m.val, x, 0)
    scale = oracle.csr_absmv(m.rowptr, m.colind, m.val, x)
    rp, ci, v = mhdc.to_device(m)
    xd = torch.from_numpy(x).cuda()
    s = torch.cuda.current_stream()
    rs = vendor.RocSparse(s)
    for analysed in (False, True):
        info = rs.analysis(m.n, m.nnz, rp, ci, v) if analysed else None
        y = torch.full_like(xd, float("nan"))
        rs.csrmv(m.n, m.nnz, rp, ci, v, info, xd, y)
        torch.cuda.synchronize()
        assert_spmv_close(y, m, x, Y_ref=yref, absAx=scale)
        rs.free_info(info)
    rs.close()
