"""The selector's host-side rules, exported by the library and callable
without a GPU: the byte-model judge of mhdc_select and the candidate list
of mhdc_select_refine (the grid of Sec. 6.4.1 around a decision).  The
offline evaluation (learned.evaluate) calls the same functions."""
import os

import pytest

from tests.conftest import ROOT

LIB = os.path.join(ROOT, "paper_2105_04937_amd", "libmhdc.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libmhdc.so not built")


def test_judge_keep():
    from paper_2105_04937_amd import mhdc
    assert mhdc.judge_keep(100.0, 80.0, 0.25)
    assert not mhdc.judge_keep(100.0 + 1e-9, 80.0, 0.25)
    assert mhdc.judge_keep(80.0, 80.0, 0.0)
    assert not mhdc.judge_keep(81.0, 80.0, 0.0)
    assert mhdc.judge_keep(1e12, 1.0, 1e12)


@pytest.mark.parametrize("decision,want", [
    ((0.5, 64), [(0.5, 32), (0.5, 128), (0.6, 64), (0.6, 256), (0.5, 4096)]),
    ((0.6, 256), [(0.6, 128), (0.6, 512), (0.5, 256), (0.7, 256), (0.6, 4096)]),
    ((0.9, 4096), [(0.9, 2048), (0.8, 4096), (0.6, 256)]),
    ((0.5, 32), [(0.5, 64), (0.6, 32), (0.6, 256), (0.5, 4096)]),
    ((0.7, 2048), [(0.7, 1024), (0.7, 4096), (0.6, 2048), (0.8, 2048), (0.6, 256)]),
])
def test_refine_candidates(decision, want):
    """Halved / doubled n_b, theta -+ 0.1, the policy (0.6, 256) and the
    decision's theta at n_b = 4096, inside theta 0.5..0.9 and n_b 32..4096,
    each once and never the decision itself."""
    from paper_2105_04937_amd import mhdc
    assert mhdc.refine_candidates(*decision) == want

