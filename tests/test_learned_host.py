"""Host logic of the selector's training pipeline (no GPU): the folding of
the input standardisation into the first layer."""
import numpy as np

from oracle import selector as S
from paper_2105_04937_amd import learned


def test_fold_standardisation_matches_standardised_inputs():
    """The folded first layer computes on raw features what the trained
    network computed on standardised ones (FP32 storage rounding aside), for
    both network kinds."""
    rng = np.random.default_rng(4)
    X = rng.uniform(0, 0.3, size=(50, 66))
    mu, sd = X.mean(0), X.std(0) + 1e-6
    for n_out, count in ((2, S.N_PARAMS), (40, S.N_PARAMS_SCORER)):
        p = S.init_params(3, n_out).astype(np.float64) + rng.normal(0, 0.05, count)
        want, _ = S.forward(p, (X - mu) / sd)
        got, _ = S.forward(learned.fold_standardisation(p, mu, sd).astype(np.float64), X)
        assert np.allclose(got, want, rtol=1e-4, atol=1e-4 * np.abs(want).max())
