"""GPU PCA training of the motion model against the FP64 oracle PCA (direct
SVD of the centred training matrix) on the same FP32 training DVFs."""
import numpy as np
import pytest

import oracle
from paper_1004_0014_amd import synth as S
from helpers import rel_l2, rounded

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("K,n", [(3, (40, 36, 30)), (5, (33, 29, 21)), (2, (64, 64, 40))])
def test_pca_train_matches_oracle(K, n):
    from paper_1004_0014_amd import _lib
    g = S.Grid(n, (5.0, 5.5, 7.0))
    phis = 2 * np.pi * np.arange(1, 10) / 10
    d_t, d = rounded(np.stack([S.analytic_dvf(g, p, K) for p in phis]), torch.float32)
    mean, U, sing, wt = _lib.pca_train(g, d_t.cuda(), K)
    mo, Uo, so, wo = oracle.pca(d, K)
    assert rel_l2(mean.cpu().numpy(), mo) <= 1e-6
    for k in range(K):
        assert rel_l2(U[k].cpu().numpy(), Uo[k]) <= 2e-5, k
    np.testing.assert_allclose(sing, so, rtol=1e-6)
    np.testing.assert_allclose(wt, wo, rtol=1e-5, atol=1e-6 * np.abs(wo).max())
