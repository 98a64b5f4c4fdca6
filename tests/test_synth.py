"""Checks of the seeded input generators: the PCA motion model (eq. (1),
section 2.1; section 3's 9 training DVFs) against a direct SVD of the training
matrix, its exactness for the rank-R analytic motion, and phantom determinism."""
import numpy as np
import pytest

from paper_1004_0014_amd import synth as S


@pytest.mark.parametrize("K", [2, 3, 4, 5])
def test_pca_matches_direct_svd(K):
    g = S.Grid((20, 18, 16), (6.0, 6.0, 8.0))
    m = S.pca_model(g, K)
    phis = 2 * np.pi * np.arange(1, 10) / 10
    X = np.stack([S.analytic_dvf(g, p, K).ravel() for p in phis], 1)
    Xc = X - X.mean(1, keepdims=True)
    u, s, _ = np.linalg.svd(Xc, full_matrices=False)
    np.testing.assert_allclose(m.sing[:K], s[:K], rtol=1e-10)
    assert s[K] < 1e-10 * s[0]                       # the motion has rank K exactly
    assert np.all(s[:K - 1] > 1.05 * s[1:K])         # distinct: directions well defined
    Uf = m.U.reshape(K, -1)
    np.testing.assert_allclose(Uf @ Uf.T, np.eye(K), atol=1e-12)
    for k in range(K):
        a = np.abs(u[:, k])
        j = np.flatnonzero(a >= (1 - 1e-5) * a.max())[0]
        uk = u[:, k] * np.sign(u[j, k])                 # sign rule
        np.testing.assert_allclose(Uf[k], uk, atol=1e-10)
    np.testing.assert_allclose(m.mean.ravel(), X.mean(1), atol=1e-12)
    np.testing.assert_allclose(m.w_train, Xc.T @ Uf.T, atol=1e-9)


def test_test_motion_lies_in_model_span():
    g = S.Grid((16, 16, 12), (8.0, 8.0, 10.0))
    m = S.pca_model(g, 3)
    for phi in (0.3, 2.0, 4.4):
        w = S.truth_w(m, phi, 1.5)
        x = m.mean + np.tensordot(w, m.U, axes=(0, 0))
        np.testing.assert_allclose(x, S.analytic_dvf(g, phi, 3, 1.5), atol=1e-10)


def test_phantom_deterministic_and_bounded():
    g = S.grid_for("tiny")
    a = S.phantom(g, seed=0)
    b = S.phantom(g, seed=0)
    assert np.array_equal(a, b)
    assert not np.array_equal(a, S.phantom(g, seed=1))
    assert a.min() >= 0.0 and 0.015 < a.max() < 0.03
    # body, lung and tumour levels present
    flat = S.phantom(g, texture=0.0)
    assert set(np.unique(flat)) == {0.0, 0.004, 0.02}
    tc = S.tumor_center(g)
    i = np.round((tc - np.array(g.origin)) / np.array(g.spacing)).astype(int)
    assert flat[i[2], i[1], i[0]] == 0.02


def test_oracle_pca_matches_pattern_pca():
    """oracle.pca (direct SVD of the centred training matrix) against the
    input generator's exact Gram-matrix PCA: same mean, fields, singular
    values and training coefficients."""
    import oracle
    g = S.Grid((18, 16, 12), (6.0, 6.0, 8.0))
    for K in (3, 5):
        m = S.pca_model(g, K)
        phis = 2 * np.pi * np.arange(1, 10) / 10
        d = np.stack([S.analytic_dvf(g, p, K) for p in phis])
        mean, U, sing, wt = oracle.pca(d, K)
        np.testing.assert_allclose(mean, m.mean, atol=1e-12)
        np.testing.assert_allclose(U, m.U, atol=1e-10)
        np.testing.assert_allclose(sing, m.sing[:K], rtol=1e-10)
        np.testing.assert_allclose(wt, m.w_train, atol=1e-8)


def test_training_dvfs_are_the_model_phases():
    """The stacked training DVFs are the analytic motion at the model's
    training phases (rounded to FP32)."""
    g = S.Grid((10, 9, 7), (6.0, 6.0, 8.0))
    d = S.training_dvfs(g, 3)
    assert d.dtype == np.float32 and d.shape == (9, 3) + g.shape
    for j in range(9):
        ref = S.analytic_dvf(g, 2 * np.pi * (j + 1) / 10, 3)
        np.testing.assert_allclose(d[j], ref, rtol=1e-6, atol=1e-6 * np.abs(ref).max())
