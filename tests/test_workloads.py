"""Host checks of the seeded input generators (no GPU needed)."""
import numpy as np

from paper_2203_15031_amd import workloads as W


def test_sparse_regression_shape_and_coefficients():
    X, Y, beta = W.sparse_regression()
    assert X.shape == (250, 500) and Y.shape == (250, 2) and beta.shape == (500,)
    assert np.all(beta[:5] == 2.0) and np.all(beta[5:10] == -1.0) and np.all(beta[10:] == 0.0)
    assert Y.flags["C_CONTIGUOUS"]
    # the noise of each response has the stated scale (250 draws: within 20%)
    for r, s in enumerate((3.0, 5.0)):
        e = Y[:, r] - X @ beta
        assert abs(e.std() / s - 1.0) < 0.2


def test_sparse_regression_is_seeded():
    a = W.sparse_regression(n=40, p=30, sigmas=(1.0, 2.0, 4.0), seed=7)
    b = W.sparse_regression(n=40, p=30, sigmas=(1.0, 2.0, 4.0), seed=7)
    c = W.sparse_regression(n=40, p=30, sigmas=(1.0, 2.0, 4.0), seed=8)
    for u, v in zip(a, b):
        assert np.array_equal(u, v)
    assert not np.array_equal(a[0], c[0])
    assert a[1].shape == (40, 3)


def test_named_workloads_are_seeded_with_their_shapes():
    for name in ("ar1_n100_p200", "er_n200_p1000"):
        w = W.workload(name)
        X1 = W.generate(name)
        X2 = W.generate(name)
        assert X1.shape == (w.n, w.p)
        assert np.array_equal(X1, X2)
        assert np.all(np.isfinite(X1))


def test_exact_covariance_designs():
    # the designs with a prescribed sample covariance hold it to rounding
    X = W.star_band_design(n=200, arms=40, lambda0=0.15, gap=3e-5)
    n, p = X.shape
    S = X.T @ X / n
    assert np.abs(X.mean(0)).max() < 1e-12
    np.testing.assert_allclose(np.diag(S), 1.0, atol=1e-12)
    np.testing.assert_allclose(S[0, 1:41], 0.15 - 3e-5, atol=1e-12)
    assert np.abs(S[1:41, 1:41] - np.eye(40)).max() < 1e-12
    assert abs(S[41, 42] - 0.6) < 1e-12
