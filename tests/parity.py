"""Comparison helpers shared by the GPU parity tests (no test functions here).

Tolerances follow the stated bar: normwise relative error
max |R_gpu - R_ref| / max |R_ref| per result, 1e-6 for the double form and
1e-4 for the mixed form, and an identical support away from the
threshold: oracle zeros whose KKT slack lambda_k - |g_jk| exceeds tau, and
oracle nonzeros with |beta_jk| > tau, must match (tau = the same bar).
"""
import numpy as np


def rel_err(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.abs(b).max()
    if den == 0:
        return float(np.abs(a).max())
    return float(np.abs(a - b).max() / den)


def standardized_cov(X):
    X = np.asarray(X, dtype=np.float64)
    Xs = (X - X.mean(0)) / X.std(0)
    return Xs.T @ Xs / X.shape[0]


def _mismatch(B_gpu, B_orc, G, sigma_orc, lambda0, tau, off):
    lam = lambda0 * np.asarray(sigma_orc)[None, :]
    orc_zero = (B_orc == 0) & off
    orc_nz = (B_orc != 0) & off
    sure_zero = orc_zero & ((lam - np.abs(G)) > tau)
    sure_nz = orc_nz & (np.abs(B_orc) > tau)
    mism = int(((B_gpu != 0) & sure_zero).sum() + ((B_gpu == 0) & sure_nz).sum())
    excluded = int(off.sum() - sure_zero.sum() - sure_nz.sum())
    return mism, excluded


def support_mismatch(B_gpu, B_orc, S, sigma_orc, lambda0, tau):
    """Entries outside the +-tau margin whose zero/nonzero status differs.

    B_* on the standardised scale; S the standardised covariance.  Oracle
    zeros need KKT slack lambda_k - |g_jk| > tau (g = S[:, k] - S beta_k),
    oracle nonzeros |beta_jk| > tau; both directions are checked.  Returns
    (n_mismatch, n_excluded)."""
    import scipy.sparse as sps
    G = S - np.asarray(sps.csc_matrix(B_orc).__rmatmul__(S))
    p = B_orc.shape[0]
    return _mismatch(B_gpu, B_orc, G, sigma_orc, lambda0, tau, ~np.eye(p, dtype=bool))


def standardize(X):
    X = np.asarray(X, dtype=np.float64)
    return (X - X.mean(0)) / X.std(0)


def support_mismatch_cols(B_gpu_cols, B_orc_cols, Xs, cols, sigma_orc_cols, lambda0, tau):
    """support_mismatch for the listed response columns only.

    B_*_cols: p x m (column i = beta of response cols[i], standardised
    scale); Xs: the standardised data.  The gradients g = Xs^T (x_k - Xs
    beta_k) / n are formed from the data, so S is never needed."""
    n, p = Xs.shape
    cols = np.asarray(cols)
    G = Xs.T @ (Xs[:, cols] - Xs @ B_orc_cols) / n
    off = np.ones((p, cols.size), dtype=bool)
    off[cols, np.arange(cols.size)] = False
    return _mismatch(B_gpu_cols, B_orc_cols, G, sigma_orc_cols, lambda0, tau, off)


def omega_invariants(Om, B, sigma_std=None):
    """Exact symmetry and the AND-rule support of the symmetrised estimate."""
    Om = np.asarray(Om)
    B = np.asarray(B)
    assert np.array_equal(Om, Om.T), "Omega is not bitwise symmetric"
    p = B.shape[0]
    off = ~np.eye(p, dtype=bool)
    both = (B != 0) & (B.T != 0)
    assert np.array_equal((Om != 0) & off, both & off), "Omega support is not the AND rule"
