"""GPU parity of the scaled-lasso entry (spmesl_scaled_lasso) against the oracle.

The entry treats each response as SPMESL treats one of its variables:
design and response columns centred and scaled to unit variance, response r
regressed on the design columns only by Algorithm 1, results unscaled by
Proposition 1.  The reference is the oracle's Algorithm 1 (exact mode,
tol 1e-13) on the oracle's standardised design and response, unscaled here.
Bar: normwise relative error 1e-6 (double form) and an identical support
away from the threshold.
"""
import ctypes as C
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from paper_2203_15031_amd import workloads as W
from tests.parity import rel_err

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
BAR = 1e-6


@pytest.fixture(scope="module")
def sp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2203_15031_amd import spmesl
    return spmesl


@pytest.fixture(scope="module")
def ctx(sp):
    c = sp.Context(0)
    yield c
    c.close()


def gpu(A):
    return torch.from_numpy(np.ascontiguousarray(A)).to(DEV)


def reference(X, Y, lam0):
    """Per response: (beta on the caller's scale, sigma on the caller's scale,
    beta and sigma of the standardised problem, standardised design and
    response)."""
    Xs, _, c = oracle.standardize(X)
    out = []
    for r in range(Y.shape[1]):
        ys2, _, cy = oracle.standardize(Y[:, r:r + 1])
        ys = ys2[:, 0]
        b, s, _, _, st = oracle.scaled_lasso(Xs, ys, lam0, tol=1e-13)
        assert st == 0
        out.append((b * c / cy[0], s / cy[0], b, s, Xs, ys))
    return out


def check(beta_gpu, sig_gpu, ref, lam0, scale):
    """Parity of one response against its reference."""
    b_orig, s_orig, b_std, s_std, Xs, ys = ref
    b_ref, s_ref = (b_orig, s_orig) if scale == "original" else (b_std, s_std)
    assert rel_err(beta_gpu, b_ref) <= BAR
    assert abs(sig_gpu - s_ref) <= BAR * abs(s_ref)
    # support away from the threshold (standardised scale: the gradient
    # x_j^T (y - X beta) / n of the reference against lambda = sigma lambda0)
    n = Xs.shape[0]
    g = Xs.T @ (ys - Xs @ b_std) / n
    lam = lam0 * s_std
    sure_zero = (b_std == 0) & (lam - np.abs(g) > BAR)
    sure_nz = np.abs(b_std) > BAR
    assert not np.any((beta_gpu != 0) & sure_zero)
    assert not np.any((beta_gpu == 0) & sure_nz)


@pytest.mark.parametrize("scale", ["original", "standardized"])
def test_section3_example(ctx, scale):
    # Section 3's example behind Fig. 2: p = 500, n = 250, two responses
    # (sigma = 3, 5) on one design, lambda0 = sqrt(2 log p / n)
    X, Y, _ = W.sparse_regression()
    n, p = X.shape
    lam0 = math.sqrt(2 * math.log(p) / n)
    beta, sig, outer, st, stats = ctx.scaled_lasso(gpu(X), gpu(Y), lam0, tol=1e-8, output_scale=scale)
    assert st == 0
    refs = reference(X, Y, lam0)
    beta, sig, outer = beta.cpu().numpy(), sig.cpu().numpy(), outer.cpu().numpy()
    for r in range(Y.shape[1]):
        check(beta[:, r], sig[r], refs[r], lam0, scale)
    # fewer than ten sigma updates per response, as the paper observes
    assert np.all(outer >= 1) and np.all(outer < 10)
    assert stats["columns"] == Y.shape[1]


@pytest.mark.parametrize("r,lam0", [(0.6, 0.3), (-0.45, 0.2), (0.25, 0.3)])
def test_one_predictor_closed_form(ctx, r, lam0):
    # one standardised predictor with correlation r (Eq. (1)):
    # sigma^2 = (1 - r^2) / (1 - lam0^2), beta = r - sign(r) lam0 sigma when
    # |r| > lam0, else beta = 0 and sigma = 1
    X = W.orthogonal_pairs_design(40, [r], np.random.default_rng(11))
    y, x = X[:, 0], X[:, 1:2]
    beta, sig, _, st, _ = ctx.scaled_lasso(gpu(x), gpu(y), lam0, tol=1e-12, output_scale="standardized")
    assert st == 0
    if abs(r) > lam0:
        s_cf = math.sqrt((1 - r * r) / (1 - lam0 * lam0))
        b_cf = r - math.copysign(lam0 * s_cf, r)
    else:
        s_cf, b_cf = 1.0, 0.0
    assert abs(float(sig) - s_cf) < 1e-9
    assert abs(float(beta[0]) - b_cf) < 1e-9


def _sparse_responses(n, p, m, k, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, p)) * rng.uniform(0.5, 3.0, p) + rng.uniform(-2, 2, p)
    B = np.zeros((p, m))
    for r in range(m):
        idx = rng.choice(p, k, replace=False)
        B[idx, r] = rng.choice([-1.0, 1.0], k) * rng.uniform(0.5, 2.0, k)
    Y = X @ B + rng.standard_normal((n, m)) * rng.uniform(0.5, 3.0, m) + 5.0
    return X, np.ascontiguousarray(Y)


@pytest.mark.parametrize("n,p,m,k", [(77, 130, 37, 6), (200, 64, 5, 3), (300, 700, 9, 12)])
def test_many_responses_ragged(ctx, n, p, m, k):
    X, Y = _sparse_responses(n, p, m, k, seed=n + p + m)
    lam0 = math.sqrt(2 * math.log(p) / n)
    beta, sig, outer, st, _ = ctx.scaled_lasso(gpu(X), gpu(Y), lam0, tol=1e-8)
    assert st == 0
    refs = reference(X, Y, lam0)
    beta, sig = beta.cpu().numpy(), sig.cpu().numpy()
    for r in range(m):
        check(beta[:, r], sig[r], refs[r], lam0, "original")


def test_many_responses_sharing_one_signal(ctx):
    # 96 responses of Section 3's example (sigma from 1 to 8): the responses
    # correlate strongly with one another, and none may enter another's
    # working set; every eighth response is checked against the oracle
    X, Y, _ = W.sparse_regression(sigmas=np.linspace(1.0, 8.0, 96))
    n, p = X.shape
    lam0 = math.sqrt(2 * math.log(p) / n)
    beta, sig, outer, st, stats = ctx.scaled_lasso(gpu(X), gpu(Y), lam0, tol=1e-8)
    assert st == 0
    assert stats["max_working_set"] <= 32
    pick = list(range(0, 96, 8))
    refs = reference(X, Y[:, pick], lam0)
    beta, sig = beta.cpu().numpy(), sig.cpu().numpy()
    for i, r in enumerate(pick):
        check(beta[:, r], sig[r], refs[i], lam0, "original")


def test_wide_working_set_escalates(ctx):
    # 48 strong coefficients: the working set outgrows 32 coordinates and
    # the response is finished by the 128-coordinate tier
    X, Y = _sparse_responses(600, 160, 2, 48, seed=9)
    lam0 = 0.1
    beta, sig, _, st, stats = ctx.scaled_lasso(gpu(X), gpu(Y), lam0, tol=1e-8)
    assert st == 0
    assert stats["max_working_set"] > 32
    refs = reference(X, Y, lam0)
    beta, sig = beta.cpu().numpy(), sig.cpu().numpy()
    for r in range(2):
        check(beta[:, r], sig[r], refs[r], lam0, "original")


def test_responses_are_independent(ctx):
    # response r never enters another response's regression: solving the
    # responses together or one at a time gives the same results
    X, Y = _sparse_responses(120, 90, 4, 5, seed=4)
    lam0 = 0.25
    beta, sig, _, st, _ = ctx.scaled_lasso(gpu(X), gpu(Y), lam0, tol=1e-10)
    assert st == 0
    for r in range(4):
        b1, s1, _, st1, _ = ctx.scaled_lasso(gpu(X), gpu(Y[:, r]), lam0, tol=1e-10)
        assert st1 == 0
        assert rel_err(b1.cpu().numpy(), beta[:, r].cpu().numpy()) < 1e-9
        assert abs(float(s1) - float(sig[r])) < 1e-9 * float(sig[r])


def test_errors(ctx, sp):
    X, Y = _sparse_responses(50, 20, 2, 3, seed=1)
    Xd, Yd = gpu(X), gpu(Y)
    with pytest.raises(sp.SpmeslError) as e:
        ctx.scaled_lasso(Xd, gpu(np.ones((50, 1))), 0.2)
    assert e.value.code == sp.EZEROVAR
    Yn = Y.copy()
    Yn[3, 1] = np.nan
    with pytest.raises(sp.SpmeslError) as e:
        ctx.scaled_lasso(Xd, gpu(Yn), 0.2)
    assert e.value.code == sp.ENONFINITE
    # through the C ABI: a precision other than double, and ldy < m
    lib = sp.load()
    beta = torch.empty((20, 2), dtype=torch.float64, device=DEV)
    sig = torch.empty((2,), dtype=torch.float64, device=DEV)
    prob = ctx.problem(Xd)
    for prec, ldy in ((sp.MIXED, 2), (sp.FP64, 1)):
        opt = ctx.options(0.2, 1e-8, prec)
        st = lib.spmesl_scaled_lasso(ctx._h, C.byref(prob), C.c_void_p(Yd.data_ptr()), 2, ldy, C.byref(opt),
                                     C.c_void_p(beta.data_ptr()), C.c_void_p(sig.data_ptr()), None, None)
        assert st == sp.EINVAL
