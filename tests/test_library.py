"""Host-side checks of the HIP library (no GPU needed)."""
import ctypes
import json
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "spmesl.h")
GOLDEN = os.path.join(ROOT, "tests", "golden")


def _lib():
    from paper_2203_15031_amd import spmesl
    return spmesl.load()


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(spmesl_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for f in ("spmesl_create", "spmesl_destroy", "spmesl_solve", "spmesl_solve_batch",
              "spmesl_workspace_size", "spmesl_set_workspace", "spmesl_covariance",
              "spmesl_symmetrize", "spmesl_lambda_pb", "spmesl_scaled_lasso"):
        assert f in names


def test_library_exports_every_declared_symbol():
    lib = _lib()
    missing = [f for f in declared_functions() if not hasattr(lib, f)]
    assert not missing, missing


def test_penalty_levels_worked_example():
    from paper_2203_15031_amd import spmesl
    g = json.load(open(os.path.join(GOLDEN, "penalty_levels.json")))
    tol = 0.5 * 10 ** -g["printed_decimals"]
    assert abs(spmesl.lambda_ub(g["n"], g["p"]) - g["lambda_ub"]) <= tol
    assert abs(spmesl.lambda_univ(g["n"], g["p"]) - g["lambda_univ"]) <= tol
    lam, k = spmesl.lambda_pb(g["n"], g["p"])
    assert abs(lam - g["lambda_pb"]) <= tol and abs(k - g["k"]) <= tol


def test_penalty_levels_against_oracle():
    import oracle
    from paper_2203_15031_amd import spmesl
    for n, p in [(100, 1000), (250, 500), (400, 5000), (1000, 20000), (30, 3)]:
        lam, k = spmesl.lambda_pb(n, p)
        lo, ko = oracle.lambda_pb(n, p)
        assert abs(lam - lo) < 1e-12 * lo and abs(k - ko) < 1e-9 * ko
        assert spmesl.lambda_ub(n, p) == pytest.approx(oracle.lambda_ub(n, p), rel=1e-15)
        assert spmesl.lambda_univ(n, p) == pytest.approx(oracle.lambda_univ(n, p), rel=1e-15)


def test_normal_quantile_accuracy():
    # the library's Phi^-1 (AS 241) through lambda_pb's building block:
    # L_n(t) = Phi^-1(1 - t)/sqrt(n) with k = p t; check against scipy via
    # the root equation at many p
    from scipy.stats import norm
    from paper_2203_15031_amd import spmesl
    for p in (10, 57, 100, 1000, 12345, 1e6):
        lam, k = spmesl.lambda_pb(1.0, p)
        L = norm.ppf(1 - k / p)
        assert abs(lam - np.sqrt(2) * L) < 1e-13 * abs(L)
        assert abs(k - (L ** 4 + 2 * L ** 2)) < 1e-9 * k


def test_workspace_size_and_validation():
    from paper_2203_15031_amd import spmesl
    lib = _lib()
    for prec in (0, 1, 2):
        prob = spmesl.Problem(1, 400, 5000, 5000)  # pointer value only checked for NULL
        opt = spmesl.Options(0.2, 1e-8, 0, 0, 0, prec, 0, 0)
        sz = ctypes.c_size_t()
        assert lib.spmesl_workspace_size(ctypes.byref(prob), ctypes.byref(opt), ctypes.byref(sz)) == 0
        # S, the O(n p) state, and the dense tiers' workgroup slices (a
        # quarter of the rest of the plan at most, 16 MB at least)
        s_bytes = (8 if prec == 0 else 4) * 5000 * 5000
        assert s_bytes < sz.value < 1.25 * (s_bytes + 64 * 2 ** 20) + 16 * 2 ** 20
    bad = [spmesl.Problem(1, 1, 10, 10), spmesl.Problem(1, 10, 1, 1), spmesl.Problem(1, 10, 10, 5),
           spmesl.Problem(0, 10, 10, 10)]
    opt = spmesl.Options(0.2, 1e-8, 0, 0, 0, 0, 0, 0)
    for prob in bad:
        sz = ctypes.c_size_t()
        assert lib.spmesl_workspace_size(ctypes.byref(prob), ctypes.byref(opt), ctypes.byref(sz)) == -1
    prob = spmesl.Problem(1, 10, 10, 10)
    for o in (spmesl.Options(0.0, 1e-8, 0, 0, 0, 0, 0, 0), spmesl.Options(0.2, 0.0, 0, 0, 0, 0, 0, 0),
              spmesl.Options(0.2, 1e-8, 0, 0, 0, 3, 0, 0), spmesl.Options(0.2, 1e-8, 0, 0, 0, 0, 2, 0)):
        sz = ctypes.c_size_t()
        assert lib.spmesl_workspace_size(ctypes.byref(prob), ctypes.byref(o), ctypes.byref(sz)) == -1


def test_tuning_cache_roundtrip(tmp_path):
    # the autotuner's cache: stored entries come back, keyed by device,
    # precision and shape, and a hit skips the tuning call
    from paper_2203_15031_amd import tuning

    class FakeCtx:
        def __init__(self):
            self.tuned = 0
            self.set = None

        def autotune(self, X, lam, tol, prec, reps=5):
            self.tuned += 1
            return {"dense_block": 16, "fill_blocks": 128, "kkt_rows": 2, "screen_permille": 900, "fill_split": 1}, 0.25

        def set_tuning(self, t):
            self.set = dict(t)

    class FakeX:
        shape = (400, 5000)

    path = str(tmp_path / "t.json")
    c = FakeCtx()
    t, ms, hit = tuning.tuned(c, FakeX(), 0.2, precision="mixed", path=path, device_name="gpu")
    assert not hit and c.tuned == 1 and ms == 0.25 and t["fill_blocks"] == 128
    t2, ms2, hit2 = tuning.tuned(c, FakeX(), 0.2, precision="mixed", path=path, device_name="gpu")
    assert hit2 and c.tuned == 1 and t2 == t and c.set == t and ms2 == 0.25
    # another precision or shape is another entry
    tuning.tuned(c, FakeX(), 0.2, precision="fp64", path=path, device_name="gpu")
    assert c.tuned == 2
    data = tuning.load(path)
    assert tuning.key("gpu", "mixed", 400, 5000) in data and len(data) == 2
