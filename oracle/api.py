"""ctypes binding of the C oracle (test infrastructure only).

Arrays cross as float64; data matrices are passed row-major (n, p) and
transposed here to the column-major layout the C code walks.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "spmesl_oracle.c")
_LIB = None

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)
_lp = C.POINTER(C.c_int64)


def lib_path(mutant: int = 0) -> str:
    name = "liboracle.so" if mutant == 0 else f"liboracle_m{mutant}.so"
    return os.path.join(_HERE, name)


def build(mutant: int = 0, out: str | None = None) -> str:
    """Compile the oracle with gcc (-O2, OpenMP).  mutant > 0 plants a mistake."""
    out = out or lib_path(mutant)
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
           f"-DORACLE_MUTANT={int(mutant)}", _SRC, "-o", out + ".tmp", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


def _setup(lib):
    lib.oracle_standardize.argtypes = [C.c_int64, C.c_int64, _dp, _dp, _dp, _dp]
    lib.oracle_standardize.restype = C.c_int
    lib.oracle_scaled_lasso.argtypes = [C.c_int64, C.c_int64, _dp, _dp, C.c_int64,
                                        C.c_double, C.c_double, C.c_int, C.c_int,
                                        _dp, _dp, _dp, _ip, _ip]
    lib.oracle_scaled_lasso.restype = C.c_int
    lib.oracle_symmetrize.argtypes = [C.c_int64, _dp]
    lib.oracle_symmetrize.restype = None
    lib.oracle_spmesl.argtypes = [C.c_int64, C.c_int64, _dp, C.c_double, C.c_double,
                                  C.c_int, C.c_int, C.c_int, _dp, _dp, _dp, _dp,
                                  _dp, _dp, _ip, _ip, _ip, C.c_int]
    lib.oracle_spmesl.restype = C.c_int
    lib.oracle_spmesl_columns.argtypes = [C.c_int64, C.c_int64, _dp, C.c_double,
                                          C.c_double, C.c_int, C.c_int, C.c_int64, _lp,
                                          _dp, _dp, _dp, _dp, _ip, _ip, _ip, C.c_int]
    lib.oracle_spmesl_columns.restype = C.c_int
    lib.oracle_omega_subset.argtypes = [C.c_int64, C.c_int64, _lp, _dp, _dp, _dp, _dp]
    lib.oracle_omega_subset.restype = None
    for f in ("oracle_lambda_ub", "oracle_lambda_univ"):
        getattr(lib, f).argtypes = [C.c_double, C.c_double]
        getattr(lib, f).restype = C.c_double
    lib.oracle_lambda_pb.argtypes = [C.c_double, C.c_double, _dp]
    lib.oracle_lambda_pb.restype = C.c_double
    return lib


def load(mutant: int = 0):
    """Load (building when absent) the oracle library."""
    global _LIB
    if mutant == 0 and _LIB is not None:
        return _LIB
    path = lib_path(mutant)
    if mutant != 0 or not os.path.exists(path) or \
            os.path.getmtime(path) < os.path.getmtime(_SRC):
        build(mutant)
    lib = _setup(C.CDLL(path))
    if mutant == 0:
        _LIB = lib
    return lib


def _p(a):
    return a.ctypes.data_as(_dp)


def _colmajor(X):
    X = np.asarray(X, dtype=np.float64)
    return np.ascontiguousarray(X.T)  # (p, n) C-order == column-major (n, p)


def standardize(X, lib=None):
    """Returns (Xs row-major, mean, c) or raises on a C error code."""
    lib = lib or load()
    n, p = X.shape
    Xc = _colmajor(X)
    Xs = np.empty_like(Xc)
    mean = np.empty(p)
    c = np.empty(p)
    st = lib.oracle_standardize(n, p, _p(Xc), _p(Xs), _p(mean), _p(c))
    if st != 0:
        raise OracleError(st)
    return Xs.T.copy(), mean, c


class OracleError(RuntimeError):
    def __init__(self, code):
        super().__init__(f"oracle status {code}")
        self.code = code


def scaled_lasso(X, y, lambda0, tol=1e-8, skip=-1, max_outer=1000, max_sweeps=1000000,
                 beta0=None, sigma0=1.0, lib=None):
    """Algorithm 1 on (y, X) as given (no standardisation).

    Returns (beta, sigma, n_outer, n_sweeps, status)."""
    lib = lib or load()
    n, p = X.shape
    Xc = _colmajor(X)
    y = np.ascontiguousarray(y, dtype=np.float64)
    beta = np.zeros(p) if beta0 is None else np.array(beta0, dtype=np.float64)
    sig = C.c_double(sigma0)
    e = np.empty(n)
    no, ns = C.c_int(0), C.c_int(0)
    st = lib.oracle_scaled_lasso(n, p, _p(Xc), _p(y), skip, lambda0, tol, max_outer,
                                 max_sweeps, _p(beta), C.byref(sig), _p(e),
                                 C.byref(no), C.byref(ns))
    if st == -1:
        raise OracleError(st)
    return beta, sig.value, no.value, ns.value, st


def spmesl(X, lambda0, tol=1e-8, original_scale=True, max_outer=1000,
           max_sweeps=1000000, nthreads=0, lib=None):
    """Algorithm 2 (+ Proposition 1 when original_scale).

    Returns a dict with B (p x p, column k = beta_{-k}), sigma, Omega, Omega1,
    mean, c, n_outer, n_sweeps, col_status, status."""
    lib = lib or load()
    n, p = X.shape
    Xc = _colmajor(X)
    B = np.empty((p, p))       # C-order buffer used column-major: B_cm[k, j] = b_jk
    Om = np.empty((p, p))
    Om1 = np.empty((p, p))
    sigma = np.empty(p)
    mean = np.empty(p)
    c = np.empty(p)
    no = np.empty(p, dtype=np.int32)
    ns = np.empty(p, dtype=np.int32)
    cs = np.empty(p, dtype=np.int32)
    st = lib.oracle_spmesl(n, p, _p(Xc), lambda0, tol, max_outer, max_sweeps,
                           1 if original_scale else 0, _p(B), _p(sigma), _p(Om), _p(Om1),
                           _p(mean), _p(c), no.ctypes.data_as(_ip), ns.ctypes.data_as(_ip),
                           cs.ctypes.data_as(_ip), nthreads)
    if st in (-1, -2, -4):
        raise OracleError(st)
    return dict(B=B.T.copy(), sigma=sigma, Omega=Om.T.copy(), Omega1=Om1.T.copy(),
                mean=mean, c=c, n_outer=no, n_sweeps=ns, col_status=cs, status=st)


def spmesl_columns(X, lambda0, cols, tol=1e-8, max_outer=1000, max_sweeps=1000000,
                   nthreads=0, lib=None):
    """Algorithm 1 for the listed response columns only (standardised scale).

    Returns dict with B (p x m, column i = beta_{-cols[i]}), sigma (m), mean, c,
    n_outer, n_sweeps, col_status, status."""
    lib = lib or load()
    n, p = X.shape
    Xc = _colmajor(X)
    cols = np.ascontiguousarray(cols, dtype=np.int64)
    m = cols.size
    Bc = np.empty((max(m, 1), p))
    sg = np.empty(max(m, 1))
    mean = np.empty(p)
    c = np.empty(p)
    no = np.empty(max(m, 1), dtype=np.int32)
    ns = np.empty(max(m, 1), dtype=np.int32)
    cs = np.empty(max(m, 1), dtype=np.int32)
    st = lib.oracle_spmesl_columns(n, p, _p(Xc), lambda0, tol, max_outer, max_sweeps, m,
                                   cols.ctypes.data_as(_lp), _p(Bc), _p(sg), _p(mean), _p(c),
                                   no.ctypes.data_as(_ip), ns.ctypes.data_as(_ip),
                                   cs.ctypes.data_as(_ip), nthreads)
    if st in (-1, -2, -4):
        raise OracleError(st)
    return dict(B=Bc[:m].T.copy(), sigma=sg[:m].copy(), mean=mean, c=c,
                n_outer=no[:m].copy(), n_sweeps=ns[:m].copy(), col_status=cs[:m].copy(),
                status=st)


def spmesl_subset(X, lambda0, cols, tol=1e-8, original_scale=False, max_outer=1000,
                  max_sweeps=1000000, nthreads=0, lib=None):
    """Algorithm 1 for the listed columns (ascending, distinct) and the
    symmetrised estimate on the pairs inside the set.

    Returns spmesl_columns' dict (standardised B and sigma of the listed
    columns) plus Omega_sub (m x m): the block of Omega for the pairs of
    listed columns, on the data's scale when original_scale."""
    lib = lib or load()
    cols = np.ascontiguousarray(cols, dtype=np.int64)
    if cols.size > 1 and not np.all(np.diff(cols) > 0):
        raise ValueError("cols must be ascending and distinct")
    r = spmesl_columns(X, lambda0, cols, tol=tol, max_outer=max_outer,
                       max_sweeps=max_sweeps, nthreads=nthreads, lib=lib)
    p = X.shape[1]
    m = cols.size
    Bc = np.ascontiguousarray(r["B"].T)  # (m, p) C-order == column-major (p, m)
    sg = np.ascontiguousarray(r["sigma"])
    Om = np.empty((max(m, 1), max(m, 1)))
    cc = np.ascontiguousarray(r["c"]) if original_scale else None
    lib.oracle_omega_subset(p, m, cols.ctypes.data_as(_lp), _p(Bc), _p(sg),
                            _p(cc) if cc is not None else None, Om.ctypes.data_as(_dp))
    r["Omega_sub"] = Om[:m, :m].T.copy()
    return r


def symmetrize(W, lib=None):
    """Algorithm 2's symmetrisation of a (p x p) matrix; returns a new array."""
    lib = lib or load()
    p = W.shape[0]
    Wc = np.ascontiguousarray(np.asarray(W, dtype=np.float64).T)
    lib.oracle_symmetrize(p, _p(Wc))
    return Wc.T.copy()


def lambda_ub(n, p, lib=None):
    return (lib or load()).oracle_lambda_ub(float(n), float(p))


def lambda_univ(n, p, lib=None):
    return (lib or load()).oracle_lambda_univ(float(n), float(p))


def lambda_pb(n, p, lib=None):
    """Returns (lambda_pb, k)."""
    k = C.c_double(0.0)
    lam = (lib or load()).oracle_lambda_pb(float(n), float(p), C.byref(k))
    return lam, k.value
