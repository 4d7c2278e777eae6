"""Python binding of libspmesl.so (the C ABI in include/spmesl.h).

Argument marshalling only: every step of the solve runs in the library's HIP
kernels.  PyTorch supplies device memory (inputs, outputs, workspace) and the
current HIP stream.  There is no fallback path: if the library is not built
the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libspmesl.so")

OK = 0
EINVAL = -1
ENONFINITE = -2
EZEROVAR = -3
EDEGENERATE = -4
ENOCONV = -5
EHIP = -6
ENOMEM = -7
EWORKSET = -8

FP64, FP32, MIXED = 0, 1, 2
SCALE_ORIGINAL, SCALE_STANDARDIZED = 0, 1
FLAG_TIMING = 1
FLAG_EAGER = 2
FLAG_FULL_KKT = 4
FLAG_DATA_FORM = 8
MAX_WORKING_SET = 128
NOALLOC_SCRATCH_BYTES = 64 << 20

_PRECISION = {"fp64": FP64, "fp32": FP32, "mixed": MIXED}
_SCALE = {"original": SCALE_ORIGINAL, "standardized": SCALE_STANDARDIZED}
_NAMES = {OK: "OK", EINVAL: "EINVAL", ENONFINITE: "ENONFINITE", EZEROVAR: "EZEROVAR",
          EDEGENERATE: "EDEGENERATE", ENOCONV: "ENOCONV", EHIP: "EHIP", ENOMEM: "ENOMEM",
          EWORKSET: "EWORKSET"}


class SpmeslError(RuntimeError):
    def __init__(self, code: int, msg: str = ""):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


class Problem(C.Structure):
    _fields_ = [("X", C.c_void_p), ("n", C.c_int64), ("p", C.c_int64), ("ldx", C.c_int64),
                ("B0", C.c_void_p), ("sigma0", C.c_void_p)]


class Options(C.Structure):
    _fields_ = [("lambda0", C.c_double), ("tol", C.c_double), ("max_outer", C.c_int32),
                ("max_sweeps", C.c_int32), ("max_rounds", C.c_int32), ("precision", C.c_int32),
                ("output_scale", C.c_int32), ("flags", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [(f, C.c_int64) for f in (
        "columns", "total_outer", "max_outer", "total_sweeps", "total_updates", "total_rounds",
        "max_working_set", "nnz_B", "columns_noconv", "polish_kkt_checks", "polish_added",
        "sum_working_set", "resolved_columns", "escalated_columns")] + \
        [(f, C.c_double) for f in (
            "ms_standardize", "ms_covariance", "ms_solve", "ms_polish", "ms_output", "ms_total")]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class Tuning(C.Structure):
    _fields_ = [("dense_block", C.c_int32), ("fill_blocks", C.c_int32), ("kkt_rows", C.c_int32),
                ("screen_permille", C.c_int32), ("fill_split", C.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class Result(C.Structure):
    _fields_ = [("B", C.c_void_p), ("sigma", C.c_void_p), ("Omega", C.c_void_p),
                ("stats", C.POINTER(Stats))]


_lib = None


def load():
    """Load libspmesl.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2203_15031_amd/build.py")
    lib = C.CDLL(LIB_PATH)
    vp, i64 = C.c_void_p, C.c_int64
    lib.spmesl_create.argtypes = [C.POINTER(vp), C.c_int, vp]
    lib.spmesl_create.restype = C.c_int
    lib.spmesl_destroy.argtypes = [vp]
    lib.spmesl_destroy.restype = None
    lib.spmesl_set_stream.argtypes = [vp, vp]
    lib.spmesl_set_stream.restype = C.c_int
    lib.spmesl_last_error.argtypes = [vp]
    lib.spmesl_last_error.restype = C.c_char_p
    lib.spmesl_version.argtypes = []
    lib.spmesl_version.restype = C.c_char_p
    lib.spmesl_workspace_size.argtypes = [C.POINTER(Problem), C.POINTER(Options), C.POINTER(C.c_size_t)]
    lib.spmesl_workspace_size.restype = C.c_int
    lib.spmesl_set_workspace.argtypes = [vp, vp, C.c_size_t]
    lib.spmesl_set_workspace.restype = C.c_int
    lib.spmesl_solve.argtypes = [vp, C.POINTER(Problem), C.POINTER(Options), C.POINTER(Result)]
    lib.spmesl_solve.restype = C.c_int
    lib.spmesl_solve_batch.argtypes = [vp, C.c_int, C.POINTER(Problem), C.POINTER(Options),
                                       C.POINTER(C.c_double), C.POINTER(Result), C.POINTER(C.c_int)]
    lib.spmesl_batch_workspace_size.argtypes = [vp, C.c_int, C.POINTER(Problem), C.POINTER(Options),
                                                C.POINTER(C.c_size_t)]
    lib.spmesl_batch_workspace_size.restype = C.c_int
    lib.spmesl_solve_async.argtypes = [vp, C.POINTER(Problem), C.POINTER(Options), C.POINTER(Result), vp]
    lib.spmesl_solve_async.restype = C.c_int
    lib.spmesl_solve_noalloc.argtypes = [vp, C.POINTER(Problem), C.POINTER(Options), C.POINTER(Result), vp]
    lib.spmesl_solve_noalloc.restype = C.c_int
    lib.spmesl_solve_batch.restype = C.c_int
    lib.spmesl_covariance.argtypes = [vp, C.POINTER(Problem), C.c_int, vp, vp, vp]
    lib.spmesl_covariance.restype = C.c_int
    lib.spmesl_scaled_lasso.argtypes = [vp, C.POINTER(Problem), vp, i64, i64, C.POINTER(Options), vp, vp, vp,
                                        C.POINTER(Stats)]
    lib.spmesl_scaled_lasso.restype = C.c_int
    lib.spmesl_scaled_lasso_workspace_size.argtypes = [i64, i64, i64, C.POINTER(C.c_size_t)]
    lib.spmesl_scaled_lasso_workspace_size.restype = C.c_int
    lib.spmesl_symmetrize.argtypes = [vp, i64, vp, vp]
    lib.spmesl_symmetrize.restype = C.c_int
    lib.spmesl_set_tuning.argtypes = [vp, C.POINTER(Tuning)]
    lib.spmesl_set_tuning.restype = C.c_int
    lib.spmesl_get_tuning.argtypes = [vp, C.POINTER(Tuning)]
    lib.spmesl_get_tuning.restype = C.c_int
    lib.spmesl_autotune.argtypes = [vp, C.POINTER(Problem), C.POINTER(Options), C.POINTER(Result), C.c_int,
                                    C.POINTER(Tuning), C.POINTER(C.c_double)]
    lib.spmesl_autotune.restype = C.c_int
    lib.spmesl_kernel_times.argtypes = [vp, C.c_int, C.POINTER(C.c_char_p), C.POINTER(C.c_double)]
    lib.spmesl_kernel_times.restype = C.c_int
    for f in ("spmesl_lambda_univ", "spmesl_lambda_ub"):
        getattr(lib, f).argtypes = [C.c_double, C.c_double]
        getattr(lib, f).restype = C.c_double
    lib.spmesl_lambda_pb.argtypes = [C.c_double, C.c_double, C.POINTER(C.c_double),
                                     C.POINTER(C.c_double)]
    lib.spmesl_lambda_pb.restype = C.c_int
    _lib = lib
    return lib


# ---------------------------------------------------------------------------
# penalty levels (host)
# ---------------------------------------------------------------------------

def lambda_univ(n, p):
    return load().spmesl_lambda_univ(float(n), float(p))


def lambda_ub(n, p):
    return load().spmesl_lambda_ub(float(n), float(p))


def lambda_pb(n, p):
    """Returns (lambda_pb, k)."""
    lam, k = C.c_double(), C.c_double()
    st = load().spmesl_lambda_pb(float(n), float(p), C.byref(lam), C.byref(k))
    if st != OK:
        raise SpmeslError(st, "lambda_pb")
    return lam.value, k.value


# ---------------------------------------------------------------------------
# context
# ---------------------------------------------------------------------------

def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


def _check_X(X):
    if not isinstance(X, torch.Tensor) or X.dtype != torch.float64 or not X.is_cuda:
        raise TypeError("X must be a float64 CUDA tensor")
    if X.dim() != 2 or X.stride(1) != 1:
        raise ValueError("X must be 2-D with unit column stride (row-major)")


@dataclass
class SolveResult:
    B: torch.Tensor | None
    sigma: torch.Tensor | None
    Omega: torch.Tensor | None
    status: int
    stats: dict


class Context:
    """One library context bound to a device; enqueues on torch's current stream."""

    def __init__(self, device: int | None = None):
        lib = load()
        self.device = torch.cuda.current_device() if device is None else int(device)
        self._h = C.c_void_p()
        with torch.cuda.device(self.device):
            stream = torch.cuda.current_stream().cuda_stream
            st = lib.spmesl_create(C.byref(self._h), self.device, C.c_void_p(stream))
        if st != OK:
            raise SpmeslError(st, "spmesl_create")
        self._ws = None

    def close(self):
        if self._h:
            load().spmesl_destroy(self._h)
            self._h = C.c_void_p()
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- helpers ------------------------------------------------------------
    def _err(self):
        return load().spmesl_last_error(self._h).decode()

    def _bind_stream(self):
        s = torch.cuda.current_stream(self.device).cuda_stream
        load().spmesl_set_stream(self._h, C.c_void_p(s))

    def _workspace(self, nbytes: int):
        """Workspace from torch's allocator, grown on demand."""
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=f"cuda:{self.device}")
            base = self._ws.data_ptr()
            off = (-base) % 256
            st = load().spmesl_set_workspace(self._h, C.c_void_p(base + off), nbytes + 256 - off)
            if st != OK:
                raise SpmeslError(st, self._err())

    @staticmethod
    def options(lambda0, tol=1e-8, precision="fp64", output_scale="original", max_outer=0,
                max_sweeps=0, max_rounds=0, timing=False, eager=False, full_kkt=False, data_form=False):
        return Options(float(lambda0), float(tol), int(max_outer), int(max_sweeps),
                       int(max_rounds), _PRECISION[precision] if isinstance(precision, str) else int(precision),
                       _SCALE[output_scale] if isinstance(output_scale, str) else int(output_scale),
                       (FLAG_TIMING if timing else 0) | (FLAG_EAGER if eager else 0)
                       | (FLAG_FULL_KKT if full_kkt else 0) | (FLAG_DATA_FORM if data_form else 0))

    @staticmethod
    def problem(X):
        _check_X(X)
        n, p = X.shape
        return Problem(X.data_ptr(), n, p, X.stride(0))

    def workspace_size(self, X, opt):
        prob = self.problem(X)
        sz = C.c_size_t()
        st = load().spmesl_workspace_size(C.byref(prob), C.byref(opt), C.byref(sz))
        if st != OK:
            raise SpmeslError(st, "workspace_size")
        return sz.value

    # -- entry points -------------------------------------------------------
    def solve(self, X, lambda0, tol=1e-8, precision="fp64", output_scale="original",
              want=("B", "sigma", "Omega"), out=None, max_outer=0, max_sweeps=0, max_rounds=0,
              timing=False, check=True, eager=False, full_kkt=False, B0=None, sigma0=None,
              data_form=False) -> SolveResult:
        """Full SPMESL of X (n x p float64 CUDA tensor).

        Returns B (p x p, column k = beta of response k), sigma (p) and the
        symmetrised Omega (p x p).  `out` may hold preallocated output
        tensors.  Raises SpmeslError on any code other than OK and (when
        check is False) ENOCONV.  eager=True enqueues kernel by kernel
        instead of replaying the context's graph of a repeated call.
        full_kkt=True (mixed form) makes the double polish prove every column
        with a full KKT pass over S.  B0 (p x p) and sigma0 (p), float64 CUDA
        tensors in the scale of the outputs, warm-start the column solves
        (either may be None).  data_form=True (double only) solves without
        forming S (Algorithm 3's data form)."""
        opt = self.options(lambda0, tol, precision, output_scale, max_outer, max_sweeps,
                           max_rounds, timing, eager, full_kkt, data_form)
        prob, res, out, stats = self._prepare(X, opt, want, out)
        self._warm(prob, X, B0, sigma0)
        st = load().spmesl_solve(self._h, C.byref(prob), C.byref(opt), C.byref(res))
        if st != OK and (check or st != ENOCONV):
            raise SpmeslError(st, self._err())
        return SolveResult(out.get("B"), out.get("sigma"), out.get("Omega"), st, stats.as_dict())

    def solve_async(self, X, lambda0, status, tol=1e-8, precision="fp64", output_scale="original",
                    want=("B", "sigma", "Omega"), out=None, eager=False, data_form=False) -> SolveResult:
        """Enqueue a full solve on torch's current stream without waiting.

        `status` is a one-element int32 CUDA tensor that receives the status
        code when the solve completes on the stream.  Returns the output
        tensors (valid once the stream has reached that point); stats are
        not reported."""
        if status.dtype != torch.int32 or status.device != X.device or status.numel() < 1:
            raise ValueError("status must be an int32 tensor on the device of X")
        opt = self.options(lambda0, tol, precision, output_scale, eager=eager, data_form=data_form)
        prob, res, out, _ = self._prepare(X, opt, want, out)
        st = load().spmesl_solve_async(self._h, C.byref(prob), C.byref(opt), C.byref(res),
                                       C.c_void_p(status.data_ptr()))
        if st != OK:
            raise SpmeslError(st, self._err())
        return SolveResult(out.get("B"), out.get("sigma"), out.get("Omega"), OK, {})

    def solve_noalloc(self, X, lambda0, status, out, tol=1e-8, precision="fp64",
                      output_scale="original"):
        """spmesl_solve_noalloc: the solve of solve_async in the library's fixed
        scratch array (no allocation by the library).  `out` holds the
        caller's B / sigma / Omega tensors (any may be None); `status` a
        one-element int32 CUDA tensor that receives the status code."""
        if status.dtype != torch.int32 or status.device != X.device or status.numel() < 1:
            raise ValueError("status must be an int32 tensor on the device of X")
        opt = self.options(lambda0, tol, precision, output_scale)
        prob = self.problem(X)
        for name in ("B", "sigma", "Omega"):
            t = out.get(name)
            if t is not None and (t.dtype != torch.float64 or not t.is_contiguous() or t.device != X.device):
                raise ValueError(f"{name} must be a contiguous float64 tensor on {X.device}")
        res = Result(_ptr(out.get("B")).value, _ptr(out.get("sigma")).value,
                     _ptr(out.get("Omega")).value, None)
        self._bind_stream()
        st = load().spmesl_solve_noalloc(self._h, C.byref(prob), C.byref(opt), C.byref(res),
                                         C.c_void_p(status.data_ptr()))
        if st != OK:
            raise SpmeslError(st, self._err())
        return SolveResult(out.get("B"), out.get("sigma"), out.get("Omega"), OK, {})

    @staticmethod
    def _warm(prob, X, B0, sigma0):
        p = prob.p
        for name, t, shape in (("B0", B0, (p, p)), ("sigma0", sigma0, (p,))):
            if t is None:
                continue
            if t.dtype != torch.float64 or not t.is_contiguous() or t.device != X.device or tuple(t.shape) != shape:
                raise ValueError(f"{name} must be a contiguous float64 tensor of shape {shape} on {X.device}")
            setattr(prob, name, t.data_ptr())

    def _prepare(self, X, opt, want, out):
        prob = self.problem(X)
        p = prob.p
        dev = X.device
        out = dict(out or {})
        for name, shape in (("B", (p, p)), ("sigma", (p,)), ("Omega", (p, p))):
            if name in want and out.get(name) is None:
                out[name] = torch.empty(shape, dtype=torch.float64, device=dev)
        for name in ("B", "sigma", "Omega"):
            if name in out and out[name] is not None:
                t = out[name]
                if t.dtype != torch.float64 or not t.is_contiguous() or t.device != dev:
                    raise ValueError(f"{name} must be a contiguous float64 tensor on {dev}")
        stats = Stats()
        res = Result(_ptr(out.get("B")).value, _ptr(out.get("sigma")).value,
                     _ptr(out.get("Omega")).value, C.pointer(stats))
        self._workspace(self.workspace_size(X, opt) + 4096)
        self._bind_stream()
        return prob, res, out, stats

    def solve_batch(self, Xs, lambda0s, tol=1e-8, precision="fp64", output_scale="original",
                    check=True, outs=None, eager=False, data_form=False):
        """Solve several datasets (uneven n, p) in one library call; lambda0s
        is one value or one per dataset.  `outs` may hold one dict of
        preallocated B / sigma / Omega tensors per dataset (a repeated call
        with the same tensors replays the context's graph of the batch)."""
        m = len(Xs)
        if not isinstance(lambda0s, (list, tuple)):
            lambda0s = [lambda0s] * m
        opt = self.options(lambda0s[0] if m else 1.0, tol, precision, output_scale, eager=eager,
                           data_form=data_form)
        probs = (Problem * m)(*[self.problem(X) for X in Xs])
        lams = (C.c_double * m)(*[float(v) for v in lambda0s])
        stats = [Stats() for _ in range(m)]
        ress = (Result * m)()
        outs = list(outs) if outs is not None else [None] * m
        need = 0
        for i, X in enumerate(Xs):
            p = X.shape[1]
            o = outs[i]
            if o is None:
                o = dict(B=torch.empty((p, p), dtype=torch.float64, device=X.device),
                         sigma=torch.empty((p,), dtype=torch.float64, device=X.device),
                         Omega=torch.empty((p, p), dtype=torch.float64, device=X.device))
                outs[i] = o
            ress[i] = Result(_ptr(o.get("B")).value, _ptr(o.get("sigma")).value,
                             _ptr(o.get("Omega")).value, C.pointer(stats[i]))
        sz = C.c_size_t()
        st = load().spmesl_batch_workspace_size(self._h, m, probs, C.byref(opt), C.byref(sz))
        if st != OK:
            raise SpmeslError(st, "batch_workspace_size")
        need = sz.value
        self._workspace(need + 4096)
        self._bind_stream()
        unset = 1  # no status code is positive: a slot the call did not write
        status = (C.c_int * max(m, 1))(*([unset] * max(m, 1)))
        st = load().spmesl_solve_batch(self._h, m, probs, C.byref(opt), lams, ress, status)
        # check=False returns the per-data-set statuses when the call reached
        # every data set (a data set's own error does not stop the others)
        if st != OK and (check or any(status[i] == unset for i in range(m))):
            raise SpmeslError(st, self._err())
        return [SolveResult(outs[i].get("B"), outs[i].get("sigma"), outs[i].get("Omega"), status[i],
                            stats[i].as_dict()) for i in range(m)]

    def covariance(self, X, precision="fp64"):
        """Standardise X and form S; returns (S, mean, scale)."""
        prec = _PRECISION[precision] if isinstance(precision, str) else int(precision)
        prob = self.problem(X)
        p = prob.p
        dt = torch.float64 if prec == FP64 else torch.float32
        S = torch.empty((p, p), dtype=dt, device=X.device)
        mean = torch.empty((p,), dtype=torch.float64, device=X.device)
        scale = torch.empty((p,), dtype=torch.float64, device=X.device)
        opt = self.options(1.0, 1.0, prec)
        self._workspace(self.workspace_size(X, opt) + 4096)
        self._bind_stream()
        st = load().spmesl_covariance(self._h, C.byref(prob), prec, _ptr(S), _ptr(mean), _ptr(scale))
        if st != OK:
            raise SpmeslError(st, self._err())
        return S, mean, scale

    def scaled_lasso(self, X, Y, lambda0, tol=1e-8, output_scale="original", max_outer=0, max_sweeps=0,
                     max_rounds=0, check=True):
        """Scaled lassos of the responses Y (n x m, or n) on the design X (n x p).

        Returns (beta (p x m, or p), sigma (m, or a 0-d tensor), outer
        (int32, sigma updates per response), status, stats)."""
        _check_X(X)
        vec = Y.dim() == 1
        Y2 = Y.unsqueeze(1) if vec else Y
        if Y2.dtype != torch.float64 or Y2.device != X.device or Y2.dim() != 2 or Y2.stride(1) != 1:
            raise ValueError("Y must be a float64 tensor on the device of X, 1-D or 2-D row-major")
        if Y2.shape[0] != X.shape[0]:
            raise ValueError("Y must have as many rows as X")
        n, p = X.shape
        m = Y2.shape[1]
        beta = torch.empty((p, m), dtype=torch.float64, device=X.device)
        sigma = torch.empty((m,), dtype=torch.float64, device=X.device)
        outer = torch.empty((m,), dtype=torch.int32, device=X.device)
        opt = self.options(lambda0, tol, "fp64", output_scale, max_outer, max_sweeps, max_rounds)
        sz = C.c_size_t()
        st = load().spmesl_scaled_lasso_workspace_size(n, p, m, C.byref(sz))
        if st != OK:
            raise SpmeslError(st, "scaled_lasso_workspace_size")
        self._workspace(sz.value + 4096)
        self._bind_stream()
        stats = Stats()
        prob = self.problem(X)
        st = load().spmesl_scaled_lasso(self._h, C.byref(prob), _ptr(Y2), m, Y2.stride(0), C.byref(opt),
                                        _ptr(beta), _ptr(sigma), _ptr(outer), C.byref(stats))
        if st != OK and (check or st != ENOCONV):
            raise SpmeslError(st, self._err())
        if vec:
            return beta[:, 0], sigma[0], outer[0], st, stats.as_dict()
        return beta, sigma, outer, st, stats.as_dict()

    # -- launch shapes and the autotuner ------------------------------------
    def set_tuning(self, tuning=None):
        """Set the context's launch shapes (a dict of spmesl_tuning fields;
        None resets them to the defaults)."""
        if tuning is None:
            st = load().spmesl_set_tuning(self._h, None)
        else:
            t = Tuning(**{k: int(v) for k, v in tuning.items()})
            st = load().spmesl_set_tuning(self._h, C.byref(t))
        if st != OK:
            raise SpmeslError(st, self._err())

    def get_tuning(self):
        t = Tuning()
        st = load().spmesl_get_tuning(self._h, C.byref(t))
        if st != OK:
            raise SpmeslError(st, self._err())
        return t.as_dict()

    def autotune(self, X, lambda0, tol=1e-8, precision="fp64", output_scale="original", reps=5, out=None,
                 data_form=False):
        """spmesl_autotune on this problem: returns (tuning dict, ms per solve);
        the context keeps the chosen shapes."""
        opt = self.options(lambda0, tol, precision, output_scale, data_form=data_form)
        prob, res, out, _ = self._prepare(X, opt, ("B", "sigma", "Omega"), out)
        best = Tuning()
        ms = C.c_double()
        st = load().spmesl_autotune(self._h, C.byref(prob), C.byref(opt), C.byref(res), int(reps),
                                    C.byref(best), C.byref(ms))
        if st != OK:
            raise SpmeslError(st, self._err())
        return best.as_dict(), ms.value

    def kernel_times(self):
        """[(name, ms)] of each launch step of the last solve run with timing=True."""
        lib = load()
        n = lib.spmesl_kernel_times(self._h, 0, None, None)
        if n < 0:
            raise SpmeslError(n, self._err())
        names = (C.c_char_p * max(n, 1))()
        ms = (C.c_double * max(n, 1))()
        n = lib.spmesl_kernel_times(self._h, n, names, ms)
        return [(names[i].decode(), float(ms[i])) for i in range(n)]

    def symmetrize(self, Omega1):
        if Omega1.dtype != torch.float64 or not Omega1.is_cuda or not Omega1.is_contiguous():
            raise TypeError("Omega1 must be a contiguous float64 CUDA tensor")
        p = Omega1.shape[0]
        out = torch.empty_like(Omega1)
        self._bind_stream()
        st = load().spmesl_symmetrize(self._h, p, _ptr(Omega1), _ptr(out))
        if st != OK:
            raise SpmeslError(st, self._err())
        return out


_default = {}


def context(device: int | None = None) -> Context:
    d = torch.cuda.current_device() if device is None else int(device)
    if d not in _default:
        _default[d] = Context(d)
    return _default[d]


def solve(X, lambda0, tol=1e-8, precision="fp64", **kw) -> SolveResult:
    """spmesl_solve on X's device with a cached context."""
    return context(X.device.index).solve(X, lambda0, tol, precision, **kw)
