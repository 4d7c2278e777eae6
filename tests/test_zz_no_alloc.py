"""GPU test of spmesl_solve_noalloc, the entry point that allocates nothing.

It runs spmesl_solve_async's solve in the library's fixed per-GPU scratch
array.  Two calls in a row (the second on a smaller problem, so the array
still holds the first call's contents) must give the results of
spmesl_solve_async on the same inputs, and both must meet the parity bar
against the oracle.  A problem that does not fit the array is refused
before anything is enqueued.
"""
import ctypes as C

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from paper_2203_15031_amd import workloads as W
from tests.parity import rel_err

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _outs(p):
    return dict(B=torch.full((p, p), 5.0, dtype=torch.float64, device=DEV),
                sigma=torch.full((p,), 5.0, dtype=torch.float64, device=DEV),
                Omega=torch.full((p, p), 5.0, dtype=torch.float64, device=DEV))


def test_noalloc_matches_async_on_two_calls():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2203_15031_amd import spmesl as sp
    ctx = sp.Context(0)
    try:
        cases = [("er_n200_p1000", "mixed", 1e-4), ("ar1_n100_p200", "mixed", 1e-4),
                 ("er_n200_p1000", "fp64", 1e-6), ("ar1_n100_p200", "fp64", 1e-6)]
        for name, prec, bar in cases:
            w = W.workload(name)
            X = W.generate(name)
            Xg = torch.from_numpy(X).to(DEV)
            p = X.shape[1]
            st_a = torch.full((1,), 99, dtype=torch.int32, device=DEV)
            st_n = torch.full((1,), 99, dtype=torch.int32, device=DEV)
            ref = ctx.solve_async(Xg, w.lambda0, st_a, tol=w.tol, precision=prec, out=_outs(p))
            torch.cuda.synchronize()
            got = ctx.solve_noalloc(Xg, w.lambda0, st_n, _outs(p), tol=w.tol, precision=prec)
            torch.cuda.synchronize()
            assert int(st_a.item()) == sp.OK and int(st_n.item()) == sp.OK, (name, prec)
            for t in ("B", "sigma", "Omega"):
                assert torch.equal(getattr(got, t), getattr(ref, t)), (name, prec, t)
            orc = oracle.spmesl(X, w.lambda0, tol=1e-12)
            for t in ("B", "sigma", "Omega"):
                err = rel_err(getattr(got, t).cpu().numpy(), orc[t])
                assert err <= bar, (name, prec, t, err)
    finally:
        ctx.close()


def test_noalloc_refuses_a_problem_beyond_the_scratch():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2203_15031_amd import spmesl as sp
    lib = sp.load()
    ctx = sp.Context(0)
    try:
        # n = 400, p = 5000 in the mixed form needs about 143 MiB of scratch
        X = torch.zeros((400, 5000), dtype=torch.float64, device=DEV)
        opt = ctx.options(0.2, 1e-8, "mixed")
        assert ctx.workspace_size(X, opt) > sp.NOALLOC_SCRATCH_BYTES
        status = torch.full((1,), 99, dtype=torch.int32, device=DEV)
        prob = ctx.problem(X)
        res = sp.Result(None, None, None, None)
        st = lib.spmesl_solve_noalloc(ctx._h, C.byref(prob), C.byref(opt), C.byref(res),
                                      C.c_void_p(status.data_ptr()))
        assert st == sp.ENOMEM
        torch.cuda.synchronize()
        assert int(status.item()) == 99  # nothing was enqueued
        # and the entry point still works afterwards
        Xs = torch.from_numpy(W.generate("ar1_n100_p200")).to(DEV)
        r = ctx.solve_noalloc(Xs, 0.3, status, _outs(200), precision="fp64")
        torch.cuda.synchronize()
        assert int(status.item()) == sp.OK
        assert torch.equal(r.Omega, r.Omega.T)
    finally:
        ctx.close()
