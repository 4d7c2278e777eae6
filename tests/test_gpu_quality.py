"""GPU: the estimation-quality measures (Section 4.1) computed from the
library's Omega-hat equal those computed from the oracle's on the same data
(the four networks of Section 4.1 at p = 100, lambda_univ), and the Table 3
and 4 study runs end to end on a few datasets."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from paper_2203_15031_amd import quality as Q
from paper_2203_15031_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2203_15031_amd import spmesl
    c = spmesl.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("kind", ["ar1", "ar4", "sf", "hub"])
@pytest.mark.parametrize("prec,bar", [("fp64", 1e-6), ("mixed", 1e-4)])
def test_measures_match_oracle(ctx, kind, prec, bar):
    n, p = 60, 100
    om0 = Q.network(kind, p, 5)
    X = W.sample_from_precision(n, om0, np.random.default_rng(17))
    lam = Q.penalty("univ", n, p)
    ref = oracle.spmesl(X, lam, tol=1e-12, original_scale=True)["Omega"]
    r = ctx.solve(torch.from_numpy(X).to("cuda:0"), lam, 1e-8, prec, want=("Omega",))
    om = r.Omega.cpu().numpy()
    assert Q.edge_counts(om, om0) == Q.edge_counts(ref, om0)
    a, b = Q.measures(om, om0), Q.measures(ref, om0)
    for k in ("edges", "SEN", "SPE", "FDR", "MISR", "MCC"):
        assert a[k] == b[k], (k, a[k], b[k])
    assert abs(a["Frobenius"] - b["Frobenius"]) <= bar * max(1.0, np.abs(ref).max()) * p


def test_simulation_runs(ctx):
    res = Q.simulate("ar1", datasets=3, n=250, p=500, precision="mixed")
    lv = res["levels"]
    assert res["true_edges"] == 499 and set(lv) == {"SPMESL-P", "SPMESL-2", "SPMESL-4"}
    # the larger the penalty level, the fewer edges (lambda_pb < lambda_univ < lambda_ub)
    assert lv["SPMESL-P"]["edges"][0] >= lv["SPMESL-2"]["edges"][0] >= lv["SPMESL-4"]["edges"][0]
    assert all(0.0 <= lv[m][k][0] <= 100.0 for m in lv for k in ("SEN", "SPE", "FDR", "MISR", "MCC"))
