"""Estimation quality of SPMESL, as the paper's simulation study measures it.

Section 4.1 defines, and Section 4.3 reports (Tables 3-4), scores of an
estimate Omega-hat against the true precision matrix
Omega0 by edge recovery over the pairs j < k (an edge is a nonzero entry):

    SEN  = TP / (TP + FN)             SPE = TN / (TN + FP)
    FDR  = FP / (TP + FP)             MISR = (FP + FN) / (p (p - 1) / 2)
    MCC  = (TP TN - FP FN) / sqrt((TP + FP)(TP + FN)(TN + FP)(TN + FN))

(reported in percent, as in Tables 3 and 4), the number of estimated edges
|E-hat|, and the estimation error ||Omega-hat - Omega0||_F.  `simulate`
repeats the study of those tables: p = 500, n = 250, samples X ~ N(0,
Omega0^-1) for the four networks of Section 4.1 (`workloads.paper_network`),
50 datasets per network, and SPMESL at the three penalty levels lambda_pb
(SPMESL-P), lambda_univ (SPMESL-2) and lambda_ub (SPMESL-4) of Section 2.2.
The estimates come from the library's solver on the GPU; this module only
draws data and counts.

    python -m paper_2203_15031_amd.quality [--datasets 50] [--precision mixed]
"""
from __future__ import annotations

import argparse
import json
import math
import sys

import numpy as np

from . import workloads

# order of the penalty levels in the paper's tables
LEVELS = (("SPMESL-P", "pb"), ("SPMESL-2", "univ"), ("SPMESL-4", "ub"))
NETWORKS = (("AR(1)", "ar1"), ("AR(4)", "ar4"), ("Scale-Free", "sf"), ("Hub", "hub"))


def edge_counts(omega_hat: np.ndarray, omega0: np.ndarray) -> tuple[int, int, int, int]:
    """TP, FP, TN, FN over the pairs j < k (an edge is a nonzero entry)."""
    p = omega0.shape[0]
    iu = np.triu_indices(p, 1)
    est = omega_hat[iu] != 0
    true = omega0[iu] != 0
    tp = int(np.sum(est & true))
    fp = int(np.sum(est & ~true))
    tn = int(np.sum(~est & ~true))
    fn = int(np.sum(~est & true))
    return tp, fp, tn, fn


def measures(omega_hat: np.ndarray, omega0: np.ndarray) -> dict:
    """|E-hat|, SEN, SPE, FDR, MISR, MCC (percent) and ||Omega-hat - Omega0||_F.

    A ratio whose denominator is zero is reported as 0."""
    tp, fp, tn, fn = edge_counts(omega_hat, omega0)
    p = omega0.shape[0]

    def ratio(a, b):
        return 100.0 * a / b if b else 0.0

    den = math.sqrt(float(tp + fp) * (tp + fn) * (tn + fp) * (tn + fn))
    return {
        "edges": tp + fp,
        "SEN": ratio(tp, tp + fn),
        "SPE": ratio(tn, tn + fp),
        "FDR": ratio(fp, tp + fp),
        "MISR": ratio(fp + fn, p * (p - 1) // 2),
        "MCC": 100.0 * (float(tp) * tn - float(fp) * fn) / den if den else 0.0,
        "Frobenius": float(np.linalg.norm(omega_hat - omega0)),
    }


def penalty(level: str, n: int, p: int) -> float:
    """lambda_pb, lambda_univ or lambda_ub of Section 2.2 (library host helpers)."""
    from . import spmesl
    if level == "pb":
        return spmesl.lambda_pb(n, p)[0]
    if level == "univ":
        return spmesl.lambda_univ(n, p)
    if level == "ub":
        return spmesl.lambda_ub(n, p)
    raise ValueError(level)


def network(kind: str, p: int, seed: int) -> np.ndarray:
    return workloads.paper_network(kind, p, np.random.default_rng(seed))


def simulate(kind: str, datasets: int = 50, n: int = 250, p: int = 500, seed: int = 11,
             precision: str = "mixed", tol: float = 1e-8, device: int = 0) -> dict:
    """Means and standard errors of `measures` over `datasets` samples of
    one network, for each penalty level.  One network per kind (seeded), one
    sample matrix per dataset (seeded by a SeedSequence spawn)."""
    import torch
    from . import spmesl
    om0 = network(kind, p, seed)
    lams = {lv: penalty(lv, n, p) for _, lv in LEVELS}
    ctx = spmesl.Context(device)
    rows = {name: [] for name, _ in LEVELS}
    for child in np.random.SeedSequence(seed).spawn(datasets):
        X = workloads.sample_from_precision(n, om0, np.random.default_rng(child))
        Xd = torch.from_numpy(X).to(f"cuda:{device}")
        for name, lv in LEVELS:
            r = ctx.solve(Xd, lams[lv], tol, precision, want=("Omega",))
            rows[name].append(measures(r.Omega.cpu().numpy(), om0))
    out = {"network": kind, "p": p, "n": n, "datasets": datasets, "precision": precision,
           "true_edges": int(np.count_nonzero(np.triu(om0, 1))),
           "lambda": {name: lams[lv] for name, lv in LEVELS}, "levels": {}}
    for name, _ in LEVELS:
        vals = {k: np.array([m[k] for m in rows[name]], dtype=float) for k in rows[name][0]}
        out["levels"][name] = {k: (float(v.mean()), float(v.std(ddof=1) / math.sqrt(len(v))) if len(v) > 1 else 0.0)
                               for k, v in vals.items()}
    return out


def format_table(results: list[dict]) -> str:
    keys = ("edges", "SEN", "SPE", "FDR", "MISR", "MCC", "Frobenius")
    lines = ["| Network | Method | |E-hat| | SEN | SPE | FDR | MISR | MCC | Frobenius |",
             "|---|---|---:|---:|---:|---:|---:|---:|---:|"]
    for res in results:
        label = dict((k, v) for v, k in NETWORKS)[res["network"]]
        for name, _ in LEVELS:
            cells = [f"{res['levels'][name][k][0]:.2f} ({res['levels'][name][k][1]:.2f})" for k in keys]
            lines.append(f"| {label} (|E|={res['true_edges']}) | {name} | " + " | ".join(cells) + " |")
    return "\n".join(lines)


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--datasets", type=int, default=50)
    ap.add_argument("--n", type=int, default=250)
    ap.add_argument("--p", type=int, default=500)
    ap.add_argument("--seed", type=int, default=11)
    ap.add_argument("--precision", default="mixed", choices=("fp64", "fp32", "mixed"))
    ap.add_argument("--networks", default="ar1,ar4,sf,hub")
    ap.add_argument("--json", default=None, help="also write the results as JSON to this path")
    a = ap.parse_args(argv)
    results = []
    for kind in a.networks.split(","):
        res = simulate(kind, a.datasets, a.n, a.p, a.seed, a.precision)
        results.append(res)
        print(f"[quality] {kind} done", flush=True)
    print(format_table(results), flush=True)
    if a.json:
        with open(a.json, "w") as fh:
            json.dump(results, fh, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
