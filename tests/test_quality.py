"""Edge-recovery measures and Frobenius error (Section 4.1), pinned by hand
counts on a small example, by their limiting cases, and the generators by
the true edge counts the paper prints for its networks (Tables 3 and 4)."""
import math

import numpy as np

from paper_2203_15031_amd import quality as Q
from paper_2203_15031_amd import workloads as W


def test_hand_example():
    # true edges (0,1), (1,2); estimated edges (0,1), (2,3) over p = 4:
    # TP 1, FP 1 (2,3), FN 1 (1,2), TN 6 - 3 = 3
    om0 = np.eye(4)
    om0[0, 1] = om0[1, 0] = 0.4
    om0[1, 2] = om0[2, 1] = -0.3
    est = np.eye(4) * 2.0
    est[0, 1] = est[1, 0] = 0.1
    est[2, 3] = est[3, 2] = 0.2
    assert Q.edge_counts(est, om0) == (1, 1, 3, 1)
    m = Q.measures(est, om0)
    assert m["edges"] == 2
    assert math.isclose(m["SEN"], 50.0) and math.isclose(m["SPE"], 75.0)
    assert math.isclose(m["FDR"], 50.0) and math.isclose(m["MISR"], 100.0 * 2 / 6)
    # (1 * 3 - 1 * 1) / sqrt(2 * 2 * 4 * 4) = 2 / 8
    assert math.isclose(m["MCC"], 25.0)
    # diagonal 1 -> 2 on four entries, (0,1) 0.4 -> 0.1 twice, (1,2) -0.3 -> 0
    # twice, (2,3) 0 -> 0.2 twice
    fro = math.sqrt(4 * 1.0 + 2 * 0.09 + 2 * 0.09 + 2 * 0.04)
    assert math.isclose(m["Frobenius"], fro)


def test_limiting_cases():
    om0 = np.eye(6)
    om0[0, 3] = om0[3, 0] = 0.5
    om0[4, 5] = om0[5, 4] = 0.2
    m = Q.measures(om0.copy(), om0)
    assert m["SEN"] == 100.0 and m["SPE"] == 100.0 and m["FDR"] == 0.0
    assert m["MISR"] == 0.0 and math.isclose(m["MCC"], 100.0) and m["Frobenius"] == 0.0
    # no estimated edge: nothing found, no false discovery, MCC undefined -> 0
    m = Q.measures(np.eye(6), om0)
    assert m["edges"] == 0 and m["SEN"] == 0.0 and m["FDR"] == 0.0 and m["MCC"] == 0.0
    assert math.isclose(m["MISR"], 100.0 * 2 / 15)
    # every pair estimated: all true edges found, SPE 0
    full = np.ones((6, 6))
    m = Q.measures(full, om0)
    assert m["SEN"] == 100.0 and m["SPE"] == 0.0 and math.isclose(m["FDR"], 100.0 * 13 / 15)


def test_networks_true_edge_counts():
    # |E| of the paper's tables at p = 500: AR(1) 499, AR(4) 1990, scale-free
    # 495 (five 100-node trees); hubs vary with the draw (551 in the paper)
    counts = {k: int(np.count_nonzero(np.triu(Q.network(k, 500, 11), 1))) for _, k in Q.NETWORKS}
    assert counts["ar1"] == 499 and counts["ar4"] == 1990 and counts["sf"] == 495
    assert 500 <= counts["hub"] <= 600
    for _, k in Q.NETWORKS:
        om = Q.network(k, 500, 11)
        assert np.allclose(om, om.T) and np.linalg.eigvalsh(om).min() > 0


def test_scale_free_steps_alone_positive_definite():
    # The stated steps (i)-(iv) give a positive definite precision matrix for
    # the scale-free trees drawn for the study: no diagonal shift is applied
    # to them (unit diagonal), unlike the hub subnetworks.
    om = Q.network("sf", 500, 11)
    assert np.array_equal(np.diag(om), np.ones(500))
    assert np.linalg.eigvalsh(om).min() > 0.05
    hub = Q.network("hub", 500, 11)
    assert np.diag(hub).min() > 1.0
    # with linear preferential attachment (the Barabasi-Albert model) the
    # steps alone fail for most 100-node trees: their hubs have many leaves
    rng = np.random.default_rng(5)
    pd = 0
    for _ in range(40):
        T = W.subnetwork_precision(W._tree_edges(100, rng, power=1.0), 100, rng)
        pd += np.linalg.eigvalsh(T).min() > 0
    assert pd <= 8
