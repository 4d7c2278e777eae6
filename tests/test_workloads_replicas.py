"""The replicated headline workload used by the batched benchmark figure."""
import numpy as np

from paper_2203_15031_amd import workloads as W


def test_replicas_start_with_the_workload_and_differ():
    Xs = W.generate_replicas("blockar_n400_p5000", 3)
    w = W.workload("blockar_n400_p5000")
    assert len(Xs) == 3
    assert all(X.shape == (w.n, w.p) for X in Xs)
    assert np.array_equal(Xs[0], W.generate("blockar_n400_p5000"))
    assert not np.array_equal(Xs[1], Xs[0]) and not np.array_equal(Xs[2], Xs[1])
    # deterministic in the workload's seed
    again = W.generate_replicas("blockar_n400_p5000", 3)
    assert all(np.array_equal(a, b) for a, b in zip(Xs, again))
