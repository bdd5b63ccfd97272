"""Serving with continuous batching (paper_1601_06681_amd.serving): requests that join
and leave the batch while it runs get bit for bit the results they get alone; the
admitted workspaces never exceed the HBM budget."""
import math

import numpy as np
import pytest



def _requests():
    from paper_1601_06681_amd import workloads as W
    lam = math.hypot(*W.EULER_U0) + W.EULER_C0
    reqs = []
    for i, n in enumerate((12, 17, 9, 14)):
        reqs.append(dict(id=len(reqs), kind="euler", n=n, degree=3, steps=3 + i % 2,
                         dt=0.25 / n / (20 * lam)))
    for n in (4, 6, 5, 7):
        reqs.append(dict(id=len(reqs), kind="transport", n=n, degree=2, beta=(1.0, 0.7, 0.3), sigma=1.0))
    order = [0, 4, 1, 5, 2, 6, 3, 7]
    return [reqs[i] for i in order]


@pytest.mark.gpu
def test_served_results_equal_alone_within_budget():
    import torch
    from paper_1601_06681_amd import serving as S
    reqs = _requests()
    alone = [S.solve_alone(r, 1e-10, keep=True) for r in reqs]
    need = [S.footprint(r) for r in reqs]
    budget = sum(sorted(need)[-3:])          # at most about three members at a time
    arrivals = [0.0, 0.0, 0.002, 0.004, 0.004, 0.01, 0.02, 0.02]
    out = S.Server(budget, rounds=3).run(reqs, arrivals, keep=True)
    assert out["peak_bytes"] <= budget
    assert out["batches"] >= 3                # membership changed while running
    for i, (dt, iters, u) in enumerate(alone):
        assert torch.equal(out["solutions"][i], u), i
    assert np.all(out["latency"] > 0)


def test_fifo_latency_recursion():
    from paper_1601_06681_amd import serving as S
    lat, end = S.fifo_latencies([0.0, 1.0, 1.5, 10.0], [2.0, 1.0, 1.0, 0.5])
    np.testing.assert_allclose(lat, [2.0, 2.0, 2.5, 0.5])
    assert end == 10.5
