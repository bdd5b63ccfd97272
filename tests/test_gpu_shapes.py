"""Launch shapes and the autotuner (ehdg_tune_set, ehdg_launch_shape, autotune.py).

Race check: the iterates must not depend on how the sweep is laid out over workgroups.
Each element's local solve reads only the previous iterate (Jacobi), so any tiles-per-
workgroup count and either workgroup order must give bitwise the same iterates.  A shape
that let a workgroup read traces another workgroup of the same launch had already
overwritten, or that skipped or doubled a tile, would show up here.  The residual norms are
summed per workgroup, so their last bits may differ between shapes: the iteration counts
must agree and the histories within 1e-12 relative.
"""
import json

import numpy as np
import pytest

from tests._cases import gpu_transport, swe_random_fns

pytestmark = pytest.mark.gpu

SHAPES = [(0, 0), (0, 1), (4, 0), (8, 1), (64, 0)]


@pytest.fixture(autouse=True)
def clean_registry():
    from paper_1601_06681_amd import ehdg as E
    E.ehdg_tune_clear()
    yield
    E.ehdg_tune_clear()


def _swe(n, p, dt, periodic, seed, precision=0):
    from paper_1601_06681_amd.ehdg import EHDG_SWE, Problem
    prob = Problem(EHDG_SWE, 2, n, periodic=(1, 1, 0) if periodic else (0, 0, 0), degree=p, Phi=1.0, dt=dt,
                   precision=precision)
    prob.set_initial(swe_random_fns(seed))
    return prob


FAMILIES = {
    "transport2d_p3": (dict(pde=0, dim=2, degree=3, precision=0),
                       lambda: gpu_transport((23, 17), (1.0, 1.0), 3, (1.0, 0.5), 1.0)),
    "transport3d_p2": (dict(pde=0, dim=3, degree=2, precision=0),
                       lambda: gpu_transport((7, 6, 5), (1.0, 1.0, 1.0), 2, (-0.5, 0.9, 0.4), 1.0)),
    "swe_walls_p2": (dict(pde=1, dim=2, degree=2, precision=0), lambda: _swe((13, 11), 2, 2e-3, False, 5)),
    "transport2d_fp32_p2": (dict(pde=0, dim=2, degree=2, precision=3),
                            lambda: gpu_transport((19, 21), (1.0, 1.0), 2, (-0.8, 0.6), 1.0, precision=3)),
}


@pytest.mark.parametrize("fam", list(FAMILIES))
def test_iterates_do_not_depend_on_the_launch_shape(fam):
    import torch
    from paper_1601_06681_amd import ehdg as E
    key, make = FAMILIES[fam]
    tol = 1e-6 if key["precision"] == 3 else 1e-10
    runs = []
    for tpg, rev in SHAPES:
        E.ehdg_tune_set(key["pde"], key["dim"], key["degree"], key["precision"], tpg, rev)
        prob = make()
        shape = E.ehdg_launch_shape(prob.h)
        assert shape[2] == rev and (tpg == 0 or shape[0] >= tpg)
        sols = []
        done = 0
        for k in (1, 5, 9):
            prob.iterate(k - done)
            done = k
            sols.append(prob.solution().clone())
        prob.close()
        prob = make()
        if key["pde"] == 1:
            rc, its = prob.step(2, tol, 1000)
            it, hist = sum(its), None
        else:
            rc, it, res = prob.solve(tol, 5000)
            hist = prob.residuals(0, it)
        runs.append((shape, sols, it, hist, prob.solution().clone()))
        prob.close()
    base = runs[0]
    assert len({r[0][1] for r in runs}) > 1  # the shapes really differ (workgroup counts)
    for shape, sols, it, hist, u in runs[1:]:
        for a, b in zip(sols, base[1]):
            assert torch.equal(a, b), shape
        assert it == base[2], (shape, it, base[2])
        assert torch.equal(u, base[4]), shape
        if hist is not None:
            np.testing.assert_allclose(hist, base[3], rtol=1e-12, atol=0)


def test_batch_uses_each_members_tuned_shape():
    """A member set up with a tuned shape gets the same shape in a batch: bitwise its solo
    result (iteration count, residual history, solution)."""
    from paper_1601_06681_amd import ehdg as E
    E.ehdg_tune_set(0, 2, 3, 0, 8, 1)
    cases = [((23, 17), 3, (1.0, 0.5)), ((12, 30), 2, (-0.4, 0.9))]
    solo = []
    for n, p, beta in cases:
        prob = gpu_transport(n, (1.0, 1.0), p, beta, 1.0)
        rc, it, res = prob.solve(1e-10, 5000)
        solo.append((it, prob.residuals(0, it), prob.solution().clone()))
        prob.close()
    members = [gpu_transport(n, (1.0, 1.0), p, beta, 1.0) for n, p, beta in cases]
    assert E.ehdg_launch_shape(members[0].h)[2] == 1
    batch = E.Batch(members)
    rc, its, _ = batch.solve(1e-10, 5000)
    for i, prob in enumerate(members):
        assert its[i] == solo[i][0]
        np.testing.assert_array_equal(prob.residuals(0, its[i]), solo[i][1])
        assert bool((prob.solution() == solo[i][2]).all())
    batch.close()
    for prob in members:
        prob.close()


def test_autotuner_picks_times_and_caches_a_shape(tmp_path):
    from paper_1601_06681_amd import autotune as A
    from paper_1601_06681_amd import ehdg as E
    path = str(tmp_path / "tune.json")
    out = A.tune(lambda: _swe((64, 64), 3, 1e-3, True, 1), 1, 2, 3, 0, sweeps=40, path=path)
    assert len(out["timings"]) == len(A.DEFAULT_CANDIDATES)
    assert all(r["sweep_us"] > 0 for r in out["timings"])
    best = out["best"]
    assert best["sweep_us"] == min(r["sweep_us"] for r in out["timings"])
    data = json.load(open(path))
    row = data[A.arch()][A.family_key(1, 2, 3, 0)]
    assert row["tiles_per_group"] == best["tiles_per_group"] and row["reverse_order"] == best["reverse_order"]
    # a problem set up now gets the tuned shape; load() re-registers it after a clear
    E.ehdg_tune_clear()
    assert A.load(path)
    prob = _swe((64, 64), 3, 1e-3, True, 1)
    tpg, groups, rev = E.ehdg_launch_shape(prob.h)
    assert rev == best["reverse_order"]
    assert best["tiles_per_group"] == 0 or tpg >= best["tiles_per_group"]
    prob.close()
    # batch mode: rounds of a batch of such problems through the batched sweep
    out = A.tune(lambda: _swe((32, 32), 3, 1e-3, True, 2), 1, 2, 3, 0, sweeps=10, candidates=((0, 0), (16, 0)),
                 save=False, batch=3)
    assert len(out["timings"]) == 2 and out["best"]["context"] == "batch"
    assert all(r["sweep_us"] > 0 for r in out["timings"])
