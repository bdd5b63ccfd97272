"""Batches of independent problems (ehdg_batch_*), through the C ABI.

A batch advances many problems together.  A round of sweeps is one launch per family over
a (problem, tile range) table (or, switched on, one persistent launch per precision for the
2D transport and shallow-water members), replayed from a captured HIP graph.  Each member gets exactly the work it gets alone, so the bar is
bitwise: every member's iteration counts, residual history and solution equal those of the
same problem advanced on its own, with graphs or without.  One member of each batch is also
checked against the FP64 oracle (same iteration count, 1e-10).
"""
import numpy as np
import pytest

from oracle import ehdg as O
from tests._cases import gpu_transport, oracle_swe, oracle_transport, rel_err, swe_random_fns

pytestmark = pytest.mark.gpu

# mixed families (2D / 3D transport, degrees 2..4, ragged meshes, flow directions), two
# members sharing one family
STEADY = [
    dict(n=(16, 12), L=(1.0, 1.0), p=2, beta=(1.0, 0.5), sigma=1.0),
    dict(n=(9, 21), L=(1.0, 0.8), p=3, beta=(-0.7, 0.4), sigma=0.6),
    dict(n=(30, 7), L=(1.0, 1.0), p=4, beta=(0.3, -1.0), sigma=1.5),
    dict(n=(6, 5, 4), L=(1.0, 1.0, 1.0), p=2, beta=(1.0, 0.7, 0.3), sigma=1.0),
    dict(n=(17, 3), L=(1.0, 1.0), p=2, beta=(1.0, 0.5), sigma=1.0),
    dict(n=(5, 4, 3), L=(1.0, 0.9, 0.8), p=3, beta=(-0.6, 0.8, -1.0), sigma=0.5),
]


def _transport(c, **kw):
    return gpu_transport(c["n"], c["L"], c["p"], c["beta"], c["sigma"], **kw)


def _u(prob):
    return prob.solution().cpu().numpy().reshape(prob.nel, -1)


def test_batch_solve_equals_solo_and_oracle():
    from paper_1601_06681_amd.ehdg import Batch
    solo = []
    for c in STEADY:
        prob = _transport(c)
        rc, it, res = prob.solve(1e-10, 5000)
        solo.append((it, res, prob.solution().clone(), prob.residuals(0, it)))
        prob.close()
    members = [_transport(c) for c in STEADY]
    batch = Batch(members)
    rc, its, ress = batch.solve(1e-10, 5000)
    assert rc == 0
    for i, prob in enumerate(members):
        it, res, u, hist = solo[i]
        assert its[i] == it, (i, its[i], it)
        assert ress[i] == res
        assert bool((prob.solution() == u).all()), i
        np.testing.assert_array_equal(prob.residuals(0, it), hist)
    c = STEADY[1]
    op, F, _, _ = oracle_transport(c["n"], c["L"], c["p"], c["beta"], c["sigma"])
    ref = O.solve(op, F, np.zeros((op.mesh.nel, op.ref.Np)), tol=1e-10, max_iter=5000)
    assert its[1] == ref["iters"]
    assert rel_err(_u(members[1]), ref["u"]) < 1e-10
    batch.close()


def _swe(n, p, dt, periodic, seed):
    from paper_1601_06681_amd.ehdg import EHDG_SWE, Problem
    per = (1, 1, 0) if periodic else (0, 0, 0)
    prob = Problem(EHDG_SWE, 2, n, L=(1.0, 1.0), periodic=per, degree=p, Phi=1.0, dt=dt)
    prob.set_initial(swe_random_fns(seed))
    return prob


def _be_members():
    import torch
    out = [lambda: _swe((16, 16), 3, 1e-3, True, 1), lambda: _swe((12, 10), 2, 2e-3, False, 2),
           lambda: _swe((9, 13), 4, 5e-4, True, 3)]

    def transport_be():
        c = dict(n=(10, 8), L=(1.0, 1.0), p=3, beta=(0.6, -0.8), sigma=0.5)
        op, F, ue, f = oracle_transport(c["n"], c["L"], c["p"], c["beta"], c["sigma"], dt=0.02)
        u0 = op.interpolate(lambda X: np.cos(3 * X[..., 0]) * np.sin(2 * X[..., 1]))
        prob = _transport(c, dt=0.02)
        prob.set_initial(torch.tensor(u0.reshape(op.mesh.nel, 1, -1), device=prob.device))
        return prob
    out.append(transport_be)
    return out


def test_batch_step_equals_solo_and_oracle():
    from paper_1601_06681_amd.ehdg import Batch
    makers = _be_members()
    solo = []
    for mk in makers:
        prob = mk()
        rc, its = prob.step(4, 1e-10, 1000)
        solo.append((its, prob.solution().clone()))
        prob.close()
    members = [mk() for mk in makers]
    batch = Batch(members)
    rc, its = batch.step(4, 1e-10, 1000)
    assert rc == 0
    for i, prob in enumerate(members):
        assert its[i] == solo[i][0], (i, its[i], solo[i][0])
        assert bool((prob.solution() == solo[i][1]).all()), i
    # two more steps continue each member from where the batch left it
    rc, its2 = batch.step(2, 1e-10, 1000)
    assert rc == 0 and all(len(v) == 2 and min(v) > 0 for v in its2)
    # member 0 against the oracle over the first 4 steps
    op = oracle_swe((16, 16), 3, 1.0, 1e-3, True)
    fns = swe_random_fns(1)
    u0 = op.interpolate([lambda X, fn=fn: fn(X, np) for fn in fns])
    ref_u, ref_its = O.be_steps(op, u0, 4, tol=1e-10)
    assert its[0] == ref_its
    batch.close()


def test_batch_iteration_cap_and_refinement_member():
    from paper_1601_06681_amd import ehdg as E
    members = [_transport(c) for c in STEADY[:3]]
    batch = E.Batch(members)
    rc, its, ress = batch.solve(1e-10, 5, allow=(E.EHDG_OK, E.EHDG_ERR_NOT_CONVERGED))
    assert rc == E.EHDG_ERR_NOT_CONVERGED and its == [5, 5, 5]
    batch.close()
    low = _transport(STEADY[0], precision=1, inner=2)
    with pytest.raises(E.EhdgError) as ei:
        E.Batch([members[0], low])
    assert ei.value.code == E.EHDG_ERR_UNSUPPORTED
    with pytest.raises(E.EhdgError) as ei:
        E.Batch([members[0], members[0]])
    assert ei.value.code == E.EHDG_ERR_INVALID_ARG


def test_batch_mixed_precision_steps_equal_solo():
    """FP64 and plain FP32 shallow-water members in one batch, stepped at one tolerance
    (1e-6, within reach of both precisions): the FP32 members' sweeps run in the FP32
    batched sweep and their step completions in the FP32 step kernel; every member equals
    its solo run at the same tolerance bitwise."""
    from paper_1601_06681_amd.ehdg import EHDG_SWE, Batch, Problem

    def mk(n, p, dt, prec, seed):
        prob = Problem(EHDG_SWE, 2, n, L=(1.0, 1.0), periodic=(1, 1, 0), degree=p, Phi=1.0, dt=dt, precision=prec)
        prob.set_initial(swe_random_fns(seed))
        return prob
    specs = [((16, 16), 3, 1e-3, 3, 1), ((12, 10), 2, 2e-3, 0, 2), ((9, 13), 4, 5e-4, 3, 3), ((11, 7), 1, 1e-3, 0, 4)]
    tol = 1e-6
    solo = []
    for sp in specs:
        prob = mk(*sp)
        rc, its = prob.step(3, tol, 1000)
        solo.append((its, prob.solution().clone()))
        prob.close()
    members = [mk(*sp) for sp in specs]
    batch = Batch(members)
    rc, its = batch.step(3, tol, 1000)
    assert rc == 0
    for i, prob in enumerate(members):
        assert its[i] == solo[i][0], (i, its[i], solo[i][0])
        assert bool((prob.solution() == solo[i][1]).all()), i
    batch.close()
    for prob in members:
        prob.close()


def test_batch_graph_replays_equal_eager_launches():
    """The rounds replayed from the captured graph give bitwise the eager launches' results,
    over several calls with unrelated eager GPU work and synchronizations between them:
    advance (sweeps and step completions in every round), then solve."""
    import torch
    from paper_1601_06681_amd.ehdg import Batch
    def members():
        out = [_transport(c) for c in STEADY[:3]] + [mk() for mk in _be_members()[:2]]
        return out
    runs = []
    for graph in (True, False):
        ms = members()
        batch = Batch(ms)
        batch.set_graph(graph)
        states, sols = [], []
        for k in range(4):
            x = torch.randn(1 << 20, device=ms[0].device)
            y = (x * 2.0).sum()                       # eager work between replays
            torch.cuda.synchronize()
            states.append(batch.advance(7, 1e-10, step_targets=[10 ** 6] * len(ms)))
            sols.append([p.solution().clone() for p in ms])
            del x, y
        runs.append((states, sols))
        batch.close()
        for p in ms:
            p.close()
    (s1, u1), (s2, u2) = runs
    assert s1 == s2
    for a, b in zip(u1, u2):
        for x, y in zip(a, b):
            assert torch.equal(x, y)


def _pinned_reports(batch, count):
    import torch
    return [torch.empty(batch.report_bytes(), dtype=torch.uint8, pin_memory=True) for _ in range(count)]


def test_async_launches_equal_advance_and_retire_members_early():
    """ehdg_batch_launch / _poll / _get_solution: three launches queued ahead, reports read
    in order without waiting, each member retired from the first report that shows it
    finished while later launches are still queued.  The retired solutions and the
    members' iteration counts equal those of the same batch driven by ehdg_batch_advance
    (and so those of each problem alone), bitwise."""
    import torch
    from paper_1601_06681_amd import ehdg as E

    def members():
        return [_transport(c) for c in STEADY[:4]] + [mk() for mk in _be_members()[:3]]
    targets = [0, 0, 0, 0, 4, 3, 5]
    ref = members()
    rb = E.Batch(ref)
    while True:
        st = rb.advance(16, 1e-10, targets)
        if all(s == 1 for s in st):
            break
    ref_u = [p.solution().clone() for p in ref]
    ref_it = [p.iters() for p in ref]
    rb.close()

    ms = members()
    b = E.Batch(ms)
    b.set_graph(False)
    reps = _pinned_reports(b, 3)
    inflight = []
    for r in reps:
        b.launch(16, 1e-10, targets, r)
        inflight.append(r)
    with pytest.raises(E.EhdgError) as ei:       # a report buffer of a pending launch
        b.launch(16, 1e-10, targets, reps[0])
    assert ei.value.code == E.EHDG_ERR_INVALID_ARG
    with pytest.raises(E.EhdgError) as ei:       # synchronous calls wait for the reports
        b.advance(1, 1e-10, targets)
    assert ei.value.code == E.EHDG_ERR_INVALID_ARG
    got, polls, reports = {}, 0, 0
    while len(got) < len(ms):
        st = b.poll()
        polls += 1
        if st is None:
            continue
        reports += 1
        r = inflight.pop(0)
        for k, s in enumerate(st):
            assert s in (0, 1)
            if s == 1 and k not in got:
                got[k] = b.solution(k)
        if len(got) < len(ms):
            b.launch(16, 1e-10, targets, r)
            inflight.append(r)
    while inflight:                              # drain the launches still queued
        if b.poll() is not None:
            inflight.pop(0)
    with pytest.raises(E.EhdgError) as ei:       # nothing pending
        b.poll()
    assert ei.value.code == E.EHDG_ERR_INVALID_ARG
    assert reports >= 2 and polls >= reports
    torch.cuda.synchronize()
    for k, p in enumerate(ms):
        assert torch.equal(got[k], ref_u[k]), k
        assert p.iters() == ref_it[k], k
    b.close()
    for p in ref + ms:
        p.close()


def test_async_solution_needs_a_finished_report():
    import torch
    from paper_1601_06681_amd import ehdg as E
    ms = [_transport(c) for c in STEADY[:2]]
    b = E.Batch(ms)
    out = torch.empty(ms[0].nel, ms[0].m, ms[0].Np, dtype=torch.float64, device=ms[0].device)
    with pytest.raises(E.EhdgError) as ei:       # no report read yet
        b.solution(0, out)
    assert ei.value.code == E.EHDG_ERR_INVALID_ARG
    rep = _pinned_reports(b, 1)[0]
    b.launch(2, 1e-10, None, rep)                # steady members: no step targets needed
    st = None
    while st is None:
        st = b.poll()
    assert st == [0, 0]                          # two rounds: nobody has converged
    with pytest.raises(E.EhdgError) as ei:
        b.solution(1, out)
    assert ei.value.code == E.EHDG_ERR_INVALID_ARG
    b.close()
    be = [mk() for mk in _be_members()[:1]]
    bb = E.Batch(be)
    with pytest.raises(E.EhdgError) as ei:       # backward-Euler members need targets
        bb.launch(2, 1e-10, None, _pinned_reports(bb, 1)[0])
    assert ei.value.code == E.EHDG_ERR_INVALID_ARG
    bb.close()
    for p in ms + be:
        p.close()


def test_persistent_and_per_family_launches_agree():
    """2D transport and shallow-water members (FP64 and plain FP32) swept by the persistent
    launch and by one launch per family: bitwise the same iterates, counts and histories."""
    import torch
    from paper_1601_06681_amd.ehdg import EHDG_SWE, Batch, Problem

    def members():
        out = [_transport(c, precision=prec) for c in STEADY[:3] if len(c["n"]) == 2 for prec in (0, 3)]
        for n, p, prec, seed in (((12, 10), 2, 0, 1), ((9, 13), 3, 3, 2)):
            prob = Problem(EHDG_SWE, 2, n, L=(1.0, 1.0), periodic=(1, 1, 0), degree=p, Phi=1.0, dt=1e-3,
                           precision=prec)
            prob.set_initial(swe_random_fns(seed))
            out.append(prob)
        return out
    runs = []
    for persist in (True, False):
        ms = members()
        b = Batch(ms)
        b.set_persistent(persist)
        st = b.advance(40, 1e-6, [0] * 6 + [3, 3])
        runs.append((st, [p.iters() for p in ms], [p.solution().clone() for p in ms],
                     [p.residuals(0, min(p.iters(), 8)) if p.pde == 0 else None for p in ms]))
        b.close()
        for p in ms:
            p.close()
    (s1, i1, u1, h1), (s2, i2, u2, h2) = runs
    assert s1 == s2 and i1 == i2
    for a, c in zip(u1, u2):
        assert torch.equal(a, c)
    for a, c in zip(h1, h2):
        if a is not None:
            np.testing.assert_array_equal(a, c)
