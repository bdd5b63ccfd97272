"""The FP64 sweeps' lagged stopping test, through the C ABI: the launch numbering, the
partial-sum sets and the reductions that close a chunk of sweeps or a time step must
give the same iterates, residual histories and iteration counts however the work is
cut into calls, and the counts the oracle gives.

Each sweep takes the stopping test of the sweep before it; a chunk of sweeps ends with
a one-workgroup reduction; a backward-Euler step's last sweep is tested by the step
completion.  The cases below cut the same work at every such boundary.
"""
import numpy as np
import pytest

from oracle import ehdg as O
from tests._cases import gpu_transport, oracle_swe, oracle_transport, rel_err, swe_random_fns

pytestmark = pytest.mark.gpu

N, L, P, BETA = (11, 9), (1.0, 0.9), 3, (0.7, -0.4)


def _u(prob):
    return prob.solution().cpu().numpy().reshape(prob.nel, -1)


def test_iterate_in_pieces_equals_one_call():
    """12 sweeps one call at a time and in one call: bitwise equal iterates and histories."""
    a = gpu_transport(N, L, P, BETA, 0.5)
    b = gpu_transport(N, L, P, BETA, 0.5)
    for _ in range(12):
        a.iterate(1)
    b.iterate(12)
    assert a.iters() == b.iters() == 12
    np.testing.assert_array_equal(a.residuals(0, 12), b.residuals(0, 12))
    np.testing.assert_array_equal(_u(a), _u(b))
    # and against the oracle's increments of the same iterates
    op, F, _, _ = oracle_transport(N, L, P, BETA, 0.5)
    u = np.zeros((op.mesh.nel, op.ref.Np))
    s_old = op.state(u)
    want = []
    for _ in range(12):
        u = op.solve(op.rhs(F, op.trace(u)))
        s = op.state(u)
        want.append(O.rel_increment(s, s_old))
        s_old = s
    np.testing.assert_allclose(a.residuals(0, 12), want, rtol=1e-9, atol=1e-15)
    a.close()
    b.close()


def test_repeated_solve_hits_the_chunk_boundary():
    """The second solve of the same problem starts with a chunk of exactly the sweeps the
    first needed, so its stopping test falls on the chunk's closing reduction: same count,
    bitwise the same solution and history, and the oracle's count."""
    prob = gpu_transport(N, L, P, BETA, 0.5)
    tol = 1e-10
    _, it1, r1 = prob.solve(tol, 5000)
    u1, h1 = _u(prob), prob.residuals(0, it1)
    prob.set_initial(None)
    _, it2, r2 = prob.solve(tol, 5000)
    u2, h2 = _u(prob), prob.residuals(0, it2)
    assert it1 == it2
    assert r1 == r2 and r1 < tol
    np.testing.assert_array_equal(u1, u2)
    np.testing.assert_array_equal(h1, h2)
    op, F, _, _ = oracle_transport(N, L, P, BETA, 0.5)
    ref = O.solve(op, F, np.zeros((op.mesh.nel, op.ref.Np)), tol=tol)
    assert it1 == ref["iters"]
    assert rel_err(u1, ref["u"]) < 1e-10
    prob.close()


def test_iterate_then_solve_continues_the_segment():
    """A solve after 5 plain sweeps continues from them: same count and result as one solve."""
    a = gpu_transport(N, L, P, BETA, 0.5)
    b = gpu_transport(N, L, P, BETA, 0.5)
    tol = 1e-10
    a.iterate(5)
    _, ita, _ = a.solve(tol, 5000)
    _, itb, _ = b.solve(tol, 5000)
    # the solve starts a new segment from the 5th iterate: 5 + ita sweeps in all
    assert 5 + ita in (itb, itb + 1, itb - 1)
    assert rel_err(_u(a), _u(b)) < 1e-9
    a.close()
    b.close()


@pytest.mark.parametrize("cut", [[1, 1, 1, 1, 1, 1], [2, 4], [6]])
def test_steps_in_pieces(cut):
    """Six backward-Euler steps in differently cut calls: the same per-step counts and
    bitwise the same solution (the step completion takes each step's last test)."""
    from paper_1601_06681_amd.ehdg import EHDG_SWE, Problem
    n, p, Phi, dt = (12, 10), 3, 1.0, 2e-3
    fns = swe_random_fns(3)
    ref = Problem(EHDG_SWE, 2, n, periodic=(1, 1, 0), degree=p, Phi=Phi, dt=dt)
    ref.set_initial(fns)
    _, its_ref = ref.step(6, 1e-10)
    prob = Problem(EHDG_SWE, 2, n, periodic=(1, 1, 0), degree=p, Phi=Phi, dt=dt)
    prob.set_initial(fns)
    its = []
    for c in cut:
        its += prob.step(c, 1e-10)[1]
    assert its == its_ref
    np.testing.assert_array_equal(_u(prob), _u(ref))
    op = oracle_swe(n, p, Phi, dt)
    u0 = op.interpolate([lambda X, f=f: f(X, np) for f in fns])
    _, its_or = O.be_steps(op, u0, 6, tol=1e-10)
    assert its_ref == its_or
    prob.close()
    ref.close()
