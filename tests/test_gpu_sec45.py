"""Sec. 4.5 on the GPU: time-dependent 3D transport, a Gaussian moving along the diagonal
of the unit cube, 8^3 hexahedra, degree 4, backward Euler with dt = 0.01, 240 steps.

The paper does not state beta; the exact solution moves with speed 0.2 per axis, read as
beta = (0.2, 0.2, 0.2) with f = 0.  Inflow data are the exact solution at the new time
level, refreshed before every step.  The paper reports 9 iterations per step under its
tolerance criterion (successive L2 errors against the exact solution differing by less
than 1e-10, the criterion of Sec. 4.1).

Checked here:
  * the library's own stopping test (relative trace increment 1e-10): the GPU's
    iterations per step equal the oracle's on the first steps, the solution after them
    agrees with the oracle's (1e-10), and over all 240 steps the count stays constant
    (the paper's observation) and the error against the exact solution stays small;
  * the paper's criterion on the first steps: one sweep at a time on the GPU, the L2
    error of each GPU iterate by the oracle's quadrature, stopping as the paper states;
    the iterations per step equal the oracle's under the same criterion (15; the paper
    prints 9, a disagreement recorded with the reading of beta).
"""
import numpy as np
import pytest

from oracle import ehdg as O
from oracle.mesh import StructuredMesh
from oracle.transport import Transport
from tests._cases import rel_err

pytestmark = pytest.mark.gpu

N, P, DT, STEPS = 8, 4, 0.01, 240
BETA = (0.2, 0.2, 0.2)


def _ue(t):
    def fn(X, xp=np):
        return xp.exp(-5 * ((X[..., 0] - 0.2 * t) ** 2 + (X[..., 1] - 0.2 * t) ** 2 + (X[..., 2] - 0.2 * t) ** 2))
    return fn


def _gpu():
    from paper_1601_06681_amd.ehdg import EHDG_TRANSPORT, Problem
    prob = Problem(EHDG_TRANSPORT, 3, (N, N, N), L=(1.0, 1.0, 1.0), degree=P, beta=BETA, sigma=0.0, dt=DT)
    prob.set_initial([_ue(0.0)])
    return prob


def _u(prob):
    return prob.solution().cpu().numpy().reshape(prob.nel, -1)


def _oracle_op(n):
    """The oracle operator of step n (t_n -> t_{n+1}), with the inflow data at t_{n+1}."""
    t1 = (n + 1) * DT
    return Transport(StructuredMesh((N, N, N)), P, BETA, sigma=0.0, dt=DT, g=lambda X: _ue(t1)(X, np))


def _err_diff(op, t):
    ex = lambda X: _ue(t)(X, np)
    return lambda un, uo: abs(O.l2_norm(op, un, ex) - O.l2_norm(op, uo, ex)) < 1e-10


def test_sec45_library_stopping_test_240_steps():
    prob = _gpu()
    its = []
    ref_u, ref_its = None, []
    for n in range(STEPS):
        prob.set_forcing(None, _ue((n + 1) * DT))
        rc, it = prob.step(1, 1e-10, 1000)
        its.append(it[0])
        if n < 3:
            op = _oracle_op(n)
            if ref_u is None:
                ref_u = op.interpolate(lambda X: _ue(0.0)(X, np))
            out = O.solve(op, op.load(None, ref_u), ref_u, tol=1e-10, max_iter=1000)
            ref_u = out["u"]
            ref_its.append(out["iters"])
            if n == 2:
                assert its == ref_its, (its, ref_its)
                assert rel_err(_u(prob), ref_u) < 1e-10
    assert max(its) - min(its) <= 1, (min(its), max(its))
    op = _oracle_op(STEPS - 1)
    err = O.l2_norm(op, _u(prob), lambda X: _ue(STEPS * DT)(X, np))
    ref = O.l2_norm(op, np.zeros_like(_u(prob)), lambda X: _ue(STEPS * DT)(X, np))
    print(f"\n[sec45] iterations per step: {its[:5]} ... {its[-5:]}")
    # backward Euler is first order in time: over T = 2.4 with dt = 0.01 its error is of
    # order T dt max|u_tt| / 2 (u_tt = (beta . grad)^2 u, about 0.1 here): a few 1e-3
    # relative to ||u||; the space error at p = 4 on 8^3 is far smaller
    assert err < 2e-2 * ref, (err, ref)
    print(f"\n[sec45] library test 1e-10: iterations per step {min(its)}..{max(its)} over {STEPS} steps, "
          f"relative L2 error at t = {STEPS * DT:.2f}: {err / ref:.2e}")
    prob.close()


def test_sec45_paper_criterion_first_steps():
    import torch
    prob = _gpu()
    steps = 3
    u_gpu = torch.as_tensor(np.ascontiguousarray(_u(prob)).reshape(prob.nel, 1, -1), device=prob.device)
    ref_u, gpu_its, ref_its = None, [], []
    for n in range(steps):
        op = _oracle_op(n)
        crit = _err_diff(op, (n + 1) * DT)
        if ref_u is None:
            ref_u = op.interpolate(lambda X: _ue(0.0)(X, np))
        out = O.solve(op, op.load(None, ref_u), ref_u, criterion=crit, max_iter=200)
        ref_u = out["u"]
        ref_its.append(out["iters"])
        # GPU: the step's iterates one sweep at a time from the traces of u^n
        prob.set_forcing(None, _ue((n + 1) * DT))
        prob.set_initial(u_gpu)
        prev, k = _u(prob), 0
        while True:
            prob.iterate(1)
            k += 1
            cur = _u(prob)
            if crit(cur, prev) or k >= 200:
                break
            prev = cur
        gpu_its.append(k)
        u_gpu = prob.solution().clone()
        assert rel_err(cur, ref_u) < 1e-10, n
    assert gpu_its == ref_its, (gpu_its, ref_its)
    print(f"\n[sec45] paper criterion: GPU iterations per step {gpu_its}, oracle {ref_its}, paper 9")
    prob.close()
