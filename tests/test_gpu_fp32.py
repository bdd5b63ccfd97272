"""Parity of the plain FP32 form (EHDG_FP32) with the FP64 oracle, through the C ABI.

The FP32 form keeps the traces, g and the condensed operator T in FP32 and
applies T on the FP32 matrix cores.  Only the increment norms of the stopping test
are accumulated in FP64, and the element solution is recovered in FP64 from the FP32
traces.  Its error against the FP64 oracle is rounding.  One sweep rounds the
operator, the data and the new traces at u = 2^-24 = 6.0e-8, and its FP32
accumulation over I inputs adds at most I u |T| |in| (random-walk sqrt(I) u in
practice).  For the families here I <= 96 and |T| |in| / |out| <= ~10, so one sweep
errs by at most ~1e-6 of max|s|.  The contraction keeps the sum of the sweeps'
errors below that bound over (1 - rho).  Bars:
  * iterates 1..9: 3e-5 of max|u| (9 sweeps x 1e-6, times the 3x gap between the
    node-value norm of u and the trace norm);
  * converged (increment 1e-6): 1e-4 of max|u| against the oracle's fixed point.
    This is the stopping error, tol rho / (1 - rho) with rho <= 0.9, plus the FP32
    fixed-point shift of ~1e-6 / (1 - rho).
"""
import numpy as np
import pytest

from oracle import ehdg as O
from tests._cases import gpu_transport, oracle_swe, oracle_transport, rel_err, swe_initial_fns, swe_random_fns

pytestmark = pytest.mark.gpu

FP32 = 3
ITER_TOL32 = 3e-5
CONV_TOL32 = 1e-4


def _u(prob):
    return prob.solution().cpu().numpy().reshape(prob.nel, -1)


@pytest.mark.parametrize("p,beta", [(2, (1.0, 0.5)), (3, (-0.8, 0.3)), (4, (0.4, -1.1)), (2, (0.0, -0.7)),
                                    (6, (-0.6, -0.9)), (1, (1.0, 0.0))])
def test_fp32_transport2d_iterates(p, beta):
    n, L = (13, 7), (1.0, 0.8)
    op, F, _, _ = oracle_transport(n, L, p, beta, 1.0)
    prob = gpu_transport(n, L, p, beta, 1.0, precision=FP32)
    u = np.zeros((op.mesh.nel, op.ref.Np))
    done = 0
    for k in (1, 2, 5, 9):
        u, _ = O.iterate(op, F, u, k - done)
        prob.iterate(k - done)
        done = k
        err = rel_err(_u(prob), u)
        assert err < ITER_TOL32, (k, err)
    prob.close()


@pytest.mark.parametrize("p,beta", [(1, (1.0, 0.7, 0.3)), (3, (1.0, 0.7, 0.3)), (4, (-0.5, 0.9, -0.4)),
                                    (2, (0.0, 1.0, -0.6))])
def test_fp32_transport3d_iterates(p, beta):
    n, L = (9, 7, 5), (1.0, 1.0, 0.7)
    op, F, _, _ = oracle_transport(n, L, p, beta, 1.0)
    prob = gpu_transport(n, L, p, beta, 1.0, precision=FP32)
    u = np.zeros((op.mesh.nel, op.ref.Np))
    done = 0
    for k in (1, 3, 7):
        u, _ = O.iterate(op, F, u, k - done)
        prob.iterate(k - done)
        done = k
        err = rel_err(_u(prob), u)
        assert err < ITER_TOL32, (k, err)
    prob.close()


# (n, p, beta): the first column of the element's own state among the inputs is
# S = (active axes) x (face nodes); the sweep takes the previous state rows for the
# increment from its gathered registers by lane transposes that depend on S mod 4
@pytest.mark.parametrize("n,p,beta", [
    ((13, 7), 3, (1.0, 0.5)),          # S = 8: 0 mod 4
    ((13, 7), 2, (-0.8, 0.6)),         # S = 6: 2 mod 4
    ((13, 7), 2, (1.0, 0.0)),          # S = 3: 3 mod 4
    ((13, 7), 4, (0.0, -0.9)),         # S = 5: 1 mod 4
    ((9, 7, 5), 2, (1.0, 0.7, 0.3)),   # S = 27: 3 mod 4
    ((9, 7, 5), 2, (0.0, 1.0, -0.6)),  # S = 18: 2 mod 4
    ((9, 7, 5), 3, (1.0, 0.7, 0.3)),   # S = 48: 0 mod 4
])
def test_fp32_increments_match_oracle_history(n, p, beta):
    """The plain FP32 sweep's recorded relative increments ||s^k - s^(k-1)|| / ||s^k||
    against the oracle's FP64 ones over the first 10 sweeps, where each is above 1e-3 and
    FP32 rounding (about 1e-7 of ||s||) moves it by less than 1e-4 of itself."""
    L = (1.0, 0.8, 0.7)[:len(n)]
    op, F, _, _ = oracle_transport(n, L, p, beta, 1.0)
    k = 10
    ref = O.solve(op, F, np.zeros((op.mesh.nel, op.ref.Np)), tol=0.0, max_iter=k)
    prob = gpu_transport(n, L, p, beta, 1.0, precision=FP32)
    from paper_1601_06681_amd import ehdg as E
    prob.solve(0.0, k, allow=(E.EHDG_OK, E.EHDG_ERR_NOT_CONVERGED))
    hist = prob.residuals(0, k)
    want = np.asarray(ref["hist"][:k])
    assert want.min() > 1e-3, want
    np.testing.assert_allclose(hist, want, rtol=1e-4)
    prob.close()


@pytest.mark.parametrize("n", [(8, 8), (37, 29)])
def test_fp32_transport2d_converged(n):
    """The 8 x 8 degree-2 workload (and a ragged mesh) solved to an increment of 1e-6:
    the sweep count is within 2 of the oracle's for the same tolerance, the solution
    within CONV_TOL32 of the oracle's fixed point, and the residual history follows
    the oracle's to 1e-3 relative plus 1e-7 absolute: rounding every new trace value
    to FP32 moves ||s^{k+1} - s^k|| by at most u ||s^{k+1}||, so the relative increment
    carries an absolute error of about u = 6e-8, which near 1e-6 exceeds 1e-3 of it."""
    p, beta, sigma = 2, (1.0, 0.5), 1.0
    op, F, _, _ = oracle_transport(n, (1.0, 1.0), p, beta, sigma)
    ref = O.solve(op, F, np.zeros((op.mesh.nel, op.ref.Np)), tol=1e-6, max_iter=5000)
    lim = O.solve(op, F, np.zeros((op.mesh.nel, op.ref.Np)), tol=1e-14, max_iter=5000)
    prob = gpu_transport(n, (1.0, 1.0), p, beta, sigma, precision=FP32)
    rc, iters, res = prob.solve(1e-6, 5000)
    assert rc == 0 and res < 1e-6
    assert abs(iters - ref["iters"]) <= 2, (iters, ref["iters"])
    assert rel_err(_u(prob), lim["u"]) < CONV_TOL32
    k = min(iters, ref["iters"]) - 2
    np.testing.assert_allclose(prob.residuals(0, k), ref["hist"][:k], rtol=1e-3, atol=1e-7)
    prob.close()


@pytest.mark.parametrize("periodic", [True, False])
@pytest.mark.parametrize("p", [2, 4, 6])
def test_fp32_swe_iterates(p, periodic):
    n, Phi, dt = (11, 9), 1.3, 2e-3
    op = oracle_swe(n, p, Phi, dt, periodic)
    fns = swe_random_fns(p)
    u0 = op.interpolate([lambda X, fn=fn: fn(X, np) for fn in fns])
    F = op.load(u0)
    from paper_1601_06681_amd.ehdg import EHDG_SWE, Problem
    prob = Problem(EHDG_SWE, 2, n, periodic=(1, 1, 0) if periodic else (0, 0, 0), degree=p, Phi=Phi, dt=dt,
                   precision=FP32)
    prob.set_initial(fns)
    u, done = u0, 0
    for k in (1, 2, 6):
        u, _ = O.iterate(op, F, u, k - done)
        prob.iterate(k - done)
        done = k
        err = rel_err(_u(prob), u)
        assert err < ITER_TOL32, (k, err)
    prob.close()


def test_fp32_swe_steps_hump():
    """Five backward-Euler steps of the Gaussian hump at an increment of 1e-6 per step:
    step counts within 1 of the oracle's at the same tolerance, the solution within
    CONV_TOL32 of the oracle's tightly converged steps."""
    from paper_1601_06681_amd.ehdg import EHDG_SWE, Problem
    n, p, Phi, dt = (16, 16), 4, 1.0, 1e-3
    op = oracle_swe(n, p, Phi, dt, True)
    fns = swe_initial_fns(0)
    u0 = op.interpolate([lambda X, fn=fn: fn(X, np) for fn in fns])
    _, its_ref = O.be_steps(op, u0, 5, tol=1e-6)
    lim_u, _ = O.be_steps(op, u0, 5, tol=1e-13)
    prob = Problem(EHDG_SWE, 2, n, periodic=(1, 1, 0), degree=p, Phi=Phi, dt=dt, precision=FP32)
    prob.set_initial(fns)
    rc, its = prob.step(5, 1e-6, 1000)
    assert rc == 0
    assert all(abs(a - b) <= 1 for a, b in zip(its, its_ref)), (its, its_ref)
    assert rel_err(_u(prob), lim_u) < CONV_TOL32
    prob.close()


def test_fp32_euler_steps():
    from oracle.euler import Euler
    from oracle.mesh import StructuredMesh
    from paper_1601_06681_amd.ehdg import EHDG_EULER, Problem
    from tests.test_gpu_euler import _fns
    n, p, dt, U0, c0 = (12, 10), 3, 4e-3, (0.5, 0.25), 1.0
    op = Euler(StructuredMesh(n, periodic=(True, True)), p, U0, c0, dt)
    fns = _fns(3)
    u0 = op.interpolate([lambda X, fn=fn: fn(X, np) for fn in fns])
    lim_u, _ = O.be_steps(op, u0, 3, tol=1e-13)
    prob = Problem(EHDG_EULER, 2, n, periodic=(1, 1, 0), degree=p, dt=dt, U0=U0, c0=c0, precision=FP32)
    prob.set_initial(fns)
    rc, its = prob.step(3, 1e-6, 1000)
    assert rc == 0
    assert rel_err(_u(prob), lim_u) < CONV_TOL32
    prob.close()


def test_fp32_tight_tolerance_keeps_fp32_accuracy():
    """A tolerance far below FP32 rounding buys no accuracy: the rounded iteration either
    stalls near u (NOT_CONVERGED at the cap) or reaches an exact fixed point of the
    rounded map (increment 0), and either way its result stays at FP32 accuracy,
    within CONV_TOL32 of the oracle's fixed point."""
    from paper_1601_06681_amd import ehdg as E
    n, p, beta, sigma = (8, 8), 2, (1.0, 0.5), 1.0
    op, F, _, _ = oracle_transport(n, (1.0, 1.0), p, beta, sigma)
    lim = O.solve(op, F, np.zeros((op.mesh.nel, op.ref.Np)), tol=1e-14, max_iter=5000)
    prob = gpu_transport(n, (1.0, 1.0), p, beta, sigma, precision=FP32)
    rc, iters, res = prob.solve(1e-12, 400, allow=(E.EHDG_OK, E.EHDG_ERR_NOT_CONVERGED))
    assert np.isfinite(res) and (res < 1e-12 or iters == 400)
    assert rel_err(_u(prob), lim["u"]) < CONV_TOL32
    prob.close()


def test_fp32_members_in_a_batch_equal_solo():
    """Plain FP32 members in a batch (the persistent FP32 sweep) give bitwise their solo
    results: iteration counts, residual histories, solutions."""
    from paper_1601_06681_amd import ehdg as E
    cases = [((13, 7), 2, (1.0, 0.5)), ((20, 11), 4, (-0.6, 0.9)), ((9, 9), 3, (0.0, -0.7))]
    solo = []
    for n, p, beta in cases:
        prob = gpu_transport(n, (1.0, 1.0), p, beta, 1.0, precision=FP32)
        rc, it, res = prob.solve(1e-6, 5000)
        solo.append((it, prob.solution().clone(), prob.residuals(0, it)))
        prob.close()
    members = [gpu_transport(n, (1.0, 1.0), p, beta, 1.0, precision=FP32) for n, p, beta in cases]
    batch = E.Batch(members)
    rc, its, _ = batch.solve(1e-6, 5000)
    assert rc == 0
    for i, prob in enumerate(members):
        assert its[i] == solo[i][0]
        assert bool((prob.solution() == solo[i][1]).all()), i
        np.testing.assert_array_equal(prob.residuals(0, its[i]), solo[i][2])
    batch.close()
    for prob in members:
        prob.close()
