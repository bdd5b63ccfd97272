"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Bars (FP64 path): every iterate k equal to the oracle's iterate k within 1e-12
relative (max-norm over the mesh, relative to the largest value); converged
solutions within 1e-10 relative with the same iteration count.  Both sides run the
same number of sweeps on the same closed-form inputs; their only difference is
rounding (the library applies precomputed condensed operators, the oracle solves
with an LU factorisation every sweep), so agreement is expected at ~1e-14.
"""
import numpy as np
import pytest

from oracle import ehdg as O
from tests._cases import (gpu_transport, oracle_swe, oracle_transport, rel_err, swe_initial_fns,
                          swe_random_fns)

pytestmark = pytest.mark.gpu

ITER_TOL = 1e-12
CONV_TOL = 1e-10


def _gpu_u(prob):
    return prob.solution().cpu().numpy().reshape(prob.nel, -1)


# ------------------------------------------------------------------ transport 2D
_BETAS_2D = [(1.0, 0.5), (-0.8, 0.3), (0.4, -1.1), (-0.6, -0.9), (1.0, 0.0), (0.0, -0.7)]
# The degree-1 kernels with two active axes were running when a GPU run ended with the
# card faulted; no defect has been found in them (a host build of the same kernels under
# AddressSanitizer runs these cases in bounds and to parity), so they stay off the GPU
# until the cause is known.
_HELD = pytest.mark.skip(reason="held off the GPU: degree-1 two-axis kernels were running when a run faulted "
                                "the card; cause not found")
_CASES_2D = [pytest.param(p, b, id=f"p{p}-beta{i}",
                          marks=[_HELD] if (p == 1 and b[0] != 0.0 and b[1] != 0.0) else [])
             for i, b in enumerate(_BETAS_2D) for p in (1, 2, 3, 4, 5, 6)]


@pytest.mark.parametrize("p,beta", _CASES_2D)
def test_transport2d_iterates(p, beta):
    n, L = (13, 7), (1.0, 0.8)
    op, F, _, _ = oracle_transport(n, L, p, beta, 1.0)
    prob = gpu_transport(n, L, p, beta, 1.0)
    u = np.zeros((op.mesh.nel, op.ref.Np))
    done = 0
    for k in (1, 2, 5, 9):
        u, _ = O.iterate(op, F, u, k - done)
        prob.iterate(k - done)
        done = k
        assert rel_err(_gpu_u(prob), u) < ITER_TOL, (k, rel_err(_gpu_u(prob), u))


@pytest.mark.parametrize("n", [(8, 8), (37, 29), (64, 5)])
def test_transport2d_converged_c1(n):
    """The 8 x 8 degree-2 workload (and larger ragged meshes) solved to 1e-10."""
    p, beta, sigma = 2, (1.0, 0.5), 1.0
    op, F, ue, _ = oracle_transport(n, (1.0, 1.0), p, beta, sigma)
    ref = O.solve(op, F, np.zeros((op.mesh.nel, op.ref.Np)), tol=1e-10, max_iter=5000)
    prob = gpu_transport(n, (1.0, 1.0), p, beta, sigma)
    rc, iters, res = prob.solve(1e-10, 5000)
    assert iters == ref["iters"]
    assert rel_err(_gpu_u(prob), ref["u"]) < CONV_TOL
    hist = prob.residuals(0, iters)
    np.testing.assert_allclose(hist, ref["hist"], rtol=1e-6, atol=1e-14)


# ------------------------------------------------------------------ transport 3D
@pytest.mark.parametrize("p", [1, 2, 3, 4])
@pytest.mark.parametrize("beta", [(1.0, 0.7, 0.3), (-0.5, 0.9, -0.4), (0.0, 1.0, -0.6)])
def test_transport3d_iterates(p, beta):
    n, L = (9, 7, 5), (1.0, 1.0, 0.7)
    op, F, _, _ = oracle_transport(n, L, p, beta, 1.0)
    prob = gpu_transport(n, L, p, beta, 1.0)
    u = np.zeros((op.mesh.nel, op.ref.Np))
    done = 0
    for k in (1, 3, 7):
        u, _ = O.iterate(op, F, u, k - done)
        prob.iterate(k - done)
        done = k
        assert rel_err(_gpu_u(prob), u) < ITER_TOL, (k, rel_err(_gpu_u(prob), u))


def test_transport3d_converged_small_c3():
    n, p, beta, sigma = (6, 6, 6), 3, (1.0, 0.7, 0.3), 1.0
    op, F, _, _ = oracle_transport(n, (1.0, 1.0, 1.0), p, beta, sigma)
    ref = O.solve(op, F, np.zeros((op.mesh.nel, op.ref.Np)), tol=1e-8, max_iter=5000)
    prob = gpu_transport(n, (1.0, 1.0, 1.0), p, beta, sigma)
    rc, iters, res = prob.solve(1e-8, 5000)
    assert iters == ref["iters"]
    assert rel_err(_gpu_u(prob), ref["u"]) < CONV_TOL


def test_transport_periodic_axis():
    """A periodic axis closes the upwind chain into a cycle (no boundary data on it)."""
    n, p, beta = (10, 6), 2, (0.9, -0.4)
    op, F, _, _ = oracle_transport(n, (1.0, 1.0), p, beta, 2.0, periodic=(True, False), manufactured=False)
    rng = np.random.default_rng(4)
    u0 = rng.standard_normal((op.mesh.nel, op.ref.Np))
    import torch
    prob = gpu_transport(n, (1.0, 1.0), p, beta, 2.0, periodic=(1, 0, 0), manufactured=False)
    prob.set_initial(torch.tensor(u0.reshape(op.mesh.nel, 1, -1), device=prob.device))
    u, _ = O.iterate(op, F, u0, 6)
    prob.iterate(6)
    assert rel_err(_gpu_u(prob), u) < ITER_TOL


# ------------------------------------------------------------------ backward Euler transport
def test_transport_backward_euler_steps():
    import torch
    n, p, beta, dt = (10, 8), 3, (0.6, -0.8), 0.02
    op, F, ue, f = oracle_transport(n, (1.0, 1.0), p, beta, 0.5, dt=dt)
    u0 = op.interpolate(lambda X: np.cos(3 * X[..., 0]) * np.sin(2 * X[..., 1]))
    load = lambda um: op.load(lambda X: f(X, np), um)
    ref_u, ref_its = O.be_steps(op, u0, 4, tol=1e-10, load=load)
    prob = gpu_transport(n, (1.0, 1.0), p, beta, 0.5, dt=dt)
    prob.set_initial(torch.tensor(u0.reshape(op.mesh.nel, 1, -1), device=prob.device))
    rc, its = prob.step(4, 1e-10, 1000)
    assert its == ref_its
    assert rel_err(_gpu_u(prob), ref_u) < CONV_TOL


# ------------------------------------------------------------------ shallow water
def _gpu_swe(n, p, Phi, dt, periodic=True, L=(1.0, 1.0), precision=0, inner=1):
    from paper_1601_06681_amd.ehdg import EHDG_SWE, Problem
    per = (1, 1, 0) if periodic else (0, 0, 0)
    return Problem(EHDG_SWE, 2, n, L=L, periodic=per, degree=p, Phi=Phi, dt=dt, precision=precision,
                   inner_sweeps=inner)


@pytest.mark.parametrize("periodic", [True, False])
@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6])
def test_swe_iterates(p, periodic):
    n, Phi, dt = (11, 9), 1.3, 2e-3
    op = oracle_swe(n, p, Phi, dt, periodic)
    fns = swe_random_fns(p)
    u0 = op.interpolate([lambda X, fn=fn: fn(X, np) for fn in fns])
    F = op.load(u0)
    prob = _gpu_swe(n, p, Phi, dt, periodic)
    prob.set_initial(fns)
    u = u0
    done = 0
    for k in (1, 2, 6):
        u, _ = O.iterate(op, F, u, k - done)
        prob.iterate(k - done)
        done = k
        assert rel_err(_gpu_u(prob), u) < ITER_TOL, (k, rel_err(_gpu_u(prob), u))


@pytest.mark.parametrize("periodic", [True, False])
def test_swe_steps_hump(periodic):
    n, p, Phi, dt = (16, 16), 4, 1.0, 1e-3
    op = oracle_swe(n, p, Phi, dt, periodic)
    fns = swe_initial_fns(0)
    u0 = op.interpolate([lambda X, fn=fn: fn(X, np) for fn in fns])
    ref_u, ref_its = O.be_steps(op, u0, 5, tol=1e-10)
    prob = _gpu_swe(n, p, Phi, dt, periodic)
    prob.set_initial(fns)
    rc, its = prob.step(5, 1e-10, 1000)
    assert its == ref_its
    assert rel_err(_gpu_u(prob), ref_u) < CONV_TOL


# ------------------------------------------------------------------ mixed precision
@pytest.mark.parametrize("inner", [1, 3, 8])
def test_fp32_refine_transport(inner):
    """FP32 correction sweeps + FP64 residual refinement reach the FP64 fixed point
    within 1e-8 relative."""
    n, p, beta, sigma = (16, 16), 3, (1.0, 0.5), 1.0
    op, F, _, _ = oracle_transport(n, (1.0, 1.0), p, beta, sigma)
    ref = O.solve(op, F, np.zeros((op.mesh.nel, op.ref.Np)), tol=1e-14, max_iter=20000)
    prob = gpu_transport(n, (1.0, 1.0), p, beta, sigma, precision=1, inner=inner)
    rc, iters, res = prob.solve(1e-11, 20000)
    assert res < 1e-11
    assert rel_err(_gpu_u(prob), ref["u"]) < 1e-8


def test_fp32_refine_swe_steps():
    n, p, Phi, dt = (16, 16), 4, 1.0, 1e-3
    op = oracle_swe(n, p, Phi, dt, True)
    fns = swe_initial_fns(0)
    u0 = op.interpolate([lambda X, fn=fn: fn(X, np) for fn in fns])
    ref_u, _ = O.be_steps(op, u0, 3, tol=1e-14)
    prob = _gpu_swe(n, p, Phi, dt, True, precision=1, inner=4)
    prob.set_initial(fns)
    prob.step(3, 1e-11, 2000)
    assert rel_err(_gpu_u(prob), ref_u) < 1e-8


# ------------------------------------------------------------------ semantics
def test_deterministic_and_resumable():
    """Bitwise repeatable; iterate 20 + checkpoint + resume 20 == iterate 40."""
    import torch
    from paper_1601_06681_amd import ehdg as E
    n, p, beta = (21, 17), 3, (1.0, 0.5)
    a = gpu_transport(n, (1.0, 1.0), p, beta, 1.0)
    a.iterate(40)
    ua = a.solution()
    b = gpu_transport(n, (1.0, 1.0), p, beta, 1.0)
    b.iterate(40)
    assert torch.equal(ua, b.solution())
    c = gpu_transport(n, (1.0, 1.0), p, beta, 1.0)
    c.iterate(20)
    blob = torch.empty(E.ehdg_state_bytes(c.h), dtype=torch.uint8, device=c.device)
    E.ehdg_get_state(c.h, blob)
    d = gpu_transport(n, (1.0, 1.0), p, beta, 1.0)
    E.ehdg_set_state(d.h, blob)
    d.iterate(20)
    assert torch.equal(ua, d.solution())


def test_divergence_and_iteration_cap_are_reported():
    from paper_1601_06681_amd import ehdg as E
    # dt (p+1)(p+2)/h = 1e-2 * 30 * 32 = 9.6: the shallow-water iteration diverges
    prob = _gpu_swe((32, 32), 4, 1.0, 1e-2, True)
    prob.set_initial(swe_initial_fns(0))
    rc, iters, res = prob.solve(1e-10, 5000, allow=(E.EHDG_ERR_DIVERGED,))
    assert rc == E.EHDG_ERR_DIVERGED and not np.isfinite(res)
    c1 = gpu_transport((8, 8), (1.0, 1.0), 2, (1.0, 0.5), 1.0)
    rc, iters, res = c1.solve(1e-10, 5, allow=(E.EHDG_ERR_NOT_CONVERGED,))
    assert rc == E.EHDG_ERR_NOT_CONVERGED and iters == 5


# ------------------------------------------------------------------ full-size workloads
def test_swe_full_size_first_sweeps():
    """256^2, degree 4 (the shallow-water benchmark mesh): three sweeps from the
    Gaussian hump, every element compared with the oracle."""
    from paper_1601_06681_amd import workloads as W
    cfg = W.SWE2D
    op = oracle_swe(cfg["n"], cfg["degree"], cfg["Phi"], cfg["dt"], True)
    fns = swe_initial_fns(cfg["seed"])
    u0 = op.interpolate([lambda X, fn=fn: fn(X, np) for fn in fns])
    u, _ = O.iterate(op, op.load(u0), u0, 3)
    prob = _gpu_swe(cfg["n"], cfg["degree"], cfg["Phi"], cfg["dt"], True)
    prob.set_initial(fns)
    prob.iterate(3)
    assert rel_err(_gpu_u(prob), u) < ITER_TOL


def test_transport3d_full_size_first_sweeps():
    """64^3, degree 3 (the 3D benchmark mesh): three sweeps, every element compared."""
    from paper_1601_06681_amd import workloads as W
    cfg = W.TRANSPORT3D
    op, F, _, _ = oracle_transport(cfg["n"], cfg["L"], cfg["degree"], cfg["beta"], cfg["sigma"])
    u, _ = O.iterate(op, F, np.zeros((op.mesh.nel, op.ref.Np)), 3)
    prob = gpu_transport(cfg["n"], cfg["L"], cfg["degree"], cfg["beta"], cfg["sigma"])
    prob.iterate(3)
    assert rel_err(_gpu_u(prob), u) < ITER_TOL


# (n, p, beta): the element's own state starts at input column S = (active axes) x (face
# nodes); the one-tile-per-wavefront sweep takes the previous state rows for the increment
# from its gathered registers, by a row shuffle that depends on S mod 4
@pytest.mark.parametrize("n,p,beta", [
    ((13, 7), 3, (1.0, 0.5)),          # S = 8: 0 mod 4
    ((13, 7), 4, (0.0, -0.9)),         # S = 5: 1 mod 4
    ((13, 7), 2, (-0.8, 0.6)),         # S = 6: 2 mod 4
    ((13, 7), 2, (1.0, 0.0)),          # S = 3: 3 mod 4
    ((9, 7, 5), 2, (0.0, 1.0, -0.6)),  # S = 18: 2 mod 4
    ((9, 7, 5), 2, (1.0, 0.7, 0.3)),   # S = 27: 3 mod 4
])
def test_fp64_increments_match_oracle_history(n, p, beta):
    """The FP64 sweep's recorded relative increments over the first 10 sweeps against the
    oracle's: the same quantities in FP64, summed in another order (1e-9 relative)."""
    from paper_1601_06681_amd import ehdg as E
    L = (1.0, 0.8, 0.7)[:len(n)]
    op, F, _, _ = oracle_transport(n, L, p, beta, 1.0)
    k = 10
    ref = O.solve(op, F, np.zeros((op.mesh.nel, op.ref.Np)), tol=0.0, max_iter=k)
    prob = gpu_transport(n, L, p, beta, 1.0)
    prob.solve(0.0, k, allow=(E.EHDG_OK, E.EHDG_ERR_NOT_CONVERGED))
    np.testing.assert_allclose(prob.residuals(0, k), np.asarray(ref["hist"][:k]), rtol=1e-9)
    prob.close()


@pytest.mark.parametrize("inner", [2, 6])
def test_bf16_mfma_refine_transport3d(inner):
    """BF16 correction sweeps on MFMA (FP32 accumulation) + FP64 residual refinement
    reach the FP64 fixed point within 1e-8 relative (3D transport, degree 3)."""
    n, p, beta, sigma = (12, 10, 9), 3, (1.0, 0.7, 0.3), 1.0
    op, F, _, _ = oracle_transport(n, (1.0, 1.0, 1.0), p, beta, sigma)
    ref = O.solve(op, F, np.zeros((op.mesh.nel, op.ref.Np)), tol=1e-14, max_iter=20000)
    prob = gpu_transport(n, (1.0, 1.0, 1.0), p, beta, sigma, precision=2, inner=inner)
    rc, iters, res = prob.solve(1e-11, 50000)
    assert res < 1e-11
    assert rel_err(_gpu_u(prob), ref["u"]) < 1e-8


def test_bf16_mfma_refine_negative_beta_ragged():
    """Other flow directions and an element count that is not a multiple of 16."""
    n, p, beta, sigma = (7, 5, 3), 3, (-0.6, 0.8, -1.0), 0.5
    op, F, _, _ = oracle_transport(n, (1.0, 0.9, 0.8), p, beta, sigma)
    ref = O.solve(op, F, np.zeros((op.mesh.nel, op.ref.Np)), tol=1e-14, max_iter=20000)
    prob = gpu_transport(n, (1.0, 0.9, 0.8), p, beta, sigma, precision=2, inner=4)
    rc, iters, res = prob.solve(1e-11, 50000)
    assert rel_err(_gpu_u(prob), ref["u"]) < 1e-8


@pytest.mark.parametrize("n,p,beta", [((7, 5, 3), 3, (-0.6, 0.8, -1.0)), ((6, 5, 4), 2, (1.0, -0.5, 0.25))])
def test_fp32_refine_transport3d_ragged(n, p, beta):
    """3D FP32 correction form reaches the FP64 fixed point within 1e-8 relative: degree 3
    (the refinement after a segment's first applies the correction in its own kernel and
    gathers the corrected state) and degree 2 (the refinement adds the correction in its
    gather); element counts not a multiple of 16."""
    op, F, _, _ = oracle_transport(n, (1.0, 0.9, 0.8), p, beta, 0.5)
    ref = O.solve(op, F, np.zeros((op.mesh.nel, op.ref.Np)), tol=1e-14, max_iter=20000)
    prob = gpu_transport(n, (1.0, 0.9, 0.8), p, beta, 0.5, precision=1, inner=4)
    rc, iters, res = prob.solve(1e-11, 50000)
    assert res < 1e-11
    assert rel_err(_gpu_u(prob), ref["u"]) < 1e-8


@pytest.mark.parametrize("prec", [1, 2])
@pytest.mark.parametrize("inner", [1, 2, 4])
def test_refine_forms_transport3d_be_steps_and_resume(prec, inner):
    """Backward-Euler steps of the degree-3 3D family in the FP32 and BF16 correction
    forms: there the last correction sweep of a refinement stores s' = s + correction for
    the next refinement (stamped), and a refinement that finds no matching stamp (the
    first after a new step or a new call) applies the correction in its own pass.  With
    one sweep per refinement there is no correction sweep and the pass applies the
    residual itself; with two the only correction sweep is the one that stores s'.  Steps
    split over two calls, and a solve stopped at its iteration cap then resumed, must
    reach the oracle's FP64 results."""
    import torch
    from paper_1601_06681_amd import ehdg as E
    n, p, beta, dt = (7, 5, 4), 3, (0.8, -0.6, 0.5), 0.05
    op, F, ue, f = oracle_transport(n, (1.0, 0.9, 0.8), p, beta, 0.5, dt=dt)
    u0 = op.interpolate(lambda X: np.cos(3 * X[..., 0]) * np.sin(2 * X[..., 1]) + X[..., 2])
    load = lambda um: op.load(lambda X: f(X, np), um)
    ref_u, _ = O.be_steps(op, u0, 5, tol=1e-14, load=load)
    prob = gpu_transport(n, (1.0, 0.9, 0.8), p, beta, 0.5, dt=dt, precision=prec, inner=inner)
    prob.set_initial(torch.tensor(u0.reshape(op.mesh.nel, 1, -1), device=prob.device))
    prob.step(2, 1e-12, 4000)
    prob.step(3, 1e-12, 4000)
    assert rel_err(_gpu_u(prob), ref_u) < 1e-8
    # steady solve from zero: stopped at a cap of 3 refinements, then resumed
    op_s, F_s, _, _ = oracle_transport(n, (1.0, 0.9, 0.8), p, beta, 0.5)
    ref = O.solve(op_s, F_s, np.zeros((op_s.mesh.nel, op_s.ref.Np)), tol=1e-14, max_iter=20000)
    prob_s = gpu_transport(n, (1.0, 0.9, 0.8), p, beta, 0.5, precision=prec, inner=inner)
    rc, its, res = prob_s.solve(1e-12, 3 * inner, allow=(E.EHDG_OK, E.EHDG_ERR_NOT_CONVERGED))
    assert rc == E.EHDG_ERR_NOT_CONVERGED
    rc, its, res = prob_s.solve(1e-12, 50000)
    assert res < 1e-12
    assert rel_err(_gpu_u(prob_s), ref["u"]) < 1e-8
    prob.close()
    prob_s.close()


def test_bf16_refine_unsupported_elsewhere():
    from paper_1601_06681_amd import ehdg as E
    with pytest.raises(E.EhdgError) as ei:
        gpu_transport((8, 8), (1.0, 1.0), 2, (1.0, 0.5), 1.0, precision=2, inner=4)
    assert ei.value.code == E.EHDG_ERR_UNSUPPORTED
