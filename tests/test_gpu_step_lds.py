"""The step completion with the stacked operator in LDS, through the C ABI.

A single problem whose family's stacked operator fits in LDS, on a mesh that fills at least
half of a round of that kernel's workgroups, completes its backward-Euler steps with the
operator-in-LDS kernel (each wavefront one element tile, all row tiles of the operator
applied from LDS); a batch member completes them with the shared-tile kernel.  Both take
each row tile's k tiles in the same order and add the C entries after the products, so a
problem stepped alone and as the only member of a batch must agree bitwise: iteration
counts and solution.  The batched path is pinned against the oracle by the batch tests.
"""
import numpy as np
import pytest

from tests._cases import swe_random_fns

pytestmark = pytest.mark.gpu


def _swe(n, p, dt, periodic, seed, precision=0):
    from paper_1601_06681_amd.ehdg import EHDG_SWE, Problem
    per = (1, 1, 0) if periodic else (0, 0, 0)
    prob = Problem(EHDG_SWE, 2, n, L=(1.0, 1.0), periodic=per, degree=p, Phi=1.0, dt=dt, precision=precision)
    prob.set_initial(swe_random_fns(seed))
    return prob


def _solo_equals_batch(make, steps, tol):
    from paper_1601_06681_amd.ehdg import Batch
    prob = make()
    rc, its = prob.step(steps, tol, 1000)
    assert rc == 0 and len(its) == steps and min(its) > 0
    u = prob.solution().clone()
    prob.close()
    member = make()
    batch = Batch([member])
    rc, bits = batch.step(steps, tol, 1000)
    assert rc == 0
    assert list(bits[0]) == list(its), (bits[0], its)
    assert bool((member.solution() == u).all())
    batch.close()
    member.close()


# (mesh, degree, dt, periodic): the shallow-water benchmark mesh and degree (4096 element
# tiles), a ragged non-periodic mesh (2071 tiles, the last one 3 elements), and degree 2
@pytest.mark.parametrize("n,p,dt,periodic", [
    ((256, 256), 4, 5e-5, True),
    ((181, 183), 4, 5e-5, False),
    ((256, 256), 2, 1e-4, True),
])
def test_swe_step_lds_equals_shared_tile(n, p, dt, periodic):
    print(f"swe step lds n={n} p={p}", flush=True)
    _solo_equals_batch(lambda: _swe(n, p, dt, periodic, 5), 3, 1e-10)


def test_swe_step_lds_plain_fp32_equals_shared_tile():
    """Plain FP32 traces (the FP32 state and g, FP64 contraction)."""
    print("swe step lds fp32", flush=True)
    _solo_equals_batch(lambda: _swe((256, 256), 4, 5e-5, True, 6, precision=3), 3, 1e-6)


def test_transport_be_step_lds_equals_shared_tile():
    """2D transport backward-Euler steps, degree 3 on 256 x 256."""
    import torch
    from tests._cases import gpu_transport
    print("transport be step lds", flush=True)

    def make():
        prob = gpu_transport((256, 256), (1.0, 1.0), 3, (0.6, -0.8), 0.5, dt=0.002)
        nel, np_ = prob.nel, 16
        x = torch.linspace(0.0, 1.0, nel * np_, dtype=torch.float64, device=prob.device)
        prob.set_initial(torch.cos(3.0 * x).reshape(nel, 1, np_))
        return prob
    _solo_equals_batch(make, 2, 1e-10)


def test_transport3d_be_step_lds_equals_shared_tile():
    """3D transport backward-Euler steps, degree 2 on 32^3 (every axis an inflow axis)."""
    import torch
    from tests._cases import gpu_transport
    print("transport3d be step lds", flush=True)

    def make():
        prob = gpu_transport((32, 32, 32), (1.0, 1.0, 1.0), 2, (1.0, 0.7, 0.3), 1.0, dt=0.01)
        nel, np_ = prob.nel, 27
        x = torch.linspace(0.0, 1.0, nel * np_, dtype=torch.float64, device=prob.device)
        prob.set_initial(torch.sin(5.0 * x).reshape(nel, 1, np_))
        return prob
    _solo_equals_batch(make, 2, 1e-10)


def test_euler_step_lds_equals_shared_tile():
    """Linearized Euler, degree 2 on a ragged 182 x 181 mesh with walls."""
    from paper_1601_06681_amd.ehdg import EHDG_EULER, Problem
    from tests.test_gpu_euler import C0, U0, _fns
    print("euler step lds", flush=True)

    def make():
        prob = Problem(EHDG_EULER, 2, (182, 181), L=(1.0, 1.0), periodic=(0, 0, 0), degree=2, dt=2e-4, U0=U0, c0=C0,
                       rho0=1.0)
        prob.set_initial(_fns(2))
        return prob
    _solo_equals_batch(make, 2, 1e-10)


def test_swe_full_size_steps_match_oracle():
    """The benchmark workload itself (256^2, degree 4, the Gaussian hump, dt 5e-5): two
    backward-Euler steps with the operator-in-LDS step completion against the oracle's,
    the same iteration counts and the element solution within the parity tolerance."""
    from oracle import ehdg as O
    from paper_1601_06681_amd import workloads as W
    from tests._cases import oracle_swe, rel_err, swe_initial_fns
    from tests.test_gpu_parity import CONV_TOL, _gpu_swe, _gpu_u
    print("swe full-size steps vs oracle", flush=True)
    cfg = W.SWE2D
    op = oracle_swe(cfg["n"], cfg["degree"], cfg["Phi"], cfg["dt"], True)
    fns = swe_initial_fns(cfg["seed"])
    u0 = op.interpolate([lambda X, fn=fn: fn(X, np) for fn in fns])
    ref_u, ref_its = O.be_steps(op, u0, 2, tol=1e-10)
    prob = _gpu_swe(cfg["n"], cfg["degree"], cfg["Phi"], cfg["dt"], True)
    prob.set_initial(fns)
    rc, its = prob.step(2, 1e-10, 1000)
    assert its == ref_its
    assert rel_err(_gpu_u(prob), ref_u) < CONV_TOL
    prob.close()
