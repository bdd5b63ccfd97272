"""Pins of the linearized-Euler eHDG oracle (CPU only).

* the eHDG limit equals classical DG with the upwind flux A^+ w^- + A^- w^+, assembled
  without traces (periodic and no-incoming-wave boundaries);
* entropy-only data (rho' alone, with rho0 = c0 = 1) make the Euler iteration the
  transport iteration with beta = U0 and the backward-Euler mass term, iterate by
  iterate, with u', v', p' identically zero;
* the symmetrised energy ||rho' - p'||^2 + ||u'||^2 + ||v'||^2 + ||p'||^2 does not grow
  over a backward-Euler step on a periodic mesh (rho0 = c0 = 1);
* the trace formula reproduces upwinding on each characteristic field.
"""
import numpy as np
import pytest

from oracle import ehdg as O
from oracle import fourier
from oracle.euler import Euler, abs_matrix, dg_euler, flux_matrices
from oracle.mesh import StructuredMesh
from oracle.transport import Transport


@pytest.mark.parametrize("periodic", [True, False])
@pytest.mark.parametrize("p", [1, 2, 3])
def test_fixed_point_equals_upwind_dg(p, periodic):
    m = StructuredMesh((4, 5), periodic=(periodic, periodic))
    op = Euler(m, p, (0.5, 0.25), 1.0, 0.01)
    U0 = np.random.default_rng(p).standard_normal((m.nel, 4 * op.ref.Np))
    F = op.load(U0)
    out = O.solve(op, F, U0, tol=1e-15, max_iter=3000)
    Ud = dg_euler(op, F)
    assert np.abs(out["u"] - Ud).max() / np.abs(Ud).max() < 1e-12


def test_fixed_point_general_state():
    m = StructuredMesh((5, 3), L=(1.2, 0.8), periodic=(True, False))
    op = Euler(m, 2, (-0.3, 0.6), 1.4, 0.02, rho0=1.3)
    U0 = np.random.default_rng(9).standard_normal((m.nel, 4 * op.ref.Np))
    F = op.load(U0)
    out = O.solve(op, F, U0, tol=1e-15, max_iter=3000)
    Ud = dg_euler(op, F)
    assert np.abs(out["u"] - Ud).max() / np.abs(Ud).max() < 1e-12


@pytest.mark.parametrize("U0", [(0.5, 0.25), (-0.4, 0.7)])
def test_entropy_mode_is_transport(U0):
    m = StructuredMesh((6, 5))
    p, dt = 2, 0.02
    op = Euler(m, p, U0, 1.0, dt)
    tr = Transport(m, p, U0, sigma=0.0, dt=dt)
    rho = np.random.default_rng(3).standard_normal((m.nel, op.ref.Np))
    z = np.zeros_like(rho)
    W0 = np.concatenate([rho, z, z, z], axis=1)
    we, wt = W0, rho
    Np = op.ref.Np
    for _ in range(6):
        we, _ = O.iterate(op, op.load(W0), we, 1)
        wt, _ = O.iterate(tr, tr.load(None, rho), wt, 1)
        assert np.abs(we[:, :Np] - wt).max() < 1e-12 * np.abs(wt).max()
        assert np.abs(we[:, Np:]).max() == 0.0


def test_energy_non_increasing_per_step():
    m = StructuredMesh((6, 6), periodic=(True, True))
    op = Euler(m, 3, (0.5, 0.25), 1.0, 0.01)
    Np = op.ref.Np
    u = np.random.default_rng(4).standard_normal((m.nel, 4 * Np))

    def energy(U):
        r, a, b, pp = (U[:, i * Np:(i + 1) * Np] for i in range(4))
        q = lambda X: np.einsum("ei,ij,ej->", X, op.M, X)
        return q(r - pp) + q(a) + q(b) + q(pp)

    e_prev = energy(u)
    for _ in range(4):
        u, _ = O.be_steps(op, u, 1, tol=1e-14)
        e = energy(u)
        assert e <= e_prev * (1 + 1e-12)
        e_prev = e


def test_trace_upwinds_each_characteristic():
    """what = (I+S)/2 w^- + (I-S)/2 w^+: its characteristic amplitudes are the upwind ones."""
    Ax, Ay = flux_matrices((0.5, 0.25), 1.0, 1.0)
    rng = np.random.default_rng(0)
    for nvec in ((1, 0), (-1, 0), (0, 1), (0, -1)):
        An = nvec[0] * Ax + nvec[1] * Ay
        lam, V = np.linalg.eig(An)
        S = np.linalg.solve(abs_matrix(An), An)
        wm, wp = rng.standard_normal(4), rng.standard_normal(4)
        what = 0.5 * (np.eye(4) + S) @ wm + 0.5 * (np.eye(4) - S) @ wp
        a_hat = np.linalg.solve(V, what)
        a_up = np.where(lam.real > 0, np.linalg.solve(V, wm), np.linalg.solve(V, wp))
        np.testing.assert_allclose(a_hat, a_up, atol=1e-13)


def test_fourier_rate_matches_iteration():
    N, p, dt = 6, 2, 0.01
    h = 1.0 / N
    mk = lambda mesh: Euler(StructuredMesh((3, 3), L=(3 * h, 3 * h), periodic=(True, True)), p, (0.5, 0.25), 1.0, dt)
    B0, Bf, _ = fourier.blocks(mk, 2)
    rho, _ = fourier.spectral_radius(B0, Bf, (N, N))
    m = StructuredMesh((N, N), periodic=(True, True))
    op = Euler(m, p, (0.5, 0.25), 1.0, dt)
    u = np.random.default_rng(5).standard_normal((m.nel, 4 * op.ref.Np))
    F = np.zeros_like(u)
    u, _ = O.iterate(op, F, u, 60)
    n0 = np.linalg.norm(u)
    u, _ = O.iterate(op, F, u, 40)
    observed = (np.linalg.norm(u) / n0) ** (1 / 40)
    assert abs(observed - rho) < 0.03 * rho, (observed, rho)
