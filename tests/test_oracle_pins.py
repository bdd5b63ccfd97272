"""Pins of the oracle's eHDG iteration to results fixed by mathematics (CPU only).

Each test checks the oracle against something other than itself:
* the eHDG limit against two direct global solves (upwind HDG with the trace as an
  unknown, and classical upwind/Godunov DG with no trace at all);
* optimal h-convergence on manufactured solutions;
* the closed-form p = 0 iteration in 1D;
* monotone decay of the |beta.n|-weighted trace error (energy argument of Theorem 1);
* the Bloch-wave spectral radius against the observed asymptotic rate, the
  p = 0 closed form 2 dt / h, and Theorem 2's contraction bound;
* conservation identities of both operators.
"""
import numpy as np
import pytest

from oracle import direct, ehdg, fourier
from oracle.mesh import StructuredMesh
from oracle.swe import ShallowWater
from oracle.transport import Transport

pi = np.pi


def _c1_like(b, sig):
    ue = lambda X: np.sin(pi * X[..., 0]) * np.cos(pi * X[..., 1])
    f = lambda X: (b[0] * pi * np.cos(pi * X[..., 0]) * np.cos(pi * X[..., 1])
                   - b[1] * pi * np.sin(pi * X[..., 0]) * np.sin(pi * X[..., 1]) + sig * ue(X))
    return ue, f


def _c3_like(b, sig):
    ue = lambda X: np.sin(pi * X[..., 0]) * np.cos(pi * X[..., 1]) * np.sin(pi * X[..., 2])
    f = lambda X: (b[0] * pi * np.cos(pi * X[..., 0]) * np.cos(pi * X[..., 1]) * np.sin(pi * X[..., 2])
                   - b[1] * pi * np.sin(pi * X[..., 0]) * np.sin(pi * X[..., 1]) * np.sin(pi * X[..., 2])
                   + b[2] * pi * np.sin(pi * X[..., 0]) * np.cos(pi * X[..., 1]) * np.cos(pi * X[..., 2])
                   + sig * ue(X))
    return ue, f


# ---------------------------------------------------------------------------- P1/P2
@pytest.mark.parametrize("p", [1, 2, 3, 4])
@pytest.mark.parametrize("b", [(1.0, 0.5), (-0.7, 0.4), (0.3, -1.0)])
def test_transport2d_fixed_point_equals_direct_solves(p, b):
    ue, f = _c1_like(b, 1.0)
    m = StructuredMesh((4, 4))
    op = Transport(m, p, b, sigma=1.0, g=ue)
    F = op.load(f)
    out = ehdg.solve(op, F, np.zeros((m.nel, op.ref.Np)), tol=1e-15, max_iter=3000)
    Uh = direct.hdg_transport(op, F)
    Ud = direct.dg_transport(op, F)
    scale = np.abs(Uh).max()
    assert np.abs(out["u"] - Uh).max() / scale < 1e-12
    assert np.abs(Ud - Uh).max() / scale < 1e-12


@pytest.mark.parametrize("p", [1, 2, 3])
def test_transport3d_fixed_point_equals_direct_solves(p):
    b = (1.0, 0.7, 0.3)
    ue, f = _c3_like(b, 1.0)
    m = StructuredMesh((2, 3, 2))
    op = Transport(m, p, b, sigma=1.0, g=ue)
    F = op.load(f)
    out = ehdg.solve(op, F, np.zeros((m.nel, op.ref.Np)), tol=1e-15, max_iter=3000)
    Uh = direct.hdg_transport(op, F)
    Ud = direct.dg_transport(op, F)
    scale = np.abs(Uh).max()
    assert np.abs(out["u"] - Uh).max() / scale < 1e-12
    assert np.abs(Ud - Uh).max() / scale < 1e-12


def test_transport_backward_euler_fixed_point():
    b = (1.0, -0.5)
    m = StructuredMesh((4, 4))
    op = Transport(m, 2, b, sigma=0.0, dt=0.05, g=lambda X: np.cos(X[..., 0] + X[..., 1]))
    rng = np.random.default_rng(1)
    um = rng.standard_normal((m.nel, op.ref.Np))
    F = op.load(None, um)
    out = ehdg.solve(op, F, um, tol=1e-15, max_iter=3000)
    Uh = direct.hdg_transport(op, F)
    assert np.abs(out["u"] - Uh).max() / np.abs(Uh).max() < 1e-12


@pytest.mark.parametrize("periodic", [True, False])
@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_swe_fixed_point_equals_direct_solves(p, periodic):
    m = StructuredMesh((4, 4), periodic=(periodic, periodic))
    op = ShallowWater(m, p, 1.0, 1e-3)
    U0 = np.random.default_rng(p).standard_normal((m.nel, 3 * op.ref.Np))
    F = op.load(U0)
    out = ehdg.solve(op, F, U0, tol=1e-15, max_iter=3000)
    Uh = direct.hdg_swe(op, F)
    Ud = direct.dg_swe(op, F)
    scale = np.abs(Uh).max()
    assert np.abs(out["u"] - Uh).max() / scale < 1e-12
    assert np.abs(Ud - Uh).max() / scale < 1e-12


def test_swe_fixed_point_general_phi():
    m = StructuredMesh((3, 4), L=(1.5, 2.0), periodic=(True, True))
    op = ShallowWater(m, 3, 2.5, 4e-3)
    U0 = np.random.default_rng(7).standard_normal((m.nel, 3 * op.ref.Np))
    F = op.load(U0)
    out = ehdg.solve(op, F, U0, tol=1e-15, max_iter=3000)
    Ud = direct.dg_swe(op, F)
    assert np.abs(out["u"] - Ud).max() / np.abs(Ud).max() < 1e-12


# ---------------------------------------------------------------------------- P6
@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_transport2d_optimal_rate(p):
    b = (1.0, 0.5)
    ue, f = _c1_like(b, 1.0)
    errs = []
    for N in (4, 8, 16):
        m = StructuredMesh((N, N))
        op = Transport(m, p, b, sigma=1.0, g=ue)
        out = ehdg.solve(op, op.load(f), np.zeros((m.nel, op.ref.Np)), tol=1e-14, max_iter=3000)
        errs.append(ehdg.l2_norm(op, out["u"], ue))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(rates - (p + 1)) < 0.3), rates


@pytest.mark.parametrize("p", [1, 2])
def test_transport3d_optimal_rate(p):
    b = (1.0, 0.7, 0.3)
    ue, f = _c3_like(b, 1.0)
    errs = []
    for N in (2, 4, 8):
        m = StructuredMesh((N, N, N))
        op = Transport(m, p, b, sigma=1.0, g=ue)
        out = ehdg.solve(op, op.load(f), np.zeros((m.nel, op.ref.Np)), tol=1e-14, max_iter=3000)
        errs.append(ehdg.l2_norm(op, out["u"], ue))
    rate = np.log2(errs[1] / errs[2])
    assert abs(rate - (p + 1)) < 0.35, errs


@pytest.mark.parametrize("p", [1, 2, 3])
def test_swe_single_step_spatial_rate(p):
    """One backward-Euler step with forcing chosen so the exact discrete-in-time
    solution is a given smooth field: isolates the spatial error (rate p+1)."""
    Phi, dt = 1.0, 1e-3     # dt (p+1)(p+2)/h < 1 on every mesh, so the iteration converges
    ph = lambda X: np.cos(2 * pi * X[..., 0]) * np.sin(2 * pi * X[..., 1])
    uu = lambda X: np.sin(2 * pi * X[..., 0]) * np.cos(2 * pi * X[..., 1])
    vv = lambda X: np.cos(2 * pi * X[..., 0] + 2 * pi * X[..., 1])
    # residual of the BE-discretised PDE with u^m = 0 and u^{m+1} = (ph, uu, vv):
    #   ph/dt + Phi (u_x + v_y) = r1,  u/dt + ph_x = r2,  v/dt + ph_y = r3
    def r1(X):
        x, y = X[..., 0], X[..., 1]
        ux = 2 * pi * np.cos(2 * pi * x) * np.cos(2 * pi * y)
        vy = -2 * pi * np.sin(2 * pi * x + 2 * pi * y)
        return ph(X) / dt + Phi * (ux + vy)
    def r2(X):
        return uu(X) / dt - 2 * pi * np.sin(2 * pi * X[..., 0]) * np.sin(2 * pi * X[..., 1])
    def r3(X):
        return vv(X) / dt + 2 * pi * np.cos(2 * pi * X[..., 0]) * np.cos(2 * pi * X[..., 1])
    errs = []
    for N in (4, 8, 16):
        m = StructuredMesh((N, N), periodic=(True, True))
        op = ShallowWater(m, p, Phi, dt)
        Xq = m.physical(np.arange(m.nel), op.ref.xi_q)
        w = op.ref.w_q * op.J
        F = np.concatenate([(r1(Xq) * w) @ op.Psi_q, Phi * (r2(Xq) * w) @ op.Psi_q,
                            Phi * (r3(Xq) * w) @ op.Psi_q], axis=1)
        U0 = np.zeros((m.nel, 3 * op.ref.Np))
        out = ehdg.solve(op, F, U0, tol=1e-14, max_iter=3000)
        Np = op.ref.Np
        e = [ehdg.l2_norm(op, out["u"][:, i * Np:(i + 1) * Np], fn) for i, fn in enumerate((ph, uu, vv))]
        errs.append(np.sqrt(np.sum(np.square(e))))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert rates[-1] > p + 1 - 0.35, (errs, rates)


# ---------------------------------------------------------------------------- P3
@pytest.mark.parametrize("sig", [0.0, 1.0, 3.0])
def test_p0_1d_closed_form_iteration(sig):
    """p = 0, beta > 0 in 1D: e_j^{k+1} = (e_j^k + e_{j-1}^k) / (2 + sigma h / beta)."""
    N, beta = 12, 0.8
    m = StructuredMesh((N,))
    op = Transport(m, 0, (beta,), sigma=sig)
    h = 1.0 / N
    e = np.random.default_rng(0).standard_normal((N, 1))
    F = np.zeros_like(e)
    for _ in range(5):
        e_next, _ = ehdg.iterate(op, F, e, 1)
        expect = (e[:, 0] + np.concatenate([[0.0], e[:-1, 0]])) / (2 + sig * h / beta)
        np.testing.assert_allclose(e_next[:, 0], expect, rtol=1e-13, atol=1e-15)
        e = e_next


# ---------------------------------------------------------------------------- P4
def _weighted_trace_energy(op, S):
    """sum over faces of int |beta.n| (state error)^2 for constant beta."""
    E = 0.0
    for f in range(2 * op.d):
        if op.bn[f] <= 0:
            continue
        pts, wf, Pf, Mu = op.face[f]
        Mf = np.einsum("q,qa,qb->ab", wf, Mu, Mu)
        E += op.bn[f] * np.einsum("ea,ab,eb->", S[:, f], Mf, S[:, f])
    return E


@pytest.mark.parametrize("d,p,b,sig", [(2, 1, (1.0, 0.5), 0.0), (2, 3, (-0.4, 1.0), 1.0),
                                       (2, 4, (1.0, 1.0), 0.0), (3, 2, (1.0, 0.7, 0.3), 1.0)])
def test_trace_error_energy_is_non_increasing(d, p, b, sig):
    n = (5, 4) if d == 2 else (3, 3, 2)
    m = StructuredMesh(n)
    op = Transport(m, p, b, sigma=sig)
    F = np.zeros((m.nel, op.ref.Np))
    u = np.random.default_rng(3).standard_normal((m.nel, op.ref.Np))
    E_prev = _weighted_trace_energy(op, op.state(u))
    for _ in range(40):
        u, _ = ehdg.iterate(op, F, u, 1)
        E = _weighted_trace_energy(op, op.state(u))
        assert E <= E_prev * (1 + 1e-12) + 1e-300
        E_prev = E


# ---------------------------------------------------------------------------- P12/P15
def _swe_blocks(p, h, dt, Phi=1.0):
    mk = lambda mesh: ShallowWater(StructuredMesh((3, 3), L=(3 * h, 3 * h), periodic=(True, True)), p, Phi, dt)
    B0, Bf, _ = fourier.blocks(mk, 2)
    return B0, Bf


@pytest.mark.parametrize("N,dt", [(8, 0.1), (8, 0.05), (16, 0.02)])
def test_swe_p0_spectral_radius_closed_form(N, dt):
    """p = 0: the checkerboard velocity mode is amplified by -2 dt / h."""
    B0, Bf = _swe_blocks(0, 1.0 / N, dt)
    rho, _ = fourier.spectral_radius(B0, Bf, (N, N))
    assert abs(rho - 2 * dt / (1.0 / N)) < 1e-12


@pytest.mark.parametrize("p,dt", [(1, 0.02), (2, 0.01), (3, 0.004)])
def test_swe_fourier_radius_matches_observed_rate(p, dt):
    N = 6
    B0, Bf = _swe_blocks(p, 1.0 / N, dt)
    rho, _ = fourier.spectral_radius(B0, Bf, (N, N))
    m = StructuredMesh((N, N), periodic=(True, True))
    op = ShallowWater(m, p, 1.0, dt)
    u = np.random.default_rng(5).standard_normal((m.nel, 3 * op.ref.Np))
    F = np.zeros_like(u)
    u, _ = ehdg.iterate(op, F, u, 60)
    n0 = np.linalg.norm(u)
    u, _ = ehdg.iterate(op, F, u, 40)
    observed = (np.linalg.norm(u) / n0) ** (1 / 40)
    assert abs(observed - rho) < 0.02 * rho, (observed, rho)


def _skeleton_norm2(op, U):
    """sum over element boundaries of int (phi^2 + Phi |vel|^2) (Theorem 2's E_h norm)."""
    ph, u, v = op.face_values(U)
    tot = 0.0
    for f in range(4):
        pts, w = op.ref.face_quadrature(f)
        Jf = op.mesh.h[1 - f // 2] / 2.0
        Mu = op.ref.face_trace_basis(f, pts)
        Mf = np.einsum("q,qa,qb->ab", w * Jf, Mu, Mu)
        for X, wt in ((ph, 1.0), (u, op.Phi), (v, op.Phi)):
            tot += wt * np.einsum("ea,ab,eb->", X[:, f], Mf, X[:, f])
    return tot


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_swe_theorem2_contraction_bound(p):
    """Where B > 0 and C < 1 (Theorem 2), ||iterate||^2_{E_h} <= C^k ||initial||^2_{E_h}."""
    N, dt, Phi = 8, 1e-4, 1.0
    h = 1.0 / N
    X = h / (dt * (p + 1) * (p + 2))
    A = max((Phi + np.sqrt(Phi)) / 2, (1 + np.sqrt(Phi)) / 2)
    B = min(X + (np.sqrt(Phi) - Phi) / 2, X + (0.0 - 1 - np.sqrt(Phi)) / 2)
    C = A / B
    assert B > 0 and C < 1
    m = StructuredMesh((N, N), periodic=(True, True))
    op = ShallowWater(m, p, Phi, dt)
    u = np.random.default_rng(p).standard_normal((m.nel, 3 * op.ref.Np))
    n0 = _skeleton_norm2(op, u)
    F = np.zeros_like(u)
    for k in range(1, 8):
        u, _ = ehdg.iterate(op, F, u, 1)
        assert _skeleton_norm2(op, u) <= C ** k * n0 * (1 + 1e-10)


def test_c2_shape_is_outside_convergent_regime():
    """256^2, p = 4, dt = 1e-3 (the shallow-water workload's stated step): the Bloch
    analysis gives rho(T) = dt (p+1)(p+2) / h = 7.68 > 1 at the checkerboard mode."""
    B0, Bf = _swe_blocks(4, 1.0 / 256, 1e-3)
    rho = np.max(np.abs(np.linalg.eigvals(fourier.symbol(B0, Bf, [np.pi, np.pi]))))
    assert abs(rho - 7.68) < 1e-9
    # and the step used instead, dt = 5e-5, lies inside Theorem 2 (C < 1) and converges
    B0, Bf = _swe_blocks(4, 1.0 / 256, 5e-5)
    ks = np.linspace(0, 2 * np.pi, 16, endpoint=False)
    rho = max(np.max(np.abs(np.linalg.eigvals(fourier.symbol(B0, Bf, [a, c])))) for a in ks for c in ks)
    assert rho < 0.5


# ---------------------------------------------------------------------------- P11/P14
def test_swe_momentum_conserved_every_iterate_and_mass_at_fixed_point():
    m = StructuredMesh((5, 4), periodic=(True, True))
    op = ShallowWater(m, 3, 1.0, 2e-3)
    U0 = np.random.default_rng(11).standard_normal((m.nel, 3 * op.ref.Np))
    F = op.load(U0)
    Np = op.ref.Np
    integ = lambda X: np.sum(X @ op.M.sum(axis=0))          # int over the mesh
    ph0, u0, v0 = op.split(U0)
    u = U0.copy()
    for _ in range(6):
        u, _ = ehdg.iterate(op, F, u, 1)
        _, uu, vv = op.split(u)
        assert abs(integ(uu) - integ(u0)) < 1e-12 * np.abs(u0).sum()
        assert abs(integ(vv) - integ(v0)) < 1e-12 * np.abs(v0).sum()
    out = ehdg.solve(op, F, U0, tol=1e-15, max_iter=500)
    assert abs(integ(op.split(out["u"])[0]) - integ(ph0)) < 1e-11 * np.abs(ph0).sum()


def test_swe_energy_non_increasing_per_step():
    m = StructuredMesh((6, 6), periodic=(True, True))
    op = ShallowWater(m, 2, 1.0, 5e-3)
    u = np.random.default_rng(2).standard_normal((m.nel, 3 * op.ref.Np))
    energy = lambda U: sum(np.einsum("ei,ij,ej->", X, op.M, X) for X in op.split(U))
    e_prev = energy(u)
    for _ in range(4):
        u, _ = ehdg.be_steps(op, u, 1, tol=1e-14)
        e = energy(u)
        assert e <= e_prev * (1 + 1e-12)
        e_prev = e


def test_transport_global_conservation_at_fixed_point():
    b, sig = (1.0, 0.5), 1.0
    ue, f = _c1_like(b, sig)
    m = StructuredMesh((6, 6))
    op = Transport(m, 3, b, sigma=sig, g=ue)
    F = op.load(f)
    out = ehdg.solve(op, F, np.zeros((m.nel, op.ref.Np)), tol=1e-15, max_iter=3000)
    U = out["u"]
    uh = op.trace(U)
    lhs = sig * np.sum(U @ op.M.sum(axis=0))
    for f_ in range(4):
        nb = op.nbr[f_]
        pts, wf, Pf, Mu = op.face[f_]
        bnd = nb < 0
        lhs += op.bn[f_] * np.sum((uh[bnd, f_] @ Mu.T) * wf[None])
    assert abs(lhs - F.sum()) < 1e-12 * np.abs(F).sum()
