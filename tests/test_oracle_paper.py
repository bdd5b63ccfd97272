"""The oracle against the numbers the paper prints (CPU only).

Table 1 (iterations to the paper's stopping criteria for the steady problems of
Sections 4.1-4.3) and Table 2 (iterations per backward-Euler step, Sections 4.4
and 4.5) are stored verbatim under tests/golden/.  The paper does not state its
basis, quadrature or exact iteration-count convention, so counts are compared
within a band: +-15% for Table 1, [-1, +2] iterations for Table 2.
"""
import os

import numpy as np
import pytest

from oracle import ehdg
from oracle.mesh import StructuredMesh
from oracle.swe import ShallowWater
from oracle.transport import Transport

pi = np.pi
GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _table(name):
    rows = []
    with open(os.path.join(GOLD, name)) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                rows.append([int(v) for v in line.split()])
    return np.array(rows)


T1 = _table("table1_iterations.txt")
T2 = _table("table2_iterations.txt")


def _t1(nel2d=None, nel3d=None, p=None, col=None):
    for r in T1:
        if (nel2d is None or r[0] == nel2d) and (nel3d is None or r[1] == nel3d) and r[2] == p:
            return r[col]
    raise KeyError


def _t2(nel2d=None, nel3d=None, p=None, col=None):
    for r in T2:
        if (nel2d is None or r[0] == nel2d) and (nel3d is None or r[1] == nel3d) and r[2] == p:
            return r[col]
    raise KeyError


def _err_diff_criterion(op, exact):
    """|  ||u^k - u_e|| - ||u^{k-1} - u_e||  | < 1e-10  (Section 4.1's criterion)."""
    return lambda un, uo: abs(ehdg.l2_norm(op, un, exact) - ehdg.l2_norm(op, uo, exact)) < 1e-10


# Section 4.1: beta = (y, x), u_e = sin(pi x) cos(pi y) / pi, inflow x = 0 and y = 0
@pytest.mark.parametrize("N", [4, 8])
@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_table1_smooth_2d(N, p):
    beta = lambda X: np.stack([X[..., 1], X[..., 0]], axis=-1)
    ue = lambda X: np.sin(pi * X[..., 0]) * np.cos(pi * X[..., 1]) / pi
    f = lambda X: (X[..., 1] * np.cos(pi * X[..., 0]) * np.cos(pi * X[..., 1])
                   - X[..., 0] * np.sin(pi * X[..., 0]) * np.sin(pi * X[..., 1]))
    m = StructuredMesh((N, N))
    op = Transport(m, p, beta, div_beta=lambda X: np.zeros(X.shape[:-1]), g=ue)
    out = ehdg.solve(op, op.load(f), np.zeros((m.nel, op.ref.Np)), criterion=_err_diff_criterion(op, ue),
                     max_iter=1000)
    paper = _t1(nel2d=N * N, p=p, col=3)
    assert abs(out["iters"] - paper) <= 0.15 * paper, (out["iters"], paper)


# Section 4.2: beta = (1 + sin(pi y / 2), 2), [0,2]^2, f = 0, piecewise inflow data
@pytest.mark.parametrize("N", [4, 8])
@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_table1_discontinuous_2d(N, p):
    beta = lambda X: np.stack([1 + np.sin(pi * X[..., 1] / 2), 2 + 0 * X[..., 0]], axis=-1)

    def g(X):
        x, y = X[..., 0], X[..., 1]
        out = np.where(np.isclose(x, 0.0), 1.0, 0.0)
        return np.where(np.isclose(y, 0.0) & (x > 0) & (x <= 1), np.sin(pi * x) ** 6, out)

    m = StructuredMesh((N, N), L=(2.0, 2.0))
    op = Transport(m, p, beta, div_beta=lambda X: np.zeros(X.shape[:-1]), g=g)
    crit = lambda un, uo: ehdg.l2_norm(op, un - uo) < 1e-10
    out = ehdg.solve(op, np.zeros((m.nel, op.ref.Np)), np.zeros((m.nel, op.ref.Np)), criterion=crit,
                     max_iter=1000)
    paper = _t1(nel2d=N * N, p=p, col=4)
    assert abs(out["iters"] - paper) <= 0.15 * paper, (out["iters"], paper)


# Section 4.3: beta = (z, x, y), u_e = sin(pi x) cos(pi y) sin(pi z) / pi
@pytest.mark.parametrize("N", [2, 4])
@pytest.mark.parametrize("p", [1, 2, 3])
def test_table1_steady_3d(N, p):
    beta = lambda X: np.stack([X[..., 2], X[..., 0], X[..., 1]], axis=-1)
    ue = lambda X: np.sin(pi * X[..., 0]) * np.cos(pi * X[..., 1]) * np.sin(pi * X[..., 2]) / pi

    def f(X):
        x, y, z = X[..., 0], X[..., 1], X[..., 2]
        return (z * np.cos(pi * x) * np.cos(pi * y) * np.sin(pi * z)
                - x * np.sin(pi * x) * np.sin(pi * y) * np.sin(pi * z)
                + y * np.sin(pi * x) * np.cos(pi * y) * np.cos(pi * z))

    m = StructuredMesh((N, N, N))
    op = Transport(m, p, beta, div_beta=lambda X: np.zeros(X.shape[:-1]), g=ue)
    out = ehdg.solve(op, op.load(f), np.zeros((m.nel, op.ref.Np)), criterion=_err_diff_criterion(op, ue),
                     max_iter=1000)
    paper = _t1(nel3d=N ** 3, p=p, col=5)
    assert abs(out["iters"] - paper) <= 0.15 * paper, (out["iters"], paper)


# Section 4.4: standing wave with walls, Phi = 1; first backward-Euler step
@pytest.mark.parametrize("N", [4, 8])
@pytest.mark.parametrize("p", [1, 2, 3, 4])
@pytest.mark.parametrize("dt,col", [(1e-3, 3), (1e-4, 4)])
def test_table2_shallow_water(N, p, dt, col):
    s2 = np.sqrt(2.0)

    def exact(t):
        return [lambda X: np.cos(pi * X[..., 0]) * np.cos(pi * X[..., 1]) * np.cos(s2 * pi * t),
                lambda X: np.sin(pi * X[..., 0]) * np.cos(pi * X[..., 1]) * np.sin(s2 * pi * t) / s2,
                lambda X: np.cos(pi * X[..., 0]) * np.sin(pi * X[..., 1]) * np.sin(s2 * pi * t) / s2]

    m = StructuredMesh((N, N))
    op = ShallowWater(m, p, 1.0, dt)
    u = op.interpolate(exact(0.0))
    ex = exact(dt)
    Np = op.ref.Np
    err = lambda U: np.sqrt(sum(ehdg.l2_norm(op, U[:, i * Np:(i + 1) * Np], ex[i]) ** 2 for i in range(3)))
    out = ehdg.solve(op, op.load(u), u, criterion=lambda un, uo: abs(err(un) - err(uo)) < 1e-10, max_iter=200)
    paper = _t2(nel2d=N * N, p=p, col=col)
    assert -1 <= out["iters"] - paper <= 2, (out["iters"], paper)


# Section 4.5 setup (beta = (0.2, 0.2, 0.2): the Gaussian moves with speed 0.2 per axis, f = 0)
@pytest.mark.parametrize("N", [2, 4])
@pytest.mark.parametrize("p", [1, 2, 3])
@pytest.mark.parametrize("dt,col", [(1e-3, 5), (1e-4, 6)])
def test_table2_advection_3d(N, p, dt, col):
    ue_t = lambda t: (lambda X: np.exp(-5 * ((X[..., 0] - 0.2 * t) ** 2 + (X[..., 1] - 0.2 * t) ** 2
                                             + (X[..., 2] - 0.2 * t) ** 2)))
    m = StructuredMesh((N, N, N))
    op = Transport(m, p, (0.2, 0.2, 0.2), sigma=0.0, dt=dt, g=ue_t(dt))
    u = op.interpolate(ue_t(0.0))
    out = ehdg.solve(op, op.load(None, u), u, criterion=_err_diff_criterion(op, ue_t(dt)), max_iter=200)
    paper = _t2(nel3d=N ** 3, p=p, col=col)
    assert -1 <= out["iters"] - paper <= 2, (out["iters"], paper)
