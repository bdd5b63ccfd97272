"""Pins of the oracle's variable-velocity branch (CPU only).

The oracle's per-element operator for a velocity field beta(x) carries a div(beta)
volume term, a per-element inverse and an L2-projected trace (oracle/transport.py).
They are pinned against things outside that code:

* An independently assembled classical upwind DG solve in strong form
  (oracle.direct.dg_transport_variable): (beta.grad u + sigma u, v)_K plus the inflow
  jump |beta.n| (u^- - u^ext) at the face Gauss points.  It has no div(beta) term, no
  lift and no trace unknown.  The paper's local equation (eq. transportLocal)
  integrates by parts to exactly this form, so with polynomial velocities (exact
  Gauss quadrature) the eHDG fixed point must equal it to rounding.  A sign or factor
  error on the div(beta) term, in the lifts or in the projected trace breaks this.
* The optimal (p+1) h-convergence the paper reports for its Section 4.1 and 4.3
  problems (beta = (y, x) and (z, x, y)) and for a manufactured problem with
  div(beta) != 0 and a reaction term.
* A planted mistake: the same oracle built with the div(beta) term negated must fail
  the first pin (so the pin can see that term).
"""
import numpy as np
import pytest

from oracle import ehdg as O
from oracle.direct import dg_transport_variable
from oracle.mesh import StructuredMesh
from oracle.transport import Transport

pi = np.pi


def _zero(X):
    return np.zeros(X.shape[:-1])


def sec41():
    """Section 4.1: beta = (y, x), u_e = sin(pi x) cos(pi y) / pi on [0, 1]^2."""
    beta = lambda X: np.stack([X[..., 1], X[..., 0]], -1)
    ue = lambda X: np.sin(pi * X[..., 0]) * np.cos(pi * X[..., 1]) / pi
    f = lambda X: (X[..., 1] * np.cos(pi * X[..., 0]) * np.cos(pi * X[..., 1])
                   - X[..., 0] * np.sin(pi * X[..., 0]) * np.sin(pi * X[..., 1]))
    return (1.0, 1.0), beta, _zero, 0.0, f, ue


def sec43():
    """Section 4.3: beta = (z, x, y), u_e = sin(pi x) cos(pi y) sin(pi z) / pi on [0, 1]^3."""
    beta = lambda X: np.stack([X[..., 2], X[..., 0], X[..., 1]], -1)
    ue = lambda X: np.sin(pi * X[..., 0]) * np.cos(pi * X[..., 1]) * np.sin(pi * X[..., 2]) / pi

    def f(X):
        x, y, z = X[..., 0], X[..., 1], X[..., 2]
        return (z * np.cos(pi * x) * np.cos(pi * y) * np.sin(pi * z)
                - x * np.sin(pi * x) * np.sin(pi * y) * np.sin(pi * z)
                + y * np.sin(pi * x) * np.cos(pi * y) * np.cos(pi * z))
    return (1.0, 1.0, 1.0), beta, _zero, 0.0, f, ue


def compressive2d():
    """beta = (-1 - x y / 2, 1/2 + x^2 / 4): inflow on x = 1.5 and y = 0, div(beta) = -y/2,
    reaction 0.3; manufactured u_e = cos(2x + y), f = beta.grad u_e + sigma u_e."""
    sigma = 0.3
    beta = lambda X: np.stack([-1 - 0.5 * X[..., 0] * X[..., 1], 0.5 + 0.25 * X[..., 0] ** 2], -1)
    div = lambda X: -0.5 * X[..., 1]
    ue = lambda X: np.cos(2 * X[..., 0] + X[..., 1])

    def f(X):
        b, s = beta(X), np.sin(2 * X[..., 0] + X[..., 1])
        return -2 * b[..., 0] * s - b[..., 1] * s + sigma * ue(X)
    return (1.5, 0.8), beta, div, sigma, f, ue


def expanding3d():
    """beta = (1 + x/2, 1/2 + 3x/10, -(4/5 + y/5)): div(beta) = 1/2, inflow on x = 0, y = 0
    and z = 1, reaction 0.2; manufactured u_e = exp(-x) sin(y + 2z) + z."""
    sigma = 0.2
    beta = lambda X: np.stack([1 + 0.5 * X[..., 0], 0.5 + 0.3 * X[..., 0], -(0.8 + 0.2 * X[..., 1])], -1)
    div = lambda X: np.full(X.shape[:-1], 0.5)
    ue = lambda X: np.exp(-X[..., 0]) * np.sin(X[..., 1] + 2 * X[..., 2]) + X[..., 2]

    def f(X):
        x, y, z = X[..., 0], X[..., 1], X[..., 2]
        b = beta(X)
        ux = -np.exp(-x) * np.sin(y + 2 * z)
        uy = np.exp(-x) * np.cos(y + 2 * z)
        uz = 2 * np.exp(-x) * np.cos(y + 2 * z) + 1.0
        return b[..., 0] * ux + b[..., 1] * uy + b[..., 2] * uz + sigma * ue(X)
    return (1.0, 0.9, 1.1), beta, div, sigma, f, ue


PROBLEMS = {"sec41": sec41, "sec43": sec43, "compressive2d": compressive2d, "expanding3d": expanding3d}


def _op(name, n, p, negate_div=False):
    L, beta, div, sigma, f, ue = PROBLEMS[name]()
    divf = (lambda X: -div(X)) if negate_div else div
    op = Transport(StructuredMesh(n, L=L), p, beta, sigma=sigma, div_beta=divf, g=ue)
    return op, op.load(f), ue


def _limit(op, F, tol=1e-15):
    out = O.solve(op, F, np.zeros((op.mesh.nel, op.ref.Np)), tol=tol, max_iter=5000)
    assert out["converged"]
    return out["u"]


def _rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


EQ_CASES = ([("sec41", n, p) for n in ((4, 4), (5, 3)) for p in (1, 2, 3, 4)]
            + [("compressive2d", n, p) for n in ((4, 4), (5, 3)) for p in (1, 2, 3, 4)]
            + [("sec43", n, p) for n in ((2, 2, 2), (3, 2, 2)) for p in (1, 2, 3)]
            + [("expanding3d", n, p) for n in ((2, 2, 2), (2, 3, 2)) for p in (1, 2, 3)])


@pytest.mark.parametrize("name,n,p", EQ_CASES)
def test_variable_limit_equals_strong_form_upwind_dg(name, n, p):
    """eHDG fixed point (Algorithm 1 iterated to a 1e-15 increment) = strong-form upwind
    DG, within 1e-12 relative (observed ~1e-14)."""
    op, F, _ = _op(name, n, p)
    u = _limit(op, F)
    ref = dg_transport_variable(op, F)
    assert _rel(u, ref) < 1e-12, _rel(u, ref)


@pytest.mark.parametrize("name,n", [("compressive2d", (4, 4)), ("expanding3d", (2, 2, 2))])
def test_planted_div_beta_sign_error_is_caught(name, n):
    """The oracle built with -div(beta) in its volume term no longer matches the DG solve:
    the equivalence pin sees the div(beta) term (both fields have div(beta) != 0)."""
    p = 2
    op, F, _ = _op(name, n, p, negate_div=True)
    u = _limit(op, F, tol=1e-13)
    ref = dg_transport_variable(_op(name, n, p)[0], F)
    assert _rel(u, ref) > 1e-3


RATE_CASES = ([("sec41", p, (4, 8, 16)) for p in (1, 2, 3)]
              + [("compressive2d", p, (4, 8, 16)) for p in (1, 2, 3)]
              + [("sec43", p, (2, 4, 8)) for p in (1, 2)]
              + [("expanding3d", 1, (2, 4, 8))])


@pytest.mark.parametrize("name,p,Ns", RATE_CASES)
def test_variable_h_rate_is_optimal(name, p, Ns):
    """L2 error of the eHDG limit against the exact solution decays at rate p+1 (the
    paper's 'optimal' h-convergence for its Sections 4.1 and 4.3), within +-0.3 on the
    last refinement, and the error drops on every refinement."""
    errs = []
    for N in Ns:
        d = len(PROBLEMS[name]()[0])
        op, F, ue = _op(name, (N,) * d, p)
        errs.append(O.l2_norm(op, _limit(op, F, tol=1e-13), ue))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 0.5), rates
    assert abs(rates[-1] - (p + 1)) < 0.3, (errs, rates)
