"""Pins of the oracle's reference element against textbook values (CPU only)."""
import numpy as np
import pytest

from oracle.basis import RefElement, gll_nodes_weights, gauss_legendre, lagrange_eval, lagrange_deriv
from oracle.mesh import StructuredMesh

# Closed-form GLL nodes and weights (textbook values of the Lobatto rule)
GLL = {
    1: ([-1, 1], [1, 1]),
    2: ([-1, 0, 1], [1 / 3, 4 / 3, 1 / 3]),
    3: ([-1, -1 / np.sqrt(5), 1 / np.sqrt(5), 1], [1 / 6, 5 / 6, 5 / 6, 1 / 6]),
    4: ([-1, -np.sqrt(3 / 7), 0, np.sqrt(3 / 7), 1], [1 / 10, 49 / 90, 32 / 45, 49 / 90, 1 / 10]),
}


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_gll_closed_form(p):
    x, w = gll_nodes_weights(p)
    np.testing.assert_allclose(x, GLL[p][0], atol=1e-15)
    np.testing.assert_allclose(w, GLL[p][1], rtol=1e-14)


@pytest.mark.parametrize("p", range(1, 9))
def test_gll_exactness(p):
    # the Lobatto rule with p+1 points integrates x^k exactly for k <= 2p-1
    x, w = gll_nodes_weights(p)
    for k in range(2 * p):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.sum(w * x ** k) - exact) < 1e-13


@pytest.mark.parametrize("q", range(1, 10))
def test_gauss_exactness(q):
    x, w = gauss_legendre(q)
    for k in range(2 * q):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.sum(w * x ** k) - exact) < 1e-13


@pytest.mark.parametrize("p", range(1, 7))
def test_lagrange_cardinal_and_derivative(p):
    x, _ = gll_nodes_weights(p)
    np.testing.assert_allclose(lagrange_eval(x, x), np.eye(p + 1), atol=1e-14)
    t = np.linspace(-1, 1, 13)
    D = lagrange_deriv(x, t)
    # derivatives of 1 and of x reproduced exactly by the interpolant
    np.testing.assert_allclose(D.sum(axis=1), 0.0, atol=1e-11)
    np.testing.assert_allclose(D @ x, 1.0, atol=1e-11)
    np.testing.assert_allclose(D @ x ** p, p * t ** (p - 1), atol=1e-10)


@pytest.mark.parametrize("d,p", [(2, 1), (2, 3), (3, 1), (3, 2), (3, 3)])
def test_face_nodes_match_across_neighbours(d, p):
    """Both sides of a face list the same physical points in the same order."""
    mesh = StructuredMesh((3,) * d, L=(1.0,) * d, periodic=(True,) * d)
    ref = RefElement(p, d)
    for f in range(2 * d):
        nb = mesh.neighbour(f)
        for e in range(mesh.nel):
            xm = mesh.physical(e, ref.face_node_xi(f))[0]
            xp = mesh.physical(nb[e], ref.face_node_xi(f ^ 1))[0]
            diff = np.abs(np.mod(xm - xp + 0.5, 1.0) - 0.5)     # periodic distance
            assert diff.max() < 1e-14


@pytest.mark.parametrize("d,p", [(2, 2), (3, 2)])
def test_face_trace_basis_is_volume_restriction(d, p):
    """mu_a on a face equals the restriction of the volume basis of the a-th face node."""
    ref = RefElement(p, d)
    for f in range(2 * d):
        pts, _ = ref.face_quadrature(f)
        np.testing.assert_allclose(ref.basis(pts)[:, ref.face_nodes[f]], ref.face_trace_basis(f, pts),
                                   atol=1e-14)


def test_mass_matrix_integrates_constants():
    for d, p in [(1, 3), (2, 2), (3, 2)]:
        ref = RefElement(p, d)
        Psi = ref.basis(ref.xi_q)
        M = np.einsum("q,qj,qi->ij", ref.w_q, Psi, Psi)
        assert abs(M.sum() - 2.0 ** d) < 1e-13
