"""Exact spectral radius of the eHDG iteration on periodic uniform meshes (oracle).

TEST INFRASTRUCTURE ONLY (part of the CPU oracle; never imported by the product path).

On a periodic uniform mesh with constant coefficients the homogeneous iteration
u^{k+1}_K = B_0 u^k_K + sum_f B_f u^k_{nb(K,f)} is translation invariant, so it is
block-diagonalised by Bloch waves u_K = v exp(i theta . idx(K)).  The symbol is
S(theta) = B_0 + sum_f B_f exp(i theta . delta_f) and the spectral radius of the
iteration on an N_0 x N_1 (x N_2) mesh is the largest |eigenvalue| of S(theta) over
theta = 2 pi k / N.  The blocks are extracted by applying one homogeneous sweep of
the operator's own Algorithm-1 pieces to unit vectors on a 3^d periodic mesh.
"""
import itertools
import numpy as np

from .mesh import StructuredMesh


def blocks(make_op, d):
    """B_0 and B_f (f = 0..2d-1) from one homogeneous sweep on a periodic 3^d mesh.

    make_op(mesh) -> operator object (with trace / rhs / solve).
    """
    mesh = StructuredMesh((3,) * d, L=None, periodic=(True,) * d)
    op = make_op(mesh)
    n = op.A.shape[-1]
    c = mesh.elem(np.array([1] * d))
    B0 = np.zeros((n, n))
    Bf = [np.zeros((n, n)) for _ in range(2 * d)]
    zeroF = np.zeros((mesh.nel, n))
    for j in range(n):
        U = np.zeros((mesh.nel, n))
        U[c, j] = 1.0
        Un = op.solve(op.rhs(zeroF, op.trace(U)))
        B0[:, j] = Un[c]
        for f in range(2 * d):
            K = mesh.neighbour(f ^ 1)[c]          # element whose face-f neighbour is c
            Bf[f][:, j] = Un[K]
    return B0, Bf, op


def symbol(B0, Bf, theta):
    d = len(theta)
    S = B0.astype(np.complex128).copy()
    for f in range(2 * d):
        ax, side = f // 2, f % 2
        S += Bf[f] * np.exp(1j * theta[ax] * (-1 if side == 0 else 1))
    return S


def spectral_radius(B0, Bf, n_per_axis):
    """max over theta = 2 pi k / N of rho(S(theta)); returns (rho, theta_argmax)."""
    d = len(n_per_axis)
    best, arg = -1.0, None
    for ks in itertools.product(*[range(n) for n in n_per_axis]):
        th = [2 * np.pi * ks[a] / n_per_axis[a] for a in range(d)]
        r = np.max(np.abs(np.linalg.eigvals(symbol(B0, Bf, th))))
        if r > best:
            best, arg = r, th
    return best, arg
