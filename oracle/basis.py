"""Reference-element ingredients for the oracle: nodes, quadrature, Lagrange basis.

TEST INFRASTRUCTURE ONLY.  This package is the slow, plain FP64 CPU oracle that
the HIP path is checked against; nothing in the product path may import it.

The paper builds its discrete spaces from polynomials of degree p on each element
and on each face (Section 2, definition of the broken spaces V_h and Lambda_h).
It does not say which basis or quadrature is used.  Reading used here: tensor
products of degree-p Lagrange polynomials on Gauss-Lobatto-Legendre (GLL) nodes,
so that on a face the element basis restricted to that face is again a tensor
Lagrange basis on the face nodes, and Gauss-Legendre quadrature with p+2 points
per direction for every volume and face integral (exact for all integrands of the
constant-coefficient operators, which have degree at most 2p+1 per direction).

Degree p = 0 is allowed as a special case (one node at the element centre), used
only by the closed-form p = 0 checks of the iteration.
"""
import numpy as np


def legendre(n, x):
    """Return (P_n(x), P_n'(x)) by the three-term recurrence, elementwise on x."""
    x = np.asarray(x, dtype=np.float64)
    p0 = np.ones_like(x)
    if n == 0:
        return p0, np.zeros_like(x)
    p1 = x.copy()
    for k in range(2, n + 1):
        p0, p1 = p1, ((2 * k - 1) * x * p1 - (k - 1) * p0) / k
    # derivative from (1 - x^2) P_n' = n (P_{n-1} - x P_n), valid off the endpoints
    with np.errstate(divide="ignore", invalid="ignore"):
        dp = n * (p0 - x * p1) / (1.0 - x * x)
    end = np.isclose(np.abs(x), 1.0)
    if np.any(end):
        # P_n'(+-1) = (+-1)^(n+1) n (n+1) / 2
        dp = np.where(end, np.sign(x) ** (n + 1) * n * (n + 1) / 2.0, dp)
    return p1, dp


def gll_nodes_weights(p):
    """Gauss-Lobatto-Legendre nodes (ascending) and weights for degree p >= 1.

    Nodes: -1, +1 and the p-1 roots of P_p'.  Weights: 2 / (p (p+1) P_p(x)^2).
    The interior roots are found by Newton's method on q(x) = (1-x^2) P_p'(x),
    started from the Chebyshev-Gauss-Lobatto points.
    """
    if p == 0:
        return np.array([0.0]), np.array([2.0])
    x = -np.cos(np.pi * np.arange(p + 1) / p)
    for _ in range(100):
        pn, dpn = legendre(p, x)
        # q = (1-x^2) P_p' ; q' = -p(p+1) P_p (Legendre ODE)
        q = (1.0 - x * x) * dpn
        dq = -p * (p + 1) * pn
        step = np.zeros_like(x)
        step[1:-1] = q[1:-1] / dq[1:-1]
        x = x - step
        if np.max(np.abs(step)) < 1e-16:
            break
    x[0], x[-1] = -1.0, 1.0
    pn, _ = legendre(p, x)
    w = 2.0 / (p * (p + 1) * pn * pn)
    return x, w


def gauss_legendre(q):
    """Gauss-Legendre points and weights on [-1, 1] (library primitive)."""
    return np.polynomial.legendre.leggauss(q)


def lagrange_eval(nodes, x):
    """Matrix L[i, j] = l_j(x_i) of the Lagrange basis on `nodes`, by the product formula."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = len(nodes)
    L = np.ones((len(x), n))
    for j in range(n):
        for m in range(n):
            if m != j:
                L[:, j] *= (x - nodes[m]) / (nodes[j] - nodes[m])
    return L


def lagrange_deriv(nodes, x):
    """Matrix D[i, j] = l_j'(x_i), by differentiating the product formula term by term."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = len(nodes)
    D = np.zeros((len(x), n))
    for j in range(n):
        for k in range(n):
            if k == j:
                continue
            term = np.full(len(x), 1.0 / (nodes[j] - nodes[k]))
            for m in range(n):
                if m != j and m != k:
                    term *= (x - nodes[m]) / (nodes[j] - nodes[m])
            D[:, j] += term
    return D


def tensor_index(p, d):
    """Multi-indices (a_0, ..., a_{d-1}) of tensor nodes, axis 0 fastest: array (N, d)."""
    n = p + 1
    idx = np.indices((n,) * d).reshape(d, -1).T          # last axis varies fastest
    return idx[:, ::-1].copy()                            # make axis 0 fastest


def face_axes(f):
    """Face f in 0..2d-1: axis f // 2, side f % 2 (0 = minus side, 1 = plus side)."""
    return f // 2, f % 2


class RefElement:
    """Tensor GLL element of degree p in d dimensions with (p+2)-point GL quadrature.

    Node a = a_0 + (p+1) a_1 + (p+1)^2 a_2 (axis 0 fastest).  Faces 0..2d-1 are
    (axis 0 minus, axis 0 plus, axis 1 minus, ...).  On a face, nodes are ordered by
    the tangential indices in increasing axis order, first tangential axis fastest,
    so two elements sharing a face list the shared physical points in the same order.
    """

    def __init__(self, p, d, nquad=None):
        self.p, self.d = p, d
        self.nodes1, self.gllw1 = gll_nodes_weights(p)
        q = p + 2 if nquad is None else nquad
        self.xq1, self.wq1 = gauss_legendre(q)
        self.nq1 = q
        self.Np = (p + 1) ** d
        self.nf = (p + 1) ** (d - 1)
        self.nidx = tensor_index(p, d)                     # (Np, d)
        self.qidx = tensor_index(q - 1, d)                 # (Nq, d)
        self.xi_nodes = self.nodes1[self.nidx]             # (Np, d) reference coords
        self.xi_q = self.xq1[self.qidx]                    # (Nq, d)
        self.w_q = np.prod(self.wq1[self.qidx], axis=1)    # (Nq,)
        # face nodes: indices into the volume nodes, and their reference coordinates
        self.face_nodes = []
        for f in range(2 * d):
            ax, side = face_axes(f)
            val = 0 if side == 0 else p
            sel = np.nonzero(self.nidx[:, ax] == val)[0]
            # tangential ordering: sort by tangential indices, first tangential axis fastest
            tang = [a for a in range(d) if a != ax]
            keys = tuple(self.nidx[sel, a] for a in tang)   # lexsort: last key is the primary one
            order = np.lexsort(keys) if len(keys) else np.arange(len(sel))
            self.face_nodes.append(sel[order])

    def basis(self, xi):
        """Psi[i, j] = psi_j(xi_i) for reference points xi (n, d)."""
        xi = np.atleast_2d(xi)
        out = np.ones((xi.shape[0], self.Np))
        for a in range(self.d):
            La = lagrange_eval(self.nodes1, xi[:, a])      # (n, p+1)
            out *= La[:, self.nidx[:, a]]
        return out

    def grad_basis(self, xi):
        """G[a][i, j] = d psi_j / d xi_a at reference points xi (n, d)."""
        xi = np.atleast_2d(xi)
        Ls = [lagrange_eval(self.nodes1, xi[:, a]) for a in range(self.d)]
        Ds = [lagrange_deriv(self.nodes1, xi[:, a]) for a in range(self.d)]
        G = []
        for a in range(self.d):
            g = np.ones((xi.shape[0], self.Np))
            for b in range(self.d):
                M = Ds[b] if b == a else Ls[b]
                g *= M[:, self.nidx[:, b]]
            G.append(g)
        return G

    def face_quadrature(self, f):
        """Reference points (nq_f, d) and weights on face f (tensor GL in the tangential axes)."""
        ax, side = face_axes(f)
        tang = [a for a in range(self.d) if a != ax]
        if self.d == 1:
            pts = np.array([[-1.0 if side == 0 else 1.0]])
            return pts, np.array([1.0])
        qi = tensor_index(self.nq1 - 1, self.d - 1)
        pts = np.zeros((qi.shape[0], self.d))
        pts[:, ax] = -1.0 if side == 0 else 1.0
        for t, a in enumerate(tang):
            pts[:, a] = self.xq1[qi[:, t]]
        w = np.prod(self.wq1[qi], axis=1)
        return pts, w

    def face_trace_basis(self, f, xi):
        """Mu[i, a] = mu_a(xi_i): the face Lagrange basis (tangential tensor GLL) on face f."""
        ax, _ = face_axes(f)
        tang = [a for a in range(self.d) if a != ax]
        xi = np.atleast_2d(xi)
        if self.d == 1:
            return np.ones((xi.shape[0], 1))
        fidx = tensor_index(self.p, self.d - 1)
        out = np.ones((xi.shape[0], fidx.shape[0]))
        for t, a in enumerate(tang):
            La = lagrange_eval(self.nodes1, xi[:, a])
            out *= La[:, fidx[:, t]]
        return out

    def face_node_xi(self, f):
        """Reference coordinates (nf, d) of the face-f nodes, in face order."""
        if self.p == 0:
            ax, side = face_axes(f)
            pt = np.zeros((1, self.d))
            pt[0, ax] = -1.0 if side == 0 else 1.0
            return pt
        return self.xi_nodes[self.face_nodes[f]]
