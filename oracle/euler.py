"""eHDG for the 2D linearized Euler equations, backward Euler in time (oracle).

TEST INFRASTRUCTURE ONLY (part of the CPU oracle; never imported by the product path).

The paper treats transport and linearized shallow water and states that other
hyperbolic systems follow the same construction (Section 3, first paragraph).
This operator applies that construction to the acoustics-plus-advection system
linearized about a uniform state (rho0, U0, p0 = rho0 c0^2 / gamma):

    w_t + A_x w_x + A_y w_y = 0,   w = (rho', u', v', p'),
    A_x = [[U, rho0, 0, 0], [0, U, 0, 1/rho0], [0, 0, U, 0], [0, rho0 c0^2, 0, U]],
    A_y = [[V, 0, rho0, 0], [0, V, 0, 0], [0, 0, V, 1/rho0], [0, 0, rho0 c0^2, V]].

Upwind HDG local equation at iterate k+1 (the systems analogue of eq. transportLocalk1):

    (w/dt, v)_K - (A_x w, v_x)_K - (A_y w, v_y)_K + <A_n w + |A_n| (w - what^k), v>_dK
        = (w^m/dt, v)_K,

and the trace from the conservation condition [[A_n w + |A_n| (w - what)]] = 0:

    what = (I + S)/2 w^- + (I - S)/2 w^+,   S = sign(A_{n^-}) = |A_n|^{-1} A_n,

the systems analogue of eq. transportLocale.  |A_n| = V |Lambda| V^{-1} from the
eigen-decomposition (real spectrum U.n, U.n, U.n +- c0).  Boundary reading (no
incoming waves): what = (I + S)/2 w^-.
Unknown layout per element: [rho (Np), u (Np), v (Np), p (Np)].
"""
import numpy as np
import scipy.linalg

from .basis import RefElement
from .mesh import StructuredMesh


def flux_matrices(U0, rho0, c0):
    U, V = U0
    Ax = np.array([[U, rho0, 0, 0], [0, U, 0, 1 / rho0], [0, 0, U, 0], [0, rho0 * c0 ** 2, 0, U]], dtype=float)
    Ay = np.array([[V, 0, rho0, 0], [0, V, 0, 0], [0, 0, V, 1 / rho0], [0, 0, rho0 * c0 ** 2, V]], dtype=float)
    return Ax, Ay


def abs_matrix(A):
    """|A| = V |Lambda| V^{-1} for a real-diagonalisable A."""
    lam, V = np.linalg.eig(A)
    lam, V = lam.real, V.real
    return (V * np.abs(lam)) @ np.linalg.inv(V)


class Euler:
    def __init__(self, mesh: StructuredMesh, p, U0, c0, dt, rho0=1.0):
        assert mesh.d == 2
        self.mesh, self.p, self.d = mesh, p, 2
        self.ref = ref = RefElement(p, 2)
        self.dt = float(dt)
        self.Ax, self.Ay = flux_matrices(U0, rho0, c0)
        h = mesh.h
        self.J = np.prod(h / 2.0)
        Np = ref.Np
        Psi = ref.basis(ref.xi_q)
        G = ref.grad_basis(ref.xi_q)
        wq = ref.w_q * self.J
        M = np.einsum("q,qj,qi->ij", wq, Psi, Psi)
        Kx = np.einsum("q,qj,qi->ij", wq, Psi, G[0] * (2.0 / h[0]))     # (psi_j, dpsi_i/dx)
        Ky = np.einsum("q,qj,qi->ij", wq, Psi, G[1] * (2.0 / h[1]))
        self.M = M
        n = 4 * Np
        A = np.kron(np.eye(4), M / self.dt) - np.kron(self.Ax, Kx) - np.kron(self.Ay, Ky)
        self.nvec = [mesh.normal(f) for f in range(4)]
        self.An, self.absAn, self.S = [], [], []
        self.lifts = []
        for f in range(4):
            pts, w = ref.face_quadrature(f)
            Jf = h[1 - f // 2] / 2.0
            Pf = ref.basis(pts)
            Mu = ref.face_trace_basis(f, pts)
            E = np.einsum("q,qj,qi->ij", w * Jf, Pf, Pf)
            Lf = np.einsum("q,qa,qi->ia", w * Jf, Mu, Pf)                 # <mu_a, psi_i>_f
            An = self.nvec[f][0] * self.Ax + self.nvec[f][1] * self.Ay
            aA = abs_matrix(An)
            self.An.append(An)
            self.absAn.append(aA)
            self.S.append(np.linalg.solve(aA, An))
            A += np.kron(An + aA, E)
            self.lifts.append(np.kron(aA, Lf))                               # acts on what_f (4 x nf)
        self.A = A
        self.lu = scipy.linalg.lu_factor(A)
        self.Psi_fn = [ref.basis(ref.face_node_xi(f)) for f in range(4)]
        self.nbr = [mesh.neighbour(f) for f in range(4)]
        self.Psi_q = Psi

    def face_values(self, U):
        """w at the face nodes: (nel, 4 faces, 4 fields, nf)."""
        Np = self.ref.Np
        out = []
        for f in range(4):
            out.append(np.stack([U[:, c * Np:(c + 1) * Np] @ self.Psi_fn[f].T for c in range(4)], axis=1))
        return np.stack(out, axis=1)

    def trace(self, U):
        """what at every element-face node: (nel, 4, 4 fields, nf)."""
        fv = self.face_values(U)
        out = np.empty_like(fv)
        I4 = np.eye(4)
        for f in range(4):
            fo = f ^ 1
            nb = self.nbr[f]
            Sm = self.S[f]
            wm = fv[:, f]                                                    # (nel, 4, nf)
            wp = np.zeros_like(wm)
            inner = nb >= 0
            wp[inner] = fv[nb[inner], fo]
            out[:, f] = (np.einsum("ab,ebn->ean", 0.5 * (I4 + Sm), wm)
                         + np.einsum("ab,ebn->ean", 0.5 * (I4 - Sm), wp))
        return out

    def rhs(self, F, what):
        r = F.copy()
        for f in range(4):
            r += what[:, f].reshape(what.shape[0], -1) @ self.lifts[f].T
        return r

    def solve(self, R):
        return scipy.linalg.lu_solve(self.lu, R.T).T

    def load(self, um):
        """(w^m / dt, v) per field."""
        Np = self.ref.Np
        return np.concatenate([um[:, c * Np:(c + 1) * Np] @ self.M.T / self.dt for c in range(4)], axis=1)

    def state(self, U):
        """Per-side outgoing part c_f = (I + S_f)/2 w at the face nodes: (nel, 4, 4, nf).
        On an interior face what = c^- + c^+."""
        fv = self.face_values(U)
        I4 = np.eye(4)
        return np.stack([np.einsum("ab,ebn->ean", 0.5 * (I4 + self.S[f]), fv[:, f]) for f in range(4)], axis=1)

    def interpolate(self, fns):
        X = self.mesh.physical(np.arange(self.mesh.nel), self.ref.xi_nodes)
        return np.concatenate([fn(X) for fn in fns], axis=1)


def dg_euler(op, F):
    """Classical DG with the upwind flux A^+ w^- + A^- w^+ (A^+- = (A_n +- |A_n|)/2);
    boundary faces take no incoming waves (w^+ = 0).  No trace unknowns."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    mesh, ref = op.mesh, op.ref
    Np = ref.Np
    n = 4 * Np
    h = mesh.h
    Psi = ref.basis(ref.xi_q)
    G = ref.grad_basis(ref.xi_q)
    wq = ref.w_q * op.J
    M = np.einsum("q,qj,qi->ij", wq, Psi, Psi)
    Kx = np.einsum("q,qj,qi->ij", wq, Psi, G[0] * (2.0 / h[0]))
    Ky = np.einsum("q,qj,qi->ij", wq, Psi, G[1] * (2.0 / h[1]))
    Avol = np.kron(np.eye(4), M / op.dt) - np.kron(op.Ax, Kx) - np.kron(op.Ay, Ky)
    rows, cols, vals = [], [], []

    def add(r0, c0, B):
        ii, jj = np.nonzero(B)
        rows.extend(r0 + ii)
        cols.extend(c0 + jj)
        vals.extend(B[ii, jj])

    nbr = [mesh.neighbour(f) for f in range(4)]
    for e in range(mesh.nel):
        add(e * n, e * n, Avol)
        for f in range(4):
            pts, w = ref.face_quadrature(f)
            Jf = h[1 - f // 2] / 2.0
            Pm = ref.basis(pts)
            pts_o = pts.copy()
            pts_o[:, f // 2] = -pts[:, f // 2]
            Po = ref.basis(pts_o)
            An = op.An[f]
            aA = abs_matrix(An)
            Ap, Am = 0.5 * (An + aA), 0.5 * (An - aA)
            add(e * n, e * n, np.kron(Ap, np.einsum("q,qi,qj->ij", w * Jf, Pm, Pm)))
            nb = nbr[f][e]
            if nb >= 0:
                add(e * n, nb * n, np.kron(Am, np.einsum("q,qi,qj->ij", w * Jf, Pm, Po)))
    Amat = sp.csr_matrix((vals, (rows, cols)), shape=(mesh.nel * n,) * 2)
    return spla.spsolve(Amat.tocsc(), F.reshape(-1)).reshape(mesh.nel, n)
