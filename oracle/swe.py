"""eHDG local solver and trace for the linearized shallow-water system (oracle).

TEST INFRASTRUCTURE ONLY (part of the CPU oracle; never imported by the product path).

Unknowns per element: geopotential phi, velocity (u, v); mean geopotential Phi > 0
constant; Coriolis, friction and wind stress are zero (the paper's own test, Section
4.4, and every workload here).  Backward Euler in time (Section 3, the SWE system and
the three local equations of its eHDG solver), written for iterate k+1:

  (phi/dt, w1) - (Phi vel, grad w1) + <Phi vel.n + sqrt(Phi) (phi - phihat^k), w1>_dK
        = (phi^m/dt, w1)
  (Phi u/dt, w2) - (Phi phi, d w2/dx) + <Phi phihat^k n_1, w2>_dK = (Phi u^m/dt, w2)
  (Phi v/dt, w3) - (Phi phi, d w3/dy) + <Phi phihat^k n_2, w3>_dK = (Phi v^m/dt, w3)

with the trace phihat^k = {{phi^k}} + sqrt(Phi) {{vel^k . n}}, where each side uses its
own outward normal, so the trace is single-valued on a face.
Wall boundary reading (zero normal mass flux Phi vel.n + sqrt(Phi)(phi - phihat) = 0):
phihat = phi^- + sqrt(Phi) vel^-.n^-.

Unknown layout per element: [phi (Np), u (Np), v (Np)].
"""
import numpy as np
import scipy.linalg

from .basis import RefElement
from .mesh import StructuredMesh


class ShallowWater:
    def __init__(self, mesh: StructuredMesh, p, Phi, dt):
        assert mesh.d == 2
        self.mesh, self.p, self.d = mesh, p, 2
        self.ref = ref = RefElement(p, 2)
        self.Phi, self.dt = float(Phi), float(dt)
        self.sq = np.sqrt(self.Phi)
        h = mesh.h
        J = np.prod(h / 2.0)
        self.J = J
        Np = ref.Np
        Psi = ref.basis(ref.xi_q)
        G = ref.grad_basis(ref.xi_q)
        wq = ref.w_q * J
        M = np.einsum("q,qj,qi->ij", wq, Psi, Psi)
        Kx = np.einsum("q,qj,qi->ij", wq, Psi, G[0] * (2.0 / h[0]))      # (psi_j, dpsi_i/dx)
        Ky = np.einsum("q,qj,qi->ij", wq, Psi, G[1] * (2.0 / h[1]))
        self.M = M
        Phi, sq, dt = self.Phi, self.sq, self.dt
        A = np.zeros((3 * Np, 3 * Np))
        P, U, V = slice(0, Np), slice(Np, 2 * Np), slice(2 * Np, 3 * Np)
        A[P, P] += M / dt
        A[P, U] += -Phi * Kx
        A[P, V] += -Phi * Ky
        A[U, P] += -Phi * Kx
        A[U, U] += Phi * M / dt
        A[V, P] += -Phi * Ky
        A[V, V] += Phi * M / dt
        self.lifts = []
        self.nvec = [mesh.normal(f) for f in range(4)]
        for f in range(4):
            pts, w = ref.face_quadrature(f)
            Jf = h[1 - f // 2] / 2.0
            Pf = ref.basis(pts)
            Mu = ref.face_trace_basis(f, pts)
            E = np.einsum("q,qj,qi->ij", w * Jf, Pf, Pf)
            n1, n2 = self.nvec[f]
            A[P, P] += sq * E
            A[P, U] += Phi * n1 * E
            A[P, V] += Phi * n2 * E
            Lf = np.einsum("q,qa,qi->ia", w * Jf, Mu, Pf)                # <mu_a, psi_i>_f
            lift = np.zeros((3 * Np, Lf.shape[1]))
            lift[P] = sq * Lf
            lift[U] = -Phi * n1 * Lf
            lift[V] = -Phi * n2 * Lf
            self.lifts.append(lift)
        self.A = A
        self.lu = scipy.linalg.lu_factor(A)
        self.Psi_fn = [ref.basis(ref.face_node_xi(f)) for f in range(4)]
        self.nbr = [mesh.neighbour(f) for f in range(4)]
        self.Psi_q = Psi

    def split(self, U):
        Np = self.ref.Np
        return U[:, :Np], U[:, Np:2 * Np], U[:, 2 * Np:]

    def face_values(self, U):
        """(phi, u, v) at the face nodes: three arrays (nel, 4, nf)."""
        ph, u, v = self.split(U)
        fv = lambda X: np.stack([X @ self.Psi_fn[f].T for f in range(4)], axis=1)
        return fv(ph), fv(u), fv(v)

    def trace(self, U):
        """phihat at every element-face node: (nel, 4, nf)."""
        ph, u, v = self.face_values(U)
        out = np.empty_like(ph)
        for f in range(4):
            fo = f ^ 1
            nb = self.nbr[f]
            n1, n2 = self.nvec[f]
            vn_m = u[:, f] * n1 + v[:, f] * n2
            inner = nb >= 0
            ph_p = np.zeros_like(ph[:, f])
            vn_p = np.zeros_like(vn_m)
            ph_p[inner] = ph[nb[inner], fo]
            # the neighbour's own outward normal is -n
            vn_p[inner] = -(u[nb[inner], fo] * n1 + v[nb[inner], fo] * n2)
            th = 0.5 * (ph[:, f] + ph_p) + self.sq * 0.5 * (vn_m + vn_p)
            bnd = ~inner
            th[bnd] = ph[bnd, f] + self.sq * vn_m[bnd]
            out[:, f] = th
        return out

    def rhs(self, F, phat):
        r = F.copy()
        for f in range(4):
            r += phat[:, f, :] @ self.lifts[f].T
        return r

    def solve(self, R):
        return scipy.linalg.lu_solve(self.lu, R.T).T

    def load(self, um):
        """Backward-Euler right-hand side (phi^m/dt, w1), (Phi u^m/dt, w2), (Phi v^m/dt, w3)."""
        ph, u, v = self.split(um)
        dt, Phi = self.dt, self.Phi
        return np.concatenate([ph @ self.M.T / dt, Phi * (u @ self.M.T) / dt, Phi * (v @ self.M.T) / dt], axis=1)

    def state(self, U):
        """Per-side characteristic halves c_f = (phi + sqrt(Phi) vel.n_f) / 2 at face nodes: (nel, 4, nf).

        On an interior face phihat = c^- + c^+, so these are what each element
        contributes to the next trace.
        """
        ph, u, v = self.face_values(U)
        out = np.empty_like(ph)
        for f in range(4):
            n1, n2 = self.nvec[f]
            out[:, f] = 0.5 * (ph[:, f] + self.sq * (u[:, f] * n1 + v[:, f] * n2))
        return out

    def interpolate(self, fns):
        X = self.mesh.physical(np.arange(self.mesh.nel), self.ref.xi_nodes)
        return np.concatenate([fn(X) for fn in fns], axis=1)
