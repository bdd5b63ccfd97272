"""Upwind HDG local operator and eHDG trace for scalar transport (oracle).

TEST INFRASTRUCTURE ONLY (part of the CPU oracle; never imported by the product path).

Local equation (Section 3, eq. transportLocal; with the backward-Euler L2 term of
the time-dependent paragraph after Theorem 1 and a reaction term sigma*u):

    -(u, div(beta v))_K + <beta.n u + |beta.n| (u - uhat), v>_dK
        + (sigma + 1/dt) (u, v)_K = (f, v)_K + (u^m / dt, v)_K

Moving <|beta.n| uhat, v> to the right-hand side leaves the element operator

    A = -(psi_j, div(beta psi_i)) + sum_f <(beta.n + |beta.n|) psi_j, psi_i>_f
        + (sigma + 1/dt) (psi_j, psi_i)

and one lift per face, Lift_f[i, a] = <|beta.n| mu_a, psi_i>_f, acting on the
face-nodal values of uhat.  The eHDG trace (eq. transportLocale) is

    uhat^k = {{u^k sgn(beta.n)}} + {{u^k}},  2{{w}} = w^- + w^+,

taken as an element of the face polynomial space: for constant beta it is applied
at the face nodes (exact, since beta.n is constant on a face); for variable beta it
is applied pointwise at the face quadrature points and L2-projected onto the face
space.  Boundary reading: on the inflow boundary (beta.n^- < 0) uhat = g (its
interpolant at the face nodes for constant beta); elsewhere on the boundary, where
the formula has no neighbour, uhat = u^- (the element's own value).

Every integral is a plain quadrature sum over tensor Gauss points; nothing is
factored or fused.
"""
import numpy as np
import scipy.linalg

from .basis import RefElement
from .mesh import StructuredMesh


class Transport:
    """Upwind HDG transport on a structured mesh.

    beta: constant vector (length d) or callable beta(x) -> (..., d).
    div_beta: callable div(beta)(x) -> (...), required when beta is a callable.
    sigma: reaction coefficient; dt: backward-Euler step (None for steady).
    g: callable inflow boundary data g(x) -> (...), or None (zero).
    """

    def __init__(self, mesh: StructuredMesh, p, beta, sigma=0.0, dt=None, div_beta=None, g=None):
        self.mesh, self.p, self.d = mesh, p, mesh.d
        self.ref = RefElement(p, mesh.d)
        self.sigma = float(sigma)
        self.dt = dt
        self.const = not callable(beta)
        self.g = g
        d, ref = self.d, self.ref
        h = mesh.h
        J = np.prod(h / 2.0)
        if self.const:
            b = np.asarray(beta, dtype=np.float64)
            self.beta_vec = b
            self.beta = lambda x: np.broadcast_to(b, np.shape(x)[:-1] + (d,))
            self.div_beta = lambda x: np.zeros(np.shape(x)[:-1])
        else:
            self.beta = beta
            self.div_beta = div_beta
        self.J = J
        # reference basis data
        Psi = ref.basis(ref.xi_q)                                   # (Nq, Np)
        G = ref.grad_basis(ref.xi_q)                                # d x (Nq, Np)
        self.Psi_q = Psi
        self.Psi_fn = [ref.basis(ref.face_node_xi(f)) for f in range(2 * d)]   # (nf, Np)
        react = self.sigma + (0.0 if dt is None else 1.0 / dt)
        self.react = react
        face = []
        for f in range(2 * d):
            pts, w = ref.face_quadrature(f)
            Jf = np.prod([h[a] / 2.0 for a in range(d) if a != f // 2]) if d > 1 else 1.0
            face.append((pts, w * Jf, ref.basis(pts), ref.face_trace_basis(f, pts)))
        self.face = face
        nvec = [mesh.normal(f) for f in range(2 * d)]
        self.nvec = nvec
        if self.const:
            bgrad = sum(self.beta_vec[a] * G[a] * (2.0 / h[a]) for a in range(d))   # (Nq, Np): beta.grad psi_i
            wq = ref.w_q * J
            A = -np.einsum("q,qj,qi->ij", wq, Psi, bgrad) + react * np.einsum("q,qj,qi->ij", wq, Psi, Psi)
            lifts = []
            self.bn = np.array([self.beta_vec @ nvec[f] for f in range(2 * d)])
            for f in range(2 * d):
                pts, wf, Pf, Mu = face[f]
                bn = self.bn[f]
                A += (bn + abs(bn)) * np.einsum("q,qj,qi->ij", wf, Pf, Pf)
                lifts.append(abs(bn) * np.einsum("q,qa,qi->ia", wf, Mu, Pf))
            self.A = A
            self.lifts = lifts
            self.lu = scipy.linalg.lu_factor(A)
            self.M = np.einsum("q,qj,qi->ij", wq, Psi, Psi)
        else:
            nel = mesh.nel
            Xq = mesh.physical(np.arange(nel), ref.xi_q)            # (nel, Nq, d)
            B = self.beta(Xq)                                       # (nel, Nq, d)
            divB = self.div_beta(Xq)                                # (nel, Nq)
            wq = ref.w_q * J
            bgrad = sum(B[:, :, a, None] * G[a][None] * (2.0 / h[a]) for a in range(d))  # (nel,Nq,Np)
            A = -np.einsum("q,qj,eqi->eij", wq, Psi, bgrad)
            A -= np.einsum("q,eq,qj,qi->eij", wq, divB, Psi, Psi)
            A += react * np.einsum("q,qj,qi->ij", wq, Psi, Psi)[None]
            lifts = []
            for f in range(2 * d):
                pts, wf, Pf, Mu = face[f]
                Xf = mesh.physical(np.arange(nel), pts)
                bn = self.beta(Xf) @ nvec[f]                         # (nel, nqf)
                A += np.einsum("q,eq,qj,qi->eij", wf, bn + np.abs(bn), Pf, Pf)
                lifts.append(np.einsum("q,eq,qa,qi->eia", wf, np.abs(bn), Mu, Pf))
            self.A = A
            self.lifts = lifts
            self.Ainv = np.linalg.inv(A)
            self.M = np.einsum("q,qj,qi->ij", wq, Psi, Psi)
        # beta.n^- at every face node of every element (for the trace's sign)
        self.bn_nodes = np.zeros((mesh.nel, 2 * d, ref.nf if p > 0 else 1))
        for f in range(2 * d):
            Xn = mesh.physical(np.arange(mesh.nel), ref.face_node_xi(f))
            self.bn_nodes[:, f, :] = self.beta(Xn) @ nvec[f]
        self.nbr = [mesh.neighbour(f) for f in range(2 * d)]

    # ---- pieces of Algorithm 1 -------------------------------------------------
    def face_values(self, U):
        """u^- at the face nodes of every face: (nel, 2d, nf)."""
        return np.stack([U @ self.Psi_fn[f].T for f in range(2 * self.d)], axis=1)

    def trace(self, U):
        """uhat = {{u sgn(beta.n)}} + {{u}} on every element face: nodal values (nel, 2d, nf).

        Constant beta: beta.n is constant on each face and the formula is applied at
        the face nodes, which reproduces the upwind restriction exactly.
        Variable beta: beta.n may vanish at isolated points of a face, so the formula
        is applied pointwise at the face quadrature points and the result is
        L2-projected onto the face polynomial space (the trace space Lambda_h).
        """
        if self.const:
            return self._trace_nodal(U)
        return self._trace_projected(U)

    def _trace_nodal(self, U):
        fv = self.face_values(U)
        out = np.empty_like(fv)
        for f in range(2 * self.d):
            fo = f ^ 1                       # the same face seen from the neighbour
            nb = self.nbr[f]
            um = fv[:, f, :]
            sm = np.sign(self.bn_nodes[:, f, :])
            inner = nb >= 0
            up = np.zeros_like(um)
            up[inner] = fv[nb[inner], fo, :]
            sp = -sm
            uh = 0.5 * (um * sm + up * sp) + 0.5 * (um + up)
            bnd = ~inner
            if np.any(bnd):
                xb = self.mesh.physical(np.nonzero(bnd)[0], self.ref.face_node_xi(f))
                gval = self.g(xb) if self.g is not None else np.zeros(xb.shape[:2])
                inflow = sm[bnd] < 0
                uh[bnd] = np.where(inflow, gval, um[bnd])
            out[:, f, :] = uh
        return out

    def _trace_projected(self, U):
        nel, d = self.mesh.nel, self.d
        out = np.empty((nel, 2 * d, self.ref.nf))
        for f in range(2 * d):
            fo = f ^ 1
            nb = self.nbr[f]
            pts, wf, Pf, Mu = self.face[f]
            pts_o = pts.copy()
            pts_o[:, f // 2] = -pts[:, f // 2]
            Po = self.ref.basis(pts_o)                     # neighbour's basis at the same points
            Xf = self.mesh.physical(np.arange(nel), pts)
            sm = np.sign(self.beta(Xf) @ self.nvec[f])     # (nel, nq)
            um = U @ Pf.T
            inner = nb >= 0
            up = np.zeros_like(um)
            up[inner] = U[nb[inner]] @ Po.T
            uh = 0.5 * (um * sm - up * sm) + 0.5 * (um + up)
            bnd = ~inner
            if np.any(bnd):
                gval = self.g(Xf[bnd]) if self.g is not None else np.zeros(um[bnd].shape)
                uh[bnd] = np.where(sm[bnd] < 0, gval, um[bnd])
            Mf = np.einsum("q,qa,qb->ab", wf, Mu, Mu)
            out[:, f, :] = np.linalg.solve(Mf, ((uh * wf[None]) @ Mu).T).T
        return out

    def rhs(self, F, uhat):
        """F + sum_f Lift_f uhat_f."""
        r = F.copy()
        for f in range(2 * self.d):
            if self.const:
                r += uhat[:, f, :] @ self.lifts[f].T
            else:
                r += np.einsum("eia,ea->ei", self.lifts[f], uhat[:, f, :])
        return r

    def solve(self, R):
        """Apply A^{-1} to every element's right-hand side (rows of R)."""
        if self.const:
            return scipy.linalg.lu_solve(self.lu, R.T).T
        return np.einsum("eij,ej->ei", self.Ainv, R)

    def load(self, f=None, um=None):
        """(f, psi_i)_K (+ (u^m/dt, psi_i)_K) for every element: (nel, Np)."""
        nel = self.mesh.nel
        F = np.zeros((nel, self.ref.Np))
        if f is not None:
            Xq = self.mesh.physical(np.arange(nel), self.ref.xi_q)
            F += (f(Xq) * (self.ref.w_q * self.J)[None]) @ self.Psi_q
        if um is not None and self.dt is not None:
            F += (um @ self.M.T) / self.dt
        return F

    def state(self, U):
        """Upwind traces produced by each element: face values where beta.n^- > 0, else 0."""
        return self.face_values(U) * (self.bn_nodes > 0)

    def interpolate(self, fn):
        """Nodal interpolant of fn at the GLL nodes of every element: (nel, Np)."""
        X = self.mesh.physical(np.arange(self.mesh.nel), self.ref.xi_nodes)
        return fn(X)
