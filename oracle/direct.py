"""Direct (non-iterative) global solves that pin the eHDG fixed point (oracle).

TEST INFRASTRUCTURE ONLY (part of the CPU oracle; never imported by the product path).

Two independent global systems, assembled element by element and solved with a
sparse LU (scipy.sparse.linalg.spsolve):

* hdg_*: the upwind HDG system of Section 3: the local equations with the trace as
  an unknown, closed by the conservation condition on every interior face
  <[[flux]], mu>_e = 0 for all mu in the face trace space; boundary faces carry the
  boundary rule (transport: uhat = g on inflow, uhat = u^- elsewhere; shallow water:
  zero normal mass flux on walls).
* dg_*: a classical upwind discontinuous Galerkin method with no trace unknown:
  the upwind flux beta.n u^upwind for transport and the exact Riemann (Godunov)
  flux for shallow water.  It is built from textbook fluxes, not from the HDG
  formulas, so agreement with the eHDG limit checks the trace formulas themselves.
  For a velocity field beta(x) (dg_transport_variable) the DG form is the strong one,
  with no div(beta) term, so agreement also checks the HDG operator's volume term.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def _face_ids(mesh):
    """Unique face id for every (element, face); interior faces are shared."""
    d = mesh.d
    fid = -np.ones((mesh.nel, 2 * d), dtype=np.int64)
    nxt = 0
    nbr = [mesh.neighbour(f) for f in range(2 * d)]
    for e in range(mesh.nel):
        for f in range(2 * d):
            if fid[e, f] >= 0:
                continue
            fid[e, f] = nxt
            nb = nbr[f][e]
            if nb >= 0:
                fid[nb, f ^ 1] = nxt
            nxt += 1
    return fid, nxt, nbr


# --------------------------------------------------------------------------------
# transport (constant beta)
# --------------------------------------------------------------------------------
def _transport_face_mats(op, f):
    pts, wf, Pf, Mu = op.face[f]
    return pts, wf, Pf, Mu


def hdg_transport(op, F):
    """Global upwind HDG solve for a constant-beta Transport operator. Returns U (nel, Np)."""
    assert op.const
    mesh, ref, d = op.mesh, op.ref, op.d
    Np, nf = ref.Np, ref.nf
    fid, nface, nbr = _face_ids(mesh)
    nu = mesh.nel * Np
    ntot = nu + nface * nf
    rows, cols, vals = [], [], []
    rhs = np.zeros(ntot)

    def add(r0, c0, B):
        ii, jj = np.nonzero(B)
        rows.extend(r0 + ii)
        cols.extend(c0 + jj)
        vals.extend(B[ii, jj])

    for e in range(mesh.nel):
        add(e * Np, e * Np, op.A)
        rhs[e * Np:(e + 1) * Np] = F[e]
        for f in range(2 * d):
            add(e * Np, nu + fid[e, f] * nf, -op.lifts[f])
    # face equations
    done = np.zeros(nface, dtype=bool)
    for e in range(mesh.nel):
        for f in range(2 * d):
            k = fid[e, f]
            if done[k]:
                continue
            done[k] = True
            r0 = nu + k * nf
            nb = nbr[f][e]
            if nb < 0:
                bn = op.bn[f]
                Pn = op.Psi_fn[f]                   # (nf, Np) values at face nodes
                add(r0, r0, np.eye(nf))
                if bn < 0:
                    xb = mesh.physical(e, ref.face_node_xi(f))[0]
                    rhs[r0:r0 + nf] = op.g(xb) if op.g is not None else 0.0
                else:
                    add(r0, e * Np, -Pn)
                continue
            # conservation: sum over both sides of <beta.n u + |beta.n| (u - uhat), mu_a>
            for (el, fl) in ((e, f), (nb, f ^ 1)):
                pts, wf, Pf, Mu = op.face[fl]
                bn = op.bn[fl]
                add(r0, el * Np, np.einsum("q,qa,qj->aj", wf, Mu, Pf) * (bn + abs(bn)))
                add(r0, r0, -abs(bn) * np.einsum("q,qa,qb->ab", wf, Mu, Mu))
    Amat = sp.csr_matrix((vals, (rows, cols)), shape=(ntot, ntot))
    x = spla.spsolve(Amat.tocsc(), rhs)
    return x[:nu].reshape(mesh.nel, Np)


def dg_transport(op, F):
    """Classical upwind DG (flux beta.n u^upwind) for constant beta. Returns U (nel, Np)."""
    assert op.const
    mesh, ref, d = op.mesh, op.ref, op.d
    Np = ref.Np
    h = mesh.h
    J = op.J
    Psi = ref.basis(ref.xi_q)
    G = ref.grad_basis(ref.xi_q)
    wq = ref.w_q * J
    b = op.beta_vec
    # volume: -(u, beta.grad v) + react (u, v)
    bgrad = sum(b[a] * G[a] * (2.0 / h[a]) for a in range(d))
    Avol = -np.einsum("q,qj,qi->ij", wq, Psi, bgrad) + op.react * np.einsum("q,qj,qi->ij", wq, Psi, Psi)
    nbr = [mesh.neighbour(f) for f in range(2 * d)]
    rows, cols, vals = [], [], []
    rhs = F.reshape(-1).copy()

    def add(r0, c0, B):
        ii, jj = np.nonzero(B)
        rows.extend(r0 + ii)
        cols.extend(c0 + jj)
        vals.extend(B[ii, jj])

    for e in range(mesh.nel):
        add(e * Np, e * Np, Avol)
        for f in range(2 * d):
            pts, wf, Pf, Mu = op.face[f]
            bn = op.bn[f]
            if bn > 0:
                add(e * Np, e * Np, bn * np.einsum("q,qj,qi->ij", wf, Pf, Pf))
            elif bn < 0:
                nb = nbr[f][e]
                if nb >= 0:
                    # neighbour's polynomial at the same physical points (its face f^1)
                    pts_o = pts.copy()
                    ax = f // 2
                    pts_o[:, ax] = -pts[:, ax]
                    Po = ref.basis(pts_o)
                    add(e * Np, nb * Np, bn * np.einsum("q,qj,qi->ij", wf, Po, Pf))
                else:
                    # boundary data enters through its interpolant at the face nodes,
                    # the same representation the HDG trace uses
                    Xn = mesh.physical(e, ref.face_node_xi(f))[0]
                    gn = op.g(Xn) if op.g is not None else np.zeros(Xn.shape[0])
                    gv = Mu @ gn
                    rhs[e * Np:(e + 1) * Np] -= bn * np.einsum("q,q,qi->i", wf, gv, Pf)
    Amat = sp.csr_matrix((vals, (rows, cols)), shape=(mesh.nel * Np,) * 2)
    return spla.spsolve(Amat.tocsc(), rhs).reshape(mesh.nel, Np)


# --------------------------------------------------------------------------------
# shallow water
# --------------------------------------------------------------------------------
def hdg_swe(op, F):
    """Global HDG solve (unknowns U and phihat) for a ShallowWater operator."""
    mesh, ref = op.mesh, op.ref
    Np, nf = ref.Np, ref.nf
    n = 3 * Np
    fid, nface, nbr = _face_ids(mesh)
    nu = mesh.nel * n
    ntot = nu + nface * nf
    rows, cols, vals = [], [], []
    rhs = np.zeros(ntot)
    Phi, sq = op.Phi, op.sq

    def add(r0, c0, B):
        ii, jj = np.nonzero(B)
        rows.extend(r0 + ii)
        cols.extend(c0 + jj)
        vals.extend(B[ii, jj])

    for e in range(mesh.nel):
        add(e * n, e * n, op.A)
        rhs[e * n:(e + 1) * n] = F[e]
        for f in range(4):
            add(e * n, nu + fid[e, f] * nf, -op.lifts[f])
    done = np.zeros(nface, dtype=bool)
    for e in range(mesh.nel):
        for f in range(4):
            k = fid[e, f]
            if done[k]:
                continue
            done[k] = True
            r0 = nu + k * nf
            nb = nbr[f][e]
            sides = ((e, f),) if nb < 0 else ((e, f), (nb, f ^ 1))
            for (el, fl) in sides:
                pts, w = ref.face_quadrature(fl)
                Jf = mesh.h[1 - fl // 2] / 2.0
                Pf = ref.basis(pts)
                Mu = ref.face_trace_basis(fl, pts)
                W = np.einsum("q,qa,qj->aj", w * Jf, Mu, Pf)
                n1, n2 = op.nvec[fl]
                # flux Phi vel.n + sqrt(Phi) (phi - phihat), tested with mu_a
                add(r0, el * n, sq * W)
                add(r0, el * n + Np, Phi * n1 * W)
                add(r0, el * n + 2 * Np, Phi * n2 * W)
                add(r0, r0, -sq * np.einsum("q,qa,qb->ab", w * Jf, Mu, Mu))
    Amat = sp.csr_matrix((vals, (rows, cols)), shape=(ntot, ntot))
    x = spla.spsolve(Amat.tocsc(), rhs)
    return x[:nu].reshape(mesh.nel, n)


def dg_swe(op, F):
    """DG with the exact Riemann (Godunov) flux for the linear shallow-water system.

    At a face with normal n (own side -, neighbour +) the Riemann state is
      phi*  = (phi^- + phi^+)/2 + sqrt(Phi) (vn^- - vn^+)/2,
      vn*   = (vn^- + vn^+)/2 + (phi^- - phi^+) / (2 sqrt(Phi)),   vn = vel.n,
    and the numerical fluxes are Phi vn* (mass) and Phi phi* n (momentum).
    Walls use the mirror state phi^+ = phi^-, vn^+ = -vn^-.
    """
    mesh, ref = op.mesh, op.ref
    Np = ref.Np
    n = 3 * Np
    h = mesh.h
    Phi, sq, dt = op.Phi, op.sq, op.dt
    Psi = ref.basis(ref.xi_q)
    G = ref.grad_basis(ref.xi_q)
    wq = ref.w_q * op.J
    M = np.einsum("q,qj,qi->ij", wq, Psi, Psi)
    Kx = np.einsum("q,qj,qi->ij", wq, Psi, G[0] * (2.0 / h[0]))
    Ky = np.einsum("q,qj,qi->ij", wq, Psi, G[1] * (2.0 / h[1]))
    P, U, V = slice(0, Np), slice(Np, 2 * Np), slice(2 * Np, 3 * Np)
    Avol = np.zeros((n, n))
    Avol[P, P] = M / dt
    Avol[P, U] = -Phi * Kx
    Avol[P, V] = -Phi * Ky
    Avol[U, U] = Phi * M / dt
    Avol[U, P] = -Phi * Kx
    Avol[V, V] = Phi * M / dt
    Avol[V, P] = -Phi * Ky
    nbr = [mesh.neighbour(f) for f in range(4)]
    rows, cols, vals = [], [], []

    def add(r0, c0, B):
        ii, jj = np.nonzero(B)
        rows.extend(r0 + ii)
        cols.extend(c0 + jj)
        vals.extend(B[ii, jj])

    for e in range(mesh.nel):
        add(e * n, e * n, Avol)
        for f in range(4):
            pts, w = ref.face_quadrature(f)
            Jf = h[1 - f // 2] / 2.0
            wf = w * Jf
            Pm = ref.basis(pts)
            pts_o = pts.copy()
            pts_o[:, f // 2] = -pts[:, f // 2]
            Po = ref.basis(pts_o)
            n1, n2 = op.nvec[f]
            nb = nbr[f][e]
            # linear maps from element unknowns to (phi, vn) at face quadrature points
            def phi_of(Pq):
                Z = np.zeros((Pq.shape[0], n)); Z[:, P] = Pq; return Z
            def vn_of(Pq):
                Z = np.zeros((Pq.shape[0], n)); Z[:, U] = n1 * Pq; Z[:, V] = n2 * Pq; return Z
            ph_m, vn_m = phi_of(Pm), vn_of(Pm)
            if nb >= 0:
                ph_p, vn_p = phi_of(Po), vn_of(Po)      # neighbour's vel dotted with OUR normal
                blocks = [(e, 0.5 * ph_m + 0.5 * sq * vn_m, 0.5 * vn_m + 0.5 / sq * ph_m),
                          (nb, 0.5 * ph_p - 0.5 * sq * vn_p, 0.5 * vn_p - 0.5 / sq * ph_p)]
            else:
                # mirror state: phi* = phi^- + sqrt(Phi) vn^-, vn* = 0
                blocks = [(e, ph_m + sq * vn_m, 0.0 * vn_m)]
            for (el, phs, vns) in blocks:
                B = np.zeros((n, n))
                B[P] = Phi * np.einsum("q,qi,qj->ij", wf, Pm, vns)
                B[U] = Phi * n1 * np.einsum("q,qi,qj->ij", wf, Pm, phs)
                B[V] = Phi * n2 * np.einsum("q,qi,qj->ij", wf, Pm, phs)
                add(e * n, el * n, B)
    Amat = sp.csr_matrix((vals, (rows, cols)), shape=(mesh.nel * n,) * 2)
    return spla.spsolve(Amat.tocsc(), F.reshape(-1)).reshape(mesh.nel, n)


# --------------------------------------------------------------------------------
# transport (variable beta): classical upwind DG in strong form
# --------------------------------------------------------------------------------
def dg_transport_variable(op, F):
    """Classical upwind DG for beta.grad u + react u = f with a velocity field beta(x).

    Strong (non-integrated) form of Lesaint-Raviart / Johnson-Pitkaranta type: on every
    element K and for every test function v,

        (beta.grad u + react u, v)_K + sum over inflow points of dK of
            |beta.n| (u^- - u^ext) v  =  (f, v)_K,

    where a face quadrature point is an inflow point of K when beta(x).n^- < 0 there,
    u^ext is the upwind neighbour's polynomial at the same physical point, or on the
    domain boundary the L2 projection of g onto the face polynomials (the same data
    the HDG trace carries).  Nothing here uses div(beta), the HDG lifts or a trace
    unknown: the paper's local equation eq. transportLocal integrates by parts to this
    form pointwise (its volume term -(u, div(beta v)) becomes (beta.grad u, v) minus
    <beta.n u, v> on dK), so where the quadrature integrates both forms exactly
    (polynomial beta of low degree) the eHDG fixed point equals this solve to rounding,
    and a wrong sign or factor on the div(beta) term of the HDG operator shows up as a
    mismatch.  op: a variable-beta Transport (its mesh, reference element, beta, react,
    boundary data g).  Returns U (nel, Np).
    """
    mesh, ref, d = op.mesh, op.ref, op.d
    Np = ref.Np
    nel = mesh.nel
    h = mesh.h
    Psi = ref.basis(ref.xi_q)                                   # (Nq, Np)
    G = ref.grad_basis(ref.xi_q)                                # d x (Nq, Np)
    wq = ref.w_q * op.J
    Xq = mesh.physical(np.arange(nel), ref.xi_q)                # (nel, Nq, d)
    B = op.beta(Xq)                                             # (nel, Nq, d)
    # (beta.grad psi_j, psi_i)_K + react (psi_j, psi_i)_K per element
    dpsi = np.stack([G[a] * (2.0 / h[a]) for a in range(d)], axis=-1)      # (Nq, Np, d)
    bgrad = np.einsum("eqa,qja->eqj", B, dpsi)                            # beta.grad psi_j
    Avol = np.einsum("q,eqj,qi->eij", wq, bgrad, Psi) + op.react * np.einsum("q,qj,qi->ij", wq, Psi, Psi)[None]
    nbr = [mesh.neighbour(f) for f in range(2 * d)]
    rows, cols, vals = [], [], []
    rhs = F.reshape(-1).copy()

    def add(r0, c0, M):
        ii, jj = np.nonzero(M)
        rows.extend(r0 + ii)
        cols.extend(c0 + jj)
        vals.extend(M[ii, jj])

    for e in range(nel):
        add(e * Np, e * Np, Avol[e])
    for f in range(2 * d):
        pts, w = ref.face_quadrature(f)
        Jf = np.prod([h[a] / 2.0 for a in range(d) if a != f // 2]) if d > 1 else 1.0
        wf = w * Jf
        Pm = ref.basis(pts)                                     # own basis at the face points
        pts_o = pts.copy()
        pts_o[:, f // 2] = -pts[:, f // 2]
        Po = ref.basis(pts_o)                                   # neighbour's basis, same points
        Mu = ref.face_trace_basis(f, pts)                       # face polynomials (for g's projection)
        Mf = np.einsum("q,qa,qb->ab", wf, Mu, Mu)
        nvec = mesh.normal(f)
        Xf = mesh.physical(np.arange(nel), pts)                 # (nel, nqf, d)
        bn = op.beta(Xf) @ nvec                                 # (nel, nqf)
        wt = np.where(bn < 0, -bn, 0.0) * wf[None]              # |beta.n| w at inflow points
        for e in range(nel):
            if not np.any(wt[e]):
                continue
            add(e * Np, e * Np, np.einsum("q,qi,qj->ij", wt[e], Pm, Pm))
            nb = nbr[f][e]
            if nb >= 0:
                add(e * Np, nb * Np, -np.einsum("q,qi,qj->ij", wt[e], Pm, Po))
            elif op.g is not None:
                gq = op.g(Xf[e:e + 1])[0]                       # g at the face points
                coef = np.linalg.solve(Mf, Mu.T @ (wf * gq))    # L2 projection onto the face space
                rhs[e * Np:(e + 1) * Np] += np.einsum("q,qi,q->i", wt[e], Pm, Mu @ coef)
    Amat = sp.csr_matrix((vals, (rows, cols)), shape=(nel * Np,) * 2)
    return spla.spsolve(Amat.tocsc(), rhs).reshape(nel, Np)
