"""Algorithm 1 of the paper (the eHDG fixed-point iteration), volume form (oracle).

TEST INFRASTRUCTURE ONLY (part of the CPU oracle; never imported by the product path).

Algorithm 1 (Section 3): from an initial guess u^0 compute the trace uhat^0 with the
trace formula; then repeat: solve every element's local equation for u^{k+1} with the
trace uhat^k, compute uhat^{k+1} from u^{k+1}, check convergence.

The operator objects (Transport, ShallowWater, Euler) supply the pieces:
trace(U), rhs(F, trace), solve(R) and state(U).

Convergence check (the paper states its criteria only for its experiments): the
relative l2 norm of the increment of the per-element state that forms the next
trace, ||s(u^{k+1}) - s(u^k)||_2 / ||s(u^{k+1})||_2 < tol, where s is the upwind
outflow trace for transport and the per-side characteristic half-state for the
systems (each operator's `state`).  If ||s(u^{k+1})|| = 0 the absolute norm is used.
The count returned is the number of local solves performed up to and including
the first one after which the check holds (the initial trace is not counted).
The paper's own experiment criteria are available through `criterion`.
"""
import numpy as np


def rel_increment(s_new, s_old):
    num = np.sqrt(np.sum((s_new - s_old) ** 2))
    den = np.sqrt(np.sum(s_new ** 2))
    return num / den if den > 0 else num


def solve(op, F, u0, tol=1e-10, max_iter=10000, criterion=None, history=False):
    """Run Algorithm 1.  Returns dict(u, iters, res, converged, hist, states).

    criterion: optional callable (u_new, u_old) -> bool replacing the default check.
    """
    u = u0.copy()
    uhat = op.trace(u)
    res_hist = []
    s_old = op.state(u)
    for k in range(max_iter):
        u_new = op.solve(op.rhs(F, uhat))
        uhat = op.trace(u_new)
        s_new = op.state(u_new)
        r = rel_increment(s_new, s_old)
        res_hist.append(r)
        done = criterion(u_new, u) if criterion is not None else (r < tol)
        u, s_old = u_new, s_new
        if done:
            return dict(u=u, iters=k + 1, res=r, converged=True, hist=np.array(res_hist))
        if not np.isfinite(r):
            break
    return dict(u=u, iters=len(res_hist), res=res_hist[-1] if res_hist else np.nan,
                converged=False, hist=np.array(res_hist))


def iterate(op, F, u0, n):
    """Exactly n sweeps of Algorithm 1 (no convergence check).  Returns (u^n, u^{n-1})."""
    u = u0.copy()
    uprev = u
    uhat = op.trace(u)
    for _ in range(n):
        uprev = u
        u = op.solve(op.rhs(F, uhat))
        uhat = op.trace(u)
    return u, uprev


def be_steps(op, u0, nsteps, tol=1e-10, max_iter=10000, load=None, criterion=None):
    """Backward-Euler steps; each step runs Algorithm 1 warm-started from the previous
    step's solution (Section 4.4: the initial guess of a step is the previous solution).

    load(um) -> F builds the step's right-hand side (the operator's `load` by default).
    Returns (u_final, iterations per step).
    """
    u = u0.copy()
    its = []
    for _ in range(nsteps):
        F = (load or op.load)(u)
        out = solve(op, F, u, tol=tol, max_iter=max_iter,
                    criterion=(None if criterion is None else criterion))
        if not out["converged"]:
            raise RuntimeError("eHDG did not converge within a backward-Euler step")
        u = out["u"]
        its.append(out["iters"])
    return u, its


def l2_norm(op, U, fn=None, nquad_extra=1):
    """||u_h - fn||_{L2(Omega)} (fn callable of x, or None for ||u_h||), by Gauss quadrature."""
    from .basis import RefElement
    ref = op.ref
    q = RefElement(ref.p, ref.d, nquad=ref.p + 2 + nquad_extra)
    Psi = ref.basis(q.xi_q)
    mesh = op.mesh
    vals = U @ Psi.T
    if fn is not None:
        X = mesh.physical(np.arange(mesh.nel), q.xi_q)
        vals = vals - fn(X)
    return np.sqrt(np.sum(vals ** 2 * (q.w_q * op.J)[None]))
