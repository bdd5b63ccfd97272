"""Shared test-case builders: the same closed-form inputs for the oracle (numpy, at
its own points) and for the HIP path (torch, at the library's points)."""
import numpy as np

from oracle.mesh import StructuredMesh
from oracle.swe import ShallowWater
from oracle.transport import Transport
from paper_1601_06681_amd import workloads as W


def oracle_transport(n, L, p, beta, sigma, dt=None, periodic=None, manufactured=True):
    d = len(n)
    mesh = StructuredMesh(n, L=L[:d], periodic=periodic)
    if manufactured:
        ue, f = (W.transport_manufactured_2d if d == 2 else W.transport_manufactured_3d)(beta, sigma)
    else:
        ue, f = None, None
    op = Transport(mesh, p, tuple(beta[:d]), sigma=sigma, dt=dt, g=(lambda X: ue(X, np)) if ue else None)
    F = op.load((lambda X: f(X, np)) if f else None)
    return op, F, ue, f


def gpu_transport(n, L, p, beta, sigma, dt=0.0, periodic=(0, 0, 0), precision=0, inner=1, manufactured=True):
    from paper_1601_06681_amd.ehdg import EHDG_TRANSPORT, Problem
    d = len(n)
    prob = Problem(EHDG_TRANSPORT, d, n, L=L, periodic=periodic, degree=p, beta=beta, sigma=sigma, dt=dt,
                   precision=precision, inner_sweeps=inner)
    if manufactured:
        ue, f = (W.transport_manufactured_2d if d == 2 else W.transport_manufactured_3d)(beta, sigma)
        prob.set_forcing([f], ue)
    prob.set_initial(None)
    return prob


def oracle_swe(n, p, Phi, dt, periodic=True, L=(1.0, 1.0)):
    mesh = StructuredMesh(n, L=L, periodic=(periodic, periodic))
    return ShallowWater(mesh, p, Phi, dt)


def swe_initial_fns(seed=0, width=0.05, L=(1.0, 1.0)):
    return W.gaussian_hump(W.hump_centre(seed), width=width, L=L)


def swe_random_fns(seed):
    """A smooth random periodic initial state (three fields), for parity cases."""
    rng = np.random.default_rng(seed)
    a = rng.uniform(-1, 1, (3, 3))

    def mk(i):
        def fn(X, xp=np):
            x, y = X[..., 0], X[..., 1]
            return (a[i, 0] * xp.sin(2 * np.pi * x + a[i, 1]) * xp.cos(2 * np.pi * y)
                    + a[i, 2] * xp.cos(4 * np.pi * y + a[i, 0]))
        return fn
    return [mk(0), mk(1), mk(2)]


def rel_err(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    scale = max(np.abs(b).max(), 1e-300)
    return np.abs(a - b).max() / scale
