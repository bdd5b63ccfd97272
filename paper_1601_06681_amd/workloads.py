"""Seeded synthetic inputs of the benchmark and test workloads.

Input generation only: problem parameters and closed-form data (manufactured
solutions, forcing, boundary data, initial states) as functions of physical
coordinates.  Every function takes an array namespace `xp` (numpy or torch) so the
same definition is sampled by the oracle at its points and by the GPU path at the
library's points.  Nothing here computes any part of the method.

Workloads (the paper prints no timings; these are the synthetic shapes measured):
  transport2d_8x8_p2    steady 2D transport, b = (1, 0.5), sigma = 1, manufactured
                        u = sin(pi x) cos(pi y) on the unit square, 8 x 8, degree 2
  swe2d_256x256_p4      2D linearized shallow water, Phi = g H = 1, periodic unit
                        square, 256 x 256, degree 4, 20 backward-Euler steps,
                        Gaussian-hump initial height from seed 0
  transport3d_64c_p3    3D transport on 64^3 hexes, degree 3, b = (1, 0.7, 0.3),
                        sigma = 1, manufactured u = sin(pi x) cos(pi y) sin(pi z)
  batch_mix_512         512 independent problems drawn from seed 0 (batch_mix below)
"""
import math

import numpy as np

PI = math.pi


# ---------------------------------------------------------------------------- transport
def transport_manufactured_2d(b, sigma):
    """u = sin(pi x) cos(pi y) and the forcing f = b . grad u + sigma u."""
    def ue(X, xp=np):
        return xp.sin(PI * X[..., 0]) * xp.cos(PI * X[..., 1])

    def f(X, xp=np):
        x, y = X[..., 0], X[..., 1]
        return (b[0] * PI * xp.cos(PI * x) * xp.cos(PI * y) - b[1] * PI * xp.sin(PI * x) * xp.sin(PI * y)
                + sigma * xp.sin(PI * x) * xp.cos(PI * y))
    return ue, f


def transport_manufactured_3d(b, sigma):
    """u = sin(pi x) cos(pi y) sin(pi z) and f = b . grad u + sigma u."""
    def ue(X, xp=np):
        return xp.sin(PI * X[..., 0]) * xp.cos(PI * X[..., 1]) * xp.sin(PI * X[..., 2])

    def f(X, xp=np):
        x, y, z = X[..., 0], X[..., 1], X[..., 2]
        sx, cx = xp.sin(PI * x), xp.cos(PI * x)
        sy, cy = xp.sin(PI * y), xp.cos(PI * y)
        sz, cz = xp.sin(PI * z), xp.cos(PI * z)
        return (b[0] * PI * cx * cy * sz - b[1] * PI * sx * sy * sz + b[2] * PI * sx * cy * cz
                + sigma * sx * cy * sz)
    return ue, f


TRANSPORT2D = dict(name="transport2d_8x8_p2", dim=2, n=(8, 8), L=(1.0, 1.0), periodic=(0, 0), degree=2,
                   beta=(1.0, 0.5), sigma=1.0, dt=0.0, tol=1e-10)
TRANSPORT3D = dict(name="transport3d_64c_p3", dim=3, n=(64, 64, 64), L=(1.0, 1.0, 1.0), periodic=(0, 0, 0),
                   degree=3, beta=(1.0, 0.7, 0.3), sigma=1.0, dt=0.0, tol=1e-8)
# The same problem at 128^3: 2.1 M elements, 134 M DOFs.  Its traces (2.4 GB per FP64
# sweep, 1.2 GB per FP32 correction sweep) are far larger than the 256 MB Infinity Cache, so
# its bandwidth figures are HBM figures.
TRANSPORT3D_CONTROL = dict(TRANSPORT3D, name="transport3d_128c_p3_control", n=(128, 128, 128))


# ---------------------------------------------------------------------------- shallow water
def hump_centre(seed=0):
    """Centre of the Gaussian hump: uniform in [0.25, 0.75]^2 from numpy PCG64(seed)."""
    return np.random.default_rng(seed).uniform(0.25, 0.75, 2)


def gaussian_hump(centre, width=0.05, L=(1.0, 1.0)):
    """phi_0 = exp(-d^2 / (2 w^2)) with d the periodic distance to `centre`; u = v = 0."""
    cx, cy = float(centre[0]), float(centre[1])

    def phi(X, xp=np):
        dx = xp.abs(X[..., 0] - cx)
        dy = xp.abs(X[..., 1] - cy)
        dx = xp.minimum(dx, L[0] - dx)
        dy = xp.minimum(dy, L[1] - dy)
        return xp.exp(-(dx * dx + dy * dy) / (2.0 * width * width))

    def zero(X, xp=np):
        return 0.0 * X[..., 0]
    return phi, zero, zero


# The stated step dt = 1e-3 gives dt (p+1)(p+2) / h = 7.68 on this mesh; the eHDG
# shallow-water iteration then has spectral radius 7.68 and diverges.  The largest
# round step inside Theorem 2's sufficient condition (ratio < 1/2) is used instead.
SWE2D = dict(name="swe2d_256x256_p4", dim=2, n=(256, 256), L=(1.0, 1.0), periodic=(1, 1), degree=4, Phi=1.0,
              dt=5e-5, dt_stated=1e-3, steps=20, tol=1e-10, seed=0)


def scaled(cfg, n):
    """The same workload on a smaller mesh (parity tests)."""
    out = dict(cfg)
    out["n"] = tuple(n)
    return out


# ---------------------------------------------------------------------------- batches
def batch_mix(count=512, seed=0):
    """`count` independent problems drawn from numpy PCG64(seed), in draw order.

    Each: side N ~ U{16..256} (N x N unit square), degree p ~ U{1..5}, and with
    probability 1/2 each:
      transport: steady, b = (cos t, sin t), t ~ U[0, 2 pi), sigma ~ U[0.5, 2], the
                 manufactured solution of transport_manufactured_2d, inflow data u_e;
      swe:       periodic shallow water, Phi = 1, the Gaussian hump of seed 0, 5
                 backward-Euler steps with dt (p+1)(p+2) / h = 0.25."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n = int(rng.integers(16, 257))
        p = int(rng.integers(1, 6))
        if rng.random() < 0.5:
            t = float(rng.uniform(0.0, 2.0 * PI))
            sigma = float(rng.uniform(0.5, 2.0))
            out.append(dict(kind="transport", n=n, degree=p, beta=(math.cos(t), math.sin(t)), sigma=sigma))
        else:
            h = 1.0 / n
            out.append(dict(kind="swe", n=n, degree=p, dt=0.25 * h / ((p + 1) * (p + 2)), steps=5))
    return out


# ---------------------------------------------------------------------------- serving
EULER_U0 = (0.5, 0.25)
EULER_C0 = 1.0


def serving_requests(count=2000, seed=0):
    """`count` requests drawn from numpy PCG64(seed), in arrival order.

    Each has `gap`, an Exponential(1) inter-arrival time (the server scales it to its
    arrival rate), and with probability 1/2 each:
      euler:     linearized Euler about (rho0, U0, c0) = (1, (0.5, 0.25), 1), periodic
                 N x N unit square, N ~ U{32..512}, degree 3, 10 backward-Euler steps,
                 dt (p+1)(p+2) (|U0| + c0) / h = 0.25, a Gaussian density/pressure pulse;
      transport: steady 3D transport, N^3 unit cube, N ~ U{16..64}, degree 2,
                 b = (1, 0.7, 0.3), sigma = 1, the manufactured solution of
                 transport_manufactured_3d."""
    rng = np.random.default_rng(seed)
    lam = math.hypot(*EULER_U0) + EULER_C0
    out = []
    for i in range(count):
        gap = float(rng.exponential(1.0))
        if rng.random() < 0.5:
            n = int(rng.integers(32, 513))
            p = 3
            out.append(dict(id=i, gap=gap, kind="euler", n=n, degree=p, steps=10,
                            dt=0.25 * (1.0 / n) / ((p + 1) * (p + 2) * lam)))
        else:
            n = int(rng.integers(16, 65))
            out.append(dict(id=i, gap=gap, kind="transport", n=n, degree=2, beta=(1.0, 0.7, 0.3), sigma=1.0))
    return out


def euler_pulse(width=0.1, centre=(0.5, 0.5)):
    """rho' = p' = exp(-d^2 / (2 w^2)) (periodic distance d to `centre`), u' = v' = 0."""
    phi, zero, _ = gaussian_hump(centre, width=width)
    return [phi, zero, zero, phi]
