"""Structured meshes of axis-aligned boxes for the oracle.

TEST INFRASTRUCTURE ONLY (part of the CPU oracle; never imported by the product path).

Section 2 of the paper partitions the domain into non-overlapping elements K_j,
with skeleton E_h of uniquely defined faces and outward normals n^- on the element
and n^+ = -n^- on its neighbour.  Every workload here is a uniform grid of boxes on
[0, L_0] x ... x [0, L_{d-1}], optionally periodic per axis.
Element index e = i_0 + N_0 (i_1 + N_1 i_2).
"""
import numpy as np


class StructuredMesh:
    def __init__(self, n, L=None, periodic=None):
        self.n = tuple(int(v) for v in n)
        self.d = len(self.n)
        self.L = tuple(float(v) for v in (L if L is not None else (1.0,) * self.d))
        self.periodic = tuple(bool(v) for v in (periodic if periodic is not None else (False,) * self.d))
        self.h = np.array([self.L[a] / self.n[a] for a in range(self.d)])
        self.nel = int(np.prod(self.n))
        idx = np.indices(self.n[::-1]).reshape(self.d, -1).T[:, ::-1]   # (nel, d), axis 0 fastest
        self.ijk = idx.copy()
        self.x0 = self.ijk * self.h                                      # lower corner per element

    def elem(self, ijk):
        e = 0
        stride = 1
        for a in range(self.d):
            e += ijk[..., a] * stride
            stride *= self.n[a]
        return e

    def neighbour(self, f):
        """Neighbour element across face f for every element, -1 on a non-periodic boundary."""
        ax, side = f // 2, f % 2
        step = -1 if side == 0 else 1
        nb = self.ijk.copy()
        nb[:, ax] += step
        out = np.full(self.nel, -1, dtype=np.int64)
        if self.periodic[ax]:
            nb[:, ax] %= self.n[ax]
            return self.elem(nb)
        ok = (nb[:, ax] >= 0) & (nb[:, ax] < self.n[ax])
        out[ok] = self.elem(nb[ok])
        return out

    def normal(self, f):
        v = np.zeros(self.d)
        v[f // 2] = -1.0 if f % 2 == 0 else 1.0
        return v

    def physical(self, e, xi):
        """Physical coordinates of reference points xi (n, d) in elements e (m,) -> (m, n, d)."""
        e = np.atleast_1d(e)
        return self.x0[e][:, None, :] + (np.atleast_2d(xi)[None, :, :] + 1.0) * 0.5 * self.h[None, None, :]
