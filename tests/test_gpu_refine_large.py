"""The FP32 correction form of the degree-3 3D transport family above 64 MB of FP32 state
(73 x 71 x 72 hexahedra: 373 176 elements x 48 values x 4 B = 71.6 MB; the last tile of 16
elements is ragged, 8 elements), where the correction and the residual are stored
element-major and swept by k_inner32_aos (below that size the component-major form runs,
which the small parity cases cover against the oracle).

At this size the oracle takes too long, so the checks are properties that hold at any
size, against the FP64 path (itself pinned to the oracle on smaller meshes and on the
first sweeps of 64^3): the corrected form converges to the FP64 fixed point (Section 3:
the refinement's residual is the FP64 one, so its fixed point is the FP64 one), with 1, 2
and 8 sweeps per refinement (no correction sweep; the only one, which stores s'; seven
plain ones and the last); and backward-Euler steps split over two calls equal the FP64
steps.  Bars: the solves stop at relative increments of 1e-11 (FP64: 1e-12), whose
stopping error is below 1e-9 relative for these contraction rates; 1e-8 is asserted.
"""
import numpy as np
import pytest

from tests._cases import gpu_transport, rel_err

pytestmark = pytest.mark.gpu

N, L, P = (73, 71, 72), (1.0, 0.9, 1.1), 3
BETA, SIGMA = (1.0, 0.7, 0.3), 1.0


def _u(prob):
    return prob.solution().cpu().numpy().reshape(prob.nel, -1)


@pytest.fixture(scope="module")
def fp64_fixed_point():
    prob = gpu_transport(N, L, P, BETA, SIGMA)
    rc, its, res = prob.solve(1e-12, 100000)
    assert res < 1e-12
    u = _u(prob)
    prob.close()
    return u


@pytest.mark.parametrize("inner", [1, 2, 8])
def test_fp32_form_element_major_reaches_fp64_fixed_point(fp64_fixed_point, inner):
    prob = gpu_transport(N, L, P, BETA, SIGMA, precision=1, inner=inner)
    assert prob.nel * 48 * 4 > 64 << 20 and prob.nel % 16 != 0
    rc, its, res = prob.solve(1e-11, 100000)
    assert res < 1e-11
    err = rel_err(_u(prob), fp64_fixed_point)
    print(f"\n[large] FP32 form, {inner} sweeps per refinement: {its} equivalent sweeps, rel err {err:.2e}")
    assert err < 1e-8
    prob.close()


def test_bf16_form_eight_tiles_per_wavefront_reaches_fp64_fixed_point(fp64_fixed_point):
    """The BF16 correction sweep takes 8 tiles per wavefront once the grid at 4 would need
    more than one round of resident workgroups.  At 100 or more registers per lane at most
    5 wavefronts fit per SIMD, at most 1280 workgroups of 4 wavefronts: 64^3 (16 384 tiles)
    runs 4 per wavefront, this mesh (23 324 tiles) 8, with the last correction sweep
    storing s'."""
    prob = gpu_transport(N, L, P, BETA, SIGMA, precision=2, inner=8)
    rc, its, res = prob.solve(1e-11, 100000)
    assert res < 1e-11
    err = rel_err(_u(prob), fp64_fixed_point)
    print(f"\n[large] BF16 form, 8 sweeps per refinement: {its} equivalent sweeps, rel err {err:.2e}")
    assert err < 1e-8
    prob.close()


def test_fp32_form_element_major_be_steps_equal_fp64():
    import torch
    dt = 0.05
    u0 = None
    out = {}
    for prec in (0, 1):
        prob = gpu_transport(N, L, P, BETA, SIGMA, dt=dt, precision=prec, inner=4 if prec else 1)
        if u0 is None:
            X = prob.points("nodes")
            u0 = (torch.cos(3 * X[..., 0]) * torch.sin(2 * X[..., 1]) + X[..., 2]).reshape(prob.nel, 1, -1)
        prob.set_initial(u0.contiguous())
        prob.step(1, 1e-12, 4000)
        prob.step(2, 1e-12, 4000)
        out[prec] = _u(prob)
        prob.close()
    err = rel_err(out[1], out[0])
    print(f"\n[large] FP32 form BE steps against FP64: rel err {err:.2e}")
    assert err < 1e-8
