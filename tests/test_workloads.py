"""Seeded workload generators and the serving queue model, on the CPU.

The manufactured forcings are checked against central differences of their exact
solutions (so a dropped term or a wrong sign fails), the generators against the ranges
and formulas their docstrings state, and the first-in-first-out queue against a case
worked by hand.
"""
import math

import numpy as np

from paper_1601_06681_amd import serving as S
from paper_1601_06681_amd import workloads as W


def _fd_forcing(ue, b, sigma, X, h=1e-5):
    """b . grad ue + sigma ue by central differences."""
    out = sigma * ue(X)
    for a in range(X.shape[-1]):
        e = np.zeros(X.shape[-1])
        e[a] = h
        out = out + b[a] * (ue(X + e) - ue(X - e)) / (2 * h)
    return out


def test_manufactured_forcing_2d():
    rng = np.random.default_rng(1)
    X = rng.uniform(0.0, 1.0, (200, 2))
    for b, sigma in (((1.0, 0.5), 1.0), ((-0.3, 2.0), 0.0), ((0.0, -1.0), 2.5)):
        ue, f = W.transport_manufactured_2d(b, sigma)
        np.testing.assert_allclose(f(X), _fd_forcing(ue, b, sigma, X), atol=1e-8)


def test_manufactured_forcing_3d():
    rng = np.random.default_rng(2)
    X = rng.uniform(0.0, 1.0, (200, 3))
    for b, sigma in (((1.0, 0.7, 0.3), 1.0), ((-0.6, 0.8, -1.0), 0.5)):
        ue, f = W.transport_manufactured_3d(b, sigma)
        np.testing.assert_allclose(f(X), _fd_forcing(ue, b, sigma, X), atol=1e-8)


def test_batch_mix_ranges_and_determinism():
    a, b = W.batch_mix(512, seed=0), W.batch_mix(512, seed=0)
    assert a == b
    assert a != W.batch_mix(512, seed=1)
    kinds = [r["kind"] for r in a]
    assert 0.4 < kinds.count("swe") / len(a) < 0.6
    # the draw is the whole specified mix: degree-1 transport members are present
    assert any(r["kind"] == "transport" and r["degree"] == 1 for r in a)
    for r in a:
        assert 16 <= r["n"] <= 256
        if r["kind"] == "transport":
            assert 1 <= r["degree"] <= 5
            assert math.isclose(math.hypot(*r["beta"]), 1.0, rel_tol=1e-12)
            assert 0.5 <= r["sigma"] <= 2.0
        else:
            p, h = r["degree"], 1.0 / r["n"]
            assert 1 <= p <= 5 and r["steps"] == 5
            assert math.isclose(r["dt"] * (p + 1) * (p + 2) / h, 0.25, rel_tol=1e-12)


def test_serving_requests_ranges_and_determinism():
    a = W.serving_requests(2000, seed=0)
    assert a == W.serving_requests(2000, seed=0)
    assert [r["id"] for r in a] == list(range(2000))
    gaps = np.array([r["gap"] for r in a])
    assert (gaps > 0).all() and 0.9 < gaps.mean() < 1.1   # Exponential(1)
    lam = math.hypot(*W.EULER_U0) + W.EULER_C0
    for r in a:
        if r["kind"] == "euler":
            assert 32 <= r["n"] <= 512 and r["degree"] == 3 and r["steps"] == 10
            assert math.isclose(r["dt"] * 4 * 5 * lam * r["n"], 0.25, rel_tol=1e-12)
        else:
            assert 16 <= r["n"] <= 64 and r["degree"] == 2
            assert r["beta"] == (1.0, 0.7, 0.3) and r["sigma"] == 1.0


def test_fifo_latencies_by_hand():
    # arrivals 0, 1, 1.5 with services 2, 1, 0.5: starts 0, 2, 3; ends 2, 3, 3.5
    lat, end = S.fifo_latencies([0.0, 1.0, 1.5], [2.0, 1.0, 0.5])
    np.testing.assert_allclose(lat, [2.0, 2.0, 2.0])
    assert end == 3.5
    # an idle server starts each request on arrival
    lat, end = S.fifo_latencies([0.0, 10.0], [1.0, 2.0])
    np.testing.assert_allclose(lat, [1.0, 2.0])
    assert end == 12.0


def test_gaussian_hump_is_periodic():
    phi, zero, _ = W.gaussian_hump((0.1, 0.9), width=0.05)
    X = np.array([[0.1, 0.9], [0.0, 0.5], [1.0, 0.5], [0.5, 0.0], [0.5, 1.0], [0.95, 0.05]])
    v = phi(X)
    assert v[0] == 1.0
    # opposite sides of the torus agree (up to the rounding of 1 - 0.9 against 0.1)
    assert math.isclose(v[1], v[2], rel_tol=1e-12) and math.isclose(v[3], v[4], rel_tol=1e-12)
    # (0.95, 0.05) is 0.15 from the centre along each axis once both axes wrap
    assert math.isclose(v[5], math.exp(-(2 * 0.15 ** 2) / (2 * 0.05 ** 2)), rel_tol=1e-12)
    assert (zero(X) == 0.0).all()
