"""Host-side ring arithmetic (csrc/ring.h): the per-step sweep counts live in a device
ring of 65,536 entries, and a read of `count` entries from logical index `first` is at
most two copies.  Compiled with g++ (no GPU) and checked against the plain definition,
slot of logical entry i = i mod cap, at the wrap point and on random cases."""
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1601_06681_amd", "csrc")

DRIVER = r"""
#include <cstdio>
#include "ring.h"
int main() {
  long long first, count, cap;
  while (std::scanf("%lld %lld %lld", &first, &count, &cap) == 3) {
    const ehdg::RingSpan r = ehdg::ring_span(first, count, cap);
    std::printf("%zu %zu %zu %zu\n", r.off0, r.n0, r.off1, r.n1);
  }
  return 0;
}
"""


@pytest.fixture(scope="module")
def ring_bin(tmp_path_factory):
    d = tmp_path_factory.mktemp("ring")
    src = d / "drv.cpp"
    src.write_text(DRIVER)
    exe = d / "drv"
    subprocess.run(["g++", "-std=c++17", "-O1", "-I", CSRC, str(src), "-o", str(exe)], check=True)
    return str(exe)


def _spans(exe, cases):
    inp = "".join(f"{f} {c} {k}\n" for f, c, k in cases)
    out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout.split("\n")
    return [tuple(int(v) for v in line.split()) for line in out if line.strip()]


def _slots(span):
    off0, n0, off1, n1 = span
    return list(range(off0, off0 + n0)) + list(range(off1, off1 + n1))


def test_wrap_point_of_the_step_ring(ring_bin):
    cap = 1 << 16
    cases = [(0, 5, cap), (cap - 3, 3, cap), (cap - 3, 7, cap), (cap, 4, cap), (3 * cap + 10, cap, cap),
             (cap - 1, cap, cap), (100_000, 10, cap), (5, 0, cap)]
    for case, span in zip(cases, _spans(ring_bin, cases)):
        first, count, k = case
        assert _slots(span) == [(first + i) % k for i in range(count)], (case, span)
        assert span[1] + span[3] == count
    # a read that straddles the end is exactly two copies
    assert _spans(ring_bin, [(cap - 3, 7, cap)])[0] == (cap - 3, 3, 0, 4)


def test_random_reads_match_the_definition(ring_bin):
    rng = np.random.default_rng(11)
    cases = []
    for _ in range(400):
        cap = int(rng.integers(1, 50))
        cases.append((int(rng.integers(0, 10 * cap)), int(rng.integers(0, cap + 1)), cap))
    for case, span in zip(cases, _spans(ring_bin, cases)):
        first, count, k = case
        assert _slots(span) == [(first + i) % k for i in range(count)], (case, span)
