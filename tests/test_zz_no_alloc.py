"""ehdg_batch_create_static (batch tables in the library's static device array, no
workspace) against ehdg_batch_create (tables in a caller workspace), through the C ABI.

Both create the same tables and launch the same kernels, so a member's iteration
counts, residuals and solution must be bitwise equal.  Two static batches are created
in a row: the second with fewer, smaller members reuses the device array, and the first
is then refused (its tables were replaced)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _members(kinds):
    from paper_1601_06681_amd import workloads as W
    from paper_1601_06681_amd.ehdg import EHDG_SWE, EHDG_TRANSPORT, Problem
    out = []
    for kind, n, p, extra in kinds:
        if kind == "transport":
            beta, sigma = extra
            prob = Problem(EHDG_TRANSPORT, 2, (n, n), degree=p, beta=beta, sigma=sigma)
            ue, f = W.transport_manufactured_2d(beta, sigma)
            prob.set_forcing([f], ue)
            prob.set_initial(None)
        else:
            prob = Problem(EHDG_SWE, 2, (n, n), periodic=(1, 1, 0), degree=p, Phi=1.0, dt=extra)
            prob.set_initial(W.gaussian_hump(W.hump_centre(0)))
        out.append(prob)
    return out


def _reset(probs, kinds):
    from paper_1601_06681_amd import workloads as W
    for prob, (kind, *_rest) in zip(probs, kinds):
        prob.set_initial(None if kind == "transport" else W.gaussian_hump(W.hump_centre(0)))


def _solve_both(kinds):
    """Steady members solved and BE members stepped through a workspace batch, then the
    same from the same initial states through a static batch.  Returns both results."""
    import torch
    from paper_1601_06681_amd.ehdg import Batch
    probs = _members(kinds)
    tr = [p for p, k in zip(probs, kinds) if k[0] == "transport"]
    sw = [p for p, k in zip(probs, kinds) if k[0] == "swe"]
    results = []
    for static in (False, True):
        _reset(probs, kinds)
        out = {}
        if tr:
            b = Batch(tr, static=static)
            out["tr"] = b.solve(1e-10, 20000)
            out["tr_u"] = [p.solution().clone() for p in tr]
            out["tr_hist"] = [p.residuals(0, it) for p, it in zip(tr, out["tr"][1])]
            b.close()
        if sw:
            b = Batch(sw, static=static)
            out["sw"] = b.step(3, 1e-10, 1000)
            out["sw_u"] = [p.solution().clone() for p in sw]
            b.close()
        results.append(out)
    torch.cuda.synchronize()
    return probs, results


def _assert_same(a, b):
    import torch
    if "tr" in a:
        assert a["tr"][1] == b["tr"][1]
        assert a["tr"][2] == b["tr"][2]
        for x, y in zip(a["tr_u"], b["tr_u"]):
            assert torch.equal(x, y)
        for x, y in zip(a["tr_hist"], b["tr_hist"]):
            np.testing.assert_array_equal(x, y)
    if "sw" in a:
        assert a["sw"][1] == b["sw"][1]
        for x, y in zip(a["sw_u"], b["sw_u"]):
            assert torch.equal(x, y)


KINDS_LARGE = [("transport", 40, 3, ((1.0, 0.5), 1.0)), ("transport", 23, 2, ((-0.7, 0.4), 0.8)),
               ("transport", 64, 4, ((0.3, -1.0), 1.5)), ("swe", 32, 3, 1e-3), ("swe", 48, 4, 5e-4)]
KINDS_SMALL = [("transport", 12, 2, ((0.6, 0.8), 1.2)), ("swe", 16, 2, 1e-3)]


def test_static_batch_matches_workspace_batch_twice():
    from paper_1601_06681_amd import ehdg as E
    probs1, (ws1, st1) = _solve_both(KINDS_LARGE)
    _assert_same(ws1, st1)
    # the first static batch (kept alive) is refused once a second one replaces its tables
    keep = E.Batch([probs1[0]], static=True)
    probs2, (ws2, st2) = _solve_both(KINDS_SMALL)
    _assert_same(ws2, st2)
    with pytest.raises(E.EhdgError) as ei:
        keep.solve(1e-10, 100)
    assert ei.value.code == E.EHDG_ERR_INVALID_ARG
    keep.close()
    for p in probs1 + probs2:
        p.close()
