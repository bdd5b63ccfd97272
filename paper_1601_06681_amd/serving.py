"""Serving independent eHDG problems on one GPU with continuous batching.

Requests arrive over time.  Every tick the server:
  1. admits the requests that have arrived, in arrival order, while the sum of the
     admitted members' device workspaces stays within an HBM budget (a request that
     does not fit waits; its problem is set up on admission);
  2. rebuilds the batch if its membership changed (a host-side table, one small upload)
     and advances every member by a fixed number of rounds with ehdg_batch_advance
     (one launch per operator family per round: all members progress together);
  3. retires the members that finished: their solution is read and their workspace is
     released.
A member's state lives in its own workspace, so leaving and re-forming the batch does
not change its iterates: its result is bit for bit the result of solving it alone.

The comparison is the plain FP64 first-in-first-out server, which sets up and solves one
request at a time; its latencies follow from the measured service times and the same
arrival times.
"""
import time
from collections import deque

import numpy as np

from . import ehdg as E
from . import workloads as W


def make_problem(req):
    """The device problem of one request, with its data and initial state set."""
    if req["kind"] == "euler":
        prob = E.Problem(E.EHDG_EULER, 2, (req["n"], req["n"]), L=(1.0, 1.0), periodic=(1, 1, 0),
                         degree=req["degree"], dt=req["dt"], U0=W.EULER_U0, c0=W.EULER_C0, rho0=1.0)
        prob.set_initial(W.euler_pulse())
    else:
        prob = E.Problem(E.EHDG_TRANSPORT, 3, (req["n"],) * 3, L=(1.0, 1.0, 1.0), degree=req["degree"],
                         beta=req["beta"], sigma=req["sigma"])
        ue, f = W.transport_manufactured_3d(req["beta"], req["sigma"])
        prob.set_forcing([f], ue)
        prob.set_initial(None)
    return prob


def footprint(req):
    """Device bytes the request's problem occupies (its workspace)."""
    if req["kind"] == "euler":
        d = E.make_desc(E.EHDG_EULER, 2, (req["n"], req["n"]), periodic=(1, 1, 0), degree=req["degree"],
                        dt=req["dt"], U0=W.EULER_U0, c0=W.EULER_C0)
    else:
        d = E.make_desc(E.EHDG_TRANSPORT, 3, (req["n"],) * 3, degree=req["degree"], beta=req["beta"],
                        sigma=req["sigma"])
    return E.ehdg_workspace_bytes(d)


def solve_alone(req, tol, keep=False):
    """Plain FP64, one request at a time: (service seconds, iterations, solution or None)."""
    torch = E._torch()
    torch.cuda.synchronize()
    t = time.perf_counter()
    prob = make_problem(req)
    if req["kind"] == "euler":
        rc, its = prob.step(req["steps"], tol, 10000)
        iters = int(sum(its))
    else:
        rc, iters, _ = prob.solve(tol, 100000)
    u = prob.solution()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    out = u if keep else None
    prob.close()
    return dt, iters, out


def fifo_latencies(arrivals, service):
    """Latencies of a one-at-a-time first-in-first-out server."""
    end, lat = 0.0, []
    for a, s in zip(arrivals, service):
        start = max(a, end)
        end = start + s
        lat.append(end - a)
    return np.array(lat), end


class Server:
    """Continuous batching over ehdg_batch_advance (see the module docstring)."""

    def __init__(self, hbm_budget, rounds=8, tol=1e-10):
        self.budget = int(hbm_budget)
        self.rounds = int(rounds)
        self.tol = float(tol)

    def run(self, requests, arrivals, keep=False):
        """Serves `requests` arriving at `arrivals` (seconds from the start, ascending).
        Returns per-request latency (s) and finish time, the makespan, tick and batch
        counts, and the solutions if `keep`."""
        torch = E._torch()
        n = len(requests)
        need = [footprint(r) for r in requests]
        if max(need) > self.budget:
            raise ValueError("a request is larger than the HBM budget")
        pending = deque(range(n))
        active, probs, targets = [], {}, {}
        used = 0
        finish = np.zeros(n)
        result = {}
        ticks = batches = 0
        peak = 0
        batch, members = None, None
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        while pending or active:
            now = time.perf_counter() - t0
            while pending and arrivals[pending[0]] <= now and used + need[pending[0]] <= self.budget:
                i = pending.popleft()
                probs[i] = make_problem(requests[i])
                targets[i] = requests[i].get("steps", 0)
                used += need[i]
                peak = max(peak, used)
                active.append(i)
            if not active:
                wait = arrivals[pending[0]] - (time.perf_counter() - t0)
                if wait > 0:
                    time.sleep(wait)
                continue
            if members != active:
                if batch is not None:
                    batch.close()
                batch = E.Batch([probs[i] for i in active])
                members = list(active)
                batches += 1
            state = batch.advance(self.rounds, self.tol, [targets[i] for i in active])
            ticks += 1
            if 2 in state:
                bad = [active[k] for k, s in enumerate(state) if s == 2]
                raise RuntimeError(f"requests {bad} diverged")
            done = [active[k] for k, s in enumerate(state) if s == 1]
            if done:
                for i in done:
                    u = probs[i].solution()
                    if keep:
                        result[i] = u
                for i in done:
                    probs[i].close()
                    del probs[i]
                    used -= need[i]
                torch.cuda.synchronize()
                tnow = time.perf_counter() - t0
                for i in done:
                    finish[i] = tnow
                active = [i for i in active if i not in done]
        if batch is not None:
            batch.close()
        makespan = time.perf_counter() - t0
        lat = finish - np.asarray(arrivals)
        return dict(latency=lat, finish=finish, makespan=makespan, ticks=ticks, batches=batches, peak_bytes=peak,
                    solutions=result if keep else None)
