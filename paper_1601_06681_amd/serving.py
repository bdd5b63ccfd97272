"""Serving independent eHDG problems on one GPU with continuous batching.

Requests arrive over time; each is one problem (set-up, a steady solve or a number of
backward-Euler steps, its solution).  The server keeps the GPU busy with one batch of
the admitted problems and changes the batch between short launches:

  * Admission.  Arrived requests are admitted in arrival order while the sum of the
    admitted problems' device workspaces stays within an HBM budget.  With `max_active`
    set, at most that many problems are in the batch and at most `lookahead` more are
    admitted ahead of them (set up, waiting to join in arrival order); max_active = 1 is
    first-in-first-out service with the next requests' set-up overlapped.
  * Set-up overlapped with the batch.  A worker thread sets up each admitted problem
    (host operator build, data sampled on the device) on a second stream; the GPU keeps
    sweeping the batch meanwhile.  An event on that stream orders the batch after the
    set-up when the problem joins.
  * Asynchronous rounds.  The batch is advanced by launches of `rounds` rounds each
    (ehdg_batch_launch); up to `depth` launches are queued ahead, so the GPU never waits
    for the host.  Each launch ends with a copy of every member's control block into a
    pinned host buffer; the server reads it when the launch's event has completed
    (ehdg_batch_poll, which never waits).
  * Retirement as members finish.  A member that a report shows finished is retired at
    once: its solution is queued into an output tensor (ehdg_batch_get_solution, valid
    while later launches are still queued, since rounds leave a finished member
    unchanged), its workspace is released, and the batch is rebuilt without it.  Its
    latency ends when that copy has completed.
A member's state lives in its own workspace, so leaving and re-forming the batch does not
change its iterates: its result is bit for bit its result alone.

The comparison is the plain FP64 first-in-first-out server, which sets up and solves one
request at a time; its latencies follow from the measured service times and the same
arrival times.
"""
import queue
import sys
import threading
import time
from collections import deque

import numpy as np

from . import ehdg as E
from . import workloads as W

CTRL_BYTES = 64  # one member's control block in a launch report


def make_problem(req):
    """The device problem of one request, with its data and initial state set (on the
    current stream)."""
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


class _SetupWorker:
    """Sets up admitted requests on its own thread and stream, in admission order."""

    def __init__(self, requests, torch):
        self.requests = requests
        self.torch = torch
        self.stream = torch.cuda.Stream()
        self.todo = queue.Queue()
        self.done = queue.Queue()
        self.thread = threading.Thread(target=self._loop, daemon=True)
        self.thread.start()

    def _loop(self):
        torch = self.torch
        while True:
            i = self.todo.get()
            if i is None:
                return
            try:
                with torch.cuda.stream(self.stream):
                    prob = make_problem(self.requests[i])
                    ev = torch.cuda.Event()
                    ev.record(self.stream)
                self.done.put((i, prob, ev, None))
            except Exception as exc:  # reported by the serving thread
                self.done.put((i, None, None, exc))

    def stop(self):
        self.todo.put(None)
        self.thread.join()


class Server:
    """Continuous batching with overlapped set-up and asynchronous launches (see the
    module docstring)."""

    def __init__(self, hbm_budget, rounds=8, tol=1e-10, max_active=None, lookahead=2, depth=2, graphs=False):
        self.budget = int(hbm_budget)
        self.rounds = int(rounds)
        self.tol = float(tol)
        self.max_active = max_active
        self.lookahead = int(lookahead)
        self.depth = int(depth)
        self.graphs = bool(graphs)

    def run(self, requests, arrivals, keep=False):
        """Serves `requests` arriving at `arrivals` (seconds from the start, ascending).
        Returns per-request latency (s) and finish time, the makespan, launch and batch
        counts, the peak admitted workspace, and the solutions if `keep`."""
        torch = E._torch()
        n = len(requests)
        need = [footprint(r) for r in requests]
        if max(need) > self.budget:
            raise ValueError("a request is larger than the HBM budget")
        cap = None if self.max_active is None else self.max_active + self.lookahead
        main = torch.cuda.Stream()
        worker = _SetupWorker(requests, torch)
        # one pinned report buffer per launch in flight, sized for every request at once
        bufs = [torch.empty(CTRL_BYTES * n, dtype=torch.uint8, pin_memory=True) for _ in range(self.depth)]
        free_bufs = list(range(self.depth))
        pending = deque(range(n))
        probs = {}                 # admitted, set up, not yet closed
        used = admitted = 0
        peak = 0
        ready = deque()            # set up, waiting to join the batch (arrival order)
        members = []               # request ids of the current batch, in batch order
        batch = None
        inflight = deque()         # (batch, members, buffer index), oldest first
        old = []                   # replaced batches: [batch, event after its last work]
        refs = {}                  # request id -> live batches that hold its handle
        retired = set()
        retiring = deque()         # (ids, outputs, event after their solution copies)
        finish = np.zeros(n)
        result = {}
        launches = batches = 0
        done_count = 0
        t0 = time.perf_counter()

        def drop_batch(b, mem):
            b.close()
            for i in mem:
                refs[i] -= 1
                if refs[i] == 0 and i in retired:
                    p = probs.pop(i)
                    p.workspace.record_stream(main)  # reuse waits for main's queued work
                    p.close()

        # the serving thread sleeps whenever it waits; a short switch interval hands it the
        # interpreter soon after the set-up thread's Python work
        switch = sys.getswitchinterval()
        sys.setswitchinterval(2e-4)
        try:
            with torch.cuda.stream(main):
                while done_count < n:
                    now = time.perf_counter() - t0
                    progress = False
                    # admission: set-up starts on the worker
                    while (pending and arrivals[pending[0]] <= now and used + need[pending[0]] <= self.budget
                           and (cap is None or admitted < cap)):
                        i = pending.popleft()
                        used += need[i]
                        admitted += 1
                        peak = max(peak, used)
                        worker.todo.put(i)
                        progress = True
                    # finished set-ups join at the next rebuild, after their set-up stream work
                    while True:
                        try:
                            i, prob, ev, exc = worker.done.get_nowait()
                        except queue.Empty:
                            break
                        if exc is not None:
                            raise exc
                        main.wait_event(ev)
                        probs[i] = prob
                        refs[i] = 0
                        ready.append(i)
                        progress = True
                    # reports of completed launches, oldest first
                    while inflight:
                        b, mem, k = inflight[0]
                        st = b.poll()
                        if st is None:
                            break
                        inflight.popleft()
                        free_bufs.append(k)
                        progress = True
                        ids, outs = [], []
                        for j, s in enumerate(st):
                            i = mem[j]
                            if s == 2:
                                raise RuntimeError(f"request {i} diverged")
                            if s == 1 and i not in retired:
                                outs.append(b.solution(j))
                                ids.append(i)
                                retired.add(i)
                                used -= need[i]
                                admitted -= 1
                        if ids:
                            ev = torch.cuda.Event()
                            ev.record(main)
                            retiring.append((ids, outs, ev))
                            for rec in old:
                                if rec[0][0] is b:
                                    rec[1] = ev
                    # results whose copies have completed
                    while retiring and retiring[0][2].query():
                        ids, outs, _ = retiring.popleft()
                        tnow = time.perf_counter() - t0
                        for i, u in zip(ids, outs):
                            finish[i] = tnow
                            if keep:
                                result[i] = u
                        done_count += len(ids)
                        progress = True
                    # replaced batches whose work has all completed
                    keep_old = []
                    for rec in old:
                        (b, mem), ev = rec
                        if any(x[0] is b for x in inflight) or (ev is not None and not ev.query()):
                            keep_old.append(rec)
                        else:
                            drop_batch(b, mem)
                    old = keep_old
                    # rebuild the batch when members left or set-up problems can join
                    live = [i for i in members if i not in retired]
                    room = len(ready) if self.max_active is None else max(0, self.max_active - len(live))
                    join = [ready.popleft() for _ in range(min(room, len(ready)))]
                    if join or len(live) != len(members):
                        live += join
                        if batch is not None:
                            ev = torch.cuda.Event()
                            ev.record(main)
                            old.append([(batch, members), ev])
                        batch, members = None, live
                        if live:
                            batch = E.Batch([probs[i] for i in live], stream=main)
                            if not self.graphs:
                                batch.set_graph(False)
                            for i in live:
                                refs[i] += 1
                            batches += 1
                    # keep up to `depth` launches queued
                    while batch is not None and free_bufs and len(inflight) < self.depth:
                        k = free_bufs.pop()
                        targets = [requests[i].get("steps", 0) for i in members]
                        batch.launch(self.rounds, self.tol, targets, bufs[k])
                        inflight.append((batch, members, k))
                        launches += 1
                        progress = True
                    if not progress:
                        wait = 1e-4                 # lets the set-up thread run
                        if not inflight and not retiring and not probs and pending:
                            wait = min(max(arrivals[pending[0]] - (time.perf_counter() - t0), wait), 1e-3)
                        time.sleep(wait)
            main.synchronize()
        finally:
            sys.setswitchinterval(switch)
            worker.stop()
        makespan = time.perf_counter() - t0
        for rec in old:
            (b, mem), _ = rec
            drop_batch(b, mem)
        if batch is not None:
            drop_batch(batch, members)
        for p in probs.values():
            p.close()
        lat = finish - np.asarray(arrivals)
        return dict(latency=lat, finish=finish, makespan=makespan, launches=launches, batches=batches,
                    peak_bytes=peak, solutions=result if keep else None)
