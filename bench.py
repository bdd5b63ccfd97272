"""Benchmark of the eHDG hot path on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--no-forms]
                [--no-3d] [--no-control] [--no-variable] [--no-batch] [--no-serving]

A step is one backward-Euler time step of the linearized shallow-water workload
(256 x 256 periodic quads, degree 4, 3 fields, 4 915 200 DOFs): build the step's
right-hand side, sweep the eHDG iteration (gather neighbour traces, apply the
condensed local operator, write new traces, FP64 residual) until the relative trace
increment is below 1e-10, recover the element solution.  K = 20 steps is the whole
workload.  The printed value is whole-job throughput: DOFs x sweeps / wall time of
the K timed steps, inputs resident in HBM.

Further sections of the same JSON line (each can be switched off): 64^3 steady
transport in FP64 and the mixed-precision forms, the same at 128^3 as a control whose
traces cannot stay in the Infinity Cache, Section 4.1 / 4.3 variable-velocity
transport (per-element operators), a batch of 512 mixed problems, and a serving run.

One JSON line on stdout; progress on stderr.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK = 8.0e12          # MI355X HBM3E, bytes/s
FP64_PEAK = 78.6e12        # MI355X FP64 vector / matrix, flop/s
BF16_PEAK = 2.5e15


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_src_sha():
    with open(os.path.join(ROOT, "paper_1601_06681_amd", "csrc", "kernels.hip"), "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def traffic_from_profiles(kernel_tag, per_launch_alg_bytes):
    """HBM bytes per launch from committed rocprofv3 --pmc summaries, if they were
    taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", f"{kernel_tag}_pmc.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("kernel_src_sha") != kernel_src_sha():
        return None
    return d.get("hbm_bytes_per_dispatch")


def swe_problem(cfg, precision=0, inner=1):
    from paper_1601_06681_amd.ehdg import EHDG_SWE, Problem
    return Problem(EHDG_SWE, 2, cfg["n"], L=cfg["L"], periodic=(1, 1, 0), degree=cfg["degree"], Phi=cfg["Phi"],
                   dt=cfg["dt"], precision=precision, inner_sweeps=inner)


def time_sweeps(torch, prob, n):
    """Average duration of one sweep launch over n back-to-back sweeps, HIP events on
    the stream the library launches on (torch's current stream)."""
    st = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    prob.iterate(2)
    torch.cuda.synchronize()
    e0.record(st)
    prob.iterate(n)
    e1.record(st)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3 / n


def host_description():
    """CPU model and the cores this process may run on (the GPU machine's host)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, len(os.sched_getaffinity(0))


def cpu_baseline_swe(cfg, fns, target_s=10.0, threads=None):
    """The oracle (numpy FP64 volume form) on whole backward-Euler steps of the same
    workload, as many as fit in about target_s seconds, with BLAS/LAPACK threads = all
    (threads None) or the given count."""
    import numpy as np
    from threadpoolctl import threadpool_info, threadpool_limits
    from oracle import ehdg as O
    from oracle.mesh import StructuredMesh
    from oracle.swe import ShallowWater
    mesh = StructuredMesh(cfg["n"], L=cfg["L"], periodic=(True, True))
    op = ShallowWater(mesh, cfg["degree"], cfg["Phi"], cfg["dt"])
    u = op.interpolate([lambda X, fn=fn: fn(X, np) for fn in fns])
    dofs = mesh.nel * 3 * op.ref.Np
    sweeps, steps = 0, 0
    with threadpool_limits(limits=threads):
        used = max([t.get("num_threads", 1) for t in threadpool_info()] + [1])
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < target_s and steps < cfg["steps"]:
            out = O.solve(op, op.load(u), u, tol=cfg["tol"], max_iter=1000)
            u = out["u"]
            sweeps += out["iters"]
            steps += 1
        dt = time.perf_counter() - t0
    model, host_cores = host_description()
    return {"value": dofs * sweeps / dt, "unit": "DOF-updates/s", "cores": int(used), "kind": "oracle",
            "sample": f"{steps} backward-Euler steps ({sweeps} sweeps) of the same 256x256 p=4 workload, "
                      f"numpy FP64 volume-form Algorithm 1, {int(used)} BLAS thread(s), {dt:.1f} s",
            "host_cores": host_cores, "cpu_model": model}


def run_swe(args, torch):
    from paper_1601_06681_amd import workloads as W
    cfg = W.SWE2D
    fns = W.gaussian_hump(W.hump_centre(cfg["seed"]))
    prob = swe_problem(cfg)
    dofs = prob.nel * prob.m * prob.Np
    log(f"[bench] swe2d {cfg['n']} p={cfg['degree']} dofs={dofs} dt={cfg['dt']}")
    # warmup
    prob.set_initial(fns)
    if args.warmup:
        prob.step(args.warmup, cfg["tol"], 1000)
    prob.set_initial(fns)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc, its = prob.step(args.steps, cfg["tol"], 1000)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sweeps = int(sum(its))
    value = dofs * sweeps / wall
    log(f"[bench] {args.steps} steps, {sweeps} sweeps, {wall * 1e3:.3f} ms, {value:.3e} DOF-updates/s")
    u64 = prob.solution()

    # roofline of the dominant kernel (the FP64 sweep)
    t_sweep = time_sweeps(torch, prob, 200)
    S, nel = prob.S, prob.nel
    alg_bytes = 3 * S * 8 * nel            # read own state, read g, write new state (neighbour reads cached)
    achieved = alg_bytes / t_sweep
    roofline = {"bound": "hbm", "achieved": achieved / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                "frac": achieved / HBM_PEAK,
                "traffic": traffic_from_profiles("swe_sweep_p4_256x256", alg_bytes),
                "kernel": "k_sweep_mfma<SweFam<5>> (FP64 matrix-core sweep, residual fused)",
                "alg_bytes_per_launch": alg_bytes, "avg_launch_us": t_sweep * 1e6}
    log(f"[bench] sweep {t_sweep * 1e6:.2f} us/launch, {achieved / 1e9:.0f} GB/s algorithmic")

    # spectral radius of the shallow-water sweep at the stated step (Bloch-wave analysis of
    # the iteration: dt (p+1)(p+2) / h, pinned against the exact symbol in the CPU tests);
    # above 1 the iteration diverges, which is why the workload runs at cfg["dt"]
    h = cfg["L"][0] / cfg["n"][0]
    rho_stated = cfg["dt_stated"] * (cfg["degree"] + 1) * (cfg["degree"] + 2) / h
    out = {
        "metric": "DOF-updates/s per eHDG iteration", "value": value, "unit": "DOF-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": wall * 1e3 / max(args.steps, 1),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": cfg["name"], "mesh": "256x256 periodic unit square", "degree": cfg["degree"],
                   "fields": 3, "dofs": dofs, "Phi": cfg["Phi"], "dt": cfg["dt"], "dt_stated": cfg["dt_stated"],
                   "rho_at_stated_dt": rho_stated, "rho_formula": "dt (p+1)(p+2) / h",
                   "be_steps": args.steps, "rel_tol": cfg["tol"], "sweeps": sweeps,
                   "iters_per_step": its},
        "roofline": roofline,
    }
    if not args.no_forms:
        # accuracy of every form against the FP64 form run to 1e-13 per step (a tightly
        # converged reference of the same discretization); the FP64 form's own error at the
        # benchmark tolerance is stated the same way
        ref = swe_problem(cfg)
        ref.set_initial(fns)
        ref.step(args.steps, 1e-13, 5000)
        u_ref = ref.solution()
        ref.close()

        def rel(u):
            return float(((u - u_ref).abs().max() / u_ref.abs().max()).item())
        out["config"]["rel_err_vs_tight_fp64"] = rel(u64)
        forms = {}
        for name, prec, inner, tol in (("fp32_refine_s4", 1, 4, cfg["tol"]), ("fp32_plain", 3, 1, 1e-6)):
            pf = swe_problem(cfg, precision=prec, inner=inner)
            pf.set_initial(fns)
            if args.warmup:
                pf.step(args.warmup, tol, 1000)
            pf.set_initial(fns)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rc, itsf = pf.step(args.steps, tol, 1000)
            torch.cuda.synchronize()
            wf = time.perf_counter() - t0
            err = rel(pf.solution())
            forms[name] = {
                "value": dofs * sum(itsf) / wf, "ms_per_step": wf * 1e3 / max(args.steps, 1), "rel_tol": tol,
                "equivalent_sweeps": int(sum(itsf)), "rel_err_vs_tight_fp64": err,
                "speedup_vs_fp64_form": wall / wf}
            log(f"[bench] {name}: {wf * 1e3:.3f} ms, err vs tight fp64 {err:.2e}")
            pf.close()
        out["forms"] = forms
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle) ...")
        cb = cpu_baseline_swe(cfg, fns)
        one = cpu_baseline_swe(cfg, fns, target_s=8.0, threads=1)
        cb["single_thread"] = {k: one[k] for k in ("value", "unit", "cores", "sample")}
        out["cpu_baseline"] = cb
        log(f"[bench] cpu baseline {cb['value']:.3e} DOF-updates/s ({cb['cores']} threads), "
            f"{one['value']:.3e} (1 thread); host {cb['host_cores']} cores, {cb['cpu_model']}")
    prob.close()
    return out


def run_transport3d(torch, args, cfg=None):
    """64^3 hexes (or cfg's mesh), degree 3, steady transport.  Time to a relative trace
    increment of 1e-8 for plain FP64, the FP32- and BF16-MFMA-correction forms with FP64
    refinement, and plain FP32; and each form's time to a solution within 1e-8 of a
    tightly converged FP64 reference (the FP64 form at an increment of 1e-13): the outer
    tolerance is tightened until the error is reached, so the speed-ups compare equal
    accuracy."""
    from paper_1601_06681_amd import workloads as W
    from paper_1601_06681_amd.ehdg import EHDG_TRANSPORT, Problem
    cfg = cfg or W.TRANSPORT3D
    ue, f = W.transport_manufactured_3d(cfg["beta"], cfg["sigma"])

    def make(precision=0, inner=1):
        prob = Problem(EHDG_TRANSPORT, 3, cfg["n"], L=cfg["L"], degree=cfg["degree"], beta=cfg["beta"],
                       sigma=cfg["sigma"], precision=precision, inner_sweeps=inner)
        prob.set_forcing([f], ue)
        return prob

    def solve_timed(prob, tol, cap=100000):
        prob.set_initial(None)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, iters, res = prob.solve(tol, cap, allow=(0, 4))
        u = prob.solution()
        torch.cuda.synchronize()
        return time.perf_counter() - t0, iters, res, u

    p64 = make()
    solve_timed(p64, cfg["tol"])                       # warm-up (kernel loading, caches)
    t64, it64, res64, u64 = solve_timed(p64, cfg["tol"])
    _, it_ref, res_ref, u_ref = solve_timed(p64, 1e-13)
    u_ref = u_ref.clone()
    dofs = p64.nel * p64.Np
    p64.set_initial(None)
    t_sweep = time_sweeps(torch, p64, 50)
    alg_bytes = 3 * p64.S * 8 * p64.nel
    flops = 2 * p64.S * p64.I * p64.nel
    ex = p64.points("nodes")
    err_exact = float(((u64[:, 0, :] - ue(ex, torch)).abs().max()).item())

    def rel(u):
        return float(((u - u_ref).abs().max() / u_ref.abs().max()).item())
    out = {"workload": cfg["name"], "dofs": dofs, "rel_tol": cfg["tol"],
           "reference": {"rel_tol": 1e-13, "sweeps": it_ref, "rel_res": res_ref},
           "fp64": {"time_to_tol_ms": t64 * 1e3, "sweeps": it64, "rel_res": res64,
                    "dof_updates_per_s": dofs * it64 / t64, "max_err_vs_manufactured": err_exact,
                    "rel_err_vs_reference": rel(u64),
                    "sweep_us": t_sweep * 1e6, "sweep_alg_bytes": alg_bytes,
                    "sweep_hbm_frac": alg_bytes / t_sweep / HBM_PEAK,
                    "sweep_fp64_frac": flops / t_sweep / FP64_PEAK},
           "roofline": {"bound": "hbm", "achieved": alg_bytes / t_sweep / 1e9, "peak": HBM_PEAK / 1e9,
                        "unit": "GB/s", "frac": alg_bytes / t_sweep / HBM_PEAK,
                        "traffic": traffic_from_profiles("transport3d_sweep_p3_64x64x64", alg_bytes)
                        if cfg is W.TRANSPORT3D else None,
                        "kernel": "k_sweep_mfma<TransportFam<3, 3, 4>> (FP64 matrix-core sweep, residual fused)",
                        "alg_bytes_per_launch": alg_bytes, "avg_launch_us": t_sweep * 1e6}}
    log(f"[bench] 3d {cfg['name']} fp64: {it64} sweeps in {t64 * 1e3:.2f} ms; sweep {t_sweep * 1e6:.1f} us "
        f"({alg_bytes / t_sweep / 1e9:.0f} GB/s, {flops / t_sweep / 1e12:.1f} TF/s); err vs reference "
        f"{rel(u64):.2e}")
    # 24 correction sweeps per FP64 refinement: of 4 to 48, the fastest to an error of 1e-8
    # for the BF16 form at 64^3 and 128^3, within 5% of the fastest (32) for the FP32 form
    forms = (("fp64", 0, 1), ("fp32_refine_s24", 1, 24), ("bf16_mfma_refine_s24", 2, 24), ("fp32_plain", 3, 1))
    equal = {}
    for name, prec, inner in forms:
        pr = p64 if prec == 0 else make(prec, inner)
        # plain FP32 cannot reach increments far below its rounding: it runs at 1e-6 (its
        # accuracy floor is stated by the error), capped at twice the FP64 sweep count
        tol_form = 1e-6 if prec == 3 else cfg["tol"]
        cap = 2 * it_ref + 100
        if prec:
            solve_timed(pr, tol_form, cap)
            t, it, res, u = solve_timed(pr, tol_form, cap)
            err = rel(u)
            out[name] = {"time_to_tol_ms": t * 1e3, "rel_tol": tol_form, "equivalent_sweeps": it, "rel_res": res,
                         "rel_err_vs_reference": err, "speedup_vs_fp64_form": t64 / t}
            log(f"[bench] 3d {cfg['name']} {name}: {t * 1e3:.2f} ms, {it} equivalent sweeps, err vs reference "
                f"{err:.2e}")
        # time to an error of at most 1e-8 against the reference
        row = None
        for tol in ((1e-6, 1e-7) if prec == 3 else (1e-8, 1e-9, 1e-10, 1e-11)):
            t, it, res, u = solve_timed(pr, tol, cap)
            err = rel(u)
            row = {"rel_tol": tol, "time_ms": t * 1e3, "equivalent_sweeps": it, "rel_err_vs_reference": err,
                   "reached": err <= 1e-8}
            if err <= 1e-8:
                break
        equal[name] = row
        log(f"[bench] 3d {cfg['name']} {name} at error <= 1e-8: tol {row['rel_tol']:.0e}, "
            f"{row['time_ms']:.2f} ms, err {row['rel_err_vs_reference']:.2e}")
        if prec:
            pr.close()
    base = equal["fp64"]["time_ms"]
    for row in equal.values():
        row["speedup_vs_fp64_form"] = base / row["time_ms"] if row["reached"] else None
    out["at_error_1e-8"] = equal
    p64.close()
    return out


# Section 4.1's velocity beta = (y, x) (div beta = 0)
VARIABLE_BETA_2D = (lambda X, xp: xp.stack([X[..., 1], X[..., 0]], -1), None)


def run_variable(torch, args):
    """Transport with a velocity field (per-element operators): Section 4.1's problem
    (beta = (y, x), 256 x 256, degree 4) and Section 4.3's (beta = (z, x, y), 16^3,
    degree 3), solved to a relative trace increment of 1e-10 from zero."""
    from paper_1601_06681_amd.ehdg import EHDG_TRANSPORT, Problem, ehdg_set_forcing
    pi = 3.141592653589793
    cases = [
        ("sec4.1 beta=(y,x) 256x256 p4", (256, 256), 4, VARIABLE_BETA_2D[0],
         lambda X, xp: xp.sin(pi * X[..., 0]) * xp.cos(pi * X[..., 1]) / pi,
         lambda X, xp: (X[..., 1] * xp.cos(pi * X[..., 0]) * xp.cos(pi * X[..., 1])
                        - X[..., 0] * xp.sin(pi * X[..., 0]) * xp.sin(pi * X[..., 1]))),
        ("sec4.3 beta=(z,x,y) 16^3 p3", (16, 16, 16), 3,
         lambda X, xp: xp.stack([X[..., 2], X[..., 0], X[..., 1]], -1),
         lambda X, xp: xp.sin(pi * X[..., 0]) * xp.cos(pi * X[..., 1]) * xp.sin(pi * X[..., 2]) / pi,
         lambda X, xp: (X[..., 2] * xp.cos(pi * X[..., 0]) * xp.cos(pi * X[..., 1]) * xp.sin(pi * X[..., 2])
                        - X[..., 0] * xp.sin(pi * X[..., 0]) * xp.sin(pi * X[..., 1]) * xp.sin(pi * X[..., 2])
                        + X[..., 1] * xp.sin(pi * X[..., 0]) * xp.cos(pi * X[..., 1]) * xp.cos(pi * X[..., 2]))),
    ]
    out = []
    for name, n, p, beta, ue, f in cases:
        t0 = time.perf_counter()
        prob = Problem(EHDG_TRANSPORT, len(n), n, degree=p, velocity=(beta, None))
        torch.cuda.synchronize()
        t_setup = time.perf_counter() - t0
        X = prob.points("quad")
        # inflow data: the exact solution at the boundary nodes (its interpolant)
        Xb = prob.boundary_points()
        ehdg_set_forcing(prob.h, f(X, torch).to(torch.float64)[:, None, :].contiguous(),
                         ue(Xb, torch).to(torch.float64).contiguous())
        res = []
        for _ in range(2):                       # the first solve warms up
            prob.set_initial(None)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            rc, iters, rr = prob.solve(1e-10, 200000)
            u = prob.solution()
            torch.cuda.synchronize()
            res.append((time.perf_counter() - t1, iters, rr, u))
        t, iters, rr, u = res[-1]
        err = float((u[:, 0, :] - ue(prob.points("nodes"), torch)).abs().max().item())
        prob.set_initial(None)
        t_sweep = time_sweeps(torch, prob, 100)
        alg = (prob.S * prob.I + 3 * prob.S) * 8 * prob.nel
        dofs = prob.nel * prob.Np
        tag = "variable_sweep_p4_256x256" if len(n) == 2 else None
        row = {"workload": name, "dofs": dofs, "setup_s": t_setup, "sweeps": iters, "rel_res": rr,
               "time_to_tol_ms": t * 1e3, "dof_updates_per_s": dofs * iters / t, "max_err_vs_exact": err,
               "roofline": {"bound": "hbm", "achieved": alg / t_sweep / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                            "frac": alg / t_sweep / HBM_PEAK,
                            "traffic": traffic_from_profiles(tag, alg) if tag else None,
                            "kernel": f"k_sweep_var<TransportFam<{len(n)}, {len(n)}, {p + 1}>> (per-element "
                                      "operators streamed, residual fused)",
                            "alg_bytes_per_launch": alg, "avg_launch_us": t_sweep * 1e6}}
        log(f"[bench] variable {name}: setup {t_setup:.2f} s, {iters} sweeps in {t * 1e3:.1f} ms, sweep "
            f"{t_sweep * 1e6:.1f} us ({alg / t_sweep / 1e9:.0f} GB/s), err {err:.2e}")
        out.append(row)
        prob.close()
    return out


def run_batch(torch, args):
    """Batched uneven solves: the batch_mix problems (seed 0) in plain FP32, with launch
    shapes from the autotuner and rounds replayed from a captured HIP graph (one sweep
    launch per family and round).  The steady transport members are solved to
    an increment of 1e-6, the shallow-water members take 5 backward-Euler steps at 1e-6.
    Compared with the same batch launched without the graph, with the persistent sweep
    launch (one per round for every member) instead of the per-family launches, and with
    the first problems of each kind solved one by one.  Members the library refuses (degree-1 transport with both
    velocity components non-zero) are counted and left out."""
    import tempfile
    from paper_1601_06681_amd import autotune as A
    from paper_1601_06681_amd import workloads as W
    from paper_1601_06681_amd.ehdg import EHDG_FP32, EHDG_SWE, EHDG_TRANSPORT, Batch, Problem
    drawn = W.batch_mix(args.batch_size, 0)
    specs = [sp for sp in drawn if not (sp["kind"] == "transport" and sp["degree"] == 1
                                        and sp["beta"][0] != 0.0 and sp["beta"][1] != 0.0)]
    hump = W.gaussian_hump(W.hump_centre(0))
    tol = 1e-6

    def make(sp):
        if sp["kind"] == "transport":
            prob = Problem(EHDG_TRANSPORT, 2, (sp["n"], sp["n"]), L=(1.0, 1.0), degree=sp["degree"], beta=sp["beta"],
                           sigma=sp["sigma"], precision=EHDG_FP32)
            ue, f = W.transport_manufactured_2d(sp["beta"], sp["sigma"])
            prob.set_forcing([f], ue)
            prob.set_initial(None)
        else:
            prob = Problem(EHDG_SWE, 2, (sp["n"], sp["n"]), L=(1.0, 1.0), periodic=(1, 1, 0), degree=sp["degree"],
                           Phi=1.0, dt=sp["dt"], precision=EHDG_FP32)
            prob.set_initial(hump)
        return prob

    # launch shapes: the autotuner in batch mode (a round of 8 problems of 128 x 128 of the
    # family through the batched sweep) for each family in the batch
    t0 = time.perf_counter()
    cache = os.path.join(tempfile.mkdtemp(prefix="ehdg_tune_"), "tune.json")
    tuned = {}
    for kind, p in sorted({(sp["kind"], sp["degree"]) for sp in specs}):
        rep = dict(kind=kind, n=128, degree=p, beta=(0.96, 0.28), sigma=1.0,
                   dt=0.25 / 128 / ((p + 1) * (p + 2)), steps=5)
        pde = EHDG_TRANSPORT if kind == "transport" else EHDG_SWE
        out = A.tune(lambda rep=rep: make(rep), pde, 2, p, EHDG_FP32, sweeps=30, path=cache, batch=8)
        tuned[f"{kind}_p{p}"] = {k: out["best"][k] for k in ("tiles_per_group", "reverse_order", "sweep_us")}
    t_tune = time.perf_counter() - t0
    log(f"[bench] batch: autotuned {len(tuned)} families in {t_tune:.1f} s")
    t0 = time.perf_counter()
    probs = [make(sp) for sp in specs]
    torch.cuda.synchronize()
    log(f"[bench] batch: {len(probs)} problems set up in {time.perf_counter() - t0:.1f} s")
    tr = [i for i, sp in enumerate(specs) if sp["kind"] == "transport"]
    sw = [i for i, sp in enumerate(specs) if sp["kind"] == "swe"]
    dofs = [p.nel * p.m * p.Np for p in probs]
    out = {"workload": f"batch_mix_{len(drawn)}", "problems": len(specs), "transport": len(tr), "swe": len(sw),
           "left_out_degree1_two_axis_transport": len(drawn) - len(specs), "precision": "fp32", "rel_tol": tol,
           "elements": int(sum(p.nel for p in probs)), "dofs": int(sum(dofs)), "autotune_s": t_tune,
           "tuned_shapes": tuned}

    def timed(fn):
        torch.cuda.synchronize()
        t = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return r, time.perf_counter() - t

    def reset(idx):
        for i in idx:
            probs[i].set_initial(None if specs[i]["kind"] == "transport" else hump)

    bt = Batch([probs[i] for i in tr])
    bs = Batch([probs[i] for i in sw])
    for graph, persist in ((True, False), (False, False), (True, True)):
        bt.set_graph(graph)
        bs.set_graph(graph)
        bt.set_persistent(persist)
        bs.set_persistent(persist)
        bt.solve(tol, 100000)                  # warm-up: kernel loading, graph capture, predictions
        bs.step(1, tol, 1000)
        reset(tr)
        reset(sw)
        (rc_t, its_t, _), wall_t = timed(lambda: bt.solve(tol, 100000))
        (rc_s, its_s), wall_s = timed(lambda: bs.step(5, tol, 1000))
        upd_t = sum(dofs[i] * its_t[k] for k, i in enumerate(tr))
        upd_s = sum(dofs[i] * sum(its_s[k]) for k, i in enumerate(sw))
        row = {"transport_solve_ms": wall_t * 1e3, "transport_sweeps_total": int(sum(its_t)),
               "swe_5_steps_ms": wall_s * 1e3, "swe_sweeps_total": int(sum(sum(v) for v in its_s)),
               "dof_updates_per_s": (upd_t + upd_s) / (wall_t + wall_s)}
        name = ("batched_graph" if graph else "batched_eager") if not persist else "persistent_graph"
        out[name] = row
        log(f"[bench] batch ({name}): transport {wall_t * 1e3:.1f} ms, swe "
            f"{wall_s * 1e3:.1f} ms, {row['dof_updates_per_s']:.3e} DOF-updates/s")
    # the same problems one after another (the first args.batch_solo of each kind)
    k = args.batch_solo
    reset(tr[:k])
    reset(sw[:k])
    upd, wall = 0, 0.0
    for i in tr[:k]:
        (rc, it, _), w = timed(lambda: probs[i].solve(tol, 100000))
        upd += dofs[i] * it
        wall += w
    for i in sw[:k]:
        (rc, its), w = timed(lambda: probs[i].step(5, tol, 1000))
        upd += dofs[i] * sum(its)
        wall += w
    out["one_by_one_first"] = {"problems_per_kind": k, "dof_updates_per_s": upd / wall}
    log(f"[bench] batch: one by one (first {k} of each kind) {upd / wall:.3e} DOF-updates/s")
    bt.close()
    bs.close()
    for p in probs:
        p.close()
    from paper_1601_06681_amd.ehdg import ehdg_tune_clear
    ehdg_tune_clear()
    return out


def run_serving(torch, args):
    """Serving with continuous batching: the serving_requests stream (seed 0) arriving as a
    Poisson process at 0.8 x the capacity of the plain FP64 first-in-first-out server
    (measured: every request set up and solved alone, one after another), served by the
    continuous-batching server within an HBM budget.  Latency percentiles and throughput
    of both."""
    import numpy as np
    from paper_1601_06681_amd import serving as S
    from paper_1601_06681_amd import workloads as W
    reqs = W.serving_requests(args.serve_count, 0)
    for kind in ("euler", "transport"):         # warm-up: kernel loading
        S.solve_alone(next(r for r in reqs if r["kind"] == kind), 1e-10)
    t = time.perf_counter()
    service = np.array([S.solve_alone(r, 1e-10)[0] for r in reqs])
    log(f"[bench] serving: {len(reqs)} requests alone in {time.perf_counter() - t:.1f} s, "
        f"mean service {service.mean() * 1e3:.2f} ms")
    rate = 0.8 / service.mean()
    arrivals = np.cumsum([r["gap"] for r in reqs]) / rate
    fifo_lat, fifo_end = S.fifo_latencies(arrivals, service)
    server = S.Server(args.serve_hbm_gb * 2 ** 30, rounds=args.serve_rounds, depth=args.serve_depth,
                      max_active=args.serve_max_active or None, lookahead=args.serve_lookahead)
    out = server.run(reqs, arrivals)
    lat = out["latency"]
    log(f"[bench] serving: batched run done ({out['makespan']:.1f} s)")
    # capacity: everything queued at once (the FIFO capacity is 1 / mean service time)
    sat = server.run(reqs, np.zeros(len(reqs)))
    log(f"[bench] serving: saturated run done ({sat['makespan']:.1f} s)")
    # one member at a time: first in, first out, with the next requests' set-up overlapped
    one = S.Server(args.serve_hbm_gb * 2 ** 30, rounds=args.serve_rounds, depth=2, max_active=1,
                   lookahead=args.serve_lookahead).run(reqs, arrivals)

    def pct(x):
        return {"p50_ms": float(np.percentile(x, 50) * 1e3), "p99_ms": float(np.percentile(x, 99) * 1e3)}
    res = {"workload": f"serving_{len(reqs)}", "requests": len(reqs),
           "euler": sum(r["kind"] == "euler" for r in reqs), "arrival_rate_per_s": rate,
           "fifo_fp64": {**pct(fifo_lat), "throughput_per_s": len(reqs) / fifo_end,
                         "mean_service_ms": float(service.mean() * 1e3)},
           "continuous_batching": {**pct(lat), "throughput_per_s": len(reqs) / out["makespan"],
                                   "launches": out["launches"], "batches": out["batches"],
                                   "peak_workspace_gb": out["peak_bytes"] / 2 ** 30,
                                   "hbm_budget_gb": args.serve_hbm_gb, "rounds_per_launch": args.serve_rounds,
                                   "launches_queued_ahead": args.serve_depth,
                                   "max_active": args.serve_max_active or None,
                                   "lookahead": args.serve_lookahead},
           "one_member_overlapped_setup": {**pct(one["latency"]), "throughput_per_s": len(reqs) / one["makespan"],
                                           "launches": one["launches"], "rounds_per_launch": args.serve_rounds,
                                           "launches_queued_ahead": 2},
           "capacity_per_s": {"fifo_fp64": float(1.0 / service.mean()),
                              "continuous_batching": len(reqs) / sat["makespan"]}}
    log(f"[bench] serving: FIFO p50 {res['fifo_fp64']['p50_ms']:.1f} ms p99 {res['fifo_fp64']['p99_ms']:.1f} ms; "
        f"batched p50 {res['continuous_batching']['p50_ms']:.1f} ms p99 {res['continuous_batching']['p99_ms']:.1f} ms; "
        f"capacity {res['capacity_per_s']['fifo_fp64']:.1f} vs {res['capacity_per_s']['continuous_batching']:.1f} /s; "
        f"one member p50 {res['one_member_overlapped_setup']['p50_ms']:.1f} ms "
        f"p99 {res['one_member_overlapped_setup']['p99_ms']:.1f} ms")
    return res


def run_counter_sample(torch, args):
    """For rocprofv3 --pmc runs: a plain device-to-device copy of 256 MiB (the
    calibration kernel: it must fetch and write exactly 256 MiB each), then 20 FP64
    sweeps and 2 backward-Euler steps of the shallow-water workload, unless --no-3d
    5 sweeps of the 64^3 transport workload, and unless --no-variable 20 sweeps of
    Section 4.1's variable-velocity problem at 256 x 256, degree 4."""
    from paper_1601_06681_amd import workloads as W
    n = 256 * 1024 * 1024 // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    del a, b
    cfg = W.SWE2D
    prob = swe_problem(cfg)
    prob.set_initial(W.gaussian_hump(W.hump_centre(cfg["seed"])))
    torch.cuda.synchronize()
    prob.iterate(20)
    torch.cuda.synchronize()
    prob.set_initial(W.gaussian_hump(W.hump_centre(cfg["seed"])))
    prob.step(2, cfg["tol"], 1000)
    torch.cuda.synchronize()
    prob.close()
    if not args.no_3d:
        from paper_1601_06681_amd.ehdg import EHDG_TRANSPORT, Problem
        c3 = W.TRANSPORT3D
        p3 = Problem(EHDG_TRANSPORT, 3, c3["n"], L=c3["L"], degree=c3["degree"], beta=c3["beta"], sigma=c3["sigma"])
        p3.iterate(5)
        torch.cuda.synchronize()
        p3.close()
    if not args.no_variable:
        from paper_1601_06681_amd.ehdg import EHDG_TRANSPORT, Problem
        pv = Problem(EHDG_TRANSPORT, 2, (256, 256), degree=4, velocity=VARIABLE_BETA_2D)
        pv.set_initial(None)
        pv.iterate(20)
        torch.cuda.synchronize()
        pv.close()
    log("[bench] counter sample done")


PMC_KERNELS = {  # summary tag -> kernel name prefix (as rocprofv3 prints it)
    "swe_sweep_p4_256x256": "void ehdg::k_sweep_mfma<ehdg::SweFam<5>, true>",
    "swe_step_p4_256x256": "void ehdg::k_step_lds<ehdg::SweFam<5>, double>",
    "transport3d_sweep_p3_64x64x64": "void ehdg::k_sweep_mfma<ehdg::TransportFam<3, 3, 4>, true>",
    "variable_sweep_p4_256x256": "void ehdg::k_sweep_var<ehdg::TransportFam<2, 2, 5> >",
}


def summarize_pmc(fetch_dir, write_dir):
    """Writes profiles/<tag>_pmc.json from two rocprofv3 --pmc runs of --counter-sample
    (FETCH_SIZE, then WRITE_SIZE).  Each counter is scaled by what it reads for the
    256 MiB device-to-device copy in the same run (which moves exactly 256 MiB each way)."""
    import csv
    import statistics

    def load(d, counter):
        rows = list(csv.DictReader(open(os.path.join(d, "run_counter_collection.csv"))))
        out = {}
        for r in rows:
            if r["Counter_Name"] == counter:
                out.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
        return out

    fetch, write = load(fetch_dir, "FETCH_SIZE"), load(write_dir, "WRITE_SIZE")
    copy_kib = 256 * 1024.0
    f_copy = max(v for k, vs in fetch.items() if k.startswith("__amd_rocclr_copyBuffer") for v in vs)
    w_copy = max(v for k, vs in write.items() if k.startswith("__amd_rocclr_copyBuffer") for v in vs)
    ff, fw = copy_kib / f_copy, copy_kib / w_copy
    sha = kernel_src_sha()
    for tag, prefix in PMC_KERNELS.items():
        fk = [v for k, vs in fetch.items() if k.startswith(prefix) for v in vs]
        wk = [v for k, vs in write.items() if k.startswith(prefix) for v in vs]
        if not fk or not wk:
            continue
        fm, wm = statistics.median(fk), statistics.median(wk)
        d = {"kernel": prefix, "kernel_src_sha": sha, "dispatches": [len(fk), len(wk)],
             "fetch_kib_per_dispatch_raw": fm, "write_kib_per_dispatch_raw": wm,
             "copy_calibration": {"copy_bytes": 256 * 1024 * 1024, "fetch_kib_raw": f_copy, "write_kib_raw": w_copy,
                                  "fetch_factor": ff, "write_factor": fw},
             "hbm_bytes_per_dispatch": (fm * ff + wm * fw) * 1024.0,
             "commands": ["rocprofv3 --pmc FETCH_SIZE --output-format csv -d <fetch_dir> -o run -- "
                          "python3 bench.py --counter-sample",
                          "rocprofv3 --pmc WRITE_SIZE --output-format csv -d <write_dir> -o run -- "
                          "python3 bench.py --counter-sample",
                          "python bench.py --summarize-pmc <fetch_dir> <write_dir>"]}
        path = os.path.join(ROOT, "profiles", f"{tag}_pmc.json")
        with open(path, "w") as fh:
            json.dump(d, fh, indent=1)
        log(f"[pmc] {tag}: {d['hbm_bytes_per_dispatch'] / 1e6:.2f} MB per dispatch -> {path}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="swe2d")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true")
    ap.add_argument("--no-3d", action="store_true")
    ap.add_argument("--no-control", action="store_true",
                    help="skip the 128^3 transport control (traces far larger than the Infinity Cache)")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-variable", action="store_true")
    ap.add_argument("--batch-size", type=int, default=512)
    ap.add_argument("--batch-solo", type=int, default=16,
                    help="problems of each kind timed one by one for the comparison")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serve-count", type=int, default=2000)
    ap.add_argument("--serve-hbm-gb", type=float, default=64.0)
    ap.add_argument("--serve-rounds", type=int, default=16, help="rounds per launch")
    ap.add_argument("--serve-depth", type=int, default=3, help="launches queued ahead")
    ap.add_argument("--serve-max-active", type=int, default=2, help="batch members at most (0: no limit)")
    ap.add_argument("--serve-lookahead", type=int, default=2, help="requests set up ahead of the batch")
    ap.add_argument("--counter-sample", action="store_true",
                    help="only the copy-calibration kernel and a few sweeps, for rocprofv3 --pmc")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write profiles/*_pmc.json from two --pmc runs of --counter-sample (no GPU needed)")
    args = ap.parse_args()
    if args.summarize_pmc:
        summarize_pmc(*args.summarize_pmc)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only: the eHDG sweep of one mesh is measured "
                                   "on a single MI355X (multi-GPU sharding is a design, not a measured path)"}))
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    torch.cuda.init()
    if args.workload != "swe2d":
        print(json.dumps({"error": f"unknown workload {args.workload}"}))
        sys.exit(2)
    if args.counter_sample:
        run_counter_sample(torch, args)
        return
    out = run_swe(args, torch)
    if not args.no_3d:
        out["transport3d"] = run_transport3d(torch, args)
        # the 64^3 transport sweep (the largest single-GPU workload of the hot path) as a
        # second roofline figure beside the headline's
        out["roofline_transport3d"] = out["transport3d"]["roofline"]
    if not args.no_control:
        from paper_1601_06681_amd import workloads as W
        out["transport3d_control"] = run_transport3d(torch, args, W.TRANSPORT3D_CONTROL)
    if not args.no_variable:
        out["variable_velocity"] = run_variable(torch, args)
    if not args.no_batch:
        out["batch"] = run_batch(torch, args)
    if not args.no_serving:
        out["serving"] = run_serving(torch, args)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
