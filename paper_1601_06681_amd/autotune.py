"""Launch-shape autotuner for the plain eHDG sweeps (FP64 and FP32).

A sweep applies the condensed local operator to tiles of 16 elements, and a launch gives
each workgroup a contiguous range of tiles.  How many tiles per workgroup (and so how many
workgroups, in how many rounds) and in which order the workgroups take their ranges decide
how well the launch hides load latency and how neighbour reads share the L2 caches.  The
arithmetic of every element is the same in any shape, so the iterates do not change.  For
a problem family (pde, dim, degree, precision) the tuner:
  * times the plain sweep of a representative problem (or a round of a batch of such
    problems, for batched use) with HIP events, for each candidate shape (the default of
    one round of resident workgroups, fixed tile counts, and both workgroup orders);
  * keeps the fastest and registers it with the library (ehdg_tune_set), so that problems
    of that family set up afterwards in this process use it;
  * caches the result in a JSON file keyed by the GPU architecture and the family.
load() applies a cache.

Cache file: $EHDG_TUNE_CACHE, else ~/.cache/ehdg/tune.json.
"""
import json
import os

from . import ehdg as E

DEFAULT_CANDIDATES = ((0, 0), (0, 1), (4, 0), (8, 0), (16, 0), (32, 0), (64, 0))
BATCH_CANDIDATES = ((0, 0), (8, 0), (16, 0), (32, 0), (64, 0), (32, 1))


def cache_path(path=None):
    if path:
        return path
    return os.environ.get("EHDG_TUNE_CACHE") or os.path.join(os.path.expanduser("~"), ".cache", "ehdg", "tune.json")


def arch(device=0):
    import torch
    props = torch.cuda.get_device_properties(device)
    return getattr(props, "gcnArchName", None) or props.name


def family_key(pde, dim, degree, precision):
    return f"pde{int(pde)}-dim{int(dim)}-p{int(degree)}-prec{int(precision)}"


def _read(path):
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def load(path=None, device=0):
    """Registers every cached shape of this GPU architecture; returns them by family key."""
    data = _read(cache_path(path)).get(arch(device), {})
    for key, row in data.items():
        E.ehdg_tune_set(row["pde"], row["dim"], row["degree"], row["precision"], row["tiles_per_group"],
                        row["reverse_order"])
    return data


def time_sweeps(prob, sweeps):
    """Average time of one plain sweep over `sweeps` back-to-back sweeps (HIP events on the
    stream the library launches on)."""
    import torch
    st = torch.cuda.current_stream()
    prob.iterate(3)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(st)
    prob.iterate(sweeps)
    e1.record(st)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3 / sweeps


def time_batch_rounds(probs, rounds):
    """Average time of one round (a sweep of every member) of a batch of `probs`."""
    import torch
    st = torch.cuda.current_stream()
    batch = E.Batch(probs)
    allow = (E.EHDG_OK, E.EHDG_ERR_NOT_CONVERGED)
    batch.solve(0.0, 3, allow=allow)            # graph capture, kernel loading
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(st)
    batch.solve(0.0, rounds, allow=allow)       # tolerance 0: exactly `rounds` rounds
    e1.record(st)
    torch.cuda.synchronize()
    batch.close()
    return e0.elapsed_time(e1) / 1e3 / rounds


def tune(make_problem, pde, dim, degree, precision, sweeps=100, candidates=None, path=None, save=True, device=0,
         batch=1):
    """Times the plain sweep under each candidate shape (tiles per workgroup, reversed
    order) and registers the fastest for the family.  make_problem must set up a new
    problem of that family (it is called after each candidate is registered).  batch = 1:
    the sweep of one problem alone; batch > 1: a round of a batch of that many problems
    (the batched sweep, where more tiles per workgroup amortize each table entry's fixed
    cost).  Returns {"best": {...}, "timings": [...]}; saves it in the cache
    when save is true."""
    if candidates is None:
        candidates = BATCH_CANDIDATES if batch > 1 else DEFAULT_CANDIDATES
    timings = []
    for tpg, rev in candidates:
        E.ehdg_tune_set(pde, dim, degree, precision, tpg, rev)
        probs = [make_problem() for _ in range(max(1, batch))]
        eff_tpg, groups, eff_rev = E.ehdg_launch_shape(probs[0].h)
        t = time_sweeps(probs[0], sweeps) if batch <= 1 else time_batch_rounds(probs, sweeps)
        for prob in probs:
            prob.close()
        timings.append({"tiles_per_group": int(tpg), "reverse_order": int(rev), "effective_tiles_per_group": eff_tpg,
                        "groups": groups, "sweep_us": t * 1e6})
    best = min(timings, key=lambda r: r["sweep_us"])
    E.ehdg_tune_set(pde, dim, degree, precision, best["tiles_per_group"], best["reverse_order"])
    row = {"pde": int(pde), "dim": int(dim), "degree": int(degree), "precision": int(precision),
           "tiles_per_group": best["tiles_per_group"], "reverse_order": best["reverse_order"],
           "sweep_us": best["sweep_us"], "context": "batch" if batch > 1 else "solo"}
    if save:
        p = cache_path(path)
        data = _read(p)
        data.setdefault(arch(device), {})[family_key(pde, dim, degree, precision)] = row
        os.makedirs(os.path.dirname(os.path.abspath(p)), exist_ok=True)
        tmp = p + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(data, fh, indent=1)
        os.replace(tmp, p)
    return {"best": row, "timings": timings}
