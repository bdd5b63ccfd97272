"""Python binding of the eHDG C ABI (include/ehdg.h): argument marshalling only.

Every function below has the name of the C entry point it calls.  Device memory
and streams come from PyTorch (ROCm); all computation happens in libehdg.so.
`Problem` bundles a handle with its workspace tensor and samples closed-form data
at the library's own reference points.
"""
import ctypes

import numpy as np

from . import _lib
from ._lib import (EHDG_BF16_REFINE, EHDG_ERR_DIVERGED, EHDG_ERR_HIP, EHDG_ERR_INVALID_ARG, EHDG_ERR_NOT_CONVERGED,
                   EHDG_ERR_UNSUPPORTED, EHDG_ERR_WORKSPACE_TOO_SMALL, EHDG_FP32, EHDG_FP32_REFINE, EHDG_FP64, EHDG_EULER, EHDG_OK,
                   EHDG_SWE, EHDG_TRANSPORT, ehdg_desc)

__all__ = [
    "EhdgError", "Problem", "Batch", "make_desc", *_lib.EXPORTED,
    "EHDG_TRANSPORT", "EHDG_SWE", "EHDG_EULER", "EHDG_FP64", "EHDG_FP32_REFINE", "EHDG_BF16_REFINE", "EHDG_FP32",
]


class EhdgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"ehdg error {code}: {msg}")
        self.code = code


def _torch():
    import torch
    return torch


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _check(rc, h=None, ok=(EHDG_OK,)):
    if rc in ok:
        return rc
    lib = _lib.load()
    msg = lib.ehdg_error_string(rc).decode()
    if h is not None:
        last = lib.ehdg_last_error(h).decode()
        if last:
            msg += f" ({last})"
    raise EhdgError(rc, msg)


def _stream_ptr(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def make_desc(pde, dim, n, L=(1.0, 1.0, 1.0), periodic=(0, 0, 0), degree=1, beta=(0.0, 0.0, 0.0), sigma=0.0,
              Phi=1.0, dt=0.0, precision=EHDG_FP64, inner_sweeps=1, U0=(0.0, 0.0), c0=1.0, rho0=1.0):
    d = ehdg_desc()
    d.pde, d.dim, d.degree = int(pde), int(dim), int(degree)
    for a in range(3):
        d.n[a] = int(n[a]) if a < len(n) else 1
        d.L[a] = float(L[a]) if a < len(L) else 1.0
        d.periodic[a] = int(periodic[a]) if a < len(periodic) else 0
        d.beta[a] = float(beta[a]) if a < len(beta) else 0.0
    d.sigma, d.Phi, d.dt = float(sigma), float(Phi), float(dt)
    d.U0[0], d.U0[1] = float(U0[0]), float(U0[1])
    d.c0, d.rho0 = float(c0), float(rho0)
    d.precision, d.inner_sweeps = int(precision), int(inner_sweeps)
    return d


# ---------------------------------------------------------------------------- C ABI
def ehdg_reference_points(degree):
    lib = _lib.load()
    x = np.zeros(degree + 1)
    q = np.zeros(degree + 2)
    w = np.zeros(degree + 2)
    _check(lib.ehdg_reference_points(degree, x.ctypes.data_as(ctypes.c_void_p), q.ctypes.data_as(ctypes.c_void_p),
                                     w.ctypes.data_as(ctypes.c_void_p)))
    return x, q, w


def ehdg_workspace_bytes(desc):
    lib = _lib.load()
    out = ctypes.c_size_t(0)
    _check(lib.ehdg_workspace_bytes(ctypes.byref(desc), ctypes.byref(out)))
    return out.value


def ehdg_setup(desc, workspace, stream=None):
    lib = _lib.load()
    h = ctypes.c_void_p()
    _check(lib.ehdg_setup(ctypes.byref(desc), _ptr(workspace), workspace.numel() * workspace.element_size(),
                          _stream_ptr(stream), ctypes.byref(h)))
    return h


def ehdg_variable_workspace_bytes(desc):
    lib = _lib.load()
    out = ctypes.c_size_t(0)
    _check(lib.ehdg_variable_workspace_bytes(ctypes.byref(desc), ctypes.byref(out)))
    return out.value


def _host_f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def ehdg_setup_variable(desc, beta_q, div_beta_q, beta_face, workspace, stream=None):
    """beta_q, div_beta_q (or None), beta_face: host arrays in the C ABI's layouts."""
    lib = _lib.load()
    bq, dq, bf = _host_f64(beta_q), _host_f64(div_beta_q), _host_f64(beta_face)
    vp = lambda a: None if a is None else a.ctypes.data_as(ctypes.c_void_p)
    h = ctypes.c_void_p()
    _check(lib.ehdg_setup_variable(ctypes.byref(desc), vp(bq), vp(dq), vp(bf), _ptr(workspace),
                                   workspace.numel() * workspace.element_size(), _stream_ptr(stream),
                                   ctypes.byref(h)))
    return h


def ehdg_set_forcing(h, forcing_q=None, bc=None):
    _check(_lib.load().ehdg_set_forcing(h, _ptr(forcing_q), _ptr(bc)), h)


def ehdg_set_initial(h, u0=None):
    _check(_lib.load().ehdg_set_initial(h, _ptr(u0)), h)


def ehdg_iterate(h, n_iters):
    _check(_lib.load().ehdg_iterate(h, int(n_iters)), h)


def ehdg_solve(h, rel_tol, max_iters, allow=(EHDG_OK,)):
    it = ctypes.c_int32(0)
    res = ctypes.c_double(0.0)
    rc = _lib.load().ehdg_solve(h, float(rel_tol), int(max_iters), ctypes.byref(it), ctypes.byref(res))
    _check(rc, h, ok=allow)
    return rc, it.value, res.value


def ehdg_step(h, n_steps, rel_tol, max_iters_per_step, allow=(EHDG_OK,)):
    its = np.zeros(max(n_steps, 1), dtype=np.int32)
    rc = _lib.load().ehdg_step(h, int(n_steps), float(rel_tol), int(max_iters_per_step),
                               its.ctypes.data_as(ctypes.c_void_p))
    _check(rc, h, ok=allow)
    return rc, its[:n_steps].tolist()


def ehdg_get_solution(h, out):
    _check(_lib.load().ehdg_get_solution(h, _ptr(out)), h)


def ehdg_get_residuals(h, first, count):
    out = np.zeros(max(count, 1))
    _check(_lib.load().ehdg_get_residuals(h, int(first), int(count), out.ctypes.data_as(ctypes.c_void_p)), h)
    return out[:count]


def ehdg_sizes(h):
    n_el = ctypes.c_int64(0)
    vals = [ctypes.c_int32(0) for _ in range(5)]
    _check(_lib.load().ehdg_sizes(h, ctypes.byref(n_el), *[ctypes.byref(v) for v in vals]), h)
    m, n_p, s, i, iters = (v.value for v in vals)
    return dict(n_el=n_el.value, m=m, n_p=n_p, S=s, I=i, iters=iters)


def ehdg_state_bytes(h):
    out = ctypes.c_size_t(0)
    _check(_lib.load().ehdg_state_bytes(h, ctypes.byref(out)), h)
    return out.value


def ehdg_get_state(h, dst):
    _check(_lib.load().ehdg_get_state(h, _ptr(dst), dst.numel() * dst.element_size()), h)


def ehdg_set_state(h, src):
    _check(_lib.load().ehdg_set_state(h, _ptr(src), src.numel() * src.element_size()), h)


def ehdg_destroy(h):
    _check(_lib.load().ehdg_destroy(h))


def ehdg_error_string(code):
    return _lib.load().ehdg_error_string(int(code)).decode()


def ehdg_last_error(h):
    return _lib.load().ehdg_last_error(h).decode()


def _aligned_bytes(torch, nbytes, device):
    """A uint8 tensor of nbytes whose data pointer is 256-byte aligned (the ABI's workspace rule)."""
    raw = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    off = (-raw.data_ptr()) % 256
    return raw[off:off + nbytes]


def _handle_array(handles):
    arr = (ctypes.c_void_p * len(handles))()
    for i, h in enumerate(handles):
        arr[i] = h.value if isinstance(h, ctypes.c_void_p) else h
    return arr


def _check_batch(rc, b, ok=(EHDG_OK,)):
    if rc in ok:
        return rc
    lib = _lib.load()
    msg = lib.ehdg_error_string(rc).decode()
    if b is not None:
        last = lib.ehdg_batch_last_error(b).decode()
        if last:
            msg += f" ({last})"
    raise EhdgError(rc, msg)


def ehdg_batch_workspace_bytes(handles):
    out = ctypes.c_size_t(0)
    _check(_lib.load().ehdg_batch_workspace_bytes(_handle_array(handles), len(handles), ctypes.byref(out)))
    return out.value


def ehdg_batch_create(handles, workspace, stream=None):
    b = ctypes.c_void_p()
    _check(_lib.load().ehdg_batch_create(_handle_array(handles), len(handles), _ptr(workspace),
                                         workspace.numel() * workspace.element_size(), _stream_ptr(stream),
                                         ctypes.byref(b)))
    return b


def ehdg_batch_create_static(handles, stream=None):
    b = ctypes.c_void_p()
    _check(_lib.load().ehdg_batch_create_static(_handle_array(handles), len(handles), _stream_ptr(stream),
                                                ctypes.byref(b)))
    return b


def ehdg_batch_solve(b, n, rel_tol, max_iters, allow=(EHDG_OK,)):
    its = np.zeros(n, dtype=np.int32)
    res = np.zeros(n)
    rc = _lib.load().ehdg_batch_solve(b, float(rel_tol), int(max_iters), its.ctypes.data_as(ctypes.c_void_p),
                                      res.ctypes.data_as(ctypes.c_void_p))
    _check_batch(rc, b, ok=allow)
    return rc, its.tolist(), res.tolist()


def ehdg_batch_step(b, n, n_steps, rel_tol, max_iters_per_step, allow=(EHDG_OK,)):
    its = np.zeros((n, max(n_steps, 1)), dtype=np.int32)
    rc = _lib.load().ehdg_batch_step(b, int(n_steps), float(rel_tol), int(max_iters_per_step),
                                     its.ctypes.data_as(ctypes.c_void_p))
    _check_batch(rc, b, ok=allow)
    return rc, its[:, :n_steps].tolist()


def ehdg_batch_advance(b, n, rounds, rel_tol, step_targets=None):
    state = np.zeros(n, dtype=np.int32)
    tg = None
    if step_targets is not None:
        tg = np.ascontiguousarray(step_targets, dtype=np.int32)
    rc = _lib.load().ehdg_batch_advance(b, int(rounds), float(rel_tol),
                                        tg.ctypes.data_as(ctypes.c_void_p) if tg is not None else None,
                                        state.ctypes.data_as(ctypes.c_void_p))
    _check_batch(rc, b)
    return state.tolist()


def ehdg_batch_set_persistent(b, enabled):
    _check_batch(_lib.load().ehdg_batch_set_persistent(b, 1 if enabled else 0), b)


def ehdg_batch_report_bytes(b):
    n = ctypes.c_size_t(0)
    _check_batch(_lib.load().ehdg_batch_report_bytes(b, ctypes.byref(n)), b)
    return n.value


def ehdg_batch_launch(b, rounds, rel_tol, step_targets, report):
    """Queues `rounds` rounds and a report into `report` (a pinned host tensor of at least
    ehdg_batch_report_bytes bytes); returns at once."""
    tg = None
    if step_targets is not None:
        tg = np.ascontiguousarray(step_targets, dtype=np.int32)
    rc = _lib.load().ehdg_batch_launch(b, int(rounds), float(rel_tol),
                                       tg.ctypes.data_as(ctypes.c_void_p) if tg is not None else None,
                                       _ptr(report), report.numel() * report.element_size())
    _check_batch(rc, b)


def ehdg_batch_poll(b, n):
    """The oldest pending launch's member states if its work has completed, else None."""
    state = np.zeros(n, dtype=np.int32)
    ready = ctypes.c_int32(0)
    _check_batch(_lib.load().ehdg_batch_poll(b, state.ctypes.data_as(ctypes.c_void_p), ctypes.byref(ready)), b)
    return state.tolist() if ready.value else None


def ehdg_batch_get_solution(b, member, out):
    _check_batch(_lib.load().ehdg_batch_get_solution(b, int(member), _ptr(out)), b)


def ehdg_tune_set(pde, dim, degree, precision, tiles_per_group, reverse_order=0):
    _check(_lib.load().ehdg_tune_set(int(pde), int(dim), int(degree), int(precision), int(tiles_per_group),
                                     int(reverse_order)))


def ehdg_tune_clear():
    _check(_lib.load().ehdg_tune_clear())


def ehdg_launch_shape(h):
    """(tiles per workgroup, workgroups, reversed order) of the handle's plain sweeps."""
    tpg, ng, rev = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_int32(0)
    _check(_lib.load().ehdg_launch_shape(h, ctypes.byref(tpg), ctypes.byref(ng), ctypes.byref(rev)), h)
    return tpg.value, ng.value, rev.value


def ehdg_batch_set_graph(b, enabled):
    _check_batch(_lib.load().ehdg_batch_set_graph(b, int(bool(enabled))), b)


def ehdg_batch_destroy(b):
    _check(_lib.load().ehdg_batch_destroy(b))


def ehdg_batch_last_error(b):
    return _lib.load().ehdg_batch_last_error(b).decode()


# ---------------------------------------------------------------------------- convenience
class Batch:
    """Several Problems advanced together (ehdg_batch_*).  The Problems must outlive it."""

    def __init__(self, problems, stream=None, static=False):
        """static: tables in the library's static device array (ehdg_batch_create_static),
        no workspace allocated; one static batch per device at a time."""
        self.problems = list(problems)
        handles = [p.h for p in self.problems]
        self.workspace = None
        if static:
            self.b = ehdg_batch_create_static(handles, stream)
            return
        torch = _torch()
        nbytes = ehdg_batch_workspace_bytes(handles)
        self.workspace = _aligned_bytes(torch, max(nbytes, 256), self.problems[0].device)
        self.b = ehdg_batch_create(handles, self.workspace, stream)

    def solve(self, tol, max_iters=100000, allow=(EHDG_OK,)):
        return ehdg_batch_solve(self.b, len(self.problems), tol, max_iters, allow)

    def step(self, n_steps, tol, max_iters=100000, allow=(EHDG_OK,)):
        return ehdg_batch_step(self.b, len(self.problems), n_steps, tol, max_iters, allow)

    def set_graph(self, enabled):
        """Rounds replayed from a captured HIP graph (True, the default) or launched one by one."""
        ehdg_batch_set_graph(self.b, enabled)

    def set_persistent(self, enabled):
        """2D transport and shallow-water sweeps in the persistent launch (True) or in one
        launch per family (False, the default)."""
        ehdg_batch_set_persistent(self.b, enabled)

    def advance(self, rounds, tol, step_targets=None):
        """Member states after `rounds` more rounds: 0 running, 1 finished, 2 failed."""
        return ehdg_batch_advance(self.b, len(self.problems), rounds, tol, step_targets)

    def report_bytes(self):
        return ehdg_batch_report_bytes(self.b)

    def launch(self, rounds, tol, step_targets, report):
        """Queues `rounds` rounds and their report (pinned host tensor); does not wait."""
        ehdg_batch_launch(self.b, rounds, tol, step_targets, report)

    def poll(self):
        """Member states of the oldest pending launch once it has completed, else None."""
        return ehdg_batch_poll(self.b, len(self.problems))

    def solution(self, k, out=None):
        """Queues member k's solution (finished in the last report read) into `out`."""
        p = self.problems[k]
        if out is None:
            out = p.torch.empty(p.nel, p.m, p.Np, dtype=p.torch.float64, device=p.device)
        ehdg_batch_get_solution(self.b, k, out)
        return out

    def close(self):
        if self.b is not None:
            ehdg_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Problem:
    """A handle with its device workspace.  Closed-form data are sampled on the device
    at the physical points implied by the library's reference points."""

    def __init__(self, pde, dim, n, L=(1.0, 1.0, 1.0), periodic=(0, 0, 0), degree=1, beta=(0.0, 0.0, 0.0),
                 sigma=0.0, Phi=1.0, dt=0.0, precision=EHDG_FP64, inner_sweeps=1, device="cuda", stream=None,
                 U0=(0.0, 0.0), c0=1.0, rho0=1.0, velocity=None):
        """velocity: (beta_fn, div_fn) for transport with a velocity field (ehdg_setup_variable);
        beta_fn(X, xp) -> (..., dim), div_fn(X, xp) -> (...) or None for div beta = 0."""
        torch = _torch()
        self.torch = torch
        self.desc = make_desc(pde, dim, n, L, periodic, degree, beta, sigma, Phi, dt, precision, inner_sweeps,
                              U0, c0, rho0)
        self.pde, self.dim, self.p = pde, dim, degree
        self.n = tuple(int(v) for v in n[:dim])
        self.L = tuple(float(v) for v in L[:dim])
        self.periodic = tuple(int(v) for v in periodic[:dim])
        self.device = torch.device(device)
        self.stream = stream
        self.gll, self.gq, self.gw = ehdg_reference_points(degree)
        if velocity is None:
            nbytes = ehdg_workspace_bytes(self.desc)
            self.workspace = _aligned_bytes(torch, nbytes, self.device)
            self.h = ehdg_setup(self.desc, self.workspace, stream)
        else:
            self.nel = int(np.prod(self.n))
            bq, dq, bf = self.velocity_samples(*velocity)
            nbytes = ehdg_variable_workspace_bytes(self.desc)
            self.workspace = _aligned_bytes(torch, nbytes, self.device)
            self.h = ehdg_setup_variable(self.desc, bq, dq, bf, self.workspace, stream)
        sz = ehdg_sizes(self.h)
        self.nel, self.m, self.Np, self.S, self.I = sz["n_el"], sz["m"], sz["n_p"], sz["S"], sz["I"]

    def close(self):
        if self.h is not None:
            ehdg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- sampling points --------------------------------------------------------
    def _elem_corners(self):
        torch = self.torch
        e = torch.arange(self.nel, device=self.device, dtype=torch.int64)
        idx = []
        r = e
        for a in range(self.dim):
            idx.append(r % self.n[a])
            r = r // self.n[a]
        h = [self.L[a] / self.n[a] for a in range(self.dim)]
        return torch.stack([idx[a].double() * h[a] for a in range(self.dim)], dim=-1), h

    def _tensor_ref(self, pts1d):
        torch = self.torch
        k = len(pts1d)
        g = torch.tensor(pts1d, dtype=torch.float64, device=self.device)
        grids = torch.meshgrid(*([g] * self.dim), indexing="ij")       # last axis fastest
        return torch.stack([grids[self.dim - 1 - a].reshape(-1) for a in range(self.dim)], dim=-1)  # axis 0 fastest

    def points(self, which="nodes"):
        """Physical points (n_el, npts, dim): 'nodes' (GLL) or 'quad' (Gauss)."""
        x0, h = self._elem_corners()
        ref = self._tensor_ref(self.gll if which == "nodes" else self.gq)
        hh = self.torch.tensor(h, dtype=self.torch.float64, device=self.device)
        return x0[:, None, :] + (ref[None, :, :] + 1.0) * 0.5 * hh

    def face_quad_points(self):
        """Physical Gauss points of every element face: (n_el, 2 dim, (p+2)^(dim-1), dim), face f
        on axis f // 2 at its minus (f even) or plus end, tangential axes first-fastest."""
        torch = self.torch
        x0, h = self._elem_corners()
        hh = torch.tensor(h, dtype=torch.float64, device=self.device)
        d = self.dim
        g = torch.tensor(self.gq, dtype=torch.float64, device=self.device)
        k = len(self.gq)
        out = []
        for f in range(2 * d):
            ax = f // 2
            tang = [t for t in range(d) if t != ax]
            ref = torch.zeros(k ** (d - 1), d, dtype=torch.float64, device=self.device)
            ref[:, ax] = -1.0 if f % 2 == 0 else 1.0
            idx = torch.arange(k ** (d - 1), device=self.device)
            for j, t in enumerate(tang):
                ref[:, t] = g[(idx // (k ** j)) % k]
            out.append(x0[:, None, :] + (ref[None] + 1.0) * 0.5 * hh)
        return torch.stack(out, dim=1)

    def velocity_samples(self, beta_fn, div_fn=None):
        """Host arrays (beta_q, div_beta_q, beta_face) of ehdg_setup_variable from callables (X, xp)."""
        torch = self.torch
        Xq = self.points("quad")
        bq = torch.as_tensor(beta_fn(Xq, torch), dtype=torch.float64).permute(0, 2, 1).contiguous()
        dq = None
        if div_fn is not None:
            dq = torch.as_tensor(div_fn(Xq, torch), dtype=torch.float64).expand(Xq.shape[:2]).contiguous()
        Xf = self.face_quad_points()
        Bf = torch.as_tensor(beta_fn(Xf, torch), dtype=torch.float64)           # (nel, 2d, nqf, d)
        axis = torch.arange(2 * self.dim, device=Bf.device) // 2
        bf = torch.gather(Bf, 3, axis[None, :, None, None].expand(*Bf.shape[:3], 1))[..., 0].contiguous()
        cpu = lambda t: None if t is None else t.cpu().numpy()
        return cpu(bq), cpu(dq), cpu(bf)

    def boundary_points(self):
        """Face-node points of every non-periodic side, in the C ABI's bc layout: (nbc, dim)."""
        torch = self.torch
        out = []
        h = [self.L[a] / self.n[a] for a in range(self.dim)]
        g = torch.tensor(self.gll, dtype=torch.float64, device=self.device)
        for side in range(2 * self.dim):
            ax = side // 2
            if self.periodic[ax]:
                continue
            tang = [t for t in range(self.dim) if t != ax]
            # faces: tangential element indices (first fastest); nodes: tangential node indices
            shape = [self.n[t] for t in tang]
            fidx = torch.stack(torch.meshgrid(*[torch.arange(s, device=self.device) for s in shape[::-1]],
                                              indexing="ij"), dim=-1).reshape(-1, len(tang)).flip(-1)
            nidx = torch.stack(torch.meshgrid(*[torch.arange(self.p + 1, device=self.device)] * len(tang),
                                              indexing="ij"), dim=-1).reshape(-1, len(tang)).flip(-1)
            pts = torch.zeros(fidx.shape[0], nidx.shape[0], self.dim, dtype=torch.float64, device=self.device)
            pts[..., ax] = 0.0 if side % 2 == 0 else self.L[ax]
            for j, t in enumerate(tang):
                pts[..., t] = fidx[:, None, j].double() * h[t] + (g[nidx[None, :, j]] + 1.0) * 0.5 * h[t]
            out.append(pts.reshape(-1, self.dim))
        if not out:
            return torch.zeros(0, self.dim, dtype=torch.float64, device=self.device)
        return torch.cat(out, dim=0)

    # -- data ---------------------------------------------------------------------
    def set_forcing(self, f_fns=None, g_fn=None):
        """f_fns: list of callables (X, xp) -> values, one per field (or None); g_fn: inflow data."""
        torch = self.torch
        fq = None
        if f_fns is not None:
            X = self.points("quad")
            fq = torch.stack([torch.as_tensor(fn(X, torch), dtype=torch.float64, device=self.device).expand(X.shape[:2])
                              if fn is not None else torch.zeros(X.shape[:2], dtype=torch.float64,
                                                                 device=self.device) for fn in f_fns], dim=1)
            fq = fq.contiguous()
        bc = None
        if g_fn is not None:
            Xb = self.boundary_points()
            bc = g_fn(Xb, torch).to(torch.float64).contiguous() if Xb.shape[0] else None
        ehdg_set_forcing(self.h, fq, bc)

    def set_initial(self, u0=None):
        """u0: tensor (n_el, m, N_p), list of callables per field, or None."""
        torch = self.torch
        if u0 is not None and not isinstance(u0, torch.Tensor):
            X = self.points("nodes")
            u0 = torch.stack([fn(X, torch).to(torch.float64) for fn in u0], dim=1).contiguous()
        ehdg_set_initial(self.h, u0)

    def solution(self):
        out = self.torch.empty(self.nel, self.m, self.Np, dtype=self.torch.float64, device=self.device)
        ehdg_get_solution(self.h, out)
        return out

    def iterate(self, n):
        ehdg_iterate(self.h, n)

    def solve(self, tol, max_iters=100000, allow=(EHDG_OK,)):
        return ehdg_solve(self.h, tol, max_iters, allow)

    def step(self, n_steps, tol, max_iters=100000, allow=(EHDG_OK,)):
        return ehdg_step(self.h, n_steps, tol, max_iters, allow)

    def residuals(self, first, count):
        return ehdg_get_residuals(self.h, first, count)

    def iters(self):
        return ehdg_sizes(self.h)["iters"]
