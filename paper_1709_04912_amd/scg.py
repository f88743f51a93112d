"""Python binding of libscg (include/scg.h): argument marshalling only.

Every computation runs in the HIP library; PyTorch supplies device memory
and streams. Importing this module loads libscg.so and raises if it is
missing: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libscg.so")

SCG_OK, SCG_EINVAL, SCG_ENOMEM, SCG_EDEVICE = 0, -1, -2, -3
SCG_ENOCONV, SCG_ENAN, SCG_EBREAKDOWN = -4, -5, -6
SCG_EAGAIN, SCG_EINPROGRESS, SCG_ENOTFOUND = -7, -8, -9
SCG_F32, SCG_F64 = 0, 1
VARIANTS = {"CG": 0, "S_CG": 1, "S_CG_CD": 2, "S_PCG": 3, "S_CG_K": 4, "S_CG_3OP": 5,
            "PCG": 6, "S_PCG_K": 7}
SCG_FLAG_NO_PERTURB = 1


class scg_geom(C.Structure):
    _fields_ = [("n", C.c_int32), ("n_angles", C.c_int32), ("n_bins", C.c_int32)]


class scg_params(C.Structure):
    _fields_ = [("variant", C.c_int32), ("prec", C.c_int32), ("eps", C.c_double),
                ("gamma0", C.c_double), ("a", C.c_double), ("max_iter", C.c_int32),
                ("max_trials", C.c_int32), ("tv_kappa", C.c_double),
                ("precond_mu", C.c_double), ("flags", C.c_uint32), ("restart_k", C.c_int32)]


class scg_report(C.Structure):
    _fields_ = [("status", C.c_int32), ("k", C.c_int32), ("steps", C.c_int32),
                ("trials_total", C.c_int32), ("ell", C.c_int32), ("reserved", C.c_int32),
                ("f_out", C.c_double), ("tv_out", C.c_double)]


class scg_trace_entry(C.Structure):
    _fields_ = [("k", C.c_int32), ("accepted", C.c_int32), ("trials", C.c_int32),
                ("ell", C.c_int32), ("f_half", C.c_double), ("tv_x", C.c_double),
                ("gamma", C.c_double), ("beta", C.c_double), ("alpha", C.c_double)]


class scg_kernel_time(C.Structure):
    _fields_ = [("launches", C.c_int64), ("total_ms", C.c_double),
                ("tail_launches", C.c_int64), ("tail_ms", C.c_double)]


class scg_tuning(C.Structure):
    _fields_ = [("project_groups", C.c_int32), ("backproject_split", C.c_int32),
                ("project_angles", C.c_int32), ("swizzle", C.c_int32),
                ("backproject_mirror", C.c_int32), ("project_mirror", C.c_int32)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


KERNEL_CLASSES = ("project", "backproject", "tv", "trials", "vector", "stage", "filter",
                  "control")


class ScgError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {lib.scg_strerror(status).decode()} ({status})")


def _load() -> C.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libscg.so not built ({LIB_PATH}); run __graft_entry__.build()")
    L = C.CDLL(LIB_PATH)
    vp, i32, dbl = C.c_void_p, C.c_int32, C.c_double
    L.scg_plan_create.argtypes = [C.POINTER(scg_geom), C.c_int, C.POINTER(vp)]
    L.scg_plan_destroy.argtypes = [vp]
    L.scg_plan_destroy.restype = None
    L.scg_workspace_bytes.argtypes = [vp, C.POINTER(scg_params), C.POINTER(C.c_size_t)]
    L.scg_project.argtypes = [vp, C.c_int, vp, vp, vp]
    L.scg_backproject.argtypes = [vp, C.c_int, vp, vp, vp]
    L.scg_tv.argtypes = [vp, C.c_int, vp, dbl, vp, C.POINTER(dbl), vp]
    L.scg_filter.argtypes = [vp, C.c_int, dbl, vp, vp, vp]
    L.scg_solve.argtypes = [vp, C.POINTER(scg_params), vp, vp, vp, vp, C.c_size_t,
                            C.POINTER(scg_report), C.POINTER(scg_trace_entry), i32,
                            C.POINTER(i32), i32, vp]
    L.scg_solve_static.argtypes = [vp, C.POINTER(scg_params), vp, vp, vp,
                                   C.POINTER(scg_report), C.POINTER(scg_trace_entry), i32,
                                   C.POINTER(i32), i32, vp]
    L.scg_static_workspace_bytes.argtypes = []
    L.scg_static_workspace_bytes.restype = C.c_size_t
    L.scg_profile.argtypes = [vp, C.c_uint32]
    L.scg_profile_read.argtypes = [vp, C.POINTER(scg_kernel_time)]
    L.scg_profile_every.argtypes = [vp, i32]
    L.scg_plan_get_tuning.argtypes = [vp, C.c_int, C.POINTER(scg_tuning)]
    L.scg_plan_set_tuning.argtypes = [vp, C.c_int, C.POINTER(scg_tuning)]
    L.scg_plan_autotune.argtypes = [vp, C.c_int, vp, C.POINTER(scg_tuning)]
    L.scg_default_params.argtypes = [C.POINTER(scg_params)]
    L.scg_default_params.restype = None
    L.scg_strerror.argtypes = [C.c_int]
    L.scg_strerror.restype = C.c_char_p
    for name in ("scg_plan_create", "scg_workspace_bytes", "scg_project", "scg_backproject",
                 "scg_tv", "scg_filter", "scg_solve", "scg_solve_static", "scg_profile",
                 "scg_profile_read", "scg_profile_every",
                 "scg_plan_get_tuning", "scg_plan_set_tuning", "scg_plan_autotune"):
        getattr(L, name).restype = C.c_int
    return L


lib = _load()


def _check(rc: int, where: str, ok=(SCG_OK,)):
    if rc not in ok:
        raise ScgError(rc, where)
    return rc


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def _prec_of(t: torch.Tensor) -> int:
    if t.dtype == torch.float32:
        return SCG_F32
    if t.dtype == torch.float64:
        return SCG_F64
    raise TypeError("tensors must be float32 or float64")


def _dev(t: torch.Tensor, n: int, name: str):
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous device tensor")
    if t.numel() != n:
        raise ValueError(f"{name} has {t.numel()} elements, expected {n}")
    return C.c_void_p(t.data_ptr())


@dataclass
class Report:
    status: int
    k: int
    steps: int
    trials_total: int
    ell: int
    f_out: float
    tv_out: float


class Plan:
    """A parallel-beam geometry on one device (scg_plan_create)."""

    def __init__(self, n: int, n_angles: int, n_bins: int, device: int = 0):
        self.n, self.n_angles, self.n_bins = int(n), int(n_angles), int(n_bins)
        self.device = int(device)
        g = scg_geom(self.n, self.n_angles, self.n_bins)
        h = C.c_void_p()
        _check(lib.scg_plan_create(C.byref(g), self.device, C.byref(h)), "scg_plan_create")
        self._h = h

    @property
    def J(self) -> int:
        return self.n * self.n

    @property
    def L(self) -> int:
        return self.n_angles * self.n_bins

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            torch.cuda.synchronize(self.device)
            lib.scg_plan_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- operators ---------------------------------------------------------
    def project(self, x: torch.Tensor, out: Optional[torch.Tensor] = None, stream=None):
        """y = A x (scg_project)."""
        if out is None:
            out = torch.empty(self.L, dtype=x.dtype, device=x.device)
        _check(lib.scg_project(self._h, _prec_of(x), _dev(x, self.J, "x"), _dev(out, self.L, "y"),
                               C.c_void_p(_stream_handle(stream))), "scg_project")
        return out

    def backproject(self, y: torch.Tensor, out: Optional[torch.Tensor] = None, stream=None):
        """x = A^T y (scg_backproject)."""
        if out is None:
            out = torch.empty(self.J, dtype=y.dtype, device=y.device)
        _check(lib.scg_backproject(self._h, _prec_of(y), _dev(y, self.L, "y"),
                                   _dev(out, self.J, "x"), C.c_void_p(_stream_handle(stream))),
               "scg_backproject")
        return out

    def tv(self, x: torch.Tensor, kappa: float = 0.0, subgrad: bool = False, stream=None):
        """TV(x) and optionally a subgradient (scg_tv)."""
        s = torch.empty(self.J, dtype=x.dtype, device=x.device) if subgrad else None
        val = C.c_double()
        _check(lib.scg_tv(self._h, _prec_of(x), _dev(x, self.J, "x"), float(kappa),
                          C.c_void_p(s.data_ptr()) if s is not None else None, C.byref(val),
                          C.c_void_p(_stream_handle(stream))), "scg_tv")
        return (val.value, s) if subgrad else val.value

    def filter(self, r: torch.Tensor, mu: float = 0.0, out: Optional[torch.Tensor] = None,
               stream=None):
        """F^T C F per projection (scg_filter)."""
        if out is None:
            out = torch.empty(self.L, dtype=r.dtype, device=r.device)
        _check(lib.scg_filter(self._h, _prec_of(r), float(mu), _dev(r, self.L, "r"),
                              _dev(out, self.L, "out"), C.c_void_p(_stream_handle(stream))),
               "scg_filter")
        return out

    # -- launch shapes -----------------------------------------------------
    def tuning(self, prec: int = SCG_F32) -> dict:
        t = scg_tuning()
        _check(lib.scg_plan_get_tuning(self._h, prec, C.byref(t)), "scg_plan_get_tuning")
        return t.as_dict()

    def set_tuning(self, prec: int = SCG_F32, project_groups: int = 4,
                   backproject_split: int = 2, project_angles: int = 8, swizzle: int = 0,
                   backproject_mirror: int = 0, project_mirror: int = 0):
        t = scg_tuning(project_groups, backproject_split, project_angles, swizzle,
                       backproject_mirror, project_mirror)
        _check(lib.scg_plan_set_tuning(self._h, prec, C.byref(t)), "scg_plan_set_tuning")

    def autotune(self, prec: int = SCG_F32, stream=None) -> dict:
        """Times every launch shape of A and A^T and keeps the fastest."""
        t = scg_tuning()
        _check(lib.scg_plan_autotune(self._h, prec, C.c_void_p(_stream_handle(stream)),
                                     C.byref(t)), "scg_plan_autotune")
        return t.as_dict()

    # -- kernel timing -----------------------------------------------------
    def profile(self, classes=(), every: int = 1):
        """Times the named kernel classes inside scg_solve (scg_profile), one
        launch in `every` of each (scg_profile_every)."""
        mask = 0
        for c in classes:
            mask |= 1 << KERNEL_CLASSES.index(c)
        _check(lib.scg_profile(self._h, mask), "scg_profile")
        _check(lib.scg_profile_every(self._h, int(every)), "scg_profile_every")

    def profile_read(self) -> dict:
        """Per class: (launches, total_ms, tail_launches, tail_ms); the tail
        launches were enqueued after the solve had stopped and did no work."""
        arr = (scg_kernel_time * len(KERNEL_CLASSES))()
        _check(lib.scg_profile_read(self._h, arr), "scg_profile_read")
        return {name: (arr[i].launches, arr[i].total_ms, arr[i].tail_launches, arr[i].tail_ms)
                for i, name in enumerate(KERNEL_CLASSES)}

    # -- solver ------------------------------------------------------------
    def params(self, eps: float, gamma0: float, variant: str = "S_CG", prec: int = SCG_F32,
               a: float = 0.975, max_iter: int = 1000, max_trials: int = 100,
               kappa: float = 0.0, mu: float = 0.0, flags: int = 0,
               restart_k: int = 2) -> scg_params:
        p = scg_params()
        lib.scg_default_params(C.byref(p))
        p.variant = VARIANTS[variant] if isinstance(variant, str) else int(variant)
        p.prec = int(prec)
        p.eps, p.gamma0, p.a = float(eps), float(gamma0), float(a)
        p.max_iter, p.max_trials = int(max_iter), int(max_trials)
        p.tv_kappa, p.precond_mu, p.flags = float(kappa), float(mu), int(flags)
        p.restart_k = int(restart_k)
        return p

    def f(self, y: torch.Tensor, x: torch.Tensor, stream=None) -> float:
        """f(x) = 1/2 ||y - A x||^2 evaluated by the library: scg_solve of
        plain CG from x0 = x with max_iter = 0 reports f at its start point
        (FP64 accumulation)."""
        p = self.params(eps=1e-300, gamma0=0.0, variant="CG", prec=_prec_of(y), max_iter=0)
        _, rep, _ = self.solve(y, p, x0=x, trace=False, stream=stream)
        return rep.f_out

    def workspace_bytes(self, params: scg_params) -> int:
        n = C.c_size_t()
        _check(lib.scg_workspace_bytes(self._h, C.byref(params), C.byref(n)),
               "scg_workspace_bytes")
        return n.value

    def workspace(self, params: scg_params) -> torch.Tensor:
        return torch.empty(self.workspace_bytes(params), dtype=torch.uint8,
                           device=f"cuda:{self.device}")

    def solve(self, y: torch.Tensor, params: scg_params, x0: Optional[torch.Tensor] = None,
              out: Optional[torch.Tensor] = None, ws: Optional[torch.Tensor] = None,
              trace: bool = True, forced=None, stream=None):
        """Runs scg_solve; returns (x, Report, trace list). Statuses
        SCG_ENOCONV, SCG_ENAN and SCG_EBREAKDOWN are reported, not raised."""
        if ws is None:
            ws = self.workspace(params)
        need = self.workspace_bytes(params)
        return self._run("scg_solve", y, params, x0, out, trace, forced, stream,
                         (C.c_void_p(ws.data_ptr()), need))

    def solve_static(self, y: torch.Tensor, params: scg_params,
                     x0: Optional[torch.Tensor] = None, out: Optional[torch.Tensor] = None,
                     trace: bool = True, forced=None, stream=None):
        """scg_solve_static: scg_solve on the library's static device workspace
        (no device allocation by the library); out must be given by callers
        that allocate nothing themselves."""
        return self._run("scg_solve_static", y, params, x0, out, trace, forced, stream, ())

    def _run(self, fn, y, params, x0, out, trace, forced, stream, ws_args):
        prec = _prec_of(y)
        if prec != params.prec:
            raise ValueError("params.prec does not match the tensor dtype")
        if out is None:
            out = torch.empty(self.J, dtype=y.dtype, device=y.device)
        cap = params.max_iter + 1 if trace else 0
        tr = (scg_trace_entry * max(cap, 1))()
        rep = scg_report()
        fptr, flen = None, 0
        if forced is not None:
            flat = []
            for nt, am in forced:
                flat += [int(nt), int(am)]
            farr = (C.c_int32 * max(len(flat), 1))(*flat)
            fptr, flen = farr, len(forced)
        rc = getattr(lib, fn)(self._h, C.byref(params), _dev(y, self.L, "y"),
                              _dev(x0, self.J, "x0") if x0 is not None else None,
                              _dev(out, self.J, "x_out"), *ws_args,
                              C.byref(rep), tr if trace else None, cap, fptr, flen,
                              C.c_void_p(_stream_handle(stream)))
        _check(rc, fn, ok=(SCG_OK, SCG_ENOCONV, SCG_ENAN, SCG_EBREAKDOWN))
        report = Report(rep.status, rep.k, rep.steps, rep.trials_total, rep.ell, rep.f_out,
                        rep.tv_out)
        entries = []
        if trace:
            for e in tr[:max(rep.steps, 0)]:
                entries.append({"k": e.k, "accepted": e.accepted, "trials": e.trials,
                                "ell": e.ell, "f_half": e.f_half, "tv_x": e.tv_x,
                                "gamma": e.gamma, "beta": e.beta, "alpha": e.alpha})
        return out, report, entries


def static_workspace_bytes() -> int:
    """Bytes of scg_solve_static's per-device workspace."""
    return int(lib.scg_static_workspace_bytes())


# ---------------------------------------------------------------------------
# Batch engine (scg_batch_*)
# ---------------------------------------------------------------------------

class scg_batch_stats(C.Structure):
    _fields_ = [("active", C.c_int32), ("slots", C.c_int32), ("groups", C.c_int32),
                ("graph_updates", C.c_int32), ("arena_bytes", C.c_uint64),
                ("arena_used", C.c_uint64), ("submitted", C.c_uint64),
                ("retired", C.c_uint64), ("macro_steps", C.c_uint64),
                ("graph_builds", C.c_uint64), ("rebuild_ns", C.c_uint64)]


SCG_BATCH_NO_GRAPH = 1


def _bind_batch(L):
    vp = C.c_void_p
    L.scg_batch_create.argtypes = [C.c_int, C.c_size_t, C.c_int, C.c_uint32, C.POINTER(vp)]
    L.scg_batch_destroy.argtypes = [vp]
    L.scg_batch_destroy.restype = None
    L.scg_batch_submit.argtypes = [vp, vp, C.POINTER(scg_params), vp, vp, vp,
                                   C.POINTER(C.c_uint64)]
    L.scg_batch_step.argtypes = [vp, C.c_int]
    L.scg_batch_poll.argtypes = [vp, C.c_uint64, C.POINTER(scg_report)]
    L.scg_batch_cancel.argtypes = [vp, C.c_uint64]
    L.scg_batch_get_stats.argtypes = [vp, C.POINTER(scg_batch_stats)]
    L.scg_batch_stream.argtypes = [vp]
    L.scg_batch_stream.restype = vp
    L.scg_batch_wait_stream.argtypes = [vp, vp]
    for name in ("scg_batch_create", "scg_batch_submit", "scg_batch_step", "scg_batch_poll",
                 "scg_batch_cancel", "scg_batch_get_stats", "scg_batch_wait_stream"):
        getattr(L, name).restype = C.c_int


_bind_batch(lib)


class Batch:
    """Many resident solves advanced together (scg_batch_*). The tensors of a
    submitted solve are kept referenced until its report has been polled."""

    def __init__(self, arena_bytes: int, max_slots: int = 64, device: int = 0,
                 graph: bool = True):
        self.device = device
        self._h = C.c_void_p()
        flags = 0 if graph else SCG_BATCH_NO_GRAPH
        _check(lib.scg_batch_create(device, int(arena_bytes), int(max_slots), flags,
                                    C.byref(self._h)), "scg_batch_create")
        self._keep = {}
        self._stream = torch.cuda.ExternalStream(lib.scg_batch_stream(self._h),
                                                 device=f"cuda:{device}")

    @property
    def stream(self):
        return self._stream

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib.scg_batch_destroy(self._h)
            self._h = C.c_void_p()
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def submit(self, plan: "Plan", y: torch.Tensor, params: scg_params,
               x0: Optional[torch.Tensor] = None, out: Optional[torch.Tensor] = None):
        """Admits a solve; returns (ticket, out) or None when the batch has no
        free slot or arena room (SCG_EAGAIN)."""
        if _prec_of(y) != params.prec:
            raise ValueError("params.prec does not match the tensor dtype")
        if out is None:
            out = torch.empty(plan.J, dtype=y.dtype, device=y.device)
        # y (and x0) come from torch's current stream: the batch's work waits
        # for what is enqueued there
        _check(lib.scg_batch_wait_stream(
            self._h, C.c_void_p(_stream_handle(torch.cuda.current_stream(y.device)))),
            "scg_batch_wait_stream")
        t = C.c_uint64()
        rc = lib.scg_batch_submit(self._h, plan._h, C.byref(params), _dev(y, plan.L, "y"),
                                  _dev(x0, plan.J, "x0") if x0 is not None else None,
                                  _dev(out, plan.J, "x_out"), C.byref(t))
        if rc == SCG_EAGAIN:
            return None
        _check(rc, "scg_batch_submit")
        self._keep[t.value] = (plan, y, x0, out)
        return t.value, out

    def step(self, iters: int = 1) -> int:
        """Runs `iters` iterations of every active solve and retires the
        finished ones; returns the number still active."""
        rc = lib.scg_batch_step(self._h, int(iters))
        if rc < 0:
            raise ScgError(rc, "scg_batch_step")
        return rc

    def poll(self, ticket: int):
        """The Report of a retired ticket (once), or None while it runs."""
        rep = scg_report()
        rc = lib.scg_batch_poll(self._h, int(ticket), C.byref(rep))
        if rc == SCG_EINPROGRESS:
            return None
        _check(rc, "scg_batch_poll")
        self._keep.pop(int(ticket), None)
        return Report(rep.status, rep.k, rep.steps, rep.trials_total, rep.ell, rep.f_out,
                      rep.tv_out)

    def cancel(self, ticket: int):
        _check(lib.scg_batch_cancel(self._h, int(ticket)), "scg_batch_cancel")
        self._keep.pop(int(ticket), None)

    def stats(self) -> dict:
        s = scg_batch_stats()
        _check(lib.scg_batch_get_stats(self._h, C.byref(s)), "scg_batch_get_stats")
        return {name: getattr(s, name) for name, _ in s._fields_ if name != "reserved"}
