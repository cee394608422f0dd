"""Python binding of libfdw (the C-ABI in include/fdw.h): argument marshalling only.

Every step of the solver runs in the HIP kernels of libfdw.so; PyTorch provides device
memory (the caller-owned workspaces and arrays) and the stream.  Importing this module on a
machine without the built library raises ImportError: there is no CPU fallback.

The solver is the explicit leapfrog discretisation of the regularised Cauchy problem of
arXiv 2005.11931 (Section 2, equation (2.1); grid and zero Dirichlet data of Section 3.3).
"""
from __future__ import annotations

import ctypes
import math
import os
from typing import List, Optional, Sequence, Tuple

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libfdw.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"libfdw.so is not built ({LIB_PATH}); run `python -m paper_2005_11931_amd.build`")

_lib = ctypes.CDLL(LIB_PATH)

FDW_F32, FDW_F64 = 0, 1
FDW_OK, FDW_EINVAL, FDW_ECFL, FDW_ESTATE, FDW_ENOMEM, FDW_EHIP, FDW_EUNSTABLE, FDW_ENOTSUP = 0, -1, -2, -3, -4, -5, -6, -7
FDW_ESYNC = -8
FDW_ALLOW_UNSTABLE, FDW_ALLOW_ZERO_H = 1, 2
FDW_CFG_TIME_BLOCK, FDW_CFG_SEGMENT_ROWS, FDW_CFG_USE_GRAPH, FDW_CFG_BATCH_MODE, FDW_CFG_TIMING = 1, 2, 3, 4, 5
FDW_CFG_LANE_COLUMNS, FDW_CFG_ADJ_TIME_BLOCK, FDW_CFG_ADJ_LANE_COLUMNS, FDW_CFG_ADJ_SEGMENT_ROWS = 6, 7, 8, 9
FDW_CFG_CHECK_ENERGY, FDW_CFG_TEST_BARRIER_FLAG, FDW_CFG_ITEM_ORDER, FDW_CFG_STREAM_POLICY = 10, 11, 12, 13
FDW_CFG_SMALL_TILES, FDW_CFG_TILE_ROWS = 14, 15

EXPORTED = [
    "fdw_workspace_bytes", "fdw_init", "fdw_set_coeff", "fdw_step_n", "fdw_energy", "fdw_record_traces",
    "fdw_misfit", "fdw_adjoint_workspace_bytes", "fdw_record_checkpoints", "fdw_adjoint", "fdw_get_state", "fdw_set_state", "fdw_reset",
    "fdw_member_distance",
    "fdw_steps_taken", "fdw_configure", "fdw_get_config", "fdw_autotune", "fdw_kernel_time", "fdw_last_error",
    "fdw_status_string", "fdw_destroy", "fdw_misfit_noalloc", "fdw_noalloc_last_error", "fdw_autotune_adjoint",
    "fdw_adi_workspace_bytes", "fdw_adi_init", "fdw_adi_step_n", "fdw_adi_get_state", "fdw_adi_reset",
    "fdw_adi_last_error", "fdw_adi_destroy",
]


class fdw_problem(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("x0", ctypes.c_double), ("x1", ctypes.c_double), ("y0", ctypes.c_double), ("y1", ctypes.c_double),
        ("tau", ctypes.c_double), ("T", ctypes.c_double),
        ("dtype", ctypes.c_int32), ("flags", ctypes.c_uint32),
    ]


_vp = ctypes.c_void_p
_lib.fdw_workspace_bytes.argtypes = [ctypes.POINTER(fdw_problem), ctypes.c_int32]
_lib.fdw_workspace_bytes.restype = ctypes.c_size_t
_lib.fdw_init.argtypes = [ctypes.POINTER(fdw_problem), ctypes.c_int32, _vp, ctypes.c_size_t,
                          ctypes.POINTER(_vp), ctypes.POINTER(_vp), _vp, ctypes.POINTER(_vp)]
_lib.fdw_init.restype = ctypes.c_int
_lib.fdw_set_coeff.argtypes = [_vp, ctypes.c_int32, _vp, _vp]
_lib.fdw_step_n.argtypes = [_vp, ctypes.c_int64, _vp]
_lib.fdw_energy.argtypes = [_vp, ctypes.POINTER(ctypes.c_double)]
_lib.fdw_record_traces.argtypes = [_vp, ctypes.c_int32, _vp, ctypes.c_int32, _vp]
_lib.fdw_misfit.argtypes = [_vp, ctypes.c_int32, _vp, _vp, ctypes.c_int64, ctypes.c_int32, _vp, _vp]
_lib.fdw_adjoint_workspace_bytes.argtypes = [_vp, ctypes.c_int32, ctypes.c_int32]
_lib.fdw_record_checkpoints.argtypes = [_vp, ctypes.c_int32, ctypes.c_int32, _vp, ctypes.c_size_t]
_lib.fdw_record_checkpoints.restype = ctypes.c_int
_lib.fdw_adjoint_workspace_bytes.restype = ctypes.c_size_t
_lib.fdw_adjoint.argtypes = [_vp, ctypes.c_int32, _vp, ctypes.c_int32, _vp, ctypes.c_int32, _vp, ctypes.c_size_t,
                             _vp, _vp]
_lib.fdw_get_state.argtypes = [_vp, ctypes.c_int32, _vp, _vp, ctypes.POINTER(ctypes.c_int64)]
_lib.fdw_set_state.argtypes = [_vp, ctypes.c_int32, _vp, _vp, ctypes.c_int64]
_lib.fdw_reset.argtypes = [_vp, ctypes.c_int32]
_lib.fdw_member_distance.argtypes = [_vp, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)]
_lib.fdw_member_distance.restype = ctypes.c_int
_lib.fdw_steps_taken.argtypes = [_vp, ctypes.c_int32]
_lib.fdw_steps_taken.restype = ctypes.c_int64
_lib.fdw_configure.argtypes = [_vp, ctypes.c_int32, ctypes.c_int64]
_lib.fdw_get_config.argtypes = [_vp, ctypes.c_int32]
_lib.fdw_get_config.restype = ctypes.c_int64
_lib.fdw_autotune.argtypes = [_vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)]
_lib.fdw_autotune_adjoint.argtypes = [_vp, ctypes.c_int32, _vp, ctypes.c_int32, _vp, ctypes.c_int32, _vp,
                                      ctypes.c_size_t, _vp, ctypes.POINTER(ctypes.c_int64)]
_lib.fdw_autotune_adjoint.restype = ctypes.c_int
_lib.fdw_adi_workspace_bytes.argtypes = [ctypes.POINTER(fdw_problem)]
_lib.fdw_adi_workspace_bytes.restype = ctypes.c_size_t
_lib.fdw_adi_init.argtypes = [ctypes.POINTER(fdw_problem), ctypes.c_double, _vp, ctypes.c_size_t, _vp, _vp, _vp, _vp,
                              _vp, ctypes.POINTER(_vp)]
_lib.fdw_adi_init.restype = ctypes.c_int
_lib.fdw_adi_step_n.argtypes = [_vp, ctypes.c_int64]
_lib.fdw_adi_step_n.restype = ctypes.c_int
_lib.fdw_adi_get_state.argtypes = [_vp, _vp, _vp, ctypes.POINTER(ctypes.c_int64)]
_lib.fdw_adi_get_state.restype = ctypes.c_int
_lib.fdw_adi_reset.argtypes = [_vp]
_lib.fdw_adi_reset.restype = ctypes.c_int
_lib.fdw_adi_last_error.argtypes = [_vp]
_lib.fdw_adi_last_error.restype = ctypes.c_char_p
_lib.fdw_adi_destroy.argtypes = [_vp]
_lib.fdw_adi_destroy.restype = None
_lib.fdw_kernel_time.argtypes = [_vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
_lib.fdw_kernel_time.restype = ctypes.c_int
_lib.fdw_last_error.argtypes = [_vp]
_lib.fdw_last_error.restype = ctypes.c_char_p
_lib.fdw_status_string.argtypes = [ctypes.c_int]
_lib.fdw_status_string.restype = ctypes.c_char_p
_lib.fdw_misfit_noalloc.argtypes = [ctypes.c_int32, _vp, _vp, ctypes.c_int64, ctypes.c_int32, _vp, _vp, _vp]
_lib.fdw_misfit_noalloc.restype = ctypes.c_int
_lib.fdw_noalloc_last_error.argtypes = []
_lib.fdw_noalloc_last_error.restype = ctypes.c_char_p
_lib.fdw_destroy.argtypes = [_vp]
_lib.fdw_destroy.restype = None
for _name in ("fdw_set_coeff", "fdw_step_n", "fdw_energy", "fdw_record_traces", "fdw_misfit", "fdw_adjoint",
              "fdw_get_state", "fdw_set_state", "fdw_reset", "fdw_configure", "fdw_autotune"):
    getattr(_lib, _name).restype = ctypes.c_int


class FdwError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_lib.fdw_status_string(status).decode()} ({status}): {msg}")
        self.status = status


def lib() -> ctypes.CDLL:
    return _lib


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream_handle(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def torch_dtype(dtype: int) -> torch.dtype:
    return torch.float32 if dtype == FDW_F32 else torch.float64


def problem(nx: int, ny: int, tau: float, nsteps: int, dtype: int = FDW_F64, x0: float = -1.0, x1: float = 1.0,
            y0: float = -1.0, y1: float = 1.0, flags: int = 0) -> fdw_problem:
    return fdw_problem(nx, ny, x0, x1, y0, y1, tau, nsteps * tau, dtype, flags)


def problem_from_case(case, dtype: int = FDW_F64, flags: int = 0) -> fdw_problem:
    return fdw_problem(case.nx, case.ny, case.x0, case.x1, case.y0, case.y1, case.tau, case.nsteps * case.tau, dtype,
                       flags)


class Solver:
    """One context of libfdw: `count` members (count > 1 is a batched family).

    u0, u1 and the coefficients are device tensors [ny][nx] in the storage dtype.
    """

    def __init__(self, problems: Sequence[fdw_problem], u0: Sequence[torch.Tensor], u1: Sequence[torch.Tensor],
                 device: str = "cuda:0"):
        self.device = torch.device(device)
        self.count = len(problems)
        self.problems = list(problems)
        arr = (fdw_problem * self.count)(*problems)
        ws = _lib.fdw_workspace_bytes(arr, self.count)
        if ws == 0:
            raise FdwError(FDW_EINVAL, "invalid problem description")
        self.dtypes = [p.dtype for p in problems]
        self.dtype = problems[0].dtype  # the first member's (a family may mix FP32 and FP64 members)
        self.tdtype = torch_dtype(self.dtype)
        self.workspace = torch.empty(ws, dtype=torch.uint8, device=self.device)
        self._keep = [t.contiguous() for t in list(u0) + list(u1)]
        for t, p in zip(u0, problems):
            assert t.dtype == torch_dtype(p.dtype) and tuple(t.shape) == (p.ny, p.nx), (t.dtype, t.shape)
        u0p = (_vp * self.count)(*[t.data_ptr() for t in self._keep[: self.count]])
        u1p = (_vp * self.count)(*[t.data_ptr() for t in self._keep[self.count:]])
        ctx = _vp()
        self.stream = _stream_handle(self.device)
        st = _lib.fdw_init(arr, self.count, _vp(self.workspace.data_ptr()), ws, u0p, u1p, _vp(self.stream),
                           ctypes.byref(ctx))
        if st != 0:
            raise FdwError(st, "fdw_init failed")
        self.ctx = ctx
        self._h = [None] * self.count
        self._gen = [0] * self.count  # bumped whenever a member's coefficient is set
        self._traces = [None] * self.count
        self._ckpt = None  # (member, ckpt_every, workspace) of an armed checkpoint recording

    # -- helpers
    def _check(self, st: int):
        if st != 0:
            raise FdwError(st, _lib.fdw_last_error(self.ctx).decode())

    def close(self):
        if getattr(self, "ctx", None):
            torch.cuda.synchronize(self.device)
            _lib.fdw_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- API
    def set_coeff(self, h1: torch.Tensor, h2: Optional[torch.Tensor] = None, member: int = 0):
        h1 = h1.contiguous()
        h2 = None if h2 is None else h2.contiguous()
        self._h[member] = (h1, h2)
        self._gen[member] += 1
        self._check(_lib.fdw_set_coeff(self.ctx, member, _ptr(h1), _ptr(h2)))

    def step(self, n: int, energy: bool = False) -> Optional[torch.Tensor]:
        e = torch.empty((self.count, n), dtype=torch.float64, device=self.device) if (energy and n > 0) else None
        self._check(_lib.fdw_step_n(self.ctx, int(n), _ptr(e)))
        return e

    def step_into(self, n: int, energy_out: Optional[torch.Tensor]):
        self._check(_lib.fdw_step_n(self.ctx, int(n), _ptr(energy_out)))

    def energy(self) -> List[float]:
        out = (ctypes.c_double * self.count)()
        self._check(_lib.fdw_energy(self.ctx, out))
        return list(out)

    def record_traces(self, receivers: Optional[torch.Tensor], member: int = 0) -> Optional[torch.Tensor]:
        if receivers is None or receivers.numel() == 0:
            self._check(_lib.fdw_record_traces(self.ctx, member, None, 0, None))
            self._traces[member] = None
            return None
        p = self.problems[member]
        N = int(round(p.T / p.tau))
        rec = receivers.to(device=self.device, dtype=torch.int32).contiguous()
        R = rec.shape[0]
        tr = torch.zeros((N + 1, R), dtype=torch_dtype(p.dtype), device=self.device)
        self._traces[member] = (rec, tr)
        self._check(_lib.fdw_record_traces(self.ctx, member, _ptr(rec), R, _ptr(tr)))
        return tr

    def misfit(self, traces: torch.Tensor, d: torch.Tensor, member: int = 0,
               want_grad: bool = True) -> Tuple[torch.Tensor, Optional[torch.Tensor]]:
        traces = traces.contiguous()
        d = d.to(torch.float64).contiguous()
        J = torch.empty((), dtype=torch.float64, device=self.device)
        g = torch.empty(d.shape, dtype=torch.float64, device=self.device) if want_grad else None
        self._check(_lib.fdw_misfit(self.ctx, member, _ptr(traces), _ptr(d), traces.shape[0], traces.shape[1],
                                    _ptr(J), _ptr(g)))
        return J, g

    def _adjoint_workspace(self, member: int, ckpt_every: int) -> torch.Tensor:
        nb = _lib.fdw_adjoint_workspace_bytes(self.ctx, member, ckpt_every)
        if nb == 0:
            raise FdwError(FDW_EINVAL, "fdw_adjoint_workspace_bytes failed")
        return torch.empty(nb, dtype=torch.uint8, device=self.device)

    def record_checkpoints(self, ckpt_every: Optional[int] = 64, member: int = 0):
        """Store the adjoint's checkpoints during the coming forward run of `member` (which must
        be at step 0), so that `adjoint` with the same ckpt_every skips its replay.
        ckpt_every=None stops the recording."""
        if ckpt_every is None:
            self._check(_lib.fdw_record_checkpoints(self.ctx, member, 1, None, 0))
            self._ckpt = None
            return
        ws = self._adjoint_workspace(member, ckpt_every)
        self._check(_lib.fdw_record_checkpoints(self.ctx, member, ckpt_every, _ptr(ws), ws.numel()))
        self._ckpt = (member, ckpt_every, ws)

    def adjoint(self, receivers: torch.Tensor, trace_grad: torch.Tensor, ckpt_every: int = 64, member: int = 0,
                separate: bool = False):
        p = self.problems[member]
        rec = receivers.to(device=self.device, dtype=torch.int32).contiguous()
        tg = trace_grad.to(device=self.device, dtype=torch.float64).contiguous()
        if self._ckpt is not None and self._ckpt[0] == member and self._ckpt[1] == ckpt_every:
            ws = self._ckpt[2]  # the library checks whether the recording is complete
        else:
            ws = self._adjoint_workspace(member, ckpt_every)
        nb = ws.numel()
        g1 = torch.empty((p.ny, p.nx), dtype=torch.float64, device=self.device)
        g2 = torch.empty((p.ny, p.nx), dtype=torch.float64, device=self.device) if separate else None
        self._check(_lib.fdw_adjoint(self.ctx, member, _ptr(rec), rec.shape[0], _ptr(tg), ckpt_every, _ptr(ws), nb,
                                     _ptr(g1), _ptr(g2)))
        return (g1, g2) if separate else g1

    def get_state(self, member: int = 0) -> Tuple[torch.Tensor, torch.Tensor, int]:
        p = self.problems[member]
        u = torch.empty((p.ny, p.nx), dtype=torch_dtype(p.dtype), device=self.device)
        du = torch.empty_like(u)
        n = ctypes.c_int64()
        self._check(_lib.fdw_get_state(self.ctx, member, _ptr(u), _ptr(du), ctypes.byref(n)))
        return u, du, int(n.value)

    def set_state(self, u: torch.Tensor, du: torch.Tensor, n: int, member: int = 0):
        u, du = u.contiguous(), du.contiguous()
        self._check(_lib.fdw_set_state(self.ctx, member, _ptr(u), _ptr(du), int(n)))
        torch.cuda.current_stream(self.device).synchronize()

    def distance(self, a: int, b: int) -> float:
        """L2 distance sqrt(dx dy sum (u_a - u_b)^2) of two members' current fields."""
        out = ctypes.c_double()
        self._check(_lib.fdw_member_distance(self.ctx, a, b, ctypes.byref(out)))
        return float(out.value)

    def reset(self, member: int = 0):
        self._check(_lib.fdw_reset(self.ctx, member))

    def steps_taken(self, member: int = 0) -> int:
        return int(_lib.fdw_steps_taken(self.ctx, member))

    def configure(self, key: int, value: int):
        self._check(_lib.fdw_configure(self.ctx, key, int(value)))

    def config(self, key: int) -> int:
        return int(_lib.fdw_get_config(self.ctx, key))

    def kernel_time(self) -> Tuple[float, int]:
        """(total ms, launches) of the stencil launches since the last call (FDW_CFG_TIMING = 1)."""
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        self._check(_lib.fdw_kernel_time(self.ctx, ctypes.byref(ms), ctypes.byref(n)))
        return float(ms.value), int(n.value)

    def autotune(self, steps: int = 0) -> Tuple[int, int, int]:
        """Returns (time_block, segment_rows, lane_columns)."""
        out = (ctypes.c_int64 * 3)()
        self._check(_lib.fdw_autotune(self.ctx, int(steps), out))
        return int(out[0]), int(out[1]), int(out[2])

    def autotune_adjoint(self, receivers: torch.Tensor, trace_grad: torch.Tensor, ckpt_every: int = 64,
                         member: int = 0) -> Tuple[int, int, int]:
        """Tune the reverse sweep on this gradient problem (uses the recorded checkpoints when the
        forward run stored them).  Returns (adj_time_block, adj_segment_rows, adj_lane_columns)."""
        p = self.problems[member]
        rec = receivers.to(device=self.device, dtype=torch.int32).contiguous()
        tg = trace_grad.to(device=self.device, dtype=torch.float64).contiguous()
        if self._ckpt is not None and self._ckpt[0] == member and self._ckpt[1] == ckpt_every:
            ws = self._ckpt[2]
        else:
            ws = self._adjoint_workspace(member, ckpt_every)
        g = torch.empty((p.ny, p.nx), dtype=torch.float64, device=self.device)
        out = (ctypes.c_int64 * 3)()
        self._check(_lib.fdw_autotune_adjoint(self.ctx, member, _ptr(rec), rec.shape[0], _ptr(tg), ckpt_every,
                                              _ptr(ws), ws.numel(), _ptr(g), out))
        return int(out[0]), int(out[1]), int(out[2])


def misfit_noalloc(traces: torch.Tensor, d: torch.Tensor, J_out: torch.Tensor,
                   grad_out: Optional[torch.Tensor] = None) -> None:
    """fdw_misfit_noalloc: J_out[()] = sum (traces - d)^2 and grad_out = 2 (traces - d), with no
    context, no workspace and no device allocation (the outputs are the caller's)."""
    dt = FDW_F32 if traces.dtype == torch.float32 else FDW_F64
    assert traces.is_contiguous() and d.is_contiguous() and d.dtype == torch.float64 and traces.shape == d.shape
    assert J_out.dtype == torch.float64 and (grad_out is None or grad_out.dtype == torch.float64)
    rows, R = traces.shape
    st = _lib.fdw_misfit_noalloc(dt, _ptr(traces), _ptr(d), rows, R, _ptr(J_out), _ptr(grad_out),
                                 _vp(_stream_handle(traces.device)))
    if st != 0:
        raise FdwError(st, _lib.fdw_noalloc_last_error().decode())


class ImplicitSolver:
    """The implicit factorized scheme with cyclic-reduction line solves (fdw_adi_*)."""

    def __init__(self, problem: fdw_problem, sigma: float, u0: torch.Tensor, u1: torch.Tensor, h1: torch.Tensor,
                 h2: Optional[torch.Tensor] = None, device: str = "cuda:0"):
        self.device = torch.device(device)
        self.problem = problem
        self.tdtype = torch_dtype(problem.dtype)
        ws = _lib.fdw_adi_workspace_bytes(ctypes.byref(problem))
        if ws == 0:
            raise FdwError(FDW_EINVAL, "invalid problem description")
        self.workspace = torch.empty(ws, dtype=torch.uint8, device=self.device)
        self._keep = [t.contiguous() for t in (u0, u1, h1) + (() if h2 is None else (h2,))]
        for t in self._keep:
            assert t.dtype == self.tdtype and tuple(t.shape) == (problem.ny, problem.nx), (t.dtype, t.shape)
        ctx = _vp()
        st = _lib.fdw_adi_init(ctypes.byref(problem), float(sigma), _vp(self.workspace.data_ptr()), ws,
                               _ptr(self._keep[0]), _ptr(self._keep[1]), _ptr(self._keep[2]),
                               None if h2 is None else _ptr(self._keep[3]), _vp(_stream_handle(self.device)),
                               ctypes.byref(ctx))
        if st != 0:
            raise FdwError(st, "fdw_adi_init failed")
        self.ctx = ctx

    def _check(self, st: int):
        if st != 0:
            raise FdwError(st, _lib.fdw_adi_last_error(self.ctx).decode())

    def step(self, n: int):
        self._check(_lib.fdw_adi_step_n(self.ctx, int(n)))

    def get_state(self) -> Tuple[torch.Tensor, torch.Tensor, int]:
        p = self.problem
        u = torch.empty((p.ny, p.nx), dtype=self.tdtype, device=self.device)
        du = torch.empty_like(u)
        n = ctypes.c_int64()
        self._check(_lib.fdw_adi_get_state(self.ctx, _ptr(u), _ptr(du), ctypes.byref(n)))
        return u, du, int(n.value)

    def reset(self):
        self._check(_lib.fdw_adi_reset(self.ctx))

    def close(self):
        if getattr(self, "ctx", None):
            torch.cuda.synchronize(self.device)
            _lib.fdw_adi_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def implicit_solver_for_case(case, sigma: float = 0.25, dtype: int = FDW_F64, device: str = "cuda:0",
                             flags: int = 0) -> ImplicitSolver:
    td = torch_dtype(dtype)
    t = lambda a: torch.as_tensor(a, dtype=td, device=device)
    return ImplicitSolver(problem_from_case(case, dtype, flags), sigma, t(case.u0), t(case.u1), t(case.h1),
                          None if case.h2 is None else t(case.h2), device=device)


def solver_for_case(case, dtype: int = FDW_F64, device: str = "cuda:0", flags: int = 0, separate_h2: bool = False):
    """Build a single-member Solver from an inputs.Case and set its coefficient."""
    td = torch_dtype(dtype)
    u0 = torch.as_tensor(case.u0, dtype=td, device=device)
    u1 = torch.as_tensor(case.u1, dtype=td, device=device)
    s = Solver([problem_from_case(case, dtype, flags)], [u0], [u1], device=device)
    h1 = torch.as_tensor(case.h1, dtype=td, device=device)
    h2 = None
    if case.h2 is not None or separate_h2:
        h2 = torch.as_tensor(case.h1 if case.h2 is None else case.h2, dtype=td, device=device)
    s.set_coeff(h1, h2)
    return s


def family_solver(cases, dtype=FDW_F32, device: str = "cuda:0", flags: int = 0) -> Solver:
    """A batched Solver over `cases`; dtype is one storage type for all members, or a list with
    one per member (a family may hold FP64 members among FP32 ones)."""
    dts = list(dtype) if isinstance(dtype, (list, tuple)) else [dtype] * len(cases)
    u0 = [torch.as_tensor(c.u0, dtype=torch_dtype(d), device=device) for c, d in zip(cases, dts)]
    u1 = [torch.as_tensor(c.u1, dtype=torch_dtype(d), device=device) for c, d in zip(cases, dts)]
    s = Solver([problem_from_case(c, d, flags) for c, d in zip(cases, dts)], u0, u1, device=device)
    for m, (c, d) in enumerate(zip(cases, dts)):
        td = torch_dtype(d)
        s.set_coeff(torch.as_tensor(c.h1, dtype=td, device=device),
                    None if c.h2 is None else torch.as_tensor(c.h2, dtype=td, device=device), member=m)
    return s


class FdwMisfit(torch.autograd.Function):
    """loss = sum_{n,r} (u^n(receiver r) - d_{n,r})^2 as a function of the nodal depth h (h1 = h2 = h).

    forward: set the coefficient, run the leapfrog solve recording traces and the adjoint's
    checkpoints, FP64 misfit (libfdw).
    backward: adjoint source 2 (traces - d) * grad_output, reverse leapfrog from the recorded
    checkpoints (libfdw) -> dL/dh.  If the solver's coefficient was set again after this
    loss's forward (another loss on the same solver, a line search), the loss's own depth is
    set back first and the adjoint replays the forward run from the initial data.
    """

    @staticmethod
    def forward(ctx, h: torch.Tensor, solver: Solver, receivers: torch.Tensor, d_obs: torch.Tensor,
                ckpt_every: int = 64):
        p = solver.problems[0]
        N = int(round(p.T / p.tau))
        hs = h.detach().to(solver.tdtype).clone()
        solver.set_coeff(hs)
        solver.record_checkpoints(ckpt_every)
        tr = solver.record_traces(receivers)
        solver.step(N)
        J, g = solver.misfit(tr, d_obs)
        ctx.solver = solver
        ctx.receivers = receivers
        ctx.ckpt = ckpt_every
        ctx.h_dtype = h.dtype
        ctx.h_solver = hs
        ctx.gen = solver._gen[0]
        ctx.save_for_backward(g)
        solver.record_traces(None)
        return J

    @staticmethod
    def backward(ctx, grad_out):
        (g,) = ctx.saved_tensors
        tg = g * grad_out.to(torch.float64)
        if ctx.solver._gen[0] != ctx.gen:
            # the solver moved on to another depth: back to this loss's (the adjoint replays)
            ctx.solver.set_coeff(ctx.h_solver)
            ctx.gen = ctx.solver._gen[0]
        grad_h = ctx.solver.adjoint(ctx.receivers, tg, ckpt_every=ctx.ckpt)
        return grad_h.to(ctx.h_dtype), None, None, None, None
