"""ctypes wrapper of the FP64 CPU oracle (fdw_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the benchmark's
CPU-baseline leg, never by the library.  It shares no code with the GPU path; the two meet
only in the seeded input generators.

Every function here calls straight into the C oracle; see fdw_oracle.c for the definitions
and their citations in the paper.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fdw_oracle.c")
_LIBDIR = os.path.join(_HERE, "_lib")
_LIB = os.path.join(_LIBDIR, "libfdwref.so")
_lock = threading.Lock()
_lib = None

_DP = ctypes.POINTER(ctypes.c_double)
_IP = ctypes.POINTER(ctypes.c_int)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, OpenMP, no floating-point contraction)."""
    os.makedirs(_LIBDIR, exist_ok=True)
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
               _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)
            lib = ctypes.CDLL(_LIB)
            lib.fdwref_faces.argtypes = [ctypes.c_int, ctypes.c_int, _DP, _DP, _DP, _DP]
            lib.fdwref_apply.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, _DP, _DP, _DP, _DP]
            lib.fdwref_start.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                         _DP, _DP, _DP, _DP, _DP, _DP]
            lib.fdwref_step.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                        _DP, _DP, _DP, _DP, _DP, _DP]
            lib.fdwref_energy.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                          _DP, _DP, _DP, _DP]
            lib.fdwref_energy.restype = ctypes.c_double
            lib.fdwref_forward.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                           _DP, _DP, _DP, _DP, ctypes.c_long, _DP, ctypes.c_int, _IP, _DP, _DP, _DP]
            lib.fdwref_forward.restype = ctypes.c_int
            lib.fdwref_forward_ld.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                              ctypes.c_double, _DP, _DP, _DP, _DP, ctypes.c_long, ctypes.c_int, _IP,
                                              _DP, ctypes.c_int, ctypes.POINTER(ctypes.c_long), _DP, _DP, _DP]
            lib.fdwref_forward_ld.restype = ctypes.c_int
            lib.fdwref_adi_forward.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                               ctypes.c_double, ctypes.c_double, _DP, _DP, _DP, _DP, ctypes.c_long,
                                               _DP, _DP]
            lib.fdwref_adi_forward.restype = ctypes.c_int
            lib.fdwref_tridiag.argtypes = [ctypes.c_int, _DP, _DP, _DP, _DP, _DP]
            lib.fdwref_misfit.argtypes = [ctypes.c_long, ctypes.c_int, _DP, _DP]
            lib.fdwref_misfit.restype = ctypes.c_double
            lib.fdwref_adjoint.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                           _DP, _DP, _DP, _DP, ctypes.c_long, ctypes.c_int, _IP, _DP, ctypes.c_long,
                                           _DP, _DP]
            lib.fdwref_adjoint.restype = ctypes.c_int
            lib.fdwref_threads.restype = ctypes.c_int
            _lib = lib
    return _lib


def _d(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_DP)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def threads() -> int:
    return int(_load().fdwref_threads())


def faces(h1: np.ndarray, h2: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    h1, h2 = _f64(h1), _f64(h2)
    ny, nx = h1.shape
    hx, hy = np.empty_like(h1), np.empty_like(h1)
    _load().fdwref_faces(nx, ny, _d(h1), _d(h2), _d(hx), _d(hy))
    return hx, hy


def apply(hx: np.ndarray, hy: np.ndarray, v: np.ndarray, dx: float, dy: float) -> np.ndarray:
    hx, hy, v = _f64(hx), _f64(hy), _f64(v)
    ny, nx = v.shape
    out = np.empty_like(v)
    _load().fdwref_apply(nx, ny, dx, dy, _d(hx), _d(hy), _d(v), _d(out))
    return out


def start(hx, hy, u0, u1, dx, dy, tau, f0=None) -> np.ndarray:
    hx, hy, u0, u1 = _f64(hx), _f64(hy), _f64(u0), _f64(u1)
    f0 = None if f0 is None else _f64(f0)
    ny, nx = u0.shape
    out = np.empty_like(u0)
    _load().fdwref_start(nx, ny, dx, dy, tau, _d(hx), _d(hy), _d(u0), _d(u1), _d(f0), _d(out))
    return out


def step(hx, hy, u_prev, u_cur, dx, dy, tau, f=None) -> np.ndarray:
    hx, hy, u_prev, u_cur = _f64(hx), _f64(hy), _f64(u_prev), _f64(u_cur)
    f = None if f is None else _f64(f)
    ny, nx = u_cur.shape
    out = np.empty_like(u_cur)
    _load().fdwref_step(nx, ny, dx, dy, tau, _d(hx), _d(hy), _d(u_prev), _d(u_cur), _d(f), _d(out))
    return out


def energy(hx, hy, u_n, u_np1, dx, dy, tau) -> float:
    hx, hy, u_n, u_np1 = _f64(hx), _f64(hy), _f64(u_n), _f64(u_np1)
    ny, nx = u_n.shape
    return float(_load().fdwref_energy(nx, ny, dx, dy, tau, _d(hx), _d(hy), _d(u_n), _d(u_np1)))


def forward(nx: int, ny: int, dx: float, dy: float, tau: float, h1, h2, u0, u1, nsteps: int,
            want_energy: bool = False, receivers: Optional[np.ndarray] = None):
    """Forward solve; returns dict(u_prev, u_cur, energy, traces)."""
    h1 = _f64(h1)
    h2 = h1 if h2 is None else _f64(h2)
    u0, u1 = _f64(u0), _f64(u1)
    assert h1.shape == (ny, nx) and h2.shape == (ny, nx) and u0.shape == (ny, nx) and u1.shape == (ny, nx)
    e = np.empty(max(nsteps, 1)) if want_energy else None
    R = 0 if receivers is None else int(len(receivers))
    rec = None
    tr = None
    if R:
        rec = np.ascontiguousarray(receivers, dtype=np.int32)
        tr = np.empty((nsteps + 1, R))
    up = np.empty((ny, nx))
    uc = np.empty((ny, nx))
    rc = _load().fdwref_forward(nx, ny, dx, dy, tau, _d(h1), _d(h2), _d(u0), _d(u1), int(nsteps), _d(e), R,
                                None if rec is None else rec.ctypes.data_as(_IP), _d(tr), _d(up), _d(uc))
    if rc != 0:
        raise ValueError(f"fdwref_forward failed ({rc})")
    return dict(u_prev=up, u_cur=uc, energy=None if e is None else e[:nsteps], traces=tr)


def forward_case(case, nsteps: Optional[int] = None, want_energy: bool = False, receivers=None):
    n = case.nsteps if nsteps is None else nsteps
    rec = case.receivers if receivers is None else receivers
    return forward(case.nx, case.ny, case.dx, case.dy, case.tau, case.h1, case.h2, case.u0, case.u1, n,
                   want_energy=want_energy, receivers=rec)


def forward_ld(nx: int, ny: int, dx: float, dy: float, tau: float, h1, h2, u0, u1, nsteps: int,
               receivers: Optional[np.ndarray] = None, marks=()):
    """The forward definition evaluated in x87 extended precision (long double); results
    rounded to FP64.  Returns dict(u_prev, u_cur, traces, marks) with marks[k] = u^k for each
    requested step k <= nsteps."""
    h1 = _f64(h1)
    h2 = h1 if h2 is None else _f64(h2)
    u0, u1 = _f64(u0), _f64(u1)
    assert h1.shape == (ny, nx) and h2.shape == (ny, nx) and u0.shape == (ny, nx) and u1.shape == (ny, nx)
    R = 0 if receivers is None else int(len(receivers))
    rec = tr = None
    if R:
        rec = np.ascontiguousarray(receivers, dtype=np.int32)
        tr = np.empty((nsteps + 1, R))
    up = np.empty((ny, nx))
    uc = np.empty((ny, nx))
    mk = np.ascontiguousarray(sorted(set(int(k) for k in marks)), dtype=np.int64)
    assert mk.size == 0 or (mk[0] >= 0 and mk[-1] <= nsteps)
    mo = np.empty((mk.size, ny, nx)) if mk.size else None
    rc = _load().fdwref_forward_ld(nx, ny, dx, dy, tau, _d(h1), _d(h2), _d(u0), _d(u1), int(nsteps), R,
                                   None if rec is None else rec.ctypes.data_as(_IP), _d(tr), int(mk.size),
                                   mk.ctypes.data_as(ctypes.POINTER(ctypes.c_long)) if mk.size else None,
                                   None if mo is None else mo.ctypes.data_as(_DP), _d(up), _d(uc))
    if rc != 0:
        raise ValueError(f"fdwref_forward_ld failed ({rc})")
    return dict(u_prev=up, u_cur=uc, traces=tr, marks={int(k): mo[q] for q, k in enumerate(mk)})


def forward_case_ld(case, nsteps: Optional[int] = None, receivers=None, marks=()):
    n = case.nsteps if nsteps is None else nsteps
    rec = case.receivers if receivers is None else receivers
    return forward_ld(case.nx, case.ny, case.dx, case.dy, case.tau, case.h1, case.h2, case.u0, case.u1, n,
                      receivers=rec, marks=marks)


def misfit(traces: np.ndarray, d: np.ndarray) -> float:
    traces, d = _f64(traces), _f64(d)
    assert traces.shape == d.shape
    return float(_load().fdwref_misfit(traces.shape[0], traces.shape[1], _d(traces), _d(d)))


def adjoint(nx: int, ny: int, dx: float, dy: float, tau: float, h1, h2, u0, u1, nsteps: int,
            receivers: np.ndarray, trace_grad: np.ndarray, ckpt_every: int = 0, separate: bool = False):
    """Gradient of a trace loss with respect to the nodal coefficients.

    Returns dL/dh (h1 = h2 = h, summed) or, with separate=True, (dL/dh1, dL/dh2).
    """
    h1 = _f64(h1)
    h2 = h1 if h2 is None else _f64(h2)
    u0, u1 = _f64(u0), _f64(u1)
    rec = np.ascontiguousarray(receivers, dtype=np.int32)
    R = int(len(rec))
    tg = _f64(trace_grad)
    assert tg.shape == (nsteps + 1, R)
    g1 = np.empty((ny, nx))
    g2 = np.empty((ny, nx)) if separate else None
    rc = _load().fdwref_adjoint(nx, ny, dx, dy, tau, _d(h1), _d(h2), _d(u0), _d(u1), int(nsteps), R,
                                rec.ctypes.data_as(_IP), _d(tg), int(ckpt_every), _d(g1), _d(g2))
    if rc != 0:
        raise ValueError(f"fdwref_adjoint failed ({rc})")
    return (g1, g2) if separate else g1


def adi_forward(nx: int, ny: int, dx: float, dy: float, tau: float, sigma: float, h1, h2, u0, u1, nsteps: int):
    """The implicit factorized scheme (Section 3.3 / Section 4); returns dict(u_prev, u_cur)."""
    h1 = _f64(h1)
    h2 = h1 if h2 is None else _f64(h2)
    u0, u1 = _f64(u0), _f64(u1)
    assert h1.shape == (ny, nx) and h2.shape == (ny, nx) and u0.shape == (ny, nx) and u1.shape == (ny, nx)
    up = np.empty((ny, nx))
    uc = np.empty((ny, nx))
    rc = _load().fdwref_adi_forward(nx, ny, dx, dy, tau, sigma, _d(h1), _d(h2), _d(u0), _d(u1), int(nsteps),
                                    _d(up), _d(uc))
    if rc != 0:
        raise ValueError(f"fdwref_adi_forward failed ({rc})")
    return dict(u_prev=up, u_cur=uc)


def adi_forward_case(case, sigma: float = 0.25, nsteps: Optional[int] = None):
    n = case.nsteps if nsteps is None else nsteps
    return adi_forward(case.nx, case.ny, case.dx, case.dy, case.tau, sigma, case.h1, case.h2, case.u0, case.u1, n)


def tridiag(lo, di, up, rhs) -> np.ndarray:
    lo, di, up, rhs = _f64(lo), _f64(di), _f64(up), _f64(rhs)
    x = np.empty_like(rhs)
    _load().fdwref_tridiag(int(rhs.size), _d(lo), _d(di), _d(up), _d(rhs), _d(x))
    return x
