"""FP64 CPU oracle of the T2S2-FDLBM D2Q9 step (arXiv 1911.12913).

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The GPU library
never imports, links or calls it; the two share no code.  Inputs come from
``workloads`` (problem definitions only).

The arithmetic lives in ``t2s2_oracle.c`` (plain C, materialised arrays, one
loop per stage of the paper's Sec. 2D sequence); this module builds it with
gcc, loads it through ctypes and adds the time step of eq 3.1.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "t2s2_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

XI = 1.0          # lattice speed (reading: xi = 1)
CS2 = XI * XI / 3.0


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no fast-math, no FP contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call([
            "gcc", "-std=c11", "-O2", "-fPIC", "-shared", "-fopenmp",
            "-ffp-contract=off", "-fno-fast-math", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB)
        d, i, l, p = ctypes.c_double, ctypes.c_int, ctypes.c_long, ctypes.c_void_p
        lib.oracle_run.argtypes = [i, i, p, p, i, i, d, d, d, d, d, d, d, d, p, d, i, p, l]
        lib.oracle_run.restype = i
        lib.oracle_run_family.argtypes = [i, i, p, p, i, i, d, d, d, d, d, d, d, d, p, d, p, p, p,
                                          l]
        lib.oracle_run_family.restype = i
        lib.oracle_init.argtypes = [i, i, p, p, p, p, d, d, d, p]
        lib.oracle_init.restype = i
        lib.oracle_moments.argtypes = [i, i, p, d, d, d, d, p, p, p]
        lib.oracle_moments.restype = i
        lib.oracle_set_threads.argtypes = [i]
        lib.oracle_set_threads.restype = i
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def set_threads(n: int | None) -> int:
    """Thread count of the oracle's OpenMP loops (None: leave as is); returns
    the count in effect."""
    return int(_load().oracle_set_threads(int(n) if n is not None else 0))


# ----------------------------------------------------------- parameters

def min_spacing(case) -> float:
    """Minimum node spacing over both axes, including the periodic seam."""
    out = math.inf
    for c, per, period in ((case.x, case.periodic_x, case.period_x),
                           (case.y, case.periodic_y, case.period_y)):
        d = np.diff(c)
        if per:
            d = np.append(d, c[0] + period - c[-1])
        out = min(out, float(np.min(d)))
    return out


def time_step(case) -> float:
    """eq 3.1: dt = CFL * dx_min / xi (an explicit case.dt overrides)."""
    if case.dt is not None:
        return float(case.dt)
    return case.cfl * min_spacing(case) / XI


def tau(case) -> float:
    """Relaxation time; reading nu = c_s^2 tau."""
    return case.nu / CS2


def inv_tau(case) -> float:
    return 0.0 if math.isinf(case.nu) else CS2 / case.nu


# ------------------------------------------------------------------ API

def init(case, offset: float = 1.0, noneq: bool = True) -> np.ndarray:
    """Initial state phi = f~ - offset*w, shape (9, ny, nx), from the case's
    macroscopic fields (f^eq, plus the eq 3.5 correction when grad0 is set)."""
    lib = _load()
    ny, nx = case.ny, case.nx
    rho = np.ascontiguousarray(case.rho0, dtype=np.float64)
    ux = np.ascontiguousarray(case.ux0, dtype=np.float64)
    uy = np.ascontiguousarray(case.uy0, dtype=np.float64)
    grad = None
    if noneq and case.grad0 is not None:
        grad = np.ascontiguousarray(case.grad0, dtype=np.float64)
    phi = np.empty((9, ny, nx), dtype=np.float64)
    t = tau(case) if not math.isinf(case.nu) else 0.0
    rc = lib.oracle_init(nx, ny, _ptr(rho), _ptr(ux), _ptr(uy),
                         _ptr(grad) if grad is not None else None,
                         t, time_step(case), float(offset), _ptr(phi))
    if rc != 0:
        raise ValueError(f"oracle_init failed ({rc})")
    return phi


def run(case, phi: np.ndarray, nsteps: int, *, offset: float = 1.0, scheme: int = 1,
        A: float | None = None, eta: float | None = None, dt: float | None = None,
        threads: int | None = None, btilde=None, bbar=None) -> np.ndarray:
    """Advance a copy of phi by nsteps; returns the new state.

    scheme 1: T2S2-FDLBM1 family with h = A dt (A = 0.5 default, A = 0 is
    Guo's T1S2); scheme 2: T2S2-FDLBM2; scheme 3: the eq 2.13 family with
    gradient weights btilde = (B~0, B~1, B~2) on L(f^n), L(f*), L(f^{n+1})
    and collision weights bbar = (B-0, B-1, B-2) on Omega(f^n), Omega(f*),
    Omega(f^{n+1}) (None: (1/2, 0, 1/2) in the explicit form of eqs
    2.19-2.20; a given bbar always takes the node-by-node solve of the
    implicit weight, also at (1/2, 0, 1/2))."""
    lib = _load()
    if threads is None:
        # small grids: thread start-up costs more than the stage loops
        threads = 1 if case.nx * case.ny < 16384 else (os.cpu_count() or 1)
    set_threads(threads)
    out = np.ascontiguousarray(phi, dtype=np.float64).copy()
    assert out.shape == (9, case.ny, case.nx)
    x = np.ascontiguousarray(case.x, dtype=np.float64)
    y = np.ascontiguousarray(case.y, dtype=np.float64)
    uw = np.ascontiguousarray(case.u_wall, dtype=np.float64).reshape(8)
    args = (case.nx, case.ny, _ptr(x), _ptr(y), int(case.periodic_x),
            int(case.periodic_y), float(case.period_x), float(case.period_y),
            float(dt if dt is not None else time_step(case)), inv_tau(case),
            float(case.A if A is None else A), float(case.eta if eta is None else eta),
            float(case.force[0]), float(case.force[1]), _ptr(uw), float(offset))
    if scheme == 3:
        bt = np.ascontiguousarray(btilde, dtype=np.float64).reshape(3)
        bb = None if bbar is None else np.ascontiguousarray(bbar, dtype=np.float64).reshape(3)
        rc = lib.oracle_run_family(*args, _ptr(bt), _ptr(bb) if bb is not None else None,
                                   _ptr(out), int(nsteps))
    else:
        rc = lib.oracle_run(*args, int(scheme), _ptr(out), int(nsteps))
    if rc != 0:
        raise ValueError(f"oracle_run failed ({rc})")
    return out


def moments(case, phi: np.ndarray, offset: float = 1.0, dt: float | None = None):
    """(rho - offset, u, v) of eq 3.3, each [ny][nx]."""
    lib = _load()
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    ny, nx = phi.shape[1:]
    d = np.empty((ny, nx))
    u = np.empty((ny, nx))
    v = np.empty((ny, nx))
    rc = lib.oracle_moments(nx, ny, _ptr(phi), float(offset),
                            float(dt if dt is not None else time_step(case)),
                            float(case.force[0]), float(case.force[1]),
                            _ptr(d), _ptr(u), _ptr(v))
    if rc != 0:
        raise ValueError(f"oracle_moments failed ({rc})")
    return d, u, v
