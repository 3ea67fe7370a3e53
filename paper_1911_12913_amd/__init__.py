"""MI355X D2Q9 T2S2-FDLBM step library: Python binding of libt2s2.so.

Argument marshalling only.  Every step of the method runs in the HIP
kernels behind the C-ABI declared in include/t2s2.h; PyTorch provides device
memory and the current HIP stream.  There is no CPU fallback: without the
built library (python -m paper_1911_12913_amd.build) or without a GPU, the
calls raise.
"""
from __future__ import annotations

import ctypes
import math
import os
from typing import Optional, Sequence

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libt2s2.so")

OK, ERR_INVALID_ARG, ERR_HIP, ERR_UNSUPPORTED, ERR_NONFINITE, ERR_NOT_BOUND = range(6)
F64, F32_DEV, BF16_DEV, F16_DEV, BF16_SR_DEV, F16_SR_DEV = range(6)
STORAGE = {"f64": F64, "f32": F32_DEV, "bf16": BF16_DEV, "f16": F16_DEV, "bf16sr": BF16_SR_DEV,
           "f16sr": F16_SR_DEV}
NDIAG = 6
DIAG_NAMES = ("mass_excess", "kinetic_energy", "max_speed", "nonfinite", "momentum_x",
              "momentum_y")
NGRE = 5
GRE_NAMES = ("sum_diff2", "sum_ref2", "sum_u2", "gre", "residual")


class T2S2Error(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"t2s2 error {code}: {msg}")
        self.code = code


class Config(ctypes.Structure):
    """Mirror of struct t2s2_config (include/t2s2.h)."""

    _fields_ = [
        ("nu", ctypes.c_double),
        ("cfl", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("eta", ctypes.c_double),
        ("A", ctypes.c_double),
        ("force", ctypes.c_double * 2),
        ("u_wall", (ctypes.c_double * 2) * 4),
        ("periodic_x", ctypes.c_int),
        ("periodic_y", ctypes.c_int),
        ("period_x", ctypes.c_double),
        ("period_y", ctypes.c_double),
        ("storage", ctypes.c_int),
        ("scheme", ctypes.c_int),
        ("btilde", ctypes.c_double * 3),
        ("bbar", ctypes.c_double * 3),
    ]


class StabilityParams(ctypes.Structure):
    """Mirror of struct t2s2_stability_params (include/t2s2.h)."""

    _fields_ = [
        ("model", ctypes.c_int),
        ("eta", ctypes.c_double),
        ("A", ctypes.c_double),
        ("b2bar", ctypes.c_double),
        ("b2tilde", ctypes.c_double),
        ("u", ctypes.c_double * 2),
        ("nk", ctypes.c_int),
        ("full_kx", ctypes.c_int),
        ("squarings", ctypes.c_int),
        ("btilde", ctypes.c_double * 3),
        ("bbar", ctypes.c_double * 3),
    ]


STAB_MODELS = {"paper": 0, "fdlbm1": 1, "fdlbm2": 2, "family": 3}

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libt2s2.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} not found: build it with "
                           "`python -m paper_1911_12913_amd.build`")
    # Load torch's HIP runtime first so the library binds to the same one
    # (two HIP runtimes in one process do not share devices or memory).
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    vp, i, d, sz, i64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t, ctypes.c_int64
    sig = {
        "t2s2_create": (i, [ctypes.POINTER(Config), vp, i, vp, i, ctypes.POINTER(vp)]),
        "t2s2_state_bytes": (sz, [vp]),
        "t2s2_workspace_bytes": (sz, [vp]),
        "t2s2_bind": (i, [vp, vp, vp, vp, vp]),
        "t2s2_init_macro": (i, [vp, vp, vp, vp, vp]),
        "t2s2_init_distributions": (i, [vp, vp]),
        "t2s2_step": (i, [vp, i64]),
        "t2s2_graph_capture": (i, [vp, i]),
        "t2s2_graph_step": (i, [vp, i64]),
        "t2s2_current": (i, [vp]),
        "t2s2_steps_taken": (i64, [vp]),
        "t2s2_dt": (d, [vp]),
        "t2s2_moments": (i, [vp, vp, vp, vp]),
        "t2s2_read_distributions": (i, [vp, vp]),
        "t2s2_diagnostics": (i, [vp, ctypes.POINTER(ctypes.c_double)]),
        "t2s2_diagnostics_noalloc": (i, [vp, vp]),
        "t2s2_velocity_error": (i, [vp, vp, vp, ctypes.POINTER(ctypes.c_double)]),
        "t2s2_stencil_weights": (i, [vp, vp, vp]),
        "t2s2_omega": (d, [vp]),
        "t2s2_adjoint_state_bytes": (sz, [vp]),
        "t2s2_adjoint_scratch_bytes": (sz, [vp]),
        "t2s2_bind_adjoint": (i, [vp, vp]),
        "t2s2_adjoint_seed_velocity": (i, [vp, vp, vp, vp, vp]),
        "t2s2_adjoint_step": (i, [vp, vp, vp, vp, vp]),
        "t2s2_step_save_s": (i, [vp, vp, vp, vp]),
        "t2s2_adjoint_step_stored": (i, [vp, vp, vp, vp, vp, vp, vp]),
        "t2s2_adjoint_init_macro": (i, [vp, vp, vp, vp, vp, vp, vp, vp]),
        "t2s2_adjoint_read": (i, [vp, vp, vp]),
        "t2s2_adjoint_load": (i, [vp, vp, vp]),
        "t2s2_stability_map": (i, [ctypes.POINTER(StabilityParams), vp, vp, i, vp, vp]),
        "t2s2_copy_probe": (i, [vp, vp, i64, i, vp]),
        "t2s2_destroy": (None, [vp]),
        "t2s2_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def exported_symbols() -> Sequence[str]:
    return ("t2s2_create", "t2s2_state_bytes", "t2s2_workspace_bytes", "t2s2_bind",
            "t2s2_init_macro", "t2s2_init_distributions", "t2s2_step", "t2s2_graph_capture",
            "t2s2_graph_step", "t2s2_current",
            "t2s2_steps_taken", "t2s2_dt", "t2s2_moments", "t2s2_read_distributions",
            "t2s2_diagnostics", "t2s2_diagnostics_noalloc", "t2s2_velocity_error", "t2s2_stencil_weights", "t2s2_omega", "t2s2_adjoint_state_bytes",
            "t2s2_adjoint_scratch_bytes", "t2s2_bind_adjoint", "t2s2_adjoint_seed_velocity",
            "t2s2_adjoint_step", "t2s2_step_save_s", "t2s2_adjoint_step_stored",
            "t2s2_adjoint_init_macro", "t2s2_adjoint_read",
            "t2s2_adjoint_load", "t2s2_stability_map", "t2s2_copy_probe", "t2s2_destroy",
            "t2s2_last_error")


def _check(rc: int):
    if rc != OK:
        msg = _lib.t2s2_last_error()
        raise T2S2Error(rc, msg.decode() if msg else "")


def make_config(*, nu: float, cfl: float = 0.0, dt: float = 0.0, eta: float = 0.01,
                A: float = 0.5, force=(0.0, 0.0), u_wall=None, periodic_x: bool = True,
                periodic_y: bool = True, period_x: float = 0.0, period_y: float = 0.0,
                storage="f64", scheme: int = 1, btilde=(0.0, 1.0, 0.0),
                bbar=(0.5, 0.0, 0.5)) -> Config:
    """scheme 1: T2S2-FDLBM1 family (A = 1/2 FDLBM1, A = 0 T1S2); scheme 2:
    T2S2-FDLBM2; scheme 3: the eq 2.13 family with gradient weights btilde
    on L(f^n), L(f*), L(f^{n+1}) and collision weights bbar on Omega(f^n),
    Omega(f*), Omega(f^{n+1})."""
    cfg = Config()
    cfg.nu = float(nu)
    cfg.cfl = float(cfl)
    cfg.dt = float(dt) if dt else 0.0
    cfg.eta = float(eta)
    cfg.A = float(A)
    cfg.force[0], cfg.force[1] = float(force[0]), float(force[1])
    if u_wall is not None:
        for s in range(4):
            cfg.u_wall[s][0] = float(u_wall[s][0])
            cfg.u_wall[s][1] = float(u_wall[s][1])
    cfg.periodic_x = int(bool(periodic_x))
    cfg.periodic_y = int(bool(periodic_y))
    cfg.period_x = float(period_x)
    cfg.period_y = float(period_y)
    cfg.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
    cfg.scheme = int(scheme)
    for k in range(3):
        cfg.btilde[k] = float(btilde[k])
        cfg.bbar[k] = float(bbar[k])
    return cfg


class Context:
    """Owns a t2s2_ctx and the torch tensors bound to it (two state buffers
    and the workspace) on one HIP device and stream.

    Stream order: the library launches on the bound stream.  Every call
    below first makes the bound stream wait for the caller's current stream
    (so inputs written there are complete), and afterwards makes the current
    stream wait for the bound stream (so returned tensors, and later work on
    the current stream, see the call's results).  Device tensors handed to
    the library are marked as used by the bound stream (record_stream), so
    the caching allocator does not reuse their memory before the bound
    stream is done with them.  With the two streams the same, this is a
    no-op."""

    def __init__(self, cfg: Config, x, y, device=None, stream=None):
        import numpy as np
        import torch

        lib = load_library()
        if not torch.cuda.is_available():
            raise RuntimeError("t2s2 needs a HIP device (torch.cuda.is_available() is False)")
        self._torch = torch
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        xs = np.ascontiguousarray(x, dtype=np.float64)
        ys = np.ascontiguousarray(y, dtype=np.float64)
        self.nx, self.ny = int(xs.shape[0]), int(ys.shape[0])
        self.cfg = cfg
        h = ctypes.c_void_p()
        _check(lib.t2s2_create(ctypes.byref(cfg), xs.ctypes.data, self.nx, ys.ctypes.data,
                               self.ny, ctypes.byref(h)))
        self._h = h
        nbytes = int(lib.t2s2_state_bytes(h))
        wbytes = int(lib.t2s2_workspace_bytes(h))
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            # torch's caching allocator returns >= 512-byte aligned blocks
            self.state = [torch.empty(nbytes, dtype=torch.uint8, device=self.device)
                          for _ in range(2)]
            self.workspace = torch.empty(wbytes, dtype=torch.uint8, device=self.device)
            cur = self._enter()
            rc = lib.t2s2_bind(h, self.state[0].data_ptr(), self.state[1].data_ptr(),
                               self.workspace.data_ptr(), self.stream.cuda_stream)
            self._leave(cur, self.state + [self.workspace])
            _check(rc)

    # -- lifetime
    def close(self):
        if getattr(self, "_h", None):
            _lib.t2s2_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- stream order
    def _enter(self):
        """Bound stream after the caller's current stream; returns the current
        stream if it differs from the bound one, else None."""
        cur = self._torch.cuda.current_stream(self.device)
        if cur.cuda_stream == self.stream.cuda_stream:
            return None
        self.stream.wait_stream(cur)
        return cur

    def _leave(self, cur, tensors=()):
        """Current stream after the bound stream; tensors used by the call are
        recorded as in use on the bound stream."""
        if cur is None:
            return
        for x in tensors:
            if x is not None:
                x.record_stream(self.stream)
        cur.wait_stream(self.stream)

    def _call(self, fn, *args, tensors=()):
        """One C-ABI call, ordered against the caller's current stream."""
        cur = self._enter()
        rc = fn(self._h, *args)
        self._leave(cur, tensors)
        _check(rc)

    # -- helpers
    def _f64(self, a, shape):
        t = self._torch
        a = t.as_tensor(a, dtype=t.float64, device=self.device).contiguous()
        if tuple(a.shape) != tuple(shape):
            raise ValueError(f"expected shape {shape}, got {tuple(a.shape)}")
        return a

    @staticmethod
    def _ptr(x):
        return x.data_ptr() if x is not None else None

    @property
    def dt(self) -> float:
        return float(_lib.t2s2_dt(self._h))

    @property
    def steps_taken(self) -> int:
        return int(_lib.t2s2_steps_taken(self._h))

    @property
    def current(self) -> int:
        return int(_lib.t2s2_current(self._h))

    # -- the C-ABI calls
    def init_macro(self, rho, ux, uy, grad=None):
        shp = (self.ny, self.nx)
        r, u, v = self._f64(rho, shp), self._f64(ux, shp), self._f64(uy, shp)
        g = self._f64(grad, (4,) + shp) if grad is not None else None
        self._call(_lib.t2s2_init_macro, r.data_ptr(), u.data_ptr(), v.data_ptr(),
                   self._ptr(g), tensors=(r, u, v, g))

    def init_distributions(self, g):
        gd = self._f64(g, (9, self.ny, self.nx))
        self._call(_lib.t2s2_init_distributions, gd.data_ptr(), tensors=(gd,))

    def step(self, n: int = 1):
        self._call(_lib.t2s2_step, int(n))

    def graph_capture(self, steps_per_graph: int):
        """Record steps_per_graph (even) steps into a HIP graph; needs the
        context to be bound to a non-default stream."""
        self._call(_lib.t2s2_graph_capture, int(steps_per_graph))

    def graph_step(self, n: int):
        self._call(_lib.t2s2_graph_step, int(n))

    def moments(self):
        t = self._torch
        out = [t.empty((self.ny, self.nx), dtype=t.float64, device=self.device) for _ in range(3)]
        self._call(_lib.t2s2_moments, *[o.data_ptr() for o in out], tensors=out)
        return tuple(out)

    def velocity_error(self, ux_ref, uy_ref) -> dict:
        """Global relative error of the velocity against a reference field
        (t2s2_velocity_error): ``gre`` = E(u) of eq 3.6 (normalised by the
        reference), ``residual`` = the Sec. 3C form (normalised by the
        current field; pass the previous output's velocity), and the sums."""
        t = self._torch
        refs = [t.as_tensor(r, dtype=t.float64, device=self.device).contiguous()
                for r in (ux_ref, uy_ref)]
        for r in refs:
            if tuple(r.shape) != (self.ny, self.nx):
                raise ValueError(f"reference field must be ({self.ny}, {self.nx})")
        out = (ctypes.c_double * NGRE)()
        self._call(_lib.t2s2_velocity_error, refs[0].data_ptr(), refs[1].data_ptr(), out,
                   tensors=refs)
        return dict(zip(GRE_NAMES, list(out)))

    def read_distributions(self):
        t = self._torch
        g = t.empty((9, self.ny, self.nx), dtype=t.float64, device=self.device)
        self._call(_lib.t2s2_read_distributions, g.data_ptr(), tensors=(g,))
        return g

    @property
    def omega(self) -> float:
        return float(_lib.t2s2_omega(self._h))

    # -- raw state buffers (checkpoint / restore)
    def state_tensor(self):
        """The bound buffer holding the current state (raw storage bytes)."""
        return self.state[self.current]

    def save_state(self):
        """A copy of the current state buffer, made on the bound stream."""
        t = self._torch
        out = t.empty_like(self.state_tensor())
        cur = self._enter()
        with t.cuda.stream(self.stream):
            out.copy_(self.state_tensor())
        self._leave(cur, (out,))
        return out

    def restore_state(self, saved):
        """Copy a saved state buffer back into the current one, on the bound
        stream."""
        t = self._torch
        cur = self._enter()
        with t.cuda.stream(self.stream):
            self.state_tensor().copy_(saved)
        self._leave(cur, (saved,))

    # -- adjoint
    def enable_adjoint(self):
        """Allocate and bind the adjoint scratch (idempotent)."""
        if getattr(self, "adjoint_scratch", None) is None:
            t = self._torch
            n = int(_lib.t2s2_adjoint_scratch_bytes(self._h))
            self.adjoint_scratch = t.empty(n, dtype=t.uint8, device=self.device)
            self._call(_lib.t2s2_bind_adjoint, self.adjoint_scratch.data_ptr(),
                       tensors=(self.adjoint_scratch,))

    def adjoint_buffer(self):
        t = self._torch
        return t.empty(int(_lib.t2s2_adjoint_state_bytes(self._h)), dtype=t.uint8,
                       device=self.device)

    def adjoint_seed_velocity(self, state, gu, gv, lam):
        shp = (self.ny, self.nx)
        gu = self._f64(gu, shp) if gu is not None else None
        gv = self._f64(gv, shp) if gv is not None else None
        self._call(_lib.t2s2_adjoint_seed_velocity, state.data_ptr(), self._ptr(gu),
                   self._ptr(gv), lam.data_ptr(), tensors=(state, gu, gv, lam))

    def adjoint_step(self, state, lam_np1, lam_n, dnu=None):
        """lam_n from lam_np1 through the step taken from `state`; adds the
        step's contribution to dL/dnu into the device scalar dnu if given."""
        self._call(_lib.t2s2_adjoint_step, state.data_ptr(), lam_np1.data_ptr(),
                   lam_n.data_ptr(), self._ptr(dnu), tensors=(state, lam_np1, lam_n, dnu))

    def step_save_s(self, src, dst, s_out):
        """One step from the state buffer src into dst, storing S into s_out
        (an adjoint_buffer())."""
        self._call(_lib.t2s2_step_save_s, src.data_ptr(), dst.data_ptr(), s_out.data_ptr(),
                   tensors=(src, dst, s_out))

    def adjoint_step_stored(self, state_n, state_np1, s_n, lam_np1, lam_n, dnu=None):
        """adjoint_step with the step's new state and S from step_save_s."""
        self._call(_lib.t2s2_adjoint_step_stored, state_n.data_ptr(), state_np1.data_ptr(),
                   s_n.data_ptr(), lam_np1.data_ptr(), lam_n.data_ptr(), self._ptr(dnu),
                   tensors=(state_n, state_np1, s_n, lam_np1, lam_n, dnu))

    def adjoint_init_macro(self, lam0, rho, ux, uy):
        t = self._torch
        shp = (self.ny, self.nx)
        r, u, v = self._f64(rho, shp), self._f64(ux, shp), self._f64(uy, shp)
        out = [t.empty(shp, dtype=t.float64, device=self.device) for _ in range(3)]
        self._call(_lib.t2s2_adjoint_init_macro, lam0.data_ptr(), r.data_ptr(), u.data_ptr(),
                   v.data_ptr(), *[o.data_ptr() for o in out],
                   tensors=[lam0, r, u, v] + out)
        return tuple(out)

    def adjoint_read(self, lam):
        t = self._torch
        out = t.empty((9, self.ny, self.nx), dtype=t.float64, device=self.device)
        self._call(_lib.t2s2_adjoint_read, lam.data_ptr(), out.data_ptr(), tensors=(lam, out))
        return out

    def adjoint_load(self, dense):
        d = self._f64(dense, (9, self.ny, self.nx))
        lam = self.adjoint_buffer()
        self._call(_lib.t2s2_adjoint_load, d.data_ptr(), lam.data_ptr(), tensors=(d, lam))
        return lam

    def diagnostics_noalloc(self, out=None):
        """t2s2_diagnostics_noalloc: the diagnostics of the current state into
        a device FP64 tensor of NDIAG values (allocated here when out is None;
        the library allocates nothing), asynchronous."""
        t = self._torch
        if out is None:
            out = t.empty(NDIAG, dtype=t.float64, device=self.device)
        if out.dtype != t.float64 or out.numel() < NDIAG or not out.is_contiguous():
            raise ValueError(f"out must be a contiguous float64 tensor of >= {NDIAG} values")
        self._call(_lib.t2s2_diagnostics_noalloc, out.data_ptr(), tensors=(out,))
        return out

    def diagnostics(self, raise_nonfinite: bool = True) -> dict:
        out = (ctypes.c_double * NDIAG)()
        cur = self._enter()
        rc = _lib.t2s2_diagnostics(self._h, out)
        self._leave(cur)
        if rc != OK and not (rc == ERR_NONFINITE and not raise_nonfinite):
            _check(rc)
        return dict(zip(DIAG_NAMES, list(out)))


def context_for_case(case, storage="f64", device=None, stream=None, **overrides) -> Context:
    """Context for a workloads.Case-like object (x, y, periodic flags, nu,
    cfl/dt, eta, A, force, u_wall), bound to `stream` (a torch stream;
    default: the current stream)."""
    kw = dict(nu=case.nu, cfl=case.cfl, dt=case.dt or 0.0, eta=case.eta, A=case.A,
              force=case.force, u_wall=case.u_wall, periodic_x=case.periodic_x,
              periodic_y=case.periodic_y, period_x=case.period_x, period_y=case.period_y,
              storage=storage)
    kw.update(overrides)
    return Context(make_config(**kw), case.x, case.y, device=device, stream=stream)


def stability_map(model, omega, r, *, eta, u=(0.0, 0.0), A=0.5, b2bar=0.5, b2tilde=0.0,
                  nk=33, full_kx=True, squarings=30, btilde=(0.0, 1.0, 0.0),
                  bbar=(0.5, 0.0, 0.5), device=None, stream=None):
    """Largest spectral radius of the growth matrix over the mode grid for
    each (omega[i], r[i]) (t2s2_stability_map); returns a device tensor."""
    import torch

    lib = load_library()
    dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    w = torch.as_tensor(omega, dtype=torch.float64, device=dev).contiguous().reshape(-1)
    rr = torch.as_tensor(r, dtype=torch.float64, device=dev).contiguous().reshape(-1)
    if w.shape != rr.shape:
        raise ValueError("omega and r must have the same number of points")
    out = torch.empty_like(w)
    prm = StabilityParams()
    prm.model = STAB_MODELS[model] if isinstance(model, str) else int(model)
    prm.eta, prm.A, prm.b2bar, prm.b2tilde = float(eta), float(A), float(b2bar), float(b2tilde)
    prm.u[0], prm.u[1] = float(u[0]), float(u[1])
    prm.nk, prm.full_kx, prm.squarings = int(nk), int(bool(full_kx)), int(squarings)
    for k in range(3):
        prm.btilde[k] = float(btilde[k])
        prm.bbar[k] = float(bbar[k])
    with torch.cuda.device(dev):
        st = stream if stream is not None else torch.cuda.current_stream(dev)
        _check(lib.t2s2_stability_map(ctypes.byref(prm), w.data_ptr(), rr.data_ptr(), w.numel(),
                                      out.data_ptr(), st.cuda_stream))
    return out


def copy_probe(src, dst, stream=None):
    """Reference copy of a nine-plane state (t2s2_copy_probe): `src` and
    `dst` are device tensors of the same dtype (8, 4 or 2 bytes per element)
    and a number of elements divisible by 9; asynchronous on `stream`."""
    import torch

    lib = load_library()
    if src.dtype != dst.dtype or src.numel() != dst.numel() or src.numel() % 9:
        raise ValueError("src and dst: same dtype and size, a multiple of 9 elements")
    if not (src.is_contiguous() and dst.is_contiguous()):
        raise ValueError("src and dst must be contiguous")
    with torch.cuda.device(src.device):
        st = stream if stream is not None else torch.cuda.current_stream(src.device)
        _check(lib.t2s2_copy_probe(src.data_ptr(), dst.data_ptr(), src.numel() // 9,
                                   src.element_size(), st.cuda_stream))
