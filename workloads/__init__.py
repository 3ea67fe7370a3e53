"""Seeded synthetic workloads: meshes, flow parameters and initial macroscopic
fields of the paper's test flows (Sec. 3).

This module holds the *problem definitions* only (node coordinates, the
physical parameters, closed-form initial and reference fields, seeded noise).
It holds none of the method's arithmetic: no equilibrium, no collision, no
difference operator, no time step.  Both the GPU library's tests and the CPU
oracle take their inputs from here; nothing else is shared between them.

Mesh maps:
  * uniform periodic axis, node-centred, N unique nodes on [lo, lo + L);
  * tanh-stretched walled axis of eq 3.9 / eq 3.11:
        y_j = (a + tanh(c mu_j)) / (2a),  a = tanh(c),  mu_j = (2j - N)/N,
    j = 0..N (N intervals, N+1 nodes, walls at 0 and 1).  The cavity uses the
    same mu_j on both axes (the printed mu_j = j/N of eq 3.11 maps [0,1] onto
    [1/2, 1], which contradicts the stated clustering at the walls).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np


@dataclasses.dataclass
class Case:
    """A flow problem on a separable Cartesian mesh.

    Arrays of the initial state are [ny][nx] in float64.  ``grad0`` is None or
    a (4, ny, nx) array (du/dx, du/dy, dv/dx, dv/dy) used by the eq 3.5
    initial non-equilibrium correction.  ``u_wall`` is (4, 2): left, right,
    bottom, top wall velocity; corner nodes take the left/right value.
    ``dt`` of None means: derive it from ``cfl`` (eq 3.1).
    """

    name: str
    x: np.ndarray
    y: np.ndarray
    periodic_x: bool
    periodic_y: bool
    period_x: float
    period_y: float
    nu: float
    cfl: float
    eta: float
    A: float = 0.5
    dt: Optional[float] = None
    force: tuple = (0.0, 0.0)
    u_wall: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros((4, 2)))
    rho0: Optional[np.ndarray] = None
    ux0: Optional[np.ndarray] = None
    uy0: Optional[np.ndarray] = None
    grad0: Optional[np.ndarray] = None
    nsteps: int = 0
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def nx(self) -> int:
        return int(self.x.shape[0])

    @property
    def ny(self) -> int:
        return int(self.y.shape[0])


# ------------------------------------------------------------------ meshes

def uniform_periodic(n: int, lo: float, length: float):
    """n node-centred coordinates lo + i*length/n, i = 0..n-1, and the period."""
    return lo + np.arange(n, dtype=np.float64) * (length / n), float(length)


def tanh_walled(n_intervals: int, c: float) -> np.ndarray:
    """Walled axis on [0, 1] clustered at both walls (eq 3.9 / eq 3.11 map)."""
    a = math.tanh(c)
    j = np.arange(n_intervals + 1, dtype=np.float64)
    mu = (2.0 * j - n_intervals) / n_intervals
    y = (a + np.tanh(c * mu)) / (2.0 * a)
    y[0], y[-1] = 0.0, 1.0
    return y


def sinusoidal_periodic(n: int, eps: float):
    """Smooth non-uniform periodic axis x = zeta + eps sin(zeta) on [0, 2pi)."""
    z = np.arange(n, dtype=np.float64) * (2.0 * math.pi / n)
    return z + eps * np.sin(z), 2.0 * math.pi


# ---------------------------------------------------------- Taylor-Green

def tgv_fields(x, y, k1, k2, u0, nu, t, rho0=1.0, cs2=1.0 / 3.0):
    """Closed form eq 3.4 on the tensor mesh: rho, u, v and the four velocity
    gradients.  The pressure part decays at twice the velocity rate (it is
    quadratic in the velocity amplitude); rho = rho0 + (p - p0)/cs2."""
    X, Y = np.meshgrid(x, y, indexing="xy")
    decay = math.exp(-nu * (k1 * k1 + k2 * k2) * t)
    u = -u0 * np.cos(k1 * X) * np.sin(k2 * Y) * decay
    v = u0 * (k1 / k2) * np.sin(k1 * X) * np.cos(k2 * Y) * decay
    dp = -(u0 * u0 / 4.0) * (np.cos(2 * k1 * X) + (k1 * k1) / (k2 * k2) * np.cos(2 * k2 * Y)) * decay * decay
    rho = rho0 + dp / cs2
    dudx = u0 * k1 * np.sin(k1 * X) * np.sin(k2 * Y) * decay
    dudy = -u0 * k2 * np.cos(k1 * X) * np.cos(k2 * Y) * decay
    dvdx = u0 * (k1 * k1 / k2) * np.cos(k1 * X) * np.cos(k2 * Y) * decay
    dvdy = -u0 * k1 * np.sin(k1 * X) * np.sin(k2 * Y) * decay
    return rho, u, v, np.stack([dudx, dudy, dvdx, dvdy])


def tgv_case(nx, ny, *, lo=0.0, length=2 * math.pi, k1=1.0, k2=1.0, u0=0.01, nu=0.01,
             cfl=0.5, eta=0.01, A=0.5, dt=None, nsteps=0, noneq_init=True, name=None):
    x, px = uniform_periodic(nx, lo, length)
    y, py = uniform_periodic(ny, lo, length)
    rho, u, v, grad = tgv_fields(x, y, k1, k2, u0, nu, 0.0)
    return Case(name=name or f"tgv{nx}x{ny}", x=x, y=y, periodic_x=True, periodic_y=True,
                period_x=px, period_y=py, nu=nu, cfl=cfl, eta=eta, A=A, dt=dt,
                rho0=rho, ux0=u, uy0=v, grad0=grad if noneq_init else None, nsteps=nsteps,
                meta=dict(k1=k1, k2=k2, u0=u0))


# ---------------------------------------------------------------- cavity

def cavity_case(n_intervals, *, c=1.5, lid=0.1, re=1000.0, cfl=0.9, eta=0.1, A=0.5,
                noise=1e-6, seed=0, nsteps=0, name=None):
    """Lid-driven cavity of height 1 on the doubly stretched mesh (eq 3.11).
    Rest state rho = 1 plus U(-noise, noise) on u and v at interior nodes
    (numpy PCG64, ``seed``).  nu = lid * 1 / Re."""
    x = tanh_walled(n_intervals, c)
    y = tanh_walled(n_intervals, c)
    n = n_intervals + 1
    rho = np.ones((n, n))
    u = np.zeros((n, n))
    v = np.zeros((n, n))
    if noise > 0:
        rng = np.random.Generator(np.random.PCG64(seed))
        u[1:-1, 1:-1] = rng.uniform(-noise, noise, size=(n - 2, n - 2))
        v[1:-1, 1:-1] = rng.uniform(-noise, noise, size=(n - 2, n - 2))
    uw = np.zeros((4, 2))
    uw[3, 0] = lid
    return Case(name=name or f"cavity{n}", x=x, y=y, periodic_x=False, periodic_y=False,
                period_x=0.0, period_y=0.0, nu=lid / re, cfl=cfl, eta=eta, A=A,
                u_wall=uw, rho0=rho, ux0=u, uy0=v, nsteps=nsteps,
                meta=dict(c=c, lid=lid, re=re))


# ------------------------------------------------------------ Poiseuille

def poiseuille_case(nx=10, ny_intervals=20, *, c=1.5, re=10.0, force=0.01, dt_over_y1=None,
                    cfl=0.1, eta=0.1, A=0.5, nsteps=0, name=None):
    """Force-driven channel of height H = 1 (eq 3.7, mesh eq 3.9): x periodic
    with nx unique nodes zeta_i = i/nx, y walled and tanh-stretched.  With
    u0 = F H^2 / (8 nu) and Re = H u0 / nu, nu = sqrt(F H^3 / (8 Re))."""
    x = np.arange(nx, dtype=np.float64) / nx
    y = tanh_walled(ny_intervals, c)
    nu = math.sqrt(force / (8.0 * re))
    n = y.shape[0]
    rho = np.ones((n, nx))
    z = np.zeros((n, nx))
    dt = None if dt_over_y1 is None else dt_over_y1 * float(y[1] - y[0])
    return Case(name=name or f"poiseuille{nx}x{n}", x=x, y=y, periodic_x=True, periodic_y=False,
                period_x=1.0, period_y=0.0, nu=nu, cfl=cfl, eta=eta, A=A, dt=dt,
                force=(force, 0.0), rho0=rho, ux0=z, uy0=z.copy(), nsteps=nsteps,
                meta=dict(u0=force / (8.0 * nu), c=c, re=re))


def couette_case(nx=8, ny_intervals=20, *, c=1.5, lid=0.01, nu=0.05, cfl=0.5, eta=0.1,
                 A=0.5, nsteps=0, name=None):
    """Plane Couette flow between a resting bottom wall (y = 0) and a top wall
    moving at ``lid`` (y = 1); x periodic.  Steady closed form u = lid * y."""
    x = np.arange(nx, dtype=np.float64) / nx
    y = tanh_walled(ny_intervals, c) if c > 0 else np.linspace(0.0, 1.0, ny_intervals + 1)
    n = y.shape[0]
    uw = np.zeros((4, 2))
    uw[3, 0] = lid
    return Case(name=name or f"couette{nx}x{n}", x=x, y=y, periodic_x=True, periodic_y=False,
                period_x=1.0, period_y=0.0, nu=nu, cfl=cfl, eta=eta, A=A, u_wall=uw,
                rho0=np.ones((n, nx)), ux0=np.zeros((n, nx)), uy0=np.zeros((n, nx)),
                nsteps=nsteps, meta=dict(lid=lid))


def poiseuille_profile(y, u0, H=1.0):
    """Closed form eq 3.7 (read y/H for the printed y/h)."""
    return 4.0 * u0 * (y / H) * (1.0 - y / H)


# -------------------------------------------------------- adjoint probes

def probe_nodes(nx, ny, count=64, seed=2):
    """``count`` distinct interior nodes (i, j), seeded (PCG64)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    flat = rng.choice((nx - 2) * (ny - 2), size=count, replace=False)
    i = 1 + flat % (nx - 2)
    j = 1 + flat // (nx - 2)
    return np.stack([i, j], axis=1).astype(np.int64)


def gaussian_velocity(nx, ny, std=1e-3, seed=1):
    """N(0, std^2) on u and v at interior nodes (PCG64)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    u = np.zeros((ny, nx))
    v = np.zeros((ny, nx))
    u[1:-1, 1:-1] = rng.normal(0.0, std, size=(ny - 2, nx - 2))
    v[1:-1, 1:-1] = rng.normal(0.0, std, size=(ny - 2, nx - 2))
    return u, v


def random_state(shape, scale, seed):
    """Seeded uniform array in [-scale, scale) (PCG64)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(-scale, scale, size=shape)


def rel_l2(a, b):
    """||a - b||_2 / ||b||_2 (eq 3.6 form)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = float(np.sqrt(np.sum(b * b)))
    return float(np.sqrt(np.sum((a - b) ** 2))) / (nb if nb > 0 else 1.0)
