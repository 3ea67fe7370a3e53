"""Pins of the oracle's torch twin (oracle/twin.py) on the CPU.

The twin restates the step of Sec. 2D (eqs 2.19-2.23, 2.32-2.38, eq 3.10 at
the walls) in torch operations so that autograd gives the exact gradient of
the discrete map; it is the reference of the GPU adjoint.  Here it is tied
to the C oracle, which is pinned to the paper in test_oracle_pins.py, and its
autograd gradient is checked against central differences of its own forward
map.  No GPU is involved.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W

torch = pytest.importorskip("torch")
from oracle.twin import Twin  # noqa: E402


def _channel(walls_in_x, n_along=12, n_across=16):
    """Couette channel with walls on one axis only (tanh-stretched, one wall
    moving along it), the other axis periodic; seeded velocity noise."""
    case = W.couette_case(nx=n_along, ny_intervals=n_across, c=1.5, lid=0.05, nu=0.02,
                          cfl=0.6, eta=0.1)
    if walls_in_x:
        case.x, case.y = case.y.copy(), case.x.copy()
        case.periodic_x, case.periodic_y = False, True
        case.period_x, case.period_y = 0.0, 1.0
        case.u_wall = np.zeros((4, 2))
        case.u_wall[1, 1] = 0.05
    shape = (case.ny, case.nx)
    case.rho0 = np.ones(shape)
    case.ux0, case.uy0 = W.gaussian_velocity(case.nx, case.ny, std=1e-3, seed=4)
    return case


def _case(kind):
    if kind == "cavity33":
        return W.cavity_case(32, lid=0.1, re=400.0, cfl=0.9, eta=0.1, noise=1e-3, seed=3)
    if kind == "tgv20x17":
        # ragged periodic grid (no dimension a multiple of anything) and
        # non-equilibrium initial state (eq 3.5)
        return W.tgv_case(20, 17, u0=0.05, nu=0.01, cfl=0.7, eta=0.3)
    if kind == "channel_y_walls":
        return _channel(False)
    if kind == "channel_x_walls":
        return _channel(True)
    if kind == "cavity_t1s2":
        return W.cavity_case(20, lid=0.1, re=400.0, cfl=0.2, eta=0.1, noise=1e-3, seed=5,
                             A=0.0)
    raise ValueError(kind)


@pytest.mark.parametrize("kind", ["cavity33", "tgv20x17", "channel_y_walls",
                                  "channel_x_walls", "cavity_t1s2"])
def test_twin_run_equals_c_oracle(kind):
    """Twin.run (stage by stage in torch) and oracle.run (plain C) give the
    same state after 30 steps, walls and the quadratic ghost of the first
    interior node included, to 1e-14 relative (both FP64, same stage order;
    only rounding of the two codes may differ)."""
    case = _case(kind)
    phi0 = oracle.init(case)
    ref = oracle.run(case, phi0, 30)
    tw = Twin(case)
    out = tw.run(torch.from_numpy(phi0.copy()), case.nu, 30).numpy()
    err = W.rel_l2(out, ref)
    assert err <= 1e-14, err
    # a single step too, where any difference is one stage's
    one = tw.step(torch.from_numpy(phi0.copy()), oracle.CS2 / case.nu).numpy()
    assert W.rel_l2(one, oracle.run(case, phi0, 1)) <= 1e-15


def test_twin_equilibrium_init_equals_c_oracle():
    """Twin.init (f~ = f^eq(rho, u), Sec. 3) equals the C oracle's
    initialisation without the eq 3.5 correction."""
    case = W.cavity_case(16, lid=0.1, re=400.0, noise=1e-3, seed=2)
    rho = 1.0 + W.random_state((case.ny, case.nx), 1e-3, 9)
    case.rho0 = rho
    tw = Twin(case)
    phi = tw.init(torch.from_numpy(rho), torch.from_numpy(case.ux0),
                  torch.from_numpy(case.uy0)).numpy()
    ref = oracle.init(case, noneq=False)
    assert W.rel_l2(phi, ref) <= 1e-15


def test_twin_ghost_is_quadratic_at_the_wall():
    """Twin._pad: on a walled axis the point one past the wall is
    3 f_0 - 3 f_1 + f_2, so a quadratic profile continues exactly (reading of
    the missing upwind point next to a wall)."""
    case = _channel(False)
    tw = Twin(case)
    j = torch.arange(case.ny, dtype=torch.float64)
    f = (0.3 + 0.2 * j - 0.05 * j * j)[:, None].expand(case.ny, case.nx).contiguous()
    p = tw._pad(f, 0, False)
    n = case.ny
    assert float((p[1] - (0.3 - 0.2 - 0.05)).abs().max()) <= 1e-15
    assert float((p[n + 2] - (0.3 + 0.2 * n - 0.05 * n * n)).abs().max()) <= 1e-13


def _loss_fn(case, nsteps, probes, target):
    tw = Twin(case)
    rho0 = torch.ones(case.ny, case.nx, dtype=torch.float64)
    pj, pi = torch.as_tensor(probes[:, 1]), torch.as_tensor(probes[:, 0])

    def loss(u0, v0, nu):
        phi = tw.run(tw.init(rho0, u0, v0), nu, nsteps)
        _, _, u, v = Twin.moments(phi)
        return ((u[pj, pi] - target[0]) ** 2 + (v[pj, pi] - target[1]) ** 2).mean()

    return loss


@pytest.mark.parametrize("kind", ["cavity", "tgv"])
def test_twin_autograd_matches_central_differences(kind):
    """Autograd through the twin (the adjoint's reference) against
    Richardson-extrapolated central differences of the twin's forward map:
    a directional derivative with respect to the initial velocity and the
    derivative with respect to nu, after 12 steps."""
    if kind == "cavity":
        case = W.cavity_case(14, lid=0.1, re=400.0, cfl=0.9, eta=0.1, noise=0.0)
    else:
        case = W.tgv_case(16, 12, u0=0.02, nu=0.01, cfl=0.8, eta=0.1, noneq_init=False)
    nsteps = 12
    probes = W.probe_nodes(case.nx, case.ny, 8, seed=2)
    target = torch.from_numpy(W.random_state((2, 8), 0.01, 5))
    loss = _loss_fn(case, nsteps, probes, target)
    u0, v0 = W.gaussian_velocity(case.nx, case.ny, std=1e-2, seed=1)
    if kind == "tgv":
        u0, v0 = u0 + case.ux0, v0 + case.uy0
    du, dv = W.gaussian_velocity(case.nx, case.ny, std=1.0, seed=7)
    tu = torch.tensor(u0, requires_grad=True)
    tv = torch.tensor(v0, requires_grad=True)
    tnu = torch.tensor(case.nu, dtype=torch.float64, requires_grad=True)
    loss(tu, tv, tnu).backward()
    dir_ad = float((tu.grad * torch.from_numpy(du)).sum() + (tv.grad * torch.from_numpy(dv)).sum())
    nu_ad = float(tnu.grad)

    def fd(fun, h):
        return (fun(h) - fun(-h)) / (2 * h)

    def richardson(fun, h):
        return (4 * fd(fun, h / 2) - fd(fun, h)) / 3

    with torch.no_grad():
        U0, V0 = torch.from_numpy(u0), torch.from_numpy(v0)
        DU, DV = torch.from_numpy(du), torch.from_numpy(dv)
        along_u = lambda e: float(loss(U0 + e * DU, V0 + e * DV, case.nu))  # noqa: E731
        along_nu = lambda e: float(loss(U0, V0, case.nu * (1 + e))) / case.nu  # noqa: E731
        dir_fd = richardson(along_u, 1e-4)
        nu_fd = richardson(along_nu, 1e-4)
    assert abs(dir_ad - dir_fd) <= 1e-7 * abs(dir_fd), (dir_ad, dir_fd)
    assert abs(nu_ad - nu_fd) <= 1e-7 * abs(nu_fd), (nu_ad, nu_fd)
