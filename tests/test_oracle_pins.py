"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: values the
paper prints (tests/golden), closed forms (relaxation factor, Fourier growth
factor, Taylor-Green decay, Couette profile, uniform forcing), exact
invariants (rest state, conservation), an independent implementation of
Guo's T1S2 scheme, and convergence orders.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import workloads as W
from lattice_ref import CS2, EX, EY, W as WQ

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def _paper_tgv(nx=32, ny=128, **kw):
    """Taylor vortex of Sec. 3A: [-pi, pi]^2, k1 = 1, k2 = 4, u0 = 0.01, nu = 0.001."""
    kw.setdefault("eta", 0.01)
    return W.tgv_case(nx, ny, lo=-math.pi, length=2 * math.pi, k1=1.0, k2=4.0, u0=0.01,
                      nu=0.001, **kw)


def _tc(nu=0.001, k1=1.0, k2=4.0):
    return math.log(2.0) / (nu * (k1 * k1 + k2 * k2))


def _tgv_errors(case, phi, n, dt):
    _, u, v = oracle.moments(case, phi)
    m = case.meta
    _, ua, va, _ = W.tgv_fields(case.x, case.y, m["k1"], m["k2"], m["u0"], case.nu, n * dt)
    return W.rel_l2(u, ua), W.rel_l2(v, va)


# ------------------------------------------------------------- lattice

def test_equilibrium_moments_eq_3_2():
    """f^eq of eq 3.2 on D2Q9 has moments rho, rho u, rho cs2 I + rho u u."""
    case = W.tgv_case(8, 8)
    rng = np.random.Generator(np.random.PCG64(5))
    case.rho0 = 1.0 + rng.uniform(-0.05, 0.05, (8, 8))
    case.ux0 = rng.uniform(-0.1, 0.1, (8, 8))
    case.uy0 = rng.uniform(-0.1, 0.1, (8, 8))
    case.grad0 = None
    f = oracle.init(case, offset=0.0)
    ex, ey = EX[:, None, None], EY[:, None, None]
    r = case.rho0
    np.testing.assert_allclose(f.sum(0), r, rtol=1e-15, atol=0)
    np.testing.assert_allclose((ex * f).sum(0), r * case.ux0, rtol=1e-13, atol=1e-17)
    np.testing.assert_allclose((ey * f).sum(0), r * case.uy0, rtol=1e-13, atol=1e-17)
    np.testing.assert_allclose((ex * ex * f).sum(0), r * CS2 + r * case.ux0 ** 2, rtol=1e-14)
    np.testing.assert_allclose((ex * ey * f).sum(0), r * case.ux0 * case.uy0, rtol=1e-12,
                               atol=1e-17)
    np.testing.assert_allclose((ey * ey * f).sum(0), r * CS2 + r * case.uy0 ** 2, rtol=1e-14)
    assert np.all(np.isfinite(f))


# ------------------------------------------------- P1: parameter readings

def test_time_step_and_iteration_counts_table_4():
    """xi = 1, dx_min = smallest spacing, t_c = ln2 / (nu (k1^2 + k2^2)):
    Table 4's dt (4 digits) and iteration counts are reproduced exactly."""
    g = _gold("tgv_tables.json")["table4_32x128_at_2tc"]["rows"]
    for row in g:
        case = _paper_tgv(cfl=row["cfl"])
        dt = oracle.time_step(case)
        assert abs(dt - row["dt"]) < 1e-4  # printed to 4 decimals (some truncated)
        assert int(math.floor(2.0 * _tc() / dt)) == row["iterations"]


def test_time_step_and_iteration_counts_table_8():
    """Poiseuille mesh (eq 3.9): dt = CFL * y1 and floor(20 / dt) match Table 8."""
    for row in _gold("poiseuille_table8.json")["rows"]:
        case = W.poiseuille_case(cfl=row["cfl"])
        dt = oracle.time_step(case)
        assert dt == pytest.approx(row["cfl"] * (case.y[1] - case.y[0]), rel=1e-15)
        assert abs(dt - row["dt"]) < 1e-4
        assert int(math.floor(20.0 / dt)) == row["iterations"]


# ------------------------------------------------- P2: collision algebra

@pytest.mark.parametrize("A", [0.5, 0.0])
@pytest.mark.parametrize("omega", [0.3, 1.7, 3.5])
def test_uniform_relaxation_closed_form(A, omega):
    """A uniform state relaxes as f~ - f^eq = r^n delta, r = (2 - w)/(2 + w)
    (trapezoidal collision), for a perturbation with no mass or momentum."""
    case = W.tgv_case(6, 6, nu=0.1)
    dt = omega * case.nu / CS2
    rho, ux, uy = 1.02, 0.03, -0.02
    case.rho0 = np.full((6, 6), rho)
    case.ux0 = np.full((6, 6), ux)
    case.uy0 = np.full((6, 6), uy)
    case.grad0 = None
    case.dt = dt
    feq = oracle.init(case, offset=1.0)
    delta = 1e-4 * WQ * (EX * EX - EY * EY)
    phi0 = feq + delta[:, None, None]
    n = 7
    phi = oracle.run(case, phi0, n, A=A)
    r = (2.0 - omega) / (2.0 + omega)
    expect = feq + (r ** n) * delta[:, None, None]
    # feq itself is re-evaluated every step (rounding ~1e-18 at its 1e-2 scale)
    np.testing.assert_allclose(phi - feq, expect - feq, rtol=1e-10, atol=1e-16)


# ------------------------------------- P3: advection operator and march

def _mixed_symbol(theta, s, eta):
    central = 1j * np.sin(theta)
    if s > 0:
        up = (3.0 - 4.0 * np.exp(-1j * theta) + np.exp(-2j * theta)) / 2.0
    else:
        up = -(3.0 - 4.0 * np.exp(1j * theta) + np.exp(2j * theta)) / 2.0
    return (1.0 - eta) * central + eta * up


@pytest.mark.parametrize("A,eta", [(0.5, 0.3), (0.5, 0.0), (0.0, 0.3), (0.5, 1.0)])
def test_collisionless_fourier_growth(A, eta):
    """No collision (tau -> infinity): each population is advected by
    f^{n+1} = (1 + dt L + h dt L^2) f, so a Fourier mode is multiplied by
    g = 1 + dt lam + h dt lam^2 per step, lam = -sum_a xi_a d(theta_a)/dx_a."""
    n = 16
    case = W.tgv_case(n, n, nu=math.inf, eta=eta, A=A)
    dx = 2 * math.pi / n
    dt = 0.2 * dx  # inside the stability region of the pure-upwind case
    case.dt = dt
    kx, ky = 2, 3
    X, Y = np.meshgrid(case.x, case.y, indexing="xy")
    rng = np.random.Generator(np.random.PCG64(11))
    a = 1e-3 * (rng.normal(size=9) + 1j * rng.normal(size=9))
    mode = np.exp(1j * (kx * X + ky * Y))
    phi0 = np.real(a[:, None, None] * mode[None])
    steps = 40
    phi = oracle.run(case, phi0, steps, A=A, eta=eta)
    h = A * dt
    expect = np.empty_like(phi)
    for q in range(9):
        lam = 0.0
        if EX[q]:
            lam -= EX[q] * _mixed_symbol(kx * dx, EX[q], eta) / dx
        if EY[q]:
            lam -= EY[q] * _mixed_symbol(ky * dx, EY[q], eta) / dx
        g = 1.0 + dt * lam + h * dt * lam * lam
        expect[q] = np.real(a[q] * g ** steps * mode)
    # tolerance on the initial amplitude: strongly damped modes end far below it
    np.testing.assert_allclose(phi, expect, rtol=0, atol=1e-12 * np.abs(phi0).max())


# --------------------------------------------------- P4: fixed point

@pytest.mark.parametrize("case_fn", ["tgv", "cavity", "poiseuille_noforce"])
def test_rest_state_is_exact_fixed_point(case_fn):
    """rho = 1, u = 0 stays put; in deviation storage the state is exactly 0."""
    if case_fn == "tgv":
        case = W.tgv_case(12, 10)
    elif case_fn == "cavity":
        case = W.cavity_case(10, noise=0.0)
        case.u_wall[:] = 0.0
    else:
        case = W.poiseuille_case(force=0.01)
        case.force = (0.0, 0.0)
    phi0 = np.zeros((9, case.ny, case.nx))
    phi = oracle.run(case, phi0, 25)
    assert np.count_nonzero(phi) == 0


# --------------------------------------------------- P5: conservation

def test_mass_and_momentum_conserved_on_periodic_stretched_mesh():
    """On a periodic separable mesh sum J rho and sum J (sum xi f~) are
    invariants (J = x'(i) y'(j)): the stencil weights sum to zero and the
    metric weighting telescopes."""
    x, px = W.sinusoidal_periodic(24, 0.3)
    y, py = W.sinusoidal_periodic(20, 0.25)
    case = W.tgv_case(24, 20, nu=0.02, cfl=0.5, eta=0.1)
    case.x, case.y, case.period_x, case.period_y = x, y, px, py
    rho, u, v, grad = W.tgv_fields(x, y, 1.0, 1.0, 0.03, 0.02, 0.0)
    case.rho0, case.ux0, case.uy0, case.grad0 = rho, u, v, grad
    phi0 = oracle.init(case) + W.random_state((9, 20, 24), 1e-4, 3)

    def jac(c, period):
        cm = np.roll(c, 1)
        cm[0] -= period
        cp = np.roll(c, -1)
        cp[-1] += period
        return (cp - cm) / 2.0

    J = jac(y, py)[:, None] * jac(x, px)[None, :]

    def invariants(phi):
        return (np.sum(J * phi.sum(0)), np.sum(J * (EX[:, None, None] * phi).sum(0)),
                np.sum(J * (EY[:, None, None] * phi).sum(0)))

    m0, jx0, jy0 = invariants(phi0)
    phi = oracle.run(case, phi0, 400)
    m1, jx1, jy1 = invariants(phi)
    total = np.sum(J)
    assert abs(m1 - m0) <= 1e-14 * total
    assert abs(jx1 - jx0) <= 1e-14 * total
    assert abs(jy1 - jy0) <= 1e-14 * total
    assert np.abs(phi - phi0).max() > 1e-4  # the state did evolve


# --------------------------------------------- P6: reduction to T1S2

def _t1s2_numpy(f, dx, dy, dt, tau, eta, nsteps):
    """Guo's explicit FDLBM (eqs 2.18-2.20) written directly in numpy on a
    uniform periodic grid, absolute populations."""
    ex, ey, w = EX[:, None, None], EY[:, None, None], WQ[:, None, None]

    def d(g, axis, s):
        c = (np.roll(g, -1, axis) - np.roll(g, 1, axis)) / 2.0
        if s > 0:
            up = (3 * g - 4 * np.roll(g, 1, axis) + np.roll(g, 2, axis)) / 2.0
        else:
            up = -(3 * g - 4 * np.roll(g, -1, axis) + np.roll(g, -2, axis)) / 2.0
        return (1 - eta) * c + eta * up

    for _ in range(nsteps):
        rho = f.sum(0)
        ux = (ex * f).sum(0) / rho
        uy = (ey * f).sum(0) / rho
        eu = ex * ux + ey * uy
        feq = w * rho * (1 + 3 * eu + 4.5 * eu ** 2 - 1.5 * (ux ** 2 + uy ** 2))
        fphys = (2 * tau * f + dt * feq) / (2 * tau + dt)
        fplus = ((2 * tau - dt) * f + 2 * dt * feq) / (2 * tau + dt)
        L = np.zeros_like(f)
        for q in range(9):
            if EX[q]:
                L[q] -= EX[q] * d(fphys[q], 1, EX[q]) / dx
            if EY[q]:
                L[q] -= EY[q] * d(fphys[q], 0, EY[q]) / dy
        f = fplus + dt * L
    return f


def test_A0_reduces_to_independent_t1s2():
    """Remark I: A = 0 of the general two-stage march is Guo's T1S2-FDLBM."""
    case = W.tgv_case(16, 12, u0=0.05, nu=0.02, cfl=0.25, eta=0.2, A=0.0)
    phi0 = oracle.init(case, offset=0.0)
    phi = oracle.run(case, phi0, 60, offset=0.0)
    ref = _t1s2_numpy(phi0.copy(), 2 * math.pi / 16, 2 * math.pi / 12,
                      oracle.time_step(case), oracle.tau(case), 0.2, 60)
    dev = phi - WQ[:, None, None]
    # both sides carry absolute populations (~0.44): rounding ~5e-17 per operation
    np.testing.assert_allclose(dev, ref - WQ[:, None, None], rtol=0, atol=2e-14)


def test_A_half_differs_from_t1s2():
    """Sanity: the T2S2-FDLBM1 march is not T1S2 (h = dt/2 matters)."""
    case = W.tgv_case(16, 12, u0=0.05, nu=0.02, cfl=0.25, eta=0.2)
    phi0 = oracle.init(case)
    a = oracle.run(case, phi0, 30, A=0.5)
    b = oracle.run(case, phi0, 30, A=0.0)
    assert np.abs(a - b).max() > 1e-6 * np.abs(a).max()


# ------------------------------------------------------ P7: time order

@pytest.mark.parametrize("A,lo,hi", [(0.5, 1.75, 2.25), (0.0, 0.85, 1.15)])
def test_temporal_order_by_step_halving(A, lo, hi):
    """At a fixed mesh, velocity differences between dt, dt/2, dt/4 runs to
    the same final time shrink as dt^2 for T2S2-FDLBM1 and as dt for T1S2
    (Sec. 3B, Table 6, and the temporal-order statement of Sec. 4)."""
    us = []
    for k in range(3):
        n = 400 * 2 ** k
        case = W.tgv_case(16, 16, nu=0.05, dt=10.0 / n, eta=0.01, A=A)
        phi = oracle.run(case, oracle.init(case), n)
        _, u, v = oracle.moments(case, phi)
        us.append(np.stack([u, v]))
    order = math.log2(np.linalg.norm(us[0] - us[1]) / np.linalg.norm(us[1] - us[2]))
    assert lo <= order <= hi, order


# ------------------------------------------- P8: paper worked examples

@pytest.mark.parametrize("row", [r for r in _gold("tgv_tables.json")
                                 ["table1_32x128_dt_pi_over_640_at_tc"]["rows"]
                                 if not (r["scheme"] == "T1S2" and r["eta"] != 0.01)])
def test_table_1_errors(row):
    """Table 1: E(u), E(v) of the three difference schemes at t_c; the
    printed values discriminate the reading of eta (upwind weight)."""
    A = 0.5 if row["scheme"] == "T2S2-1" else 0.0
    case = _paper_tgv(dt=math.pi / 640, eta=row["eta"], A=A)
    n = int(math.floor(_tc() / case.dt))
    phi = oracle.run(case, oracle.init(case), n, threads=8)
    eu, ev = _tgv_errors(case, phi, n, case.dt)
    assert eu == pytest.approx(row["Eu"], rel=0.05)
    assert ev == pytest.approx(row["Ev"], rel=0.05)


def test_table_2_coarse_grid():
    g = _gold("tgv_tables.json")["table2_dt_pi_over_640_at_tc"]
    case = _paper_tgv(16, 64, dt=math.pi / 640)
    n = int(math.floor(_tc() / case.dt))
    phi = oracle.run(case, oracle.init(case), n, threads=8)
    eu, _ = _tgv_errors(case, phi, n, case.dt)
    assert eu == pytest.approx(g["Eu"][0], rel=0.05)


@pytest.mark.parametrize("idx", [0, 1, 5])
def test_table_4_errors(idx):
    """Table 4 at 2 t_c: T2S2-FDLBM1 at CFL 0.8 / 0.9 and T1S2 at CFL 0.2."""
    row = _gold("tgv_tables.json")["table4_32x128_at_2tc"]["rows"][idx]
    A = 0.5 if row["scheme"] == "T2S2-1" else 0.0
    case = _paper_tgv(cfl=row["cfl"], A=A)
    dt = oracle.time_step(case)
    n = row["iterations"]
    phi = oracle.run(case, oracle.init(case), n, threads=8)
    eu, _ = _tgv_errors(case, phi, n, dt)
    assert eu == pytest.approx(row["GRE"], rel=0.10)


def test_t1s2_unstable_and_t2s2_stable_at_large_cfl():
    """Sec. 3A: T1S2 fails beyond CFL 0.3; T2S2-FDLBM1 works at CFL 0.9."""
    g = _gold("tgv_tables.json")["table3_t1s2_unstable_from_cfl"]
    case = _paper_tgv(cfl=0.6, A=0.0)
    n = int(_tc() / oracle.time_step(case))
    phi = oracle.run(case, oracle.init(case), n, threads=8)
    eu, _ = _tgv_errors(case, phi, n, oracle.time_step(case)) if np.all(np.isfinite(phi)) else (np.inf, 0)
    assert not eu < 0.1
    case = _paper_tgv(cfl=g["t2s2_stable_cfl"], A=0.5)
    n = int(_tc() / oracle.time_step(case))
    phi = oracle.run(case, oracle.init(case), n, threads=8)
    eu, _ = _tgv_errors(case, phi, n, oracle.time_step(case))
    assert eu < 0.02


# ------------------------------- P9: Taylor-Green closed form (32^2 set)

def test_tgv_second_order_convergence_and_viscosity():
    """[0, 2pi]^2, U0 = 0.01, nu = 0.01, CFL 0.5: GRE against eq 3.4 at a
    fixed time falls at second order over 16^2, 32^2, 64^2, and the energy
    decay rate gives nu within 2% on 32^2 (reading nu = cs2 tau)."""
    T = 1000 * 0.5 * 2 * math.pi / 32
    errs = []
    for n in (16, 32, 64):
        case = W.tgv_case(n, n, nu=0.01, cfl=0.5, eta=0.01)
        dt = oracle.time_step(case)
        steps = int(round(T / dt))
        phi = oracle.run(case, oracle.init(case), steps, threads=8)
        eu, _ = _tgv_errors(case, phi, steps, dt)
        errs.append(eu)
        if n == 32:
            _, u, v = oracle.moments(case, phi)
            e0 = np.sum(case.ux0 ** 2 + case.uy0 ** 2)
            nu_eff = -math.log(np.sum(u ** 2 + v ** 2) / e0) / (4.0 * steps * dt)
            assert nu_eff == pytest.approx(0.01, rel=0.02)
    assert math.log2(errs[0] / errs[1]) >= 1.7
    assert math.log2(errs[1] / errs[2]) >= 1.7


# --------------------------------------------------- walls and forcing

@pytest.mark.parametrize("eta", [0.1, 1.0])
def test_couette_flow_exact_on_uniform_mesh(eta):
    """Plane Couette flow: the non-equilibrium part is uniform, so the wall
    extrapolation (eq 3.10) and the stencils are exact; the steady state is
    u = U y to round-off."""
    case = W.couette_case(c=0.0, eta=eta, lid=0.01, nu=0.05, cfl=0.5)
    n = int(60.0 / oracle.time_step(case))
    phi = oracle.run(case, oracle.init(case), n, threads=1)
    _, u, v = oracle.moments(case, phi)
    ua = np.broadcast_to((0.01 * case.y)[:, None], u.shape)
    assert W.rel_l2(u, ua) < 1e-9
    assert np.abs(v).max() < 1e-14


def test_uniform_forcing_closed_form():
    """Uniform periodic state under a body force (eq 3.12 with the eq 3.3
    moment shift): u^n = u^0 + n dt F exactly, rho unchanged."""
    case = W.tgv_case(8, 8, nu=0.1)
    case.rho0 = np.full((8, 8), 1.0)
    case.ux0 = np.full((8, 8), 0.01)
    case.uy0 = np.full((8, 8), -0.02)
    case.grad0 = None
    case.force = (1e-3, 2e-3)
    case.dt = 0.05
    phi0 = oracle.init(case)
    _, u0, v0 = oracle.moments(case, phi0)
    phi = oracle.run(case, phi0, 100)
    d, u, v = oracle.moments(case, phi)
    assert np.abs(d).max() < 1e-15
    np.testing.assert_allclose(u, u0 + 100 * 0.05 * 1e-3, rtol=1e-12)
    np.testing.assert_allclose(v, v0 + 100 * 0.05 * 2e-3, rtol=1e-12)
    assert np.ptp(u) == 0.0 and np.ptp(v) == 0.0


def test_poiseuille_converges_to_eq_3_7():
    """Force-driven channel (eq 3.7) on the eq 3.9 mesh: the steady profile
    approaches the parabola at least at first order under refinement."""
    errs = []
    for ny in (20, 40):
        case = W.poiseuille_case(ny_intervals=ny, dt_over_y1=0.9, eta=0.1)
        prof = W.poiseuille_profile(case.y, case.meta["u0"])
        case.ux0 = np.broadcast_to(prof[:, None], (case.ny, case.nx)).copy()
        n = int(150.0 / oracle.time_step(case))
        phi = oracle.run(case, oracle.init(case), n, threads=1)
        _, u, _ = oracle.moments(case, phi)
        errs.append(W.rel_l2(u, np.broadcast_to(prof[:, None], u.shape)))
    assert errs[0] < 0.05
    assert math.log2(errs[0] / errs[1]) >= 1.0


@pytest.mark.parametrize("vwall", [0.01, -0.02])
def test_couette_flow_between_x_walls(vwall):
    """Couette flow turned by 90 degrees: walls at x = 0, 1 (the left wall
    moving along y), y periodic; steady v = V (1 - x) to round-off."""
    case = W.couette_case(c=0.0, eta=0.1, lid=0.0, nu=0.05, cfl=0.5)
    case.x, case.y = case.y.copy(), case.x.copy()
    case.periodic_x, case.periodic_y = False, True
    case.period_x, case.period_y = 0.0, 1.0
    case.rho0 = np.ones((case.ny, case.nx))
    case.ux0 = np.zeros((case.ny, case.nx))
    case.uy0 = np.zeros((case.ny, case.nx))
    case.u_wall = np.zeros((4, 2))
    case.u_wall[0, 1] = vwall
    n = int(60.0 / oracle.time_step(case))
    phi = oracle.run(case, oracle.init(case), n, threads=1)
    _, u, v = oracle.moments(case, phi)
    va = np.broadcast_to((vwall * (1.0 - case.x))[None, :], v.shape)
    assert W.rel_l2(v, va) < 1e-9
    assert np.abs(u).max() < 1e-14


def _ghost_case(eta, walls_in_x):
    """Uniform channel, collisionless (nu = inf), A = 0, resting walls on one
    axis and a periodic other axis."""
    case = W.couette_case(nx=6, ny_intervals=10, c=0.0, lid=0.0, nu=math.inf, cfl=0.4,
                          eta=eta, A=0.0)
    if walls_in_x:
        case.x, case.y = case.y.copy(), case.x.copy()
        case.periodic_x, case.periodic_y = False, True
        case.period_x, case.period_y = 0.0, 1.0
    return case


@pytest.mark.parametrize("walls_in_x", [False, True])
@pytest.mark.parametrize("eta", [1.0, 0.37])
def test_wall_adjacent_stencil_takes_the_quadratic_ghost(eta, walls_in_x):
    """The missing upwind point next to a wall (reading: quadratic ghost
    f_-1 = 3 f_0 - 3 f_1 + f_2, so the upwind difference of eq 2.38 there
    equals the central one).  Closed form of one collisionless step at A = 0
    (P = Q = f~, S = R = P, eq 2.23) from a state whose only non-zero
    populations are the two moving across the walls, equal to each other and
    varying across the channel as phi: the momentum is zero everywhere, so
    the wall extrapolation of eq 3.10 copies the first interior node onto the
    resting wall (R_0 = R_1).  For the population moving away from the wall
    at the first interior node, D = (R_2 - R_0)/2 = (phi_2 - phi_1)/2 for
    every eta; a linear ghost would give (1 - eta)(phi_2 - phi_1)/2.  The
    population moving toward that wall takes the regular upwind points
    (j + 1, j + 2).  Both walls, both axes."""
    case = _ghost_case(eta, walls_in_x)
    n_across = case.nx if walls_in_x else case.ny
    rng = np.random.Generator(np.random.PCG64(11))
    phi = rng.uniform(-1e-3, 1e-3, size=n_across)
    q_up, q_down = (1, 3) if walls_in_x else (2, 4)   # +xi and -xi across the walls
    g0 = np.zeros((9, case.ny, case.nx))
    prof = phi[None, :] if walls_in_x else phi[:, None]
    g0[q_up] = np.broadcast_to(prof, (case.ny, case.nx))
    g0[q_down] = g0[q_up]
    out = oracle.run(case, g0, 1, threads=1)
    dt = oracle.time_step(case)
    r = dt / (1.0 / (n_across - 1))   # dt / spacing, uniform mesh
    p = phi

    def across(a, j):
        return a[:, j] if walls_in_x else a[j, :]

    # bottom (or left) wall, first interior node j = 1, R_0 = R_1 = phi_1
    up_exp = p[1] - r * (p[2] - p[1]) / 2
    down_exp = p[1] + r * ((1 - eta) * (p[2] - p[1]) / 2 - eta * (3 * p[1] - 4 * p[2] + p[3]) / 2)
    np.testing.assert_allclose(across(out[q_up], 1), up_exp, rtol=0, atol=1e-17)
    np.testing.assert_allclose(across(out[q_down], 1), down_exp, rtol=0, atol=1e-17)
    # top (or right) wall, j = n - 2: mirrored, R_{n-1} = R_{n-2}
    m = n_across - 2
    down_exp = p[m] + r * (p[m] - p[m - 1]) / 2
    up_exp = p[m] - r * ((1 - eta) * (p[m] - p[m - 1]) / 2
                         + eta * (3 * p[m] - 4 * p[m - 1] + p[m - 2]) / 2)
    np.testing.assert_allclose(across(out[q_down], m), down_exp, rtol=0, atol=1e-17)
    np.testing.assert_allclose(across(out[q_up], m), up_exp, rtol=0, atol=1e-17)
    # the regular interior node j = 3 for comparison (no ghost involved)
    j = 3
    up_exp = p[j] - r * ((1 - eta) * (p[j + 1] - p[j - 1]) / 2
                         + eta * (3 * p[j] - 4 * p[j - 1] + p[j - 2]) / 2)
    np.testing.assert_allclose(across(out[q_up], j), up_exp, rtol=0, atol=1e-17)


def test_cavity_mirror_symmetry():
    """A lid moving left gives the mirror image (x -> 1 - x, u -> -u) of a lid
    moving right on the symmetric mesh: the side walls and corners are
    treated alike."""
    a = W.cavity_case(24, noise=0.0, lid=0.1, re=100.0)
    b = W.cavity_case(24, noise=0.0, lid=0.1, re=100.0)
    b.u_wall[3, 0] = -0.1
    pa = oracle.run(a, oracle.init(a), 300)
    pb = oracle.run(b, oracle.init(b), 300)
    _, ua, va = oracle.moments(a, pa)
    _, ub, vb = oracle.moments(b, pb)
    scale = np.abs(ua).max()
    assert np.abs(ub[:, ::-1] + ua).max() < 1e-12 * scale
    assert np.abs(vb[:, ::-1] - va).max() < 1e-12 * scale
    assert np.abs(va).max() > 1e-3 * scale  # the flow is two-dimensional


# ---------------------------------------------------- representation

def test_absolute_and_deviation_representations_agree():
    """offset = 0 (the paper's f~) and offset = 1 (f~ - w) give the same
    state up to FP64 rounding at the scale of w."""
    case = W.tgv_case(16, 16, u0=0.02, nu=0.02, cfl=0.6, eta=0.05)
    a = oracle.run(case, oracle.init(case, offset=0.0), 200, offset=0.0)
    b = oracle.run(case, oracle.init(case, offset=1.0), 200, offset=1.0)
    assert np.abs((a - WQ[:, None, None]) - b).max() < 1e-14


@pytest.mark.parametrize("omega,stable", [(0.46, False), (4.6, True)])
def test_tgv_cfl_09_stability_depends_on_dt_over_tau(omega, stable):
    """T2S2-FDLBM1 at CFL 0.9, eta = 0.01 on a periodic uniform grid: with
    dt / tau = 0.46 (the value a 4096^2 grid over [0, 2pi]^2 gets at
    nu = 1e-3) seeded round-off-size noise grows without bound within a few
    hundred steps; with dt / tau = 4.6 (nu = 1e-4 on 4096^2) the vortex
    decays smoothly.  The stability region of the scheme depends on tau / dt
    as well as on the CFL number (Sec. 4, von Neumann analysis); the
    throughput workload therefore runs at nu = 1e-4, same grid and work."""
    n = 64
    dt = 0.9 * 2 * math.pi / n
    nu = dt / omega * oracle.CS2
    case = W.tgv_case(n, n, u0=0.01, nu=nu, cfl=0.9, eta=0.01)
    phi = oracle.init(case) + W.random_state((9, n, n), 1e-9, 1)
    with np.errstate(all="ignore"):
        phi = oracle.run(case, phi, 400)
        _, u, v = oracle.moments(case, phi)
        umax = float(np.nanmax(np.abs(u))) if np.isfinite(u).any() else math.inf
    if stable:
        assert np.isfinite(phi).all() and umax < 0.01
    else:
        assert not np.isfinite(phi).all() or umax > 1.0


@pytest.mark.parametrize("idx", [0, 1])
def test_table_2_fdlbm2_row(idx):
    """Table 2, T2S2-FDLBM2 row (the eq 5.23 march; scheme 2 of the oracle):
    E(u) at t_c with dt = pi/640 on 16x64 and 32x128."""
    g = _gold("tgv_tables.json")["table2_fdlbm2_dt_pi_over_640_at_tc"]
    nx, ny = g["grids"][idx]
    case = _paper_tgv(nx, ny, dt=math.pi / 640)
    n = int(math.floor(_tc() / case.dt))
    phi = oracle.run(case, oracle.init(case), n, scheme=2, threads=8)
    eu, _ = _tgv_errors(case, phi, n, case.dt)
    assert eu == pytest.approx(g["Eu"][idx], rel=0.05)


def test_fdlbm2_differs_from_fdlbm1_and_reduces_with_dt():
    """The eq 5.23 march is a different scheme from eq 2.23 (their states
    differ after a few steps) and, like it, converges as dt shrinks."""
    case = W.tgv_case(24, 24, u0=0.05, nu=0.01, cfl=0.5, eta=0.05)
    phi0 = oracle.init(case)
    a = oracle.run(case, phi0, 50, scheme=1)
    b = oracle.run(case, phi0, 50, scheme=2)
    assert W.rel_l2(a, b) > 1e-6
    T = 50 * oracle.time_step(case)
    outs = []
    for k in (1, 2, 4):
        c = W.tgv_case(24, 24, u0=0.05, nu=0.01, cfl=0.5 / k, eta=0.05)
        outs.append(oracle.run(c, phi0, 50 * k, scheme=2, dt=T / (50 * k)))
    d1, d2 = W.rel_l2(outs[0], outs[1]), W.rel_l2(outs[1], outs[2])
    assert d2 < 0.6 * d1
