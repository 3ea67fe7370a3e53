"""Pins of the von Neumann oracle (oracle/stability.py, Sec. 2C).

Each check ties the growth matrices to something other than themselves: an
independently typed equilibrium, closed forms (Crank-Nicolson relaxation at
k = 0, the Taylor polynomial of the collisionless march, the Cayley form of
the B~2 = B-2 = 1/2 member), the linear response of the C oracle's actual
step, the TGV stability finding, and the paper's statement on which member
of the family has the largest stable region (Fig. 1 itself is not in the
text available here).
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from lattice_ref import CS2, EX, EY
from lattice_ref import W as WQ
from oracle import stability as S


def _feq(f):
    rho = f.sum()
    ux, uy = (EX * f).sum() / rho, (EY * f).sum() / rho
    eu = EX * ux + EY * uy
    uu = ux * ux + uy * uy
    return WQ * rho * (1 + eu / CS2 + eu ** 2 / (2 * CS2 ** 2) - uu / (2 * CS2))


@pytest.mark.parametrize("u", [(0.0, 0.0), (0.2, 0.2), (0.05, -0.11)])
def test_gamma_is_the_jacobian_of_the_equilibrium(u):
    f0 = WQ * (1 + (EX * u[0] + EY * u[1]) / CS2
               + (EX * u[0] + EY * u[1]) ** 2 / (2 * CS2 ** 2) - (u[0] ** 2 + u[1] ** 2) / (2 * CS2))
    h = 1e-6
    J = np.zeros((9, 9))
    for j in range(9):
        e = np.zeros(9)
        e[j] = h
        J[:, j] = (_feq(f0 + e) - _feq(f0 - e)) / (2 * h)
    G = S.gamma(u)
    assert np.abs(G - J).max() < 1e-8
    assert np.abs(G @ G - G).max() < 1e-13   # f^eq(f^eq(f)) = f^eq(f)


@pytest.mark.parametrize("model", ["fdlbm1", "fdlbm2", "paper"])
@pytest.mark.parametrize("omega", [0.3, 1.0, 4.6])
def test_zero_mode_relaxes_like_crank_nicolson(model, omega):
    """At k = 0 the advection symbol vanishes: three conserved modes stay
    (eigenvalue 1) and the other six relax by (2 - w)/(2 + w)."""
    G = S.growth(model, 0.0, 0.0, omega, 0.7, eta=0.1, u=(0.2, 0.2), B2bar=0.5)
    ev = np.sort(np.abs(np.linalg.eigvals(G)))
    cn = abs((2 - omega) / (2 + omega))
    expect = np.sort(np.array([1.0] * 3 + [cn] * 6))
    assert np.allclose(ev, expect, atol=1e-10)


@pytest.mark.parametrize("model,A", [("fdlbm1", 0.5), ("fdlbm1", 0.0), ("fdlbm2", None)])
def test_collisionless_growth_is_the_taylor_polynomial(model, A):
    """omega = 0: each population is advected on its own, by
    1 - r s + A (r s)^2 (A = 1/2 for FDLBM2's Heun-type predictor)."""
    th = (0.7, -1.9)
    s = S.symbol(*th, 0.2)
    r = 0.6
    G = S.growth(model, *th, 0.0, r, eta=0.2, u=(0.1, 0.0), A=A if A is not None else 0.5)
    a = 0.5 if A is None else A
    assert np.allclose(G, np.diag(1 - r * s + a * (r * s) ** 2), atol=1e-14)


@pytest.mark.parametrize("eta", [0.0, 0.1])
def test_crank_nicolson_member_never_amplifies(eta):
    """B~2 = B-2 = 1/2 in eq 4.7: Crank-Nicolson in both collision and
    advection; no mode grows for any r and omega."""
    worst = 0.0
    for omega in (0.1, 0.5, 1.0, 2.0, 5.0, 20.0):
        for r in (0.1, 0.5, 0.9, 1.5, 3.0):
            worst = max(worst, S.max_radius("paper", omega, r, 9, eta=eta, u=(0.2, 0.2),
                                            B2bar=0.5, B2tilde=0.5))
    assert worst <= 1.0 + 1e-12


@pytest.mark.parametrize("scheme", [1, 2])
def test_exact_growth_matrix_is_the_linearised_oracle_step(scheme):
    """The C oracle's step on a periodic uniform 16x16 grid, linearised by
    central differences about a uniform state and projected on a Fourier
    mode, equals the growth matrix of the implemented scheme."""
    n, mode = 16, (2, 3)
    nu = 0.02
    case = W.tgv_case(n, n, u0=0.0, nu=nu, cfl=0.6, eta=0.15)
    ux, uy = 0.05, -0.03
    case.ux0 = np.full((n, n), ux)
    case.uy0 = np.full((n, n), uy)
    case.rho0 = np.ones((n, n))
    case.grad0 = None
    phi0 = oracle.init(case, noneq=False)
    dx = 2 * math.pi / n
    dt = oracle.time_step(case)
    omega = dt / (nu / CS2)
    r = dt / dx
    th = (2 * math.pi * mode[0] / n, 2 * math.pi * mode[1] / n)
    i = np.arange(n)
    phase = np.exp(1j * (th[0] * i[None, :] + th[1] * i[:, None]))  # [y][x]
    eps = 1e-7
    Gfd = np.zeros((9, 9), dtype=np.complex128)
    for j in range(9):
        w = np.zeros((9, n, n))
        w[j] = np.real(phase)   # e_j cos(k.x): half of it rides on +k
        out_p = oracle.run(case, phi0 + eps * w, 1, scheme=scheme)
        out_m = oracle.run(case, phi0 - eps * w, 1, scheme=scheme)
        resp = (out_p - out_m) / (2 * eps)
        Gfd[:, j] = 2 * (resp * np.conj(phase)[None]).sum(axis=(1, 2)) / (n * n)
    model = "fdlbm1" if scheme == 1 else "fdlbm2"
    G = S.growth(model, *th, omega, r, eta=0.15, u=(ux, uy), A=0.5)
    assert np.abs(Gfd - G).max() < 1e-7


def _full_k_max(model, omega, r, nk, **kw):
    ths = np.linspace(-math.pi, math.pi, 2 * nk - 1)
    thy = np.linspace(0.0, math.pi, nk)
    return max(S.spectral_radius(S.growth(model, a, b, omega, r, **kw)) for a in ths for b in thy)


def test_exact_model_predicts_the_tgv_cfl_09_finding():
    """The growth matrix of the implemented FDLBM1 step has a growing mode at
    r = 0.9, eta = 0.01, dt/tau = 0.46 and none at dt/tau = 4.6 (the oracle
    runs of test_tgv_cfl_09_stability_depends_on_dt_over_tau)."""
    kw = dict(eta=0.01, u=(0.01, 0.01), A=0.5)
    assert _full_k_max("fdlbm1", 0.46, 0.9, 17, **kw) > 1.0 + 1e-4
    assert _full_k_max("fdlbm1", 4.6, 0.9, 17, **kw) <= 1.0 + 1e-12


def test_fdlbm2_unstable_where_fdlbm1_is_stable_at_cfl_09():
    """At the 4096^2 throughput setting (r = 0.9, eta = 0.01, dt/tau = 4.6)
    the exact growth matrix of the eq 5.23 step has a growing mode and the
    FDLBM1 one has none; the oracle agrees on a 64^2 Taylor-Green grid with
    the same r and dt/tau: T2S2-FDLBM2 blows up within 1500 steps, FDLBM1
    decays."""
    kw = dict(eta=0.01, u=(0.01, 0.01))
    assert _full_k_max("fdlbm2", 4.6, 0.9, 17, **kw) > 1.0 + 1e-3
    assert _full_k_max("fdlbm1", 4.6, 0.9, 17, A=0.5, **kw) <= 1.0 + 1e-12
    n = 64
    case = W.tgv_case(n, n, u0=0.01, nu=1.0, cfl=0.9, eta=0.01)
    case.nu = oracle.time_step(case) / 4.6 * CS2
    phi0 = oracle.init(case) + W.random_state((9, n, n), 1e-9, 3)
    a = oracle.run(case, phi0, 1500, scheme=1)
    b = oracle.run(case, phi0, 1500, scheme=2)
    assert np.isfinite(a).all() and np.abs(a).max() < np.abs(phi0).max()
    assert not (np.isfinite(b).all() and np.abs(b).max() < 1.0)


def test_largest_stable_region_is_the_crank_nicolson_member():
    """Sec. 2C: among the Fig. 1 settings, B-2 = 1/2, B~2 = 1/2, eta = 0.1
    gives the largest stable region in the (r, omega) plane (u = (0.2, 0.2),
    k dchi in [0, pi]^2)."""
    settings = [(0.5, 0.0, 0.1), (0.25, 0.0, 0.1), (0.0, 0.0, 0.1),
                (0.5, 0.5, 0.1), (0.5, 0.25, 0.1), (0.5, 0.0, 0.0), (0.5, 0.0, 1.0)]
    omegas = np.linspace(0.2, 3.0, 8)
    rs = np.linspace(0.1, 1.5, 8)
    area = {}
    for b2bar, b2t, eta in settings:
        area[(b2bar, b2t, eta)] = sum(
            S.max_radius("paper", w, r, 7, eta=eta, u=(0.2, 0.2), B2bar=b2bar, B2tilde=b2t)
            <= 1.0 + 1e-9 for w in omegas for r in rs)
    best = area[(0.5, 0.5, 0.1)]
    assert best == len(omegas) * len(rs)
    assert all(best >= a for a in area.values())
