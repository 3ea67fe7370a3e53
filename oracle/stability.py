"""Von Neumann analysis of the T2S2-FDLBM (Sec. 2C, eqs 4.1-4.8): CPU oracle.

TEST INFRASTRUCTURE (part of the oracle; see oracle/__init__.py).  Plain
numpy, FP64/complex128, one (k, omega, r) point at a time; the eigenvalues
come from numpy.linalg.eigvals.

The growth matrix G(k) of a perturbation f' e^{i k.x} about the global
equilibrium f^eq(rho = 1, u) (eq 4.4) is built two ways:

* ``paper``: eq 4.7 for the (B~2, B-2) family with the eq 4.8 symbol S of
  the mixed difference;
* ``fdlbm1`` / ``fdlbm2`` / ``family``: the exact linearisation of the
  implemented steps (the eq 2.23 march with h = A dt, the eq 5.23 march, and
  the eq 2.13 family with gradient weights B~ and collision weights B-),
  composed from the Jacobians of the pointwise maps and the difference
  symbol:
      fdlbm1:  G = J_Q - rS J_R (I - A rS) J_P
      fdlbm2:  G = J_Q - (rS / 2) [J_f + J_R1 (I - rS) J_Q]
      family:  G = J_Q - rS [B~0 J_f + B~1 J_R (I - A rS) J_P + B~2 J_R1 (I - rS) J_Q]
  with J_X = c_Xg I + c_Xe Gamma (the coefficients of the P, Q, R maps);
  the family with B- other than (1/2, 0, 1/2) adds the explicit collision
  terms and solves the implicit one (growth_family).

Readings (listed in the design notes):
* eq 4.8 is printed with the imaginary unit missing from two exponentials;
  the symbol of dx xi_q . D is  l(1 - eta)(sin th_x + sin th_y)
  + eta/2 [6 - 4 e^{-l th_x} - 4 e^{-l th_y} + e^{-2 l th_x} + e^{-2 l th_y}],
  l^2 = -1, th_a = kappa_a xi_qa dchi (the symbol of the mixed difference
  of eqs 2.36-2.38, eta the upwind weight);
* Gamma_ij = d f^eq_i / d f_j at rho = 1 and velocity u (through the
  moments of eq 3.3, unforced);
* in eq 4.7 the symbol multiplies from the left (it acts on the population
  it advects), as the derivation from eq 4.3 gives;
* r = dt / dx with dx the uniform spacing, xi = 1.
"""
from __future__ import annotations

import numpy as np

EX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], dtype=np.float64)
EY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], dtype=np.float64)
W = np.array([4 / 9, 1 / 9, 1 / 9, 1 / 9, 1 / 9, 1 / 36, 1 / 36, 1 / 36, 1 / 36])


def gamma(u):
    """Gamma_ij = d f^eq_i / d f_j at rho = 1, velocity u (eq 3.2, c_s^2 =
    1/3): f^eq depends on f through rho = sum f and m = sum xi f."""
    ux, uy = float(u[0]), float(u[1])
    eu = EX * ux + EY * uy
    uu = ux * ux + uy * uy
    d_rho = W * (1.0 - 4.5 * eu * eu + 1.5 * uu)         # d f^eq_i / d rho at fixed m
    d_mx = W * (3.0 * EX + 9.0 * eu * EX - 3.0 * ux)      # d f^eq_i / d m_x
    d_my = W * (3.0 * EY + 9.0 * eu * EY - 3.0 * uy)
    return d_rho[:, None] + d_mx[:, None] * EX[None, :] + d_my[:, None] * EY[None, :]


def symbol(theta_x, theta_y, eta):
    """Diagonal of S (eq 4.8, reading above): dx * symbol of xi_q . D for the
    nine directions at the mode (theta_x, theta_y) = k dchi."""
    s = np.zeros(9, dtype=np.complex128)
    for q in range(9):
        for th in (theta_x * EX[q], theta_y * EY[q]):
            s[q] += 1j * (1.0 - eta) * np.sin(th) + 0.5 * eta * (
                3.0 - 4.0 * np.exp(-1j * th) + np.exp(-2j * th))
    return s


def coefficients(A, omega):
    """Coefficients of the pointwise maps (collision transforms of the step,
    eqs 2.19-2.34): P = cPg f~ + cPe f^eq, Q = cQg f~ + cQe f^eq,
    R = cRs S + cRe f^eq(S)."""
    w = omega
    return dict(cPg=(2 - A * w) / (2 + w), cPe=(1 + A) * w / (2 + w),
                cQg=(2 - w) / (2 + w), cQe=2 * w / (2 + w),
                cRs=2 / (2 + A * w), cRe=A * w / (2 + A * w))


def growth_paper(theta_x, theta_y, omega, r, B2bar, B2tilde, eta, u):
    """Eq 4.7, with the advection symbol applied to the population it
    advects: xi_i . grad f^eq_i = xi_i . Gamma_ij grad f_j gives r S Gamma
    (S on the left; eq 4.7 prints the product the other way round)."""
    I = np.eye(9)
    G = gamma(u)
    rS = r * np.diag(symbol(theta_x, theta_y, eta))
    lhs = ((1 + omega * B2bar) * I + omega * (0.5 - 2 * B2bar) * G
           + rS @ (B2tilde * I + (0.5 - B2tilde) * G))
    rhs = ((1 - omega * (1 - B2bar)) * I + omega * (1.5 - 2 * B2bar) * G
           - rS @ ((1 - B2tilde) * I - (0.5 - B2tilde) * G))
    return np.linalg.solve(lhs, rhs)


def growth_fdlbm1(theta_x, theta_y, omega, r, A, eta, u):
    """Exact linearisation of the eq 2.23 step (h = A dt)."""
    I = np.eye(9)
    G = gamma(u)
    c = coefficients(A, omega)
    JP = c["cPg"] * I + c["cPe"] * G
    JQ = c["cQg"] * I + c["cQe"] * G
    JR = c["cRs"] * I + c["cRe"] * G
    rS = r * np.diag(symbol(theta_x, theta_y, eta))
    return JQ - rS @ JR @ (I - A * rS) @ JP


def growth_fdlbm2(theta_x, theta_y, omega, r, eta, u):
    """Exact linearisation of the eq 5.23 step: f~^{n+1} = Q + dt/2 (L(f^n)
    + L(f^{n+1})), f^{n+1} from S = Q + dt L(Q) unshifted with h = dt."""
    I = np.eye(9)
    G = gamma(u)
    c0, c1 = coefficients(0.0, omega), coefficients(1.0, omega)
    Jf = c0["cPg"] * I + c0["cPe"] * G
    JQ = c0["cQg"] * I + c0["cQe"] * G
    JR = c1["cRs"] * I + c1["cRe"] * G
    rS = r * np.diag(symbol(theta_x, theta_y, eta))
    return JQ - 0.5 * rS @ (Jf + JR @ (I - rS) @ JQ)


def growth_family(theta_x, theta_y, omega, r, A, btilde, eta, u, bbar=None):
    """Exact linearisation of the eq 2.13 family step with gradient weights
    btilde on L(f^n), L(f*), L(f^{n+1}).  With the collision weights of
    eqs 2.21 and 5.21 (bbar None):
        G = J_Q - rS [B~0 J_f + B~1 J_R(A) (I - A rS) J_P + B~2 J_R(1) (I - rS) J_Q].
    With collision weights bbar = (B-0, B-1, B-2), the right side of eq 2.13
    (dt Omega = w (Gamma - I) f, unforced)
        Y = J_f + w (Gamma - I) [B-0 J_f + B-1 J_R(A) (I - A rS) J_P] - rS [...]
    is solved for f^{n+1} from [(1 + B-2 w) I - B-2 w Gamma] f^{n+1} = Y, and
    the state is f~ = [(1 + w/2) I - (w/2) Gamma] f^{n+1} (eq 2.19)."""
    I = np.eye(9)
    G = gamma(u)
    c, c0, c1 = coefficients(A, omega), coefficients(0.0, omega), coefficients(1.0, omega)
    JP = c["cPg"] * I + c["cPe"] * G
    JQ = c["cQg"] * I + c["cQe"] * G
    JR = c["cRs"] * I + c["cRe"] * G
    Jf = c0["cPg"] * I + c0["cPe"] * G
    JR1 = c1["cRs"] * I + c1["cRe"] * G
    rS = r * np.diag(symbol(theta_x, theta_y, eta))
    b0, b1, b2 = btilde
    Jstar = JR @ (I - A * rS) @ JP
    grad = rS @ (b0 * Jf + b1 * Jstar + b2 * JR1 @ (I - rS) @ JQ)
    if bbar is None:
        return JQ - grad
    c0b, c1b, c2b = bbar
    w = omega
    Y = Jf + w * (G - I) @ (c0b * Jf + c1b * Jstar) - grad
    f_next = np.linalg.solve((1 + c2b * w) * I - c2b * w * G, Y)
    return ((1 + w / 2) * I - (w / 2) * G) @ f_next


def growth(model, theta_x, theta_y, omega, r, *, eta, u, A=0.5, B2bar=0.5, B2tilde=0.0,
           btilde=(0.0, 1.0, 0.0), bbar=None):
    if model == "paper":
        return growth_paper(theta_x, theta_y, omega, r, B2bar, B2tilde, eta, u)
    if model == "fdlbm1":
        return growth_fdlbm1(theta_x, theta_y, omega, r, A, eta, u)
    if model == "fdlbm2":
        return growth_fdlbm2(theta_x, theta_y, omega, r, eta, u)
    if model == "family":
        return growth_family(theta_x, theta_y, omega, r, A, btilde, eta, u, bbar)
    raise ValueError(model)


def spectral_radius(G):
    return float(np.max(np.abs(np.linalg.eigvals(G))))


def k_grid(nk):
    """nk x nk modes with kappa dchi in [0, pi] on both axes (Sec. 2C)."""
    th = np.linspace(0.0, np.pi, nk)
    return [(a, b) for a in th for b in th]


def max_radius(model, omega, r, nk, **kw):
    """max over the k grid of the spectral radius of G."""
    return max(spectral_radius(growth(model, a, b, omega, r, **kw)) for a, b in k_grid(nk))
