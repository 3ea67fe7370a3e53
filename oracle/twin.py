"""Torch-CPU float64 twin of the oracle, for the discrete adjoint.

TEST INFRASTRUCTURE (part of the oracle; see oracle/__init__.py).  The same
time step as t2s2_oracle.c -- stage by stage in the paper's Sec. 2D order,
through the physical f -- written with torch tensor operations so that
autograd yields the exact gradient of the discrete map.  It is checked
against the C oracle (forward) and then serves as the reference for the GPU
library's hand-written adjoint.  Unforced flows; state carried as
f~ - w (offset 1).
"""
from __future__ import annotations

import math

import torch

from . import CS2, time_step

EX = torch.tensor([0, 1, 0, -1, 0, 1, -1, -1, 1], dtype=torch.float64)
EY = torch.tensor([0, 0, 1, 0, -1, 1, 1, -1, -1], dtype=torch.float64)
W = torch.tensor([4 / 9, 1 / 9, 1 / 9, 1 / 9, 1 / 9, 1 / 36, 1 / 36, 1 / 36, 1 / 36],
                 dtype=torch.float64)


def _metric(c, per, period):
    c = torch.as_tensor(c, dtype=torch.float64)
    n = c.shape[0]
    m = torch.zeros(n, dtype=torch.float64)
    for i in range(n):
        if per:
            cm = c[n - 1] - period if i == 0 else c[i - 1]
            cp = c[0] + period if i == n - 1 else c[i + 1]
        elif i == 0 or i == n - 1:
            continue
        else:
            cm, cp = c[i - 1], c[i + 1]
        m[i] = 1.0 / ((cp - cm) / 2.0)
    return m


class Twin:
    """Oracle step in torch ops for one case (mesh, walls, eta, A, dt)."""

    def __init__(self, case, A=None, eta=None, dt=None):
        self.nx, self.ny = case.nx, case.ny
        self.per_x, self.per_y = bool(case.periodic_x), bool(case.periodic_y)
        self.mx = _metric(case.x, self.per_x, case.period_x)
        self.my = _metric(case.y, self.per_y, case.period_y)
        self.dt = float(dt if dt is not None else time_step(case))
        self.A = float(case.A if A is None else A)
        self.eta = float(case.eta if eta is None else eta)
        self.uw = torch.as_tensor(case.u_wall, dtype=torch.float64).reshape(4, 2)
        ny, nx = self.ny, self.nx
        wall = torch.zeros(ny, nx, dtype=torch.bool)
        if not self.per_x:
            wall[:, 0] = True
            wall[:, -1] = True
        if not self.per_y:
            wall[0, :] = True
            wall[-1, :] = True
        self.wall = wall
        self.interior = ~wall
        # fluid neighbour and wall velocity of every wall node
        fi = torch.arange(nx).repeat(ny, 1)
        fj = torch.arange(ny).unsqueeze(1).repeat(1, nx)
        ub = torch.zeros(ny, nx, dtype=torch.float64)
        vb = torch.zeros(ny, nx, dtype=torch.float64)
        if not self.per_x:
            fi = fi.clamp(1, nx - 2)
        if not self.per_y:
            fj = fj.clamp(1, ny - 2)
        for j in range(ny):
            for i in range(nx):
                if not wall[j, i]:
                    continue
                if not self.per_x and i == 0:
                    side = 0
                elif not self.per_x and i == nx - 1:
                    side = 1
                elif not self.per_y and j == 0:
                    side = 2
                else:
                    side = 3
                ub[j, i] = self.uw[side, 0]
                vb[j, i] = self.uw[side, 1]
        self.flat_f = (fj * nx + fi).reshape(-1)
        self.ub, self.vb = ub, vb

    # -- lattice
    @staticmethod
    def moments(a, shift_fx=0.0, shift_fy=0.0):
        s = a.sum(0)
        rho = 1.0 + s
        ux = (EX[:, None, None] * a).sum(0) / rho
        uy = (EY[:, None, None] * a).sum(0) / rho
        return s, rho, ux, uy

    @staticmethod
    def feq_dev(d, rho, ux, uy):
        eu = EX[:, None, None] * ux + EY[:, None, None] * uy
        uu = ux * ux + uy * uy
        x = eu / CS2 + eu * eu / (2 * CS2 * CS2) - uu / (2 * CS2)
        return W[:, None, None] * (d + rho * x)

    # -- mixed difference along an axis (dim 2 = x, dim 1 = y)
    def _pad(self, f, dim, per):
        n = f.shape[dim]
        if per:
            lo = f.narrow(dim, n - 2, 2)
            hi = f.narrow(dim, 0, 2)
        else:
            g_lo = 3 * f.narrow(dim, 0, 1) - 3 * f.narrow(dim, 1, 1) + f.narrow(dim, 2, 1)
            g_hi = (3 * f.narrow(dim, n - 1, 1) - 3 * f.narrow(dim, n - 2, 1)
                    + f.narrow(dim, n - 3, 1))
            lo = torch.cat([g_lo, g_lo], dim)  # index -2 only feeds wall nodes
            hi = torch.cat([g_hi, g_hi], dim)
        return torch.cat([lo, f, hi], dim)

    def _d(self, f, dim, per, sign):
        p = self._pad(f, dim, per)
        n = f.shape[dim]
        fm2, fm1 = p.narrow(dim, 0, n), p.narrow(dim, 1, n)
        f0, fp1, fp2 = p.narrow(dim, 2, n), p.narrow(dim, 3, n), p.narrow(dim, 4, n)
        central = (fp1 - fm1) / 2
        if sign > 0:
            up = (3 * f0 - 4 * fm1 + fm2) / 2
        else:
            up = -(3 * f0 - 4 * fp1 + fp2) / 2
        return (1 - self.eta) * central + self.eta * up

    def L(self, a):
        out = []
        for q in range(9):
            r = torch.zeros_like(a[q])
            ex, ey = int(EX[q]), int(EY[q])
            if ex:
                r = r - ex * self.mx[None, :] * self._d(a[q], 1, self.per_x, ex)
            if ey:
                r = r - ey * self.my[:, None] * self._d(a[q], 0, self.per_y, ey)
            out.append(r)
        return torch.stack(out)

    def nee(self, a):
        """Non-equilibrium extrapolation (eq 3.10) of an unforced physical-f or
        f~ array onto the wall nodes."""
        if self.per_x and self.per_y:
            return a
        d, rho, ux, uy = self.moments(a)
        flat = a.reshape(9, -1)
        af = flat[:, self.flat_f].reshape(a.shape)
        df, rf = d.reshape(-1)[self.flat_f].reshape(d.shape), rho.reshape(-1)[self.flat_f].reshape(d.shape)
        uf = ux.reshape(-1)[self.flat_f].reshape(d.shape)
        vf = uy.reshape(-1)[self.flat_f].reshape(d.shape)
        wall_val = self.feq_dev(df, rf, self.ub, self.vb) + (af - self.feq_dev(df, rf, uf, vf))
        return torch.where(self.wall[None], wall_val, a)

    def step(self, phi, inv_tau):
        dt, h = self.dt, self.A * self.dt
        d, rho, ux, uy = self.moments(phi)
        feq = self.feq_dev(d, rho, ux, uy)
        f = (2 * phi + dt * inv_tau * feq) / (2 + dt * inv_tau)   # eq 2.19 solved for f
        om = -(f - feq) * inv_tau
        P = f + (h / 2) * om                                      # eq 2.34
        Qp = f + (dt / 2) * om                                    # eq 2.20
        S = torch.where(self.interior[None], P + h * self.L(P), P)  # eqs 2.33, 2.35
        ds, rs, us, vs = self.moments(S)
        feqs = self.feq_dev(ds, rs, us, vs)
        R = (2 * S + h * inv_tau * feqs) / (2 + h * inv_tau)     # eq 2.32
        R = self.nee(torch.where(self.interior[None], R, S))
        out = torch.where(self.interior[None], Qp + dt * self.L(R), Qp)  # eq 2.23
        return self.nee(out)

    def init(self, rho, ux, uy):
        return self.feq_dev(rho - 1.0, rho, ux, uy)

    def run(self, phi, nu, nsteps):
        inv_tau = CS2 / nu
        for _ in range(nsteps):
            phi = self.step(phi, inv_tau)
        return phi
