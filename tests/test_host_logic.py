"""Host logic of the library without a GPU: the stencil weights, the time
step and the relaxation parameter that t2s2_create computes on the host,
against an independent construction from the paper's formulas.

The weights are rebuilt here as the matrix of L = -dt xi d/dx on one axis:
the mixed difference of eqs 2.36-2.38 (eta the upwind weight, the upwind
side mirrored for xi < 0) applied in node-index space and scaled by the
metric 1/x'(i), x'(i) = (x[i+1] - x[i-1]) / 2 with the period added across
a periodic seam; on a walled axis the upwind point outside the domain is a
quadratic ghost, f[-1] = 3 f[0] - 3 f[1] + f[2], substituted into the
formula.  The library's tap tables must equal that matrix entry by entry.
"""
import ctypes
import math

import numpy as np
import pytest

import oracle
import paper_1911_12913_amd as t2s2
import workloads as W


def _metric(c, per, period):
    n = len(c)
    m = np.zeros(n)
    for i in range(n):
        if per:
            cm = c[i - 1] - (period if i == 0 else 0.0)
            cp = c[(i + 1) % n] + (period if i == n - 1 else 0.0)
        else:
            if i == 0 or i == n - 1:
                continue
            cm, cp = c[i - 1], c[i + 1]
        m[i] = 2.0 / (cp - cm)
    return m


def _operator(c, per, period, eta, dt, sign):
    """Dense matrix of -dt * sign * d/dx on the axis (rows of wall nodes
    zero), built by applying the difference to unit vectors."""
    n = len(c)
    m = _metric(c, per, period)
    L = np.zeros((n, n))
    for j in range(n):
        f = np.zeros(n)
        f[j] = 1.0

        def at(i):
            if per:
                return f[i % n]
            if i == -1:                      # quadratic ghost below
                return 3 * f[0] - 3 * f[1] + f[2]
            if i == n:                       # and above
                return 3 * f[n - 1] - 3 * f[n - 2] + f[n - 3]
            return f[i]

        for i in range(n):
            if not per and (i == 0 or i == n - 1):
                continue
            central = (at(i + 1) - at(i - 1)) / 2.0
            if sign > 0:
                upwind = (3 * at(i) - 4 * at(i - 1) + at(i - 2)) / 2.0
            else:
                upwind = -(3 * at(i) - 4 * at(i + 1) + at(i + 2)) / 2.0
            L[i, j] = -dt * sign * m[i] * ((1 - eta) * central + eta * upwind)
    return L


def _check_axis(w, c, per, period, eta, dt):
    n = len(c)
    w = w.reshape(n, 2, 4)
    for s, sign, offs in ((0, +1, (-2, -1, 0, 1)), (1, -1, (-1, 0, 1, 2))):
        L = _operator(c, per, period, eta, dt, sign)
        rebuilt = np.zeros((n, n))
        for i in range(n):
            for k, o in enumerate(offs):
                j = i + o
                if per:
                    j %= n
                elif not 0 <= j < n:
                    assert w[i, s, k] == 0.0
                    continue
                rebuilt[i, j] += w[i, s, k]
        scale = np.abs(L).max()
        assert np.abs(rebuilt - L).max() <= 1e-14 * scale


def _create(case, eta):
    cfg = t2s2.make_config(nu=case.nu, cfl=case.cfl, eta=eta, A=0.5,
                           periodic_x=case.periodic_x, periodic_y=case.periodic_y,
                           period_x=case.period_x, period_y=case.period_y)
    lib = t2s2.load_library()
    h = ctypes.c_void_p()
    x = np.ascontiguousarray(case.x, dtype=np.float64)
    y = np.ascontiguousarray(case.y, dtype=np.float64)
    rc = lib.t2s2_create(ctypes.byref(cfg), x.ctypes.data, len(x), y.ctypes.data, len(y),
                         ctypes.byref(h))
    assert rc == t2s2.OK
    return lib, h


def _cases():
    stretched = W.tgv_case(40, 24, u0=0.01, nu=0.01, cfl=0.7)
    stretched.x, stretched.period_x = W.sinusoidal_periodic(40, 0.3)
    return [W.cavity_case(32, lid=0.1, re=400.0, cfl=0.9), stretched,
            W.poiseuille_case(10, 20, re=10.0, force=0.01)]


@pytest.mark.parametrize("eta", [0.0, 0.01, 0.1, 1.0])
@pytest.mark.parametrize("k", range(3))
def test_stencil_weights_are_the_mixed_difference_matrix(k, eta):
    case = _cases()[k]
    lib, h = _create(case, eta)
    try:
        wx = np.empty(8 * case.nx)
        wy = np.empty(8 * case.ny)
        assert lib.t2s2_stencil_weights(h, wx.ctypes.data, wy.ctypes.data) == t2s2.OK
        dt = lib.t2s2_dt(h)
        _check_axis(wx, case.x, case.periodic_x, case.period_x, eta, dt)
        _check_axis(wy, case.y, case.periodic_y, case.period_y, eta, dt)
    finally:
        lib.t2s2_destroy(h)


@pytest.mark.parametrize("k", range(3))
def test_time_step_and_omega_follow_eq_3_1(k):
    """dt = CFL x (smallest node spacing, periodic seam included) with
    xi = 1, and omega = dt / tau with tau = 3 nu; the oracle's time step
    agrees."""
    case = _cases()[k]
    lib, h = _create(case, 0.1)
    try:
        gaps = [np.diff(case.x), np.diff(case.y)]
        if case.periodic_x:
            gaps.append([case.x[0] + case.period_x - case.x[-1]])
        if case.periodic_y:
            gaps.append([case.y[0] + case.period_y - case.y[-1]])
        dmin = min(float(np.min(g)) for g in gaps)
        dt = lib.t2s2_dt(h)
        assert dt == pytest.approx(case.cfl * dmin, rel=1e-15)
        assert dt == pytest.approx(oracle.time_step(case), rel=1e-15)
        assert lib.t2s2_omega(h) == pytest.approx(dt / (3.0 * case.nu), rel=1e-15)
    finally:
        lib.t2s2_destroy(h)


def test_stencil_weights_argument_checks():
    lib = t2s2.load_library()
    assert lib.t2s2_stencil_weights(None, None, None) == t2s2.ERR_INVALID_ARG
    case = _cases()[0]
    lib, h = _create(case, 0.1)
    try:
        assert lib.t2s2_stencil_weights(h, None, None) == t2s2.OK
    finally:
        lib.t2s2_destroy(h)


def test_bench_refuses_more_than_one_gpu(capsys):
    """bench.py runs on one GPU: --gpus above 1 exits with status 2 and a
    message, before any device call."""
    import json

    import bench

    assert bench.main(["--gpus", "2"]) == 2
    rec = json.loads(capsys.readouterr().out.strip().splitlines()[-1])
    assert rec["n_gpus"] == 2 and "one GPU" in rec["error"]
