"""C-ABI checks that need no GPU: the library loads, exports every symbol
that include/t2s2.h declares, and t2s2_create validates its arguments (it
makes no device call)."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import paper_1911_12913_amd as t2s2

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "t2s2.h")).read()
    return sorted(set(re.findall(r"\b(t2s2_[a-z_]+)\s*\(", src)))


def test_header_and_binding_agree():
    assert _declared() == sorted(t2s2.exported_symbols())


def test_library_exports_every_declared_symbol():
    lib = t2s2.load_library()
    for name in _declared():
        assert hasattr(lib, name), name


def test_config_struct_layout():
    # 5 doubles, force[2], u_wall[4][2], 2 ints, 2 doubles, 2 ints, btilde[3], bbar[3]
    assert ctypes.sizeof(t2s2.Config) == 8 * 5 + 16 + 64 + 8 + 16 + 8 + 24 + 24
    assert t2s2.Config.scheme.offset == 8 * 5 + 16 + 64 + 8 + 16 + 4
    assert t2s2.Config.btilde.offset == 8 * 5 + 16 + 64 + 8 + 16 + 8
    assert t2s2.Config.bbar.offset == 8 * 5 + 16 + 64 + 8 + 16 + 8 + 24


def test_scheme_validation():
    lib = t2s2.load_library()
    for scheme, ok in ((0, True), (1, True), (2, True), (3, True), (4, False), (-1, False)):
        rc, h = _create(_good_cfg(scheme=scheme), _axis(20), _axis(20))
        assert (rc == t2s2.OK) == ok, scheme
        if h.value:
            lib.t2s2_destroy(h)
    # the family's gradient weights (eq 2.14a and the paper's ranges)
    for bt, ok in (((0.25, 0.5, 0.25), True), ((1.0, 0.0, 0.0), True), ((0.5, 0.0, 0.5), True),
                   ((0.3, 0.3, 0.3), False), ((0.2, 0.2, 0.6), False), ((-0.1, 1.1, 0.0), False),
                   ((0.5, float("nan"), 0.5), False)):
        rc, h = _create(_good_cfg(scheme=3, btilde=bt), _axis(20), _axis(20))
        assert (rc == t2s2.OK) == ok, bt
        if h.value:
            lib.t2s2_destroy(h)
    # the family's collision weights: the same ranges; all zero is (1/2, 0, 1/2)
    for bb, ok in (((0.25, 0.5, 0.25), True), ((1.0, 0.0, 0.0), True), ((0.0, 0.0, 0.0), True),
                   ((0.0, 1.0, 0.0), True), ((0.2, 0.2, 0.2), False), ((0.0, 0.4, 0.6), False),
                   ((1.1, -0.1, 0.0), False), ((0.5, 0.0, float("nan")), False)):
        rc, h = _create(_good_cfg(scheme=3, btilde=(0.0, 1.0, 0.0), bbar=bb), _axis(20),
                        _axis(20))
        assert (rc == t2s2.OK) == ok, bb
        if h.value:
            lib.t2s2_destroy(h)
    # the other schemes ignore btilde and bbar
    rc, h = _create(_good_cfg(scheme=1, btilde=(9.0, 9.0, 9.0), bbar=(9.0, 9.0, 9.0)),
                    _axis(20), _axis(20))
    assert rc == t2s2.OK
    lib.t2s2_destroy(h)


def _create(cfg, x, y):
    lib = t2s2.load_library()
    h = ctypes.c_void_p()
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    rc = lib.t2s2_create(ctypes.byref(cfg), x.ctypes.data, x.shape[0], y.ctypes.data,
                         y.shape[0], ctypes.byref(h))
    return rc, h


def _good_cfg(**kw):
    base = dict(nu=0.01, cfl=0.5, eta=0.01, periodic_x=True, periodic_y=True,
                period_x=2 * math.pi, period_y=2 * math.pi)
    base.update(kw)
    return t2s2.make_config(**base)


def _axis(n):
    return np.arange(n) * (2 * math.pi / n)


def test_create_valid_and_sizes():
    lib = t2s2.load_library()
    rc, h = _create(_good_cfg(), _axis(100), _axis(40))
    assert rc == t2s2.OK
    assert lib.t2s2_state_bytes(h) == 9 * 40 * 128 * 8
    assert lib.t2s2_workspace_bytes(h) > 0
    assert lib.t2s2_dt(h) == pytest.approx(0.5 * 2 * math.pi / 100, rel=1e-15)
    lib.t2s2_destroy(h)
    rc, h = _create(_good_cfg(storage="bf16"), _axis(100), _axis(40))
    assert rc == t2s2.OK and lib.t2s2_state_bytes(h) == 9 * 40 * 128 * 2
    lib.t2s2_destroy(h)


@pytest.mark.parametrize("kw,x,y", [
    (dict(), _axis(4), _axis(40)),                       # n < 5
    (dict(cfl=0.0), _axis(10), _axis(10)),               # cfl <= 0
    (dict(cfl=1.5), _axis(10), _axis(10)),               # cfl > 1
    (dict(nu=0.0), _axis(10), _axis(10)),                # nu <= 0
    (dict(nu=float("nan")), _axis(10), _axis(10)),
    (dict(eta=1.5), _axis(10), _axis(10)),
    (dict(A=-0.1), _axis(10), _axis(10)),
    (dict(storage=7), _axis(10), _axis(10)),
    (dict(), _axis(10)[::-1].copy(), _axis(10)),          # not increasing
    (dict(period_x=1.0), _axis(10), _axis(10)),          # period too short
    (dict(force=(float("inf"), 0.0)), _axis(10), _axis(10)),
])
def test_create_rejects_bad_arguments(kw, x, y):
    rc, h = _create(_good_cfg(**kw), x, y)
    assert rc == t2s2.ERR_INVALID_ARG
    assert not h.value
    assert len(t2s2.load_library().t2s2_last_error()) > 0


def test_calls_on_unbound_context_fail_without_device():
    lib = t2s2.load_library()
    rc, h = _create(_good_cfg(), _axis(20), _axis(20))
    assert rc == t2s2.OK
    assert lib.t2s2_step(h, 1) == t2s2.ERR_NOT_BOUND
    assert lib.t2s2_init_distributions(h, None) == t2s2.ERR_NOT_BOUND
    assert lib.t2s2_moments(h, None, None, None) == t2s2.ERR_NOT_BOUND
    assert lib.t2s2_bind(h, None, None, None, None) == t2s2.ERR_INVALID_ARG
    assert lib.t2s2_step(None, 1) == t2s2.ERR_INVALID_ARG
    assert lib.t2s2_graph_capture(h, 2) == t2s2.ERR_NOT_BOUND
    assert lib.t2s2_graph_step(h, 4) == t2s2.ERR_NOT_BOUND
    assert lib.t2s2_graph_capture(None, 2) == t2s2.ERR_INVALID_ARG
    out = (ctypes.c_double * t2s2.NGRE)()
    assert lib.t2s2_velocity_error(h, None, None, out) == t2s2.ERR_NOT_BOUND
    assert lib.t2s2_velocity_error(None, None, None, out) == t2s2.ERR_INVALID_ARG
    assert lib.t2s2_diagnostics_noalloc(h, None) == t2s2.ERR_NOT_BOUND
    assert lib.t2s2_diagnostics_noalloc(None, None) == t2s2.ERR_INVALID_ARG
    assert lib.t2s2_step_save_s(h, None, None, None) == t2s2.ERR_NOT_BOUND
    assert lib.t2s2_step_save_s(None, None, None, None) == t2s2.ERR_INVALID_ARG
    assert lib.t2s2_adjoint_step_stored(h, None, None, None, None, None, None) == t2s2.ERR_NOT_BOUND
    assert lib.t2s2_adjoint_step_stored(None, None, None, None, None, None,
                                        None) == t2s2.ERR_INVALID_ARG
    lib.t2s2_destroy(h)


def test_oversized_plane_is_unsupported():
    """The step kernel addresses one population plane with 32-bit byte
    offsets: a plane of 4 GiB or more is refused at create."""
    lib = t2s2.load_library()
    rc, h = _create(_good_cfg(), _axis(30000), _axis(30000))
    assert rc == t2s2.ERR_UNSUPPORTED and not h.value
    rc, h = _create(_good_cfg(storage=t2s2.STORAGE["f32"]), _axis(30000), _axis(30000))
    assert rc == t2s2.OK
    lib.t2s2_destroy(h)


def test_infinite_nu_is_collisionless():
    lib = t2s2.load_library()
    rc, h = _create(_good_cfg(nu=math.inf), _axis(20), _axis(20))
    assert rc == t2s2.OK
    lib.t2s2_destroy(h)


def test_stability_map_argument_checks_without_device():
    """Invalid parameters are refused before any device call; an empty map
    is a no-op."""
    lib = t2s2.load_library()

    def prm(**kw):
        p = t2s2.StabilityParams()
        p.model, p.eta, p.A, p.b2bar, p.b2tilde = 1, 0.1, 0.5, 0.5, 0.0
        p.nk, p.full_kx, p.squarings = 9, 1, 30
        for k, v in kw.items():
            setattr(p, k, v)
        return ctypes.byref(p)

    assert lib.t2s2_stability_map(prm(), None, None, 0, None, None) == t2s2.OK
    for bad in (dict(model=4), dict(eta=1.5), dict(A=-0.1), dict(nk=1), dict(nk=2000),
                dict(squarings=0), dict(squarings=61), dict(b2bar=math.nan)):
        assert lib.t2s2_stability_map(prm(**bad), None, None, 4, None, None) == t2s2.ERR_INVALID_ARG
    assert lib.t2s2_stability_map(prm(), None, None, 4, None, None) == t2s2.ERR_INVALID_ARG
    assert lib.t2s2_stability_map(None, None, None, 4, None, None) == t2s2.ERR_INVALID_ARG
    fam = t2s2.StabilityParams()
    fam.model, fam.eta, fam.A, fam.nk, fam.full_kx, fam.squarings = 3, 0.1, 0.5, 9, 1, 30
    fam.btilde[0], fam.btilde[1], fam.btilde[2] = 0.25, math.inf, 0.25
    assert lib.t2s2_stability_map(ctypes.byref(fam), None, None, 4, None, None) == t2s2.ERR_INVALID_ARG
    fam.btilde[1] = 0.5
    fam.bbar[0], fam.bbar[1], fam.bbar[2] = 0.25, math.nan, 0.25
    assert lib.t2s2_stability_map(ctypes.byref(fam), None, None, 4, None, None) == t2s2.ERR_INVALID_ARG
    fam.bbar[1] = 0.5   # valid: fails only on the NULL arrays
    assert lib.t2s2_stability_map(ctypes.byref(fam), None, None, 4, None, None) == t2s2.ERR_INVALID_ARG
    assert lib.t2s2_stability_map(ctypes.byref(fam), None, None, 0, None, None) == t2s2.OK


def test_copy_probe_argument_checks_without_device():
    """The reference copy refuses NULL, misaligned and overlapping buffers,
    empty planes and other element sizes before any device call."""
    lib = t2s2.load_library()
    a, b = 1 << 20, 1 << 30   # addresses never dereferenced: every call fails its checks
    bad = t2s2.ERR_INVALID_ARG
    assert lib.t2s2_copy_probe(None, b, 16, 8, None) == bad
    assert lib.t2s2_copy_probe(a, None, 16, 8, None) == bad
    assert lib.t2s2_copy_probe(a, b, 0, 8, None) == bad
    assert lib.t2s2_copy_probe(a, b, -5, 8, None) == bad
    assert lib.t2s2_copy_probe(a, b, 16, 3, None) == bad
    assert lib.t2s2_copy_probe(a, b, 16, 16, None) == bad
    assert lib.t2s2_copy_probe(a + 4, b, 16, 8, None) == bad
    assert lib.t2s2_copy_probe(a, a + 9 * 16 * 8 - 8, 16, 8, None) == bad   # overlap
    assert lib.t2s2_copy_probe(a + 9 * 16 * 8 - 8, a, 16, 8, None) == bad
    assert b"overlap" in lib.t2s2_last_error()
