"""GPU adjoint: per-step dot-product test, agreement with the oracle twin's
autograd, and the sqrt(N)-checkpointed rollout gradient against central
finite differences (FP64)."""
import math
import time

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
t2s2 = pytest.importorskip("paper_1911_12913_amd")
from paper_1911_12913_amd.rollout import RolloutSpec, T2S2Rollout, forward_velocity  # noqa: E402


def _spec(case, nsteps, storage="f64", checkpoint_every=None):
    return RolloutSpec(x=case.x, y=case.y, periodic_x=case.periodic_x,
                       periodic_y=case.periodic_y, period_x=case.period_x,
                       period_y=case.period_y, cfl=case.cfl, dt=case.dt or 0.0, eta=case.eta,
                       A=case.A, u_wall=case.u_wall, storage=storage, nsteps=nsteps,
                       checkpoint_every=checkpoint_every, device="cuda:0")


def _dev(a):
    return torch.as_tensor(np.asarray(a), dtype=torch.float64, device="cuda:0")


def _settle(fn, seconds=0.5):
    """Run fn repeatedly for about `seconds` (the GPU clocks come up after
    an idle or a host upload) before a timed run."""
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        for _ in range(10):
            fn()
        torch.cuda.synchronize()


def _one_walled_axis(walls_in_x):
    """Couette channel of 70 x 81 nodes (two strips across): walls on one axis only
    (tanh-stretched, one wall moving along it), the other axis periodic,
    so the adjoint's wall frame is rows only or columns only."""
    case = W.couette_case(nx=70, ny_intervals=80, c=1.5, lid=0.05, nu=0.02, cfl=0.6,
                          eta=0.1)
    if walls_in_x:
        case.x, case.y = case.y.copy(), case.x.copy()
        case.periodic_x, case.periodic_y = False, True
        case.period_x, case.period_y = 0.0, 1.0
        case.u_wall = np.zeros((4, 2))
        case.u_wall[1, 1] = 0.05
    n = (case.ny, case.nx)
    case.rho0 = np.ones(n)
    case.ux0, case.uy0 = W.gaussian_velocity(case.nx, case.ny, std=1e-3, seed=4)
    return case


@pytest.mark.parametrize("kind", ["cavity", "tgv", "cavity_t1s2", "channel_y_walls",
                                  "channel_x_walls"])
def test_adjoint_step_dot_product(kind):
    """<J v, w> = <v, J^T w> for one step: J v by central differences of the
    GPU step, J^T w by the hand-written adjoint step.  At A = 0 the step runs
    the single-stencil kernel and the adjoint's recompute the two-stencil
    one, so the test also ties the two forward kernels together.  The two
    channels have walls on one axis only."""
    if kind == "cavity":
        case = W.cavity_case(40, lid=0.1, re=400.0, cfl=0.9, eta=0.1, noise=1e-3, seed=1)
    elif kind == "cavity_t1s2":
        case = W.cavity_case(40, lid=0.1, re=400.0, cfl=0.25, eta=0.1, noise=1e-3, seed=1)
        case.A = 0.0
    elif kind.startswith("channel"):
        case = _one_walled_axis(kind == "channel_x_walls")
    else:
        case = W.tgv_case(48, 40, u0=0.05, nu=0.01, cfl=0.6, eta=0.05)
    print(f"[gpu] adjoint dot product {kind}", flush=True)
    ctx = t2s2.context_for_case(case)
    ctx.enable_adjoint()
    g0 = oracle.run(case, oracle.init(case), 20)
    v = W.random_state(g0.shape, 1.0, 21)
    w = W.random_state(g0.shape, 1.0, 22)
    eps = 1e-6 * np.abs(g0).max()

    def step_from(g):
        ctx.init_distributions(torch.from_numpy(g))
        ctx.step(1)
        return ctx.read_distributions().cpu().numpy()

    jv = (step_from(g0 + eps * v) - step_from(g0 - eps * v)) / (2 * eps)
    ctx.init_distributions(torch.from_numpy(g0))
    state = ctx.save_state()
    lam_w = ctx.adjoint_load(w)
    lam_out = ctx.adjoint_buffer()
    ctx.adjoint_step(state, lam_w, lam_out)
    jtw = ctx.adjoint_read(lam_out).cpu().numpy()
    lhs, rhs = float(np.sum(jv * w)), float(np.sum(v * jtw))
    print(f"    <Jv,w> {lhs:.12e}  <v,J^T w> {rhs:.12e}", flush=True)
    assert abs(lhs - rhs) <= 1e-8 * abs(rhs)


@pytest.mark.parametrize("kind", ["cavity", "tgv", "channel_y_walls", "channel_x_walls"])
def test_fp32_adjoint_step_dot_product(kind):
    """<J v, w> = <v, J^T w> for one FP32-storage step (FP32 arithmetic, FP64
    moment sums): J v by central differences of the GPU step, taken along
    the perturbation that survives the rounding of the two perturbed states
    to FP32 (read back from the library), J^T w by the FP32 adjoint step.
    The difference quotient of an FP32 map carries FP32 rounding of the two
    stepped states over 2 eps (about 3e-5 of the product here, where the
    FP32 J^T w itself is within 1e-5 of the FP64 one), hence 1e-4."""
    if kind == "cavity":
        case = W.cavity_case(40, lid=0.1, re=400.0, cfl=0.9, eta=0.1, noise=1e-3, seed=1)
    elif kind.startswith("channel"):
        case = _one_walled_axis(kind == "channel_x_walls")
    else:
        case = W.tgv_case(48, 40, u0=0.05, nu=0.01, cfl=0.6, eta=0.05)
    print(f"[gpu] fp32 adjoint dot product {kind}", flush=True)
    ctx = t2s2.context_for_case(case, storage="f32")
    ctx.enable_adjoint()
    g0 = oracle.run(case, oracle.init(case), 20)
    v = W.random_state(g0.shape, 1.0, 21)
    w = W.random_state(g0.shape, 1.0, 22)
    eps = 1e-3 * np.abs(g0).max()

    def load(g):
        ctx.init_distributions(torch.from_numpy(g))
        return ctx.read_distributions().cpu().numpy()  # as stored (FP32)

    def step_from(g):
        ctx.init_distributions(torch.from_numpy(g))
        ctx.step(1)
        return ctx.read_distributions().cpu().numpy()

    gp, gm = load(g0 + eps * v), load(g0 - eps * v)
    dv = (gp - gm) / (2 * eps)
    jv = (step_from(gp) - step_from(gm)) / (2 * eps)
    ctx.init_distributions(torch.from_numpy(g0))
    state = ctx.save_state()
    lam_w = ctx.adjoint_load(w)
    lam_out = ctx.adjoint_buffer()
    ctx.adjoint_step(state, lam_w, lam_out)
    jtw = ctx.adjoint_read(lam_out).cpu().numpy()
    w32 = ctx.adjoint_read(lam_w).cpu().numpy()  # w as the FP32 adjoint holds it
    lhs, rhs = float(np.sum(jv * w32)), float(np.sum(dv * jtw))
    print(f"    <Jv,w> {lhs:.9e}  <v,J^T w> {rhs:.9e}  rel {abs(lhs - rhs) / abs(rhs):.2e}",
          flush=True)
    assert abs(lhs - rhs) <= 1e-4 * abs(rhs)


@pytest.mark.parametrize("kind", ["cavity", "tgv", "channel_y_walls", "channel_x_walls"])
def test_fp32_adjoint_step_matches_fp64_adjoint_step(kind):
    """The FP32 adjoint step (its stages' algebra in FP32) against the FP64
    one on the same state and adjoint (both exactly representable in FP32):
    lambda_n and the step's dL/dnu agree to FP32 rounding."""
    if kind == "cavity":
        case = W.cavity_case(60, lid=0.1, re=400.0, cfl=0.9, eta=0.1, noise=1e-3, seed=1)
    elif kind.startswith("channel"):
        case = _one_walled_axis(kind == "channel_x_walls")
    else:
        case = W.tgv_case(150, 97, u0=0.05, nu=0.01, cfl=0.6, eta=0.05)
    print(f"[gpu] fp32 vs fp64 adjoint step {kind}", flush=True)
    g0 = oracle.run(case, oracle.init(case), 15).astype(np.float32).astype(np.float64)
    w = W.random_state(g0.shape, 1.0, 24).astype(np.float32).astype(np.float64)
    outs = {}
    for storage in ("f64", "f32"):
        ctx = t2s2.context_for_case(case, storage=storage)
        ctx.enable_adjoint()
        ctx.init_distributions(torch.from_numpy(g0))
        state = ctx.save_state()
        lam_w = ctx.adjoint_load(w)
        lam_out = ctx.adjoint_buffer()
        acc = torch.zeros(1, dtype=torch.float64, device="cuda:0")
        ctx.adjoint_step(state, lam_w, lam_out, acc)
        outs[storage] = (ctx.adjoint_read(lam_out).cpu().numpy(), float(acc.item()))
        ctx.close()
    e_l = W.rel_l2(outs["f32"][0], outs["f64"][0])
    e_nu = abs(outs["f32"][1] - outs["f64"][1]) / abs(outs["f64"][1])
    print(f"    lambda_n rel L2 {e_l:.2e}  dL/dnu rel {e_nu:.2e}", flush=True)
    assert e_l < 1e-5 and e_nu < 1e-3



def _round_16bit(g, storage):
    """Deviations rounded to the values the 16-bit form stores exactly (BF16:
    to nearest even on the FP32 bits; FP16: 2^14 g to the nearest FP16)."""
    if storage == "bf16":
        u = g.astype(np.float32).view(np.uint32).astype(np.uint64)
        u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
        return u.astype(np.uint32).view(np.float32).astype(np.float64)
    return (g * 16384.0).astype(np.float16).astype(np.float64) / 16384.0


@pytest.mark.parametrize("storage", ["bf16", "f16"])
def test_adjoint_16bit_storage_is_the_fp32_adjoint(storage):
    """On a periodic grid the adjoint step reads the state only through the
    storage type and keeps lambda in FP32 for every reduced form, so with a
    state that the 16-bit form holds exactly the BF16 and FP16 adjoints give
    the FP32-storage adjoint's lambda_n and dL/dnu bit for bit (150 x 70
    Taylor-Green, ragged strips)."""
    case = W.tgv_case(150, 70, k1=2.0, k2=1.0, u0=0.02, nu=0.005, cfl=0.6, eta=0.05)
    print(f"[gpu] 16-bit adjoint vs FP32 adjoint {storage}", flush=True)
    g = _round_16bit(oracle.run(case, oracle.init(case) + W.random_state((9, 70, 150), 1e-5, 31),
                                10), storage)
    w = W.random_state(g.shape, 1.0, 32).astype(np.float32).astype(np.float64)
    outs = {}
    for st in (storage, "f32"):
        ctx = t2s2.context_for_case(case, storage=st)
        ctx.enable_adjoint()
        ctx.init_distributions(torch.from_numpy(g))
        state = ctx.save_state()
        lam_w = ctx.adjoint_load(w)
        lam_out = ctx.adjoint_buffer()
        acc = torch.zeros(1, dtype=torch.float64, device="cuda:0")
        ctx.adjoint_step(state, lam_w, lam_out, acc)
        outs[st] = (ctx.adjoint_read(lam_out).cpu().numpy(), float(acc.item()),
                    ctx.read_distributions().cpu().numpy())
        ctx.close()
    assert np.array_equal(outs[storage][2], g) and np.array_equal(outs["f32"][2], g)
    print(f"    lambda_n bitwise {np.array_equal(outs[storage][0], outs['f32'][0])}, "
          f"dL/dnu {outs[storage][1]!r} vs {outs['f32'][1]!r}", flush=True)
    assert np.array_equal(outs[storage][0], outs["f32"][0])
    assert outs[storage][1] == outs["f32"][1]

@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_adjoint_march_block_shapes_agree(storage, monkeypatch):
    """The reverse march with blocks of four waves and of eight (forced with
    T2S2_ADJ_ROWS) gives bitwise the same lambda_n, and dL/dnu to
    round-off (the blocks' partials are summed in another grouping), on a
    walled cavity, a ragged periodic grid and the two one-walled-axis
    channels."""
    cases = [W.cavity_case(200, lid=0.1, re=400.0, cfl=0.9, eta=0.1, noise=1e-3, seed=3),
             W.tgv_case(150, 97, u0=0.05, nu=0.01, cfl=0.6, eta=0.05),
             _one_walled_axis(False), _one_walled_axis(True)]
    for case in cases:
        print(f"[gpu] adjoint block shapes {case.name} {case.nx}x{case.ny} {storage}", flush=True)
        w = W.random_state((9, case.ny, case.nx), 1.0, 23)
        outs = []
        for rows in ("4", "8"):
            monkeypatch.setenv("T2S2_ADJ_ROWS", rows)
            ctx = t2s2.context_for_case(case, storage=storage)
            ctx.enable_adjoint()
            ctx.init_macro(case.rho0, case.ux0, case.uy0)
            ctx.step(5)
            state = ctx.save_state()
            lam_w = ctx.adjoint_load(w)
            lam_out = ctx.adjoint_buffer()
            acc = torch.zeros(1, dtype=torch.float64, device="cuda:0")
            ctx.adjoint_step(state, lam_w, lam_out, acc)
            outs.append((ctx.adjoint_read(lam_out).cpu().numpy(), float(acc.item())))
            ctx.close()
        assert np.array_equal(outs[0][0], outs[1][0])
        assert abs(outs[0][1] - outs[1][1]) <= 1e-12 * abs(outs[1][1])


@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("kind", ["cavity", "tgv", "cavity_t1s2"])
def test_stored_adjoint_step_is_the_recomputing_one(kind, storage):
    """t2s2_step_save_s gives the state t2s2_step gives (bitwise; at A = 0,
    where it runs the two-stencil kernel, to rounding), and
    t2s2_adjoint_step_stored on its outputs gives bitwise the lambda_n and
    dL/dnu of t2s2_adjoint_step."""
    if kind == "tgv":
        case = W.tgv_case(48, 40, u0=0.05, nu=0.01, cfl=0.6, eta=0.05)
    else:
        case = W.cavity_case(60, lid=0.1, re=400.0, cfl=0.9, eta=0.1, noise=1e-3, seed=1)
    if kind == "cavity_t1s2":
        case.cfl, case.A = 0.25, 0.0
    print(f"[gpu] stored adjoint step {kind} {storage}", flush=True)
    ctx = t2s2.context_for_case(case, storage=storage)
    ctx.enable_adjoint()
    ctx.init_macro(case.rho0, case.ux0, case.uy0)
    ctx.step(7)
    state = ctx.save_state()
    nxt, s_n = torch.empty_like(state), ctx.adjoint_buffer()
    ctx.step_save_s(state, nxt, s_n)
    ctx.step(1)
    ref = ctx.read_distributions().cpu().numpy()
    ctx.restore_state(nxt)
    got = ctx.read_distributions().cpu().numpy()
    if case.A == 0.0:
        assert W.rel_l2(got, ref) < (1e-15 if storage == "f64" else 1e-6)
    else:
        assert np.array_equal(got, ref)
    lam_w = ctx.adjoint_load(W.random_state((9, case.ny, case.nx), 1.0, 31))
    outs = []
    for stored in (False, True):
        lam_out = ctx.adjoint_buffer()
        acc = torch.zeros(1, dtype=torch.float64, device="cuda:0")
        if stored:
            ctx.adjoint_step_stored(state, nxt, s_n, lam_w, lam_out, acc)
        else:
            ctx.adjoint_step(state, lam_w, lam_out, acc)
        outs.append((ctx.adjoint_read(lam_out).cpu().numpy(), float(acc.item())))
    assert np.array_equal(outs[0][0], outs[1][0])
    assert outs[0][1] == outs[1][1]
    ctx.close()


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_rollout_backward_with_stored_steps(storage):
    """The rollout's two backward passes (steps and S kept per segment, or
    the step recomputed inside each adjoint step) give the same gradients:
    bitwise, since both form every state and S with the same kernels."""
    case = W.cavity_case(64, lid=0.1, re=400.0, cfl=0.9, eta=0.1, noise=0.0)
    print(f"[gpu] rollout backward stored vs recomputed {storage}", flush=True)
    probes = W.probe_nodes(case.nx, case.ny, 16, seed=2)
    pj = torch.as_tensor(probes[:, 1], device="cuda:0")
    pi = torch.as_tensor(probes[:, 0], device="cuda:0")
    rho0 = _dev(np.ones((case.ny, case.nx)))
    u0, v0 = W.gaussian_velocity(case.nx, case.ny, std=1e-3, seed=1)
    grads = []
    for store in (True, False):
        spec = _spec(case, 130, storage=storage)
        spec.store_s = store
        gu, gv = _dev(u0).requires_grad_(True), _dev(v0).requires_grad_(True)
        gnu = torch.tensor(case.nu, dtype=torch.float64, device="cuda:0", requires_grad=True)
        U, V = T2S2Rollout.apply(rho0, gu, gv, gnu, spec)
        (U[pj, pi] ** 2 + V[pj, pi] ** 2).sum().backward()
        grads.append((gu.grad.cpu().numpy(), gv.grad.cpu().numpy(), gnu.grad.item()))
    assert np.array_equal(grads[0][0], grads[1][0])
    assert np.array_equal(grads[0][1], grads[1][1])
    assert grads[0][2] == grads[1][2]


def test_adjoint_matches_oracle_twin_autograd():
    """Gradients of a probe loss after 40 steps of a 33x33 cavity w.r.t. the
    initial velocity field and nu: GPU adjoint vs autograd through the
    oracle's torch twin."""
    from oracle.twin import Twin

    case = W.cavity_case(32, lid=0.1, re=400.0, cfl=0.9, eta=0.1, noise=0.0)
    nsteps = 40
    ux0, uy0 = W.gaussian_velocity(case.nx, case.ny, std=1e-3, seed=1)
    rho0 = np.ones((case.ny, case.nx))
    probes = W.probe_nodes(case.nx, case.ny, 16, seed=2)
    ut = W.random_state((2, 16), 0.02, 5)

    # oracle twin + autograd
    tw = Twin(case)
    tu = torch.tensor(ux0, requires_grad=True)
    tv = torch.tensor(uy0, requires_grad=True)
    tnu = torch.tensor(case.nu, dtype=torch.float64, requires_grad=True)
    phi = tw.run(tw.init(torch.tensor(rho0), tu, tv), tnu, nsteps)
    _, _, u, v = Twin.moments(phi)
    pj, pi = torch.as_tensor(probes[:, 1]), torch.as_tensor(probes[:, 0])
    loss = ((u[pj, pi] - torch.tensor(ut[0])) ** 2 + (v[pj, pi] - torch.tensor(ut[1])) ** 2).mean()
    loss.backward()

    # GPU rollout + hand-written adjoint
    spec = _spec(case, nsteps, checkpoint_every=7)
    gu = _dev(ux0).requires_grad_(True)
    gv = _dev(uy0).requires_grad_(True)
    gnu = torch.tensor(case.nu, dtype=torch.float64, device="cuda:0", requires_grad=True)
    U, V = T2S2Rollout.apply(_dev(rho0), gu, gv, gnu, spec)
    pjd, pid = pj.to("cuda:0"), pi.to("cuda:0")
    loss_g = ((U[pjd, pid] - _dev(ut[0])) ** 2 + (V[pjd, pid] - _dev(ut[1])) ** 2).mean()
    loss_g.backward()
    e_loss = abs(loss_g.item() - loss.item()) / abs(loss.item())
    e_u = W.rel_l2(gu.grad.cpu().numpy(), tu.grad.numpy())
    e_v = W.rel_l2(gv.grad.cpu().numpy(), tv.grad.numpy())
    e_nu = abs(gnu.grad.item() - tnu.grad.item()) / abs(tnu.grad.item())
    print(f"    loss {e_loss:.2e}  dL/du0 {e_u:.2e}  dL/dv0 {e_v:.2e}  dL/dnu {e_nu:.2e}",
          flush=True)
    assert e_loss < 1e-11 and e_u < 1e-9 and e_v < 1e-9 and e_nu < 1e-9


def _cavity513():
    """Differentiation workload: cavity on the 513 x 513 stretched mesh, Re 400."""
    return W.cavity_case(512, lid=0.1, re=400.0, cfl=0.9, eta=0.1, noise=0.0)


def _probe_loss_fn(case, nsteps, storage):
    """Loss = mean over 64 seeded interior probes of |u - u_target|^2, the
    targets from a reference run with nu_ref = 1.05 nu and no initial
    perturbation."""
    probes = W.probe_nodes(case.nx, case.ny, 64, seed=2)
    pj = torch.as_tensor(probes[:, 1], device="cuda:0")
    pi = torch.as_tensor(probes[:, 0], device="cuda:0")
    zero = np.zeros((case.ny, case.nx))
    rho0 = _dev(np.ones((case.ny, case.nx)))
    spec = _spec(case, nsteps, storage=storage)
    ut, vt = forward_velocity(spec, rho0, _dev(zero), _dev(zero), 1.05 * case.nu)
    ut, vt = ut[pj, pi].clone(), vt[pj, pi].clone()

    def loss_of(U, V):
        return ((U[pj, pi] - ut) ** 2 + (V[pj, pi] - vt) ** 2).mean()

    return spec, rho0, loss_of


@pytest.mark.parametrize("nsteps", [2000])
def test_rollout_gradient_vs_central_differences_fp64(nsteps):
    """dL/dnu and the directional derivative along a seeded direction of the
    initial velocity, adjoint vs Richardson-extrapolated central differences,
    FP64, 513x513 cavity, Re 400, CFL 0.9, N = 2000 with sqrt(N)
    checkpoints: relative agreement 1e-6."""
    case = _cavity513()
    print(f"[gpu] rollout gradient 513x513, {nsteps} steps", flush=True)
    spec, rho0, loss_of = _probe_loss_fn(case, nsteps, "f64")
    u0, v0 = W.gaussian_velocity(case.nx, case.ny, std=1e-3, seed=1)
    du, dv = W.gaussian_velocity(case.nx, case.ny, std=1e-3, seed=7)
    gu = _dev(u0).requires_grad_(True)
    gv = _dev(v0).requires_grad_(True)
    gnu = torch.tensor(case.nu, dtype=torch.float64, device="cuda:0", requires_grad=True)
    U, V = T2S2Rollout.apply(rho0, gu, gv, gnu, spec)
    L0 = loss_of(U, V)
    L0.backward()
    adj_dir = float(torch.sum(gu.grad * _dev(du)) + torch.sum(gv.grad * _dev(dv)))
    adj_nu = gnu.grad.item()

    def L_at(s_dir, nu):
        U, V = forward_velocity(spec, rho0, _dev(u0 + s_dir * du), _dev(v0 + s_dir * dv), nu)
        return loss_of(U, V).item()

    def richardson(f, h):
        d1 = (f(h) - f(-h)) / (2 * h)
        d2 = (f(h / 2) - f(-h / 2)) / h
        return (4 * d2 - d1) / 3

    fd_dir = richardson(lambda s: L_at(s, case.nu), 0.02)
    fd_nu = richardson(lambda s: L_at(0.0, case.nu + s), 1e-3 * case.nu)
    e_dir = abs(adj_dir - fd_dir) / abs(fd_dir)
    e_nu = abs(adj_nu - fd_nu) / abs(fd_nu)
    print(f"    L {L0.item():.6e}  dir adj {adj_dir:.10e} fd {fd_dir:.10e} rel {e_dir:.2e}",
          flush=True)
    print(f"    nu  adj {adj_nu:.10e} fd {fd_nu:.10e} rel {e_nu:.2e}", flush=True)
    assert e_dir < 1e-6 and e_nu < 1e-6


@pytest.mark.parametrize("nsteps", [200, 2000])
def test_fp32_adjoint_against_fp64_adjoint(nsteps):
    """The FP32 rollout gradient of the 513x513 workload (at N = 2000 the
    differentiation configuration itself: FP32, sqrt(N) checkpoints),
    reported against the FP64 one, with the wall time of the FP32 rollout
    (forward and backward)."""
    case = _cavity513()
    grads = {}
    for storage in ("f64", "f32"):
        spec, rho0, loss_of = _probe_loss_fn(case, nsteps, storage)
        u0, v0 = W.gaussian_velocity(case.nx, case.ny, std=1e-3, seed=1)
        gu = _dev(u0).requires_grad_(True)
        gv = _dev(v0).requires_grad_(True)
        gnu = torch.tensor(case.nu, dtype=torch.float64, device="cuda:0", requires_grad=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        U, V = T2S2Rollout.apply(rho0, gu, gv, gnu, spec)
        loss_of(U, V).backward()
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        grads[storage] = (gu.grad.cpu().numpy(), gv.grad.cpu().numpy(), gnu.grad.item())
        print(f"    {storage} rollout of {nsteps} steps, forward + backward: {secs:.3f} s",
              flush=True)
    e_u = W.rel_l2(np.stack(grads["f32"][:2]), np.stack(grads["f64"][:2]))
    e_nu = abs(grads["f32"][2] - grads["f64"][2]) / abs(grads["f64"][2])
    print(f"    FP32 vs FP64 adjoint, {nsteps} steps: dL/du0 rel L2 {e_u:.2e}, "
          f"dL/dnu rel {e_nu:.2e}", flush=True)
    # the FP32 forward trajectory itself drifts from the FP64 one with N
    tol = 1e-3 if nsteps <= 200 else 1e-2
    assert e_u < tol and e_nu < tol


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_adjoint_step_time_513(storage):
    """Time of one adjoint step (which recomputes the forward step it
    reverses) against one forward step, 513^2 cavity; reported."""
    case = _cavity513()
    ctx = t2s2.context_for_case(case, storage=storage)
    ctx.enable_adjoint()
    ctx.init_macro(np.ones((case.ny, case.nx)), *W.gaussian_velocity(case.nx, case.ny, 1e-3, 1))
    state = ctx.save_state()
    lam_a, lam_b = ctx.adjoint_buffer(), ctx.adjoint_buffer()
    zeros = _dev(np.zeros((case.ny, case.nx)))
    ctx.adjoint_seed_velocity(state, zeros, zeros, lam_a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for label, fn in (("forward step", lambda: ctx.step(1)),
                      ("adjoint step", lambda: ctx.adjoint_step(state, lam_a, lam_b))):
        _settle(fn)
        e0.record(ctx.stream)
        for _ in range(50):
            fn()
        e1.record(ctx.stream)
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) / 50 * 1e3
        print(f"    513^2 {storage} {label}: {us:.1f} us "
              f"({case.nx * case.ny / us:.0f} MLUPS)", flush=True)


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_adjoint_step_time_4096(storage):
    """Time of one adjoint step on the periodic 4096^2 Taylor-Green grid,
    where the state and the adjoint buffers are far larger than the caches:
    its algorithmic bytes per node (the recompute reads the state and writes
    the next state and S; the reverse march reads the state, lambda^{n+1}
    and S and writes lambda^n) over the step time, against the HBM peak;
    reported."""
    case = W.tgv_case(4096, 4096, u0=0.01, nu=1e-4, cfl=0.9, eta=0.01)
    print(f"[gpu] adjoint step 4096^2 {storage}", flush=True)
    ctx = t2s2.context_for_case(case, storage=storage)
    ctx.enable_adjoint()
    ctx.init_macro(case.rho0, case.ux0, case.uy0, case.grad0)
    state = ctx.save_state()
    lam_a, lam_b = ctx.adjoint_buffer(), ctx.adjoint_buffer()
    gu = _dev(W.random_state((case.ny, case.nx), 1.0, 3))
    ctx.adjoint_seed_velocity(state, gu, gu, lam_a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    sb = 8 if storage == "f64" else 4  # storage and arithmetic bytes per value
    per_node = {"forward step": 18 * sb, "adjoint step": 9 * (3 * sb) + 9 * (4 * sb)}
    for label, fn in (("forward step", lambda: ctx.step(1)),
                      ("adjoint step", lambda: ctx.adjoint_step(state, lam_a, lam_b))):
        _settle(fn)
        e0.record(ctx.stream)
        for _ in range(20):
            fn()
        e1.record(ctx.stream)
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) / 20 * 1e3
        gbs = per_node[label] * case.nx * case.ny / (us * 1e-6) / 1e9
        print(f"    4096^2 {storage} {label}: {us:.1f} us ({case.nx * case.ny / us:.0f} MLUPS, "
              f"{per_node[label]} B/node, {gbs:.0f} GB/s = {gbs / 8000:.3f} of 8 TB/s)", flush=True)
    lam = ctx.adjoint_read(lam_b)
    assert bool(torch.isfinite(lam).all()) and float(lam.abs().max()) > 0
    del lam
    ctx.close()
    del ctx, state, lam_a, lam_b
    torch.cuda.empty_cache()
