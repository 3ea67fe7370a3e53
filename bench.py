#!/usr/bin/env python3
"""Throughput of the D2Q9 T2S2-FDLBM step on one MI355X.

Workload: Taylor-Green vortex on a 4096 x 4096 periodic grid over [0, 2pi]^2,
U0 = 0.01, CFL = 0.9, eta = 0.01, T2S2-FDLBM1 (A = 1/2), FP64 state,
initialised with eq 3.5 (synthetic, from the closed form).  nu = 1e-4: at
nu = 1e-3 this grid has dt / tau = 0.46, where the scheme is unstable at
CFL 0.9 for every eta (the oracle blows up the same way); nu = 1e-4 gives
dt / tau = 4.6, inside the stable region, with the same work per step.
A step is one full time step of the grid (one launch of the fused kernel).

Prints one JSON line: MLUPS (lattice-node updates per second, all nodes),
the roofline of the fused step kernel (algorithmic bytes per launch / the
launch time measured with HIP events on the launch stream), and the FP64
CPU oracle timed on a bounded sample of the same workload.  The precision
forms (deviations stored in FP32, BF16 or FP16, FP32 arithmetic, FP64
moment sums) then run the same steps on the same grid; each reports its
MLUPS, its speed-up over the FP64 line and the relative L2 error of its
final velocity field against the FP64 result (which matches the oracle to
round-off) and against the closed-form decay of eq 3.4.  A plain copy of
the nine planes with the step's store policy, over buffers of the state's
size, gives the practical bandwidth ceiling beside the published peak.
Guo's T1S2-FDLBM
(A = 0, the single-stencil kernel) runs on the same grid in FP64 at
CFL 0.25, inside its stable range, for the cost of one scheme against the
other.  Last, the differentiation form: the gradient of a probe loss on the
513 x 513 cavity (2000 steps, sqrt(N) checkpoints) with respect to the
initial velocity and the viscosity, forward + backward wall time in FP32
and FP64, and the FP32 gradient against the FP64 one.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import platform
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
BYTES_PER_NODE = {"f64": 144, "f32": 72, "bf16": 36, "f16": 36, "bf16sr": 36, "f16sr": 36}
METRIC = "D2Q9 MLUPS & % HBM peak, FP64 vs FP32/BF16-store at stated L2 error"
KERNEL_SOURCES = ["paper_1911_12913_amd/csrc/t2s2_kernels.hip",
                  "paper_1911_12913_amd/csrc/t2s2_device.h",
                  "paper_1911_12913_amd/csrc/t2s2_internal.h",
                  "paper_1911_12913_amd/csrc/t2s2_api.hip",
                  "paper_1911_12913_amd/build.py"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_step_tgv4096.json")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(storage: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if
    it was taken on the current kernel sources; else None."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    entry = rec.get(storage)
    if not entry or rec.get("kernel_hash") != kernel_source_hash():
        return None
    return entry.get("bytes_per_launch")


def tgv_case(n, nu, cfl, eta):
    import workloads as W

    return W.tgv_case(n, n, u0=0.01, nu=nu, cfl=cfl, eta=eta)


def W_tgv_fields(case, t):
    import workloads as W

    m = case.meta
    return W.tgv_fields(case.x, case.y, m["k1"], m["k2"], m["u0"], case.nu, t)


def timed_windows(ctx, init, steps, warmup, warmup_s, windows):
    """Untimed steps for warmup_s seconds (clocks settle after an idle
    period), then the state is initialised again (init(ctx)), warmup
    untimed steps follow, and `windows` timed windows of exactly `steps`
    steps, each between two HIP events recorded on the library's launch
    stream, with a full synchronisation before and after each window.
    Every run thus takes the same steps from the same initial state.
    Returns (ms of each window, steps of the time-based warm-up, its
    seconds)."""
    import torch

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    extra = 0
    chunk = max(1, steps)
    while time.perf_counter() - t0 < warmup_s:
        ctx.step(chunk)
        extra += chunk
        torch.cuda.synchronize()
    warm_s = time.perf_counter() - t0
    init(ctx)
    ctx.step(warmup)
    stream = ctx.stream
    out = []
    for _ in range(windows):
        torch.cuda.synchronize()
        start = torch.cuda.Event(enable_timing=True)
        stop = torch.cuda.Event(enable_timing=True)
        start.record(stream)
        ctx.step(steps)
        stop.record(stream)
        torch.cuda.synchronize()
        out.append(start.elapsed_time(stop))
    return out, extra, warm_s


def gpu_leg(case, storage, steps, warmup, warmup_s=1.0, windows=5, **overrides):
    """One storage form on the GPU (timed_windows).  Returns the median
    window's ms, the timing record, the diagnostics, dt and the final
    velocity fields."""
    import torch

    import paper_1911_12913_amd as t2s2

    torch.cuda.set_device(0)
    ctx = t2s2.context_for_case(case, storage=storage, device="cuda:0", **overrides)
    # The initial fields go to the device once: initialising again from host
    # arrays idles the GPU for the uploads, and its clocks then take about
    # 60 steps to return (measured: the first 20-step windows after such an
    # init ran 0.60, 0.53, 0.51 ms per step against 0.505 ms steady).
    fields = [torch.as_tensor(a, dtype=torch.float64, device="cuda:0").contiguous()
              if a is not None else None
              for a in (case.rho0, case.ux0, case.uy0, case.grad0)]

    def init(c):
        c.init_macro(*fields)

    init(ctx)
    wins, extra, warm_s = timed_windows(ctx, init, steps, warmup, warmup_s, windows)
    ms = statistics.median(wins)
    timing = {"windows": len(wins), "steps_per_window": steps,
              "ms_per_step_windows": [w / steps for w in wins],
              "ms_per_step_median": ms / steps,
              "spread": (max(wins) - min(wins)) / ms,
              "warmup_steps": warmup, "warmup_s": warm_s, "warmup_time_steps": extra,
              "steps_from_init": ctx.steps_taken}
    diag = ctx.diagnostics()
    _, ux, uy = ctx.moments()
    torch.cuda.synchronize()
    dt = ctx.dt
    ctx.close()
    del fields
    return ms, timing, diag, dt, torch.stack([ux, uy])


def copy_ceiling(n, elem_bytes, reps=20, warmup=3):
    """Bandwidth of the reference nine-plane copy (t2s2_copy_probe) over
    buffers of the state's size, timed with HIP events on its stream."""
    import torch

    import paper_1911_12913_amd as t2s2

    dt = {8: torch.float64, 4: torch.float32, 2: torch.float16}[elem_bytes]
    src = torch.ones(9 * n, dtype=dt, device="cuda:0")
    dst = torch.empty_like(src)
    stream = torch.cuda.Stream()
    for _ in range(warmup):
        t2s2.copy_probe(src, dst, stream=stream)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(reps):
        t2s2.copy_probe(src, dst, stream=stream)
    stop.record(stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop) / reps
    del src, dst
    torch.cuda.empty_cache()
    return 2 * 9 * n * elem_bytes / (ms * 1e-3) / 1e9


def differentiation_leg(nsteps, storages=("f32", "f64"), reps=2):
    """The differentiation form: lid-driven cavity on the 513 x 513
    tanh-stretched mesh (c = 1.5), Re 400, CFL 0.9, nsteps steps with
    sqrt(N) checkpoints; loss = mean over 64 seeded interior probes of
    |u - u_target|^2 (targets from a run at 1.05 nu); gradient with respect
    to the initial velocity (seeded Gaussian perturbation, std 1e-3) and nu.
    Wall time of forward + backward per storage (one untimed run first), and
    the FP32 gradient against the FP64 one."""
    import numpy as np
    import torch

    import workloads as W
    from paper_1911_12913_amd.rollout import RolloutSpec, T2S2Rollout, forward_velocity

    case = W.cavity_case(512, lid=0.1, re=400.0, cfl=0.9, eta=0.1, noise=0.0)
    dev = "cuda:0"

    def t(a):
        return torch.as_tensor(np.asarray(a), dtype=torch.float64, device=dev)

    probes = W.probe_nodes(case.nx, case.ny, 64, seed=2)
    pj = torch.as_tensor(probes[:, 1], device=dev)
    pi = torch.as_tensor(probes[:, 0], device=dev)
    rho0, zero = t(np.ones((case.ny, case.nx))), t(np.zeros((case.ny, case.nx)))
    u0, v0 = W.gaussian_velocity(case.nx, case.ny, std=1e-3, seed=1)
    out, grads = {}, {}
    for st in storages:
        spec = RolloutSpec(x=case.x, y=case.y, periodic_x=case.periodic_x,
                           periodic_y=case.periodic_y, period_x=case.period_x,
                           period_y=case.period_y, cfl=case.cfl, dt=case.dt or 0.0,
                           eta=case.eta, A=case.A, u_wall=case.u_wall, storage=st,
                           nsteps=nsteps, device=dev)
        ut, vt = forward_velocity(spec, rho0, zero, zero, 1.05 * case.nu)
        ut, vt = ut[pj, pi].clone(), vt[pj, pi].clone()
        secs = []
        for r in range(reps + 1):
            gu, gv = t(u0).requires_grad_(True), t(v0).requires_grad_(True)
            gnu = torch.tensor(case.nu, dtype=torch.float64, device=dev, requires_grad=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            U, V = T2S2Rollout.apply(rho0, gu, gv, gnu, spec)
            loss = ((U[pj, pi] - ut) ** 2 + (V[pj, pi] - vt) ** 2).mean()
            loss.backward()
            torch.cuda.synchronize()
            if r > 0:
                secs.append(time.perf_counter() - t0)
        grads[st] = (torch.stack([gu.grad, gv.grad]), gnu.grad.item())
        s_mean = sum(secs) / len(secs)
        out[st] = {"rollout_s": s_mean, "unit": "s (forward + backward)",
                   "node_steps_per_s": case.nx * case.ny * nsteps / s_mean,
                   "checkpoint_every": spec.segment(), "loss": loss.item()}
    rec = {"workload": f"cavity{case.nx}x{case.ny} stretched c=1.5, Re 400, CFL 0.9, "
                       f"{nsteps} steps, sqrt(N) checkpoints, 64 probes",
           "steps": nsteps, "by_storage": out}
    if "f32" in grads and "f64" in grads:
        g32, g64 = grads["f32"], grads["f64"]
        rec["f32_vs_f64_rel_l2_dL_du0"] = rel_l2_dev(g32[0], g64[0])
        rec["f32_vs_f64_rel_dL_dnu"] = abs(g32[1] - g64[1]) / abs(g64[1])
    return rec


def rel_l2_dev(a, b) -> float:
    import torch

    return float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))


def cpu_leg(case, steps, threads):
    import oracle

    oracle.build(force=False)
    used = oracle.set_threads(threads)
    t0 = time.perf_counter()
    phi = oracle.init(case)
    t1 = time.perf_counter()
    oracle.run(case, phi, steps, threads=used)
    t2 = time.perf_counter()
    return (t2 - t1), used


def host_cpu():
    """CPU model, logical CPUs and the CPUs this process may run on."""
    model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        affinity = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        affinity = os.cpu_count() or 1
    return {"model": model, "nproc": os.cpu_count(), "affinity": affinity}


def configs_leg(threads):
    """The other workloads of the method, GPU against the oracle: the 32^2
    Taylor-Green vortex (1000 steps, FP64, the oracle in full), the 257^2
    cavity (Re 1000, FP64; 5000 GPU steps in captured 100-step graphs, the
    oracle on a 200-step prefix) and the 2049^2 cavity (Re 5000; 200 GPU
    steps per storage, the oracle on a 4-step prefix).  MLUPS of each side
    and, where both ran the same steps, the GPU state against the oracle's."""
    import numpy as np
    import torch

    import oracle
    import paper_1911_12913_amd as t2s2
    import workloads as W

    out = {}

    def gpu_time(case, storage, steps, phi0, graph=False):
        """MLUPS and ms per step of `steps` steps from phi0 (after as many
        untimed ones), and the final state."""
        s = torch.cuda.Stream() if graph else None
        ctx = t2s2.context_for_case(case, storage=storage, device="cuda:0", stream=s)
        run = ctx.step
        if graph:
            ctx.graph_capture(100)
            run = ctx.graph_step
        ctx.init_distributions(torch.from_numpy(phi0))
        run(steps)
        ctx.init_distributions(torch.from_numpy(phi0))
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(ctx.stream)
        run(steps)
        e1.record(ctx.stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        g = ctx.read_distributions().cpu().numpy()
        ctx.close()
        return case.nx * case.ny * steps / (ms * 1e-3) / 1e6, ms / steps, g

    def oracle_time(case, phi0, steps, nthreads):
        oracle.set_threads(nthreads)
        t0 = time.perf_counter()
        ref = oracle.run(case, phi0, steps, threads=nthreads)
        secs = time.perf_counter() - t0
        return case.nx * case.ny * steps / secs / 1e6, secs, ref

    # TGV 32^2: the whole configuration on both sides
    c1 = W.tgv_case(32, 32, u0=0.01, nu=0.01, cfl=0.5, eta=0.01)
    phi = oracle.init(c1)
    gm, gms, g = gpu_time(c1, "f64", 1000, phi)
    om, osec, ref = oracle_time(c1, phi, 1000, 1)
    out["tgv32x32"] = {"steps": 1000, "gpu_mlups": gm, "gpu_us_per_step": gms * 1e3,
                       "oracle_mlups": om, "oracle_threads": 1, "oracle_s": osec,
                       "rel_l2_gpu_vs_oracle": W.rel_l2(g, ref),
                       "note": "launch-bound: one 1024-node launch per step"}

    # cavity 257^2: graph-launched GPU steps, oracle prefix
    c2 = W.cavity_case(256, lid=0.1, re=1000.0, cfl=0.9, eta=0.1, noise=1e-6, seed=0)
    phi = oracle.init(c2)
    gm, gms, _ = gpu_time(c2, "f64", 5000, phi, graph=True)
    _, _, g = gpu_time(c2, "f64", 200, phi, graph=True)
    om, osec, ref = oracle_time(c2, phi, 200, threads)
    out["cavity257x257"] = {"gpu_steps": 5000, "gpu_mlups": gm, "gpu_us_per_step": gms * 1e3,
                            "launch": "captured 100-step HIP graphs", "oracle_steps": 200,
                            "oracle_mlups": om, "oracle_threads": threads, "oracle_s": osec,
                            "rel_l2_gpu_vs_oracle_200_steps": W.rel_l2(g, ref)}

    # cavity 2049^2: FP64 and the precision forms, oracle prefix
    c4 = W.cavity_case(2048, lid=0.1, re=5000.0, cfl=0.9, eta=0.05, noise=1e-6, seed=0)
    phi = oracle.init(c4)
    rec = {"gpu_steps": 200, "by_storage": {}}
    for st in ("f64", "f32", "bf16", "f16", "bf16sr", "f16sr"):
        gm, gms, _ = gpu_time(c4, st, 200, phi)
        rec["by_storage"][st] = {"gpu_mlups": gm, "gpu_us_per_step": gms * 1e3}
    om, osec, ref = oracle_time(c4, phi, 4, threads)
    _, _, g4 = gpu_time(c4, "f64", 4, phi)
    rec.update({"oracle_steps": 4, "oracle_mlups": om, "oracle_threads": threads,
                "oracle_s": osec, "rel_l2_gpu_vs_oracle_4_steps": W.rel_l2(g4, ref)})
    out["cavity2049x2049"] = rec
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000,
                    help="steps per timed window (each form runs --windows windows)")
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--warmup-s", type=float, default=1.0,
                    help="after --warmup steps, untimed steps for this many seconds")
    ap.add_argument("--windows", type=int, default=5,
                    help="timed windows of --steps steps; the median is reported")
    ap.add_argument("--n", type=int, default=4096, help="grid side")
    ap.add_argument("--storage", default="f64", choices=sorted(BYTES_PER_NODE))
    ap.add_argument("--nu", type=float, default=1e-4)
    ap.add_argument("--forms", default="f32,bf16,f16,bf16sr,f16sr",
                    help="reduced-storage forms run after the headline one, each with the "
                         "same steps; their speed-up and velocity error are reported")
    ap.add_argument("--cpu-steps", type=int, default=8,
                    help="oracle steps timed on the host with --cpu-threads threads (0 = skip)")
    ap.add_argument("--cpu-threads", type=int, default=None)
    ap.add_argument("--cpu-single-steps", type=int, default=1,
                    help="oracle steps timed on one host thread (0 = skip)")
    ap.add_argument("--t1s2-steps", type=int, default=None,
                    help="steps of the FP64 T1S2 (A = 0) line at CFL 0.25 (default: --steps; "
                         "0 = skip)")
    ap.add_argument("--adjoint-steps", type=int, default=2000,
                    help="steps of the differentiation-form rollout (513^2 cavity, forward + "
                         "backward, FP32 and FP64; 0 = skip)")
    ap.add_argument("--configs", type=int, default=1,
                    help="1: also time the 32^2, 257^2 and 2049^2 workloads against the oracle")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="after the timed region, one plain device copy of this many bytes "
                         "(reference dispatch for scaling rocprofv3 memory counters)")
    args = ap.parse_args(argv)

    if args.gpus != 1:
        print(json.dumps({"error": "the step runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        return 2

    def say(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    n, nu, cfl, eta = args.n, args.nu, 0.9, 0.01
    case = tgv_case(n, nu, cfl, eta)
    nodes = n * n
    leg = dict(warmup_s=args.warmup_s, windows=args.windows)
    say(f"tgv{n} {args.storage}: {args.windows} windows of {args.steps} steps")
    ms, timing, diag, dt, vel = gpu_leg(case, args.storage, args.steps, args.warmup, **leg)
    say(f"  ms/step windows {['%.4f' % w for w in timing['ms_per_step_windows']]}")
    if args.copy_bytes > 0:
        import torch

        a = torch.empty(args.copy_bytes, dtype=torch.uint8, device="cuda:0")
        b = torch.empty_like(a)
        a.fill_(1)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    ms_step = ms / args.steps
    mlups = nodes * args.steps / (ms * 1e-3) / 1e6
    bytes_launch = BYTES_PER_NODE[args.storage] * nodes
    achieved = bytes_launch / (ms_step * 1e-3) / 1e9
    traffic = measured_traffic(args.storage)

    # closed-form velocity (eq 3.4) at the final time, for every form's error
    import torch

    t_end = timing["steps_from_init"] * dt
    _, ue, ve, _ = W_tgv_fields(case, t_end)
    exact = torch.stack([torch.from_numpy(ue), torch.from_numpy(ve)]).to("cuda:0")
    gre = rel_l2_dev(vel, exact)

    forms = {}
    for st in [f for f in args.forms.split(",") if f and f != args.storage]:
        say(f"tgv{n} {st}")
        ms_f, tim_f, diag_f, _, vel_f = gpu_leg(case, st, args.steps, args.warmup, **leg)
        v_f = nodes * args.steps / (ms_f * 1e-3) / 1e6
        bl = BYTES_PER_NODE[st] * nodes / (ms_f / args.steps * 1e-3) / 1e9
        forms[st] = {"value": v_f, "unit": "MLUPS", "ms_per_step": ms_f / args.steps,
                     "speedup_vs_headline": v_f / mlups,
                     "rel_l2_velocity_vs_headline": rel_l2_dev(vel_f, vel),
                     "rel_l2_velocity_vs_closed_form": rel_l2_dev(vel_f, exact),
                     "hbm_frac": bl / HBM_PEAK_GBS, "bytes_per_node": BYTES_PER_NODE[st],
                     "traffic": measured_traffic(st), "nonfinite": diag_f["nonfinite"],
                     "timing": tim_f}
        del vel_f
    del exact

    t1s2 = None
    t1s2_steps = args.steps if args.t1s2_steps is None else args.t1s2_steps
    if t1s2_steps > 0:
        say(f"tgv{n} T1S2 f64")
        case0 = tgv_case(n, nu, 0.25, eta)
        ms_0, tim_0, diag_0, dt_0, vel_0 = gpu_leg(case0, "f64", t1s2_steps, args.warmup,
                                                   A=0.0, **leg)
        v_0 = nodes * t1s2_steps / (ms_0 * 1e-3) / 1e6
        _, ue0, ve0, _ = W_tgv_fields(case0, tim_0["steps_from_init"] * dt_0)
        exact0 = torch.stack([torch.from_numpy(ue0), torch.from_numpy(ve0)]).to("cuda:0")
        t1s2 = {"value": v_0, "unit": "MLUPS", "ms_per_step": ms_0 / t1s2_steps,
                "steps": t1s2_steps, "scheme": "T1S2 (A = 0)", "storage": "f64", "cfl": 0.25,
                "dt": dt_0, "kernel": "single_step_kernel",
                "hbm_frac": BYTES_PER_NODE["f64"] * nodes / (ms_0 / t1s2_steps * 1e-3) / 1e9
                / HBM_PEAK_GBS,
                "t2s2_fdlbm1_step_time_ratio": ms_step / (ms_0 / t1s2_steps),
                # Simulated time per wall-clock second: T2S2-FDLBM1 at CFL 0.9
                # against T1S2 at CFL 0.25, inside T1S2's stable range (Sec. 3A
                # gives 0.2-0.3): the paper's case for the two-stage march.
                "sim_time_per_s": dt_0 / (ms_0 / t1s2_steps * 1e-3),
                "t2s2_fdlbm1_sim_time_per_s": dt / (ms_step * 1e-3),
                "t2s2_fdlbm1_time_to_solution_speedup":
                    (dt / ms_step) / (dt_0 / (ms_0 / t1s2_steps)),
                "rel_l2_velocity_vs_closed_form": rel_l2_dev(vel_0, exact0),
                "nonfinite": diag_0["nonfinite"], "timing": tim_0}
        del vel_0, exact0

    say("copy ceilings")
    ceiling = {}
    for st in dict.fromkeys([args.storage, "f32", "bf16"]):
        eb = BYTES_PER_NODE[st] // 18
        gbs = copy_ceiling(nodes, eb)
        ceiling[f"{eb}-byte"] = {"value": gbs, "unit": "GB/s", "frac_of_peak": gbs / HBM_PEAK_GBS,
                                 "kernel": "copy_planes_kernel", "elem_bytes": eb,
                                 "storages": [k for k, v in BYTES_PER_NODE.items()
                                              if v // 18 == eb]}
    head = ceiling[f"{BYTES_PER_NODE[args.storage] // 18}-byte"]
    head["step_frac_of_ceiling"] = achieved / head["value"]
    for st, f in forms.items():
        c = ceiling.get(f"{BYTES_PER_NODE[st] // 18}-byte")
        if c:
            f["frac_of_copy_ceiling"] = f["hbm_frac"] * HBM_PEAK_GBS / c["value"]

    diff = None
    if args.adjoint_steps > 0:
        say("differentiation form")
        diff = differentiation_leg(args.adjoint_steps)

    cpu_info = host_cpu()
    # The box allots 16 host CPUs to a one-GPU job; the oracle takes that
    # share (or fewer, when fewer are available).
    threads = args.cpu_threads or min(16, cpu_info["affinity"])
    other = None
    if args.configs:
        say("other workloads against the oracle")
        other = configs_leg(threads)

    cpu = None
    if args.cpu_steps > 0:
        say("oracle on the host")
        secs, used = cpu_leg(case, args.cpu_steps, threads)
        cpu = {"value": nodes * args.cpu_steps / secs / 1e6, "unit": "MLUPS", "cores": used,
               "kind": "oracle",
               "sample": f"{args.cpu_steps} FP64 oracle steps of the same {n}x{n} TGV grid "
                         f"({secs:.1f} s, {used} OpenMP threads)",
               "host": cpu_info,
               "threads_note": "16 host CPUs are this one-GPU job's share of the box"}
        if args.cpu_single_steps > 0:
            secs1, used1 = cpu_leg(case, args.cpu_single_steps, 1)
            cpu["single_thread"] = {
                "value": nodes * args.cpu_single_steps / secs1 / 1e6, "unit": "MLUPS",
                "cores": used1,
                "sample": f"{args.cpu_single_steps} FP64 oracle step(s) of the same grid "
                          f"({secs1:.1f} s, 1 thread)"}

    rec = {
        "metric": METRIC,
        "value": mlups,
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.storage,
        "data": "synthetic (Taylor-Green closed form, eq 3.4/3.5 initial state)",
        "config": {"workload": f"tgv{n}x{n}", "grid": [n, n], "domain": "[0,2pi]^2 periodic",
                   "u0": 0.01, "nu": nu, "cfl": cfl, "eta": eta, "A": 0.5, "dt": dt,
                   "scheme": "T2S2-FDLBM1", "storage": args.storage,
                   "nu_note": "nu = 1e-3 on this grid at CFL 0.9 gives dt/tau = 0.46, where "
                              "the scheme is unstable for every eta (the oracle and the exact "
                              "von Neumann model agree); nu = 1e-4 (dt/tau = 4.6) keeps the "
                              "grid, CFL, precision and work per step"},
        "timing": timing,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "step_kernel", "bytes_per_node": BYTES_PER_NODE[args.storage],
                     "frac_of_copy_ceiling": head["step_frac_of_ceiling"]},
        "copy_ceiling": ceiling,
        "cpu_baseline": cpu,
        "rel_l2_velocity_vs_closed_form": gre,
        "precision_forms": forms,
        "t1s2": t1s2,
        "differentiation": diff,
        "other_workloads": other,
        "diagnostics_after": {k: diag[k] for k in ("kinetic_energy", "max_speed", "nonfinite")},
    }
    print(json.dumps(rec), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
