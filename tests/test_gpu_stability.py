"""GPU von Neumann stability maps (t2s2_stability_map) against the numpy
oracle (oracle/stability.py, eigenvalues by numpy.linalg.eigvals)."""
import math
import time

import numpy as np
import pytest

from oracle import stability as S

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
t2s2 = pytest.importorskip("paper_1911_12913_amd")


def _oracle_max(model, omega, r, nk, full_kx, **kw):
    thy = np.linspace(0.0, math.pi, nk)
    thx = np.linspace(-math.pi, math.pi, 2 * nk - 1) if full_kx else thy
    return max(S.spectral_radius(S.growth(model, a, b, omega, r, **kw)) for a in thx for b in thy)


CASES = [
    ("fdlbm1", dict(eta=0.01, u=(0.01, 0.01), A=0.5), True),
    ("fdlbm1", dict(eta=0.1, u=(0.2, 0.2), A=0.0), True),
    ("fdlbm2", dict(eta=0.1, u=(0.2, 0.2)), True),
    ("paper", dict(eta=0.1, u=(0.2, 0.2), B2bar=0.5, B2tilde=0.0), False),
    ("paper", dict(eta=0.1, u=(0.2, 0.2), B2bar=0.25, B2tilde=0.5), False),
    ("family", dict(eta=0.1, u=(0.2, 0.2), A=0.5, btilde=(0.25, 0.5, 0.25)), True),
    ("family", dict(eta=0.05, u=(0.05, -0.1), A=0.3, btilde=(0.15, 0.5, 0.35)), True),
    ("family", dict(eta=0.1, u=(0.2, 0.2), A=0.5, btilde=(0.0, 1.0, 0.0),
                    bbar=(0.25, 0.5, 0.25)), True),
    ("family", dict(eta=0.05, u=(0.05, -0.1), A=1.0, btilde=(0.5, 0.5, 0.0),
                    bbar=(0.5, 0.5, 0.0)), True),
]


@pytest.mark.parametrize("model,kw,full", CASES)
def test_stability_map_matches_oracle(model, kw, full):
    """Largest spectral radius over a 9 x 9 (or 17 x 9) mode grid at seeded
    (omega, r) points: GPU repeated squaring vs oracle eigenvalues, 1e-6."""
    rng = np.random.Generator(np.random.PCG64(11))
    omegas = np.concatenate([[0.46, 4.6], rng.uniform(0.05, 8.0, 10)])
    rs = np.concatenate([[0.9, 0.9], rng.uniform(0.05, 1.5, 10)])
    gkw = dict(eta=kw["eta"], u=kw["u"], A=kw.get("A", 0.5), b2bar=kw.get("B2bar", 0.5),
               b2tilde=kw.get("B2tilde", 0.0), btilde=kw.get("btilde", (0.0, 1.0, 0.0)),
               bbar=kw.get("bbar", (0.5, 0.0, 0.5)))
    print(f"[gpu] stability map {model} {kw}", flush=True)
    got = t2s2.stability_map(model, omegas, rs, nk=9, full_kx=full, squarings=30, **gkw)
    got = got.cpu().numpy()
    okw = dict(kw)
    ref = np.array([_oracle_max(model, w, r, 9, full, **okw) for w, r in zip(omegas, rs)])
    err = np.abs(got - ref) / np.maximum(ref, 1e-300)
    print(f"    max rel diff {err.max():.2e}; radii {np.round(ref[:4], 6)}", flush=True)
    assert err.max() <= 1e-6


def test_stability_map_tgv_finding_and_timing():
    """The exact FDLBM1 map over omega in [0.1, 8], r in [0.1, 1.2] (64 x 64
    points, 33 x 65 modes): the 4096^2 TGV points (r = 0.9, omega = 0.46
    unstable, 4.6 stable) as the CPU oracle runs found them; time reported."""
    omegas = np.linspace(0.1, 8.0, 64)
    rs = np.linspace(0.1, 1.2, 64)
    W_, R_ = np.meshgrid(omegas, rs, indexing="ij")
    kw = dict(eta=0.01, u=(0.01, 0.01), A=0.5)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rad = t2s2.stability_map("fdlbm1", W_.ravel(), R_.ravel(), nk=33, full_kx=True, **kw)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    rad = rad.cpu().numpy().reshape(64, 64)
    n_modes = 33 * 65
    print(f"    64x64 map x {n_modes} modes: {dt * 1e3:.1f} ms "
          f"({64 * 64 * n_modes / dt / 1e6:.1f} M growth matrices/s); "
          f"stable fraction {(rad <= 1 + 1e-9).mean():.3f}", flush=True)
    # the oracle on a bounded sample of the same map, for the rate beside it
    t0 = time.perf_counter()
    n_cpu = 0
    for w in omegas[:4]:
        for a in np.linspace(-math.pi, math.pi, 65)[:25]:
            S.spectral_radius(S.growth("fdlbm1", a, 0.3, w, 0.9, eta=0.01, u=(0.01, 0.01), A=0.5))
            n_cpu += 1
    cpu_rate = n_cpu / (time.perf_counter() - t0)
    print(f"    oracle (numpy eigvals, 1 core): {cpu_rate / 1e3:.1f} k growth matrices/s", flush=True)
    pts = t2s2.stability_map("fdlbm1", [0.46, 4.6], [0.9, 0.9], nk=33, full_kx=True, **kw)
    pts = pts.cpu().numpy()
    assert pts[0] > 1.0 + 1e-4 and pts[1] <= 1.0 + 1e-9


def test_paper_family_largest_stable_region_on_gpu():
    """Sec. 2C: B-2 = B~2 = 1/2 (eta 0.1) has the largest stable region among
    the Fig. 1 settings (u = (0.2, 0.2), modes in [0, pi]^2), on a 32 x 32
    (omega, r) map."""
    omegas = np.linspace(0.05, 4.0, 32)
    rs = np.linspace(0.05, 1.6, 32)
    W_, R_ = np.meshgrid(omegas, rs, indexing="ij")
    settings = [(0.5, 0.0, 0.1), (0.25, 0.0, 0.1), (0.0, 0.0, 0.1),
                (0.5, 0.5, 0.1), (0.5, 0.25, 0.1), (0.5, 0.0, 0.0), (0.5, 0.0, 1.0)]
    area = {}
    for b2bar, b2t, eta in settings:
        rad = t2s2.stability_map("paper", W_.ravel(), R_.ravel(), eta=eta, u=(0.2, 0.2),
                                 b2bar=b2bar, b2tilde=b2t, nk=17, full_kx=False)
        area[(b2bar, b2t, eta)] = float((rad <= 1.0 + 1e-9).float().mean())
    print("    stable fractions: " + ", ".join(f"B2={k[0]},B~2={k[1]},eta={k[2]}: {v:.3f}"
                                               for k, v in area.items()), flush=True)
    assert area[(0.5, 0.5, 0.1)] == max(area.values())
