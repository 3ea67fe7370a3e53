"""t2s2_diagnostics_noalloc (device output, reduction partials in the
library's static device array) against t2s2_diagnostics (workspace
partials, host output), through the C-ABI: two calls in a row on two
contexts, the second on a smaller mesh, each bitwise the workspace call's
values (same kernels and reduction order)."""
import ctypes

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
t2s2 = pytest.importorskip("paper_1911_12913_amd")


def _context(n, seed):
    case = W.cavity_case(n, lid=0.1, re=1000.0, cfl=0.9, eta=0.1, noise=1e-3, seed=seed)
    ctx = t2s2.context_for_case(case)
    ctx.init_distributions(torch.from_numpy(oracle.init(case)))
    ctx.step(30)
    return ctx


def test_diagnostics_noalloc_equals_workspace_diagnostics():
    lib = t2s2.load_library()
    for n, seed in ((300, 1), (40, 2)):  # the second call on a smaller mesh
        print(f"[gpu] diagnostics_noalloc cavity {n + 1}^2", flush=True)
        ctx = _context(n, seed)
        ref = ctx.diagnostics()
        out = torch.full((t2s2.NDIAG + 2,), -7.0, dtype=torch.float64, device="cuda:0")
        torch.cuda.synchronize()
        rc = lib.t2s2_diagnostics_noalloc(ctx._h, ctypes.c_void_p(out.data_ptr()))
        assert rc == t2s2.OK, lib.t2s2_last_error()
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        want = np.array([ref[k] for k in t2s2.DIAG_NAMES])
        print(f"    noalloc {got[:t2s2.NDIAG]}\n    host    {want}", flush=True)
        assert np.array_equal(got[:t2s2.NDIAG], want)
        assert np.all(got[t2s2.NDIAG:] == -7.0)  # nothing past the NDIAG values
        # and through the binding, on the context's own stream
        d = ctx.diagnostics_noalloc().cpu().numpy()
        assert np.array_equal(d, want)
        ctx.close()


def test_diagnostics_noalloc_argument_checks():
    lib = t2s2.load_library()
    ctx = _context(20, 3)
    out = torch.empty(16, dtype=torch.float64, device="cuda:0")
    assert lib.t2s2_diagnostics_noalloc(None, ctypes.c_void_p(out.data_ptr())) == t2s2.ERR_INVALID_ARG
    assert lib.t2s2_diagnostics_noalloc(ctx._h, None) == t2s2.ERR_INVALID_ARG
    assert lib.t2s2_diagnostics_noalloc(ctx._h, ctypes.c_void_p(out.data_ptr() + 4)) == \
        t2s2.ERR_INVALID_ARG
    ctx.close()


def test_diagnostics_noalloc_under_graph_capture():
    """The no-allocation variant can be recorded into a HIP graph between
    captured steps (no allocation, no host synchronisation): every replay
    writes the diagnostics of the state it has just stepped to, bitwise those
    of t2s2_diagnostics at the same point."""
    lib = t2s2.load_library()
    case = W.cavity_case(64, lid=0.1, re=1000.0, cfl=0.9, eta=0.1, noise=1e-3, seed=4)
    s = torch.cuda.Stream()
    ctx = t2s2.context_for_case(case, stream=s)
    ctx.init_distributions(torch.from_numpy(oracle.init(case)))
    out = torch.zeros(t2s2.NDIAG, dtype=torch.float64, device="cuda:0")
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        # two steps on the bound stream (the state returns to its buffer), then the diagnostics
        assert lib.t2s2_step(ctx._h, 2) == t2s2.OK
        assert lib.t2s2_diagnostics_noalloc(ctx._h, ctypes.c_void_p(out.data_ptr())) == t2s2.OK
    torch.cuda.synchronize()
    ref = t2s2.context_for_case(case)
    ref.init_distributions(torch.from_numpy(oracle.init(case)))
    for rep in range(3):
        graph.replay()
        torch.cuda.synchronize()
        ref.step(2)
        want = np.array([ref.diagnostics()[k] for k in t2s2.DIAG_NAMES])
        got = out.cpu().numpy()
        print(f"    replay {rep}: {got[:3]}", flush=True)
        assert np.array_equal(got, want), rep
    ctx.close()
    ref.close()
