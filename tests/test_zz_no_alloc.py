"""The allocation-free entry point pf_jacobian_two_phase_static: through the
C ABI, against the two-phase baseline it varies (pf_jacobian_values with
PF_METHOD_ELEMENTWISE_TWO_PHASE, same kernels: bit for bit) and against the
oracle (1e-12), on two calls in a row, the second with a smaller grid, so the
shared static scratch is reused with stale contents from the first call."""
from __future__ import annotations

import ctypes as C

import numpy as np
import pytest

import oracle
from paper_2302_10736_amd import gridgen, pf
from tests._gpu import TOL, rel_err, require_gpu, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _ptr(t):
    return C.c_void_p(t.data_ptr())


def _static_call(G, method, vm, va, p, q, j):
    """pf_jacobian_two_phase_static through the raw C ABI (ctypes), torch's current stream."""
    import torch
    L = pf.lib()
    st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    return L.pf_jacobian_two_phase_static(G.handle, int(method), int(vm.shape[0]), _ptr(vm), _ptr(va),
                                          _ptr(p) if p is not None else None, _ptr(q) if q is not None else None,
                                          _ptr(j), st)


@pytest.mark.parametrize("method", [pf.PF_METHOD_ELEMENTWISE_TWO_PHASE,
                                    pf.PF_METHOD_ELEMENTWISE_TWO_PHASE | pf.PF_EW_PRECOMPUTED])
def test_static_scratch_two_calls_larger_then_smaller(method):
    import torch
    cases = [(gridgen.grid_100k(), 2, 1), (gridgen.grid_500(), 1, 0)]  # second call: smaller grid
    handles = []
    for g, ns, case in cases:
        print(f"static two-phase: nb={g.nb} states={ns} method={method}", flush=True)
        vm_h, va_h = gridgen.states(g.nb, ns, case=case)
        G = pf.Grid.from_grid(g)
        handles.append(G)
        vm, va = to_dev(vm_h), to_dev(va_h)
        nan = lambda *s: torch.full(s, float("nan"), dtype=torch.float64, device="cuda:0")
        p, q, j = nan(ns, g.nb), nan(ns, g.nb), nan(ns, G.nnz_j)
        rc = _static_call(G, method, vm, va, p, q, j)
        assert rc == pf.PF_OK, pf.lib().pf_last_error().decode()
        p2, q2, j2 = nan(ns, g.nb), nan(ns, g.nb), nan(ns, G.nnz_j)
        pf.pf_jacobian_values(G, method, vm, va, p2, q2, j2)
        torch.cuda.synchronize()
        for a, b in ((p, p2), (q, q2), (j, j2)):
            assert np.array_equal(a.cpu().numpy(), b.cpu().numpy())
        pat = oracle.jac_pattern(oracle.ybus(g))
        for s in range(ns):
            p_o, q_o = oracle.inject_ew(g, vm_h[s], va_h[s])
            j_o = oracle.jac_ew(g, vm_h[s], va_h[s], pat)
            assert rel_err(p[s].cpu().numpy(), p_o) <= TOL
            assert rel_err(q[s].cpu().numpy(), q_o) <= TOL
            assert rel_err(j[s].cpu().numpy(), j_o) <= TOL
        # injections may be skipped (p = q = NULL)
        j3 = nan(ns, G.nnz_j)
        assert _static_call(G, method, vm, va, None, None, j3) == pf.PF_OK
        torch.cuda.synchronize()
        assert np.array_equal(j3.cpu().numpy(), j2.cpu().numpy())


def test_static_scratch_limits_and_arguments():
    import torch
    g = gridgen.make_grid(150_000, 200_000, 0.15, case=2)  # 550,000 records: beyond the static scratch
    G = pf.Grid.from_grid(g)
    vm = torch.ones(1, g.nb, dtype=torch.float64, device="cuda:0")
    j = torch.empty(1, G.nnz_j, dtype=torch.float64, device="cuda:0")
    assert _static_call(G, pf.PF_METHOD_ELEMENTWISE_TWO_PHASE, vm, vm, None, None, j) == pf.PF_EUNSUP
    assert "static scratch" in pf.lib().pf_last_error().decode()
    G2 = pf.Grid.from_grid(gridgen.grid_500())
    vm2 = torch.ones(1, G2.nb, dtype=torch.float64, device="cuda:0")
    j2 = torch.empty(1, G2.nnz_j, dtype=torch.float64, device="cuda:0")
    assert _static_call(G2, pf.PF_METHOD_ELEMENTWISE, vm2, vm2, None, None, j2) == pf.PF_EINVAL
    assert _static_call(G2, pf.PF_METHOD_ELEMENTWISE_TWO_PHASE, vm2, vm2, vm2, None, j2) == pf.PF_EINVAL


def test_static_scratch_under_graph_capture():
    """The allocation-free entry point recorded in a captured HIP graph (torch
    capture of the library's launches on the capturing stream) and replayed
    several times with eager work and input changes in between: every replay
    equals the eager call bit for bit."""
    import torch
    g = gridgen.grid_500()
    G = pf.Grid.from_grid(g)
    vm_h, va_h = gridgen.states(g.nb, 3, case=0)
    vm, va = to_dev(vm_h), to_dev(va_h)
    p, q = torch.empty_like(vm), torch.empty_like(vm)
    j = torch.empty(3, G.nnz_j, dtype=torch.float64, device="cuda:0")
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        pf.pf_jacobian_two_phase_static(G, pf.PF_METHOD_ELEMENTWISE_TWO_PHASE, vm, va, p, q, j, stream=side)
    torch.cuda.synchronize()
    gr = torch.cuda.CUDAGraph()
    with torch.cuda.graph(gr, stream=side):
        pf.pf_jacobian_two_phase_static(G, pf.PF_METHOD_ELEMENTWISE_TWO_PHASE, vm, va, p, q, j, stream=side)
    for rep in range(3):
        j.fill_(float("nan"))
        with torch.cuda.stream(side):
            gr.replay()
        torch.cuda.synchronize()
        p2, q2, j2 = torch.empty_like(p), torch.empty_like(q), torch.empty_like(j)
        pf.pf_jacobian_values(G, pf.PF_METHOD_ELEMENTWISE_TWO_PHASE, vm, va, p2, q2, j2)
        torch.cuda.synchronize()
        assert torch.equal(j, j2) and torch.equal(p, p2) and torch.equal(q, q2), rep
        vm.mul_(1.01)
        va.add_(0.02)
