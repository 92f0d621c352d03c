"""Failure paths forced from the host on a GPU handle: device allocations made
to fail by the testing hook (include/pf_testing.h).  Every kernel that runs
here runs normally; only allocation results are forced."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2302_10736_amd import gridgen, pf
from tests._gpu import TOL, rel_err, require_gpu, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _clear_hook():
    require_gpu()
    yield
    pf.pf_debug_fail_allocs(0)


def _sj(G, vm, va):
    import torch
    z = lambda *s: torch.full(s, float("nan"), dtype=torch.float64, device="cuda:0")
    p, q, j = z(1, G.nb), z(1, G.nb), z(1, G.nnz_j)
    pf.pf_jacobian_values(G, pf.PF_METHOD_ELEMENTWISE, vm, va, p, q, j)
    torch.cuda.synchronize()
    return p.cpu().numpy(), q.cpu().numpy(), j.cpu().numpy()


def test_failed_schedule_change_keeps_the_handle():
    """pf_set_schedule whose device allocation fails returns PF_ENOMEM and
    leaves tiles, lane tables, schedule and recorded graphs as they were."""
    import torch
    g = gridgen.grid_500()
    vm_h, va_h = gridgen.states(g.nb, 1, case=0)
    vm, va = to_dev(vm_h), to_dev(va_h)
    G = pf.Grid.from_grid(g)
    before = G.schedule()
    ref = _sj(G, vm, va)
    out = [torch.empty(1, G.nb, dtype=torch.float64, device="cuda:0") for _ in range(2)]
    jg = torch.empty(1, G.nnz_j, dtype=torch.float64, device="cuda:0")
    gr = pf.Graph(G, [dict(op=pf.PF_OP_JACOBIAN, method=pf.PF_METHOD_ELEMENTWISE, vm=vm, va=va, out_a=out[0],
                           out_b=out[1], jval=jg)])
    pf.pf_debug_fail_allocs(1)
    with pytest.raises(pf.PFError) as e:
        G.set_schedule(128, 3, pf.PF_ORDER_TILE_MAJOR)
    assert e.value.code == pf.PF_ENOMEM
    pf.pf_debug_fail_allocs(0)
    assert G.schedule() == before
    again = _sj(G, vm, va)
    for a, b in zip(ref, again):
        assert np.array_equal(a, b)
    gr.launch()  # the failed change did not invalidate the recording
    torch.cuda.synchronize()
    assert np.array_equal(jg.cpu().numpy(), ref[2])
    yb = oracle.ybus(g)
    j_o = oracle.jac_ew(g, vm_h[0], va_h[0], oracle.jac_pattern(yb))
    assert rel_err(again[2][0], j_o) <= TOL
    # the same change succeeds once allocations work again; results do not change
    G.set_schedule(128, 3, pf.PF_ORDER_TILE_MAJOR)
    assert G.schedule()[:3] == (128, 3, pf.PF_ORDER_TILE_MAJOR)
    after = _sj(G, vm, va)
    for a, b in zip(ref, after):
        assert np.array_equal(a, b)
    with pytest.raises(pf.PFError) as e:
        gr.launch()
    assert e.value.code == pf.PF_ESTATE
    gr.close()


def test_failed_build_reports_enomem():
    """A build whose device allocation fails returns PF_ENOMEM and no handle;
    the next build works."""
    g = gridgen.grid_500()
    pf.pf_debug_fail_allocs(1)
    with pytest.raises(pf.PFError) as e:
        pf.Grid.from_grid(g)
    assert e.value.code == pf.PF_ENOMEM
    vm_h, va_h = gridgen.states(g.nb, 1, case=0)
    G = pf.Grid.from_grid(g)
    p, q, _ = _sj(G, to_dev(vm_h), to_dev(va_h))
    p_o, _ = oracle.inject_ew(g, vm_h[0], va_h[0])
    assert rel_err(p[0], p_o) <= TOL
