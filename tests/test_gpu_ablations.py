"""GPU parity of the ablation variants of the paper's design choices.

Stored phasors (Table I): pf_phasors + pf_ybus_from_phasors, in the split
and the interleaved layout, must give bit-identical P, Q and J values to the
fused Ybus calls (which form the phasors on the fly with the same
arithmetic), and therefore the oracle's values within the parity gate.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2302_10736_amd import gridgen, pf
from tests import _grids
from tests._gpu import TOL, rel_err, require_gpu, to_dev
from tests.test_gpu_parity import star_grid

pytestmark = pytest.mark.gpu

LAYOUTS = [pf.PF_PHASOR_SPLIT, pf.PF_PHASOR_INTERLEAVED]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _phasor_case(g, vm, va, tile, spb, layout):
    import torch
    G = pf.Grid.from_grid(g)
    G.set_schedule(tile, spb)
    pf.pf_ybus(G)
    ns = vm.shape[0]
    vmd, vad = to_dev(vm), to_dev(va)
    p0, q0 = torch.empty_like(vmd), torch.empty_like(vmd)
    j0 = torch.empty(ns, G.nnz_j, dtype=torch.float64, device="cuda:0")
    pf.pf_jacobian_values(G, pf.PF_METHOD_YBUS, vmd, vad, p0, q0, j0)
    ps, qs = torch.empty_like(vmd), torch.empty_like(vmd)
    pf.pf_injections_ybus(G, vmd, vad, ps, qs)
    ph = torch.full((4 * ns * G.nb,), float("nan"), dtype=torch.float64, device="cuda:0")
    pf.pf_phasors(G, layout, vmd, vad, ph)
    p1, q1 = torch.full_like(vmd, np.nan), torch.full_like(vmd, np.nan)
    j1 = torch.full_like(j0, np.nan)
    pf.pf_ybus_from_phasors(G, layout, ns, ph, p1, q1, j1)
    p2, q2 = torch.full_like(vmd, np.nan), torch.full_like(vmd, np.nan)
    pf.pf_ybus_from_phasors(G, layout, ns, ph, p2, q2)  # injections only
    j3 = torch.full_like(j0, np.nan)
    pf.pf_ybus_from_phasors(G, layout, ns, ph, None, None, j3)  # Jacobian only
    torch.cuda.synchronize()
    h = lambda t: t.cpu().numpy()
    return dict(p0=h(p0), q0=h(q0), j0=h(j0), ps=h(ps), qs=h(qs), p1=h(p1), q1=h(q1), j1=h(j1), p2=h(p2),
                q2=h(q2), j3=h(j3), ph=h(ph))


def _check_phasor_case(g, vm, va, tile, spb, layout):
    r = _phasor_case(g, vm, va, tile, spb, layout)
    assert np.array_equal(r["p1"], r["p0"]) and np.array_equal(r["q1"], r["q0"])
    assert np.array_equal(r["j1"], r["j0"]) and np.array_equal(r["j3"], r["j0"])
    assert np.array_equal(r["p2"], r["ps"]) and np.array_equal(r["q2"], r["qs"])
    # the stored phasors themselves: V = v e^{j theta}, U = e^{j theta}
    ns, nb = vm.shape
    n = ns * nb
    ph = r["ph"]
    if layout == pf.PF_PHASOR_SPLIT:
        vre, vim, ure, uim = ph[:n], ph[n:2 * n], ph[2 * n:3 * n], ph[3 * n:]
    else:
        vre, vim, ure, uim = ph[0:2 * n:2], ph[1:2 * n:2], ph[2 * n::2], ph[2 * n + 1::2]
    assert np.max(np.abs(ure - np.cos(va.ravel()))) <= 2e-16 and np.max(np.abs(uim - np.sin(va.ravel()))) <= 2e-16
    assert np.array_equal(vre, vm.ravel() * ure) and np.array_equal(vim, vm.ravel() * uim)
    # and the oracle, state by state
    yb = oracle.ybus(g)
    pat = oracle.jac_pattern(yb)
    for s in range(ns):
        po, qo = oracle.inject_ybus(yb, vm[s], va[s])
        jo = oracle.jac_ybus(yb, vm[s], va[s], pat)
        assert rel_err(r["p1"][s], po) <= TOL and rel_err(r["q1"][s], qo) <= TOL
        assert rel_err(r["j1"][s], jo) <= TOL


@pytest.mark.parametrize("layout", LAYOUTS)
def test_phasor_variants_config0_batched(layout):
    g = gridgen.config0()
    vm, va = gridgen.states(g.nb, 5, cfg=0)
    _check_phasor_case(g, vm, va, 256, 0, layout)
    _check_phasor_case(g, vm, va, 128, 3, layout)


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("tile", [64, 512])
def test_phasor_variants_long_rows_and_ragged(layout, tile):
    # a hub row longer than any tile (the chunked long-row path) and ragged tiles
    for g in (star_grid(700, seed=1), _grids.random_small(333, 700, 8, parallel=3, isolated=7)):
        vm, va = _grids.random_state(g.nb, 3)
        _check_phasor_case(g, vm[None, :], va[None, :], tile, 1, layout)


def test_phasor_argument_checks():
    import torch
    G = pf.Grid.from_grid(gridgen.config0())
    L = pf.lib()
    vm = torch.ones(G.nb, dtype=torch.float64, device="cuda:0")
    ph = torch.empty(4 * G.nb + 2, dtype=torch.float64, device="cuda:0")
    p = torch.empty_like(vm)
    ptr = lambda t, off=0: t.data_ptr() + off
    # Ybus not assembled yet
    assert L.pf_ybus_from_phasors(G.handle, 1, 1, ptr(ph), ptr(p), ptr(p), None, None) == pf.PF_ESTATE
    pf.pf_ybus(G)
    assert L.pf_phasors(G.handle, 0, 1, ptr(vm), ptr(vm), ptr(ph), None) == pf.PF_EINVAL
    assert L.pf_phasors(G.handle, 3, 1, ptr(vm), ptr(vm), ptr(ph), None) == pf.PF_EINVAL
    assert L.pf_phasors(G.handle, 2, 1, ptr(vm), ptr(vm), ptr(ph, 8), None) == pf.PF_EINVAL  # misaligned pairs
    assert L.pf_phasors(G.handle, 1, 1, ptr(vm), ptr(vm), None, None) == pf.PF_EINVAL
    assert L.pf_ybus_from_phasors(G.handle, 1, 1, ptr(ph), None, None, None, None) == pf.PF_EINVAL  # nothing out
    assert L.pf_ybus_from_phasors(G.handle, 1, 1, ptr(ph), ptr(p), None, None, None) == pf.PF_EINVAL  # p without q
    assert L.pf_ybus_from_phasors(G.handle, 2, 1, ptr(ph, 8), ptr(p), ptr(p), None, None) == pf.PF_EINVAL
    assert L.pf_phasors(G.handle, 1, 0, None, None, None, None) == pf.PF_OK  # zero states
    assert L.pf_ybus_from_phasors(G.handle, 1, 0, None, None, None, None, None) == pf.PF_OK
    torch.cuda.synchronize()
