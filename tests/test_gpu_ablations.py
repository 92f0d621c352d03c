"""GPU parity of the ablation variants of the paper's design choices.

Stored phasors (Table I): pf_phasors + pf_ybus_from_phasors, in the split
and the interleaved layout, must give bit-identical P, Q and J values to the
fused Ybus calls (which form the phasors on the fly with the same
arithmetic), and therefore the oracle's values within the parity gate.

CSC order (PF_JAC_CSC): the Jacobian written column by column, by either
method, must be the CSR values transposed, bit for bit, and the oracle's J
transposed within the parity gate.
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
def test_phasor_variants_grid_500_batched(layout):
    g = gridgen.grid_500()
    vm, va = gridgen.states(g.nb, 5, case=0)
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
    G = pf.Grid.from_grid(gridgen.grid_500())
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


# ---------------------------------------------------------------- CSC order
def _csc_perm(jr, jc):
    """For each CSC position of the (structurally symmetric) pattern, the CSR
    position of the same entry."""
    import scipy.sparse as sp
    n = len(jr) - 1
    A = sp.csr_matrix((np.arange(1, len(jc) + 1, dtype=np.float64), jc, jr), shape=(n, n))
    T = A.T.tocsr()
    T.sort_indices()
    assert np.array_equal(T.indptr, jr) and np.array_equal(T.indices, jc)  # symmetric pattern
    return T.data.astype(np.int64) - 1


def _grid_perms(G, bus_off=None):
    """CSC -> CSR position map of every grid of a handle, in global J numbering
    (the exported pattern lists each grid's 2 nb_g + 1 row pointers, then the
    next grid's)."""
    _, _, jr, jc = G.pattern()
    _, joff = G.offsets()
    bo = np.array([0, G.nb]) if bus_off is None else np.asarray(bus_off)
    perm = np.empty(G.nnz_j, np.int64)
    r0 = 0
    for k in range(G.ngrids):
        a, b = int(joff[k]), int(joff[k + 1])
        rows = jr[r0:r0 + 2 * int(bo[k + 1] - bo[k]) + 1]
        assert rows[0] == 0 and rows[-1] == b - a
        perm[a:b] = a + _csc_perm(rows, jc[a:b])
        r0 += len(rows)
    assert r0 == len(jr)
    return perm


def _csc_case(g, vm, va, tile, spb, bus_off=None, br_off=None, method=pf.PF_METHOD_ELEMENTWISE):
    import torch
    G = pf.Grid.from_grid(g, bus_off, br_off)
    G.set_schedule(tile, spb)
    if method == pf.PF_METHOD_YBUS:
        pf.pf_ybus(G)
    ns = vm.shape[0]
    vmd, vad = to_dev(vm), to_dev(va)
    p0, q0 = torch.empty_like(vmd), torch.empty_like(vmd)
    j0 = torch.empty(ns, G.nnz_j, dtype=torch.float64, device="cuda:0")
    pf.pf_jacobian_values(G, method, vmd, vad, p0, q0, j0)
    p1, q1 = torch.full_like(vmd, np.nan), torch.full_like(vmd, np.nan)
    j1 = torch.full_like(j0, np.nan)
    pf.pf_jacobian_values(G, method | pf.PF_JAC_CSC, vmd, vad, p1, q1, j1)
    torch.cuda.synchronize()
    perm = _grid_perms(G, bus_off)
    j0h, j1h = j0.cpu().numpy(), j1.cpu().numpy()
    assert np.array_equal(p1.cpu().numpy(), p0.cpu().numpy()) and np.array_equal(q1.cpu().numpy(), q0.cpu().numpy())
    for s in range(ns):
        assert np.array_equal(j1h[s], j0h[s][perm]), s  # the CSR values transposed, bit for bit
    return G, j1h


@pytest.mark.parametrize("method", [pf.PF_METHOD_ELEMENTWISE, pf.PF_METHOD_YBUS])
def test_csc_grid_500_against_oracle(method):
    import scipy.sparse as sp
    g = gridgen.grid_500()
    vm, va = gridgen.states(g.nb, 2, case=0)
    G, jcsc = _csc_case(g, vm, va, 256, 0, method=method)
    yr, yc, jr, jc = G.pattern()
    yb = oracle.ybus(g)
    pat = oracle.jac_pattern(yb)
    for s in range(2):
        jo = (oracle.jac_ew(g, vm[s], va[s], pat) if method == pf.PF_METHOD_ELEMENTWISE
              else oracle.jac_ybus(yb, vm[s], va[s], pat))
        A = sp.csr_matrix((jo, pat[1], pat[0]), shape=(2 * g.nb, 2 * g.nb))
        # CSC values = column by column: the CSR data of the transpose
        T = A.T.tocsr()
        T.sort_indices()
        assert rel_err(jcsc[s], T.data) <= TOL


@pytest.mark.parametrize("method", [pf.PF_METHOD_ELEMENTWISE, pf.PF_METHOD_YBUS])
@pytest.mark.parametrize("tile", [64, 256, 512])
def test_csc_edge_grids(tile, method):
    for g in (_grids.random_small(80, 150, 21, parallel=9, isolated=4), star_grid(700, seed=1),
              star_grid(600, seed=2, parallel=40), _grids.two_bus(0.01, 0.1, 0.02, 1.03, 0.04, flip=True)):
        vm, va = _grids.random_state(g.nb, 3)
        _csc_case(g, vm[None, :], va[None, :], tile, 1, method=method)


@pytest.mark.parametrize("method", [pf.PF_METHOD_ELEMENTWISE, pf.PF_METHOD_YBUS])
def test_csc_batched_and_multigrid(method):
    g = gridgen.grid_500()
    vm, va = gridgen.states(g.nb, 11, case=0)
    _csc_case(g, vm, va, 128, 3, method=method)
    grids = [_grids.random_small(n, int(n * 1.4), 70 + n, parallel=n % 4) for n in (5, 40, 300, 17, 2)]
    grids.append(star_grid(530, seed=9))
    big, bo, ro = gridgen.concat(grids)
    vm, va = _grids.random_state(big.nb, 7)
    _csc_case(big, vm[None, :], va[None, :], 256, 0, bo, ro, method=method)


def test_csc_other_methods_unsupported():
    import torch
    G = pf.Grid.from_grid(gridgen.grid_500())
    pf.pf_ybus(G)
    vm = torch.ones(G.nb, dtype=torch.float64, device="cuda:0")
    j = torch.empty(G.nnz_j, dtype=torch.float64, device="cuda:0")
    for m in (pf.PF_METHOD_ELEMENTWISE_TWO_PHASE, pf.PF_METHOD_ELEMENTWISE_ATOMIC):
        with pytest.raises(pf.PFError) as e:
            pf.pf_jacobian_values(G, m | pf.PF_JAC_CSC, vm, vm, None, None, j)
        assert e.value.code == pf.PF_EUNSUP


# ------------------------------------------------- precomputed branch constants
@pytest.mark.parametrize("case", ["grid_500_x3", "parallel_isolated", "hub_600_parallel"])
def test_precomputed_constants_same_values(case):
    """PF_EW_PRECOMPUTED reads the constants the branch kernel would derive:
    the two-phase results are bit-identical, copy-add stays within the gate."""
    import torch
    if case == "grid_500_x3":
        g = gridgen.grid_500()
        vm, va = gridgen.states(g.nb, 3, case=0)
    else:
        g = (_grids.random_small(80, 150, 21, parallel=9, isolated=4) if case == "parallel_isolated"
             else star_grid(600, seed=2, parallel=40))
        vm, va = _grids.random_state(g.nb, 3)
        vm, va = vm[None, :], va[None, :]
    G = pf.Grid.from_grid(g)
    ns = vm.shape[0]
    vmd, vad = to_dev(vm), to_dev(va)
    out = {}
    for name, m in (("tp", pf.PF_METHOD_ELEMENTWISE_TWO_PHASE),
                    ("tp_pre", pf.PF_METHOD_ELEMENTWISE_TWO_PHASE | pf.PF_EW_PRECOMPUTED),
                    ("ca_pre", pf.PF_METHOD_ELEMENTWISE_ATOMIC | pf.PF_EW_PRECOMPUTED)):
        p, q = torch.full_like(vmd, np.nan), torch.full_like(vmd, np.nan)
        j = torch.full((ns, G.nnz_j), np.nan, dtype=torch.float64, device="cuda:0")
        pf.pf_jacobian_values(G, m, vmd, vad, p, q, j)
        torch.cuda.synchronize()
        out[name] = (p.cpu().numpy(), q.cpu().numpy(), j.cpu().numpy())
    for a, b in zip(out["tp"], out["tp_pre"]):
        assert np.array_equal(a, b)
    yb = oracle.ybus(g)
    pat = oracle.jac_pattern(yb)
    scale = None
    for s in range(ns):
        po, qo = oracle.inject_ew(g, vm[s], va[s])
        jo = oracle.jac_ew(g, vm[s], va[s], pat)
        p, q, j = (x[s] for x in out["ca_pre"])
        assert rel_err(p, po, scale) <= TOL and rel_err(q, qo, scale) <= TOL and rel_err(j, jo, scale) <= TOL


def test_precomputed_flag_scope_and_graphs():
    import torch
    G = pf.Grid.from_grid(gridgen.grid_500())
    pf.pf_ybus(G)
    vm = to_dev(np.ones((2, G.nb)))
    va = to_dev(np.zeros((2, G.nb)))
    j = torch.empty(2, G.nnz_j, dtype=torch.float64, device="cuda:0")
    for m in (pf.PF_METHOD_ELEMENTWISE, pf.PF_METHOD_YBUS):
        with pytest.raises(pf.PFError) as e:
            pf.pf_jacobian_values(G, m | pf.PF_EW_PRECOMPUTED, vm, va, None, None, j)
        assert e.value.code == pf.PF_EUNSUP
    # a recorded two-phase evaluation with precomputed constants (its scratch is
    # allocated before recording) replays to the eager result
    vm = to_dev(gridgen.states(G.nb, 2, case=0)[0])
    va = to_dev(gridgen.states(G.nb, 2, case=0)[1])
    m = pf.PF_METHOD_ELEMENTWISE_TWO_PHASE | pf.PF_EW_PRECOMPUTED
    j_eager = torch.empty_like(j)
    pf.pf_jacobian_values(G, m, vm, va, None, None, j_eager)
    G2 = pf.Grid.from_grid(gridgen.grid_500())  # fresh handle: no scratch yet
    gr = pf.Graph(G2, [dict(op=pf.PF_OP_JACOBIAN, method=m, vm=vm, va=va, jval=j)])
    for _ in range(3):
        j.fill_(float("nan"))
        gr.launch()
        torch.cuda.synchronize()
        assert torch.equal(j, j_eager)
    gr.close()


def test_variants_grid_100k_full_size():
    """The 100k-bus benchmark grid: CSC output and both stored-phasor layouts
    against the fused kernels, bit for bit, and the fused kernels' oracle
    parity (covered in test_gpu_parity) carries over."""
    g = gridgen.grid_100k()
    vm, va = gridgen.states(g.nb, 1, case=1)
    _csc_case(g, vm, va, 256, 0)
    _csc_case(g, vm, va, 256, 0, method=pf.PF_METHOD_YBUS)
    for layout in LAYOUTS:
        r = _phasor_case(g, vm, va, 256, 0, layout)
        assert np.array_equal(r["p1"], r["p0"]) and np.array_equal(r["q1"], r["q0"])
        assert np.array_equal(r["j1"], r["j0"]) and np.array_equal(r["p2"], r["ps"])


@pytest.mark.parametrize("n", [1, 2, 3, 1001, (1 << 20) + 1, 5_000_000, (16 << 20) + 5])
def test_stream_copy(n):
    """The bandwidth probe copies every element, odd lengths included, with
    two pairs of doubles per thread and (past 8M pairs) one."""
    import torch
    src = torch.randn(n + 2, dtype=torch.float64, device="cuda:0")[:n]  # the first n of a larger buffer
    dst = torch.full((n + 2,), float("nan"), dtype=torch.float64, device="cuda:0")
    pf.pf_stream_copy(src, dst[:n])
    torch.cuda.synchronize()
    assert torch.equal(dst[:n], src)
    assert torch.isnan(dst[n:]).all()  # nothing written past the end
