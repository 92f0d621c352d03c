"""GPU parity: every C-ABI call against the CPU oracle, element by element.

Gate: for each output array (P, Q, J values, Ybus values, g_vm, g_va) and
each state, max|gpu - oracle| <= 1e-12 max|oracle|.  Tiny hand-made grids
whose sums cancel almost completely (many parallel branches on one bus
pair) are gated against the largest term instead of the result.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2302_10736_amd import gridgen, pf
from tests import _grids
from tests._gpu import TOL, compare_grid, gpu_all, oracle_all, rel_err, require_gpu, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def check_single(g, vm, va, tile=256, spb=0, use_scale=False, lam=True, order=pf.PF_ORDER_AUTO):
    """Build a handle, run every call on states [ns, nb], compare each state."""
    G = pf.Grid.from_grid(g)
    G.set_schedule(tile, spb, order)
    ns = vm.shape[0]
    rng = np.random.default_rng(5)
    lp = rng.normal(size=vm.shape) if lam else None
    lq = rng.normal(size=vm.shape) if lam else None
    gres = gpu_all(G, vm, va, lp, lq)
    for s in range(ns):
        ores = oracle_all(g, vm[s], va[s], None if lp is None else lp[s], None if lq is None else lq[s])
        compare_grid(gres, ores, s, slice(None), slice(None), slice(None), use_scale=use_scale)
    return gres


def test_grid_500_every_call():
    g = gridgen.grid_500()
    vm, va = gridgen.states(g.nb, 1, case=0)
    check_single(g, vm, va)


def star_grid(n_leaf, seed=0, parallel=0):
    """A hub bus with n_leaf branches (long row) plus a ring among the leaves."""
    rng = np.random.default_rng(seed)
    nb = n_leaf + 1
    f = [0] * n_leaf + list(range(1, nb - 1))
    t = list(range(1, nb)) + list(range(2, nb))
    for _ in range(parallel):
        k = int(rng.integers(0, n_leaf))
        f.append(0); t.append(k + 1)
    n = len(f)
    flip = rng.random(n) < 0.5
    fb = np.where(flip, t, f).astype(np.int32)
    tb = np.where(flip, f, t).astype(np.int32)
    tap = np.where(rng.random(n) < 0.3, rng.uniform(0.9, 1.1, n), 1.0)
    shift = np.where(tap != 1.0, rng.uniform(-0.1, 0.1, n), 0.0)
    return gridgen.Grid(nb, n, fb, tb, rng.uniform(0.001, 0.05, n), rng.uniform(0.01, 0.3, n),
                        rng.uniform(0, 0.1, n), tap, shift, rng.uniform(0, 0.02, nb), rng.uniform(-0.1, 0.1, nb))


EDGE_GRIDS = {
    "parallel_isolated": lambda: _grids.random_small(80, 150, 21, parallel=9, isolated=4),
    "two_bus": lambda: _grids.two_bus(0.01, 0.1, 0.02, 1.03, 0.04),
    "two_bus_flip": lambda: _grids.two_bus(0.01, 0.1, 0.02, 1.03, 0.04, flip=True),
    "many_parallel_pair": lambda: _grids.random_small(2, 30, 2, parallel=10),
    "hub_700": lambda: star_grid(700, seed=1),
    "hub_600_parallel": lambda: star_grid(600, seed=2, parallel=40),
    "ragged_tiles": lambda: _grids.random_small(333, 700, 8, parallel=3, isolated=7),
}


@pytest.mark.parametrize("tile", [64, 128, 256, 512])
@pytest.mark.parametrize("name", sorted(EDGE_GRIDS))
def test_edge_grids(name, tile):
    g = EDGE_GRIDS[name]()
    vm, va = _grids.random_state(g.nb, 3)
    use_scale = name == "many_parallel_pair"
    check_single(g, vm[None, :], va[None, :], tile=tile, use_scale=use_scale)


def test_shunt_only_buses():
    nb = 7
    gs = np.linspace(0, 0.02, nb)
    bs = np.linspace(-0.1, 0.1, nb)
    e = np.zeros(0)
    g = gridgen.Grid(nb, 0, np.zeros(0, np.int32), np.zeros(0, np.int32), e, e, e, e, e, gs, bs)
    vm, va = _grids.random_state(nb, 4)
    gres = check_single(g, vm[None], va[None], lam=True)
    assert np.allclose(gres["p_ew"][0], vm ** 2 * gs, rtol=1e-15, atol=0)
    assert np.allclose(gres["q_ew"][0], -(vm ** 2) * bs, rtol=1e-15, atol=0)


@pytest.mark.parametrize("order", [pf.PF_ORDER_TILE_MAJOR, pf.PF_ORDER_STATE_MAJOR, pf.PF_ORDER_GROUPED])
@pytest.mark.parametrize("spb", [0, 1, 3, 8, 64])
def test_batched_states_ragged(spb, order):
    g = gridgen.grid_500()
    vm, va = gridgen.states(g.nb, 37, case=0)
    check_single(g, vm, va, tile=128, spb=spb, order=order)


def test_zero_states_is_a_no_op():
    import torch
    G = pf.Grid.from_grid(gridgen.grid_500())
    e = torch.empty(0, G.nb, dtype=torch.float64, device="cuda:0")
    ej = torch.empty(0, G.nnz_j, dtype=torch.float64, device="cuda:0")
    pf.pf_injections_elementwise(G, e, e, e, e)
    pf.pf_jacobian_values(G, pf.PF_METHOD_ELEMENTWISE, e, e, e, e, ej)
    pf.pf_injections_vjp(G, e, e, e, e, e, e)


def test_multigrid_every_call():
    grids = [_grids.random_small(n, int(n * 1.4), 70 + n, parallel=n % 4, isolated=(n % 3 if n > 3 else 0))
             for n in (5, 40, 300, 17, 2)]
    grids.append(star_grid(530, seed=9))
    big, bo, ro = gridgen.concat(grids)
    G = pf.Grid.from_grid(big, bo, ro)
    assert G.ngrids == len(grids)
    ns = 3
    rng = np.random.default_rng(1)
    vm = rng.uniform(0.9, 1.1, (ns, big.nb))
    va = rng.normal(0, 0.2, (ns, big.nb))
    lp = rng.normal(size=vm.shape)
    lq = rng.normal(size=vm.shape)
    gres = gpu_all(G, vm, va, lp, lq)
    y_off, j_off = G.offsets()
    for k, g in enumerate(grids):
        bsl = slice(bo[k], bo[k + 1])
        for s in range(ns):
            ores = oracle_all(g, vm[s, bsl], va[s, bsl], lp[s, bsl], lq[s, bsl])
            compare_grid(gres, ores, s, bsl, slice(j_off[k], j_off[k + 1]), slice(y_off[k], y_off[k + 1]),
                         use_scale=g.nb == 2, br_sl=slice(ro[k], ro[k + 1]))


def test_determinism_across_runs_and_schedules():
    g = _grids.random_small(900, 1600, 33, parallel=12, isolated=5)
    vm, va = _grids.random_state(g.nb, 6)
    rng = np.random.default_rng(2)
    # the last two states keep every angle difference within pi/4 (whole
    # waves take the sine/cosine shortcut) except at 1 % of the buses, so a
    # record's wave takes the shortcut under some tile sizes and not others
    small = rng.normal(0, 0.01, (2, g.nb))
    small[1, rng.choice(g.nb, g.nb // 100, replace=False)] = rng.uniform(1.0, 3.0, g.nb // 100)
    vm = np.stack([vm, rng.uniform(0.9, 1.1, g.nb), rng.uniform(0.9, 1.1, g.nb), rng.uniform(0.95, 1.05, g.nb),
                   rng.uniform(0.95, 1.05, g.nb)])
    va = np.stack([va, rng.normal(0, 0.3, g.nb), rng.normal(0, 0.3, g.nb), small[0], small[1]])
    lp, lq = rng.normal(size=vm.shape), rng.normal(size=vm.shape)
    G = pf.Grid.from_grid(g)
    ref = gpu_all(G, vm, va, lp, lq)
    for s in range(vm.shape[0]):
        compare_grid(ref, oracle_all(g, vm[s], va[s], lp[s], lq[s]), s, slice(None), slice(None), slice(None))
    # every method but copy-add (atomic adds in no fixed order) is bitwise reproducible
    fixed = [k for k in ref if not k.endswith("_ca")]
    for _ in range(3):
        again = gpu_all(G, vm, va, lp, lq)
        for k in fixed:
            assert np.array_equal(ref[k], again[k]), k
    for tile in (64, 128, 512):
        for spb in (1, 2):
            for order in (pf.PF_ORDER_TILE_MAJOR, pf.PF_ORDER_STATE_MAJOR, pf.PF_ORDER_GROUPED):
                G.set_schedule(tile, spb, order)
                other = gpu_all(G, vm, va, lp, lq)
                for k in fixed:
                    assert np.array_equal(ref[k], other[k]), (k, tile, spb, order)


def test_injections_and_adjoint_bitwise_across_state_chunks():
    """The injection and adjoint launches write their row outputs with plain
    stores when a tile has at most eight state chunks and with streaming
    stores above that; the adjoint walks a workgroup's states two at a time
    (an odd count repeats the last).  40 states in chunks of 1, 4, 5, 8 and
    40 (40, 10, 8, 5 and 1 chunks per tile) give the same bits, on a grid
    with parallel branches and on one without."""
    import torch
    for g in (gridgen.grid_500(), star_grid(120, seed=5, parallel=4)):
        rng = np.random.default_rng(g.nb)
        ns = 40
        vm = rng.uniform(0.9, 1.1, (ns, g.nb))
        va = rng.normal(0, 0.3, (ns, g.nb))
        lp, lq = rng.normal(size=vm.shape), rng.normal(size=vm.shape)
        G = pf.Grid.from_grid(g)
        v, a, l1, l2 = (to_dev(x) for x in (vm, va, lp, lq))
        outs = []
        for spb in (1, 4, 5, 8, 40):
            G.set_schedule(128, spb, pf.PF_ORDER_AUTO)
            r = [torch.empty_like(v) for _ in range(4)]
            pf.pf_injections_elementwise(G, v, a, r[0], r[1])
            pf.pf_injections_vjp(G, v, a, l1, l2, r[2], r[3])
            torch.cuda.synchronize()
            outs.append([x.cpu().numpy() for x in r])
        for s in (0, 17, 39):
            o = oracle_all(g, vm[s], va[s], lp[s], lq[s])
            for k, name in enumerate(("p_ew", "q_ew", "gvm", "gva")):
                assert rel_err(outs[0][k][s], o[name]) < TOL, (g.nb, s, name)
        for spb, other in zip((4, 5, 8, 40), outs[1:]):
            for k in range(4):
                assert np.array_equal(outs[0][k], other[k]), (g.nb, spb, k)


@pytest.mark.parametrize("n_leaf,parallel", [(40, 0), (100, 3), (256, 0), (250, 6), (333, 0), (700, 25)])
def test_hub_rows_bitwise_across_schedules(n_leaf, parallel):
    """Bus sums run in chunks of 16 terms fixed by the row alone, so a hub row
    gives the same bits whether its tile packs it (tile size above its branch
    ends) or walks it in pieces of the tile size (the long-row path), for
    every tile size and states per workgroup; every run matches the oracle.
    The hub sits mid-numbering, so its bus-shunt record lies inside its row.
    256 branch ends (with and without parallel branches) fill whole pieces of
    64 and 128 exactly."""
    g = star_grid(n_leaf, seed=n_leaf, parallel=parallel)
    perm = np.arange(g.nb)
    perm[0], perm[g.nb // 2] = g.nb // 2, 0
    g = gridgen.renumber(g, perm)
    rng = np.random.default_rng(n_leaf)
    ns = 3
    vm = rng.uniform(0.9, 1.1, (ns, g.nb))
    va = rng.normal(0, 0.3, (ns, g.nb))
    lp, lq = rng.normal(size=vm.shape), rng.normal(size=vm.shape)
    G = pf.Grid.from_grid(g)
    ref = gpu_all(G, vm, va, lp, lq)
    for s in range(ns):
        compare_grid(ref, oracle_all(g, vm[s], va[s], lp[s], lq[s]), s, slice(None), slice(None), slice(None))
    fixed = [k for k in ref if not k.endswith("_ca")]
    for tile in (64, 128, 512):
        for spb in (1, 2):
            G.set_schedule(tile, spb, pf.PF_ORDER_AUTO)
            other = gpu_all(G, vm, va, lp, lq)
            for k in fixed:
                assert np.array_equal(ref[k], other[k]), (k, tile, spb)


def test_graph_replays_match_eager_calls():
    """A recorded [injections, Jacobian (both methods), VJP, Jacobian in CSC order] sequence, replayed
    several times with eager work and input changes in between; every replay
    equals the eager calls bit for bit."""
    import torch
    g = _grids.random_small(700, 1000, 41, parallel=6, isolated=3)
    rng = np.random.default_rng(5)
    ns = 3
    G = pf.Grid.from_grid(g)
    pf.pf_ybus(G)
    dev = lambda a: to_dev(a)
    vm = dev(rng.uniform(0.9, 1.1, (ns, g.nb)))
    va = dev(rng.normal(0, 0.3, (ns, g.nb)))
    lp, lq = dev(rng.normal(size=(ns, g.nb))), dev(rng.normal(size=(ns, g.nb)))
    z = lambda *sh: torch.zeros(*sh, dtype=torch.float64, device="cuda:0")
    out = {k: z(ns, g.nb) for k in ("p", "q", "p2", "q2", "p3", "q3", "gvm", "gva")}
    j_ew, j_yb, j_cs = z(ns, G.nnz_j), z(ns, G.nnz_j), z(ns, G.nnz_j)
    ops = [
        dict(op=pf.PF_OP_INJECTIONS, method=pf.PF_METHOD_ELEMENTWISE, vm=vm, va=va, out_a=out["p"], out_b=out["q"]),
        dict(op=pf.PF_OP_JACOBIAN, method=pf.PF_METHOD_ELEMENTWISE, vm=vm, va=va, out_a=out["p2"], out_b=out["q2"],
             jval=j_ew),
        dict(op=pf.PF_OP_JACOBIAN, method=pf.PF_METHOD_YBUS, vm=vm, va=va, out_a=out["p3"], out_b=out["q3"], jval=j_yb),
        dict(op=pf.PF_OP_VJP, vm=vm, va=va, lam_p=lp, lam_q=lq, out_a=out["gvm"], out_b=out["gva"]),
        dict(op=pf.PF_OP_JACOBIAN, method=pf.PF_METHOD_YBUS | pf.PF_JAC_CSC, vm=vm, va=va, jval=j_cs),
    ]
    gr = pf.Graph(G, ops)

    def eager():
        e = {k: z(ns, g.nb) for k in out}
        je, jy, jc = z(ns, G.nnz_j), z(ns, G.nnz_j), z(ns, G.nnz_j)
        pf.pf_injections_elementwise(G, vm, va, e["p"], e["q"])
        pf.pf_jacobian_values(G, pf.PF_METHOD_ELEMENTWISE, vm, va, e["p2"], e["q2"], je)
        pf.pf_jacobian_values(G, pf.PF_METHOD_YBUS, vm, va, e["p3"], e["q3"], jy)
        pf.pf_injections_vjp(G, vm, va, lp, lq, e["gvm"], e["gva"])
        pf.pf_jacobian_values(G, pf.PF_METHOD_YBUS | pf.PF_JAC_CSC, vm, va, None, None, jc)
        torch.cuda.synchronize()
        return {k: v.cpu().numpy() for k, v in e.items()}, je.cpu().numpy(), jy.cpu().numpy(), jc.cpu().numpy()

    for rep in range(4):
        for t in list(out.values()) + [j_ew, j_yb, j_cs]:
            t.fill_(float("nan"))
        gr.launch()
        torch.cuda.synchronize()
        want, je, jy, jc = eager()
        for k in out:
            assert np.array_equal(out[k].cpu().numpy(), want[k]), (rep, k)
        assert np.array_equal(j_ew.cpu().numpy(), je), rep
        assert np.array_equal(j_yb.cpu().numpy(), jy), rep
        assert np.array_equal(j_cs.cpu().numpy(), jc), rep
        vm.mul_(1.0 + 0.01 * (rep + 1))  # the next replay reads the new inputs
        va.add_(0.02)
    # within tolerance of the oracle too (last inputs, state 0)
    ores = oracle_all(g, vm[0].cpu().numpy(), va[0].cpu().numpy())
    gr.launch()
    torch.cuda.synchronize()
    assert rel_err(j_ew[0].cpu().numpy(), ores["j_ew"], ores["scale"]) <= TOL
    # a schedule change invalidates the recording
    G.set_schedule(128, 0)
    with pytest.raises(pf.PFError) as e:
        gr.launch()
    assert e.value.code == pf.PF_ESTATE
    gr.close()
    with pytest.raises(pf.PFError) as e:  # Ybus op on a handle without pf_ybus
        pf.Graph(pf.Grid.from_grid(g), ops[2:3])
    assert e.value.code == pf.PF_ESTATE


def test_graph_replays_several_states_per_workgroup():
    """Injections, S+J and the VJP with 4 states per workgroup (the
    multi-state kernels; the injections and the VJP with plain row stores),
    recorded once and replayed several times with the inputs changed in
    between; every replay equals the eager calls bit for bit."""
    import torch
    g = gridgen.grid_500()
    rng = np.random.default_rng(11)
    ns = 10
    G = pf.Grid.from_grid(g)
    G.set_schedule(128, 4, pf.PF_ORDER_AUTO)
    vm = to_dev(rng.uniform(0.9, 1.1, (ns, g.nb)))
    va = to_dev(rng.normal(0, 0.3, (ns, g.nb)))
    lp, lq = to_dev(rng.normal(size=(ns, g.nb))), to_dev(rng.normal(size=(ns, g.nb)))
    z = lambda *sh: torch.zeros(*sh, dtype=torch.float64, device="cuda:0")
    out = {k: z(ns, g.nb) for k in ("p", "q", "p2", "q2", "gvm", "gva")}
    jv = z(ns, G.nnz_j)
    ops = [
        dict(op=pf.PF_OP_INJECTIONS, method=pf.PF_METHOD_ELEMENTWISE, vm=vm, va=va, out_a=out["p"], out_b=out["q"]),
        dict(op=pf.PF_OP_JACOBIAN, method=pf.PF_METHOD_ELEMENTWISE, vm=vm, va=va, out_a=out["p2"], out_b=out["q2"],
             jval=jv),
        dict(op=pf.PF_OP_VJP, vm=vm, va=va, lam_p=lp, lam_q=lq, out_a=out["gvm"], out_b=out["gva"]),
    ]
    gr = pf.Graph(G, ops)
    for rep in range(4):
        for t in list(out.values()) + [jv]:
            t.fill_(float("nan"))
        gr.launch()
        torch.cuda.synchronize()
        e = {k: z(ns, g.nb) for k in out}
        je = z(ns, G.nnz_j)
        pf.pf_injections_elementwise(G, vm, va, e["p"], e["q"])
        pf.pf_jacobian_values(G, pf.PF_METHOD_ELEMENTWISE, vm, va, e["p2"], e["q2"], je)
        pf.pf_injections_vjp(G, vm, va, lp, lq, e["gvm"], e["gva"])
        torch.cuda.synchronize()
        for k in out:
            assert np.array_equal(out[k].cpu().numpy(), e[k].cpu().numpy()), (rep, k)
        assert np.array_equal(jv.cpu().numpy(), je.cpu().numpy()), rep
        vm.mul_(1.0 + 0.01 * (rep + 1))
        va.add_(0.02)
    o = oracle_all(g, vm[3].cpu().numpy(), va[3].cpu().numpy(), lp[3].cpu().numpy(), lq[3].cpu().numpy())
    gr.launch()
    torch.cuda.synchronize()
    for k, name in (("p", "p_ew"), ("q", "q_ew"), ("gvm", "gvm"), ("gva", "gva")):
        assert rel_err(out[k][3].cpu().numpy(), o[name]) <= TOL, k
    gr.close()


def test_graph_multigrid_and_baselines():
    """A recorded sequence on a freshly built multi-grid handle (no evaluation
    call before recording) with several states: fused element-wise and Ybus
    Jacobians, the two-phase baseline (its scratch belongs to the handle from
    the build on) and the atomic copy-add baseline.  Replays
    equal the eager calls bit for bit (copy-add: to rounding, its additions
    run in no fixed order) and every grid matches the oracle."""
    import torch
    grids = [_grids.random_small(n, int(n * 1.4), 90 + n, parallel=n % 3, isolated=1) for n in (60, 7, 400)]
    grids.append(star_grid(300, seed=4))
    big, bo, ro = gridgen.concat(grids)
    G = pf.Grid.from_grid(big, bo, ro)
    pf.pf_ybus(G)
    ns = 2
    rng = np.random.default_rng(8)
    vm = to_dev(rng.uniform(0.9, 1.1, (ns, big.nb)))
    va = to_dev(rng.normal(0, 0.2, (ns, big.nb)))
    z = lambda *sh: torch.zeros(*sh, dtype=torch.float64, device="cuda:0")
    methods = (pf.PF_METHOD_ELEMENTWISE, pf.PF_METHOD_YBUS, pf.PF_METHOD_ELEMENTWISE_TWO_PHASE,
               pf.PF_METHOD_ELEMENTWISE_ATOMIC)
    outs = [(z(ns, big.nb), z(ns, big.nb), z(ns, G.nnz_j)) for _ in methods]
    ops = [dict(op=pf.PF_OP_JACOBIAN, method=m, vm=vm, va=va, out_a=o[0], out_b=o[1], jval=o[2])
           for m, o in zip(methods, outs)]
    gr = pf.Graph(G, ops)
    y_off, j_off = G.offsets()
    for rep in range(3):
        for o in outs:
            for t in o:
                t.fill_(float("nan"))
        gr.launch()
        torch.cuda.synchronize()
        for m, o in zip(methods, outs):
            e = (z(ns, big.nb), z(ns, big.nb), z(ns, G.nnz_j))
            pf.pf_jacobian_values(G, m, vm, va, *e)
            torch.cuda.synchronize()
            for a, b in zip(o, e):
                a, b = a.cpu().numpy(), b.cpu().numpy()
                if m == pf.PF_METHOD_ELEMENTWISE_ATOMIC:
                    assert rel_err(a, b) <= TOL, (rep, m)
                else:
                    assert np.array_equal(a, b), (rep, m)
        vm_h, va_h = vm.cpu().numpy(), va.cpu().numpy()
        for k, g in enumerate(grids):
            bsl = slice(bo[k], bo[k + 1])
            jsl = slice(j_off[k], j_off[k + 1])
            for s in range(ns):
                ores = oracle_all(g, vm_h[s, bsl], va_h[s, bsl])
                for m, o in zip(methods, outs):
                    key = "yb" if m == pf.PF_METHOD_YBUS else "ew"
                    assert rel_err(o[0][s, bsl].cpu().numpy(), ores["p_" + key]) <= TOL, (rep, k, s, m)
                    assert rel_err(o[2][s, jsl].cpu().numpy(), ores["j_" + key]) <= TOL, (rep, k, s, m)
        vm.mul_(1.01)
        va.add_(0.03)
    gr.close()


def test_ybus_required_before_ybus_calls():
    import torch
    G = pf.Grid.from_grid(gridgen.grid_500())
    z = torch.zeros(1, G.nb, dtype=torch.float64, device="cuda:0")
    with pytest.raises(pf.PFError) as e:
        pf.pf_injections_ybus(G, z, z, z.clone(), z.clone())
    assert e.value.code == pf.PF_ESTATE
    j = torch.zeros(1, G.nnz_j, dtype=torch.float64, device="cuda:0")
    with pytest.raises(pf.PFError) as e:
        pf.pf_jacobian_values(G, pf.PF_METHOD_YBUS, z, z, None, None, j)
    assert e.value.code == pf.PF_ESTATE


def test_jval_alignment_checked():
    import torch
    G = pf.Grid.from_grid(gridgen.grid_500())
    z = torch.zeros(1, G.nb, dtype=torch.float64, device="cuda:0")
    jbig = torch.zeros(G.nnz_j + 1, dtype=torch.float64, device="cuda:0")
    rc = pf.lib().pf_jacobian_values(G.handle, 0, 1, z.data_ptr(), z.data_ptr(), None, None,
                                     jbig.data_ptr() + 8, None)
    assert rc == pf.PF_EINVAL


# ------------------------------------------------------------------ full sizes

def test_grid_100k_full_size():
    """100k buses, one state, in the benchmark's launch configuration."""
    g = gridgen.grid_100k()
    vm, va = gridgen.states(g.nb, 1, case=1)
    G = pf.Grid.from_grid(g)
    rng = np.random.default_rng(11)
    lp, lq = rng.normal(size=vm.shape), rng.normal(size=vm.shape)
    gres = gpu_all(G, vm, va, lp, lq)
    ores = oracle_all(g, vm[0], va[0], lp[0], lq[0])
    errs = compare_grid(gres, ores, 0, slice(None), slice(None), slice(None))
    print(dict(errs))


def test_relabelled_grids():
    """Bus numbering without locality (a seeded random relabelling): remote
    buses of a tile lie anywhere in the state arrays.  Every call on the
    relabelled 500-bus grid, and S+J by both methods on the relabelled
    100k-bus grid, against the oracle on the same relabelled grid."""
    g, perm = gridgen.relabel(gridgen.grid_500(), case=0)
    vm, va = gridgen.states(g.nb, 2, case=0)
    check_single(g, vm, va)
    import torch
    g, perm = gridgen.relabel(gridgen.grid_100k(), case=1)
    vm, va = gridgen.states(g.nb, 1, case=1)
    G = pf.Grid.from_grid(g)
    pf.pf_ybus(G)
    ores = oracle_all(g, vm[0], va[0])
    vm_d, va_d = to_dev(vm), to_dev(va)
    for method, key in ((pf.PF_METHOD_ELEMENTWISE, "ew"), (pf.PF_METHOD_YBUS, "yb")):
        p = torch.empty(1, G.nb, dtype=torch.float64, device="cuda:0")
        q = torch.empty_like(p)
        j = torch.empty(1, G.nnz_j, dtype=torch.float64, device="cuda:0")
        pf.pf_jacobian_values(G, method, vm_d, va_d, p, q, j)
        torch.cuda.synchronize()
        assert rel_err(p[0].cpu().numpy(), ores["p_" + key]) <= TOL
        assert rel_err(q[0].cpu().numpy(), ores["q_" + key]) <= TOL
        assert rel_err(j[0].cpu().numpy(), ores["j_" + key]) <= TOL


def test_grid_20k_batched_sampled_states():
    """20k buses x 512 states in one launch; six sampled states compared in full."""
    import torch
    g = gridgen.grid_20k()
    B = 512
    vm, va = gridgen.states(g.nb, B, case=2, vlo=0.9, vhi=1.1, sigma=0.3)
    G = pf.Grid.from_grid(g)
    vm_d, va_d = to_dev(vm), to_dev(va)
    p = torch.empty(B, G.nb, dtype=torch.float64, device="cuda:0")
    q = torch.empty_like(p)
    j = torch.empty(B, G.nnz_j, dtype=torch.float64, device="cuda:0")
    pf.pf_jacobian_values(G, pf.PF_METHOD_ELEMENTWISE, vm_d, va_d, p, q, j)
    torch.cuda.synchronize()
    for s in (0, 1, 255, 256, 400, 511):
        ores = oracle_all(g, vm[s], va[s])
        assert rel_err(p[s].cpu().numpy(), ores["p_ew"]) <= TOL
        assert rel_err(q[s].cpu().numpy(), ores["q_ew"]) <= TOL
        assert rel_err(j[s].cpu().numpy(), ores["j_ew"]) <= TOL


def test_uneven_grids_64x4():
    """64 grids (1k-80k buses), 4 states each, one launch; every grid and state compared."""
    grids = gridgen.grids_uneven_64()
    big, bo, ro = gridgen.concat(grids)
    G = pf.Grid.from_grid(big, bo, ro)
    vm = np.concatenate([gridgen.states(gr.nb, 4, case=3, grid=k + 1)[0] for k, gr in enumerate(grids)], axis=1)
    va = np.concatenate([gridgen.states(gr.nb, 4, case=3, grid=k + 1)[1] for k, gr in enumerate(grids)], axis=1)
    gres = gpu_all(G, vm, va, with_ybus=False)
    y_off, j_off = G.offsets()
    for k, gr in enumerate(grids):
        bsl = slice(bo[k], bo[k + 1])
        yb = oracle.ybus(gr)
        pat = oracle.jac_pattern(yb)
        for s in range(4):
            p, q = oracle.inject_ew(gr, vm[s, bsl], va[s, bsl])
            jv = oracle.jac_ew(gr, vm[s, bsl], va[s, bsl], pat)
            assert rel_err(gres["p_ew"][s, bsl], p) <= TOL
            assert rel_err(gres["q_ew"][s, bsl], q) <= TOL
            assert rel_err(gres["j_ew"][s, j_off[k]:j_off[k + 1]], jv) <= TOL


def test_adjoint_100k_x32_against_oracle_and_fd():
    """100k buses x 32 states, the batched workload's launch configuration
    (automatic schedule): the injections and the VJP against the oracle on
    sampled states (the VJP as J^T lambda of the oracle Jacobian), and the VJP
    against central differences (h = 1e-7) on 1000 sampled coordinates."""
    import torch
    g = gridgen.grid_100k()
    B = 32
    vm, va = gridgen.states(g.nb, B, case=4)
    lp, lq = gridgen.adjoint_seeds(g.nb, B, case=4)
    G = pf.Grid.from_grid(g)
    vm_d, va_d, lp_d, lq_d = map(to_dev, (vm, va, lp, lq))
    gvm = torch.empty_like(vm_d)
    gva = torch.empty_like(vm_d)
    pf.pf_injections_vjp(G, vm_d, va_d, lp_d, lq_d, gvm, gva)
    p_all, q_all = torch.empty_like(vm_d), torch.empty_like(vm_d)
    pf.pf_injections_elementwise(G, vm_d, va_d, p_all, q_all)
    torch.cuda.synchronize()
    gvm_h, gva_h = gvm.cpu().numpy(), gva.cpu().numpy()
    p_h, q_h = p_all.cpu().numpy(), q_all.cpu().numpy()
    yb = oracle.ybus(g)
    pat = oracle.jac_pattern(yb)
    for s in (0, 13, 31):
        op, oq = oracle.inject_ew(g, vm[s], va[s])
        assert rel_err(p_h[s], op) <= TOL
        assert rel_err(q_h[s], oq) <= TOL
        jv = oracle.jac_ybus(yb, vm[s], va[s], pat)
        ovm, ova = oracle.vjp(g.nb, pat, jv, lp[s], lq[s])
        assert rel_err(gvm_h[s], ovm) <= TOL
        assert rel_err(gva_h[s], ova) <= TOL
    # central differences of the local objective sum_{i in N(k)} lP_i P_i + lQ_i Q_i
    coords = gridgen.sample_coords(B, g.nb, 1000, case=4)
    nbrs = [[] for _ in range(g.nb)]
    for a, c in zip(g.fbus.tolist(), g.tbus.tolist()):
        nbrs[a].append(c)
        nbrs[c].append(a)
    h = 1e-7
    chunk = 250
    worst = 0.0
    for c0 in range(0, len(coords), chunk):
        cs = coords[c0:c0 + chunk]
        n = len(cs)
        vmp = np.repeat(vm[cs[:, 0]], 2, axis=0)
        vap = np.repeat(va[cs[:, 0]], 2, axis=0)
        for r, (s, var, k) in enumerate(cs):
            arr = vmp if var == 0 else vap
            arr[2 * r, k] += h
            arr[2 * r + 1, k] -= h
        vmd, vad = to_dev(vmp), to_dev(vap)
        p = torch.empty_like(vmd)
        q = torch.empty_like(vmd)
        pf.pf_injections_elementwise(G, vmd, vad, p, q)
        torch.cuda.synchronize()
        for r, (s, var, k) in enumerate(cs):
            loc = np.array([k] + nbrs[k])
            pp = p[2 * r, loc].cpu().numpy() - p[2 * r + 1, loc].cpu().numpy()
            qq = q[2 * r, loc].cpu().numpy() - q[2 * r + 1, loc].cpu().numpy()
            fd = (lp[s, loc] @ pp + lq[s, loc] @ qq) / (2 * h)
            gv = gvm_h[s, k] if var == 0 else gva_h[s, k]
            err = abs(fd - gv) / (1 + abs(gv))
            worst = max(worst, err)
            assert err <= 1e-6, (s, var, k, fd, gv)
    print("worst FD error", worst)


def test_autograd_function():
    import torch
    from paper_2302_10736_amd.autograd import injections
    g = _grids.random_small(12, 20, 4, parallel=2, isolated=1)
    G = pf.Grid.from_grid(g)
    vm, va = _grids.random_state(g.nb, 9)
    vm_t = to_dev(vm[None]).requires_grad_(True)
    va_t = to_dev(va[None]).requires_grad_(True)
    assert torch.autograd.gradcheck(lambda a, b: injections(G, a, b), (vm_t, va_t), eps=1e-7, atol=1e-6)
    P, Q = injections(G, vm_t, va_t)
    w = torch.linspace(-1, 1, g.nb, dtype=torch.float64, device="cuda:0")
    (P * w).sum().backward()
    assert vm_t.grad is not None and va_t.grad is not None


def test_bound_calls_match_plain_calls():
    """pf.bind: arguments marshalled once, each call only calls the library;
    same results as the plain calls, also after the inputs change in place."""
    import torch
    g = gridgen.grid_500()
    vm, va = gridgen.states(g.nb, 3, case=0)
    G = pf.Grid.from_grid(g)
    pf.pf_ybus(G)
    vmd, vad = to_dev(vm), to_dev(va)
    z = lambda *sh: torch.full(sh, float("nan"), dtype=torch.float64, device="cuda:0")
    p1, q1, j1, p2, q2, j2 = z(3, G.nb), z(3, G.nb), z(3, G.nnz_j), z(3, G.nb), z(3, G.nb), z(3, G.nnz_j)
    gv1, ga1, gv2, ga2 = z(3, G.nb), z(3, G.nb), z(3, G.nb), z(3, G.nb)
    calls = [pf.bind(pf.pf_jacobian_values, G, pf.PF_METHOD_ELEMENTWISE, vmd, vad, p1, q1, j1),
             pf.bind(pf.pf_injections_vjp, G, vmd, vad, p1, q1, gv1, ga1)]
    for rep in range(2):
        for c in calls:
            c()
        pf.pf_jacobian_values(G, pf.PF_METHOD_ELEMENTWISE, vmd, vad, p2, q2, j2)
        pf.pf_injections_vjp(G, vmd, vad, p2, q2, gv2, ga2)
        torch.cuda.synchronize()
        for a, b in ((p1, p2), (q1, q2), (j1, j2), (gv1, gv2), (ga1, ga2)):
            assert torch.equal(a, b), rep
        vad.add_(0.01)  # new inputs in the same buffers
    yb_call = pf.bind(pf.pf_injections_ybus, G, vmd, vad, p1, q1)
    yb_call()
    pf.pf_injections_ybus(G, vmd, vad, p2, q2)
    torch.cuda.synchronize()
    assert torch.equal(p1, p2) and torch.equal(q1, q2)


@pytest.mark.parametrize("seed", range(12))
def test_random_hub_grids_and_schedules(seed):
    """Randomised long rows: hub buses of 65 to 1,500 branches (walked in pieces, with the chunk
    sums of one piece folded beside the next piece's), parallel branches among them, random
    schedule and batch size; every call against the oracle, and bitwise against the initial
    schedule."""
    rng = np.random.default_rng(7000 + seed)
    g = _grids.random_hubs(int(rng.integers(300, 3000)), int(rng.integers(1, 6)), 65,
                           int(rng.integers(100, 1500)), int(rng.integers(0, 30)), 7100 + seed)
    ns = int(rng.integers(1, 6))
    vm = rng.uniform(0.9, 1.1, (ns, g.nb))
    va = rng.normal(0, 0.3, (ns, g.nb))
    lp, lq = rng.normal(size=vm.shape), rng.normal(size=vm.shape)
    tile = int(rng.choice([64, 128, 256, 512]))
    spb = int(rng.choice([0, 1, 2, 3, 5]))
    order = int(rng.choice([pf.PF_ORDER_AUTO, pf.PF_ORDER_TILE_MAJOR, pf.PF_ORDER_STATE_MAJOR, pf.PF_ORDER_GROUPED]))
    print(f"seed {seed}: nb {g.nb} nl {g.nl} states {ns} schedule {tile},{spb},{order}")
    G = pf.Grid.from_grid(g)
    ref = gpu_all(G, vm, va, lp, lq)
    G.set_schedule(tile, spb, order)
    got = gpu_all(G, vm, va, lp, lq)
    for k in ref:
        if not k.endswith("_ca"):  # copy-add: atomic adds in no fixed order
            assert np.array_equal(ref[k], got[k]), k
    for s in range(ns):
        compare_grid(got, oracle_all(g, vm[s], va[s], lp[s], lq[s]), s, slice(None), slice(None), slice(None))


@pytest.mark.parametrize("seed", range(40))
def test_random_grids_and_schedules(seed):
    """Randomised sweep: grid size and shape (parallel branches, isolated
    buses, transformer share), tile size, states per workgroup, order and
    batch size drawn per seed; every call against the oracle, state by state."""
    rng = np.random.default_rng(1000 + seed)
    nb = int(rng.integers(2, 900))
    iso = int(rng.integers(0, min(5, nb - 2) + 1))
    live = nb - iso
    nl = int(rng.integers(live - 1, 2 * live + 2))
    par = int(rng.integers(0, 6))
    g = _grids.random_small(nb, max(nl, live - 1 + par), 2000 + seed, parallel=par, isolated=iso,
                            xf_frac=float(rng.uniform(0, 0.6)))
    ns = int(rng.integers(1, 6))
    vm = rng.uniform(0.9, 1.1, (ns, g.nb))
    va = rng.normal(0, 0.25, (ns, g.nb))
    tile = int(rng.choice([64, 128, 256, 512]))
    spb = int(rng.choice([0, 1, 2, 3]))
    order = int(rng.choice([pf.PF_ORDER_AUTO, pf.PF_ORDER_TILE_MAJOR, pf.PF_ORDER_STATE_MAJOR, pf.PF_ORDER_GROUPED]))
    print(f"seed {seed}: nb {g.nb} nl {g.nl} parallel {par} isolated {iso} states {ns} schedule {tile},{spb},{order}")
    check_single(g, vm, va, tile=tile, spb=spb, order=order, use_scale=g.nb <= 3)
