"""Autotuner host logic (CPU) and a device run (GPU)."""
from __future__ import annotations

import json

import numpy as np
import pytest

from paper_2302_10736_amd import autotune, gridgen, pf
from tests import _grids


def test_candidates():
    one = autotune.candidates(1)
    assert one == [(t, 1, pf.PF_ORDER_TILE_MAJOR) for t in autotune.TILES]
    many = autotune.candidates(12)
    assert (256, 0, pf.PF_ORDER_TILE_MAJOR) in many and (64, 8, pf.PF_ORDER_STATE_MAJOR) in many
    assert (128, 1, pf.PF_ORDER_GROUPED) in many
    assert all(s <= 12 for _, s, _ in many)
    assert len(many) == len(set(many)) == len(autotune.TILES) * 5 * 3  # spb in {0, 1, 2, 4, 8}, three orders


def test_tune_picks_fastest_and_caches(tmp_path):
    G = pf.Grid.from_grid(_grids.random_small(40, 60, 3), host_only=True)
    path = tmp_path / "sched.json"
    cache = autotune.ScheduleCache(str(path))
    cost = {(128, 4, pf.PF_ORDER_STATE_MAJOR): 1.0e-6}
    seen = []

    def fake(s):
        seen.append(s)
        return cost.get(tuple(s), 5.0e-6)

    res = autotune.tune(G, "jacobian_ew", 8, cache=cache, measure=fake, device="dev", lib="lib")
    assert res["schedule"] == (128, 4, pf.PF_ORDER_STATE_MAJOR)
    assert G.schedule()[:3] == (128, 4, pf.PF_ORDER_STATE_MAJOR)
    assert len(seen) == res["tried"] == len(autotune.candidates(8))
    data = json.loads(path.read_text())
    assert data[res["key"]]["schedule"] == [128, 4, pf.PF_ORDER_STATE_MAJOR]
    # a fresh handle of the same shape picks the cached schedule; other shapes do not
    G2 = pf.Grid.from_grid(_grids.random_small(40, 60, 3), host_only=True)
    assert autotune.apply(G2, "jacobian_ew", 8, cache=autotune.ScheduleCache(str(path)), device="dev",
                          lib="lib") == (128, 4, pf.PF_ORDER_STATE_MAJOR)
    assert G2.schedule()[:3] == (128, 4, pf.PF_ORDER_STATE_MAJOR)
    assert autotune.apply(G2, "jacobian_ew", 9, cache=autotune.ScheduleCache(str(path)), device="dev",
                          lib="lib") is None
    assert autotune.apply(G2, "jacobian_ew", 8, cache=autotune.ScheduleCache(str(path)), device="dev",
                          lib="other build") is None


def test_unreadable_cache_starts_empty(tmp_path):
    p = tmp_path / "bad.json"
    p.write_text("{not json")
    assert autotune.ScheduleCache(str(p)).entries == {}


def test_unknown_op_rejected():
    G = pf.Grid.from_grid(_grids.random_small(10, 12, 1), host_only=True)
    with pytest.raises(ValueError):
        autotune.problem_key(G, "jacobian", 1, "d", "l")


@pytest.mark.gpu
def test_tune_on_device_keeps_results(tmp_path):
    import torch
    from tests._gpu import to_dev
    g = gridgen.grid_500()
    G = pf.Grid.from_grid(g)
    rng = np.random.default_rng(4)
    vm, va = to_dev(rng.uniform(0.95, 1.05, (6, g.nb))), to_dev(rng.normal(0, 0.2, (6, g.nb)))
    z = lambda *s: torch.zeros(*s, dtype=torch.float64, device="cuda:0")
    p0, q0, j0 = z(6, g.nb), z(6, g.nb), z(6, G.nnz_j)
    pf.pf_jacobian_values(G, pf.PF_METHOD_ELEMENTWISE, vm, va, p0, q0, j0)
    cache = autotune.ScheduleCache(str(tmp_path / "s.json"))
    res = autotune.tune(G, "jacobian_ew", 6, cache=cache, cands=autotune.candidates(6)[::7])
    assert G.schedule()[:3] == tuple(res["schedule"]) and res["us"] > 0
    p1, q1, j1 = z(6, g.nb), z(6, g.nb), z(6, G.nnz_j)
    pf.pf_jacobian_values(G, pf.PF_METHOD_ELEMENTWISE, vm, va, p1, q1, j1)
    torch.cuda.synchronize()
    assert torch.equal(j0, j1) and torch.equal(p0, p1) and torch.equal(q0, q1)


def test_native_tuner_argument_checks():
    """pf_autotune rejects bad arguments on the host (CPU, host-only handle)."""
    import ctypes as C
    G = pf.Grid.from_grid(_grids.random_small(10, 12, 1), host_only=True)
    L = pf.lib()
    best = (C.c_int32 * 3)()
    op = pf.PfOp()
    op.op, op.method, op.nstate = pf.PF_OP_JACOBIAN, pf.PF_METHOD_ELEMENTWISE, 1
    assert L.pf_autotune(None, C.byref(op), 0, None, 5, best, None, None) == pf.PF_EINVAL
    assert L.pf_autotune(G.handle, None, 0, None, 5, best, None, None) == pf.PF_EINVAL
    assert L.pf_autotune(G.handle, C.byref(op), 0, None, 5, best, None, None) == pf.PF_ESTATE


@pytest.mark.gpu
def test_native_tuner_default_and_given_candidates():
    """pf_autotune through the C ABI: it times the default candidate set (one
    state) and a caller's list (several states), leaves the best schedule on
    the handle, and the results stay bit for bit what they were."""
    import torch
    from tests._gpu import to_dev
    g = gridgen.grid_500()
    G = pf.Grid.from_grid(g)
    rng = np.random.default_rng(9)
    for ns, cands in ((1, None), (5, [(128, 2, pf.PF_ORDER_TILE_MAJOR), (256, 0, pf.PF_ORDER_STATE_MAJOR),
                                      (64, 5, pf.PF_ORDER_TILE_MAJOR)])):
        vm, va = to_dev(rng.uniform(0.95, 1.05, (ns, g.nb))), to_dev(rng.normal(0, 0.2, (ns, g.nb)))
        z = lambda *s: torch.zeros(*s, dtype=torch.float64, device="cuda:0")
        p0, q0, j0 = z(ns, g.nb), z(ns, g.nb), z(ns, G.nnz_j)
        pf.pf_jacobian_values(G, pf.PF_METHOD_ELEMENTWISE, vm, va, p0, q0, j0)
        torch.cuda.synchronize()
        a, b, j = z(ns, g.nb), z(ns, g.nb), z(ns, G.nnz_j)
        op = dict(op=pf.PF_OP_JACOBIAN, method=pf.PF_METHOD_ELEMENTWISE, vm=vm, va=va, out_a=a, out_b=b, jval=j)
        best, us, tried = pf.pf_autotune(G, op, cands, reps=3)
        assert tried == (len(autotune.TILES) if cands is None else len(cands)) and us > 0
        assert G.schedule()[:3] == best
        if cands is not None:
            assert best in cands
        assert torch.equal(j, j0) and torch.equal(a, p0) and torch.equal(b, q0)
        p1, q1, j1 = z(ns, g.nb), z(ns, g.nb), z(ns, G.nnz_j)
        pf.pf_jacobian_values(G, pf.PF_METHOD_ELEMENTWISE, vm, va, p1, q1, j1)
        torch.cuda.synchronize()
        assert torch.equal(j1, j0) and torch.equal(p1, p0)
