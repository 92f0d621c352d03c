"""GPU parity where output element offsets pass 2^31.

290,000 states of the 500-bus grid make the Jacobian output
290,000 x 7,600 = 2.20e9 values (17.6 GB) and the branch-flow partials
290,000 x 16 x 700 = 3.25e9 values (26 GB), so every state past
state 282,563 (Jacobian) or 191,739 (flow partials) sits at an offset
that a 32-bit index would wrap.  The batch repeats eight seeded states; the
sampled states on both sides of those boundaries must equal, bit for bit,
the results of the same eight states evaluated as a small batch, which are
themselves checked against the oracle.  Results do not depend on the
schedule or on a state's position in the batch (fixed summation order), so
bitwise equality is the gate.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2302_10736_amd import gridgen, pf
from tests._gpu import TOL, rel_err, require_gpu, to_dev

pytestmark = pytest.mark.gpu

NSTATE = 290_000
NBASE = 8
NEED_BYTES = 64 << 30  # peak of the largest step below, with margin


@pytest.fixture(scope="module")
def setup():
    import torch
    require_gpu()
    free, _ = torch.cuda.mem_get_info()
    if free < NEED_BYTES:
        pytest.skip(f"needs {NEED_BYTES >> 30} GiB of free device memory, {free >> 30} GiB free")
    g = gridgen.grid_500()
    G = pf.Grid.from_grid(g)
    G.set_schedule(256, 0, pf.PF_ORDER_AUTO)
    vm, va = gridgen.states(g.nb, NBASE, case=0)
    base_vm, base_va = to_dev(vm), to_dev(va)
    idx = torch.arange(NSTATE, device="cuda:0") % NBASE
    big_vm, big_va = base_vm[idx].contiguous(), base_va[idx].contiguous()
    torch.cuda.synchronize()
    yield g, G, vm, va, base_vm, base_va, big_vm, big_va
    del big_vm, big_va
    torch.cuda.empty_cache()


def sampled(boundary):
    """States to compare: both batch ends, around the 2^31 boundary, and a few between."""
    rng = np.random.default_rng(31)
    s = {0, 1, boundary - 1, boundary, boundary + 1, NSTATE - 2, NSTATE - 1}
    s.update(int(x) for x in rng.integers(0, NSTATE, 5))
    return sorted(s)


def first_wrapping_state(per_state):
    """Smallest state whose last element lies at offset >= 2^31."""
    return (2**31 - 1) // per_state


def z(*shape):
    import torch
    return torch.empty(*shape, dtype=torch.float64, device="cuda:0")


@pytest.mark.parametrize("method", [pf.PF_METHOD_ELEMENTWISE, pf.PF_METHOD_YBUS])
def test_jacobian_values_past_2g_elements(setup, method):
    import torch
    g, G, vm, va, base_vm, base_va, big_vm, big_va = setup
    if method == pf.PF_METHOD_YBUS:
        pf.pf_ybus(G)
    nj = G.nnz_j
    assert NSTATE * nj > 2**31
    p0, q0, j0 = z(NBASE, G.nb), z(NBASE, G.nb), z(NBASE, nj)
    pf.pf_jacobian_values(G, method, base_vm, base_va, p0, q0, j0)
    p1, q1, j1 = z(NSTATE, G.nb), z(NSTATE, G.nb), z(NSTATE, nj)
    pf.pf_jacobian_values(G, method, big_vm, big_va, p1, q1, j1)
    torch.cuda.synchronize()
    p0, q0, j0 = p0.cpu().numpy(), q0.cpu().numpy(), j0.cpu().numpy()
    yb = oracle.ybus(g)
    pat = oracle.jac_pattern(yb)
    for b in range(NBASE):
        if method == pf.PF_METHOD_ELEMENTWISE:
            po, qo = oracle.inject_ew(g, vm[b], va[b])
            jo = oracle.jac_ew(g, vm[b], va[b], pat)
        else:
            po, qo = oracle.inject_ybus(yb, vm[b], va[b])
            jo = oracle.jac_ybus(yb, vm[b], va[b], pat)
        for name, got, want in (("P", p0[b], po), ("Q", q0[b], qo), ("J", j0[b], jo)):
            e = rel_err(got, want)
            assert e <= TOL, f"{name} state {b}: relative error {e:.3e}"
    for s in sampled(first_wrapping_state(nj)):
        b = s % NBASE
        assert np.array_equal(j1[s].cpu().numpy(), j0[b]), f"J differs at state {s}"
        assert np.array_equal(p1[s].cpu().numpy(), p0[b]), f"P differs at state {s}"
        assert np.array_equal(q1[s].cpu().numpy(), q0[b]), f"Q differs at state {s}"
    del p1, q1, j1
    torch.cuda.empty_cache()


def test_branch_flow_partials_past_2g_elements(setup):
    import torch
    g, G, vm, va, base_vm, base_va, big_vm, big_va = setup
    nl = G.nl
    assert NSTATE * 16 * nl > 2**31
    f0 = [z(NBASE, nl) for _ in range(4)]
    fj0 = z(NBASE, 16, nl)
    pf.pf_branch_flows(G, base_vm, base_va, *f0, fj0)
    f1 = [z(NSTATE, nl) for _ in range(4)]
    fj1 = z(NSTATE, 16, nl)
    pf.pf_branch_flows(G, big_vm, big_va, *f1, fj1)
    torch.cuda.synchronize()
    f0 = [t.cpu().numpy() for t in f0]
    fj0 = fj0.cpu().numpy()
    for b in range(NBASE):
        want = oracle.branch_flows(g, vm[b], va[b])
        for n in range(4):
            e = rel_err(f0[n][b], want[n])
            assert e <= TOL, f"flow {n} state {b}: relative error {e:.3e}"
        e = rel_err(fj0[b], oracle.branch_flow_jac(g, vm[b], va[b]))
        assert e <= TOL, f"flow partials state {b}: relative error {e:.3e}"
    for s in sampled(first_wrapping_state(16 * nl)):
        b = s % NBASE
        assert np.array_equal(fj1[s].cpu().numpy(), fj0[b]), f"flow partials differ at state {s}"
        for n in range(4):
            assert np.array_equal(f1[n][s].cpu().numpy(), f0[n][b]), f"flow {n} differs at state {s}"
    del f1, fj1
    torch.cuda.empty_cache()
