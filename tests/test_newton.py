"""Newton-Raphson loop: host logic on the CPU, the GPU-evaluated loop against
a reference loop written here on the oracle's S and Jacobian."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2302_10736_amd import gridgen, newton, pf


def test_reduced_index():
    bt = np.array([newton.SLACK, newton.PQ, newton.PV, newton.PQ])
    pvpq, pq, rows, cols = newton._reduced_index(4, bt)
    assert pvpq.tolist() == [1, 2, 3] and pq.tolist() == [1, 3]
    assert rows.tolist() == [1, 2, 3, 5, 7] and cols.tolist() == [1, 2, 3, 5, 7]


def test_reduced_map_matches_slicing():
    import scipy.sparse as sp
    g = gridgen.grid_500()
    yb = oracle.ybus(g)
    jr, jc = oracle.jac_pattern(yb)
    vm, va = gridgen.states(g.nb, 1, case=0)
    jv = oracle.jac_ew(g, vm[0], va[0], (jr, jc))
    bt = np.full(g.nb, newton.PQ)
    bt[::5] = newton.PV
    bt[0] = newton.SLACK
    _, _, rows, cols = newton._reduced_index(g.nb, bt)
    take, ind, ptr, shape = newton._reduced_map(jr, jc, rows, cols)
    A = sp.csc_matrix((jv[take], ind, ptr), shape=shape)
    B = sp.csr_matrix((jv, jc, jr), shape=(2 * g.nb, 2 * g.nb))[rows][:, cols].tocsc()
    assert A.shape == B.shape and A.nnz == B.nnz and abs(A - B).max() == 0.0


def test_case_from_state():
    g = gridgen.grid_500()
    vm, va = gridgen.states(g.nb, 1, case=0)
    p, q = oracle.inject_ew(g, vm[0], va[0])
    bt, ps, qs, vm0, va0 = newton.case_from_state(g, vm[0], va[0], p, q)
    assert bt[0] == newton.SLACK and (bt == newton.SLACK).sum() == 1
    assert np.all(vm0[bt == newton.PQ] == 1.0) and np.all(va0[bt != newton.SLACK] == 0.0)
    assert vm0[0] == vm[0][0] and va0[0] == va[0][0]


def reference_newton(g, bt, ps, qs, vm0, va0, tol, max_iter):
    """Plain Newton-Raphson on the oracle's element-wise S and Jacobian."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    yb = oracle.ybus(g)
    jr, jc = oracle.jac_pattern(yb)
    pvpq, pq, rows, cols = newton._reduced_index(g.nb, bt)
    vm, va = vm0.copy(), va0.copy()
    hist = []
    for it in range(max_iter + 1):
        p, q = oracle.inject_ew(g, vm, va)
        F = np.concatenate([p[pvpq] - ps[pvpq], q[pq] - qs[pq]])
        hist.append(float(np.max(np.abs(F))))
        if hist[-1] <= tol or it == max_iter:
            break
        jv = oracle.jac_ew(g, vm, va, (jr, jc))
        J = sp.csr_matrix((jv, jc, jr), shape=(2 * g.nb, 2 * g.nb))
        dx = spla.spsolve(J[rows][:, cols].tocsc(), -F)
        va[pvpq] += dx[:len(pvpq)]
        vm[pq] += dx[len(pvpq):]
    return vm, va, hist


@pytest.mark.gpu
@pytest.mark.parametrize("method", [pf.PF_METHOD_ELEMENTWISE, pf.PF_METHOD_YBUS, pf.PF_METHOD_ELEMENTWISE_TWO_PHASE])
def test_newton_recovers_the_state(method):
    # a mild operating point (neighbouring angles differ by a few hundredths of
    # a radian), reached from a flat start
    g = gridgen.grid_500()
    vm, va = gridgen.states(g.nb, 1, case=0, vlo=0.98, vhi=1.02, sigma=0.02)
    p, q = oracle.inject_ew(g, vm[0], va[0])
    bt, ps, qs, vm0, va0 = newton.case_from_state(g, vm[0], va[0], p, q)
    G = pf.Grid.from_grid(g)
    pf.pf_ybus(G)
    res = newton.solve(G, bt, ps, qs, vm0, va0, method=method, tol=1e-11, max_iter=12)
    assert res.converged, res.mismatch
    assert np.max(np.abs(res.vm - vm[0])) <= 1e-9 and np.max(np.abs(res.va - va[0])) <= 1e-9
    # quadratic convergence once close: each mismatch below 100 x the square of the previous
    m = res.mismatch
    for a, b in zip(m, m[1:]):
        if a < 1e-3 and b > 1e-13:
            assert b <= 100 * a * a, m
    # same iterates as the reference loop on the oracle
    rvm, rva, rhist = reference_newton(g, bt, ps, qs, vm0, va0, 1e-11, 12)
    assert len(rhist) == len(m)
    for a, b in zip(m, rhist):
        assert abs(a - b) <= 1e-9 * max(1.0, b)
    assert np.max(np.abs(res.vm - rvm)) <= 1e-12 and np.max(np.abs(res.va - rva)) <= 1e-12
