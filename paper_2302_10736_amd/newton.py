"""Newton-Raphson power flow around the evaluation kernels.

The paper computes S and the Jacobian values as the inner step of Newton's
method (Section I; it leaves the linear solve aside).  This driver closes
the loop: per iteration the GPU evaluates P, Q and all Jacobian values in
one launch (either method), the host selects the rows and columns of the
unknowns and solves the sparse linear system with SuperLU (SciPy), and the
update is applied to the device state.

Bus types follow the usual convention: one slack bus per grid (angle and
magnitude fixed), PV buses (real power and magnitude fixed; the angle is
unknown) and PQ buses (real and reactive power fixed; angle and magnitude
unknown).  Unknowns are ordered [theta(PV, PQ), v(PQ)], equations
[P(PV, PQ), Q(PQ)].
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np

from . import pf

SLACK, PV, PQ = 3, 2, 1


@dataclass
class NewtonResult:
    vm: np.ndarray
    va: np.ndarray
    converged: bool
    iterations: int
    mismatch: list = field(default_factory=list)  # max |F| before each update and at the end
    seconds_eval: float = 0.0    # device evaluation incl. copies of P, Q and J values to the host
    seconds_solve: float = 0.0   # host: reduced system and sparse LU solve


def _reduced_index(nb, bus_type):
    pvpq = np.flatnonzero((bus_type == PV) | (bus_type == PQ))
    pq = np.flatnonzero(bus_type == PQ)
    rows = np.concatenate([pvpq, nb + pq])  # P rows, then Q rows of the full J
    cols = np.concatenate([pvpq, nb + pq])  # theta columns, then v columns
    return pvpq, pq, rows, cols


def _reduced_map(jr, jc, rows, cols):
    """The reduced matrix (rows and columns of the unknowns) keeps one
    sparsity pattern: where each of its CSC entries sits in the full CSR
    value array, and its CSC index arrays.  Every iteration then forms it
    with one gather."""
    import scipy.sparse as sp
    n = len(jr) - 1
    idx = sp.csr_matrix((np.arange(1, len(jc) + 1, dtype=np.float64), jc, jr), shape=(n, n))
    red = idx[rows][:, cols].tocsc()
    red.sort_indices()
    return red.data.astype(np.int64) - 1, red.indices, red.indptr, red.shape


def solve(grid: "pf.Grid", bus_type, p_spec, q_spec, vm0, va0, method: int = pf.PF_METHOD_ELEMENTWISE,
          tol: float = 1e-10, max_iter: int = 20) -> NewtonResult:
    """Solve S(v, theta) = p_spec + j q_spec on the PV and PQ rows.

    vm0, va0 hold the fixed values (slack magnitude and angle, PV magnitudes)
    and the starting point of the unknowns.  ``method`` is any Jacobian
    method of ``pf_jacobian_values``; the handle must have had pf_ybus
    called if it is PF_METHOD_YBUS."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    import torch

    nb = grid.nb
    bus_type = np.asarray(bus_type)
    if bus_type.shape != (nb,):
        raise ValueError("bus_type must have one entry per bus")
    dev = torch.device("cuda", torch.cuda.current_device())
    yr, yc, jr, jc = grid.pattern()
    if grid.ngrids != 1:
        raise ValueError("one grid per handle (the pattern export is grid-local)")
    pvpq, pq, rows, cols = _reduced_index(nb, bus_type)
    n1 = len(pvpq)
    take, r_ind, r_ptr, r_shape = _reduced_map(jr, jc, rows, cols)
    vm = torch.as_tensor(np.asarray(vm0, dtype=np.float64), device=dev).clone()
    va = torch.as_tensor(np.asarray(va0, dtype=np.float64), device=dev).clone()
    p = torch.empty(nb, dtype=torch.float64, device=dev)
    q = torch.empty_like(p)
    j = torch.empty(grid.nnz_j, dtype=torch.float64, device=dev)
    p_spec = np.asarray(p_spec, dtype=np.float64)
    q_spec = np.asarray(q_spec, dtype=np.float64)
    res = NewtonResult(vm=None, va=None, converged=False, iterations=0)
    evaluate = pf.bind(pf.pf_jacobian_values, grid, method, vm, va, p, q, j)  # same buffers every iteration
    for it in range(max_iter + 1):
        t0 = time.perf_counter()
        evaluate()
        ph, qh, jv = p.cpu().numpy(), q.cpu().numpy(), j.cpu().numpy()
        t1 = time.perf_counter()
        res.seconds_eval += t1 - t0
        F = np.concatenate([ph[pvpq] - p_spec[pvpq], qh[pq] - q_spec[pq]])
        err = float(np.max(np.abs(F))) if F.size else 0.0
        res.mismatch.append(err)
        if err <= tol:
            res.converged = True
            break
        if it == max_iter:
            break
        Jr = sp.csc_matrix((jv[take], r_ind, r_ptr), shape=r_shape)
        dx = spla.spsolve(Jr, -F)
        res.seconds_solve += time.perf_counter() - t1
        upd_a = np.zeros(nb)
        upd_m = np.zeros(nb)
        upd_a[pvpq] = dx[:n1]
        upd_m[pq] = dx[n1:]
        va += torch.as_tensor(upd_a, device=dev)
        vm += torch.as_tensor(upd_m, device=dev)
        res.iterations = it + 1
    res.vm = vm.cpu().numpy()
    res.va = va.cpu().numpy()
    return res


def case_from_state(g, vm_true, va_true, p_true, q_true, pv_frac=0.2, seed=0, perturb=None):
    """A solvable power-flow case whose solution is a given state: bus 0 is
    the slack, a fraction of the others are PV, the rest PQ; specified
    powers are the injections at the given state.  Returns (bus_type,
    p_spec, q_spec, vm0, va0): a flat start for the unknowns, or with
    ``perturb`` the given state plus N(0, perturb) noise on the unknowns
    (power flow can have several solutions; a start near the given one
    converges to it)."""
    rng = np.random.default_rng(seed)
    nb = g.nb
    bus_type = np.full(nb, PQ)
    bus_type[rng.random(nb) < pv_frac] = PV
    bus_type[0] = SLACK
    if perturb is None:
        vm0 = np.where(bus_type == PQ, 1.0, vm_true)
        va0 = np.where(bus_type == SLACK, va_true, 0.0)
    else:
        vm0 = np.where(bus_type == PQ, vm_true + perturb * rng.standard_normal(nb), vm_true)
        va0 = np.where(bus_type == SLACK, va_true, va_true + perturb * rng.standard_normal(nb))
    return bus_type, np.asarray(p_true), np.asarray(q_true), vm0, va0
