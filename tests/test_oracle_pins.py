"""Pins of the CPU oracle against facts that do not come from the oracle itself.

* closed forms: power over a pure reactance; the two-bus pi model with an
  ideal phase-shifting transformer, built from Kirchhoff's laws;
* the power-balance identity (injections = series losses + charging and
  shunt absorption), and zero real-power sum for lossless grids;
* complex-step derivatives of the textbook polar form of the injections
  (every Jacobian column on small grids);
* exact invariants: angle-shift invariance and degree-2 homogeneity in v;
* agreement of the two independent oracle methods (eqs. (5)-(7) vs
  eqs. (1), (3), (4));
* dense brute force of eqs. (3)-(4) and the brute-force index search of
  Algorithm 2 against the closed-form slot positions;
* the VJP against complex-step gradients of lambda . S.
"""
from __future__ import annotations

import math

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import oracle
from paper_2302_10736_amd import gridgen
from tests import _grids


def rel_inf(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def term_scale(yb, vm):
    """max_i v_i sum_j |Y_ij| v_j: a bound on the terms summed into any S_i,
    the scale against which rounding of a cancelling sum is measured."""
    rows = np.repeat(np.arange(yb.nb), np.diff(yb.yrow))
    s = np.zeros(yb.nb)
    np.add.at(s, rows, np.abs(yb.y) * vm[yb.ycol])
    return float(np.max(vm * s))


def ew_all(g, vm, va):
    yb = oracle.ybus(g)
    pat = oracle.jac_pattern(yb)
    p, q = oracle.inject_ew(g, vm, va)
    j = oracle.jac_ew(g, vm, va, pat)
    return yb, pat, p, q, j


def dense_from_csr(nrow, ncol, rowptr, col, val):
    d = np.zeros((nrow, ncol), dtype=np.result_type(val, np.float64))
    for i in range(nrow):
        d[i, col[rowptr[i]:rowptr[i + 1]]] += val[rowptr[i]:rowptr[i + 1]]
    return d


# ---------------------------------------------------------------- closed forms

def test_two_bus_lossless_reactance():
    # P = v1 v2 sin(d) / x,  Q_1 = (v1^2 - v1 v2 cos d) / x  (power over a reactance)
    g = _grids.two_bus(0.0, 0.1, 0.0, 1.0, 0.0)
    vm = np.array([1.0, 1.0])
    va = np.array([0.1, 0.0])
    p_expect = 10.0 * math.sin(0.1)
    q_expect = 10.0 * (1.0 - math.cos(0.1))
    for p, q in (oracle.inject_ew(g, vm, va), oracle.inject_ybus(oracle.ybus(g), vm, va)):
        assert p[0] == pytest.approx(p_expect, rel=1e-14)
        assert p[1] == pytest.approx(-p_expect, rel=1e-14)
        assert q[0] == pytest.approx(q_expect, rel=1e-12)
        assert q[1] == pytest.approx(q_expect, rel=1e-12)


def kirchhoff_two_bus(r, x, b, tap, shift, vm, va):
    """Branch-end powers from circuit laws: an ideal transformer m e^{j phi}
    at the from side feeding a pi circuit (series 1/(r+jx), j b/2 at each end)."""
    V1 = vm[0] * np.exp(1j * va[0])
    V2 = vm[1] * np.exp(1j * va[1])
    t = tap * np.exp(1j * shift)
    Vp = V1 / t                      # secondary voltage of the ideal transformer
    Is = (Vp - V2) / (r + 1j * x)    # series current from the transformer side to bus 2
    Ip = Is + 1j * b / 2 * Vp        # current leaving the transformer secondary
    S12 = Vp * np.conj(Ip)           # ideal transformer is lossless
    S21 = V2 * np.conj(-Is + 1j * b / 2 * V2)
    return S12, S21


@pytest.mark.parametrize("flip", [False, True])
@pytest.mark.parametrize("case", [
    (0.01, 0.1, 0.02, 1.05, 0.05, (1.02, 0.98), (0.1, -0.05)),
    (0.03, 0.2, 0.08, 0.95, -0.08, (0.97, 1.04), (-0.2, 0.15)),
    (0.0, 0.05, 0.0, 1.0, 0.0, (1.0, 1.0), (0.0, 0.3)),
])
def test_two_bus_kirchhoff(case, flip):
    r, x, b, tap, shift, vm, va = case
    vm = np.array(vm)
    va = np.array(va)
    S12, S21 = kirchhoff_two_bus(r, x, b, tap, shift, vm, va)
    g = _grids.two_bus(r, x, b, tap, shift, flip=flip)
    if flip:  # branch runs from bus 1 to bus 0: swap the bus roles
        vm, va = vm[::-1].copy(), va[::-1].copy()
    for p, q in (oracle.inject_ew(g, vm, va), oracle.inject_ybus(oracle.ybus(g), vm, va)):
        got = p + 1j * q
        h, k = (1, 0) if flip else (0, 1)
        assert abs(got[h] - S12) <= 1e-14 * abs(S12)
        assert abs(got[k] - S21) <= 1e-14 * abs(S21)


def test_tap_zero_means_one():
    g1 = _grids.two_bus(0.01, 0.1, 0.02, 1.0, 0.03)
    g0 = _grids.two_bus(0.01, 0.1, 0.02, 0.0, 0.03)
    vm, va = np.array([1.01, 0.99]), np.array([0.05, -0.02])
    assert np.array_equal(np.stack(oracle.inject_ew(g1, vm, va)), np.stack(oracle.inject_ew(g0, vm, va)))


def test_bus_shunt_only():
    # An isolated bus with shunt g + jb draws v^2 (g - jb) (S = V conj(Y V)).
    g = _grids.two_bus(0.01, 0.1, 0.0, 1.0, 0.0, gs=(0.0, 0.02), bs=(0.0, 0.1))
    vm, va = np.array([1.0, 1.1]), np.array([0.0, 0.0])
    p_iso, q_iso = oracle.inject_ew(g, vm, va)
    g2 = _grids.two_bus(0.01, 0.1, 0.0, 1.0, 0.0)
    p0, q0 = oracle.inject_ew(g2, vm, va)
    assert p_iso[1] - p0[1] == pytest.approx(1.21 * 0.02, rel=1e-13)
    assert q_iso[1] - q0[1] == pytest.approx(-1.21 * 0.1, rel=1e-13)


# ------------------------------------------------------------- power balance

def balance_terms(g, vm, va):
    """Per-branch series loss z|I_s|^2 and charging -j b/2 (|V_h'|^2 + v_k^2), plus bus shunts."""
    V = vm * np.exp(1j * va)
    m = np.where(g.tap == 0, 1.0, g.tap)
    Vp = V[g.fbus] / (m * np.exp(1j * g.shift))
    z = g.r + 1j * g.x
    Is = (Vp - V[g.tbus]) / z
    series = z * np.abs(Is) ** 2
    charging = -1j * g.b / 2 * (np.abs(Vp) ** 2 + np.abs(V[g.tbus]) ** 2)
    shunt = vm ** 2 * (g.gs - 1j * g.bs)
    return np.concatenate([series, charging, shunt])


@pytest.mark.parametrize("seed", range(4))
def test_power_balance_identity(seed):
    g = _grids.random_small(40, 70, seed, parallel=4, isolated=2)
    vm, va = _grids.random_state(g.nb, seed)
    terms = balance_terms(g, vm, va)
    for p, q in (oracle.inject_ew(g, vm, va), oracle.inject_ybus(oracle.ybus(g), vm, va)):
        s = p + 1j * q
        scale = np.sum(np.abs(s)) + np.sum(np.abs(terms))
        assert abs(np.sum(s) - np.sum(terms)) <= 1e-13 * scale


def test_power_balance_grid_500():
    g = gridgen.grid_500()
    vm, va = gridgen.states(g.nb, 1, 0)
    p, q = oracle.inject_ew(g, vm[0], va[0])
    terms = balance_terms(g, vm[0], va[0])
    s = p + 1j * q
    assert abs(np.sum(s) - np.sum(terms)) <= 1e-13 * (np.sum(np.abs(s)) + np.sum(np.abs(terms)))


def test_lossless_real_power_sums_to_zero():
    g = _grids.random_small(30, 50, 11, parallel=3, lossless=True)
    vm, va = _grids.random_state(g.nb, 11)
    for p, _ in (oracle.inject_ew(g, vm, va), oracle.inject_ybus(oracle.ybus(g), vm, va)):
        assert abs(np.sum(p)) <= 1e-14 * np.sum(np.abs(p))


# ------------------------------------------------------------- complex step

def polar_injections(yb, vm, va):
    """Textbook polar form P_i = sum_j v_i v_j (G cos t_ij + B sin t_ij),
    Q_i = sum_j v_i v_j (G sin t_ij - B cos t_ij); analytic in (vm, va)."""
    rows = np.repeat(np.arange(yb.nb), np.diff(yb.yrow))
    cols = yb.ycol
    G, B = yb.y.real, yb.y.imag
    t = va[rows] - va[cols]
    w = vm[rows] * vm[cols]
    tp = w * (G * np.cos(t) + B * np.sin(t))
    tq = w * (G * np.sin(t) - B * np.cos(t))
    P = np.zeros(yb.nb, dtype=tp.dtype)
    Q = np.zeros(yb.nb, dtype=tq.dtype)
    np.add.at(P, rows, tp)
    np.add.at(Q, rows, tq)
    return P, Q


def complex_step_jacobian(yb, vm, va, h=1e-30):
    nb = yb.nb
    J = np.zeros((2 * nb, 2 * nb))
    for k in range(2 * nb):
        zm = vm.astype(np.complex128)
        za = va.astype(np.complex128)
        if k < nb:
            za[k] += 1j * h
        else:
            zm[k - nb] += 1j * h
        P, Q = polar_injections(yb, zm, za)
        J[:nb, k] = P.imag / h
        J[nb:, k] = Q.imag / h
    return J


@pytest.mark.parametrize("seed", range(3))
def test_jacobians_complex_step_small(seed):
    g = _grids.random_small(25, 45, 100 + seed, parallel=3, isolated=1)
    vm, va = _grids.random_state(g.nb, seed)
    yb, pat, p, q, j_ew = ew_all(g, vm, va)
    j_yb = oracle.jac_ybus(yb, vm, va, pat)
    Jcs = complex_step_jacobian(yb, vm, va)
    for jv in (j_ew, j_yb):
        Jd = dense_from_csr(2 * g.nb, 2 * g.nb, *pat, jv)
        assert rel_inf(Jd, Jcs) <= 1e-14
    # the polar form at real points is the injection itself
    P, Q = polar_injections(yb, vm, va)
    assert rel_inf(P, p) <= 1e-14 and rel_inf(Q, q) <= 1e-14


def test_jacobians_complex_step_grid_500():
    g = gridgen.grid_500()
    vm, va = gridgen.states(g.nb, 1, 0)
    vm, va = vm[0], va[0]
    yb, pat, _, _, j_ew = ew_all(g, vm, va)
    j_yb = oracle.jac_ybus(yb, vm, va, pat)
    Jcs = complex_step_jacobian(yb, vm, va)
    for jv in (j_ew, j_yb):
        Jd = dense_from_csr(2 * g.nb, 2 * g.nb, *pat, jv)
        assert rel_inf(Jd, Jcs) <= 1e-14


# ------------------------------------------------------------- invariants

@pytest.mark.parametrize("seed", range(3))
def test_angle_shift_and_homogeneity(seed):
    g = _grids.random_small(60, 100, 300 + seed, parallel=5, isolated=3)
    vm, va = _grids.random_state(g.nb, seed)
    yb, pat, p, q, j = ew_all(g, vm, va)
    nb = g.nb
    Jd = dense_from_csr(2 * nb, 2 * nb, *pat, j)
    scale = np.abs(Jd).sum(axis=1) + 1e-300
    # rotating every angle by the same amount leaves S unchanged
    assert np.max(np.abs(Jd[:, :nb].sum(axis=1)) / scale) <= 1e-14
    # S is homogeneous of degree 2 in v: J_v v = 2 [P; Q]
    hv = Jd[:, nb:] @ vm
    assert rel_inf(hv, 2 * np.concatenate([p, q])) <= 1e-14
    # shifting angles really leaves S unchanged
    p2, q2 = oracle.inject_ew(g, vm, va + 0.7)
    assert rel_inf(p2, p) <= 1e-13 and rel_inf(q2, q) <= 1e-13


# ------------------------------------------------------------- cross-method

@settings(max_examples=40, deadline=None)
@given(nb=st.integers(2, 30), extra=st.integers(0, 30), par=st.integers(0, 5), iso=st.integers(0, 3),
       seed=st.integers(0, 10_000))
def test_methods_agree_random(nb, extra, par, iso, seed):
    live = nb - iso
    if live < 2:
        return
    g = _grids.random_small(nb, live - 1 + extra + par, seed, parallel=par, isolated=iso)
    vm, va = _grids.random_state(g.nb, seed)
    yb, pat, p, q, j_ew = ew_all(g, vm, va)
    p2, q2 = oracle.inject_ybus(yb, vm, va)
    j_yb = oracle.jac_ybus(yb, vm, va, pat)
    sc = term_scale(yb, vm)
    assert np.max(np.abs(p - p2)) <= 1e-14 * sc * (nb + par + extra)
    assert np.max(np.abs(q - q2)) <= 1e-14 * sc * (nb + par + extra)
    assert np.max(np.abs(j_ew - j_yb)) <= 1e-14 * sc * (nb + par + extra)


def test_methods_agree_grid_500():
    g = gridgen.grid_500()
    vm, va = gridgen.states(g.nb, 1, 0)
    yb, pat, p, q, j_ew = ew_all(g, vm[0], va[0])
    p2, q2 = oracle.inject_ybus(yb, vm[0], va[0])
    assert rel_inf(p, p2) <= 1e-14 and rel_inf(q, q2) <= 1e-14
    assert rel_inf(j_ew, oracle.jac_ybus(yb, vm[0], va[0], pat)) <= 1e-14


@pytest.mark.parametrize("method", ["ew", "ybus"])
def test_relabelling_invariance(method):
    """Renumbering the buses permutes S, J and the adjoint and changes nothing
    else (a wrong bus index anywhere, say a shunt or a remote end, breaks it)."""
    import scipy.sparse as sp
    g = gridgen.grid_500()
    vm, va = gridgen.states(g.nb, 1, 0)
    lp, lq = gridgen.adjoint_seeds(g.nb, 1, 0)
    h, perm = gridgen.relabel(g, case=0)
    inv = np.argsort(perm)
    nb = g.nb

    def evaluate(gr, v, a):
        yb = oracle.ybus(gr)
        pat = oracle.jac_pattern(yb)
        if method == "ew":
            p, q = oracle.inject_ew(gr, v, a)
            j = oracle.jac_ew(gr, v, a, pat)
        else:
            p, q = oracle.inject_ybus(yb, v, a)
            j = oracle.jac_ybus(yb, v, a, pat)
        return p, q, sp.csr_matrix((j, pat[1], pat[0]), shape=(2 * nb, 2 * nb)), pat, j

    p0, q0, J0, pat0, j0 = evaluate(g, vm[0], va[0])
    p1, q1, J1, pat1, j1 = evaluate(h, vm[0][inv], va[0][inv])
    assert rel_inf(p1, p0[inv]) <= 1e-14 and rel_inf(q1, q0[inv]) <= 1e-14
    var = np.concatenate([perm, nb + perm])  # new index of each old row / column
    assert abs(J1[var][:, var] - J0).max() <= 1e-14 * abs(J0).max()
    gv0, ga0 = oracle.vjp(nb, pat0, j0, lp[0], lq[0])
    gv1, ga1 = oracle.vjp(nb, pat1, j1, lp[0][inv], lq[0][inv])
    assert rel_inf(gv1, gv0[inv]) <= 1e-14 and rel_inf(ga1, ga0[inv]) <= 1e-14


# ------------------------------------------------------------- dense brute force

def test_dense_matrix_form():
    """Eqs. (3)-(4) evaluated with dense products (the 'matrix multiplication' variant)."""
    g = _grids.random_small(20, 35, 5, parallel=2, isolated=1)
    vm, va = _grids.random_state(g.nb, 5)
    yb = oracle.ybus(g)
    pat = oracle.jac_pattern(yb)
    Y = yb.dense()
    U = np.exp(1j * va)
    V = vm * U
    Ic = Y @ V
    dSt = 1j * np.diag(V) @ (np.diag(np.conj(Ic)) - np.conj(Y @ np.diag(V)))
    dSv = np.diag(np.conj(Ic) * U) + np.diag(V) @ np.conj(Y @ np.diag(U))
    Jref = np.block([[dSt.real, dSv.real], [dSt.imag, dSv.imag]])
    Jd = dense_from_csr(2 * g.nb, 2 * g.nb, *pat, oracle.jac_ybus(yb, vm, va, pat))
    assert rel_inf(Jd, Jref) <= 1e-14
    S = V * np.conj(Ic)
    p, q = oracle.inject_ybus(yb, vm, va)
    assert rel_inf(p, S.real) <= 1e-14 and rel_inf(q, S.imag) <= 1e-14


# ------------------------------------------------------------- structure / Alg. 2

def alg2_indices(nb, yrow, ycol, jrow, jcol):
    """Algorithm 2 (brute force): for each Ybus nonzero and block (x, y), the
    position in J of (row + x nb, col + y nb), found by scanning the J row."""
    rows = np.repeat(np.arange(nb), np.diff(yrow))
    out = {}
    for bx in (0, 1):
        for by in (0, 1):
            P = np.full(len(ycol), -1, np.int64)
            for t in range(len(ycol)):
                rr = rows[t] + bx * nb
                cc = ycol[t] + by * nb
                for k in range(jrow[rr], jrow[rr + 1]):
                    if jcol[k] == cc:
                        P[t] = k
                        break
            out[(bx, by)] = P
    return out


def closed_form_slots(nb, yrow):
    nnz = int(yrow[-1])
    rows = np.repeat(np.arange(nb), np.diff(yrow))
    p = np.arange(nnz)
    return {(0, 0): yrow[rows] + p, (0, 1): yrow[rows + 1] + p,
            (1, 0): 2 * nnz + yrow[rows] + p, (1, 1): 2 * nnz + yrow[rows + 1] + p}


def test_alg2_matches_closed_form():
    g = _grids.random_small(40, 70, 9, parallel=4, isolated=2)
    yb = oracle.ybus(g)
    jrow, jcol = oracle.jac_pattern(yb)
    a = alg2_indices(g.nb, yb.yrow, yb.ycol, jrow, jcol)
    c = closed_form_slots(g.nb, yb.yrow)
    for key in a:
        assert np.array_equal(a[key], c[key])


def test_structure_counts():
    g = gridgen.grid_500()
    yb = oracle.ybus(g)
    pairs = {(min(a, b), max(a, b)) for a, b in zip(g.fbus.tolist(), g.tbus.tolist())}
    assert yb.nnz == g.nb + 2 * len(pairs) == 1900
    jrow, jcol = oracle.jac_pattern(yb)
    assert len(jcol) == 4 * yb.nnz == 7600
    assert jrow[-1] == len(jcol)
    # every diagonal is present and columns ascend within each row
    for i in range(g.nb):
        cols = yb.ycol[yb.yrow[i]:yb.yrow[i + 1]]
        assert i in cols and np.all(np.diff(cols) > 0)
    for rr in range(2 * g.nb):
        assert np.all(np.diff(jcol[jrow[rr]:jrow[rr + 1]]) > 0)


def test_paper_element_count_fixture():
    """Section V.A quotes 1,665,936 Jacobian elements for the 82k-bus case,
    i.e. 16 partials per branch; the oracle evaluates 16 per branch too."""
    import json, os
    fx = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_counts.json")))
    assert fx["jacobian_elements"] % 16 == 0
    # 16 per branch: a one-branch grid yields 16 partials (8 nonzero-pattern slots x 2 rows)
    g = _grids.two_bus(0.01, 0.1, 0.02, 1.02, 0.03)
    yb = oracle.ybus(g)
    pat = oracle.jac_pattern(yb)
    assert len(pat[1]) == 16


# ------------------------------------------------------------- VJP

@pytest.mark.parametrize("seed", range(3))
def test_vjp_complex_step(seed):
    g = _grids.random_small(30, 55, 700 + seed, parallel=3, isolated=1)
    vm, va = _grids.random_state(g.nb, seed)
    rng = np.random.default_rng(seed)
    lp, lq = rng.normal(size=g.nb), rng.normal(size=g.nb)
    yb, pat, _, _, j = ew_all(g, vm, va)
    gvm, gva = oracle.vjp(g.nb, pat, j, lp, lq)
    h = 1e-30
    ref_vm = np.zeros(g.nb)
    ref_va = np.zeros(g.nb)
    for k in range(g.nb):
        for which in (0, 1):
            zm = vm.astype(np.complex128)
            za = va.astype(np.complex128)
            (zm if which == 0 else za)[k] += 1j * h
            P, Q = polar_injections(yb, zm, za)
            d = (lp @ P.imag + lq @ Q.imag) / h
            (ref_vm if which == 0 else ref_va)[k] = d
    assert rel_inf(gvm, ref_vm) <= 1e-13
    assert rel_inf(gva, ref_va) <= 1e-13


# ------------------------------------------------------------- branch flows

@pytest.mark.parametrize("flip", [False, True])
@pytest.mark.parametrize("case", [
    (0.01, 0.1, 0.02, 1.05, 0.05, (1.02, 0.98), (0.1, -0.05)),
    (0.03, 0.2, 0.08, 0.95, -0.08, (0.97, 1.04), (-0.2, 0.15)),
])
def test_branch_flows_kirchhoff(case, flip):
    r, x, b, tap, shift, vm, va = case
    vm, va = np.array(vm), np.array(va)
    S12, S21 = kirchhoff_two_bus(r, x, b, tap, shift, vm, va)
    g = _grids.two_bus(r, x, b, tap, shift, flip=flip)
    if flip:
        vm, va = vm[::-1].copy(), va[::-1].copy()
    pf_, qf, pt, qt = oracle.branch_flows(g, vm, va)
    assert abs(pf_[0] + 1j * qf[0] - S12) <= 1e-14 * abs(S12)
    assert abs(pt[0] + 1j * qt[0] - S21) <= 1e-14 * abs(S21)


def flows_to_buses(g, flows, vm):
    pf_, qf, pt, qt = flows
    s = np.zeros(g.nb, complex)
    np.add.at(s, g.fbus, pf_ + 1j * qf)
    np.add.at(s, g.tbus, pt + 1j * qt)
    return s + vm ** 2 * (g.gs - 1j * g.bs)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_branch_flows_sum_to_ybus_injections(seed):
    g = _grids.random_small(60, 110, 100 + seed, parallel=5, isolated=2)
    vm, va = _grids.random_state(g.nb, seed)
    yb = oracle.ybus(g)
    p, q = oracle.inject_ybus(yb, vm, va)  # the other method's code path
    s = flows_to_buses(g, oracle.branch_flows(g, vm, va), vm)
    assert np.max(np.abs(s - (p + 1j * q))) <= 1e-13 * term_scale(yb, vm)


def test_branch_flows_lossless():
    g = _grids.random_small(40, 70, 7, lossless=True)
    g.b = np.zeros(g.nl)
    vm, va = _grids.random_state(g.nb, 3)
    pf_, qf, pt, qt = oracle.branch_flows(g, vm, va)
    assert np.max(np.abs(pf_ + pt)) <= 1e-13 * np.max(np.abs(pf_))


def textbook_branch_flows(g, vm, va):
    """P and Q of both ends from the branch admittances in polar form,
    P_hk = v_h^2 G_ff + v_h v_k (G_ft cos d + B_ft sin d),
    Q_hk = -v_h^2 B_ff + v_h v_k (G_ft sin d - B_ft cos d), d = theta_h - theta_k,
    with the usual pi-model branch entries (real-analytic in vm, va, so a
    complex step differentiates it)."""
    h, k = g.fbus, g.tbus
    m = np.where(g.tap == 0.0, 1.0, g.tap)
    ys = 1.0 / (g.r + 1j * g.x)
    yff = (ys + 0.5j * g.b) / m ** 2
    yft = -ys / (m * np.exp(-1j * g.shift))
    ytf = -ys / (m * np.exp(1j * g.shift))
    ytt = ys + 0.5j * g.b

    def ends(vi, vj, ti, tj, yii, yij):
        d = ti - tj
        p = vi ** 2 * yii.real + vi * vj * (yij.real * np.cos(d) + yij.imag * np.sin(d))
        q = -vi ** 2 * yii.imag + vi * vj * (yij.real * np.sin(d) - yij.imag * np.cos(d))
        return p, q
    pf_, qf = ends(vm[h], vm[k], va[h], va[k], yff, yft)
    pt, qt = ends(vm[k], vm[h], va[k], va[h], ytt, ytf)
    return pf_, qf, pt, qt


@pytest.mark.parametrize("seed", [0, 1])
def test_branch_flow_jacobian_complex_step(seed):
    g = _grids.random_small(25, 45, 200 + seed, parallel=3)
    vm, va = _grids.random_state(g.nb, seed)
    jac = oracle.branch_flow_jac(g, vm, va)
    flows = oracle.branch_flows(g, vm, va)
    ref = textbook_branch_flows(g, vm.astype(complex), va.astype(complex))
    for a, b_ in zip(flows, ref):
        assert np.max(np.abs(a - b_.real)) <= 1e-13 * np.max(np.abs(a))
    h_step = 1e-30
    want = np.zeros((16, g.nl))
    for l in range(g.nl):
        for v, (arr, bus) in enumerate(((va, g.fbus[l]), (va, g.tbus[l]), (vm, g.fbus[l]), (vm, g.tbus[l]))):
            vm_c, va_c = vm.astype(complex), va.astype(complex)
            (va_c if arr is va else vm_c)[bus] += 1j * h_step
            out = textbook_branch_flows(g, vm_c, va_c)
            for f in range(4):
                want[4 * f + v, l] = out[f][l].imag / h_step
    assert np.max(np.abs(jac - want)) <= 1e-12 * np.max(np.abs(want))
