"""Plain FP64 CPU oracle (test infrastructure only).

Only the test suite, ``__graft_entry__.smoke()`` and the benchmark's
``cpu_baseline`` leg may import this package.  The library's product path
never does; the two share no code.  The arithmetic lives in ``oracle.c``
(scalar loops, C99 complex, -ffp-contract=off); this module only marshals
numpy arrays through ctypes.  Grids are duck-typed: any object with
``nb, nl, fbus, tbus, r, x, b, tap, shift, gs, bs`` attributes.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB) or os.path.getmtime(_build.LIB) < os.path.getmtime(_build.SRC):
            _build.build()
        L = C.CDLL(_build.LIB)
        P = C.c_void_p
        i32, i64 = C.c_int32, C.c_int64
        L.orc_ybus.restype = i64
        L.orc_ybus.argtypes = [i32, i32] + [P] * 13
        L.orc_inject_ybus.restype = None
        L.orc_inject_ybus.argtypes = [i32] + [P] * 8
        L.orc_inject_ew.restype = None
        L.orc_inject_ew.argtypes = [i32, i32] + [P] * 13
        L.orc_jac_pattern.restype = None
        L.orc_jac_pattern.argtypes = [i32] + [P] * 4
        L.orc_jac_ybus.restype = i64
        L.orc_jac_ybus.argtypes = [i32] + [P] * 9
        L.orc_jac_ew.restype = i64
        L.orc_jac_ew.argtypes = [i32, i32] + [P] * 14
        L.orc_vjp.restype = None
        L.orc_vjp.argtypes = [i32] + [P] * 5
        L.orc_branch_flows.restype = None
        L.orc_branch_flows.argtypes = [i32] + [P] * 13
        L.orc_branch_flow_jac.restype = None
        L.orc_branch_flow_jac.argtypes = [i32] + [P] * 10
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _branch(g):
    return (_i32(g.fbus), _i32(g.tbus), _f64(g.r), _f64(g.x), _f64(g.b), _f64(g.tap), _f64(g.shift),
            _f64(g.gs), _f64(g.bs))


class Ybus:
    """Oracle admittance matrix in CSR (0-based, columns ascending)."""

    def __init__(self, nb, yrow, ycol, y):
        self.nb, self.yrow, self.ycol, self.y = nb, yrow, ycol, y

    @property
    def nnz(self):
        return int(self.yrow[-1])

    def dense(self) -> np.ndarray:
        d = np.zeros((self.nb, self.nb), dtype=np.complex128)
        for i in range(self.nb):
            s, e = self.yrow[i], self.yrow[i + 1]
            d[i, self.ycol[s:e]] += self.y[s:e]
        return d


def ybus(g) -> Ybus:
    arrs = _branch(g)
    cap = g.nb + 4 * g.nl
    yrow = np.zeros(g.nb + 1, np.int32)
    ycol = np.zeros(max(cap, 1), np.int32)
    yre = np.zeros(max(cap, 1))
    yim = np.zeros(max(cap, 1))
    nnz = lib().orc_ybus(g.nb, g.nl, *map(_p, arrs), _p(yrow), _p(ycol), _p(yre), _p(yim))
    if nnz < 0:
        raise MemoryError("oracle ybus allocation failed")
    return Ybus(g.nb, yrow, ycol[:nnz].copy(), yre[:nnz] + 1j * yim[:nnz])


def inject_ybus(yb: Ybus, vm, va):
    vm, va = _f64(vm), _f64(va)
    p = np.empty(yb.nb)
    q = np.empty(yb.nb)
    yre, yim = _f64(yb.y.real), _f64(yb.y.imag)
    lib().orc_inject_ybus(yb.nb, _p(yb.yrow), _p(yb.ycol), _p(yre), _p(yim), _p(vm), _p(va), _p(p), _p(q))
    return p, q


def inject_ew(g, vm, va):
    vm, va = _f64(vm), _f64(va)
    p = np.empty(g.nb)
    q = np.empty(g.nb)
    lib().orc_inject_ew(g.nb, g.nl, *map(_p, _branch(g)), _p(vm), _p(va), _p(p), _p(q))
    return p, q


def jac_pattern(yb: Ybus):
    jrow = np.zeros(2 * yb.nb + 1, np.int32)
    jcol = np.zeros(max(4 * yb.nnz, 1), np.int32)
    lib().orc_jac_pattern(yb.nb, _p(yb.yrow), _p(yb.ycol), _p(jrow), _p(jcol))
    return jrow, jcol[: 4 * yb.nnz].copy()


def jac_ybus(yb: Ybus, vm, va, pattern=None):
    jrow, jcol = pattern if pattern is not None else jac_pattern(yb)
    vm, va = _f64(vm), _f64(va)
    jval = np.zeros(max(len(jcol), 1))
    yre, yim = _f64(yb.y.real), _f64(yb.y.imag)
    miss = lib().orc_jac_ybus(yb.nb, _p(yb.yrow), _p(yb.ycol), _p(yre), _p(yim), _p(vm), _p(va),
                              _p(jrow), _p(jcol), _p(jval))
    if miss:
        raise AssertionError(f"{miss} Ybus Jacobian entries outside the pattern")
    return jval[: len(jcol)]


def jac_ew(g, vm, va, pattern):
    jrow, jcol = pattern
    vm, va = _f64(vm), _f64(va)
    jval = np.zeros(max(len(jcol), 1))
    miss = lib().orc_jac_ew(g.nb, g.nl, *map(_p, _branch(g)), _p(vm), _p(va), _p(jrow), _p(jcol), _p(jval))
    if miss:
        raise AssertionError(f"{miss} element-wise Jacobian entries outside the pattern")
    return jval[: len(jcol)]


def vjp(nb, pattern, jval, lam_p, lam_q):
    jrow, jcol = pattern
    lam = _f64(np.concatenate([lam_p, lam_q]))
    g = np.empty(2 * nb)
    lib().orc_vjp(nb, _p(jrow), _p(jcol), _p(_f64(jval)), _p(lam), _p(g))
    return g[nb:].copy(), g[:nb].copy()  # (g_vm, g_va)


def branch_flows(g, vm, va):
    """(pf, qf, pt, qt) per branch: S_hk and S_kh of eqs. (5)-(6)."""
    vm, va = _f64(vm), _f64(va)
    out = [np.empty(g.nl) for _ in range(4)]
    lib().orc_branch_flows(g.nl, *map(_p, _branch(g)[:7]), _p(vm), _p(va), *map(_p, out))
    return tuple(out)


def branch_flow_jac(g, vm, va):
    """[16, nl]: d(Pf, Qf, Pt, Qt) / d(theta_h, theta_k, v_h, v_k), four rows each."""
    vm, va = _f64(vm), _f64(va)
    jac = np.empty((16, g.nl))
    lib().orc_branch_flow_jac(g.nl, *map(_p, _branch(g)[:7]), _p(vm), _p(va), _p(jac))
    return jac
