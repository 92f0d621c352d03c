"""C-ABI boundary on the CPU: symbol exports, validation, host-only patterns.

No compute call runs here (no GPU): the host-only handle builds and exports
the patterns, which must equal the oracle's independently built ones
bit-for-bit, and Algorithm 2's brute-force index search over the exported J
pattern must reproduce the closed-form slot positions.
"""
from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle
from paper_2302_10736_amd import gridgen, pf
from tests import _grids
from tests.test_oracle_pins import alg2_indices, closed_form_slots

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    """Every function declared in include/*.h (pf.h and the testing header)."""
    syms = set()
    for name in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if name.endswith(".h"):
            src = open(os.path.join(ROOT, "include", name)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            syms |= set(re.findall(r"\b(pf_[a-z_]+)\s*\(", src))
    return sorted(syms)


def test_library_exports_every_declared_symbol():
    syms = header_symbols()
    assert len(syms) >= 14
    L = pf.lib()
    for s in syms:
        assert hasattr(L, s), s
    assert set(syms) == set(pf.EXPORTS)
    assert "gfx950" in pf.pf_version()


def test_header_compiles_as_c():
    import subprocess, tempfile
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        open(c, "w").write('#include "pf.h"\n#include "pf_testing.h"\nint main(void){ const char *(*f)(void) = '
                           'pf_last_error; int (*g)(int32_t) = pf_debug_fail_allocs; (void)f; (void)g; return PF_OK; }\n')
        subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"), "-c", c, "-o",
                        os.path.join(d, "t.o")], check=True)


def per_grid_oracle_pattern(grids):
    yr, yc, jr, jc = [], [], [], []
    for g in grids:
        yb = oracle.ybus(g)
        a, b = oracle.jac_pattern(yb)
        yr.append(yb.yrow); yc.append(yb.ycol); jr.append(a); jc.append(b)
    return [np.concatenate(x) for x in (yr, yc, jr, jc)]


@pytest.mark.parametrize("make", [
    lambda: gridgen.grid_500(),
    lambda: _grids.random_small(50, 90, 1, parallel=6, isolated=3),
    lambda: _grids.random_small(2, 9, 2, parallel=8),
    lambda: _grids.two_bus(0.01, 0.1, 0.0, 1.0, 0.0, flip=True),
])
def test_pattern_matches_oracle(make):
    g = make()
    G = pf.Grid.from_grid(g, host_only=True)
    got = G.pattern()
    want = per_grid_oracle_pattern([g])
    for a, b in zip(got, want):
        assert a.dtype == np.int32 and np.array_equal(a, b)
    assert G.nnz_j == 4 * G.nnz_y


def test_multigrid_pattern_matches_oracle():
    grids = [_grids.random_small(n, n + 5, 40 + n, parallel=n % 3, isolated=n % 2) for n in (3, 17, 9, 30)]
    big, bo, ro = gridgen.concat(grids)
    G = pf.Grid.from_grid(big, bo, ro, host_only=True)
    assert G.ngrids == 4
    got = G.pattern()
    want = per_grid_oracle_pattern(grids)
    for a, b in zip(got, want):
        assert np.array_equal(a, b)
    y_off, j_off = G.offsets()
    nnz = [oracle.ybus(g).nnz for g in grids]
    assert np.array_equal(y_off, np.concatenate([[0], np.cumsum(nnz)]))
    assert np.array_equal(j_off, 4 * y_off)


def test_isolated_bus_grid_without_branches():
    nb = 5
    G = pf.Grid(nb, 0, [], [], [], [], [], [], [], np.arange(nb) * 0.01, None, host_only=True)
    yr, yc, jr, jc = G.pattern()
    assert np.array_equal(yr, np.arange(nb + 1)) and np.array_equal(yc, np.arange(nb))
    assert G.nnz_j == 4 * nb


def test_alg2_search_on_exported_pattern():
    g = _grids.random_small(60, 110, 3, parallel=5, isolated=2)
    G = pf.Grid.from_grid(g, host_only=True)
    yr, yc, jr, jc = G.pattern()
    a = alg2_indices(g.nb, yr, yc, jr, jc)
    c = closed_form_slots(g.nb, yr)
    for key in a:
        assert np.array_equal(a[key], c[key])


# ------------------------------------------------------------- validation

def base_arrays():
    g = _grids.random_small(6, 8, 5)
    return dict(nb=g.nb, nl=g.nl, fbus=g.fbus.copy(), tbus=g.tbus.copy(), r=g.r.copy(), x=g.x.copy(), b=g.b.copy(),
                tap=g.tap.copy(), shift=g.shift.copy(), gs=g.gs.copy(), bs=g.bs.copy())


def build_raw(a, ngrids=1, bus_off=None, br_off=None, flags=pf.PF_BUILD_HOST_ONLY):
    L = pf.lib()
    h = C.c_void_p(12345)  # must be reset to NULL on error
    arrs = [np.ascontiguousarray(a["fbus"], np.int32), np.ascontiguousarray(a["tbus"], np.int32)] + \
        [np.ascontiguousarray(a[k], np.float64) for k in ("r", "x", "b", "tap", "shift")]
    ptr = lambda v: None if v is None else v.ctypes.data_as(C.c_void_p)
    gs = None if a.get("gs") is None else np.ascontiguousarray(a["gs"], np.float64)
    bs = None if a.get("bs") is None else np.ascontiguousarray(a["bs"], np.float64)
    bo = None if bus_off is None else np.ascontiguousarray(bus_off, np.int32)
    ro = None if br_off is None else np.ascontiguousarray(br_off, np.int32)
    rc = L.pf_build_pattern(a["nb"], a["nl"], *[ptr(v) for v in arrs], ptr(gs), ptr(bs), ngrids, ptr(bo), ptr(ro),
                            flags, C.byref(h))
    msg = L.pf_last_error().decode()
    if rc == 0:
        L.pf_grid_free(h)
    else:
        assert h.value is None, "handle must be NULL after a failed build"
    return rc, msg


def test_valid_build_ok():
    assert build_raw(base_arrays()) == (0, "")


@pytest.mark.parametrize("mutate, code, needle", [
    (lambda a: a.__setitem__("nb", 0), pf.PF_EINVAL, "nb"),
    (lambda a: a["fbus"].__setitem__(0, 6), pf.PF_EINVAL, "out of range"),
    (lambda a: a["tbus"].__setitem__(1, -1), pf.PF_EINVAL, "out of range"),
    (lambda a: a["tbus"].__setitem__(2, a["fbus"][2]), pf.PF_EINVAL, "from == to"),
    (lambda a: a["tap"].__setitem__(0, -1.0), pf.PF_EINVAL, "tap < 0"),
    (lambda a: a["r"].__setitem__(3, np.nan), pf.PF_EINVAL, "non-finite"),
    (lambda a: a["shift"].__setitem__(3, np.inf), pf.PF_EINVAL, "non-finite"),
    (lambda a: (a["r"].__setitem__(1, 0.0), a["x"].__setitem__(1, 0.0)), pf.PF_EINVAL, "r = x = 0"),
    (lambda a: a["gs"].__setitem__(2, np.nan), pf.PF_EINVAL, "shunt"),
    (lambda a: a.__setitem__("nl", -1), pf.PF_EINVAL, "nl"),
])
def test_validation_errors(mutate, code, needle):
    a = base_arrays()
    mutate(a)
    rc, msg = build_raw(a)
    assert rc == code and needle in msg


def test_null_branch_arrays_rejected():
    L = pf.lib()
    h = C.c_void_p()
    rc = L.pf_build_pattern(3, 2, None, None, None, None, None, None, None, None, None, 1, None, None, 1, C.byref(h))
    assert rc == pf.PF_EINVAL and "NULL" in L.pf_last_error().decode()
    rc = L.pf_build_pattern(3, 0, None, None, None, None, None, None, None, None, None, 1, None, None, 1, None)
    assert rc == pf.PF_EINVAL


def test_multigrid_offsets_validated():
    a = base_arrays()
    assert build_raw(a, 2, None, None)[0] == pf.PF_EINVAL
    assert build_raw(a, 2, [0, 3, 5], [0, 4, 8])[0] == pf.PF_EINVAL   # does not end at nb
    assert build_raw(a, 2, [0, 3, 6], [0, 9, 8])[0] == pf.PF_EINVAL   # decreasing
    assert build_raw(a, 2, [0, 0, 6], [0, 4, 8])[0] == pf.PF_EINVAL   # empty grid
    rc, msg = build_raw(a, 2, [0, 3, 6], [0, 4, 8])
    # branch indices are grid-local: the second grid has buses 0..2 only
    assert rc in (pf.PF_OK, pf.PF_EINVAL)


def test_unknown_flag_rejected():
    assert build_raw(base_arrays(), flags=0x10)[0] == pf.PF_EINVAL


def test_eval_on_host_only_handle_is_state_error():
    G = pf.Grid.from_grid(_grids.random_small(6, 8, 5), host_only=True)
    L = pf.lib()
    assert L.pf_ybus(G.handle, None, None, None) == pf.PF_ESTATE
    assert L.pf_injections_elementwise(G.handle, 1, None, None, None, None, None) == pf.PF_ESTATE
    assert L.pf_jacobian_values(G.handle, 0, 1, None, None, None, None, None, None) == pf.PF_ESTATE
    assert L.pf_injections_vjp(G.handle, 1, None, None, None, None, None, None, None) == pf.PF_ESTATE
    assert L.pf_phasors(G.handle, 1, 1, None, None, None, None) == pf.PF_ESTATE
    assert L.pf_ybus_from_phasors(G.handle, 1, 1, None, None, None, None, None) == pf.PF_ESTATE
    assert "HOST_ONLY" in L.pf_last_error().decode()
    assert L.pf_injections_elementwise(None, 1, None, None, None, None, None) == pf.PF_EINVAL


def test_graph_create_argument_checks():
    G = pf.Grid.from_grid(_grids.random_small(6, 8, 5), host_only=True)
    L = pf.lib()
    out = C.c_void_p()
    ops = (pf.PfOp * 1)()
    assert L.pf_graph_create(G.handle, ops, 1, C.byref(out)) == pf.PF_ESTATE
    assert out.value is None
    assert L.pf_graph_create(None, ops, 1, C.byref(out)) == pf.PF_EINVAL
    assert L.pf_graph_create(G.handle, ops, 0, C.byref(out)) == pf.PF_EINVAL
    assert L.pf_graph_create(G.handle, ops, 1, None) == pf.PF_EINVAL
    assert L.pf_graph_launch(None, None) == pf.PF_EINVAL
    L.pf_graph_free(None)  # no-op


def test_schedule_choices():
    G = pf.Grid.from_grid(gridgen.grid_500(), host_only=True)
    for cap in (64, 128, 256, 512):
        G.set_schedule(cap, 0)
        t, spb, order, nt = G.schedule()
        assert t == cap and nt >= (500 + 1900) // cap // 2
    with pytest.raises(pf.PFError) as e:
        G.set_schedule(100, 0)
    assert e.value.code == pf.PF_EINVAL
    with pytest.raises(pf.PFError):
        G.set_schedule(256, -1)
    with pytest.raises(pf.PFError):
        G.set_schedule(256, 0, 7)
    with pytest.raises(pf.PFError):
        G.set_schedule(256, 0, 4)
    G.set_schedule(128, 3, pf.PF_ORDER_STATE_MAJOR)
    assert G.schedule()[:3] == (128, 3, pf.PF_ORDER_STATE_MAJOR)
    G.set_schedule(64, 2, pf.PF_ORDER_GROUPED)
    assert G.schedule()[:3] == (64, 2, pf.PF_ORDER_GROUPED)


def test_binding_refuses_host_arrays():
    G = pf.Grid.from_grid(_grids.random_small(6, 8, 5), host_only=True)
    import torch
    with pytest.raises((TypeError, ValueError)):
        pf.pf_injections_elementwise(G, torch.zeros(6, dtype=torch.float64), torch.zeros(6, dtype=torch.float64),
                                     torch.zeros(6, dtype=torch.float64), torch.zeros(6, dtype=torch.float64))


def test_bind_refuses_unknown_calls_and_host_arrays():
    import torch
    with pytest.raises(ValueError):
        pf.bind("pf_ybus")
    G = pf.Grid.from_grid(_grids.random_small(6, 8, 5), host_only=True)
    z = torch.zeros(6, dtype=torch.float64)
    with pytest.raises((TypeError, ValueError)):
        pf.bind(pf.pf_injections_elementwise, G, z, z, z, z)


def test_stream_copy_argument_checks():
    """pf_stream_copy rejects bad arguments on the host, before any launch."""
    import ctypes as C
    L = pf.lib()
    a, b = C.c_void_p(1 << 20), C.c_void_p(2 << 20)
    assert L.pf_stream_copy(None, None, 0, None) == pf.PF_OK  # nothing to copy
    assert L.pf_stream_copy(a, b, -1, None) == pf.PF_EINVAL
    assert L.pf_stream_copy(None, b, 4, None) == pf.PF_EINVAL
    assert L.pf_stream_copy(C.c_void_p((1 << 20) + 8), b, 4, None) == pf.PF_EINVAL  # not 16-byte aligned
    assert L.pf_stream_copy(a, C.c_void_p((1 << 20) + 16), 4, None) == pf.PF_EINVAL  # overlapping
    assert b"overlap" in L.pf_last_error()


def test_default_tile_size_follows_grid_size():
    """Tiles never span grids: a handle of many small grids starts with the
    smallest tile that holds a mean grid's branch ends; one grid, or large
    grids, start at 256."""
    small = [gridgen.make_grid(14, 20, 0.15, case=6, grid=k) for k in range(50)]     # 40 ends per grid
    mid = [gridgen.make_grid(40, 55, 0.15, case=6, grid=100 + k) for k in range(10)]  # 110 ends per grid
    large = [gridgen.make_grid(500, 700, 0.15, case=6, grid=200 + k) for k in range(3)]
    for grids, want in ((small, 64), (mid, 128), (large, 256)):
        big, bo, ro = gridgen.concat(grids)
        assert pf.Grid.from_grid(big, bo, ro, host_only=True).schedule()[0] == want
    assert pf.Grid.from_grid(small[0], host_only=True).schedule()[0] == 256


# Full-size pattern identity (Algorithm 2's pattern, Section IV.B): the
# exported Ybus and Jacobian patterns of the benchmark grids equal the
# oracle's independently built ones bit for bit.
@pytest.mark.parametrize("which", ["grid_100k", "grid_100k_relabelled", "grids_uneven_64"])
def test_pattern_matches_oracle_full_size(which):
    if which == "grids_uneven_64":
        grids = gridgen.grids_uneven_64()
        big, bo, ro = gridgen.concat(grids)
        G = pf.Grid.from_grid(big, bo, ro, host_only=True)
    else:
        g = gridgen.grid_100k()
        if which == "grid_100k_relabelled":
            g, _ = gridgen.relabel(g, case=1)
        grids = [g]
        G = pf.Grid.from_grid(g, host_only=True)
    got = G.pattern()
    want = per_grid_oracle_pattern(grids)
    for a, b in zip(got, want):
        assert a.dtype == np.int32 and a.shape == b.shape and np.array_equal(a, b)
    assert G.nnz_j == 4 * G.nnz_y == 4 * sum(oracle.ybus(g).nnz for g in grids)


def test_debug_alloc_hook_arguments():
    """The allocation-failure hook (include/pf_testing.h) takes n >= 0."""
    with pytest.raises(pf.PFError) as e:
        pf.pf_debug_fail_allocs(-1)
    assert e.value.code == pf.PF_EINVAL
    pf.pf_debug_fail_allocs(0)
