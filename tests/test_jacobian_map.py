"""Algorithm 2 on a general target pattern (pf_jacobian_map, host) and the
in-place copy by its indices (pf_jacobian_scatter, GPU).  The expected
positions come from a dictionary of the target's (row, column) pairs built
here, independent of the library's search."""
from __future__ import annotations

import ctypes as C

import numpy as np
import pytest

from paper_2302_10736_amd import gridgen, pf
from tests import _grids


def our_entries(G):
    """(row, column) of every J entry in the exported CSR order."""
    _, _, jr, jc = G.pattern()
    rows = np.repeat(np.arange(len(jr) - 1), np.diff(jr))
    return rows, jc


def target_with_extras(G, n_extra, seed, shuffle):
    """J's pattern plus n_extra coupling entries (a series device between two
    buses adds its pair to all four blocks), as CSR; rows optionally shuffled."""
    rng = np.random.default_rng(seed)
    nb = G.nb
    rows, cols = our_entries(G)
    pairs = set(zip(rows.tolist(), cols.tolist()))
    for _ in range(n_extra):
        i, k = rng.integers(0, nb, 2)
        for a, b in ((i, k), (k, i)):
            for rb in (0, nb):
                for cb in (0, nb):
                    pairs.add((int(a) + rb, int(b) + cb))
    by_row = [[] for _ in range(2 * nb)]
    for r, c in pairs:
        by_row[r].append(c)
    ptr = [0]
    idx = []
    for r in range(2 * nb):
        cs = sorted(by_row[r])
        if shuffle:
            rng.shuffle(cs)
        idx += cs
        ptr.append(len(idx))
    return np.array(ptr, np.int32), np.array(idx, np.int32)


def expected_map(G, ptr, idx, csc=False):
    pos = {}
    for major in range(len(ptr) - 1):
        for q in range(ptr[major], ptr[major + 1]):
            pos[(major, int(idx[q])) if not csc else (int(idx[q]), major)] = q
    rows, cols = our_entries(G)
    return np.array([pos[(int(r), int(c))] for r, c in zip(rows, cols)], np.int32)


def to_csc(ptr, idx, n):
    rows = np.repeat(np.arange(n), np.diff(ptr))
    order = np.lexsort((rows, idx))
    cptr = np.zeros(n + 1, np.int32)
    np.add.at(cptr, idx + 1, 1)
    return np.cumsum(cptr).astype(np.int32), rows[order].astype(np.int32)


@pytest.fixture(scope="module")
def grid():
    return pf.Grid.from_grid(_grids.random_small(120, 200, 31, parallel=4, isolated=2), host_only=True)


def test_own_pattern_is_the_identity(grid):
    _, _, jr, jc = grid.pattern()
    m = pf.pf_jacobian_map(grid, pf.PF_LAYOUT_CSR, jr, jc)
    assert np.array_equal(m, np.arange(grid.nnz_j))


@pytest.mark.parametrize("shuffle", [False, True])
@pytest.mark.parametrize("layout", [pf.PF_LAYOUT_CSR, pf.PF_LAYOUT_CSC])
def test_superset_patterns(grid, shuffle, layout):
    ptr, idx = target_with_extras(grid, 15, 7, shuffle)
    if layout == pf.PF_LAYOUT_CSC:
        ptr, idx = to_csc(ptr, idx, 2 * grid.nb)
        if shuffle:  # unsorted columns take the linear search
            rng = np.random.default_rng(3)
            for c in range(2 * grid.nb):
                seg = idx[ptr[c]:ptr[c + 1]].copy()
                rng.shuffle(seg)
                idx[ptr[c]:ptr[c + 1]] = seg
    want = expected_map(grid, ptr, idx, csc=layout == pf.PF_LAYOUT_CSC)
    got = pf.pf_jacobian_map(grid, layout, ptr, idx)
    assert np.array_equal(got, want)


def test_missing_entry_and_malformed_targets(grid):
    _, _, jr, jc = grid.pattern()
    L = pf.lib()
    out = np.zeros(grid.nnz_j, np.int32)
    hp = lambda a: a.ctypes.data_as(C.c_void_p)
    # drop one entry of row 5: the call names the missing entry
    k = int(jr[5]) + 1
    idx = np.delete(jc, k).astype(np.int32)
    ptr = jr.copy()
    ptr[6:] -= 1
    assert L.pf_jacobian_map(grid.handle, 0, len(ptr) - 1, hp(ptr), hp(idx), hp(out)) == pf.PF_EINVAL
    assert f"(5, {jc[k]})" in L.pf_last_error().decode()
    bad = jc.copy()
    bad[0] = 2 * grid.nb  # out of range
    assert L.pf_jacobian_map(grid.handle, 0, len(jr) - 1, hp(jr), hp(bad), hp(out)) == pf.PF_EINVAL
    dec = jr.copy()
    dec[3], dec[4] = dec[4], dec[3]  # decreasing pointer
    assert L.pf_jacobian_map(grid.handle, 0, len(jr) - 1, hp(dec), hp(jc), hp(out)) == pf.PF_EINVAL
    assert L.pf_jacobian_map(grid.handle, 0, len(jr) - 2, hp(jr), hp(jc), hp(out)) == pf.PF_EINVAL  # wrong size
    assert L.pf_jacobian_map(grid.handle, 2, len(jr) - 1, hp(jr), hp(jc), hp(out)) == pf.PF_EINVAL  # layout


def test_multigrid_handle_unsupported():
    grids = [_grids.random_small(n, int(1.4 * n), n) for n in (5, 9)]
    big, bo, ro = gridgen.concat(grids)
    G = pf.Grid.from_grid(big, bo, ro, host_only=True)
    _, _, jr, jc = G.pattern()
    with pytest.raises(pf.PFError) as e:
        pf.pf_jacobian_map(G, pf.PF_LAYOUT_CSR, jr[: 2 * G.nb + 1], jc)
    assert e.value.code == pf.PF_EUNSUP


@pytest.mark.gpu
def test_scatter_into_superset_pattern():
    import torch
    from tests._gpu import require_gpu, to_dev
    require_gpu()
    g = _grids.random_small(300, 520, 41, parallel=3, isolated=2)
    G = pf.Grid.from_grid(g)
    ptr, idx = target_with_extras(G, 40, 11, shuffle=False)
    m = pf.pf_jacobian_map(G, pf.PF_LAYOUT_CSR, ptr, idx)
    rng = np.random.default_rng(4)
    ns = 3
    vm, va = to_dev(rng.uniform(0.9, 1.1, (ns, g.nb))), to_dev(rng.normal(0, 0.2, (ns, g.nb)))
    j = torch.empty(ns, G.nnz_j, dtype=torch.float64, device="cuda:0")
    pf.pf_jacobian_values(G, pf.PF_METHOD_ELEMENTWISE, vm, va, None, None, j)
    out_nnz = len(idx)
    out = torch.full((ns, out_nnz), -7.0, dtype=torch.float64, device="cuda:0")
    jm = torch.as_tensor(m, device="cuda:0")
    pf.pf_jacobian_scatter(G, j, jm, out)
    torch.cuda.synchronize()
    o, jh = out.cpu().numpy(), j.cpu().numpy()
    assert np.array_equal(o[:, m], jh)
    rest = np.setdiff1d(np.arange(out_nnz), m)
    assert len(rest) > 0 and np.all(o[:, rest] == -7.0)  # the device's extra entries are left alone
    # a map entry outside the target is skipped (the kernel guards every write)
    m2 = m.copy()
    m2[0] = out_nnz + 5
    out.fill_(-7.0)
    pf.pf_jacobian_scatter(G, j, torch.as_tensor(m2, device="cuda:0"), out)
    torch.cuda.synchronize()
    o2 = out.cpu().numpy()
    assert np.all(o2[:, m[0]] == -7.0) and np.array_equal(o2[:, m2[1:]], jh[:, 1:])
