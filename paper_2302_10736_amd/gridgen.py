"""Seeded synthetic grids, voltage states and adjoint seeds.

This module only draws random inputs.  It holds none of the power-flow
arithmetic, so both the library's GPU path and the CPU oracle can consume
its output without sharing any of the method's code.

The paper measures on MATPOWER cases from 14 to 82,000 buses and on
replicas of the 82k-bus synthetic USA case (Section V).  Those files are not
available here; these generators stand in for them, with a branch-to-bus
ratio of 1.2-1.5 (the 82k case has about 1.27, from the 16 n_l Jacobian
element count quoted in Section V.A).

Recipe (every grid):

* topology: a random spanning tree in which bus i >= 1 attaches to a parent
  drawn uniformly from [max(0, i-64), i-1] (local numbering, large
  diameter, like real grids), plus ``nl - (nb-1)`` extra edges whose ends
  are at most 10 tree hops apart; self loops and duplicate bus pairs are
  rejected, so these grids carry no parallel branches (unit tests add them
  explicitly);
* every branch draws r ~ U(0.001, 0.05), x ~ U(0.01, 0.3),
  b_charging ~ U(0, 0.1) p.u.; each end orientation is a coin flip;
* a fraction of branches (uniform, without replacement) are transformers
  with tap ~ U(0.95, 1.05) and shift ~ U(-5, 5) degrees (returned in
  radians); other branches have tap 1 and shift 0;
* 10 % of buses (uniform, without replacement) carry a shunt
  g ~ U(0, 0.02), b ~ U(-0.1, 0.1);
* states: vm ~ U(lo, hi), va ~ N(0, sigma) radians;
* adjoint seeds: lambda_P, lambda_Q ~ N(0, 1).

Streams: ``numpy.random.Generator(PCG64(SeedSequence([2302, 10736, case,
grid, stream])))`` with case numbering the workload (0: 500 buses, 1: 100k
buses, 2: 20k buses x 512 states, 3: 64 uneven grids, 4: the adjoint states
on the 100k-bus grid, 5: the size sweep), stream 0 = topology and
parameters, 1 = states, 2 = adjoint seeds, 3 = sampled coordinates,
4 = the bus relabelling of :func:`relabel`.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

SEED_ROOT = (2302, 10736)


def rng(case: int, grid: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([*SEED_ROOT, case, grid, stream])))


@dataclass
class Grid:
    nb: int
    nl: int
    fbus: np.ndarray  # int32[nl], 0-based
    tbus: np.ndarray  # int32[nl]
    r: np.ndarray     # f64[nl]
    x: np.ndarray
    b: np.ndarray     # total line charging susceptance
    tap: np.ndarray   # off-nominal ratio m (1 for lines)
    shift: np.ndarray  # radians
    gs: np.ndarray    # f64[nb] bus shunt conductance
    bs: np.ndarray    # f64[nb] bus shunt susceptance
    meta: dict = field(default_factory=dict)

    def arrays(self):
        return (self.fbus, self.tbus, self.r, self.x, self.b, self.tap, self.shift, self.gs, self.bs)


def _tree(nb: int, g: np.random.Generator) -> np.ndarray:
    """Parent of every bus i >= 1, drawn from [max(0, i-64), i-1]."""
    i = np.arange(1, nb, dtype=np.int64)
    lo = np.maximum(0, i - 64)
    return lo + np.floor(g.random(nb - 1) * (i - lo)).astype(np.int64)


def _extra_edges(nb: int, parent: np.ndarray, n_extra: int, g: np.random.Generator) -> np.ndarray:
    """``n_extra`` new bus pairs whose tree distance is 2..10 (random walks)."""
    if n_extra <= 0:
        return np.zeros((0, 2), dtype=np.int64)
    if nb < 3:
        raise ValueError("extra edges need at least 3 buses")
    child = np.arange(1, nb, dtype=np.int64)
    u = np.concatenate([child, parent])
    v = np.concatenate([parent, child])
    order = np.argsort(u, kind="stable")
    adj = v[order]
    ptr = np.zeros(nb + 1, dtype=np.int64)
    np.add.at(ptr, u + 1, 1)
    ptr = np.cumsum(ptr)
    deg = np.diff(ptr)
    existing = set(zip(np.minimum(child, parent).tolist(), np.maximum(child, parent).tolist()))
    out: list[tuple[int, int]] = []
    while len(out) < n_extra:
        m = max(64, 2 * (n_extra - len(out)))
        start = g.integers(0, nb, size=m)
        hops = g.integers(2, 11, size=m)
        cur = start.copy()
        for step in range(10):
            live = step < hops
            pick = np.floor(g.random(m) * deg[cur]).astype(np.int64)
            nxt = adj[ptr[cur] + pick]
            cur = np.where(live, nxt, cur)
        for a, c in zip(start.tolist(), cur.tolist()):
            if a == c:
                continue
            key = (min(a, c), max(a, c))
            if key in existing:
                continue
            existing.add(key)
            out.append((a, c))
            if len(out) == n_extra:
                break
    return np.asarray(out, dtype=np.int64)


def make_grid(nb: int, nl: int, xf_frac: float, case: int, grid: int = 0) -> Grid:
    if nb < 2 or nl < nb - 1:
        raise ValueError("need nb >= 2 and nl >= nb - 1 for a connected grid")
    g = rng(case, grid, 0)
    parent = _tree(nb, g)
    tree = np.stack([np.arange(1, nb, dtype=np.int64), parent], axis=1)
    extra = _extra_edges(nb, parent, nl - (nb - 1), g)
    pairs = np.concatenate([tree, extra], axis=0)
    flip = g.random(nl) < 0.5
    fbus = np.where(flip, pairs[:, 1], pairs[:, 0]).astype(np.int32)
    tbus = np.where(flip, pairs[:, 0], pairs[:, 1]).astype(np.int32)
    r = g.uniform(0.001, 0.05, nl)
    x = g.uniform(0.01, 0.3, nl)
    b = g.uniform(0.0, 0.1, nl)
    tap = np.ones(nl)
    shift = np.zeros(nl)
    nxf = int(round(xf_frac * nl))
    xf = g.choice(nl, size=nxf, replace=False)
    tap[xf] = g.uniform(0.95, 1.05, nxf)
    shift[xf] = np.deg2rad(g.uniform(-5.0, 5.0, nxf))
    gs = np.zeros(nb)
    bs = np.zeros(nb)
    nsh = int(round(0.1 * nb))
    sh = g.choice(nb, size=nsh, replace=False)
    gs[sh] = g.uniform(0.0, 0.02, nsh)
    bs[sh] = g.uniform(-0.1, 0.1, nsh)
    return Grid(nb, nl, fbus, tbus, r, x, b, tap, shift, gs, bs,
                meta={"case": case, "grid": grid, "xf_frac": xf_frac})


def states(nb: int, nstate: int, case: int, grid: int = 0, vlo: float = 0.95, vhi: float = 1.05,
           sigma: float = 0.2) -> tuple[np.ndarray, np.ndarray]:
    """vm, va as float64 [nstate, nb]."""
    g = rng(case, grid, 1)
    vm = g.uniform(vlo, vhi, (nstate, nb))
    va = g.normal(0.0, sigma, (nstate, nb))
    return vm, va


def adjoint_seeds(nb: int, nstate: int, case: int, grid: int = 0) -> tuple[np.ndarray, np.ndarray]:
    g = rng(case, grid, 2)
    return g.normal(0.0, 1.0, (nstate, nb)), g.normal(0.0, 1.0, (nstate, nb))


def sample_coords(nstate: int, nb: int, count: int, case: int, grid: int = 0) -> np.ndarray:
    """``count`` (state, var, bus) triples, var 0 = vm, 1 = va."""
    g = rng(case, grid, 3)
    return np.stack([g.integers(0, nstate, count), g.integers(0, 2, count), g.integers(0, nb, count)], axis=1)


def relabel(g: Grid, case: int, grid: int = 0) -> tuple[Grid, np.ndarray]:
    """The same grid with its buses renumbered by a seeded random permutation
    (a stress case for locality: the generator's numbering keeps neighbours
    close, real case files need not).  Returns (grid, perm) with new bus
    number perm[old]; branch order and parameters are unchanged, bus shunts
    move with their buses, and a state x of the original grid is
    ``x[..., inv]`` here with ``inv = numpy.argsort(perm)``."""
    perm = rng(case, grid, 4).permutation(g.nb)
    return renumber(g, perm), perm


def renumber(g: Grid, perm: np.ndarray) -> Grid:
    """The grid with bus i renamed perm[i] (perm a permutation of 0..nb-1)."""
    perm = np.asarray(perm)
    inv = np.argsort(perm)
    return Grid(g.nb, g.nl, perm[g.fbus].astype(np.int32), perm[g.tbus].astype(np.int32), g.r.copy(), g.x.copy(),
                g.b.copy(), g.tap.copy(), g.shift.copy(), g.gs[inv].copy(), g.bs[inv].copy(),
                meta={**g.meta, "renumbered": True})


# ---------------------------------------------------------------------------
# The five workloads


def grid_500() -> Grid:
    """500 buses, 700 branches, 15 % transformers."""
    return make_grid(500, 700, 0.15, case=0)


def grid_100k() -> Grid:
    """100,000 buses, 130,000 branches, 20 % transformers."""
    return make_grid(100_000, 130_000, 0.20, case=1)


def grid_20k() -> Grid:
    """20,000 buses, 27,000 branches, 15 % transformers (batched states)."""
    return make_grid(20_000, 27_000, 0.15, case=2)


def uneven_sizes(ngrid: int = 64) -> list[tuple[int, int]]:
    """(nb, nl) of the uneven grids: nb log-uniform in [1e3, 8e4], nl = nb U(1.2, 1.5)."""
    g = rng(3, 0, 0)
    nb = np.rint(np.exp(g.uniform(math.log(1e3), math.log(8e4), ngrid))).astype(np.int64)
    ratio = g.uniform(1.2, 1.5, ngrid)
    nl = np.rint(nb * ratio).astype(np.int64)
    return [(int(a), int(c)) for a, c in zip(nb, nl)]


def grids_uneven_64(ngrid: int = 64) -> list[Grid]:
    return [make_grid(nb, nl, 0.15, case=3, grid=k + 1) for k, (nb, nl) in enumerate(uneven_sizes(ngrid))]


def grid_hubs(nb: int = 20_000, nl: int = 27_000, nhub: int = 32, deg_lo: int = 200, deg_hi: int = 2_000,
              case: int = 6) -> Grid:
    """A generator grid (15 % transformers) plus ``nhub`` hub buses, each
    joined to a log-uniform number of distinct other buses in [deg_lo,
    deg_hi] by extra lines of the same parameter distributions (the long-row
    timing case: hub rows exceed every tile size)."""
    base = make_grid(nb, nl, 0.15, case=case)
    g = rng(case, 0, 5)
    hubs = g.choice(nb, size=nhub, replace=False)
    deg = np.rint(np.exp(g.uniform(math.log(deg_lo), math.log(deg_hi), nhub))).astype(np.int64)
    existing = set(zip(np.minimum(base.fbus, base.tbus).tolist(), np.maximum(base.fbus, base.tbus).tolist()))
    pairs = []
    for h, d in zip(hubs.tolist(), deg.tolist()):
        cand = g.permutation(nb)
        got = 0
        for c in cand.tolist():
            key = (min(h, c), max(h, c))
            if c == h or key in existing:
                continue
            existing.add(key)
            pairs.append((h, c))
            got += 1
            if got == d:
                break
    pairs = np.asarray(pairs, dtype=np.int64)
    m = len(pairs)
    flip = g.random(m) < 0.5
    fb = np.where(flip, pairs[:, 1], pairs[:, 0]).astype(np.int32)
    tb = np.where(flip, pairs[:, 0], pairs[:, 1]).astype(np.int32)
    cat = lambda a, b: np.concatenate([a, b])
    return Grid(nb, nl + m, cat(base.fbus, fb), cat(base.tbus, tb), cat(base.r, g.uniform(0.001, 0.05, m)),
                cat(base.x, g.uniform(0.01, 0.3, m)), cat(base.b, g.uniform(0.0, 0.1, m)), cat(base.tap, np.ones(m)),
                cat(base.shift, np.zeros(m)), base.gs.copy(), base.bs.copy(),
                meta={"case": case, "hubs": hubs.tolist(), "hub_degrees": deg.tolist()})


def concat(grids: list[Grid]) -> tuple[Grid, np.ndarray, np.ndarray]:
    """Concatenate grids for one multi-grid handle.

    Bus indices stay grid-local; returns (grid, bus_off[G+1], br_off[G+1])
    where grid k owns buses [bus_off[k], bus_off[k+1]) and branches
    [br_off[k], br_off[k+1]) of the concatenation.
    """
    nbs = np.array([gr.nb for gr in grids], dtype=np.int64)
    nls = np.array([gr.nl for gr in grids], dtype=np.int64)
    bus_off = np.concatenate([[0], np.cumsum(nbs)]).astype(np.int32)
    br_off = np.concatenate([[0], np.cumsum(nls)]).astype(np.int32)
    cat = lambda name: np.concatenate([getattr(gr, name) for gr in grids])
    big = Grid(int(nbs.sum()), int(nls.sum()), cat("fbus").astype(np.int32), cat("tbus").astype(np.int32),
               cat("r"), cat("x"), cat("b"), cat("tap"), cat("shift"), cat("gs"), cat("bs"),
               meta={"ngrids": len(grids)})
    return big, bus_off, br_off
