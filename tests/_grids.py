"""Small hand-built and randomised grids for unit tests (inputs only, no method arithmetic)."""
from __future__ import annotations

import numpy as np

from paper_2302_10736_amd.gridgen import Grid


def two_bus(r, x, b, tap, shift, gs=(0.0, 0.0), bs=(0.0, 0.0), flip=False) -> Grid:
    f, t = (1, 0) if flip else (0, 1)
    a = lambda v: np.array([v], dtype=np.float64)
    return Grid(2, 1, np.array([f], np.int32), np.array([t], np.int32), a(r), a(x), a(b), a(tap), a(shift),
                np.array(gs, np.float64), np.array(bs, np.float64))


def random_small(nb: int, nl: int, seed: int, parallel: int = 0, isolated: int = 0, lossless: bool = False,
                 xf_frac: float = 0.3) -> Grid:
    """Random grid with optional parallel branches and isolated buses.

    Buses ``nb - isolated .. nb - 1`` touch no branch.  ``parallel`` extra
    branches duplicate the bus pair of an existing branch (either
    orientation).  ``lossless`` sets r = 0 and bus shunt g = 0.
    """
    g = np.random.default_rng(seed)
    live = nb - isolated
    assert live >= 2
    f = []
    t = []
    for i in range(1, live):  # spanning tree over the live buses
        p = int(g.integers(0, i))
        f.append(i)
        t.append(p)
    while len(f) < nl - parallel:
        a, c = g.integers(0, live, 2)
        if a != c:
            f.append(int(a))
            t.append(int(c))
    for _ in range(parallel):
        k = int(g.integers(0, len(f)))
        if g.random() < 0.5:
            f.append(f[k]); t.append(t[k])
        else:
            f.append(t[k]); t.append(f[k])
    n = len(f)
    perm = g.permutation(n)
    fb = np.array(f, np.int32)[perm]
    tb = np.array(t, np.int32)[perm]
    r = np.zeros(n) if lossless else g.uniform(0.001, 0.05, n)
    x = g.uniform(0.01, 0.3, n)
    b = g.uniform(0.0, 0.1, n)
    tap = np.ones(n)
    shift = np.zeros(n)
    xf = g.random(n) < xf_frac
    tap[xf] = g.uniform(0.9, 1.1, xf.sum())
    shift[xf] = np.deg2rad(g.uniform(-10, 10, xf.sum()))
    gs = np.zeros(nb)
    bs = np.zeros(nb)
    sh = g.random(nb) < 0.3
    if not lossless:
        gs[sh] = g.uniform(0, 0.02, sh.sum())
    bs[sh] = g.uniform(-0.1, 0.1, sh.sum())
    return Grid(nb, n, fb, tb, r, x, b, tap, shift, gs, bs)


def random_hubs(nb: int, nhub: int, deg_lo: int, deg_hi: int, parallel: int, seed: int) -> Grid:
    """A random tree on nb buses plus nhub hub buses joined to deg_lo..deg_hi random other buses each
    (rows longer than any tile), and `parallel` duplicated branches drawn from all of them."""
    rng = np.random.default_rng(seed)
    f = [int(rng.integers(0, i)) for i in range(1, nb)]
    t = list(range(1, nb))
    for h in rng.choice(nb, size=nhub, replace=False):
        deg = int(rng.integers(deg_lo, deg_hi + 1))
        for o in rng.choice(nb, size=min(deg, nb - 1), replace=False):
            if o != h:
                f.append(int(h))
                t.append(int(o))
    for _ in range(parallel):
        k = int(rng.integers(0, len(f)))
        f.append(f[k])
        t.append(t[k])
    n = len(f)
    flip = rng.random(n) < 0.5
    fb = np.where(flip, t, f).astype(np.int32)
    tb = np.where(flip, f, t).astype(np.int32)
    tap = np.where(rng.random(n) < 0.3, rng.uniform(0.9, 1.1, n), 1.0)
    shift = np.where(tap != 1.0, rng.uniform(-0.1, 0.1, n), 0.0)
    return Grid(nb, n, fb, tb, rng.uniform(0.001, 0.05, n), rng.uniform(0.01, 0.3, n), rng.uniform(0, 0.1, n),
                tap, shift, rng.uniform(0, 0.02, nb), rng.uniform(-0.1, 0.1, nb))


def random_state(nb: int, seed: int, sigma: float = 0.2):
    g = np.random.default_rng(seed + 7919)
    return g.uniform(0.9, 1.1, nb), g.normal(0.0, sigma, nb)
