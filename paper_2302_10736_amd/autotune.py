"""Schedule autotuner.

Chooses the launch schedule of a grid handle (tile size, states per
workgroup, work order; see ``pf_set_schedule`` in include/pf.h) for one
operation and batch size by timing candidate schedules on the device, and
caches the choice in a JSON file keyed by device, library build and problem
shape.  Every schedule gives bit-identical results (all sums run in an order
fixed by the pattern), so tuning changes speed only.

    sched = autotune.tune(grid, "jacobian_ew", nstate=512)
    autotune.apply(grid, "jacobian_ew", nstate=512)   # from the cache later

The cache file is ``$PF_SCHEDULE_CACHE`` if set, else
``~/.cache/pf_mi355x/schedules.json``.
"""
from __future__ import annotations

import hashlib
import json
import os
import tempfile
from typing import Callable, Iterable, Optional, Sequence, Tuple

from . import pf

OPS = ("injections_ew", "injections_ybus", "jacobian_ew", "jacobian_ybus", "vjp", "jacobian_ew_csc",
       "jacobian_ybus_csc")
TILES = (64, 128, 256, 512)
STATES_PER_BLOCK = (1, 2, 4, 8, 16, 32, 64)

Schedule = Tuple[int, int, int]  # (tile_items, states_per_block, order)


def candidates(nstate: int, tiles: Sequence[int] = TILES) -> list:
    """Candidate schedules for a batch of ``nstate`` states.

    One state: one workgroup per tile, order irrelevant.  Several states:
    the automatic split (0) and explicit states per workgroup up to nstate,
    each in the three work orders."""
    if nstate <= 1:
        return [(t, 1, pf.PF_ORDER_TILE_MAJOR) for t in tiles]
    spbs = [0] + [s for s in STATES_PER_BLOCK if s <= nstate]
    orders = (pf.PF_ORDER_TILE_MAJOR, pf.PF_ORDER_STATE_MAJOR, pf.PF_ORDER_GROUPED)
    return [(t, s, o) for t in tiles for s in spbs for o in orders]


def default_cache_path() -> str:
    env = os.environ.get("PF_SCHEDULE_CACHE")
    if env:
        return env
    return os.path.join(os.path.expanduser("~"), ".cache", "pf_mi355x", "schedules.json")


_lib_id = None


def library_id() -> str:
    """Version string and a hash of the built library: a rebuilt library
    invalidates cached choices."""
    global _lib_id
    if _lib_id is None:
        h = hashlib.sha256()
        with open(pf.LIB_PATH, "rb") as f:
            h.update(f.read())
        _lib_id = f"{pf.pf_version()}|{h.hexdigest()[:16]}"
    return _lib_id


def problem_key(grid: "pf.Grid", op: str, nstate: int, device: str, lib: str) -> str:
    if op not in OPS:
        raise ValueError(f"unknown op {op!r}; one of {OPS}")
    return f"{device}|{lib}|nb={grid.nb}|nnzy={grid.nnz_y}|grids={grid.ngrids}|op={op}|nstate={nstate}"


class ScheduleCache:
    """A JSON file of {key: {"schedule": [tile, spb, order], "us": t, "tried": n}}."""

    def __init__(self, path: Optional[str] = None):
        self.path = path or default_cache_path()
        self.entries = {}
        if os.path.exists(self.path):
            try:
                with open(self.path) as f:
                    data = json.load(f)
                if isinstance(data, dict):
                    self.entries = data
            except (OSError, ValueError):
                self.entries = {}  # unreadable cache: start afresh

    def get(self, key: str) -> Optional[Schedule]:
        e = self.entries.get(key)
        if not e:
            return None
        t, s, o = e["schedule"]
        return int(t), int(s), int(o)

    def put(self, key: str, sched: Schedule, us: float, tried: int) -> None:
        self.entries[key] = {"schedule": list(sched), "us": us, "tried": tried}

    def save(self) -> None:
        d = os.path.dirname(self.path)
        if d:
            os.makedirs(d, exist_ok=True)
        fd, tmp = tempfile.mkstemp(dir=d or ".", prefix=".schedules.", suffix=".json")
        with os.fdopen(fd, "w") as f:
            json.dump(self.entries, f, indent=1, sort_keys=True)
        os.replace(tmp, self.path)  # atomic: readers see the old or the new file


def _device_name() -> str:
    import torch
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return f"{p.name}|{getattr(p, 'gcnArchName', '')}"


# (op name) -> (pf_op op, method)
_OP = {"injections_ew": (pf.PF_OP_INJECTIONS, pf.PF_METHOD_ELEMENTWISE),
       "injections_ybus": (pf.PF_OP_INJECTIONS, pf.PF_METHOD_YBUS),
       "jacobian_ew": (pf.PF_OP_JACOBIAN, pf.PF_METHOD_ELEMENTWISE),
       "jacobian_ybus": (pf.PF_OP_JACOBIAN, pf.PF_METHOD_YBUS),
       "jacobian_ew_csc": (pf.PF_OP_JACOBIAN, pf.PF_METHOD_ELEMENTWISE | pf.PF_JAC_CSC),
       "jacobian_ybus_csc": (pf.PF_OP_JACOBIAN, pf.PF_METHOD_YBUS | pf.PF_JAC_CSC),
       "vjp": (pf.PF_OP_VJP, pf.PF_METHOD_ELEMENTWISE)}


def synthetic_op(grid: "pf.Grid", op: str, nstate: int, seed: int = 0) -> dict:
    """``op`` on seeded synthetic device buffers (states v ~ 1 + U(-0.025,
    0.025), theta ~ N(0, 0.2), adjoint seeds ~ N(0, 1)), as a dict for
    pf_graph_create / pf_autotune."""
    import torch
    if op not in OPS:
        raise ValueError(f"unknown op {op!r}")
    dev = torch.device("cuda", torch.cuda.current_device())
    g = torch.Generator(device="cpu").manual_seed(seed)
    shape = (nstate, grid.nb)
    vm = (1.0 + 0.05 * (torch.rand(shape, generator=g, dtype=torch.float64) - 0.5)).to(dev)
    va = (0.2 * torch.randn(shape, generator=g, dtype=torch.float64)).to(dev)
    o, m = _OP[op]
    d = dict(op=o, method=m, vm=vm, va=va, out_a=torch.empty_like(vm), out_b=torch.empty_like(vm))
    if o == pf.PF_OP_VJP:
        d["lam_p"] = torch.randn(shape, generator=g, dtype=torch.float64).to(dev)
        d["lam_q"] = torch.randn(shape, generator=g, dtype=torch.float64).to(dev)
    if o == pf.PF_OP_JACOBIAN:
        d["jval"] = torch.empty((nstate, grid.nnz_j), dtype=torch.float64, device=dev)
    return d


def tune(grid: "pf.Grid", op: str, nstate: int, *, cache: Optional[ScheduleCache] = None,
         measure: Optional[Callable[[Schedule], float]] = None, cands: Optional[Iterable[Schedule]] = None,
         device: Optional[str] = None, lib: Optional[str] = None, save: bool = True) -> dict:
    """Time every candidate schedule, keep the fastest on ``grid`` and record
    it in the cache.  Returns {"schedule", "us", "tried", "key"}.  By default
    the library's native tuner (pf_autotune) times the candidates on seeded
    synthetic states (:func:`synthetic_op`); ``measure(schedule) -> seconds``
    replaces it (host-side tests)."""
    cache = cache if cache is not None else ScheduleCache()
    device = device if device is not None else _device_name()
    lib = lib if lib is not None else library_id()
    key = problem_key(grid, op, nstate, device, lib)
    cands = list(cands) if cands is not None else candidates(nstate)
    if not cands:
        raise ValueError("no candidate schedules")
    if measure is None:
        best, best_us, tried = pf.pf_autotune(grid, synthetic_op(grid, op, nstate), cands)
    else:
        best, best_t = None, float("inf")
        for c in cands:
            t = measure(c)
            if t < best_t:
                best, best_t = c, t
        grid.set_schedule(*best)
        best_us, tried = best_t * 1e6, len(cands)
    cache.put(key, best, best_us, tried)
    if save:
        cache.save()
    return {"schedule": tuple(best), "us": best_us, "tried": tried, "key": key}


def apply(grid: "pf.Grid", op: str, nstate: int, *, cache: Optional[ScheduleCache] = None,
          device: Optional[str] = None, lib: Optional[str] = None) -> Optional[Schedule]:
    """Set the cached schedule for (grid shape, op, nstate) if there is one;
    returns it, or None (the handle keeps its schedule)."""
    cache = cache if cache is not None else ScheduleCache()
    device = device if device is not None else _device_name()
    lib = lib if lib is not None else library_id()
    sched = cache.get(problem_key(grid, op, nstate, device, lib))
    if sched is not None:
        grid.set_schedule(*sched)
    return sched
