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
import time
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
    each in both work orders."""
    if nstate <= 1:
        return [(t, 1, pf.PF_ORDER_TILE_MAJOR) for t in tiles]
    spbs = [0] + [s for s in STATES_PER_BLOCK if s <= nstate]
    return [(t, s, o) for t in tiles for s in spbs for o in (pf.PF_ORDER_TILE_MAJOR, pf.PF_ORDER_STATE_MAJOR)]


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


def device_timer(grid: "pf.Grid", op: str, nstate: int, reps: int = 5, seed: int = 0,
                 warm_s: float = 0.01, samples: int = 3) -> Callable[[Schedule], float]:
    """Seconds per call of ``op`` on synthetic states under a given schedule,
    measured with HIP events around a replayed graph of ``reps`` calls (so
    the host cost of a call does not hide differences): the median of
    ``samples`` timed replays, after untimed replays for ``warm_s`` seconds
    (a tile-size change rebuilds the tables on the host, and the device runs
    slower for the first milliseconds after idling)."""
    import torch
    if op not in OPS:
        raise ValueError(f"unknown op {op!r}")
    dev = torch.device("cuda", torch.cuda.current_device())
    g = torch.Generator(device="cpu").manual_seed(seed)
    shape = (nstate, grid.nb)
    vm = (1.0 + 0.05 * (torch.rand(shape, generator=g, dtype=torch.float64) - 0.5)).to(dev)
    va = (0.2 * torch.randn(shape, generator=g, dtype=torch.float64)).to(dev)
    lp = torch.randn(shape, generator=g, dtype=torch.float64).to(dev)
    lq = torch.randn(shape, generator=g, dtype=torch.float64).to(dev)
    a, b = torch.empty_like(vm), torch.empty_like(vm)
    j = torch.empty((nstate, grid.nnz_j), dtype=torch.float64, device=dev) if op.startswith("jacobian") else None
    side = torch.cuda.Stream()

    def call(st):
        if op == "injections_ew":
            pf.pf_injections_elementwise(grid, vm, va, a, b, stream=st)
        elif op == "injections_ybus":
            pf.pf_injections_ybus(grid, vm, va, a, b, stream=st)
        elif op == "jacobian_ew":
            pf.pf_jacobian_values(grid, pf.PF_METHOD_ELEMENTWISE, vm, va, a, b, j, stream=st)
        elif op == "jacobian_ybus":
            pf.pf_jacobian_values(grid, pf.PF_METHOD_YBUS, vm, va, a, b, j, stream=st)
        elif op == "jacobian_ew_csc":
            pf.pf_jacobian_values(grid, pf.PF_METHOD_ELEMENTWISE | pf.PF_JAC_CSC, vm, va, a, b, j, stream=st)
        elif op == "jacobian_ybus_csc":
            pf.pf_jacobian_values(grid, pf.PF_METHOD_YBUS | pf.PF_JAC_CSC, vm, va, a, b, j, stream=st)
        else:
            pf.pf_injections_vjp(grid, vm, va, lp, lq, a, b, stream=st)

    def measure(sched: Schedule) -> float:
        grid.set_schedule(*sched)
        with torch.cuda.stream(side):
            call(side)
        torch.cuda.synchronize()
        gr = torch.cuda.CUDAGraph()
        with torch.cuda.graph(gr, stream=side):
            for _ in range(reps):
                call(side)
        torch.cuda.synchronize()
        tw = time.perf_counter()
        while True:
            with torch.cuda.stream(side):
                gr.replay()
            torch.cuda.synchronize()
            if time.perf_counter() - tw >= warm_s:
                break
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        ts = []
        for _ in range(max(1, samples)):
            with torch.cuda.stream(side):
                e0.record(side)
                gr.replay()
                e1.record(side)
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1) / 1e3 / reps)
        return sorted(ts)[len(ts) // 2]

    return measure


def tune(grid: "pf.Grid", op: str, nstate: int, *, cache: Optional[ScheduleCache] = None,
         measure: Optional[Callable[[Schedule], float]] = None, cands: Optional[Iterable[Schedule]] = None,
         device: Optional[str] = None, lib: Optional[str] = None, save: bool = True) -> dict:
    """Time every candidate schedule, keep the fastest on ``grid`` and record
    it in the cache.  Returns {"schedule", "us", "tried", "key"}.
    ``measure(schedule) -> seconds`` defaults to :func:`device_timer`."""
    cache = cache if cache is not None else ScheduleCache()
    device = device if device is not None else _device_name()
    lib = lib if lib is not None else library_id()
    key = problem_key(grid, op, nstate, device, lib)
    cands = list(cands) if cands is not None else candidates(nstate)
    if not cands:
        raise ValueError("no candidate schedules")
    measure = measure if measure is not None else device_timer(grid, op, nstate)
    best, best_t = None, float("inf")
    for c in cands:
        t = measure(c)
        if t < best_t:
            best, best_t = c, t
    grid.set_schedule(*best)
    cache.put(key, best, best_t * 1e6, len(cands))
    if save:
        cache.save()
    return {"schedule": best, "us": best_t * 1e6, "tried": len(cands), "key": key}


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
