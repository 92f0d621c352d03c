"""Benchmark: injection + Jacobian evaluations per second at 100k buses.

One step = one evaluation of S = P + jQ and all Jacobian values of a
100,000-bus, 130,000-branch synthetic grid (one voltage state) by the
element-wise method: one kernel launch.  To keep every step cold in the
256 MB Infinity Cache, steps rotate over R independent replicas of the
problem (grid data, state and outputs), R x 27 MB >= 512 MB.  Steps are
issued as replays of HIP graphs that record R consecutive launches: a
Python call costs about as much host time as the kernel takes, so one call
per step would measure the host.  The eager one-call-per-step rate is
reported beside it.

Printed (one JSON line): evals/s, the roofline of the dominant kernel
(algorithmic bytes per launch / average launch time, HIP events on the
launch stream), the CPU oracle's rate on the host, and side measurements:
the Ybus method under the same protocol, warm-cache rates, a plain copy of
the same byte count (the practical bandwidth ceiling at this size), 512
batched states on a 20k-bus grid, 64 uneven grids x 4 states, and the
adjoint (32 states at 100k buses) against its forward pass, the Ybus
injections with a separate phasor step in split and interleaved storage
(Table I's comparison) against the fused kernel, the headline grid with its
buses renumbered at random and then by reverse Cuthill-McKee (locality of
the remote-bus gathers), and a Newton-Raphson power flow on a 5000-bus grid
(device evaluation against host sparse solve per iteration).

Counter runs (HBM traffic of the dominant kernel):
    rocprofv3 --pmc FETCH_SIZE --output-format csv -d D1 -o f -- python3 bench.py --probe
    rocprofv3 --pmc WRITE_SIZE --output-format csv -d D2 -o w -- python3 bench.py --probe
    python3 bench.py --traffic D1/.../f_counter_collection.csv D2/.../w_counter_collection.csv
The probe runs the headline launches, as many Ybus S+J launches (their own
traffic figure) and one plain copy of a known byte count; each counter is
scaled by known bytes / counted bytes of that copy.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s
WARM_S = 0.05  # untimed replays before every timed region, seconds
# sources that decide the headline kernel's memory traffic (kernels and lane-table layout)
KERNEL_SRCS = [os.path.join(ROOT, "paper_2302_10736_amd", "csrc", f)
               for f in ("pf_kernels.hip", "pf_math.h", "pf_internal.h", "pf_api.cpp")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_ew_100k_1state_traffic.json")
HEADLINE_KERNEL = "k_ew<256, false, true, true, false>"  # element-wise S+J, one state per workgroup
COPY_PROBE_DOUBLES = 4 * 1024 * 1024  # 32 MiB read + 32 MiB written by the calibration copy


def kernel_hash():
    h = hashlib.sha256()
    for f in KERNEL_SRCS:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def traffic_from_csv(fetch_csv, write_csv):
    """Per-launch HBM bytes of the headline kernel from two rocprofv3 counter
    CSVs (FETCH_SIZE, WRITE_SIZE in KiB per dispatch), each scaled by the
    known bytes of the probe's copy kernel over what the counter read for it."""
    import csv

    def per_kernel(path, counter):
        acc = {}
        with open(path) as f:
            for row in csv.DictReader(f):
                if row.get("Counter_Name") != counter:
                    continue
                name = row["Kernel_Name"]
                key = (name, row.get("Dispatch_Id", row.get("Correlation_Id")))
                acc[key] = acc.get(key, 0.0) + float(row["Counter_Value"])
        out = {}
        for (name, _), v in acc.items():
            out.setdefault(name, []).append(v)
        return out

    def pick(d, pred, what):
        names = [n for n in d if pred(n)]
        if len(names) != 1:
            raise SystemExit(f"expected one {what} kernel in the counter file, found {names}")
        vals = d[names[0]]
        return names[0], sum(vals) / len(vals), len(vals)

    head = lambda n: "k_ew<256, false, true, true, false>" in n
    copy = lambda n: "copy" in n.lower() and "k_ew" not in n
    res = {"kernel": HEADLINE_KERNEL, "kernel_sha256_16": kernel_hash(), "copy_bytes_each_way": 8 * COPY_PROBE_DOUBLES}
    total = 0.0
    for counter, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        d = per_kernel(path, counter)
        hn, hv, hc = pick(d, head, "headline")
        # the calibration copy is by far the largest copy dispatch (state clones are 0.8 MB)
        cn = [n for n in d if copy(n)]
        if not cn:
            raise SystemExit("no copy kernel in the counter file")
        cn, cv = max(((n, max(d[n])) for n in cn), key=lambda t: t[1])
        factor = 8 * COPY_PROBE_DOUBLES / (cv * 1024.0)
        res[counter] = {"headline_kib_per_dispatch": hv, "dispatches": hc, "copy_kernel": cn,
                        "copy_kib": cv, "scale": factor, "bytes_per_launch": hv * 1024.0 * factor}
        total += hv * 1024.0 * factor
    res["bytes_per_launch"] = total
    return res


def recorded_traffic(path=TRAFFIC_FILE):
    """Counter-measured HBM bytes per launch of the headline kernel from the
    file `--traffic` wrote, or None when there is none or it was taken for
    other kernel sources (its hash differs from kernel_hash())."""
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("kernel_sha256_16") != kernel_hash():
        return None
    return t.get("bytes_per_launch")


def algorithmic_bytes(nb, nl, nnz_y, nstate, with_j=True, method="ew", vjp=False):
    """Bytes the method must move: state in/out, problem data once, outputs.

    element-wise S+J: B (16 nb [vm, va] + 16 nb [P, Q] + 8 nnzJ) + 48 nl [from, to,
    r, x, b, tap, shift] + 16 nb [shunts] + 4 (nb + 1) [row pointer];
    Ybus S+J: B (32 nb + 8 nnzJ) + 20 nnzY [column + complex value] + 4 (nb + 1);
    adjoint: B (32 nb in + 16 nb out) + grid data."""
    nnz_j = 4 * nnz_y
    per_state = 32 * nb + (8 * nnz_j if with_j else 0)
    if vjp:
        per_state = 48 * nb
    if method == "ybus":
        grid = 20 * nnz_y + 4 * (nb + 1)
    else:
        grid = 48 * nl + 16 * nb + 4 * (nb + 1)
    return nstate * per_state + grid


def make_timer(torch, side):
    """timed(fn, steps, warmup, period): time exactly `steps` launches
    fn(k, stream), issued as replays of HIP graphs that record `period`
    consecutive launches (plus one graph for the remainder), so the host cost
    of a call does not bound the rate.  Returns (seconds by HIP events on the
    launch stream around exactly those launches, wall seconds of the same
    region including the host's graph launches and the final synchronise)."""

    def timed(fn, steps, warmup, period):
        period = max(1, min(period, steps))
        with torch.cuda.stream(side):
            for k in range(max(warmup, period)):
                fn(k, side)
        torch.cuda.synchronize()

        def record(n):
            gr = torch.cuda.CUDAGraph()
            with torch.cuda.graph(gr, stream=side):
                for k in range(n):
                    fn(k, side)
            return gr
        full, rest = divmod(steps, period)
        g_full = record(period) if full else None
        g_rest = record(rest) if rest else None
        # Untimed replays for at least WARM_S seconds: after host work (grid
        # builds, schedule changes) the device has idled, and the first
        # milliseconds of work after that run measurably slower.
        tw = time.perf_counter()
        while True:
            with torch.cuda.stream(side):
                for _ in range(2):
                    (g_full or g_rest).replay()
            torch.cuda.synchronize()
            if time.perf_counter() - tw >= WARM_S:
                break
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        with torch.cuda.stream(side):
            e0.record(side)
            for _ in range(full):
                g_full.replay()
            if g_rest is not None:
                g_rest.replay()
            e1.record(side)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        return e0.elapsed_time(e1) / 1e3, wall

    return timed


SWEEP_SIZES = (118, 10_000, 82_000, 164_000, 410_000)  # the default run's sweep
SWEEP_SIZES_FULL = (118, 500, 2_000, 10_000, 30_000, 82_000, 164_000, 246_000, 328_000, 410_000)
COLD_BYTES = 512 << 20  # replicas of at least twice the 256 MB Infinity Cache per timed size


def size_sweep(torch, gridgen, pf, timed, log, sizes=SWEEP_SIZES, cold_from=82_000):
    """Device time of one evaluation (one state) by both methods, injections
    alone and with the Jacobian, over grid sizes from 118 buses to five
    replicas of an 82k-bus grid (the paper's Section V.C question, Tables VI
    and IX-X and the time-cost-ratio figure).  Grids of the same generator
    (nl = 1.27 nb, 15 % transformers); sizes above 82k are 2-5 disjoint copies
    of the 82k-bus grid in one handle, as the paper replicates its 82k case.
    From `cold_from` buses on, each timing rotates over R independent replicas
    (grid tables, state, outputs) totalling at least 512 MB, so every launch
    reads cold data from HBM; smaller grids fit the caches whatever is done
    and run warm.  Per size: microseconds per evaluation, nanoseconds per bus,
    the time-cost ratio (per-bus time over that of the 118-bus grid) and the
    Ybus / element-wise time ratio."""
    dev = torch.device("cuda:0")
    base82 = None
    rows = []
    for nb in sizes:
        if nb <= 82_000:
            g = gridgen.make_grid(nb, round(1.27 * nb), 0.15, case=5, grid=nb)
            if nb == 82_000:
                base82 = g
        else:
            if base82 is None:
                base82 = gridgen.make_grid(82_000, round(1.27 * 82_000), 0.15, case=5, grid=82_000)
            g, bo, ro = gridgen.concat([base82] * (nb // 82_000))
        offs = (bo, ro) if nb > 82_000 else (None, None)  # copies are separate grids of one handle
        vm, va = gridgen.states(g.nb, 1, case=5, grid=nb)
        G0 = pf.Grid.from_grid(g, *offs)
        per_rep = algorithmic_bytes(g.nb, g.nl, G0.nnz_y, 1) + 24 * 2 * g.nl  # + lane tables beyond branch data
        R = max(1, -(-COLD_BYTES // per_rep)) if nb >= cold_from else 1
        reps = []
        for r in range(R):
            G = G0 if r == 0 else pf.Grid.from_grid(g, *offs)
            pf.pf_ybus(G)
            reps.append((G, torch.as_tensor(vm, device=dev).clone(), torch.as_tensor(va, device=dev).clone(),
                         torch.empty(1, g.nb, dtype=torch.float64, device=dev),
                         torch.empty(1, g.nb, dtype=torch.float64, device=dev),
                         torch.empty(1, G.nnz_j, dtype=torch.float64, device=dev)))
        torch.cuda.synchronize()
        n = max(2 * R, 40)

        def t_us(fn):  # one graph of all n launches, rotating over the R replicas
            ev, _ = timed(fn, n, R, n)
            return ev / n * 1e6
        t = {
            "ew_s": t_us(lambda k, st: pf.pf_injections_elementwise(reps[k % R][0], *reps[k % R][1:5], stream=st)),
            "ew_sj": t_us(lambda k, st: pf.pf_jacobian_values(reps[k % R][0], pf.PF_METHOD_ELEMENTWISE,
                                                              *reps[k % R][1:], stream=st)),
            "ybus_s": t_us(lambda k, st: pf.pf_injections_ybus(reps[k % R][0], *reps[k % R][1:5], stream=st)),
            "ybus_sj": t_us(lambda k, st: pf.pf_jacobian_values(reps[k % R][0], pf.PF_METHOD_YBUS,
                                                                *reps[k % R][1:], stream=st)),
        }
        rows.append({"buses": g.nb, "branches": g.nl, "replicas_of_82k": nb // 82_000 if nb > 82_000 else None,
                     "cold_replicas": R, "us": t, "ns_per_bus": {k: 1e3 * v / g.nb for k, v in t.items()},
                     "ybus_over_ew": {"s": t["ybus_s"] / t["ew_s"], "sj": t["ybus_sj"] / t["ew_sj"]}})
        log(f"{g.nb:>8d} buses ({R} replicas): " + ", ".join(f"{k} {v:.2f} us" for k, v in t.items()))
        del reps, G0
        torch.cuda.empty_cache()
    ref = rows[0]["ns_per_bus"]
    for r in rows:
        r["time_cost_ratio_vs_118"] = {k: r["ns_per_bus"][k] / ref[k] for k in ref}
    return {"protocol": f"one state per evaluation, device time by HIP events over graph replays; from "
                        f"{cold_from} buses on, rotation over replicas of >= 512 MB (cold), smaller grids warm",
            "rows": rows}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--replicas", type=int, default=24)
    ap.add_argument("--no-extra", action="store_true", help="only the headline measurement")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-tune", action="store_true", help="keep the automatic schedules (skip the autotuner)")
    ap.add_argument("--sweep", action="store_true",
                    help="grid-size sweep instead of the benchmark: EW and Ybus per-bus times and time-cost ratios")
    ap.add_argument("--only", default="", help="comma list of side measurements to run")
    ap.add_argument("--probe", action="store_true",
                    help="counter-run workload: headline launches, then one copy of known size; no timing")
    ap.add_argument("--probe-batched", action="store_true",
                    help="counter-run workload: 3 batched S+J launches (20k buses x 512 states), 3 injection, "
                         "3 adjoint and 3 S+J launches (100k buses x 32 states), then one copy of known size; "
                         "no timing")
    ap.add_argument("--traffic", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write the headline kernel's HBM traffic from two counter CSVs and exit")
    args = ap.parse_args()
    if args.traffic:
        res = traffic_from_csv(*args.traffic)
        with open(TRAFFIC_FILE, "w") as f:
            json.dump(res, f, indent=1)
        print(json.dumps(res))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the library runs on a single "
              "MI355X and has no multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import torch

    import tempfile

    from paper_2302_10736_amd import autotune, gridgen, pf

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    log = lambda *a: print(*a, file=sys.stderr, flush=True)
    if args.sweep:
        timer = make_timer(torch, torch.cuda.Stream())
        print(json.dumps(size_sweep(torch, gridgen, pf, timer, log, SWEEP_SIZES_FULL)), flush=True)
        return

    if args.probe_batched:
        g2 = gridgen.grid_20k()
        vm2, va2 = gridgen.states(g2.nb, 512, case=2, vlo=0.9, vhi=1.1, sigma=0.3)
        G2 = pf.Grid.from_grid(g2)
        v2, a2 = torch.as_tensor(vm2, device=dev), torch.as_tensor(va2, device=dev)
        p2, q2 = torch.empty_like(v2), torch.empty_like(v2)
        j2 = torch.empty(512, G2.nnz_j, dtype=torch.float64, device=dev)
        for _ in range(3):
            pf.pf_jacobian_values(G2, pf.PF_METHOD_ELEMENTWISE, v2, a2, p2, q2, j2)
        torch.cuda.synchronize()
        del j2, G2
        g4 = gridgen.grid_100k()
        vm4, va4 = gridgen.states(g4.nb, 32, case=4)
        lp4, lq4 = gridgen.adjoint_seeds(g4.nb, 32, case=4)
        G4 = pf.Grid.from_grid(g4)
        v4, a4, l4p, l4q = (torch.as_tensor(x, device=dev) for x in (vm4, va4, lp4, lq4))
        o = [torch.empty_like(v4) for _ in range(4)]
        for _ in range(3):
            pf.pf_injections_elementwise(G4, v4, a4, o[0], o[1])
        for _ in range(3):
            pf.pf_injections_vjp(G4, v4, a4, l4p, l4q, o[2], o[3])
        j4 = torch.empty(32, G4.nnz_j, dtype=torch.float64, device=dev)
        for _ in range(3):
            pf.pf_jacobian_values(G4, pf.PF_METHOD_ELEMENTWISE, v4, a4, o[0], o[1], j4)
        torch.cuda.synchronize()
        del j4
        a = torch.ones(COPY_PROBE_DOUBLES, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log("probe done: 3 launches each of 20k x 512 S+J, 100k x 32 injections, adjoint and S+J; one copy of "
            f"{8 * COPY_PROBE_DOUBLES} bytes")
        return

    # ------------------------------------------------------------ workload
    g = gridgen.grid_100k()
    vm, va = gridgen.states(g.nb, 1, case=1)
    R = max(1, args.replicas)
    reps = []
    for r in range(R):
        G = pf.Grid.from_grid(g)
        reps.append(dict(
            G=G,
            vm=torch.as_tensor(vm, device=dev).clone(), va=torch.as_tensor(va, device=dev).clone(),
            p=torch.empty(1, g.nb, dtype=torch.float64, device=dev),
            q=torch.empty(1, g.nb, dtype=torch.float64, device=dev),
            j=torch.empty(1, G.nnz_j, dtype=torch.float64, device=dev)))
    G0 = reps[0]["G"]
    nnz_y, nnz_j = G0.nnz_y, G0.nnz_j
    # schedules come from the autotuner, tuned afresh (a private cache file)
    tune_cache = autotune.ScheduleCache(os.path.join(tempfile.mkdtemp(prefix="pf_bench_"), "schedules.json"))
    # The headline keeps the default schedule (256-lane tiles, one state per
    # workgroup), the one the counter probe and the kernel trace also run;
    # tile sizes 128-512 are within noise of it on cold data.
    tuned = {}
    tile, spb, order, ntiles = G0.schedule()
    log(f"grid nb={g.nb} nl={g.nl} nnzY={nnz_y} nnzJ={nnz_j} tiles={ntiles} replicas={R}")

    side = torch.cuda.Stream()  # the launch stream (default priority)

    timer = make_timer(torch, side)

    def timed(fn, steps, warmup, period=R):
        return timer(fn, steps, warmup, period)

    def eager_timed(fn, steps, warmup):
        """The same launches issued one Python call at a time (host-bound)."""
        for k in range(warmup):
            fn(k, side)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(steps):
            fn(k, side)
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    def ew_sj(k, st=None):
        d = reps[k % R]
        pf.pf_jacobian_values(d["G"], pf.PF_METHOD_ELEMENTWISE, d["vm"], d["va"], d["p"], d["q"], d["j"], stream=st)

    if args.probe:
        for k in range(2 * R):
            ew_sj(k)
        # the Ybus kernel on the same replicas, for its own traffic figure
        for d in reps:
            pf.pf_ybus(d["G"])
        torch.cuda.synchronize()
        for k in range(2 * R):
            d = reps[k % R]
            pf.pf_jacobian_values(d["G"], pf.PF_METHOD_YBUS, d["vm"], d["va"], d["p"], d["q"], d["j"])
        a = torch.ones(COPY_PROBE_DOUBLES, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"probe done: {2 * R} headline launches, {2 * R} Ybus S+J launches, one copy of "
            f"{8 * COPY_PROBE_DOUBLES} bytes")
        return

    K, W = args.steps, args.warmup
    ev_s, wall_s = timed(ew_sj, K, W)
    # value, ms_per_step and the roofline all come from this one event timing
    # of exactly K launches (device time; the wall clock of the same region
    # adds the host's graph launch and synchronise, reported beside it)
    value = K / ev_s
    avg_launch = ev_s / K
    rotated = min(R, K)
    abytes = algorithmic_bytes(g.nb, g.nl, nnz_y, 1)
    achieved = abytes / avg_launch / 1e9
    log(f"element-wise S+J: {avg_launch * 1e6:.2f} us/launch, {value:.0f} evals/s (events); "
        f"wall {wall_s / K * 1e6:.2f} us/step")

    # traffic measured by rocprofv3 counters for this exact kernel source, if recorded
    traffic = recorded_traffic()

    out = {
        "metric": "S+Jacobian evals/s at 100k buses, % HBM peak; batched & adjoint vs plain",
        "value": value,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": ev_s / K * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded generator standing in for the paper's MATPOWER cases)",
        "config": {"workload": "100k-bus grid (nb=100000, nl=130000, 20% transformers), 1 voltage state, "
                               "element-wise S + full polar Jacobian, one launch per step, steps issued as "
                               f"HIP-graph replays rotating over {rotated} cold replicas",
                   "nb": g.nb, "nl": g.nl, "nnz_y": nnz_y, "nnz_j": nnz_j, "states": 1,
                   "replicas_rotated": rotated, "replica_bytes": rotated * (abytes + 48 * g.nl),
                   "tile_items": tile, "timing": "HIP events on the launch stream around exactly `steps` launches",
                   "wall_ms_per_step": wall_s / K * 1e3},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": f"k_ew<{tile}, false, true, true, false>", "algorithmic_bytes_per_launch": abytes,
                     "avg_launch_us": avg_launch * 1e6},
    }

    extra = {}
    only = set(filter(None, args.only.split(",")))
    want = (lambda name: not args.no_extra and (not only or name in only))

    if want("repeats"):
        # spread of the headline launch time: 20 repetitions of 10 x 24 launches
        rep_us = []
        for _ in range(20):
            e, _ = timed(ew_sj, 10 * R, R)
            rep_us.append(e / (10 * R) * 1e6)
        q = np.percentile(rep_us, [10, 50, 90])
        extra["headline_repeats"] = {"repeats": 20, "launches_each": 10 * R, "p10_us": q[0], "median_us": q[1],
                                     "p90_us": q[2]}
        # the same launch over long replay windows, beside the timed steps' figure
        out["roofline"]["median_launch_us"] = q[1]
        out["roofline"]["frac_at_median"] = abytes / (q[1] * 1e-6) / 1e9 / HBM_PEAK_GBS
        log(f"headline repeats: p10 {q[0]:.2f} median {q[1]:.2f} p90 {q[2]:.2f} us")

    if want("ybus"):
        for d in reps:
            pf.pf_ybus(d["G"])
        torch.cuda.synchronize()

        def yb_sj(k, st):
            d = reps[k % R]
            pf.pf_jacobian_values(d["G"], pf.PF_METHOD_YBUS, d["vm"], d["va"], d["p"], d["q"], d["j"], stream=st)
        ev, wall = timed(yb_sj, K, W)
        yb_bytes = algorithmic_bytes(g.nb, g.nl, nnz_y, 1, method="ybus")
        extra["ybus_sj"] = {"evals_per_s": K / ev, "avg_launch_us": ev / K * 1e6,
                            "achieved_GBs": yb_bytes / (ev / K) / 1e9, "algorithmic_bytes": yb_bytes,
                            "ew_speedup_vs_ybus": (ev / K) / avg_launch}
        log(f"Ybus S+J: {ev / K * 1e6:.2f} us/launch")

    if want("two_phase"):
        # the paper's two-step structure: branch evaluation into scratch, then the bus reduction
        def tp_sj(k, st):
            d = reps[k % R]
            pf.pf_jacobian_values(d["G"], pf.PF_METHOD_ELEMENTWISE_TWO_PHASE, d["vm"], d["va"], d["p"], d["q"], d["j"],
                                  stream=st)
        ev, wall = timed(tp_sj, K, W)

        def tp_pre(k, st):
            d = reps[k % R]
            pf.pf_jacobian_values(d["G"], pf.PF_METHOD_ELEMENTWISE_TWO_PHASE | pf.PF_EW_PRECOMPUTED, d["vm"], d["va"],
                                  d["p"], d["q"], d["j"], stream=st)
        ev_pre, _ = timed(tp_pre, K, W)
        extra["ew_two_phase_sj"] = {"evals_per_s": K / ev, "avg_eval_us": ev / K * 1e6,
                                    "achieved_GBs": abytes / (ev / K) / 1e9, "launches_per_eval": 2,
                                    "fused_speedup": (ev / K) / avg_launch,
                                    "precomputed_constants_us": ev_pre / K * 1e6}
        log(f"two-phase S+J: {ev / K * 1e6:.2f} us/eval (precomputed constants {ev_pre / K * 1e6:.2f})")

    if want("copy_add"):
        # copy-add with atomic adds: zero J, shunt terms, one thread per branch adding both ends
        def ca_sj(k, st):
            d = reps[k % R]
            pf.pf_jacobian_values(d["G"], pf.PF_METHOD_ELEMENTWISE_ATOMIC, d["vm"], d["va"], d["p"], d["q"], d["j"],
                                  stream=st)
        ev, wall = timed(ca_sj, K, W)

        def ca_pre(k, st):
            d = reps[k % R]
            pf.pf_jacobian_values(d["G"], pf.PF_METHOD_ELEMENTWISE_ATOMIC | pf.PF_EW_PRECOMPUTED, d["vm"], d["va"],
                                  d["p"], d["q"], d["j"], stream=st)
        ev_pre, _ = timed(ca_pre, K, W)
        extra["ew_copy_add_atomic_sj"] = {"evals_per_s": K / ev, "avg_eval_us": ev / K * 1e6,
                                          "achieved_GBs": abytes / (ev / K) / 1e9, "launches_per_eval": 3,
                                          "fused_speedup": (ev / K) / avg_launch,
                                          "precomputed_constants_us": ev_pre / K * 1e6}
        log(f"copy-add (atomic) S+J: {ev / K * 1e6:.2f} us/eval (precomputed constants {ev_pre / K * 1e6:.2f})")

    if want("csc"):
        # the same evaluation with J written in CSC order (what sparse direct solvers take)
        def ew_csc(k, st):
            d = reps[k % R]
            pf.pf_jacobian_values(d["G"], pf.PF_METHOD_ELEMENTWISE | pf.PF_JAC_CSC, d["vm"], d["va"], d["p"], d["q"],
                                  d["j"], stream=st)
        ev, wall = timed(ew_csc, K, W)
        cb = abytes + 32 * g.nl  # + the opposite end's coupling, 16 B per branch end (lane table)
        extra["ew_sj_csc"] = {"evals_per_s": K / ev, "avg_launch_us": ev / K * 1e6,
                              "achieved_GBs": abytes / (ev / K) / 1e9, "over_csr_time": (ev / K) / avg_launch,
                              "kernel": f"k_ew_csc<{tile}, false, true>", "bytes_read_extra": cb - abytes}
        log(f"element-wise S+J, CSC order: {ev / K * 1e6:.2f} us/launch")
        for d in reps:
            pf.pf_ybus(d["G"])
        torch.cuda.synchronize()

        def yb_csc(k, st):
            d = reps[k % R]
            pf.pf_jacobian_values(d["G"], pf.PF_METHOD_YBUS | pf.PF_JAC_CSC, d["vm"], d["va"], d["p"], d["q"], d["j"],
                                  stream=st)
        ev, wall = timed(yb_csc, K, W)
        extra["ybus_sj_csc"] = {"evals_per_s": K / ev, "avg_launch_us": ev / K * 1e6,
                                "kernel": f"k_ybus_csc<{tile}, true>"}
        log(f"Ybus S+J, CSC order: {ev / K * 1e6:.2f} us/launch")

    if want("scatter"):
        # Algorithm 2's in-place copy into a larger pattern: J's entries plus the couplings of
        # 1000 series devices between random bus pairs (all four blocks), CSR
        _, _, jr0, jc0 = G0.pattern()
        rows0 = np.repeat(np.arange(2 * g.nb, dtype=np.int64), np.diff(jr0))
        rng_s = np.random.default_rng(17)
        pr = rng_s.integers(0, g.nb, (1000, 2))
        ex_r, ex_c = [], []
        for a, b in ((0, 1), (1, 0)):
            for rb in (0, g.nb):
                for cb in (0, g.nb):
                    ex_r.append(pr[:, a] + rb)
                    ex_c.append(pr[:, b] + cb)
        key = np.unique(np.concatenate([rows0 * (2 * g.nb) + jc0] +
                                       [r * (2 * g.nb) + c for r, c in zip(ex_r, ex_c)]))
        t_rows, t_cols = key // (2 * g.nb), (key % (2 * g.nb)).astype(np.int32)
        t_ptr = np.zeros(2 * g.nb + 1, np.int64)
        np.add.at(t_ptr, t_rows + 1, 1)
        t_ptr = np.cumsum(t_ptr).astype(np.int32)
        t0 = time.perf_counter()
        jmap = pf.pf_jacobian_map(G0, pf.PF_LAYOUT_CSR, t_ptr, t_cols)
        map_s = time.perf_counter() - t0
        jmap_d = torch.as_tensor(jmap, device=dev)
        outs = [torch.zeros(1, len(t_cols), dtype=torch.float64, device=dev) for _ in range(R)]

        def scat(k, st):
            d = reps[k % R]
            pf.pf_jacobian_scatter(d["G"], d["j"], jmap_d, outs[k % R], stream=st)
        ev, _ = timed(scat, K, W)
        sb = 20 * G0.nnz_j  # J read, map read, values written
        extra["jacobian_scatter_100k"] = {"avg_launch_us": ev / K * 1e6, "achieved_GBs": sb / (ev / K) / 1e9,
                                          "target_nnz": int(len(t_cols)), "map_host_s": map_s,
                                          "algorithmic_bytes": sb}
        del outs, jmap_d
        log(f"J scatter into a larger pattern: {ev / K * 1e6:.2f} us/launch (map on the host {map_s * 1e3:.0f} ms)")

    if want("flows"):
        # branch flows and their 16 partials (line-limit constraints), same grid and protocol
        for d in reps:
            d["fl"] = [torch.empty(1, g.nl, dtype=torch.float64, device=dev) for _ in range(4)]
            d["fj"] = torch.empty(1, 16, g.nl, dtype=torch.float64, device=dev)

        def flows(k, st):
            d = reps[k % R]
            pf.pf_branch_flows(d["G"], d["vm"], d["va"], *d["fl"], d["fj"], stream=st)
        ev, wall = timed(flows, K, W)
        fb = 48 * g.nl + 16 * g.nb + (32 + 128) * g.nl  # branch data + state in, flows + partials out
        extra["branch_flows_jac"] = {"evals_per_s": K / ev, "avg_launch_us": ev / K * 1e6,
                                     "achieved_GBs": fb / (ev / K) / 1e9, "algorithmic_bytes": fb}
        for d in reps:
            del d["fl"], d["fj"]
        log(f"branch flows + partials: {ev / K * 1e6:.2f} us/launch")

    if want("relabelled"):
        # the same grid with its buses renumbered at random (no locality in the
        # remote-bus gathers), same protocol: cold replicas, graph replays; and
        # the random numbering renumbered by reverse Cuthill-McKee on
        # the host (a standard fix a caller can apply before building)
        import scipy.sparse as sps
        from scipy.sparse.csgraph import reverse_cuthill_mckee
        gr_, perm_r = gridgen.relabel(g, case=1)
        adj = sps.coo_matrix((np.ones(g.nl), (gr_.fbus, gr_.tbus)), shape=(g.nb, g.nb)).tocsr()
        order = reverse_cuthill_mckee((adj + adj.T).tocsr(), symmetric_mode=True)
        perm_c = np.argsort(order)  # new number of each relabelled bus
        gc_ = gridgen.renumber(gr_, perm_c)
        res_r = {}
        for tag, gx, pfull in (("random", gr_, perm_r), ("rcm", gc_, perm_c[perm_r])):
            inv = np.argsort(pfull)
            reps_r = []
            for r in range(R):
                Gr = pf.Grid.from_grid(gx)
                pf.pf_ybus(Gr)
                reps_r.append((Gr, torch.as_tensor(vm[:, inv], device=dev).contiguous(),
                               torch.as_tensor(va[:, inv], device=dev).contiguous(),
                               torch.empty(1, g.nb, dtype=torch.float64, device=dev),
                               torch.empty(1, g.nb, dtype=torch.float64, device=dev),
                               torch.empty(1, Gr.nnz_j, dtype=torch.float64, device=dev)))
            for mname, m in (("ew_sj", pf.PF_METHOD_ELEMENTWISE), ("ybus_sj", pf.PF_METHOD_YBUS)):
                ev, wall = timed(lambda k, st, m=m: pf.pf_jacobian_values(reps_r[k % R][0], m, *reps_r[k % R][1:],
                                                                          stream=st), K, W)
                res_r[f"{tag}_{mname}_us"] = ev / K * 1e6
            res_r[f"{tag}_ew_sj_over_generator_numbering"] = res_r[f"{tag}_ew_sj_us"] / (avg_launch * 1e6)
            del reps_r
            torch.cuda.empty_cache()
        extra["relabelled_100k"] = res_r
        log(f"random bus numbering: element-wise S+J {res_r['random_ew_sj_us']:.2f} us, Ybus S+J "
            f"{res_r['random_ybus_sj_us']:.2f} us; after RCM renumbering {res_r['rcm_ew_sj_us']:.2f} / "
            f"{res_r['rcm_ybus_sj_us']:.2f} us")

    if want("copy"):
        # a plain device copy moving the same number of bytes (half read, half written)
        n = abytes // 16
        ca = [torch.ones(n, dtype=torch.float64, device=dev) for _ in range(R)]
        cb = [torch.empty(n, dtype=torch.float64, device=dev) for _ in range(R)]
        ev, wall = timed(lambda k, st: cb[k % R].copy_(ca[k % R]), K, W)
        extra["copy_same_bytes"] = {"bytes": 16 * n, "avg_launch_us": ev / K * 1e6,
                                    "GBs": 16 * n / (ev / K) / 1e9,
                                    "headline_over_copy_time": avg_launch / (ev / K)}
        # the library's streaming copy (16-byte loads, streaming stores): the
        # practical ceiling at this byte count
        evs, _ = timed(lambda k, st: pf.pf_stream_copy(ca[k % R], cb[k % R], stream=st), K, W)
        extra["stream_copy_same_bytes"] = {"bytes": 16 * n, "avg_launch_us": evs / K * 1e6,
                                           "GBs": 16 * n / (evs / K) / 1e9,
                                           "frac_hbm": 16 * n / (evs / K) / 1e9 / HBM_PEAK_GBS,
                                           "headline_over_stream_copy_time": avg_launch / (evs / K)}
        # the measured ceiling at this byte count, beside the 8 TB/s peak
        out["roofline"]["stream_copy_GBs"] = 16 * n / (evs / K) / 1e9
        out["roofline"]["frac_of_stream_copy"] = (evs / K) / avg_launch
        del ca, cb
        log(f"copy of the same bytes: {ev / K * 1e6:.2f} us (torch), {evs / K * 1e6:.2f} us (streaming copy)")

    if want("warm"):
        def ew_warm(k, st):
            d = reps[0]
            pf.pf_jacobian_values(d["G"], pf.PF_METHOD_ELEMENTWISE, d["vm"], d["va"], d["p"], d["q"], d["j"], stream=st)
        ev, wall = timed(ew_warm, K, W)
        extra["ew_sj_warm_cache"] = {"evals_per_s": K / ev, "avg_launch_us": ev / K * 1e6}
        wall = eager_timed(ew_sj, K, W)
        extra["ew_sj_eager_python_calls"] = {"evals_per_s": K / wall, "us_per_call": wall / K * 1e6,
                                             "note": "one binding call per step; bound by host time"}
        bound = [pf.bind(pf.pf_jacobian_values, d["G"], pf.PF_METHOD_ELEMENTWISE, d["vm"], d["va"], d["p"], d["q"],
                         d["j"], stream=side) for d in reps]
        wall = eager_timed(lambda k, st: bound[k % R](), K, W)
        extra["ew_sj_eager_bound_calls"] = {"evals_per_s": K / wall, "us_per_call": wall / K * 1e6,
                                            "note": "pf.bind: arguments marshalled once, one library call per step"}
        del bound

        def ew_s(k, st):
            d = reps[k % R]
            pf.pf_injections_elementwise(d["G"], d["vm"], d["va"], d["p"], d["q"], stream=st)
        ev, wall = timed(ew_s, K, W)
        extra["ew_s_only"] = {"evals_per_s": K / ev, "avg_launch_us": ev / K * 1e6,
                              "achieved_GBs": algorithmic_bytes(g.nb, g.nl, nnz_y, 1, with_j=False) / (ev / K) / 1e9}
        if "ybus_sj" in extra:
            def yb_s(k, st):
                d = reps[k % R]
                pf.pf_injections_ybus(d["G"], d["vm"], d["va"], d["p"], d["q"], stream=st)
            ev, wall = timed(yb_s, K, W)
            extra["ybus_s_only"] = {"evals_per_s": K / ev, "avg_launch_us": ev / K * 1e6}
        log("warm/S-only done")

    if want("phasor"):
        # Table I's comparison on the GPU: Ybus injections with the phasor step
        # separate (split or interleaved storage) against the fused kernel
        for d in reps:
            pf.pf_ybus(d["G"])
            d["ph"] = torch.empty(4 * g.nb, dtype=torch.float64, device=dev)
        torch.cuda.synchronize()

        def yb_fused_s(k, st):
            d = reps[k % R]
            pf.pf_injections_ybus(d["G"], d["vm"], d["va"], d["p"], d["q"], stream=st)
        ev, _ = timed(yb_fused_s, K, W)
        res = {"fused_on_the_fly": {"total_us": ev / K * 1e6}}
        for name, lay in (("split", pf.PF_PHASOR_SPLIT), ("interleaved", pf.PF_PHASOR_INTERLEAVED)):
            def ph_step(k, st, lay=lay):
                d = reps[k % R]
                pf.pf_phasors(d["G"], lay, d["vm"], d["va"], d["ph"], stream=st)

            def pw_step(k, st, lay=lay):
                d = reps[k % R]
                pf.pf_ybus_from_phasors(d["G"], lay, 1, d["ph"], d["p"], d["q"], stream=st)

            def both(k, st, lay=lay):
                ph_step(k, st, lay)
                pw_step(k, st, lay)

            def both_j(k, st, lay=lay):
                ph_step(k, st, lay)
                d = reps[k % R]
                pf.pf_ybus_from_phasors(d["G"], lay, 1, d["ph"], d["p"], d["q"], d["j"], stream=st)
            e_ph, _ = timed(ph_step, K, W)
            e_pw, _ = timed(pw_step, K, W)
            e_t, _ = timed(both, K, W)
            e_tj, _ = timed(both_j, K, W)
            res[name] = {"phasor_us": e_ph / K * 1e6, "power_us": e_pw / K * 1e6, "total_us": e_t / K * 1e6,
                         "total_with_jacobian_us": e_tj / K * 1e6}
        if "ybus_sj" in extra:
            res["fused_on_the_fly"]["total_with_jacobian_us"] = extra["ybus_sj"]["avg_launch_us"]
        extra["ybus_phasor_storage"] = res
        for d in reps:
            del d["ph"]
        log("phasor storage: " + ", ".join(f"{k} {v['total_us']:.2f} us" for k, v in res.items()))

    del reps
    torch.cuda.empty_cache()

    if want("batched"):
        g2 = gridgen.grid_20k()
        B = 512
        vm2, va2 = gridgen.states(g2.nb, B, case=2, vlo=0.9, vhi=1.1, sigma=0.3)
        G2 = pf.Grid.from_grid(g2)
        vm2d, va2d = torch.as_tensor(vm2, device=dev), torch.as_tensor(va2, device=dev)
        p2 = torch.empty(B, g2.nb, dtype=torch.float64, device=dev)
        q2 = torch.empty_like(p2)
        j2 = torch.empty(B, G2.nnz_j, dtype=torch.float64, device=dev)

        def b_sj(k, st):
            pf.pf_jacobian_values(G2, pf.PF_METHOD_ELEMENTWISE, vm2d, va2d, p2, q2, j2, stream=st)
        steps = max(20, K // 40)
        timed(b_sj, 10, 3, period=10)  # first launches on a fresh grid run slow; not counted
        ev_auto, _ = timed(b_sj, max(10, K // 100), 3, period=10)
        auto_sched = G2.schedule()
        if not args.no_tune:
            tuned["batched"] = autotune.tune(G2, "jacobian_ew", B, cache=tune_cache, save=False)
        ev, wall = timed(b_sj, steps, 5, period=10)
        bb = algorithmic_bytes(g2.nb, g2.nl, G2.nnz_y, B)
        extra["batched_20k_x512"] = {"state_evals_per_s": B * steps / ev, "avg_launch_us": ev / steps * 1e6,
                                     "achieved_GBs": bb / (ev / steps) / 1e9,
                                     "frac_hbm": bb / (ev / steps) / 1e9 / HBM_PEAK_GBS,
                                     "algorithmic_bytes": bb, "schedule": G2.schedule(),
                                     "automatic_schedule": auto_sched,
                                     "automatic_schedule_us": ev_auto / max(10, K // 100) * 1e6}
        log(f"batched: {ev / steps * 1e6:.1f} us/launch")
        # the same launch recorded by the library's own graph API (pf_graph_create / pf_graph_launch)
        pgr = pf.Graph(G2, [dict(op=pf.PF_OP_JACOBIAN, method=pf.PF_METHOD_ELEMENTWISE, vm=vm2d, va=va2d, out_a=p2,
                                 out_b=q2, jval=j2)])
        tw = time.perf_counter()
        while time.perf_counter() - tw < WARM_S:  # untimed launches first, as in timed()
            pgr.launch(stream=side)
            torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(side)
        for _ in range(steps):  # one host call per launch; the device time dominates
            pgr.launch(stream=side)
        e1.record(side)
        torch.cuda.synchronize()
        extra["batched_20k_x512"]["pf_graph_launch_us"] = e0.elapsed_time(e1) * 1e3 / steps
        pgr.close()
        # the Ybus method on the same states, tuned the same way (same grid, separate handle)
        G2y = pf.Grid.from_grid(g2)
        pf.pf_ybus(G2y)

        def b_yb(k, st):
            pf.pf_jacobian_values(G2y, pf.PF_METHOD_YBUS, vm2d, va2d, p2, q2, j2, stream=st)
        if not args.no_tune:
            tuned["batched_ybus"] = autotune.tune(G2y, "jacobian_ybus", B, cache=tune_cache, save=False)
        ev_y, _ = timed(b_yb, steps, 5, period=10)
        extra["batched_20k_x512"]["ybus_avg_launch_us"] = ev_y / steps * 1e6
        extra["batched_20k_x512"]["ybus_schedule"] = G2y.schedule()
        extra["batched_20k_x512"]["ew_speedup_vs_ybus"] = ev_y / ev
        log(f"batched Ybus: {ev_y / steps * 1e6:.1f} us/launch")
        del vm2d, va2d, p2, q2, j2, G2, G2y
        torch.cuda.empty_cache()
        ca = torch.ones(bb // 16, dtype=torch.float64, device=dev)
        cb = torch.empty_like(ca)
        evc, _ = timed(lambda k, st: cb.copy_(ca), 20, 3, period=10)
        extra["batched_20k_x512"]["copy_same_bytes_us"] = evc / 20 * 1e6
        evc, _ = timed(lambda k, st: pf.pf_stream_copy(ca, cb, stream=st), 20, 3, period=10)
        extra["batched_20k_x512"]["stream_copy_same_bytes_us"] = evc / 20 * 1e6
        del ca, cb
        torch.cuda.empty_cache()

    if want("multigrid"):
        grids = gridgen.grids_uneven_64()
        big, bo, ro = gridgen.concat(grids)
        G3 = pf.Grid.from_grid(big, bo, ro)
        vm3 = np.concatenate([gridgen.states(gr.nb, 4, case=3, grid=k + 1)[0] for k, gr in enumerate(grids)], axis=1)
        va3 = np.concatenate([gridgen.states(gr.nb, 4, case=3, grid=k + 1)[1] for k, gr in enumerate(grids)], axis=1)
        vm3d, va3d = torch.as_tensor(vm3, device=dev), torch.as_tensor(va3, device=dev)
        p3 = torch.empty(4, big.nb, dtype=torch.float64, device=dev)
        q3 = torch.empty_like(p3)
        j3 = torch.empty(4, G3.nnz_j, dtype=torch.float64, device=dev)

        def m_sj(k, st):
            pf.pf_jacobian_values(G3, pf.PF_METHOD_ELEMENTWISE, vm3d, va3d, p3, q3, j3, stream=st)
        steps = max(20, K // 40)
        if not args.no_tune:
            cands = [(t, s, o) for t in (128, 256, 512) for s in (0, 1, 4) for o in (1, 2, 3)]
            tuned["multigrid"] = autotune.tune(G3, "jacobian_ew", 4, cache=tune_cache, cands=cands, save=False)
        ev, wall = timed(m_sj, steps, 5, period=10)
        mb = algorithmic_bytes(big.nb, big.nl, G3.nnz_y, 4)
        extra["multigrid_64x4"] = {"grid_state_evals_per_s": 256 * steps / ev, "avg_launch_us": ev / steps * 1e6,
                                   "achieved_GBs": mb / (ev / steps) / 1e9,
                                   "frac_hbm": mb / (ev / steps) / 1e9 / HBM_PEAK_GBS, "algorithmic_bytes": mb,
                                   "buses": big.nb, "branches": big.nl, "schedule": G3.schedule()}
        log(f"multigrid: {ev / steps * 1e6:.1f} us/launch")
        G3y = pf.Grid.from_grid(big, bo, ro)
        pf.pf_ybus(G3y)

        def m_yb(k, st):
            pf.pf_jacobian_values(G3y, pf.PF_METHOD_YBUS, vm3d, va3d, p3, q3, j3, stream=st)
        if not args.no_tune:
            tuned["multigrid_ybus"] = autotune.tune(G3y, "jacobian_ybus", 4, cache=tune_cache, cands=cands, save=False)
        ev_y, _ = timed(m_yb, steps, 5, period=10)
        extra["multigrid_64x4"]["ybus_avg_launch_us"] = ev_y / steps * 1e6
        extra["multigrid_64x4"]["ybus_schedule"] = G3y.schedule()
        extra["multigrid_64x4"]["ew_speedup_vs_ybus"] = ev_y / ev
        log(f"multigrid Ybus: {ev_y / steps * 1e6:.1f} us/launch")
        del vm3d, va3d, p3, q3, j3, G3, G3y
        torch.cuda.empty_cache()
        ca = torch.ones(mb // 16, dtype=torch.float64, device=dev)
        cb = torch.empty_like(ca)
        evc, _ = timed(lambda k, st: cb.copy_(ca), 20, 3, period=10)
        extra["multigrid_64x4"]["copy_same_bytes_us"] = evc / 20 * 1e6
        evc, _ = timed(lambda k, st: pf.pf_stream_copy(ca, cb, stream=st), 20, 3, period=10)
        extra["multigrid_64x4"]["stream_copy_same_bytes_us"] = evc / 20 * 1e6
        del ca, cb
        torch.cuda.empty_cache()

    if want("adjoint"):
        B = 32
        vm4, va4 = gridgen.states(g.nb, B, case=4)
        lp4, lq4 = gridgen.adjoint_seeds(g.nb, B, case=4)
        G4 = pf.Grid.from_grid(g)
        t = lambda a: torch.as_tensor(a, device=dev)
        vm4d, va4d, lp4d, lq4d = t(vm4), t(va4), t(lp4), t(lq4)
        p4 = torch.empty_like(vm4d)
        q4 = torch.empty_like(vm4d)
        gv = torch.empty_like(vm4d)
        ga = torch.empty_like(vm4d)
        steps = max(50, K // 20)
        ev_f, _ = timed(lambda k, st: pf.pf_injections_elementwise(G4, vm4d, va4d, p4, q4, stream=st), steps, 5,
                        period=10)
        ev_b, _ = timed(lambda k, st: pf.pf_injections_vjp(G4, vm4d, va4d, lp4d, lq4d, gv, ga, stream=st), steps, 5,
                        period=10)
        fb = algorithmic_bytes(g.nb, g.nl, G4.nnz_y, B, with_j=False)
        bb = algorithmic_bytes(g.nb, g.nl, G4.nnz_y, B, vjp=True)
        extra["adjoint_100k_x32"] = {"forward_us": ev_f / steps * 1e6, "vjp_us": ev_b / steps * 1e6,
                                     "vjp_over_forward": ev_b / ev_f,
                                     "forward_GBs": fb / (ev_f / steps) / 1e9, "vjp_GBs": bb / (ev_b / steps) / 1e9}
        log(f"adjoint: fwd {ev_f / steps * 1e6:.1f} us, vjp {ev_b / steps * 1e6:.1f} us")
        # the headline evaluation (S + J) on the same 32 states in one launch
        j4 = torch.empty(B, G4.nnz_j, dtype=torch.float64, device=dev)
        ev_j, wall_j = timed(lambda k, st: pf.pf_jacobian_values(G4, pf.PF_METHOD_ELEMENTWISE, vm4d, va4d, p4, q4, j4,
                                                                 stream=st), steps, 5, period=10)
        jb = algorithmic_bytes(g.nb, g.nl, G4.nnz_y, B)
        extra["ew_sj_100k_x32"] = {"state_evals_per_s": B * steps / ev_j, "avg_launch_us": ev_j / steps * 1e6,
                                   "achieved_GBs": jb / (ev_j / steps) / 1e9,
                                   "frac_hbm": jb / (ev_j / steps) / 1e9 / HBM_PEAK_GBS, "algorithmic_bytes": jb,
                                   "schedule": G4.schedule()}
        log(f"100k x 32 S+J: {ev_j / steps * 1e6:.1f} us/launch")
        del j4, G4
        torch.cuda.empty_cache()

    if want("newton"):
        # the evaluation as the inner step of a Newton-Raphson power flow: 5000-bus
        # grid, 20 % PV buses, start near the solution; host sparse LU per iteration
        from paper_2302_10736_amd import newton
        g5 = gridgen.make_grid(5000, 6750, 0.15, case=2)
        vm5, va5 = gridgen.states(g5.nb, 1, case=2, vlo=0.98, vhi=1.02, sigma=0.02)
        G5 = pf.Grid.from_grid(g5)
        # specified powers: the injections at the chosen state
        p5 = torch.empty(1, g5.nb, dtype=torch.float64, device=dev)
        q5 = torch.empty_like(p5)
        pf.pf_injections_elementwise(G5, torch.as_tensor(vm5, device=dev), torch.as_tensor(va5, device=dev), p5, q5)
        case = newton.case_from_state(g5, vm5[0], va5[0], p5[0].cpu().numpy(), q5[0].cpu().numpy(),
                                      pv_frac=0.2, perturb=0.001)
        newton.solve(G5, *case, tol=1e-10, max_iter=10)  # warm-up (first-call costs)
        res = newton.solve(G5, *case, tol=1e-10, max_iter=10)
        it = max(1, res.iterations)
        extra["newton_5k"] = {"converged": res.converged, "iterations": res.iterations,
                              "max_mismatch": res.mismatch,
                              "eval_ms_per_iter": res.seconds_eval / (it + 1) * 1e3,
                              "solve_ms_per_iter": res.seconds_solve / it * 1e3,
                              "max_state_error": float(max(np.abs(res.vm - vm5[0]).max(),
                                                           np.abs(res.va - va5[0]).max())),
                              "note": "eval = device S+J plus copies to the host; solve = host SuperLU"}
        log(f"newton: {res.iterations} iterations, eval {extra['newton_5k']['eval_ms_per_iter']:.3f} ms/iter, "
            f"solve {extra['newton_5k']['solve_ms_per_iter']:.2f} ms/iter")
        del G5

    if want("hubs"):
        # long rows: 32 hub buses of 200-2000 branches each on a 20k-bus grid, against the
        # same grid without the hub lines; one state, warm (the tables fit the caches)
        res_h = {}
        for tag, gh in (("with_hubs", gridgen.grid_hubs()), ("without_hubs", gridgen.make_grid(20_000, 27_000, 0.15,
                                                                                               case=6))):
            Gh = pf.Grid.from_grid(gh)
            pf.pf_ybus(Gh)
            vmh, vah = gridgen.states(gh.nb, 1, case=6)
            vh, ah = torch.as_tensor(vmh, device=dev), torch.as_tensor(vah, device=dev)
            ph, qh = torch.empty_like(vh), torch.empty_like(vh)
            jh = torch.empty(1, Gh.nnz_j, dtype=torch.float64, device=dev)
            n = 100
            row = {"branches": gh.nl}
            for mname, fn in (("ew_s", lambda k, st: pf.pf_injections_elementwise(Gh, vh, ah, ph, qh, stream=st)),
                              ("ew_sj", lambda k, st: pf.pf_jacobian_values(Gh, pf.PF_METHOD_ELEMENTWISE, vh, ah, ph,
                                                                            qh, jh, stream=st)),
                              ("ybus_s", lambda k, st: pf.pf_injections_ybus(Gh, vh, ah, ph, qh, stream=st)),
                              ("ybus_sj", lambda k, st: pf.pf_jacobian_values(Gh, pf.PF_METHOD_YBUS, vh, ah, ph, qh,
                                                                              jh, stream=st))):
                ev, _ = timed(fn, n, 3, period=n)
                row[mname + "_us"] = ev / n * 1e6
            res_h[tag] = row
            del Gh, vh, ah, ph, qh, jh
        res_h["hub_degrees"] = {"count": 32, "min": 200, "max": 2000, "total_hub_branches":
                                res_h["with_hubs"]["branches"] - res_h["without_hubs"]["branches"]}
        extra["hubs_20k"] = res_h
        log("hubs: " + ", ".join(f"{k} {v:.2f} us" for k, v in res_h["with_hubs"].items() if k.endswith("_us")) +
            " (without hubs: " + ", ".join(f"{v:.2f}" for k, v in res_h["without_hubs"].items() if k.endswith("_us"))
            + ")")
        torch.cuda.empty_cache()

    if want("sweep"):
        extra["sweep"] = size_sweep(torch, gridgen, pf, timer, log)

    if tuned:
        extra["autotuner"] ={k: {"schedule": v["schedule"], "us": v["us"], "tried": v["tried"]}
                              for k, v in tuned.items()}
    if extra:
        out["extra"] = extra

    if not args.no_cpu:
        import oracle
        yb = oracle.ybus(g)
        pat = oracle.jac_pattern(yb)
        n = 0
        t0 = time.perf_counter()
        while True:
            oracle.inject_ew(g, vm[0], va[0])
            oracle.jac_ew(g, vm[0], va[0], pat)
            n += 1
            el = time.perf_counter() - t0
            if el >= args.cpu_seconds:
                break
        cpu_model = platform.processor() or ""
        try:
            for line in open("/proc/cpuinfo"):
                if line.startswith("model name"):
                    cpu_model = line.split(":", 1)[1].strip()
                    break
        except OSError:
            pass
        out["cpu_baseline"] = {"value": n / el, "unit": "evals/s", "cores": 1, "kind": "oracle",
                               "sample": f"{n} full element-wise S+J evaluations of the same 100k-bus grid and state "
                                         f"({el:.1f} s, one thread, {cpu_model}, nproc={os.cpu_count()})"}
        if want("cpu_batched"):
            # the batched workload's states on the oracle, one state per task over the host's cores
            # (the C oracle releases the interpreter lock, so the threads run in parallel)
            from concurrent.futures import ThreadPoolExecutor
            g2 = gridgen.grid_20k()
            vm2, va2 = gridgen.states(g2.nb, 512, case=2, vlo=0.9, vhi=1.1, sigma=0.3)
            pat2 = oracle.jac_pattern(oracle.ybus(g2))
            ns_cpu = 512
            threads = max(1, min(16, os.cpu_count() or 1))

            def one(s_):
                oracle.inject_ew(g2, vm2[s_], va2[s_])
                oracle.jac_ew(g2, vm2[s_], va2[s_], pat2)
            with ThreadPoolExecutor(max_workers=threads) as ex:
                list(ex.map(one, range(threads)))  # warm-up
                t0 = time.perf_counter()
                list(ex.map(one, range(ns_cpu)))
                el2 = time.perf_counter() - t0
            extra_cpu = {"value": ns_cpu / el2, "unit": "state-evals/s", "cores": threads, "kind": "oracle",
                         "sample": f"{ns_cpu} of the 512 states of the 20k-bus batched workload, element-wise S+J, "
                                   f"{threads} threads ({el2:.2f} s)"}
            out.setdefault("extra", {})["cpu_oracle_batched_20k"] = extra_cpu

            # the 100k x 32 adjoint workload: forward injections, then J^T lambda (J, then its transpose
            # product), one state per task
            vm4, va4 = gridgen.states(g.nb, 32, case=4)
            lp4, lq4 = gridgen.adjoint_seeds(g.nb, 32, case=4)

            def fwd(s_):
                oracle.inject_ew(g, vm4[s_], va4[s_])

            def adj(s_):
                oracle.vjp(g.nb, pat, oracle.jac_ew(g, vm4[s_], va4[s_], pat), lp4[s_], lq4[s_])
            def passes(fn, ntask, ex):  # whole passes over the tasks until at least one second has passed
                n_, t0_ = 0, time.perf_counter()
                while True:
                    list(ex.map(fn, range(ntask)))
                    n_ += 1
                    el_ = time.perf_counter() - t0_
                    if el_ >= 1.0:
                        return n_, el_
            with ThreadPoolExecutor(max_workers=threads) as ex:
                nf, el_f = passes(fwd, 32, ex)
                nbk, el_b = passes(adj, 32, ex)
            out["extra"]["cpu_oracle_adjoint_100k_x32"] = {
                "forward_state_evals_per_s": 32 * nf / el_f, "vjp_state_evals_per_s": 32 * nbk / el_b,
                "cores": threads, "kind": "oracle",
                "sample": f"the 32 states of the 100k x 32 adjoint workload, {threads} threads (forward {nf} "
                          f"passes in {el_f:.2f} s, adjoint {nbk} passes in {el_b:.2f} s)"}

            # the 64 uneven grids x 4 states, element-wise S+J, one (grid, state) per task
            grids = gridgen.grids_uneven_64()
            pats = [oracle.jac_pattern(oracle.ybus(gr)) for gr in grids]
            st3 = [gridgen.states(gr.nb, 4, case=3, grid=k + 1) for k, gr in enumerate(grids)]

            def mg(task):
                k, s_ = divmod(task, 4)
                oracle.inject_ew(grids[k], st3[k][0][s_], st3[k][1][s_])
                oracle.jac_ew(grids[k], st3[k][0][s_], st3[k][1][s_], pats[k])
            with ThreadPoolExecutor(max_workers=threads) as ex:
                nm, el_m = passes(mg, 4 * len(grids), ex)
            out["extra"]["cpu_oracle_multigrid_64x4"] = {
                "value": 4 * len(grids) * nm / el_m, "unit": "grid-state-evals/s", "cores": threads,
                "kind": "oracle",
                "sample": f"all {4 * len(grids)} grid-states of the 64-grid workload, element-wise S+J, {threads} "
                          f"threads ({nm} passes in {el_m:.2f} s)"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
