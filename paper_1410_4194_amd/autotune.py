"""Tile-shape autotuner for the marching sweeps.

The y and z sweeps give each thread one column and a segment of cells along the sweep axis;
each segment pays a short warm-up (the window of primitives and slopes it starts with, and
the one face it shares with the next segment), so long segments waste less work while short
segments expose more parallelism.  The best
length depends on the axis length, the cross-section (how many columns there are to spread
over the GPU) and the precision.  This module times candidate lengths on the GPU with the
library's own per-kernel event timing and stores the winners in a table that
``ctu.make_config`` consults when no length is given.

    python -m paper_1410_4194_amd.autotune --out tiles.json [--sizes 32 48 64 ...]

The table maps precision -> axis length -> best target length for the y sweep and for the
z sweep, measured on cubic grids of that edge holding the shock-cloud initial state (a
Mach-10 shock and a dense cloud in uniform gas, the state the bench and the serving requests
run; ``--workload kh`` tunes on the Kelvin-Helmholtz shear layer instead, which is smooth
everywhere and favours slightly longer segments at 256).  The tile shape changes results
only by rounding: a segment's first trace is a separately compiled copy of the same
formulas.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

CANDIDATES = (8, 12, 16, 24, 32, 48, 64, 96)
DEFAULT_SIZES = (32, 48, 64, 96, 128, 192, 256)
TABLE_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tiles.json")


def _time_candidate(ctu, wl, prec, seg, steps):
    cfg = ctu.make_config(wl.nx, wl.ny, wl.nz, wl.dx, wl.dy, wl.dz, wl.gamma, wl.bc, prec,
                          wl.cfl, march_seg=(seg, seg))
    g = ctu.Grid(cfg)
    g.set_primitive(wl.W)
    g.advance(2)
    g.profile_enable(True)
    g.advance(steps)
    prof = g.profile_read()
    g.close()
    y = prof["sweep1_y"][0] + prof["sweep2_y"][0]
    z = prof["sweep1_z"][0] + prof["sweep2_z"][0]
    return y / steps, z / steps


WORKLOADS = ("shock_cloud", "kh")


def tune(sizes=DEFAULT_SIZES, precs=None, candidates=CANDIDATES, steps=8, log=print,
         workload="shock_cloud"):
    from . import ctu, workloads as WL
    if workload not in WORKLOADS:
        raise ValueError(f"unknown workload {workload!r}")
    precs = precs if precs is not None else (ctu.FP64, ctu.FP32)
    table = {"candidates": list(candidates), "steps": steps, "workload": workload,
             "fp64": {}, "fp32": {}}
    for prec in precs:
        name = "fp64" if prec == ctu.FP64 else "fp32"
        for n in sizes:
            wl = WL.shock_cloud(n) if workload == "shock_cloud" else WL.kelvin_helmholtz(n, n, n)
            times = {}
            for seg in candidates:
                if seg > n + 1:
                    continue
                times[seg] = _time_candidate(ctu, wl, prec, seg, steps)
            best_y = min(times, key=lambda s: times[s][0])
            best_z = min(times, key=lambda s: times[s][1])
            table[name][str(n)] = {"y": best_y, "z": best_z,
                                   "ms": {str(s): [round(t[0], 4), round(t[1], 4)]
                                          for s, t in times.items()}}
            log(f"[autotune] {name} n={n}: y {best_y} z {best_z}  "
                + " ".join(f"{s}:{t[0]:.3f}/{t[1]:.3f}" for s, t in times.items()))
    return table


_cache = {}


def lookup(prec: int, ny: int, nz: int, path: str = TABLE_PATH):
    """Tuned (y, z) target segment lengths for a grid, from the nearest tuned axis length;
    (0, 0) (the library default) when no table exists."""
    if path not in _cache:
        try:
            with open(path) as fh:
                _cache[path] = json.load(fh)
        except (OSError, ValueError):
            _cache[path] = None
    table = _cache[path]
    if not table:
        return (0, 0)
    rows = table.get("fp64" if prec == 0 else "fp32") or {}
    if not rows:
        return (0, 0)
    sizes = sorted(int(k) for k in rows)

    def nearest(n):
        return str(min(sizes, key=lambda s: abs(s - n)))
    return (int(rows[nearest(ny)]["y"]), int(rows[nearest(nz)]["z"]))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=TABLE_PATH)
    ap.add_argument("--sizes", type=int, nargs="*", default=list(DEFAULT_SIZES))
    ap.add_argument("--steps", type=int, default=8)
    ap.add_argument("--workload", choices=WORKLOADS, default="shock_cloud")
    args = ap.parse_args()
    t0 = time.perf_counter()
    table = tune(args.sizes, steps=args.steps, workload=args.workload,
                 log=lambda *a: print(*a, file=sys.stderr, flush=True))
    table["seconds"] = round(time.perf_counter() - t0, 1)
    with open(args.out, "w") as fh:
        json.dump(table, fh, indent=1)
    print(f"[autotune] wrote {args.out}", file=sys.stderr)


if __name__ == "__main__":
    main()
