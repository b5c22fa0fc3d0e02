"""Tile-shape autotuner.

Three tile shapes change how the sweeps are launched, not what they compute:
  * march segments: the y and z sweeps give each thread one column and a segment of cells
    along the sweep axis; each segment pays a short warm-up (the window of primitives and
    slopes it starts with, and the one face it shares with the next segment), so long
    segments waste less work while short segments expose more parallelism;
  * x rows: the x sweep fused with the update gives each wavefront one or more x-rows of a
    plane, marched in chunks of 58 cells; more rows per wavefront fill more lanes of the last
    chunk of short rows but make each wavefront's march longer;
  * x chunks: the first-stage x sweep gives each wavefront that many consecutive chunks of
    its flattened plane line, paying the wavefront's set-up once for all of them.
The best shapes depend on the axis lengths, the cross-section and the precision.  This module
times candidates on the GPU with the library's own per-kernel event timing and stores the
winners in a table that ``ctu.make_config`` consults when no shape is given.

    python -m paper_1410_4194_amd.autotune --out tiles.json [--sizes 32 48 64 ...]

The table maps precision -> edge -> the best target segment length for the y and the z
sweep, the best x rows and the best x chunks, measured on cubic grids of that edge holding
the shock-cloud initial state (a Mach-10 shock and a dense cloud in uniform gas, the state
the bench and the serving requests run; ``--workload kh`` tunes on the Kelvin-Helmholtz
shear layer instead, which is smooth everywhere).  The segment length changes results only
by rounding (a segment's first trace is a separately compiled copy of the same formulas);
x rows and x chunks leave them bitwise the same.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

CANDIDATES = (4, 6, 8, 12, 16, 24, 32, 48, 64, 96)
X_ROWS = (1, 2, 3, 4, 6, 8)
X_CHUNKS = (1, 2, 4, 8, 16)
DEFAULT_SIZES = (32, 48, 64, 96, 128, 192, 256)
TABLE_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tiles.json")


def _time_shape(ctu, wl, prec, steps, classes, **shape):
    """Milliseconds per step of each kernel class in `classes` with the given tile shape."""
    cfg = ctu.make_config(wl.nx, wl.ny, wl.nz, wl.dx, wl.dy, wl.dz, wl.gamma, wl.bc, prec,
                          wl.cfl, **shape)
    g = ctu.Grid(cfg)
    g.set_primitive(wl.W)
    g.advance(2)
    g.profile_enable(True)
    g.advance(steps)
    prof = g.profile_read()
    g.close()
    return [sum(prof[k][0] for k in cls) / steps for cls in classes]


def _time_candidate(ctu, wl, prec, seg, steps):
    return _time_shape(ctu, wl, prec, steps,
                       (("sweep1_y", "sweep2_y"), ("sweep1_z", "sweep2_z")),
                       march_seg=(seg, seg), x_rows=0, x_chunks=0)


WORKLOADS = ("shock_cloud", "kh")


def tune(sizes=DEFAULT_SIZES, precs=None, candidates=CANDIDATES, steps=8, log=print,
         workload="shock_cloud", x_rows=X_ROWS, x_chunks=X_CHUNKS):
    from . import ctu, workloads as WL
    if workload not in WORKLOADS:
        raise ValueError(f"unknown workload {workload!r}")
    precs = precs if precs is not None else (ctu.FP64, ctu.FP32)
    table = {"candidates": list(candidates), "x_rows_candidates": list(x_rows),
             "x_chunks_candidates": list(x_chunks), "steps": steps, "workload": workload,
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
            log(f"[autotune] {name} n={n}: y {best_y} z {best_z}  "
                + " ".join(f"{s}:{t[0]:.3f}/{t[1]:.3f}" for s, t in times.items()))
            seg = (best_y, best_z)
            # x rows of the fused update, then x chunks of the first-stage x sweep
            rows = {r: _time_shape(ctu, wl, prec, steps, (("sweep2_x_update",),),
                                   march_seg=seg, x_rows=r, x_chunks=0)[0]
                    for r in x_rows if r <= n}
            best_r = min(rows, key=rows.get)
            chunks = {c: _time_shape(ctu, wl, prec, steps, (("sweep1_x",),),
                                     march_seg=seg, x_rows=best_r, x_chunks=c)[0]
                      for c in x_chunks}
            best_c = min(chunks, key=chunks.get)
            log(f"[autotune] {name} n={n}: x rows {best_r} ("
                + " ".join(f"{r}:{t:.3f}" for r, t in rows.items()) + f"), x chunks {best_c} ("
                + " ".join(f"{c}:{t:.3f}" for c, t in chunks.items()) + ")")
            table[name][str(n)] = {"y": best_y, "z": best_z, "x_rows": best_r,
                                   "x_chunks": best_c,
                                   "ms": {str(s): [round(t[0], 4), round(t[1], 4)]
                                          for s, t in times.items()},
                                   "ms_x_rows": {str(r): round(t, 4) for r, t in rows.items()},
                                   "ms_x_chunks": {str(c): round(t, 4)
                                                   for c, t in chunks.items()}}
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


def lookup_x(prec: int, nx: int, ny: int, path: str = TABLE_PATH):
    """Tuned (x rows, x chunks) for a grid, from the nearest tuned edge (by nx); (0, 0) (the
    library's choice) when the table has no such entry."""
    lookup(prec, ny, ny, path)  # loads the table
    table = _cache.get(path)
    rows = (table or {}).get("fp64" if prec == 0 else "fp32") or {}
    sizes = sorted(int(k) for k in rows if "x_rows" in rows[k])
    if not sizes:
        return (0, 0)
    e = rows[str(min(sizes, key=lambda s: abs(s - nx)))]
    return (int(e["x_rows"]), int(e["x_chunks"]))


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
