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
times candidates on the GPU and stores the winners in a table that ``ctu.make_config``
consults when no shape is given.  The default objective is the whole step as the library
runs it (the overlapped schedule on the grid sizes that use it, where the sweeps share the
GPU and no kernel's time is its own), each candidate timed from the same initial state;
``--objective kernels`` times the kernels a shape changes one by one instead (with per-kernel
events, which run the passes in order).

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


def _time_step(ctu, wl, prec, steps, reps=3, **shape):
    """Median milliseconds per whole step with the given tile shape and the library's default
    schedule, each of `reps` runs from the initial state (2 untimed steps, then `steps`)."""
    import torch
    cfg = ctu.make_config(wl.nx, wl.ny, wl.nz, wl.dx, wl.dy, wl.dz, wl.gamma, wl.bc, prec,
                          wl.cfl, **shape)
    g = ctu.Grid(cfg)
    out = []
    for _ in range(reps):
        g.set_primitive(wl.W)
        g.advance(2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.advance(steps)
        torch.cuda.synchronize()
        out.append((time.perf_counter() - t0) * 1e3 / steps)
    g.close()
    return sorted(out)[len(out) // 2]


def _tune_steps(ctu, wl, prec, steps, candidates, x_rows, x_chunks, log, name, n):
    """Whole-step search: segments with y = z, then y and z each with the other fixed, then x
    rows, then x chunks, each with the best of the earlier ones."""
    t = lambda **sh: _time_step(ctu, wl, prec, steps, **sh)  # noqa: E731
    segs = [s for s in candidates if s <= n + 1]
    joint = {s: t(march_seg=(s, s), x_rows=0, x_chunks=0) for s in segs}
    s0 = min(joint, key=joint.get)
    ys = {s: (joint[s] if s == s0 else t(march_seg=(s, s0), x_rows=0, x_chunks=0)) for s in segs}
    by = min(ys, key=ys.get)
    zs = {s: (ys[by] if s == s0 else t(march_seg=(by, s), x_rows=0, x_chunks=0)) for s in segs}
    bz = min(zs, key=zs.get)
    seg = (by, bz)
    rows = {r: t(march_seg=seg, x_rows=r, x_chunks=0) for r in x_rows if r <= n}
    best_r = min(rows, key=rows.get)
    chunks = {c: t(march_seg=seg, x_rows=best_r, x_chunks=c) for c in x_chunks}
    best_c = min(chunks, key=chunks.get)
    log(f"[autotune] {name} n={n}: segments y {by} z {bz} (y = z: "
        + " ".join(f"{s}:{v:.4f}" for s, v in joint.items()) + f"), x rows {best_r}, x chunks "
        f"{best_c}: {chunks[best_c]:.4f} ms per step")
    return {"y": by, "z": bz, "x_rows": best_r, "x_chunks": best_c,
            "ms_step_joint": {str(s): round(v, 4) for s, v in joint.items()},
            "ms_step_y": {str(s): round(v, 4) for s, v in ys.items()},
            "ms_step_z": {str(s): round(v, 4) for s, v in zs.items()},
            "ms_step_x_rows": {str(r): round(v, 4) for r, v in rows.items()},
            "ms_step_x_chunks": {str(c): round(v, 4) for c, v in chunks.items()}}


def _time_candidate(ctu, wl, prec, seg, steps):
    return _time_shape(ctu, wl, prec, steps,
                       (("sweep1_y", "sweep2_y"), ("sweep1_z", "sweep2_z")),
                       march_seg=(seg, seg), x_rows=0, x_chunks=0)


WORKLOADS = ("shock_cloud", "kh")


def tune(sizes=DEFAULT_SIZES, precs=None, candidates=CANDIDATES, steps=8, log=print,
         workload="shock_cloud", x_rows=X_ROWS, x_chunks=X_CHUNKS, objective="step"):
    from . import ctu, workloads as WL
    if workload not in WORKLOADS:
        raise ValueError(f"unknown workload {workload!r}")
    if objective not in ("step", "kernels"):
        raise ValueError(f"unknown objective {objective!r}")
    precs = precs if precs is not None else (ctu.FP64, ctu.FP32)
    table = {"candidates": list(candidates), "x_rows_candidates": list(x_rows),
             "x_chunks_candidates": list(x_chunks), "steps": steps, "workload": workload,
             "objective": objective, "fp64": {}, "fp32": {}}
    for prec in precs:
        name = "fp64" if prec == ctu.FP64 else "fp32"
        for n in sizes:
            wl = WL.shock_cloud(n) if workload == "shock_cloud" else WL.kelvin_helmholtz(n, n, n)
            if objective == "step":
                # at least ~20 ms of steps per timing: small grids take many more steps
                nsteps = max(steps, int(round(steps * (256 / n) ** 2)))
                table[name][str(n)] = _tune_steps(ctu, wl, prec, nsteps, candidates, x_rows,
                                                  x_chunks, log, name, n)
                continue
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


def tune_batch(precs=None, steps=200, log=print, segs=(4, 8, 12, 16, 24),
               chunks=(1, 2, 4, 8), rows=(0, 1, 2)):
    """Tile shapes for grids advanced together in a batch, timed on the 64-grid
    Kelvin-Helmholtz batch (edges from {32, ..., 128}) with one shape for every grid: the
    segment length (y and z), then the x chunks, then the x rows (0: the library's choice per
    grid), each with the best of the earlier ones.  A batch fills the GPU where one small grid
    alone does not, so it prefers less parallelism per grid than the single-grid table.  The
    shear layers evolve over a run, so the timing takes the bench's 200 steps (a 30-step
    timing picked 8-cell segments, 1.7% slower than 12 over 200 steps)."""
    from . import ctu, workloads as WL
    import torch
    precs = precs if precs is not None else (ctu.FP64, ctu.FP32)
    wls = WL.kh_batch(count=64, steps=steps)
    cells = sum(w.cells for w in wls)
    out = {}

    def rate(prec, seg, ch, rw):
        grids = [ctu.Grid.from_workload(w, prec=prec, march_seg=(seg, seg), x_rows=rw,
                                        x_chunks=ch) for w in wls]
        b = ctu.Batch(len(grids), graph=True)
        tickets = [b.submit(g, 2 + steps) for g in grids]
        b.run(2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.run(steps)
        for t in tickets:
            b.poll(t)
        torch.cuda.synchronize()
        v = cells * steps / (time.perf_counter() - t0)
        b.close()
        for g in grids:
            g.close()
        return v
    for prec in precs:
        name = "fp64" if prec == ctu.FP64 else "fp32"
        vs = {s: rate(prec, s, 4, 0) for s in segs}
        seg = max(vs, key=vs.get)
        vc = {c: rate(prec, seg, c, 0) for c in chunks}
        ch = max(vc, key=vc.get)
        vr = {r: rate(prec, seg, ch, r) for r in rows}
        rw = max(vr, key=vr.get)
        out[name] = {"march_seg": seg, "x_chunks": ch, "x_rows": rw,
                     "rate_by_seg": {str(k): round(v) for k, v in vs.items()},
                     "rate_by_x_chunks": {str(k): round(v) for k, v in vc.items()},
                     "rate_by_x_rows": {str(k): round(v) for k, v in vr.items()}}
        log(f"[autotune] batch {name}: seg {seg} ({vs}), x chunks {ch} ({vc}), x rows {rw} ({vr})")
    return out


def lookup_batch(prec: int, path: str = TABLE_PATH):
    """Tuned (segment, x rows, x chunks) for grids advanced in a batch, or None."""
    lookup(prec, 1, 1, path)  # loads the table
    e = ((_cache.get(path) or {}).get("batch") or {}).get("fp64" if prec == 0 else "fp32")
    if not e:
        return None
    return (int(e["march_seg"]), int(e["x_rows"]), int(e["x_chunks"]))


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
    ap.add_argument("--objective", choices=("step", "kernels"), default="step",
                    help="time whole steps as the library runs them (default) or the kernels "
                         "a shape changes, one by one")
    ap.add_argument("--batch-only", action="store_true",
                    help="tune only the batch shapes, into the existing table")
    args = ap.parse_args()
    log = lambda *a: print(*a, file=sys.stderr, flush=True)  # noqa: E731
    if args.batch_only:
        with open(TABLE_PATH) as fh:
            table = json.load(fh)
        table["batch"] = tune_batch(log=log)
        with open(args.out, "w") as fh:
            json.dump(table, fh, indent=1)
        print(f"[autotune] wrote {args.out}", file=sys.stderr)
        return
    t0 = time.perf_counter()
    table = tune(args.sizes, steps=args.steps, workload=args.workload, log=log,
                 objective=args.objective)
    table["batch"] = tune_batch(log=log)
    table["seconds"] = round(time.perf_counter() - t0, 1)
    with open(args.out, "w") as fh:
        json.dump(table, fh, indent=1)
    print(f"[autotune] wrote {args.out}", file=sys.stderr)


if __name__ == "__main__":
    main()
