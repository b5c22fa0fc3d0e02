"""Benchmark: CTU + PPMC + exact-Riemann steps on one MI355X.

Workload: plain FP64 shock-cloud at 256^3 on [0,1]^3 (ambient rho = p = 1, gamma = 5/3,
uniform cloud of radius 0.1 at (0.3, 0.5, 0.5) with density contrast 10, Mach-10 plane
shock with the exact Rankine-Hugoniot post-shock state for x < 0.1, outflow boundaries,
CFL 0.3), advanced with the device-side time step, state resident in HBM.  Each of
`--repeats` runs starts from the initial state, takes `warmup` untimed steps and then times
exactly `steps` steps between two device synchronizations, with no instrumentation and the
library's default schedule (the first-stage y and second-stage z sweeps on a second stream
of the grid's, overlapping the other sweeps; `--schedule` forces in order, overlapped or
fused z for the FP64 and FP32 legs); value = real cells x steps / time of the median run.  A further run of the same steps with per-kernel HIP events (recorded by the
library on its streams; timing runs every pass in order on one stream, so each kernel's
time is its own) gives the kernel times of the roofline.  The FP32 form (FP32 state, reconstruction and fluxes, FP64 Newton solve)
is timed the same way and reported beside it, with its relative L1 distance from FP64.

The JSON line also carries
  roofline: the dominant kernel's achieved bandwidth on the method's algorithmic bytes
           (read u^n, write u^(n+1): 80 B per cell update in FP64, 40 B in FP32) against the
           8 TB/s HBM peak, with its measured traffic per launch (rocprofv3 FETCH_SIZE and
           WRITE_SIZE, committed under profiles/ and tied to the kernel sources by a hash);
           `step`: the same two figures for the whole step; `valu`: VALU issue from the
           committed SQ counters; `design_streaming`: the kernel's own intermediate streams;
           `achievable`: what the library's plain streaming kernels reach on this GPU;
  batched: 64 periodic Kelvin-Helmholtz grids with per-axis edges drawn from
           {32, 48, 64, 96, 128}, 200 steps each with its own device-side time step, every pass
           one launch over all grids, replayed from a captured HIP graph; FP64 and FP32, and
           the same grids advanced one after another for comparison;
  serve:   Poisson-arriving shock-cloud requests (edges {64, 96, 128, 192}, density contrast
           log-uniform in [10, 1000], Mach uniform in [1.5, 10], radius in [0.08, 0.15], run
           to 1.5 cloud-crushing times, FP32 with the FP64 Newton solve) admitted by HBM
           footprint (2 GB budget) into a continuous batch, least estimated work first:
           p50/p99 time-to-solution and aggregate rate; serve_sweep: the same at 0.5, 1 and
           2 x the estimated capacity;
  precision_study: the 512^3 turbulent cloud (lognormal density from a k^-11/3 Gaussian
           random field, mean contrast 10, Mach-10 shock), 50 steps in FP64 and in the FP32
           form with the same time steps, relative L1 between them at steps 1, 25 and 50 (shock
           started at x = 0.1, and at x = 0.14 where it reaches the cloud);
  methods: the same 256^3 workload with PPMC + Roe/HLLE, PPMC + Roe with the H correction,
           PPMP + exact, PPMP + Roe/HLLE and PPMP + Roe with the H correction, both
           precisions (--no-methods skips them and the next leg);
  workloads: the primary step on the 256^3 turbulent cloud and Kelvin-Helmholtz layer;
  cpu_baseline: the FP64 oracle (plain C, built with OpenMP over z-planes) on all the host
           cores this process may use, on a bounded sample of the same state, with the
           serial build beside it, the core count and the CPU model.

Prints one JSON line.
"""
import argparse
import json
import os
import re
import statistics
import sys
import time

REPO = os.path.dirname(os.path.abspath(__file__))
if REPO not in sys.path:
    sys.path.insert(0, REPO)

METRIC = "cell-updates/s at 256^3 (FP64 vs FP32 CTU+PPM+exact); serve p50/p99 latency"
HBM_PEAK_GBS = 8000.0
FP64_VECTOR_PEAK_TFLOPS = 78.6    # 256 CUs x 4 SIMDs x 16 lanes x 2 (FMA) x 2.4 GHz
FP32_VECTOR_PEAK_TFLOPS = 157.3
COUNTERS_FILE = os.path.join(REPO, "profiles", "counters_shock_cloud_256.json")

# Algorithmic HBM bytes of the method per cell update: read the five conserved fields of
# u^n and write those of u^(n+1) once (the dt partials and the ghost shell add about 3%).
ALG_BYTES_PER_CELL_UPDATE = {8: 80, 4: 40}

# The kernels' own streaming design (values of the state's type per unit of work, stencil
# and neighbour reuse counted once), reported as `design_streaming`:
#   sweep1_d (per face): read 5 fields, write 5 first-stage differences
#   sweep2_y/z (per face): read 5 fields and two transverse differences (10), write 5
#   sweep2_x_update (per cell): read 5 fields, the two transverse differences (10) and the
#             y and z CTU differences (10), write the new state (5)
DESIGN_VALUES_PER_UNIT = {"sweep1": 10, "sweep2": 20, "sweep2_x_update": 30, "bc": 10}


# the paper's other reconstruction and Riemann solvers, timed on the same workload
METHODS = [("ppmc_roe", dict(riemann=1)), ("ppmc_roe_hcorr", dict(riemann=1, h_correction=1)),
           ("ppmp_exact", dict(recon=1)), ("ppmp_roe", dict(recon=1, riemann=1)),
           ("ppmp_roe_hcorr", dict(recon=1, riemann=1, h_correction=1))]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _design_values(cls, n, ng=3):
    """(units, values of the state's type) of one launch of a kernel class under the
    kernels' own streaming design, or None for classes it does not cover."""
    nx, ny, nz = n
    d = {"x": 0, "y": 1, "z": 2}
    if cls.startswith("sweep1"):
        e = [nx + 2, ny + 2, nz + 2]
        e[d[cls[-1]]] = n[d[cls[-1]]] + 1
        u = e[0] * e[1] * e[2]
        return u, DESIGN_VALUES_PER_UNIT["sweep1"] * u
    if cls == "sweep2_x_update":
        cells = nx * ny * nz
        return cells, DESIGN_VALUES_PER_UNIT["sweep2_x_update"] * cells
    if cls.startswith("sweep2"):
        e = [nx, ny, nz]
        e[d[cls[-1]]] += 1
        u = e[0] * e[1] * e[2]
        return u, DESIGN_VALUES_PER_UNIT["sweep2"] * u
    if cls == "bc_fill":  # every ghost cell of the allocated box
        u = (nx + 2 * ng) * (ny + 2 * ng) * (nz + 2 * ng) - nx * ny * nz
        return u, DESIGN_VALUES_PER_UNIT["bc"] * u
    return None


def _median(xs):
    return statistics.median(xs)


def run_gpu(wl, prec, steps, warmup, ctu, torch, repeats=5, keep_state=False,
            newton_hist=False, **method):
    """`repeats` uninstrumented runs from the initial state (warmup, then `steps` timed
    steps), then one run of the same steps with per-kernel HIP events."""
    g = ctu.Grid.from_workload(wl, prec=prec, **method)
    secs = []
    for r in range(repeats):
        if r:
            g.set_primitive(wl.W)
        g.advance(warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.advance(steps)
        torch.cuda.synchronize()
        secs.append(time.perf_counter() - t0)
    status, flags, counters = g.check()
    info = g.info()
    # per-kernel times: the same steps again, each kernel bracketed by events
    g.set_primitive(wl.W)
    g.advance(warmup)
    torch.cuda.synchronize()
    g.profile_enable(True)
    t0 = time.perf_counter()
    g.advance(steps)
    torch.cuda.synchronize()
    prof_s = time.perf_counter() - t0
    prof = g.profile_read()
    g.profile_enable(False)
    out = {"seconds": _median(secs), "runs_s": secs, "profile": prof,
           "profiled_seconds": prof_s, "status": status, "flags": flags,
           "counters": counters, "t": info.t, "steps_done": info.steps,
           "schedule": {1: "in order", 2: "overlapped", 3: "fused z"}.get(info.schedule,
                                                                          info.schedule)}
    if keep_state:
        out["state"] = g.get_state()
    if newton_hist:
        # one more (untimed) step through the instrumented sweeps
        g.profile_enable(False, newton=True)
        g.advance(1)
        out["newton_hist"] = g.newton_histogram()
        g.profile_enable(False)
    g.close()
    return out


def rel_l1(got, ref, gamma):
    """Per-field relative L1 distance of two conserved states (5, ...): sum |got - ref| over
    sum of the reference scale (rho; rho (|V| + a) for the momenta; |E|)."""
    import numpy as np
    ref = np.asarray(ref, dtype=np.float64)
    got = np.asarray(got, dtype=np.float64)
    rho = ref[0]
    V2 = (ref[1] ** 2 + ref[2] ** 2 + ref[3] ** 2) / rho ** 2
    p = np.maximum((gamma - 1.0) * (ref[4] - 0.5 * rho * V2), 1e-300)
    smom = rho * (np.sqrt(V2) + np.sqrt(gamma * p / rho))
    scales = [rho, smom, smom, smom, np.abs(ref[4])]
    return [float(np.abs(got[f] - ref[f]).sum() / scales[f].sum()) for f in range(5)]


def run_batched(ctu, torch, WL, prec, steps, warmup, count=64, compare_solo_steps=0):
    """Batched Kelvin-Helmholtz grids: warmup steps (which also capture the graph), then
    `steps` timed steps of every grid; optionally the same grids advanced one at a time."""
    wls = WL.kh_batch(count=count, steps=steps)
    cells = sum(w.cells for w in wls)
    grids = [ctu.Grid.from_workload(w, prec=prec, batch=True) for w in wls]
    b = ctu.Batch(count, graph=True)
    tickets = [b.submit(g, warmup + steps) for g in grids]
    b.run(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.run(steps)
    states = [b.poll(t)[0] for t in tickets]   # syncs the batch stream
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    assert all(s == ctu.TICKET_DONE for s in states), states
    b.close()
    out = {"grids": count, "cells": cells, "steps": steps, "warmup": warmup,
           "value": round(cells * steps / (t1 - t0), 1), "unit": "cell-updates/s",
           "ms_per_step": round(1e3 * (t1 - t0) / steps, 4), "graph": True}
    if compare_solo_steps:
        torch.cuda.synchronize()
        s0 = time.perf_counter()
        for g in grids:
            g.advance(compare_solo_steps)
        torch.cuda.synchronize()
        s1 = time.perf_counter()
        out["one_grid_at_a_time"] = {"steps": compare_solo_steps,
                                     "value": round(cells * compare_solo_steps / (s1 - s0), 1)}
    for g in grids:
        g.close()
    return out


def run_serve(ctu, WL, rate, count, hbm_budget, seed, steps_per_round=8, keep=False,
              policy="fifo"):
    from paper_1410_4194_amd import serve as S
    reqs = WL.shock_cloud_requests(count, rate=rate, seed=seed)
    requests = [S.Request(q["rid"], q["arrival"], WL.request_workload(q), q["t_end"], ctu.FP32,
                          cost=WL.estimated_steps(q) * q["n"] ** 3)
                for q in reqs]
    stats = S.serve(requests, hbm_budget=hbm_budget, max_slots=64,
                    steps_per_round=steps_per_round, graph=True, keep_states=keep, policy=policy)
    out = stats.summary()
    out.update({"rate_per_s": rate, "hbm_budget_gb": round(hbm_budget / 1e9, 2),
                "policy": policy})
    return out


def precision_study(ctu, torch, WL, n=512, steps=50, x_shock=0.1):
    """FP32 form vs FP64 on the turbulent cloud: both advanced with the FP64 grid's time step
    (read back every step), so the difference is the precision alone."""
    wl = WL.turbulent_cloud(n, x_shock=x_shock)
    g64 = ctu.Grid.from_workload(wl, prec=ctu.FP64)
    g32 = ctu.Grid.from_workload(wl, prec=ctu.FP32)
    out = {"workload": f"turbulent_cloud_{n}^3 Mach-10 shock at x={x_shock}", "steps": steps,
           "l1_by_step": {}}
    for k in range(1, steps + 1):
        dt = g64.compute_dt()
        g64.step(dt)
        g32.step(dt)
        if k in (1, steps // 2, steps):
            out["l1_by_step"][k] = rel_l1(g32.get_state(), g64.get_state(), wl.gamma)
            log(f"[bench] precision study step {k}: L1 {out['l1_by_step'][k]}")
    for g in (g64, g32):
        st = g.check()[0]
        out.setdefault("status", []).append(st)
        g.close()
    return out


# The files that define the step's kernels (device code and launch shapes): committed counter
# figures are used only while these are unchanged.  The host runtime's ABI plumbing and the
# streaming probe are not part of it.
KERNEL_SOURCES = ("ctu_common.hpp", "ctu_device.hpp", "ctu_kernels.hip", "ctu_kernels.hpp",
                  "ctu_sweeps.hip", "ctu_sweeps.hpp")


def _source_hash():
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(REPO, "paper_1410_4194_amd", "csrc")
    for f in sorted(KERNEL_SOURCES):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def _counters(prec_name):
    """Committed rocprofv3 counters of the primary step's kernels for one precision,
    {class: {"bytes": HBM bytes per launch (FETCH_SIZE and WRITE_SIZE scaled by the
    calibration), "valu_issue": fraction of SIMD cycles issuing VALU, ...}}, or None when
    they were taken from other kernel sources than these."""
    try:
        with open(COUNTERS_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("source_hash") != _source_hash():
        return None
    return t.get(prec_name)


def roofline(prof, n, eb, prec_name, rate, ng=3):
    """Roofline of the dominant kernel class (by total time over the profiled steps).

    achieved: the method's algorithmic bytes per launch (ALG_BYTES_PER_CELL_UPDATE x the
    cell updates one launch completes, i.e. every cell of the grid: each pass of a step
    covers the whole grid once) over the kernel's average launch time, against the HBM peak.
    traffic: the kernel's measured HBM bytes per launch (committed counters of the same
    kernel sources; None otherwise).  bound: the resource the counters show nearer its
    limit, the measured traffic against the HBM peak or the VALU issue fraction.
    step: the same figures for the whole step at the measured rate; valu: VALU issue from
    the committed SQ counters (dominant kernel, and weighted by kernel time over the step);
    design_streaming: the dominant kernel against its own intermediate streams."""
    cells = n[0] * n[1] * n[2]
    timed = {k: v for k, v in prof.items() if v[1] > 0}
    cls, (ms, launches) = max(timed.items(), key=lambda kv: kv[1][0])
    avg_s = ms / launches / 1e3
    per_unit = ALG_BYTES_PER_CELL_UPDATE[eb]
    alg_bytes = per_unit * cells
    achieved = alg_bytes / avg_s / 1e9
    cnt = _counters(prec_name) or {}
    k = cnt.get(cls)
    traffic = round(k["bytes"]) if k else None
    out = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": cls,
           "avg_launch_ms": round(ms / launches, 4), "launches": launches,
           "units_per_launch": cells, "unit_of_work": "cell update",
           "algorithmic_bytes_per_unit": per_unit, "algorithmic_bytes_per_launch": alg_bytes}
    steps = max(v[1] for kk, v in timed.items() if kk == cls)
    step_s = 1.0 / (rate / cells)
    out["step"] = {"algorithmic_GBps": round(per_unit * rate / 1e9, 1),
                   "algorithmic_frac": round(per_unit * rate / 1e9 / HBM_PEAK_GBS, 4)}
    if cnt and all(kk in cnt for kk in timed if kk != "dt_final"):
        step_bytes = sum(cnt[kk]["bytes"] * timed[kk][1] / steps for kk in timed if kk in cnt)
        out["step"].update({"measured_bytes": round(step_bytes),
                            "measured_bytes_per_cell_update": round(step_bytes / cells, 1),
                            "measured_GBps": round(step_bytes / step_s / 1e9, 1),
                            "measured_frac": round(step_bytes / step_s / 1e9 / HBM_PEAK_GBS, 4)})
    if k:
        meas = k["bytes"] / avg_s / 1e9
        out["measured_GBps"] = round(meas, 1)
        out["measured_frac"] = round(meas / HBM_PEAK_GBS, 4)
        valu = {"issue_frac": k.get("valu_issue"),
                "source": os.path.relpath(COUNTERS_FILE, REPO)}
        tot = sum(v[0] for kk, v in timed.items() if kk in cnt and "valu_issue" in cnt[kk])
        if tot > 0:
            valu["issue_frac_step"] = round(sum(v[0] * cnt[kk]["valu_issue"] for kk, v in
                                                timed.items() if kk in cnt and
                                                "valu_issue" in cnt[kk]) / tot, 4)
        if k.get("f64_flops") is not None and eb == 8:
            fl = k["f64_flops"] / avg_s / 1e12
            valu.update({"executed_f64_TFLOPs": round(fl, 2),
                         "executed_f64_frac": round(fl / FP64_VECTOR_PEAK_TFLOPS, 4),
                         "flop_peak_TFLOPs": FP64_VECTOR_PEAK_TFLOPS})
        out["valu"] = valu
        if valu["issue_frac"] is not None and valu["issue_frac"] > meas / HBM_PEAK_GBS:
            out["bound"] = "alu"
            out["bound_note"] = ("VALU issue above the measured traffic fraction; achieved "
                                 "and frac stay the algorithmic-bytes figures")
    dv = _design_values(cls, n, ng)
    if dv:
        out["design_streaming"] = {"bytes_per_launch": dv[1] * eb,
                                   "GBps": round(dv[1] * eb / avg_s / 1e9, 1),
                                   "frac": round(dv[1] * eb / avg_s / 1e9 / HBM_PEAK_GBS, 4)}
    return out


def bandwidth_probe(ctu, torch, gib=1, reps=5):
    """What the library's plain streaming kernels (ctu_stream_probe: one 8-byte element per
    lane, four independent loads per lane) reach on this GPU's HBM: a read-only sum, a copy
    (1 read : 1 write), an add of two arrays into a third (2 : 1) and a combine of five
    arrays into one (5 : 1, the fused update's mix), each over `gib` GiB per array, the
    best of `reps` launches timed with HIP events on torch's current stream (the stream the
    probe runs on).  Context for the roofline fraction, which stays against the published
    peak."""
    n = (gib << 30) // 8
    a = torch.empty(5 * n, dtype=torch.float64, device="cuda").uniform_()
    b = torch.empty(n, dtype=torch.float64, device="cuda").uniform_()
    c = torch.empty(max(n, ctu.stream_probe_blocks(5 * n)), dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()

    def best(kind, nn, bb, nbytes):
        ctu.stream_probe(kind, a, bb, c, nn, stream)
        torch.cuda.synchronize()
        times = []
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            ctu.stream_probe(kind, a, bb, c, nn, stream)
            e1.record(stream)
            e1.synchronize()
            times.append(e0.elapsed_time(e1) / 1e3)
        return round(nbytes / min(times) / 1e9, 1)

    nb = n * 8
    out = {"read_GBps": best(ctu.STREAM_READ, 5 * n, None, 5 * nb),
           "copy_GBps": best(ctu.STREAM_COPY, n, None, 2 * nb),
           "add_GBps": best(ctu.STREAM_ADD, n, b, 3 * nb),
           "combine5_GBps": best(ctu.STREAM_COMBINE5, n, None, 6 * nb),
           "bytes_per_array": nb, "kernel": "ctu_stream_probe"}
    del a, b, c
    torch.cuda.empty_cache()
    return out


def _host_cpu():
    """(threads this process may use, logical CPUs of the host, CPU model name)."""
    try:
        allowed = len(os.sched_getaffinity(0))
    except AttributeError:
        allowed = os.cpu_count() or 1
    env = os.environ.get("OMP_NUM_THREADS")
    threads = min(allowed, int(env)) if env and env.isdigit() and int(env) > 0 else allowed
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return threads, os.cpu_count() or 1, model


def cpu_baseline(wl, seconds_target=12.0, serial_seconds=5.0, methods=(), method_seconds=2.0):
    """The FP64 oracle on a bounded sample of the same workload: CTU steps of a box of the
    256^3 shock-cloud initial state around the shock front and the cloud's upwind edge,
    repeated for about `seconds_target`, with the OpenMP build on every core this process
    may use (OMP_NUM_THREADS caps it); the serial build on the same box beside it; then the
    box with each of `methods` ((name, config keywords)), OpenMP, about `method_seconds`
    each."""
    import oracle as O

    threads, ncpu, model = _host_cpu()
    lo, hi = (0, 64, 64), (128, 192, 192)
    cells = (hi[0] - lo[0]) * (hi[1] - lo[1]) * (hi[2] - lo[2])

    def rate(seconds, **kw):
        cfg = O.Config(wl.nx, wl.ny, wl.nz, wl.dx, wl.dy, wl.dz, wl.gamma, bc=wl.bc, cfl=wl.cfl,
                       **kw)
        u = O.state_from_primitive(cfg, wl.W)
        O.bc_fill(cfg, u)
        dt = O.compute_dt(cfg, u)
        t_total, reps = 0.0, 0
        while t_total < seconds and reps < 60:
            t0 = time.perf_counter()
            O.update_box(cfg, u, dt, lo, hi)
            t_total += time.perf_counter() - t0
            reps += 1
        del u
        return cells * reps / t_total, reps, t_total

    used = O.set_threads(threads)
    try:
        v, reps, t_total = rate(seconds_target)
        mres = {}
        for name, kw in methods:
            vm, rm, tm = rate(method_seconds, **kw)
            log(f"[bench]   oracle {name}: {vm:.4g} cell-updates/s ({rm} steps of the box)")
            mres[name] = {"value": round(vm, 1), "steps": rm, "seconds": round(tm, 1)}
    finally:
        O.set_threads(1)
    vs, rs, ts = rate(serial_seconds)
    box = f"[{lo[0]},{hi[0]})x[{lo[1]},{hi[1]})x[{lo[2]},{hi[2]})"
    out = {"value": round(v, 1), "unit": "cell-updates/s", "cores": used, "kind": "oracle",
           "sample": f"{reps} x one CTU step of the {cells}-cell box {box} (x, y, z) of the "
                     f"256^3 shock-cloud initial state, FP64 C oracle built with OpenMP over "
                     f"z-planes, {used} threads, {t_total:.1f} s",
           "host": {"cpu_model": model, "logical_cpus": ncpu, "threads_allowed": threads},
           "serial": {"value": round(vs, 1), "cores": 1, "steps": rs, "seconds": round(ts, 1)},
           "omp_speedup": round(v / vs, 2)}
    if mres:
        out["methods"] = mres
    return out


# rocprofv3 kernel names of the primary step's kernels -> the library's kernel classes
# (PPMC + exact solver for gamma 5/3: solver class 3, reconstruction 0).
_CLASS_PATTERNS = [
    (r"k_bc_fill<(double|float)>", "bc_fill"),
    (r"k_sweep_x<(double|float), 1, false, 3, 0>", "sweep1_x"),
    (r"k_sweep_march<(double|float), 1, 1, false, 3, 0>", "sweep1_y"),
    (r"k_sweep_march<(double|float), 2, 1, false, 3, 0>", "sweep1_z"),
    (r"k_sweep_march<(double|float), 1, 2, false, 3, 0>", "sweep2_y"),
    (r"k_sweep_march<(double|float), 2, 2, false, 3, 0>", "sweep2_z"),
    (r"k_sweep_x_update<(double|float), false, 3, 0>", "sweep2_x_update"),
]


def _counter_rows(d):
    """{kernel name: {counter: [value per dispatch]}} from the counter-collection CSVs of a
    rocprofv3 --pmc output directory."""
    import csv
    import glob
    rows = {}
    for path in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        with open(path) as fh:
            for r in csv.DictReader(fh):
                name = r.get("Kernel_Name", "")
                rows.setdefault(name, {}).setdefault(r["Counter_Name"], []).append(
                    float(r["Counter_Value"]))
    return rows


def _avg(xs):
    return sum(xs) / len(xs)


def summarize_counters(fetch_dir, write_dir, sq_dir, flops_dir, probe_fetch_dir,
                       probe_write_dir, out_path, command, source_hash):
    """Per-launch HBM bytes and VALU figures of the primary step's kernels from rocprofv3
    --pmc output directories, calibrated with the plain streaming kernels (whose bytes are
    known): fetch scale = bytes the read probe reads / its FETCH_SIZE; write scale = bytes
    the copy probe writes / its WRITE_SIZE.  Written as JSON, tied to the kernel sources by
    the hash of the sources the profiled runs were built from (source_hash, printed by
    `bench.py --source-hash` in the same tree before they ran)."""
    pf, pw = _counter_rows(probe_fetch_dir), _counter_rows(probe_write_dir)
    n = (1 << 30) // 8

    def probe(rows, kname, counter):
        for k, v in rows.items():
            if kname in k and counter in v:
                return _avg(v[counter])
        raise SystemExit(f"no {counter} for {kname} in the probe run")
    read_kib = probe(pf, "k_stream_read", "FETCH_SIZE")
    copy_fetch_kib = probe(pf, "k_stream_copy", "FETCH_SIZE")
    comb_fetch_kib = probe(pf, "k_stream_combine5", "FETCH_SIZE")
    copy_write_kib = probe(pw, "k_stream_copy", "WRITE_SIZE")
    comb_write_kib = probe(pw, "k_stream_combine5", "WRITE_SIZE")
    fetch_scale = (2 * n * 8 / 1024) / read_kib
    write_scale = (n * 8 / 1024) / copy_write_kib
    out = {"source_hash": source_hash, "command": command,
           "calibration": {
               "fetch_scale": round(fetch_scale, 4), "write_scale": round(write_scale, 4),
               "read_probe": {"true_kib": 2 * n * 8 // 1024, "fetch_kib": read_kib},
               "copy_probe": {"true_kib_each": n * 8 // 1024, "fetch_kib": copy_fetch_kib,
                              "write_kib": copy_write_kib},
               "combine5_probe": {"true_read_kib": 5 * n * 8 // 1024,
                                  "true_write_kib": n * 8 // 1024,
                                  "fetch_kib": comb_fetch_kib, "write_kib": comb_write_kib}}}
    fe, wr = _counter_rows(fetch_dir), _counter_rows(write_dir)
    sq = _counter_rows(sq_dir)
    fl = _counter_rows(flops_dir) if flops_dir else {}
    for kname in set(fe) | set(wr):
        for pat, cls in _CLASS_PATTERNS:
            m = re.search(pat, kname)
            if not m:
                continue
            prec = "fp64" if m.group(1) == "double" else "fp32"
            e = {"kernel": kname}
            if "FETCH_SIZE" in fe.get(kname, {}) and "WRITE_SIZE" in wr.get(kname, {}):
                e["fetch_kib"] = round(_avg(fe[kname]["FETCH_SIZE"]), 1)
                e["write_kib"] = round(_avg(wr[kname]["WRITE_SIZE"]), 1)
                e["bytes"] = round(1024 * (e["fetch_kib"] * fetch_scale +
                                           e["write_kib"] * write_scale))
            c = sq.get(kname, {})
            if "SQ_INSTS_VALU" in c and "GRBM_GUI_ACTIVE" in c and "SQ_WAVES" in c:
                insts, gui, waves = _avg(c["SQ_INSTS_VALU"]), _avg(c["GRBM_GUI_ACTIVE"]), \
                    _avg(c["SQ_WAVES"])
                # 1024 SIMDs; a wave64 VALU instruction occupies a 16-lane SIMD for 4 cycles;
                # GRBM_GUI_ACTIVE counts the busy cycles of each of the 8 XCDs
                e["valu_insts_per_wave"] = round(insts / max(waves, 1), 1)
                e["valu_issue"] = round(insts * 4 / (1024 * gui / 8), 4)
                if "SQ_WAIT_INST_ANY" in c and "SQ_WAVE_CYCLES" in c:
                    e["wait_frac"] = round(_avg(c["SQ_WAIT_INST_ANY"]) /
                                           max(_avg(c["SQ_WAVE_CYCLES"]), 1), 4)
            f = fl.get(kname, {})
            need = ("SQ_INSTS_VALU_ADD_F64", "SQ_INSTS_VALU_MUL_F64", "SQ_INSTS_VALU_FMA_F64",
                    "SQ_INSTS_VALU_TRANS_F64")
            if all(k in f for k in need):
                add, mul, fma, trans = (_avg(f[k]) for k in need)
                # per wave64 instruction: 64 lane operations, an FMA counting two flops
                e["f64_flops"] = 64 * (add + mul + trans + 2 * fma)
                e["f64_insts"] = {"add": add, "mul": mul, "fma": fma, "trans": trans}
            out.setdefault(prec, {})[cls] = e
    with open(out_path, "w") as fh:
        json.dump(out, fh, indent=1, sort_keys=True)
        fh.write("\n")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--repeats", type=int, default=5,
                    help="timed runs of the primary and FP32 legs (the median is reported)")
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--schedule", choices=("auto", "in_order", "overlap", "fused_z"),
                    default="auto",
                    help="pass order of the primary FP64 and FP32 steps (the library's choice "
                         "by default)")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-precision-study", action="store_true")
    ap.add_argument("--no-bandwidth-probe", action="store_true")
    ap.add_argument("--no-methods", action="store_true",
                    help="skip the Roe, Roe+H and PPMP legs on the same workload")
    ap.add_argument("--method-steps", type=int, default=20)
    ap.add_argument("--batch-steps", type=int, default=200)
    ap.add_argument("--serve-requests", type=int, default=16)
    ap.add_argument("--serve-load", type=float, default=0.5,
                    help="arrival rate as a fraction of the estimated capacity")
    ap.add_argument("--serve-budget-gb", type=float, default=2.0,
                    help="HBM budget of the serving loop (2 GB: admission binds from about "
                         "the estimated capacity up; the largest request needs 1.1 GB)")
    ap.add_argument("--serve-policy", choices=("fifo", "sjf"), default="sjf",
                    help="admission policy of the serving runs")
    ap.add_argument("--serve-loads", default="0.5,1,2",
                    help="arrival rates of serve_sweep, as fractions of the estimated "
                         "capacity ('' skips the sweep)")
    ap.add_argument("--precision-n", type=int, default=512)
    ap.add_argument("--source-hash", action="store_true",
                    help="print the hash of the kernel sources that counter figures are tied to")
    ap.add_argument("--stream-probe", action="store_true",
                    help="run only the plain streaming kernels, 3 launches of each (counter "
                         "calibration: 1 GiB arrays of known size)")
    ap.add_argument("--summarize-counters", nargs=7,
                    metavar=("HASH", "FETCH", "WRITE", "SQ", "FLOPS", "PROBE_FETCH", "PROBE_WRITE"),
                    help="write the committed counter file from rocprofv3 --pmc output "
                         "directories (FLOPS may be '-'); HASH: --source-hash of the profiled "
                         "tree")
    args = ap.parse_args()
    if args.summarize_counters:
        h, *d = args.summarize_counters
        summarize_counters(d[0], d[1], d[2], None if d[3] == "-" else d[3], d[4], d[5],
                           COUNTERS_FILE, "see profiles/ctu_step_shock_cloud_256.md", h)
        print(COUNTERS_FILE)
        return
    if args.source_hash:
        print(_source_hash())
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the CTU step would shard by 3D block decomposition with halo exchange, which the library does not implement)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1410_4194_amd import ctu, workloads as WL
    if args.stream_probe:
        n = (1 << 30) // 8
        a = torch.empty(5 * n, dtype=torch.float64, device="cuda").uniform_()
        b = torch.empty(n, dtype=torch.float64, device="cuda").uniform_()
        c = torch.empty(n, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        for kind, nn, bb in ((ctu.STREAM_READ, 2 * n, None), (ctu.STREAM_COPY, n, None),
                             (ctu.STREAM_COMBINE5, n, None)):
            for _ in range(3):
                ctu.stream_probe(kind, a, bb, c, nn)
        torch.cuda.synchronize()
        log(f"[bench] stream probe: 3 launches each of read ({2 * n * 8} B), copy ({n * 8} B "
            f"read and written) and combine5 ({5 * n * 8} B read, {n * 8} B written)")
        return

    log(f"[bench] building shock-cloud {args.n}^3 initial state")
    wl = WL.shock_cloud(args.n, steps=args.steps)
    n = (wl.nx, wl.ny, wl.nz)
    cells = wl.cells

    log(f"[bench] FP64: {args.repeats} runs of warmup {args.warmup} + timed {args.steps} steps, "
        "then one run with per-kernel events")
    sched = {"auto": ctu.SCHEDULE_AUTO, "in_order": ctu.SCHEDULE_IN_ORDER,
             "overlap": ctu.SCHEDULE_OVERLAP, "fused_z": ctu.SCHEDULE_FUSED_Z}[args.schedule]
    r64 = run_gpu(wl, ctu.FP64, args.steps, args.warmup, ctu, torch, repeats=args.repeats,
                  keep_state=not args.no_fp32, newton_hist=True, schedule=sched)
    v64 = cells * args.steps / r64["seconds"]
    log(f"[bench] FP64 {v64:.4g} cell-updates/s (median), runs "
        f"{[round(1e3 * s / args.steps, 4) for s in r64['runs_s']]} ms/step; "
        f"with per-kernel events {1e3 * r64['profiled_seconds'] / args.steps:.4f} ms/step")
    for k, (ms, la) in sorted(r64["profile"].items(), key=lambda kv: -kv[1][0]):
        if la:
            log(f"[bench]   {k:12s} {ms / max(la, 1):8.4f} ms/launch  x{la}")

    out = {
        "metric": METRIC, "value": round(v64, 1), "unit": "cell-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(1e3 * r64["seconds"] / args.steps, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"shock_cloud_{args.n}^3 Mach-10 chi-10 FP64 CFL 0.3",
                   "cells": cells, "grid": list(n), "parallelism": "single GPU",
                   "repeats": args.repeats, "schedule": r64["schedule"],
                   "runs_ms_per_step": [round(1e3 * s / args.steps, 4) for s in r64["runs_s"]],
                   "profiled_ms_per_step": round(1e3 * r64["profiled_seconds"] / args.steps, 4),
                   "newton_caps": r64["counters"][1], "status": r64["status"],
                   "newton_iterations_per_solve": r64.get("newton_hist")},
        "roofline": roofline(r64["profile"], n, 8, "fp64", v64),
        "kernels_ms": {k: round(v[0] / max(v[1], 1), 4) for k, v in r64["profile"].items()
                       if v[1] > 0},
    }
    if not args.no_bandwidth_probe:
        bw = bandwidth_probe(ctu, torch)
        log(f"[bench] plain streaming kernels on this GPU (GB/s): {bw}")
        out["roofline"]["achievable"] = bw
    if not args.no_fp32:
        log(f"[bench] FP32 form: {args.repeats} runs of warmup {args.warmup} + timed {args.steps} steps")
        r32 = run_gpu(wl, ctu.FP32, args.steps, args.warmup, ctu, torch, repeats=args.repeats,
                      keep_state=True, schedule=sched)
        v32 = cells * args.steps / r32["seconds"]
        log(f"[bench] FP32 {v32:.4g} cell-updates/s")
        l1 = rel_l1(r32.pop("state"), r64.pop("state"), wl.gamma)
        log(f"[bench] FP32 vs FP64 relative L1 after {args.warmup + args.steps} steps: {l1}")
        out["fp32"] = {"value": round(v32, 1), "unit": "cell-updates/s",
                       "ms_per_step": round(1e3 * r32["seconds"] / args.steps, 4),
                       "runs_ms_per_step": [round(1e3 * s / args.steps, 4) for s in r32["runs_s"]],
                       "vs_fp64": round(v32 / v64, 3),
                       "rel_l1_vs_fp64": [float(f"{e:.3e}") for e in l1],
                       "t_minus_t_fp64": r32["t"] - r64["t"],
                       "roofline": roofline(r32["profile"], n, 4, "fp32", v32),
                       "kernels_ms": {k: round(v[0] / max(v[1], 1), 4)
                                      for k, v in r32["profile"].items() if v[1] > 0}}
    if not args.no_methods:
        # the other reconstruction and Riemann solvers of the paper on the same workload
        out["methods"] = {}
        for mname, kw in METHODS:
            ng = (4 if kw.get("recon") else 3) + kw.get("h_correction", 0)
            for pname, prec, eb in (("fp64", ctu.FP64, 8), ("fp32", ctu.FP32, 4)):
                log(f"[bench] method {mname} {pname}: warmup {args.warmup}, timed {args.method_steps} steps")
                rm = run_gpu(wl, prec, args.method_steps, args.warmup, ctu, torch, repeats=1, **kw)
                vm = cells * args.method_steps / rm["seconds"]
                log(f"[bench]   {vm:.4g} cell-updates/s, status {rm['status']}, "
                    f"HLLE substitutions {rm['counters'][3]}")
                rl = roofline(rm["profile"], n, eb, f"{pname}_{mname}", vm, ng=ng)
                out["methods"][f"{mname}_{pname}"] = {
                    "value": round(vm, 1), "unit": "cell-updates/s", "steps": args.method_steps,
                    "ms_per_step": round(1e3 * rm["seconds"] / args.method_steps, 4),
                    "vs_ppmc_exact": round(vm / (v64 if prec == ctu.FP64 else
                                                 out.get("fp32", {}).get("value", v64)), 3),
                    "status": rm["status"], "hlle_substitutions": rm["counters"][3],
                    "roofline": {k: rl[k] for k in ("bound", "achieved", "peak", "unit", "frac",
                                                    "kernel", "avg_launch_ms")},
                    "kernels_ms": {k: round(v[0] / max(v[1], 1), 4)
                                   for k, v in rm["profile"].items() if v[1] > 0}}
        # the primary step on states with structure everywhere: equal face states (which skip
        # the Newton solve) are the common case in the shock-cloud's ambient gas, rarer here
        out["workloads"] = {}
        for wname, wmake in (("turbulent_cloud_256^3", lambda: WL.turbulent_cloud(args.n)),
                             ("kelvin_helmholtz_256^3", lambda: WL.kelvin_helmholtz(args.n, args.n, args.n))):
            wl2 = wmake()
            log(f"[bench] workload {wname} fp64: warmup {args.warmup}, timed {args.method_steps} steps")
            rw = run_gpu(wl2, ctu.FP64, args.method_steps, args.warmup, ctu, torch, repeats=1,
                         newton_hist=True)
            vw = wl2.cells * args.method_steps / rw["seconds"]
            h = rw.get("newton_hist") or {}
            log(f"[bench]   {vw:.4g} cell-updates/s; Newton iterations per solve {h}")
            out["workloads"][wname] = {
                "value": round(vw, 1), "unit": "cell-updates/s", "steps": args.method_steps,
                "ms_per_step": round(1e3 * rw["seconds"] / args.method_steps, 4),
                "newton_iterations_per_solve": h,
                "kernels_ms": {k: round(v[0] / max(v[1], 1), 4)
                               for k, v in rw["profile"].items() if v[1] > 0}}
            del wl2
    if not args.no_batched:
        for name, prec in (("fp64", ctu.FP64), ("fp32", ctu.FP32)):
            log(f"[bench] batched Kelvin-Helmholtz, 64 grids, {name}")
            rb = run_batched(ctu, torch, WL, prec, args.batch_steps, args.warmup,
                             compare_solo_steps=20)
            log(f"[bench]   {rb['value']:.4g} cell-updates/s over {rb['cells']} cells")
            rb["vs_plain_fp64_256"] = round(rb["value"] / v64, 3)
            out.setdefault("batched", {})[name] = rb
    if not args.no_serve:
        import numpy as np
        cap_rate = out.get("batched", {}).get("fp32", {}).get("value") or v64
        probe = WL.shock_cloud_requests(256, rate=1.0, seed=WL.BASE_SEED + 5)
        mean_work = float(np.mean([WL.estimated_steps(q) * q["n"] ** 3 for q in probe]))
        capacity = cap_rate / mean_work
        budget = int(args.serve_budget_gb * 1e9)
        loads = [float(x) for x in args.serve_loads.split(",") if x.strip()]
        runs = [args.serve_load] + [ld for ld in loads]
        done = {}
        for i, load in enumerate(runs):
            if i > 0 and load in done:
                out.setdefault("serve_sweep", []).append(done[load])
                continue
            rate = load * capacity
            log(f"[bench] serving ({args.serve_policy}): {args.serve_requests} requests at "
                f"{rate:.3f}/s ({load} x estimated capacity {capacity:.3f}/s)")
            rs = run_serve(ctu, WL, rate, args.serve_requests, budget, WL.BASE_SEED + 5,
                           policy=args.serve_policy)
            rs["load"] = load
            rs["capacity_estimate_per_s"] = round(capacity, 4)
            log(f"[bench]   p50 {rs['p50_s']} s, p99 {rs['p99_s']} s, "
                f"{rs['cell_updates_per_s']:.4g} cell-updates/s")
            done[load] = rs
            if i == 0:
                out["serve"] = rs
            else:
                out.setdefault("serve_sweep", []).append(rs)
    if not args.no_precision_study:
        log(f"[bench] precision study: {args.precision_n}^3 turbulent cloud, 50 steps, FP64 and FP32")
        out["precision_study"] = precision_study(ctu, torch, WL, n=args.precision_n)
        # the same with the shock started 0.01 from the cloud edge, so that it hits the cloud
        # within the 50 steps and the flow turns three-dimensional
        log("[bench] precision study, active variant: shock at x = 0.14")
        out["precision_study_active"] = precision_study(ctu, torch, WL, n=args.precision_n,
                                                        x_shock=0.14)
    if not args.no_cpu_baseline:
        log("[bench] CPU baseline: oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(wl, methods=() if args.no_methods else METHODS)
        log(f"[bench]   {out['cpu_baseline']['value']:.4g} cell-updates/s on "
            f"{out['cpu_baseline']['cores']} threads ({out['cpu_baseline']['host']})")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
