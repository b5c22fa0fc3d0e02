"""Benchmark: CTU + PPMC + exact-Riemann steps on one MI355X.

Workload: plain FP64 shock-cloud at 256^3 on [0,1]^3 (ambient rho = p = 1, gamma = 5/3,
uniform cloud of radius 0.1 at (0.3, 0.5, 0.5) with density contrast 10, Mach-10 plane
shock with the exact Rankine-Hugoniot post-shock state for x < 0.1, outflow boundaries,
CFL 0.3), advanced with the device-side time step.  After `warmup` untimed steps, exactly
`steps` steps are timed with the state resident in HBM; value = real cells x steps / time.
The FP32 form (FP32 state, reconstruction and fluxes, FP64 Newton solve) is timed on the
same workload and reported beside it, with its relative L1 distance from the FP64 state.

Beside the primary line's value, the same JSON line carries
  batched: 64 periodic Kelvin-Helmholtz grids with per-axis edges drawn from
           {32, 48, 64, 96, 128}, 200 steps each with its own device-side time step, every pass
           one launch over all grids, replayed from a captured HIP graph; FP64 and FP32, and
           the same grids advanced one after another for comparison;
  serve:   Poisson-arriving shock-cloud requests (edges {64, 96, 128, 192}, density contrast
           log-uniform in [10, 1000], Mach uniform in [1.5, 10], radius in [0.08, 0.15], run
           to 1.5 cloud-crushing times, FP32 with the FP64 Newton solve) admitted by HBM
           footprint (2 GB budget) into a continuous batch, least estimated work first
           (--serve-policy fifo: arrival order): p50/p99 time-to-solution and aggregate rate;
  methods: the same 256^3 workload with PPMC + Roe/HLLE, PPMC + Roe with the H correction,
           PPMP + exact, PPMP + Roe/HLLE and PPMP + Roe with the H correction, both
           precisions (--no-methods skips them and the next leg);
  workloads: the primary step on the 256^3 turbulent cloud and Kelvin-Helmholtz layer;
  cpu_baseline: the serial FP64 oracle on a bounded sample of the same state;
  roofline: the dominant kernel against the HBM and FP vector peaks, with its measured
           traffic (committed counters) and what plain streaming kernels reach here.
--precision-study runs the 512^3 turbulent cloud for 50 steps in FP64 and FP32 and reports
their relative L1 distance (also with the shock started at x = 0.14, where it reaches the
cloud within the 50 steps); --serve-sweep sweeps the serving arrival rate under both
admission policies.

Prints one JSON line.  Per-kernel durations come from HIP events the library records on
its own stream around every kernel of the timed steps.
"""
import argparse
import json
import os
import sys
import time

REPO = os.path.dirname(os.path.abspath(__file__))
if REPO not in sys.path:
    sys.path.insert(0, REPO)

METRIC = "cell-updates/s at 256^3 (FP64 vs FP32 CTU+PPM+exact); serve p50/p99 latency"
HBM_PEAK_GBS = 8000.0
FP64_VECTOR_PEAK_TFLOPS = 78.6    # 256 CUs x 4 SIMDs x 16 lanes x 2 (FMA) x 2.4 GHz
FP32_VECTOR_PEAK_TFLOPS = 157.3
TRAFFIC_FILE = os.path.join(REPO, "profiles", "traffic_shock_cloud_256.json")

# Algorithmic floating-point operations per unit of work, counted operation by operation
# along the paper's formulas (+, -, *, /, sqrt, pow, min, max, abs each count one), for the
# common path: subsonic cell, one Newton iteration with both sides on the rarefaction branch.
#   primitive conversion 12, slope step (App. A.2) 103, parabola + monotonicity + tracing
#   (App. A.3) 419, two conversions to conserved 24  -> one cell's traced states: 558
#   exact Riemann solve (App. B.1): primitives 24, sound speeds 6, PVRS 9, TSRS 19, one
#   Newton iteration 32, final f 12, u* 4, sampling 6, flux 16 -> 128
#   transverse correction (eq. transverse_evolution) of one cell: 30
#   update (eq. conserved_update) 45 + CFL bound of the new state 26 -> 71
FLOPS_FACE_STAGE1 = 558 + 128
FLOPS_FACE_STAGE2 = 558 + 30 + 128
FLOPS_CELL_UPDATE = 71

# Algorithmic HBM values (elements of the state's type) per unit of work: what the kernel
# must read and write once, with stencil and neighbour reuse counted once.
#   sweep1_d (per face): read the 5 conserved fields of a cell, write the 5 per-cell
#             differences of the first-stage fluxes
#   sweep2_y/z (per face): read 5 fields and the two transverse first-stage differences
#             (10), write the 5 per-cell differences of the CTU fluxes
#   sweep2_x_update (per cell): read 5 fields, the two transverse first-stage differences
#             (10) and the y and z CTU differences (10), write the new state (5)
#   bc_fill (per ghost cell): read and write 5 fields
VALUES_PER_UNIT = {"sweep1": 10, "sweep2": 20, "sweep2_x_update": 30, "bc": 10}


# the paper's other reconstruction and Riemann solvers, timed on the same workload
METHODS = [("ppmc_roe", dict(riemann=1)), ("ppmc_roe_hcorr", dict(riemann=1, h_correction=1)),
           ("ppmp_exact", dict(recon=1)), ("ppmp_roe", dict(recon=1, riemann=1)),
           ("ppmp_roe_hcorr", dict(recon=1, riemann=1, h_correction=1))]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _work(cls, n, ng=3):
    """(units, flops, HBM values) of one launch of a kernel class on an n grid with ng ghost
    layers (flops: exact-solver path only)."""
    nx, ny, nz = n
    d = {"x": 0, "y": 1, "z": 2}
    if cls.startswith("sweep1"):
        e = [nx + 2, ny + 2, nz + 2]
        e[d[cls[-1]]] = n[d[cls[-1]]] + 1
        u = e[0] * e[1] * e[2]
        return u, FLOPS_FACE_STAGE1 * u, VALUES_PER_UNIT["sweep1"] * u
    if cls == "sweep2_x_update":
        cells = nx * ny * nz
        faces = (nx + 1) * ny * nz
        return cells, FLOPS_FACE_STAGE2 * faces + FLOPS_CELL_UPDATE * cells, \
            VALUES_PER_UNIT["sweep2_x_update"] * cells
    if cls.startswith("sweep2"):
        e = [nx, ny, nz]
        e[d[cls[-1]]] += 1
        u = e[0] * e[1] * e[2]
        return u, FLOPS_FACE_STAGE2 * u, VALUES_PER_UNIT["sweep2"] * u
    if cls.startswith("bc_fill"):
        N = [nx + 2 * ng, ny + 2 * ng, nz + 2 * ng]
        N[d[cls[-1]]] = 2 * ng
        u = N[0] * N[1] * N[2]
        return u, 0, VALUES_PER_UNIT["bc"] * u
    if cls == "ppmp_coef":  # one launch per axis; per cell: read 5 fields, write 2
        u = (nx + 2) * (ny + 2) * (nz + 2)
        return u, 0, 7 * u
    if cls == "hcorr_eta":  # per face: 5 fields + 10 differences read, eta written; the
        # class times the x and z passes (the y sweep computes eta along y itself), so one
        # launch carries half of their faces
        u = ((nx + 1) * (ny + 2) * (nz + 2) + (nx + 2) * (ny + 2) * (nz + 1)) // 2
        return u, 0, 16 * u
    if cls == "dt_final":
        u = (ny * nz + 3) // 4
        return u, u, u
    return 0, 0, 0


def run_gpu(wl, prec, steps, warmup, ctu, torch, keep_state=False, newton_hist=False, **method):
    g = ctu.Grid.from_workload(wl, prec=prec, **method)
    g.advance(warmup)
    torch.cuda.synchronize()
    g.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.advance(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = g.profile_read()
    g.profile_enable(False)
    status, flags, counters = g.check()
    info = g.info()
    out = {"seconds": t1 - t0, "profile": prof, "status": status, "flags": flags,
           "counters": counters, "t": info.t, "steps_done": info.steps}
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
    grids = [ctu.Grid.from_workload(w, prec=prec) for w in wls]
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


def _source_hash():
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(REPO, "paper_1410_4194_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".hpp", ".cpp")):
            with open(os.path.join(csrc, f), "rb") as fh:
                h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def _traffic(cls, prec_name):
    """HBM bytes per launch from committed rocprofv3 FETCH_SIZE/WRITE_SIZE counters, scaled
    by the plain-copy calibration; None when the kernels changed since they were taken."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("source_hash") != _source_hash():
        return None
    k = t.get(prec_name, {}).get(cls)
    if not k:
        return None
    return round(k["fetch_kib"] * t["fetch_scale"] * 1024 + k["write_kib"] * t["write_scale"] * 1024)


def roofline(prof, n, eb, prec_name, ng=3, exact=True):
    """Roofline of the dominant kernel class (by total time over the timed steps): achieved
    algorithmic flops and algorithmic bytes per second against the FP vector peak and the HBM
    peak; `bound` is the resource the kernel comes closer to.  The flop counts hold for the
    exact-solver PPMC path only; other methods report the HBM side alone."""
    cls, (ms, launches) = max(((k, v) for k, v in prof.items() if v[1] > 0),
                              key=lambda kv: kv[1][0])
    avg_s = ms / launches / 1e3
    units, flops, values = _work(cls, n, ng)
    if not exact:
        hbm_frac = values * eb / avg_s / 1e9 / HBM_PEAK_GBS
        return {"bound": "hbm", "achieved": round(values * eb / avg_s / 1e9, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(hbm_frac, 4),
                "traffic": None, "kernel": cls, "avg_launch_ms": round(ms / launches, 4),
                "launches": launches, "units_per_launch": units,
                "algorithmic_bytes_per_launch": values * eb, "flops": None}
    peak_alu = FP64_VECTOR_PEAK_TFLOPS if eb == 8 else FP32_VECTOR_PEAK_TFLOPS
    alu = {"achieved": round(flops / avg_s / 1e12, 3), "peak": peak_alu, "unit": "TFLOP/s",
           "frac": round(flops / avg_s / 1e12 / peak_alu, 4), "flops_per_launch": flops}
    hbm = {"achieved": round(values * eb / avg_s / 1e9, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(values * eb / avg_s / 1e9 / HBM_PEAK_GBS, 4)}
    traffic = _traffic(cls, prec_name)
    if traffic:
        hbm["measured_GBps"] = round(traffic / avg_s / 1e9, 1)
    bound, other = ("alu", "hbm") if alu["frac"] >= hbm["frac"] else ("hbm", "alu")
    main = alu if bound == "alu" else hbm
    out = {"bound": bound, "achieved": main["achieved"], "peak": main["peak"],
           "unit": main["unit"], "frac": main["frac"], "traffic": traffic,
           "kernel": cls, "avg_launch_ms": round(ms / launches, 4), "launches": launches,
           "units_per_launch": units, "algorithmic_bytes_per_launch": values * eb,
           other: alu if other == "alu" else hbm}
    return out


def bandwidth_probe(torch, gib=2, reps=5):
    """What plain streaming kernels reach on this GPU's HBM (torch's own kernels, nothing of
    the method): a read-only sum, a copy (1 read : 1 write) and an add of two arrays into a
    third (2 : 1), each over `gib` GiB per array, the best of `reps` launches timed with HIP
    events.  Context for the roofline fraction, which stays against the published peak."""
    n = (gib << 30) // 8
    a = torch.empty(n, dtype=torch.float64, device="cuda").uniform_()
    b = torch.empty_like(a).uniform_()
    c = torch.empty_like(a)

    def best(fn, nbytes):
        fn()
        torch.cuda.synchronize()
        times = []
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            e1.synchronize()
            times.append(e0.elapsed_time(e1) / 1e3)
        return round(nbytes / min(times) / 1e9, 1)

    nb = n * 8
    out = {"read_GBps": best(lambda: a.sum(), nb), "copy_GBps": best(lambda: c.copy_(a), 2 * nb),
           "add_GBps": best(lambda: torch.add(a, b, out=c), 3 * nb), "bytes_per_array": nb}
    del a, b, c
    torch.cuda.empty_cache()
    return out


def cpu_baseline(wl, seconds_target=15.0, methods=(), method_seconds=3.0):
    """The serial FP64 oracle on a bounded sample of the same workload: one CTU step of a 64^3
    box around the shock front and the cloud's upwind edge, repeated for about
    `seconds_target`; then the same box with each of `methods` ((name, config keywords)),
    about `method_seconds` each."""
    import oracle as O

    lo, hi, cells = (0, 96, 96), (64, 160, 160), 64 ** 3

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

    v, reps, t_total = rate(seconds_target)
    out = {"value": round(v, 1), "unit": "cell-updates/s", "cores": 1, "kind": "oracle",
           "sample": f"{reps} x one CTU step of the 64^3 box [0,64)x[96,160)x[96,160) of the "
                     f"256^3 shock-cloud initial state, serial FP64 C oracle, {t_total:.1f} s"}
    if methods:
        out["methods"] = {}
        for name, kw in methods:
            vm, rm, tm = rate(method_seconds, **kw)
            log(f"[bench]   oracle {name}: {vm:.4g} cell-updates/s ({rm} steps of the box)")
            out["methods"][name] = {"value": round(vm, 1), "steps": rm, "seconds": round(tm, 1)}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
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
                    help="admission policy of the default serving run")
    ap.add_argument("--serve-sweep", action="store_true",
                    help="also sweep the arrival rate over 0.25, 0.5, 1, 2, 4 x capacity, "
                         "with both admission policies")
    ap.add_argument("--precision-study", action="store_true",
                    help="512^3 turbulent cloud, 50 steps, FP32 vs FP64 relative L1")
    ap.add_argument("--source-hash", action="store_true",
                    help="print the hash of the kernel sources that traffic figures are tied to")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run only a plain device copy of 2 GiB x 5 (counter calibration)")
    args = ap.parse_args()
    if args.source_hash:
        print(_source_hash())
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the CTU step shards by block decomposition, which this build does not run)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_probe:
        # plain copy kernel of known size: 2 GiB read + 2 GiB written per launch
        src = torch.empty(2 << 30, dtype=torch.uint8, device="cuda").random_(0, 255)
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("[bench] copy probe: 5 launches of a 2 GiB device-to-device copy")
        return
    from paper_1410_4194_amd import ctu, workloads as WL

    log(f"[bench] building shock-cloud {args.n}^3 initial state")
    wl = WL.shock_cloud(args.n, steps=args.steps)
    n = (wl.nx, wl.ny, wl.nz)
    cells = wl.cells

    log(f"[bench] FP64: warmup {args.warmup}, timed {args.steps} steps")
    r64 = run_gpu(wl, ctu.FP64, args.steps, args.warmup, ctu, torch, keep_state=not args.no_fp32,
                  newton_hist=True)
    v64 = cells * args.steps / r64["seconds"]
    log(f"[bench] FP64 {v64:.4g} cell-updates/s, {1e3 * r64['seconds'] / args.steps:.3f} ms/step")
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
                   "newton_caps": r64["counters"][1], "status": r64["status"],
                   "newton_iterations_per_solve": r64.get("newton_hist")},
        "roofline": roofline(r64["profile"], n, 8, "fp64"),
        "kernels_ms": {k: round(v[0] / max(v[1], 1), 4) for k, v in r64["profile"].items()
                       if v[1] > 0},
    }
    bw = bandwidth_probe(torch)
    log(f"[bench] plain streaming kernels on this GPU (GB/s): {bw}")
    out["roofline"]["achievable"] = bw
    if not args.no_fp32:
        log(f"[bench] FP32 form: warmup {args.warmup}, timed {args.steps} steps")
        r32 = run_gpu(wl, ctu.FP32, args.steps, args.warmup, ctu, torch, keep_state=True)
        v32 = cells * args.steps / r32["seconds"]
        log(f"[bench] FP32 {v32:.4g} cell-updates/s")
        l1 = rel_l1(r32.pop("state"), r64.pop("state"), wl.gamma)
        log(f"[bench] FP32 vs FP64 relative L1 after {args.warmup + args.steps} steps: {l1}")
        out["fp32"] = {"value": round(v32, 1), "unit": "cell-updates/s",
                       "ms_per_step": round(1e3 * r32["seconds"] / args.steps, 4),
                       "vs_fp64": round(v32 / v64, 3),
                       "rel_l1_vs_fp64": [float(f"{e:.3e}") for e in l1],
                       "t_minus_t_fp64": r32["t"] - r64["t"],
                       "roofline": roofline(r32["profile"], n, 4, "fp32")}
    if not args.no_methods:
        # the other reconstruction and Riemann solvers of the paper on the same workload
        out["methods"] = {}
        for mname, kw in METHODS:
            ng = (4 if kw.get("recon") else 3) + kw.get("h_correction", 0)
            for pname, prec, eb in (("fp64", ctu.FP64, 8), ("fp32", ctu.FP32, 4)):
                log(f"[bench] method {mname} {pname}: warmup {args.warmup}, timed {args.method_steps} steps")
                rm = run_gpu(wl, prec, args.method_steps, args.warmup, ctu, torch, **kw)
                vm = cells * args.method_steps / rm["seconds"]
                log(f"[bench]   {vm:.4g} cell-updates/s, status {rm['status']}, "
                    f"HLLE substitutions {rm['counters'][3]}")
                out["methods"][f"{mname}_{pname}"] = {
                    "value": round(vm, 1), "unit": "cell-updates/s", "steps": args.method_steps,
                    "ms_per_step": round(1e3 * rm["seconds"] / args.method_steps, 4),
                    "vs_ppmc_exact": round(vm / (v64 if prec == ctu.FP64 else
                                                 out.get("fp32", {}).get("value", v64)), 3),
                    "status": rm["status"], "hlle_substitutions": rm["counters"][3],
                    "roofline": roofline(rm["profile"], n, eb, pname, ng=ng, exact=False),
                    "kernels_ms": {k: round(v[0] / max(v[1], 1), 4)
                                   for k, v in rm["profile"].items() if v[1] > 0}}
    if not args.no_methods:
        # the primary step on states with structure everywhere: equal face states (which skip
        # the Newton solve) are the common case in the shock-cloud's ambient gas, rarer here
        out["workloads"] = {}
        for wname, wmake in (("turbulent_cloud_256^3", lambda: WL.turbulent_cloud(args.n)),
                             ("kelvin_helmholtz_256^3", lambda: WL.kelvin_helmholtz(args.n, args.n, args.n))):
            wl2 = wmake()
            log(f"[bench] workload {wname} fp64: warmup {args.warmup}, timed {args.method_steps} steps")
            rw = run_gpu(wl2, ctu.FP64, args.method_steps, args.warmup, ctu, torch, newton_hist=True)
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
        runs = [(args.serve_load, args.serve_policy)]
        if args.serve_sweep:
            runs += [(ld, pol) for ld in (0.25, 0.5, 1.0, 2.0, 4.0) for pol in ("fifo", "sjf")]
        for i, (load, policy) in enumerate(runs):
            rate = load * capacity
            log(f"[bench] serving ({policy}): {args.serve_requests} requests at {rate:.3f}/s "
                f"({load} x estimated capacity {capacity:.3f}/s)")
            rs = run_serve(ctu, WL, rate, args.serve_requests, budget, WL.BASE_SEED + 5,
                           policy=policy)
            rs["load"] = load
            rs["capacity_estimate_per_s"] = round(capacity, 4)
            log(f"[bench]   p50 {rs['p50_s']} s, p99 {rs['p99_s']} s, "
                f"{rs['cell_updates_per_s']:.4g} cell-updates/s")
            if i == 0:
                out["serve"] = rs
            else:
                out.setdefault("serve_sweep", []).append(rs)
    if args.precision_study:
        log("[bench] precision study: 512^3 turbulent cloud, 50 steps, FP64 and FP32")
        out["precision_study"] = precision_study(ctu, torch, WL)
        # the same with the shock started 0.01 from the cloud edge, so that it hits the cloud
        # within the 50 steps and the flow turns three-dimensional
        log("[bench] precision study, active variant: shock at x = 0.14")
        out["precision_study_active"] = precision_study(ctu, torch, WL, x_shock=0.14)
    if not args.no_cpu_baseline:
        log("[bench] CPU baseline: oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(wl, methods=() if args.no_methods else METHODS)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
