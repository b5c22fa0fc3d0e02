"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

One step from the same seeded input and the same dt, compared field by field with the
relative L1 metric of tests.common.rel_l1 (FP64 <= 1e-12, FP32 <= 1e-5) and cell by cell,
each cell against its own scale (tests.common.elem_err: FP64 <= 1e-10, FP32 <= 1e-4).
Per-pass checks compare the first-stage and CTU flux differences on every cell the step
computes, also cell by cell.  Workloads span
several tiles and ragged sizes, both boundary types, and the degenerate shapes (1-cell
axes, tiny grids).
"""
import math
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import oracle as O
from paper_1410_4194_amd import workloads as WL
from tests.common import (ELEM32, ELEM64, TOL32, TOL64, assert_parity, cell_scales,
                          oracle_config, oracle_state, parity_bounds, rel_l1, run_oracle)

# per-cell bound of multi-step FP64 runs, where rounding differences between the two
# implementations grow at discontinuities over the steps
MULTI64 = 1e-8


@pytest.fixture(scope="module")
def ctu():
    from paper_1410_4194_amd import ctu as _ctu
    return _ctu


def _announce(*parts):
    print("[gpu-test]", *parts, flush=True)
    sys.stdout.flush()


def _one_step(ctu, wl, prec, dt=None):
    cfg = oracle_config(wl)
    u = oracle_state(wl, cfg)
    if dt is None:
        dt = O.compute_dt(cfg, u)
    _announce(wl.name, "prec", prec, "cells", wl.cells, "dt", dt)
    g = ctu.Grid.from_workload(wl, prec=prec)
    g.step(dt)
    gpu = g.get_state()
    ref_u = u.copy()
    O.step(cfg, ref_u, dt)
    return g, gpu, O.real(cfg, ref_u), cfg, u, dt


CASES = [
    ("rough_periodic_37x11x9", lambda: WL.random_state(37, 11, 9, seed=11, spacing=(1.0, 0.5, 0.4))),
    ("rough_outflow_20x17x13", lambda: WL.random_state(20, 17, 13, seed=12, bc=(1,) * 6)),
    ("rough_mixed_70x6x5", lambda: WL.random_state(70, 6, 5, seed=13, bc=(1, 1, 0, 0, 1, 1))),
    ("smooth_supersonic_24x20x18", lambda: WL.random_state(24, 20, 18, seed=14, rough=False, mach=3.0)),
    ("sod_128x16x16", lambda: WL.sod(128, 16, 16)),
    ("sod_y_8x64x8", lambda: WL.sod(64, 8, 8, axis=1)),
    ("shock_cloud_48", lambda: WL.shock_cloud(48, steps=1)),
    ("kh_33x27x19", lambda: WL.kelvin_helmholtz(33, 27, 19)),
    ("one_cell_axes_64x1x1", lambda: WL.random_state(64, 1, 1, seed=15)),
    ("one_cell_axis_1x9x7", lambda: WL.random_state(1, 9, 7, seed=16, bc=(0, 0, 1, 1, 1, 1))),
    ("tiny_2x2x2", lambda: WL.random_state(2, 2, 2, seed=17)),
    ("single_cell", lambda: WL.random_state(1, 1, 1, seed=18)),
]


# gamma outside the compiled gas classes (5/3, 7/5): the general kernels, with the runtime
# integer root (gamma = 9/7: 2g/(g-1) = 9; gamma = 2: 4) or the general powers (gamma = 1.3)
GAMMA_CASES = [
    ("rough_gamma_1.3_19x13x11", lambda: WL.random_state(19, 13, 11, seed=19, gamma=1.3)),
    ("rough_gamma_9_7_17x12x10",
     lambda: WL.random_state(17, 12, 10, seed=20, gamma=9.0 / 7.0, bc=(1,) * 6)),
    ("smooth_gamma_2_15x10x9",
     lambda: WL.random_state(15, 10, 9, seed=21, gamma=2.0, rough=False, mach=2.0)),
]


@pytest.mark.parametrize("name,make", GAMMA_CASES, ids=[c[0] for c in GAMMA_CASES])
@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32"])
def test_one_step_general_gamma(ctu, name, make, prec):
    wl = make()
    g, gpu, ref, cfg, u0, dt = _one_step(ctu, wl, prec)
    assert_parity(gpu, ref, wl.gamma, *parity_bounds(prec), what=(name, prec))
    status, flags, counters = g.check()
    assert status == ctu.OK, (flags, counters)


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_one_step_fp64(ctu, name, make):
    wl = make()
    g, gpu, ref, cfg, u0, dt = _one_step(ctu, wl, ctu.FP64)
    assert_parity(gpu, ref, wl.gamma, TOL64, ELEM64, what=(name, "fp64"))
    status, flags, counters = g.check()
    assert status == ctu.OK, (flags, counters)


@pytest.mark.parametrize("name,make", CASES[:8], ids=[c[0] for c in CASES[:8]])
def test_one_step_fp32(ctu, name, make):
    wl = make()
    g, gpu, ref, cfg, u0, dt = _one_step(ctu, wl, ctu.FP32)
    assert gpu.dtype == np.float32
    assert_parity(gpu, ref, wl.gamma, TOL32, ELEM32, what=(name, "fp32"))


def _flux_err(gpu_f, ref_f, u, gamma):
    """Relative L1 per field over the cells the oracle computed, and the largest per-cell
    error against the cell's flux scale (its field scale times its signal speed |V| + a)."""
    mask = np.isfinite(ref_f[0])
    scales, speed = cell_scales(u, gamma)
    errs, cells = [], []
    for f in range(5):
        d = np.abs(gpu_f[f][mask] - ref_f[f][mask])
        num = d.sum()
        den = np.abs(ref_f[f][mask]).sum()
        errs.append(0.0 if num == 0.0 else num / max(den, 1e-300))
        cells.append(float(np.max(d / (scales[f][mask] * speed[mask]))))
    return np.array(errs), np.array(cells), int(mask.sum())


def _cell_diff(F, d):
    """Per-cell flux differences F(c-1/2) - F(c+1/2) along axis d of face arrays that hold
    face c+1/2 at index c, shape (5, NZ, NY, NX); NaN where a face is missing."""
    ax = {0: 2, 1: 1, 2: 0}[d]
    D = np.full_like(F, np.nan)
    for f in range(5):
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[ax] = slice(None, -1)
        hi[ax] = slice(1, None)
        D[f][tuple(hi)] = F[f][tuple(lo)] - F[f][tuple(hi)]
    return D


@pytest.mark.parametrize("name,make", [CASES[0], CASES[2], CASES[6]], ids=[CASES[0][0], CASES[2][0], CASES[6][0]])
def test_per_pass_fluxes_fp64(ctu, name, make):
    wl = make()
    cfg = oracle_config(wl)
    u = oracle_state(wl, cfg)
    dt = O.compute_dt(cfg, u)
    O.bc_fill(cfg, u)
    _, _, fstar, fhalf = O.update_box(cfg, u, dt, (0, 0, 0), (wl.nx, wl.ny, wl.nz), want_fluxes=True)
    _announce(name, "per-pass")
    g = ctu.Grid.from_workload(wl, prec=ctu.FP64)
    with pytest.raises(ctu.CtuError):  # not stored unless asked for
        g.debug_fluxes(1, 0)
    g.debug_keep_fluxes(True)
    g.step(dt)
    for d in range(3):  # the step keeps per-cell differences of each pass's fluxes
        e1, c1, n1 = _flux_err(g.debug_fluxes(0, d), _cell_diff(fstar[d], d), u, wl.gamma)
        e2, c2, n2 = _flux_err(g.debug_fluxes(1, d), _cell_diff(fhalf[d], d), u, wl.gamma)
        print(f"[parity] {name} dir {d}: F* L1 {e1.max():.2e} cell {c1.max():.2e}; "
              f"F^(n+1/2) L1 {e2.max():.2e} cell {c2.max():.2e}", flush=True)
        assert n1 > 0 and n2 > 0
        assert e1.max() <= TOL64 and c1.max() <= ELEM64, ("F*", d, e1, c1)
        assert e2.max() <= TOL64 and c2.max() <= ELEM64, ("F^{n+1/2}", d, e2, c2)
    # keeping the fluxes changes nothing else
    g2 = ctu.Grid.from_workload(wl, prec=ctu.FP64)
    g2.step(dt)
    assert np.array_equal(g2.get_state(), g.get_state())


def test_compute_dt_matches_oracle(ctu):
    for wl in (WL.random_state(19, 13, 7, seed=21), WL.shock_cloud(32, steps=1), WL.sod(64, 4, 4)):
        cfg = oracle_config(wl)
        ref = O.compute_dt(cfg, oracle_state(wl, cfg))
        for prec, tol in ((ctu.FP64, 1e-14), (ctu.FP32, 1e-6)):
            g = ctu.Grid.from_workload(wl, prec=prec)
            assert g.compute_dt() == pytest.approx(ref, rel=tol)


def test_totals_are_exact_sums(ctu):
    wl = WL.random_state(40, 30, 20, seed=22)
    g = ctu.Grid.from_workload(wl, prec=ctu.FP64)
    g.step(g.compute_dt())
    st = g.get_state()
    tot = g.totals()
    for f in range(5):
        exact = math.fsum(st[f].ravel())
        scale = math.fsum(np.abs(st[f]).ravel())
        assert abs(tot[f] - exact) <= 1e-13 * scale


def test_periodic_conservation_on_gpu(ctu):
    wl = WL.kelvin_helmholtz(48, 40, 32)
    g = ctu.Grid.from_workload(wl, prec=ctu.FP64)
    before = g.totals()
    g.advance(20)
    after = g.totals()
    st = g.get_state()
    for f in range(5):
        scale = math.fsum(np.abs(st[f]).ravel())
        assert abs(after[f] - before[f]) <= 1e-13 * max(scale, 1.0), f


def test_determinism_bitwise(ctu):
    wl = WL.shock_cloud(40, steps=1)
    out = []
    for _ in range(2):
        g = ctu.Grid.from_workload(wl, prec=ctu.FP64)
        g.advance(5)
        out.append(g.get_state())
    assert np.array_equal(out[0], out[1])


def test_invalid_step_arguments_change_nothing(ctu):
    """ctu_step with dt <= 0, NaN or infinite dt, and ctu_advance with a negative step count
    or a NaN end time are refused with CTU_EINVAL before any device work; the state, time and
    step count stay as they were, and a valid step afterwards still matches the oracle."""
    wl = WL.random_state(12, 10, 9, seed=61)
    g = ctu.Grid.from_workload(wl, prec=ctu.FP64)
    before = g.get_state()
    for dt in (0.0, -1e-3, float("nan"), float("inf")):
        with pytest.raises(ctu.CtuError) as ei:
            g.step(dt)
        assert ei.value.status == ctu.EINVAL, dt
    for nsteps, t_end in ((-1, float("inf")), (3, float("nan"))):
        with pytest.raises(ctu.CtuError) as ei:
            g.advance(nsteps, t_end=t_end)
        assert ei.value.status == ctu.EINVAL
    g.advance(0)
    assert np.array_equal(g.get_state(), before)
    info = g.info()
    assert info.steps == 0 and info.t == 0.0
    cfg = oracle_config(wl)
    u = oracle_state(wl, cfg)
    dt = O.compute_dt(cfg, u)
    g.step(dt)
    O.step(cfg, u, dt)
    assert_parity(g.get_state(), O.real(cfg, u), wl.gamma, TOL64, ELEM64, what="after refusals")


def test_advance_equals_host_loop(ctu):
    """Device-side dt (ctu_advance) gives bitwise the same steps as compute_dt + step."""
    wl = WL.sod(64, 4, 4)
    g1 = ctu.Grid.from_workload(wl, prec=ctu.FP64)
    g1.advance(10, t_end=0.2)
    g2 = ctu.Grid.from_workload(wl, prec=ctu.FP64)
    for _ in range(10):
        g2.step(g2.compute_dt())
    assert np.array_equal(g1.get_state(), g2.get_state())
    assert g1.info().t == g2.info().t and g1.info().steps == 10


def test_sod_to_t02_matches_oracle_and_exact(ctu):
    """BJ config 1: 3D Sod 128x16x16, outflow x / periodic y,z, to t = 0.2."""
    wl = WL.sod(128, 16, 16)
    g = ctu.Grid.from_workload(wl, prec=ctu.FP64)
    g.advance(10000, t_end=0.2)
    info = g.info()
    assert info.t == pytest.approx(0.2, abs=1e-14)
    st = g.get_state()
    cols = st[0].reshape(-1, 128)
    assert np.all(cols == cols[0])  # every (y, z) column identical
    wl1 = WL.sod(128, 1, 1)
    cfg1, u1, t1, n1 = run_oracle(wl1, t_end=0.2)
    assert n1 == info.steps
    ref = O.real(cfg1, u1)[:, 0, 0, :]
    # ~100 steps: rounding differences grow at the shock and contact
    assert_parity(st[:, 0, 0, :], ref, 1.4, 1e-10, MULTI64, what="sod to t=0.2")
    x = (np.arange(128) + 0.5) / 128
    ex = O.exact_solution((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), 1.4, (x - 0.5) / 0.2)
    assert np.mean(np.abs(st[0, 0, 0] - ex[0])) < 0.003


def test_nonphysical_state_is_reported(ctu):
    wl = WL.random_state(16, 8, 8, seed=23)
    g = ctu.Grid.from_workload(wl, prec=ctu.FP64)
    U = g.get_state()
    U[0, 3, 4, 5] = np.nan
    g.set_state(U)
    g.step(1e-3)
    status, flags, counters = g.check()
    assert status == ctu.ENONPHYS and flags & ctu.FLAG_NONFINITE and counters[2] > 0
    status, flags, counters = g.check()  # cleared
    assert flags == 0


def test_newton_cap_is_counted(ctu):
    wl = WL.sod(32, 2, 2)
    from paper_1410_4194_amd.ctu import make_config, Grid
    cfg = make_config(wl.nx, wl.ny, wl.nz, wl.dx, wl.dy, wl.dz, wl.gamma, wl.bc,
                      newton_max_iter=1)
    g = Grid(cfg)
    g.set_primitive(wl.W)
    g.step(g.compute_dt())
    status, flags, counters = g.check()
    assert status == ctu.ENOCONV and counters[1] > 0



@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32"])
def test_march_segments_do_not_change_results(ctu, prec):
    """The tile shape of the marching sweeps (faces per thread segment, including one-face
    segments and one segment per column) changes the launch; the result changes only by
    rounding (a segment's first trace is a separately compiled copy of the same formulas,
    whose multiply-adds the compiler may fuse differently), well inside the parity bound."""
    wl = WL.random_state(12, 37, 29, seed=77, bc=(0, 0, 1, 1, 0, 0))
    _announce("march segments", prec)
    ref = None
    for seg in ((0, 0), (1, 1), (5, 7), (38, 30), (64, 64)):
        cfg = ctu.make_config(wl.nx, wl.ny, wl.nz, wl.dx, wl.dy, wl.dz, wl.gamma, wl.bc, prec,
                              wl.cfl, march_seg=seg)
        g = ctu.Grid(cfg)
        g.set_primitive(wl.W)
        g.advance(3)
        U = g.get_state()
        g.close()
        if ref is None:
            ref = U
        else:
            assert_parity(U, ref, wl.gamma, *parity_bounds(prec), what=("segments", seg, prec))


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32"])
def test_x_tile_shapes_are_bitwise_invariant(ctu, prec):
    """The x sweeps' tile shapes (x-rows per wavefront of the fused update, 1..8, and chunks
    per wavefront of the first-stage x sweep, 1..16) change only which wavefront computes a
    cell, never its arithmetic: the state after three steps is bitwise the same, on short
    rows (several per wavefront) and ragged sizes."""
    _announce("x tile shapes", prec)
    for wl in (WL.random_state(12, 37, 29, seed=78, bc=(0, 0, 1, 1, 0, 0)),
               WL.random_state(70, 6, 5, seed=79, bc=(1, 1, 0, 0, 1, 1))):
        ref = None
        for rows, chunks in ((0, 0), (1, 1), (2, 3), (3, 16), (8, 2), (5, 7)):
            cfg = ctu.make_config(wl.nx, wl.ny, wl.nz, wl.dx, wl.dy, wl.dz, wl.gamma, wl.bc,
                                  prec, wl.cfl, march_seg=(0, 0), x_rows=rows, x_chunks=chunks)
            g = ctu.Grid(cfg)
            g.set_primitive(wl.W)
            g.advance(3)
            U = g.get_state()
            status, flags, counters = g.check()
            g.close()
            assert status == ctu.OK, (flags, counters)
            if ref is None:
                ref = U
            else:
                assert np.array_equal(U, ref), (wl.name, rows, chunks)


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32"])
def test_overlapped_passes_are_bitwise_serial(ctu, prec):
    """The overlapped schedule (the first-stage y and second-stage z sweeps on the grid's
    side stream) changes only when a pass runs, never its arithmetic: after three device-dt
    steps and two host-dt steps the state is bitwise that of every pass in order on one
    stream, for the exact solver (integer and general gamma), the Roe solver, PPMP and the H
    correction, and with per-kernel timing on (which runs the passes in order).  The fused-z
    schedule (the first-stage y sweep on the side, then both z stages in one march) solves
    the same faces with a separately compiled copy of the same formulas, whose multiply-adds
    the compiler may fuse differently: it agrees to rounding, inside the parity bound (the H
    correction takes the overlapped schedule instead, bitwise)."""
    _announce("overlapped passes", prec)
    cases = ((WL.random_state(23, 19, 17, seed=81, bc=(1, 1, 0, 0, 1, 1)), {}),
             (WL.random_state(20, 14, 12, seed=82, gamma=1.3), {"recon": 1}),
             (WL.random_state(18, 21, 13, seed=83), {"riemann": 1}),
             (WL.random_state(19, 16, 14, seed=84, bc=(1,) * 6), {"riemann": 1, "h_correction": 1}),
             (WL.random_state(17, 15, 13, seed=85, rough=False, mach=2.0),
              {"riemann": 1, "h_correction": 1, "recon": 1}),
             (WL.random_state(21, 18, 37, seed=86, bc=(2, 2, 1, 1, 0, 0)), {"recon": 1}),
             (WL.shock_cloud(48), {}))
    runs = ((ctu.SCHEDULE_IN_ORDER, False), (ctu.SCHEDULE_OVERLAP, False),
            (ctu.SCHEDULE_FUSED_Z, False), (ctu.SCHEDULE_AUTO, False),
            (ctu.SCHEDULE_OVERLAP, True), (ctu.SCHEDULE_FUSED_Z, True))
    for wl, kw in cases:
        hcorr = kw.get("h_correction", 0) == 1
        out = []
        for schedule, timing in runs:
            g = ctu.Grid.from_workload(wl, prec=prec, schedule=schedule, **kw)
            want = {ctu.SCHEDULE_AUTO: ctu.SCHEDULE_OVERLAP,
                    ctu.SCHEDULE_FUSED_Z: ctu.SCHEDULE_OVERLAP if hcorr else ctu.SCHEDULE_FUSED_Z
                    }.get(schedule, schedule)
            assert g.info().schedule == want, (schedule, g.info().schedule)
            if timing:
                g.profile_enable(True)
            g.advance(3)
            g.step(0.25 * g.compute_dt())
            g.step(0.25 * g.compute_dt())
            out.append(g.get_state())
            status, flags, counters = g.check()
            g.close()
            assert status == ctu.OK, (wl.name, kw, flags, counters)
        for k in range(1, len(runs)):
            if runs[k][0] == ctu.SCHEDULE_FUSED_Z and not hcorr:
                assert_parity(out[k], out[0], wl.gamma, *parity_bounds(prec),
                              what=("fused z", wl.name, kw, prec))
            else:
                assert np.array_equal(out[k], out[0]), (wl.name, kw, runs[k])


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32"])
def test_overlapped_long_run_is_bitwise_serial(ctu, prec):
    """A race between the two streams of the overlapped schedule (a pass reading data that the
    other stream has not finished writing) would show as a difference from the in-order
    schedule at some step.  At 128^3 the side stream's sweeps really run beside the launch
    stream's, and 200 device-dt steps of the shock-cloud (the shock running into the cloud)
    leave the state, the time and the step count bitwise those of every pass in order."""
    _announce("overlapped long run 128^3", prec)
    wl = WL.shock_cloud(128)
    res = []
    for schedule in (ctu.SCHEDULE_IN_ORDER, ctu.SCHEDULE_OVERLAP):
        g = ctu.Grid.from_workload(wl, prec=prec, schedule=schedule)
        assert g.info().schedule == schedule
        g.advance(200)
        info = g.info()
        status, flags, counters = g.check()
        assert status == ctu.OK, (schedule, flags, counters)
        res.append((g.get_state(), info.t, info.steps))
        g.close()
    assert res[0][2] == res[1][2] == 200
    assert res[0][1] == res[1][1]
    assert np.array_equal(res[0][0], res[1][0])


def test_schedule_choice_by_size(ctu):
    """The library's choice: overlapped for grids of at most CTU_OVERLAP_MAX_CELLS real cells,
    fused z above; with the H correction overlapped while one field array takes at most
    CTU_OVERLAP_MAX_FIELD_BYTES (192 MiB), in order above.  An explicit choice holds."""
    cells_limit = 20 << 20
    bytes_limit = 192 << 20
    for n, prec in ((256, ctu.FP64), (288, ctu.FP64), (256, ctu.FP32), (352, ctu.FP32)):
        cfg = ctu.make_config(n, n, n, 1.0 / n, 1.0 / n, 1.0 / n, 5.0 / 3.0, prec=prec)
        g = ctu.Grid(cfg)
        sched = g.info().schedule
        g.close()
        want = ctu.SCHEDULE_OVERLAP if n ** 3 <= cells_limit else ctu.SCHEDULE_FUSED_Z
        assert sched == want, (n, prec, sched)
        assert (n == 256) == (want == ctu.SCHEDULE_OVERLAP)
    for n in (256, 288):
        cfg = ctu.make_config(n, n, n, 1.0 / n, 1.0 / n, 1.0 / n, 1.4, riemann=ctu.RIEMANN_ROE,
                              h_correction=1)
        g = ctu.Grid(cfg)
        info = g.info()
        g.close()
        small = info.field_stride * info.elem_bytes <= bytes_limit
        assert small == (n == 256), (n, info.field_stride * info.elem_bytes)
        assert info.schedule == (ctu.SCHEDULE_OVERLAP if small else ctu.SCHEDULE_IN_ORDER), n
    for schedule in (ctu.SCHEDULE_IN_ORDER, ctu.SCHEDULE_OVERLAP, ctu.SCHEDULE_FUSED_Z):
        cfg = ctu.make_config(24, 20, 16, 1, 1, 1, 1.4, recon=ctu.RECON_PPMP, schedule=schedule)
        g = ctu.Grid(cfg)
        assert g.info().schedule == schedule
        g.close()


@pytest.mark.parametrize("schedule", [1, 2, 3], ids=["in_order", "overlap", "fused_z"])
def test_newton_histogram_counts_every_solve(ctu, schedule):
    """The instrumented sweeps count one Newton-iteration bin per exact Riemann solve: the
    bins add up to the number of solves a step makes (stage 1 on the extended transverse
    ranges, stage 2 on the real faces), in every schedule (the fused z march counts its
    second-stage solves on the real columns only), and the instrumented step gives the same
    state."""
    wl = WL.random_state(21, 14, 9, seed=5, bc=(1, 1, 0, 0, 1, 1))
    nx, ny, nz = wl.nx, wl.ny, wl.nz
    solves = ((nx + 1) * (ny + 2) * (nz + 2) + (nx + 2) * (ny + 1) * (nz + 2)
              + (nx + 2) * (ny + 2) * (nz + 1)
              + (nx + 1) * ny * nz + nx * (ny + 1) * nz + nx * ny * (nz + 1))
    _announce("newton histogram", schedule)
    plain = ctu.Grid.from_workload(wl, prec=ctu.FP64, schedule=schedule)
    plain.advance(2)
    ref = plain.get_state()
    g = ctu.Grid.from_workload(wl, prec=ctu.FP64, schedule=schedule)
    g.profile_enable(False, newton=True)
    g.advance(2)
    hist = g.newton_histogram()
    assert sum(hist.values()) == 2 * solves, hist
    assert hist["0-1"] + hist["2"] + hist["3"] > 0 and hist["cap"] == 0
    assert_parity(g.get_state(), ref, wl.gamma, TOL64, ELEM64, what="instrumented sweeps")
    capped = ctu.Grid(ctu.make_config(nx, ny, nz, wl.dx, wl.dy, wl.dz, wl.gamma, wl.bc,
                                      newton_max_iter=1, schedule=schedule))
    capped.set_primitive(wl.W)
    capped.profile_enable(False, newton=True)
    capped.step(capped.compute_dt())
    h1 = capped.newton_histogram()
    assert h1["0-1"] + h1["cap"] == solves and h1["cap"] > 0, h1


def test_near_vacuum_rarefaction(ctu):
    """Two streams moving apart faster than their escape speeds open a near-vacuum: with a
    pressure floor of 1e-40 the star pressure falls below the float range of the integer
    root's first estimate (p/p_k < 1e-30), which takes the exactly rescaled branch."""
    wl = WL.riemann_tube((1.0, -20.0, 1.0), (1.0, 20.0, 1.0), n=64, ny=2, nz=2,
                         gamma=5.0 / 3.0, name="vacuum")
    cfg = oracle_config(wl, p_floor=1e-40)
    u = oracle_state(wl, cfg)
    dt = 0.5 * O.compute_dt(cfg, u)
    _announce("near vacuum, dt", dt)
    g = ctu.Grid.from_workload(wl, prec=ctu.FP64, p_floor=1e-40)
    for _ in range(8):  # the scheme itself fails soon after (no density floor)
        g.step(dt)
        O.step(cfg, u, dt)
    gpu = g.get_state()
    ref = O.real(cfg, u)
    assert np.isfinite(ref).all()
    assert_parity(gpu, ref, wl.gamma, TOL64, MULTI64, what="near vacuum, 8 steps")

METHODS = [("ppmc_exact", {}), ("ppmc_roe", dict(riemann=1)),
           ("ppmc_roe_hcorr", dict(riemann=1, h_correction=1)), ("ppmp_exact", dict(recon=1)),
           ("ppmp_roe_hcorr", dict(recon=1, riemann=1, h_correction=1))]


@pytest.mark.parametrize("name,kw", METHODS, ids=[m[0] for m in METHODS])
@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32"])
def test_uniform_flow_is_unchanged_bitwise(ctu, name, kw, prec):
    """A uniform moving state is an exact steady solution: every face has equal states (the
    solvers' constant-state path), every flux difference is exactly zero, and ten steps leave
    the state bit for bit as it was, for every method and boundary type."""
    wl = WL.random_state(23, 17, 12, seed=90, bc=(1, 1, 0, 0, 1, 1))
    wl.W[:] = np.array([1.3, 0.4, -0.2, 0.7, 2.0])[:, None, None, None]
    _announce("uniform flow", name, "prec", prec)
    g = ctu.Grid.from_workload(wl, prec=prec, **kw)
    before = g.get_state()
    g.advance(10)
    assert np.array_equal(g.get_state(), before)
    status, flags, counters = g.check()
    assert status == ctu.OK
