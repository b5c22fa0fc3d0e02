"""Full-size parity: steps of the benchmark workloads on the GPU, checked against the oracle.

* The whole 256^3 shock-cloud grid, every cell, one step from an evolved state (the shock
  started at x = 0.17 has run into the cloud after 90 GPU steps), in FP64 and in the FP32
  form; the oracle runs its OpenMP build for this.
* The same in FP64 under the fused-z schedule (both z stages in one march), which grids above
  20M cells take by default.
* Sampled boxes of one step from the initial states of the 256^3 shock-cloud with every
  method (and under the fused-z schedule for PPMC + Roe and PPMP + exact), of the 512^3
  turbulent cloud (FP32, fused z by default), and of its FP64 steps 25 and 50.

Both sides use the same dt, so the GPU runs the same kernels and launch shapes as the
benchmark.  Every comparison checks the relative L1 norm and every cell against its own
scale (tests.common.assert_parity).
"""
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import oracle as O
from paper_1410_4194_amd import workloads as WL
from tests.common import ELEM32, ELEM64, TOL32, TOL64, assert_parity, oracle_config


def _boxes(n, special, rng, count=6, size=8):
    boxes = []
    for (cx, cy, cz) in special:
        lo = [max(0, min(n - size, c - size // 2)) for c in (cx, cy, cz)]
        boxes.append((tuple(lo), tuple(l + size for l in lo)))
    for _ in range(count):
        lo = [int(v) for v in rng.integers(0, n - size, size=3)]
        boxes.append((tuple(lo), tuple(l + size for l in lo)))
    return boxes


def _check(ctu, wl, prec, tol, special, seed, schedule=0, **method):
    print(f"[gpu-test] full size {wl.name} prec {prec} {method} schedule {schedule}", flush=True)
    cfg = oracle_config(wl, **method)
    u = O.state_from_primitive(cfg, wl.W)
    O.bc_fill(cfg, u)
    dt = O.compute_dt(cfg, u)
    g = ctu.Grid.from_workload(wl, prec=prec, schedule=schedule, **method)
    if schedule:
        assert g.info().schedule == schedule
    dt_gpu = g.compute_dt()
    assert dt_gpu == pytest.approx(dt, rel=1e-14 if prec == ctu.FP64 else 1e-6)
    g.step(dt)
    status, flags, counters = g.check()
    assert status == ctu.OK, (flags, counters)
    gpu = g.get_state()
    g.close()
    del g
    rng = np.random.default_rng(seed)
    n = wl.nx
    tol_elem = ELEM64 if prec == ctu.FP64 else ELEM32
    for lo, hi in _boxes(n, special, rng):
        ref, _ = O.update_box(cfg, u, dt, lo, hi)
        got = gpu[:, lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]]
        assert_parity(got, ref, wl.gamma, tol, tol_elem, what=(wl.name, prec, lo, hi))


def _shock_cloud_special(n):
    shock_x = int(0.1 * n)
    cloud_edge = int((0.3 - 0.1) * n)
    return [(shock_x, n // 2, n // 2), (shock_x, 3, 3), (cloud_edge, n // 2, n // 2),
            (int(0.3 * n), n // 2 + int(0.1 * n), n // 2), (0, 0, 0), (n - 1, n - 1, n - 1)]


def _oracle_threads():
    """The OpenMP oracle on this host's share of cores (at most 16)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return O.set_threads(max(1, min(16, n)))


@pytest.mark.timeout(900)
@pytest.mark.parametrize("prec,schedule", [(0, 0), (1, 0), (0, 3)],
                         ids=["fp64", "fp32", "fp64-fused_z"])
def test_shock_cloud_256_full_grid_evolved(prec, schedule):
    """Every cell of the 256^3 shock-cloud after one step from an evolved state: the GPU runs
    90 steps (its own CFL time steps) with the shock started at x = 0.17, so that it has
    entered the cloud (edge at x = 0.2) and compressed it; its state is downloaded and one more GPU step is
    compared with the oracle's step of that same state (FP64 arithmetic on the float state
    in the FP32 form), cell by cell over the whole grid.  The grid takes the library's
    schedule for its size (overlapped), and once, in FP64, the fused-z schedule that larger
    grids take (both z stages in one march)."""
    from paper_1410_4194_amd import ctu
    wl = WL.shock_cloud(256, x_shock=0.17)
    cfg = oracle_config(wl)
    print(f"[gpu-test] full grid 256^3 shock-cloud (x_shock 0.17) prec {prec} schedule "
          f"{schedule}: 90 GPU steps", flush=True)
    g = ctu.Grid.from_workload(wl, prec=prec, schedule=schedule)
    if schedule:
        assert g.info().schedule == schedule
    g.advance(90)
    U = g.get_state()
    dt = g.compute_dt()
    g.step(dt)
    status, flags, counters = g.check()
    assert status == ctu.OK, (flags, counters)
    gpu = g.get_state()
    g.close()
    del g
    # the shock has entered the cloud: cloud gas compressed above its initial density 10
    rho = U[0].astype(np.float64)
    assert rho[:, :, 50:70].max() > 14.0, rho[:, :, 50:70].max()
    threads = _oracle_threads()
    try:
        print(f"[gpu-test]   oracle step of the whole grid on {threads} threads", flush=True)
        u = O.alloc_state(cfg)
        O.real(cfg, u)[...] = U
        del U
        O.step(cfg, u, dt)
    finally:
        O.set_threads(1)
    if prec == ctu.FP64:
        assert_parity(gpu, O.real(cfg, u), wl.gamma, TOL64, ELEM64, what="256^3 full grid fp64")
    else:
        assert_parity(gpu, O.real(cfg, u), wl.gamma, TOL32, ELEM32, what="256^3 full grid fp32")


def test_shock_cloud_256_fp64(ctu=None):
    from paper_1410_4194_amd import ctu
    _check(ctu, WL.shock_cloud(256), ctu.FP64, 1e-12, _shock_cloud_special(256), seed=31)


# the paper's other reconstruction and Riemann solvers, as the benchmark times them
METHODS = [("ppmc_roe", dict(riemann=1)), ("ppmc_roe_hcorr", dict(riemann=1, h_correction=1)),
           ("ppmp_exact", dict(recon=1)), ("ppmp_roe", dict(recon=1, riemann=1)),
           ("ppmp_roe_hcorr", dict(recon=1, riemann=1, h_correction=1))]


@pytest.mark.parametrize("name,method", METHODS, ids=[m[0] for m in METHODS])
@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32"])
def test_shock_cloud_256_methods(name, method, prec):
    from paper_1410_4194_amd import ctu
    _check(ctu, WL.shock_cloud(256), prec, 1e-12 if prec == 0 else 1e-5,
           _shock_cloud_special(256), seed=33, **method)


# the fused-z schedule with the methods it has a variant for (not the H correction)
FUSED_Z_METHODS = [("ppmc_roe", dict(riemann=1)), ("ppmp_exact", dict(recon=1))]


@pytest.mark.parametrize("name,method", FUSED_Z_METHODS, ids=[m[0] for m in FUSED_Z_METHODS])
@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32"])
def test_shock_cloud_256_methods_fused_z(name, method, prec):
    from paper_1410_4194_amd import ctu
    _check(ctu, WL.shock_cloud(256), prec, 1e-12 if prec == 0 else 1e-5,
           _shock_cloud_special(256), seed=34, schedule=ctu.SCHEDULE_FUSED_Z, **method)


@pytest.mark.timeout(600)
def test_turbulent_cloud_512_fp32():
    from paper_1410_4194_amd import ctu
    wl = WL.turbulent_cloud(512)
    n = 512
    shock_x = int(0.1 * n)
    special = [(shock_x, n // 2, n // 2), (int(0.15 * n), n // 2, n // 2),
               (int(0.3 * n), n // 2, n // 2), (int(0.3 * n), n // 2 + int(0.15 * n), n // 2),
               (0, 0, 0), (n - 1, n - 1, n - 1)]
    _check(ctu, wl, ctu.FP32, 1e-5, special, seed=32)



@pytest.mark.timeout(900)
def test_turbulent_cloud_512_fp64_steps_25_and_50():
    """The FP64 reference of the precision study: steps 25 and 50 of the 512^3 turbulent
    cloud (shock started at x = 0.14 so that it reaches the cloud) against the oracle, each
    from the GPU state saved before that step, on sampled boxes."""
    from paper_1410_4194_amd import ctu
    wl = WL.turbulent_cloud(512, x_shock=0.14)
    cfg = oracle_config(wl)
    g = ctu.Grid.from_workload(wl, prec=ctu.FP64)
    n = 512
    rng = np.random.default_rng(33)
    special = [(int(0.14 * n) + 8, n // 2, n // 2), (int(0.15 * n), n // 2, n // 2),
               (int(0.16 * n), n // 2 + 20, n // 2 - 20), (0, 0, 0)]
    for k in range(1, 51):
        dt = g.compute_dt()
        if k in (25, 50):
            print(f"[gpu-test] turbulent cloud 512^3 FP64 step {k}", flush=True)
            U = g.get_state()
            u = O.alloc_state(cfg)
            O.real(cfg, u)[...] = U
            O.bc_fill(cfg, u)
            g.step(dt)
            gpu = g.get_state()
            for lo, hi in _boxes(n, special, rng, count=3):
                ref, _ = O.update_box(cfg, u, dt, lo, hi)
                got = gpu[:, lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]]
                assert_parity(got, ref, wl.gamma, TOL64, ELEM64, what=("step", k, lo))
            del u, U
        else:
            g.step(dt)
    status, flags, counters = g.check()
    assert status == ctu.OK, (flags, counters)
    g.close()