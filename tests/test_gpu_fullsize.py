"""Full-size parity: one step of the benchmark workloads on the GPU, checked on sampled boxes
that the oracle computes independently from the same seeded input.

256^3 FP64 shock-cloud (the benchmark workload) and 512^3 FP32 turbulent cloud.  Both sides
use the oracle's dt, so the GPU runs the same kernels and launch shapes as the benchmark.
Sampled boxes cover the shock front, the cloud edge, the domain corners (outflow ghosts) and
random interior points.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import oracle as O
from paper_1410_4194_amd import workloads as WL
from tests.common import oracle_config, rel_l1


def _boxes(n, special, rng, count=6, size=8):
    boxes = []
    for (cx, cy, cz) in special:
        lo = [max(0, min(n - size, c - size // 2)) for c in (cx, cy, cz)]
        boxes.append((tuple(lo), tuple(l + size for l in lo)))
    for _ in range(count):
        lo = [int(v) for v in rng.integers(0, n - size, size=3)]
        boxes.append((tuple(lo), tuple(l + size for l in lo)))
    return boxes


def _check(ctu, wl, prec, tol, special, seed, **method):
    print(f"[gpu-test] full size {wl.name} prec {prec} {method}", flush=True)
    cfg = oracle_config(wl, **method)
    u = O.state_from_primitive(cfg, wl.W)
    O.bc_fill(cfg, u)
    dt = O.compute_dt(cfg, u)
    g = ctu.Grid.from_workload(wl, prec=prec, **method)
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
    errs = []
    for lo, hi in _boxes(n, special, rng):
        ref, _ = O.update_box(cfg, u, dt, lo, hi)
        got = gpu[:, lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]]
        e = rel_l1(got, ref, wl.gamma)
        errs.append(e.max())
        assert e.max() <= tol, (lo, hi, e)
    print(f"[gpu-test]   max relative L1 over {len(errs)} boxes: {max(errs):.3e}", flush=True)


def _shock_cloud_special(n):
    shock_x = int(0.1 * n)
    cloud_edge = int((0.3 - 0.1) * n)
    return [(shock_x, n // 2, n // 2), (shock_x, 3, 3), (cloud_edge, n // 2, n // 2),
            (int(0.3 * n), n // 2 + int(0.1 * n), n // 2), (0, 0, 0), (n - 1, n - 1, n - 1)]


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
                e = rel_l1(got, ref, wl.gamma)
                assert e.max() <= 1e-12, (k, lo, e)
            del u, U
        else:
            g.step(dt)
    status, flags, counters = g.check()
    assert status == ctu.OK, (flags, counters)
    g.close()