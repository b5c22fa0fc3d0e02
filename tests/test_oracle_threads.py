"""The oracle built twice from one source, serial and with OpenMP over z-planes, must give
bit-identical steps and identical counters: every cell is computed by the same operations in
both builds, and only integer counters are summed across threads.  The threaded build is
what the full-grid GPU parity check and the all-core CPU baseline run, so it is pinned to
the serial one here, on every method and boundary type."""
import numpy as np
import pytest

import oracle as O
from paper_1410_4194_amd import workloads as WL
from tests.common import oracle_config, oracle_state

CASES = [
    ("ppmc_exact_rough_periodic", lambda: WL.random_state(21, 13, 11, seed=41), {}),
    ("ppmc_exact_shock_cloud", lambda: WL.shock_cloud(24, steps=1), {}),
    ("ppmc_roe_outflow", lambda: WL.random_state(17, 12, 9, seed=42, bc=(1,) * 6), dict(riemann=1)),
    ("ppmc_roe_h_reflect", lambda: WL.random_state(14, 12, 10, seed=43, bc=(2, 2, 0, 0, 1, 1)),
     dict(riemann=1, h_correction=1)),
    ("ppmp_exact_mixed", lambda: WL.random_state(16, 11, 13, seed=44, bc=(1, 1, 0, 0, 2, 2),
                                                 rough=False, mach=1.5), dict(recon=1)),
    ("ppmp_roe_h", lambda: WL.random_state(13, 12, 11, seed=45), dict(recon=1, riemann=1,
                                                                      h_correction=1)),
]


@pytest.fixture
def restore_serial():
    yield
    O.set_threads(1)


@pytest.mark.parametrize("name,make,method", CASES, ids=[c[0] for c in CASES])
def test_openmp_build_is_bitwise_serial(name, make, method, restore_serial):
    wl = make()
    cfg = oracle_config(wl, **method)
    u0 = oracle_state(wl, cfg)
    O.set_threads(1)
    dt = O.compute_dt(cfg, u0)
    a = u0.copy()
    sa = [O.step(cfg, a, dt) for _ in range(2)]
    n = O.set_threads(4)
    assert n == 4
    b = u0.copy()
    sb = [O.step(cfg, b, dt) for _ in range(2)]
    assert np.array_equal(a, b), name
    assert sa == sb, (sa, sb)
    # a sub-box update (the form the sampled checks use) agrees as well
    lo, hi = (1, 2, 3), (wl.nx - 1, wl.ny, wl.nz - 2)
    O.set_threads(1)
    ra, _ = O.update_box(cfg, a, dt, lo, hi)
    O.set_threads(3)
    rb, _ = O.update_box(cfg, a, dt, lo, hi)
    assert np.array_equal(ra, rb)
