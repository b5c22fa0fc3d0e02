"""The per-cell parity metric catches what the relative L1 norm dilutes: one cell made
entirely wrong in the oracle's own one-step result of the 48^3 shock-cloud changes the L1
norm by less than the FP32 bound, while its per-cell error is of order one.  (A planted
mistake, on the CPU, in the oracle's result only.)"""
import numpy as np

import oracle as O
from paper_1410_4194_amd import workloads as WL
from tests.common import ELEM32, ELEM64, TOL32, elem_err, oracle_config, oracle_state, rel_l1


def test_one_wrong_cell_fails_the_cell_bound_not_the_l1_bound():
    wl = WL.shock_cloud(48, steps=1)
    cfg = oracle_config(wl)
    u = oracle_state(wl, cfg)
    O.step(cfg, u, O.compute_dt(cfg, u))
    ref = O.real(cfg, u).copy()
    bad = ref.copy()
    bad[0, 20, 21, 22] *= 2.0
    bad[4, 20, 21, 22] *= 2.0
    l1 = rel_l1(bad, ref, wl.gamma)
    assert l1.max() < TOL32  # the L1 norm alone would pass this
    el, where = elem_err(bad, ref, wl.gamma)
    assert el.max() > 0.5 and el.max() > ELEM32 and where[0] == (20, 21, 22)
    same, _ = elem_err(ref, ref, wl.gamma)
    assert same.max() == 0.0
    # a NaN anywhere counts as the worst possible error
    bad = ref.copy()
    bad[2, 1, 2, 3] = np.nan
    el, where = elem_err(bad, ref, wl.gamma)
    assert el[2] == np.inf and where[2] == (1, 2, 3) and el.max() > ELEM64
