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


def test_condition_number_of_the_pressure():
    """kappa = 1 + kinetic / internal energy: 1 for gas at rest, about 3.3e5 in Noh's cold
    inflow (rho = 1, |V| = 1, p = 1e-6, gamma 5/3: 0.5 / 1.5e-6), and the per-cell allowance
    it sets there still fails a planted one-cell error by many orders of magnitude."""
    from tests.common import COND64, cell_condition
    wl = WL.noh(16)
    cfg = oracle_config(wl, riemann=1, h_correction=1)
    u = oracle_state(wl, cfg)
    ref = O.real(cfg, u).copy()
    kappa = cell_condition(ref, wl.gamma)
    assert abs(kappa.max() / (1.0 + 0.5 / (1e-6 / (wl.gamma - 1.0))) - 1.0) < 1e-9
    rest = WL.sod(32, 4, 4)
    ur = oracle_state(rest)
    assert np.all(cell_condition(O.real(oracle_config(rest), ur), rest.gamma) == 1.0)
    bad = ref.copy()
    bad[0, 5, 6, 7] *= 1.0 + 1e-6
    allow = np.maximum(ELEM64, COND64 * kappa)
    ratio, where = elem_err(bad, ref, wl.gamma, allow=allow)
    assert ratio[0] > 100.0 and where[0] == (5, 6, 7)
