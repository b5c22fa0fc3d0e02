"""Shared test helpers: workloads -> oracle configuration and state."""
import numpy as np

import oracle as O
from paper_1410_4194_amd import workloads as WL


def oracle_config(wl, **kw) -> O.Config:
    args = dict(cfl=wl.cfl)
    args.update(kw)
    return O.Config(wl.nx, wl.ny, wl.nz, wl.dx, wl.dy, wl.dz, wl.gamma, bc=wl.bc, **args)


def oracle_state(wl, cfg=None) -> np.ndarray:
    cfg = cfg or oracle_config(wl)
    return O.state_from_primitive(cfg, wl.W)


def run_oracle(wl, t_end=None, steps=None, cfg=None):
    """Advance with the oracle to t_end (clipping the last step) or for `steps` steps."""
    cfg = cfg or oracle_config(wl)
    u = oracle_state(wl, cfg)
    t, n = 0.0, 0
    while True:
        if steps is not None and n >= steps:
            break
        if t_end is not None and t >= t_end * (1 - 1e-14):
            break
        dt = O.compute_dt(cfg, u)
        if t_end is not None:
            dt = min(dt, t_end - t)
        O.step(cfg, u, dt)
        t += dt
        n += 1
    return cfg, u, t, n
