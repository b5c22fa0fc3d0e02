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


def rel_l1(gpu: np.ndarray, ref: np.ndarray, gamma: float) -> np.ndarray:
    """Per-field relative L1 difference of two conserved real-cell states (5, ...):
    err_f = sum |q_gpu - q_ref| / sum s_f with s = rho for mass, rho (|V| + a) for the
    momenta and E for energy (scales taken from the reference)."""
    ref = np.asarray(ref, dtype=np.float64)
    gpu = np.asarray(gpu, dtype=np.float64)
    rho = ref[0]
    V2 = (ref[1] ** 2 + ref[2] ** 2 + ref[3] ** 2) / rho ** 2
    p = np.maximum((gamma - 1.0) * (ref[4] - 0.5 * rho * V2), 1e-300)
    a = np.sqrt(gamma * p / rho)
    smom = rho * (np.sqrt(V2) + a)
    scales = [rho, smom, smom, smom, np.abs(ref[4])]
    return np.array([np.abs(gpu[f] - ref[f]).sum() / scales[f].sum() for f in range(5)])
