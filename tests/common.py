"""Shared test helpers: workloads -> oracle configuration and state, and the parity metrics
(relative L1 per field, and the largest per-cell error against each cell's own scale)."""
import json
import os

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


def cell_scales(ref: np.ndarray, gamma: float):
    """Per-cell scale of each conserved field of a state (5, ...): rho for mass,
    rho (|V| + a) for the momenta, |E| for energy; and the signal speed |V| + a."""
    ref = np.asarray(ref, dtype=np.float64)
    rho = ref[0]
    V2 = (ref[1] ** 2 + ref[2] ** 2 + ref[3] ** 2) / rho ** 2
    p = np.maximum((gamma - 1.0) * (ref[4] - 0.5 * rho * V2), 1e-300)
    speed = np.sqrt(V2) + np.sqrt(gamma * p / rho)
    smom = rho * speed
    return [np.abs(rho), smom, smom, smom, np.abs(ref[4])], speed


def rel_l1(gpu: np.ndarray, ref: np.ndarray, gamma: float) -> np.ndarray:
    """Per-field relative L1 difference of two conserved real-cell states (5, ...):
    err_f = sum |q_gpu - q_ref| / sum s_f with the scales s_f of cell_scales (taken from the
    reference)."""
    ref = np.asarray(ref, dtype=np.float64)
    gpu = np.asarray(gpu, dtype=np.float64)
    scales, _ = cell_scales(ref, gamma)
    return np.array([np.abs(gpu[f] - ref[f]).sum() / scales[f].sum() for f in range(5)])


def elem_err(gpu: np.ndarray, ref: np.ndarray, gamma: float):
    """Per-field largest cell error max_cells |q_gpu - q_ref| / s_f(cell), each cell measured
    against its own scale (cell_scales of the reference), and the index of the worst cell of
    each field.  Unlike the L1 norm this does not dilute an error confined to a few cells
    (a seam between tiles, chunks or segments)."""
    ref = np.asarray(ref, dtype=np.float64)
    gpu = np.asarray(gpu, dtype=np.float64)
    scales, _ = cell_scales(ref, gamma)
    errs, where = [], []
    for f in range(5):
        e = np.abs(gpu[f] - ref[f]) / np.maximum(scales[f], 1e-300)
        e = np.where(np.isnan(e), np.inf, e)  # a NaN on either side is the worst error
        k = int(np.argmax(e))
        errs.append(float(e.flat[k]))
        where.append(tuple(int(v) for v in np.unravel_index(k, e.shape)))
    return np.array(errs), where


# One-step parity bounds, FP64 and the FP32 form (relative L1 and per cell, as defined above).
TOL64, TOL32 = 1e-12, 1e-5
ELEM64, ELEM32 = 1e-10, 1e-4


def _report(record):
    path = os.environ.get("CTU_PARITY_REPORT")
    if path:
        with open(path, "a") as fh:
            fh.write(json.dumps(record) + "\n")


def assert_parity(gpu, ref, gamma, tol_l1, tol_elem, what=""):
    """Both bounds: relative L1 per field <= tol_l1 and every cell within tol_elem of its own
    scale.  Prints the worst cell (field, (z, y, x) index within the compared arrays)."""
    l1 = rel_l1(gpu, ref, gamma)
    el, where = elem_err(gpu, ref, gamma)
    f = int(np.argmax(el))
    print(f"[parity] {what}: relative L1 {l1.max():.2e}, worst cell {el[f]:.2e} "
          f"(field {f} at z,y,x = {where[f]})", flush=True)
    _report(dict(what=str(what), l1=float(l1.max()), elem=float(el[f]), field=f,
                 at=list(where[f]), tol_l1=tol_l1, tol_elem=tol_elem))
    assert l1.max() <= tol_l1, (what, "relative L1", l1)
    assert el.max() <= tol_elem, (what, "worst cell", el, where)
    return l1, el


def parity_bounds(prec):
    """(relative L1, per cell) one-step bounds of a precision (0 = FP64, 1 = FP32)."""
    return (TOL64, ELEM64) if prec == 0 else (TOL32, ELEM32)
