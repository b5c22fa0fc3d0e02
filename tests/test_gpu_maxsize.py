"""The largest grids one MI355X holds: 1024^3 in FP32 (153 GB of state and workspace) and,
in FP64, 1024 x 1024 x nz with nz as large as the free device memory allows (1024^3 itself
needs 306 GB).  Field offsets pass 2^32 elements here, so every index of every pass is
exercised in 64-bit form.

The state is Sod's shock tube along x, the same in every (y, z) column, written straight into
the caller-owned state buffer in its documented layout (no host copy of 10^9 cells).  Two
steps with the oracle's dt must leave every column identical bit for bit (the y and z faces
see equal states, so their flux differences vanish exactly), and column (0, 0) must match the
oracle's 1D run (FP64 <= 1e-12, FP32 <= 1e-5 relative L1); the next CFL step of the 10^9
cells must match the oracle's.
"""
import gc
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import oracle as O
from tests.common import ELEM32, TOL32, TOL64, assert_parity

MULTI64 = 1e-8  # per-cell bound after two steps

G = 1.4
NX = 1024


@pytest.fixture(scope="module")
def ctu():
    from paper_1410_4194_amd import ctu as _ctu
    return _ctu


def _announce(*parts):
    print("[gpu-test]", *parts, flush=True)
    sys.stdout.flush()


def _config(ctu, nz, prec):
    d = 1.0 / NX
    return ctu.make_config(NX, NX, nz, d, d, d, G, (1, 1, 0, 0, 0, 0), prec, 0.3)


def _largest_nz(ctu, prec, budget):
    lo, hi = 0, NX
    while lo < hi:
        mid = (lo + hi + 1) // 2
        s, w = ctu.workspace_bytes(_config(ctu, mid, prec))
        if s + w <= budget:
            lo = mid
        else:
            hi = mid - 1
    return lo


def _sod_columns():
    """Conserved Sod state along x (ny = nz = 1) and its oracle configuration."""
    d = 1.0 / NX
    cfg = O.Config(NX, 1, 1, d, d, d, G, bc=(1, 1, 0, 0, 0, 0), cfl=0.3)
    x = (np.arange(NX) + 0.5) * d
    W = np.zeros((5, 1, 1, NX))
    W[0] = np.where(x < 0.5, 1.0, 0.125)
    W[4] = np.where(x < 0.5, 1.0, 0.1)
    return cfg, O.state_from_primitive(cfg, W)


def _release():
    import torch
    gc.collect()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


@pytest.mark.parametrize("prec", [1, 0], ids=["fp32_1024^3", "fp64_largest"])
def test_largest_grid(ctu, prec):
    _release()  # cached blocks of earlier tests go back to the device first
    try:
        _run_largest(ctu, prec)
    finally:
        _release()


def _run_largest(ctu, prec):
    import torch
    free, total = torch.cuda.mem_get_info()
    budget = free - (8 << 30)
    nz = NX if prec == 1 else _largest_nz(ctu, prec, budget)
    cfg = _config(ctu, nz, prec)
    s, w = ctu.workspace_bytes(cfg)
    if s + w > budget:
        pytest.skip(f"{(s + w) / 1e9:.0f} GB do not fit in {free / 1e9:.0f} GB free")
    assert nz >= 800, nz
    _announce("largest grid", NX, NX, nz, "prec", prec, "bytes", s + w, "free", free)
    g = ctu.Grid(cfg)
    try:
        info = g.info()
        gh = info.ghost
        T = torch.float64 if prec == 0 else torch.float32
        fields = g.state.view(T)[: 5 * info.field_stride].view(5, info.field_stride)
        box = fields[:, : info.alloc_cells].view(5, nz + 2 * gh, NX + 2 * gh, NX + 2 * gh)
        real = box[:, gh:gh + nz, gh:gh + NX, gh:gh + NX]
        ocfg, u1 = _sod_columns()
        col0 = O.real(ocfg, u1)[:, 0, 0, :]
        prof = torch.tensor(col0, dtype=T, device=g.device)
        for f in range(5):
            real[f].copy_(prof[f].view(1, 1, NX).expand(nz, NX, NX))
        for _ in range(2):
            dt = O.compute_dt(ocfg, u1)
            g.step(dt)
            O.step(ocfg, u1, dt)
        status, flags, counters = g.check()
        assert status == ctu.OK, (flags, counters)
        for f in range(5):
            ref = real[f, 0:1, 0:1, :]
            assert bool((real[f] == ref).all()), f
        gpu_col = real[:, 0, 0, :].double().cpu().numpy()
        ref_col = O.real(ocfg, u1)[:, 0, 0, :]
        assert_parity(gpu_col, ref_col, G, *((TOL64, MULTI64) if prec == 0 else (TOL32, ELEM32)),
                      what=("max size column", prec))
        dt_gpu, dt_ref = g.compute_dt(), O.compute_dt(ocfg, u1)
        assert abs(dt_gpu / dt_ref - 1.0) <= (1e-12 if prec == 0 else 1e-5), (dt_gpu, dt_ref)
    finally:
        g.close()
