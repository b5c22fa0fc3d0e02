"""ctu_step_noalloc, the step whose workspace is the library's fixed device array instead of a
caller buffer, against ctu_step on grids created the usual way: two calls in a row through
the C ABI, the second on a smaller grid of the other precision with the widest method
(PPMP, Roe with the H correction, reflecting walls), each bitwise equal to ctu_step's result
(same kernels and launch shapes); and the size limit, refused before any launch."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from paper_1410_4194_amd import workloads as WL


@pytest.fixture(scope="module")
def ctu():
    from paper_1410_4194_amd import ctu as m
    return m


def _one(ctu, wl, prec, **method):
    import torch
    print(f"[gpu-test] no-alloc step {wl.name} prec {prec} {method}", flush=True)
    g = ctu.Grid.from_workload(wl, prec=prec, **method)
    dt = g.compute_dt()
    d_state = g.state.clone()  # the same initial state, in the library's layout
    torch.cuda.synchronize()
    g.step(dt)
    ref = g.get_state()
    status, flags, counters = g.check()
    assert status == ctu.OK, (flags, counters)
    ctu.step_noalloc(g.cfg, d_state, dt)
    torch.cuda.synchronize()
    g.state.copy_(d_state)  # read the no-alloc result back through the grid's gather
    torch.cuda.synchronize()
    got = g.get_state()
    g.close()
    assert np.all(np.isfinite(ref))
    diff = np.argwhere(got != ref)
    assert diff.size == 0, (wl.name, prec, diff[:5])


def test_noalloc_equals_step_twice_second_smaller(ctu):
    big = WL.random_state(40, 36, 28, seed=21, bc=(1, 1, 0, 0, 1, 1))
    small = WL.random_state(20, 14, 12, seed=22, bc=(2, 2, 0, 0, 1, 1))
    _one(ctu, big, ctu.FP64)
    _one(ctu, small, ctu.FP32, recon=1, riemann=1, h_correction=1)


def test_noalloc_refuses_a_grid_beyond_the_scratch(ctu):
    import torch
    cfg = ctu.make_config(128, 128, 128, 1 / 128, 1 / 128, 1 / 128, 5 / 3, (1,) * 6)
    _, wb = ctu.workspace_bytes(cfg)
    assert wb > ctu.NOALLOC_SCRATCH_BYTES
    dummy = torch.zeros(256, dtype=torch.uint8, device="cuda")
    with pytest.raises(ctu.CtuError) as ei:
        ctu.step_noalloc(cfg, dummy, 1e-3)
    assert ei.value.status == ctu.EINVAL and "scratch" in str(ei.value)
    assert int(dummy.sum().item()) == 0
