"""C-ABI checks that need no GPU: the library loads, exports every entry point that
include/ctu.h declares, and validates configurations on the host."""
import ctypes as C
import os
import re

import pytest

REPO = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(REPO, "include", "ctu.h")
LIB = os.path.join(REPO, "paper_1410_4194_amd", "libctu.so")


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:ctu_status|const char\*|size_t)\s+(ctu_\w+)\s*\(", text, re.M)))


@pytest.fixture(scope="module")
def ctu():
    if not os.path.exists(LIB):
        pytest.fail("libctu.so not built (python -m paper_1410_4194_amd.build)")
    from paper_1410_4194_amd import ctu as m
    return m


def test_header_declares_the_api():
    names = declared_functions()
    assert len(names) >= 20
    for must in ("ctu_grid_create", "ctu_step", "ctu_compute_dt", "ctu_advance",
                 "ctu_batch_submit", "ctu_batch_poll"):
        assert must in names


def test_library_exports_every_declared_symbol(ctu):
    lib = C.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(ctu.EXPORTS) == declared_functions()


def test_workspace_bytes_and_validation(ctu):
    cfg = ctu.make_config(256, 256, 256, 1 / 256, 1 / 256, 1 / 256, 5 / 3, (1,) * 6)
    sb, wb = ctu.workspace_bytes(cfg)
    na = 262 ** 3
    stride = (na + 63) // 64 * 64
    assert sb == 5 * stride * 8
    assert wb >= 30 * stride * 8  # first-stage and CTU fluxes, 15 fields each
    cfg32 = ctu.make_config(8, 8, 8, 1, 1, 1, 1.4, prec=ctu.FP32)
    sb32, _ = ctu.workspace_bytes(cfg32)
    assert sb32 == 5 * ((14 ** 3 + 63) // 64 * 64) * 4
    bad = [
        dict(nx=0), dict(dx=0.0), dict(gamma=1.0), dict(cfl=0.5), dict(cfl=0.0),
        dict(bc=(0, 1, 0, 0, 0, 0)), dict(bc=(3, 3, 0, 0, 0, 0)), dict(prec=7),
        dict(bc=(2, 0, 0, 0, 0, 0)), dict(nx=2, bc=(2, 2, 0, 0, 0, 0)),
        dict(nz=1, bc=(0, 0, 0, 0, 1, 2)),
        dict(newton_max_iter=0), dict(newton_tol=0.0), dict(p_floor=0.0),
        dict(march_seg=(-1, 0)), dict(march_seg=(0, 5000)),
        dict(x_rows=-1), dict(x_rows=9), dict(x_chunks=-1), dict(x_chunks=17),
        dict(schedule=-1), dict(schedule=4),
    ]
    for b in bad:
        args = dict(nx=8, ny=8, nz=8, dx=1.0, dy=1.0, dz=1.0, gamma=1.4)
        args.update({k: v for k, v in b.items() if k in args})
        extra = {k: v for k, v in b.items() if k not in args}
        c = ctu.make_config(**args, **extra)
        with pytest.raises(ctu.CtuError) as ei:
            ctu.workspace_bytes(c)
        assert ei.value.status == ctu.EINVAL
    ok = ctu.make_config(3, 8, 1, 1, 1, 1, 1.4, (ctu.BC_REFLECT, ctu.BC_OUTFLOW, 2, 2, 0, 0))
    ctu.workspace_bytes(ok)
    # PPMP: four ghost layers, six coefficient fields more, reflect needs four cells
    pp = ctu.make_config(8, 8, 8, 1, 1, 1, 1.4, recon=ctu.RECON_PPMP)
    sbp, wbp = ctu.workspace_bytes(pp)
    assert sbp == 5 * ((16 ** 3 + 63) // 64 * 64) * 8
    assert wbp >= 36 * ((16 ** 3 + 63) // 64 * 64) * 8
    with pytest.raises(ctu.CtuError):
        ctu.workspace_bytes(ctu.make_config(3, 8, 8, 1, 1, 1, 1.4, (2, 2, 0, 0, 0, 0),
                                            recon=ctu.RECON_PPMP))
    for bad_kw in (dict(recon=2), dict(riemann=2)):
        with pytest.raises(ctu.CtuError):
            ctu.workspace_bytes(ctu.make_config(8, 8, 8, 1, 1, 1, 1.4, **bad_kw))


def test_grid_create_rejects_small_workspace(ctu):
    cfg = ctu.make_config(8, 8, 8, 1, 1, 1, 1.4)
    h = C.c_void_p()
    st = ctu.lib.ctu_grid_create(C.byref(cfg), C.c_void_p(256), C.c_void_p(512), C.c_size_t(1024),
                                 None, C.byref(h))
    assert st == ctu.ENOMEM and h.value is None
    assert b"workspace" in ctu.lib.ctu_last_error()


def test_grid_size_limits(ctu):
    """More than 2^31 real cells is refused by validation; a grid whose x pass would need
    more than 2^32 - 1 work-items in one dispatch (a 5e8-cell line: every cell is a lane of
    its own row) is refused when the grid is created, before any device work."""
    with pytest.raises(ctu.CtuError) as ei:
        ctu.workspace_bytes(ctu.make_config(2048, 1024, 1025, 1, 1, 1, 1.4))
    assert ei.value.status == ctu.EINVAL
    ctu.workspace_bytes(ctu.make_config(2048, 1024, 1024, 1, 1, 1, 1.4))
    cfg = ctu.make_config(500_000_000, 1, 1, 1, 1, 1, 1.4)
    sb, wb = ctu.workspace_bytes(cfg)
    h = C.c_void_p()
    st = ctu.lib.ctu_grid_create(C.byref(cfg), C.c_void_p(256), C.c_void_p(512), C.c_size_t(wb),
                                 None, C.byref(h))
    assert st == ctu.EINVAL and h.value is None
    assert b"one launch per pass" in ctu.lib.ctu_last_error()


def test_product_path_requires_gpu(ctu):
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    cfg = ctu.make_config(8, 8, 8, 1, 1, 1, 1.4)
    with pytest.raises(RuntimeError, match="no GPU"):
        ctu.Grid(cfg)


def test_batch_workspace_and_validation(ctu):
    wb = C.c_size_t()
    assert ctu.lib.ctu_batch_workspace_bytes(64, C.byref(wb)) == ctu.OK
    assert wb.value >= 64 * (2 * 256 + 8)  # descriptors of both precisions + scalar table
    small = wb.value
    assert ctu.lib.ctu_batch_workspace_bytes(128, C.byref(wb)) == ctu.OK and wb.value > small
    for bad in (0, -1, 1 << 20):
        assert ctu.lib.ctu_batch_workspace_bytes(bad, C.byref(wb)) == ctu.EINVAL
    h = C.c_void_p()
    st = ctu.lib.ctu_batch_create(64, C.c_void_p(256), C.c_size_t(small - 1), None, 0, C.byref(h))
    assert st == ctu.ENOMEM and h.value is None
    st = ctu.lib.ctu_batch_create(64, C.c_void_p(256), C.c_size_t(small), None, 4, C.byref(h))
    assert st == ctu.EINVAL and h.value is None
    st = ctu.lib.ctu_batch_create(64, C.c_void_p(100), C.c_size_t(small), None, 0, C.byref(h))
    assert st == ctu.EINVAL and h.value is None


def test_stream_probe_validates_on_the_host(ctu):
    """The streaming probe refuses an unknown kind, a missing array and an empty range before
    anything is launched (no GPU needed); its read variant needs one double per 1024 elements."""
    lib = ctu.lib
    assert ctu.stream_probe_blocks(1) == 1 and ctu.stream_probe_blocks(1024) == 1
    assert ctu.stream_probe_blocks(1025) == 2
    fake = C.c_void_p(4096)
    for kind, a, b, c, n in ((7, fake, fake, fake, 16), (-1, fake, fake, fake, 16),
                             (0, None, None, fake, 16), (1, fake, None, None, 16),
                             (2, fake, None, fake, 16), (3, fake, None, fake, 0)):
        assert lib.ctu_stream_probe(kind, a, b, c, n, None) == ctu.EINVAL
