"""ctypes binding over the C ABI of ``libctu.so`` (include/ctu.h).

Marshalling only: every step of the timestep runs in the HIP kernels of the library.
PyTorch provides the device buffers (caller-owned, as the ABI requires) and the stream.
Importing this module raises if the library has not been built; creating a grid raises if
no GPU is visible.

torch is imported before the library is loaded so that the process holds a single HIP
runtime: torch ships its own libamdhip64 with the same soname as the system one, and
libctu.so then binds to the copy torch already loaded.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np
import torch  # noqa: F401  (must precede loading libctu.so, see above)

_HERE = os.path.dirname(os.path.abspath(__file__))
# CTU_LIBRARY selects another build of the same library (A/B timing of builds)
LIB_PATH = os.environ.get("CTU_LIBRARY") or os.path.join(_HERE, "libctu.so")

OK, EINVAL, ENOMEM, EDEVICE, ENONPHYS, ENOCONV, EAGAIN = 0, -1, -2, -3, -4, -5, -6
BC_PERIODIC, BC_OUTFLOW, BC_REFLECT = 0, 1, 2
RIEMANN_EXACT, RIEMANN_ROE = 0, 1
RECON_PPMC, RECON_PPMP = 0, 1
SCHEDULE_AUTO, SCHEDULE_IN_ORDER, SCHEDULE_OVERLAP, SCHEDULE_FUSED_Z = 0, 1, 2, 3
FP64, FP32 = 0, 1
FLAG_NONFINITE, FLAG_DENSITY, FLAG_PFLOOR, FLAG_NEWTON_CAP = 1, 2, 4, 8
TICKET_QUEUED, TICKET_RUNNING, TICKET_DONE, TICKET_FAILED, TICKET_UNKNOWN = 0, 1, 2, 3, -1
BATCH_GRAPH = 1
PROFILE_TIMING, PROFILE_NEWTON = 1, 2
NEWTON_BINS = ("0-1", "2", "3", "4", "5-8", "9-16", ">16", "cap")

EXPORTS = [
    "ctu_config_default", "ctu_workspace_bytes", "ctu_grid_create", "ctu_grid_destroy",
    "ctu_grid_info_get", "ctu_set_state", "ctu_set_primitive", "ctu_get_state",
    "ctu_compute_dt", "ctu_step", "ctu_advance", "ctu_totals", "ctu_check",
    "ctu_debug_fluxes", "ctu_debug_keep_fluxes", "ctu_batch_workspace_bytes", "ctu_batch_create", "ctu_batch_submit",
    "ctu_batch_run",
    "ctu_batch_poll", "ctu_batch_destroy", "ctu_last_error", "ctu_profile_enable",
    "ctu_profile_read", "ctu_profile_name", "ctu_newton_histogram", "ctu_stream_probe_blocks",
    "ctu_stream_probe", "ctu_step_noalloc",
]


class Config(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double),
                ("gamma", C.c_double), ("bc", C.c_int32 * 6), ("prec", C.c_int32),
                ("cfl", C.c_double), ("newton_tol", C.c_double),
                ("newton_max_iter", C.c_int32), ("p_floor", C.c_double),
                ("march_seg", C.c_int32 * 2), ("riemann", C.c_int32), ("recon", C.c_int32),
                ("h_correction", C.c_int32), ("x_rows", C.c_int32), ("x_chunks", C.c_int32),
                ("schedule", C.c_int32)]


class GridInfo(C.Structure):
    _fields_ = [("alloc_cells", C.c_int64), ("field_stride", C.c_int64),
                ("elem_bytes", C.c_int32), ("t", C.c_double), ("steps", C.c_int64),
                ("ghost", C.c_int32), ("schedule", C.c_int32)]


class CtuError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"ctu error {status}: {msg}")
        self.status = status


def _load() -> C.CDLL:
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing "
                           "(run `python -m paper_1410_4194_amd.build`)")
    lib = C.CDLL(LIB_PATH)
    vp, sz = C.c_void_p, C.c_size_t
    st = C.c_int
    sig = {
        "ctu_config_default": ([C.POINTER(Config)], st),
        "ctu_workspace_bytes": ([C.POINTER(Config), C.POINTER(sz), C.POINTER(sz)], st),
        "ctu_grid_create": ([C.POINTER(Config), vp, vp, sz, vp, C.POINTER(vp)], st),
        "ctu_grid_destroy": ([vp], st),
        "ctu_grid_info_get": ([vp, C.POINTER(GridInfo)], st),
        "ctu_set_state": ([vp, C.POINTER(vp)], st),
        "ctu_set_primitive": ([vp, C.POINTER(vp)], st),
        "ctu_get_state": ([vp, C.POINTER(vp)], st),
        "ctu_compute_dt": ([vp, C.POINTER(C.c_double)], st),
        "ctu_step": ([vp, C.c_double], st),
        "ctu_advance": ([vp, C.c_int32, C.c_double], st),
        "ctu_totals": ([vp, C.POINTER(C.c_double)], st),
        "ctu_check": ([vp, C.POINTER(C.c_uint32), C.POINTER(C.c_uint64)], st),
        "ctu_debug_fluxes": ([vp, C.c_int32, C.c_int32, C.POINTER(vp)], st),
        "ctu_debug_keep_fluxes": ([vp, C.c_int32], st),
        "ctu_batch_workspace_bytes": ([C.c_int32, C.POINTER(sz)], st),
        "ctu_batch_create": ([C.c_int32, vp, sz, vp, C.c_int32, C.POINTER(vp)], st),
        "ctu_batch_submit": ([vp, vp, C.c_int32, C.c_double, C.POINTER(C.c_uint64)], st),
        "ctu_batch_run": ([vp, C.c_int32], st),
        "ctu_batch_poll": ([vp, C.c_uint64, C.POINTER(C.c_int32), C.POINTER(C.c_double)], st),
        "ctu_batch_destroy": ([vp], st),
        "ctu_last_error": ([], C.c_char_p),
        "ctu_profile_enable": ([vp, C.c_int32], st),
        "ctu_profile_read": ([vp, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int64),
                              C.POINTER(C.c_int32)], st),
        "ctu_profile_name": ([C.c_int32], C.c_char_p),
        "ctu_newton_histogram": ([vp, C.POINTER(C.c_uint64)], st),
        "ctu_stream_probe_blocks": ([sz], sz),
        "ctu_stream_probe": ([C.c_int32, vp, vp, vp, sz, vp], st),
        "ctu_step_noalloc": ([C.POINTER(Config), vp, C.c_double, vp], st),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


lib = _load()


def _check(status: int, allow=()) -> int:
    if status != OK and status not in allow:
        raise CtuError(status, lib.ctu_last_error().decode())
    return status


def make_config(nx, ny, nz, dx, dy, dz, gamma, bc=(BC_PERIODIC,) * 6, prec=FP64, cfl=0.3,
                newton_tol=1e-6, newton_max_iter=50, p_floor=1e-20, march_seg=None,
                riemann=0, recon=0, h_correction=0, x_rows=None, x_chunks=None,
                batch=False, schedule=0) -> Config:
    """Grid configuration.  riemann: RIEMANN_EXACT or RIEMANN_ROE (with the HLLE failsafe);
    recon: RECON_PPMC or RECON_PPMP; h_correction: 1 for the H correction of the
    second-stage Roe fluxes.  Tile shapes (launch shapes only): march_seg, target cells per
    thread of the y and z sweeps; x_rows, rows per wavefront of the x sweep fused with the
    update; x_chunks, chunks per wavefront of the first-stage x sweep.  None takes the
    autotuned table (tiles.json beside this module) when it has the entry, else the library
    default; batch=True takes the shapes tuned for grids advanced in a batch (where the GPU
    is full, unlike a small grid alone), when the table has them.  schedule: SCHEDULE_AUTO
    (the library's choice by size), SCHEDULE_IN_ORDER (every pass in order on the grid's
    stream), SCHEDULE_OVERLAP (the first-stage y and second-stage z sweeps on a stream of the
    grid's own beside the others) or SCHEDULE_FUSED_Z (the first-stage y sweep beside the x
    sweep, then both z stages in one march); the first three give bitwise the same results,
    fused z the same up to rounding."""
    c = Config()
    lib.ctu_config_default(C.byref(c))
    c.nx, c.ny, c.nz = int(nx), int(ny), int(nz)
    c.dx, c.dy, c.dz = float(dx), float(dy), float(dz)
    c.gamma = float(gamma)
    for i in range(6):
        c.bc[i] = int(bc[i])
    c.prec = int(prec)
    c.cfl = float(cfl)
    c.newton_tol = float(newton_tol)
    c.newton_max_iter = int(newton_max_iter)
    c.p_floor = float(p_floor)
    if march_seg is None or x_rows is None or x_chunks is None:
        from .autotune import lookup, lookup_batch, lookup_x
        tb = lookup_batch(int(prec)) if batch else None
        if tb is not None:
            march_seg = (tb[0], tb[0]) if march_seg is None else march_seg
            x_rows = tb[1] if x_rows is None else x_rows
            x_chunks = tb[2] if x_chunks is None else x_chunks
        if march_seg is None:
            march_seg = lookup(int(prec), int(ny), int(nz))
        tx = lookup_x(int(prec), int(nx), int(ny))
        x_rows = tx[0] if x_rows is None else x_rows
        x_chunks = tx[1] if x_chunks is None else x_chunks
    c.march_seg[0], c.march_seg[1] = int(march_seg[0]), int(march_seg[1])
    c.x_rows, c.x_chunks = int(x_rows), int(x_chunks)
    c.riemann = int(riemann)
    c.recon = int(recon)
    c.h_correction = int(h_correction)
    c.schedule = int(schedule)
    return c


def workspace_bytes(cfg: Config):
    s, w = C.c_size_t(), C.c_size_t()
    _check(lib.ctu_workspace_bytes(C.byref(cfg), C.byref(s), C.byref(w)))
    return s.value, w.value


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU visible: the CTU library runs on an MI355X (gfx950) only")
    return torch


STREAM_READ, STREAM_COPY, STREAM_ADD, STREAM_COMBINE5 = 0, 1, 2, 3


def stream_probe_blocks(n: int) -> int:
    """Doubles the output of a STREAM_READ probe over n elements needs."""
    return int(lib.ctu_stream_probe_blocks(C.c_size_t(n)))


def stream_probe(kind: int, a, b, c, n: int, stream=None) -> None:
    """One launch of a plain streaming kernel (ctu_stream_probe) over torch float64 device
    tensors a, b (or None) and c, n elements; on `stream` (default: torch's current)."""
    torch = _torch()
    stream = stream if stream is not None else torch.cuda.current_stream()
    _check(lib.ctu_stream_probe(int(kind), C.c_void_p(a.data_ptr()),
                                C.c_void_p(b.data_ptr() if b is not None else 0),
                                C.c_void_p(c.data_ptr()), C.c_size_t(n),
                                C.c_void_p(stream.cuda_stream)))


NOALLOC_SCRATCH_BYTES = 128 << 20


def step_noalloc(cfg: Config, d_state, dt: float, stream=None) -> None:
    """One CTU step of the state held in the torch device tensor d_state (the library's layout,
    workspace_bytes(cfg)[0] bytes) with the library's fixed scratch as workspace
    (ctu_step_noalloc); on `stream` (default: torch's current)."""
    torch = _torch()
    stream = stream if stream is not None else torch.cuda.current_stream()
    _check(lib.ctu_step_noalloc(C.byref(cfg), C.c_void_p(d_state.data_ptr()), float(dt),
                                C.c_void_p(stream.cuda_stream)))


class Grid:
    """One grid: device state and workspace held as torch uint8 tensors."""

    def __init__(self, cfg: Config, device: str = "cuda", stream=None):
        torch = _torch()
        self.cfg = cfg
        self.n = (cfg.nx, cfg.ny, cfg.nz)
        self.dtype = np.float64 if cfg.prec == FP64 else np.float32
        sb, wb = workspace_bytes(cfg)
        self.state_bytes, self.work_bytes = sb, wb
        self.device = torch.device(device)
        self.state = torch.empty(sb, dtype=torch.uint8, device=self.device)
        self.work = torch.empty(wb, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        _check(lib.ctu_grid_create(C.byref(cfg), C.c_void_p(self.state.data_ptr()),
                                   C.c_void_p(self.work.data_ptr()), C.c_size_t(wb),
                                   C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self.handle = h

    @classmethod
    def from_workload(cls, wl, prec=FP64, stream=None, **kw) -> "Grid":
        cfg = make_config(wl.nx, wl.ny, wl.nz, wl.dx, wl.dy, wl.dz, wl.gamma, wl.bc, prec,
                          kw.pop("cfl", wl.cfl), **kw)
        g = cls(cfg, stream=stream)
        g.set_primitive(wl.W)
        return g

    def close(self):
        if getattr(self, "handle", None):
            lib.ctu_grid_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- data ------------------------------------------------------------------------------
    def _host_ptrs(self, arrays):
        arr = (C.c_void_p * 5)()
        for f in range(5):
            arr[f] = arrays[f].ctypes.data
        return arr

    def set_state(self, U: np.ndarray) -> None:
        """Conserved real-cell values, shape (5, nz, ny, nx)."""
        fields = [np.ascontiguousarray(U[f], dtype=self.dtype) for f in range(5)]
        _check(lib.ctu_set_state(self.handle, self._host_ptrs(fields)))

    def set_primitive(self, W: np.ndarray) -> None:
        """Primitive real-cell values (rho, u, v, w, p), shape (5, nz, ny, nx), float64."""
        fields = [np.ascontiguousarray(W[f], dtype=np.float64) for f in range(5)]
        _check(lib.ctu_set_primitive(self.handle, self._host_ptrs(fields)))

    def get_state(self, allow_nonphys: bool = False) -> np.ndarray:
        nx, ny, nz = self.n
        out = np.empty((5, nz, ny, nx), dtype=self.dtype)
        fields = [out[f] for f in range(5)]
        _check(lib.ctu_get_state(self.handle, self._host_ptrs(fields)),
               allow=(ENONPHYS,) if allow_nonphys else ())
        return out

    def debug_keep_fluxes(self, keep: bool = True) -> None:
        """Also store the x CTU fluxes of each step (for debug_fluxes(1, 0))."""
        _check(lib.ctu_debug_keep_fluxes(self.handle, 1 if keep else 0))

    def debug_fluxes(self, which: int, direction: int) -> np.ndarray:
        """Fluxes of the last step over the allocated box (5, NZ, NY, NX), float64."""
        nx, ny, nz = self.n
        g2 = 2 * self.info().ghost
        out = np.empty((5, nz + g2, ny + g2, nx + g2), dtype=np.float64)
        _check(lib.ctu_debug_fluxes(self.handle, which, direction,
                                    self._host_ptrs([out[f] for f in range(5)])))
        return out

    # -- stepping -------------------------------------------------------------------------
    def compute_dt(self) -> float:
        dt = C.c_double()
        _check(lib.ctu_compute_dt(self.handle, C.byref(dt)))
        return dt.value

    def step(self, dt: float) -> None:
        _check(lib.ctu_step(self.handle, float(dt)))

    def advance(self, nsteps: int, t_end: float = float("inf")) -> None:
        _check(lib.ctu_advance(self.handle, int(nsteps), float(t_end)))

    def totals(self) -> np.ndarray:
        out = (C.c_double * 5)()
        _check(lib.ctu_totals(self.handle, out))
        return np.array(out[:])

    def check(self):
        flags = C.c_uint32()
        cnt = (C.c_uint64 * 4)()
        status = lib.ctu_check(self.handle, C.byref(flags), cnt)
        return status, flags.value, list(cnt)

    def profile_enable(self, on: bool = True, newton: bool = False) -> None:
        """Per-kernel event timing (on), and/or the Newton-iteration histogram (newton)."""
        mode = (PROFILE_TIMING if on else 0) | (PROFILE_NEWTON if newton else 0)
        _check(lib.ctu_profile_enable(self.handle, mode))

    def newton_histogram(self) -> dict:
        out = (C.c_uint64 * 8)()
        _check(lib.ctu_newton_histogram(self.handle, out))
        return dict(zip(NEWTON_BINS, [int(v) for v in out]))

    def profile_read(self) -> dict:
        """{kernel class: (total ms, launches)} accumulated since profile_enable."""
        n = 32
        ms = (C.c_double * n)()
        la = (C.c_int64 * n)()
        cnt = C.c_int32()
        _check(lib.ctu_profile_read(self.handle, n, ms, la, C.byref(cnt)))
        return {lib.ctu_profile_name(k).decode(): (ms[k], la[k]) for k in range(cnt.value)}

    def info(self) -> GridInfo:
        info = GridInfo()
        _check(lib.ctu_grid_info_get(self.handle, C.byref(info)))
        return info


class Batch:
    """Continuous batch of independent grids (ctu_batch_* in ctu.h): every pass of a step is
    one launch over all running grids of a precision."""

    def __init__(self, max_slots: int, graph: bool = False, stream=None, device: str = "cuda"):
        torch = _torch()
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        wb = C.c_size_t()
        _check(lib.ctu_batch_workspace_bytes(int(max_slots), C.byref(wb)))
        self.work = torch.empty(wb.value, dtype=torch.uint8, device=torch.device(device))
        h = C.c_void_p()
        _check(lib.ctu_batch_create(int(max_slots), C.c_void_p(self.work.data_ptr()),
                                    C.c_size_t(wb.value), C.c_void_p(self.stream.cuda_stream),
                                    BATCH_GRAPH if graph else 0, C.byref(h)))
        self.handle = h
        self._grids = {}  # ticket -> grid, keeps submitted grids alive

    def submit(self, grid: Grid, nsteps: int, t_end: float = float("inf")) -> Optional[int]:
        """Ticket, or None when every slot is taken."""
        t = C.c_uint64()
        s = _check(lib.ctu_batch_submit(self.handle, grid.handle, int(nsteps), float(t_end),
                                        C.byref(t)), allow=(EAGAIN,))
        if s == EAGAIN:
            return None
        self._grids[t.value] = grid
        return t.value

    def run(self, steps: int) -> None:
        _check(lib.ctu_batch_run(self.handle, int(steps)))

    def poll(self, ticket: int):
        """(state, t); a DONE or FAILED ticket releases its slot and grid."""
        state = C.c_int32()
        t = C.c_double()
        _check(lib.ctu_batch_poll(self.handle, C.c_uint64(ticket), C.byref(state), C.byref(t)))
        if state.value in (TICKET_DONE, TICKET_FAILED, TICKET_UNKNOWN):
            self._grids.pop(ticket, None)
        return state.value, t.value

    def close(self):
        if getattr(self, "handle", None):
            lib.ctu_batch_destroy(self.handle)
            self.handle = None
            self._grids = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
