"""CPU oracle for the CTU step (TEST INFRASTRUCTURE ONLY): PPMC or PPMP reconstruction, the
exact or the Roe/HLLE Riemann solver, the optional H correction.

Thin ctypes wrapper over ``libctu_oracle.so`` (plain serial FP64 C, see ctu_oracle.c), or,
after ``set_threads(n)``, over the OpenMP build of the same source (``libctu_oracle_omp.so``,
bit-identical results).
Only the tests, the smoke check and the benchmark's CPU-baseline leg import this package;
the GPU library never does.  Arrays are numpy float64; a conserved state is a (5, NZ, NY, NX)
array over the allocated box (``Config.ng`` ghost layers per side: 3 with PPMC, 4 with PPMP,
one more with the H correction), fields (rho, mx, my, mz, E).
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field
from typing import Optional, Sequence, Tuple

import numpy as np

NG = 3  # ghost layers of the PPMC configuration (Config.ng in general)
BC_PERIODIC = 0
BC_OUTFLOW = 1
BC_REFLECT = 2
RIEMANN_EXACT, RIEMANN_ROE = 0, 1
RECON_PPMC, RECON_PPMP = 0, 1

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBPATH = os.environ.get("CTU_ORACLE_LIB") or os.path.join(_HERE, "libctu_oracle.so")
# the OpenMP build of the same source (z-planes shared among threads, bit-identical results)
_LIBPATH_OMP = None if os.environ.get("CTU_ORACLE_LIB") else os.path.join(_HERE, "libctu_oracle_omp.so")
_lib = None
_libs = {}


class _Config(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double),
                ("gamma", C.c_double), ("bc", C.c_int * 6), ("cfl", C.c_double),
                ("newton_tol", C.c_double), ("newton_max_iter", C.c_int),
                ("p_floor", C.c_double), ("riemann", C.c_int), ("h_correction", C.c_int),
                ("recon", C.c_int)]


class _Stats(C.Structure):
    _fields_ = [("solves", C.c_long), ("newton_iters", C.c_long),
                ("newton_capped", C.c_long), ("p_floored", C.c_long), ("hlle", C.c_long)]


_dp = C.POINTER(C.c_double)


def _load():
    global _lib
    if _lib is None:
        _lib = _open(_LIBPATH)
    return _lib


def set_threads(n: int) -> int:
    """Threads of the whole-grid operations (step, update_box): 1 selects the serial build,
    n > 1 the OpenMP build with n threads.  Returns the count in effect (1 when only the
    serial library is available, e.g. a library given by CTU_ORACLE_LIB)."""
    global _lib
    if n <= 1 or _LIBPATH_OMP is None:
        _lib = _open(_LIBPATH)
        return 1
    _lib = _open(_LIBPATH_OMP)
    return int(_lib.ref_threads(int(n)))


def threads() -> int:
    """Threads the whole-grid operations currently use."""
    return int(_load().ref_threads(0))


def _open(path):
    if path in _libs:
        return _libs[path]
    if not os.path.exists(path):
        from . import build as _b  # noqa: F401  (build on first use)
        _b.build()
    lib = C.CDLL(path)
    lib.ref_threads.argtypes = [C.c_int]
    lib.ref_threads.restype = C.c_int
    lib.ref_cons_to_prim.argtypes = [_dp, C.c_double, C.c_double, _dp]
    lib.ref_cons_to_prim.restype = C.c_int
    lib.ref_prim_to_cons.argtypes = [_dp, C.c_double, _dp]
    lib.ref_char_project.argtypes = [_dp, C.c_double, C.c_double, _dp]
    lib.ref_char_unproject.argtypes = [_dp, C.c_double, C.c_double, _dp]
    lib.ref_plmc_slope.argtypes = [_dp, _dp, _dp, C.c_double, _dp]
    lib.ref_ppmc.argtypes = [_dp, C.c_double, C.c_double, _dp, _dp, _dp]
    lib.ref_riemann_star.argtypes = [_dp, _dp, C.c_double, C.c_double, C.c_int, C.c_double,
                                     _dp, _dp, C.POINTER(C.c_int)]
    lib.ref_riemann_star.restype = C.c_int
    lib.ref_riemann_sample.argtypes = [_dp, _dp, C.c_double, C.c_double, C.c_double,
                                       C.c_double, _dp]
    lib.ref_riemann_sample.restype = C.c_int
    lib.ref_riemann_wave_speeds.argtypes = [_dp, _dp, C.c_double, C.c_double, C.c_double, _dp]
    lib.ref_riemann_flux.argtypes = [_dp, _dp, C.c_double, C.c_double, C.c_int, C.c_double,
                                     _dp, C.POINTER(_Stats)]
    lib.ref_ppmp.argtypes = [_dp, C.c_double, C.c_double, C.c_double, _dp, _dp, _dp]
    lib.ref_ppmp_flattening.argtypes = [_dp]
    lib.ref_ppmp_flattening.restype = C.c_double
    lib.ref_ppmp_steepening.argtypes = [_dp, C.c_double, C.c_double]
    lib.ref_ppmp_steepening.restype = C.c_double
    lib.ref_ghost_width.argtypes = [C.POINTER(_Config)]
    lib.ref_ghost_width.restype = C.c_int
    lib.ref_roe_flux.argtypes = [_dp, _dp, C.c_double, C.c_double, C.c_double, _dp,
                                 C.POINTER(_Stats)]
    lib.ref_roe_flux.restype = C.c_int
    lib.ref_bc_fill.argtypes = [C.POINTER(_Config), C.POINTER(_dp)]
    lib.ref_bc_fill.restype = C.c_int
    lib.ref_compute_dt.argtypes = [C.POINTER(_Config), C.POINTER(_dp)]
    lib.ref_compute_dt.restype = C.c_double
    lib.ref_ctu_update_box.argtypes = [C.POINTER(_Config), C.POINTER(_dp), C.c_double,
                                       C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(_dp),
                                       C.POINTER(_dp), C.POINTER(_dp), C.POINTER(_Stats)]
    lib.ref_ctu_update_box.restype = C.c_int
    lib.ref_ctu_step.argtypes = [C.POINTER(_Config), C.POINTER(_dp), C.c_double,
                                 C.POINTER(_Stats)]
    lib.ref_ctu_step.restype = C.c_int
    _libs[path] = lib
    return lib


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


def _vec(x, n) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(n))
    return a


@dataclass
class Config:
    """Grid and solver parameters (mirrors the oracle's C struct)."""
    nx: int
    ny: int
    nz: int
    dx: float
    dy: float
    dz: float
    gamma: float
    bc: Sequence[int] = (BC_PERIODIC,) * 6
    cfl: float = 0.3
    newton_tol: float = 1e-6
    newton_max_iter: int = 50
    p_floor: float = 1e-20
    riemann: int = 0          # RIEMANN_EXACT or RIEMANN_ROE
    h_correction: int = 0     # 1: H correction of the second-stage Roe fluxes
    recon: int = 0            # RECON_PPMC or RECON_PPMP

    def _c(self) -> _Config:
        c = _Config()
        c.nx, c.ny, c.nz = self.nx, self.ny, self.nz
        c.dx, c.dy, c.dz = self.dx, self.dy, self.dz
        c.gamma = self.gamma
        for i in range(6):
            c.bc[i] = int(self.bc[i])
        c.cfl = self.cfl
        c.newton_tol = self.newton_tol
        c.newton_max_iter = self.newton_max_iter
        c.p_floor = self.p_floor
        c.riemann = self.riemann
        c.h_correction = self.h_correction
        c.recon = self.recon
        return c

    @property
    def ng(self) -> int:
        """Ghost layers per side (3 for PPMC; 4 for PPMP or with the H correction)."""
        return int(_load().ref_ghost_width(C.byref(self._c())))

    @property
    def alloc_shape(self) -> Tuple[int, int, int]:
        g = self.ng
        return (self.nz + 2 * g, self.ny + 2 * g, self.nx + 2 * g)


@dataclass
class Stats:
    solves: int = 0
    newton_iters: int = 0
    newton_capped: int = 0
    p_floored: int = 0
    hlle: int = 0


def _stats_out(s: _Stats) -> Stats:
    return Stats(s.solves, s.newton_iters, s.newton_capped, s.p_floored, s.hlle)


# --- pointwise pieces ----------------------------------------------------------------------

def cons_to_prim(U, gamma: float, p_floor: float = 1e-20) -> np.ndarray:
    lib = _load()
    U = _vec(U, 5)
    W = np.zeros(5)
    lib.ref_cons_to_prim(_ptr(U), gamma, p_floor, _ptr(W))
    return W


def prim_to_cons(W, gamma: float) -> np.ndarray:
    lib = _load()
    W = _vec(W, 5)
    U = np.zeros(5)
    lib.ref_prim_to_cons(_ptr(W), gamma, _ptr(U))
    return U


def char_project(d, rho: float, a: float) -> np.ndarray:
    lib = _load()
    d = _vec(d, 5)
    xi = np.zeros(5)
    lib.ref_char_project(_ptr(d), rho, a, _ptr(xi))
    return xi


def char_unproject(xi, rho: float, a: float) -> np.ndarray:
    lib = _load()
    xi = _vec(xi, 5)
    d = np.zeros(5)
    lib.ref_char_unproject(_ptr(xi), rho, a, _ptr(d))
    return d


def plmc_slope(wm, w0, wp, gamma: float) -> np.ndarray:
    lib = _load()
    wm, w0, wp = _vec(wm, 5), _vec(w0, 5), _vec(wp, 5)
    dw = np.zeros(5)
    lib.ref_plmc_slope(_ptr(wm), _ptr(w0), _ptr(wp), gamma, _ptr(dw))
    return dw


def ppmc(w5x5, dtodx: float, gamma: float):
    """PPMC of the centre cell of a 5-cell stencil of rotated primitives.

    Returns (W*_L, W*_R, W_L, W_R): traced states and the monotonized face values."""
    lib = _load()
    w = np.ascontiguousarray(np.asarray(w5x5, dtype=np.float64).reshape(5, 5))
    wl, wr, wlr = np.zeros(5), np.zeros(5), np.zeros(10)
    lib.ref_ppmc(_ptr(w), dtodx, gamma, _ptr(wl), _ptr(wr), _ptr(wlr))
    return wl, wr, wlr[:5].copy(), wlr[5:].copy()


def riemann_star(WL, WR, gamma: float, tol: float = 1e-6, max_iter: int = 50,
                 p_floor: float = 1e-20):
    """Star pressure and velocity of the exact Riemann problem; WL, WR = (rho, u, p)."""
    lib = _load()
    wl, wr = _vec(WL, 3), _vec(WR, 3)
    ps, us = C.c_double(), C.c_double()
    capped = C.c_int()
    it = lib.ref_riemann_star(_ptr(wl), _ptr(wr), gamma, tol, max_iter, p_floor,
                              C.byref(ps), C.byref(us), C.byref(capped))
    return ps.value, us.value, it, bool(capped.value)


def riemann_sample(WL, WR, pstar: float, ustar: float, gamma: float, S: float):
    lib = _load()
    wl, wr = _vec(WL, 3), _vec(WR, 3)
    out = np.zeros(3)
    side = lib.ref_riemann_sample(_ptr(wl), _ptr(wr), pstar, ustar, gamma, S, _ptr(out))
    return out, side


def riemann_wave_speeds(WL, WR, pstar: float, ustar: float, gamma: float) -> np.ndarray:
    lib = _load()
    wl, wr = _vec(WL, 3), _vec(WR, 3)
    out = np.zeros(5)
    lib.ref_riemann_wave_speeds(_ptr(wl), _ptr(wr), pstar, ustar, gamma, _ptr(out))
    return out


def exact_solution(WL, WR, gamma: float, xi: np.ndarray, tol: float = 1e-14,
                   max_iter: int = 200) -> np.ndarray:
    """Exact Riemann solution (rho, u, p) at similarity coordinates xi = (x - x0)/t."""
    ps, us, _, _ = riemann_star(WL, WR, gamma, tol, max_iter)
    out = np.zeros((3, len(xi)))
    for n, s in enumerate(np.asarray(xi, dtype=np.float64)):
        out[:, n], _ = riemann_sample(WL, WR, ps, us, gamma, float(s))
    return out


def riemann_flux(UL, UR, gamma: float, tol: float = 1e-6, max_iter: int = 50,
                 p_floor: float = 1e-20):
    lib = _load()
    ul, ur = _vec(UL, 5), _vec(UR, 5)
    F = np.zeros(5)
    st = _Stats()
    lib.ref_riemann_flux(_ptr(ul), _ptr(ur), gamma, tol, max_iter, p_floor, _ptr(F),
                         C.byref(st))
    return F, _stats_out(st)


def ppmp(w7x5, dtodx: float, dx: float, gamma: float):
    """PPMP traced face states of the centre cell of 7 rotated primitive states; returns
    (WsL, WsR, WL_mono, WR_mono)."""
    lib = _load()
    w = _vec(w7x5, 35)
    L, R, LR = np.zeros(5), np.zeros(5), np.zeros(10)
    lib.ref_ppmp(_ptr(w), dtodx, dx, gamma, _ptr(L), _ptr(R), _ptr(LR))
    return L, R, LR[:5].copy(), LR[5:].copy()


def ppmp_coefficients(w7x5, gamma: float, dx: float):
    """(flattening F, steepening eta) of the centre cell of 7 rotated primitive states."""
    lib = _load()
    w = _vec(w7x5, 35)
    return (float(lib.ref_ppmp_flattening(_ptr(w))),
            float(lib.ref_ppmp_steepening(_ptr(w), gamma, dx)))


def roe_flux(UL, UR, gamma: float, p_floor: float = 1e-20, eta_h: float = 0.0):
    """Roe flux with the HLLE failsafe; returns (F, used_hlle, stats)."""
    lib = _load()
    ul, ur = _vec(UL, 5), _vec(UR, 5)
    F = np.zeros(5)
    st = _Stats()
    used = lib.ref_roe_flux(_ptr(ul), _ptr(ur), gamma, p_floor, eta_h, _ptr(F), C.byref(st))
    return F, bool(used), _stats_out(st)


# --- whole-grid operations ------------------------------------------------------------------

def _field_ptrs(u: np.ndarray):
    assert u.dtype == np.float64 and u.flags.c_contiguous and u.shape[0] == 5
    arr = (_dp * 5)()
    for f in range(5):
        arr[f] = u[f].ctypes.data_as(_dp)
    return arr


def alloc_state(cfg: Config) -> np.ndarray:
    return np.zeros((5,) + cfg.alloc_shape, dtype=np.float64)


def bc_fill(cfg: Config, u: np.ndarray) -> None:
    if _load().ref_bc_fill(C.byref(cfg._c()), _field_ptrs(u)) != 0:
        raise ValueError("a reflecting boundary needs >= 3 cells on its axis")


def compute_dt(cfg: Config, u: np.ndarray) -> float:
    return float(_load().ref_compute_dt(C.byref(cfg._c()), _field_ptrs(u)))


def step(cfg: Config, u: np.ndarray, dt: float) -> Stats:
    """One CTU step in place (ghost fill included)."""
    st = _Stats()
    rc = _load().ref_ctu_step(C.byref(cfg._c()), _field_ptrs(u), dt, C.byref(st))
    if rc != 0:
        raise ValueError("oracle step failed")
    return _stats_out(st)


def update_box(cfg: Config, u: np.ndarray, dt: float, lo, hi, want_fluxes: bool = False):
    """u^{n+1} on the real-cell box [lo, hi) (x, y, z order) of a ghost-filled state.

    Returns (out, stats) with out of shape (5, nz_box, ny_box, nx_box); with want_fluxes
    also the first-stage and CTU flux arrays, each (3, 5) + alloc_shape (face i+1/2 at i)."""
    lib = _load()
    lo3 = (C.c_int * 3)(*[int(v) for v in lo])
    hi3 = (C.c_int * 3)(*[int(v) for v in hi])
    shape = tuple(int(hi[a] - lo[a]) for a in (2, 1, 0))
    out = np.zeros((5,) + shape)
    st = _Stats()
    fs_arr = fh_arr = None
    fstar = fhalf = None
    if want_fluxes:
        fstar = np.full((3, 5) + cfg.alloc_shape, np.nan)
        fhalf = np.full((3, 5) + cfg.alloc_shape, np.nan)
        fs_arr = (_dp * 15)()
        fh_arr = (_dp * 15)()
        for d in range(3):
            for f in range(5):
                fs_arr[d * 5 + f] = fstar[d, f].ctypes.data_as(_dp)
                fh_arr[d * 5 + f] = fhalf[d, f].ctypes.data_as(_dp)
    rc = lib.ref_ctu_update_box(C.byref(cfg._c()), _field_ptrs(u), dt, lo3, hi3,
                                _field_ptrs(out), fs_arr, fh_arr, C.byref(st))
    if rc != 0:
        raise ValueError("invalid box")
    if want_fluxes:
        return out, _stats_out(st), fstar, fhalf
    return out, _stats_out(st)


def real(cfg: Config, u: np.ndarray) -> np.ndarray:
    """View of the real cells of an allocated state."""
    g = cfg.ng
    return u[:, g:g + cfg.nz, g:g + cfg.ny, g:g + cfg.nx]


def state_from_primitive(cfg: Config, W: np.ndarray) -> np.ndarray:
    """Allocated conserved state from real-cell primitives W of shape (5, nz, ny, nx).

    Uses the oracle's own EOS conversion, cell by cell in a numpy-vectorized restatement of
    ref_prim_to_cons (same operation order)."""
    g = cfg.gamma
    u = alloc_state(cfg)
    rho, vx, vy, vz, p = (np.asarray(W[q], dtype=np.float64) for q in range(5))
    r = real(cfg, u)
    r[0] = rho
    r[1] = rho * vx
    r[2] = rho * vy
    r[3] = rho * vz
    r[4] = p / (g - 1.0) + 0.5 * rho * (vx * vx + vy * vy + vz * vz)
    return u
