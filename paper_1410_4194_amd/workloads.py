"""Seeded synthetic inputs (initial conditions) for the CTU timestep.

This module only builds input fields; it holds none of the timestep's arithmetic.  Every
generator returns a :class:`Workload` whose primitive fields ``W`` = (rho, u, v, w, p) are
float64 arrays of shape (5, nz, ny, nx) over the real cells, x fastest.  The GPU library
and the CPU oracle each convert them to conserved variables with their own code.

Workloads follow the test problems of the paper (Sec. 4) and the shock-cloud setup of
Sec. 5, with synthetic stand-ins where the paper used data that is not available
(its turbulent "realistic cloud" is replaced by a seeded lognormal random field).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

BASE_SEED = 14104194
PERIODIC = 0
OUTFLOW = 1
REFLECT = 2


@dataclass
class Workload:
    name: str
    nx: int
    ny: int
    nz: int
    dx: float
    dy: float
    dz: float
    gamma: float
    bc: Tuple[int, int, int, int, int, int]
    W: np.ndarray                      # (5, nz, ny, nx) primitives, float64
    cfl: float = 0.3
    steps: Optional[int] = None
    t_end: Optional[float] = None
    meta: dict = field(default_factory=dict)

    @property
    def cells(self) -> int:
        return self.nx * self.ny * self.nz


def _centres(n: int, d: float) -> np.ndarray:
    return (np.arange(n, dtype=np.float64) + 0.5) * d


def normal_shock(mach: float, rho1: float, p1: float, gamma: float):
    """Exact Rankine-Hugoniot state behind a plane shock of Mach number `mach` running into
    gas at rest (rho1, p1).  Returns (rho2, u2, p2, shock_speed)."""
    m2 = mach * mach
    a1 = math.sqrt(gamma * p1 / rho1)
    vs = mach * a1
    rho2 = rho1 * (gamma + 1.0) * m2 / ((gamma - 1.0) * m2 + 2.0)
    p2 = p1 * (2.0 * gamma * m2 - (gamma - 1.0)) / (gamma + 1.0)
    u2 = vs * (1.0 - rho1 / rho2)
    return rho2, u2, p2, vs


def strong_shock_limit(mach: float, rho1: float, p1: float, gamma: float):
    """Strong-shock limits of Sec. 5.1: (rho, v, p) behind a Mach `mach` shock."""
    a1 = math.sqrt(gamma * p1 / rho1)
    vs = mach * a1
    return ((gamma + 1.0) / (gamma - 1.0) * rho1, 2.0 / (gamma + 1.0) * vs,
            2.0 * gamma / (gamma + 1.0) * mach * mach * p1)


def cloud_crushing_time(radius: float, chi: float, shock_speed: float) -> float:
    """t_cc = r_cl chi^(1/2) / v_s (Sec. 5, eq. t_cc)."""
    return radius * math.sqrt(chi) / shock_speed


# ------------------------------------------------------------------------------------------
# 1D Riemann problems embedded in 3D (Sec. 4.1)
# ------------------------------------------------------------------------------------------

def riemann_tube(left, right, n: int = 128, ny: int = 1, nz: int = 1, axis: int = 0,
                 gamma: float = 1.4, x0: float = 0.5, t_end: float = 0.2, cfl: float = 0.3,
                 name: str = "riemann") -> Workload:
    """Shock tube along `axis` on [0, 1] with n cells; cubic cells; outflow along the tube,
    periodic across it.  left/right = (rho, u_normal, p)."""
    dims = [ny, nz]
    shape3 = [n, ny, nz] if axis == 0 else ([ny, n, nz] if axis == 1 else [ny, nz, n])
    nx_, ny_, nz_ = shape3
    d = 1.0 / n
    xc = _centres(n, d)
    lm = xc < x0
    W = np.zeros((5, nz_, ny_, nx_))
    bshape = [1, 1, 1]
    bshape[2 - axis] = n
    lm = lm.reshape(bshape)
    W[0] = np.where(lm, left[0], right[0])
    W[1 + axis] = np.where(lm, left[1], right[1])
    W[4] = np.where(lm, left[2], right[2])
    bc = [PERIODIC] * 6
    bc[2 * axis] = OUTFLOW
    bc[2 * axis + 1] = OUTFLOW
    del dims
    return Workload(name, nx_, ny_, nz_, d, d, d, gamma, tuple(bc), W, cfl=cfl, t_end=t_end,
                    meta={"axis": axis, "x0": x0, "left": tuple(left), "right": tuple(right)})


def sod(n: int = 128, ny: int = 16, nz: int = 16, axis: int = 0) -> Workload:
    """Sod tube, (1, 0, 1) | (0.125, 0, 0.1), gamma 1.4, t = 0.2 (Sec. 4.1.1; standard
    right state)."""
    return riemann_tube((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), n, ny, nz, axis, 1.4, 0.5, 0.2,
                        name=f"sod_{n}x{ny}x{nz}")


def strong_shock_tube(n: int = 100, ny: int = 1, nz: int = 1) -> Workload:
    """Strong shock tube (10, 0, 100) | (1, 0, 1), gamma 1.4, t = 0.07 (Sec. 4.1.2)."""
    return riemann_tube((10.0, 0.0, 100.0), (1.0, 0.0, 1.0), n, ny, nz, 0, 1.4, 0.5, 0.07,
                        name="strong_shock")


def strong_rarefaction(n: int = 128, ny: int = 1, nz: int = 1) -> Workload:
    """Einfeldt 123 problem (1, -2, 0.4) | (1, 2, 0.4), gamma 1.4, t = 0.15 (Sec. 4.1.3)."""
    return riemann_tube((1.0, -2.0, 0.4), (1.0, 2.0, 0.4), n, ny, nz, 0, 1.4, 0.5, 0.15,
                        name="strong_rarefaction")


def blast_waves(n: int = 400, ny: int = 1, nz: int = 1) -> Workload:
    """Interacting blast waves (Sec. 4.1.5): rho = 1, u = 0, gamma 1.4 on x in [0, 1] with
    p = 1000 for x < 0.1, p = 100 for x > 0.9 and p = 0.01 between; reflecting walls at both
    ends of x, periodic across; t = 0.038."""
    d = 1.0 / n
    xc = _centres(n, d)
    p = np.where(xc < 0.1, 1000.0, np.where(xc > 0.9, 100.0, 0.01))
    W = np.zeros((5, nz, ny, n))
    W[0] = 1.0
    W[4] = p.reshape(1, 1, n)
    bc = (REFLECT, REFLECT, PERIODIC, PERIODIC, PERIODIC, PERIODIC)
    return Workload(f"blast_waves_{n}", n, ny, nz, d, d, d, 1.4, bc, W, cfl=0.3, t_end=0.038)


def implosion(n: int = 400, nz: int = 1) -> Workload:
    """Implosion (Sec. 4.2.1): the quadrant [0, 0.3]^2 with reflecting walls on all four
    sides; rho = 0.125, p = 0.14 inside the diamond x + y < 0.15, rho = 1, p = 1 outside, at
    rest, gamma 1.4; periodic along z (nz copies of the 2D problem); t = 0.045 (early) or
    2.5 (jet).  The initial state is symmetric under x <-> y, and so is the exact solution."""
    d = 0.3 / n
    xc = _centres(n, d)
    inside = (xc.reshape(1, n) + xc.reshape(n, 1)) < 0.15
    W = np.zeros((5, nz, n, n))
    W[0] = np.where(inside, 0.125, 1.0)
    W[4] = np.where(inside, 0.14, 1.0)
    bc = (REFLECT, REFLECT, REFLECT, REFLECT, PERIODIC, PERIODIC)
    return Workload(f"implosion_{n}", n, n, nz, d, d, d, 1.4, bc, W, cfl=0.3, t_end=0.045)


def noh(n: int = 64, p0: float = 1e-6) -> Workload:
    """Noh's strong shock in 3D (Sec. 4.3.1): the octant [0, 1]^3 at rho = 1 moving at unit
    speed toward the origin, gamma 5/3, reflecting walls at x = 0, y = 0, z = 0.  The paper
    starts from zero pressure and sets the outer faces from the analytic solution; here the
    pressure is p0 (the pressure floor keeps the solver defined) and the outer faces are
    outflow, which leaves the solution inside r < 1 - t untouched.  Analytic: shock at
    r = t/3, density 64 behind it, (1 + t/r)^2 ahead of it."""
    d = 1.0 / n
    xc = _centres(n, d)
    z, y, x = np.meshgrid(xc, xc, xc, indexing="ij")
    r = np.sqrt(x * x + y * y + z * z)
    W = np.zeros((5, n, n, n))
    W[0] = 1.0
    W[1] = -x / r
    W[2] = -y / r
    W[3] = -z / r
    W[4] = p0
    bc = (REFLECT, OUTFLOW, REFLECT, OUTFLOW, REFLECT, OUTFLOW)
    return Workload(f"noh_{n}^3", n, n, n, d, d, d, 5.0 / 3.0, bc, W, cfl=0.3, t_end=0.6)


def shock_duct(nx: int = 96, ny: int = 16, nz: int = 1, mach: float = 6.0,
               amp: float = 1e-3) -> Workload:
    """A plane shock aligned with the grid running down a duct (the carbuncle setting of
    Sec. 4.3.1 and App. C): gas at rest (rho = 1, p = 1/gamma, gamma 1.4) ahead of a Mach
    `mach` shock that starts at x = 0.5, the Rankine-Hugoniot state behind it, cell width
    1/ny, walls across y, outflow along x, periodic along z.  One cell ahead of the shock on
    the duct's centre line has its density raised by the fraction `amp`: a scheme prone to
    the carbuncle grows that seed into cross-flow, a dissipative one carries it as a small
    contact."""
    g = 1.4
    d = 1.0 / ny
    rho2, u2, p2, _ = normal_shock(mach, 1.0, 1.0 / g, g)
    post = (_centres(nx, d) < 0.5).reshape(1, 1, nx)
    W = np.zeros((5, nz, ny, nx))
    W[0] = np.where(post, rho2, 1.0)
    W[1] = np.where(post, u2, 0.0)
    W[4] = np.where(post, p2, 1.0 / g)
    W[0, :, ny // 2, int(0.8 * ny)] *= 1.0 + amp
    bc = (OUTFLOW, OUTFLOW, REFLECT, REFLECT, PERIODIC, PERIODIC)
    return Workload(f"shock_duct_{nx}x{ny}x{nz}", nx, ny, nz, d, d, d, g, bc, W, cfl=0.3)


# ------------------------------------------------------------------------------------------
# Shock-cloud problems (Sec. 5)
# ------------------------------------------------------------------------------------------

def shock_cloud(n: int = 256, mach: float = 10.0, chi: float = 10.0, radius: float = 0.1,
                centre=(0.3, 0.5, 0.5), x_shock: float = 0.1, gamma: float = 5.0 / 3.0,
                steps: Optional[int] = 100, cfl: float = 0.3) -> Workload:
    """Uniform spherical cloud (density contrast chi, pressure equilibrium) in ambient gas
    (rho, p) = (1, 1) at rest on [0, 1]^3, hit by a plane shock moving in +x whose
    post-shock state (x < x_shock) is the exact Rankine-Hugoniot state.  Outflow on all
    faces; the zero-gradient x- face then feeds post-shock gas, like the paper's inflow."""
    d = 1.0 / n
    x = _centres(n, d)
    X = x[None, None, :]
    Y = x[None, :, None]
    Z = x[:, None, None]
    r2 = (X - centre[0]) ** 2 + (Y - centre[1]) ** 2 + (Z - centre[2]) ** 2
    rho = np.where(r2 <= radius * radius, chi, 1.0) * np.ones((n, n, n))
    rho2, u2, p2, vs = normal_shock(mach, 1.0, 1.0, gamma)
    post = np.broadcast_to(X < x_shock, (n, n, n))
    W = np.zeros((5, n, n, n))
    W[0] = np.where(post, rho2, rho)
    W[1] = np.where(post, u2, 0.0)
    W[4] = np.where(post, p2, 1.0)
    return Workload(f"shock_cloud_{n}^3", n, n, n, d, d, d, gamma, (OUTFLOW,) * 6, W, cfl=cfl,
                    steps=steps,
                    meta={"mach": mach, "chi": chi, "radius": radius, "shock_speed": vs,
                          "post_shock": (rho2, u2, p2), "t_cc": cloud_crushing_time(radius, chi, vs)})


def shock_cloud_requests(count: int, rate: float, seed: int = BASE_SEED + 5,
                         sizes: Sequence[int] = (64, 96, 128, 192),
                         chi_range=(10.0, 1000.0), mach_range=(1.5, 10.0),
                         radius_range=(0.08, 0.15), t_cc_factor: float = 1.5,
                         gamma: float = 5.0 / 3.0):
    """Poisson-arriving shock-cloud solve requests: arrival times (seconds after the first
    possible arrival, exponential gaps of mean 1/rate) and per request a grid edge drawn
    from `sizes`, a cloud density contrast log-uniform in chi_range, a shock Mach number
    uniform in mach_range and a cloud radius uniform in radius_range; each runs to
    t_cc_factor cloud-crushing times.  Returns a list of dicts; the initial state is built
    by ``request_workload``."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=count)
    arrivals = np.cumsum(gaps) - gaps[0]
    out = []
    for i in range(count):
        n = int(rng.choice(np.asarray(sizes)))
        chi = float(10.0 ** rng.uniform(math.log10(chi_range[0]), math.log10(chi_range[1])))
        mach = float(rng.uniform(*mach_range))
        radius = float(rng.uniform(*radius_range))
        vs = normal_shock(mach, 1.0, 1.0, gamma)[3]
        out.append({"rid": i, "arrival": float(arrivals[i]), "n": n, "chi": chi, "mach": mach,
                    "radius": radius, "gamma": gamma,
                    "t_end": t_cc_factor * cloud_crushing_time(radius, chi, vs)})
    return out


def request_workload(req: dict) -> Workload:
    """Initial state of one request from ``shock_cloud_requests``."""
    return shock_cloud(req["n"], mach=req["mach"], chi=req["chi"], radius=req["radius"],
                       gamma=req["gamma"], steps=None)


def estimated_steps(req: dict, cfl: float = 0.3) -> float:
    """Rough step count of a request: t_end over the CFL step of the post-shock gas (the
    fastest signal of the initial state)."""
    rho2, u2, p2, _ = normal_shock(req["mach"], 1.0, 1.0, req["gamma"])
    speed = u2 + math.sqrt(req["gamma"] * p2 / rho2)
    return req["t_end"] / (cfl / req["n"] / speed)


def gaussian_random_field(n: int, slope: float, seed: int) -> np.ndarray:
    """Zero-mean Gaussian random field on an n^3 periodic grid with power spectrum
    P(k) ~ k^slope (white noise filtered by |k|^(slope/2), k = 0 removed)."""
    rng = np.random.default_rng(seed)
    white = rng.standard_normal((n, n, n))
    fk = np.fft.rfftn(white)
    kx = np.fft.rfftfreq(n) * n
    ky = np.fft.fftfreq(n) * n
    k2 = kx[None, None, :] ** 2 + ky[None, :, None] ** 2 + ky[:, None, None] ** 2
    k2[0, 0, 0] = 1.0
    filt = k2 ** (slope / 4.0)
    filt[0, 0, 0] = 0.0
    fk *= filt
    g = np.fft.irfftn(fk, s=(n, n, n), axes=(0, 1, 2))
    return g


def turbulent_cloud(n: int = 512, mach: float = 10.0, mean_chi: float = 10.0,
                    sigma_ln: float = 1.0, radius: float = 0.15, centre=(0.3, 0.5, 0.5),
                    x_shock: float = 0.1, gamma: float = 5.0 / 3.0, steps: int = 50,
                    seed: int = BASE_SEED + 3, cfl: float = 0.3) -> Workload:
    """Cloud with a lognormal density, rho = max(1, A exp(sigma g)), g a unit-variance
    Gaussian random field with P(k) ~ k^(-11/3) (normalized over the cloud), A set by
    bisection so the cloud-mean density equals mean_chi; pressure equilibrium, Mach shock
    as in :func:`shock_cloud`.  Synthetic stand-in for the paper's turbulent cloud."""
    d = 1.0 / n
    x = _centres(n, d)
    X = x[None, None, :]
    Y = x[None, :, None]
    Z = x[:, None, None]
    inside = ((X - centre[0]) ** 2 + (Y - centre[1]) ** 2 + (Z - centre[2]) ** 2) <= radius ** 2
    g = gaussian_random_field(n, -11.0 / 3.0, seed)
    gi = g[inside]
    gi = (gi - gi.mean()) / gi.std()
    lo, hi = 1e-6, 1e6
    for _ in range(200):
        A = math.sqrt(lo * hi)
        m = np.maximum(1.0, A * np.exp(sigma_ln * gi)).mean()
        if m < mean_chi:
            lo = A
        else:
            hi = A
    A = math.sqrt(lo * hi)
    rho = np.ones((n, n, n))
    rho[inside] = np.maximum(1.0, A * np.exp(sigma_ln * gi))
    rho2, u2, p2, vs = normal_shock(mach, 1.0, 1.0, gamma)
    post = np.broadcast_to(X < x_shock, (n, n, n))
    W = np.zeros((5, n, n, n))
    W[0] = np.where(post, rho2, rho)
    W[1] = np.where(post, u2, 0.0)
    W[4] = np.where(post, p2, 1.0)
    return Workload(f"turbulent_cloud_{n}^3", n, n, n, d, d, d, gamma, (OUTFLOW,) * 6, W,
                    cfl=cfl, steps=steps, meta={"mach": mach, "mean_chi": mean_chi, "A": A,
                                                "shock_speed": vs})


# ------------------------------------------------------------------------------------------
# Periodic problems
# ------------------------------------------------------------------------------------------

def kelvin_helmholtz(nx: int, ny: int, nz: int, gamma: float = 1.4, steps: int = 200,
                     cfl: float = 0.3) -> Workload:
    """3D shear layer on [0, 1]^3 (cell widths 1/n per axis): rho = 2, u = -0.5 for
    1/3 < y < 2/3, else rho = 1, u = +0.5; v = 0.01 sin(2 pi x); p = 2.5; periodic
    (Sec. 4.2.3, extended to 3D with a v-only perturbation)."""
    dx, dy, dz = 1.0 / nx, 1.0 / ny, 1.0 / nz
    x = _centres(nx, dx)[None, None, :]
    y = _centres(ny, dy)[None, :, None]
    band = np.broadcast_to((y > 1.0 / 3.0) & (y < 2.0 / 3.0), (nz, ny, nx))
    W = np.zeros((5, nz, ny, nx))
    W[0] = np.where(band, 2.0, 1.0)
    W[1] = np.where(band, -0.5, 0.5)
    W[2] = np.broadcast_to(0.01 * np.sin(2.0 * np.pi * x), (nz, ny, nx))
    W[4] = 2.5
    return Workload(f"kh_{nx}x{ny}x{nz}", nx, ny, nz, dx, dy, dz, gamma, (PERIODIC,) * 6, W,
                    cfl=cfl, steps=steps)


def kh_batch(count: int = 64, edges: Sequence[int] = (32, 48, 64, 96, 128),
             seed: int = BASE_SEED + 4, steps: int = 200) -> List[Workload]:
    """`count` Kelvin-Helmholtz problems with per-axis edges drawn uniformly from `edges`."""
    rng = np.random.default_rng(seed)
    sizes = rng.choice(np.asarray(edges), size=(count, 3))
    return [kelvin_helmholtz(int(a), int(b), int(c), steps=steps) for a, b, c in sizes]


def sound_wave(n: int, axis: int = 0, amp: float = 1e-6, gamma: float = 5.0 / 3.0,
               periods: float = 1.0, cfl: float = 0.3) -> Workload:
    """Right-moving linear sound wave along `axis` (rho0 = 1, a0 = 1), periodic; after
    `periods` periods the exact solution equals the initial state."""
    shape = [1, 1, 1]
    shape[axis] = n
    nx, ny, nz = shape
    d = 1.0 / n
    s = np.sin(2.0 * np.pi * _centres(n, d))
    bshape = [1, 1, 1]
    bshape[2 - axis] = n
    s = s.reshape(bshape)
    p0 = 1.0 / gamma
    W = np.zeros((5, nz, ny, nx))
    W[0] = 1.0 + amp * s
    W[1 + axis] = amp * s
    W[4] = p0 + amp * s
    return Workload(f"sound_{n}_{'xyz'[axis]}", nx, ny, nz, d, d, d, gamma, (PERIODIC,) * 6, W,
                    cfl=cfl, t_end=periods)


def diagonal_advection(n: int, nz: int = 1, gamma: float = 5.0 / 3.0, amp: float = 0.1,
                       cfl: float = 0.3) -> Workload:
    """Density wave rho = 1 + amp sin(2 pi (x + y)) advected with V = (1, 1, 0) at uniform
    pressure 1 on a periodic n x n x nz box (cell width 1/n): exact solution is a
    translation, periodic in time with period 1."""
    d = 1.0 / n
    x = _centres(n, d)[None, None, :]
    y = _centres(n, d)[None, :, None]
    W = np.zeros((5, nz, n, n))
    W[0] = np.broadcast_to(1.0 + amp * np.sin(2.0 * np.pi * (x + y)), (nz, n, n))
    W[1] = 1.0
    W[2] = 1.0
    W[4] = 1.0
    return Workload(f"diag_adv_{n}", n, n, nz, d, d, d, gamma, (PERIODIC,) * 6, W, cfl=cfl,
                    t_end=1.0)


def random_state(nx: int, ny: int, nz: int, seed: int, rough: bool = True,
                 gamma: float = 1.4, bc=(PERIODIC,) * 6, mach: float = 1.0,
                 spacing=(1.0, 1.0, 1.0)) -> Workload:
    """Random positive state for parity and invariance tests.  rough=True draws independent
    cell values (discontinuities everywhere, every limiter branch exercised); rough=False
    draws a few random Fourier modes (smooth)."""
    rng = np.random.default_rng(seed)
    W = np.zeros((5, nz, ny, nx))
    if rough:
        W[0] = 10.0 ** rng.uniform(-0.5, 0.5, size=(nz, ny, nx))
        W[4] = 10.0 ** rng.uniform(-0.5, 0.5, size=(nz, ny, nx))
        for q in (1, 2, 3):
            W[q] = mach * rng.uniform(-1.0, 1.0, size=(nz, ny, nx))
    else:
        z, y, x = np.meshgrid(np.arange(nz) / nz, np.arange(ny) / ny, np.arange(nx) / nx,
                              indexing="ij")
        for q in range(5):
            acc = np.zeros((nz, ny, nx))
            for _ in range(3):
                k = rng.integers(0, 3, size=3)
                ph = rng.uniform(0, 2 * np.pi)
                acc += rng.uniform(0.1, 0.3) * np.sin(2 * np.pi * (k[0] * x + k[1] * y + k[2] * z) + ph)
            W[q] = (1.0 + 0.5 * acc) if q in (0, 4) else mach * acc
    dx, dy, dz = (s / n for s, n in zip(spacing, (nx, ny, nz)))
    return Workload(f"random_{'rough' if rough else 'smooth'}_{nx}x{ny}x{nz}_s{seed}", nx, ny,
                    nz, dx, dy, dz, gamma, tuple(bc), W)
