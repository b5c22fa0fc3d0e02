"""Pins of the oracle's Roe solver and its HLLE failsafe (Sec. 2.3.2-2.3.3, App. B.2) and of
the H-correction eigenvalue floor (App. C).

What fixes the answer, independently of the oracle's own formulas:
* consistency: equal states give the physical flux f(U) exactly;
* Roe's property: the jump across a single shock or contact is one eigenvector of the
  Roe matrix, so an isolated stationary or moving shock, or a contact, gets the exact
  upwind flux;
* completeness of the eigen-decomposition: with the H-correction speed above every
  |lambda| the flux collapses to the local Lax-Friedrichs flux (F_L + F_R)/2 - eta dU/2,
  which involves no eigenvector at all;
* mirror symmetry; second-order agreement with the exact solver on weak waves;
* the HLLE flux in its textbook form (b+ F_L - b- F_R + b+ b- dU) / (b+ - b-) on the
  Einfeldt 1-2-3 problem, where the linearization produces a negative intermediate state.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_1410_4194_amd import workloads as WL


def cons(w, g):
    """Conserved (rho, mx, my, mz, E) of primitives (rho, u, v, w, p), written out here."""
    r, u, v, ww, p = w
    return np.array([r, r * u, r * v, r * ww, p / (g - 1.0) + 0.5 * r * (u * u + v * v + ww * ww)])


def phys_flux(w, g):
    r, u, v, ww, p = w
    E = p / (g - 1.0) + 0.5 * r * (u * u + v * v + ww * ww)
    return np.array([r * u, r * u * u + p, r * u * v, r * u * ww, (E + p) * u])


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


@pytest.mark.parametrize("w", [(1.0, 0.3, -0.2, 0.5, 1.0), (0.125, -0.7, 0.1, 0.0, 0.1),
                               (2.0, 5.0, 1.0, 1.0, 1.0), (1.0, -4.0, 0.0, 0.2, 0.5)])
def test_equal_states_give_physical_flux(w):
    g = 1.4
    U = cons(w, g)
    F, used, st = O.roe_flux(U, U, g)
    assert not used
    assert _rel(F, phys_flux(w, g)) <= 4e-16


@pytest.mark.parametrize("mach", [1.5, 3.0, 10.0])
@pytest.mark.parametrize("g", [1.4, 5.0 / 3.0])
def test_stationary_shock_is_exact(mach, g):
    """Shock frame: upstream (1, M a, 1) | downstream from the Rankine-Hugoniot jump.  The
    jump is the eigenvector of speed 0, so the Roe flux equals the common physical flux."""
    rho2, u2_lab, p2, vs = WL.normal_shock(mach, 1.0, 1.0, g)
    wl = (1.0, vs, 0.0, 0.0, 1.0)
    wr = (rho2, vs - u2_lab, 0.0, 0.0, p2)
    FL, FR = phys_flux(wl, g), phys_flux(wr, g)
    assert _rel(FL, FR) <= 1e-13
    F, used, _ = O.roe_flux(cons(wl, g), cons(wr, g), g)
    assert not used
    assert _rel(F, FL) <= 1e-12


@pytest.mark.parametrize("mach", [1.2, 2.0, 6.0])
def test_moving_shock_gets_upwind_flux(mach):
    """Lab frame, shock moving right into gas at rest on the right: one wave of speed
    v_s > 0 with the subsonic side moving slower, so the Roe flux is the left flux."""
    g = 1.4
    rho2, u2, p2, vs = WL.normal_shock(mach, 1.0, 1.0, g)
    wl = (rho2, u2, 0.0, 0.0, p2)
    wr = (1.0, 0.0, 0.0, 0.0, 1.0)
    F, used, _ = O.roe_flux(cons(wl, g), cons(wr, g), g)
    assert not used
    # the subsonic check: the Roe acoustic speeds straddle 0
    assert _rel(F, phys_flux(wl, g)) <= 1e-12


@pytest.mark.parametrize("u", [0.0, 0.4, -0.3])
def test_contact_and_shear_get_upwind_flux(u):
    """Density and transverse-velocity jumps at equal u and p: contact and shear waves of
    speed u; the flux is the upwind physical flux (either side when u = 0)."""
    g = 1.4
    wl = (1.0, u, 0.3, -0.1, 1.0)
    wr = (0.2, u, -0.5, 0.7, 1.0)
    F, used, _ = O.roe_flux(cons(wl, g), cons(wr, g), g)
    assert not used
    up = phys_flux(wl if u >= 0.0 else wr, g)
    if u == 0.0:
        assert np.allclose(F, up, rtol=0, atol=1e-15)
    else:
        assert _rel(F, up) <= 1e-13


@pytest.mark.parametrize("seed", range(8))
def test_large_eta_gives_local_lax_friedrichs(seed):
    """|lambda| -> max(|lambda|, eta) with eta above every eigenvalue: the dissipation term
    becomes eta * sum(xi R) = eta * dU, so the flux is (F_L + F_R)/2 - eta (U_R - U_L)/2."""
    rng = np.random.default_rng(100 + seed)
    g = 1.4 if seed % 2 else 5.0 / 3.0
    wl = (10 ** rng.uniform(-0.5, 0.5), rng.uniform(-0.5, 0.5), rng.uniform(-1, 1),
          rng.uniform(-1, 1), 10 ** rng.uniform(-0.3, 0.3))
    wr = (10 ** rng.uniform(-0.5, 0.5), rng.uniform(-0.5, 0.5), rng.uniform(-1, 1),
          rng.uniform(-1, 1), 10 ** rng.uniform(-0.3, 0.3))
    UL, UR = cons(wl, g), cons(wr, g)
    eta = 50.0
    F, used, _ = O.roe_flux(UL, UR, g, eta_h=eta)
    if used:
        pytest.skip("HLLE branch for this draw")
    llf = 0.5 * (phys_flux(wl, g) + phys_flux(wr, g)) - 0.5 * eta * (UR - UL)
    assert _rel(F, llf) <= 1e-13


@pytest.mark.parametrize("seed", range(10))
def test_mirror_symmetry(seed):
    """Reflecting x: (L, R) -> (mirror R, mirror L) negates the mass, transverse-momentum and
    energy fluxes and keeps the normal-momentum flux; both branches."""
    rng = np.random.default_rng(200 + seed)
    g = 1.4
    mach = 0.5 if seed < 5 else 4.0  # large jumps reach the HLLE branch
    ws = [(10 ** rng.uniform(-1, 1), mach * rng.uniform(-1, 1), rng.uniform(-1, 1),
           rng.uniform(-1, 1), 10 ** rng.uniform(-1, 1)) for _ in range(2)]
    wl, wr = ws
    F, used, _ = O.roe_flux(cons(wl, g), cons(wr, g), g)
    m = lambda w: (w[0], -w[1], w[2], w[3], w[4])
    Fm, used_m, _ = O.roe_flux(cons(m(wr), g), cons(m(wl), g), g)
    assert used == used_m
    exp = np.array([-F[0], F[1], -F[2], -F[3], -F[4]])
    assert np.max(np.abs(Fm - exp)) <= 1e-13 * max(np.max(np.abs(F)), 1.0)


def test_weak_waves_agree_with_exact_to_second_order():
    """For jumps of size d the Roe and exact Godunov fluxes differ by O(d^2) or better."""
    g = 1.4
    base = np.array([1.0, 0.2, 0.1, -0.1, 1.0])
    dirv = np.array([0.7, -0.4, 0.3, 0.2, 0.9])
    errs = []
    for d in (1e-1, 5e-2, 2.5e-2):
        wl, wr = base - 0.5 * d * dirv, base + 0.5 * d * dirv
        Fr, used, _ = O.roe_flux(cons(wl, g), cons(wr, g), g)
        Fe, _ = O.riemann_flux(cons(wl, g), cons(wr, g), g, tol=1e-14)
        errs.append(np.max(np.abs(Fr - Fe)))
    assert errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.5, errs


def test_123_problem_falls_back_to_hlle():
    """Einfeldt's 1-2-3 problem: the linearized intermediate state has negative pressure,
    so the HLLE flux is returned; it matches the textbook HLL form with the bounding speeds
    min(u_L - a_L, lambda-) and max(u_R + a_R, lambda+), and its mass and energy fluxes
    vanish by symmetry."""
    g = 1.4
    wl, wr = (1.0, -2.0, 0.0, 0.0, 0.4), (1.0, 2.0, 0.0, 0.0, 0.4)
    UL, UR = cons(wl, g), cons(wr, g)
    F, used, st = O.roe_flux(UL, UR, g)
    assert used and st.hlle == 1
    # Roe-averaged speeds (equal densities: plain means)
    HL = (UL[4] + wl[4]) / wl[0]
    HR = (UR[4] + wr[4]) / wr[0]
    ut, Ht = 0.5 * (wl[1] + wr[1]), 0.5 * (HL + HR)
    at = math.sqrt((g - 1.0) * (Ht - 0.5 * ut * ut))
    aL, aR = math.sqrt(g * 0.4), math.sqrt(g * 0.4)
    bm = min(ut - at, wl[1] - aL, 0.0)
    bp = max(ut + at, wr[1] + aR, 0.0)
    hll = (bp * phys_flux(wl, g) - bm * phys_flux(wr, g) + bp * bm * (UR - UL)) / (bp - bm)
    assert _rel(F, hll) <= 1e-14
    assert F[0] == pytest.approx(0.0, abs=1e-15) and F[4] == pytest.approx(0.0, abs=1e-15)


def test_hlle_keeps_positive_states():
    """Where the fallback fires, a first-order Godunov update with the HLLE flux keeps the
    cell averages positive (the property that motivates the failsafe), on strong random
    rarefactions."""
    g = 1.4
    rng = np.random.default_rng(7)
    fired = 0
    for _ in range(200):
        r, p = 10 ** rng.uniform(-1, 1), 10 ** rng.uniform(-2, 1)
        a = math.sqrt(g * p / r)
        du = rng.uniform(1.0, 6.0) * a
        wl, wr = (r, -du, 0.0, 0.0, p), (r * rng.uniform(0.8, 1.2), du, 0.0, 0.0, p)
        UL, UR = cons(wl, g), cons(wr, g)
        F, used, _ = O.roe_flux(UL, UR, g)
        if not used:
            continue
        fired += 1
        # left cell after one step with dt/dx chosen at CFL 0.5 of the largest speed
        smax = max(abs(wl[1]) + a, abs(wr[1]) + math.sqrt(g * wr[4] / wr[0]))
        lam = 0.5 / smax
        Un = UL - lam * (F - phys_flux(wl, g))
        assert Un[0] > 0.0
        assert Un[4] - 0.5 * Un[1] ** 2 / Un[0] > 0.0
    assert fired > 20


def test_supersonic_shortcuts():
    g = 1.4
    wl = (1.0, 3.0, 0.1, 0.2, 1.0)
    wr = (0.5, 2.5, -0.1, 0.0, 0.8)
    F, used, _ = O.roe_flux(cons(wl, g), cons(wr, g), g)
    assert np.array_equal(F, phys_flux(wl, g)) or _rel(F, phys_flux(wl, g)) <= 4e-16
    ml = (wr[0], -wr[1], wr[2], wr[3], wr[4])
    mr = (wl[0], -wl[1], wl[2], wl[3], wl[4])
    F2, used2, _ = O.roe_flux(cons(ml, g), cons(mr, g), g)
    assert _rel(F2, phys_flux(mr, g)) <= 4e-16


# --- whole CTU step with the Roe solver ----------------------------------------------------

from tests.common import oracle_config, oracle_state, run_oracle  # noqa: E402


def test_roe_step_keeps_uniform_flow():
    wl = WL.random_state(9, 7, 6, seed=3)
    wl.W[:] = np.array([1.3, 0.4, -0.2, 0.7, 2.0])[:, None, None, None]
    cfg = oracle_config(wl, riemann=O.RIEMANN_ROE)
    u = oracle_state(wl, cfg)
    before = O.real(cfg, u).copy()
    O.step(cfg, u, 0.5 * O.compute_dt(cfg, u))
    assert np.array_equal(O.real(cfg, u), before)


def test_roe_step_conserves_on_periodic_grid():
    wl = WL.random_state(11, 9, 8, seed=4)
    cfg = oracle_config(wl, riemann=O.RIEMANN_ROE)
    u = oracle_state(wl, cfg)
    r0 = O.real(cfg, u).reshape(5, -1).copy()
    for _ in range(3):
        O.step(cfg, u, O.compute_dt(cfg, u))
    r1 = O.real(cfg, u).reshape(5, -1)
    for f in range(5):
        assert abs(math.fsum(r1[f]) - math.fsum(r0[f])) <= 1e-13 * math.fsum(np.abs(r0[f]))


def test_roe_sod_matches_exact_solution():
    """Sod to t = 0.2 with the Roe solver: mean density error against the exact solution is
    as small as with the exact solver (the solvers differ only inside the waves)."""
    wl = WL.sod(128, 1, 1)
    cfg = oracle_config(wl, riemann=O.RIEMANN_ROE)
    cfg, u, t, n = run_oracle(wl, t_end=0.2, cfg=cfg)
    x = (np.arange(128) + 0.5) / 128
    ex = O.exact_solution((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), 1.4, (x - 0.5) / 0.2)
    r = O.real(cfg, u)[:, 0, 0, :]
    assert np.mean(np.abs(r[0] - ex[0])) < 0.004


def test_roe_strong_rarefaction_stays_physical():
    """The 1-2-3 problem to t = 0.15: HLLE keeps density and pressure positive where the
    linearization alone would not."""
    wl = WL.strong_rarefaction(128, 1, 1)
    cfg = oracle_config(wl, riemann=O.RIEMANN_ROE)
    u = oracle_state(wl, cfg)
    t, hlle = 0.0, 0
    while t < 0.15 * (1 - 1e-14):
        dt = min(O.compute_dt(cfg, u), 0.15 - t)
        hlle += O.step(cfg, u, dt).hlle
        t += dt
    r = O.real(cfg, u)[:, 0, 0, :]
    p = 0.4 * (r[4] - 0.5 * r[1] ** 2 / r[0])
    assert np.all(r[0] > 0) and np.all(p > 0)
    assert hlle > 0
