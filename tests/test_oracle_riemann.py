"""Pins of the oracle's exact Riemann solver (App. B.1) against physics it must satisfy.

None of these checks re-evaluates the solver's own pressure function: shocks are checked
with the Rankine-Hugoniot conservation laws, rarefactions with isentropy and the Riemann
invariants, the star pressure with closed forms derived independently (two-rarefaction
formula; symmetric two-shock collision solved from the jump conditions), and the sampling
with Galilean invariance and the flux identities of any consistent Riemann solver.
"""
import math

import numpy as np
import pytest

RNG_SEED = 14104194


def _states(rng, n, gamma):
    """Random non-vacuum left/right states (rho, u, p)."""
    out = []
    while len(out) < n:
        rl, rr, pl, pr = 10.0 ** rng.uniform(-3, 3, size=4)
        ul, ur = rng.uniform(-5, 5, size=2)
        al, ar = math.sqrt(gamma * pl / rl), math.sqrt(gamma * pr / rr)
        if ur - ul >= 2.0 * (al + ar) / (gamma - 1.0) * 0.95:
            continue  # (near-)vacuum generation: the floors define the answer there
        out.append(((rl, ul, pl), (rr, ur, pr)))
    return out


def _energy(rho, u, p, gamma):
    return p / (gamma - 1.0) + 0.5 * rho * u * u


def _rh_residuals(pre, post, s, gamma):
    """Mass, momentum and energy flux jumps across a discontinuity moving at speed s."""
    (r1, u1, p1), (r2, u2, p2) = pre, post
    m1, m2 = r1 * (u1 - s), r2 * (u2 - s)
    q1, q2 = r1 * u1 * (u1 - s) + p1, r2 * u2 * (u2 - s) + p2
    e1 = _energy(r1, u1, p1, gamma) * (u1 - s) + p1 * u1
    e2 = _energy(r2, u2, p2, gamma) * (u2 - s) + p2 * u2
    scale_m = abs(r1 * (abs(u1) + abs(s))) + abs(r2 * (abs(u2) + abs(s)))
    scale_q = abs(r1 * (u1 * u1 + abs(u1 * s))) + p1 + p2 + abs(r2 * (u2 * u2 + abs(u2 * s)))
    scale_e = (abs(_energy(r1, u1, p1, gamma)) * (abs(u1) + abs(s)) + abs(p1 * u1)
               + abs(_energy(r2, u2, p2, gamma)) * (abs(u2) + abs(s)) + abs(p2 * u2))
    return abs(m1 - m2) / scale_m, abs(q1 - q2) / scale_q, abs(e1 - e2) / scale_e


@pytest.mark.parametrize("gamma", [1.4, 5.0 / 3.0])
def test_shocks_satisfy_rankine_hugoniot(oracle, gamma):
    rng = np.random.default_rng(RNG_SEED)
    n_shocks = 0
    for WL, WR in _states(rng, 300, gamma):
        ps, us, _, capped = oracle.riemann_star(WL, WR, gamma, tol=1e-14, max_iter=200)
        assert not capped
        sp = oracle.riemann_wave_speeds(WL, WR, ps, us, gamma)
        if ps > WL[2]:
            star, _ = oracle.riemann_sample(WL, WR, ps, us, gamma, 0.5 * (sp[1] + us))
            assert max(_rh_residuals(WL, star, sp[0], gamma)) < 1e-11
            n_shocks += 1
        if ps > WR[2]:
            star, _ = oracle.riemann_sample(WL, WR, ps, us, gamma, 0.5 * (sp[3] + us))
            assert max(_rh_residuals(WR, star, sp[4], gamma)) < 1e-11
            n_shocks += 1
    assert n_shocks > 100


@pytest.mark.parametrize("gamma", [1.4, 5.0 / 3.0])
def test_rarefactions_are_isentropic_simple_waves(oracle, gamma):
    rng = np.random.default_rng(RNG_SEED + 1)
    n_rare = 0
    for WL, WR in _states(rng, 300, gamma):
        ps, us, _, _ = oracle.riemann_star(WL, WR, gamma, tol=1e-14, max_iter=200)
        sp = oracle.riemann_wave_speeds(WL, WR, ps, us, gamma)
        for side, W, head, tail, sgn in ((0, WL, sp[0], sp[1], 1.0), (1, WR, sp[4], sp[3], -1.0)):
            if ps > W[2]:
                continue
            n_rare += 1
            r0, u0, p0 = W
            a0 = math.sqrt(gamma * p0 / r0)
            entropy0 = p0 / r0 ** gamma
            inv0 = u0 + sgn * 2.0 * a0 / (gamma - 1.0)
            # star state on this side of the contact, and three points inside the fan
            xs = [0.5 * (tail + us)] + [head + f * (tail - head) for f in (0.25, 0.5, 0.75)]
            for n, S in enumerate(xs):
                (r, u, p), _ = oracle.riemann_sample(WL, WR, ps, us, gamma, S)
                a = math.sqrt(gamma * p / r)
                assert abs(p / r ** gamma - entropy0) <= 1e-11 * entropy0
                inv = u + sgn * 2.0 * a / (gamma - 1.0)
                assert abs(inv - inv0) <= 1e-11 * (abs(inv0) + a0)
                if n > 0:  # inside the fan the sample sits on the characteristic u -/+ a = S
                    assert abs((u - sgn * a) - S) <= 1e-11 * (abs(S) + a0 + abs(u0))
    assert n_rare > 100


@pytest.mark.parametrize("gamma", [1.4, 5.0 / 3.0])
def test_contact_continuity(oracle, gamma):
    rng = np.random.default_rng(RNG_SEED + 2)
    for WL, WR in _states(rng, 100, gamma):
        ps, us, _, _ = oracle.riemann_star(WL, WR, gamma, tol=1e-14, max_iter=200)
        eps = 1e-9 * (1.0 + abs(us))
        left, sl = oracle.riemann_sample(WL, WR, ps, us, gamma, us - eps)
        right, sr = oracle.riemann_sample(WL, WR, ps, us, gamma, us + eps)
        assert (sl, sr) == (0, 1)
        assert left[2] == ps and right[2] == ps
        assert left[1] == us and right[1] == us


@pytest.mark.parametrize("gamma", [1.4, 5.0 / 3.0])
def test_two_rarefaction_closed_form(oracle, gamma):
    """When both waves are rarefactions the star pressure has a closed form."""
    rng = np.random.default_rng(RNG_SEED + 3)
    z = (gamma - 1.0) / (2.0 * gamma)
    checked = 0
    for WL, WR in _states(rng, 400, gamma):
        ps, us, _, _ = oracle.riemann_star(WL, WR, gamma, tol=1e-14, max_iter=200)
        if ps >= min(WL[2], WR[2]) or ps <= 1e-5:
            continue
        (rl, ul, pl), (rr, ur, pr) = WL, WR
        al, ar = math.sqrt(gamma * pl / rl), math.sqrt(gamma * pr / rr)
        exact = ((al + ar - 0.5 * (gamma - 1.0) * (ur - ul)) / (al / pl ** z + ar / pr ** z)) ** (1.0 / z)
        assert abs(ps - exact) <= 1e-11 * exact
        checked += 1
    assert checked > 30
    # Einfeldt "123" problem: symmetric two-rarefaction case, u* = 0 exactly.
    ps, us, _, _ = oracle.riemann_star((1.0, -2.0, 0.4), (1.0, 2.0, 0.4), 1.4, 1e-14, 200)
    a = math.sqrt(1.4 * 0.4)
    exact = (((2 * a - 0.2 * 4.0) / (2 * a / 0.4 ** (0.4 / 2.8))) ** (2.8 / 0.4))
    assert abs(ps - exact) <= 1e-11 * exact and us == 0.0


@pytest.mark.parametrize("gamma", [1.4, 5.0 / 3.0])
@pytest.mark.parametrize("U,rho,p", [(1.0, 1.0, 1.0), (10.0, 2.0, 0.5), (0.3, 0.1, 3.0)])
def test_symmetric_collision_from_jump_conditions(oracle, gamma, U, rho, p):
    """Two equal streams colliding at +/-U stop the gas between two shocks.  Mass, momentum
    and energy conservation across the right shock give a quadratic for its speed s:
    s^2 + (3-gamma)U s/2 - ((gamma-1)U^2/2 + gamma p/rho) = 0, and p* = p + rho U (U + s)."""
    b = 0.5 * (3.0 - gamma) * U
    c = -(0.5 * (gamma - 1.0) * U * U + gamma * p / rho)
    s = 0.5 * (-b + math.sqrt(b * b - 4.0 * c))
    p_exact = p + rho * U * (U + s)
    ps, us, _, _ = oracle.riemann_star((rho, U, p), (rho, -U, p), gamma, 1e-14, 200)
    assert abs(ps - p_exact) <= 1e-12 * p_exact
    assert abs(us) <= 1e-13 * U
    sp = oracle.riemann_wave_speeds((rho, U, p), (rho, -U, p), ps, us, gamma)
    assert abs(sp[4] - s) <= 1e-12 * (abs(s) + U)


@pytest.mark.parametrize("gamma", [1.4, 5.0 / 3.0])
def test_galilean_invariance(oracle, gamma):
    rng = np.random.default_rng(RNG_SEED + 4)
    for WL, WR in _states(rng, 60, gamma):
        V = rng.uniform(-3, 3)
        ps, us, _, _ = oracle.riemann_star(WL, WR, gamma, 1e-14, 200)
        WLs = (WL[0], WL[1] + V, WL[2])
        WRs = (WR[0], WR[1] + V, WR[2])
        ps2, us2, _, _ = oracle.riemann_star(WLs, WRs, gamma, 1e-14, 200)
        scale = abs(us) + abs(V) + math.sqrt(gamma * max(WL[2] / WL[0], WR[2] / WR[0]))
        assert abs(ps2 - ps) <= 1e-11 * ps
        assert abs(us2 - (us + V)) <= 1e-11 * scale
        for S in rng.uniform(-6, 6, size=5):
            a, _ = oracle.riemann_sample(WL, WR, ps, us, gamma, S)
            b, _ = oracle.riemann_sample(WLs, WRs, ps2, us2, gamma, S + V)
            if abs(S - us) < 1e-6 * scale:
                continue
            assert abs(b[0] - a[0]) <= 1e-9 * a[0]
            assert abs(b[1] - (a[1] + V)) <= 1e-9 * scale
            assert abs(b[2] - a[2]) <= 1e-9 * a[2]


def test_newton_tolerance(oracle):
    """At the default tolerance 1e-6 the quadratic convergence leaves ~1e-12 relative error."""
    rng = np.random.default_rng(RNG_SEED + 5)
    for WL, WR in _states(rng, 300, 1.4):
        p6, _, it, capped = oracle.riemann_star(WL, WR, 1.4, 1e-6, 50)
        p14, _, _, _ = oracle.riemann_star(WL, WR, 1.4, 1e-14, 200)
        assert not capped and it <= 20
        if p14 > 1e-5:
            assert abs(p6 - p14) <= 1e-9 * p14


def test_sod_wave_positions(oracle):
    """Sod tube (rho, u, p) = (1, 0, 1) | (0.125, 0, 0.1), gamma = 1.4: the rarefaction head
    moves at -a_L, and the sampled profile at t = 0.2 has the four features in order."""
    WL, WR = (1.0, 0.0, 1.0), (0.125, 0.0, 0.1)
    ps, us, _, _ = oracle.riemann_star(WL, WR, 1.4, 1e-14, 200)
    sp = oracle.riemann_wave_speeds(WL, WR, ps, us, 1.4)
    assert sp[0] == pytest.approx(-math.sqrt(1.4), rel=1e-15)
    x = 0.5 + 0.2 * sp
    assert x[0] < x[1] < x[2] < x[3] == x[4]
    # star pressure and velocity of the Sod problem (textbook values, 5 digits)
    assert ps == pytest.approx(0.30313, abs=1e-5)
    assert us == pytest.approx(0.92745, abs=1e-5)


def _flux_of_state(U, gamma):
    """Euler x-flux f(u) of eq. (x_flux) for a conserved state."""
    rho, mx, my, mz, E = U
    u, v, w = mx / rho, my / rho, mz / rho
    p = (gamma - 1.0) * (E - 0.5 * rho * (u * u + v * v + w * w))
    return np.array([rho * u, rho * u * u + p, rho * u * v, rho * u * w, (E + p) * u])


@pytest.mark.parametrize("gamma", [1.4, 5.0 / 3.0])
def test_flux_consistency_mirror_and_contact(oracle, gamma):
    rng = np.random.default_rng(RNG_SEED + 6)
    for _ in range(100):
        rho, p = 10.0 ** rng.uniform(-2, 2, size=2)
        u, v, w = rng.uniform(-3, 3, size=3)
        U = oracle.prim_to_cons((rho, u, v, w, p), gamma)
        F, _ = oracle.riemann_flux(U, U, gamma)
        ref = _flux_of_state(U, gamma)
        assert np.allclose(F, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())
    for WL, WR in _states(rng, 100, gamma):
        vl, wl, vr, wr = rng.uniform(-1, 1, size=4)
        UL = oracle.prim_to_cons((WL[0], WL[1], vl, wl, WL[2]), gamma)
        UR = oracle.prim_to_cons((WR[0], WR[1], vr, wr, WR[2]), gamma)
        F, _ = oracle.riemann_flux(UL, UR, gamma, tol=1e-14, max_iter=200)
        # mirror image: swap sides and reverse the normal velocity
        UR_m = oracle.prim_to_cons((WL[0], -WL[1], vl, wl, WL[2]), gamma)
        UL_m = oracle.prim_to_cons((WR[0], -WR[1], vr, wr, WR[2]), gamma)
        Fm, _ = oracle.riemann_flux(UL_m, UR_m, gamma, tol=1e-14, max_iter=200)
        scale = np.abs(F).max() + 1e-300
        assert abs(Fm[0] + F[0]) <= 1e-9 * scale
        assert abs(Fm[1] - F[1]) <= 1e-9 * scale
        assert abs(Fm[4] + F[4]) <= 1e-9 * scale
    # stationary contact: no mass flux, momentum flux equals the pressure
    for rl, rr, p in [(1.0, 0.125, 1.0), (3.0, 0.01, 0.2)]:
        UL = oracle.prim_to_cons((rl, 0.0, 0.3, -0.1, p), gamma)
        UR = oracle.prim_to_cons((rr, 0.0, -0.7, 0.2, p), gamma)
        F, _ = oracle.riemann_flux(UL, UR, gamma)
        assert F[0] == 0.0 and F[1] == p and F[4] == 0.0


def test_pressure_floor_applied(oracle):
    """A conserved state with negative internal energy is converted with p = p_floor."""
    U = np.array([1.0, 2.0, 0.0, 0.0, 1.0])  # kinetic energy 2 > E
    W = oracle.cons_to_prim(U, 1.4, 1e-20)
    assert W[4] == 1e-20
    F, st = oracle.riemann_flux(U, U, 1.4)
    assert st.p_floored == 2 and np.all(np.isfinite(F))
