"""Pins of the oracle's PPMP reconstruction (App. A.4) and of the CTU step with it.

What fixes the answer, independently of the oracle's own formulas:
* a uniform state traces to itself;
* on a linear profile no limiter, steepening or flattening acts and the parabola is the
  line (w6 = 0), so the characteristic tracing of CW84 must reproduce the linearized
  characteristic solution at the half step: each approaching wave carries its Riemann
  invariant (p -/+ rho a u, rho - p/a^2, v, w) from x_face - lambda dt/2, a wave moving away
  keeps the reference state's value; the error is second order in the amplitude (a sign
  slip in any correction leaves a first-order error);
* waves moving away from a face leave its state at the interpolated value;
* a shock confined to a cell pair is flattened to first order (states = cell averages),
  an expansion is not;
* a smeared contact is steepened toward its neighbours, a sound wave is not;
* mirror symmetry; whole-step invariants (uniform flow, conservation, Sod accuracy).
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_1410_4194_amd import workloads as WL
from tests.common import oracle_config, oracle_state, run_oracle

G = 1.4


def _linear_stencil(base, grad, eps):
    return np.array([base + eps * grad * (s - 3) for s in range(7)])


def _char_exact(base, grad, eps, dtodx, face):
    """Linearized characteristic solution at the half step at the face x = face/2 (cell
    centre at 0, unit width) for the linear profile base + eps*grad*x; the waves that do not
    approach the face take the value of the fastest approaching wave's foot point (the
    reference state)."""
    rho0, u0, v0, w0, p0 = base
    a0 = math.sqrt(G * p0 / rho0)
    C = rho0 * a0
    lam = np.array([u0 - a0, u0, u0 + a0])
    xf = 0.5 * face
    def val(x):
        return base + eps * grad * x
    if face > 0:  # right face: waves with lambda > 0 approach; reference is lambda+
        ref = xf - 0.5 * dtodx * max(lam[2], 0.0)
        foot = [xf - 0.5 * dtodx * l if l > 0 else ref for l in lam]
    else:
        ref = xf - 0.5 * dtodx * min(lam[0], 0.0)
        foot = [xf - 0.5 * dtodx * l if l < 0 else ref for l in lam]
    wm, wz, wp = val(foot[0]), val(foot[1]), val(foot[2])
    # the transverse velocities follow the advection wave's own foot point (the face itself
    # when that wave moves away)
    adv = xf - 0.5 * dtodx * (max(lam[1], 0.0) if face > 0 else min(lam[1], 0.0))
    wt = val(adv)
    Jm = wm[4] - C * wm[1]          # carried by u - a
    S0 = wz[0] - wz[4] / a0 ** 2    # carried by u
    Jp = wp[4] + C * wp[1]          # carried by u + a
    p = 0.5 * (Jp + Jm)
    u = 0.5 * (Jp - Jm) / C
    rho = S0 + p / a0 ** 2
    return np.array([rho, u, wt[2], wt[3], p])


def test_uniform_state_traces_to_itself():
    w = np.tile([1.3, 0.4, -0.2, 0.7, 2.0], (7, 1))
    L, R, _, _ = O.ppmp(w, 0.3, 0.1, G)
    assert np.allclose(L, w[3], rtol=2e-16, atol=0) and np.allclose(R, w[3], rtol=2e-16, atol=0)


@pytest.mark.parametrize("u0", [1.8, 0.4, -0.5, -2.1])
def test_linear_waves_traced_to_second_order(u0):
    """Supersonic right/left and subsonic both ways: the traced states converge to the
    linearized characteristic solution with error O(eps^2)."""
    base = np.array([1.0, u0, 0.3, -0.2, 1.0])
    grad = np.array([0.7, -0.5, 0.4, 0.9, 0.6])
    dtodx = 0.3
    errs = {1: [], -1: []}
    for eps in (1e-2, 5e-3, 2.5e-3):
        w = _linear_stencil(base, grad, eps)
        L, R, WLm, WRm = O.ppmp(w, dtodx, 0.1, G)
        # the interpolated faces of a line are exact
        assert np.allclose(WLm, base - 0.5 * eps * grad, rtol=0, atol=1e-14)
        assert np.allclose(WRm, base + 0.5 * eps * grad, rtol=0, atol=1e-14)
        errs[1].append(np.max(np.abs(R - _char_exact(base, grad, eps, dtodx, 1))) / eps)
        errs[-1].append(np.max(np.abs(L - _char_exact(base, grad, eps, dtodx, -1))) / eps)
    for face in (1, -1):
        e = errs[face]
        if e[0] < 1e-12:  # exact up to rounding (no wave reaches this face)
            continue
        assert e[0] < 0.05 and e[0] / e[1] > 1.8 and e[1] / e[2] > 1.8, (face, e)


def test_waves_moving_away_leave_the_face_unchanged():
    """Flow supersonic to the right: no wave reaches the left face, whose traced state is
    the interpolated (monotonized) value."""
    rng = np.random.default_rng(3)
    w = np.array([[1.0 + 0.1 * rng.standard_normal(), 3.0 + 0.1 * rng.standard_normal(),
                   rng.standard_normal(), rng.standard_normal(), 1.0 + 0.1 * rng.standard_normal()]
                  for _ in range(7)])
    L, R, WLm, WRm = O.ppmp(w, 0.2, 0.1, G)
    assert np.allclose(L, WLm, rtol=4e-16, atol=0)


def test_sharp_shock_is_flattened_to_first_order():
    """Pressure jumps by 10x between cells 3 and 4 of the stencil (compression): the cells
    next to the jump are flattened completely and trace to their own averages."""
    w = np.array([[1.0, 1.0, 0.0, 0.0, 10.0]] * 4 + [[0.3, 0.0, 0.0, 0.0, 1.0]] * 3)
    # shift so the jump sits between the centre cell and its right neighbour
    F, eta = O.ppmp_coefficients(w, G, 0.1)
    assert F == 1.0
    L, R, _, _ = O.ppmp(w, 0.0, 0.1, G)
    assert np.allclose(L, w[3], rtol=2e-16, atol=0) and np.allclose(R, w[3], rtol=2e-16, atol=0)


@pytest.mark.parametrize("p2,expect", [(10.0, 0.0), (10.5, 1.0)])
def test_flattening_takes_the_neighbour_by_pressure_gradient(p2, expect):
    """Hand-evaluated stencils, shock between the right neighbour and the cell after it
    (p = 10 | 1, compression).  The centre cell's own coefficient is 0 (small jump across
    it); the right neighbour's is 1.  With p_{i+1} - p_{i-1} = 0 the rule takes the left
    neighbour (F = 0); with p_{i+1} - p_{i-1} = -0.5 < 0 it takes the right one (F = 1)."""
    p = np.array([10.0, 10.0, p2, 10.0, 10.0, 1.0, 1.0])
    u = np.array([1.0, 1.0, 1.0, 1.0, 1.0, 0.0, 0.0])
    w = np.stack([np.ones(7), u, np.zeros(7), np.zeros(7), p], axis=1)
    F, eta = O.ppmp_coefficients(w, G, 0.1)
    assert F == expect


def test_expansion_is_not_flattened():
    w = np.array([[1.0, -1.0, 0.0, 0.0, 10.0]] * 4 + [[0.3, 1.0, 0.0, 0.0, 1.0]] * 3)
    F, eta = O.ppmp_coefficients(w, G, 0.1)
    assert F == 0.0


def test_weak_pressure_jump_is_not_flattened():
    w = np.array([[1.0, 0.2, 0.0, 0.0, 1.2]] * 4 + [[1.0, 0.0, 0.0, 0.0, 1.0]] * 3)
    F, eta = O.ppmp_coefficients(w, G, 0.1)
    assert F == 0.0


def test_smeared_contact_is_steepened():
    """A density step spread over a few cells at uniform pressure and velocity: the centre
    cell (an inflection of the profile) is steepened, and its face densities move toward the
    neighbouring plateaus."""
    rho = np.array([1.0, 1.0, 1.15, 2.0, 2.85, 3.0, 3.0])
    w = np.stack([rho, np.full(7, 0.1), np.zeros(7), np.zeros(7), np.ones(7)], axis=1)
    F, eta = O.ppmp_coefficients(w, G, 0.1)
    assert F == 0.0 and eta > 0.5
    L, R, WLm, WRm = O.ppmp(w, 0.0, 0.1, G)
    # reference: the same stencil with the jump too small to steepen gives the plain values
    assert WRm[0] > 0.5 * (rho[3] + rho[4]) and WLm[0] < 0.5 * (rho[2] + rho[3])


def test_sound_wave_is_not_steepened():
    """Density and pressure jump together (p ~ rho^gamma): condition on the pressure jump."""
    rho = np.array([1.0, 1.0, 1.15, 2.0, 2.85, 3.0, 3.0])
    w = np.stack([rho, np.zeros(7), np.zeros(7), np.zeros(7), rho ** G], axis=1)
    F, eta = O.ppmp_coefficients(w, G, 0.1)
    assert eta == 0.0


@pytest.mark.parametrize("seed", range(6))
def test_mirror_symmetry(seed):
    rng = np.random.default_rng(50 + seed)
    w = np.stack([10 ** rng.uniform(-0.5, 0.5, 7), rng.uniform(-1, 1, 7), rng.uniform(-1, 1, 7),
                  rng.uniform(-1, 1, 7), 10 ** rng.uniform(-0.5, 0.5, 7)], axis=1)
    m = w[::-1].copy()
    m[:, 1] *= -1.0
    L, R, _, _ = O.ppmp(w, 0.25, 0.1, G)
    Lm, Rm, _, _ = O.ppmp(m, 0.25, 0.1, G)
    flip = np.array([1.0, -1.0, 1.0, 1.0, 1.0])
    assert np.allclose(Lm, flip * R, rtol=1e-13, atol=1e-14)
    assert np.allclose(Rm, flip * L, rtol=1e-13, atol=1e-14)


# --- whole CTU step with PPMP ---------------------------------------------------------------

def _cfg(wl, **kw):
    return oracle_config(wl, recon=O.RECON_PPMP, **kw)


def test_ppmp_uses_four_ghost_layers():
    wl = WL.random_state(5, 4, 6, seed=1)
    assert _cfg(wl).ng == 4 and oracle_config(wl).ng == 3


def test_ppmp_step_keeps_uniform_flow():
    wl = WL.random_state(9, 7, 6, seed=3)
    wl.W[:] = np.array([1.3, 0.4, -0.2, 0.7, 2.0])[:, None, None, None]
    cfg = _cfg(wl)
    u = oracle_state(wl, cfg)
    before = O.real(cfg, u).copy()
    O.step(cfg, u, 0.5 * O.compute_dt(cfg, u))
    assert np.array_equal(O.real(cfg, u), before)


@pytest.mark.parametrize("riemann", [0, 1], ids=["exact", "roe"])
def test_ppmp_step_conserves_on_periodic_grid(riemann):
    wl = WL.random_state(11, 9, 8, seed=4)
    cfg = _cfg(wl, riemann=riemann)
    u = oracle_state(wl, cfg)
    r0 = O.real(cfg, u).reshape(5, -1).copy()
    for _ in range(3):
        O.step(cfg, u, O.compute_dt(cfg, u))
    r1 = O.real(cfg, u).reshape(5, -1)
    for f in range(5):
        assert abs(math.fsum(r1[f]) - math.fsum(r0[f])) <= 1e-13 * math.fsum(np.abs(r0[f]))


def test_ppmp_one_dimensional_columns_identical():
    wl = WL.sod(32, 3, 4)
    cfg = _cfg(wl)
    u = oracle_state(wl, cfg)
    for _ in range(3):
        O.step(cfg, u, O.compute_dt(cfg, u))
    r = O.real(cfg, u)
    for f in range(5):
        cols = r[f].reshape(-1, 32)
        assert np.all(cols == cols[0])


def test_ppmp_sod_accuracy_and_sharper_contact():
    """Sod to t = 0.2 at 128 cells: close to the exact solution, and the contact region is
    resolved at least as well as with PPMC (the behaviour the paper reports for PPMP)."""
    x = (np.arange(128) + 0.5) / 128
    ex = O.exact_solution((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), 1.4, (x - 0.5) / 0.2)
    res = {}
    for name, recon in (("ppmp", O.RECON_PPMP), ("ppmc", O.RECON_PPMC)):
        wl = WL.sod(128, 1, 1)
        cfg = oracle_config(wl, recon=recon)
        cfg, u, t, n = run_oracle(wl, t_end=0.2, cfg=cfg)
        r = O.real(cfg, u)[0, 0, 0]
        contact = (x > 0.6) & (x < 0.78)
        res[name] = (np.mean(np.abs(r - ex[0])), np.mean(np.abs(r[contact] - ex[0][contact])))
    assert res["ppmp"][0] < 0.003, res
    assert res["ppmp"][1] <= res["ppmc"][1], res


def test_ppmp_reflect_equals_mirrored_periodic_box():
    """The mirror-box identity with four ghost layers (bit for bit)."""
    n = [8, 5, 4]
    bc = (2, 2, 0, 0, 0, 0)
    wl = WL.random_state(*n, seed=12, bc=bc)
    cfg = _cfg(wl)
    u = oracle_state(wl, cfg)
    dt = 0.5 * O.compute_dt(cfg, u)
    O.step(cfg, u, dt)
    M = np.flip(wl.W, axis=3).copy()
    M[1] *= -1.0
    W2 = np.concatenate([wl.W, M], axis=3)
    cfg2 = O.Config(16, 5, 4, wl.dx, wl.dy, wl.dz, wl.gamma, bc=(0,) * 6, cfl=wl.cfl,
                    recon=O.RECON_PPMP)
    u2 = O.state_from_primitive(cfg2, W2)
    O.step(cfg2, u2, dt)
    assert np.array_equal(O.real(cfg, u), O.real(cfg2, u2)[..., :8])


def test_ppmp_blast_waves_stay_physical():
    wl = WL.blast_waves(100)
    cfg = _cfg(wl)
    u0 = O.real(cfg, oracle_state(wl, cfg)).copy()
    cfg, u, t, n = run_oracle(wl, t_end=wl.t_end, cfg=cfg)
    r = O.real(cfg, u)
    assert np.all(r[0] > 0)
    assert abs(r[0].sum() - u0[0].sum()) <= 1e-12 * u0[0].sum()
