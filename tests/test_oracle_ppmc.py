"""Pins of the oracle's PPMC reconstruction (App. A.3, with the PLMC slope step of App. A.2).

The characteristic projections are checked against an eigen-decomposition computed by numpy
from the primitive-form Euler Jacobian (Sec. 2: dw/dt + A(w) dw/dx = 0); the parabola and the
tracing integrals against Gauss-Legendre quadrature of the CW84 parabola; the corrections
against the general rule "each wave family moving toward a face is traced with its own speed,
the others keep the reference (fastest-wave) trace"; plus mirror symmetry, exactness on
uniform and linear data, and the monotonicity the limiter steps exist to guarantee.
"""
import math

import numpy as np
import pytest

SEED = 14104194
GL_X, GL_W = np.polynomial.legendre.leggauss(3)  # exact for the quadratic parabola


def jacobian(w, gamma):
    """A(w) of the 1D primitive Euler system with two passively advected velocities."""
    rho, u, _, _, p = w
    A = np.zeros((5, 5))
    A[0, 0], A[0, 1] = u, rho
    A[1, 1], A[1, 4] = u, 1.0 / rho
    A[2, 2] = u
    A[3, 3] = u
    A[4, 1], A[4, 4] = gamma * p, u
    return A


def eig_projectors(w, gamma):
    """(eigenvalues, list of (lambda, P)) where P projects onto each eigenspace of A."""
    A = jacobian(w, gamma)
    lam, R = np.linalg.eig(A)
    lam = lam.real
    R = R.real
    L = np.linalg.inv(R)
    groups = {}
    for k in range(5):
        key = round(lam[k], 9)
        groups.setdefault(key, []).append(k)
    out = []
    for key, ks in groups.items():
        P = sum(np.outer(R[:, k], L[k, :]) for k in ks)
        out.append((lam[ks[0]], P))
    return out


def parabola_avg(WL, WR, wc, s0, s1):
    """Average over [s0, s1] (cell-unit coordinate, 0 = left face) of the CW84 parabola
    a(x) = W_L + x (dW + w6 (1 - x)), dW = W_R - W_L, w6 = 6 w - 3 (W_L + W_R)."""
    WL, WR, wc = map(np.asarray, (WL, WR, wc))
    if s1 - s0 == 0.0:
        x = np.array([s0])
        return WL + x[0] * ((WR - WL) + (6 * wc - 3 * (WL + WR)) * (1 - x[0]))
    xs = 0.5 * (s1 - s0) * GL_X + 0.5 * (s1 + s0)
    tot = 0.0
    for x, wt in zip(xs, GL_W):
        tot = tot + 0.5 * wt * (WL + x * ((WR - WL) + (6 * wc - 3 * (WL + WR)) * (1 - x)))
    return tot


def random_w(rng, gamma, n=5, smooth=False):
    base = np.array([10 ** rng.uniform(-1, 1), rng.uniform(-2, 2), rng.uniform(-1, 1),
                     rng.uniform(-1, 1), 10 ** rng.uniform(-1, 1)])
    w = np.empty((n, 5))
    for k in range(n):
        pert = rng.normal(size=5) * (0.02 if smooth else 0.3)
        w[k] = base * (1 + pert * np.array([1, 0, 0, 0, 1])) + pert * np.array([0, 1, 1, 1, 0])
    w[:, 0] = np.abs(w[:, 0]) + 1e-3
    w[:, 4] = np.abs(w[:, 4]) + 1e-3
    return w


def test_projection_round_trip(oracle):
    rng = np.random.default_rng(SEED)
    for _ in range(200):
        d = rng.normal(size=5) * 10 ** rng.uniform(-3, 3)
        rho, a = 10 ** rng.uniform(-2, 2), 10 ** rng.uniform(-2, 2)
        back = oracle.char_unproject(oracle.char_project(d, rho, a), rho, a)
        # rounding scale of each component: the round trip mixes dp/a^2 with rho du/a
        mix = abs(d[4]) / a ** 2 + rho * abs(d[1]) / a
        scale = np.abs(d) + np.array([mix, mix * a / rho, 0.0, 0.0, mix * a * a])
        assert np.all(np.abs(back - d) <= 1e-14 * scale)


@pytest.mark.parametrize("gamma", [1.4, 5.0 / 3.0])
def test_projection_matches_eigenvectors(oracle, gamma):
    """unproject(e_k) spans the eigenspaces of A and project is its inverse, with the
    component order (u-a, u [entropy], u [v], u [w], u+a)."""
    rng = np.random.default_rng(SEED + 1)
    for _ in range(50):
        w = random_w(rng, gamma, 1)[0]
        rho, u, p = w[0], w[1], w[4]
        a = math.sqrt(gamma * p / rho)
        A = jacobian(w, gamma)
        lam = [u - a, u, u, u, u + a]
        for k in range(5):
            e = np.zeros(5)
            e[k] = 1.0
            r = oracle.char_unproject(e, rho, a)
            assert np.allclose(A @ r, lam[k] * r, rtol=1e-12, atol=1e-12 * (abs(u) + a) * np.abs(r).max())
        # project diagonalizes A
        d = rng.normal(size=5)
        assert np.allclose(oracle.char_project(A @ d, rho, a),
                           np.array(lam) * oracle.char_project(d, rho, a),
                           rtol=1e-11, atol=1e-11 * (abs(u) + a) * np.abs(d).max() * (rho + 1 / a ** 2 + rho / a))


def test_uniform_state_is_exact(oracle):
    rng = np.random.default_rng(SEED + 2)
    for _ in range(50):
        w0 = random_w(rng, 1.4, 1)[0]
        w = np.tile(w0, (5, 1))
        sl, sr, WL, WR = oracle.ppmc(w, rng.uniform(0, 0.4), 1.4)
        assert np.array_equal(sl, w0) and np.array_equal(sr, w0)


def test_linear_data_gives_exact_face_values(oracle):
    """On linear data the limiter is inactive and, at dt = 0, the traced states are the
    face values of the line."""
    rng = np.random.default_rng(SEED + 3)
    for _ in range(50):
        w0 = random_w(rng, 1.4, 1)[0]
        slope = rng.normal(size=5) * 1e-3 * np.abs(w0).clip(0.1)
        w = np.array([w0 + (k - 2) * slope for k in range(5)])
        sl, sr, WL, WR = oracle.ppmc(w, 0.0, 1.4)
        assert np.allclose(WL, w0 - 0.5 * slope, rtol=1e-13, atol=1e-14)
        assert np.allclose(WR, w0 + 0.5 * slope, rtol=1e-13, atol=1e-14)
        assert np.allclose(sl, WL, rtol=0, atol=1e-15) and np.allclose(sr, WR, rtol=0, atol=1e-15)


@pytest.mark.parametrize("gamma", [1.4, 5.0 / 3.0])
def test_tracing_matches_characteristic_rule(oracle, gamma):
    """General statement of the tracing: for each eigenspace k of A(w_c), its component of
    W*_R is that of the parabola averaged over the last beta_k of the cell when the wave
    moves toward the right face (lambda_k > 0), and of the reference average (fastest wave
    lambda^p) otherwise; mirror image at the left face with alpha_k and lambda^m."""
    rng = np.random.default_rng(SEED + 4)
    n_cases = {"sub+": 0, "sub-": 0, "sup+": 0, "sup-": 0}
    for trial in range(400):
        w = random_w(rng, gamma, 5, smooth=(trial % 2 == 0))
        if trial % 4 == 1:
            w[:, 1] += 4 * math.sqrt(gamma * w[2, 4] / w[2, 0])  # supersonic to the right
        if trial % 4 == 3:
            w[:, 1] -= 4 * math.sqrt(gamma * w[2, 4] / w[2, 0])  # supersonic to the left
        dtodx = rng.uniform(0.0, 0.15)
        sl, sr, WL, WR = oracle.ppmc(w, dtodx, gamma)
        wc = w[2]
        a = math.sqrt(gamma * wc[4] / wc[0])
        lam_m, lam_p = wc[1] - a, wc[1] + a
        ref_L = parabola_avg(WL, WR, wc, 0.0, dtodx * max(-lam_m, 0.0))
        ref_R = parabola_avg(WL, WR, wc, 1.0 - dtodx * max(lam_p, 0.0), 1.0)
        exp_L = np.zeros(5)
        exp_R = np.zeros(5)
        for lam, P in eig_projectors(wc, gamma):
            if lam < 0:
                exp_L += P @ parabola_avg(WL, WR, wc, 0.0, -dtodx * lam)
            else:
                exp_L += P @ ref_L
            if lam > 0:
                exp_R += P @ parabola_avg(WL, WR, wc, 1.0 - dtodx * lam, 1.0)
            else:
                exp_R += P @ ref_R
        scale = np.abs(w).max(axis=0) + 1e-12
        assert np.all(np.abs(sl - exp_L) <= 1e-10 * scale), (trial, sl, exp_L)
        assert np.all(np.abs(sr - exp_R) <= 1e-10 * scale), (trial, sr, exp_R)
        key = ("sup" if abs(wc[1]) > a else "sub") + ("+" if wc[1] > 0 else "-")
        n_cases[key] += 1
    assert min(n_cases.values()) > 20


@pytest.mark.parametrize("gamma", [1.4, 5.0 / 3.0])
def test_mirror_symmetry(oracle, gamma):
    """Reflecting the stencil and the normal velocity swaps the two traced states."""
    rng = np.random.default_rng(SEED + 5)
    flip = np.array([1.0, -1.0, 1.0, 1.0, 1.0])
    for trial in range(200):
        w = random_w(rng, gamma, 5, smooth=(trial % 3 == 0))
        dtodx = rng.uniform(0.0, 0.2)
        sl, sr, _, _ = oracle.ppmc(w, dtodx, gamma)
        wm = (w[::-1] * flip).copy()
        sl2, sr2, _, _ = oracle.ppmc(wm, dtodx, gamma)
        scale = np.abs(w).max(axis=0) + 1e-12
        assert np.all(np.abs(sl2 - sr * flip) <= 1e-12 * scale)
        assert np.all(np.abs(sr2 - sl * flip) <= 1e-12 * scale)


def test_reconstruction_is_monotone(oracle):
    """After the limiter steps the face values lie between neighbouring averages, and the
    parabola has no extremum inside the cell unless the final clamp (which the paper
    applies after the steep-gradient fix) pinned one face value to a neighbour bound."""
    rng = np.random.default_rng(SEED + 6)
    n_monotone = 0
    for _ in range(500):
        w = random_w(rng, 1.4, 5)
        _, _, WL, WR = oracle.ppmc(w, 0.0, 1.4)
        wc, wm, wp = w[2], w[1], w[3]
        loL, hiL = np.minimum(wc, wm), np.maximum(wc, wm)
        loR, hiR = np.minimum(wc, wp), np.maximum(wc, wp)
        assert np.all(WL >= loL) and np.all(WL <= hiL)
        assert np.all(WR >= loR) and np.all(WR <= hiR)
        dW = WR - WL
        w6 = 6 * wc - 3 * (WL + WR)
        # derivative of the parabola is dW + w6 (1 - 2x): same sign at both ends (or zero)
        d0, d1 = dW + w6, dW - w6
        tol = 1e-12 * (np.abs(dW) + np.abs(w6))
        bad = d0 * d1 < -tol * (np.abs(d0) + np.abs(d1))
        on_bound = (WL == loL) | (WL == hiL) | (WR == loR) | (WR == hiR)
        assert np.all(~bad | on_bound)
        n_monotone += int(np.sum(~bad))
    assert n_monotone > 2000


def test_steep_gradient_fix(oracle):
    """Monotone data whose interpolated parabola overshoots: the fix moves one face value so
    the parabola's slope vanishes at the other face (CW84's steepening condition)."""
    rows = []
    for vals in ([0.0, 0.0, 0.1, 1.0, 1.0], [1.0, 1.0, 0.9, 0.0, 0.0], [0.0, 0.0, 0.9, 1.0, 1.0]):
        w = np.tile(np.array([1.0, 0.0, 0.0, 0.0, 1.0]), (5, 1))
        w[:, 2] = vals  # transverse velocity: a passively advected component
        _, _, WL, WR = oracle.ppmc(w, 0.0, 1.4)
        c = vals[2]
        dW, w6 = WR[2] - WL[2], 6 * c - 3 * (WL[2] + WR[2])
        rows.append((dW + w6, dW - w6))
        # one end of the parabola is flat, and it stays monotone
        assert min(abs(dW + w6), abs(dW - w6)) <= 1e-15
        assert (dW + w6) * (dW - w6) >= -1e-15
    assert len(rows) == 3


def test_limiter_zeroes_slope_at_extremum(oracle):
    w = np.array([[1.0, 0.0, 0.0, 0.0, 1.0], [2.0, 0.0, 0.0, 0.0, 1.0], [1.5, 0.0, 0.0, 0.0, 1.0]])
    dw = oracle.plmc_slope(w[0], w[1], w[2], 1.4)
    assert dw[0] == 0.0
    # monotone density-only data: MC slope = min(central, 2 left, 2 right)
    w = np.array([[1.0, 0, 0, 0, 1.0], [1.1, 0, 0, 0, 1.0], [1.5, 0, 0, 0, 1.0]])
    dw = oracle.plmc_slope(w[0], w[1], w[2], 1.4)
    assert dw[0] == pytest.approx(0.2, rel=1e-14)
    w = np.array([[1.0, 0, 0, 0, 1.0], [1.3, 0, 0, 0, 1.0], [1.35, 0, 0, 0, 1.0]])
    dw = oracle.plmc_slope(w[0], w[1], w[2], 1.4)
    assert dw[0] == pytest.approx(0.1, rel=1e-13)
