"""Values the paper prints, kept as text fixtures under tests/golden/ (each with its
citation), against the input generators and the oracle.

* test_problems.txt: the initial states of the test problems of Sec. 4.1-4.2 (with the
  readings of the printed inconsistencies noted in the fixture) against the seeded
  generators that feed both the oracle and the GPU;
* noh_3d.txt: the densities Sec. 4.3.1 prints for Noh's problem (16 immediately ahead of
  the shock, 64 behind it): consistent with the jump conditions, and met by the oracle's
  Roe + H correction run on a 32^3 octant.
"""
import os

import numpy as np
import pytest

import oracle as O
from paper_1410_4194_amd import workloads as WL
from tests.common import oracle_config, run_oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _records(name):
    out = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.split("#", 1)[0].split()
            if line:
                out.append(line)
    return out


def _kv(name):
    return {r[0]: float(r[1]) for r in _records(name)}


TUBES = {r[1]: [float(v) for v in r[2:]] for r in _records("test_problems.txt") if r[0] == "tube"}
OTHER = {r[0]: [float(v) for v in r[1:]] for r in _records("test_problems.txt") if r[0] != "tube"}
MAKERS = {"sod": lambda: WL.sod(64, 2, 2), "strong_shock": lambda: WL.strong_shock_tube(64),
          "strong_rarefaction": lambda: WL.strong_rarefaction(64)}


@pytest.mark.parametrize("name", sorted(MAKERS))
def test_shock_tubes(name):
    rl, ul, pl, rr, ur, pr, x0, gamma, t_end = TUBES[name]
    wl = MAKERS[name]()
    x = (np.arange(wl.nx) + 0.5) * wl.dx
    left, right = x < x0, x > x0
    for f, (a, b) in ((0, (rl, rr)), (1, (ul, ur)), (4, (pl, pr))):
        assert np.all(wl.W[f][..., left] == a) and np.all(wl.W[f][..., right] == b), (name, f)
    assert np.all(wl.W[2] == 0) and np.all(wl.W[3] == 0)
    assert wl.gamma == gamma and wl.t_end == t_end
    assert abs(wl.nx * wl.dx - 1.0) < 1e-15


def test_interacting_blast_waves():
    rho, p_left, p_mid, p_right, xa, xb, gamma, t_end = OTHER["blast"]
    wl = WL.blast_waves(400)
    x = (np.arange(wl.nx) + 0.5) * wl.dx
    p = wl.W[4][0, 0]
    assert np.all(p[x < xa] == p_left) and np.all(p[x > xb] == p_right)
    assert np.all(p[(x > xa) & (x < xb)] == p_mid)
    assert np.all(wl.W[0] == rho) and np.all(wl.W[1:4] == 0)
    assert wl.bc[:2] == (WL.REFLECT, WL.REFLECT)
    assert wl.gamma == gamma and wl.t_end == t_end


def test_implosion():
    side, diag, r_in, p_in, r_out, p_out, gamma, t_end = OTHER["implosion"]
    wl = WL.implosion(60, nz=2)
    assert abs(wl.nx * wl.dx - side) < 1e-15 and abs(wl.ny * wl.dy - side) < 1e-15
    xc = (np.arange(wl.nx) + 0.5) * wl.dx
    inside = (xc[None, :] + xc[:, None]) < diag
    for k in range(wl.nz):
        assert np.all(wl.W[0, k][inside] == r_in) and np.all(wl.W[4, k][inside] == p_in)
        assert np.all(wl.W[0, k][~inside] == r_out) and np.all(wl.W[4, k][~inside] == p_out)
    assert np.all(wl.W[1:4] == 0)
    assert wl.bc[:4] == (WL.REFLECT,) * 4
    assert wl.gamma == gamma and wl.t_end == t_end


def test_kelvin_helmholtz():
    r_band, u_band, r_out, u_out, p, gamma, amp = OTHER["kh"]
    wl = WL.kelvin_helmholtz(12, 12, 4)
    y = (np.arange(wl.ny) + 0.5) * wl.dy
    x = (np.arange(wl.nx) + 0.5) * wl.dx
    band = (y > 1 / 3) & (y < 2 / 3)
    assert np.all(wl.W[0][:, band] == r_band) and np.all(wl.W[1][:, band] == u_band)
    assert np.all(wl.W[0][:, ~band] == r_out) and np.all(wl.W[1][:, ~band] == u_out)
    assert np.all(wl.W[4] == p) and wl.gamma == gamma
    assert np.allclose(wl.W[2], amp * np.sin(2 * np.pi * x)[None, None, :], rtol=0, atol=1e-17)


def test_noh_printed_densities_follow_the_jump_conditions():
    g = _kv("noh_3d.txt")
    gamma, n = g["gamma"], int(g["dimensions"])
    # ahead of the shock, at the shock radius t/3: rho0 (1 + 3)^(n-1)
    assert g["pre_shock_density"] == g["rho0"] * 4.0 ** (n - 1)
    # a strong shock compresses by (gamma + 1)/(gamma - 1)
    assert abs(g["post_shock_density"] - g["pre_shock_density"] * (gamma + 1) / (gamma - 1)) < 1e-12


def test_oracle_noh_meets_the_printed_densities():
    """Roe + H correction, 32^3 octant to t = 0.6 (about 73 steps, a few seconds): the
    pre-shock gas follows rho0 (1 + t/r)^2 to 1%, and the shocked shell between the
    wall-heated core and the shock reaches the printed 64 to 15%."""
    g = _kv("noh_3d.txt")
    n = 32
    wl = WL.noh(n)
    assert wl.gamma == g["gamma"] and np.all(wl.W[0] == g["rho0"])
    cfg, u, t, steps = run_oracle(wl, t_end=wl.t_end, cfg=oracle_config(wl, riemann=1, h_correction=1))
    rho = O.real(cfg, u)[0]
    xc = (np.arange(n) + 0.5) / n
    z, y, x = np.meshgrid(xc, xc, xc, indexing="ij")
    r = np.sqrt(x * x + y * y + z * z)
    pre = (r > 0.28) & (r < 0.38)
    assert np.abs(rho[pre] / (g["rho0"] * (1 + t / r[pre]) ** 2) - 1).mean() < 0.01
    post = (r > 0.08) & (r < 0.17)
    assert abs(rho[post].mean() / g["post_shock_density"] - 1) < 0.15
