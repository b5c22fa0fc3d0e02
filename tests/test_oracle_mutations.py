"""Mutation sweep: plants plausible mistakes in the oracle (on the CPU) and checks that the
pin tests catch every one.  Each mutation is a garbled equation of the paper taken
literally, a sign or index slip, or a dropped term.  Opt-in (about five minutes): run with
CTU_MUTATIONS=1.
"""
import os
import subprocess
import sys
import tempfile

import pytest

REPO = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(REPO, "oracle", "ctu_oracle.c")

M=[
 ("xi0 printed sign", "xi[0] = 0.5 * (d[4] / a2 - rho * d[1] / a);", "xi[0] = -0.5 * (d[4] / a2 + rho * d[1] / a);"),
 ("B printed alpha^p", "B[q] = ILm - ppm_IL(ap, dw[q], w6[q]);", "B[q] = 0.5 * am * (dw[q] + w6[q] * (1.0 + (2.0 / 3.0) * ap)) - ppm_IL(ap, dw[q], w6[q]);"),
 ("D printed", "D[q] = IRp - ppm_IR(b0, dw[q], w6[q]);", "D[q] = IRp - 0.5 * b0 * (dw[q] + w6[q] * (1.0 + (2.0 / 3.0) * b0));"),
 ("w6 printed", "w6[q] = 6.0 * c - 3.0 * (wl + wr);", "w6[q] = 6.0 * c - 3.0 * (wl - wr);"),
 ("right fan +", "double c = 2.0 / (gamma + 1.0) * (ar - 0.5 * (gamma - 1.0) * (ur - S));", "double c = 2.0 / (gamma + 1.0) * (ar + 0.5 * (gamma - 1.0) * (ur - S));"),
 ("transverse sign", "Uh[side][f] = ustar + h1 * (Fs[t1][f][x1] - Fs[t1][f][xc]) +", "Uh[side][f] = ustar - h1 * (Fs[t1][f][x1] - Fs[t1][f][xc]) +"),
 ("transverse t2 drop", "h2 * (Fs[t2][f][x2] - Fs[t2][f][xc]);", "0.0 * (Fs[t2][f][x2] - Fs[t2][f][xc]);"),
 ("update sign y", "v = v + dtd[1] * (Fh[1][f][hm[1]] - Fh[1][f][hp[1]]);", "v = v - dtd[1] * (Fh[1][f][hm[1]] - Fh[1][f][hp[1]]);"),
 ("transverse vel side", "double vt = (u >= 0.0) ? WL[2] : WR[2];", "double vt = (u >= 0.0) ? WR[2] : WL[2];"),
 ("minmod not MC", "if (2.0 * fabs(dl) < m) m = 2.0 * fabs(dl);", "if (fabs(dl) < m) m = fabs(dl);"),
 ("Q30 swap", "ul[q] = Us[d][1][rot[d][q]][xc];\n              ur[q] = Us[d][0][rot[d][q]][xn];", "ul[q] = Us[d][0][rot[d][q]][xc];\n              ur[q] = Us[d][1][rot[d][q]][xn];"),
 ("IR sign", "return 0.5 * beta * (dw - w6 * (1.0 - (2.0 / 3.0) * beta));", "return 0.5 * beta * (dw - w6 * (1.0 + (2.0 / 3.0) * beta));"),
 ("IL half", "return 0.5 * alpha * (dw + w6 * (1.0 + (2.0 / 3.0) * alpha));", "return alpha * (dw + w6 * (1.0 + (2.0 / 3.0) * alpha));"),
 ("shock density", "out[0] = rl * (pstar / pl + gm) / (pstar / pl * gm + 1.0);", "out[0] = rl * (pstar / pl + gm) / (pstar / pl + gm * 1.0);"),
 ("rare density exp", "out[0] = rl * pow(pstar / pl, 1.0 / gamma);", "out[0] = rl * pow(pstar / pl, gamma);"),
 ("ustar sign", "*ustar = 0.5 * (ul + ur + fr - fl);", "*ustar = 0.5 * (ul + ur + fl - fr);"),
 ("energy flux no transverse KE", "double E = p / (gamma - 1.0) + 0.5 * rho * (u * u + vt * vt + wt * wt);", "double E = p / (gamma - 1.0) + 0.5 * rho * (u * u);"),
 ("contact corr sign", "WsL[0] += E[0] - E[4] / a2;", "WsL[0] += E[0] + E[4] / a2;"),
 ("acoustic corr u", "WsR[1] += 0.5 * (C[1] - C[4] / (a * rho));", "WsR[1] += 0.5 * (C[1] + C[4] / (a * rho));"),
 ("lambda0 cond", "if (l0 > 0.0) {\n    WsR[0] += D[0]", "if (l0 < 0.0) {\n    WsR[0] += D[0]"),
 ("parabola WR", "double wr = 0.5 * (wp[q] + wc[q]) - (dwp[q] - dwc[q]) / 6.0;", "double wr = 0.5 * (wp[q] + wc[q]) + (dwp[q] - dwc[q]) / 6.0;"),
 ("steep fix", "if ((wr - wl) * (wl - (3.0 * c - 2.0 * wr)) < 0.0) wl = 3.0 * c - 2.0 * wr;", "if ((wr - wl) * (wl - (3.0 * c - 2.0 * wr)) < 0.0) wl = 2.0 * c - wr;"),
 ("clamp dropped", "wl = fmin(hi, fmax(lo, wl));", "wl = wl;"),
 ("dt direction", "double ty = c->dy / (fabs(W[2]) + a);", "double ty = c->dx / (fabs(W[2]) + a);"),
 ("outflow mirror", "src = (q < 0) ? 0 : n[axis] - 1;", "src = (q < 0) ? -q - 1 : 2 * n[axis] - q - 1;"),
 ("fprime rare exponent", "*df = 1.0 / (rho_k * a_k) * pow(p / p_k, -(gamma + 1.0) / (2.0 * gamma));", "*df = 1.0 / (rho_k * a_k) * pow(p / p_k, (gamma + 1.0) / (2.0 * gamma));"),
 ("fan u", "out[1] = c + S;", "out[1] = c;"),
 ("half dt transverse", "double h1 = 0.5 * dt / dd[t1];", "double h1 = dt / dd[t1];"),
 ("reflect mirror off by one", "src = (q < 0) ? -1 - q : 2 * n[axis] - 1 - q;", "src = (q < 0) ? -q : 2 * n[axis] - 2 - q;"),
 ("reflect no flip", "flip = -1.0;", "flip = 1.0;"),
 ("reflect flips wrong component", "u[f][dst_i] = (f == 1 + axis) ? flip", "u[f][dst_i] = (f == 1 + (axis + 1) % 3) ? flip"),
 ("roe s3 printed", "s[3] = C[0] * wt + C[2] + C[3] * wt + C[4] * wt;", "s[3] = C[0] * wt + C[2] + C[3] * 2.0 + C[4] * wt;"),
 ("roe xi4 sign", "xi[4] = dU[0] * Na * (0.5 * gp * V2 - ut * at)", "xi[4] = dU[0] * Na * (0.5 * gp * V2 + ut * at)"),
 ("roe dissipation sign", "F[q] = 0.5 * (FL[q] + FR[q] - s[q]);", "F[q] = 0.5 * (FL[q] + FR[q] + s[q]);"),
 ("roe never falls back", "if (!failed) {\n    for (int q = 0; q < 5; ++q) F[q] = 0.5", "if (1) {\n    for (int q = 0; q < 5; ++q) F[q] = 0.5"),
 ("hlle bm without roe speed", "double bm = fmin(fmin(lm, WL[1] - aL), 0.0);", "double bm = fmin(WL[1] - aL, 0.0);"),
 ("roe plain mean velocity", "double ut = (sl * WL[1] + sr * WR[1]) / (sl + sr);", "double ut = 0.5 * (WL[1] + WR[1]);"),
 ("eta ignored", "double am = fmax(fabs(lm), eta_h), a0 = fmax(fabs(l0), eta_h)", "double am = fabs(lm), a0 = fmax(fabs(l0), eta_h)"),
 ("ppmp printed concavity", "if (!(d2m * d2p < 0.0)) return 0.0;", "if (!(d2m * d2p > 0.0)) return 0.0;"),
 ("ppmp printed rho_R steepening", "WR[0] = WR[0] * (1.0 - eta) + (wp[0] - 0.5 * dwp[0]) * eta;", "WR[0] = WR[0] * (1.0 - eta) + (wm[0] - 0.5 * dwp[0]) * eta;"),
 ("ppmp printed chi^p_L", "((mL[1] - pL[1]) + (mL[4] - pL[4]) / CL)", "((mL[1] - pL[1]) - (mL[4] + pL[4]) / CL)"),
 ("ppmp printed monotonicity 3", "< 0.0) WR[q] = 3.0 * c - 2.0 * WL[q];", "< 0.0) WL[q] = 3.0 * c - 2.0 * WL[q];"),
 ("ppmp chi0 zeroing sign", "if (lam[1] > 0.0) chi0L = 0.0;", "if (lam[1] < 0.0) chi0L = 0.0;"),
 ("ppmp flattening branch swap", "return (p[4] - p[2] < 0.0) ? fmax(F0, Fp) : fmax(F0, Fm);", "return (p[4] - p[2] < 0.0) ? fmax(F0, Fm) : fmax(F0, Fp);"),
 ("ppmp transverse from reference", "WsL[2] = oL[2];", "WsL[2] = mL[2];"),
 ("ppmp no expansion test", "if (u[3] - u[1] > 0.0) return 0.0;", "if (0) return 0.0;"),
 ("ppmp chi^m_R sign", "WsR[1] = pR[1] - CR * chimR;", "WsR[1] = pR[1] + CR * chimR;"),
 ("hcorr own face only", "eta_h = fmax(eta_h, eta[t][box_index(&E[t], m[0], m[1], m[2])]);\n                  eta_h = fmax(eta_h, eta[t][box_index(&E[t], cc[0], cc[1], cc[2])]);", "(void)m;"),
 ("hcorr eta without half", "eta[d][box_index(&E[d], i, j, k)] = 0.5 * fabs(sR - sL);", "eta[d][box_index(&E[d], i, j, k)] = fabs(sR - sL);"),
 ("hcorr eta from first-stage states", "ctu_face_states(c, d, cl, dt, &X, Us, Fs, Uh);\n            for (int side = 0; side < 2; ++side) ref_cons_to_prim(Uh[side], g, c->p_floor, w[side]);", "ctu_face_states(c, d, cl, 0.0, &X, Us, Fs, Uh);\n            for (int side = 0; side < 2; ++side) ref_cons_to_prim(Uh[side], g, c->p_floor, w[side]);"),
 ("clamp before the steep-gradient fix", "    if ((wr - wl) * (wl - (3.0 * c - 2.0 * wr)) < 0.0) wl = 3.0 * c - 2.0 * wr;\n    if ((wr - wl) * ((3.0 * c - 2.0 * wl) - wr) < 0.0) wr = 3.0 * c - 2.0 * wl;\n    /* Step 5: bound the face values by the neighbouring cell averages. */\n    double lo = fmin(c, wm[q]), hi = fmax(c, wm[q]);\n    wl = fmin(hi, fmax(lo, wl));\n    lo = fmin(c, wp[q]);\n    hi = fmax(c, wp[q]);\n    wr = fmin(hi, fmax(lo, wr));", "    double lo = fmin(c, wm[q]), hi = fmax(c, wm[q]);\n    wl = fmin(hi, fmax(lo, wl));\n    lo = fmin(c, wp[q]);\n    hi = fmax(c, wp[q]);\n    wr = fmin(hi, fmax(lo, wr));\n    if ((wr - wl) * (wl - (3.0 * c - 2.0 * wr)) < 0.0) wl = 3.0 * c - 2.0 * wr;\n    if ((wr - wl) * ((3.0 * c - 2.0 * wl) - wr) < 0.0) wr = 3.0 * c - 2.0 * wl;"),
 ("own rho for slopes", "  double rho = w0[0];\n  double a = sound_speed(w0, gamma);", "  double rho = wm[0];\n  double a = sound_speed(wm, gamma);"),
]

PINS = ["tests/test_oracle_riemann.py", "tests/test_oracle_roe.py", "tests/test_oracle_ppmc.py",
        "tests/test_oracle_ppmp.py", "tests/test_oracle_hcorr.py", "tests/test_oracle_step.py"]


# Readings that no printed value or closed form fixes: a mutation to the other reading is
# expected to survive every pin (strict, so that a pin that starts catching it is noticed).
# App. C takes eta from "the left and right input states" and corrects the second-stage
# fluxes only; the oracle reads these as the second-stage (transverse-corrected) states, the
# one reading that needs the extra ghost layer the paper adds.  Where the first- and
# second-stage states differ, nothing printed gives a value to compare with: parity of the
# stage choice is unpinned.
UNPINNED_READINGS = {"hcorr eta from first-stage states"}


def _params():
    out = []
    for m in M:
        marks = ()
        if m[0] in UNPINNED_READINGS:
            marks = pytest.mark.xfail(strict=True, reason="a reading no printed value fixes")
        out.append(pytest.param(*m, id=m[0], marks=marks))
    return out


def test_every_mutation_finds_its_text():
    """The sweep is opt-in, so an edit of the oracle could leave a mutation without its
    target; this runs in the default suite and names any such mutation."""
    src = open(SRC).read()
    missing = [m[0] for m in M if src.count(m[1]) < 1]
    assert not missing, missing


@pytest.mark.slow
@pytest.mark.skipif(not os.environ.get("CTU_MUTATIONS"), reason="opt-in: set CTU_MUTATIONS=1")
@pytest.mark.parametrize("name,old,new", _params())
def test_pins_catch_mutation(name, old, new, tmp_path):
    src = open(SRC).read()
    assert src.count(old) >= 1, name
    c = tmp_path / "mutant.c"
    c.write_text(src.replace(old, new, 1))
    so = tmp_path / "mutant.so"
    subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared",
                    "-I" + os.path.join(REPO, "oracle"), str(c), "-o", str(so), "-lm"], check=True)
    env = dict(os.environ, CTU_ORACLE_LIB=str(so))
    env.pop("CTU_MUTATIONS", None)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider"] + PINS,
                       cwd=REPO, env=env, capture_output=True, text=True, timeout=900)
    assert r.returncode != 0, f"mutation '{name}' survived the pin tests"
