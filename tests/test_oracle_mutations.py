"""Planted mistakes in the oracle must fail its pins.

Each case copies the oracle's C source, plants one plausible mistake (a
dropped term, a wrong sign, a swapped index, the paper's printed form where a
reading corrects it), builds the copy on the CPU and runs the pin tests
against it.  A mutant that passes every pin would mean the pins do not
constrain that part of the oracle.
"""
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "cshoracle.c")
SRC3 = os.path.join(ROOT, "oracle", "cshoracle3.c")

MUTANTS = {
    # eq. (28) as printed: 1/2 - max(lam0, 0) k instead of 1/2 + min(lam0, 0) k
    "eq28_printed_sign": ("w_lo[m] = w[m] - (0.5 + k * fmin(lam0, 0.0)) * dwm[m];",
                          "w_lo[m] = w[m] - (0.5 - k * fmax(lam0, 0.0)) * dwm[m];"),
    # eq. (31) not added (CTU-only tracing with an HLL flux)
    "eq31_dropped": ("for (int m = 0; m < NV; ++m) w_hi[m] -= k * ((lam[a] - lamM) * pa) * R[m][a];",
                     "(void)0;"),
    # MC limiter without the extremum clause
    "mc_no_extremum_clause": ("if (dl * dr <= 0.0) return 0.0;", ""),
    # transverse predictor with the wrong sign
    "transverse_sign": ("xlo[s + m] -= ky * Bdw[m];", "xlo[s + m] += ky * Bdw[m];"),
    # transverse predictor dropped on the y faces
    "transverse_dropped_y": ("yhi[s + m] -= kx * Adw[m];", "(void)Adw;"),
    # flux: Pxy u term dropped from the Exy flux
    "flux_exy_term": ("F[4] = U[4] * u + pxy * u + pxx * v;", "F[4] = U[4] * u + pxx * v;"),
    # flux: y-flux of Exx with the wrong stress component
    "flux_y_exx": ("G[3] = U[3] * v + 2.0 * pxy * u;", "G[3] = U[3] * v + 2.0 * w[IXX] * u;"),
    # left eigenvector with a sign error
    "left_eigvec_sign": ("{0.0, q / (2.0 * c), -1.0 / (2.0 * c), -pxy / (2.0 * pxx * pxx), 1.0 / (2.0 * pxx), 0.0},",
                         "{0.0, -q / (2.0 * c), -1.0 / (2.0 * c), -pxy / (2.0 * pxx * pxx), 1.0 / (2.0 * pxx), 0.0},"),
    # Jacobian as printed in eq. (16): no transverse compression term Pyy u_x
    "jacobian_printed": ("A[IYY][IU] = pyy;", "A[IYY][IU] = 0.0;"),
    # y Jacobian with a transposed entry
    "jac_y_index": ("B[IXY][IU] = pyy;", "B[IU][IXY] = pyy;"),
    # HLL with the wrong sign of the dissipation term
    "hll_sign": ("flux[m] = (sr * Fl[m] - sl * Fr[m] + sl * sr * (Ur[m] - Ul[m])) / (sr - sl);",
                 "flux[m] = (sr * Fl[m] - sl * Fr[m] - sl * sr * (Ur[m] - Ul[m])) / (sr - sl);"),
    # update with the y flux difference scaled by dx
    "update_dy": ("const double cx = dt / g->dx, cy = twod ? dt / g->dy : 0.0;",
                  "const double cx = dt / g->dx, cy = twod ? dt / g->dx : 0.0;"),
    # kick on the wrong velocity component
    "kick_component": ("w[IV] += dt * ay;", "w[IV] += dt * ax;"),
    # CFL rate without the y term
    "cfl_no_y": ("if (twod) s += (fabs(w[IV]) + sqrt(3.0 * w[IYY] / w[IR])) / g->dy;", ""),
    # outflow ghost copies the second cell instead of the edge cell.  (Reflecting
    # ghost -2 alone would be an equivalent mutant: with MC the slope of ghost
    # -1 is zero whatever ghost -2 holds.)
    "bc_outflow": ("if (i < 0) return 0;", "if (i < 0) return 1;"),
    # periodic wrap off by one
    "bc_periodic": ("return (r < 0) ? r + n : r;", "return (r < 0) ? r + n - 1 : r;"),
    # KT: dissipation with the wrong sign, local speed without |u|, stage
    # without the 1/2 of the midpoint rule, reconstruction without the limiter
    "kt_dissipation_sign": ("flux[m] = 0.5 * (Fl[m] + Fr[m]) - 0.5 * a * (Ur[m] - Ul[m]);",
                            "flux[m] = 0.5 * (Fl[m] + Fr[m]) + 0.5 * a * (Ur[m] - Ul[m]);"),
    "kt_speed_no_u": ("double rl = fabs(wl[iv]) + sqrt(3.0 * wl[ip] / wl[IR]);",
                      "double rl = sqrt(3.0 * wl[ip] / wl[IR]);"),
    "kt_midpoint_half": ("Us[m * n + c] = U[m * n + c] + 0.5 * dt * L[c * NV + m];",
                         "Us[m * n + c] = U[m * n + c] + dt * L[c * NV + m];"),
    "kt_unlimited_x": ("sxl[s + m] = orc_mc(w[m] - wl[m], 0.5 * (wr[m] - wl[m]), wr[m] - w[m]);",
                       "sxl[s + m] = 0.5 * (wr[m] - wl[m]);"),
    # Fourier amplitudes: the angle as printed, arctan(y / x) (two quadrants
    # only); the disc mass taken over the region instead of the whole grid;
    # the mode number off by one
    "fourier_atan_printed": ("const double phi = atan2(y, x);", "const double phi = atan(y / x);"),
    "fourier_mass_in_region": ("            mass[j] += sigma * cell;\n            if (fabs(x) > X || fabs(y) > Y || (x == 0.0 && y == 0.0)) continue;",
                               "            if (fabs(x) > X || fabs(y) > Y || (x == 0.0 && y == 0.0)) continue;\n            mass[j] += sigma * cell;"),
    # HLLC: contact speed with the stress jump reversed; transverse star velocity
    # without the shear-stress jump; the normal energy's stress flux halved;
    # the star sides exchanged
    "hllc_sstar_sign": ("const double ss = (wr[inn] - wl[inn] + D[0] * wl[in] - D[1] * wr[in]) / (D[0] - D[1]);",
                        "const double ss = (wl[inn] - wr[inn] + D[0] * wl[in] - D[1] * wr[in]) / (D[0] - D[1]);"),
    "hllc_vstar_no_stress": ("const double vs = (wr[IXY] - wl[IXY] + D[0] * wl[it] - D[1] * wr[it]) / (D[0] - D[1]);",
                             "const double vs = (D[0] * wl[it] - D[1] * wr[it]) / (D[0] - D[1]);"),
    "hllc_energy_flux": ("Ns[inn] = 2.0 * pnn * ss;", "Ns[inn] = pnn * ss;"),
    "hllc_sides": ("} else if (S[1] >= 0.0) {", "} else if (S[1] <= 0.0) {"),
    # three dimensions: a flux term dropped, a Jacobian entry on the wrong
    # velocity, a shear eigenvector sign, half the transverse predictor on the
    # high faces, the CFL sum without z
    "flux3_term": ("F[pidx(i, j)] = U[pidx(i, j)] * uk + w[pidx(k, i)] * w[1 + j] + w[pidx(k, j)] * w[1 + i];",
                   "F[pidx(i, j)] = U[pidx(i, j)] * uk + w[pidx(k, i)] * w[1 + j];"),
    "jac3_entry": ("A[r][1 + i] += w[pidx(j, k)];", "A[r][1 + i] += w[pidx(i, k)];"),
    "eigen3_shear_sign": ("R[pidx(n, ts)][cidx] = pnn;", "R[pidx(n, ts)][cidx] = -pnn;"),
    "transverse3_half": ("hi[m] -= kf[o2] * Adw[o2][m];", "hi[m] -= 0.5 * kf[o2] * Adw[o2][m];"),
    "cfl3_no_z": ("for (int k = 0; k < 3; ++k) s += (fabs(w[1 + k])", "for (int k = 0; k < 2; ++k) s += (fabs(w[1 + k])"),
    # validity check (Sec. 2, positive-definite stress): the determinant test
    # dropped; the finiteness test dropped (an infinite Exx leaves every sign
    # test true)
    "physical_no_det": ("w[IXX] > 0.0 && w[IYY] > 0.0 &&\n                   w[IXX] * w[IYY] - w[IXY] * w[IXY] > 0.0;",
                        "w[IXX] > 0.0 && w[IYY] > 0.0;"),
    "physical_no_isfinite": ("for (int m = 0; m < NV; ++m) good = good && isfinite(w[m]);", ""),
    # branch pattern: the limiter's one-sided cases exchanged; the HLL S_L
    # code on the wrong side of the tie
    "branch_mc_sides": ("return l <= r ? ORC_MC_LEFT : ORC_MC_RIGHT;", "return l <= r ? ORC_MC_RIGHT : ORC_MC_LEFT;"),
    "branch_hll_left": ("codes[0] = l1 < l0;", "codes[0] = l1 > l0;"),
    "fourier_mode_index": ("re[(size_t)j * mmax + m - 1] += sigma * cos(m * phi) * cell;",
                           "re[(size_t)j * mmax + m - 1] += sigma * cos((m + 1) * phi) * cell;"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_fails_a_pin(name, tmp_path):
    old, new = MUTANTS[name]
    # the site must be unique within a file; a statement the 2-D and 3-D
    # oracles share is planted in both
    srcs = {p: open(p).read() for p in (SRC, SRC3)}
    assert all(t.count(old) <= 1 for t in srcs.values()) and any(t.count(old) for t in srcs.values()), \
        f"mutation site not found uniquely: {name}"
    for p, t in srcs.items():
        (tmp_path / os.path.basename(p)).write_text(t.replace(old, new))
    for h in ("cshoracle.h",):
        (tmp_path / h).write_text(open(os.path.join(ROOT, "oracle", h)).read())
    lib = tmp_path / "libmut.so"
    subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                    "-o", str(lib), str(tmp_path / "cshoracle.c"), str(tmp_path / "cshoracle3.c"), "-lm"],
                   check=True, cwd=tmp_path)
    env = dict(os.environ, CSH_ORACLE_LIB=str(lib), OMP_NUM_THREADS="4")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_branch_pins.py"),
                        os.path.join(ROOT, "tests", "test_oracle_pins.py"),
                        os.path.join(ROOT, "tests", "test_oracle_kt_pins.py"),
                        os.path.join(ROOT, "tests", "test_oracle_fourier_pins.py"),
                        os.path.join(ROOT, "tests", "test_oracle_hllc_pins.py"),
                        os.path.join(ROOT, "tests", "test_oracle3_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"mutant {name} passed every pin:\n{r.stdout[-2000:]}"
