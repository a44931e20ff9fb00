/*
 * FP64 CPU oracle for the collisionless-stellar-hydrodynamics sweep.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or helper with
 * the HIP implementation.
 *
 * What it computes: one step of the MUSCL-Hancock scheme with characteristic
 * tracing and an HLL Riemann flux for the Boltzmann moment equations (BME) of
 * Mitchell, Vorobyov & Hensler, "Collisionless Stellar Hydrodynamics as an
 * Efficient Alternative to N-body Methods" (arXiv:1210.5246):
 *   - equations: Sec. 2, eqs. (2)-(4), closed with zero heat flux Q_ijk = 0;
 *   - conserved / primitive variables: Sec. 3.3, eq. (10) and the W vector of
 *     eq. (11), here in 2-D with the full symmetric stress tensor;
 *   - eigen-system: Sec. 3.3, eqs. (14)-(18), re-derived for the full 2-D
 *     tensor (see the readings below);
 *   - slopes, projection, MC limiter, back-projection: Sec. 3.3, eqs. (19)-(26);
 *   - interface extrapolation and characteristic tracing: Sec. 3.3,
 *     eqs. (27)-(32) (eqs. 40-45 of Stone et al. 2008, which the paper follows);
 *   - HLL flux and the unsplit conservative update: Sec. 3.3;
 *   - operator-split external-gravity kick after the hydro step: Sec. 3.3,
 *     last paragraph.
 *
 * Formulation (deliberately literal and slow): the left/right eigenvectors are
 * built as dense 6x6 matrices, every projection is a dense mat-vec, and the
 * tracing corrections are explicit per-wave sums.  Everything is FP64 and
 * row-at-a-time; OpenMP only splits independent rows/cells.
 *
 * Readings of the paper taken here (each one is listed with its reason in
 * the design notes of the repository):
 *   R1  full symmetric 2-D tensor (Pxy kept), fluxes from eqs. (2)-(4);
 *   R2  the primitive Jacobian is derived from the conservative flux
 *       (the printed eq. (16) lacks rho in entry (1,2) and the transverse
 *       compression terms); eigenvalues ordered to match the eigenvector columns;
 *   R3  MC limiter returns 0 when the one-sided differences differ in sign;
 *   R4  eq. (28) is read with the domain-of-dependence sign:
 *       w_R,i-1/2 = w_i - [1/2 + min(lambda0,0) dt/(2dx)] dw;
 *   R5  eqs. (31)-(32) are added to eqs. (29)-(30); a wave with lambda == 0
 *       goes into the HLL-correction sum, so each wave is counted once;
 *   R6  dimensionally unsplit: each x-face state also receives the transverse
 *       predictor -(dt/2dy) B(w) dw_y (and y-face states -(dt/2dx) A(w) dw_x);
 *   R7  HLL signal speeds: Davis estimates with a = sqrt(3 Pnn / rho);
 *   R8  CFL: s = max[(|u|+a_x)/dx + (|v|+a_y)/dy] (1-D: (|u|+a_x)/dx);
 *   R9  boundaries: periodic wrap or zero-gradient outflow, 2 ghost cells;
 *   R10 fixed external potential of a flat rotation curve,
 *       a = -vc^2 (x, y) / (x^2 + y^2 + rc^2), applied as an exact kick of the
 *       velocity after the hydro step (rho and P unchanged).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "cshoracle.h"

#ifdef _OPENMP
#include <omp.h>
#endif

enum { NV = 6 };
enum { IR = 0, IU = 1, IV = 2, IXX = 3, IXY = 4, IYY = 5 };

/* ---------------------------------------------------------------------- */
/* Variables.  Sec. 2: E_ij = Pi_ij + rho u_i u_j, Pi_ij = rho sigma^2_ij.   */
/* ---------------------------------------------------------------------- */

void orc_cons(const double w[NV], double U[NV])
{
    double rho = w[IR], u = w[IU], v = w[IV];
    U[0] = rho;
    U[1] = rho * u;
    U[2] = rho * v;
    U[3] = w[IXX] + rho * u * u;
    U[4] = w[IXY] + rho * u * v;
    U[5] = w[IYY] + rho * v * v;
}

void orc_prim(const double U[NV], double w[NV])
{
    double rho = U[0];
    double u = U[1] / rho, v = U[2] / rho;
    w[IR] = rho;
    w[IU] = u;
    w[IV] = v;
    w[IXX] = U[3] - rho * u * u;
    w[IXY] = U[4] - rho * u * v;
    w[IYY] = U[5] - rho * v * v;
}

/* Physical flux in x: the k = x divergence terms of eqs. (2)-(4),
 * F = (rho u, rho u u + Pxx, rho v u + Pxy, Exx u + 2 Pxx u,
 *      Exy u + Pxy u + Pxx v, Eyy u + 2 Pxy v).
 * For Pxy = 0 this is the 2-D restriction of the F column of eq. (10). */
void orc_flux_x(const double U[NV], double F[NV])
{
    double w[NV];
    orc_prim(U, w);
    double rho = w[IR], u = w[IU], v = w[IV];
    double pxx = w[IXX], pxy = w[IXY];
    F[0] = rho * u;
    F[1] = rho * u * u + pxx;
    F[2] = rho * v * u + pxy;
    F[3] = U[3] * u + 2.0 * pxx * u;
    F[4] = U[4] * u + pxy * u + pxx * v;
    F[5] = U[5] * u + 2.0 * pxy * v;
}

/* Physical flux in y: the k = y divergence terms of eqs. (2)-(4),
 * G = (rho v, rho u v + Pxy, rho v v + Pyy, Exx v + 2 Pxy u,
 *      Exy v + Pyy u + Pxy v, Eyy v + 2 Pyy v). */
void orc_flux_y(const double U[NV], double G[NV])
{
    double w[NV];
    orc_prim(U, w);
    double rho = w[IR], u = w[IU], v = w[IV];
    double pxy = w[IXY], pyy = w[IYY];
    G[0] = rho * v;
    G[1] = rho * u * v + pxy;
    G[2] = rho * v * v + pyy;
    G[3] = U[3] * v + 2.0 * pxy * u;
    G[4] = U[4] * v + pyy * u + pxy * v;
    G[5] = U[5] * v + 2.0 * pyy * v;
}

/* ---------------------------------------------------------------------- */
/* Eigen-system (Sec. 3.3, eqs. (12)-(18), reading R2).                     */
/* ---------------------------------------------------------------------- */

/* Primitive Jacobian in x, A = dF~/dW, rows of the quasi-linear system
 *   rho_t + u rho_x + rho u_x = 0
 *   u_t + u u_x + Pxx_x / rho = 0
 *   v_t + u v_x + Pxy_x / rho = 0
 *   Pxx_t + u Pxx_x + 3 Pxx u_x = 0
 *   Pxy_t + u Pxy_x + 2 Pxy u_x + Pxx v_x = 0
 *   Pyy_t + u Pyy_x + Pyy u_x + 2 Pxy v_x = 0
 * which follows from eqs. (2)-(4) with Q = 0. */
void orc_jac_x(const double w[NV], double A[NV][NV])
{
    memset(A, 0, sizeof(double) * NV * NV);
    double rho = w[IR], u = w[IU];
    double pxx = w[IXX], pxy = w[IXY], pyy = w[IYY];
    for (int k = 0; k < NV; ++k) A[k][k] = u;
    A[IR][IU] = rho;
    A[IU][IXX] = 1.0 / rho;
    A[IV][IXY] = 1.0 / rho;
    A[IXX][IU] = 3.0 * pxx;
    A[IXY][IU] = 2.0 * pxy;
    A[IXY][IV] = pxx;
    A[IYY][IU] = pyy;
    A[IYY][IV] = 2.0 * pxy;
}

/* Primitive Jacobian in y, B = dG~/dW (the same moment equations, k = y):
 *   rho_t + v rho_y + rho v_y = 0
 *   u_t + v u_y + Pxy_y / rho = 0
 *   v_t + v v_y + Pyy_y / rho = 0
 *   Pxx_t + v Pxx_y + Pxx v_y + 2 Pxy u_y = 0
 *   Pxy_t + v Pxy_y + 2 Pxy v_y + Pyy u_y = 0
 *   Pyy_t + v Pyy_y + 3 Pyy v_y = 0 */
void orc_jac_y(const double w[NV], double B[NV][NV])
{
    memset(B, 0, sizeof(double) * NV * NV);
    double rho = w[IR], v = w[IV];
    double pxx = w[IXX], pxy = w[IXY], pyy = w[IYY];
    for (int k = 0; k < NV; ++k) B[k][k] = v;
    B[IR][IV] = rho;
    B[IU][IXY] = 1.0 / rho;
    B[IV][IYY] = 1.0 / rho;
    B[IXX][IU] = 2.0 * pxy;
    B[IXX][IV] = pxx;
    B[IXY][IU] = pyy;
    B[IXY][IV] = 2.0 * pxy;
    B[IYY][IV] = 3.0 * pyy;
}

/* Eigenvalues and dense eigenvectors of A (x-direction).
 * a = sqrt(3 Pxx / rho) is the directional sound speed of eq. (15) with
 * gamma = 3; c = sqrt(Pxx / rho) is the shear speed that the off-diagonal
 * stress adds (the paper notes the non-diagonal system has more waves,
 * Sec. 3.3 before eq. (14)).  Waves, in increasing speed:
 *   lam = (u - a, u - c, u, u, u + c, u + a).
 * R[:, k] is the right eigenvector of wave k, L[k, :] the left one, L R = I.
 * For Pxy = 0 the fast pair and the rho/contact columns reduce to those of
 * eqs. (17)-(18). */
void orc_eigen_x(const double w[NV], double lam[NV], double R[NV][NV], double L[NV][NV])
{
    double rho = w[IR], u = w[IU];
    double pxx = w[IXX], pxy = w[IXY], pyy = w[IYY];
    double a = sqrt(3.0 * pxx / rho);
    double c = sqrt(pxx / rho);
    double q = pxy / pxx;

    lam[0] = u - a;
    lam[1] = u - c;
    lam[2] = u;
    lam[3] = u;
    lam[4] = u + c;
    lam[5] = u + a;

    /* right eigenvectors, one per column */
    double r[NV][NV] = {
        {rho, -a, -a * q, 3.0 * pxx, 3.0 * pxy, pyy + 2.0 * pxy * q}, /* u - a */
        {0.0, 0.0, -c, 0.0, pxx, 2.0 * pxy},                         /* u - c */
        {1.0, 0.0, 0.0, 0.0, 0.0, 0.0},                              /* u: density */
        {0.0, 0.0, 0.0, 0.0, 0.0, 1.0},                              /* u: Pyy */
        {0.0, 0.0, c, 0.0, pxx, 2.0 * pxy},                          /* u + c */
        {rho, a, a * q, 3.0 * pxx, 3.0 * pxy, pyy + 2.0 * pxy * q},  /* u + a */
    };
    for (int k = 0; k < NV; ++k)
        for (int m = 0; m < NV; ++m) R[m][k] = r[k][m];

    double l[NV][NV] = {
        {0.0, -1.0 / (2.0 * a), 0.0, 1.0 / (6.0 * pxx), 0.0, 0.0},
        {0.0, q / (2.0 * c), -1.0 / (2.0 * c), -pxy / (2.0 * pxx * pxx), 1.0 / (2.0 * pxx), 0.0},
        {1.0, 0.0, 0.0, -rho / (3.0 * pxx), 0.0, 0.0},
        {0.0, 0.0, 0.0, -pyy / (3.0 * pxx) + 4.0 * pxy * pxy / (3.0 * pxx * pxx), -2.0 * q, 1.0},
        {0.0, -q / (2.0 * c), 1.0 / (2.0 * c), -pxy / (2.0 * pxx * pxx), 1.0 / (2.0 * pxx), 0.0},
        {0.0, 1.0 / (2.0 * a), 0.0, 1.0 / (6.0 * pxx), 0.0, 0.0},
    };
    memcpy(L, l, sizeof(l));
}

/* The y-direction system is the x-direction one with the roles of the axes
 * exchanged: with S the permutation (rho, u, v, Pxx, Pxy, Pyy) ->
 * (rho, v, u, Pyy, Pxy, Pxx) (S = S^-1), B(w) = S A(S w) S, so
 * R_y = S R_x(S w), L_y = L_x(S w) S, lam_y = lam_x(S w). */
static const int SWAPXY[NV] = {IR, IV, IU, IYY, IXY, IXX};

void orc_eigen_y(const double w[NV], double lam[NV], double R[NV][NV], double L[NV][NV])
{
    double ws[NV], Rs[NV][NV], Ls[NV][NV];
    for (int m = 0; m < NV; ++m) ws[m] = w[SWAPXY[m]];
    orc_eigen_x(ws, lam, Rs, Ls);
    for (int m = 0; m < NV; ++m)
        for (int k = 0; k < NV; ++k) {
            R[m][k] = Rs[SWAPXY[m]][k];
            L[k][m] = Ls[k][SWAPXY[m]];
        }
}

/* ---------------------------------------------------------------------- */
/* Slope limiting (Sec. 3.3, eqs. (19)-(26)).                               */
/* ---------------------------------------------------------------------- */

static double sgn(double x) { return (x > 0.0) ? 1.0 : ((x < 0.0) ? -1.0 : 0.0); }

/* Monotonised-central limiter of eq. (25), with the standard TVD clause
 * (reading R3): zero at a local extremum of the characteristic variable. */
double orc_mc(double dl, double dc, double dr)
{
    if (dl * dr <= 0.0) return 0.0;
    double m = fmin(fmin(2.0 * fabs(dl), fabs(dc)), 2.0 * fabs(dr));
    return sgn(dc) * m;
}

static void matvec(const double M[NV][NV], const double x[NV], double y[NV])
{
    for (int i = 0; i < NV; ++i) {
        double s = 0.0;
        for (int k = 0; k < NV; ++k) s += M[i][k] * x[k];
        y[i] = s;
    }
}

/* Which argument of eq. (25) the MC limiter takes (branch codes of
 * orc_branches): 0 at an extremum (the TVD clause, reading R3), else the
 * first minimal one of |dc| (1), 2|dl| (2), 2|dr| (3). */
static int mc_branch(double dl, double dc, double dr)
{
    if (dl * dr <= 0.0) return ORC_MC_OFF;
    const double c = fabs(dc), l = 2.0 * fabs(dl), r = 2.0 * fabs(dr);
    if (c <= l && c <= r) return ORC_MC_CENTRED;
    return l <= r ? ORC_MC_LEFT : ORC_MC_RIGHT;
}

/* Limited primitive slope of the centre cell from its two neighbours along
 * one direction (dir 0 = x, 1 = y): differences eqs. (19)-(21), projection on
 * the left eigenvectors eqs. (22)-(24), MC limiting eq. (25), projection back
 * on the right eigenvectors eq. (26).  codes (optional) receives the branch
 * each wave's limiter takes. */
static void limited_slope(int dir, const double wm[NV], const double w0[NV], const double wp[NV],
                          double dwm[NV], int codes[NV])
{
    double lam[NV], R[NV][NV], L[NV][NV];
    if (dir == 0) orc_eigen_x(w0, lam, R, L);
    else orc_eigen_y(w0, lam, R, L);

    double dL[NV], dC[NV], dR[NV];
    for (int m = 0; m < NV; ++m) {
        dL[m] = w0[m] - wm[m];
        dC[m] = (wp[m] - wm[m]) / 2.0;
        dR[m] = wp[m] - w0[m];
    }
    double uL[NV], uC[NV], uR[NV], um[NV];
    matvec(L, dL, uL);
    matvec(L, dC, uC);
    matvec(L, dR, uR);
    for (int k = 0; k < NV; ++k) um[k] = orc_mc(uL[k], uC[k], uR[k]);
    if (codes)
        for (int k = 0; k < NV; ++k) codes[k] = mc_branch(uL[k], uC[k], uR[k]);
    for (int m = 0; m < NV; ++m) {
        double s = 0.0;
        for (int k = 0; k < NV; ++k) s += um[k] * R[m][k];
        dwm[m] = s;
    }
}

void orc_limited_slope(int dir, const double wm[NV], const double w0[NV], const double wp[NV],
                       double dwm[NV])
{
    limited_slope(dir, wm, w0, wp, dwm, NULL);
}

/* ---------------------------------------------------------------------- */
/* Interface states (Sec. 3.3, eqs. (27)-(32)).                             */
/* ---------------------------------------------------------------------- */

/* Time-centred states on the two faces of a cell along direction dir, from the
 * cell's primitive state w and its limited slope dwm along dir.
 *   w_hi = state on the high face (i+1/2), the "w_L,i+1/2" of the paper;
 *   w_lo = state on the low face (i-1/2), the "w_R,i-1/2" of the paper.
 * k = dt / (2 dh).  lamM / lam0 are the largest / smallest eigenvalues.
 *   eq. (27): w~_hi = w + [1/2 - k max(lamM, 0)] dwm
 *   eq. (28): w~_lo = w - [1/2 + k min(lam0, 0)] dwm          (reading R4)
 *   eq. (29): w_hi += k sum_{lam_a > 0} (lamM - lam_a) (l_a . dwm) r_a
 *   eq. (31): w_hi -= k sum_{lam_a <= 0} (lam_a - lamM) (l_a . dwm) r_a  (R5)
 *   eq. (30): w_lo += k sum_{lam_a < 0} (lam0 - lam_a) (l_a . dwm) r_a
 *   eq. (32): w_lo -= k sum_{lam_a >= 0} (lam_a - lam0) (l_a . dwm) r_a  (R5) */
static void trace(int dir, const double w[NV], const double dwm[NV], double k,
                  double w_lo[NV], double w_hi[NV], int codes[2])
{
    double lam[NV], R[NV][NV], L[NV][NV];
    if (dir == 0) orc_eigen_x(w, lam, R, L);
    else orc_eigen_y(w, lam, R, L);
    double lamM = lam[0], lam0 = lam[0];
    for (int a = 1; a < NV; ++a) {
        lamM = fmax(lamM, lam[a]);
        lam0 = fmin(lam0, lam[a]);
    }
    if (codes) {  /* the two kinks of eqs. (27)-(28) */
        codes[0] = lamM > 0.0;
        codes[1] = lam0 < 0.0;
    }

    for (int m = 0; m < NV; ++m) {
        w_hi[m] = w[m] + (0.5 - k * fmax(lamM, 0.0)) * dwm[m];
        w_lo[m] = w[m] - (0.5 + k * fmin(lam0, 0.0)) * dwm[m];
    }

    for (int a = 0; a < NV; ++a) {
        double pa = 0.0; /* l_a . dwm */
        for (int m = 0; m < NV; ++m) pa += L[a][m] * dwm[m];

        /* high face: eq. (29) for right-moving waves, eq. (31) for the rest */
        if (lam[a] > 0.0) {
            for (int m = 0; m < NV; ++m) w_hi[m] += k * ((lamM - lam[a]) * pa) * R[m][a];
        } else {
            for (int m = 0; m < NV; ++m) w_hi[m] -= k * ((lam[a] - lamM) * pa) * R[m][a];
        }
        /* low face: eq. (30) for left-moving waves, eq. (32) for the rest */
        if (lam[a] < 0.0) {
            for (int m = 0; m < NV; ++m) w_lo[m] += k * ((lam0 - lam[a]) * pa) * R[m][a];
        } else {
            for (int m = 0; m < NV; ++m) w_lo[m] -= k * ((lam[a] - lam0) * pa) * R[m][a];
        }
    }
}

void orc_trace(int dir, const double w[NV], const double dwm[NV], double k,
               double w_lo[NV], double w_hi[NV])
{
    trace(dir, w, dwm, k, w_lo, w_hi, NULL);
}

/* ---------------------------------------------------------------------- */
/* HLL Riemann flux (Sec. 3.3; signal speeds reading R7).                   */
/* ---------------------------------------------------------------------- */

/* Branches of the HLL flux (codes of orc_branches): which face state sets
 * S_L (0 left, 1 right; the first on a tie), whether S_L >= 0, which sets S_R
 * (0 left, 1 right; the first on a tie), whether S_R <= 0. */
static void hll_branches(int dir, const double wl[NV], const double wr[NV], int codes[4])
{
    int iv = (dir == 0) ? IU : IV;
    int ip = (dir == 0) ? IXX : IYY;
    double al = sqrt(3.0 * wl[ip] / wl[IR]);
    double ar = sqrt(3.0 * wr[ip] / wr[IR]);
    double l0 = wl[iv] - al, l1 = wr[iv] - ar;
    double r0 = wl[iv] + al, r1 = wr[iv] + ar;
    codes[0] = l1 < l0;
    codes[1] = fmin(l0, l1) >= 0.0;
    codes[2] = r1 > r0;
    codes[3] = fmax(r0, r1) <= 0.0;
}

void orc_hll(int dir, const double wl[NV], const double wr[NV], double flux[NV])
{
    double Ul[NV], Ur[NV], Fl[NV], Fr[NV];
    orc_cons(wl, Ul);
    orc_cons(wr, Ur);
    int iv = (dir == 0) ? IU : IV;      /* normal velocity */
    int ip = (dir == 0) ? IXX : IYY;    /* normal stress */
    if (dir == 0) {
        orc_flux_x(Ul, Fl);
        orc_flux_x(Ur, Fr);
    } else {
        orc_flux_y(Ul, Fl);
        orc_flux_y(Ur, Fr);
    }
    double al = sqrt(3.0 * wl[ip] / wl[IR]);
    double ar = sqrt(3.0 * wr[ip] / wr[IR]);
    double sl = fmin(wl[iv] - al, wr[iv] - ar);
    double sr = fmax(wl[iv] + al, wr[iv] + ar);
    if (sl >= 0.0) {
        for (int m = 0; m < NV; ++m) flux[m] = Fl[m];
    } else if (sr <= 0.0) {
        for (int m = 0; m < NV; ++m) flux[m] = Fr[m];
    } else {
        for (int m = 0; m < NV; ++m)
            flux[m] = (sr * Fl[m] - sl * Fr[m] + sl * sr * (Ur[m] - Ul[m])) / (sr - sl);
    }
}


/* ---------------------------------------------------------------------- */
/* HLLC Riemann flux for the BME (the solver of the paper's runs, Sec. 4.1; */
/* its BME form is reading H1).                                             */
/* ---------------------------------------------------------------------- */
/*
 * Reading H1 (the paper names HLLC but gives no BME form): Toro's three-wave
 * solver with the outer speeds of HLL (reading R7) and one contact wave S*.
 * The star region between S_L and S_R has one velocity (S*, v*) and one pair
 * of normal-direction stresses (Pnn*, Pnt*) on both sides of the contact;
 * with D_K = rho_K (S_K - u_K):
 *   S*   = [Pnn_R - Pnn_L + D_L u_L - D_R u_R] / (D_L - D_R)
 *   Pnn* = Pnn_K + D_K (S* - u_K)             (the same for K = L, R)
 *   v*   = [Pnt_R - Pnt_L + D_L v_L - D_R v_R] / (D_L - D_R)
 *   Pnt* = Pnt_K + D_K (v* - v_K)             (the same for K = L, R)
 * (u, v the normal and transverse velocity).  Each conserved density of the
 * star state on side K follows from the jump condition across S_K, with the
 * star flux written as q* S* + N*, N* the non-advective part of the flux
 * evaluated with the star quantities:
 *   q*_K (S_K - S*) = q_K (S_K - u_K) + N* - N_K,
 *   N = (0, Pnn, Pnt, 2 Pnn u, Pnt u + Pnn v, 2 Pnt v) for
 *   q = (rho, rho u, rho v, Enn, Ent, Ett).
 * The jump conditions across S_L, S* and S_R then all hold, the fan average
 * equals the HLL state, and an isolated contact (jumps in rho and Ptt only)
 * is kept exactly.  The flux is F_L, F*_L, F*_R or F_R by the sign pattern
 * of S_L, S*, S_R.
 */
void orc_hllc_star(int dir, const double wl[NV], const double wr[NV], double speeds[3], double UsL[NV],
                   double UsR[NV])
{
    const int in = (dir == 0) ? IU : IV;     /* normal velocity / momentum */
    const int it = (dir == 0) ? IV : IU;     /* transverse */
    const int inn = (dir == 0) ? IXX : IYY;  /* normal-normal stress / energy */
    const int itt = (dir == 0) ? IYY : IXX;  /* transverse-transverse */
    const double *w[2] = {wl, wr};
    double U[2][NV];
    orc_cons(wl, U[0]);
    orc_cons(wr, U[1]);
    double a[2];
    for (int k = 0; k < 2; ++k) a[k] = sqrt(3.0 * w[k][inn] / w[k][IR]);
    const double S[2] = {fmin(wl[in] - a[0], wr[in] - a[1]), fmax(wl[in] + a[0], wr[in] + a[1])};
    double D[2];
    for (int k = 0; k < 2; ++k) D[k] = w[k][IR] * (S[k] - w[k][in]);
    const double ss = (wr[inn] - wl[inn] + D[0] * wl[in] - D[1] * wr[in]) / (D[0] - D[1]);
    const double vs = (wr[IXY] - wl[IXY] + D[0] * wl[it] - D[1] * wr[it]) / (D[0] - D[1]);
    const double pnn = wl[inn] + D[0] * (ss - wl[in]);
    const double pnt = wl[IXY] + D[0] * (vs - wl[it]);
    /* non-advective flux parts with the star quantities */
    double Ns[NV];
    Ns[IR] = 0.0;
    Ns[in] = pnn;
    Ns[it] = pnt;
    Ns[inn] = 2.0 * pnn * ss;
    Ns[IXY] = pnt * ss + pnn * vs;
    Ns[itt] = 2.0 * pnt * vs;
    for (int k = 0; k < 2; ++k) {
        const double *wk = w[k];
        const double u = wk[in], v = wk[it];
        double N[NV];
        N[IR] = 0.0;
        N[in] = wk[inn];
        N[it] = wk[IXY];
        N[inn] = 2.0 * wk[inn] * u;
        N[IXY] = wk[IXY] * u + wk[inn] * v;
        N[itt] = 2.0 * wk[IXY] * v;
        double *Us = k == 0 ? UsL : UsR;
        for (int m = 0; m < NV; ++m) Us[m] = (U[k][m] * (S[k] - u) + Ns[m] - N[m]) / (S[k] - ss);
    }
    speeds[0] = S[0];
    speeds[1] = ss;
    speeds[2] = S[1];
}

void orc_hllc(int dir, const double wl[NV], const double wr[NV], double flux[NV])
{
    double Ul[NV], Ur[NV], Fl[NV], Fr[NV], S[3], UsL[NV], UsR[NV];
    orc_cons(wl, Ul);
    orc_cons(wr, Ur);
    if (dir == 0) {
        orc_flux_x(Ul, Fl);
        orc_flux_x(Ur, Fr);
    } else {
        orc_flux_y(Ul, Fl);
        orc_flux_y(Ur, Fr);
    }
    orc_hllc_star(dir, wl, wr, S, UsL, UsR);
    if (S[0] >= 0.0) {
        for (int m = 0; m < NV; ++m) flux[m] = Fl[m];
    } else if (S[1] >= 0.0) {
        for (int m = 0; m < NV; ++m) flux[m] = Fl[m] + S[0] * (UsL[m] - Ul[m]);
    } else if (S[2] > 0.0) {
        for (int m = 0; m < NV; ++m) flux[m] = Fr[m] + S[2] * (UsR[m] - Ur[m]);
    } else {
        for (int m = 0; m < NV; ++m) flux[m] = Fr[m];
    }
}

/* ---------------------------------------------------------------------- */
/* Stepping the whole grid.                                                 */
/* ---------------------------------------------------------------------- */

static int map_index(int i, int n, int bc)
{
    if (bc == ORC_BC_PERIODIC) {
        int r = i % n;
        return (r < 0) ? r + n : r;
    }
    if (i < 0) return 0;
    if (i >= n) return n - 1;
    return i;
}

/* Acceleration of the fixed external potential (reading R10). */
static void external_accel(const orc_grid *g, int i, int j, double *ax, double *ay)
{
    double x = g->x0 + (i + 0.5) * g->dx;
    double y = (g->ny > 1) ? g->y0 + (j + 0.5) * g->dy : 0.0;
    double f = -g->vc * g->vc / (x * x + y * y + g->rc * g->rc);
    *ax = f * x;
    *ay = (g->ny > 1) ? f * y : 0.0;
}

/* Operator-split kick (Sec. 3.3, last paragraph): velocities gain dt * a,
 * density and stress are unchanged. */
static void kick(const orc_grid *g, int i, int j, double dt, double U[NV])
{
    if (g->vc == 0.0) return;
    double ax, ay, w[NV];
    external_accel(g, i, j, &ax, &ay);
    orc_prim(U, w);
    w[IU] += dt * ax;
    w[IV] += dt * ay;
    orc_cons(w, U);
}

/*
 * One step on a padded block.  Wp holds primitive states of an
 * (nxi+4) x (nyi+4) block (2-D) or nxi+4 cells (1-D), 2 ghost cells per side,
 * cell-major with 6 values per cell.  Uin holds the conserved states of the
 * nxi x nyi interior, Uout receives them after the step.  (gi0, gj0) is the
 * global index of the interior's first cell (for the external potential).
 * Fx / Fy (optional) receive the face fluxes: Fx[(nxi+1) * nyi], face i-1/2 of
 * interior cell i at column i; Fy[nxi * (nyi+1)].
 */
typedef void (*riemann_fn)(int dir, const double wl[NV], const double wr[NV], double flux[NV]);

static riemann_fn solver_fn(int solver)
{
    return solver == ORC_SOLVER_HLLC ? orc_hllc : orc_hll;
}

/*
 * The four time-centred face states of one cell (1-D: the two x ones) from
 * its primitive state w and its neighbours along x (wxm, wxp) and y (wym,
 * wyp): limited slopes (eqs. (19)-(26)), tracing (eqs. (27)-(32)) and, in
 * 2-D, the transverse predictor of the unsplit scheme (reading R6).  The
 * states land at offset s of xlo, xhi, ylo, yhi.  codes (optional) receives
 * the branches taken: per direction the six limiter codes and the two
 * tracing kinks.
 */
static void cell_faces(int twod, const double *w, const double *wxm, const double *wxp, const double *wym,
                       const double *wyp, double kx, double ky, double *xlo, double *xhi, double *ylo,
                       double *yhi, size_t s, int codes[16])
{
    double dwx[NV], dwy[NV] = {0, 0, 0, 0, 0, 0};
    limited_slope(0, wxm, w, wxp, dwx, codes);
    trace(0, w, dwx, kx, xlo + s, xhi + s, codes ? codes + NV : NULL);
    if (twod) {
        limited_slope(1, wym, w, wyp, dwy, codes ? codes + 8 : NULL);
        trace(1, w, dwy, ky, ylo + s, yhi + s, codes ? codes + 8 + NV : NULL);
        /* transverse predictor terms (reading R6) */
        double A[NV][NV], B[NV][NV], Adw[NV], Bdw[NV];
        orc_jac_x(w, A);
        orc_jac_y(w, B);
        matvec(A, dwx, Adw);
        matvec(B, dwy, Bdw);
        for (int m = 0; m < NV; ++m) {
            xlo[s + m] -= ky * Bdw[m];
            xhi[s + m] -= ky * Bdw[m];
            ylo[s + m] -= kx * Adw[m];
            yhi[s + m] -= kx * Adw[m];
        }
    }
}

static void step_block(const orc_grid *g, double dt, int nxi, int nyi, int twod,
                       const double *Wp, const double *Uin, int gi0, int gj0,
                       double *Uout, double *Fx, double *Fy, riemann_fn riemann)
{
    const int px = nxi + 4;                 /* padded row length */
    const int sx = nxi + 2, sy = twod ? nyi + 2 : 1;   /* cells -1..n */
    const double kx = dt / (2.0 * g->dx);
    const double ky = twod ? dt / (2.0 * g->dy) : 0.0;

#define WP(i, j) (Wp + ((size_t)((j) + (twod ? 2 : 0)) * px + (size_t)((i) + 2)) * NV)
#define SIDX(i, j) (((size_t)((j) + (twod ? 1 : 0)) * sx + (size_t)((i) + 1)) * NV)

    size_t ns = (size_t)sx * sy * NV;
    double *xlo = malloc(ns * sizeof(double)), *xhi = malloc(ns * sizeof(double));
    double *ylo = twod ? malloc(ns * sizeof(double)) : NULL;
    double *yhi = twod ? malloc(ns * sizeof(double)) : NULL;

    /* slopes and face states of interior cells and a one-cell ring */
    #pragma omp parallel for schedule(static)
    for (int jj = 0; jj < sy; ++jj) {
        int j = twod ? jj - 1 : 0;
        for (int i = -1; i <= nxi; ++i)
            cell_faces(twod, WP(i, j), WP(i - 1, j), WP(i + 1, j), twod ? WP(i, j - 1) : NULL,
                       twod ? WP(i, j + 1) : NULL, kx, ky, xlo, xhi, ylo, yhi, SIDX(i, j), NULL);
    }

    /* fluxes through every face of the interior */
    double *fx = malloc((size_t)(nxi + 1) * nyi * NV * sizeof(double));
    double *fy = twod ? malloc((size_t)nxi * (nyi + 1) * NV * sizeof(double)) : NULL;
    #pragma omp parallel for schedule(static)
    for (int j = 0; j < nyi; ++j)
        for (int i = 0; i <= nxi; ++i) /* face i-1/2 between cells i-1 and i */
            riemann(0, xhi + SIDX(i - 1, j), xlo + SIDX(i, j),
                    fx + ((size_t)j * (nxi + 1) + i) * NV);
    if (twod) {
        #pragma omp parallel for schedule(static)
        for (int j = 0; j <= nyi; ++j) /* face j-1/2 between cells j-1 and j */
            for (int i = 0; i < nxi; ++i)
                riemann(1, yhi + SIDX(i, j - 1), ylo + SIDX(i, j),
                        fy + ((size_t)j * nxi + i) * NV);
    }

    /* unsplit conservative update, then the source kick */
    const double cx = dt / g->dx, cy = twod ? dt / g->dy : 0.0;
    #pragma omp parallel for schedule(static)
    for (int j = 0; j < nyi; ++j)
        for (int i = 0; i < nxi; ++i) {
            size_t c = ((size_t)j * nxi + i) * NV;
            const double *fm = fx + ((size_t)j * (nxi + 1) + i) * NV;
            const double *fp = fm + NV;
            for (int m = 0; m < NV; ++m) {
                double du = -cx * (fp[m] - fm[m]);
                if (twod) {
                    const double *gm = fy + ((size_t)j * nxi + i) * NV;
                    const double *gp = fy + ((size_t)(j + 1) * nxi + i) * NV;
                    du -= cy * (gp[m] - gm[m]);
                }
                Uout[c + m] = Uin[c + m] + du;
            }
            kick(g, gi0 + i, gj0 + j, dt, Uout + c);
        }

    if (Fx) memcpy(Fx, fx, (size_t)(nxi + 1) * nyi * NV * sizeof(double));
    if (Fy && twod) memcpy(Fy, fy, (size_t)nxi * (nyi + 1) * NV * sizeof(double));
    free(xlo);
    free(xhi);
    free(ylo);
    free(yhi);
    free(fx);
    free(fy);
#undef WP
#undef SIDX
}

static int grid_ok(const orc_grid *g)
{
    if (g->nx < 1 || g->ny < 1) return 0;
    if (!(g->dx > 0.0)) return 0;
    if (g->ny > 1 && !(g->dy > 0.0)) return 0;
    if (g->bcx != ORC_BC_PERIODIC && g->bcx != ORC_BC_OUTFLOW) return 0;
    if (g->bcy != ORC_BC_PERIODIC && g->bcy != ORC_BC_OUTFLOW) return 0;
    return 1;
}

/* Padded primitive block around the interior [i0, i0+nxi) x [j0, j0+nyi). */
static double *padded_prim(const orc_grid *g, const double *U, int i0, int j0, int nxi, int nyi)
{
    int twod = g->ny > 1;
    int px = nxi + 4, py = twod ? nyi + 4 : 1;
    size_t n = (size_t)g->nx * g->ny;
    double *Wp = malloc((size_t)px * py * NV * sizeof(double));
    #pragma omp parallel for schedule(static)
    for (int jj = 0; jj < py; ++jj)
        for (int ii = 0; ii < px; ++ii) {
            int gi = map_index(i0 + ii - 2, g->nx, g->bcx);
            int gj = twod ? map_index(j0 + jj - 2, g->ny, g->bcy) : 0;
            size_t c = (size_t)gj * g->nx + gi;
            double Uc[NV];
            for (int m = 0; m < NV; ++m) Uc[m] = U[m * n + c];
            orc_prim(Uc, Wp + ((size_t)jj * px + ii) * NV);
        }
    return Wp;
}

int orc_step(const orc_grid *g, double dt, const double *U, double *Unew)
{
    return orc_step_rs(g, ORC_SOLVER_HLL, dt, U, Unew);
}

int orc_step_rs(const orc_grid *g, int solver, double dt, const double *U, double *Unew)
{
    if (!grid_ok(g)) return -1;
    int twod = g->ny > 1;
    size_t n = (size_t)g->nx * g->ny;
    double *Wp = padded_prim(g, U, 0, 0, g->nx, g->ny);
    double *Uin = malloc(n * NV * sizeof(double)), *Uout = malloc(n * NV * sizeof(double));
    for (size_t c = 0; c < n; ++c)
        for (int m = 0; m < NV; ++m) Uin[c * NV + m] = U[m * n + c];
    step_block(g, dt, g->nx, g->ny, twod, Wp, Uin, 0, 0, Uout, NULL, NULL, solver_fn(solver));
    for (size_t c = 0; c < n; ++c)
        for (int m = 0; m < NV; ++m) Unew[m * n + c] = Uout[c * NV + m];
    free(Wp);
    free(Uin);
    free(Uout);
    return 0;
}

int orc_step_cells(const orc_grid *g, double dt, const double *U, int64_t ncells,
                   const int64_t *cells, double *out)
{
    return orc_step_cells_rs(g, ORC_SOLVER_HLL, dt, U, ncells, cells, out);
}

int orc_step_cells_rs(const orc_grid *g, int solver, double dt, const double *U, int64_t ncells,
                      const int64_t *cells, double *out)
{
    if (!grid_ok(g)) return -1;
    int twod = g->ny > 1;
    size_t n = (size_t)g->nx * g->ny;
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t s = 0; s < ncells; ++s) {
        int64_t c = cells[s];
        int i = (int)(c % g->nx), j = (int)(c / g->nx);
        double *Wp = padded_prim(g, U, i, j, 1, 1);
        double Uin[NV], Uout[NV];
        for (int m = 0; m < NV; ++m) Uin[m] = U[m * n + (size_t)c];
        step_block(g, dt, 1, 1, twod, Wp, Uin, i, j, Uout, NULL, NULL, solver_fn(solver));
        for (int m = 0; m < NV; ++m) out[s * NV + m] = Uout[m];
        free(Wp);
    }
    return 0;
}

int orc_fluxes(const orc_grid *g, double dt, const double *U, double *Fx, double *Fy)
{
    return orc_fluxes_rs(g, ORC_SOLVER_HLL, dt, U, Fx, Fy);
}

int orc_fluxes_rs(const orc_grid *g, int solver, double dt, const double *U, double *Fx, double *Fy)
{
    if (!grid_ok(g)) return -1;
    int twod = g->ny > 1;
    int nx = g->nx, ny = g->ny;
    size_t n = (size_t)nx * ny;
    double *Wp = padded_prim(g, U, 0, 0, nx, ny);
    double *Uin = malloc(n * NV * sizeof(double)), *Uout = malloc(n * NV * sizeof(double));
    for (size_t c = 0; c < n; ++c)
        for (int m = 0; m < NV; ++m) Uin[c * NV + m] = U[m * n + c];
    size_t nfx = (size_t)(nx + 1) * ny, nfy = (size_t)nx * (ny + 1);
    double *fx = malloc(nfx * NV * sizeof(double));
    double *fy = twod ? malloc(nfy * NV * sizeof(double)) : NULL;
    step_block(g, dt, nx, ny, twod, Wp, Uin, 0, 0, Uout, fx, fy, solver_fn(solver));
    for (size_t f = 0; f < nfx; ++f)
        for (int m = 0; m < NV; ++m) Fx[m * nfx + f] = fx[f * NV + m];
    if (twod && Fy)
        for (size_t f = 0; f < nfy; ++f)
            for (int m = 0; m < NV; ++m) Fy[m * nfy + f] = fy[f * NV + m];
    free(Wp);
    free(Uin);
    free(Uout);
    free(fx);
    free(fy);
    return 0;
}

/*
 * Branch pattern of one step: which side of every kink of the scheme each
 * decision falls on (the limiter's cases, the tracing coefficients' max/min
 * with 0, the HLL speed estimates' min/max and their clipping).  Where two
 * states give the same pattern, the step is one smooth function on the
 * segment between them (up to a switch and back), so a central difference
 * across it is a derivative.  Layout, all int:
 *   per extended cell (j = -1..ny in 2-D, 0 in 1-D; i = -1..nx; x fastest):
 *     16 codes: x limiter codes of the six waves, x tracing kinks (lamM > 0,
 *     lam0 < 0), then the same 8 along y (zero in 1-D);
 *   per x face i-1/2 (j = 0..ny-1, i = 0..nx): the 4 HLL codes;
 *   per y face j-1/2 (j = 0..ny, i = 0..nx-1), 2-D only: the 4 HLL codes.
 */
int64_t orc_branch_count(const orc_grid *g)
{
    int twod = g->ny > 1;
    int64_t sx = g->nx + 2, sy = twod ? g->ny + 2 : 1;
    int64_t n = 16 * sx * sy + 4 * (int64_t)(g->nx + 1) * g->ny;
    if (twod) n += 4 * (int64_t)g->nx * (g->ny + 1);
    return n;
}

int orc_branches(const orc_grid *g, double dt, const double *U, int *codes)
{
    if (!grid_ok(g)) return -1;
    int twod = g->ny > 1;
    int nx = g->nx, ny = g->ny;
    const int px = nx + 4, sx = nx + 2, sy = twod ? ny + 2 : 1;
    const double kx = dt / (2.0 * g->dx), ky = twod ? dt / (2.0 * g->dy) : 0.0;
    double *Wp = padded_prim(g, U, 0, 0, nx, ny);
    size_t ns = (size_t)sx * sy * NV;
    double *xlo = malloc(ns * sizeof(double)), *xhi = malloc(ns * sizeof(double));
    double *ylo = twod ? malloc(ns * sizeof(double)) : NULL;
    double *yhi = twod ? malloc(ns * sizeof(double)) : NULL;
#define WP(i, j) (Wp + ((size_t)((j) + (twod ? 2 : 0)) * px + (size_t)((i) + 2)) * NV)
#define CELL(i, j) ((size_t)((j) + (twod ? 1 : 0)) * sx + (size_t)((i) + 1))
    #pragma omp parallel for schedule(static)
    for (int jj = 0; jj < sy; ++jj) {
        int j = twod ? jj - 1 : 0;
        for (int i = -1; i <= nx; ++i) {
            int *c = codes + 16 * CELL(i, j);
            for (int m = 0; m < 16; ++m) c[m] = 0;
            cell_faces(twod, WP(i, j), WP(i - 1, j), WP(i + 1, j), twod ? WP(i, j - 1) : NULL,
                       twod ? WP(i, j + 1) : NULL, kx, ky, xlo, xhi, ylo, yhi, CELL(i, j) * NV, c);
        }
    }
    int *fxc = codes + 16 * (size_t)sx * sy;
    #pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i <= nx; ++i)
            hll_branches(0, xhi + CELL(i - 1, j) * NV, xlo + CELL(i, j) * NV,
                         fxc + 4 * ((size_t)j * (nx + 1) + i));
    if (twod) {
        int *fyc = fxc + 4 * (size_t)(nx + 1) * ny;
        #pragma omp parallel for schedule(static)
        for (int j = 0; j <= ny; ++j)
            for (int i = 0; i < nx; ++i)
                hll_branches(1, yhi + CELL(i, j - 1) * NV, ylo + CELL(i, j) * NV,
                             fyc + 4 * ((size_t)j * nx + i));
    }
#undef WP
#undef CELL
    free(Wp);
    free(xlo);
    free(xhi);
    free(ylo);
    free(yhi);
    return 0;
}

/* Largest CFL rate of the state (reading R8): the timestep is C / s. */
double orc_max_signal_speed(const orc_grid *g, const double *U)
{
    int twod = g->ny > 1;
    size_t n = (size_t)g->nx * g->ny;
    double smax = 0.0;
    #pragma omp parallel for reduction(max : smax) schedule(static)
    for (size_t c = 0; c < n; ++c) {
        double Uc[NV], w[NV];
        for (int m = 0; m < NV; ++m) Uc[m] = U[m * n + c];
        orc_prim(Uc, w);
        double s = (fabs(w[IU]) + sqrt(3.0 * w[IXX] / w[IR])) / g->dx;
        if (twod) s += (fabs(w[IV]) + sqrt(3.0 * w[IYY] / w[IR])) / g->dy;
        if (s > smax) smax = s;
    }
    return smax;
}

/* 1 if every cell has rho > 0 and a positive-definite, finite stress. */
int orc_physical(const orc_grid *g, const double *U)
{
    size_t n = (size_t)g->nx * g->ny;
    int ok = 1;
    #pragma omp parallel for reduction(& : ok) schedule(static)
    for (size_t c = 0; c < n; ++c) {
        double Uc[NV], w[NV];
        for (int m = 0; m < NV; ++m) Uc[m] = U[m * n + c];
        orc_prim(Uc, w);
        int good = w[IR] > 0.0 && w[IXX] > 0.0 && w[IYY] > 0.0 &&
                   w[IXX] * w[IYY] - w[IXY] * w[IXY] > 0.0;
        for (int m = 0; m < NV; ++m) good = good && isfinite(w[m]);
        ok &= good;
    }
    return ok;
}

/* Field conversions for whole arrays (SoA [6][n]). */
void orc_cons_field(int64_t n, const double *W, double *U)
{
    #pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < n; ++c) {
        double w[NV], u[NV];
        for (int m = 0; m < NV; ++m) w[m] = W[m * n + c];
        orc_cons(w, u);
        for (int m = 0; m < NV; ++m) U[m * n + c] = u[m];
    }
}

void orc_prim_field(int64_t n, const double *U, double *W)
{
    #pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < n; ++c) {
        double u[NV], w[NV];
        for (int m = 0; m < NV; ++m) u[m] = U[m * n + c];
        orc_prim(u, w);
        for (int m = 0; m < NV; ++m) W[m * n + c] = w[m];
    }
}

/* Threads the OpenMP loops of this oracle use. */
int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads the following parallel loops use (n >= 1); no effect without OpenMP. */
void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ---------------------------------------------------------------------- */
/* Kurganov-Tadmor central scheme (Sec. 3.2, eqs. (5)-(8)).                */
/* ---------------------------------------------------------------------- */
/*
 * Readings (the section leaves them open):
 *   K1 reconstruction: piecewise-linear in the primitive variables, each
 *      component limited on its own with the MC limiter of eq. (25) (no
 *      characteristic projection: the scheme needs no eigenvectors);
 *   K2 local speed of eq. (7): the spectral radius of dF/dU at the two face
 *      states, |u_n| + a_n with a_n the directional sound speed of eq. (8),
 *      gamma = 3;
 *   K3 time integration: the Runge-Kutta midpoint rule
 *        U* = U^n + dt/2 L(U^n),  U^{n+1} = U^n + dt L(U*),
 *      L = -(H_{i+1/2} - H_{i-1/2})/dx - (H_{j+1/2} - H_{j-1/2})/dy (eq. (5),
 *      unsplit in 2-D), then the external kick as for the other scheme.
 */

/* Numerical flux of eq. (6) in direction dir from the states on the two sides
 * of a face: wl = u^- (left), wr = u^+ (right). */
void orc_kt_flux(int dir, const double wl[NV], const double wr[NV], double flux[NV])
{
    double Ul[NV], Ur[NV], Fl[NV], Fr[NV];
    orc_cons(wl, Ul);
    orc_cons(wr, Ur);
    int iv = (dir == 0) ? IU : IV, ip = (dir == 0) ? IXX : IYY;
    if (dir == 0) {
        orc_flux_x(Ul, Fl);
        orc_flux_x(Ur, Fr);
    } else {
        orc_flux_y(Ul, Fl);
        orc_flux_y(Ur, Fr);
    }
    double rl = fabs(wl[iv]) + sqrt(3.0 * wl[ip] / wl[IR]);
    double rr = fabs(wr[iv]) + sqrt(3.0 * wr[ip] / wr[IR]);
    double a = fmax(rl, rr);
    for (int m = 0; m < NV; ++m) flux[m] = 0.5 * (Fl[m] + Fr[m]) - 0.5 * a * (Ur[m] - Ul[m]);
}

/* L(U) on the interior of a padded block (same padding as step_block). */
static void kt_rhs(const orc_grid *g, int nxi, int nyi, int twod, const double *Wp, double *L)
{
    const int px = nxi + 4;
    const int sx = nxi + 2, sy = twod ? nyi + 2 : 1;
#define WP(i, j) (Wp + ((size_t)((j) + (twod ? 2 : 0)) * px + (size_t)((i) + 2)) * NV)
#define SIDX(i, j) (((size_t)((j) + (twod ? 1 : 0)) * sx + (size_t)((i) + 1)) * NV)
    size_t ns = (size_t)sx * sy * NV;
    double *sxl = malloc(ns * sizeof(double)), *syl = twod ? malloc(ns * sizeof(double)) : NULL;
    /* component-wise MC slopes of every cell and its one-cell ring (K1) */
    #pragma omp parallel for schedule(static)
    for (int jj = 0; jj < sy; ++jj) {
        int j = twod ? jj - 1 : 0;
        for (int i = -1; i <= nxi; ++i) {
            const double *w = WP(i, j), *wl = WP(i - 1, j), *wr = WP(i + 1, j);
            size_t s = SIDX(i, j);
            for (int m = 0; m < NV; ++m)
                sxl[s + m] = orc_mc(w[m] - wl[m], 0.5 * (wr[m] - wl[m]), wr[m] - w[m]);
            if (twod) {
                const double *wd = WP(i, j - 1), *wu = WP(i, j + 1);
                for (int m = 0; m < NV; ++m)
                    syl[s + m] = orc_mc(w[m] - wd[m], 0.5 * (wu[m] - wd[m]), wu[m] - w[m]);
            }
        }
    }
    const double idx = 1.0 / g->dx, idy = twod ? 1.0 / g->dy : 0.0;
    #pragma omp parallel for schedule(static)
    for (int j = 0; j < nyi; ++j)
        for (int i = 0; i < nxi; ++i) {
            double hp[NV], hm[NV], wl[NV], wr[NV];
            size_t c = ((size_t)j * nxi + i) * NV;
            /* x faces: i+1/2 (cells i, i+1) and i-1/2 (cells i-1, i) */
            for (int m = 0; m < NV; ++m) {
                wl[m] = WP(i, j)[m] + 0.5 * sxl[SIDX(i, j) + m];
                wr[m] = WP(i + 1, j)[m] - 0.5 * sxl[SIDX(i + 1, j) + m];
            }
            orc_kt_flux(0, wl, wr, hp);
            for (int m = 0; m < NV; ++m) {
                wl[m] = WP(i - 1, j)[m] + 0.5 * sxl[SIDX(i - 1, j) + m];
                wr[m] = WP(i, j)[m] - 0.5 * sxl[SIDX(i, j) + m];
            }
            orc_kt_flux(0, wl, wr, hm);
            for (int m = 0; m < NV; ++m) L[c + m] = -(hp[m] - hm[m]) * idx;
            if (twod) {
                for (int m = 0; m < NV; ++m) {
                    wl[m] = WP(i, j)[m] + 0.5 * syl[SIDX(i, j) + m];
                    wr[m] = WP(i, j + 1)[m] - 0.5 * syl[SIDX(i, j + 1) + m];
                }
                orc_kt_flux(1, wl, wr, hp);
                for (int m = 0; m < NV; ++m) {
                    wl[m] = WP(i, j - 1)[m] + 0.5 * syl[SIDX(i, j - 1) + m];
                    wr[m] = WP(i, j)[m] - 0.5 * syl[SIDX(i, j) + m];
                }
                orc_kt_flux(1, wl, wr, hm);
                for (int m = 0; m < NV; ++m) L[c + m] -= (hp[m] - hm[m]) * idy;
            }
        }
    free(sxl);
    free(syl);
#undef WP
#undef SIDX
}

/* One step of the KT scheme (readings K1-K3), U -> Unew. */
int orc_step_kt(const orc_grid *g, double dt, const double *U, double *Unew)
{
    if (!grid_ok(g)) return -1;
    int twod = g->ny > 1;
    size_t n = (size_t)g->nx * g->ny;
    double *Us = malloc(n * NV * sizeof(double)), *L = malloc(n * NV * sizeof(double));
    /* stage 1: U* = U + dt/2 L(U) */
    double *Wp = padded_prim(g, U, 0, 0, g->nx, g->ny);
    kt_rhs(g, g->nx, g->ny, twod, Wp, L);
    free(Wp);
    for (size_t c = 0; c < n; ++c)
        for (int m = 0; m < NV; ++m) Us[m * n + c] = U[m * n + c] + 0.5 * dt * L[c * NV + m];
    /* stage 2: U^{n+1} = U + dt L(U*) */
    Wp = padded_prim(g, Us, 0, 0, g->nx, g->ny);
    kt_rhs(g, g->nx, g->ny, twod, Wp, L);
    free(Wp);
    for (int j = 0; j < g->ny; ++j)
        for (int i = 0; i < g->nx; ++i) {
            size_t c = (size_t)j * g->nx + i;
            double u[NV];
            for (int m = 0; m < NV; ++m) u[m] = U[m * n + c] + dt * L[c * NV + m];
            kick(g, i, j, dt, u);
            for (int m = 0; m < NV; ++m) Unew[m * n + c] = u[m];
        }
    free(Us);
    free(L);
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Global Fourier amplitudes of the surface density (Sec. 4.4).            */
/* ---------------------------------------------------------------------- */
/*
 * A_m = |integral over the region of Sigma exp(i m phi) dx dy| / M_d, with
 * Sigma the density of the 2-D state.  Readings:
 *   F1 M_d is the mass of the whole grid (sum of rho dx dy over all cells);
 *   F2 phi is the polar angle of the cell centre in all four quadrants
 *      (atan2(y, x)); a cell centred exactly on the origin has no angle and
 *      is left out of the integral (it stays in M_d);
 *   F3 the integral is the midpoint sum over the cells whose centres lie in
 *      the closed rectangle [-X, X] x [-Y, Y] about the coordinate origin.
 * Row sums are formed independently and added in row order, so the result
 * does not depend on the thread count.  A[m - 1] receives A_m, m = 1..mmax.
 */
int orc_fourier_amplitudes(const orc_grid *g, const double *U, int mmax, double X, double Y, double *A)
{
    if (!grid_ok(g) || g->ny < 2 || mmax < 1) return -1;
    const int nx = g->nx, ny = g->ny;
    const double cell = g->dx * g->dy;
    double *re = calloc((size_t)ny * mmax, sizeof(double));
    double *im = calloc((size_t)ny * mmax, sizeof(double));
    double *mass = calloc((size_t)ny, sizeof(double));
    #pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j) {
        const double y = g->y0 + (j + 0.5) * g->dy;
        for (int i = 0; i < nx; ++i) {
            const double x = g->x0 + (i + 0.5) * g->dx;
            const double sigma = U[(size_t)j * nx + i];
            mass[j] += sigma * cell;
            if (fabs(x) > X || fabs(y) > Y || (x == 0.0 && y == 0.0)) continue;
            const double phi = atan2(y, x);
            for (int m = 1; m <= mmax; ++m) {
                re[(size_t)j * mmax + m - 1] += sigma * cos(m * phi) * cell;
                im[(size_t)j * mmax + m - 1] += sigma * sin(m * phi) * cell;
            }
        }
    }
    double M = 0.0;
    for (int j = 0; j < ny; ++j) M += mass[j];
    for (int m = 1; m <= mmax; ++m) {
        double sr = 0.0, si = 0.0;
        for (int j = 0; j < ny; ++j) {
            sr += re[(size_t)j * mmax + m - 1];
            si += im[(size_t)j * mmax + m - 1];
        }
        A[m - 1] = sqrt(sr * sr + si * si) / M;
    }
    free(re);
    free(im);
    free(mass);
    return 0;
}
