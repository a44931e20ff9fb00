/*
 * FP64 CPU oracle of the three-dimensional moment equations: the ten-moment
 * system (rho, rho u_i, E_ij = P_ij + rho u_i u_j, i <= j) with zero heat flux
 * (Sec. 2, eqs. (2)-(4) in three dimensions; the paper's stated extension with
 * ten eigenvalues, Sec. 3.3) advanced by the characteristic MUSCL-Hancock
 * scheme of Sec. 3.3 with an HLL flux, unsplit in three directions.
 *
 * TEST INFRASTRUCTURE ONLY (see cshoracle.c).  Plain C99, dense 10 x 10
 * eigenvector matrices (the right ones written from the eigen-analysis, the
 * left ones by Gauss-Jordan inversion), literal per-wave sums in the tracing,
 * a three-branch HLL.  Readings as in two dimensions (R1-R9, R12), with:
 *   T1 the transverse predictor of each face state carries the Jacobian
 *      terms of both other directions;
 *   T2 the CFL rate is the sum of (|u_k| + a_k) / dh_k over the three axes;
 *   T3 no external potential.
 *
 * Layout: structure of arrays [10][nz][ny][nx], x fastest; primitive
 * W = (rho, u, v, w, Pxx, Pxy, Pxz, Pyy, Pyz, Pzz), conserved
 * U = (rho, rho u, rho v, rho w, Exx, Exy, Exz, Eyy, Eyz, Ezz).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "cshoracle.h"

enum { N3 = 10 };
enum { R3 = 0 };

/* index of P_ij (and E_ij) in the 10-vector, i, j in 0..2 */
static int pidx(int i, int j)
{
    static const int t[3][3] = {{4, 5, 6}, {5, 7, 8}, {6, 8, 9}};
    return t[i][j];
}

void orc3_cons(const double w[N3], double U[N3])
{
    const double rho = w[R3];
    U[R3] = rho;
    for (int i = 0; i < 3; ++i) U[1 + i] = rho * w[1 + i];
    for (int i = 0; i < 3; ++i)
        for (int j = i; j < 3; ++j) U[pidx(i, j)] = w[pidx(i, j)] + rho * w[1 + i] * w[1 + j];
}

void orc3_prim(const double U[N3], double w[N3])
{
    const double rho = U[R3];
    w[R3] = rho;
    for (int i = 0; i < 3; ++i) w[1 + i] = U[1 + i] / rho;
    for (int i = 0; i < 3; ++i)
        for (int j = i; j < 3; ++j) w[pidx(i, j)] = U[pidx(i, j)] - rho * w[1 + i] * w[1 + j];
}

/* Flux along axis k of eqs. (2)-(4) with Q = 0:
 *   rho u_k,  rho u_i u_k + P_ik,  E_ij u_k + P_ki u_j + P_kj u_i. */
void orc3_flux(int k, const double U[N3], double F[N3])
{
    double w[N3];
    orc3_prim(U, w);
    const double uk = w[1 + k];
    F[R3] = U[1 + k];
    for (int i = 0; i < 3; ++i) F[1 + i] = U[1 + i] * uk + w[pidx(i, k)];
    for (int i = 0; i < 3; ++i)
        for (int j = i; j < 3; ++j)
            F[pidx(i, j)] = U[pidx(i, j)] * uk + w[pidx(k, i)] * w[1 + j] + w[pidx(k, j)] * w[1 + i];
}

/* Primitive Jacobian along axis k: W_t + A W_k = 0 with
 *   rho:  u_k d rho + rho d u_k
 *   u_i:  u_k d u_i + d P_ik / rho
 *   P_ij: u_k d P_ij + P_ij d u_k + P_ik d u_j + P_jk d u_i. */
void orc3_jac(int k, const double w[N3], double A[N3][N3])
{
    memset(A, 0, sizeof(double) * N3 * N3);
    const double rho = w[R3], uk = w[1 + k];
    for (int m = 0; m < N3; ++m) A[m][m] = uk;
    A[R3][1 + k] += rho;
    for (int i = 0; i < 3; ++i) A[1 + i][pidx(i, k)] += 1.0 / rho;
    for (int i = 0; i < 3; ++i)
        for (int j = i; j < 3; ++j) {
            const int r = pidx(i, j);
            A[r][1 + k] += w[r];
            A[r][1 + j] += w[pidx(i, k)];
            A[r][1 + i] += w[pidx(j, k)];
        }
}

/* Gauss-Jordan inverse with partial pivoting (returns 0 if singular). */
static int invert(const double M[N3][N3], double Inv[N3][N3])
{
    double a[N3][2 * N3];
    for (int i = 0; i < N3; ++i)
        for (int j = 0; j < N3; ++j) {
            a[i][j] = M[i][j];
            a[i][N3 + j] = (i == j) ? 1.0 : 0.0;
        }
    for (int c = 0; c < N3; ++c) {
        int p = c;
        for (int r = c + 1; r < N3; ++r)
            if (fabs(a[r][c]) > fabs(a[p][c])) p = r;
        if (a[p][c] == 0.0) return 0;
        if (p != c)
            for (int j = 0; j < 2 * N3; ++j) {
                double t = a[c][j];
                a[c][j] = a[p][j];
                a[p][j] = t;
            }
        const double d = a[c][c];
        for (int j = 0; j < 2 * N3; ++j) a[c][j] /= d;
        for (int r = 0; r < N3; ++r) {
            if (r == c) continue;
            const double f = a[r][c];
            if (f != 0.0)
                for (int j = 0; j < 2 * N3; ++j) a[r][j] -= f * a[c][j];
        }
    }
    for (int i = 0; i < N3; ++i)
        for (int j = 0; j < N3; ++j) Inv[i][j] = a[i][N3 + j];
    return 1;
}

/* Eigen-system along axis n (eigenvalues ascending):
 *   u - a, u - c (shear t1), u - c (shear t2), u (4: rho, P_t1t1, P_t1t2,
 *   P_t2t2), u + c (t1), u + c (t2), u + a,
 * a = sqrt(3 P_nn / rho), c = sqrt(P_nn / rho), t1 < t2 the other two axes.
 * Right eigenvectors (columns), with q_t = P_nt / P_nn:
 *   u +- a: (rho, +-a at u_n, +-a q_t at u_t, 3 P_nn, 3 P_nt,
 *            P_tt' + P_nt q_t' + P_nt' q_t at P_tt')
 *   u +- c, shear t: (+-c at u_t, P_nn at P_nt, P_nt' (1 + [t' == t]) at P_tt')
 *   u: the unit vectors of rho, P_t1t1, P_t1t2, P_t2t2.
 * The left eigenvectors are the rows of R^-1. */
int orc3_eigen(int n, const double w[N3], double lam[N3], double R[N3][N3], double L[N3][N3])
{
    const int t1 = (n == 0) ? 1 : 0, t2 = (n == 2) ? 1 : 2;
    const int t[2] = {t1, t2};
    const double rho = w[R3], un = w[1 + n], pnn = w[pidx(n, n)];
    const double a = sqrt(3.0 * pnn / rho), c = sqrt(pnn / rho);
    double q[3] = {0, 0, 0};
    for (int s = 0; s < 2; ++s) q[t[s]] = w[pidx(n, t[s])] / pnn;
    memset(R, 0, sizeof(double) * N3 * N3);
    /* columns 0 and 9: u -+ a */
    for (int col = 0; col < 2; ++col) {
        const int cidx = col == 0 ? 0 : 9;
        const double sg = col == 0 ? -1.0 : 1.0;
        R[R3][cidx] = rho;
        R[1 + n][cidx] = sg * a;
        for (int s = 0; s < 2; ++s) R[1 + t[s]][cidx] = sg * a * q[t[s]];
        R[pidx(n, n)][cidx] = 3.0 * pnn;
        for (int s = 0; s < 2; ++s) R[pidx(n, t[s])][cidx] = 3.0 * w[pidx(n, t[s])];
        for (int s = 0; s < 2; ++s)
            for (int r = s; r < 2; ++r) {
                const int ts = t[s], tr = t[r];
                R[pidx(ts, tr)][cidx] = w[pidx(ts, tr)] + w[pidx(n, ts)] * q[tr] + w[pidx(n, tr)] * q[ts];
            }
        lam[cidx] = un + sg * a;
    }
    /* shear waves: columns 1, 2 (u - c) and 7, 8 (u + c) */
    for (int s = 0; s < 2; ++s)
        for (int sgn_i = 0; sgn_i < 2; ++sgn_i) {
            const int cidx = sgn_i == 0 ? 1 + s : 7 + s;
            const double sg = sgn_i == 0 ? -1.0 : 1.0;
            const int ts = t[s];
            R[1 + ts][cidx] = sg * c;
            R[pidx(n, ts)][cidx] = pnn;
            for (int r = 0; r < 2; ++r) {
                const int tr = t[r];
                R[pidx(ts, tr)][cidx] = (tr == ts) ? 2.0 * w[pidx(n, ts)] : w[pidx(n, tr)];
            }
            lam[cidx] = un + sg * c;
        }
    /* contacts: columns 3..6 */
    R[R3][3] = 1.0;
    R[pidx(t1, t1)][4] = 1.0;
    R[pidx(t1, t2)][5] = 1.0;
    R[pidx(t2, t2)][6] = 1.0;
    for (int cidx = 3; cidx <= 6; ++cidx) lam[cidx] = un;
    return invert((const double(*)[N3])R, L);
}

static void matvec3(const double M[N3][N3], const double x[N3], double y[N3])
{
    for (int i = 0; i < N3; ++i) {
        double s = 0.0;
        for (int k = 0; k < N3; ++k) s += M[i][k] * x[k];
        y[i] = s;
    }
}

/* Limited slope along axis n: eqs. (19)-(26) with the 10-wave system. */
void orc3_limited_slope(int n, const double wm[N3], const double w0[N3], const double wp[N3], double dwm[N3])
{
    double lam[N3], R[N3][N3], L[N3][N3];
    orc3_eigen(n, w0, lam, R, L);
    double dL[N3], dC[N3], dR[N3], aL[N3], aC[N3], aR[N3], am[N3];
    for (int m = 0; m < N3; ++m) {
        dL[m] = w0[m] - wm[m];
        dC[m] = (wp[m] - wm[m]) / 2.0;
        dR[m] = wp[m] - w0[m];
    }
    matvec3((const double(*)[N3])L, dL, aL);
    matvec3((const double(*)[N3])L, dC, aC);
    matvec3((const double(*)[N3])L, dR, aR);
    for (int k = 0; k < N3; ++k) am[k] = orc_mc(aL[k], aC[k], aR[k]);
    for (int m = 0; m < N3; ++m) {
        double s = 0.0;
        for (int k = 0; k < N3; ++k) s += am[k] * R[m][k];
        dwm[m] = s;
    }
}

/* Face states along axis n, eqs. (27)-(32) with readings R4, R5 (every wave
 * counted once, the HLL terms added). */
void orc3_trace(int n, const double w[N3], const double dwm[N3], double k, double w_lo[N3], double w_hi[N3])
{
    double lam[N3], R[N3][N3], L[N3][N3];
    orc3_eigen(n, w, lam, R, L);
    double lamM = lam[0], lam0 = lam[0];
    for (int a = 1; a < N3; ++a) {
        lamM = fmax(lamM, lam[a]);
        lam0 = fmin(lam0, lam[a]);
    }
    for (int m = 0; m < N3; ++m) {
        w_hi[m] = w[m] + (0.5 - k * fmax(lamM, 0.0)) * dwm[m];
        w_lo[m] = w[m] - (0.5 + k * fmin(lam0, 0.0)) * dwm[m];
    }
    for (int a = 0; a < N3; ++a) {
        double pa = 0.0;
        for (int m = 0; m < N3; ++m) pa += L[a][m] * dwm[m];
        if (lam[a] > 0.0) {
            for (int m = 0; m < N3; ++m) w_hi[m] += k * ((lamM - lam[a]) * pa) * R[m][a];
        } else {
            for (int m = 0; m < N3; ++m) w_hi[m] -= k * ((lam[a] - lamM) * pa) * R[m][a];
        }
        if (lam[a] < 0.0) {
            for (int m = 0; m < N3; ++m) w_lo[m] += k * ((lam0 - lam[a]) * pa) * R[m][a];
        } else {
            for (int m = 0; m < N3; ++m) w_lo[m] -= k * ((lam[a] - lam0) * pa) * R[m][a];
        }
    }
}

/* HLL flux along axis n with Davis speeds, a = sqrt(3 P_nn / rho). */
void orc3_hll(int n, const double wl[N3], const double wr[N3], double flux[N3])
{
    double Ul[N3], Ur[N3], Fl[N3], Fr[N3];
    orc3_cons(wl, Ul);
    orc3_cons(wr, Ur);
    orc3_flux(n, Ul, Fl);
    orc3_flux(n, Ur, Fr);
    const int ip = pidx(n, n);
    const double al = sqrt(3.0 * wl[ip] / wl[R3]), ar = sqrt(3.0 * wr[ip] / wr[R3]);
    const double sl = fmin(wl[1 + n] - al, wr[1 + n] - ar);
    const double sr = fmax(wl[1 + n] + al, wr[1 + n] + ar);
    if (sl >= 0.0) {
        for (int m = 0; m < N3; ++m) flux[m] = Fl[m];
    } else if (sr <= 0.0) {
        for (int m = 0; m < N3; ++m) flux[m] = Fr[m];
    } else {
        for (int m = 0; m < N3; ++m)
            flux[m] = (sr * Fl[m] - sl * Fr[m] + sl * sr * (Ur[m] - Ul[m])) / (sr - sl);
    }
}

/* ghost index maps: periodic wrap, or the nearest edge cell (zero gradient) */
static int map3(int i, int n, int bc)
{
    if (bc == ORC_BC_PERIODIC) return ((i % n) + n) % n;
    return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

static int grid3_ok(const orc_grid3 *g)
{
    for (int a = 0; a < 3; ++a) {
        if (g->n[a] < 1 || !(g->h[a] > 0.0)) return 0;
        if (g->bc[a] != ORC_BC_PERIODIC && g->bc[a] != ORC_BC_OUTFLOW) return 0;
    }
    return 1;
}

/*
 * One step for the box of cells [o0, o0 + b0) x [o1, o1 + b1) x [o2, o2 + b2):
 * primitive block with 2 ghost layers per side (index maps of the boundary
 * conditions), face states of the box and a one-cell ring, HLL fluxes of the
 * box's faces, unsplit update.  Uout: [10][b2][b1][b0] of the box.
 */
static void step3_box(const orc_grid3 *g, double dt, const double *U, const int o[3], const int b[3], double *Uout)
{
    const size_t ncell = (size_t)g->n[0] * g->n[1] * g->n[2];
    const int p[3] = {b[0] + 4, b[1] + 4, b[2] + 4};
    const size_t np = (size_t)p[0] * p[1] * p[2];
    double *Wp = malloc(np * N3 * sizeof(double));
    for (int kk = 0; kk < p[2]; ++kk)
        for (int jj = 0; jj < p[1]; ++jj)
            for (int ii = 0; ii < p[0]; ++ii) {
                const int gi = map3(o[0] + ii - 2, g->n[0], g->bc[0]);
                const int gj = map3(o[1] + jj - 2, g->n[1], g->bc[1]);
                const int gk = map3(o[2] + kk - 2, g->n[2], g->bc[2]);
                const size_t c = ((size_t)gk * g->n[1] + gj) * g->n[0] + gi;
                double Uc[N3];
                for (int m = 0; m < N3; ++m) Uc[m] = U[m * ncell + c];
                orc3_prim(Uc, Wp + (((size_t)kk * p[1] + jj) * p[0] + ii) * N3);
            }
#define WP3(i, j, k) (Wp + ((((size_t)(k) + 2) * p[1] + (size_t)(j) + 2) * p[0] + (size_t)(i) + 2) * N3)
    /* face states of the box and its ring: s[axis][lo/hi] */
    const int r[3] = {b[0] + 2, b[1] + 2, b[2] + 2};
    const size_t nr = (size_t)r[0] * r[1] * r[2];
    double *fs = malloc(nr * 6 * N3 * sizeof(double));
#define FS(i, j, k, ax, hi) (fs + (((((size_t)(k) + 1) * r[1] + (size_t)(j) + 1) * r[0] + (size_t)(i) + 1) * 6 + (ax) * 2 + (hi)) * N3)
    const double kf[3] = {dt / (2.0 * g->h[0]), dt / (2.0 * g->h[1]), dt / (2.0 * g->h[2])};
    for (int k = -1; k <= b[2]; ++k)
        for (int j = -1; j <= b[1]; ++j)
            for (int i = -1; i <= b[0]; ++i) {
                const double *w = WP3(i, j, k);
                double dw[3][N3], Adw[3][N3];
                const int step[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
                for (int ax = 0; ax < 3; ++ax) {
                    const double *wm = WP3(i - step[ax][0], j - step[ax][1], k - step[ax][2]);
                    const double *wp = WP3(i + step[ax][0], j + step[ax][1], k + step[ax][2]);
                    orc3_limited_slope(ax, wm, w, wp, dw[ax]);
                    double A[N3][N3];
                    orc3_jac(ax, w, A);
                    matvec3((const double(*)[N3])A, dw[ax], Adw[ax]);
                }
                for (int ax = 0; ax < 3; ++ax) {
                    double *lo = FS(i, j, k, ax, 0), *hi = FS(i, j, k, ax, 1);
                    orc3_trace(ax, w, dw[ax], kf[ax], lo, hi);
                    /* transverse predictor terms of the two other axes (T1) */
                    for (int o2 = 0; o2 < 3; ++o2) {
                        if (o2 == ax) continue;
                        for (int m = 0; m < N3; ++m) {
                            lo[m] -= kf[o2] * Adw[o2][m];
                            hi[m] -= kf[o2] * Adw[o2][m];
                        }
                    }
                }
            }
    /* fluxes and update */
    for (int k = 0; k < b[2]; ++k)
        for (int j = 0; j < b[1]; ++j)
            for (int i = 0; i < b[0]; ++i) {
                const int step[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
                double du[N3] = {0};
                for (int ax = 0; ax < 3; ++ax) {
                    double fm[N3], fp[N3];
                    const int di = step[ax][0], dj = step[ax][1], dk = step[ax][2];
                    orc3_hll(ax, FS(i - di, j - dj, k - dk, ax, 1), FS(i, j, k, ax, 0), fm);
                    orc3_hll(ax, FS(i, j, k, ax, 1), FS(i + di, j + dj, k + dk, ax, 0), fp);
                    const double cfac = dt / g->h[ax];
                    for (int m = 0; m < N3; ++m) du[m] -= cfac * (fp[m] - fm[m]);
                }
                const size_t gc = ((size_t)(o[2] + k) * g->n[1] + (o[1] + j)) * g->n[0] + (o[0] + i);
                const size_t bc = ((size_t)k * b[1] + j) * b[0] + i;
                const size_t nb = (size_t)b[0] * b[1] * b[2];
                for (int m = 0; m < N3; ++m) Uout[m * nb + bc] = U[m * ncell + gc] + du[m];
            }
#undef FS
#undef WP3
    free(fs);
    free(Wp);
}

/* One step of the whole grid, in boxes of full rows x 4 x 4 cells (bounded memory). */
int orc3_step(const orc_grid3 *g, double dt, const double *U, double *Unew)
{
    if (!grid3_ok(g)) return -1;
    const size_t ncell = (size_t)g->n[0] * g->n[1] * g->n[2], plane = (size_t)g->n[0] * g->n[1];
    const int e = 4, nby = (g->n[1] + e - 1) / e, nbz = (g->n[2] + e - 1) / e;
    #pragma omp parallel for schedule(dynamic, 1)
    for (int s = 0; s < nby * nbz; ++s) {
        const int o[3] = {0, (s % nby) * e, (s / nby) * e};
        const int b[3] = {g->n[0], o[1] + e <= g->n[1] ? e : g->n[1] - o[1], o[2] + e <= g->n[2] ? e : g->n[2] - o[2]};
        const size_t nb = (size_t)b[0] * b[1] * b[2];
        double *out = malloc(nb * N3 * sizeof(double));
        step3_box(g, dt, U, o, b, out);
        for (int k = 0; k < b[2]; ++k)
            for (int j = 0; j < b[1]; ++j)
                for (int i = 0; i < b[0]; ++i)
                    for (int m = 0; m < N3; ++m)
                        Unew[m * ncell + (size_t)(o[2] + k) * plane + (size_t)(o[1] + j) * g->n[0] + i] =
                            out[m * nb + ((size_t)k * b[1] + j) * b[0] + i];
        free(out);
    }
    return 0;
}

/* Updated conserved states of the listed cells (flat index (k ny + j) nx + i): out[ncells][10]. */
int orc3_step_cells(const orc_grid3 *g, double dt, const double *U, int64_t ncells, const int64_t *cells,
                    double *out)
{
    if (!grid3_ok(g)) return -1;
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t s = 0; s < ncells; ++s) {
        const int64_t c = cells[s];
        const int o[3] = {(int)(c % g->n[0]), (int)((c / g->n[0]) % g->n[1]), (int)(c / ((int64_t)g->n[0] * g->n[1]))};
        const int b[3] = {1, 1, 1};
        double u[N3];
        step3_box(g, dt, U, o, b, u);
        for (int m = 0; m < N3; ++m) out[s * N3 + m] = u[m];
    }
    return 0;
}

/* CFL rate (T2): max over cells of sum_k (|u_k| + sqrt(3 P_kk / rho)) / h_k. */
double orc3_max_signal_speed(const orc_grid3 *g, const double *U)
{
    const size_t ncell = (size_t)g->n[0] * g->n[1] * g->n[2];
    double smax = 0.0;
    #pragma omp parallel for reduction(max : smax) schedule(static)
    for (int64_t c = 0; c < (int64_t)ncell; ++c) {
        double Uc[N3], w[N3];
        for (int m = 0; m < N3; ++m) Uc[m] = U[m * ncell + c];
        orc3_prim(Uc, w);
        double s = 0.0;
        for (int k = 0; k < 3; ++k) s += (fabs(w[1 + k]) + sqrt(3.0 * w[pidx(k, k)] / w[R3])) / g->h[k];
        smax = fmax(smax, s);
    }
    return smax;
}
