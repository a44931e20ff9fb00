/*
 * FP64 CPU oracle for the collisionless-stellar-hydrodynamics sweep.
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the
 * CPU-baseline leg of the benchmark, never by the product path.
 *
 * Arrays at this interface are structure-of-arrays, [6][ny][nx], x fastest,
 * in the variable order
 *   conserved U = (rho, rho u, rho v, Exx, Exy, Eyy),  E_ij = P_ij + rho u_i u_j
 *   primitive W = (rho, u, v, Pxx, Pxy, Pyy).
 * ny == 1 selects the one-dimensional scheme (no y terms at all).
 */
#ifndef CSHORACLE_H
#define CSHORACLE_H

#include <stdint.h>

#define ORC_BC_PERIODIC 0
#define ORC_BC_OUTFLOW 1

typedef struct {
    int nx, ny;
    double dx, dy;
    int bcx, bcy;
    double x0, y0; /* lower-left domain corner; cell centre x0 + (i + 1/2) dx */
    double vc, rc; /* external flat-rotation-curve potential; vc == 0: none */
} orc_grid;

void orc_cons(const double w[6], double U[6]);
void orc_prim(const double U[6], double w[6]);
void orc_flux_x(const double U[6], double F[6]);
void orc_flux_y(const double U[6], double G[6]);
void orc_jac_x(const double w[6], double A[6][6]);
void orc_jac_y(const double w[6], double B[6][6]);
void orc_eigen_x(const double w[6], double lam[6], double R[6][6], double L[6][6]);
void orc_eigen_y(const double w[6], double lam[6], double R[6][6], double L[6][6]);
double orc_mc(double dl, double dc, double dr);
void orc_limited_slope(int dir, const double wm[6], const double w0[6], const double wp[6],
                       double dwm[6]);
void orc_trace(int dir, const double w[6], const double dwm[6], double k, double w_lo[6],
               double w_hi[6]);
void orc_hll(int dir, const double wl[6], const double wr[6], double flux[6]);

/* One step U -> Unew (may not alias), timestep dt.  Returns 0, or -1 on a bad grid. */
int orc_step(const orc_grid *g, double dt, const double *U, double *Unew);

/* Riemann solver of the characteristic scheme (the plain entry points use HLL). */
#define ORC_SOLVER_HLL 0
#define ORC_SOLVER_HLLC 1
void orc_hllc(int dir, const double wl[6], const double wr[6], double flux[6]);
void orc_hllc_star(int dir, const double wl[6], const double wr[6], double speeds[3], double UsL[6],
                   double UsR[6]);
int orc_step_rs(const orc_grid *g, int solver, double dt, const double *U, double *Unew);
int orc_step_cells_rs(const orc_grid *g, int solver, double dt, const double *U, int64_t ncells,
                      const int64_t *cells, double *out);
int orc_fluxes_rs(const orc_grid *g, int solver, double dt, const double *U, double *Fx, double *Fy);
/* The step for selected cells only: cells[s] = j * nx + i, out[s][6] (cell-major). */
int orc_step_cells(const orc_grid *g, double dt, const double *U, int64_t ncells,
                   const int64_t *cells, double *out);
/* Face fluxes of the step: Fx [6][ny][nx+1] (column i = face i-1/2),
 * Fy [6][ny+1][nx] (row j = face j-1/2); Fy unused in 1-D. */
int orc_fluxes(const orc_grid *g, double dt, const double *U, double *Fx, double *Fy);
double orc_max_signal_speed(const orc_grid *g, const double *U);
int orc_physical(const orc_grid *g, const double *U);
/* Branch pattern of one step (the side of every kink each decision takes);
 * orc_branch_count gives the number of codes.  Limiter codes: */
#define ORC_MC_OFF 0
#define ORC_MC_CENTRED 1
#define ORC_MC_LEFT 2
#define ORC_MC_RIGHT 3
int64_t orc_branch_count(const orc_grid *g);
int orc_branches(const orc_grid *g, double dt, const double *U, int *codes);
/* Whole-field conversions, SoA [6][n]. */
void orc_cons_field(int64_t n, const double *W, double *U);
void orc_prim_field(int64_t n, const double *U, double *W);
int orc_num_threads(void);
void orc_set_num_threads(int n);

/* Kurganov-Tadmor central scheme: numerical flux of eq. (6) and one step. */
void orc_kt_flux(int dir, const double wl[6], const double wr[6], double flux[6]);
int orc_step_kt(const orc_grid *g, double dt, const double *U, double *Unew);

/* Global Fourier amplitudes A_1..A_mmax of the density (Sec. 4.4); region [-X, X] x [-Y, Y]. */
int orc_fourier_amplitudes(const orc_grid *g, const double *U, int mmax, double X, double Y, double *A);

/* ---- three dimensions (cshoracle3.c): ten-moment system, HLL ---- */
typedef struct {
    int n[3];      /* cells along x, y, z */
    double h[3];   /* cell sizes */
    int bc[3];     /* ORC_BC_PERIODIC / ORC_BC_OUTFLOW per axis */
} orc_grid3;

void orc3_cons(const double w[10], double U[10]);
void orc3_prim(const double U[10], double w[10]);
void orc3_flux(int k, const double U[10], double F[10]);
void orc3_jac(int k, const double w[10], double A[10][10]);
int orc3_eigen(int n, const double w[10], double lam[10], double R[10][10], double L[10][10]);
void orc3_limited_slope(int n, const double wm[10], const double w0[10], const double wp[10], double dwm[10]);
void orc3_trace(int n, const double w[10], const double dwm[10], double k, double w_lo[10], double w_hi[10]);
void orc3_hll(int n, const double wl[10], const double wr[10], double flux[10]);
int orc3_step(const orc_grid3 *g, double dt, const double *U, double *Unew);
int orc3_step_cells(const orc_grid3 *g, double dt, const double *U, int64_t ncells, const int64_t *cells,
                    double *out);
double orc3_max_signal_speed(const orc_grid3 *g, const double *U);

#endif
