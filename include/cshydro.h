/*
 * cshydro -- collisionless stellar hydrodynamics on AMD Instinct MI355X (gfx950).
 *
 * C ABI of the Godunov sweep for the Boltzmann moment equations (BME) of
 * Mitchell, Vorobyov & Hensler, "Collisionless Stellar Hydrodynamics as an
 * Efficient Alternative to N-body Methods" (arXiv:1210.5246):
 *   continuity, momentum and second-moment equations, Sec. 2, eqs. (2)-(4),
 *   closed with zero heat flux (Q_ijk = 0), advanced by the MUSCL-Hancock
 *   scheme with characteristic tracing and an HLL Riemann flux of Sec. 3.3,
 *   eqs. (10)-(32), on a uniform 1-D or 2-D grid, with the full symmetric 2-D
 *   stress tensor.
 *
 * Conventions for every entry point:
 *   - All state arrays are DEVICE pointers owned by the caller, structure of
 *     arrays [6][ny][nx] with x fastest (1-D: ny = 1), contiguous, element type
 *     double (CSH_F64) or float (CSH_F32) as chosen at init.
 *       conserved U = (rho, rho u, rho v, Exx, Exy, Eyy), E_ij = P_ij + rho u_i u_j
 *       primitive W = (rho, u, v, Pxx, Pxy, Pyy), P_ij = rho sigma^2_ij (Sec. 2)
 *   - Work is enqueued on the HIP stream given at init and is asynchronous
 *     unless a function says it synchronises.
 *   - Return value: CSH_OK (0) or a negative CSH_ERR_* code; csh_last_error()
 *     returns a message for the calling thread's last error.  No C++ exception
 *     crosses this interface.
 *   - A handle is not thread-safe; distinct handles are independent.
 *   - Launch shape: each 2-D sweep kernel marches a wavefront over a segment
 *     of rows whose length the library chooses from the grid size; the 3-D
 *     sweep runs one workgroup of four wavefronts per compute unit, each
 *     marching along z through an equal share of the grid's planes.
 *     Environment variables, for tuning only, override these choices (a
 *     positive integer; anything else is ignored); results agree to rounding
 *     for any value:
 *       CSH_ROWS     rows per segment of the characteristic sweeps, read when
 *                    a 2-D handle is created;
 *       CSH_KT_ROWS  rows per segment of the Kurganov-Tadmor step, read at
 *                    every 2-D launch (a recorded graph keeps the value it
 *                    was recorded with);
 *       CSH_PLANES   the most planes the 3-D sweep marches in one piece;
 *       CSH_WG3      workgroups of the 3-D sweep;
 *     the last two are read at every csh3_step and whenever csh3_run_cfl
 *     records its graph (a recorded graph keeps the values it was recorded
 *     with).
 */
#ifndef CSHYDRO_H
#define CSHYDRO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CSH_OK 0
#define CSH_ERR_ARG (-1)         /* invalid argument (sizes, pointers, enum values)  */
#define CSH_ERR_HIP (-2)         /* a HIP runtime call failed                         */
#define CSH_ERR_NONPHYSICAL (-3) /* a state with rho <= 0, non-positive-definite stress or a
                                    non-finite value was produced or supplied            */

#define CSH_BC_PERIODIC 0 /* wrap-around ghost cells                                */
#define CSH_BC_OUTFLOW 1  /* zero-gradient ghost cells (copy of the edge cell)      */

#define CSH_F64 0
#define CSH_F32 1

#define CSH_SCHEME_MUSCL_HLL 0 /* MUSCL-Hancock, characteristic tracing, HLL (Sec. 3.3) -- default */
#define CSH_SCHEME_KT 1        /* Kurganov-Tadmor central scheme, RK2 midpoint (Sec. 3.2)          */
#define CSH_SCHEME_MUSCL_HLLC 2 /* the characteristic sweep with the HLLC flux of the paper's runs    */

typedef struct csh_grid csh_grid;
typedef struct csh_batch csh_batch;

const char *csh_last_error(void);

/*
 * Create a grid handle and convert primitive to conserved state.
 * nx >= 1, ny >= 1 (ny == 1: one-dimensional scheme, no y terms), one plane
 * (nx ny elements) smaller than 4 GiB; dx, dy > 0
 * (dy unused in 1-D); bc_x, bc_y: CSH_BC_*; dtype: CSH_F64 or CSH_F32.
 * W: device, primitive fields [6][ny][nx], read only.  U: device, receives the
 * conserved state [6][ny][nx] (the definitions of Sec. 2).  stream: a
 * hipStream_t (NULL: the null stream).  Synchronises; returns
 * CSH_ERR_NONPHYSICAL (handle still created) if some cell of W has rho <= 0,
 * Pxx <= 0, Pyy <= 0, Pxx Pyy - Pxy^2 <= 0 or a non-finite value.
 * The handle owns small device scalars (and, once csh_adjoint_step is used,
 * the adjoint workspace); free it with csh_destroy.
 */
int csh_init_state(csh_grid **h, int nx, int ny, double dx, double dy, int bc_x, int bc_y,
                   int dtype, const void *W, void *U, void *stream);

/*
 * Convert primitive fields W into conserved state U on an existing handle
 * (the conversion and validation of csh_init_state; clears the handle's
 * non-physical flag first).  W, U: device [6][ny][nx] of the handle's dtype.
 * Synchronises.
 */
int csh_set_state(csh_grid *h, const void *W, void *U);

/*
 * Select the scheme csh_step, csh_run_cfl and csh_run_dts use:
 *   CSH_SCHEME_MUSCL_HLL (default): the characteristic MUSCL-Hancock sweep with
 *     HLL fluxes of Sec. 3.3;
 *   CSH_SCHEME_MUSCL_HLLC: the same sweep with an HLLC flux (the solver of the
 *     paper's runs, Sec. 4.1; the paper gives no BME form): Davis outer speeds,
 *     contact S* = (Pnn_R - Pnn_L + D_L u_L - D_R u_R) / (D_L - D_R),
 *     D_K = rho_K (S_K - u_K), one star velocity (S*, v*) and one pair of
 *     normal stresses (Pnn*, Pnt*) on both sides of the contact, each star
 *     density from the jump condition across its outer wave; isolated
 *     contacts are kept exactly;
 *   CSH_SCHEME_KT: the Kurganov-Tadmor central scheme of Sec. 3.2, eqs. (5)-(8):
 *     local-speed flux H = (F(u-) + F(u+))/2 - a/2 (u+ - u-), a = max |u_n| +
 *     sqrt(3 P_nn / rho) over the two face states, faces reconstructed by
 *     component-wise MC-limited linear primitive profiles, two stages of the
 *     Runge-Kutta midpoint rule per step, then the kick.  On a 2-D grid both
 *     stages run in one launch (the intermediate state is never stored); on a
 *     1-D grid two launches, and the first call allocates one state-sized
 *     stage buffer the handle keeps.
 * csh_fluxes returns the faces of either characteristic sweep and CSH_ERR_ARG
 * under CSH_SCHEME_KT; csh_adjoint_step is that of CSH_SCHEME_MUSCL_HLL and
 * returns CSH_ERR_ARG under the other schemes.  Synchronises.
 */
int csh_set_scheme(csh_grid *h, int scheme);

#define CSH_FOURIER_MAX_M 16

/*
 * Global Fourier amplitudes of the surface density, the spiral-growth
 * diagnostic of Sec. 4.4:
 *   A_m = | sum over cells centred in [-X, X] x [-Y, Y] of rho exp(i m phi) |
 *         / sum over all cells of rho ,   m = 1 .. m_max,
 * with phi the polar angle (all four quadrants) of the cell centre
 * (x0 + (i + 1/2) dx, y0 + (j + 1/2) dy) (the same corner convention as
 * csh_set_potential; each coordinate a product and a sum rounded separately)
 * and rho the density plane of U.  A cell centred exactly on the origin has
 * no angle and is left out of the numerator.
 * U: device state [6][ny][nx] in the handle's dtype (only the density plane is
 * read).  A: host array of m_max doubles.  1 <= m_max <= CSH_FOURIER_MAX_M,
 * X, Y > 0 (pass HUGE_VAL for the whole grid).  2-D handles only.  The sums
 * are formed in a fixed order (deterministic).  The first call allocates a
 * 270 KB workspace the handle keeps.  Synchronises the handle's stream.
 * Errors: CSH_ERR_ARG, CSH_ERR_HIP.
 */
int csh_fourier_amplitudes(csh_grid *h, const void *U, double x0, double y0, double X, double Y, int m_max,
                           double *A);

/*
 * For callers that cannot allocate device memory (code under stream or graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * amplitudes as csh_fourier_amplitudes, computed by the same kernels, with no
 * allocation, no host copy and no synchronisation.
 * The partial sums live in a statically sized device array of the library
 * (CSH_FOURIER_MAX_M and 1024 partial rows: 1024 x 33 doubles, 264 KiB),
 * one per GPU, held until the process ends; its address on the current device
 * is looked up on the first call on that device (no allocation).
 * A_dev: caller-owned DEVICE array of m_max doubles, written in stream order
 * on the handle's stream (read it after that stream has reached this call).
 * Arguments otherwise as csh_fourier_amplitudes; m_max > CSH_FOURIER_MAX_M is
 * rejected (the array's limit).  Every call on one GPU shares that GPU's
 * array: calls that overlap in time on one GPU (other streams, other threads)
 * race and must be serialised by the caller.  Nothing in the array needs
 * clearing: each call writes every partial sum it reads.
 * Errors: CSH_ERR_ARG, CSH_ERR_HIP.
 */
int csh_fourier_amplitudes_noalloc(csh_grid *h, const void *U, double x0, double y0, double X, double Y,
                                   int m_max, double *A_dev);

/*
 * Fixed external potential of a flat rotation curve, Phi = vc^2/2 ln(R^2 + rc^2)
 * centred on the coordinate origin (the analytic stand-in for the halo of
 * Sec. 4.4), applied after every step as an exact operator-split kick
 * u_i += dt a_i with a = -grad Phi, rho and P unchanged (Sec. 3.3, last
 * paragraph).  (x0, y0) are the coordinates of the grid's lower-left corner:
 * cell (i, j) is centred at (x0 + (i + 1/2) dx, y0 + (j + 1/2) dy) (1-D: y = 0).
 * vc == 0 switches the source off.
 */
int csh_set_potential(csh_grid *h, double vc, double rc, double x0, double y0);

/*
 * One sweep U -> U_new with timestep dt (host value): slopes, characteristic
 * limiting and tracing, HLL flux at every face, the unsplit conservative update
 * (Sec. 3.3, eqs. (19)-(32)) and the source kick if set.  U and U_new are
 * distinct device buffers [6][ny][nx].  Also reduces the CFL rate of U_new on
 * the device (read it with csh_last_signal_speed).  Asynchronous: a
 * non-physical output is reported by the next synchronising call.
 */
int csh_step(csh_grid *h, double dt, const void *U, void *U_new);

/*
 * s = max over cells of (|u| + a_x)/dx + (|v| + a_y)/dy (1-D: (|u| + a_x)/dx),
 * a_d = sqrt(3 P_dd / rho) (Sec. 3.2, eq. (8) with gamma = 3); the CFL
 * timestep is C / s.  Reads U, synchronises, writes *s (host).
 * Returns CSH_ERR_NONPHYSICAL if a cell of U, or an output of an earlier
 * asynchronous call on this handle, was not physical.
 */
int csh_max_signal_speed(csh_grid *h, const void *U, double *s);

/* s of the output of the last csh_step / csh_run_cfl (fused reduction, no pass
 * over the state).  Synchronises; errors as csh_max_signal_speed. */
int csh_last_signal_speed(csh_grid *h, double *s);

/*
 * The HLL face fluxes of the sweep of U with timestep dt (the time-centred
 * fluxes the update of csh_step uses; no source term).  Fx: device
 * [6][ny][nx+1], column i holds face i-1/2; Fy: device [6][ny+1][nx], row j
 * holds face j-1/2 (ignored in 1-D, may be NULL).  Asynchronous.
 */
int csh_fluxes(csh_grid *h, double dt, const void *U, void *Fx, void *Fy);

/*
 * Advance nsteps steps with the timestep chosen on the device every step:
 * dt_n = C / s_n (C = cfl, s_n the rate of the state at the start of the step),
 * clipped so that the time, starting from 0 at this call, does not pass t_end
 * (t_end <= 0: no clipping; steps after t_end is reached have dt = 0 and leave
 * the state unchanged).  U: device state, updated in place on return (the
 * steps alternate between U and U_work, a caller-owned device buffer of the
 * same size).  dt_log: device array of nsteps doubles receiving each step's
 * timestep, or NULL.  No host synchronisation between steps; the sequence is
 * captured once as a HIP graph per (nsteps, buffers, cfl, t_end) and replayed.
 */
int csh_run_cfl(csh_grid *h, int nsteps, double cfl, double t_end, void *U, void *U_work,
                double *dt_log);

/*
 * nsteps steps as csh_run_cfl (t_end none), keeping every state: states is a
 * caller-owned device array [nsteps][6][ny][nx] of the handle's dtype (nsteps
 * times the state size), and states[k] receives the state after step k + 1;
 * the first step reads U0 (device, read only, not inside states).  dt_log:
 * as for csh_run_cfl.  The states are bitwise those csh_run_cfl passes
 * through.  For reverse passes that keep the whole trajectory in memory (a
 * 512 x 512 FP64 run of 200 steps is 2.5 GB).  The steps are launched on the
 * handle's stream directly (no graph: the state array is usually new at every
 * call); asynchronous.
 */
int csh_run_cfl_states(csh_grid *h, int nsteps, double cfl, const void *U0, void *states, double *dt_log);

/*
 * Advance nsteps steps with given timesteps: step k uses dts[k] (device array
 * of nsteps doubles, read when the step runs).  U is updated in place (U_work
 * as for csh_run_cfl); captured once as a HIP graph per (nsteps, buffers, dts)
 * and replayed.  Replays a recorded run exactly (the timesteps of csh_run_cfl's
 * dt_log reproduce its states bit for bit).
 */
int csh_run_dts(csh_grid *h, int nsteps, const double *dts, void *U, void *U_work);

/*
 * Adjoint of one sweep at frozen timestep dt:
 *   lam = (d step_dt(U) / d U)^T lam_next,
 * the exact transpose of the linearisation of csh_step about U (limiter and
 * HLL branches fixed at U; at ties the subgradient of the first minimal
 * argument), external kick included.  U, lam_next: device, read only;
 * lam: device output; all [6][ny][nx] of the handle's dtype (CSH_F64 only).
 * Does not touch the handle's CFL state.  The first call allocates a workspace
 * of 66 (nx + 2)(ny + 2) + 6 (nx + 4)(ny + 2) doubles (1-D: 66 (nx + 2) +
 * 6 (nx + 4)) that the handle keeps until csh_destroy.  Asynchronous.
 */
int csh_adjoint_step(csh_grid *h, double dt, const void *U, const void *lam_next, void *lam);

/*
 * Transpose of the primitive-to-conserved map of csh_init_state (Sec. 2:
 * U = (rho, rho u, rho v, Pxx + rho u^2, Pxy + rho u v, Pyy + rho v^2)) at W:
 * lam_W = (dU/dW)^T lam_U, to carry a gradient with respect to the initial
 * conserved state back to the primitive fields (density, velocity, stress).
 * W, lam_U: device, read; lam_W: device output; [6][ny][nx] FP64.  Asynchronous.
 */
int csh_init_state_adjoint(csh_grid *h, const void *W, const void *lam_U, void *lam_W);

/* Release the handle (synchronises its stream first). */
int csh_destroy(csh_grid *h);

/* ---- many independent 1-D problems of uneven length, one launch ---------------------------- */

/*
 * ntubes independent 1-D tubes, tube k on cells offsets[k] .. offsets[k+1]-1
 * of concatenated SoA arrays [6][offsets[ntubes]]; each tube spans [0, 1]
 * (dx = 1 / its length) with outflow ends.  offsets: HOST array of ntubes + 1
 * nondecreasing values, offsets[0] = 0, every length >= 1.
 * W: device primitive fields, read; U: device, receives the conserved state.
 * dtype: CSH_F64.  Synchronises; errors as csh_init_state.
 */
int csh_batch_init(csh_batch **b, int ntubes, const int64_t *offsets, int dtype, const void *W,
                   void *U, void *stream);

/*
 * Advance every tube nsteps steps, each with its own CFL timestep
 * dt = cfl / s_k recomputed on the device after every step, in one persistent
 * launch (workgroups take whole tubes, longest first, from a device queue;
 * replayed from a captured HIP graph).  U is updated in place (U_work: caller
 * buffer of the same size).  dt_out: device array [ntubes][nsteps] of the
 * timesteps taken, or NULL.  threads: workgroup size (64, 128, 256, 512 or
 * 1024), or 0 for the size chosen by csh_batch_autotune (256 if never tuned).
 */
int csh_batch_run(csh_batch *b, int nsteps, double cfl, void *U, void *U_work, double *dt_out,
                  int threads);

/*
 * Synchronises the batch's stream and reports whether any state a step of an
 * earlier csh_batch_run produced was not physical (rho <= 0, stress not
 * positive-definite, or non-finite): CSH_ERR_NONPHYSICAL, else CSH_OK.
 * csh_batch_run is asynchronous and checks every new state on the device; the
 * flag stays set for the life of the batch (as the non-physical flag of a
 * grid handle until csh_set_state).
 */
int csh_batch_status(csh_batch *b);

/*
 * Time the candidate workgroup sizes on this device for this batch (a few
 * steps each, on scratch copies of U; U is not modified), keep the fastest
 * as the batch's default and write it to *best_threads.  Synchronises.
 * The choice is persisted: one line "<key> <threads>" per batch shape in the
 * file CSH_TUNE_CACHE names (the value "off" disables it; default
 * $HOME/.cache/cshydro/batch_autotune.txt), with key
 * "arch=<gcnArchName>;cus=<compute units>;tubes=<ntubes>;cells=<total cells>;maxlen=<longest tube>";
 * a later call for the same shape on the same kind of device takes the
 * recorded size without probing (the last record of a key wins).
 */
int csh_batch_autotune(csh_batch *b, int probe_steps, double cfl, const void *U, int *best_threads);

int csh_batch_destroy(csh_batch *b);

/* ======================================================================
 * Three dimensions: the ten-moment system (Sec. 2, eqs. (2)-(4) in three
 * dimensions; ten eigenvalues, Sec. 3.3), FP64, HLL, no external potential.
 * U = (rho, rho u, rho v, rho w, Exx, Exy, Exz, Eyy, Eyz, Ezz) and
 * W = (rho, u, v, w, Pxx, Pxy, Pxz, Pyy, Pyz, Pzz), device arrays
 * [10][nz][ny][nx] (x fastest).  The scheme is the characteristic sweep of
 * Sec. 3.3 along all three axes: MC slopes of the ten wave amplitudes, the
 * Hancock predictor with the transverse terms of both other axes, HLL fluxes
 * with Davis speeds, the unsplit update; timestep C / max over cells of
 * sum_k (|u_k| + sqrt(3 P_kk / rho)) / h_k.
 * ====================================================================== */
typedef struct csh3_grid csh3_grid;

/* Message of the last failed csh3_* call on this thread. */
const char *csh3_last_error(void);

/*
 * Create a 3-D handle and convert W to U (one component, nx ny nz doubles,
 * smaller than 4 GiB; validation as csh_init_state:
 * rho > 0 and a positive-definite stress, else CSH_ERR_NONPHYSICAL with the
 * handle still returned).  A step needs no workspace: the handle holds only
 * its timestep slots and error flag.  stream: the HIP stream all work of the
 * handle runs on (NULL: the null stream), on the device current at this
 * call, whose compute-unit count the handle records (the sweep runs one
 * workgroup per compute unit).
 */
int csh3_init_state(csh3_grid **h, int nx, int ny, int nz, double dx, double dy, double dz, int bc_x, int bc_y,
                    int bc_z, const void *W, void *U, void *stream);

/* One step with a host timestep: U -> U_new (distinct buffers).  Synchronises;
 * CSH_ERR_NONPHYSICAL if the new state is not physical. */
int csh3_step(csh3_grid *h, double dt, const void *U, void *U_new);

/* Largest CFL rate of U (dt = C / s).  Synchronises. */
int csh3_max_signal_speed(csh3_grid *h, const void *U, double *s);

/* The CFL rate of the output of the last step, reduced inside that step. */
int csh3_last_signal_speed(csh3_grid *h, double *s);

/* nsteps steps with dt = cfl / s chosen on the device from each step's input,
 * replayed from a captured HIP graph (recorded once per argument set).  U is
 * advanced in place, U_work is scratch of the same size, dt_log (device,
 * nsteps doubles) receives the timesteps.  Synchronises. */
int csh3_run_cfl(csh3_grid *h, int nsteps, double cfl, void *U, void *U_work, double *dt_log);

/* Free the handle (NULL is ignored). */
void csh3_destroy(csh3_grid *h);

#ifdef __cplusplus
}
#endif

#endif /* CSHYDRO_H */
