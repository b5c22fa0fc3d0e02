/*
 * ctu_oracle.h -- CPU oracle for one unsplit CTU timestep of the 3D Euler equations
 * (PPMC reconstruction with characteristic tracing + exact Riemann solver).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU library against the
 * paper (Schneider & Robertson, "Cholla", arXiv:1410.4194).  Only the test suite, the smoke
 * check and the CPU-baseline leg of the benchmark load it.  The GPU product path never links,
 * loads or calls it, and it shares no source, header, table or helper with the GPU library.
 *
 * Plain, serial, double precision C, built with -O2 -ffp-contract=off (no FMA contraction).
 * Every function follows the algorithm steps in the order the paper states them; where the
 * printed equations are garbled the reading taken is stated beside the code.
 *
 * Parity status: every function here is pinned by tests against closed forms, conservation
 * laws, jump conditions, invariants or brute force (see tests/test_oracle_*.py).
 *
 * Layout: conserved state is structure-of-arrays, 5 fields (rho, rho*u, rho*v, rho*w, E),
 * each over the allocated box (nx+2g)(ny+2g)(nz+2g) with x fastest, g = ref_ghost_width();
 * real cell (i,j,k), 0 <= i < nx, sits at (i+g) + NX*((j+g) + NY*(k+g)), NX = nx+2g,
 * NY = ny+2g.  g = 3 for PPMC: its stencil reaches two cells to each side and the CTU
 * transverse correction one more.
 */
#ifndef CTU_ORACLE_H
#define CTU_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

#define REF_BC_PERIODIC 0
#define REF_BC_OUTFLOW 1
#define REF_BC_REFLECT 2
#define REF_RIEMANN_EXACT 0 /* exact solver, Newton star pressure (App. B.1) */
#define REF_RIEMANN_ROE 1   /* Roe solver with the HLLE failsafe (App. B.2) */
#define REF_RECON_PPMC 0    /* PPM with characteristic limiting and tracing (App. A.3) */
#define REF_RECON_PPMP 1    /* PPM in the primitive variables, CW84 (App. A.4) */

typedef struct {
  int nx, ny, nz;          /* real cells per axis, >= 1 */
  double dx, dy, dz;       /* cell widths */
  double gamma;            /* ratio of specific heats */
  int bc[6];               /* x-, x+, y-, y+, z-, z+ : REF_BC_* */
  double cfl;              /* Courant number C0 */
  double newton_tol;       /* relative tolerance on the star-pressure change */
  int newton_max_iter;     /* iteration cap of the Newton loop */
  double p_floor;          /* pressure floor applied on every primitive conversion */
  int riemann;             /* REF_RIEMANN_* */
  int h_correction;        /* 1: H correction of the second-stage Roe fluxes (App. C) */
  int recon;               /* REF_RECON_* */
} ref_config;

/* Ghost layers of the state arrays: 3 for PPMC (stencil of two cells plus one for the
 * transverse correction), 4 when PPMP (three-cell stencil) or the H correction (which reads
 * second-stage states one cell beyond the boundary) is used. */
int ref_ghost_width(const ref_config* c);

typedef struct {
  long solves;             /* Riemann problems solved */
  long newton_iters;       /* Newton iterations summed over all solves */
  long newton_capped;      /* solves that hit newton_max_iter without converging */
  long p_floored;          /* primitive conversions whose pressure was raised to p_floor */
  long hlle;               /* Roe solves that fell back to the HLLE flux */
} ref_stats;

/* --- pointwise pieces (exposed for the pin tests) ------------------------------------ */

/* Conserved (rho, m1, m2, m3, E) -> primitive (rho, v1, v2, v3, p) with p >= p_floor.
 * Returns 1 when the floor was applied, else 0.  Ideal-gas EOS p = (gamma-1) rho e. */
int ref_cons_to_prim(const double U[5], double gamma, double p_floor, double W[5]);
void ref_prim_to_cons(const double W[5], double gamma, double U[5]);

/* Projection of a primitive difference d = (drho, du, dv, dw, dp) onto the characteristic
 * variables of a cell with density rho and sound speed a, and back. */
void ref_char_project(const double d[5], double rho, double a, double xi[5]);
void ref_char_unproject(const double xi[5], double rho, double a, double d[5]);

/* Monotonized-central limited slope of cell c from the characteristic differences
 * (the PLMC slope step that PPMC applies to cells c-1, c, c+1).  w_m, w_0, w_p are the
 * rotated primitives (rho, normal v, two transverse v, p) of cells c-1, c, c+1. */
void ref_plmc_slope(const double wm[5], const double w0[5], const double wp[5], double gamma,
                    double dw[5]);

/* PPMC: given rotated primitives of cells c-2..c+2 (w[0]..w[4]) and dtodx = dt/dx along
 * the sweep, return the time-evolved face states W*_L (left face of cell c) and W*_R
 * (right face of cell c), in rotated primitives.  If WLR_out is not NULL it receives the
 * monotonized face values before tracing: WLR_out[0..4] = W_L, WLR_out[5..9] = W_R. */
void ref_ppmc(const double w[5][5], double dtodx, double gamma, double WsL[5], double WsR[5],
              double* WLR_out);

/* PPMP (App. A.4): given rotated primitives of cells c-3..c+3 (w[0]..w[6]), dtodx = dt/dx
 * and the cell width dx along the sweep, return the traced face states W*_L, W*_R of cell
 * c.  WLR_out as for ref_ppmc (after steepening, flattening and the monotonicity fixes). */
void ref_ppmp(const double w[7][5], double dtodx, double dx, double gamma, double WsL[5],
              double WsR[5], double* WLR_out);

/* The two PPMP coefficients of cell c (slot 3 of w[7][5]): the shock-flattening F_c and the
 * contact-steepening eta_c, both in [0, 1]. */
double ref_ppmp_flattening(const double w[7][5]);
double ref_ppmp_steepening(const double w[7][5], double gamma, double dx);

/* Exact Riemann problem, star region: left (rho, u, p), right (rho, u, p).
 * Returns the Newton iteration count; *capped = 1 if the cap was reached. */
int ref_riemann_star(const double WL[3], const double WR[3], double gamma, double tol,
                     int max_iter, double p_floor, double* pstar, double* ustar, int* capped);

/* Exact Riemann solution sampled at similarity coordinate S = x/t.  The solver itself
 * samples at S = 0; other S serve the exact-solution checks.  out = (rho, u, p).
 * Returns 0 when the sample lies left of the contact, 1 when right. */
int ref_riemann_sample(const double WL[3], const double WR[3], double pstar, double ustar,
                       double gamma, double S, double out[3]);

/* Wave speeds of the exact solution: out[0..4] = left wave head, left wave tail (equal to
 * the shock speed for a shock), contact, right wave tail, right wave head. */
void ref_riemann_wave_speeds(const double WL[3], const double WR[3], double pstar,
                             double ustar, double gamma, double out[5]);

/* Exact-solver interface flux from rotated conserved states UL, UR (normal momentum in
 * slot 1).  F is in the same rotated order. */
void ref_riemann_flux(const double UL[5], const double UR[5], double gamma, double tol,
                      int max_iter, double p_floor, double F[5], ref_stats* st);

/* Roe flux (App. B.2) from rotated conserved states UL, UR (taken through their primitive
 * form with the pressure floor, as the solver starts from primitives), with the HLLE flux substituted
 * when an intermediate Roe state has a non-positive density or pressure.  eta_h is the
 * H-correction speed (App. C; 0 for none).  Returns 1 when HLLE was used, else 0. */
int ref_roe_flux(const double UL[5], const double UR[5], double gamma, double p_floor,
                 double eta_h, double F[5], ref_stats* st);

/* --- whole-grid operations ----------------------------------------------------------- */

/* Ghost fill: x faces, then y, then z, each over the full extent of the other two axes
 * (ghosts included), so edge and corner ghosts end up consistent.  Periodic ghosts copy the
 * real cell one period away, outflow ghosts the edge cell, reflecting ghosts their mirror
 * image across the wall with the wall-normal momentum negated (needs as many cells on the
 * axis as there are ghost layers; returns -1 without filling otherwise). */
int ref_bc_fill(const ref_config* c, double* const u[5]);

/* CFL time step over the real cells: C0 * min(dx/(|u|+a), dy/(|v|+a), dz/(|w|+a)). */
double ref_compute_dt(const ref_config* c, double* const u[5]);

/* u^{n+1} for the real cells of the box [lo, hi) (per-axis, real-cell coordinates) from a
 * ghost-filled state u (not modified).  out[q] are compact arrays of the box, x fastest.
 * Optional debug outputs (NULL to skip), each an array of 3*5 pointers (dir-major) to
 * arrays over the allocated box, face i+1/2 stored at cell i:
 *   fstar: first-stage fluxes F*, G*, H* on the extended range;
 *   fhalf: CTU fluxes F^{n+1/2}, G^{n+1/2}, H^{n+1/2} on the faces of the box's cells.
 * Returns 0 on success, -1 on an invalid box. */
int ref_ctu_update_box(const ref_config* c, double* const u[5], double dt, const int lo[3],
                       const int hi[3], double* const out[5], double* const* fstar,
                       double* const* fhalf, ref_stats* st);

/* One full CTU step in place: ghost fill, then u^{n+1} on every real cell. */
int ref_ctu_step(const ref_config* c, double* const u[5], double dt, ref_stats* st);

/* Threads used by ref_ctu_update_box (and so ref_ctu_step): the OpenMP build of this source
 * shares the z-planes of every loop among them (n > 0 sets the count; returns the count in
 * effect); the serial build ignores n and returns 1.  Both builds give identical results. */
int ref_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
