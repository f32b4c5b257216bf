/*
 * mco.h -- plain FP64 CPU oracle of the 2D wave-propagation step.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the HIP library under paper_1308_1464_amd/.
 *
 * What it computes (the paper gives the method in words only; the formulas
 * are those of the finite-volume wave-propagation method it names):
 *   - per-edge normal Riemann solves: waves W^p, speeds s^p and the
 *     fluctuations A-dQ (amdq) and A+dQ (apdq) from the two adjacent cell
 *     states and their auxiliary values (paper, section 2, "Threading the
 *     Riemann solver"; LeVeque, Finite Volume Methods for Hyperbolic
 *     Problems (2002), ch. 3, 4, 9, 15),
 *   - wave limiters and the second-order correction flux (paper, section
 *     1.2 and Table 1, "Limiters"; LeVeque 2002, ch. 6),
 *   - the conservative cell update and Godunov dimensional splitting
 *     (LeVeque 2002, ch. 6 and ch. 19),
 *   - the CFL max-speed reduction and the variable time-step rule (paper,
 *     section 1.2, "Dynamic time stepping"; LeVeque 2002, ch. 4/5).
 *
 * All arrays are host FP64, structure-of-arrays [meqn][ny][nx], x fastest.
 */
#ifndef MCO_H
#define MCO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    MCO_ADVECTION = 0,   /* meqn 1, mwaves 1 */
    MCO_ACOUSTICS = 1,   /* meqn 3 (p,u,v), mwaves 2 */
    MCO_ACOUSTICS_VC = 2,/* meqn 3, mwaves 2, maux 2 (rho, c) */
    MCO_SW_ROE = 3,      /* meqn 3 (h,hu,hv), mwaves 3, Roe + Harten-Hyman */
    MCO_EULER_ROE = 4,   /* meqn 4 (rho,rho u,rho v,E), mwaves 4, Roe + HH, HLLE fallback */
    MCO_SW_HLLE = 5      /* meqn 3, mwaves 3 (slot 2 empty) */
};

enum { MCO_LIM_NONE = 0, MCO_LIM_MINMOD = 1, MCO_LIM_SUPERBEE = 2,
       MCO_LIM_VANLEER = 3, MCO_LIM_MC = 4, MCO_LIM_FIRST_ORDER = 5 };

enum { MCO_BC_PERIODIC = 0, MCO_BC_EXTRAP = 1 };

/* status bits returned by the solvers and the step */
enum { MCO_ST_NONPHYS = 1,   /* h, rho or p <= 0, or a NaN, in an input state */
       MCO_ST_FALLBACK = 2,  /* Euler: the HLLE fallback was taken */
       MCO_ST_BADARG = 4,
       MCO_ST_STALLED = 8 }; /* run2d: more than 1000 consecutive rejections */

typedef struct {
    double g;      /* gravity (shallow water) */
    double gamma;  /* ratio of specific heats (Euler) */
    double rho;    /* density (constant-coefficient acoustics) */
    double K;      /* bulk modulus (constant-coefficient acoustics) */
    double u, v;   /* advection velocity */
} mco_params;

/* meqn, mwaves, maux of a solver; returns 0, or -1 for an unknown solver */
int mco_dims(int solver, int* meqn, int* mwaves, int* maux);

/* One edge.  ixy = 1: x-normal, 2: y-normal.  ql, qr: meqn values;
 * auxl, auxr: maux values or NULL.  wave: [mwaves][meqn]; s: [mwaves];
 * amdq, apdq: [meqn].  Returns status bits. */
int mco_rp1(int solver, const mco_params* P, int ixy,
            const double* ql, const double* qr,
            const double* auxl, const double* auxr,
            double* wave, double* s, double* amdq, double* apdq);

/* n independent edges, structure-of-arrays: ql, qr [meqn][n];
 * aux [2][maux][n] (left block then right block) or NULL;
 * waves [mwaves][meqn][n], speeds [mwaves][n], amdq/apdq [meqn][n].
 * Returns the OR of the per-edge status bits. */
int mco_rp2(int solver, const mco_params* P, int ixy, int64_t n,
            const double* ql, const double* qr, const double* aux,
            double* waves, double* speeds, double* amdq, double* apdq);

/* wave-limiter function phi(theta) */
double mco_phi(int limiter, double theta);

/* One dimensionally split step (x-sweep, then y-sweep on the result, each
 * with the full dt).  q, qout: [meqn][ny][nx]; aux: [maux][ny][nx] or NULL.
 * smax_out (may be NULL): max over counted x-edges of |s|/dx and over
 * counted y-edges of |s|/dy.  nthreads <= 1 runs single-threaded.
 * Returns status bits. */
int mco_step2d(int solver, const mco_params* P, int nx, int ny, double dx, double dy,
               const double* q, const double* aux, double dt, int limiter, int bc,
               double* qout, double* smax_out, int nthreads);

/* Max over x-edges of |s|/dx and y-edges of |s|/dy at the given state (the
 * dt_0 pre-pass).  Returns status bits. */
int mco_max_speed(int solver, const mco_params* P, int nx, int ny, double dx, double dy,
                  const double* q, const double* aux, int bc, double* smax_out, int nthreads);

/* Variable time-step driver: dt_0 = cfl_target / smax(q^0); then each step
 * with dt_n gives cfl_n = dt_n * smax_n; cfl_n > cfl_max rejects the step and
 * retries with dt = cfl_target / smax_n; otherwise the step is accepted and
 * dt_{n+1} = cfl_target / smax_n.  Runs nsteps accepted steps, in place on q.
 * dt_hist (may be NULL): nsteps accepted dt values; t_out, nrej_out may be
 * NULL.  Returns status bits. */
int mco_run2d(int solver, const mco_params* P, int nx, int ny, double dx, double dy,
              double* q, const double* aux, int limiter, int bc,
              double cfl_target, double cfl_max, int nsteps,
              double* dt_hist, double* t_out, int* nrej_out, int nthreads);

#ifdef __cplusplus
}
#endif
#endif
