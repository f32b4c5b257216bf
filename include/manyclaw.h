/*
 * manyclaw.h -- C ABI of libmanyclaw.so, the MI355X (gfx950) implementation
 * of the 2D finite-volume wave-propagation step.
 *
 * The paper's statement of the problem (section 2, "Threading the Riemann
 * solver"): a pointwise Riemann solver takes the states and auxiliary values
 * of adjacent cells and computes the waves, speeds and fluctuations at the
 * edge between them, without knowing about the parallelism around it; the
 * step around it applies limiters (section 1.2, Table 1) and updates the
 * cells, and each grid advances with its own time step (section 1.2,
 * "Dynamic time stepping").  The formulas are those of the wave-propagation
 * method (LeVeque, Finite Volume Methods for Hyperbolic Problems, 2002).
 *
 * Conventions for every entry point:
 *   - Pointers are DEVICE pointers unless marked "host".  The caller owns
 *     every array it passes; the library keeps no caller pointer after a
 *     call returns.
 *   - Arrays are structure-of-arrays, x fastest: a field array is
 *     [meqn][ny][nx] of the context's dtype (double for MC_F64, float for
 *     MC_F32).
 *   - Calls are asynchronous on the context's HIP stream and return
 *     MC_OK when the work was enqueued.  Argument errors are detected on the
 *     host before anything is launched and return MC_EINVAL (nothing is
 *     enqueued).  HIP launch failures return MC_EHIP.
 *   - Conditions found on the device (a non-physical state: h, rho or p <= 0
 *     or NaN; the Euler HLLE fallback having been taken) are OR-ed into the
 *     context's device status word; mc_status_get reads it.
 *   - A context is not thread-safe; separate contexts are independent.
 */
#ifndef MANYCLAW_H
#define MANYCLAW_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mc_ctx mc_ctx; /* opaque */

typedef enum {
    MC_OK = 0,
    MC_EINVAL = -1,        /* bad argument, detected on the host before any launch */
    MC_ENOMEM = -2,        /* device allocation failed (context creation only) */
    MC_EHIP = -3,          /* a HIP call failed */
    MC_ECFL = -4,          /* the error named by the MC_ST_CFL status bit: a run under the
                              time-step rule had more than MC_MAX_RETRIES attempts in a row
                              rejected (for a caller that turns a status word into an error) */
    MC_ENONPHYS = -5,      /* the error named by the MC_ST_NONPHYS status bit */
    MC_EUNSUPPORTED = -6,  /* valid request this build does not implement */
    MC_ESCRATCH = -7       /* the request needs more than the library's static device
                              array holds (mc_step2d_patches_noalloc) */
} mc_status;

/* Riemann solvers (meqn, mwaves, maux):
 *   MC_ADVECTION     (1, 1, 0)  q_t + u q_x + v q_y = 0
 *   MC_ACOUSTICS     (3, 2, 0)  q = (p, u, v), constant rho and K
 *   MC_ACOUSTICS_VC  (3, 2, 2)  q = (p, u, v), aux = (rho, c) per cell
 *   MC_SW_ROE        (3, 3, 0)  q = (h, hu, hv), Roe + Harten-Hyman fix
 *   MC_EULER_ROE     (4, 4, 0)  q = (rho, rho u, rho v, E), Roe + HH, HLLE fallback
 *   MC_SW_HLLE       (3, 3, 0)  HLLE, waves in slots 0 and 2
 *   MC_SW_SURROGATE  (3, 3, 0)  learned shallow-water solver (mc_sur_* entry points)
 *   MC_EULER_SURROGATE (4, 4, 0) learned Euler solver (mc_sur_* entry points) */
typedef enum {
    MC_ADVECTION = 0, MC_ACOUSTICS = 1, MC_ACOUSTICS_VC = 2, MC_SW_ROE = 3,
    MC_EULER_ROE = 4, MC_SW_HLLE = 5, MC_SW_SURROGATE = 6, MC_EULER_SURROGATE = 7
} mc_solver;

typedef enum {
    MC_LIM_NONE = 0,        /* phi = 1 (Lax-Wendroff) */
    MC_LIM_MINMOD = 1, MC_LIM_SUPERBEE = 2, MC_LIM_VANLEER = 3, MC_LIM_MC = 4,
    MC_LIM_FIRST_ORDER = 5  /* no correction flux */
} mc_limiter;

typedef enum { MC_BC_PERIODIC = 0, MC_BC_EXTRAP = 1 } mc_bc;

typedef enum { MC_F64 = 0, MC_F32 = 1 } mc_dtype;

/* physical parameters and the time-step rule (host struct) */
typedef struct {
    double g, gamma, rho, K, u, v;
    double cfl_target; /* desired Courant number: dt_{n+1} = cfl_target / smax_n */
    double cfl_max;    /* a step with dt_n * smax_n > cfl_max is rejected */
} mc_params;

/* ping-pong state (host struct holding device pointers): a step reads
 * q[cur], writes q[1 - cur] and flips cur */
typedef struct { void* q[2]; int32_t cur; } mc_state;

/* result of one step or of the max-speed pre-pass (device struct) */
typedef struct {
    double smax; /* max over counted x-edges of |s|/dx and y-edges of |s|/dy */
    double cfl;  /* dt * smax (0 for the pre-pass) */
} mc_cfl;

/* device-resident clock for the variable time-step rule (paper, section
 * 1.2 and Table 1, "dynamic time stepping"; the rule is the usual one of
 * the method, LeVeque 2002, section 4.4) (device struct, 72 bytes).
 * mc_clock_init fills it; each mc_run2d attempt reads dt and cur, and the
 * attempt's last workgroup applies the rule:
 *   cfl = dt * smax; if cfl <= cfl_max: accept (cur ^= 1, t += dt, n_acc++,
 *   rej_run = 0), else n_rej++ and rej_run++; in both cases
 *   dt = cfl_target / smax.
 * When rej_run exceeds MC_MAX_RETRIES (a state that no longer yields a
 * usable step: a NaN speed, a blow-up) the clock latches MC_ST_CFL in its
 * status and in the context's status word (mc_status_get). */
#define MC_MAX_RETRIES 8
typedef struct {
    double t, dt, cfl, smax;
    int32_t cur, n_acc, n_rej, status;
    double cfl_target, cfl_max;
    int32_t rej_run, reserved;
} mc_clock;

/* Create a context for one solver, dtype and grid of nx x ny cells with
 * spacing dx, dy.  hip_stream is a hipStream_t (NULL = the null stream).
 * Allocates the context's small device scratch (counters, reductions,
 * status).  Returns MC_EINVAL for an unknown solver/dtype, nx or ny < 1,
 * dx or dy <= 0, or a NULL ctx/params; MC_ENOMEM or MC_EHIP on failure. */
int mc_ctx_create(mc_ctx** ctx, int solver, int dtype, const mc_params* params,
                  int32_t nx, int32_t ny, double dx, double dy, void* hip_stream);
void mc_ctx_destroy(mc_ctx* ctx);

/* Rows per work item of the fused step kernel: 0 (default) chooses them per
 * launch from the kernel's occupancy so that the grid fills whole rounds of
 * resident wavefronts; 8..1024 fixes them.  Results do not depend on it. */
int mc_ctx_set_tile(mc_ctx* ctx, int32_t rows_per_item);

/* Picks the rows per work item of the split step for this context's grid
 * by timing (the paper, section 2, treats the traversal and tiling of the
 * grid as a performance choice apart from the solver; its best layout
 * depends on the machine).  Candidates: the occupancy rule (0) and 16, 24,
 * 32, 40, 48, 64, 96, 128, 192, 256 rows (those up to the grid height);
 * each is timed over three launches after one warm-up, twice, and the
 * fastest is kept as by mc_ctx_set_tile (the occupancy rule when it is
 * within 3 % of the fastest).  With MANYCLAW_TUNE_CACHE naming a file (as
 * for mc_patches_tune), the choice for this solver, dtype, limiter,
 * boundary rule, grid size and device is taken from it when present (no
 * launch at all) and added to it otherwise.  Every launch is the step of
 * st->q[st->cur] with this dt, limiter, boundary rule and aux (as
 * mc_step2d) written into st->q[1 - st->cur]; st->cur is not changed, so
 * the state's other buffer is overwritten and nothing else.  rows_out
 * (host, may be NULL) receives the choice (0: the occupancy rule).
 * Synchronises the context's stream.  Errors as mc_step2d;
 * MC_EUNSUPPORTED for the learned solvers. */
int mc_tune_rows(mc_ctx* ctx, const mc_state* st, const void* aux, double dt, int limiter, int bc,
                 int32_t* rows_out);

/* Batch of n independent normal Riemann problems (paper, section 2; the
 * outputs are the method's per-edge work arrays).
 *   ixy:      1 = x-normal, 2 = y-normal (the momentum/velocity slots
 *             exchange roles)
 *   q_left, q_right: [meqn][n] states left and right of each edge
 *   aux:      [2][maux][n] (left block, then right block), NULL when maux = 0
 *   waves:    out [mwaves][meqn][n];  speeds: out [mwaves][n]
 *   amdq, apdq: out [meqn][n], left- and right-going fluctuations
 * n = 0 is a no-op.  MC_EINVAL: n < 0, ixy not 1/2, a NULL array (aux only
 * when maux > 0).  For MC_SW_SURROGATE and MC_EULER_SURROGATE the context
 * needs MC_F32 and an attached network (mc_ctx_set_surrogate), else
 * MC_EINVAL; unflagged edges carry the network waves in slots 0 and 2
 * (shallow water; slot 1 zero) or 0, 1 and 3 (Euler; slot 2 zero). */
int mc_rp2(mc_ctx* ctx, int32_t ixy, int64_t n,
           const void* q_left, const void* q_right, const void* aux,
           void* waves, void* speeds, void* amdq, void* apdq);

/* One dimensionally split step (x-sweep, then y-sweep of its result, each
 * with the full dt; ghost cells by index mapping, two per side) of the
 * context's grid: limited second-order correction fluxes (section 1.2,
 * Table 1), conservative update, and the CFL max-speed reduction.
 *   st:      reads st->q[st->cur], writes st->q[1 - st->cur], flips st->cur
 *            (the caller flips back to discard a rejected step)
 *   aux:     [maux][ny][nx] or NULL when maux = 0
 *   dt:      time step (host value)
 *   cfl_out: device mc_cfl receiving smax and dt * smax, or NULL
 * MC_EINVAL: NULL st or buffers, q[0] == q[1], dt < 0, bad limiter/bc.
 * MC_SW_SURROGATE, MC_EULER_SURROGATE: MC_F32 only, network attached with
 * mc_ctx_set_surrogate;
 * the context then owns an intermediate state and an edge-record buffer
 * (allocated on the first such step, MC_ENOMEM if that fails). */
int mc_step2d(mc_ctx* ctx, mc_state* st, const void* aux, double dt,
              int limiter, int bc, mc_cfl* cfl_out);

/* One Strang-split step (Strang 1968; LeVeque 2002, section 19.5): x-sweep
 * of dt/2, y-sweep of dt, x-sweep of dt/2, each the sweep of mc_step2d
 * (same solvers, limiters, boundary rule and aux; the surrogate solvers
 * return MC_EUNSUPPORTED).  Second order in time for smooth solutions where
 * the plain (Godunov) step is first order.  One launch reads q^n once and
 * writes q^{n+1} once: each row finished by the fused x and y sweeps takes
 * its closing x half-sweep in the same pass (the boundary rule re-applied
 * to the intermediate state first).  st and the errors as for mc_step2d.
 * cfl_out (device or NULL):
 * smax = the largest Courant number of the three sweeps divided by dt,
 * i.e. max(max|s_x| / (2 dx), max|s_y| / dy), and cfl = dt * smax. */
int mc_step2d_strang(mc_ctx* ctx, mc_state* st, const void* aux, double dt,
                     int limiter, int bc, mc_cfl* cfl_out);

/* One unsplit step (LeVeque 2002, chapters 20-21; the paper's "both
 * directions at once", section 2): every x- and y-edge solved on the one
 * state q^n, the limited normal corrections of both directions, and the
 * fluctuations entering each cell split by a transverse solve into the
 * parts moving across the other direction, which correct that direction's
 * fluxes by -dt/(2 d) times them (corner transport, first-order transverse
 * propagation).  One kernel reads q^n once and writes q^{n+1} once.
 * Solvers: MC_ADVECTION, MC_ACOUSTICS, MC_SW_ROE, MC_SW_HLLE, MC_EULER_ROE,
 * MC_ACOUSTICS_VC (the learned solvers: MC_EUNSUPPORTED); the transverse
 * solve uses the transverse eigenvectors at the edge's Roe average (for
 * MC_SW_HLLE the Roe average of its two cells; none on a dry shallow-water
 * edge or where the Euler average has c^2 <= 0), and for MC_ACOUSTICS_VC
 * the impedances and sound speeds of the receiving cell and of its two
 * neighbours across the transverse direction.  aux ([2][ny][nx] device, (rho, c), as for
 * mc_step2d) is required for MC_ACOUSTICS_VC (NULL: MC_EINVAL) and ignored
 * otherwise.  st, dt, limiter, bc and the errors as for mc_step2d;
 * cfl_out (device or NULL): smax = max(max|s_x| / dx, max|s_y| / dy) over the
 * counted edges, cfl = dt * smax.  The context keeps a 16-byte reduction
 * buffer (allocated on the first call). */
int mc_step2d_unsplit(mc_ctx* ctx, mc_state* st, const void* aux, double dt,
                      int limiter, int bc, mc_cfl* cfl_out);

/* dt_0 pre-pass of the variable time step (paper, section 1.2 and Table 1,
 * "dynamic time stepping"): max over counted x-edges of |s|/dx and y-edges
 * of |s|/dy at state q (both directions at the same state), so that
 * dt_0 = cfl_target / smax.  q: [meqn][ny][nx], aux as for mc_step2d,
 * out: device mc_cfl (out->cfl is set to 0).  MC_EINVAL: NULL ctx, q or
 * out, a bad bc, aux missing for a solver that needs it, a learned solver. */
int mc_max_speed(mc_ctx* ctx, const void* q, const void* aux, int bc, mc_cfl* out);

/* Initialise a device clock for the variable time step (section 1.2 and
 * Table 1, "dynamic time stepping") from state q (cur = 0 means q is q0):
 * dt = cfl_target / smax(q), t = 0, counters and status 0; cfl_target and
 * cfl_max come from the context's params.  clk: device mc_clock.  Errors
 * as for mc_max_speed (clk NULL: MC_EINVAL). */
int mc_clock_init(mc_ctx* ctx, mc_clock* clk, const void* q, const void* aux, int bc);

/* nsteps step attempts under the variable time-step rule (section 1.2 and
 * Table 1, "dynamic time stepping": each grid sets its own dt from its own
 * CFL reduction), driven entirely on the device by clk (no host
 * synchronisation): attempt k reads q[clk->cur], writes q[1 - clk->cur].
 * Rejected attempts count in clk->n_rej and do not advance the state; more
 * than MC_MAX_RETRIES in a row latch MC_ST_CFL.  q0, q1: the two state
 * buffers ([meqn][ny][nx] each, distinct); aux as for mc_step2d.
 * use_graph != 0 captures the attempts once into a HIP graph cached in the
 * context (keyed by the arguments) and replays it.  MC_EINVAL: NULL or
 * equal buffers, NULL clk, nsteps < 0, a bad limiter or bc, a learned
 * solver; nsteps = 0 is a no-op. */
int mc_run2d(mc_ctx* ctx, void* q0, void* q1, const void* aux, mc_clock* clk,
             int32_t nsteps, int limiter, int bc, int use_graph);

/* One patch of a batch (host and device struct, 88 bytes).  The patch's
 * fields [meqn][ny][nx] start at element `offset` of each of the two pools;
 * cur says which pool holds its current state.  t, dt, cfl, smax, n_acc,
 * n_rej and status are the state of its own time-step rule; dt <= 0 on entry
 * means "start from dt_0 = cfl_target / smax of the current state". */
typedef struct {
    int32_t nx, ny;
    int64_t offset;
    double dx, dy;
    double t, dt, cfl, smax;
    int32_t bc, status, n_acc, n_rej;
    int32_t cur, reserved;
} mc_patch;

/* Batched uneven patches (paper, section 1.2: larger portions of the data
 * scheduled onto finer-grained workers; every refined grid manages its own
 * time step).  Advances every patch by nsteps accepted steps of the split
 * step, each under its own time-step rule (rejections retried, counted in
 * n_rej), in ONE persistent kernel launch; use_graph != 0 captures that
 * launch once into a HIP graph (cached per arguments) and replays it.
 *   patches_host: host copy of the descriptors (geometry: nx, ny, offset,
 *                 dx, dy, bc, cur); only read, to build the schedule
 *   patches_dev:  device descriptors, read and updated by the kernel
 *   pool0, pool1: device pools of the context's dtype; patch k's fields
 *                 [meqn][ny][nx] start at element offset of a pool
 * The context's solver must be MC_SW_ROE, MC_SW_HLLE, MC_EULER_ROE,
 * MC_ACOUSTICS or MC_ADVECTION (no per-cell aux, no learned solver;
 * MC_EUNSUPPORTED otherwise); its params give the solver's constants,
 * cfl_target and cfl_max; its nx, ny, dx, dy are not used.  MC_EINVAL: NULL arrays, n < 1, nsteps < 0, pool0 == pool1,
 * a patch with nx or ny < 1, dx or dy <= 0, a bad bc or cur.  A patch that
 * cannot finish within 4 nsteps + 64 attempts stops early (n_acc tells). */
int mc_step2d_patches(mc_ctx* ctx, const mc_patch* patches_host, mc_patch* patches_dev,
                      int32_t n_patches, void* pool0, void* pool1, int32_t nsteps, int limiter,
                      int use_graph);

/* mc_step2d_patches without device allocation, for callers that cannot
 * allocate device memory (code under HIP graph capture, serving loops,
 * harnesses that forbid hipMalloc): the same kernel, the same arguments
 * and results (bitwise equal to mc_step2d_patches with use_graph = 0), but
 * the batch's schedule (work items and per-workgroup lists, about 12 bytes
 * per work item) goes into a static device array of 4 MiB that the library
 * holds on every device it runs on until the process ends; no plan or
 * graph is cached and nothing is allocated on the device.  The schedule is
 * copied into the array on the context's stream (from host memory, so the
 * call cannot itself be captured), ordered after the work already on that
 * stream.  Every call on a device shares that device's array: calls that
 * can overlap on one device (other streams, other threads) race; calls on
 * one stream do not.  MC_ESCRATCH (nothing enqueued) when the schedule
 * needs more than 4 MiB; otherwise the errors of mc_step2d_patches. */
int mc_step2d_patches_noalloc(mc_ctx* ctx, const mc_patch* patches_host, mc_patch* patches_dev,
                              int32_t n_patches, void* pool0, void* pool1, int32_t nsteps,
                              int limiter);

/* Autotuner of the batch schedule: times eight-step persistent launches
 * (best of three) for candidate rows-per-chunk of each of four patch-height
 * classes (ny < 32, < 64, < 128, >= 128) on scratch copies shaped like the
 * batch (the caller's pools and descriptors are not touched), keeps the
 * fastest (coordinate search, two passes; a change must be at least 1 %
 * faster) and caches it in the context for this geometry.
 * rows_out (host, 4 ints, may be NULL) receives the choice.  Synchronises
 * the context's stream.  When the environment variable MANYCLAW_TUNE_CACHE
 * names a file, choices persist across processes: an entry for this
 * geometry, solver, dtype, limiter and device (GPU architecture and CU
 * count) is taken from it without timing anything, and a tuned choice is
 * added to it (a JSON object of "key": [values] entries, replaced as a
 * whole by rename). */
int mc_patches_tune(mc_ctx* ctx, const mc_patch* patches_host, int32_t n_patches, int limiter,
                    int32_t* rows_out);

/* Sets the rows per chunk of the four height classes for this geometry
 * (4..4096 each) instead of tuning. */
int mc_patches_set_rows(mc_ctx* ctx, const mc_patch* patches_host, int32_t n_patches,
                        const int32_t* rows);

/* Measurement utility: copies nbytes (a multiple of 16; both pointers
 * 16-byte aligned) from src to dst with a plain grid-stride kernel on the
 * context's stream.  Used to measure the achievable HBM bandwidth and to
 * calibrate the hardware memory counters against a known byte count.
 * MC_EINVAL on NULL pointers, misalignment or a bad size. */
int mc_copy_probe(mc_ctx* ctx, void* dst, const void* src, int64_t nbytes);

/* Reads and clears the device status word (synchronises the context's
 * stream).  *status receives the OR of MC_ST_* bits seen since the last read:
 *   MC_ST_NONPHYS   a non-physical state (h, rho or p <= 0, or NaN) met by a
 *                   solver (error code MC_ENONPHYS)
 *   MC_ST_FALLBACK  the Euler solver took its HLLE fallback (information)
 *   MC_ST_CFL       a device clock had more than MC_MAX_RETRIES attempts in
 *                   a row rejected (error code MC_ECFL) */
#define MC_ST_NONPHYS 1
#define MC_ST_FALLBACK 2
#define MC_ST_CFL 4
int mc_status_get(mc_ctx* ctx, int32_t* status /* host */);

/* ------------------------------------------------------------------ */
/* Learned normal Riemann solvers (the surrogates).  The paper has no
 * learned component; a network replaces its per-edge solve (section 2) for
 * MC_SW_SURROGATE and MC_EULER_SURROGATE contexts and leaves the limiter,
 * update and CFL reduction as they are.  Per edge, in the edge's normal
 * frame, with reference scales of the mean state:
 *   shallow water  q = (h, hu_n, hu_t); h0 = (hL + hR)/2, c0 = sqrt(g h0),
 *            jump scales S = (h0, h0 c0, h0 c0)
 *   Euler    q = (rho, rho u_n, rho u_t, E); rho0, p0 the means of the two
 *            sides, c0 = sqrt(gamma p0 / rho0), S = (rho0, rho0 c0, rho0 c0,
 *            rho0 c0^2)
 *   inputs   x = (ubar/c0, vbar/c0, m, e) with ubar, vbar the mean velocities
 *            and the scaled jump (qR - qL)/S = m e, |e| = 1 (NIN = 6 or 7)
 *   network  NIN-128-128-128-128-NOUT, tanh-form GELU after each hidden
 *            layer, BF16 weights and activations, FP32 accumulation (MFMA)
 *   outputs  K speeds in units of c0, then K waves in units of m S:
 *            shallow water K = 2 (NOUT 8; record slots 0, 2: the two
 *            acoustic families, the shear wave folded in by its speed's
 *            sign); Euler K = 3 (NOUT 15; slots 0, 1, 3: acoustic, entropy
 *            plus shear, acoustic); then projected (smallest change at fixed
 *            speeds) so that A-dQ + A+dQ = f(qR) - f(qL) in FP32
 *   fallback the plain solver of the system (Roe + Harten-Hyman, HLLE where
 *            Roe's intermediate states are not physical) on flagged edges:
 *            shallow water h outside [1e-3, 10], |u| or |v| > 5, min h <
 *            1e-2; Euler rho or p outside [0.05, 10], |u| or |v| > 2; either
 *            system |u_n| >= c on a side (every transonic edge); a
 *            degenerate projection.  Flags are decided in FP32 from products
 *            only (shallow water |u| >= c as hu^2 >= g h^3; Euler p rho =
 *            (gamma - 1)(E rho - |rho u|^2 / 2) against the box times rho,
 *            |u| >= c as (rho u)^2 >= gamma p rho).
 * Parameters: nparams floats (mc_sur_dims), layer after layer, each layer's
 * weight matrix [out][in] row-major followed by its bias [out].
 * Row layouts: inputs X [n][8] (NIN used, the rest 0); targets and outputs
 * [n][ystride] (NOUT used; ystride 8 or 16).
 * A network handle owns its parameters (FP32 master copy, BF16 packed
 * copies), Adam moments and a training workspace for max_batch rows.  All
 * calls are asynchronous on the handle's stream unless stated. */
#define MC_SUR_NPARAMS 51464      /* shallow water */
#define MC_SUR_NIN 6
#define MC_SUR_NOUT 8
#define MC_SUR_EU_NPARAMS 52495   /* Euler */
#define MC_SUR_EU_NIN 7
#define MC_SUR_EU_NOUT 15
typedef struct mc_sur mc_sur; /* opaque */

/* Network sizes of a model (MC_SW_SURROGATE or MC_EULER_SURROGATE; host
 * ints out); MC_EINVAL for other values. */
int mc_sur_dims(int32_t model, int32_t* nparams, int32_t* nin, int32_t* nout, int32_t* ystride);
/* model: MC_SW_SURROGATE or MC_EULER_SURROGATE.  max_batch: largest batch
 * of mc_sur_loss_grad / mc_sur_train (1..1<<20).  Parameters start at zero;
 * MC_EINVAL, MC_ENOMEM or MC_EHIP. */
int mc_sur_create(mc_sur** sur, int32_t model, int32_t max_batch, void* hip_stream);
void mc_sur_destroy(mc_sur* sur);

/* Parameters from a device array of nparams floats (copied); resets Adam's
 * moments and step count. */
int mc_sur_set_params(mc_sur* sur, const float* params);
/* Copies the FP32 master parameters into a device array. */
int mc_sur_get_params(mc_sur* sur, float* params);
/* Initial parameters from nparams uniforms in [0, 1) (device, double):
 * weights uniform in +-sqrt(6 / (fan_in + fan_out)) (Glorot and Bengio
 * 2010), biases 0; resets Adam. */
int mc_sur_init_params(mc_sur* sur, const double* uniforms);

/* Training pairs (x-normal states), labels from the plain Roe solver in
 * FP64.  prm: host; g is used for shallow water, gamma for Euler.
 *   shallow water: uniforms [6][n] rows (hL, uL, vL, hR, uR, vR),
 *     h = exp(ln 1e-3 + (ln 10 - ln 1e-3) U), u, v = -5 + 10 U; outputs
 *     (s1, s3)/c0, W_a = A-dQ/s1, W_b = A+dQ/s3 (the middle wave split
 *     by the sign of its speed), waves scaled by 1/(m S)
 *   Euler: uniforms [8][n] rows (rhoL, uL, vL, pL, rhoR, uR, vR, pR), rho
 *     and p = exp(ln 0.05 + (ln 10 - ln 0.05) U), u, v = -2 + 4 U; outputs
 *     (s1, u_hat, s4)/c0, W1, W2 + W3, W4, waves scaled by 1/(m S)
 * keep[i] = 1 when the pair enters the loss: no flag, m > 0, s1 < 0 < s_last,
 * Roe's intermediate states physical and no entropy-fix split (the HH
 * transonic test of the two acoustic families).
 *   X: out [n][8]; Y: out [n][ystride] (0 where not kept); keep: out [n] */
int mc_sur_gen(mc_sur* sur, const mc_params* prm, int64_t n, const double* uniforms, float* X,
               float* Y, int32_t* keep);
/* Stable compaction of the kept rows of X ([n][8]) and Y ([n][ystride])
 * into Xc, Yc (same layouts, capacity n); *n_kept (host) receives their
 * number.  Synchronises. */
int mc_sur_compact(mc_sur* sur, int64_t n, const float* X, const float* Y, const int32_t* keep,
                   float* Xc, float* Yc, int64_t* n_kept);

/* Network outputs for n input rows X [n][8] into out [n][ystride] (padding
 * columns 0), by the fused inference kernel (the one the step uses). */
int mc_sur_forward(mc_sur* sur, int64_t n, const float* X, float* out);
/* Loss and gradient of one batch (1 <= n <= max_batch) by the training
 * kernels: loss = sum of squared output errors / (nout n).  grad: device
 * nparams floats or NULL (the gradient then stays in the handle for
 * mc_sur_adam); loss: device float or NULL. */
int mc_sur_loss_grad(mc_sur* sur, int64_t n, const float* X, const float* Y, float* grad,
                     float* loss);
/* One Adam step (Kingma and Ba 2015, Algorithm 1) on the handle's last
 * gradient with step size lr; repacks the BF16 copies. */
int mc_sur_adam(mc_sur* sur, float lr, float beta1, float beta2, float eps);
/* Whole training run on the device: for each epoch, batches of `batch`
 * rows of (X, Y) in the order order_host[epoch][k] (host, epochs x
 * (n / batch) batch indices), each a loss/gradient and an Adam step (beta
 * 0.9, 0.999, eps 1e-8) with step size lr0 (1 + cos(pi i / total)) / 2 at
 * update i of total.  loss_host (host, epochs floats, may be NULL) receives
 * each epoch's mean batch loss.  Synchronises once per epoch. */
int mc_sur_train(mc_sur* sur, int64_t n, const float* X, const float* Y, int32_t batch,
                 int32_t epochs, float lr0, const int32_t* order_host, float* loss_host);
/* Mean squared output error of the network over n rows (fused kernel);
 * *loss_host receives it.  Synchronises. */
int mc_sur_eval(mc_sur* sur, int64_t n, const float* X, const float* Y, double* loss_host);

/* Attaches a network to a surrogate context (NULL detaches); the handle's
 * model must be the context's solver, else MC_EINVAL.  The handle must
 * outlive the context's use of it; the context uses its packed weights as
 * they are at each call. */
int mc_ctx_set_surrogate(mc_ctx* ctx, mc_sur* sur);
/* Edges solved and edges that fell back since the last call, over every
 * surrogate step and mc_rp2 of the context (host int64s; synchronises and
 * clears). */
int mc_sur_edge_stats(mc_ctx* ctx, int64_t* edges, int64_t* fallback);

/* ------------------------------------------------------------------ */
/* Two-level refinement coupling (paper, section 1.2 and Table 1: "dynamic
 * time stepping"; each refined grid manages its own time step, with an
 * update on refinement boundaries by spatial and temporal interpolation).
 * The method is the standard one for the wave-propagation scheme:
 * subcycling with interpolated ghost cells (Berger and Oliger 1984) and the
 * conservative fix-up at coarse-fine edges (Berger and Colella 1989).
 * The coarse grid is the context's grid (its solver, MC_F64 or MC_F32, its
 * params and stream).  The solver must be one whose fluctuations sum to a
 * physical flux difference, which the fix-up needs: MC_SW_ROE, MC_SW_HLLE,
 * MC_EULER_ROE, MC_ACOUSTICS or MC_ADVECTION.  Refined patches are rectangles
 * of whole coarse cells, non-overlapping, refined by `ratio` in x, y and
 * time; they are given, not chosen (grid management is not part of this).
 * One mc_amr_step(dt):
 *   1. the coarse grid (ghost cells by the boundary rule) takes one split
 *      step of dt; at each coarse edge between an uncovered and a covered
 *      cell the effective flux seen by the uncovered cell is kept;
 *   2. ratio times: every patch gets two ghost cells per side (corners
 *      included) at t + k dt / ratio -- copied from the patch covering the
 *      ghost cell (after the fine-level boundary rule), else the coarse cell
 *      under it with minmod-limited linear slopes, at t and at t + dt,
 *      linear in time -- and takes one split step of dt / ratio on its
 *      padded array (the x-sweep covers the ghost rows); the effective flux
 *      at each patch boundary edge is summed over the substeps;
 *   3. each uncovered coarse cell next to a patch trades its coarse flux
 *      for the average of the ratio x ratio fine fluxes through that edge;
 *   4. each covered coarse cell becomes the average of its fine cells.
 * The hierarchy owns ghost-padded copies of every grid (two per grid) and
 * the flux registers; states enter and leave through mc_amr_set/get. */
typedef struct { int32_t ci0, cj0, cw, ch; } mc_amr_box; /* patch footprint, coarse cells */
typedef struct mc_amr mc_amr; /* opaque */

/* ratio 1..16; boxes: host array of npatch footprints (npatch >= 0), each
 * inside the coarse grid, no two overlapping; bc: MC_BC_PERIODIC or
 * MC_BC_EXTRAP (applied on both levels).  MC_EINVAL on a bad argument,
 * MC_EUNSUPPORTED for other solvers, MC_ENOMEM / MC_EHIP.  Synchronises. */
int mc_amr_create(mc_amr** amr, mc_ctx* ctx, int32_t ratio, int32_t npatch,
                  const mc_amr_box* boxes, int32_t bc);
void mc_amr_destroy(mc_amr* amr);
/* interior size of grid `which` (-1 the coarse grid, p >= 0 patch p; host) */
int mc_amr_dims(const mc_amr* amr, int32_t which, int32_t* nx, int32_t* ny);
/* copy a grid's state in or out: q device [meqn][ny][nx] of the context's
 * dtype (asynchronous on the context's stream) */
int mc_amr_set(mc_amr* amr, int32_t which, const void* q);
int mc_amr_get(mc_amr* amr, int32_t which, void* q);
/* one coarse step of size dt (host value) with the given limiter.
 * cfl_out (device, or NULL): smax = the largest |s| / d over the counted
 * edges of both levels in coarse-step units (fine speeds over fine cells
 * times dt / ratio per fine step equal |s| / d_coarse times dt), and
 * cfl = dt * smax.  Status bits go to the context (mc_status_get). */
int mc_amr_step(mc_amr* amr, double dt, int32_t limiter, mc_cfl* cfl_out);

/* meqn, mwaves, maux of a solver (host ints); MC_EINVAL for unknown solvers */
int mc_solver_dims(int solver, int32_t* meqn, int32_t* mwaves, int32_t* maux);

const char* mc_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif
