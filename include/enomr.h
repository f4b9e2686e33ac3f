/*
 * enomr.h - C ABI of the MI355X (gfx950) ENO-MR library.
 *
 * ENO-MR is the finite-difference scheme of H. Shen, "An efficient class of
 * increasingly high-order ENO schemes with multi-resolution" (arXiv 2311.15504):
 * per-face flux reconstruction over nested candidate stencils (orders 5..17),
 * global Lax-Friedrichs splitting, characteristic projection at Roe-averaged
 * faces for the Euler equations, and SSP-RK3 time stepping.
 *
 * Conventions shared by every call
 * --------------------------------
 * - All array arguments are DEVICE pointers on the context's device, owned by
 *   the caller, FP64 unless stated, C-contiguous.  State arrays are laid out
 *   [variable][y][x] (x fastest) and hold interior cells only; the library
 *   applies the boundary conditions itself (periodic wrap or zero-gradient
 *   copy) when it reads neighbours.
 * - Every call is asynchronous and ordered on the context's HIP stream.  The
 *   library keeps no pointer beyond the work it has enqueued.
 * - Argument errors are returned at once (ENOMR_EINVAL, ENOMR_EORDER) and
 *   nothing is enqueued.  HIP failures return ENOMR_EHIP.  A non-physical state
 *   met on the device (rho <= 0, p <= 0, NaN) is latched in a device status word
 *   and reported by enomr_check() as ENOMR_ENONPHYS.  The library never aborts
 *   or prints; enomr_last_error() gives a message for the calling thread.
 * - Stencil-index logs (uint8) hold, per face, per characteristic field and
 *   per sign (+ then -), the position of the chosen stencil in the order's
 *   candidate list (0 = the full stencil, see enomr_coefficients()).
 */
#ifndef ENOMR_H
#define ENOMR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    ENOMR_OK = 0,
    ENOMR_EINVAL = 1,    /* bad argument or shape                          */
    ENOMR_EORDER = 2,    /* order not odd in 5..17                         */
    ENOMR_ENOMEM = 3,    /* device allocation failed                       */
    ENOMR_EHIP = 4,      /* a HIP runtime call failed                      */
    ENOMR_ENONPHYS = 5,  /* non-physical state met on the device           */
    ENOMR_ENODEV = 6     /* no usable gfx950 device                        */
} enomr_status;

enum { ENOMR_ADVECTION = 0, ENOMR_BURGERS = 1, ENOMR_EULER = 2 };
enum { ENOMR_PERIODIC = 0, ENOMR_OUTFLOW = 1 };
enum { ENOMR_SPLIT_NONE = 0, ENOMR_SPLIT_LF = 1 };
enum { ENOMR_CHARACTERISTIC = 0, ENOMR_COMPONENTWISE = 1 };
enum { ENOMR_ALPHA_LINE = 0, ENOMR_ALPHA_FIELD = 1 };

/*
 * A conservation law on a uniform grid (Sec. 2.1, Eq. 1DHCL; Sec. 4.3-4.4).
 *   ndim     1 or 2.  1D states are [nvar][nx]; 2D states [nvar][ny][nx].
 *   system   ENOMR_ADVECTION (u_t + a u_x = 0, nvar 1, ndim 1),
 *            ENOMR_BURGERS (u_t + (u^2/2)_x = 0, nvar 1, ndim 1),
 *            ENOMR_EULER (nvar 3 in 1D: rho, rho u, E; nvar 4 in 2D:
 *            rho, rho u, rho v, E; ideal gas with ratio gamma).
 *   nx, ny   interior nodes per axis (ny = 1 in 1D); at least 2r+1 and at
 *            most 2^31 each; in 2D also ny <= 2097120 and nx*ny <= 2^32
 *            (ENOMR_EINVAL otherwise).
 *   hx, hy   node spacing.
 *   order    2r-1, odd in 5..17.
 *   bc_x/y   ENOMR_PERIODIC or ENOMR_OUTFLOW (zero-gradient copy).
 *   split    scalar laws only: ENOMR_SPLIT_LF (global Lax-Friedrichs,
 *            Eq. LF_Flux_Split) or ENOMR_SPLIT_NONE (reconstruct f itself as
 *            f^+, valid when f'(u) >= 0).  Euler always splits.
 *   gamma    ratio of specific heats (Euler).
 *   adv_speed  the constant a (advection).
 * Euler operator variants (zero-initialised fields give the scheme as the
 * paper runs it: characteristic reconstruction, one alpha per line, no
 * source):
 *   recon    ENOMR_CHARACTERISTIC (project G+- onto the Roe-face eigenvectors,
 *            Sec. 4 preamble) or ENOMR_COMPONENTWISE (reconstruct each
 *            conserved component of G+- = (F +- alpha U)/2 as it is).
 *   alpha_mode  ENOMR_ALPHA_LINE (alpha = max over the line of |u_n|+c,
 *            Eq. LF_Flux_Split) or ENOMR_ALPHA_FIELD (characteristic field k
 *            splits with alpha_k = max over the line of |lambda_k|, lambda =
 *            u_n-c, u_n, [u_n,] u_n+c: w+-_k = (l_k.F +- alpha_k l_k.U)/2).
 *            ENOMR_ALPHA_FIELD needs ENOMR_CHARACTERISTIC.
 *   gravity  2D Euler only: adds the source g [0, 0, rho, rho v] of the
 *            Rayleigh-Taylor problem (Sec. 4.4) to dU/dt; 0 = no source.
 * Batched execution and the adjoint take the default operator only.
 */
typedef struct {
    int32_t ndim;
    int32_t system;
    int64_t nx, ny;
    double hx, hy;
    int32_t order;
    int32_t bc_x, bc_y;
    int32_t split;
    double gamma;
    double adv_speed;
    int32_t recon;
    int32_t alpha_mode;
    double gravity;
} enomr_problem;

typedef struct enomr_ctx enomr_ctx;

/* Context on `device` issuing work on `hip_stream` (a hipStream_t; NULL = the
   null stream).  Uploads the coefficient tables.  *out owned by the caller
   until enomr_destroy(). */
enomr_status enomr_create(int device, void *hip_stream, enomr_ctx **out);
enomr_status enomr_destroy(enomr_ctx *ctx);
enomr_status enomr_set_stream(enomr_ctx *ctx, void *hip_stream);

/* Message describing the last error returned on the calling thread. */
const char *enomr_last_error(void);

/*
 * Host-only: the candidate list of `order` and its coefficients as the library
 * uses them (Sec. 3.1 Eq. Candidates, Tables Flux_reconstruction1/2 and
 * ISCoe1/2).  mn receives 2*ncand ints (m, n) for stencils S_{j-m}^{j+n} in
 * selection order; a and b receive 17 doubles per candidate, entry l+m for
 * offset l.  Any output pointer may be NULL.  Needs no GPU.
 */
enomr_status enomr_coefficients(int order, int32_t *ncand, int32_t *mn, double *a, double *b);

/*
 * Bare scalar ENO-MR reconstruction (Sec. 3.2, Steps 1-3.2) at n faces.
 * f_with_halo: n + 2r - 1 values; face i lies between array entries i+r-1 and
 * i+r.  sign = +1 reconstructs f^+ (centred on the left cell), -1 reconstructs
 * f^- (the mirror image, centred on the right cell).  fhat: n values.
 * idx (nullable): n bytes.  0 <= n <= 2^38 (ENOMR_EINVAL otherwise).
 */
enomr_status enomr_recon_faces(enomr_ctx *ctx, int order, int sign, int64_t n,
                               const double *f_with_halo, double *fhat, uint8_t *idx);

/* Bytes of device workspace that enomr_rhs/dt/ssprk3_step/advance need for
   `prob`. */
enomr_status enomr_workspace_size(const enomr_problem *prob, size_t *bytes);

/*
 * dU/dt = L(U) (Sec. 2.1 Eq. 1DWENOFD, dimension by dimension), with alpha of
 * each line computed from U (Eq. LF_Flux_Split).  ws: workspace of
 * enomr_workspace_size() bytes.  idx (nullable) receives the stencil log:
 *   scalar 1D: [nx+1][2];  Euler 1D: [nx+1][3][2];
 *   Euler 2D: x-faces [ny][nx+1][4][2] followed by y-faces [ny+1][nx][4][2].
 * Face f of a line lies between cells f-1 and f (f = 0..n; for periodic lines
 * faces 0 and n are the same face and carry the same values).
 */
enomr_status enomr_rhs(enomr_ctx *ctx, const enomr_problem *prob, const double *U,
                       double *dUdt, uint8_t *idx, void *ws);

/*
 * enomr_rhs without a workspace and without any device allocation, for
 * callers that cannot allocate (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  Same operator and log layout as
 * enomr_rhs.  The per-line alphas live in a library-owned device array of
 * 131072 doubles (1 MiB) per device, held until the process ends: a problem
 * needs ceil32(na * ny) + na * (2D ? nx : 1) doubles of it (na = 3 with
 * per-field alphas, else 1); a larger one is ENOMR_EINVAL with a message.  In
 * 2D, dUdt also holds the y sweep's part of L until the x sweep completes it
 * in place, so dUdt must not alias U (ENOMR_EINVAL).  Every call on a device
 * shares its array: calls that overlap on one device (other streams or
 * threads) race; calls ordered on one stream do not.
 */
enomr_status enomr_rhs_noalloc(enomr_ctx *ctx, const enomr_problem *prob, const double *U, double *dUdt,
                               uint8_t *idx);

/*
 * Time step from the CFL rule, written to the device scalar *dt_dev:
 *   1D: dt = cfl / (max(|u|+c) / hx), scalar laws use max|f'(u)|;
 *   2D: dt = cfl / (max(|u|+c)/hx + max(|v|+c)/hy).
 * With per-field alphas the maxima are taken over the three field speeds,
 * whose largest is |u|+c: the step is the same.
 */
enomr_status enomr_dt(enomr_ctx *ctx, const enomr_problem *prob, const double *U, double cfl,
                      double *dt_dev, void *ws);

/*
 * One SSP-RK3 step (Sec. 2.3 Eq. TVD3rdRK) of U in place with the step size in
 * the device scalar *dt_dev.  idx_log (nullable): the three stages' stencil
 * logs back to back, each laid out as for enomr_rhs.
 */
enomr_status enomr_ssprk3_step(enomr_ctx *ctx, const enomr_problem *prob, double *U,
                               const double *dt_dev, void *ws, uint8_t *idx_log);

/*
 * nsteps SSP-RK3 steps of U in place, each with dt from the CFL rule at the
 * start of the step.  If t_end > 0 the run stops at t_end: the step that would
 * pass it is shortened to end there and later steps do nothing.  dt_log
 * (nullable, device, nsteps doubles) receives the step sizes used.
 */
enomr_status enomr_advance(enomr_ctx *ctx, const enomr_problem *prob, double *U, double cfl,
                           int64_t nsteps, double t_end, void *ws, double *dt_log);

/* Wait for the context's stream, then return and clear the device status
   (ENOMR_OK or ENOMR_ENONPHYS). */
enomr_status enomr_check(enomr_ctx *ctx);

/*
 * Kernel timing.  Between enomr_profile_start() and enomr_profile_stop() every
 * launch the context makes is bracketed by HIP events on its stream.  stop()
 * waits for the stream and writes, per kernel class, the summed device time in
 * milliseconds (ms[3]) and the number of launches (launches[3]); classes:
 * 0 = x (or 1D) sweep kernels, 1 = y sweep kernels, 2 = alpha / dt / fills.
 * Either pointer may be NULL.
 */
enomr_status enomr_profile_start(enomr_ctx *ctx);
enomr_status enomr_profile_stop(enomr_ctx *ctx, double *ms, int64_t *launches);

/*
 * Linear SSP-RK(m, m-1) (Sec. 2.3, Eq. lSSPRK, coefficients Eq. lSSPRK_Coe,
 * read as alpha_{m,m-1} = (2/m) alpha_{m-1,m-2}) for scalar 1D problems
 * (ENOMR_ADVECTION, ENOMR_BURGERS), the time stepping of the paper's linear
 * convergence tests (Sec. 4.1):
 *   u^(0) = u^n,  u^(s) = u^(s-1) + dt/2 L(u^(s-1)),  s = 1..m-1,
 *   u^{n+1} = sum_{k<m-1} alpha_{m,k} u^(k) + alpha_{m,m-1} (u^(m-1) + dt/2 L(u^(m-1))).
 * The coefficients are computed in exact rational arithmetic and rounded to
 * the nearest doubles.  U: device [nx]; dt is fixed; 2 <= m <= 18.
 * ws: device workspace of enomr_lssp_workspace_size(prob, m) bytes.
 */
enomr_status enomr_lssp_workspace_size(const enomr_problem *prob, int m, size_t *bytes);
enomr_status enomr_lssp_advance(enomr_ctx *ctx, const enomr_problem *prob, double *U, double dt, int64_t nsteps,
                                int m, void *ws);

/*
 * Frozen-stencil discrete adjoint (1D Euler problems).
 *
 * With the stencil choices, the per-stage alpha and the step size fixed from a
 * forward pass, one SSP-RK3 step (Sec. 2.3, Eq. TVD3rdRK) of the operator
 * (Sec. 2.1 Eq. 1DWENOFD with the LF split of Eq. LF_Flux_Split, the Roe-face
 * projection and the chosen stencils of Sec. 3.2) is a smooth map of U; these
 * calls apply the transpose of its Jacobian.
 *
 * enomr_record_steps: nsteps SSP-RK3 steps of U in place with dt from the CFL
 *   rule (bitwise the steps enomr_advance takes), recording per step k:
 *   stages[k] = [U^n, U^(1), U^(2)] (3 states), idx_log[k] = the three stages'
 *   stencil logs (layout of enomr_rhs, 3 * log size bytes), alpha_log[3k..3k+2]
 *   = each stage's alpha, dt_log[k] = the step size.
 * enomr_adjoint_steps: lam (in: adjoint of the state after the recorded steps;
 *   out: adjoint of the state before them), through the recorded steps in
 *   reverse order.
 * enomr_rhs_adjoint: lam_U = (dL/dU)^T lam_dUdt at state U with frozen idx (one
 *   stage log) and alpha (device scalar); lam_U must not alias lam_dUdt
 *   (ENOMR_EINVAL).
 * All arrays are device arrays; ws as from enomr_workspace_size().
 */
enomr_status enomr_rhs_adjoint(enomr_ctx *ctx, const enomr_problem *prob, const double *U, const uint8_t *idx,
                               const double *alpha_dev, const double *lam_dUdt, double *lam_U, void *ws);
enomr_status enomr_record_steps(enomr_ctx *ctx, const enomr_problem *prob, double *U, double cfl, int64_t nsteps,
                                double *stages, uint8_t *idx_log, double *alpha_log, double *dt_log, void *ws);
enomr_status enomr_adjoint_steps(enomr_ctx *ctx, const enomr_problem *prob, int64_t nsteps, const double *stages,
                                 const uint8_t *idx_log, const double *alpha_log, const double *dt_log, double *lam,
                                 void *ws);

/*
 * Batched execution: many independent 1D and 2D Euler problems (uneven
 * sizes and orders) advanced together from captured hipGraphs.  Each problem
 * advances with its own per-stage alphas and CFL time step exactly as
 * enomr_advance() would advance it alone, and its result is bitwise equal to
 * that run.  1D problems: one persistent launch for all steps, in which a
 * workgroup takes a whole problem from a work queue (longest first) and runs
 * all its steps.  2D problems: stage by stage, one launch per order for the
 * alphas (and dt), one for the y faces and one for the x faces of all that
 * order's problems (a tile per workgroup, largest problems first), the
 * orders as parallel branches of a one-step graph replayed once per step.
 * With both kinds, the 1D launch runs on a stream of its own beside the 2D
 * steps.
 *
 * enomr_batch_create: probs[nprob] (ENOMR_EULER, ndim 1 or 2, any order
 * 5..17), U[nprob] device pointers to the problems' states ([3][nx] or
 * [4][ny][nx]), bound to the batch for its lifetime and advanced in place.
 * The batch allocates its own workspace (2 stage states per problem; for 2D
 * also L_y and the per-line alphas).  autotune = 1 times one step of the 1D
 * problems on scratch copies for each tile width (64, 128, 256 faces) and
 * keeps the fastest; 0 uses 128; 64, 128 or 256 use that width; any other
 * value is ENOMR_EINVAL.  autotune = 1 also times one step of the 2D
 * problems for each tile shape of the 2D sweeps (64 x 4, 32 x 8, 16 x 16
 * faces x lines) and keeps the fastest; otherwise the 2D sweeps use 32 x 8.
 * The tile shape does not change any result.
 * enomr_batch_advance: nsteps SSP-RK3 steps of every problem at CFL `cfl`.
 * enomr_batch_info: the 1D kernel's tile width, its workgroups plus those of
 * the largest 2D sweep launch, and the autotune times (ms, for widths
 * 64/128/256; zeros without autotune).  Any pointer may be NULL.
 * enomr_batch_info2d: the 2D sweeps' tile shape and its autotune times (ms,
 * for 64 x 4, 32 x 8, 16 x 16; zeros without autotune).  Any pointer may be
 * NULL.
 * enomr_batch_set_tile2d: use the 2D tile shape tile_faces x tile_lines (one
 * of the three) from the next advance on; waits for the context's stream and
 * rebuilds the 2D step's graph.  Other shapes: ENOMR_EINVAL.
 */
typedef struct enomr_batch enomr_batch;
enomr_status enomr_batch_create(enomr_ctx *ctx, int32_t nprob, const enomr_problem *probs, double *const *U,
                                int autotune, enomr_batch **out);
enomr_status enomr_batch_advance(enomr_batch *batch, double cfl, int64_t nsteps);
enomr_status enomr_batch_info(const enomr_batch *batch, int32_t *tile_faces, int32_t *workgroups,
                              double *tune_ms);
enomr_status enomr_batch_info2d(const enomr_batch *batch, int32_t *tile_faces, int32_t *tile_lines,
                                double *tune_ms);
enomr_status enomr_batch_set_tile2d(enomr_batch *batch, int32_t tile_faces, int32_t tile_lines);
enomr_status enomr_batch_destroy(enomr_batch *batch);

#ifdef __cplusplus
}
#endif

#endif /* ENOMR_H */
