/*
 * thiim.h -- C-ABI of the MI355X (gfx950) THIIM library.
 *
 * The library iterates the Time Harmonic Inverse Iteration Method (THIIM) of
 * Malas et al., "Optimization of an electromagnetics code with multicore
 * wavefront diamond blocking and multi-dimensional intra-tile
 * parallelization" (arXiv:1510.05218): the leapfrog update of Sec. I-A,
 * Eq. (3)/(4) (Eq. (5) for cells with negative permittivity) on a Yee grid,
 * with the six field components split into twelve parts as in Eq. (6)/(7)
 * (Berenger PML), in double-complex arithmetic.  Per cell it keeps the 40
 * double-complex arrays counted in Sec. III (12 split fields, 28 coefficient
 * arrays).
 *
 * Conventions (all calls):
 *   - Grid arrays are [nz][ny][nx] (x fastest) of interleaved complex128
 *     (re, im), the layout of Listings 1 and 2.  N = nx*ny*nz.
 *   - Units: eps0 = mu0 = c0 = 1, mu_r = 1, grid step h.
 *   - Split components, in the order used by every field buffer:
 *       0 H_xy  1 H_xz  2 H_yx  3 H_yz  4 H_zx  5 H_zy
 *       6 E_xy  7 E_xz  8 E_yx  9 E_yz 10 E_zx 11 E_zy
 *     (F_ab = part of field component F_a driven by the other field's
 *     component b, the naming of Listings 1 and 2.)
 *   - Coefficient arrays, in the order used by thiim_get_coeffs:
 *       t_q = q, c_q = 12 + q (q = 0..11), Src of H_xy, H_yx, E_xy, E_yx
 *       = 24..27 (Sec. III: 4*3 + 8*2 = 28 arrays).
 *   - Boundaries: ghost values beyond the z walls are zero (homogeneous
 *     Dirichlet, Sec. II-B); x and y are periodic (Sec. I-A, production
 *     setting) or Dirichlet.
 *   - Ownership: the caller allocates every buffer (the workspace included);
 *     the library never allocates device memory.  A context borrows its
 *     workspace and must be destroyed before the workspace is freed.  Inputs
 *     are read during thiim_create only.
 *   - Errors: every int-returning call returns THIIM_OK (0) or a negative
 *     status; nothing aborts or throws across the ABI.  thiim_last_error()
 *     gives a message for the calling thread's last failure.
 *   - Streams: work is enqueued on grid.stream (a hipStream_t; NULL = the
 *     null stream).  thiim_iterate only enqueues; calls documented as
 *     "synchronising" wait for the stream and report device faults.
 */
#ifndef THIIM_H
#define THIIM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define THIIM_OK 0
#define THIIM_EINVAL (-1)    /* invalid argument */
#define THIIM_ENOMEM (-2)    /* workspace too small */
#define THIIM_EDEVICE (-3)   /* HIP runtime or device error */
#define THIIM_EDIVERGED (-4) /* residual not finite, or grown 1e6-fold over the
                              * smallest one the solve reached */
#define THIIM_ENOTCONV (-5)  /* iteration limit reached before tolerance */

#define THIIM_PERIODIC 0
#define THIIM_DIRICHLET 1

/* Sweep implementations of one THIIM iteration (all give the same result;
 * the fused and blocked forms are bit-identical to the naive one). */
#define THIIM_KERNEL_AUTO 0    /* library's choice */
#define THIIM_KERNEL_NAIVE 1   /* one in-place sweep per half-step */
#define THIIM_KERNEL_FUSED 2   /* H and E half-steps in one HBM pass */
#define THIIM_KERNEL_BLOCKED 3 /* t_block iterations per HBM pass */

/* Coefficient storage (both give bit-identical iterates). */
#define THIIM_STORAGE_FULL 0    /* the 28 coefficient arrays of the paper's
                                 * layout (40 double-complex arrays per cell
                                 * with the 12 fields) */
#define THIIM_STORAGE_COMPACT 1 /* per-cell eps and the 4 Src arrays; t and c
                                 * derived in the sweeps from eps and per-plane
                                 * tables by the same formulas */

/* Arithmetic of thiim_solve. */
#define THIIM_PRECISION_FP64 0  /* every sweep in complex128 */
#define THIIM_PRECISION_MIXED 1 /* defect correction: FP64 residual, correction
                                 * accumulation and norms; the correction
                                 * equation (I - M) d = r approximated by
                                 * complex64 sweeps d <- M d + r (M: the linear
                                 * part of one THIIM iteration).  Needs
                                 * THIIM_STORAGE_COMPACT. */

typedef struct thiim_ctx thiim_ctx;

typedef struct {
    int nx, ny, nz;   /* cells, PML planes included; each >= 2 */
    int bc_x, bc_y;   /* THIIM_PERIODIC or THIIM_DIRICHLET */
    double h;         /* grid step (> 0) */
    double tau;       /* pseudo-time step, 0 < tau <= h / sqrt(3) */
    int kernel;       /* THIIM_KERNEL_* */
    int t_block;      /* iterations per pass for THIIM_KERNEL_BLOCKED: 0 (auto,
                       * = 2), 1 or 2; a remainder runs through the fused sweep.
                       * With THIIM_PRECISION_MIXED, 3 is also allowed; the
                       * complex64 inner sweeps run 2 iterations per pass on
                       * 32 x 32 regions for 0 (auto), 1 and 2, and 3 on
                       * 32 x 16 regions for 3 */
    int tile_x, tile_y; /* fused sweep: tile 64x8, 32x8, 64x4 or 16x16; blocked
                         * sweep: region 64x8, 64x6 or 32x16 (columns x rows) of
                         * which the centre (x-2T) x (y-2T) is stored; 0x0 = auto */
    int z_chunk;      /* z planes per workgroup stream (0 = auto) */
    int storage;      /* THIIM_STORAGE_FULL or THIIM_STORAGE_COMPACT */
    int precision;    /* THIIM_PRECISION_FP64 or THIIM_PRECISION_MIXED */
    int adjoint;      /* 1: reserve the buffers of thiim_adjoint_grad (51 more
                       * arrays; needs THIIM_STORAGE_COMPACT), else 0 */
    void *stream;     /* hipStream_t */
} thiim_grid;

typedef struct {
    /* Device pointer, 2*N doubles: (eps', eps'') per cell.  The relative
     * permittivity is eps' - i eps'' in the paper's exp(+i w t) convention
     * (eps'' >= 0 absorbs); eps' > 0 uses the forward update Eq. (3),
     * eps' < 0 the back iteration Eq. (5); eps' == 0 is rejected. */
    const double *eps;
    /* Host pointers, nz doubles each: PML conductivities.  sigma_e[k] is
     * added to the material conductivity (w eps'') of the two E parts with a
     * z difference (E_xy, E_yx) at plane k; sigma_h[k] is the magnetic
     * conductivity of H_xy, H_yx at plane k.  Other parts get no PML term. */
    const double *sigma_e;
    const double *sigma_h;
    /* Device pointers, 2*N doubles each, or NULL for zero: the source terms
     * S_H and S_E of Eq. (3)/(4) for the x and y components, in the order
     * S_Hx, S_Hy, S_Ex, S_Ey.  Each enters the Src array of the part with a
     * z difference (H_xy, H_yx, E_xy, E_yx). */
    const double *src[4];
} thiim_coeffs;

/* Bytes of device workspace a context on this grid needs: the coefficient
 * data (full: 28 arrays; compact: 5 arrays), two 12-array field buffers,
 * per-plane tables and reduction scratch; 256-byte aligned. */
int thiim_workspace_bytes(const thiim_grid *g, size_t *bytes);

/* Validates the inputs, builds the coefficient data on the device (Eq.
 * (3)-(5) solved for the new value: the 28 arrays with full storage; eps,
 * the 4 Src arrays and per-plane tables with compact storage; the complex64
 * records with mixed precision), zeroes the fields (x0 = 0) and
 * records ||P Phi(0)||_2 for thiim_residual (P: sum of each split pair).
 * omega: angular frequency in units of c0/h.  Synchronising.  On failure
 * *out is NULL. */
int thiim_create(const thiim_grid *g, const thiim_coeffs *m, double omega,
                 void *workspace, size_t workspace_bytes, thiim_ctx **out);

/* Enqueues n >= 0 THIIM iterations x <- Phi(x) (H half-step, Eq. (4), then
 * E half-step, Eq. (3)/(5)).  Asynchronous. */
int thiim_iterate(thiim_ctx *ctx, int n);

/* Relative residual of the physical fields of the current state,
 * ||P (Phi(x) - x)||_2 / ||P Phi(0)||_2, accumulated in FP64 on the device.
 * Does not advance x.  Synchronising; THIIM_EDIVERGED if not finite. */
int thiim_residual(thiim_ctx *ctx, double *rel_res);

/* Iterates until thiim_residual <= tol or max_it sweeps, from the current
 * state.  FP64: the residual is checked every check_every (>= 1) iterations.
 * MIXED: each defect-correction step is one FP64 sweep (the residual) plus
 * complex64 inner sweeps d <- M d + r: check_every of them (rounded up to
 * whole blocked passes, at least one averaging window), or, with
 * check_every = 0, an adaptive count (doubled while a step gains less than
 * 0.3).  The correction added to x is the mean of d over the last
 * Kp = round(2 pi / (omega tau T)) passes of T sweeps -- one period of the
 * modes that an iteration only rotates by e^{-i omega tau}, which the
 * complex64 rounding would otherwise leave in x for ever; those passes sum
 * d into a complex64 buffer as they store it, and x += sum / Kp follows in
 * FP64 once per correction.  A split pair whose
 * two parts have identical coefficients on a plane (the z pairs everywhere,
 * the x and y pairs off the PML) enters a correction through its sum only,
 * half to each part: a MIXED solve determines the physical fields P x, not
 * how such a pair is split.
 * *iters (sweeps done, both precisions) and *rel_res may be NULL.
 * Synchronising; THIIM_ENOTCONV when max_it is reached first;
 * THIIM_EDIVERGED when a residual is not finite or exceeds 1e6 times the
 * smallest one reached so far (e.g. a medium with gain, eps'' < 0). */
int thiim_solve(thiim_ctx *ctx, double tol, int max_it, int check_every,
                int *iters, double *rel_res);

/* Gradient of the absorption functional
 *     J = sum_p w_p eps''_p |E_p|^2
 * (E_p: the physical E field of the current state at cell p, each component
 * the sum of its two split parts, Eq. (6)/(7)) with respect to eps' and
 * eps'' of every cell, by the adjoint method.  One THIIM iteration is
 * x <- M x + c (Sec. I-A, Eq. (3)-(5)); with g = dJ/dx and lam the solution of
 * (I - M^T) lam = g (the transposed iteration lam <- M^T lam + g from
 * lam = 0: the E half-step transposed, then the H half-step transposed),
 *     dJ/dtheta_p = [theta = eps''] w_p |E_p|^2
 *                 + 2 Re sum over the six E parts q of p of lam_q dPhi_q/dtheta_p,
 * dPhi_q/dtheta from the closed forms of t, c and Src of the E parts (the
 * only coefficients that depend on eps; the PML profiles are held fixed).
 * The current state should be converged (thiim_solve); it is not changed.
 *   weight    device, N doubles: w_p
 *   tol > 0   solve to ||P(M^T lam + g - lam)_E|| / ||P g_E|| <= tol by
 *             defect correction: r = M^T lam + g - lam, then m sweeps
 *             d <- M^T d + r (m = max(check_every, 2 Kp), doubled while a
 *             step gains less than 0.3) and lam += the mean of d over the last
 *             Kp = round(2 pi / (omega tau)) sweeps (one rotation period of the
 *             modes an iteration rotates by e^{-i omega tau}; the plain
 *             transposed iteration converges much more slowly where the PML
 *             conductivity is small), until tol or max_it sweeps
 *             (THIIM_ENOTCONV; the outputs are still written).  On a
 *             THIIM_PRECISION_MIXED context the inner sweeps run in
 *             complex64, two per pass of a temporally blocked transposed
 *             sweep (32 x 16 regions, the blocked forward sweep's z chunk),
 *             and the mean runs over the passes of one period,
 *             round(2 pi / (2 omega tau)); the defect, lam and the norms stay
 *             in FP64.
 *   tol <= 0  exactly max_it plain transposed iterations lam <- M^T lam + g
 *             from lam = 0 (check_every unused)
 *   grad_eps  device, 2*N doubles: (dJ/deps', dJ/deps'') per cell
 *   J, iters (transposed sweeps run), rel_res  host, may be NULL
 * Needs a context created with grid.adjoint = 1 (compact storage); the FP64
 * transposed sweep uses the fused tile and z chunk.  Synchronising. */
int thiim_adjoint_grad(thiim_ctx *ctx, const double *weight, double tol, int max_it,
                       int check_every, double *grad_eps, double *J, int *iters,
                       double *rel_res);

/* ---- auto-tuner ------------------------------------------------------- */

/* Chosen sweep configuration. */
typedef struct {
    int kernel;               /* THIIM_KERNEL_FUSED or THIIM_KERNEL_BLOCKED */
    int tile_x, tile_y;       /* fused tile or blocked region */
    int t_block;              /* iterations per pass (1 fused, 2 blocked) */
    int z_chunk;              /* planes per workgroup stream */
    double ms_per_iteration;  /* measured (of the configuration applied) */
    double model_ms;          /* modelled (see below) */
    int candidates, timed;    /* configurations considered / timed */
    /* thiim_batch_autotune: time per iteration of the batch with the best
     * single configuration for all problems (the one described above) and
     * with each grid's own thiim_autotune choice; per_grid = 1 when the
     * latter was faster and applied.  thiim_autotune: one_for_all_ms = the
     * measured time, per_grid_ms = 0, per_grid = 0. */
    double one_for_all_ms, per_grid_ms;
    int per_grid;
} thiim_tuning;

/* Picks the sweep configuration of thiim_iterate for this context: every
 * fused tile and blocked region crossed with z chunks (16 planes to nz, and
 * the round-quantisation choice of each geometry with its neighbours) is
 * scored by a traffic / capacity model (HBM bytes per cell with tile halos
 * and z-chunk overlap, stretched by the rounds of one-workgroup-per-CU that
 * the launch needs); the configurations within 1.3x of the best score (at
 * most 10) are timed over trial_iters iterations each, from the current
 * state into the spare buffer (the state does not advance), and the fastest
 * is kept.  All configurations give bit-identical iterates.
 * out may be NULL.  Synchronising. */
int thiim_autotune(thiim_ctx *ctx, int trial_iters, thiim_tuning *out);

/* Applies a sweep configuration chosen earlier (by thiim_autotune on a
 * context of the same grid, e.g. one kept in a tuner cache keyed by grid,
 * storage, precision and device) without timing anything: kernel FUSED or
 * BLOCKED, a tile / region that thiim_autotune can choose, 1 <= z_chunk <=
 * nz; the other fields are ignored.  All configurations give bit-identical
 * iterates.  THIIM_EINVAL on anything else (the context is unchanged). */
int thiim_apply_tuning(thiim_ctx *ctx, const thiim_tuning *tuning);

/* ---- batches ------------------------------------------------------------ */

/* A batch advances n contexts together: grids of any size (compact storage,
 * one common stream, each context's own sweep configuration).  Contexts with
 * the same configuration share one persistent launch per pass: the resident
 * workgroups take the concatenated tiles of all of them from a device work
 * queue (one counter per XCD; the last workgroup of a pass clears them for
 * the next).  The passes of each
 * 64 iterations are captured once in a HIP graph and replayed (eager
 * launches on the null stream, which cannot be captured).  A batch borrows
 * its contexts and a small device workspace (the per-launch item tables and
 * the queue counters); destroy it before them, and do not run two calls on
 * one batch at the same time. */
typedef struct thiim_batch thiim_batch;

int thiim_batch_workspace_bytes(int n, size_t *bytes);
int thiim_batch_create(thiim_ctx *const *ctxs, int n, void *workspace,
                       size_t workspace_bytes, thiim_batch **out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * batch as thiim_batch_create without a workspace.  Its item tables and
 * work-queue counters live in a static device array of the library (256 KiB
 * per device, held until the process ends), so n <= 128 (THIIM_EINVAL
 * beyond).  All contexts must be on one device; the first call on a device
 * looks up the array's address there.  One such batch per device at a time:
 * the array keeps the last batch's tables (re-uploaded by every new batch;
 * the queue counters are zeroed when the batch is made and every pass leaves
 * them zero), so a second call on a device
 * whose static batch is still alive fails with THIIM_EINVAL; destroy the
 * first (thiim_batch_destroy, which then waits for the batch's stream).
 * Calls on one batch from several threads at once race, as for any batch.
 * No device memory is allocated or freed. */
int thiim_batch_create_static(thiim_ctx *const *ctxs, int n, thiim_batch **out);

/* n iterations of every context.  Asynchronous (uploads the item tables, a
 * synchronising copy, when the batch changed). */
int thiim_batch_iterate(thiim_batch *batch, int n);

/* thiim_residual of every context into rel_res[n].  Synchronising. */
int thiim_batch_residual(thiim_batch *batch, double *rel_res);

/* Iterates all contexts, checking every check_every iterations, and stops
 * advancing each one as soon as its residual is <= tol; iters[i] and
 * rel_res[i] (may be NULL) receive its iteration count and final residual.
 * THIIM_ENOTCONV if any context reached max_it first.  Synchronising.
 * When every context was created with THIIM_PRECISION_MIXED, this runs the
 * mixed-precision solver of thiim_solve for all of them at once: per step,
 * each active problem's FP64 residual sweep, then the complex64 inner passes
 * of all problems with the same T as one batched launch per pass (captured
 * in a HIP graph per active set), each problem averaging its own window;
 * check_every = inner sweeps per step (0: adaptive, driven by the slowest
 * problem); iters[i] counts sweeps as thiim_solve does.  Contexts may not
 * mix the two precisions. */
int thiim_batch_solve(thiim_batch *batch, double tol, int max_it, int check_every,
                      int *iters, double *rel_res);

/* Picks the sweep configurations of the batch by timing the batched passes
 * themselves (trial passes from the current states into the spare buffers,
 * so the states do not advance), two ways, and keeps the faster: one
 * configuration for every problem (blocked regions 32x16, 64x8, 64x6 and
 * fused tiles 64x8, 32x8, with each problem's automatic z chunk or a fixed
 * one), and per grid shape the choice of thiim_autotune on one problem of
 * that shape alone.  In a batch the launch is filled by all problems
 * together, so the two can differ.  out describes the best single
 * configuration (z_chunk = 0: each problem's automatic chunk) and both
 * timings.  out may be NULL.  Synchronising. */
int thiim_batch_autotune(thiim_batch *batch, int trial_iters, thiim_tuning *out);

void thiim_batch_destroy(thiim_batch *batch);

/* Device-to-device copies of the 12 split fields, one buffer of 12*2*N
 * doubles in component order.  get: synchronising. */
int thiim_get_fields(thiim_ctx *ctx, double *dst);
int thiim_set_fields(thiim_ctx *ctx, const double *src);

/* Device copy of the 28 coefficient arrays (28*2*N doubles), expanded from
 * the compact storage when that is in use.  Synchronising. */
int thiim_get_coeffs(thiim_ctx *ctx, double *dst);

/* ---- measurement ------------------------------------------------------- */

/* Streaming probe of the practical HBM bandwidth, with the sweeps' access
 * forms (16-byte buffer loads, non-temporal 16-byte stores) and no THIIM
 * arithmetic: nin input arrays of n complex128 values at src (array stride
 * `stride` values) and nout output arrays at dst (same stride);
 * out_j = in_j for j < nout, the inputs beyond nout added into out_0.
 * (nin, nout) = (1, 1) is a plain copy, (13, 12) streams the arrays of one
 * compact-storage sweep pass (eps and 12 fields in, 12 fields out).  Device
 * buffers, 16-byte aligned, each array under 4 GiB.  Enqueued on `stream`
 * (a hipStream_t); asynchronous. */
int thiim_stream_probe(const double *src, double *dst, long long n, long long stride, int nin,
                       int nout, void *stream);

/* Iterations done since create / set_fields. */
int thiim_iterations(const thiim_ctx *ctx, long long *n);

/* Releases the context (not the workspace).  NULL is allowed. */
void thiim_destroy(thiim_ctx *ctx);

/* Message of the calling thread's last failure ("" if none). */
const char *thiim_last_error(void);

/* Name of a status code. */
const char *thiim_status_str(int status);

#ifdef __cplusplus
}
#endif

#endif /* THIIM_H */
