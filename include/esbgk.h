/*
 * esbgk.h -- C ABI of the MI355X kinetic IMEX engine for the 2D-space /
 * 2D-velocity ES-BGK equation with a coupled Euler / ES-BGK domain
 * decomposition (Caparello & Tenna, arXiv 2512.03586).
 *
 * The engine advances the coupled system of Sec. 3 with Algorithm 1
 * ("High-order Domain Decomposition Method for the ES-BGK Equation"): each
 * step runs the regime update of Sec. 3.1.2, then the IMEX Runge-Kutta stages
 * (eqs. RKEI1-RKEI2 for the kinetic cells, eqs. RKEuler-RKEuler_2 for the
 * fluid cells), coupling the two models after every stage (Sec. 3.3, Remark
 * rem_coupling), and the final update.
 *
 * Conventions for every entry point:
 *  - Grid: nx * ny cells on the periodic box [0,lx] x [0,ly] (Sec. 3.2), cell
 *    index c = i + nx*j.  Velocity grid: nv nodes per direction on
 *    [-vmax, vmax], midpoint nodes v_a = -vmax + (a + 1/2) dv, dv = 2 vmax/nv,
 *    node index k = a + nv*b (x-velocity fastest).  nv must be a multiple of 4,
 *    4 <= nv <= 64.
 *  - "Device pointer" means memory on the GPU the context was created on,
 *    owned by the caller; the library only reads / writes it in the order of
 *    the given stream.  Host pointers are named as such.
 *  - Streams are passed as `void *` and are hipStream_t handles (NULL = the
 *    default stream).  Every call is asynchronous on its stream unless it says
 *    it synchronizes.
 *  - The library never allocates device memory: all state lives in the
 *    workspace the caller hands to esbgk_create().
 *  - Return codes: ESBGK_OK, or a negative error (below).  esbgk_last_error()
 *    returns a thread-local message for the last failing call.  No C++
 *    exception crosses this interface.  A context is used from one host thread
 *    and one stream at a time.
 */
#ifndef ESBGK_H
#define ESBGK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes */
#define ESBGK_OK 0
#define ESBGK_EINVAL (-1)    /* null / misaligned pointer, bad size, non-physical input */
#define ESBGK_ENOMEM (-2)    /* workspace too small */
#define ESBGK_EDEVICE (-3)   /* a HIP call failed */
#define ESBGK_ENONPHYS (-4)  /* a step met rho <= 0, T <= 0, a non-SPD ES tensor or NaN */

/* ---- enumerations of esbgk_config fields */
enum { ESBGK_ARS222 = 0, ESBGK_ARS233 = 1 };                  /* scheme */
enum { ESBGK_UPWIND1 = 0, ESBGK_MINMOD2 = 1 };                /* recon */
enum { ESBGK_FP64 = 0, ESBGK_FP32 = 1, ESBGK_BF16 = 2, ESBGK_MIXED = 3 }; /* precision of f */
enum { ESBGK_IND_PLAIN = 0, ESBGK_IND_FROZEN = 1, ESBGK_IND_LEARNED = 2 }; /* indicator */
enum { ESBGK_COUPLE_STAGE = 0, ESBGK_COUPLE_STEP = 1 };       /* coupling */

/*
 * Problem definition.
 *  scheme      IMEX tableau: ARS(2,3,3) as printed in Sec. 3.4.2, or
 *              ARS(2,2,2) (the second-order member of the same family).
 *  recon       transport / Euler reconstruction: piecewise constant (upwind)
 *              or minmod-limited piecewise linear; upwind flux for the
 *              kinetic transport (the Lax-Friedrichs flux of Sec. 3.2 with
 *              dissipation |v|), Rusanov flux for Euler.
 *  precision   storage and arithmetic of f: FP64; FP32; BF16 storage with
 *              FP32 arithmetic; or MIXED: the state f^n in FP32, FP32
 *              arithmetic, and 16-bit storage of two increments, f^(2) - f^n
 *              and P - f^(3) (P the partial sum of the final combination,
 *              implicit term of the last stage included; f^(3) kept in FP32),
 *              ARS(2,3,3) only.  FP32 velocity sums are compensated.  The
 *              implicit term of an earlier stage enters the stage sums as
 *              (f^(j) - f*_j)/(dt a_jj), equal to (tau/eps)(Ghat_j - f^(j))
 *              for the exact relaxation, except with 16-bit stage arrays,
 *              which re-evaluate Ghat_j.  Per-cell
 *              quantities are FP64 always, and so are the 2x2 ES-tensor
 *              algebra and the 6x6 conservation solve.
 *  indicator   PLAIN: the breakdown criteria of Sec. 3.1.2 every step;
 *              FROZEN: the partition set by esbgk_set_mask() is kept (as in
 *              the order-of-accuracy test, Sec. 4.1.1); LEARNED: the MLP
 *              predictor between plain checks every learned_k steps.
 *  ce_set      0 = the paper's Chapman-Enskog constants (2/3, 5/2, 2/3),
 *              1 = the 2D-consistent set (1, 2, 1).
 *  correction  1 = six-moment discrete-conservation correction of the
 *              sampled Gaussian (exact discrete conservation), 0 = none.
 *  coupling    STAGE = Algorithm 1; STEP = low-order coupling (LOC).
 *  beta        ES-BGK parameter (Pr = 1/(1-beta)); tau the relaxation
 *              constant (rate tau/eps); dt > 0 fixed step, else
 *              dt = cfl * min(dx, dy) / vmax; eta, delta the thresholds of
 *              criteria crit:CompEuler and eqKintoFluid1.
 */
typedef struct esbgk_config {
    int32_t nx, ny, nv;
    int32_t scheme, recon, precision, indicator, ce_set, correction, coupling;
    int32_t learned_k;
    int32_t reserved;
    double lx, ly, vmax;
    double beta, tau, cfl, dt;
    double eta, delta;
} esbgk_config;

typedef struct esbgk_ctx esbgk_ctx;

/* Host-side diagnostics, filled by esbgk_get_stats(). */
typedef struct esbgk_stats {
    int64_t steps;          /* steps taken since the last esbgk_set_state() */
    double time;            /* simulated time */
    double dt;              /* step used */
    int32_t n_kinetic;      /* kinetic cells after the last regime update */
    int32_t n_buffer;       /* fluid cells inside a kinetic stencil */
    int32_t error_flags;    /* bit 0 rho<=0, bit 1 T<=0, bit 2 ES tensor not SPD, bit 3 NaN */
    int32_t reserved;
    int64_t kinetic_cell_steps; /* sum over steps of the kinetic-cell count */
} esbgk_stats;

/* Kernel classes timed by esbgk_kernel_times(). */
enum { ESBGK_K_STAGE2 = 0, ESBGK_K_STAGE3 = 1, ESBGK_K_FINAL = 2, ESBGK_K_FILL = 3, ESBGK_K_COUNT = 4 };

/* Bytes of device workspace a context with this configuration needs (f
 * buffers, per-cell arrays, lists).  Pure function of cfg; EINVAL on a bad
 * configuration. */
int esbgk_workspace_size(const esbgk_config *cfg, size_t *bytes);

/* Create a context on the current HIP device.  d_workspace: device pointer,
 * 256-byte aligned, at least esbgk_workspace_size() bytes, owned by the caller
 * and kept alive until esbgk_destroy().  cfg is copied.  ENOMEM if bytes is
 * too small, EINVAL for a bad configuration. */
int esbgk_create(const esbgk_config *cfg, void *d_workspace, size_t bytes, esbgk_ctx **out);

/* Destroy the host-side context (the workspace is not freed). */
void esbgk_destroy(esbgk_ctx *ctx);

/* Message of the last failing call on this host thread ("" if none). */
const char *esbgk_last_error(void);

/* Initial macroscopic state (Sec. 4: every test starts from moments).
 * d_rho, d_ux, d_uy, d_T, d_eps: device FP64 arrays of nc = nx*ny values
 * (density, velocity, temperature, local Knudsen number eps > 0).  Sets
 * U = (rho, rho u, rho|u|^2/2 + rho T), t = 0 and, as in the paper's tests,
 * an all-fluid partition; cells become kinetic at the first regime update and
 * then receive f = Mhat(U) (eq. Coupling_FluKin).  Validates finiteness and
 * rho > 0, T > 0, eps > 0 (synchronizes on the stream to do so; EINVAL). */
int esbgk_set_state(esbgk_ctx *ctx, const double *d_rho, const double *d_ux, const double *d_uy,
                    const double *d_T, const double *d_eps, void *stream);

/* Set the partition (device uint8, nc values, 1 = kinetic).  Cells turning
 * kinetic receive f = Mhat(U); cells turning fluid keep U = moments(f). */
int esbgk_set_mask(esbgk_ctx *ctx, const uint8_t *d_mask, void *stream);

/* Set the full phase-space state: d_f device FP64 [nc][nv*nv]; every cell
 * becomes kinetic and takes U = moments(f) (eq. Coupling_KinFlu). Requires a
 * prior esbgk_set_state() (for eps). */
int esbgk_set_f(esbgk_ctx *ctx, const double *d_f, void *stream);

/* Advance nsteps steps of Algorithm 1 (asynchronous). */
int esbgk_step(esbgk_ctx *ctx, int nsteps, void *stream);

/* Cell moments at the current time: device FP64 arrays of nc values.  For
 * kinetic cells they are the moments of f (H3), for fluid cells the Euler
 * state.  Any output pointer may be NULL. */
int esbgk_get_moments(esbgk_ctx *ctx, double *d_rho, double *d_ux, double *d_uy, double *d_T,
                      void *stream);

/* Conserved variables, device FP64 SoA [4][nc] = (rho, rho ux, rho uy, E). */
int esbgk_get_conserved(esbgk_ctx *ctx, double *d_U, void *stream);

/* Current partition, device uint8 [nc], 1 = kinetic. */
int esbgk_get_mask(esbgk_ctx *ctx, uint8_t *d_mask, void *stream);

/* Distribution function, device FP64 [nc][nv*nv] (converted from the storage
 * precision).  Only kinetic cells hold meaningful values. */
int esbgk_get_f(esbgk_ctx *ctx, double *d_f, void *stream);

/* L1 distance of eq. eqKintoFluid1 of each kinetic cell at the current time,
 * device FP64 [nc] (0 for fluid cells); the regime update reads these. */
int esbgk_get_l1(esbgk_ctx *ctx, double *d_l1, void *stream);

/* Kinetic-cell list of the last regime update, in the engine's processing
 * order (8x8 cell tiles, row-major inside a tile, tiles row-major).
 * d_cells device int32 [nc]; h_count host int32 receives the count.
 * Synchronizes on the stream. */
int esbgk_get_kinetic_cells(esbgk_ctx *ctx, int32_t *d_cells, int32_t *h_count, void *stream);

/* Diagnostics (synchronizes on the stream).  Returns ENONPHYS when the
 * device error flag is set. */
int esbgk_get_stats(esbgk_ctx *ctx, esbgk_stats *h_out, void *stream);

/* Kernel timing for measurement: while enabled, every launch of the kernel
 * classes above is bracketed by HIP events on its stream (host-side event
 * objects; no device memory).  esbgk_kernel_times() synchronizes, and fills
 * h_ms[ESBGK_K_COUNT] with the summed durations (milliseconds) and
 * h_launches[ESBGK_K_COUNT] with the launch counts since the last reset. */
int esbgk_set_timing(esbgk_ctx *ctx, int enable);
int esbgk_kernel_times(esbgk_ctx *ctx, double *h_ms, int64_t *h_launches, int reset);

/* Stateless regime indicator, the same device code the step runs
 * (Sec. 3.1.2, criterion crit:CompEuler, Remark, eq. eqKintoFluid1):
 *   lambda = largest |eigenvalue| of S_1 - I from central differences of
 *   (ux, uy, T), mask_new = (lambda > eta) || (mask_old && l1 > delta).
 * d_prim device FP64 SoA [4][nc] = (rho, ux, uy, T); d_eps, d_l1 FP64 [nc];
 * d_mask_old, d_mask_new uint8 [nc]; d_lambda FP64 [nc] (may be NULL).
 * Uses cfg's grid, beta, tau, ce_set, eta, delta.  Every operation is a
 * correctly rounded IEEE double operation in a fixed order (no contraction). */
int esbgk_indicator(const esbgk_config *cfg, const double *d_prim, const double *d_eps,
                    const double *d_l1, const uint8_t *d_mask_old, uint8_t *d_mask_new,
                    double *d_lambda, void *stream);

/* ====================================================================
 * Learned regime indicator (an addition to the paper's method; it has no
 * counterpart there).  A network predicts, from the macroscopic state at the
 * start of a step, which cells the plain criterion of Sec. 3.1.2 marks
 * kinetic at any of the next K = learned_k steps.  With indicator = LEARNED
 * the engine runs the plain criterion P only every K steps (the fallback and
 * the judge of the prediction) and keeps the mask P | prediction for the next
 * K steps, so that the regime update, the compaction and the fluid -> kinetic
 * fills run once per K steps.
 *
 * Features of a cell (192 BF16 values): over its periodic 5 x 5 stencil
 * (k = 5 (dj + 2) + (di + 2)), for stencil cell s and centre c,
 *   x[7k+0] = rho_s/rho_c - 1, x[7k+1] = ux_s - ux_c, x[7k+2] = uy_s - uy_c,
 *   x[7k+3] = T_s/T_c - 1, x[7k+4] = eps_s/(eps_s + 0.01),
 *   x[7k+5] = A_s/(A_s + 1e-4) with A = eps^2 |grad u|^2,
 *   x[7k+6] = B_s/(B_s + 1e-4) with B = eps^2 |grad T|^2 / T,
 *   x[175] = the mask in use at c, x[176..191] = 0
 * (central differences; FP64 + - * / in a fixed order, rounded FP32 -> BF16).
 * Network: z = w3 . relu(W2^T relu(W1^T x + b1) + b2) + b3, 64 and 64 hidden
 * units, weights used in BF16, biases in FP32, hidden activations stored in
 * BF16, FP32 accumulation on the matrix cores.  Parameters travel as one flat
 * FP32 vector of esbgk_mlp_param_count() values: W1 [192][64] (row = input),
 * b1 [64], W2 [64][64], b2 [64], w3 [64], b3.  Training minimizes the mean
 * weighted logistic loss w_pos y softplus(-z) + (1 - y) softplus(z) with
 * bias-corrected Adam (beta1 0.9, beta2 0.999, eps 1e-8).
 * ==================================================================== */

typedef struct esbgk_mlp esbgk_mlp;

/* Number of parameters (16577). */
int esbgk_mlp_param_count(void);

/* Device bytes for a network that trains on batches of up to max_batch
 * samples (parameters, Adam moments, BF16 copies, gradient partials). */
int esbgk_mlp_workspace_size(int max_batch, size_t *bytes);

/* Create a network in the caller's device workspace (256-byte aligned, kept
 * alive until esbgk_mlp_destroy()).  Weights are undefined until
 * esbgk_mlp_set_weights(). */
int esbgk_mlp_create(int max_batch, void *d_workspace, size_t bytes, esbgk_mlp **out);
void esbgk_mlp_destroy(esbgk_mlp *net);
const char *esbgk_mlp_last_error(void);

/* Load / read the flat FP32 parameter vector (device pointers).  Loading
 * resets the Adam state. */
int esbgk_mlp_set_weights(esbgk_mlp *net, const float *d_params, void *stream);
int esbgk_mlp_get_weights(esbgk_mlp *net, float *d_params, void *stream);

/* Per-cell derived fields of nsnap snapshots on an nx x ny periodic grid of
 * size lx x ly.  d_fields: device FP64 [nsnap][6][nx*ny] = (rho, ux, uy, T,
 * eps, mask in use as 0.0 / 1.0); d_derived: device FP64 [nsnap][3][nx*ny]
 * (eps/(eps+0.01), A/(A+1e-4), B/(B+1e-4)). */
int esbgk_mlp_derived(int nx, int ny, double lx, double ly, const double *d_fields, int nsnap,
                      double *d_derived, void *stream);

/* Feature rows of n samples of nsnap snapshots: d_samples device int32
 * [n][2] = (snapshot, cell); d_X device [n][192] BF16 bit patterns.  A
 * sample outside [0, nsnap) x [0, nx*ny) gets a row of zeros. */
int esbgk_mlp_features(int nx, int ny, const double *d_fields, const double *d_derived, int nsnap,
                       const int32_t *d_samples, int n, uint16_t *d_X, void *stream);

/* Logits of n feature rows (device FP32 [n]); any n >= 0. */
int esbgk_mlp_forward(esbgk_mlp *net, const uint16_t *d_X, int n, float *d_logits, void *stream);

/* Gradient of the mean weighted logistic loss over n <= max_batch samples
 * (labels d_y device FP32 [n], 0 or 1) with respect to the parameters,
 * written to d_grad (device FP32, flat order); d_loss (device FP32, may be
 * NULL) receives the loss.  Deterministic (fixed reduction order). */
int esbgk_mlp_gradients(esbgk_mlp *net, const uint16_t *d_X, const float *d_y, int n, float w_pos,
                        float *d_grad, float *d_loss, void *stream);

/* One Adam step on the same gradient (learning rate lr > 0). */
int esbgk_mlp_train_step(esbgk_mlp *net, const uint16_t *d_X, const float *d_y, int n, float w_pos,
                         float lr, float *d_loss, void *stream);

/* Attach the predictor to a context configured with indicator = LEARNED:
 * mask = P | (logit > threshold) at every check step.  With net = NULL the
 * mask is P dilated by `dilation` cells along x and y (Chebyshev distance),
 * the plain-every-K baseline.  The network must outlive its use. */
int esbgk_set_learned(esbgk_ctx *ctx, esbgk_mlp *net, float threshold, int dilation);

/* Judge counters of the learned indicator since esbgk_set_state(), summed
 * over the check steps after the first: h_out[0] checks, h_out[1] cells
 * with P = 1 outside the mask that was in use (missed), h_out[2] cells in
 * the mask in use with P = 0 (extra), h_out[3] cells with P = 1.
 * Synchronizes on the stream. */
int esbgk_get_learned_stats(esbgk_ctx *ctx, int64_t *h_out, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* ESBGK_H */
