/*
 * mbh.h -- C ABI of libmbh, the MI355X (gfx950) batched LISA massive-black-
 * hole-binary log-likelihood of Katz, Marsat, Chua, Babak & Larson (2020),
 * arXiv:2005.01827.
 *
 * The library evaluates, for a batch of walkers, -ln L = 1/2 <d-h|d-h>
 * summed over the TDI channels A, E, T (Sec. II, Eqs. NLL, innerprod,
 * innerprodsum), where the template h is built as in Sec. II.A: harmonic-mode
 * amplitude and phase on a sparse frequency grid (Eq. amp_and_phase), the
 * time-frequency map t_lm(f) (Eq. t_f) with the t < 0 cut, the Fourier-domain
 * LISA response (Eq. response and the A, E, T combinations), cubic-spline
 * interpolation onto the dense grid f_k = k df, and a noise-weighted inner
 * product with the data.  The data and PSD are uploaded once per context
 * (Sec. II.A: done once before sampling).
 *
 * Conventions shared by all entry points
 *   - Pointers named *_dev are device pointers (hipMalloc'd or torch CUDA
 *     tensors); *_host pointers are host memory.  The caller owns every
 *     buffer it passes; the context owns its device copies and workspaces.
 *   - 'stream' is a hipStream_t passed as void* (NULL = the null stream).
 *     Calls are asynchronous on that stream unless stated otherwise.  A
 *     context must not be used from two host threads or two streams at the
 *     same time.
 *   - Calls never abort.  They return an mbh_status; mbh_last_error() gives
 *     the message of the last failure on that context.
 *   - A walker whose parameters are physically invalid (q outside (0,1],
 *     |a_i| > 0.99, M_T <= 0, D_L <= 0, any NaN/inf) or whose template has
 *     no active mode gets ln L = -inf (resp. the data-only value) with
 *     status MBH_OK, so that a sampler simply rejects it.
 *
 * Parameters: params[B][11] float64, in the paper's order (Sec. II):
 *   M_T [Msun, detector frame], q = m2/m1 in (0,1], a1, a2 (aligned spins,
 *   a1 of the heavier body), D_L [Gpc], phi_ref, iota, lambda, beta, psi
 *   (SSB frame, radians), t_ref [s]; t_coal = t0 + t_ref.
 */
#ifndef MBH_H
#define MBH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mbh_ctx mbh_ctx;

typedef enum {
    MBH_OK = 0,
    MBH_EINVAL = -1,  /* bad argument: null pointer, size, mode list, layout */
    MBH_ENOMEM = -2,  /* device or host allocation failed                  */
    MBH_EHIP = -3,    /* a HIP runtime call failed                          */
    MBH_EBATCH = -4   /* B > max_batch of the context                       */
} mbh_status;

typedef enum {
    MBH_FP64 = 0,     /* whole path in double precision                     */
    MBH_FP32C = 1     /* dense stage: FP64 phase, FP32 template, residual d - h
                         formed and summed in float-float against the whitened
                         data held as an FP32 pair (about 48 bits)           */
} mbh_precision;

typedef struct {
    double df;             /* 1/T_obs [Hz]; dense bins f_k = k df                  */
    int64_t k0;            /* first dense bin (k0 >= 1)                            */
    int64_t n;             /* number of dense bins; k0 + n <= 2^31                 */
    const double *data;    /* host, [3][n][2]: A, E, T complex128 interleaved      */
    const double *psd;     /* host, [3][n]: one-sided S_n of A, E, T (all > 0)     */
    int n_modes;           /* 1..6                                                 */
    int modes[6][2];       /* (l,m) subset of (2,2),(3,3),(4,4),(2,1),(3,2),(4,3)  */
    int n_sparse;          /* sparse knots per mode, 8..1024 (256 in the configs)  */
    double t0;             /* [s]; t_coal = t0 + t_ref                             */
    int precision;         /* mbh_precision                                        */
    int max_batch;         /* largest B any call on this context will use          */
} mbh_ctx_desc;

/* Create a context: validates the descriptor, allocates device memory for
 * the data, the weights 4 df / S_n, the per-channel prefix sums of
 * 4 df |d|^2 / S_n and all per-walker workspaces for max_batch walkers, and
 * uploads the data (Sec. II.A: data and PSD are transferred once).
 * Synchronous.  On failure *out is NULL and nothing is leaked. */
mbh_status mbh_ctx_create(const mbh_ctx_desc *desc, mbh_ctx **out);

/* Free every resource of the context (NULL is allowed). Synchronous. */
void mbh_ctx_destroy(mbh_ctx *ctx);

/* Message of the last failure on ctx (static text if ctx is NULL). */
const char *mbh_last_error(const mbh_ctx *ctx);

/* Sec. II (11-parameter list, Eq. amp_and_phase, Eq. t_f): per walker, the
 * physical constants; per mode, the frequency support [f_start, f_end] from
 * the root of t_lm(f) = 0 and the ringdown cut; the sparse log-spaced knots
 * and A_lm, phi_lm, t_lm at them.  params_dev: device [B][11]. Results stay
 * in the context workspace. */
mbh_status mbh_waveform_gen(mbh_ctx *ctx, const double *params_dev, int B, void *stream);

/* Sec. II (Eq. response, A/E/T from X/Y/Z) and Sec. II.A (spline setup):
 * T^{A,E,T}_lm(f_j, t_lm(f_j)) at every knot, the orbital delay phase folded
 * into the phase, then not-a-knot cubic-spline coefficients of the eight
 * real functions per mode.  Requires a preceding mbh_waveform_gen with the
 * same B on the same stream: MBH_EINVAL (nothing launched) otherwise. */
mbh_status mbh_response(mbh_ctx *ctx, int B, void *stream);

/* Sec. II.A (dense interpolation) and Eqs. NLL, innerprod, innerprodsum:
 * interpolate every mode onto the dense bins of its band, sum modes per
 * channel, and reduce, per walker, out7_dev[B][7] = {ln L, <d|h>_A, <d|h>_E,
 * <d|h>_T, <h|h>_A, <h|h>_E, <h|h>_T} (device).  The reduction is
 * deterministic (fixed order, no floating-point atomics).  Requires that
 * the last call to fill the workspace was mbh_response, mbh_loglike_batch,
 * mbh_autotune or mbh_set_sparse with the same B (or mbh_template, B = 1) on
 * the same stream: MBH_EINVAL (nothing launched) otherwise.  B = 0 is a no-op. */
mbh_status mbh_interp_and_inner(mbh_ctx *ctx, int B, double *out7_dev, void *stream);

/* The three stages above in one call, launched as one captured HIP graph per
 * batch size after the first call: logL_dev[B] (device) receives ln L.  The
 * graph reads params_dev and writes logL_dev directly (its first and last
 * kernels are pointed at the caller's buffers before each launch), so both
 * buffers must stay valid until the work on 'stream' has completed.  On
 * the FP64 path the dense stage accumulates only the residual sums here (ln L
 * needs nothing else), so ln L is bitwise the value mbh_interp_and_inner
 * returns. */
mbh_status mbh_loglike_batch(mbh_ctx *ctx, const double *params_dev, int B, double *logL_dev, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * stages and kernels as mbh_loglike_batch, launched directly on 'stream'
 * (no graph, no events), with every per-call workspace (sparse stage, spline
 * coefficients, work-item lists, counters, partial sums) taken from one
 * fixed 64 MiB device array per GPU that the library holds until the
 * process ends, instead of the context's workspace.  The call allocates and
 * frees nothing.  params_dev[B][11] and logL_dev[B] are device buffers of
 * the caller; ln L is bitwise the value mbh_loglike_batch returns.
 * Limits: B <= max_batch, and the workspace of B walkers (about 0.55 MB per
 * walker with 6 modes, 256 knots and the 2^25-s grid, so about 100 walkers;
 * more for fewer modes, knots or bins) must fit in 64 MiB: MBH_EBATCH with
 * the required size in mbh_last_error otherwise.  MBH_EINVAL if the
 * context's device is not the current one; MBH_EHIP if the array's device
 * address could not be taken when the context was created.
 * All calls on one GPU share the array, whatever their context: calls
 * that overlap in time on one GPU (two streams, two host threads) race and
 * give wrong results; serialize them.  The array keeps the last call's
 * contents; the call writes every value before reading it. */
mbh_status mbh_loglike_batch_noalloc(mbh_ctx *ctx, const double *params_dev, int B, double *logL_dev, void *stream);

/* Dense template of one walker on the context's grid, h_dev[3][n][2]
 * (device, complex128 interleaved), built by the same kernels as the
 * likelihood.  Used to synthesise injections on the device. */
mbh_status mbh_template(mbh_ctx *ctx, const double *params_dev, double *h_dev, void *stream);

/* Copy the sparse stage of walker w (after mbh_response) to host buffers;
 * any pointer may be NULL.  band_host[nm][4] = {active, klo, khi, 0};
 * fband_host[nm][2] = {f_start, f_end}; f_host[nm][ns] knots;
 * fn_host[nm][8][ns] = A, phi, Re/Im T^A, Re/Im T^E, Re/Im T^T;
 * coef_host[nm][8][ns-1][4], the cubic of interval i in powers of f - f_i
 * (c0 + c1 (f - f_i) + c2 (f - f_i)^2 + c3 (f - f_i)^3).  Synchronous on
 * 'stream'. */
mbh_status mbh_get_sparse(mbh_ctx *ctx, int w, int64_t *band_host, double *fband_host, double *f_host,
                          double *fn_host, double *coef_host, void *stream);

/* Replace the sparse stage of walkers 0..B-1 with caller-supplied knots and
 * knot values (host, same layouts as mbh_get_sparse) and recompute the spline
 * coefficients on the device; a following mbh_interp_and_inner evaluates
 * exactly those functions.  Lets the dense stage be checked in isolation.
 * Synchronous on 'stream'. */
mbh_status mbh_set_sparse(mbh_ctx *ctx, int B, const int64_t *band_host, const double *fband_host,
                          const double *f_host, const double *fn_host, void *stream);

/* Kernel timing for measurement.  With on != 0, mbh_loglike_batch launches
 * its kernels directly (the same kernels and launch shapes as the captured
 * graph) and brackets the dense interpolation + inner-product kernel with HIP
 * events on the caller's stream.  mbh_get_timing synchronizes on those
 * events and returns the summed dense-kernel time [ms] and the number of
 * timed launches since the last mbh_set_timing call; outputs may be NULL. */
mbh_status mbh_set_timing(mbh_ctx *ctx, int on);
mbh_status mbh_get_timing(mbh_ctx *ctx, double *dense_ms_total, int64_t *count);

/* Launch shape of the dense interpolation + inner-product kernel (the
 * batching over sources of Sec. II.A).  blocks_per_cu (1..32) workgroups per
 * compute unit take (walker, tile) work items from a counter (a tile is 512
 * to 8192 bins, chosen per context); with one_per_walker != 0 each walker's
 * tiles go to one workgroup instead (an unbalanced reference schedule for
 * load-balance measurements).
 * ln L is bitwise identical under every shape.  Drops the context's captured
 * graphs.  Synchronous.  Default: 8 blocks per CU, tiled. */
mbh_status mbh_set_schedule(mbh_ctx *ctx, int blocks_per_cu, int one_per_walker);
mbh_status mbh_get_schedule(const mbh_ctx *ctx, int *blocks_per_cu, int *one_per_walker);

/* Autotuner: run the sparse stages once for params_dev[B][11] (device,
 * 1 <= B <= max_batch), time the dense kernel with HIP events for every
 * blocks_per_cu in {2, 3, 4, 6, 8, 9, 12, 16, 24, 32} (median of reps in
 * 1..100 launches), and keep the fastest as the context's tiled schedule.
 * best_bpc_host and best_ms_host (may be NULL) receive the choice and its
 * median time [ms].
 * Synchronous on 'stream'. */
mbh_status mbh_autotune(mbh_ctx *ctx, const double *params_dev, int B, int reps, int *best_bpc_host,
                        double *best_ms_host, void *stream);

/* ------------------------------------------------------------------------
 * Learned proposal for the sampler: an affine-coupling normalizing flow (a
 * density q(u) that can be both sampled and evaluated), used as the
 * independence proposal of a Metropolis-Hastings step next to the stretch
 * move of Sec. III.A.  FP32, on standardized sampling coordinates u.
 *
 * Layer l (0..L-1) reorders the dim coordinates by a permutation
 * perm[l][0..dim); the first nc[l] reordered coordinates (nc = ceil(dim/2)
 * for even l, floor(dim/2) for odd l) pass through unchanged and condition
 * an MLP  nc -> H (tanh) -> H (tanh) -> 2 nt  (nt = dim - nc) whose output o
 * gives s = tanh(o[0..nt)) and t = o[nt..2nt); the other nt reordered
 * coordinates map as y = x exp(s) + t.  z = f(u) after L layers and
 *   log q(u) = -|z|^2/2 - (dim/2) ln(2 pi) + sum_l sum_j s_lj.
 * Parameters are one flat FP32 array, per layer in this order, each linear
 * map stored input-major (W[i][j] multiplies input i into output j):
 *   W1[nc][H], b1[H], W2[H][H], b2[H], W3[H][2 nt], b3[2 nt].
 * Limits: 2 <= dim <= 32, 1 <= L <= 32, 16 <= H <= 256, 1 <= max_batch <= 2^20.
 * Device arrays are FP32 and row-major: u, z [n][dim], logq [n].
 * ------------------------------------------------------------------------ */
typedef struct mbh_flow mbh_flow;

/* Create a flow for batches of up to max_batch rows.  perm_host[L][dim]
 * (host; each row a permutation of 0..dim-1) fixes the coordinate order of
 * every layer; NULL draws the permutations from 'seed'.  Initial weights are
 * drawn from 'seed' (uniform, scale 1/sqrt(fan-in)) except W3 and b3, which
 * start at zero so that the initial flow is the identity map.  Synchronous;
 * on failure *out is NULL and nothing is leaked.  EINVAL also if one
 * layer's small weights (W1, b1, b2, W3, b3) and two hidden activations of
 * 16 rows do not fit the current device's LDS per workgroup (about 87 KB at
 * dim = 32, H = 256; under 64 KB for every dim up to H = 160). */
mbh_status mbh_flow_create(int dim, int n_layers, int hidden, int max_batch, const int *perm_host, uint64_t seed,
                           mbh_flow **out);
void mbh_flow_destroy(mbh_flow *flow);
/* Message of the last failure on the flow (static text if flow is NULL). */
const char *mbh_flow_last_error(const mbh_flow *flow);
/* Length of the flat parameter array (-1 if flow is NULL). */
int64_t mbh_flow_num_params(const mbh_flow *flow);
/* perm_host[L][dim] and nc_host[L] (host); either may be NULL. */
mbh_status mbh_flow_get_layout(const mbh_flow *flow, int *perm_host, int *nc_host);
/* Copy the flat parameter array to / from host memory.  set_params also
 * clears the Adam moments and step count.  Synchronous. */
mbh_status mbh_flow_get_params(mbh_flow *flow, float *params_host);
mbh_status mbh_flow_set_params(mbh_flow *flow, const float *params_host);
/* z_dev = f(u_dev) and logq_dev = log q(u_dev) for n <= max_batch rows
 * (logq_dev may be NULL; z_dev may not alias u_dev). */
mbh_status mbh_flow_forward(mbh_flow *flow, const float *u_dev, int n, float *z_dev, float *logq_dev, void *stream);
/* u_dev = f^{-1}(z_dev) and logq_dev = log q(u_dev) (may be NULL): with
 * z ~ N(0, I) this draws u ~ q. */
mbh_status mbh_flow_inverse(mbh_flow *flow, const float *z_dev, int n, float *u_dev, float *logq_dev, void *stream);
/* Training loss  -(1/n) sum_i log q(u_i)  (host, double) and its gradient
 * with respect to the flat parameters (grad_host, may be NULL).  The
 * gradient stays on the device for mbh_flow_adam.  Every reduction runs in
 * a fixed order, so results are bitwise reproducible.  Synchronous. */
mbh_status mbh_flow_loss_grad(mbh_flow *flow, const float *u_dev, int n, double *loss_host, float *grad_host,
                              void *stream);
/* One Adam step (beta1 = 0.9, beta2 = 0.999, eps = 1e-8, bias-corrected)
 * on the gradient of the last mbh_flow_loss_grad; EINVAL if there is none. */
mbh_status mbh_flow_adam(mbh_flow *flow, float lr, void *stream);

/* Library version (major*100 + minor). */
int mbh_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MBH_H */
