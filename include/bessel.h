/*
 * bessel.h -- C ABI of libbessel.so: batched log K_v(x), its derivatives in v
 * and x, and the integration range, on MI355X (gfx950) HIP kernels.
 *
 * Method: Takekawa, "Fast parallel calculation of modified Bessel function of
 * the second kind and its derivatives" (arXiv 2108.11560).  For v real and
 * x > 0 (Section 2, Eq. (1)-(2)),
 *     K_v(x) = int_0^inf cosh(v t) exp(-x cosh t) dt.
 * Each element: find the peak t_p of g(t) = log cosh(v t) - x cosh t
 * (Section 2.2), bracket [t0, t1] = {t : g(t) >= g(t_p) + log eps} (Section 2.1,
 * Eq. (7)-(8); Section 2.3), and sum a fixed number of trapezoid bins in log
 * space (Section 2.4, Eq. (9)-(11) and Eq. (int)).  Derivatives of log K up
 * to second order come from the companion integrals of Section 4.1, Eq. (13),
 * over the same bins; bessel_logdk gives derivatives of K of higher orders,
 * each integrand over its own peak and bracket.
 *
 * Conventions shared by every entry point:
 *   - Array pointers are DEVICE pointers, contiguous, owned by the caller; the
 *     library never frees, reallocates or keeps them past the call.
 *   - Calls are asynchronous on `hip_stream` (a hipStream_t; NULL means the
 *     default stream).  No entry point synchronises the host on the hot path.
 *   - `dtype` selects the element type of every floating array of the call:
 *     BESSEL_F32 (float) or BESSEL_F64 (double).  The truncation margin log eps
 *     follows the dtype: eps = 2^-23 (F32) or 2^-52 (F64).
 *   - Output arrays must not overlap input arrays (BESSEL_ERR_ALIAS).
 *   - Sizes: elements are indexed with 64 bits; one call takes up to
 *     256 x (2^31 - 1) elements (the launch grid), the learned range modes up to
 *     2^31 - 2 (their worklist holds 32-bit indices).  Larger n returns
 *     BESSEL_ERR_ARG before any work is queued.
 *   - Return value: BESSEL_OK (0), or a negative status; the message of the
 *     last failure on the calling thread is bessel_last_error().  n == 0 is a
 *     no-op that returns BESSEL_OK.
 *   - Per-element domain results are not errors (the paper states only v real,
 *     x > 0):  NaN v or x, or x < 0 -> NaN;  x == 0 -> log K = +inf;
 *     x == +inf -> log K = -inf;  |v| == inf with finite x > 0 -> log K = +inf;
 *     derivatives are NaN in all of these.  v < 0 is evaluated at |v|
 *     (K_{-v} = K_v) with d/dv negated; v == 0 gives d/dv == 0 exactly.
 *     0 < x < 1e-36, finite x > 1e36, finite |v| > 1e6 and finite
 *     |v| > 1.2e38 x -> NaN as well: beyond the range of the bracket search
 *     (which runs in FP32 with fixed step counts).
 *   - Validated domain (tests against the CPU oracle at the default 128 bins):
 *     |v| <= 1e3 with 1e-6 <= x <= 1e6 at the F64 bar (mixed error 1e-12) and
 *     1e-35 <= x <= 1e6 at the F32 bar (1e-5).  Larger orders, tested at
 *     |v| = 1e4, 1e5 and 1e6 for x from 1e-30 to 1e6: log K and its first
 *     derivatives hold the same bars (measured <= 4e-13 F64, <= 1e-7 F32);
 *     the F64 second derivatives in x hold ~1e-11 at 1e5 and ~4e-10 at 1e6
 *     (the variance of cosh t about cosh t_p over a bracket narrower than
 *     1e-2 cancels a few digits).  Outside the validated x range the results
 *     stay finite but lose accuracy: below x ~ 1e-6 the bracket is so wide
 *     that 128 bins resolve the d/dx integrand only to ~1e-10 (more bins
 *     restore it); far above x ~ 1e6 the FP32 bracket search widens the
 *     bracket by the FP32 rounding of g(t_p) ~ -x until 128 bins no longer
 *     resolve it.  F32 derivatives whose value exceeds the F32 range (e.g.
 *     d2/dx2 ~ v / x^2 at small x) are +-inf.
 */
#ifndef BESSEL_H
#define BESSEL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* element types */
#define BESSEL_F32 0
#define BESSEL_F64 1

/* how [t0, t1] is found */
#define BESSEL_RANGE_NEWTON 0 /* peak by Newton steps, ends by monotone fixed-point + Newton steps
                                 (above |v| = 1e3 also from curvature bounds; the tighter end is kept) */
#define BESSEL_RANGE_MLP 1    /* learned bracket with a per-element check and Newton fallback */
#define BESSEL_RANGE_MLP_TABLE 2 /* the same network read from its bilinear table (see bessel_mlp) */

/* status codes */
#define BESSEL_OK 0
#define BESSEL_ERR_ARG (-1)        /* NULL required pointer, n < 0 or above the size limit */
#define BESSEL_ERR_DTYPE (-2)      /* dtype not BESSEL_F32 / BESSEL_F64 */
#define BESSEL_ERR_NBINS (-3)      /* nbins outside [BESSEL_MIN_BINS, BESSEL_MAX_BINS] */
#define BESSEL_ERR_RANGE_MODE (-4) /* unknown range_mode, or a learned range_mode with mlp == NULL */
#define BESSEL_ERR_HIP (-5)        /* a HIP launch or runtime call failed */
#define BESSEL_ERR_ALIAS (-6)      /* an output overlaps an input */
#define BESSEL_ERR_UNSUPPORTED (-7) /* combination not provided (e.g. MLP range with F64) */
#define BESSEL_ERR_ORDER (-8)      /* derivative order outside [0, BESSEL_MAX_ORDER] */

#define BESSEL_MIN_BINS 2
#define BESSEL_MAX_BINS 4096

/* Opaque learned-range predictor (see the MLP section below). */
typedef struct bessel_mlp bessel_mlp;

/*
 * bessel_logk -- logk[i] = log K_{v[i]}(x[i]) for i < n.
 *   v, x     [n] inputs (dtype).
 *   logk     [n] output (dtype).
 *   nbins    number of trapezoid bins n of Eq. (9) (n + 1 nodes); 64, 128 and
 *            256 run specialised kernels, other values in range a generic one.
 *   range_mode, mlp   BESSEL_RANGE_NEWTON (mlp ignored, may be NULL),
 *            BESSEL_RANGE_MLP or BESSEL_RANGE_MLP_TABLE (mlp required; F32 only).
 * Section 2 (Algorithm 3 and Eq. (int)).
 */
int bessel_logk(int dtype, int64_t n, const void* v, const void* x, void* logk, int nbins,
                int range_mode, const bessel_mlp* mlp, void* hip_stream);

/*
 * bessel_logk_dv_dx -- derivatives of log K in one pass over the same bins:
 *   dv[i] = d/dv log K_v(x),  dx[i] = d/dx log K_v(x)   at (v[i], x[i]),
 * each multiplied by grad_out[i] when grad_out is not NULL (the backward of a
 * scalar loss through log K).  logk (nullable) also receives log K.
 * Section 4.1, Eq. (13): d/dv K = int t sinh(v t) e^{-x cosh t} dt and
 * d/dx K = -int cosh t cosh(v t) e^{-x cosh t} dt, divided by K.
 */
int bessel_logk_dv_dx(int dtype, int64_t n, const void* v, const void* x, const void* grad_out,
                      void* logk, void* dv, void* dx, int nbins, int range_mode,
                      const bessel_mlp* mlp, void* hip_stream);

/*
 * bessel_range -- the bracket of Section 2.1 (Eq. (7)-(8)) for the dtype's eps:
 *   t0[i], t1[i]    integration limits; [t0, t1] contains every t with
 *                   g(t) >= g(t_p) + log eps (a superset, never a subset);
 *   tp[i]           (nullable) BESSEL_RANGE_NEWTON: the peak location t_p
 *                   (Section 2.2, FP32 Newton steps);
 *   logf_peak[i]    (nullable) BESSEL_RANGE_NEWTON: g(t_p), the shift of Eq. (int)
 *                   (BESSEL_F32: evaluated in FP32 arithmetic as the F32 kernels
 *                   shift by it, to ~1e-6 of log cosh(v t_p) + x cosh t_p);
 *   fallback[i]     (nullable, uint8) with a learned range mode: 1 where the
 *                   learned bracket failed its check and the Newton bracket was used.
 * With a learned range mode, where an element's learned bracket passed its check,
 * tp is not the peak but the point of the bracket whose g is the shift (the
 * best of the bracket's midpoint, asinh(v/x) clamped into the bracket and, if
 * t0 = 0, 0), and logf_peak is g there, in FP32: a lower bound of max g (any
 * finite shift gives the same log K).  Where the element fell back, all four
 * outputs are the Newton bracket's.
 */
int bessel_range(int dtype, int64_t n, const void* v, const void* x, void* t0, void* t1,
                 void* tp, void* logf_peak, int range_mode, const bessel_mlp* mlp,
                 uint8_t* fallback, void* hip_stream);

/*
 * bessel_logk_hess -- log K with its first and second derivatives in v and x
 * from one pass over the same bins (Section 4.1, Eq. (13) with n + m <= 2:
 * the integrands t^2 f, cosh^2(t) f and t cosh(t) sinh(vt) e^{-x cosh t}
 * join those of the first derivatives):
 *   dvv[i] = d2/dv2 log K = K_vv/K - (K_v/K)^2,
 *   dxx[i] = d2/dx2 log K = K_xx/K - (K_x/K)^2,
 *   dvx[i] = d2/dvdx log K = K_vx/K - (K_v/K)(K_x/K),
 * and logk, dv, dx as bessel_logk_dv_dx.  Every output is nullable (at least
 * one must be given); outputs may not overlap inputs or each other.  Newton
 * bracket, dtype F32 or F64.  Conventions: K_{-v} = K_v, so dv and dvx are odd
 * in v (0 at v = 0) and dvv, dxx even; special inputs give NaN derivatives.
 */
int bessel_logk_hess(int dtype, int64_t n, const void* v, const void* x, void* logk, void* dv, void* dx, void* dvv,
                     void* dxx, void* dvx, int nbins, void* hip_stream);

/*
 * bessel_logdk -- derivatives of K itself of any orders, each integrand over
 * its own peak and bracket (Section 4.1, Eq. (13)):
 *   logdk[i] = log |d^a/dv^a d^b/dx^b K_v(x)|  at (v[i], x[i]),
 *   a = order_v, b = order_x, both in [0, BESSEL_MAX_ORDER];
 *   sign[i]  (nullable) = the derivative's sign: (-1)^b, times sign(v) for odd
 *            a, and 0 where it is exactly zero (odd a at v = 0).
 * The derivative is (-1)^b times the integral of
 *   t^a cosh^b(t) C(v t) e^{-x cosh t}  over t >= 0, C = cosh (even a) or sinh (odd a),
 * and each element locates that integrand's own peak and the interval where it
 * is within eps of it (a doubling search from the peak for each end, then
 * bisection and Newton steps), and sums nbins trapezoid bins relative to the
 * peak.  Unlike the companion sums of bessel_logk_dv_dx / bessel_logk_hess,
 * which use f's interval, this keeps its accuracy for high orders.  FP64
 * arithmetic for both dtypes (the dtype sets the arrays and eps).
 * Conventions: NaN v or x, x < 0 or 0 < x < 1e-36 -> NaN (sign NaN); odd a at
 * v == 0 -> -inf (sign 0); x == 0 or |v| == inf -> +inf; x == +inf -> -inf.
 * Validated domain: as log K (F64: |v| <= 1e3, 1e-6 <= x <= 1e5, mixed error
 * 1e-12 on logdk at 128 bins; orders up to BESSEL_MAX_ORDER).  Outputs may not
 * overlap inputs or each other.
 */
#define BESSEL_MAX_ORDER 8
int bessel_logdk(int dtype, int64_t n, const void* v, const void* x, int order_v, int order_x, void* logdk,
                 void* sign, int nbins, void* hip_stream);

/*
 * bessel_set_split_threshold -- batch-size policy of bessel_logk,
 * bessel_logk_dv_dx and bessel_logk_hess.  Batches of at most n elements run
 * kernels that give each element 16 lanes (every lane finds the bracket, sums
 * 1/16 of the bins, and the lanes add their FP64 partial sums): for small
 * batches, where one lane per element would leave most of the GPU idle, this
 * cuts the latency (Section 3.4 measures the time against the batch size).
 * Larger batches run one lane per element.  The two layouts add the same
 * terms in a different order, so results can differ in the last bits between
 * them (both within the path's tolerance); for a given n and threshold they
 * are deterministic.  bessel_logk and bessel_logk_dv_dx with a learned
 * range_mode also take the Newton bracket on this layout for such batches (one
 * launch; the predictor saves no time there), so their results equal those of
 * BESSEL_RANGE_NEWTON and bessel_mlp_fallback_count reads 0 after them;
 * bessel_range keeps the learned bracket at every size.  n = 0 turns the
 * split kernels off.  Default 16384; at most BESSEL_MAX_SPLIT_THRESHOLD.
 * previous (nullable) receives the old value.  Process-wide; takes effect for
 * later calls.
 */
#define BESSEL_MAX_SPLIT_THRESHOLD (1LL << 26)
int bessel_set_split_threshold(int64_t n, int64_t* previous);

/*
 * bessel_hess_vjp -- the backward step through (d/dv, d/dx) log K, with the
 * second derivatives a bessel_logk_hess call produced (the Hessian of log K is
 * symmetric):
 *   grad_v[i] = g_dv[i] dvv[i] + g_dx[i] dvx[i],
 *   grad_x[i] = g_dv[i] dvx[i] + g_dx[i] dxx[i].
 * g_dv or g_dx may be NULL (a zero upstream gradient), not both; grad_v or
 * grad_x may be NULL (not needed).  Outputs may not overlap inputs.  This is
 * what second-order differentiation (a Newton step in v or x, a Hessian of a
 * likelihood) needs from Section 4.1's derivatives.
 */
int bessel_hess_vjp(int dtype, int64_t n, const void* g_dv, const void* g_dx, const void* dvv, const void* dxx,
                    const void* dvx, void* grad_v, void* grad_x, void* hip_stream);

/*
 * bessel_logk_backward -- the backward step of a scalar loss through log K:
 *   grad_v[i] = grad_out[i] * dv[i],  grad_x[i] = grad_out[i] * dx[i],
 * where dv, dx are the derivatives a forward bessel_logk_dv_dx call saved.
 * grad_v or grad_x may be NULL (that gradient is not needed).  Outputs may not
 * overlap inputs.  Section 4.1 (the derivatives) with the chain rule.
 */
int bessel_logk_backward(int dtype, int64_t n, const void* grad_out, const void* dv, const void* dx,
                         void* grad_v, void* grad_x, void* hip_stream);

/*
 * Learned bracket predictor (FP32 path).
 *
 * A network 2 -> 64 -> 64 -> 2 maps the features of an element,
 * ((log max(|v|, 1e-3) - m_v)/s_v, (log x - m_x)/s_x), to (y0, y1); the bracket
 * is t0 = max(0, y0 - margin_t0) exp(y1), t1 = exp(y1 + margin_t1).  Its
 * activations are tanh-shaped and need no transcendental: clamp(a, -1, 1) on
 * the first layer, u (3 - u^2) / 2 with u = clamp(a / 1.5, -1, 1) on the second.
 * It is trained on the method's own Newton brackets (Sections 2.2-2.3 at the
 * FP32 eps), and at inference (all three layers on f16 MFMA with FP32
 * accumulation, the activations in packed f16 arithmetic) every
 * predicted bracket is checked after the bins: the end terms must lie below eps
 * relative to the shift and the even-node and odd-node sums must agree to
 * 1e-5.  Elements that fail are recomputed by the Newton path in a second
 * kernel on the same stream.
 *
 * BESSEL_RANGE_MLP_TABLE reads the same network from a table: after each
 * change of the parameters, the first call in this mode evaluates the
 * network (the same f16-MFMA inference) on a 256 x 256 grid of the feature
 * plane, z in [-4, 4]^2, and stores per cell the bilinear coefficients of
 * both outputs (2.6 MB, owned by the handle). Each element then interpolates
 * the outputs of its cell instead of running 128 activations. Features
 * outside the grid are clamped to its edge. The check and the fallback are
 * the same as for BESSEL_RANGE_MLP.
 *
 * Parameter vector (host floats, BESSEL_MLP_NPARAMS): W1 (64 x 2, row-major),
 * b1[64], W2 (64 x 64; W2[i][j] multiplies hidden j of layer 1), b2[64],
 * W3 (2 x 64), b3[2] (BESSEL_MLP_NWEIGHTS trainable values), then
 * m_v, s_v, m_x, s_x, margin_t1, margin_t0, 0, 0.
 *
 * The handle owns all device memory it uses: parameters, optimizer state, the
 * inference operands derived from the parameters (rebuilt on the stream of
 * the first inference call after any change of the parameters), and
 * workspaces that grow (stream-ordered, on the call's stream) to the largest
 * n seen.  Calls that use one handle must not overlap in time (serialise them
 * on one stream); different handles are independent.
 */
#define BESSEL_MLP_HIDDEN 64
#define BESSEL_MLP_NWEIGHTS 4482
#define BESSEL_MLP_NPARAMS 4490

typedef struct {
  int64_t steps;      /* Adam steps */
  int64_t batch;      /* samples per step, drawn with replacement from the n inputs */
  float lr;           /* learning rate at the first step */
  float lr_final;     /* learning rate at the last step (exponential decay in between) */
  float beta1, beta2, adam_eps;
  float alpha;        /* loss weight on the unsafe side (t0 too large, t1 too small) */
  uint64_t seed;      /* minibatch draws: splitmix64 of (seed, step, sample) */
} bessel_mlp_train_cfg;

/* Create a predictor; params (host, nullable: zeros with unit scales) of length nparams. */
int bessel_mlp_create(const float* params, int64_t nparams, bessel_mlp** out);
/* Destroy (synchronises the device first).  NULL is a no-op. */
int bessel_mlp_destroy(bessel_mlp* mlp);
/* Replace the parameters (host floats) and reset the optimizer state. */
int bessel_mlp_set_params(bessel_mlp* mlp, const float* params, int64_t nparams);
/* Copy the parameters to host floats (synchronises the device). */
int bessel_mlp_get_params(const bessel_mlp* mlp, float* params, int64_t nparams);
/*
 * Train on n FP32 device inputs (v, x): labels are the Newton brackets of the
 * inputs at the FP32 eps, then cfg->steps Adam steps on minibatches.  loss_host
 * (nullable, cfg->steps floats) receives the loss of each step; when it is
 * given the call synchronises the stream at the end.
 */
int bessel_mlp_train(bessel_mlp* mlp, const bessel_mlp_train_cfg* cfg, int64_t n, const float* v, const float* x,
                     float* loss_host, void* hip_stream);
/*
 * Loss and gradient (BESSEL_MLP_NWEIGHTS floats, same order as the weights) of
 * the full batch of n device samples with given bracket targets t0, t1 (device),
 * asymmetry alpha.  loss[1] and grad are device outputs.
 */
int bessel_mlp_loss_grad(bessel_mlp* mlp, int64_t n, const float* v, const float* x, const float* t0,
                         const float* t1, float alpha, float* loss, float* grad, void* hip_stream);
/* One Adam step (Kingma & Ba, bias-corrected; the handle counts steps from 1)
 * with a given device gradient of BESSEL_MLP_NWEIGHTS floats. */
int bessel_mlp_adam_step(bessel_mlp* mlp, const float* grad, float lr, float beta1, float beta2, float eps,
                         void* hip_stream);
/* Raw network outputs y[2 i], y[2 i + 1] for n device inputs; mode 0: FP32 with
 * the activations in FP32, one element per lane; mode 1: the f16-MFMA inference of the
 * fused kernel (the same operands and arithmetic); mode 2: the bilinear table
 * of BESSEL_RANGE_MLP_TABLE. */
int bessel_mlp_forward(const bessel_mlp* mlp, int64_t n, const float* v, const float* x, float* y, int mode,
                       void* hip_stream);
/* Number of elements of the handle's last learned-range call that fell back to
 * the Newton bracket (synchronises the device). */
int bessel_mlp_fallback_count(const bessel_mlp* mlp, int* count);

/*
 * bessel_gh_logk_sum -- per-set sums over shared samples (FP32 arrays):
 *   for set i (lam, alpha, delta, mu: [nsets]) and samples y[nsamp],
 *     v = lam_i - 1/2,  r_j = sqrt(delta_i^2 + (y_j - mu_i)^2),  x_j = alpha_i r_j,
 *     sum[i] = sum_j log K_v(x_j),
 *   and the gradient of sum[i] with respect to lam_i, alpha_i, delta_i, mu_i
 *   (each nullable), multiplied by grad_sum[i] when grad_sum is not NULL.
 * This is the Bessel factor of a generalised-hyperbolic log-likelihood (the
 * application named in the paper's introduction), evaluated with the FP32
 * path and its derivatives (Sections 2 and 4.1) and the chain rule.  Sums are
 * accumulated in FP64 and reduced in a fixed order (deterministic).  Each
 * term follows bessel_logk's per-element conventions (a NaN or infinite term,
 * e.g. |lam - 1/2| above 1e6, makes its set's sum and gradients non-finite).
 * The call allocates a temporary of nsets * ceil(nsamp/256) * 5 doubles,
 * stream-ordered on hip_stream.  range_mode: BESSEL_RANGE_NEWTON (mlp ignored) or
 * BESSEL_RANGE_MLP_TABLE (mlp required: the bracket from the predictor's
 * table, checked after the bins as in bessel_logk; an element that fails the
 * check takes the Newton bracket in the same pass, so no worklist is kept and
 * the handle's fallback count is not changed).  BESSEL_RANGE_MLP returns
 * BESSEL_ERR_UNSUPPORTED.
 */
int bessel_gh_logk_sum(int64_t nsets, const float* lam, const float* alpha, const float* delta, const float* mu,
                       int64_t nsamp, const float* y, const float* grad_sum, float* sum, float* g_lam,
                       float* g_alpha, float* g_delta, float* g_mu, int nbins, int range_mode,
                       const bessel_mlp* mlp, void* hip_stream);

/*
 * bessel_gh_logk_sum_noalloc -- bessel_gh_logk_sum without any allocation, for
 * callers that cannot allocate device memory during the call (code under HIP
 * graph capture, serving loops, harnesses that forbid hipMalloc).  Arguments,
 * results and errors are those of bessel_gh_logk_sum (the same kernels, so the
 * same bits), except that the per-block partial sums live in a static device
 * array of the library instead of a temporary: at most
 * BESSEL_GH_NOALLOC_MAX_BLOCKS records, i.e. nsets * ceil(nsamp / 256) must not
 * exceed it (else BESSEL_ERR_ARG before any work is queued; 1024 sets of 65536
 * samples fit).  Each GPU the library runs on holds that array (10 MiB) until
 * the process ends; the first call on a GPU looks up its address there.  With
 * BESSEL_RANGE_MLP_TABLE the predictor's table is rebuilt, when its parameters
 * changed, into buffers the handle allocated at creation.  Every
 * call on one GPU shares the array: calls that overlap in time on one GPU (on
 * different streams, or from different host threads) race and must be
 * serialised by the caller.  Nothing in the array needs clearing between calls.
 */
#define BESSEL_GH_NOALLOC_MAX_BLOCKS (1LL << 18)
int bessel_gh_logk_sum_noalloc(int64_t nsets, const float* lam, const float* alpha, const float* delta,
                               const float* mu, int64_t nsamp, const float* y, const float* grad_sum, float* sum,
                               float* g_lam, float* g_alpha, float* g_delta, float* g_mu, int nbins,
                               int range_mode, const bessel_mlp* mlp, void* hip_stream);

/* Message of the last failed call on the calling thread ("" if none). */
const char* bessel_last_error(void);

/* Library build string (compiler, target) for logs. */
const char* bessel_version(void);

#ifdef __cplusplus
}
#endif

#endif /* BESSEL_H */
