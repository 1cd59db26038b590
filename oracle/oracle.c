/*
 * oracle.c -- CPU oracle for log K_v(x), its derivatives in v and x, the
 * truncation interval of the integral, and the paper's own range-and-trapezoid
 * algorithm.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or constant generator with the GPU library; the GPU library
 * never calls it.
 *
 * Arithmetic is x87 long double (64-bit mantissa, unit roundoff 2^-64), about
 * three decimal digits beyond the FP64 results it checks.
 *
 * Method (Takekawa, "Fast parallel calculation of modified Bessel function of
 * the second kind and its derivatives", arXiv 2108.11560):
 *   Section 2, Eq. (1)-(2):  K_v(x) = int_0^inf f(t) dt,
 *                            f(t) = cosh(v t) exp(-x cosh t),  v real, x > 0.
 *   Section 2.1, Eq. (3)-(5): g = log f = log cosh(v t) - x cosh t,
 *                            g' = v tanh(v t) - x sinh t,
 *                            g'' = v^2 sech^2(v t) - x cosh t.
 *   Section 2.1, Eq. (7)-(8): the truncation set {t : g(t) >= g(t_p) + log eps}.
 *   Section 4.1, Eq. (13):    derivatives of f in v and x, integrated the same way.
 *
 * Two families of entry points:
 *
 *  (1) oracle_logk_batch / oracle_logk_hess_batch / oracle_range_exact: the
 *      plain definitions.  log K is
 *      the integral of Eq. (1) computed by adaptive Gauss-Legendre quadrature
 *      (not the paper's fixed-bin trapezoid), split at the exact peak of g and
 *      truncated where g has fallen 60 nats below the peak (neglected mass below
 *      1e-26 relative on x >= 1e-3).  d/dv log K and d/dx log K are the
 *      companion integrals of Eq. (13) with the exp(-x cosh t) factor present:
 *        d/dv K = int t sinh(v t) exp(-x cosh t) dt,
 *        d/dx K = -int cosh(t) cosh(v t) exp(-x cosh t) dt.
 *      The second derivatives differentiate these once more under the
 *      integral (Eq. (13) with n + m = 2):
 *        d2/dv2 K  = int t^2 cosh(v t) exp(-x cosh t) dt,
 *        d2/dx2 K  = int cosh^2(t) cosh(v t) exp(-x cosh t) dt,
 *        d2/dvdx K = -int t cosh(t) sinh(v t) exp(-x cosh t) dt,
 *      and those of log K follow from K''/K - (K'/K)^2 and
 *      K_vx/K - (K_v/K)(K_x/K).
 *      The peak and the level crossings are found by plain bisection.
 *
 *  (2) oracle_method_batch: Algorithms 1-3 and Eq. (int) of Section 2 in the
 *      paper's order, with the readings listed at that function.
 *
 * Domain conventions for both (the paper states only v real, x > 0):
 *   NaN v or x, or x < 0     -> NaN outputs;
 *   x == 0                   -> log K = +inf, derivatives NaN;
 *   x == +inf                -> log K = -inf, derivatives NaN;
 *   |v| == inf, finite x > 0 -> log K = +inf, derivatives NaN;
 *   v < 0                    -> evaluated at |v| (K_{-v} = K_v), d/dv and
 *                               d2/dvdx negated;
 *   v == 0                   -> d/dv log K = d2/dvdx log K = 0 exactly.
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>
#include <pthread.h>

typedef long double ld;

#define LN2L 0.693147180559945309417232121458176568L

/* ---------------------------------------------------------------------- */
/* The log-integrand and its t-derivatives (Section 2.1, Eq. (3)-(5)).      */
/* ---------------------------------------------------------------------- */

/* log cosh z written so it cannot overflow: |z| + log(1 + e^{-2|z|}) - log 2. */
static ld log_cosh(ld z) {
  ld a = fabsl(z);
  return a + log1pl(expl(-2.0L * a)) - LN2L;
}

/* g_{v,x}(t) = log cosh(v t) - x cosh t  (Eq. 3). */
static ld g_vx(ld v, ld x, ld t) { return log_cosh(v * t) - x * coshl(t); }

/* g'_{v,x}(t) = v tanh(v t) - x sinh t  (Eq. 4). */
static ld dg_vx(ld v, ld x, ld t) { return v * tanhl(v * t) - x * sinhl(t); }

/* g''_{v,x}(t) = v^2 sech^2(v t) - x cosh t  (Eq. 5). */
static ld d2g_vx(ld v, ld x, ld t) {
  ld c = coshl(v * t);
  ld sech2 = isinf(c) ? 0.0L : 1.0L / (c * c);
  return v * v * sech2 - x * coshl(t);
}

/* ---------------------------------------------------------------------- */
/* Exact peak and truncation interval by bisection (Section 2.1-2.3).       */
/* ---------------------------------------------------------------------- */

/* Peak t_p of g.  Section 2.1: if v^2 <= x, g decreases on t >= 0 and t_p = 0;
 * otherwise g' > 0 on (0, t_p) and g' < 0 beyond, with a single root.  Since
 * tanh <= 1, g'(t) <= v - x sinh t < 0 for t > asinh(v/x), so the root lies in
 * (0, asinh(v/x)].  Bisection until the interval stops shrinking. */
static ld exact_peak(ld v, ld x) {
  if (v * v <= x) return 0.0L;
  ld lo = 0.0L, hi = asinhl(v / x) + 1.0L;
  for (int it = 0; it < 400; ++it) {
    ld mid = 0.5L * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (dg_vx(v, x, mid) > 0.0L) lo = mid; else hi = mid;
  }
  return 0.5L * (lo + hi);
}

/* Root of F(t) = g(t) - G + L on [a, b], where F(a) and F(b) have opposite
 * signs, by bisection.  Returns the end where F <= 0, so the returned interval
 * always contains the set where F > 0. */
static ld level_cross(ld v, ld x, ld G, ld L, ld a, ld b) {
  ld Fa = g_vx(v, x, a) - G + L;
  for (int it = 0; it < 400; ++it) {
    ld mid = 0.5L * (a + b);
    if (mid == a || mid == b) break;
    ld Fm = g_vx(v, x, mid) - G + L;
    if ((Fm > 0.0L) == (Fa > 0.0L)) { a = mid; Fa = Fm; } else { b = mid; }
  }
  /* a and b are adjacent; return the one with F <= 0. */
  return (Fa <= 0.0L) ? a : b;
}

/* Upper crossing of g = G - L for t > t_p: double the step from t_p until
 * F < 0 (g is strictly decreasing beyond t_p), then bisect. */
static ld upper_cross(ld v, ld x, ld tp, ld G, ld L) {
  ld step = 1.0L;
  while (g_vx(v, x, tp + step) - G + L > 0.0L) step *= 2.0L;
  return level_cross(v, x, G, L, tp, tp + step);
}

/* Lower crossing on [0, t_p]: 0 if F(0) > 0, otherwise bisection (g is
 * increasing on [0, t_p]). */
static ld lower_cross(ld v, ld x, ld tp, ld G, ld L) {
  if (g_vx(v, x, 0.0L) - G + L > 0.0L) return 0.0L;
  return level_cross(v, x, G, L, tp, 0.0L);
}

/* ---------------------------------------------------------------------- */
/* Gauss-Legendre rule computed at start-up (Newton iteration on P_n).      */
/* ---------------------------------------------------------------------- */

#define GL_N 20
static ld gl_node[GL_N], gl_wt[GL_N];
static pthread_once_t gl_once = PTHREAD_ONCE_INIT;

static void gl_init(void) {
  for (int i = 0; i < GL_N; ++i) {
    ld z = cosl(3.14159265358979323846264338327950288L * ((ld)i + 0.75L) / ((ld)GL_N + 0.5L));
    ld dp = 0.0L;
    for (int it = 0; it < 100; ++it) {
      /* Legendre recurrence: (k+1) P_{k+1} = (2k+1) z P_k - k P_{k-1}. */
      ld p0 = 1.0L, p1 = z;
      for (int k = 1; k < GL_N; ++k) {
        ld p2 = ((2.0L * k + 1.0L) * z * p1 - (ld)k * p0) / ((ld)k + 1.0L);
        p0 = p1; p1 = p2;
      }
      dp = (ld)GL_N * (z * p1 - p0) / (z * z - 1.0L);
      ld dz = p1 / dp;
      z -= dz;
      if (fabsl(dz) <= 1e-21L * fabsl(z) + 1e-30L) {
        /* one more evaluation for the weight at the converged node */
        p0 = 1.0L; p1 = z;
        for (int k = 1; k < GL_N; ++k) {
          ld p2 = ((2.0L * k + 1.0L) * z * p1 - (ld)k * p0) / ((ld)k + 1.0L);
          p0 = p1; p1 = p2;
        }
        dp = (ld)GL_N * (z * p1 - p0) / (z * z - 1.0L);
        break;
      }
    }
    gl_node[i] = z;
    gl_wt[i] = 2.0L / ((1.0L - z * z) * dp * dp);
  }
}

/* ---------------------------------------------------------------------- */
/* Adaptive quadrature of up to six integrands, scaled by exp(-G):          */
/*   I0 = int exp(g - G) dt                    (K_v(x) e^{-G})              */
/*   I1 = int t tanh(v t) exp(g - G) dt        (d/dv K e^{-G}, v >= 0)      */
/*   I2 = int cosh(t) exp(g - G) dt            (-d/dx K e^{-G})             */
/*   I3 = int t^2 exp(g - G) dt                (d2/dv2 K e^{-G})            */
/*   I4 = int cosh^2(t) exp(g - G) dt          (d2/dx2 K e^{-G})            */
/*   I5 = int t cosh(t) tanh(v t) exp(g - G) dt (-d2/dvdx K e^{-G})         */
/* (exp(g) = cosh(v t) exp(-x cosh t), so t tanh(v t) exp(g) is the          */
/* t sinh(v t) exp(-x cosh t) of d/dv, and so on.)  `level` 0 integrates I0, */
/* 1 also I1-I2, 2 all six.                                                  */
/* ---------------------------------------------------------------------- */

#define NQ 6

typedef struct {
  ld v, x, G;
  ld tol[NQ];
  int level;
} quad_ctx;

static void gl_panel(const quad_ctx* c, ld a, ld b, ld r[NQ]) {
  ld mid = 0.5L * (a + b), hw = 0.5L * (b - a);
  ld s[NQ] = {0.0L, 0.0L, 0.0L, 0.0L, 0.0L, 0.0L};
  for (int i = 0; i < GL_N; ++i) {
    ld t = mid + hw * gl_node[i];
    ld e = expl(g_vx(c->v, c->x, t) - c->G);
    s[0] += gl_wt[i] * e;
    if (c->level >= 1) {
      ld th = t * tanhl(c->v * t), ch = coshl(t);
      s[1] += gl_wt[i] * th * e;
      s[2] += gl_wt[i] * ch * e;
      if (c->level >= 2) {
        s[3] += gl_wt[i] * t * t * e;
        s[4] += gl_wt[i] * ch * ch * e;
        s[5] += gl_wt[i] * th * ch * e;
      }
    }
  }
  for (int k = 0; k < NQ; ++k) r[k] = hw * s[k];
}

static void gl_adapt(const quad_ctx* c, ld a, ld b, const ld whole[NQ], int depth, ld acc[NQ]) {
  ld m = 0.5L * (a + b);
  ld left[NQ], right[NQ], fine[NQ];
  gl_panel(c, a, m, left);
  gl_panel(c, m, b, right);
  int ok = 1;
  for (int k = 0; k < NQ; ++k) {
    fine[k] = left[k] + right[k];
    if (!(fabsl(fine[k] - whole[k]) <= c->tol[k])) ok = 0;
  }
  if (ok || depth >= 48 || m <= a || m >= b) {
    for (int k = 0; k < NQ; ++k) acc[k] += fine[k];
    return;
  }
  gl_adapt(c, a, m, left, depth + 1, acc);
  gl_adapt(c, m, b, right, depth + 1, acc);
}

/* Integrate over [lo, hi] split at tp: a coarse pass over 8 panels per side
 * sets the absolute tolerances (4e-18 of each integral, a little above the
 * long double rounding floor of a 20-point sum), then every panel is refined
 * adaptively.  An accepted panel's two-half estimate is far more accurate than
 * its difference from the one-panel estimate. */
static void integrate(quad_ctx* c, ld lo, ld tp, ld hi, ld out[NQ]) {
  const int P = 8;
  ld est[NQ] = {0.0L, 0.0L, 0.0L, 0.0L, 0.0L, 0.0L};
  ld edges[2][2] = {{lo, tp}, {tp, hi}};
  for (int s = 0; s < 2; ++s) {
    ld a = edges[s][0], b = edges[s][1];
    if (!(b > a)) continue;
    for (int p = 0; p < P; ++p) {
      ld r[NQ];
      gl_panel(c, a + (b - a) * p / P, a + (b - a) * (p + 1) / P, r);
      for (int k = 0; k < NQ; ++k) est[k] += fabsl(r[k]);
    }
  }
  for (int k = 0; k < NQ; ++k) {
    c->tol[k] = (est[k] > 0.0L) ? 4e-18L * est[k] : INFINITY;
    out[k] = 0.0L;
  }
  for (int s = 0; s < 2; ++s) {
    ld a = edges[s][0], b = edges[s][1];
    if (!(b > a)) continue;
    for (int p = 0; p < P; ++p) {
      ld pa = a + (b - a) * p / P, pb = a + (b - a) * (p + 1) / P;
      ld whole[NQ];
      gl_panel(c, pa, pb, whole);
      gl_adapt(c, pa, pb, whole, 0, out);
    }
  }
}

/* Margin below the peak at which the oracle truncates the integral. */
#define ORACLE_MARGIN 60.0L

/* One element of the plain definition: out[0] = log K; with level >= 1 also
 * out[1] = d/dv log K, out[2] = d/dx log K; with level 2 also
 * out[3] = d2/dv2 log K, out[4] = d2/dx2 log K, out[5] = d2/dvdx log K. */
static void logk_one(double vin, double xin, int level, double out[NQ]) {
  const int nout = level == 0 ? 1 : level == 1 ? 3 : NQ;
  ld nan_ = NAN;
  if (isnan(vin) || isnan(xin) || xin < 0.0 || xin == 0.0 || isinf(xin) || isinf(vin)) {
    out[0] = (isnan(vin) || isnan(xin) || xin < 0.0) ? nan_
             : (xin == 0.0) ? INFINITY : isinf(xin) ? -INFINITY : INFINITY;
    for (int k = 1; k < nout; ++k) out[k] = nan_;
    return;
  }
  ld sgn = (vin < 0.0) ? -1.0L : 1.0L;
  ld v = fabsl((ld)vin), x = (ld)xin;
  ld tp = exact_peak(v, x);
  ld G = g_vx(v, x, tp);
  ld lo = lower_cross(v, x, tp, G, ORACLE_MARGIN);
  ld hi = upper_cross(v, x, tp, G, ORACLE_MARGIN);
  quad_ctx c;
  c.v = v; c.x = x; c.G = G; c.level = level;
  ld I[NQ];
  integrate(&c, lo, tp, hi, I);
  out[0] = (double)(G + logl(I[0]));
  if (level >= 1) {
    ld lv = I[1] / I[0], lx = -I[2] / I[0];
    out[1] = (v == 0.0L) ? 0.0 : (double)(sgn * lv);
    out[2] = (double)lx;
    if (level >= 2) {
      out[3] = (double)(I[3] / I[0] - lv * lv);
      out[4] = (double)(I[4] / I[0] - lx * lx);
      out[5] = (v == 0.0L) ? 0.0 : (double)(sgn * (-I[5] / I[0] - lv * lx));
    }
  }
}

/* ---------------------------------------------------------------------- */
/* Threading helper: a static partition of [0, n) over pthreads.           */
/* ---------------------------------------------------------------------- */

typedef void (*elem_fn)(void* ctx, int64_t i);
typedef struct { elem_fn fn; void* ctx; int64_t n; int64_t next; pthread_mutex_t mu; } pool_t;

static void* pool_worker(void* arg) {
  pool_t* p = (pool_t*)arg;
  for (;;) {
    pthread_mutex_lock(&p->mu);
    int64_t b = p->next;
    p->next += 8;
    pthread_mutex_unlock(&p->mu);
    if (b >= p->n) break;
    int64_t e = b + 8 < p->n ? b + 8 : p->n;
    for (int64_t i = b; i < e; ++i) p->fn(p->ctx, i);
  }
  return NULL;
}

static void run_pool(elem_fn fn, void* ctx, int64_t n, int nthreads) {
  pthread_once(&gl_once, gl_init);
  pool_t p;
  p.fn = fn; p.ctx = ctx; p.n = n; p.next = 0;
  pthread_mutex_init(&p.mu, NULL);
  if (nthreads < 1) nthreads = 1;
  if (nthreads > 256) nthreads = 256;
  pthread_t th[256];
  int started = 0;
  for (int k = 1; k < nthreads; ++k)
    if (pthread_create(&th[started], NULL, pool_worker, &p) == 0) ++started;
  pool_worker(&p);
  for (int k = 0; k < started; ++k) pthread_join(th[k], NULL);
  pthread_mutex_destroy(&p.mu);
}

/* ---------------------------------------------------------------------- */
/* (1) Plain definitions: batch entry points.                              */
/* ---------------------------------------------------------------------- */

typedef struct { const double *v, *x; double *logk, *dv, *dx; } logk_args;

static void logk_elem(void* ctx, int64_t i) {
  logk_args* a = (logk_args*)ctx;
  double o[NQ];
  int want = (a->dv != NULL) || (a->dx != NULL);
  logk_one(a->v[i], a->x[i], want ? 1 : 0, o);
  a->logk[i] = o[0];
  if (a->dv) a->dv[i] = o[1];
  if (a->dx) a->dx[i] = o[2];
}

/* log K_v(x) for n pairs; dv and dx (nullable) receive d/dv and d/dx of log K. */
int oracle_logk_batch(int64_t n, const double* v, const double* x, double* logk,
                      double* dv, double* dx, int nthreads) {
  if (n < 0 || (n > 0 && (!v || !x || !logk))) return -1;
  logk_args a = {v, x, logk, dv, dx};
  run_pool(logk_elem, &a, n, nthreads);
  return 0;
}

typedef struct { const double *v, *x; double* out; } hess_args;

static void hess_elem(void* ctx, int64_t i) {
  hess_args* a = (hess_args*)ctx;
  logk_one(a->v[i], a->x[i], 2, a->out + NQ * i);
}

/* log K and its first and second derivatives for n pairs: out[6 i + k] holds
 * log K, d/dv, d/dx, d2/dv2, d2/dx2, d2/dvdx of log K at (v[i], x[i]). */
int oracle_logk_hess_batch(int64_t n, const double* v, const double* x, double* out, int nthreads) {
  if (n < 0 || (n > 0 && (!v || !x || !out))) return -1;
  hess_args a = {v, x, out};
  run_pool(hess_elem, &a, n, nthreads);
  return 0;
}

typedef struct { const double *v, *x; double log_eps; double *tp, *G, *t0, *t1; } range_args;

static void range_elem(void* ctx, int64_t i) {
  range_args* a = (range_args*)ctx;
  ld v = fabsl((ld)a->v[i]), x = (ld)a->x[i];
  if (!(x > 0.0L) || isinf(x) || isnan(v) || isinf(v)) {
    a->tp[i] = a->G[i] = a->t0[i] = a->t1[i] = NAN;
    return;
  }
  ld L = -(ld)a->log_eps;
  ld tp = exact_peak(v, x);
  ld G = g_vx(v, x, tp);
  a->tp[i] = (double)tp;
  a->G[i] = (double)G;
  a->t0[i] = (double)lower_cross(v, x, tp, G, L);
  a->t1[i] = (double)upper_cross(v, x, tp, G, L);
}

/* Exact peak t_p, G = g(t_p), and the interval [t0, t1] = {t : g(t) >= G + log_eps}
 * (Eq. 7-8) for n pairs; log_eps < 0 is the log of the truncation ratio. */
int oracle_range_exact(int64_t n, const double* v, const double* x, double log_eps,
                       double* tp, double* G, double* t0, double* t1, int nthreads) {
  if (n < 0 || (n > 0 && (!v || !x || !tp || !G || !t0 || !t1)) || !(log_eps < 0.0)) return -1;
  range_args a = {v, x, log_eps, tp, G, t0, t1};
  run_pool(range_elem, &a, n, nthreads);
  return 0;
}

/* ---------------------------------------------------------------------- */
/* (2) The paper's algorithm (Algorithms 1-3, Eq. (int)).                   */
/*                                                                          */
/* Readings taken where the text is garbled or silent:                      */
/*  - FindRange searches m over the integers (the text of Section 2.2); with */
/*    halve_ok == 0 it starts at m = 0 and only doubles, as the algorithm    */
/*    box prints it.                                                         */
/*  - FindZero keeps F(first) < 0 <= F(second) and returns the F < 0 end;    */
/*    the Newton step starts from the current F < 0 end and is clipped to the */
/*    closed interval between it and the bisection point; the loop stops     */
/*    when that end moved less than tol, or after max_iter steps.            */
/*  - The truncation set uses g >= g(t_p) + log eps (Eq. 8).                 */
/*  - Eq. (int): the trapezoid weight c_m multiplies exp(g(t_m) - g(t_p));   */
/*    it does not sit inside the exponent.                                   */
/* ---------------------------------------------------------------------- */

typedef struct { ld v, x, G, L; int kind; } fz_fn;  /* kind 0: F = g'; kind 1: F = g - G + L */

static ld fz_F(const fz_fn* f, ld t) {
  return f->kind == 0 ? dg_vx(f->v, f->x, t) : g_vx(f->v, f->x, t) - f->G + f->L;
}
static ld fz_dF(const fz_fn* f, ld t) {
  return f->kind == 0 ? d2g_vx(f->v, f->x, t) : dg_vx(f->v, f->x, t);
}

/* Algorithm 1 (FindRange): from t0 with F(t0) >= 0, return [t_s, t_e] =
 * [t0 + 2^m, t0 + 2^{m+1}] with F(t_s) >= 0 > F(t_e). */
static void find_range(const fz_fn* f, ld t0, int halve_ok, ld* ts, ld* te) {
  int m = 0;
  if (fz_F(f, t0 + 2.0L) >= 0.0L || !halve_ok) {
    while (fz_F(f, t0 + ldexpl(1.0L, m + 1)) >= 0.0L && m < 16000) ++m;
    *ts = t0 + ldexpl(1.0L, m);
    *te = t0 + ldexpl(1.0L, m + 1);
    return;
  }
  /* F(t0 + 2) < 0: step m down while F(t0 + 2^m) < 0. */
  while (m > -60 && fz_F(f, t0 + ldexpl(1.0L, m)) < 0.0L) --m;
  *ts = (m > -60) ? t0 + ldexpl(1.0L, m) : t0;
  *te = t0 + ldexpl(1.0L, m + 1);
}

/* Algorithm 2 (FindZero): a is the F < 0 end, b the F >= 0 end. */
static ld find_zero(const fz_fn* f, ld a, ld b, ld tol, int max_iter) {
  int i = 0;
  for (;;) {
    ld a_prev = a;
    ld ts = a + 0.5L * (b - a);
    ld dF = fz_dF(f, a);
    ld tn = a - fz_F(f, a) / dF;
    /* clip into the closed interval between a and ts */
    ld lo = a < ts ? a : ts, hi = a < ts ? ts : a;
    if (!(tn >= lo)) tn = lo;  /* also catches NaN */
    if (tn > hi) tn = hi;
    if (fz_F(f, ts) < 0.0L) {
      a = ts;
    } else if (fz_F(f, tn) < 0.0L) {
      a = tn; b = ts;
    } else {
      b = tn;
    }
    ++i;
    if (fabsl(a - a_prev) < tol || i >= max_iter) break;
  }
  return a;
}

typedef struct {
  const double *v, *x; int nbins; double log_eps; int halve_ok; double tol; int max_iter;
  double *logk, *tp, *t0, *t1;
} method_args;

static void method_elem(void* ctx, int64_t i) {
  method_args* a = (method_args*)ctx;
  ld v = fabsl((ld)a->v[i]), x = (ld)a->x[i];
  if (!(x > 0.0L) || isinf(x) || isnan(v) || isinf(v)) {
    a->logk[i] = NAN;
    if (a->tp) a->tp[i] = NAN;
    if (a->t0) a->t0[i] = NAN;
    if (a->t1) a->t1[i] = NAN;
    return;
  }
  ld leps = (ld)a->log_eps;
  /* Algorithm 3: peak. */
  ld tp = 0.0L;
  if (d2g_vx(v, x, 0.0L) > 0.0L) {
    fz_fn fp = {v, x, 0.0L, 0.0L, 0};
    ld ts, te;
    find_range(&fp, 0.0L, a->halve_ok, &ts, &te);
    tp = find_zero(&fp, te, ts, (ld)a->tol, a->max_iter);
  }
  ld G = g_vx(v, x, tp);
  fz_fn fr = {v, x, G, -leps, 1};
  /* lower end */
  ld t0 = 0.0L;
  if (g_vx(v, x, 0.0L) - G <= leps) t0 = find_zero(&fr, 0.0L, tp, (ld)a->tol, a->max_iter);
  /* upper end */
  ld ts, te;
  find_range(&fr, tp, a->halve_ok, &ts, &te);
  ld t1 = find_zero(&fr, te, ts, (ld)a->tol, a->max_iter);
  /* Eq. (int): log K = g(t_p) + log sum_m h c_m exp(g(t_m) - g(t_p)). */
  int n = a->nbins;
  ld h = (t1 - t0) / (ld)n;
  ld s = 0.0L;
  for (int m = 0; m <= n; ++m) {
    ld cm = (m == 0 || m == n) ? 0.5L : 1.0L;
    s += cm * expl(g_vx(v, x, t0 + (ld)m * h) - G);
  }
  a->logk[i] = (double)(G + logl(h * s));
  if (a->tp) a->tp[i] = (double)tp;
  if (a->t0) a->t0[i] = (double)t0;
  if (a->t1) a->t1[i] = (double)t1;
}

/* The paper's LogBesselK (Algorithm 3) for n pairs with nbins trapezoid bins,
 * truncation margin log_eps (< 0), FindZero tolerance tol and iteration cap
 * max_iter (the paper uses tol = 1, max_iter = 10).  tp, t0, t1 nullable. */
int oracle_method_batch(int64_t n, const double* v, const double* x, int nbins, double log_eps,
                        int halve_ok, double tol, int max_iter, double* logk, double* tp,
                        double* t0, double* t1, int nthreads) {
  if (n < 0 || (n > 0 && (!v || !x || !logk)) || nbins < 1 || !(log_eps < 0.0) || max_iter < 1)
    return -1;
  method_args a = {v, x, nbins, log_eps, halve_ok, tol, max_iter, logk, tp, t0, t1};
  run_pool(method_elem, &a, n, nthreads);
  return 0;
}

/* ---------------------------------------------------------------------- */
/* Brute-force check: a plain trapezoid with nbins bins over [lo, hi] of the */
/* three integrands, unscaled by any peak (for small tests of the adaptive   */
/* rule).  Returns log of the three integrals' values (I1 divided by its    */
/* sign convention as in logk_one).                                         */
/* ---------------------------------------------------------------------- */

int oracle_trapezoid_brute(double vin, double xin, double lo, double hi, int64_t nbins, double out[3]) {
  if (nbins < 1 || !(hi > lo) || !(xin > 0.0)) return -1;
  ld v = fabsl((ld)vin), x = (ld)xin;
  ld tp = exact_peak(v, x);
  ld G = g_vx(v, x, tp);
  ld h = ((ld)hi - (ld)lo) / (ld)nbins;
  ld s0 = 0.0L, s1 = 0.0L, s2 = 0.0L;
  for (int64_t m = 0; m <= nbins; ++m) {
    ld t = (ld)lo + (ld)m * h;
    ld w = (m == 0 || m == nbins) ? 0.5L : 1.0L;
    ld e = w * expl(g_vx(v, x, t) - G);
    s0 += e;
    s1 += t * tanhl(v * t) * e;
    s2 += coshl(t) * e;
  }
  out[0] = (double)(G + logl(h * s0));
  out[1] = (double)(s1 / s0);
  out[2] = (double)(-s2 / s0);
  return 0;
}

/* ---------------------------------------------------------------------- */
/* (3) General derivatives of K itself (Section 4.1, Eq. (13)), each over  */
/*     its own integrand's peak and truncation interval.                    */
/*                                                                          */
/* For orders a (in v) and b (in x), differentiating under the integral of  */
/* Eq. (1):                                                                 */
/*   d^a/dv^a d^b/dx^b K_v(x) = (-1)^b int_0^inf t^a cosh^b(t) C_a(v t)     */
/*                                          exp(-x cosh t) dt,              */
/* C_a = cosh for even a and sinh for odd a.  With v >= 0 the integrand is  */
/* >= 0, and its log                                                        */
/*   g_ab(t) = a log t + b log cosh t + log C_a(v t) - x cosh t             */
/* has one peak (g_ab' = sinh(t) (phi(t) - x) with                          */
/* phi = (a/t + b tanh t + v T(v t)) / sinh t strictly decreasing; T = tanh */
/* for even a and coth for odd a), as the text states for these integrands. */
/* The oracle integrates exp(g_ab - G_ab) by the same adaptive              */
/* Gauss-Legendre rule over the integrand's own interval at 60 nats below   */
/* its own peak, both found by bisection.  The sign of the derivative is     */
/* (-1)^b, times sign(v) for odd a; for odd a at v = 0 it is exactly zero.   */
/* ---------------------------------------------------------------------- */

/* log sinh z for z > 0, accurate as z -> 0: z - log 2 + log(1 - e^{-2z}). */
static ld log_sinh(ld z) { return z - LN2L + logl(-expm1l(-2.0L * z)); }

typedef struct { ld v, x; int a, b; } gab_fn;

static ld gab_val(const gab_fn* f, ld t) {
  if (t <= 0.0L) return (f->a == 0) ? -f->x : -INFINITY;  /* a = 0: g(0) = -x */
  ld vt = f->v * t;
  ld lc = (f->a & 1) ? log_sinh(vt) : log_cosh(vt);
  return (ld)f->a * logl(t) + (ld)f->b * log_cosh(t) + lc - f->x * coshl(t);
}

static ld gab_der(const gab_fn* f, ld t) {
  ld vt = f->v * t;
  ld T = (f->a & 1) ? 1.0L / tanhl(vt) : tanhl(vt);
  return (ld)f->a / t + (ld)f->b * tanhl(t) + f->v * T - f->x * sinhl(t);
}

/* Peak: at 0 when a = 0 and b + v^2 <= x (g_ab'' (0) = b + v^2 - x <= 0 and
 * phi decreasing), otherwise the single root of g_ab' in (0, inf). */
static ld gab_peak(const gab_fn* f) {
  if (f->a == 0 && (ld)f->b + f->v * f->v <= f->x) return 0.0L;
  ld hi = 1.0L, lo;
  while (gab_der(f, hi) > 0.0L) hi *= 2.0L;
  lo = hi;
  while (lo > 0.0L && !(gab_der(f, lo) > 0.0L)) lo *= 0.5L;
  for (int it = 0; it < 400; ++it) {
    ld mid = 0.5L * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (gab_der(f, mid) > 0.0L) lo = mid; else hi = mid;
  }
  return 0.5L * (lo + hi);
}

/* Level crossing of g_ab = G - L between p (F >= 0) and q (F < 0). */
static ld gab_cross(const gab_fn* f, ld G, ld L, ld p, ld q) {
  for (int it = 0; it < 400; ++it) {
    ld mid = 0.5L * (p + q);
    if (mid == p || mid == q) break;
    if (gab_val(f, mid) - G + L >= 0.0L) p = mid; else q = mid;
  }
  return q;
}

static void gab_panel(const gab_fn* f, ld G, ld a, ld b, ld* r) {
  ld mid = 0.5L * (a + b), hw = 0.5L * (b - a), s = 0.0L;
  for (int i = 0; i < GL_N; ++i) s += gl_wt[i] * expl(gab_val(f, mid + hw * gl_node[i]) - G);
  *r = hw * s;
}

static void gab_adapt(const gab_fn* f, ld G, ld tol, ld a, ld b, ld whole, int depth, ld* acc) {
  ld m = 0.5L * (a + b), left, right;
  gab_panel(f, G, a, m, &left);
  gab_panel(f, G, m, b, &right);
  if (fabsl(left + right - whole) <= tol || depth >= 48 || m <= a || m >= b) {
    *acc += left + right;
    return;
  }
  gab_adapt(f, G, tol, a, m, left, depth + 1, acc);
  gab_adapt(f, G, tol, m, b, right, depth + 1, acc);
}

static double logdk_one(double vin, double xin, int a, int b, double* sign) {
  if (isnan(vin) || isnan(xin) || xin < 0.0) { *sign = NAN; return NAN; }
  double s = (b & 1) ? -1.0 : 1.0;
  if ((a & 1) && vin < 0.0) s = -s;
  if ((a & 1) && vin == 0.0) { *sign = 0.0; return -INFINITY; }
  *sign = s;
  if (xin == 0.0) return INFINITY;
  if (isinf(xin)) return -INFINITY;
  if (isinf(vin)) return INFINITY;
  gab_fn f = {fabsl((ld)vin), (ld)xin, a, b};
  ld tp = gab_peak(&f);
  ld G = gab_val(&f, tp);
  ld L = ORACLE_MARGIN;
  ld lo = 0.0L, hi;
  if (tp > 0.0L && !(gab_val(&f, 0.0L) - G + L >= 0.0L)) lo = gab_cross(&f, G, L, tp, 0.0L);
  ld step = (tp > 0.0L) ? tp : 1.0L;
  while (gab_val(&f, tp + step) - G + L >= 0.0L) step *= 2.0L;
  hi = gab_cross(&f, G, L, tp, tp + step);
  /* 8 panels per side; absolute tolerance 4e-18 of the coarse estimate */
  const int P = 8;
  ld edges[2][2] = {{lo, tp}, {tp, hi}}, est = 0.0L, acc = 0.0L;
  for (int e = 0; e < 2; ++e)
    for (int p = 0; p < P && edges[e][1] > edges[e][0]; ++p) {
      ld r, pa = edges[e][0] + (edges[e][1] - edges[e][0]) * p / P;
      gab_panel(&f, G, pa, edges[e][0] + (edges[e][1] - edges[e][0]) * (p + 1) / P, &r);
      est += r;
    }
  ld tol = 4e-18L * est;
  for (int e = 0; e < 2; ++e)
    for (int p = 0; p < P && edges[e][1] > edges[e][0]; ++p) {
      ld pa = edges[e][0] + (edges[e][1] - edges[e][0]) * p / P;
      ld pb = edges[e][0] + (edges[e][1] - edges[e][0]) * (p + 1) / P, whole;
      gab_panel(&f, G, pa, pb, &whole);
      gab_adapt(&f, G, tol, pa, pb, whole, 0, &acc);
    }
  return (double)(G + logl(acc));
}

typedef struct { const double *v, *x; int a, b; double *out, *sign; } dk_args;

static void dk_elem(void* ctx, int64_t i) {
  dk_args* d = (dk_args*)ctx;
  double s;
  d->out[i] = logdk_one(d->v[i], d->x[i], d->a, d->b, &s);
  if (d->sign) d->sign[i] = s;
}

/* log |d^a/dv^a d^b/dx^b K_v(x)| for n pairs, and (nullable) its sign.
 * Conventions: NaN v or x, or x < 0 -> NaN (sign NaN); odd a at v = 0 ->
 * -inf (sign 0: the derivative is zero); x == 0 -> +inf; x == +inf -> -inf;
 * |v| == inf -> +inf. */
int oracle_logdk_batch(int64_t n, const double* v, const double* x, int a, int b, double* out,
                       double* sign, int nthreads) {
  if (n < 0 || a < 0 || b < 0 || (n > 0 && (!v || !x || !out))) return -1;
  dk_args d = {v, x, a, b, out, sign};
  run_pool(dk_elem, &d, n, nthreads);
  return 0;
}
