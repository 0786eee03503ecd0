/*
 * ta_oracle.c -- plain FP64 CPU oracle for the piecewise trigonometric
 * approximations of Goyal & Arora, "A Novel SIMD-Optimized Implementation for
 * Fast and Memory-Efficient Trigonometric Computation" (arXiv 2502.10831).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  The GPU library never
 * links, includes or calls anything here, and this file includes nothing from
 * the GPU sources: the two share no code, tables or constants.
 *
 * Every function is a direct, slow, obviously-correct statement of what the
 * paper defines, evaluated in IEEE double with libm.  Where the paper is silent
 * the reading taken is stated next to the code.
 *
 * Readings of the paper used here (each one also listed in the design notes):
 *  R1  Coefficients.  Section 2 prints radian coefficients truncated to two
 *      decimals and says full precision was used.  Appendix A (eqs. 5-10)
 *      gives every segment as tan t = (a t + b)/(c t + d) with small integer
 *      a, b, c, d and t in degrees.  The radian coefficients are a*180/pi and
 *      c*180/pi with b, d unchanged, so the unrounded coefficients are the integer form
 *      with t = rho*180/pi.  (The tests check that truncating these values to
 *      two decimals gives all 42 numbers printed in Section 2.)
 *  R2  Reduction.  Section 3 reduces the angle to [0, pi/2] "along with the
 *      resulting sign" and the pseudocode returns sign * f(red).  The only
 *      fold for which sign*f(red) can equal sin, cos and tan in every quadrant
 *      is red = arcsin|sin x| = arccos|cos x|, with the signs of sin x and
 *      cos x.  It is computed here from libm sin/cos with atan2, which gives
 *      both red and its complement pi/2 - red to full relative precision.
 *  R3  Segment index.  The pseudocode divides by 0.261; Section 2 defines the
 *      pieces on uniform pi/12 intervals.  The index is floor(red/(pi/12)),
 *      with red = pi/2 placed in the last piece (closed at pi/2).
 *  R4  Square root and reciprocal.  Section 3 replaces them by the fast
 *      inverse square root (Algorithm 1).  The oracle of the method uses true
 *      sqrt and division; the FISR form is provided separately
 *      (ta_or_*_fisr) because it is what the paper's error tables measured.
 *  R5  Pieces above 45 degrees are evaluated about the 90-degree end:
 *      a t + b = (90 a + b) - a w with w = 90 - t, which is the same affine
 *      function (exact algebra) but keeps D = c t + d accurate near the pole
 *      where c*90 + d = 0 for the last piece.
 *  R6  Tan guard.  proposed_tan returns +inf when |red - pi/2| < 1e-3, before
 *      the sign is applied.  Off by default; TA_OR_TAN_GUARD turns it on.
 *  R7  Specials (paper silent): NaN or +-Inf in -> NaN out; sin and tan keep
 *      the sign of a zero input, cos(+-0) = 1.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define TA_OR_TAN_GUARD 1u

/* Appendix A integer coefficients, degrees: tan t ~ (a t + b)/(c t + d).
 * Piece 0: eq. (9), 0-15 deg.   Piece 1: eq. (5), 15-30 deg.
 * Piece 2: eq. (6), 30-45 deg.  Piece 3: eq. (7), 45-60 deg.
 * Piece 4: eq. (8), 60-75 deg.  Piece 5: eq. (10), 75-90 deg. */
static const double OR_A[6] = {11.0, 10.0, 6.0, 10.0, 4.0, 1.0};
static const double OR_B[6] = {0.0, 10.0, 46.0, 217.0, 297.0, 542.0};
static const double OR_C[6] = {-1.0, -4.0, -5.0, -13.0, -10.0, -11.0};
static const double OR_D[6] = {632.0, 657.0, 541.0, 1252.0, 910.0, 990.0};

/* Degrees per radian in double (the unrounded coefficients, reading R1). */
static double or_k(void) { return 180.0 / M_PI; }

/* ---- reduction (Section 3, reading R2) ---------------------------------- */

/* Fold angle rho in [0, pi/2], its complement v = pi/2 - rho (computed
 * directly, not by subtraction), and the signs of sin x and cos x. */
void ta_or_fold(double x, double *rho, double *v, int *neg_s, int *neg_c) {
  double s = sin(x), c = cos(x);
  *rho = atan2(fabs(s), fabs(c));
  *v = atan2(fabs(c), fabs(s));
  *neg_s = signbit(s) ? 1 : 0;
  *neg_c = signbit(c) ? 1 : 0;
}

/* ---- segment index (Section 2 intervals, reading R3) -------------------- */
int ta_or_segment(double rho) {
  int k = (int)floor(rho / (M_PI / 12.0));
  if (k > 5) k = 5;
  if (k < 0) k = 0;
  return k;
}

/* ---- one piece: numerator and denominator of tan (Appendix A, eqs. 5-10) ---
 * Degree units.  t = rho*180/pi, w = v*180/pi.  For pieces 3-5 the same
 * affine forms are written about 90 degrees (reading R5). */
void ta_or_piece(int k, double rho, double v, double *num, double *den) {
  double K = or_k();
  if (k <= 2) {
    double t = rho * K;
    *num = OR_A[k] * t + OR_B[k];
    *den = OR_C[k] * t + OR_D[k];
  } else {
    double w = v * K;
    *num = (90.0 * OR_A[k] + OR_B[k]) - OR_A[k] * w;
    *den = (90.0 * OR_C[k] + OR_D[k]) - OR_C[k] * w;
  }
}

/* Appendix A.4: sin = N/sqrt(N^2 + D^2), cos = D/sqrt(N^2 + D^2), tan = N/D
 * (the quadratic under the root in A.4 is N^2 + D^2 expanded).  Unsigned
 * values on [0, pi/2] for piece k. */
void ta_or_piece_scs(int k, double rho, double v, double *s, double *c,
                     double *t) {
  double n, d;
  ta_or_piece(k, rho, v, &n, &d);
  double h = sqrt(n * n + d * d);
  *s = n / h;
  *c = d / h;
  *t = n / d;
}

/* ---- the method: proposed sin / cos / tan (Section 2 + Section 3) -------- */
static void or_eval(double x, unsigned flags, double *ys, double *yc,
                    double *yt) {
  if (isnan(x) || isinf(x)) { /* reading R7 */
    *ys = *yc = *yt = NAN;
    return;
  }
  double rho, v;
  int ns, nc;
  ta_or_fold(x, &rho, &v, &ns, &nc);
  int k = ta_or_segment(rho);
  double s, c, t;
  ta_or_piece_scs(k, rho, v, &s, &c, &t);
  *ys = ns ? -s : s;
  *yc = nc ? -c : c;
  if ((flags & TA_OR_TAN_GUARD) && v < 1e-3) { /* reading R6 */
    *yt = INFINITY;
  } else {
    *yt = (ns != nc) ? -t : t;
  }
}

double ta_or_sin(double x) { double s, c, t; or_eval(x, 0, &s, &c, &t); return s; }
double ta_or_cos(double x) { double s, c, t; or_eval(x, 0, &s, &c, &t); return c; }
double ta_or_tan(double x, unsigned flags) {
  double s, c, t;
  or_eval(x, flags, &s, &c, &t);
  return t;
}

/* Array form: any of ys / yc / yt may be NULL.  nthreads <= 0 uses OpenMP's
 * default.  Returns the number of threads used. */
int ta_or_map(const double *x, int64_t n, double *ys, double *yc, double *yt,
              unsigned flags, int nthreads) {
  int used = 1;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel
  {
#pragma omp single
    used = omp_get_num_threads();
#pragma omp for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
      double s, c, t;
      or_eval(x[i], flags, &s, &c, &t);
      if (ys) ys[i] = s;
      if (yc) yc[i] = c;
      if (yt) yt[i] = t;
    }
  }
#else
  (void)nthreads;
  for (int64_t i = 0; i < n; ++i) {
    double s, c, t;
    or_eval(x[i], flags, &s, &c, &t);
    if (ys) ys[i] = s;
    if (yc) yc[i] = c;
    if (yt) yt[i] = t;
  }
#endif
  return used;
}

/* Per-element diagnostics: fold angle, complement, piece index and the
 * signs, so a checker can evaluate a neighbouring piece. */
void ta_or_fold_map(const double *x, int64_t n, double *rho, double *v,
                    int32_t *k, int32_t *neg_s, int32_t *neg_c) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double r, w;
    int a, b;
    ta_or_fold(x[i], &r, &w, &a, &b);
    rho[i] = r;
    v[i] = w;
    k[i] = ta_or_segment(r);
    neg_s[i] = a;
    neg_c[i] = b;
  }
}

/* ---- Taylor baseline (Section 3 and the Taylor columns of Tables 1-3) ----
 * Taylor-N is the first N non-zero Maclaurin terms evaluated on the same
 * folded angle rho, with the same signs as the proposed functions. */
static double or_fact(int m) {
  double f = 1.0;
  for (int i = 2; i <= m; ++i) f *= (double)i;
  return f;
}

/* Tangent-series coefficients T_{2j+1} = tan^{(2j+1)}(0)/(2j+1)! as exact
 * rationals: 1, 1/3, 2/15, 17/315, 62/2835, 1382/155925, 21844/6081075,
 * 929569/638512875, 6404582/10854718875. */
static const double OR_TAN_NUM[9] = {1.0, 1.0, 2.0, 17.0, 62.0, 1382.0,
                                     21844.0, 929569.0, 6404582.0};
static const double OR_TAN_DEN[9] = {1.0, 3.0, 15.0, 315.0, 2835.0,
                                     155925.0, 6081075.0, 638512875.0,
                                     10854718875.0};

static void or_taylor_eval(double x, int terms, double *ys, double *yc,
                           double *yt) {
  if (isnan(x) || isinf(x)) {
    *ys = *yc = *yt = NAN;
    return;
  }
  double rho, v;
  int ns, nc;
  ta_or_fold(x, &rho, &v, &ns, &nc);
  double s = 0.0, c = 0.0, t = 0.0;
  for (int j = 0; j < terms; ++j) {
    double sg = (j % 2) ? -1.0 : 1.0;
    s += sg * pow(rho, 2 * j + 1) / or_fact(2 * j + 1);
    c += sg * pow(rho, 2 * j) / or_fact(2 * j);
    t += OR_TAN_NUM[j] / OR_TAN_DEN[j] * pow(rho, 2 * j + 1);
  }
  *ys = ns ? -s : s;
  *yc = nc ? -c : c;
  *yt = (ns != nc) ? -t : t;
}

/* Also returns, per element, the sum of the absolute values of the terms
 * (scale of the rounding error of any evaluation order). */
void ta_or_taylor_map(const double *x, int64_t n, int terms, double *ys,
                      double *yc, double *yt, double *abs_s, double *abs_c,
                      double *abs_t) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double s, c, t;
    or_taylor_eval(x[i], terms, &s, &c, &t);
    if (ys) ys[i] = s;
    if (yc) yc[i] = c;
    if (yt) yt[i] = t;
    if (abs_s || abs_c || abs_t) {
      double rho, v;
      int a, b;
      double as = 0, ac = 0, at = 0;
      if (!(isnan(x[i]) || isinf(x[i]))) {
        ta_or_fold(x[i], &rho, &v, &a, &b);
        for (int j = 0; j < terms; ++j) {
          as += pow(rho, 2 * j + 1) / or_fact(2 * j + 1);
          ac += pow(rho, 2 * j) / or_fact(2 * j);
          at += OR_TAN_NUM[j] / OR_TAN_DEN[j] * pow(rho, 2 * j + 1);
        }
      }
      if (abs_s) abs_s[i] = as;
      if (abs_c) abs_c[i] = ac;
      if (abs_t) abs_t[i] = at;
    }
  }
}

/* ---- derivative of the method (Appendix A.4 differentiated) -------------
 * On piece k, with N = a t + b, D = c t + d, t = rho*K (K = 180/pi):
 *   dS/drho = K (ad - bc) D / Q^{3/2},  dC/drho = -K (ad - bc) N / Q^{3/2},
 *   dT/drho = K (ad - bc) / D^2,        Q = N^2 + D^2.
 * The fold rho = arcsin|sin x| has d rho/dx = sign(sin x) * sign(cos x), and
 * the outputs carry the signs of sin x, cos x and their product.  The value
 * returned is the derivative of the selected piece (one-sided at the
 * discontinuities at 15, 30, 60 and 75 degrees and at the kink at 45).
 * `shift` evaluates piece k + shift (clamped to 0..5) instead: next to a
 * jump node either neighbouring piece is a correct result (the boundary
 * tie-break reading), and its derivative is the neighbour's. */
static void or_grad_eval(double x, int shift, double *gs, double *gc,
                         double *gt) {
  if (isnan(x) || isinf(x)) {
    *gs = *gc = *gt = NAN;
    return;
  }
  double rho, v;
  int ns, nc;
  ta_or_fold(x, &rho, &v, &ns, &nc);
  int k = ta_or_segment(rho) + shift;
  if (k < 0) k = 0;
  if (k > 5) k = 5;
  double n, d;
  ta_or_piece(k, rho, v, &n, &d);
  double K = or_k();
  double det = OR_A[k] * OR_D[k] - OR_B[k] * OR_C[k];
  double q = n * n + d * d;
  double dS = K * det * d / (q * sqrt(q));
  double dC = -K * det * n / (q * sqrt(q));
  double dT = K * det / (d * d);
  double sig_s = ns ? -1.0 : 1.0, sig_c = nc ? -1.0 : 1.0;
  double drho_dx = sig_s * sig_c;
  *gs = sig_s * dS * drho_dx;
  *gc = sig_c * dC * drho_dx;
  *gt = sig_s * sig_c * dT * drho_dx;
}

void ta_or_grad_map(const double *x, int64_t n, int shift, double *gs,
                    double *gc, double *gt) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double a, b, c;
    or_grad_eval(x[i], shift, &a, &b, &c);
    if (gs) gs[i] = a;
    if (gc) gc[i] = b;
    if (gt) gt[i] = c;
  }
}

/* ---- the paper's literal arithmetic (Section 3, Algorithms 1-4) ---------
 * Radian coefficients a*K, c*K; sin/cos helpers multiply the linear form by
 * the fast inverse square root of the quadratic; the tan helper multiplies by
 * the square of the fast inverse square root of the denominator.  `divisor`
 * is the piece width used for the index (pi/12, or the pseudocode's 0.261;
 * the index is clamped to the last piece).  Returns unsigned values on
 * [0, pi/2] for the folded angle rho; used only to reproduce the error
 * columns of Tables 1-3. */
static double or_fisr(double number) {
  /* Algorithm 1: magic constant, one Newton-Raphson step. */
  double x2 = number * 0.5;
  int64_t i;
  memcpy(&i, &number, sizeof i);
  i = (int64_t)0x5fe6eb50c7b537a9LL - (i >> 1);
  double y;
  memcpy(&y, &i, sizeof y);
  y = y * (1.5 - (x2 * y * y));
  return y;
}

/* Algorithms 2-4 on one folded angle `ang` in [0, pi/2]: piece index
 * floor(ang/divisor) (clamped to the last piece), radian coefficients
 * a = a_k*K, c = c_k*K with b, d unchanged, the quadratic x ang^2 + y ang + z
 * with x = a^2 + c^2, y = 2(ab + cd), z = b^2 + d^2 (Appendix A.4), and the
 * fast inverse square root in place of 1/sqrt and of the division. */
static void or_fisr_eval(double ang, double divisor, double *ys, double *yc,
                         double *yt) {
  double K = or_k();
  int k = (int)floor(ang / divisor);
  if (k > 5) k = 5;
  if (k < 0) k = 0;
  double a = OR_A[k] * K, b = OR_B[k], c = OR_C[k] * K, d = OR_D[k];
  double qx = a * a + c * c, qy = 2.0 * (a * b + c * d), qz = b * b + d * d;
  double poly_s = a * ang + b;          /* Algorithm 2: poly */
  double ang2 = ang * ang;              /* Algorithm 2: ang2 */
  double inner = qx * ang2 + qy * ang + qz;
  double inv = or_fisr(inner);
  *ys = poly_s * inv;
  double poly_c = c * ang + d;          /* Algorithm 3 */
  *yc = poly_c * inv;
  double tmp = or_fisr(c * ang + d);    /* Algorithm 4 */
  *yt = poly_s * (tmp * tmp);
}

void ta_or_fisr_map(const double *rho, int64_t n, double divisor, double *ys,
                    double *yc, double *yt) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double s, c, t;
    or_fisr_eval(rho[i], divisor, &s, &c, &t);
    if (ys) ys[i] = s;
    if (yc) yc[i] = c;
    if (yt) yt[i] = t;
  }
}

/* The paper's arithmetic on angles x: the Section 3 fold and signs around
 * or_fisr_eval, and proposed_tan's guard (+inf, unsigned, when the folded
 * angle is within 1e-3 of pi/2) when TA_OR_TAN_GUARD is set. */
void ta_or_paper_map(const double *x, int64_t n, double divisor,
                     unsigned flags, double *ys, double *yc, double *yt) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double s = NAN, c = NAN, t = NAN;
    if (!(isnan(x[i]) || isinf(x[i]))) {
      double rho, v;
      int ns, nc;
      ta_or_fold(x[i], &rho, &v, &ns, &nc);
      or_fisr_eval(rho, divisor, &s, &c, &t);
      s = ns ? -s : s;
      c = nc ? -c : c;
      t = (ns != nc) ? -t : t;
      if ((flags & TA_OR_TAN_GUARD) && v < 1e-3) t = INFINITY;
    }
    if (ys) ys[i] = s;
    if (yc) yc[i] = c;
    if (yt) yt[i] = t;
  }
}

/* ---- the method in extended precision ------------------------------------
 * The same definitions (readings R1-R7) evaluated in x87 long double (64-bit
 * significand) from double inputs, to check FP64 outputs: each result here is
 * within a few units of 2^-64 of the exact value of the formulas at x, about
 * 2^-10 of an FP64 ulp.  glibc's sinl/cosl reduce any double argument
 * accurately, so the fold keeps full relative precision near the zeros of
 * sin and cos.  `shift` evaluates the piece k + shift (clamped to 0..5)
 * instead of the piece k that rho falls in: a checker uses shift = -1 and +1
 * for inputs whose rho is within rounding distance of a piece boundary. */
static long double or_kl(void) { return 180.0L / acosl(-1.0L); }

void ta_or_fold_ld(double x, long double *rho, long double *v, int *neg_s,
                   int *neg_c) {
  long double s = sinl((long double)x), c = cosl((long double)x);
  *rho = atan2l(fabsl(s), fabsl(c));
  *v = atan2l(fabsl(c), fabsl(s));
  *neg_s = signbit(s) ? 1 : 0;
  *neg_c = signbit(c) ? 1 : 0;
}

static int or_segment_ld(long double rho) {
  int k = (int)floorl(rho / (acosl(-1.0L) / 12.0L));
  if (k > 5) k = 5;
  if (k < 0) k = 0;
  return k;
}

static void or_piece_ld(int k, long double rho, long double v,
                        long double *num, long double *den) {
  long double K = or_kl();
  if (k <= 2) {
    long double t = rho * K;
    *num = (long double)OR_A[k] * t + (long double)OR_B[k];
    *den = (long double)OR_C[k] * t + (long double)OR_D[k];
  } else {
    long double w = v * K;
    *num = (90.0L * OR_A[k] + OR_B[k]) - (long double)OR_A[k] * w;
    *den = (90.0L * OR_C[k] + OR_D[k]) - (long double)OR_C[k] * w;
  }
}

static void or_eval_ld(double x, unsigned flags, int shift, long double *ys,
                       long double *yc, long double *yt) {
  if (isnan(x) || isinf(x)) {
    *ys = *yc = *yt = NAN;
    return;
  }
  long double rho, v;
  int ns, nc;
  ta_or_fold_ld(x, &rho, &v, &ns, &nc);
  int k = or_segment_ld(rho) + shift;
  if (k < 0) k = 0;
  if (k > 5) k = 5;
  long double n, d;
  or_piece_ld(k, rho, v, &n, &d);
  long double h = sqrtl(n * n + d * d);
  long double s = n / h, c = d / h, t = n / d;
  *ys = ns ? -s : s;
  *yc = nc ? -c : c;
  if ((flags & TA_OR_TAN_GUARD) && v < 1e-3L) {
    *yt = INFINITY;
  } else {
    *yt = (ns != nc) ? -t : t;
  }
}

int ta_or_map_ld(const double *x, int64_t n, long double *ys, long double *yc,
                 long double *yt, unsigned flags, int shift) {
  int used = 1;
#pragma omp parallel
  {
#ifdef _OPENMP
#pragma omp single
    used = omp_get_num_threads();
#endif
#pragma omp for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
      long double s, c, t;
      or_eval_ld(x[i], flags, shift, &s, &c, &t);
      if (ys) ys[i] = s;
      if (yc) yc[i] = c;
      if (yt) yt[i] = t;
    }
  }
  return used;
}

/* Fold angle, complement (both long double) and piece index per element. */
void ta_or_fold_map_ld(const double *x, int64_t n, long double *rho,
                       long double *v, int32_t *k) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    long double r = NAN, w = NAN;
    int a, b;
    if (!(isnan(x[i]) || isinf(x[i]))) ta_or_fold_ld(x[i], &r, &w, &a, &b);
    rho[i] = r;
    v[i] = w;
    k[i] = isnan(r) ? -1 : or_segment_ld(r);
  }
}

/* Derivative of the selected piece (as ta_or_grad_map) in long double;
 * `shift` as in ta_or_map_ld. */
static void or_grad_eval_ld(double x, int shift, long double *gs,
                            long double *gc, long double *gt) {
  if (isnan(x) || isinf(x)) {
    *gs = *gc = *gt = NAN;
    return;
  }
  long double rho, v;
  int ns, nc;
  ta_or_fold_ld(x, &rho, &v, &ns, &nc);
  int k = or_segment_ld(rho) + shift;
  if (k < 0) k = 0;
  if (k > 5) k = 5;
  long double n, d;
  or_piece_ld(k, rho, v, &n, &d);
  long double det = (long double)OR_A[k] * OR_D[k] -
                    (long double)OR_B[k] * OR_C[k];
  long double q = n * n + d * d;
  long double Kdet = or_kl() * det;
  long double dS = Kdet * d / (q * sqrtl(q));
  long double dC = -Kdet * n / (q * sqrtl(q));
  long double dT = Kdet / (d * d);
  long double sig_s = ns ? -1.0L : 1.0L, sig_c = nc ? -1.0L : 1.0L;
  long double drho_dx = sig_s * sig_c;
  *gs = sig_s * dS * drho_dx;
  *gc = sig_c * dC * drho_dx;
  *gt = sig_s * sig_c * dT * drho_dx;
}

void ta_or_grad_map_ld(const double *x, int64_t n, int shift, long double *gs,
                       long double *gc, long double *gt) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    long double a, b, c;
    or_grad_eval_ld(x[i], shift, &a, &b, &c);
    if (gs) gs[i] = a;
    if (gc) gc[i] = b;
    if (gt) gt[i] = c;
  }
}
