/*
 * Drives every entry point of the C oracle over special values, random
 * doubles of every magnitude and the piece nodes; built with AddressSanitizer
 * and UndefinedBehaviorSanitizer by tests/test_sanitizers.py.  Exit status 0
 * when every call returned and the outputs have the expected NaN pattern.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void ta_or_fold(double x, double *rho, double *v, int *neg_s, int *neg_c);
int ta_or_segment(double rho);
void ta_or_piece(int k, double rho, double v, double *num, double *den);
void ta_or_piece_scs(int k, double rho, double v, double *s, double *c,
                     double *t);
double ta_or_sin(double x);
double ta_or_cos(double x);
double ta_or_tan(double x, unsigned flags);
int ta_or_map(const double *x, int64_t n, double *ys, double *yc, double *yt,
              unsigned flags, int nthreads);
void ta_or_fold_map(const double *x, int64_t n, double *rho, double *v,
                    int32_t *k, int32_t *neg_s, int32_t *neg_c);
void ta_or_taylor_map(const double *x, int64_t n, int terms, double *ys,
                      double *yc, double *yt, double *abs_s, double *abs_c,
                      double *abs_t);
void ta_or_grad_map(const double *x, int64_t n, int shift, double *gs,
                    double *gc, double *gt);
void ta_or_fisr_map(const double *rho, int64_t n, double divisor, double *ys,
                    double *yc, double *yt);
void ta_or_paper_map(const double *x, int64_t n, double divisor,
                     unsigned flags, double *ys, double *yc, double *yt);
int ta_or_map_ld(const double *x, int64_t n, long double *ys, long double *yc,
                 long double *yt, unsigned flags, int shift);
void ta_or_fold_map_ld(const double *x, int64_t n, long double *rho,
                       long double *v, int32_t *k);
void ta_or_grad_map_ld(const double *x, int64_t n, int shift, long double *gs,
                       long double *gc, long double *gt);

static uint64_t state = 2024873u;
static double next_uniform(void) { /* splitmix64 */
  uint64_t z = (state += 0x9e3779b97f4a7c15ull);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  z ^= z >> 31;
  return (double)(z >> 11) * 0x1p-53;
}

int main(void) {
  enum { NSPEC = 12, NRAND = 4000 };
  const int64_t n = NSPEC + NRAND;
  double *x = malloc(sizeof(double) * n);
  double *a = malloc(sizeof(double) * n), *b = malloc(sizeof(double) * n);
  double *c = malloc(sizeof(double) * n), *d = malloc(sizeof(double) * n);
  double *e = malloc(sizeof(double) * n), *f = malloc(sizeof(double) * n);
  long double *la = malloc(sizeof(long double) * n);
  long double *lb = malloc(sizeof(long double) * n);
  long double *lc = malloc(sizeof(long double) * n);
  int32_t *k = malloc(sizeof(int32_t) * n), *s1 = malloc(sizeof(int32_t) * n);
  int32_t *s2 = malloc(sizeof(int32_t) * n);
  if (!x || !a || !b || !c || !d || !e || !f || !la || !lb || !lc || !k || !s1 ||
      !s2)
    return 2;
  const double spec[NSPEC] = {0.0, -0.0, NAN, INFINITY, -INFINITY, 5e-324,
                              -5e-324, 1.7976931348623157e308, M_PI / 2,
                              M_PI / 12, M_PI / 4, 1e22};
  for (int i = 0; i < NSPEC; ++i) x[i] = spec[i];
  for (int i = 0; i < NRAND; ++i) {
    const double m = pow(10.0, -30.0 + 330.0 * next_uniform());
    x[NSPEC + i] = next_uniform() < 0.5 ? -m : m;
  }
  ta_or_map(x, n, a, b, c, 0u, 2);
  ta_or_map(x, n, a, b, c, 1u, 0);
  ta_or_fold_map(x, n, a, b, k, s1, s2);
  for (int terms = 5; terms <= 9; terms += 2)
    ta_or_taylor_map(x, n, terms, a, b, c, d, e, f);
  ta_or_grad_map(x, n, 0, a, b, c);
  ta_or_grad_map(x, n, 1, a, b, c);
  ta_or_grad_map(x, n, -1, a, b, c);
  for (int i = 0; i < n; ++i) d[i] = fabs(fmod(x[i], M_PI / 2));
  ta_or_fisr_map(d, n, M_PI / 12, a, b, c);
  ta_or_fisr_map(d, n, 0.261, a, b, c);
  ta_or_paper_map(x, n, 0.261, 1u, a, b, c);
  for (int shift = -1; shift <= 1; ++shift) {
    ta_or_map_ld(x, n, la, lb, lc, 0u, shift);
    ta_or_grad_map_ld(x, n, shift, la, lb, lc);
  }
  ta_or_fold_map_ld(x, n, la, lb, k);
  for (int kk = 0; kk < 6; ++kk) {
    double num, den, ss, cc, tt;
    ta_or_piece(kk, 0.1, M_PI / 2 - 0.1, &num, &den);
    ta_or_piece_scs(kk, 0.1, M_PI / 2 - 0.1, &ss, &cc, &tt);
  }
  double rho, v;
  int ns, nc;
  ta_or_fold(-0.0, &rho, &v, &ns, &nc);
  if (ta_or_segment(M_PI / 2) != 5 || ta_or_segment(0.0) != 0) return 3;
  /* NaN exactly for NaN and +-Inf inputs */
  ta_or_map(x, n, a, b, c, 0u, 1);
  for (int64_t i = 0; i < n; ++i) {
    const int special = isnan(x[i]) || isinf(x[i]);
    if ((isnan(a[i]) != 0) != special || (isnan(b[i]) != 0) != special) {
      fprintf(stderr, "unexpected NaN pattern at x = %a\n", x[i]);
      return 4;
    }
  }
  if (!signbit(ta_or_sin(-0.0)) || ta_or_cos(-0.0) != 1.0 ||
      !signbit(ta_or_tan(-0.0, 0u)))
    return 5;
  free(x); free(a); free(b); free(c); free(d); free(e); free(f);
  free(la); free(lb); free(lc); free(k); free(s1); free(s2);
  puts("oracle driver ok");
  return 0;
}
