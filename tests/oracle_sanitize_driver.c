/* Drives every entry point of the CPU oracle (oracle/dfpr_oracle.c) on
 * small graphs, including the degenerate cases (one vertex, no edges, an
 * empty batch, a batch touching every vertex), for a build with
 * AddressSanitizer and UndefinedBehaviorSanitizer.  Test infrastructure:
 * compiled and run by tests/test_oracle_sanitized.py.  Exits 0 when every
 * call succeeds and every rank vector is finite and sums to 1. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_pagerank(int32_t, int64_t, const int32_t *, const int32_t *, double,
                    double, int32_t, int32_t, const double *, double *,
                    int32_t *, double *, double *);
int oracle_df_bb(int32_t, int64_t, const int32_t *, const int32_t *, int64_t,
                 const int32_t *, const int32_t *, int64_t, const int32_t *,
                 const uint8_t *, const double *, double, double, double,
                 int32_t, double *, uint8_t *, int32_t *, double *, int64_t *,
                 int64_t *, int64_t *);
int oracle_dt_bb(int32_t, int64_t, const int32_t *, const int32_t *, int64_t,
                 const int32_t *, const int32_t *, int64_t, const int32_t *,
                 const double *, double, double, int32_t, double *, uint8_t *,
                 int32_t *, double *, int64_t *, int64_t *, int64_t *);
int oracle_residual(int32_t, int64_t, const int32_t *, const int32_t *, double,
                    const double *, int32_t, double *, double *);

static int bad = 0;

static void check(const char *what, int rc, const double *R, int32_t n) {
  double s = 0.0;
  int finite = 1;
  for (int32_t v = 0; v < n; ++v) {
    s += R[v];
    if (!isfinite(R[v])) finite = 0;
  }
  if (rc != 0 || !finite || fabs(s - 1.0) > 1e-9) {
    printf("%s: rc=%d finite=%d sum=%.17g\n", what, rc, finite, s);
    bad = 1;
  }
}

/* ring 0->1->...->n-1->0, chords v->(3v+1)%n, and a self-loop on every
 * vertex (the loops are explicit for the oracle) */
static int64_t make_graph(int32_t n, int32_t *src, int32_t *dst, int drop_every) {
  int64_t m = 0;
  for (int32_t v = 0; v < n; ++v) {
    src[m] = v; dst[m] = v; ++m;
    if (n > 1 && (drop_every == 0 || v % drop_every != 0)) {
      src[m] = v; dst[m] = (v + 1) % n; ++m;
    }
    int32_t c = (int32_t)((3 * (int64_t)v + 1) % n);
    if (c != v && c != (v + 1) % n) { src[m] = v; dst[m] = c; ++m; }
  }
  return m;
}

static void run(int32_t n) {
  const double alpha = 0.85, tol = 1e-10;
  int32_t *ps = malloc(sizeof(int32_t) * 3 * (size_t)n);
  int32_t *pd = malloc(sizeof(int32_t) * 3 * (size_t)n);
  int32_t *cs = malloc(sizeof(int32_t) * 3 * (size_t)n);
  int32_t *cd = malloc(sizeof(int32_t) * 3 * (size_t)n);
  int32_t *srcs = malloc(sizeof(int32_t) * (size_t)n);
  double *R0 = malloc(sizeof(double) * (size_t)n);
  double *R1 = malloc(sizeof(double) * (size_t)n);
  uint8_t *aff = malloc((size_t)n);
  uint8_t *marks = calloc((size_t)n, 1);
  int32_t it = 0;
  double a = 0, b = 0;
  int64_t im = 0, wv = 0, we = 0;
  const int64_t mp = make_graph(n, ps, pd, 0);
  const int64_t mc = make_graph(n, cs, cd, 4);   /* every 4th ring edge deleted */
  int64_t nb = 0;
  for (int32_t v = 0; v < n; v += 4) srcs[nb++] = v;
  char what[64];
  snprintf(what, sizeof what, "pagerank n=%d", n);
  check(what, oracle_pagerank(n, mp, ps, pd, alpha, 1e-13, 500, 1, NULL, R0, &it, &a, &b),
        R0, n);
  snprintf(what, sizeof what, "residual n=%d", n);
  if (oracle_residual(n, mp, ps, pd, alpha, R0, 1, &a, &b) != 0 || a > 1e-12) {
    printf("%s: linf=%g\n", what, a);
    bad = 1;
  }
  snprintf(what, sizeof what, "df n=%d", n);
  check(what, oracle_df_bb(n, mp, ps, pd, mc, cs, cd, nb, srcs, NULL, R0, alpha, tol,
                           tol / 1000, 500, R1, aff, &it, &a, &im, &wv, &we), R1, n);
  snprintf(what, sizeof what, "df empty batch n=%d", n);
  check(what, oracle_df_bb(n, mp, ps, pd, mp, ps, pd, 0, srcs, NULL, R0, alpha, tol,
                           tol / 1000, 500, R1, NULL, &it, &a, &im, &wv, &we), R1, n);
  for (int32_t v = 0; v < n; ++v) marks[v] = 1;
  snprintf(what, sizeof what, "df all marked n=%d", n);
  check(what, oracle_df_bb(n, mp, ps, pd, mc, cs, cd, 0, srcs, marks, R0, alpha, tol,
                           tol / 1000, 500, R1, aff, &it, &a, &im, &wv, &we), R1, n);
  snprintf(what, sizeof what, "dt n=%d", n);
  check(what, oracle_dt_bb(n, mp, ps, pd, mc, cs, cd, nb, srcs, R0, alpha, tol, 500, R1,
                           aff, &it, &a, &im, &wv, &we), R1, n);
  snprintf(what, sizeof what, "dt empty batch n=%d", n);
  check(what, oracle_dt_bb(n, mp, ps, pd, mp, ps, pd, 0, srcs, R0, alpha, tol, 500, R1,
                           NULL, &it, &a, &im, &wv, &we), R1, n);
  free(ps); free(pd); free(cs); free(cd); free(srcs); free(R0); free(R1); free(aff);
  free(marks);
}

int main(void) {
  const int32_t sizes[] = {1, 2, 7, 64, 1000};
  for (size_t i = 0; i < sizeof sizes / sizeof sizes[0]; ++i) run(sizes[i]);
  /* a bad argument is rejected, not read */
  double R[1];
  int32_t it;
  double a, b;
  const int32_t s = 5, d = 0;
  if (oracle_pagerank(1, 1, &s, &d, 0.85, 1e-13, 10, 1, NULL, R, &it, &a, &b) != -1) {
    printf("out-of-range edge accepted\n");
    bad = 1;
  }
  if (!bad) printf("oracle sanitized run ok\n");
  return bad;
}
