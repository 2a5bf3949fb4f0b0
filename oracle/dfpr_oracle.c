/*
 * CPU oracle for Dynamic Frontier PageRank -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously correct fp64 code that the tests, the smoke check
 * and the benchmark's CPU-baseline leg use to check the HIP library.  The
 * product path never links, loads or calls it; it shares no code, header or
 * table with the HIP sources.
 *
 * Everything follows "Lock-Free Computation of PageRank in Dynamic Graphs"
 * (arXiv 2407.19562):
 *   - Eq. 1 (Section 3.1): R[v] = alpha * sum_{u in in(v)} R[u]/|out(u)|
 *                                 + (1 - alpha)/n, every R starting at 1/n.
 *   - Algorithm 3 (Static, barrier-based): Jacobi sweeps with two vectors,
 *     stop on the L-infinity change.  Here the stop is on the L1 change
 *     instead, tight enough (default 1e-13) that the result is the fixed
 *     point to near fp64 rounding; the column-stochastic transition matrix
 *     makes every sweep an alpha-contraction in L1, so the L1 error bound is
 *     alpha/(1-alpha) times the last L1 change.
 *   - Algorithm 1 (DF, barrier-based): initial marking of the out-neighbours
 *     of every batch source in the previous and current graph, then Jacobi
 *     sweeps over the affected set; a vertex whose rank moves by more than
 *     the frontier tolerance marks its out-neighbours; stop when the
 *     L-infinity change of a sweep is <= tol.
 *   - Algorithm 7 (Dynamic Traversal, barrier-based; Section 3.5.2): every
 *     vertex reachable in the current graph from those out-neighbours is
 *     affected, then the same sweeps without any further marking.
 *
 * Graphs arrive as CSR built here by a counting sort.  The caller (the
 * Python layer of the oracle) supplies edge sets that already carry the
 * self-loops of Section 5.1.3 when that reading is wanted.
 *
 * Parity pins for every function live in the CPU tests: closed forms,
 * the sum-to-one invariant, dense linear solves, brute force over all
 * 4-vertex digraphs, the marking example of Section 4.1.2 (and, derived
 * by hand from Algorithm 7, its traversal marking), reachability from a
 * library breadth-first search, and which ranks a change can move.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Counting sort of the edges by `key` (dst for in-rows, src for out-rows):
 * off[n+1] row offsets, col[m] the other endpoint.  Rows keep input order. */
static void build_csr(int32_t n, int64_t m, const int32_t *key,
                      const int32_t *other, int64_t *off, int32_t *col) {
  memset(off, 0, sizeof(int64_t) * ((size_t)n + 1));
  for (int64_t e = 0; e < m; ++e) off[key[e] + 1]++;
  for (int32_t v = 0; v < n; ++v) off[v + 1] += off[v];
  int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
  memcpy(fill, off, sizeof(int64_t) * (size_t)n);
  for (int64_t e = 0; e < m; ++e) col[fill[key[e]]++] = other[e];
  free(fill);
}

/* Returns 0 on success, -1 on a bad argument, -2 on allocation failure. */
static int check_edges(int32_t n, int64_t m, const int32_t *src,
                       const int32_t *dst) {
  if (n <= 0 || m < 0) return -1;
  for (int64_t e = 0; e < m; ++e)
    if (src[e] < 0 || src[e] >= n || dst[e] < 0 || dst[e] >= n) return -1;
  return 0;
}

int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* One Jacobi sweep of Eq. 1 over every vertex: Rn <- T(R).  in-rows via
 * (ioff, icol); outdeg[u] = |out(u)| in the given edge set. */
static void jacobi_sweep(int32_t n, const int64_t *ioff, const int32_t *icol,
                         const int64_t *outdeg, double alpha, const double *R,
                         double *Rn) {
  const double base = (1.0 - alpha) / (double)n;
#pragma omp parallel for schedule(dynamic, 2048)
  for (int32_t v = 0; v < n; ++v) {
    double r = base;
    for (int64_t k = ioff[v]; k < ioff[v + 1]; ++k) {
      int32_t u = icol[k];
      r += alpha * R[u] / (double)outdeg[u];
    }
    Rn[v] = r;
  }
}

/*
 * Static PageRank (Eq. 1, Algorithm 3) on the edge set (src, dst).
 * R starts at 1/n (or at `init` when non-null).  Sweeps until the L1
 * change is <= l1_tol or max_iters sweeps were made.  threads <= 0 keeps
 * the OpenMP default.  Outputs: R_out[n], *iters, *last_l1, *last_linf.
 */
int oracle_pagerank(int32_t n, int64_t m, const int32_t *src,
                    const int32_t *dst, double alpha, double l1_tol,
                    int32_t max_iters, int32_t threads, const double *init,
                    double *R_out, int32_t *iters, double *last_l1,
                    double *last_linf) {
  if (check_edges(n, m, src, dst) || !R_out || !(alpha > 0 && alpha < 1))
    return -1;
#ifdef _OPENMP
  if (threads > 0) omp_set_num_threads(threads);
#endif
  int64_t *ioff = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
  int32_t *icol = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m ? m : 1));
  int64_t *outdeg = (int64_t *)calloc((size_t)n, sizeof(int64_t));
  double *Rn = (double *)malloc(sizeof(double) * (size_t)n);
  if (!ioff || !icol || !outdeg || !Rn) {
    free(ioff); free(icol); free(outdeg); free(Rn);
    return -2;
  }
  build_csr(n, m, dst, src, ioff, icol);
  for (int64_t e = 0; e < m; ++e) outdeg[src[e]]++;
  double *R = R_out;
  for (int32_t v = 0; v < n; ++v) R[v] = init ? init[v] : 1.0 / (double)n;
  int32_t it = 0;
  double l1 = INFINITY, linf = INFINITY;
  while (it < max_iters) {
    jacobi_sweep(n, ioff, icol, outdeg, alpha, R, Rn);
    ++it;
    l1 = 0.0;
    linf = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : l1) reduction(max : linf)
    for (int32_t v = 0; v < n; ++v) {
      double d = fabs(Rn[v] - R[v]);
      l1 += d;
      if (d > linf) linf = d;
    }
    memcpy(R, Rn, sizeof(double) * (size_t)n);
    if (l1 <= l1_tol) break;
  }
  if (iters) *iters = it;
  if (last_l1) *last_l1 = l1;
  if (last_linf) *last_linf = linf;
  free(ioff); free(icol); free(outdeg); free(Rn);
  return 0;
}

/*
 * Timing helper for the CPU baseline: exactly `sweeps` Jacobi sweeps of
 * Eq. 1 (no stop test) from 1/n, returning the in-edges gathered per sweep
 * in *edges_per_sweep.  The CSR build is outside the timed part the caller
 * measures only when it times oracle_sweeps_prepared; here everything runs.
 */
int oracle_sweeps(int32_t n, int64_t m, const int32_t *src,
                  const int32_t *dst, double alpha, int32_t sweeps,
                  int32_t threads, double *R_out, double *build_seconds,
                  double *sweep_seconds) {
  if (check_edges(n, m, src, dst) || !R_out) return -1;
#ifdef _OPENMP
  if (threads > 0) omp_set_num_threads(threads);
  double t0 = omp_get_wtime();
#endif
  int64_t *ioff = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
  int32_t *icol = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m ? m : 1));
  int64_t *outdeg = (int64_t *)calloc((size_t)n, sizeof(int64_t));
  double *Rn = (double *)malloc(sizeof(double) * (size_t)n);
  if (!ioff || !icol || !outdeg || !Rn) {
    free(ioff); free(icol); free(outdeg); free(Rn);
    return -2;
  }
  build_csr(n, m, dst, src, ioff, icol);
  for (int64_t e = 0; e < m; ++e) outdeg[src[e]]++;
  for (int32_t v = 0; v < n; ++v) R_out[v] = 1.0 / (double)n;
#ifdef _OPENMP
  double t1 = omp_get_wtime();
#endif
  for (int32_t s = 0; s < sweeps; ++s) {
    jacobi_sweep(n, ioff, icol, outdeg, alpha, R_out, Rn);
    memcpy(R_out, Rn, sizeof(double) * (size_t)n);
  }
#ifdef _OPENMP
  double t2 = omp_get_wtime();
  if (build_seconds) *build_seconds = t1 - t0;
  if (sweep_seconds) *sweep_seconds = t2 - t1;
#else
  if (build_seconds) *build_seconds = -1;
  if (sweep_seconds) *sweep_seconds = -1;
#endif
  free(ioff); free(icol); free(outdeg); free(Rn);
  return 0;
}

/*
 * Dynamic Frontier, barrier-based (Algorithm 1; Section 4.1).
 *
 * Inputs: the previous edge set (psrc, pdst; mp edges) and the current one
 * (csrc, cdst; mc edges), the batch sources bsrc[nb] (the u of every
 * (u, v) in the deletions and insertions), optional extra initial marks
 * marks0[n] (may be null), the previous ranks Rprev[n].
 * Marking: every v' in (G^{t-1} U G^t).out(u) for every batch source u
 * becomes affected.  Then per iteration, for every vertex affected at the
 * start of that iteration: r from Eq. 1 on G^t with the previous
 * iteration's ranks, dr = |r - R[v]|, Rnew[v] = r, and dr > ftol marks
 * every out-neighbour in G^t (taking effect from the next iteration).
 * dR = max |Rnew - R| over all vertices; swap; stop when dR <= tol or after
 * max_iters iterations.
 *
 * Outputs: R_out[n]; affected_out[n] (1 if ever affected; may be null);
 * *iters; *last_dR; initial_marked (count after the marking step);
 * *work_vertices (sum over iterations of the affected count) and
 * *work_edges (sum of in-degrees in G^t of those vertices).
 */
int oracle_df_bb(int32_t n, int64_t mp, const int32_t *psrc,
                 const int32_t *pdst, int64_t mc, const int32_t *csrc,
                 const int32_t *cdst, int64_t nb, const int32_t *bsrc,
                 const uint8_t *marks0,
                 const double *Rprev, double alpha, double tol, double ftol,
                 int32_t max_iters, double *R_out, uint8_t *affected_out,
                 int32_t *iters, double *last_dR, int64_t *initial_marked,
                 int64_t *work_vertices, int64_t *work_edges) {
  if (check_edges(n, mp, psrc, pdst) || check_edges(n, mc, csrc, cdst) ||
      !Rprev || !R_out || nb < 0)
    return -1;
  for (int64_t i = 0; i < nb; ++i)
    if (bsrc[i] < 0 || bsrc[i] >= n) return -1;
  int64_t *poff = malloc(sizeof(int64_t) * ((size_t)n + 1));
  int32_t *pcol = malloc(sizeof(int32_t) * (size_t)(mp ? mp : 1));
  int64_t *coff = malloc(sizeof(int64_t) * ((size_t)n + 1));
  int32_t *ccol = malloc(sizeof(int32_t) * (size_t)(mc ? mc : 1));
  int64_t *ioff = malloc(sizeof(int64_t) * ((size_t)n + 1));
  int32_t *icol = malloc(sizeof(int32_t) * (size_t)(mc ? mc : 1));
  uint8_t *VA = calloc((size_t)n, 1);
  uint8_t *VAnext = calloc((size_t)n, 1);
  double *R = malloc(sizeof(double) * (size_t)n);
  double *Rn = malloc(sizeof(double) * (size_t)n);
  int rc = 0;
  if (!poff || !pcol || !coff || !ccol || !ioff || !icol || !VA || !VAnext ||
      !R || !Rn) {
    rc = -2;
    goto done;
  }
  build_csr(n, mp, psrc, pdst, poff, pcol);   /* G^{t-1}.out */
  build_csr(n, mc, csrc, cdst, coff, ccol);   /* G^t.out     */
  build_csr(n, mc, cdst, csrc, ioff, icol);   /* G^t.in      */

  /* Initial marking (Algorithm 1, before the first iteration); marks0
     adds marks made elsewhere (vertex removal: the out-neighbours of the
     removed sources, which the vertex set here no longer holds). */
  if (marks0)
    for (int32_t v = 0; v < n; ++v) VA[v] = marks0[v] ? 1 : 0;
  for (int64_t i = 0; i < nb; ++i) {
    int32_t u = bsrc[i];
    for (int64_t k = poff[u]; k < poff[u + 1]; ++k) VA[pcol[k]] = 1;
    for (int64_t k = coff[u]; k < coff[u + 1]; ++k) VA[ccol[k]] = 1;
  }
  int64_t marked = 0;
  for (int32_t v = 0; v < n; ++v) marked += VA[v];
  if (initial_marked) *initial_marked = marked;

  for (int32_t v = 0; v < n; ++v) R[v] = Rn[v] = Rprev[v];
  memcpy(VAnext, VA, (size_t)n);
  const double base = (1.0 - alpha) / (double)n;
  int32_t it = 0;
  double dR = 0.0;
  int64_t wv = 0, we = 0;
  while (it < max_iters) {
    for (int32_t v = 0; v < n; ++v) {
      if (!VA[v]) continue;
      double r = base;
      for (int64_t k = ioff[v]; k < ioff[v + 1]; ++k) {
        int32_t u = icol[k];
        r += alpha * R[u] / (double)(coff[u + 1] - coff[u]);
      }
      double dr = fabs(r - R[v]);
      Rn[v] = r;
      wv += 1;
      we += ioff[v + 1] - ioff[v];
      if (dr > ftol)
        for (int64_t k = coff[v]; k < coff[v + 1]; ++k) VAnext[ccol[k]] = 1;
    }
    ++it;
    dR = 0.0;
    for (int32_t v = 0; v < n; ++v) {
      double d = fabs(Rn[v] - R[v]);
      if (d > dR) dR = d;
    }
    double *t = R; R = Rn; Rn = t;
    /* Unaffected vertices hold equal values in both vectors, and affected
       ones are rewritten every iteration, so the swap is all that is needed;
       keep the two vectors equal on vertices affected from now on. */
    for (int32_t v = 0; v < n; ++v) {
      if (VAnext[v] && !VA[v]) Rn[v] = R[v];
      VA[v] = VAnext[v];
    }
    if (dR <= tol) break;
  }
  memcpy(R_out, R, sizeof(double) * (size_t)n);
  if (affected_out) memcpy(affected_out, VA, (size_t)n);
  if (iters) *iters = it;
  if (last_dR) *last_dR = dR;
  if (work_vertices) *work_vertices = wv;
  if (work_edges) *work_edges = we;
done:
  free(poff); free(pcol); free(coff); free(ccol); free(ioff); free(icol);
  free(VA); free(VAnext); free(R); free(Rn);
  return rc;
}

/* Marks v and every vertex reachable from it in the CSR (off, col),
 * depth first with an explicit stack.  A vertex is marked when it is
 * pushed, so the stack never holds more than n entries; a vertex already
 * marked was reached by an earlier search, which marked all it reaches. */
static void visit_dfs(int32_t v, const int64_t *off, const int32_t *col,
                      uint8_t *VA, int32_t *stack) {
  if (VA[v]) return;
  int64_t top = 0;
  VA[v] = 1;
  stack[top++] = v;
  while (top > 0) {
    int32_t x = stack[--top];
    for (int64_t k = off[x]; k < off[x + 1]; ++k) {
      int32_t y = col[k];
      if (!VA[y]) {
        VA[y] = 1;
        stack[top++] = y;
      }
    }
  }
}

/*
 * Dynamic Traversal, barrier-based (Algorithm 7; Section 3.5.2).
 *
 * Inputs as for oracle_df_bb, without the frontier tolerance.
 * Marking: for every batch source u and every v' in (G^{t-1} U G^t).out(u),
 * v' and every vertex reachable from v' in G^t become affected.  Then
 * Jacobi iterations of Eq. 1 on G^t over the affected set from Rprev: per
 * iteration r for every affected v with the previous iteration's ranks,
 * Rnew[v] = r; dR = max |Rnew - R|; swap; stop when dR <= tol or after
 * max_iters iterations.  Nothing is marked during the iterations.
 *
 * Outputs: R_out[n]; affected_out[n] (may be null); *iters; *last_dR;
 * *marked (the affected count); *work_vertices and *work_edges as for
 * oracle_df_bb.
 */
int oracle_dt_bb(int32_t n, int64_t mp, const int32_t *psrc,
                 const int32_t *pdst, int64_t mc, const int32_t *csrc,
                 const int32_t *cdst, int64_t nb, const int32_t *bsrc,
                 const double *Rprev, double alpha, double tol,
                 int32_t max_iters, double *R_out, uint8_t *affected_out,
                 int32_t *iters, double *last_dR, int64_t *marked,
                 int64_t *work_vertices, int64_t *work_edges) {
  if (check_edges(n, mp, psrc, pdst) || check_edges(n, mc, csrc, cdst) ||
      !Rprev || !R_out || nb < 0)
    return -1;
  for (int64_t i = 0; i < nb; ++i)
    if (bsrc[i] < 0 || bsrc[i] >= n) return -1;
  int64_t *poff = malloc(sizeof(int64_t) * ((size_t)n + 1));
  int32_t *pcol = malloc(sizeof(int32_t) * (size_t)(mp ? mp : 1));
  int64_t *coff = malloc(sizeof(int64_t) * ((size_t)n + 1));
  int32_t *ccol = malloc(sizeof(int32_t) * (size_t)(mc ? mc : 1));
  int64_t *ioff = malloc(sizeof(int64_t) * ((size_t)n + 1));
  int32_t *icol = malloc(sizeof(int32_t) * (size_t)(mc ? mc : 1));
  uint8_t *VA = calloc((size_t)(n ? n : 1), 1);
  int32_t *stack = malloc(sizeof(int32_t) * (size_t)(n ? n : 1));
  double *R = malloc(sizeof(double) * (size_t)(n ? n : 1));
  double *Rn = malloc(sizeof(double) * (size_t)(n ? n : 1));
  int rc = 0;
  if (!poff || !pcol || !coff || !ccol || !ioff || !icol || !VA || !stack ||
      !R || !Rn) {
    rc = -2;
    goto done;
  }
  build_csr(n, mp, psrc, pdst, poff, pcol);   /* G^{t-1}.out */
  build_csr(n, mc, csrc, cdst, coff, ccol);   /* G^t.out     */
  build_csr(n, mc, cdst, csrc, ioff, icol);   /* G^t.in      */

  /* Marking (Algorithm 7, before the first iteration): searches in G^t
     from the previous and current out-neighbours of every batch source. */
  for (int64_t i = 0; i < nb; ++i) {
    int32_t u = bsrc[i];
    for (int64_t k = poff[u]; k < poff[u + 1]; ++k)
      visit_dfs(pcol[k], coff, ccol, VA, stack);
    for (int64_t k = coff[u]; k < coff[u + 1]; ++k)
      visit_dfs(ccol[k], coff, ccol, VA, stack);
  }
  int64_t cnt = 0;
  for (int32_t v = 0; v < n; ++v) cnt += VA[v];
  if (marked) *marked = cnt;

  for (int32_t v = 0; v < n; ++v) R[v] = Rn[v] = Rprev[v];
  const double base = (1.0 - alpha) / (double)n;
  int32_t it = 0;
  double dR = 0.0;
  int64_t wv = 0, we = 0;
  while (it < max_iters) {
    for (int32_t v = 0; v < n; ++v) {
      if (!VA[v]) continue;
      double r = base;
      for (int64_t k = ioff[v]; k < ioff[v + 1]; ++k) {
        int32_t u = icol[k];
        r += alpha * R[u] / (double)(coff[u + 1] - coff[u]);
      }
      Rn[v] = r;
      wv += 1;
      we += ioff[v + 1] - ioff[v];
    }
    ++it;
    dR = 0.0;
    for (int32_t v = 0; v < n; ++v) {
      double d = fabs(Rn[v] - R[v]);
      if (d > dR) dR = d;
    }
    /* unaffected vertices hold Rprev in both vectors */
    double *t = R; R = Rn; Rn = t;
    if (dR <= tol) break;
  }
  memcpy(R_out, R, sizeof(double) * (size_t)n);
  if (affected_out) memcpy(affected_out, VA, (size_t)n);
  if (iters) *iters = it;
  if (last_dR) *last_dR = dR;
  if (work_vertices) *work_vertices = wv;
  if (work_edges) *work_edges = we;
done:
  free(poff); free(pcol); free(coff); free(ccol); free(ioff); free(icol);
  free(VA); free(stack); free(R); free(Rn);
  return rc;
}

/*
 * Residual of Eq. 1 at R: max over v of |T(R)[v] - R[v]| and the L1 sum,
 * on the edge set (src, dst).  A property check usable at any size.
 */
int oracle_residual(int32_t n, int64_t m, const int32_t *src,
                    const int32_t *dst, double alpha, const double *R,
                    int32_t threads, double *linf, double *l1) {
  if (check_edges(n, m, src, dst) || !R) return -1;
#ifdef _OPENMP
  if (threads > 0) omp_set_num_threads(threads);
#endif
  int64_t *ioff = malloc(sizeof(int64_t) * ((size_t)n + 1));
  int32_t *icol = malloc(sizeof(int32_t) * (size_t)(m ? m : 1));
  int64_t *outdeg = calloc((size_t)n, sizeof(int64_t));
  double *Rn = malloc(sizeof(double) * (size_t)n);
  if (!ioff || !icol || !outdeg || !Rn) {
    free(ioff); free(icol); free(outdeg); free(Rn);
    return -2;
  }
  build_csr(n, m, dst, src, ioff, icol);
  for (int64_t e = 0; e < m; ++e) outdeg[src[e]]++;
  jacobi_sweep(n, ioff, icol, outdeg, alpha, R, Rn);
  double a = 0.0, s = 0.0;
  for (int32_t v = 0; v < n; ++v) {
    double d = fabs(Rn[v] - R[v]);
    s += d;
    if (d > a) a = d;
  }
  if (linf) *linf = a;
  if (l1) *l1 = s;
  free(ioff); free(icol); free(outdeg); free(Rn);
  return 0;
}
