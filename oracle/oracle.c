/*
 * oracle.c -- plain FP64 CPU oracle for early-abandoning pruned DTW.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path (the HIP library and
 * its Python binding) may include, link or call this file.  Only the test
 * suite, the smoke check and the benchmark's cpu_baseline leg use it.
 *
 * Every function here is the plain definition written out, in double
 * precision, with no blocking, no fusion and no pruning, except
 * oracle_eap_model(), which is a model of the paper's EAPrunedDTW line sweep
 * (Section 4, Algorithm 3) kept only to check the threshold contract and the
 * worked example's printed pruning facts; it is never used as a reference
 * value for the GPU.
 *
 * Paper: Herrmann & Webb, "Early Abandoning PrunedDTW and its application to
 * similarity search" (arXiv 2010.05371).
 *
 * Conventions (readings of the paper):
 *  - rows i = 1..lS index S, columns j = 1..lT index T (1-based, as in Eq. 1-5);
 *  - cost(a, b) = (a - b)^2 (Section 2, "usually the squared Euclidean distance");
 *  - Sakoe-Chiba window r: a cell is admissible iff |i - j| <= r (Section 2.1);
 *  - z-normalisation uses the population standard deviation; a flat window
 *    (variance at most 1e-14 of its mean square) normalises to all zeros.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_INF (INFINITY)

/* ------------------------------------------------------------------------- */
/* z-normalisation (two-pass, population sigma).                             */
/* The paper inherits this step from the UCR Suite it embeds its DTW in      */
/* (Section 5, experimental setup); it is not spelled out there.             */
/* ------------------------------------------------------------------------- */
/* A window is flat when its variance is at most 1e-14 of its mean square   */
/* E[x^2] = var + mean^2 (sigma at most 1e-7 of its RMS: variation at the    */
/* float32 rounding level of its values); a flat window normalises to zeros. */
#define ORACLE_FLAT_REL 1e-14

static int oracle_flat(double mean, double var) {
  return !(var > ORACLE_FLAT_REL * (var + mean * mean));
}

void oracle_znorm(const double *x, int64_t m, double *z) {
  double mean = 0.0;
  for (int64_t t = 0; t < m; ++t) mean += x[t];
  mean /= (double)m;
  double var = 0.0;
  for (int64_t t = 0; t < m; ++t) {
    double dv = x[t] - mean;
    var += dv * dv;
  }
  var /= (double)m;
  double sd = oracle_flat(mean, var) ? 0.0 : sqrt(var);
  for (int64_t t = 0; t < m; ++t) z[t] = (sd > 0.0) ? (x[t] - mean) / sd : 0.0;
}

/* mean and population sigma of every window (two-pass; 0 for a flat window), */
/* for the stats tests. */
void oracle_window_stats(const double *x, int64_t n, int64_t m, double *mu, double *sigma) {
  for (int64_t k = 0; k + m <= n; ++k) {
    double mean = 0.0;
    for (int64_t t = 0; t < m; ++t) mean += x[k + t];
    mean /= (double)m;
    double var = 0.0;
    for (int64_t t = 0; t < m; ++t) {
      double dv = x[k + t] - mean;
      var += dv * dv;
    }
    var /= (double)m;
    mu[k] = mean;
    sigma[k] = oracle_flat(mean, var) ? 0.0 : sqrt(var);
  }
}

/* ------------------------------------------------------------------------- */
/* Full-matrix banded DTW (Section 2, Eq. 1-5, window of Section 2.1).       */
/* M has (lS+1) x (lT+1) cells; M(0,0)=0, M(i,0)=M(0,j)=+inf, cells outside   */
/* the window are +inf and never computed.                                    */
/* ------------------------------------------------------------------------- */
typedef struct {
  double *M;       /* (lS+1)*(lT+1) */
  int64_t cap;     /* cells allocated */
} dtw_ws;

static int ws_reserve(dtw_ws *w, int64_t cells) {
  if (w->cap >= cells) return 0;
  free(w->M);
  w->M = (double *)malloc((size_t)cells * sizeof(double));
  w->cap = w->M ? cells : 0;
  return w->M ? 0 : -1;
}

static inline double min3d(double a, double b, double c) {
  double m = a < b ? a : b;
  return m < c ? m : c;
}

/* Fills the whole matrix; returns M(lS, lT). */
static double dtw_matrix(dtw_ws *w, const double *S, int64_t lS, const double *T, int64_t lT,
                         int64_t r) {
  const int64_t W = lT + 1;
  if (ws_reserve(w, (lS + 1) * W) != 0) return NAN;
  double *M = w->M;
  for (int64_t c = 0; c < (lS + 1) * W; ++c) M[c] = ORACLE_INF;
  M[0] = 0.0;
  for (int64_t i = 1; i <= lS; ++i) {
    int64_t jlo = i - r, jhi = i + r;
    if (jlo < 1) jlo = 1;
    if (jhi > lT) jhi = lT;
    for (int64_t j = jlo; j <= jhi; ++j) {
      double d = S[i - 1] - T[j - 1];
      double cost = d * d;
      M[i * W + j] = cost + min3d(M[(i - 1) * W + j], M[i * W + j - 1], M[(i - 1) * W + j - 1]);
    }
  }
  return M[lS * W + lT];
}

/* Weighted DTW (an elastic distance with DTW's recurrence and another cost,
 * the paper's closing outlook): cell (i, j) costs wt[|i-j|] (S_i - T_j)^2.
 * wt has at least max(lS, lT) entries. */
static double wdtw_matrix(dtw_ws *w, const double *S, int64_t lS, const double *T, int64_t lT,
                          int64_t r, const double *wt) {
  const int64_t W = lT + 1;
  if (ws_reserve(w, (lS + 1) * W) != 0) return NAN;
  double *M = w->M;
  for (int64_t c = 0; c < (lS + 1) * W; ++c) M[c] = ORACLE_INF;
  M[0] = 0.0;
  for (int64_t i = 1; i <= lS; ++i) {
    int64_t jlo = i - r, jhi = i + r;
    if (jlo < 1) jlo = 1;
    if (jhi > lT) jhi = lT;
    for (int64_t j = jlo; j <= jhi; ++j) {
      double d = S[i - 1] - T[j - 1];
      double cost = wt[i > j ? i - j : j - i] * d * d;
      M[i * W + j] = cost + min3d(M[(i - 1) * W + j], M[i * W + j - 1], M[(i - 1) * W + j - 1]);
    }
  }
  return M[lS * W + lT];
}

/* The modified logistic weight of weighted DTW (Jeong, Jeong & Omitaomu,
 * Pattern Recognition 2011): w(k) = 1 / (1 + exp(-g (k - mc))) for a phase
 * difference k = |i - j|, with mc half the series length (the longer one for
 * unequal lengths) and the maximum weight 1.  Fills wt[0..len). */
void oracle_wdtw_weights(int64_t len, double g, double *wt) {
  const double mc = (double)len / 2.0;
  for (int64_t k = 0; k < len; ++k) wt[k] = 1.0 / (1.0 + exp(-g * ((double)k - mc)));
}

double oracle_wdtw(const double *S, int64_t lS, const double *T, int64_t lT, int64_t r,
                   double g) {
  const int64_t L = lS > lT ? lS : lT;
  double *wt = malloc((size_t)(L > 0 ? L : 1) * sizeof(double));
  dtw_ws w = {0, 0};
  if (!wt) return NAN;
  oracle_wdtw_weights(L, g, wt);
  double v = (lS == 0 && lT == 0) ? 0.0 : (lS == 0 || lT == 0) ? ORACLE_INF
                                                                : wdtw_matrix(&w, S, lS, T, lT, r, wt);
  free(w.M);
  free(wt);
  return v;
}

/* The edit distance with real penalty, ERP (Chen & Ng, VLDB 2004), an elastic
 * distance of the kind the paper's closing outlook names: DTW's three-move
 * structure, where a diagonal move costs |S_i - T_j| and a vertical or
 * horizontal move aligns its point with the gap value g at cost |S_i - g| or
 * |T_j - g|.  Full (lS+1) x (lT+1) matrix under the Sakoe-Chiba window applied
 * to every cell, borders included: M(0,0) = 0, M(0,j) = M(0,j-1) + |T_j - g|
 * and M(i,0) = M(i-1,0) + |S_i - g| while |i - j| <= r, every cell outside the
 * window +inf; then
 *   M(i,j) = min(M(i-1,j-1) + |S_i - T_j|, M(i-1,j) + |S_i - g|, M(i,j-1) + |T_j - g|). */
double oracle_erp(const double *S, int64_t lS, const double *T, int64_t lT, int64_t r, double g) {
  const int64_t W = lT + 1;
  double *M = (double *)malloc((size_t)((lS + 1) * W) * sizeof(double));
  if (!M) return NAN;
  for (int64_t c = 0; c < (lS + 1) * W; ++c) M[c] = ORACLE_INF;
  M[0] = 0.0;
  for (int64_t j = 1; j <= lT && j <= r; ++j) M[j] = M[j - 1] + fabs(T[j - 1] - g);
  for (int64_t i = 1; i <= lS && i <= r; ++i) M[i * W] = M[(i - 1) * W] + fabs(S[i - 1] - g);
  for (int64_t i = 1; i <= lS; ++i) {
    int64_t jlo = i - r, jhi = i + r;
    if (jlo < 1) jlo = 1;
    if (jhi > lT) jhi = lT;
    for (int64_t j = jlo; j <= jhi; ++j) {
      const double diag = M[(i - 1) * W + j - 1] + fabs(S[i - 1] - T[j - 1]);
      const double up = M[(i - 1) * W + j] + fabs(S[i - 1] - g);
      const double left = M[i * W + j - 1] + fabs(T[j - 1] - g);
      M[i * W + j] = min3d(diag, up, left);
    }
  }
  const double v = M[lS * W + lT];
  free(M);
  return v;
}

/* Nearest neighbour of the query under ERP (the search of Section 2.2 with
 * the outlook's other distance): every offset k of x, its window z-normalised
 * (oracle_znorm) as the rows, the z-normalised query as the columns; the first
 * offset of the smallest distance.  Returns 0, or -1 when out of memory. */
int oracle_erp_nn_search(const double *q, int64_t m, const double *x, int64_t n, int64_t r,
                         double g, int64_t *out_k, double *out_d) {
  double *zq = malloc((size_t)m * sizeof(double)), *zc = malloc((size_t)m * sizeof(double));
  if (!zq || !zc) {
    free(zq);
    free(zc);
    return -1;
  }
  oracle_znorm(q, m, zq);
  int64_t best_k = -1;
  double best = ORACLE_INF;
  for (int64_t k = 0; k + m <= n; ++k) {
    oracle_znorm(x + k, m, zc);
    const double d = oracle_erp(zc, m, zq, m, r, g);
    if (d < best) {
      best = d;
      best_k = k;
    }
  }
  free(zq);
  free(zc);
  *out_k = best_k;
  *out_d = best;
  return 0;
}

double oracle_dtw(const double *S, int64_t lS, const double *T, int64_t lT, int64_t r) {
  if (lS == 0 && lT == 0) return 0.0;          /* Eq. 2 */
  if (lS == 0 || lT == 0) return ORACLE_INF;   /* Eq. 3-4 */
  dtw_ws w = {0, 0};
  double v = dtw_matrix(&w, S, lS, T, lT, r);
  free(w.M);
  return v;
}

/* Writes the whole (lS+1)x(lT+1) DTW matrix (for tests of single cells). */
int oracle_dtw_matrix(const double *S, int64_t lS, const double *T, int64_t lT, int64_t r,
                      double *out) {
  dtw_ws w = {0, 0};
  double v = dtw_matrix(&w, S, lS, T, lT, r);
  if (isnan(v) && !w.M) return -1;
  memcpy(out, w.M, (size_t)((lS + 1) * (lT + 1)) * sizeof(double));
  free(w.M);
  return 0;
}

/* Threshold contract (Section 2.2): the early-abandoned value is the DTW when
 * it does not exceed ub and +inf when it strictly exceeds it.  Ties are kept. */
double oracle_eap(const double *S, int64_t lS, const double *T, int64_t lT, int64_t r, double ub) {
  double v = oracle_dtw(S, lS, T, lT, r);
  return (v <= ub) ? v : ORACLE_INF;
}

/* ------------------------------------------------------------------------- */
/* Optimal warping path and its gradient (Section 2: warping path, several   */
/* optimal paths possible).  Backtrack from (lS,lT) to (1,1); among the       */
/* admissible predecessors take the smallest value, ties broken               */
/* diagonal > top (i-1,j) > left (i,j-1).                                    */
/* d DTW / d S(i) = sum over path cells (i,j) of 2(S(i)-T(j)) * gout,         */
/* d DTW / d T(j) = -sum over path cells (i,j) of 2(S(i)-T(j)) * gout.        */
/* min_gap receives the smallest relative gap between the chosen predecessor  */
/* and the best other finite predecessor along the path (a tie detector).     */
/* Returns the path length (number of cells) or -1; +inf distance => zero     */
/* gradients and length 0.                                                    */
/* ------------------------------------------------------------------------- */
int64_t oracle_dtw_grad(const double *S, int64_t lS, const double *T, int64_t lT, int64_t r,
                        double gout, double *dS, double *dT, int64_t *path_i, int64_t *path_j,
                        double *dist, double *min_gap) {
  for (int64_t i = 0; i < lS; ++i) dS[i] = 0.0;
  for (int64_t j = 0; j < lT; ++j) dT[j] = 0.0;
  if (min_gap) *min_gap = ORACLE_INF;
  if (lS == 0 || lT == 0) {
    if (dist) *dist = (lS == 0 && lT == 0) ? 0.0 : ORACLE_INF;
    return 0;
  }
  dtw_ws w = {0, 0};
  double v = dtw_matrix(&w, S, lS, T, lT, r);
  if (!w.M) return -1;
  if (dist) *dist = v;
  if (!(v < ORACLE_INF)) {
    free(w.M);
    return 0;
  }
  const int64_t W = lT + 1;
  const double *M = w.M;
  int64_t i = lS, j = lT, len = 0;
  for (;;) {
    double d = S[i - 1] - T[j - 1];
    double g = 2.0 * d * gout;
    dS[i - 1] += g;
    dT[j - 1] -= g;
    if (path_i) path_i[len] = i;
    if (path_j) path_j[len] = j;
    ++len;
    if (i == 1 && j == 1) break;
    double vd = M[(i - 1) * W + (j - 1)];
    double vt = M[(i - 1) * W + j];
    double vl = M[i * W + (j - 1)];
    double best = min3d(vd, vt, vl);
    int step; /* 0 diag, 1 top, 2 left */
    if (vd == best) step = 0;
    else if (vt == best) step = 1;
    else step = 2;
    if (min_gap) {
      double other = ORACLE_INF;
      if (step != 0 && vd < other) other = vd;
      if (step != 1 && vt < other) other = vt;
      if (step != 2 && vl < other) other = vl;
      if (other < ORACLE_INF) {
        double scale = fabs(best) > 1e-300 ? fabs(best) : 1.0;
        double gap = (other - best) / scale;
        if (gap < *min_gap) *min_gap = gap;
      }
    }
    if (step == 0) { --i; --j; }
    else if (step == 1) { --i; }
    else { --j; }
  }
  free(w.M);
  return len;
}

/* ------------------------------------------------------------------------- */
/* Multi-threaded drivers.  Threads get contiguous static slices; each slice */
/* is reduced in order, then slices are reduced in order, so the result does  */
/* not depend on the thread count.                                            */
/* ------------------------------------------------------------------------- */
typedef struct {
  const double *q;
  int64_t m;
  const double *x;
  int64_t r;
  const int64_t *offsets; /* candidate offsets to evaluate */
  int64_t lo, hi;         /* slice [lo,hi) of offsets[] */
  double *out;            /* per-offset distances (indexed like offsets[]) */
  int err;
  const double *wt;       /* weighted DTW: weights by |i-j| (NULL: DTW) */
} nn_job;

static void *nn_worker(void *arg) {
  nn_job *jb = (nn_job *)arg;
  double *zq = (double *)malloc((size_t)jb->m * sizeof(double));
  double *zc = (double *)malloc((size_t)jb->m * sizeof(double));
  dtw_ws w = {0, 0};
  if (!zq || !zc) { jb->err = -1; goto done; }
  oracle_znorm(jb->q, jb->m, zq);
  for (int64_t t = jb->lo; t < jb->hi; ++t) {
    int64_t k = jb->offsets[t];
    oracle_znorm(jb->x + k, jb->m, zc);
    double v = jb->wt ? wdtw_matrix(&w, zq, jb->m, zc, jb->m, jb->r, jb->wt)
                      : dtw_matrix(&w, zq, jb->m, zc, jb->m, jb->r);
    if (!w.M) { jb->err = -1; goto done; }
    jb->out[t] = v;
  }
done:
  free(zq);
  free(zc);
  free(w.M);
  return NULL;
}

/* Distances d_k = DTW(z(query), z(x[k..k+m)), window r) for the listed
 * offsets (Section 2.2's candidates T_1..T_m, Section 5's subsequence search).
 * Returns 0 on success. */
static int nn_dists_impl(const double *q, int64_t m, const double *x, int64_t n, int64_t r,
                         const int64_t *offsets, int64_t noff, int nthreads, double *out,
                         const double *wt);

int oracle_nn_dists(const double *q, int64_t m, const double *x, int64_t n, int64_t r,
                    const int64_t *offsets, int64_t noff, int nthreads, double *out) {
  return nn_dists_impl(q, m, x, n, r, offsets, noff, nthreads, out, NULL);
}

/* Weighted-DTW distances of the listed candidates (weights of
 * oracle_wdtw_weights for length m and parameter g). */
int oracle_nn_dists_w(const double *q, int64_t m, const double *x, int64_t n, int64_t r,
                      double g, const int64_t *offsets, int64_t noff, int nthreads,
                      double *out) {
  if (m <= 0) return -2;
  double *wt = malloc((size_t)m * sizeof(double));
  if (!wt) return -1;
  oracle_wdtw_weights(m, g, wt);
  int rc = nn_dists_impl(q, m, x, n, r, offsets, noff, nthreads, out, wt);
  free(wt);
  return rc;
}

static int nn_dists_impl(const double *q, int64_t m, const double *x, int64_t n, int64_t r,
                         const int64_t *offsets, int64_t noff, int nthreads, double *out,
                         const double *wt) {
  for (int64_t t = 0; t < noff; ++t)
    if (offsets[t] < 0 || offsets[t] + m > n) return -2;
  if (nthreads < 1) nthreads = 1;
  if (nthreads > 256) nthreads = 256;
  pthread_t th[256];
  int live[256];
  nn_job jobs[256];
  int64_t per = (noff + nthreads - 1) / nthreads;
  for (int t = 0; t < nthreads; ++t) {
    int64_t lo = (int64_t)t * per, hi = lo + per;
    if (lo > noff) lo = noff;
    if (hi > noff) hi = noff;
    jobs[t] = (nn_job){q, m, x, r, offsets, lo, hi, out, 0, wt};
    live[t] = pthread_create(&th[t], NULL, nn_worker, &jobs[t]) == 0;
    if (!live[t]) nn_worker(&jobs[t]);
  }
  int err = 0;
  for (int t = 0; t < nthreads; ++t) {
    if (live[t]) pthread_join(th[t], NULL);
    if (jobs[t].err) err = jobs[t].err;
  }
  return err;
}

/* Brute-force nearest neighbour over every offset k in [k_begin, k_end):
 * the lexicographic minimum of (d_k, k), i.e. the smallest offset among equal
 * minimal distances (a sequential scan that only replaces its best on a
 * strictly better candidate, Section 2.2). */
int oracle_nn_search(const double *q, int64_t m, const double *x, int64_t n, int64_t r,
                     int64_t k_begin, int64_t k_end, int nthreads, int64_t *best_k,
                     double *best_d) {
  if (m <= 0 || n < m || k_begin < 0 || k_end > n - m + 1 || k_begin >= k_end) return -2;
  int64_t noff = k_end - k_begin;
  int64_t *offs = (int64_t *)malloc((size_t)noff * sizeof(int64_t));
  double *d = (double *)malloc((size_t)noff * sizeof(double));
  if (!offs || !d) { free(offs); free(d); return -1; }
  for (int64_t t = 0; t < noff; ++t) offs[t] = k_begin + t;
  int rc = oracle_nn_dists(q, m, x, n, r, offs, noff, nthreads, d);
  if (rc == 0) {
    int64_t bk = -1;
    double bd = ORACLE_INF;
    for (int64_t t = 0; t < noff; ++t) {
      if (bk < 0 || d[t] < bd) { bd = d[t]; bk = offs[t]; }
    }
    *best_k = bk;
    *best_d = bd;
  }
  free(offs);
  free(d);
  return rc;
}

typedef struct {
  const double *X, *Y;   /* rows of length L */
  int64_t L, r;
  const int64_t *ia, *ib; /* pair p = (X[ia[p]], Y[ib[p]]) */
  int64_t lo, hi;
  double *out;
  int err;
} pair_job;

static void *pair_worker(void *arg) {
  pair_job *jb = (pair_job *)arg;
  dtw_ws w = {0, 0};
  for (int64_t p = jb->lo; p < jb->hi; ++p) {
    const double *a = jb->X + jb->ia[p] * jb->L;
    const double *b = jb->Y + jb->ib[p] * jb->L;
    double v = dtw_matrix(&w, a, jb->L, b, jb->L, jb->r);
    if (!w.M) { jb->err = -1; break; }
    jb->out[p] = v;
  }
  free(w.M);
  return NULL;
}

/* DTW of listed pairs (X[ia[p]], Y[ib[p]]), all of length L, window r. */
int oracle_dtw_pairs(const double *X, const double *Y, int64_t L, int64_t r, const int64_t *ia,
                     const int64_t *ib, int64_t npairs, int nthreads, double *out) {
  if (L <= 0) {
    for (int64_t p = 0; p < npairs; ++p) out[p] = 0.0;
    return 0;
  }
  if (nthreads < 1) nthreads = 1;
  if (nthreads > 256) nthreads = 256;
  pthread_t th[256];
  int live[256];
  pair_job jobs[256];
  int64_t per = (npairs + nthreads - 1) / nthreads;
  for (int t = 0; t < nthreads; ++t) {
    int64_t lo = (int64_t)t * per, hi = lo + per;
    if (lo > npairs) lo = npairs;
    if (hi > npairs) hi = npairs;
    jobs[t] = (pair_job){X, Y, L, r, ia, ib, lo, hi, out, 0};
    live[t] = pthread_create(&th[t], NULL, pair_worker, &jobs[t]) == 0;
    if (!live[t]) pair_worker(&jobs[t]);
  }
  int err = 0;
  for (int t = 0; t < nthreads; ++t) {
    if (live[t]) pthread_join(th[t], NULL);
    if (jobs[t].err) err = jobs[t].err;
  }
  return err;
}

/* ------------------------------------------------------------------------- */
/* Model of the paper's EAPrunedDTW line sweep (Section 4, Algorithm 3),      */
/* with a Sakoe-Chiba window (the paper states its algorithms without one;   */
/* a cell is admissible iff |i - j| <= r, Section 2.1) and with the          */
/* cost recomputed for every column of the last stage.  Kept only to check   */
/* the threshold contract and the worked example; never a reference value.   */
/*                                                                           */
/* Lines run over `li` and columns over `co`; co is the shorter series and,  */
/* at equal lengths, lines run over S.  Outputs: the value (or +inf), the    */
/* number of evaluated cells, and, if trace is non-NULL, per line the value  */
/* of the pruning point at the end of the line (trace[i-1]), 0 if the line    */
/* was not completed.  abandon_i / abandon_j receive the cell at which the     */
/* sweep gave up (0,0 if it did not).                                         */
/* ------------------------------------------------------------------------- */
double oracle_eap_model(const double *S, int64_t lS, const double *T, int64_t lT, int64_t r,
                        double ub, int64_t *cells, int64_t *trace, int64_t *abandon_i,
                        int64_t *abandon_j) {
  const double *li = S, *co = T;
  int64_t nli = lS, nco = lT;
  if (lT > lS) { li = T; co = S; nli = lT; nco = lS; }
  if (cells) *cells = 0;
  if (abandon_i) *abandon_i = 0;
  if (abandon_j) *abandon_j = 0;
  if (nli == 0 && nco == 0) return 0.0;
  if (nco == 0) return ORACLE_INF;
  if (nli - nco > r) return ORACLE_INF; /* no admissible path */
  if (trace) for (int64_t i = 0; i < nli; ++i) trace[i] = 0;

  double *a = (double *)malloc((size_t)(nco + 1) * sizeof(double));
  double *b = (double *)malloc((size_t)(nco + 1) * sizeof(double));
  if (!a || !b) { free(a); free(b); return NAN; }
  for (int64_t j = 0; j <= nco; ++j) a[j] = b[j] = ORACLE_INF;
  double *above = a, *line = b;
  above[0] = 0.0;              /* the origin cell (0,0) sits in the row above line 1 */
  int64_t left_edge = 1;       /* first column not known to be > ub (grows only) */
  int64_t tail_above = 1;      /* first column of the > ub tail of the line above */
  int64_t ncells = 0;
  double result = ORACLE_INF;
  int done = 0;

  for (int64_t i = 1; i <= nli && !done; ++i) {
    int64_t wlo = i - r < 1 ? 1 : i - r;
    int64_t whi = i + r > nco ? nco : i + r;
    if (left_edge < wlo) left_edge = wlo;
    int64_t tail = 0;          /* column after the last cell <= ub seen on this line */
    int64_t j = left_edge;
    line[j - 1] = ORACLE_INF;  /* the column left of the border is beyond ub */
    const double li_i = li[i - 1];
#define COST(jj) ((li_i - co[(jj) - 1]) * (li_i - co[(jj) - 1]))
    /* 1) cells left of the border's continuation: left neighbour is > ub */
    while (j == left_edge && j < tail_above) {
      line[j] = COST(j) + (above[j] < above[j - 1] ? above[j] : above[j - 1]);
      ++ncells;
      if (line[j] <= ub) tail = j + 1;
      else ++left_edge;
      ++j;
    }
    /* 2) ordinary cells with all three dependencies */
    while (j < tail_above) {
      line[j] = COST(j) + min3d(line[j - 1], above[j], above[j - 1]);
      ++ncells;
      if (line[j] <= ub) tail = j + 1;
      ++j;
    }
    /* 3) the column of the previous line's pruning point: no top dependency */
    if (j <= whi) {
      if (j == left_edge) {
        line[j] = COST(j) + above[j - 1];
        ++ncells;
        if (line[j] <= ub) tail = j + 1;
        else { /* the two borders collide: nothing on this line is <= ub */
          if (abandon_i) *abandon_i = (li == S) ? i : j;
          if (abandon_j) *abandon_j = (li == S) ? j : i;
          done = 1;
          break;
        }
      } else {
        line[j] = COST(j) + (line[j - 1] < above[j - 1] ? line[j - 1] : above[j - 1]);
        ++ncells;
        if (line[j] <= ub) tail = j + 1;
      }
      ++j;
    } else if (j == left_edge) { /* the left border ran through the whole line */
      if (abandon_i) *abandon_i = (li == S) ? i : j - 1;
      if (abandon_j) *abandon_j = (li == S) ? j - 1 : i;
      done = 1;
      break;
    }
    /* 4) beyond the previous pruning point: only the left dependency */
    while (j == tail && j <= whi) {
      line[j] = COST(j) + line[j - 1];
      ++ncells;
      if (line[j] <= ub) tail = j + 1;
      ++j;
    }
#undef COST
    tail_above = tail;
    if (trace) trace[i - 1] = tail;
    double *t = above; above = line; line = t;
  }
  if (!done && tail_above > nco) result = above[nco];
  if (cells) *cells = ncells;
  free(a);
  free(b);
  return result;
}

/* ------------------------------------------------------------------------- */
/* Lower bounds for the search (Section 2.2: a cheap lb <= DTW lets a        */
/* candidate be skipped when lb is strictly above ub; the paper names        */
/* LB_Kim and LB_Keogh, and its experiments (Section 5) keep the UCR Suite's */
/* three: LB_Kim, LB_Keogh with the query's envelope and LB_Keogh with the   */
/* candidate's).  The paper gives no formulas; these are the plain           */
/* definitions, each a sum of costs that every admissible warping path pays. */
/* ------------------------------------------------------------------------- */

/* Envelope of a[0..n) under window r: U[t] = max a[t-r..t+r], L[t] = min,
 * the window clipped to [0, n). */
void oracle_envelope(const double *a, int64_t n, int64_t r, double *U, double *L) {
  for (int64_t t = 0; t < n; ++t) {
    int64_t lo = t - r < 0 ? 0 : t - r;
    int64_t hi = t + r > n - 1 ? n - 1 : t + r;
    double u = a[lo], l = a[lo];
    for (int64_t s = lo + 1; s <= hi; ++s) {
      if (a[s] > u) u = a[s];
      if (a[s] < l) l = a[s];
    }
    U[t] = u;
    L[t] = l;
  }
}

static inline double sqd(double a, double b) { return (a - b) * (a - b); }

/* LB_Kim over two series of equal length m (cells (i, j), 0-based, cost
 * (q_i - c_j)^2).  Every warping path from (0,0) to (m-1,m-1) moves max(i,j)
 * and min(i,j) up by at most one per step, so for each level a = 1..L it
 * visits a cell with max(i,j) = a-1 (front set F_a) and a cell with
 * min(i,j) = m-a (back set B_a, both coordinates >= m-a).  Those 2L sets are
 * pairwise disjoint when 2L <= m, so the sum over them of the cheapest cell is
 * a lower bound for any window (a set's cells outside the window only lower
 * its minimum).  L = min(3, m/2). */
double oracle_lb_kim(const double *q, const double *c, int64_t m) {
  int64_t L = m / 2 < 3 ? m / 2 : 3;
  double lb = 0.0;
  for (int64_t a = 1; a <= L; ++a) {
    int64_t f = a - 1, b = m - a;
    double mf = INFINITY, mb = INFINITY;
    for (int64_t s = 0; s <= f; ++s) {
      /* front: (s, f) and (f, s) */
      if (sqd(q[s], c[f]) < mf) mf = sqd(q[s], c[f]);
      if (sqd(q[f], c[s]) < mf) mf = sqd(q[f], c[s]);
    }
    for (int64_t s = b; s < m; ++s) {
      /* back: (s, b) and (b, s) */
      if (sqd(q[s], c[b]) < mb) mb = sqd(q[s], c[b]);
      if (sqd(q[b], c[s]) < mb) mb = sqd(q[b], c[s]);
    }
    lb += mf + mb;
  }
  return lb;
}

/* LB_Keogh: sum over t of the squared distance from a[t] to [L[t], U[t]].
 * With U, L the envelope of the other series under window r, every path
 * visits each t of `a` at least once, paired with a point of the other series
 * within r of t, so this is a lower bound of DTW under window r. */
double oracle_lb_keogh(const double *a, const double *U, const double *L, int64_t m) {
  double lb = 0.0;
  for (int64_t t = 0; t < m; ++t) {
    if (a[t] > U[t]) lb += sqd(a[t], U[t]);
    else if (a[t] < L[t]) lb += sqd(a[t], L[t]);
  }
  return lb;
}

/* The three bounds of each listed candidate k of the z-normalised search:
 *  kim[t] = LB_Kim(z(q), z(x[k..k+m)))
 *  eq[t]  = LB_Keogh(z(x[k..k+m)); envelope of z(q) under r)
 *  ec[t]  = LB_Keogh(z(q); candidate envelope), where the candidate envelope is
 *           the envelope of the whole series x under r at positions k..k+m-1,
 *           z-normalised with the candidate's mean and sigma (all zeros when
 *           sigma is zero).  Near the candidate's ends that window reaches
 *           past the candidate, which only widens the envelope.
 * Between two series of length m a window of m-1 already admits every path
 * (Section 2.1), so a wider window is taken as m-1 (it would only widen the
 * series envelope).  Returns 0 on success. */
int oracle_nn_lower_bounds(const double *q, int64_t m, const double *x, int64_t n, int64_t r,
                           const int64_t *offsets, int64_t noff, double *kim, double *eq,
                           double *ec) {
  if (m <= 0 || n < m || r < 0) return -2;
  if (r > m - 1) r = m - 1;
  for (int64_t t = 0; t < noff; ++t)
    if (offsets[t] < 0 || offsets[t] + m > n) return -2;
  double *zq = malloc((size_t)m * sizeof(double)), *zc = malloc((size_t)m * sizeof(double));
  double *Uq = malloc((size_t)m * sizeof(double)), *Lq = malloc((size_t)m * sizeof(double));
  double *Uc = malloc((size_t)m * sizeof(double)), *Lc = malloc((size_t)m * sizeof(double));
  double *Ux = malloc((size_t)n * sizeof(double)), *Lx = malloc((size_t)n * sizeof(double));
  int rc = -1;
  if (!zq || !zc || !Uq || !Lq || !Uc || !Lc || !Ux || !Lx) goto done;
  oracle_znorm(q, m, zq);
  oracle_envelope(zq, m, r, Uq, Lq);
  oracle_envelope(x, n, r, Ux, Lx);
  for (int64_t t = 0; t < noff; ++t) {
    const int64_t k = offsets[t];
    double mean = 0.0, var = 0.0;
    for (int64_t s = 0; s < m; ++s) mean += x[k + s];
    mean /= (double)m;
    for (int64_t s = 0; s < m; ++s) var += sqd(x[k + s], mean);
    var /= (double)m;
    const double sd = oracle_flat(mean, var) ? 0.0 : sqrt(var);
    for (int64_t s = 0; s < m; ++s) {
      zc[s] = sd > 0.0 ? (x[k + s] - mean) / sd : 0.0;
      Uc[s] = sd > 0.0 ? (Ux[k + s] - mean) / sd : 0.0;
      Lc[s] = sd > 0.0 ? (Lx[k + s] - mean) / sd : 0.0;
    }
    kim[t] = oracle_lb_kim(zq, zc, m);
    eq[t] = oracle_lb_keogh(zc, Uq, Lq, m);
    ec[t] = oracle_lb_keogh(zq, Uc, Lc, m);
  }
  rc = 0;
done:
  free(zq); free(zc); free(Uq); free(Lq); free(Uc); free(Lc); free(Ux); free(Lx);
  return rc;
}

/* Nearest-neighbour search with the lower-bound cascade in front of the DTW
 * (the UCR Suite arrangement the paper's experiments use, Section 5): a
 * sequential scan of every offset that skips a candidate as soon as one of
 * LB_Kim, LB_Keogh(query envelope), LB_Keogh(candidate envelope), in that
 * order, is strictly above the best distance so far; the others get the full
 * DTW under window r.  Since every bound is a lower bound, the answer is the
 * brute-force answer (same lexicographic minimum of (distance, offset)).
 * counts[0..3] = candidates skipped by each bound, then candidates whose DTW
 * was computed.  Single-threaded; for small inputs.  Returns 0 on success. */
int oracle_nn_search_lb(const double *q, int64_t m, const double *x, int64_t n, int64_t r,
                        int64_t *best_k, double *best_d, int64_t *counts) {
  if (m <= 0 || n < m || r < 0) return -2;
  const int64_t K = n - m + 1;
  double *kim = malloc((size_t)K * sizeof(double)), *eq = malloc((size_t)K * sizeof(double));
  double *ec = malloc((size_t)K * sizeof(double)), *zq = malloc((size_t)m * sizeof(double));
  double *zc = malloc((size_t)m * sizeof(double));
  int64_t *offs = malloc((size_t)K * sizeof(int64_t));
  dtw_ws w = {0, 0};
  int rc = -1;
  if (!kim || !eq || !ec || !zq || !zc || !offs) goto done;
  for (int64_t k = 0; k < K; ++k) offs[k] = k;
  if ((rc = oracle_nn_lower_bounds(q, m, x, n, r, offs, K, kim, eq, ec)) != 0) goto done;
  rc = -1;
  oracle_znorm(q, m, zq);
  for (int i = 0; i < 4; ++i) counts[i] = 0;
  double bd = INFINITY;
  int64_t bk = -1;
  for (int64_t k = 0; k < K; ++k) {
    if (kim[k] > bd) { ++counts[0]; continue; }
    if (eq[k] > bd) { ++counts[1]; continue; }
    if (ec[k] > bd) { ++counts[2]; continue; }
    ++counts[3];
    oracle_znorm(x + k, m, zc);
    const double d = dtw_matrix(&w, zq, m, zc, m, r);
    if (!w.M) goto done;
    if (bk < 0 || d < bd) { bd = d; bk = k; }
  }
  *best_k = bk;
  *best_d = bd;
  rc = 0;
done:
  free(kim); free(eq); free(ec); free(zq); free(zc); free(offs); free(w.M);
  return rc;
}

/* ------------------------------------------------------------------------- */
/* k nearest neighbours of the search (the k-NN use named with NN1 in        */
/* Section 2.2): the k smallest (d_k, k) pairs in lexicographic order, i.e.  */
/* the k best offsets with ties going to the smaller offset, over every       */
/* offset (no exclusion of overlapping offsets).  Plain definition: every     */
/* distance, then a sort.  Fewer than k offsets: all of them.                 */
/* ------------------------------------------------------------------------- */
typedef struct {
  double d;
  int64_t k;
} knn_item;

static int knn_cmp(const void *a, const void *b) {
  const knn_item *x = (const knn_item *)a, *y = (const knn_item *)b;
  if (x->d < y->d) return -1;
  if (x->d > y->d) return 1;
  return (x->k > y->k) - (x->k < y->k);
}

int oracle_knn_search(const double *q, int64_t m, const double *x, int64_t n, int64_t r,
                      int64_t kk, int nthreads, int64_t *out_k, double *out_d, int64_t *out_cnt) {
  if (m <= 0 || n < m || kk < 1) return -2;
  const int64_t K = n - m + 1;
  int64_t *offs = malloc((size_t)K * sizeof(int64_t));
  double *d = malloc((size_t)K * sizeof(double));
  knn_item *it = malloc((size_t)K * sizeof(knn_item));
  int rc = -1;
  if (!offs || !d || !it) goto done;
  for (int64_t t = 0; t < K; ++t) offs[t] = t;
  if ((rc = oracle_nn_dists(q, m, x, n, r, offs, K, nthreads, d)) != 0) goto done;
  for (int64_t t = 0; t < K; ++t) it[t] = (knn_item){d[t], t};
  qsort(it, (size_t)K, sizeof(knn_item), knn_cmp);
  const int64_t c = kk < K ? kk : K;
  for (int64_t t = 0; t < c; ++t) {
    out_k[t] = it[t].k;
    out_d[t] = it[t].d;
  }
  *out_cnt = c;
  rc = 0;
done:
  free(offs); free(d); free(it);
  return rc;
}

/* ------------------------------------------------------------------------- */
/* Leave-one-out nearest neighbour over one set of series (the NN1            */
/* classification use of Section 2.2): for each series i, the series j != i  */
/* with the smallest DTW under window r, the smaller index among equal        */
/* distances.  Plain definition: every pair i < j through oracle_dtw_pairs,   */
/* then the minimum of each row and column.  N >= 2.                          */
/* ------------------------------------------------------------------------- */
int oracle_nn1(const double *X, int64_t N, int64_t L, int64_t r, int nthreads, int64_t *out_j,
               double *out_d) {
  if (N < 2 || L < 1) return -2;
  const int64_t P = N * (N - 1) / 2;
  int64_t *ia = malloc((size_t)P * sizeof(int64_t)), *ib = malloc((size_t)P * sizeof(int64_t));
  double *D = malloc((size_t)P * sizeof(double));
  int rc = -1;
  if (!ia || !ib || !D) goto done;
  int64_t p = 0;
  for (int64_t i = 0; i < N; ++i)
    for (int64_t j = i + 1; j < N; ++j) {
      ia[p] = i;
      ib[p] = j;
      ++p;
    }
  if ((rc = oracle_dtw_pairs(X, X, L, r, ia, ib, P, nthreads, D)) != 0) goto done;
  for (int64_t i = 0; i < N; ++i) {
    out_j[i] = -1;
    out_d[i] = INFINITY;
  }
  for (p = 0; p < P; ++p) {
    const int64_t i = ia[p], j = ib[p];
    /* j > i: for row i, j is visited in increasing order; for row j, i too */
    if (out_j[i] < 0 || D[p] < out_d[i] || (D[p] == out_d[i] && j < out_j[i])) {
      out_d[i] = D[p];
      out_j[i] = j;
    }
    if (out_j[j] < 0 || D[p] < out_d[j] || (D[p] == out_d[j] && i < out_j[j])) {
      out_d[j] = D[p];
      out_j[j] = i;
    }
  }
  rc = 0;
done:
  free(ia); free(ib); free(D);
  return rc;
}

/* Nearest neighbour of every series of a test set Q [nq][L] among a separate
 * reference set R [nr][L] (NN1 classification): for each i, the j with the
 * smallest DTW(Q_i, R_j) under window r, the smaller j among equal distances.
 * Plain definition: every (i, j) through oracle_dtw_pairs, then row minima. */
int oracle_nn1_ref(const double *Q, int64_t nq, const double *R, int64_t nr, int64_t L,
                   int64_t r, int nthreads, int64_t *out_j, double *out_d) {
  if (nq < 1 || nr < 1 || L < 1) return -2;
  const int64_t P = nq * nr;
  int64_t *ia = malloc((size_t)P * sizeof(int64_t)), *ib = malloc((size_t)P * sizeof(int64_t));
  double *D = malloc((size_t)P * sizeof(double));
  int rc = -1;
  if (!ia || !ib || !D) goto done;
  for (int64_t i = 0, p = 0; i < nq; ++i)
    for (int64_t j = 0; j < nr; ++j, ++p) {
      ia[p] = i;
      ib[p] = j;
    }
  if ((rc = oracle_dtw_pairs(Q, R, L, r, ia, ib, P, nthreads, D)) != 0) goto done;
  for (int64_t i = 0; i < nq; ++i) {
    out_j[i] = 0;
    out_d[i] = D[i * nr];
    for (int64_t j = 1; j < nr; ++j)
      if (D[i * nr + j] < out_d[i]) {
        out_d[i] = D[i * nr + j];
        out_j[i] = j;
      }
  }
  rc = 0;
done:
  free(ia); free(ib); free(D);
  return rc;
}

/* ------------------------------------------------------------------------- */
/* The paper's method on the CPU: a nearest-neighbour scan (Section 5's       */
/* search) whose distance is the EAPrunedDTW model above (Algorithm 3) with  */
/* the best-so-far as its bound.  The offsets are split into contiguous      */
/* ranges, one per thread, scanned in order; every thread reads the shared   */
/* best-so-far before each candidate and publishes a value at most it under  */
/* a lock (ties: the smaller offset).  Each candidate is z-normalised; lines */
/* run over the candidate, columns over the query.  Since the model returns  */
/* the exact DTW whenever it does not exceed the bound, the answer is the     */
/* brute-force answer.  *cells receives the evaluated cells of all           */
/* candidates.  Test and baseline infrastructure only.  Returns 0 on success. */
/* ------------------------------------------------------------------------- */
typedef struct {
  const double *zq, *x;
  int64_t m, r;
  const int64_t *offsets;
  int64_t lo, hi;
  pthread_mutex_t *mu;
  volatile double *bsf;
  volatile int64_t *bk;
  int64_t cells;
  int err;
} eap_scan_job;

static void *eap_scan_worker(void *arg) {
  eap_scan_job *jb = (eap_scan_job *)arg;
  double *zc = malloc((size_t)jb->m * sizeof(double));
  if (!zc) { jb->err = -1; return NULL; }
  for (int64_t t = jb->lo; t < jb->hi; ++t) {
    const int64_t k = jb->offsets[t];
    oracle_znorm(jb->x + k, jb->m, zc);
    const double ub = *jb->bsf;
    int64_t cells = 0;
    const double v = oracle_eap_model(zc, jb->m, jb->zq, jb->m, jb->r, ub, &cells, NULL, NULL,
                                      NULL);
    jb->cells += cells;
    if (v <= ub) {
      pthread_mutex_lock(jb->mu);
      if (v < *jb->bsf || (v == *jb->bsf && (*jb->bk < 0 || k < *jb->bk))) {
        *jb->bsf = v;
        *jb->bk = k;
      }
      pthread_mutex_unlock(jb->mu);
    }
  }
  free(zc);
  return NULL;
}

int oracle_eap_scan(const double *q, int64_t m, const double *x, int64_t n, int64_t r,
                    const int64_t *offsets, int64_t noff, int nthreads, int64_t *best_k,
                    double *best_d, int64_t *cells) {
  if (m <= 0 || n < m || r < 0 || noff <= 0) return -2;
  for (int64_t t = 0; t < noff; ++t)
    if (offsets[t] < 0 || offsets[t] + m > n) return -2;
  if (nthreads < 1) nthreads = 1;
  if (nthreads > 256) nthreads = 256;
  double *zq = malloc((size_t)m * sizeof(double));
  if (!zq) return -1;
  oracle_znorm(q, m, zq);
  pthread_mutex_t mu = PTHREAD_MUTEX_INITIALIZER;
  volatile double bsf = ORACLE_INF;
  volatile int64_t bk = -1;
  pthread_t th[256];
  int live[256];
  eap_scan_job jobs[256];
  const int64_t per = (noff + nthreads - 1) / nthreads;
  for (int t = 0; t < nthreads; ++t) {
    int64_t lo = (int64_t)t * per, hi = lo + per;
    if (lo > noff) lo = noff;
    if (hi > noff) hi = noff;
    jobs[t] = (eap_scan_job){zq, x, m, r, offsets, lo, hi, &mu, &bsf, &bk, 0, 0};
    live[t] = pthread_create(&th[t], NULL, eap_scan_worker, &jobs[t]) == 0;
    if (!live[t]) eap_scan_worker(&jobs[t]);
  }
  int rc = 0;
  int64_t total = 0;
  for (int t = 0; t < nthreads; ++t) {
    if (live[t]) pthread_join(th[t], NULL);
    if (jobs[t].err) rc = jobs[t].err;
    total += jobs[t].cells;
  }
  free(zq);
  *best_k = bk;
  *best_d = bsf;
  if (cells) *cells = total;
  return rc;
}

