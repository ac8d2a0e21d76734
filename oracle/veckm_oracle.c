/*
 * FP64 CPU oracle for the event encoder and the two-layer perceptron.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no header, table or helper with the HIP
 * library.
 *
 * What it computes (plain definitions, no pooling, no tables):
 *
 *   Neighbourhood (Sec. 2.1, Eqn. 1, with an optional temporal radius rt):
 *     N(q) = { k : |x_k - x_q| <= rx, |y_k - y_q| <= ry, and
 *                  (rt < 0  or  |t_k - t_q| <= rt) }.
 *     rt < 0 is the paper's own neighbourhood: the whole slice in time.
 *
 *   Encoding (Sec. 2.2.1, Eqn. 10; count of Eqn. 17; Algorithm 1 final
 *   normalisation step):
 *     emb_q[j] = (1/|N(q)|) * sum_{k in N(q)} exp(+i * (A[j,0] dx + A[j,1] dy
 *                                                      + A[j,2] dt)),
 *     with (dx, dy, dt) = (x_k - x_q, y_k - y_q, t_k - t_q) formed in exact
 *     64-bit integers, so the result depends only on relative coordinates.
 *     This is the row of the adjacency-matrix product of the predecessor
 *     method that the paper reformulates (Sec. 2.1, last paragraphs).
 *     Output is planar: [Re emb[0..D-1], Im emb[0..D-1]].
 *
 *   Perceptron (Sec. 2.1, Eqns. 5-6): flow = W2 * relu(W1 * x + b1) + b2,
 *     W1 is [hidden][in], W2 is [2][hidden] (row-major).
 *
 * Two neighbour searches are provided and produce bit-identical sums,
 * because both accumulate the neighbours in increasing event index:
 *   search 0: literal O(n) scan per query (the adjacency row);
 *   search 1: pixel buckets over the (x, y) bounding box, candidates merged
 *             and sorted by event index before summation.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -fPIC -shared (no FMA
 * contraction, so every sum is evaluated in the written order).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

static inline int64_t iabs64(int64_t v) { return v < 0 ? -v : v; }

static inline int in_window(int64_t dx, int64_t dy, int64_t dt,
                            int32_t rx, int32_t ry, int32_t rt) {
  if (iabs64(dx) > rx || iabs64(dy) > ry) return 0;
  if (rt >= 0 && iabs64(dt) > rt) return 0;
  return 1;
}

/* Adds the phase of one neighbour to the running sums. */
static inline void add_phase(const double* A, int32_t D, int64_t dx, int64_t dy,
                             int64_t dt, double* re, double* im) {
  for (int32_t j = 0; j < D; ++j) {
    double th = A[3 * j + 0] * (double)dx + A[3 * j + 1] * (double)dy +
                A[3 * j + 2] * (double)dt;
    re[j] += cos(th);
    im[j] += sin(th);
  }
}

static int cmp_i64(const void* a, const void* b) {
  int64_t x = *(const int64_t*)a, y = *(const int64_t*)b;
  return (x > y) - (x < y);
}

/* Returns 0 on success, -1 on bad arguments, -2 on allocation failure. */
int oracle_encode(const int32_t* ev, int64_t n, const int64_t* queries, int64_t m,
                  const double* A, int32_t D, int32_t rx, int32_t ry, int32_t rt,
                  int32_t search, double* emb, int64_t* cnt, int32_t nthreads) {
  if (!ev || !A || !emb || D <= 0 || rx < 0 || ry < 0 || n < 0 || m < 0) return -1;
  if (nthreads <= 0) nthreads = omp_get_max_threads();

  /* pixel buckets for search 1 */
  int64_t xmin = 0, ymin = 0, bw = 0, bh = 0;
  int64_t *start = NULL, *list = NULL;
  if (search == 1 && n > 0) {
    int64_t xmax = ev[0], ymax = ev[1];
    xmin = ev[0]; ymin = ev[1];
    for (int64_t k = 1; k < n; ++k) {
      if (ev[4 * k] < xmin) xmin = ev[4 * k];
      if (ev[4 * k] > xmax) xmax = ev[4 * k];
      if (ev[4 * k + 1] < ymin) ymin = ev[4 * k + 1];
      if (ev[4 * k + 1] > ymax) ymax = ev[4 * k + 1];
    }
    bw = xmax - xmin + 1; bh = ymax - ymin + 1;
    start = (int64_t*)calloc((size_t)(bw * bh + 1), sizeof(int64_t));
    list = (int64_t*)malloc((size_t)n * sizeof(int64_t));
    if (!start || !list) { free(start); free(list); return -2; }
    for (int64_t k = 0; k < n; ++k)
      start[(ev[4 * k + 1] - ymin) * bw + (ev[4 * k] - xmin) + 1]++;
    for (int64_t p = 0; p < bw * bh; ++p) start[p + 1] += start[p];
    int64_t* fill = (int64_t*)malloc((size_t)(bw * bh) * sizeof(int64_t));
    if (!fill) { free(start); free(list); return -2; }
    memcpy(fill, start, (size_t)(bw * bh) * sizeof(int64_t));
    for (int64_t k = 0; k < n; ++k)  /* increasing k: each bucket is sorted */
      list[fill[(ev[4 * k + 1] - ymin) * bw + (ev[4 * k] - xmin)]++] = k;
    free(fill);
  }

  int failed = 0;
#pragma omp parallel num_threads(nthreads)
  {
    double* re = (double*)malloc((size_t)D * sizeof(double));
    double* im = (double*)malloc((size_t)D * sizeof(double));
    int64_t cap = 1024;
    int64_t* nb = (int64_t*)malloc((size_t)cap * sizeof(int64_t));
    if (!re || !im || !nb) {
#pragma omp atomic write
      failed = 1;
    }
#pragma omp for schedule(dynamic, 8)
    for (int64_t i = 0; i < m; ++i) {
      if (failed) continue;
      int64_t q = queries ? queries[i] : i;
      int64_t xq = ev[4 * q], yq = ev[4 * q + 1], tq = ev[4 * q + 2];
      for (int32_t j = 0; j < D; ++j) { re[j] = 0.0; im[j] = 0.0; }
      int64_t c = 0;
      if (search != 1) {
        for (int64_t k = 0; k < n; ++k) {
          int64_t dx = ev[4 * k] - xq, dy = ev[4 * k + 1] - yq, dt = ev[4 * k + 2] - tq;
          if (!in_window(dx, dy, dt, rx, ry, rt)) continue;
          ++c;
          add_phase(A, D, dx, dy, dt, re, im);
        }
      } else {
        int64_t nn = 0;
        for (int64_t py = yq - ry; py <= yq + ry; ++py) {
          if (py < ymin || py >= ymin + bh) continue;
          for (int64_t px = xq - rx; px <= xq + rx; ++px) {
            if (px < xmin || px >= xmin + bw) continue;
            int64_t b = (py - ymin) * bw + (px - xmin);
            for (int64_t s = start[b]; s < start[b + 1]; ++s) {
              int64_t k = list[s];
              if (rt >= 0 && iabs64((int64_t)ev[4 * k + 2] - tq) > rt) continue;
              if (nn == cap) {
                cap *= 2;
                int64_t* g = (int64_t*)realloc(nb, (size_t)cap * sizeof(int64_t));
                if (!g) { failed = 1; break; }
                nb = g;
              }
              nb[nn++] = k;
            }
          }
        }
        qsort(nb, (size_t)nn, sizeof(int64_t), cmp_i64);
        for (int64_t s = 0; s < nn; ++s) {
          int64_t k = nb[s];
          add_phase(A, D, ev[4 * k] - xq, ev[4 * k + 1] - yq, ev[4 * k + 2] - tq, re, im);
        }
        c = nn;
      }
      double* row = emb + (size_t)i * 2 * (size_t)D;
      for (int32_t j = 0; j < D; ++j) {
        row[j] = c > 0 ? re[j] / (double)c : 0.0;
        row[D + j] = c > 0 ? im[j] / (double)c : 0.0;
      }
      if (cnt) cnt[i] = c;
    }
    free(re); free(im); free(nb);
  }
  free(start); free(list);
  return failed ? -2 : 0;
}

/* flow[i] = W2 * relu(W1 * x[i] + b1) + b2 in FP64. */
int oracle_mlp(const double* x, int64_t m, int32_t in_dim, int32_t hidden,
               const double* W1, const double* b1, const double* W2,
               const double* b2, double* out, int32_t nthreads) {
  if (!x || !W1 || !b1 || !W2 || !b2 || !out || in_dim <= 0 || hidden <= 0) return -1;
  if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(static) num_threads(nthreads)
  for (int64_t i = 0; i < m; ++i) {
    const double* xi = x + (size_t)i * (size_t)in_dim;
    double o0 = 0.0, o1 = 0.0;
    for (int32_t r = 0; r < hidden; ++r) {
      double h = b1[r];
      const double* w = W1 + (size_t)r * (size_t)in_dim;
      for (int32_t c = 0; c < in_dim; ++c) h += w[c] * xi[c];
      if (h < 0.0) h = 0.0;
      o0 += W2[r] * h;
      o1 += W2[hidden + r] * h;
    }
    out[2 * i] = o0 + b2[0];
    out[2 * i + 1] = o1 + b2[1];
  }
  return 0;
}
