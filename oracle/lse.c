/*
 * lse.c -- plain FP64 message log-sum-exp for the CPU oracle (test
 * infrastructure: only the test suite, the smoke entry point and the
 * benchmark's CPU-baseline leg load it; the product library never does).
 *
 * One call computes one message of the bipartite iteration (Section 3,
 * Theorem tree_dual_var and eq. q: the log of the product K (u * gamma)),
 *
 *     m(x) = log sum_y exp( w(y) - C(x, y) / eps ),   x = 0 .. n_dst - 1,
 *
 * with w(y) = Lam_(k,j)(y) + log gamma_k(y) given by the caller and the cost
 * either the squared Euclidean distance of the support points or an explicit
 * matrix.  Each row is the textbook two-pass stabilised sum: its maximum
 * first, then the sum of exp(v - max), then the log.  An all -inf row gives
 * -inf.  Rows are independent and each is summed sequentially over y, so the
 * result does not depend on the number of threads.  Nothing is blocked,
 * fused or reordered beyond that.
 */
#include <math.h>
#include <stdint.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* Threads for one call: `threads` if positive, else every thread the OpenMP
 * runtime offers (OMP_NUM_THREADS or the processor count).  Passed as a
 * num_threads clause, so no call changes the default of later calls. */
static int team_size(int threads) {
#ifdef _OPENMP
  return threads > 0 ? threads : omp_get_max_threads();
#else
  (void)threads;
  return 1;
#endif
}

/* Squared-Euclidean cost C(x, y) = sum_d (xs[x*dim+d] - ys[y*dim+d])^2.
 * xs: [n_dst * dim], ys: [n_src * dim], w: [n_src], out: [n_dst].
 * threads <= 0: every available thread. */
void oracle_message_sqeuclid(const double* xs, const double* ys, const double* w, int64_t n_dst, int64_t n_src,
                             int dim, double eps, double* out, int threads) {
  const int nt = team_size(threads);
  (void)nt;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 16) num_threads(nt)
#endif
  for (int64_t x = 0; x < n_dst; ++x) {
    const double* px = xs + x * dim;
    double mx = -INFINITY;
    for (int64_t y = 0; y < n_src; ++y) {
      double c = 0.0;
      for (int d = 0; d < dim; ++d) {
        const double t = px[d] - ys[y * dim + d];
        c += t * t;
      }
      const double v = w[y] - c / eps;
      if (v > mx) mx = v;
    }
    if (!(mx > -INFINITY)) {
      out[x] = -INFINITY;
      continue;
    }
    double s = 0.0;
    for (int64_t y = 0; y < n_src; ++y) {
      double c = 0.0;
      for (int d = 0; d < dim; ++d) {
        const double t = px[d] - ys[y * dim + d];
        c += t * t;
      }
      s += exp(w[y] - c / eps - mx);
    }
    out[x] = mx + log(s);
  }
}

/* Explicit cost.  cost holds C as an n_rows x n_cols row-major float32 matrix
 * of the edge; transposed = 0: C(x, y) = cost[x * n_src + y] (the message's
 * rows are the matrix rows), 1: C(x, y) = cost[y * n_dst + x]. */
void oracle_message_explicit(const float* cost, int transposed, const double* w, int64_t n_dst, int64_t n_src,
                             double eps, double* out, int threads) {
  const int nt = team_size(threads);
  (void)nt;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 16) num_threads(nt)
#endif
  for (int64_t x = 0; x < n_dst; ++x) {
    double mx = -INFINITY;
    for (int64_t y = 0; y < n_src; ++y) {
      const double c = transposed ? (double)cost[y * n_dst + x] : (double)cost[x * n_src + y];
      const double v = w[y] - c / eps;
      if (v > mx) mx = v;
    }
    if (!(mx > -INFINITY)) {
      out[x] = -INFINITY;
      continue;
    }
    double s = 0.0;
    for (int64_t y = 0; y < n_src; ++y) {
      const double c = transposed ? (double)cost[y * n_dst + x] : (double)cost[x * n_src + y];
      s += exp(w[y] - c / eps - mx);
    }
    out[x] = mx + log(s);
  }
}

int oracle_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
