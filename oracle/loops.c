/*
 * mu-mode product written as plain loops -- TEST INFRASTRUCTURE ONLY (part of the CPU
 * oracle; never linked into the product library).
 *
 * Section 2 of the paper defines the mu-mode product W = V x_mu L of an order-d tensor
 * V (sizes n_1..n_d) with an n_mu x n_mu matrix L entry by entry:
 *     w(i_1..i_d) = sum_{j=1}^{n_mu} L(i_mu, j) v(i_1..i_{mu-1}, j, i_{mu+1}..i_d).
 * With vec(V) stacked by columns (Lemma 1: i_1 fastest), the entry (a, i, b) with
 * a < nlo = n_1..n_{mu-1}, i < n_mu, b < nhi = n_{mu+1}..n_d sits at a + nlo (i + n_mu b).
 * The loops below run over the output entries and sum over j in increasing order,
 * starting from zero; nothing is blocked or reordered.  OpenMP splits the (b, i) pairs
 * over threads, which changes no arithmetic; products of fewer than 2^22 multiply-adds
 * stay on one thread (thread start-up would cost more than they do).
 */
#include <stdint.h>

#define PAR_MIN_WORK ((int64_t)1 << 22)

void oracle_mode_product(int64_t nlo, int64_t nmu, int64_t nhi, const double *L,
                         const double *Lt, const double *v, double *w) {
  const int par = nlo * nmu * nmu * nhi >= PAR_MIN_WORK;
  if (nlo == 1) {
    /* mode 1: the same sums with i innermost, reading L through its transpose
       Lt[j][i] = L[i][j] so that the inner loop runs over contiguous memory; every
       output entry still accumulates over j in increasing order from zero */
#pragma omp parallel for schedule(static) if (par)
    for (int64_t b = 0; b < nhi; ++b) {
      double *wb = w + nmu * b;
      const double *vb = v + nmu * b;
      for (int64_t i = 0; i < nmu; ++i) wb[i] = 0.0;
      for (int64_t j = 0; j < nmu; ++j) {
        const double vj = vb[j];
        const double *lj = Lt + j * nmu;
        for (int64_t i = 0; i < nmu; ++i) wb[i] += lj[i] * vj;
      }
    }
    return;
  }
#pragma omp parallel for collapse(2) schedule(static) if (par)
  for (int64_t b = 0; b < nhi; ++b) {
    for (int64_t i = 0; i < nmu; ++i) {
      double *wi = w + nlo * (i + nmu * b);
      for (int64_t a = 0; a < nlo; ++a) wi[a] = 0.0;
      for (int64_t j = 0; j < nmu; ++j) {
        const double lij = L[i * nmu + j];
        const double *vj = v + nlo * (j + nmu * b);
        for (int64_t a = 0; a < nlo; ++a) wi[a] += lij * vj[a];
      }
    }
  }
}

/* Threads the loops run on from now on (n >= 1); used to time the oracle on one core. */
void oracle_set_threads(int n) {
#ifdef _OPENMP
  extern void omp_set_num_threads(int);
  if (n >= 1) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

/* Threads OpenMP would use (reported beside oracle timings). */
int oracle_threads(void) {
  int t = 1;
#pragma omp parallel
  {
#pragma omp single
    {
#ifdef _OPENMP
      extern int omp_get_num_threads(void);
      t = omp_get_num_threads();
#endif
    }
  }
  return t;
}
