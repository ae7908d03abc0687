/*
 * ORACLE -- test infrastructure only. Nothing in the product path may link,
 * load or call this file; only the tests, the smoke check and the benchmark's
 * CPU-baseline leg do.
 *
 * Plain CPU FP64 evaluation of the discrete convolution sum with singularity
 * subtraction, written straight from its definition:
 *
 *   discrete sum (paper Section 6, Eq. direct-sum): u_i = sum_{j, i != j} G(r_i, r_j) f_j w_j
 *   Yukawa with subtraction (Section 4.3, Eq. yukawa-conv-ss and the analytic term 4 pi f / k^2):
 *       u_i = sum_{j: d_ij > 0} (f_j - f_i) exp(-k d_ij) / d_ij w_j + 4 pi f_i / k^2
 *   Coulomb with Gaussian subtraction (Section 4.3, Eqs. coulomb-conv-ss, correction_term):
 *       u_i = sum_{j: d_ij > 0} (f_j - f_i exp(-d_ij^2 / a^2)) / d_ij w_j + 2 pi a^2 f_i
 *   plain kernels (no subtraction): u_i = sum_{j: d_ij > 0} G(d_ij) f_j w_j with
 *       G = exp(-k d)/d (Yukawa) or 1/d (Coulomb).
 *
 * "i != j" is read as "distance exactly zero is skipped", which is the same
 * thing when all points are distinct and also defines separate target sets.
 * Every target's sum is accumulated with Neumaier's compensated summation in
 * source order; exp and sqrt are the host C library's.
 *
 * Threads split the targets into contiguous blocks; each target is owned by one
 * thread, so the result does not depend on the thread count.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>

enum { K_YUKAWA_SS = 0, K_COULOMB_SS = 1, K_YUKAWA = 2, K_COULOMB = 3 };

typedef struct {
  int kernel;
  double kappa, alpha;
  const double *sx, *sy, *sz, *sf, *sw;
  int64_t ns;
  const double *tx, *ty, *tz, *tf;
  int64_t t0, t1;
  double *out;
  double *abs_out; /* optional: sum of |term| per target */
} job_t;

static void *run_block(void *arg) {
  job_t *jb = (job_t *)arg;
  const double pi = 3.14159265358979323846;
  for (int64_t i = jb->t0; i < jb->t1; ++i) {
    const double xi = jb->tx[i], yi = jb->ty[i], zi = jb->tz[i];
    const double fi = jb->tf ? jb->tf[i] : 0.0;
    double s = 0.0, c = 0.0, sabs = 0.0;
    for (int64_t j = 0; j < jb->ns; ++j) {
      const double dx = xi - jb->sx[j], dy = yi - jb->sy[j], dz = zi - jb->sz[j];
      const double d2 = dx * dx + dy * dy + dz * dz;
      const double d = sqrt(d2);
      if (d == 0.0) continue;
      double term;
      switch (jb->kernel) {
        case K_YUKAWA_SS:
          term = (jb->sf[j] - fi) * exp(-jb->kappa * d) / d * jb->sw[j];
          break;
        case K_COULOMB_SS:
          term = (jb->sf[j] - fi * exp(-d2 / (jb->alpha * jb->alpha))) / d * jb->sw[j];
          break;
        case K_YUKAWA:
          term = exp(-jb->kappa * d) / d * jb->sf[j] * jb->sw[j];
          break;
        default:
          term = 1.0 / d * jb->sf[j] * jb->sw[j];
          break;
      }
      /* Neumaier compensated sum */
      const double t = s + term;
      if (fabs(s) >= fabs(term))
        c += (s - t) + term;
      else
        c += (term - t) + s;
      s = t;
      sabs += fabs(term);
    }
    double u = s + c;
    if (jb->kernel == K_YUKAWA_SS) u += 4.0 * pi * fi / (jb->kappa * jb->kappa);
    if (jb->kernel == K_COULOMB_SS) u += 2.0 * pi * jb->alpha * jb->alpha * fi;
    jb->out[i] = u;
    if (jb->abs_out) jb->abs_out[i] = sabs;
  }
  return NULL;
}

/* Returns 0 on success, -1 on bad arguments. Targets' f (tf) is required for the
 * subtracted kernels and ignored otherwise. */
int oracle_direct(int kernel, double kappa, double alpha, const double *sx, const double *sy,
                  const double *sz, const double *sf, const double *sw, int64_t ns,
                  const double *tx, const double *ty, const double *tz, const double *tf,
                  int64_t nt, double *out, double *abs_out, int nthreads) {
  if (kernel < 0 || kernel > 3 || ns < 0 || nt < 0 || !out) return -1;
  if ((kernel == K_YUKAWA_SS || kernel == K_COULOMB_SS) && !tf) return -1;
  if (nthreads < 1) nthreads = 1;
  if (nthreads > 256) nthreads = 256;
  if (nt < nthreads) nthreads = nt > 0 ? (int)nt : 1;
  pthread_t th[256];
  job_t jobs[256];
  for (int t = 0; t < nthreads; ++t) {
    jobs[t] = (job_t){kernel, kappa, alpha, sx, sy, sz, sf, sw, ns, tx, ty, tz, tf,
                      nt * t / nthreads, nt * (t + 1) / nthreads, out, abs_out};
  }
  for (int t = 1; t < nthreads; ++t) pthread_create(&th[t], NULL, run_block, &jobs[t]);
  run_block(&jobs[0]);
  for (int t = 1; t < nthreads; ++t) pthread_join(th[t], NULL);
  return 0;
}
