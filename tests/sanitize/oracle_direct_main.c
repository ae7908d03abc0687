/* Test driver: runs the oracle's C direct sum (oracle/direct.c, linked in) on
 * inputs read from a file, so that the sum can be built and run as a
 * standalone program under the host sanitizers.
 *   oracle_direct_main IN OUT KERNEL NS NT THREADS KAPPA ALPHA
 * IN holds sx sy sz sf sw (NS doubles each) then tx ty tz tf (NT doubles
 * each); OUT receives out and abs_out (NT doubles each). Exit status: 0 on
 * success, 2 on bad usage or I/O, 3 when the sum rejects its arguments. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_direct(int kernel, double kappa, double alpha, const double *sx, const double *sy,
                  const double *sz, const double *sf, const double *sw, int64_t ns,
                  const double *tx, const double *ty, const double *tz, const double *tf,
                  int64_t nt, double *out, double *abs_out, int nthreads);

int main(int argc, char **argv) {
  if (argc != 9) return 2;
  const int kernel = atoi(argv[3]);
  const int64_t ns = atoll(argv[4]), nt = atoll(argv[5]);
  const int threads = atoi(argv[6]);
  const double kappa = atof(argv[7]), alpha = atof(argv[8]);
  if (ns < 1 || nt < 1) return 2;
  double *in = malloc(sizeof(double) * (size_t)(5 * ns + 4 * nt));
  double *res = malloc(sizeof(double) * (size_t)(2 * nt));
  if (!in || !res) return 2;
  FILE *f = fopen(argv[1], "rb");
  if (!f) return 2;
  const size_t want = (size_t)(5 * ns + 4 * nt);
  const size_t got = fread(in, sizeof(double), want, f);
  fclose(f);
  if (got != want) return 2;
  const double *s = in, *t = in + 5 * ns;
  const int rc = oracle_direct(kernel, kappa, alpha, s, s + ns, s + 2 * ns, s + 3 * ns,
                               s + 4 * ns, ns, t, t + nt, t + 2 * nt, t + 3 * nt, nt, res,
                               res + nt, threads);
  if (rc != 0) return 3;
  f = fopen(argv[2], "wb");
  if (!f) return 2;
  const size_t put = fwrite(res, sizeof(double), (size_t)(2 * nt), f);
  fclose(f);
  free(in);
  free(res);
  return put == (size_t)(2 * nt) ? 0 : 2;
}
