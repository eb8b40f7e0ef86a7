/*
 * FP64 periodic 3x3x3 cross-correlation for the learned-start network oracle -- test
 * infrastructure only (used by oracle/cnn_oracle.py; never by the product library).
 *
 * out[z][y][x][o] = b[o] + sum_t sum_i w[o][t][i] x[(z+dz)%n][(y+dy)%n][(x+dx)%n][i]
 * with tap t = (dz+1)*9 + (dy+1)*3 + (dx+1), fields channels-last [z][y][x][c], plain loops
 * over every output cell, tap and input channel in double precision, one accumulator per
 * output channel.  It computes exactly the definition that cnn_oracle.conv writes with
 * array shifts, and is pinned to it by the CPU tests; it exists only because the array form
 * is too slow on 256^3 grids.
 */
#include <stdlib.h>

#define MAX_COUT 64

__attribute__((target_clones("avx2", "default")))
static void conv_row(const double* x, int cin, long long n, const double* wt, const double* b, int cout, long long z,
                     long long y, double* out) {
  double acc[MAX_COUT];
  for (long long xx = 0; xx < n; ++xx) {
    for (int o = 0; o < cout; ++o) acc[o] = b[o];
    for (int t = 0; t < 27; ++t) {
      const long long zz = (z + t / 9 - 1 + n) % n, yy = (y + (t / 3) % 3 - 1 + n) % n, xs = (xx + t % 3 - 1 + n) % n;
      const double* p = x + ((zz * n + yy) * n + xs) * cin;
      const double* w = wt + (long long)t * cin * cout;
      for (int i = 0; i < cin; ++i) {
        const double xi = p[i];
        const double* wi = w + (long long)i * cout;
        for (int o = 0; o < cout; ++o) acc[o] += wi[o] * xi;
      }
    }
    double* q = out + ((z * n + y) * n + xx) * cout;
    for (int o = 0; o < cout; ++o) q[o] = acc[o];
  }
}

/* w: [cout][27][cin] as in the parameter vector; returns 0, or -1 when cout > 64 or out of memory */
int conv3_periodic(const double* x, int cin, int n, const double* w, const double* b, int cout, double* out) {
  if (cout > MAX_COUT || cout < 1 || cin < 1) return -1;
  /* the weights as [27][cin][cout], so that the innermost loop runs over independent accumulators */
  double* wt = (double*)malloc(sizeof(double) * 27 * cin * cout);
  if (!wt) return -1;
  for (int o = 0; o < cout; ++o)
    for (int t = 0; t < 27; ++t)
      for (int i = 0; i < cin; ++i) wt[((long long)t * cin + i) * cout + o] = w[((long long)o * 27 + t) * cin + i];
  const long long nn = n;
#pragma omp parallel for collapse(2) schedule(static)
  for (long long z = 0; z < nn; ++z)
    for (long long y = 0; y < nn; ++y) conv_row(x, cin, nn, wt, b, cout, z, y, out);
  free(wt);
  return 0;
}
