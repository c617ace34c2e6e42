/* Host driver for the C oracle kernels (oracle/oracle_c.c), so that they can
 * be built and run under AddressSanitizer and UndefinedBehaviorSanitizer.
 * stdin: M N k p g_mode sigma eps L abar G Z, then Y (3M), aY (M), X (3N),
 * aX (N), wX (N).  stdout: f (3M), U, s (M), the p = 1 pair sums (5M) and
 * the k nearest neighbours of every reference point among the reference
 * (N k, as float32 coordinates). */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void ora_forces(int64_t M, int64_t N, const double* Y, const double* aY, const double* X, const double* aX,
                const double* wX, double p, int g_mode, double sigma, double eps, double L, double abar, double G,
                double Z, double* f_out, double* U_out, double* s_out);
void ora_pair_sums(int64_t M, int64_t N, const double* aY, const double* X, const double* aX, const double* wX,
                   int g_mode, double sigma, double abar, double* out);
void ora_knn(int64_t n, const float* P, int k, int64_t nq, const int64_t* queries, int64_t* out);

static double* read_n(int64_t n) {
  double* a = (double*)malloc(sizeof(double) * (size_t)n);
  for (int64_t i = 0; i < n; ++i)
    if (scanf("%lf", &a[i]) != 1) exit(2);
  return a;
}

int main(void) {
  long long M, N;
  int k, g_mode;
  double p, sigma, eps, L, abar, G, Z;
  if (scanf("%lld %lld %d %lf %d %lf %lf %lf %lf %lf %lf", &M, &N, &k, &p, &g_mode, &sigma, &eps, &L, &abar, &G,
            &Z) != 11)
    return 2;
  double* Y = read_n(3 * M);
  double* aY = read_n(M);
  double* X = read_n(3 * N);
  double* aX = read_n(N);
  double* wX = read_n(N);
  double* f = (double*)malloc(sizeof(double) * (size_t)(3 * M));
  double* s = (double*)malloc(sizeof(double) * (size_t)M);
  double* ps = (double*)malloc(sizeof(double) * (size_t)(5 * M));
  double U = 0.0;
  ora_forces(M, N, Y, aY, X, aX, wX, p, g_mode, sigma, eps, L, abar, G, Z, f, &U, s);
  ora_pair_sums(M, N, aY, X, aX, wX, g_mode, sigma, abar, ps);
  float* P = (float*)malloc(sizeof(float) * (size_t)(3 * N));
  int64_t* q = (int64_t*)malloc(sizeof(int64_t) * (size_t)N);
  int64_t* nn = (int64_t*)malloc(sizeof(int64_t) * (size_t)(N * k));
  for (int64_t i = 0; i < 3 * N; ++i) P[i] = (float)X[i];
  for (int64_t i = 0; i < N; ++i) q[i] = i;
  ora_knn(N, P, k, N, q, nn);
  for (int64_t i = 0; i < 3 * M; ++i) printf("%.17g ", f[i]);
  printf("%.17g ", U);
  for (int64_t i = 0; i < M; ++i) printf("%.17g ", s[i]);
  for (int64_t i = 0; i < 5 * M; ++i) printf("%.17g ", ps[i]);
  for (int64_t i = 0; i < N * k; ++i) printf("%lld ", (long long)nn[i]);
  printf("\n");
  free(Y); free(aY); free(X); free(aX); free(wX); free(f); free(s); free(ps); free(P); free(q); free(nn);
  return 0;
}
