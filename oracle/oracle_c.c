/*
 * FP64 CPU oracle kernels (plain C loops, OpenMP over template points).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the Python oracle (oracle/ref.py)
 * for sizes where NumPy broadcasting would be slow.  The library never
 * links or calls it, and it shares no code with the HIP path.
 *
 * ora_forces: the shape-weighted pair force of eq. (5) with g from
 *   Sec. IV / eq. (10), s from eq. (3) and the distance law of eqs. (4),
 *   (11): f_i = coef * sum_j w_j g_ij ((|r|^2+eps^2)/L^2)^((p-1)/2) r_ij,
 *   r_ij = y_i - x_j, coef = -(G/Z); the energy
 *   U = (G/Z) sum_ij w_j g_ij L^(1-p) q^((p+1)/2) / (p+1);
 *   optionally (s_out != NULL) the absolute-sum scale of each force,
 *   s_i = (G/Z) sum_j |w_j g_ij h_ij| |r_ij|.
 * ora_knn: k nearest neighbours in float32 squared distance, evaluated as
 *   ((dx*dx + dy*dy) + dz*dz) with every operation rounded to float32 (the
 *   file is compiled with -ffp-contract=off), ties broken by index.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>

void ora_forces(int64_t M, int64_t N, const double* Y, const double* aY, const double* X,
                const double* aX, const double* wX, double p, int g_mode, double sigma,
                double eps, double L, double abar, double G, double Z, double* f_out,
                double* U_out, double* s_out) {
  double Utot = 0.0;
  const double hp = 0.5 * (p - 1.0);
#pragma omp parallel for schedule(static) reduction(+ : Utot)
  for (int64_t i = 0; i < M; ++i) {
    double fx = 0.0, fy = 0.0, fz = 0.0, u = 0.0, sa = 0.0;
    for (int64_t j = 0; j < N; ++j) {
      double rx = Y[3 * i + 0] - X[3 * j + 0];
      double ry = Y[3 * i + 1] - X[3 * j + 1];
      double rz = Y[3 * i + 2] - X[3 * j + 2];
      double q = rx * rx + ry * ry + rz * rz + eps * eps;
      double da = aY[i] - aX[j];
      double s = exp(-(da * da) / (sigma * sigma));
      double g = (g_mode == 1) ? (aY[i] / abar) * (aX[j] / abar) * s : (g_mode == 2 ? 1.0 : s);
      double h = (hp == 0.0) ? 1.0 : pow(q / (L * L), hp);
      double c = wX[j] * g * h;
      fx += c * rx;
      fy += c * ry;
      fz += c * rz;
      u += c * q;
      if (s_out) sa += fabs(c) * sqrt(rx * rx + ry * ry + rz * rz);
    }
    if (s_out) s_out[i] = (G / Z) * sa;
    f_out[3 * i + 0] = -(G / Z) * fx;
    f_out[3 * i + 1] = -(G / Z) * fy;
    f_out[3 * i + 2] = -(G / Z) * fz;
    Utot += u;
  }
  *U_out = (G / Z) * Utot / (p + 1.0);
}

/* ora_pair_sums (p = 1 only, where h = 1 and the pair weight
 * c_ij = w_j g_ij does not depend on the pose): per template row i the sums
 * over the reference S0_i = sum_j c_ij, Sx_i = sum_j c_ij x_j (3) and
 * Sxx_i = sum_j c_ij |x_j|^2, out[5 i ...].  With them eq. 5 reads
 * f_i = -(G/Z) (y_i S0_i - Sx_i) for any pose. */
void ora_pair_sums(int64_t M, int64_t N, const double* aY, const double* X, const double* aX,
                   const double* wX, int g_mode, double sigma, double abar, double* out) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < M; ++i) {
    double s0 = 0.0, sx = 0.0, sy = 0.0, sz = 0.0, sq = 0.0;
    for (int64_t j = 0; j < N; ++j) {
      double da = aY[i] - aX[j];
      double s = exp(-(da * da) / (sigma * sigma));
      double g = (g_mode == 1) ? (aY[i] / abar) * (aX[j] / abar) * s : (g_mode == 2 ? 1.0 : s);
      double c = wX[j] * g;
      s0 += c;
      sx += c * X[3 * j + 0];
      sy += c * X[3 * j + 1];
      sz += c * X[3 * j + 2];
      sq += c * (X[3 * j + 0] * X[3 * j + 0] + X[3 * j + 1] * X[3 * j + 1] + X[3 * j + 2] * X[3 * j + 2]);
    }
    out[5 * i + 0] = s0;
    out[5 * i + 1] = sx;
    out[5 * i + 2] = sy;
    out[5 * i + 3] = sz;
    out[5 * i + 4] = sq;
  }
}

static float sq32(const float* P, int64_t a, int64_t b) {
  float dx = P[3 * a + 0] - P[3 * b + 0];
  float dy = P[3 * a + 1] - P[3 * b + 1];
  float dz = P[3 * a + 2] - P[3 * b + 2];
  float xx = dx * dx;
  float yy = dy * dy;
  float zz = dz * dz;
  float s = xx + yy;
  return s + zz;
}

void ora_knn(int64_t n, const float* P, int k, int64_t nq, const int64_t* queries, int64_t* out) {
#pragma omp parallel
  {
    float* bd = (float*)malloc(sizeof(float) * (size_t)k);
    int64_t* bi = (int64_t*)malloc(sizeof(int64_t) * (size_t)k);
#pragma omp for schedule(dynamic, 16)
    for (int64_t r = 0; r < nq; ++r) {
      int64_t q = queries[r];
      int cnt = 0;
      for (int64_t j = 0; j < n; ++j) {
        float d = sq32(P, q, j);
        /* candidates arrive in increasing index, so an equal distance never
           displaces an earlier (smaller-index) entry */
        if (cnt == k && !(d < bd[k - 1])) continue;
        int pos = (cnt < k) ? cnt : k - 1;
        while (pos > 0 && d < bd[pos - 1]) {
          bd[pos] = bd[pos - 1];
          bi[pos] = bi[pos - 1];
          --pos;
        }
        bd[pos] = d;
        bi[pos] = j;
        if (cnt < k) ++cnt;
      }
      for (int s = 0; s < k; ++s) out[r * k + s] = bi[s];
    }
    free(bd);
    free(bi);
  }
}

/* Thread count of the loops above (for timing the oracle on one thread and
 * on all host threads). */
int ora_threads(void) { return omp_get_max_threads(); }
void ora_set_threads(int n) { omp_set_num_threads(n); }
