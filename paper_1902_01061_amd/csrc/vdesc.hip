// Vector shape descriptor: soft histogram of normals (Sec. III-A lists
// histograms of normals among the local shape features).
//
// normals_kernel: the covariance (1/k, centred at the neighbourhood mean) of
// each point's k nearest neighbours, in FP64, and its unit eigenvector of the
// smallest eigenvalue (for a symmetric positive semi-definite matrix the
// singular vectors are the eigenvectors); its sign is arbitrary.
// hist_kernel: h_i[b] = (1/k) sum over the neighbours j of the tent weight of
// u = |n_i . n_j| at bin b, centres b / (D - 1): u spreads a unit weight over
// its two nearest centres.  |.| removes the sign, and the tents make h a
// continuous function of the normals.  One wave per block; each lane keeps
// its D partial sums in its own LDS column (no bank conflicts).
#include "common.h"
#include "launch.h"

namespace sgr {

namespace {

constexpr int HN_BT = 64;

__global__ __launch_bounds__(256) void normals_kernel(const float* __restrict__ X, const float* __restrict__ Y,
                                                      const float* __restrict__ Zc, int n, int k,
                                                      const int32_t* __restrict__ idx, double* __restrict__ nrm) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int32_t* nb = idx + (int64_t)i * k;
  double m[3] = {0, 0, 0};
  for (int s = 0; s < k; ++s) {
    const int j = nb[s] >= 0 ? nb[s] : i;
    m[0] += (double)X[j];
    m[1] += (double)Y[j];
    m[2] += (double)Zc[j];
  }
  const double invk = 1.0 / (double)k;
  for (int c = 0; c < 3; ++c) m[c] *= invk;
  double C[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int s = 0; s < k; ++s) {
    const int j = nb[s] >= 0 ? nb[s] : i;
    const double e[3] = {(double)X[j] - m[0], (double)Y[j] - m[1], (double)Zc[j] - m[2]};
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) C[r * 3 + c] += e[r] * e[c];
  }
  for (int e = 0; e < 9; ++e) C[e] *= invk;
  double sv[3], u[3][3], v[3][3];
  svd3(C, sv, u, v);
  for (int c = 0; c < 3; ++c) nrm[(int64_t)i * 3 + c] = v[2][c];
}

__global__ __launch_bounds__(HN_BT) void hist_kernel(int n, int k, int D, const int32_t* __restrict__ idx,
                                                     const double* __restrict__ nrm, float* __restrict__ h_out) {
  __shared__ double s_h[32 * HN_BT];
  const int i = blockIdx.x * HN_BT + threadIdx.x;
  for (int b = 0; b < D; ++b) s_h[b * HN_BT + threadIdx.x] = 0.0;
  if (i >= n) return;
  const double ni[3] = {nrm[(int64_t)i * 3], nrm[(int64_t)i * 3 + 1], nrm[(int64_t)i * 3 + 2]};
  const int32_t* nb = idx + (int64_t)i * k;
  const double scale = (double)(D - 1);
  bool bad = false;
  for (int s = 0; s < k; ++s) {
    const int j = nb[s] >= 0 ? nb[s] : i;
    const double* nj = nrm + (int64_t)j * 3;
    double u = fabs(ni[0] * nj[0] + ni[1] * nj[1] + ni[2] * nj[2]);
    if (!(u == u)) {  // a normal from non-finite coordinates
      bad = true;
      continue;
    }
    u = u > 1.0 ? 1.0 : u;
    const double pos = u * scale;
    const int b0 = min((int)floor(pos), D - 2);
    const double fr = pos - (double)b0;
    s_h[b0 * HN_BT + threadIdx.x] += 1.0 - fr;
    s_h[(b0 + 1) * HN_BT + threadIdx.x] += fr;
  }
  const double invk = 1.0 / (double)k;
  for (int b = 0; b < D; ++b) h_out[(int64_t)i * D + b] = bad ? NAN : (float)(s_h[b * HN_BT + threadIdx.x] * invk);
}

// Local polynomial descriptor (Sec. III-A lists local polynomial coefficients
// among the features): per point, its k neighbours in the frame of their
// covariance (1/k, centred at their mean; tangent axes of the two largest
// eigenvalues, normal of the smallest), coordinates divided by rho =
// sqrt(trace); the least-squares quadric h = c0 + c1 u + c2 v + c3 u^2 + c4 uv
// + c5 v^2 from its 6x6 normal equations (Cholesky, FP64); out = [mu1, mu2,
// r]: the eigenvalues mu1 >= mu2 of the Hessian [[2 c3, c4], [c4, 2 c5]],
// negated and swapped when their sum is negative (the normal's sign is
// arbitrary), and the RMS residual.  None of the three changes with rotation,
// translation, scale or the signs and in-plane rotation of the frame.  NaN
// when rho = 0 or the normal equations are singular (neighbours on a line).
__global__ __launch_bounds__(256) void poly_kernel(const float* __restrict__ X, const float* __restrict__ Y,
                                                   const float* __restrict__ Zc, int n, int k,
                                                   const int32_t* __restrict__ idx, float* __restrict__ out) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int32_t* nb = idx + (int64_t)i * k;
  double m[3] = {0, 0, 0};
  for (int s = 0; s < k; ++s) {
    const int j = nb[s] >= 0 ? nb[s] : i;
    m[0] += (double)X[j];
    m[1] += (double)Y[j];
    m[2] += (double)Zc[j];
  }
  const double invk = 1.0 / (double)k;
  for (int c = 0; c < 3; ++c) m[c] *= invk;
  double C[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int s = 0; s < k; ++s) {
    const int j = nb[s] >= 0 ? nb[s] : i;
    const double e[3] = {(double)X[j] - m[0], (double)Y[j] - m[1], (double)Zc[j] - m[2]};
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) C[r * 3 + c] += e[r] * e[c];
  }
  for (int e = 0; e < 9; ++e) C[e] *= invk;
  const double rho = sqrt(C[0] + C[4] + C[8]);
  float* o = out + (int64_t)i * 3;
  if (!(rho > 0.0)) {
    o[0] = o[1] = o[2] = NAN;
    return;
  }
  double sv[3], uu[3][3], vv[3][3];
  svd3(C, sv, uu, vv);  // vv[0], vv[1]: tangent axes; vv[2]: normal
  const double irho = 1.0 / rho;
  // normal equations over phi = (1, u, v, u^2, u v, v^2): packed lower triangle
  double A[21], b[6];
  for (int e = 0; e < 21; ++e) A[e] = 0.0;
  for (int e = 0; e < 6; ++e) b[e] = 0.0;
  for (int s = 0; s < k; ++s) {
    const int j = nb[s] >= 0 ? nb[s] : i;
    const double e[3] = {(double)X[j] - m[0], (double)Y[j] - m[1], (double)Zc[j] - m[2]};
    const double u = (e[0] * vv[0][0] + e[1] * vv[0][1] + e[2] * vv[0][2]) * irho;
    const double v = (e[0] * vv[1][0] + e[1] * vv[1][1] + e[2] * vv[1][2]) * irho;
    const double h = (e[0] * vv[2][0] + e[1] * vv[2][1] + e[2] * vv[2][2]) * irho;
    const double phi[6] = {1.0, u, v, u * u, u * v, v * v};
    int t = 0;
    for (int r = 0; r < 6; ++r) {
      for (int c = 0; c <= r; ++c) A[t++] += phi[r] * phi[c];
      b[r] += phi[r] * h;
    }
  }
  // Cholesky A = L L^T in place (packed lower triangle), then two solves
  bool ok = true;
  double scale = 0.0;
  for (int r = 0, t = 0; r < 6; t += ++r + 1) scale = fmax(scale, A[t]);
  for (int r = 0; r < 6; ++r) {
    const int rr = r * (r + 1) / 2;
    for (int c = 0; c <= r; ++c) {
      const int cc = c * (c + 1) / 2;
      double acc = A[rr + c];
      for (int q = 0; q < c; ++q) acc -= A[rr + q] * A[cc + q];
      if (c == r) {
        if (!(acc > 1e-13 * scale)) ok = false;
        A[rr + r] = sqrt(fmax(acc, 0.0));
      } else {
        A[rr + c] = acc / A[cc + c];
      }
    }
  }
  if (!ok) {
    o[0] = o[1] = o[2] = NAN;
    return;
  }
  double y[6], cf[6];
  for (int r = 0; r < 6; ++r) {
    const int rr = r * (r + 1) / 2;
    double acc = b[r];
    for (int q = 0; q < r; ++q) acc -= A[rr + q] * y[q];
    y[r] = acc / A[rr + r];
  }
  for (int r = 5; r >= 0; --r) {
    double acc = y[r];
    for (int q = r + 1; q < 6; ++q) acc -= A[q * (q + 1) / 2 + r] * cf[q];
    cf[r] = acc / A[r * (r + 1) / 2 + r];
  }
  // Hessian eigenvalues and the sign convention
  const double a11 = 2.0 * cf[3], a12 = cf[4], a22 = 2.0 * cf[5];
  const double mean = 0.5 * (a11 + a22), dev = sqrt(0.25 * (a11 - a22) * (a11 - a22) + a12 * a12);
  double mu1 = mean + dev, mu2 = mean - dev;
  if (mu1 + mu2 < 0.0) {
    const double t = mu1;
    mu1 = -mu2;
    mu2 = -t;
  }
  double r2 = 0.0;
  for (int s = 0; s < k; ++s) {
    const int j = nb[s] >= 0 ? nb[s] : i;
    const double e[3] = {(double)X[j] - m[0], (double)Y[j] - m[1], (double)Zc[j] - m[2]};
    const double u = (e[0] * vv[0][0] + e[1] * vv[0][1] + e[2] * vv[0][2]) * irho;
    const double v = (e[0] * vv[1][0] + e[1] * vv[1][1] + e[2] * vv[1][2]) * irho;
    const double h = (e[0] * vv[2][0] + e[1] * vv[2][1] + e[2] * vv[2][2]) * irho;
    const double d = h - (cf[0] + cf[1] * u + cf[2] * v + cf[3] * u * u + cf[4] * u * v + cf[5] * v * v);
    r2 += d * d;
  }
  o[0] = (float)mu1;
  o[1] = (float)mu2;
  o[2] = (float)sqrt(r2 * invk);
}

}  // namespace

size_t poly_workspace(int n, int k) {
  return 256 + (((size_t)n * k * 4 + 255) & ~(size_t)255) + grid_knn_workspace(n, k);
}

hipError_t launch_poly(const float* x, const float* y, const float* z, int n, int k, float* out, void* ws,
                       hipStream_t st) {
  char* p = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(ws) + 255) & ~(uintptr_t)255);
  int32_t* idx = reinterpret_cast<int32_t*>(p);
  p += ((size_t)n * k * 4 + 255) & ~(size_t)255;
  hipError_t e = launch_grid_knn(x, y, z, n, k, nullptr, idx, p, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(poly_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, x, y, z, n, k, idx, out);
  return hipGetLastError();
}

size_t normal_hist_workspace(int n, int k) {
  // base alignment, neighbour lists, normals, grid-search scratch
  return 256 + (((size_t)n * k * 4 + 255) & ~(size_t)255) + (((size_t)n * 24 + 255) & ~(size_t)255) +
         grid_knn_workspace(n, k);
}

hipError_t launch_normal_hist(const float* x, const float* y, const float* z, int n, int k, int D, float* h_out,
                              void* ws, hipStream_t st) {
  char* p = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(ws) + 255) & ~(uintptr_t)255);
  int32_t* idx = reinterpret_cast<int32_t*>(p);
  p += ((size_t)n * k * 4 + 255) & ~(size_t)255;
  double* nrm = reinterpret_cast<double*>(p);
  p += ((size_t)n * 24 + 255) & ~(size_t)255;
  hipError_t e = launch_grid_knn(x, y, z, n, k, nullptr, idx, p, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(normals_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, x, y, z, n, k, idx, nrm);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(hist_kernel, dim3((unsigned)((n + HN_BT - 1) / HN_BT)), dim3(HN_BT), 0, st, n, k, D, idx, nrm,
                     h_out);
  return hipGetLastError();
}

}  // namespace sgr
