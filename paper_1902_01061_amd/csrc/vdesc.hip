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

}  // namespace

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
