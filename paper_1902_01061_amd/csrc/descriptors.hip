// Global moments (Sec. III-B: centroid, covariance and its largest
// eigenvalue, for the scale).  The local shape descriptors (Sec. III-A) come
// from the grid search in knn_grid.hip.
#include "common.h"
#include "launch.h"

namespace sgr {

// Centroid, covariance (1/n) and its largest eigenvalue; two passes over
// the cloud in one block with a fixed-order FP64 reduction (deterministic).
__device__ inline __attribute__((always_inline)) void moments_body(const float* __restrict__ X,
                                                                   const float* __restrict__ Y,
                                                                   const float* __restrict__ Zc, int64_t n,
                                                                   double* __restrict__ out, double* lds,
                                                                   double* cen) {
  double s[3] = {0, 0, 0};
  for (int64_t i = threadIdx.x; i < n; i += 1024) {
    s[0] += X[i];
    s[1] += Y[i];
    s[2] += Zc[i];
  }
  block_sum<3, 1024>(s, lds);
  if (threadIdx.x == 0) {
    for (int c = 0; c < 3; ++c) cen[c] = s[c] / (double)n;
  }
  __syncthreads();
  const double cx = cen[0], cy = cen[1], cz = cen[2];
  double v[6] = {0, 0, 0, 0, 0, 0};
  for (int64_t i = threadIdx.x; i < n; i += 1024) {
    const double ex = X[i] - cx, ey = Y[i] - cy, ez = Zc[i] - cz;
    v[0] += ex * ex;
    v[1] += ey * ey;
    v[2] += ez * ez;
    v[3] += ex * ey;
    v[4] += ex * ez;
    v[5] += ey * ez;
  }
  block_sum<6, 1024>(v, lds);
  if (threadIdx.x == 0) {
    double C[6];
    for (int c = 0; c < 6; ++c) C[c] = v[c] / (double)n;
    double lam[3];
    eig_psd3(C, lam);
    out[0] = cx;
    out[1] = cy;
    out[2] = cz;
    for (int c = 0; c < 6; ++c) out[3 + c] = C[c];
    out[9] = lam[0];
  }
}

__global__ __launch_bounds__(1024) void moments_kernel(const float* __restrict__ X, const float* __restrict__ Y,
                                                       const float* __restrict__ Zc, int64_t n, double* __restrict__ out) {
  __shared__ double lds[16 * 6];
  __shared__ double cen[3];
  moments_body(X, Y, Zc, n, out, lds, cen);
}

// One block per cloud; cloud c writes out[10 c .. 10 c + 9].
__global__ __launch_bounds__(1024) void moments_batch_kernel(const CloudDesc* __restrict__ clouds,
                                                             double* __restrict__ out) {
  __shared__ double lds[16 * 6];
  __shared__ double cen[3];
  const CloudDesc& c = clouds[blockIdx.x];
  moments_body(gptr(c.x), gptr(c.y), gptr(c.z), c.n, out + 10 * (int64_t)blockIdx.x, lds, cen);
}

hipError_t launch_moments_batch(const CloudDesc* clouds, int n_clouds, double* out, hipStream_t st) {
  hipLaunchKernelGGL(moments_batch_kernel, dim3(n_clouds), dim3(1024), 0, st, clouds, out);
  return hipGetLastError();
}

hipError_t launch_moments(const float* x, const float* y, const float* z, int64_t n, double* out, hipStream_t st) {
  hipLaunchKernelGGL(moments_kernel, dim3(1), dim3(1024), 0, st, x, y, z, n, out);
  return hipGetLastError();
}

}  // namespace sgr
