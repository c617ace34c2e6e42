// Change detection after registration (the application of Sec. I and
// Sec. IV: parts of the registered template with no similar reference part
// nearby show the change).  For every template point i, posed by the final
// registration pose, with j its nearest reference point within tau:
//   bit 0: there is none (nothing near it),
//   bit 1: (a_i - a_j)^2 > sigma^2 (-ln s_min)   (the nearest point's shape
//          similarity exp(-(a_i - a_j)^2 / sigma^2) of eq. 3 is below s_min).
// Both decisions are taken in a precision a reader can reproduce: the posed
// point is formed in FP64 without fused operations and rounded once to
// FP32, the nearest point and the distance test use the FP32 key
// ((dx*dx + dy*dy) + dz*dz) with ties by index, and the shape test compares
// the exact FP64 curvature difference squared with an FP64 threshold.
#include "common.h"
#include "launch.h"

namespace sgr {

// T(y) = s R y + t, evaluated as s ((R_r0 y0 + R_r1 y1) + R_r2 y2) + t_r.
__global__ __launch_bounds__(256) void posed_exact_kernel(const float* __restrict__ x, const float* __restrict__ y,
                                                          const float* __restrict__ z, int M,
                                                          const double* __restrict__ pose, float* __restrict__ ox,
                                                          float* __restrict__ oy, float* __restrict__ oz) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= M) return;
  const double s = pose[0];
  const double p0 = (double)x[i], p1 = (double)y[i], p2 = (double)z[i];
  double o[3];
  for (int r = 0; r < 3; ++r) {  // every operation rounded on its own (this file is built without fusion)
    const double a = __dmul_rn(pose[1 + 3 * r], p0);
    const double b = __dmul_rn(pose[2 + 3 * r], p1);
    const double c = __dmul_rn(pose[3 + 3 * r], p2);
    o[r] = __dadd_rn(__dmul_rn(s, __dadd_rn(__dadd_rn(a, b), c)), pose[10 + r]);
  }
  ox[i] = (float)o[0];
  oy[i] = (float)o[1];
  oz[i] = (float)o[2];
}

__global__ __launch_bounds__(256) void change_flags_kernel(const float* __restrict__ aY, const float* __restrict__ aX,
                                                           const int32_t* __restrict__ nn, const float* __restrict__ key,
                                                           int M, float tau2, double shape_thr,
                                                           uint8_t* __restrict__ flags) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= M) return;
  const int j = nn[i];
  uint8_t f = 0;
  if (j < 0) {
    f = 1;  // no reference point within tau (or a non-finite posed point)
  } else {
    const double da = (double)aY[i] - (double)aX[j];
    if (da * da > shape_thr) f |= 2;
  }
  flags[i] = f;
}

size_t change_workspace(int M, int N) { return grid_knn_workspace(N, 1) + 3 * (((size_t)M * 4 + 255) & ~size_t(255)); }

hipError_t launch_change(const float* yx, const float* yy, const float* yz, const float* aY, int M, const float* xx,
                         const float* xy, const float* xz, const float* aX, int N, const double* pose, float tau2,
                         double shape_thr, uint8_t* flags, int32_t* nn, float* key, void* ws, hipStream_t st) {
  char* p = (char*)ws;
  const size_t qb = ((size_t)M * 4 + 255) & ~size_t(255);
  float* qx = (float*)p;
  float* qy = (float*)(p + qb);
  float* qz = (float*)(p + 2 * qb);
  void* gws = p + 3 * qb;
  hipLaunchKernelGGL(posed_exact_kernel, dim3((M + 255) / 256), dim3(256), 0, st, yx, yy, yz, M, pose, qx, qy, qz);
  if (hipError_t e = launch_grid_nn(xx, xy, xz, N, qx, qy, qz, M, tau2, nn, key, gws, st)) return e;
  hipLaunchKernelGGL(change_flags_kernel, dim3((M + 255) / 256), dim3(256), 0, st, aY, aX, nn, key, M, tau2, shape_thr,
                     flags);
  return hipGetLastError();
}

}  // namespace sgr
