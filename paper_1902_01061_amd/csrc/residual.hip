// Registration residual (the RMSE of Sec. V): with correspondences,
// sqrt(mean |T(y_i) - x_corr(i)|^2) over i with corr(i) >= 0; without, the
// one-sided nearest-neighbour RMSE template -> reference.  The nearest
// neighbour is chosen by float32 squared distance of the float32-rounded
// transformed point (ties by index, reference streamed through LDS); the
// distance that enters the mean is recomputed in FP64.
#include "common.h"
#include "launch.h"

namespace sgr {

constexpr int RS_BT = 256;

__global__ __launch_bounds__(RS_BT) void residual_kernel(const float* __restrict__ yx, const float* __restrict__ yy,
                                                         const float* __restrict__ yz, int M,
                                                         const float* __restrict__ xx, const float* __restrict__ xy,
                                                         const float* __restrict__ xz, int N,
                                                         const double* __restrict__ pose,
                                                         const int32_t* __restrict__ corr, double* __restrict__ part) {
  __shared__ float4 tile[RS_BT];
  __shared__ double lds[(RS_BT / 64) * 2];
  const int i = blockIdx.x * RS_BT + threadIdx.x;
  const bool valid = i < M;
  double T[3] = {0, 0, 0};
  if (valid) {
    const double s = pose[0];
    const double p0 = yx[i], p1 = yy[i], p2 = yz[i];
    for (int r = 0; r < 3; ++r)
      T[r] = s * (pose[1 + 3 * r] * p0 + pose[2 + 3 * r] * p1 + pose[3 + 3 * r] * p2) + pose[10 + r];
  }
  double v[2] = {0, 0};
  if (corr) {
    if (valid && corr[i] >= 0 && corr[i] < N) {
      const int j = corr[i];
      const double dx = T[0] - xx[j], dy = T[1] - xy[j], dz = T[2] - xz[j];
      v[0] = dx * dx + dy * dy + dz * dz;
      v[1] = 1.0;
    }
  } else {
    const float qx = (float)T[0], qy = (float)T[1], qz = (float)T[2];
    float best = INFINITY;
    int bj = -1;
    for (int base = 0; base < N; base += RS_BT) {
      const int j = base + threadIdx.x;
      __syncthreads();
      tile[threadIdx.x] = (j < N) ? make_float4(xx[j], xy[j], xz[j], 0.f) : make_float4(0.f, 0.f, 0.f, 0.f);
      __syncthreads();
      const int cnt = min(RS_BT, N - base);
      for (int jj = 0; jj < cnt; ++jj) {
        const float4 p = tile[jj];
        const float dx = __fsub_rn(p.x, qx), dy = __fsub_rn(p.y, qy), dz = __fsub_rn(p.z, qz);
        const float d2 = __fadd_rn(__fadd_rn(__fmul_rn(dx, dx), __fmul_rn(dy, dy)), __fmul_rn(dz, dz));
        if (d2 < best) {
          best = d2;
          bj = base + jj;
        }
      }
    }
    if (valid && bj >= 0) {
      const double dx = T[0] - xx[bj], dy = T[1] - xy[bj], dz = T[2] - xz[bj];
      v[0] = dx * dx + dy * dy + dz * dz;
      v[1] = 1.0;
    }
  }
  block_sum<2, RS_BT>(v, lds);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = v[0];
    part[2 * blockIdx.x + 1] = v[1];
  }
}

__global__ __launch_bounds__(256) void residual_final_kernel(const double* __restrict__ part, int nblk,
                                                             double* __restrict__ out) {
  __shared__ double lds[4 * 2];
  double v[2] = {0, 0};
  for (int b = threadIdx.x; b < nblk; b += 256) {
    v[0] += part[2 * b];
    v[1] += part[2 * b + 1];
  }
  block_sum<2, 256>(v, lds);
  if (threadIdx.x == 0) out[0] = v[1] > 0 ? sqrt(v[0] / v[1]) : NAN;
}

int residual_blocks(int M) { return (M + RS_BT - 1) / RS_BT; }

hipError_t launch_residual(const float* yx, const float* yy, const float* yz, int M, const float* xx, const float* xy,
                           const float* xz, int N, const double* pose, const int32_t* corr, double* part, int nblk,
                           double* rmse_out, hipStream_t st) {
  hipLaunchKernelGGL(residual_kernel, dim3(nblk), dim3(RS_BT), 0, st, yx, yy, yz, M, xx, xy, xz, N, pose, corr, part);
  hipLaunchKernelGGL(residual_final_kernel, dim3(1), dim3(256), 0, st, part, nblk, rmse_out);
  return hipGetLastError();
}

}  // namespace sgr
