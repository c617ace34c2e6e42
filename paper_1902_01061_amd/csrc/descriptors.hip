// Local shape descriptor (Sec. III-A: curvature of the local neighbourhood)
// and global moments (Sec. III-B: covariance eigenvalues for the scale).
//
// knn_desc_kernel: exact brute-force k nearest neighbours of every point,
// one query per lane.  The reference points stream through LDS in tiles of
// 256 (coalesced SoA loads, one float4 per lane); every lane reads the same
// LDS word (broadcast).  The running top-k sits in registers as a sorted
// list; a candidate closer than the current k-th is placed by a branch-free
// compare-exchange pass.  Distances are float32 ((dx*dx + dy*dy) + dz*dz)
// with each operation rounded (no contraction), ties broken by index, so
// the neighbour lists are fully determined.  The neighbourhood covariance
// (1/k, centred) and its eigenvalues are then taken in FP64 and the
// curvature is the PCA surface variation lambda_min / trace.
#include "common.h"
#include "launch.h"

namespace sgr {

constexpr int KNN_BT = 256;

template <int KC>
__device__ inline void knn_desc_body(const float* __restrict__ X, const float* __restrict__ Y,
                                     const float* __restrict__ Zc, int n, int k, float* __restrict__ a_out,
                                     int32_t* __restrict__ idx_out, int qblock, float4* tile) {
  const int q = qblock * KNN_BT + threadIdx.x;
  const bool valid = q < n;
  const float qx = valid ? X[q] : 0.f;
  const float qy = valid ? Y[q] : 0.f;
  const float qz = valid ? Zc[q] : 0.f;
  // Sorted ascending.  Slots [0, KC-k) hold -inf sentinels that never move,
  // so bd[KC-1] is always the k-th best distance.
  float bd[KC];
  int bi[KC];
#pragma unroll
  for (int s = 0; s < KC; ++s) {
    bd[s] = (s < KC - k) ? -INFINITY : INFINITY;
    bi[s] = -1;
  }
  for (int base = 0; base < n; base += KNN_BT) {
    const int j = base + threadIdx.x;
    __syncthreads();
    tile[threadIdx.x] = (j < n) ? make_float4(X[j], Y[j], Zc[j], 0.f) : make_float4(0.f, 0.f, 0.f, 0.f);
    __syncthreads();
    const int cnt = min(KNN_BT, n - base);
    for (int jj = 0; jj < cnt; ++jj) {
      const float4 p = tile[jj];
      const float dx = __fsub_rn(p.x, qx);
      const float dy = __fsub_rn(p.y, qy);
      const float dz = __fsub_rn(p.z, qz);
      const float d2 = __fadd_rn(__fadd_rn(__fmul_rn(dx, dx), __fmul_rn(dy, dy)), __fmul_rn(dz, dz));
      if (d2 < bd[KC - 1]) {
        float cd = d2;
        int ci = base + jj;
#pragma unroll
        for (int s = 0; s < KC; ++s) {
          const bool sw = cd < bd[s];
          const float td = bd[s];
          const int ti = bi[s];
          bd[s] = sw ? cd : td;
          bi[s] = sw ? ci : ti;
          cd = sw ? td : cd;
          ci = sw ? ti : ci;
        }
      }
    }
  }
  if (!valid) return;
  // Neighbourhood covariance in FP64 (1/k, centred at the neighbourhood mean).
  double m[3] = {0, 0, 0};
#pragma unroll
  for (int s = 0; s < KC; ++s) {
    if (s < KC - k) continue;
    const int id = bi[s] >= 0 ? bi[s] : q;
    m[0] += (double)X[id];
    m[1] += (double)Y[id];
    m[2] += (double)Zc[id];
  }
  const double invk = 1.0 / (double)k;
  m[0] *= invk;
  m[1] *= invk;
  m[2] *= invk;
  double C[6] = {0, 0, 0, 0, 0, 0};
  bool missing = false;
#pragma unroll
  for (int s = 0; s < KC; ++s) {
    if (s < KC - k) continue;
    missing |= bi[s] < 0;
    const int id = bi[s] >= 0 ? bi[s] : q;
    const double ex = (double)X[id] - m[0], ey = (double)Y[id] - m[1], ez = (double)Zc[id] - m[2];
    C[0] += ex * ex;
    C[1] += ey * ey;
    C[2] += ez * ez;
    C[3] += ex * ey;
    C[4] += ex * ez;
    C[5] += ey * ez;
    if (idx_out) idx_out[(int64_t)q * k + (s - (KC - k))] = bi[s];
  }
#pragma unroll
  for (int c = 0; c < 6; ++c) C[c] *= invk;
  double lam[3];
  eig_psd3(C, lam);
  const double tr = C[0] + C[1] + C[2];
  float a = (tr > 0.0) ? (float)(lam[2] / tr) : 0.f;
  if (missing) a = NAN;  // non-finite coordinates: no complete neighbourhood
  if (a_out) a_out[q] = a;
}

template <int KC>
__global__ __launch_bounds__(KNN_BT) void knn_desc_kernel(const float* __restrict__ X, const float* __restrict__ Y,
                                                          const float* __restrict__ Zc, int n, int k,
                                                          float* __restrict__ a_out, int32_t* __restrict__ idx_out) {
  __shared__ float4 tile[KNN_BT];
  knn_desc_body<KC>(X, Y, Zc, n, k, a_out, idx_out, blockIdx.x, tile);
}

// Many clouds in one launch: block b works on query block blocks[b].y of
// cloud blocks[b].x.
template <int KC>
__global__ __launch_bounds__(KNN_BT) void knn_desc_batch_kernel(const CloudDesc* __restrict__ clouds,
                                                                const int2* __restrict__ blocks, int k) {
  __shared__ float4 tile[KNN_BT];
  const int2 b = blocks[blockIdx.x];
  const CloudDesc& c = clouds[b.x];
  knn_desc_body<KC>(c.x, c.y, c.z, c.n, k, c.a_out, nullptr, b.y, tile);
}

// Centroid, covariance (1/n) and its largest eigenvalue; two passes over
// the cloud in one block with a fixed-order FP64 reduction (deterministic).
__device__ inline void moments_body(const float* __restrict__ X, const float* __restrict__ Y,
                                    const float* __restrict__ Zc, int64_t n, double* __restrict__ out, double* lds,
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
  moments_body(c.x, c.y, c.z, c.n, out + 10 * (int64_t)blockIdx.x, lds, cen);
}

hipError_t launch_knn_desc(const float* x, const float* y, const float* z, int n, int k, float* a_out,
                           int32_t* idx_out, hipStream_t st) {
  const dim3 grid((n + KNN_BT - 1) / KNN_BT), block(KNN_BT);
  if (k <= 8)
    hipLaunchKernelGGL(knn_desc_kernel<8>, grid, block, 0, st, x, y, z, n, k, a_out, idx_out);
  else if (k <= 16)
    hipLaunchKernelGGL(knn_desc_kernel<16>, grid, block, 0, st, x, y, z, n, k, a_out, idx_out);
  else if (k <= 24)
    hipLaunchKernelGGL(knn_desc_kernel<24>, grid, block, 0, st, x, y, z, n, k, a_out, idx_out);
  else
    hipLaunchKernelGGL(knn_desc_kernel<32>, grid, block, 0, st, x, y, z, n, k, a_out, idx_out);
  return hipGetLastError();
}

hipError_t launch_knn_desc_batch(const CloudDesc* clouds, const int2* blocks, int n_blocks, int k, hipStream_t st) {
  const dim3 grid(n_blocks), block(KNN_BT);
  if (k <= 8)
    hipLaunchKernelGGL(knn_desc_batch_kernel<8>, grid, block, 0, st, clouds, blocks, k);
  else if (k <= 16)
    hipLaunchKernelGGL(knn_desc_batch_kernel<16>, grid, block, 0, st, clouds, blocks, k);
  else if (k <= 24)
    hipLaunchKernelGGL(knn_desc_batch_kernel<24>, grid, block, 0, st, clouds, blocks, k);
  else
    hipLaunchKernelGGL(knn_desc_batch_kernel<32>, grid, block, 0, st, clouds, blocks, k);
  return hipGetLastError();
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
