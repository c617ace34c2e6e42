// Visiting order of the template points for the force kernel: a stable sort
// by curvature.  The force on a point does not depend on the order, but a
// block of the force kernel then holds points whose similarity coordinates
// b = (a - abar) sqrt(log2 e) / sigma span a narrow range, so the block can
// centre the expanded similarity exponent on that range (eq. 3) and use one
// FMA per pair.  b is an increasing function of a, so sorting the FP32
// curvatures orders b.  Radix sort is stable: equal curvatures keep their
// index order and the permutation is deterministic.
#include <hipcub/hipcub.hpp>

#include "launch.h"

namespace sgr {

namespace {

constexpr size_t kAlign = 256;

size_t up(size_t b) { return (b + kAlign - 1) & ~(kAlign - 1); }

__global__ __launch_bounds__(256) void iota_kernel(int* __restrict__ v, int n) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) v[i] = i;
}

// keys[off[r] + i] = aY_r[i], idx[off[r] + i] = i for every registration r
__global__ __launch_bounds__(256) void seg_gather_kernel(const RegDesc* __restrict__ regs,
                                                         const int* __restrict__ off, float* __restrict__ keys,
                                                         int* __restrict__ idx) {
  const int r = blockIdx.y;
  const int M = regs[r].M;
  const float* __restrict__ a = gptr(regs[r].aY);
  const int o = off[r];
  for (int i = blockIdx.x * 256 + threadIdx.x; i < M; i += gridDim.x * 256) {
    keys[o + i] = a[i];
    idx[o + i] = i;
  }
}

size_t temp_bytes(int64_t n, int nseg) {
  size_t tb = 0;
  if (nseg <= 1)
    (void)hipcub::DeviceRadixSort::SortPairs(nullptr, tb, (const float*)nullptr, (float*)nullptr,
                                             (const int*)nullptr, (int*)nullptr, (int)n, 0, 32, (hipStream_t)0);
  else
    (void)hipcub::DeviceSegmentedRadixSort::SortPairs(nullptr, tb, (const float*)nullptr, (float*)nullptr,
                                                      (const int*)nullptr, (int*)nullptr, (int)n, nseg,
                                                      (const int*)nullptr, (const int*)nullptr, 0, 32, (hipStream_t)0);
  return tb;
}

}  // namespace

size_t sort_perm_workspace(int64_t n, int nseg) {
  // keys in (batch), keys out, index in, radix-sort temporaries
  return 3 * up((size_t)n * 4) + up(temp_bytes(n, nseg)) + kAlign;
}

hipError_t launch_sort_perm(const float* aY, int M, int* perm, void* ws, hipStream_t st) {
  char* p = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(ws) + kAlign - 1) & ~(uintptr_t)(kAlign - 1));
  float* keys_out = reinterpret_cast<float*>(p);
  p += up((size_t)M * 4);
  int* idx = reinterpret_cast<int*>(p);
  p += up((size_t)M * 4);
  size_t tb = temp_bytes(M, 1);
  hipLaunchKernelGGL(iota_kernel, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, st, idx, M);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return hipcub::DeviceRadixSort::SortPairs(p, tb, aY, keys_out, idx, perm, M, 0, 32, st);
}

hipError_t launch_sort_perm_batch(const RegDesc* regs, int B, const int* off, int64_t total, int max_M, int* perm,
                                  void* ws, hipStream_t st) {
  char* p = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(ws) + kAlign - 1) & ~(uintptr_t)(kAlign - 1));
  float* keys_in = reinterpret_cast<float*>(p);
  p += up((size_t)total * 4);
  float* keys_out = reinterpret_cast<float*>(p);
  p += up((size_t)total * 4);
  int* idx = reinterpret_cast<int*>(p);
  p += up((size_t)total * 4);
  size_t tb = temp_bytes(total, B);
  const unsigned gx = (unsigned)std::min<int64_t>(64, (max_M + 255) / 256);
  hipLaunchKernelGGL(seg_gather_kernel, dim3(gx, (unsigned)B), dim3(256), 0, st, regs, off, keys_in, idx);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (B == 1) return hipcub::DeviceRadixSort::SortPairs(p, tb, keys_in, keys_out, idx, perm, (int)total, 0, 32, st);
  return hipcub::DeviceSegmentedRadixSort::SortPairs(p, tb, keys_in, keys_out, idx, perm, (int)total, B, off, off + 1,
                                                     0, 32, st);
}

}  // namespace sgr
