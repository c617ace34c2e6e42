// Pose-independent pair sums of the p = 1 law (eq. 5 with h = 1; eqs. 3, 10).
//
// With p = 1 the pair weight c_ij = exp2(lw_j - (b_i - b_j)^2), lw_j the
// log2 of the reference mass (times a_j / abar for eq. 10), depends on the
// descriptors and masses only, never on the pose.  The force on template
// point i is then linear in its posed position y_i:
//   f_i = -(G / Z) g_i sum_j c_ij (y_i - x_j) = -(G / Z) g_i (y_i S0_i - S1_i),
// with S0_i = sum_j c_ij and S1_i = sum_j c_ij x_j, and its energy term is
// g_i ((|y_i|^2 + eps^2) S0_i - 2 y_i . S1_i + S2_i) with S2_i = sum_j c_ij
// |x_j|^2 (x_j relative to the reference centroid, as everywhere).
//
// psum_kernel forms S0, S1, S2 once per registration (scalar descriptors;
// the vector-descriptor kernel writes the same sums itself), one pass over all
// pairs: a block of 1 024 template points (visiting order, four per lane)
// against one chunk of the reference, staged through LDS 256 points at a
// time; every lane sums a tile's 256 terms per point in FP32 and adds them
// to FP64 sums, as the force kernel does.  psum_reduce_kernel adds the chunks in a fixed order.  pinv_kernel
// is then the whole per-iteration force: O(M) work that poses the template
// exactly as the force kernel does (FP64 pose, FP32 posed point), forms the
// forces in FP64 and writes the same per-block wrench partials for the
// update kernel.
#include <algorithm>

#include "common.h"
#include "launch.h"

namespace sgr {

namespace {

constexpr int PS_BT = 256;
constexpr int PS_NQ = 5;  // S0, S1 (3), S2

// Sums of template point bi's pair weights over reference points [j0, j1)
// into t (FP64), one LDS tile of PS_BT points at a time (every thread of the
// block calls it with the same range).
__device__ inline void pair_sums(float bi, const float4* __restrict__ ref4, const float* __restrict__ lw, int j0,
                                 int j1, float4* s_x, float* s_l, float* s_q, double* t) {
  for (int base = j0; base < j1; base += PS_BT) {
    __syncthreads();
    {
      const int j = base + threadIdx.x;
      float4 X = make_float4(0.f, 0.f, 0.f, 0.f);
      float l = -INFINITY;  // exp2(-inf) = 0: beyond the range
      if (j < j1) {
        X = ref4[j];
        l = lw[j];
      }
      s_x[threadIdx.x] = X;
      s_l[threadIdx.x] = l;
      s_q[threadIdx.x] = __builtin_fmaf(X.x, X.x, __builtin_fmaf(X.y, X.y, X.z * X.z));
    }
    __syncthreads();
    const int n = min(PS_BT, j1 - base);
    float a0 = 0.f, ax = 0.f, ay = 0.f, az = 0.f, aq = 0.f;
    for (int jj = 0; jj < n; ++jj) {
      const float4 X = s_x[jj];
      const float d = bi - X.w;
      const float c = __builtin_amdgcn_exp2f(__builtin_fmaf(-d, d, s_l[jj]));
      a0 += c;
      ax = __builtin_fmaf(c, X.x, ax);
      ay = __builtin_fmaf(c, X.y, ay);
      az = __builtin_fmaf(c, X.z, az);
      aq = __builtin_fmaf(c, s_q[jj], aq);
    }
    t[0] += (double)a0;
    t[1] += (double)ax;
    t[2] += (double)ay;
    t[3] += (double)az;
    t[4] += (double)aq;
  }
}

// One block: PS_R * 256 template points (visiting order), PS_R per lane,
// against one chunk of the reference; every staged point is read from LDS
// once for the lane's PS_R points.
constexpr int PS_R = 4;

__global__ __launch_bounds__(PS_BT) void psum_kernel(const float4* __restrict__ tm4, int M,
                                                     const float4* __restrict__ ref4, const float* __restrict__ lw,
                                                     int N, int chunk_len, double* __restrict__ part) {
  __shared__ float4 s_x[PS_BT];
  __shared__ float s_l[PS_BT], s_q[PS_BT];
  const int n_iblk = (M + PS_BT * PS_R - 1) / (PS_BT * PS_R);
  const int iblk = blockIdx.x % n_iblk, chunk = blockIdx.x / n_iblk;
  const int ip0 = iblk * PS_BT * PS_R + threadIdx.x;
  float bi[PS_R];
#pragma unroll
  for (int r = 0; r < PS_R; ++r) bi[r] = ip0 + r * PS_BT < M ? tm4[ip0 + r * PS_BT].w : 0.f;
  const int j0 = chunk * chunk_len, j1 = min(N, j0 + chunk_len);
  double t[PS_R][PS_NQ];
#pragma unroll
  for (int r = 0; r < PS_R; ++r)
#pragma unroll
    for (int q = 0; q < PS_NQ; ++q) t[r][q] = 0.0;
  for (int base = j0; base < j1; base += PS_BT) {
    __syncthreads();
    {
      const int j = base + threadIdx.x;
      float4 X = make_float4(0.f, 0.f, 0.f, 0.f);
      float l = -INFINITY;  // exp2(-inf) = 0: beyond the range
      if (j < j1) {
        X = ref4[j];
        l = lw[j];
      }
      s_x[threadIdx.x] = X;
      s_l[threadIdx.x] = l;
      s_q[threadIdx.x] = __builtin_fmaf(X.x, X.x, __builtin_fmaf(X.y, X.y, X.z * X.z));
    }
    __syncthreads();
    const int n = min(PS_BT, j1 - base);
    float a[PS_R][PS_NQ];
#pragma unroll
    for (int r = 0; r < PS_R; ++r)
#pragma unroll
      for (int q = 0; q < PS_NQ; ++q) a[r][q] = 0.f;
    for (int jj = 0; jj < n; ++jj) {
      const float4 X = s_x[jj];
      const float l = s_l[jj], xq = s_q[jj];
#pragma unroll
      for (int r = 0; r < PS_R; ++r) {
        const float d = bi[r] - X.w;
        const float c = __builtin_amdgcn_exp2f(__builtin_fmaf(-d, d, l));
        a[r][0] += c;
        a[r][1] = __builtin_fmaf(c, X.x, a[r][1]);
        a[r][2] = __builtin_fmaf(c, X.y, a[r][2]);
        a[r][3] = __builtin_fmaf(c, X.z, a[r][3]);
        a[r][4] = __builtin_fmaf(c, xq, a[r][4]);
      }
    }
#pragma unroll
    for (int r = 0; r < PS_R; ++r)
#pragma unroll
      for (int q = 0; q < PS_NQ; ++q) t[r][q] += (double)a[r][q];
  }
#pragma unroll
  for (int r = 0; r < PS_R; ++r) {
    const int ip = ip0 + r * PS_BT;
    if (ip < M) {
      double* o = part + ((int64_t)chunk * M + ip) * PS_NQ;
#pragma unroll
      for (int q = 0; q < PS_NQ; ++q) o[q] = t[r][q];
    }
  }
}

// Batched form: block (r, b) of tblk takes template points [256 b, 256 b +
// 256) of registration r against its whole reference, and writes their sums
// at template offset poff[r].
__global__ __launch_bounds__(PS_BT) void psum_batch_kernel(const RegDesc* __restrict__ regs,
                                                           const int2* __restrict__ tblk,
                                                           const int* __restrict__ poff,
                                                           const float4* __restrict__ ref4,
                                                           const float* __restrict__ lw, double* __restrict__ S) {
  __shared__ float4 s_x[PS_BT];
  __shared__ float s_l[PS_BT], s_q[PS_BT];
  const int2 rb = tblk[blockIdx.x];
  const RegDesc g = reg_at(regs, rb.x);
  const int ip = rb.y * PS_BT + threadIdx.x;
  const float bi = ip < g.M ? g.tm4[ip].w : 0.f;
  double t[PS_NQ] = {0.0, 0.0, 0.0, 0.0, 0.0};
  pair_sums(bi, ref4 + g.ref_off, lw + g.ref_off, 0, g.N, s_x, s_l, s_q, t);
  if (ip < g.M) {
    double* o = S + ((int64_t)poff[rb.x] + ip) * PS_NQ;
#pragma unroll
    for (int q = 0; q < PS_NQ; ++q) o[q] = t[q];
  }
}

__global__ __launch_bounds__(256) void psum_reduce_kernel(const double* __restrict__ part, int M, int n_chunks,
                                                          double* __restrict__ S) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)M * PS_NQ) return;
  double s = 0.0;
  for (int c = 0; c < n_chunks; ++c) s += part[(int64_t)c * M * PS_NQ + e];
  S[e] = s;
}

// Wrench terms of template point ip (visiting order) of one registration:
// the posed point as the force kernel forms it (FP64 pose, rounded once to
// FP32), then its force and energy from the pair sums s, in FP64.
template <bool WU>
__device__ inline void pinv_point(const float4* __restrict__ tm4, const float2* __restrict__ tmx, const double* s,
                                  int ip, const double* __restrict__ pose, const Derived& D, int t, double* w) {
  double sR[9], cv[3];
  const double sc = pose[0];
#pragma unroll
  for (int e = 0; e < 9; ++e) sR[e] = sc * pose[1 + e];
#pragma unroll
  for (int r = 0; r < 3; ++r)
    cv[r] = sR[3 * r] * D.ybar0[0] + sR[3 * r + 1] * D.ybar0[1] + sR[3 * r + 2] * D.ybar0[2] + pose[10 + r] -
            D.xbar[r];
  // eq. (12), reading: iteration t uses 0.1 G1 + 0.9 G1 / (1 + exp(-(t - 1 - E/2)))
  const double G = 0.1 * D.G1 + 0.9 * D.G1 / (1.0 + exp(-(((double)t - 1.0) - 0.5 * D.E)));
  const double coef = -(G / D.Z) * D.coefL;
  const double ucoef = (G / D.Z) * D.coefL / (D.p + 1.0);
  const float4 T = tm4[ip];
  const double ex = (double)T.x - D.ybar0[0], ey = (double)T.y - D.ybar0[1], ez = (double)T.z - D.ybar0[2];
  // the posed point relative to xbar, rounded once to FP32
  const float pxf = (float)(sR[0] * ex + sR[1] * ey + sR[2] * ez + cv[0]);
  const float pyf = (float)(sR[3] * ex + sR[4] * ey + sR[5] * ez + cv[1]);
  const float pzf = (float)(sR[6] * ex + sR[7] * ey + sR[8] * ez + cv[2]);
  const double px = pxf, py = pyf, pz = pzf;
  const double tx = px * s[0] - s[1], ty = py * s[0] - s[2], tz = pz * s[0] - s[3];
  const float2 A2 = tmx[ip];
  const double gi = D.g_mode == 1.0 ? (double)A2.x / D.abar : 1.0;
  const double mi = (double)A2.y;
  const double fx = coef * gi * tx, fy = coef * gi * ty, fz = coef * gi * tz;
  const double cx = px - cv[0], cy = py - cv[1], cz = pz - cv[2];
  w[WR_F + 0] = mi * fx;
  w[WR_F + 1] = mi * fy;
  w[WR_F + 2] = mi * fz;
  w[WR_K + 0] = fx * cx;
  w[WR_K + 1] = fx * cy;
  w[WR_K + 2] = fx * cz;
  w[WR_K + 3] = fy * cx;
  w[WR_K + 4] = fy * cy;
  w[WR_K + 5] = fy * cz;
  w[WR_K + 6] = fz * cx;
  w[WR_K + 7] = fz * cy;
  w[WR_K + 8] = fz * cz;
  if constexpr (WU)
    w[WR_U] = ucoef * gi * ((px * px + py * py + pz * pz + D.eps2) * s[0] - 2.0 * (px * s[1] + py * s[2] + pz * s[3]) +
                            s[4]);
}

__global__ __launch_bounds__(256) void pack_plain_kernel(const float* __restrict__ x, const float* __restrict__ y,
                                                         const float* __restrict__ z, const float* __restrict__ mY, int M,
                                                         float4* __restrict__ tm4, float2* __restrict__ tmx) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= M) return;
  tm4[i] = make_float4(x[i], y[i], z[i], 0.f);
  tmx[i] = make_float2(0.f, mY ? mY[i] : 1.f);
}

template <bool WU>
__global__ __launch_bounds__(PS_BT) void pinv_kernel(const float4* __restrict__ tm4, const float2* __restrict__ tmx,
                                                     const double* __restrict__ S, int M,
                                                     const double* __restrict__ pose, const Derived* __restrict__ dv,
                                                     int t, double* __restrict__ wpart) {
  __shared__ double s_red[(PS_BT / 64) * 13];
  double w[13];
#pragma unroll
  for (int e = 0; e < 13; ++e) w[e] = 0.0;
  const int ip = blockIdx.x * PS_BT + threadIdx.x;
  if (ip < M) pinv_point<WU>(tm4, tmx, S + (int64_t)ip * PS_NQ, ip, pose, *dv, t, w);
  block_sum<13, PS_BT>(w, s_red);
  if (threadIdx.x == 0) {
    double* o = wpart + (int64_t)blockIdx.x * WR_STRIDE;
#pragma unroll
    for (int e = 0; e < 13; ++e) o[e] = w[e];
  }
}

// Batched form: block (r, b) of tblk, wrench slot regs[r].wslot0 + b (regs
// here describe the slot layout of this kernel: one slot per 256 points).
template <bool WU>
__global__ __launch_bounds__(PS_BT) void pinv_batch_kernel(const RegDesc* __restrict__ regs,
                                                           const int2* __restrict__ tblk,
                                                           const int* __restrict__ poff,
                                                           const double* __restrict__ S,
                                                           const double* __restrict__ poses,
                                                           const Derived* __restrict__ dvs, int t,
                                                           double* __restrict__ wpart) {
  __shared__ double s_red[(PS_BT / 64) * 13];
  const int2 rb = tblk[blockIdx.x];
  const RegDesc g = reg_at(regs, rb.x);
  double w[13];
#pragma unroll
  for (int e = 0; e < 13; ++e) w[e] = 0.0;
  const int ip = rb.y * PS_BT + threadIdx.x;
  if (ip < g.M)
    pinv_point<WU>(g.tm4, g.tmx, S + ((int64_t)poff[rb.x] + ip) * PS_NQ, ip, poses + 13 * (int64_t)rb.x, dvs[rb.x],
                   t, w);
  block_sum<13, PS_BT>(w, s_red);
  if (threadIdx.x == 0) {
    double* o = wpart + ((int64_t)g.wslot0 + rb.y) * WR_STRIDE;
#pragma unroll
    for (int e = 0; e < 13; ++e) o[e] = w[e];
  }
}

}  // namespace

// Reference chunks of psum_kernel: about 4 blocks per CU, and up to 24 while
// every block keeps at least 4e6 pairs (more rounds of shorter chunks even
// out the end of a large launch; on a small pair each block's fixed start
// and end would dominate).
int pinv_chunks(int M, int N, int n_cu) {
  const int n_iblk = (M + PS_BT * PS_R - 1) / (PS_BT * PS_R);
  const int n_t = (N + PS_BT - 1) / PS_BT;
  const int64_t lo = int64_t(4) * n_cu, hi = int64_t(24) * n_cu;
  const int64_t target = std::min(hi, std::max(lo, (int64_t)M * N / 4000000));
  const int nc = (int)((target + n_iblk - 1) / n_iblk);
  return std::max(1, std::min(nc, n_t));
}

int pinv_blocks(int M) { return (M + PS_BT - 1) / PS_BT; }

hipError_t launch_psum(const float4* tm4, int M, const float4* ref4, const float* lw, int N, int n_chunks,
                       double* part, double* S, hipStream_t st) {
  if (M <= 0) return hipSuccess;
  const int n_t = (N + PS_BT - 1) / PS_BT;
  const int chunk_len = (n_t + n_chunks - 1) / n_chunks * PS_BT;  // whole tiles
  const int nc = (N + chunk_len - 1) / chunk_len;                // chunks actually used
  const int n_iblk = (M + PS_BT * PS_R - 1) / (PS_BT * PS_R);
  hipLaunchKernelGGL(psum_kernel, dim3((unsigned)(n_iblk * nc)), dim3(PS_BT), 0, st, tm4, M, ref4, lw, N, chunk_len,
                     part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_psum_reduce(part, M, nc, S, st);
}

hipError_t launch_psum_reduce(const double* part, int M, int n_chunks, double* S, hipStream_t st) {
  if (M <= 0) return hipSuccess;
  const int64_t ne = (int64_t)M * PS_NQ;
  hipLaunchKernelGGL(psum_reduce_kernel, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, st, part, M, n_chunks, S);
  return hipGetLastError();
}

hipError_t launch_pack_plain(const float* x, const float* y, const float* z, const float* mY, int M, float4* tm4,
                             float2* tmx, hipStream_t st) {
  if (M <= 0) return hipSuccess;
  hipLaunchKernelGGL(pack_plain_kernel, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, st, x, y, z, mY, M, tm4, tmx);
  return hipGetLastError();
}

hipError_t launch_psum_batch(const RegDesc* regs, const int2* tblk, int n_tblk, const int* poff, const float4* ref4,
                             const float* lw, double* S, hipStream_t st) {
  if (n_tblk <= 0) return hipSuccess;
  hipLaunchKernelGGL(psum_batch_kernel, dim3((unsigned)n_tblk), dim3(PS_BT), 0, st, regs, tblk, poff, ref4, lw, S);
  return hipGetLastError();
}

hipError_t launch_pinv_batch(const RegDesc* regs_p, const int2* tblk, int n_tblk, const int* poff, const double* S,
                             const double* poses, const Derived* dvs, int t, bool wu, double* wpart, hipStream_t st) {
  if (n_tblk <= 0) return hipSuccess;
  const dim3 grid((unsigned)n_tblk), block(PS_BT);
  if (wu)
    hipLaunchKernelGGL(pinv_batch_kernel<true>, grid, block, 0, st, regs_p, tblk, poff, S, poses, dvs, t, wpart);
  else
    hipLaunchKernelGGL(pinv_batch_kernel<false>, grid, block, 0, st, regs_p, tblk, poff, S, poses, dvs, t, wpart);
  return hipGetLastError();
}

hipError_t launch_pinv(const float4* tm4, const float2* tmx, const double* S, int M, const double* pose,
                       const Derived* dv, int t, bool wu, double* wpart, hipStream_t st) {
  const dim3 grid((unsigned)pinv_blocks(M)), block(PS_BT);
  if (wu)
    hipLaunchKernelGGL(pinv_kernel<true>, grid, block, 0, st, tm4, tmx, S, M, pose, dv, t, wpart);
  else
    hipLaunchKernelGGL(pinv_kernel<false>, grid, block, 0, st, tm4, tmx, S, M, pose, dv, t, wpart);
  return hipGetLastError();
}

}  // namespace sgr
