// Mixed-precision form of the p = 1 shape-weighted force: the similarity-
// weighted sums over the reference are a matrix product and run on the
// matrix cores.
//
// For p = 1 the force needs, per template point i,
//   S_i = sum_j c_ij [1, x_j, y_j, z_j],   c_ij = exp2(lw_j - (b_i - b_j)^2),
// and f_i = kappa g'_i (y_i S_i[0] - S_i[1..3]).  Writing P = (c_ij) (M x N)
// and V = (1, x_hi, y_hi, z_hi, x_lo, y_lo, z_lo, 0) (N x 8, each coordinate
// split into a bf16 head and a bf16 tail), S = P V is a dense contraction
// over the long reference dimension.  The pair weights are formed on the
// FP32 VALU (one FMA and one exp2 per pair with the exponent expanded about
// the block's range of b, as in the FP32 kernel; one sub more otherwise),
// rounded to bf16 (round to nearest even, unbiased) and fed as the A operand of
// v_mfma_f32_16x16x32_bf16; V is the B operand; accumulation is FP32 per
// 256-point tile and FP64 across tiles.  Each wave owns 4 blocks of 16
// template rows and reuses each B fragment four times.
//
// Operand layout (16x16x32): lane l holds A[l % 16][8 (l / 16) + e] and
// B[8 (l / 16) + e][l % 16] for e = 0..7; the result D[4 (l / 16) + e][l % 16]
// for e = 0..3.
#include "common.h"
#include "launch.h"

namespace sgr {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int MX_BT = 256;  // 4 waves
constexpr int MX_RB = 4;    // row blocks of 16 per wave: 64 template points per wave
constexpr int MX_TJ = 256;  // reference points per LDS tile
constexpr int MX_PTS = MX_BT / 64 * MX_RB * 16;  // template points per block (256)

template <bool WF>
__global__ __launch_bounds__(MX_BT) void force_mixed_kernel(ForceArgs A) {
  __shared__ float2 s_bl[MX_TJ];           // (b_j, lw_j), or (d_j, lw_j - d_j^2) in the expanded form
  __shared__ __bf16 s_vt[16][MX_TJ];       // V transposed; rows 8..15 stay zero (unused B columns)
  __shared__ double s_T[MX_BT / 64][64][8];
  __shared__ double s_red[(MX_BT / 64) * 13];

  const int n_iblk = (A.M + MX_PTS - 1) / MX_PTS;
  const int iblk = blockIdx.x % n_iblk;
  const int chunk = blockIdx.x / n_iblk;
  const Derived& D = *A.dv;
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int i_wave = iblk * MX_PTS + w * 64;  // first template position of this wave
  const bool packed = A.tm4 != nullptr;
  // b of the template point at visiting position ip (< M)
  auto b_at = [&](int ip) -> float {
    return packed ? A.tm4[ip].w : (float)(((double)A.aY[ip] - D.abar) * D.bscale);
  };

#pragma unroll
  for (int r = 8; r < 16; ++r) s_vt[r][threadIdx.x] = (__bf16)0.0f;

  float bi[MX_RB];
  float lo = INFINITY, hi = -INFINITY;
#pragma unroll
  for (int rb = 0; rb < MX_RB; ++rb) {
    const int ip = i_wave + rb * 16 + (l & 15);
    bi[rb] = 0.f;
    if (ip < A.M) {
      bi[rb] = b_at(ip);
      lo = fminf(lo, bi[rb]);
      hi = fmaxf(hi, bi[rb]);
    }
  }
  // expanded exponent centred on the block's range of b (one FMA per weight)
  block_range<MX_BT>(lo, hi, s_red);
  float beta;
  const bool expd = expanded_centre(lo, hi, D, false, beta);
  float al[MX_RB];
#pragma unroll
  for (int rb = 0; rb < MX_RB; ++rb) al[rb] = 2.f * (bi[rb] - beta);

  double T[MX_RB][4];
#pragma unroll
  for (int rb = 0; rb < MX_RB; ++rb)
    for (int e = 0; e < 4; ++e) T[rb][e] = 0.0;

  const int col = l & 15, kq = 8 * (l >> 4);
  const int j0 = chunk * A.chunk_len;
  const int j1 = min(A.N, j0 + A.chunk_len);
  for (int base = j0; base < j1; base += MX_TJ) {
    __syncthreads();
    {
      const int t = threadIdx.x;
      const int j = base + t;
      float4 X = make_float4(0.f, 0.f, 0.f, 0.f);
      float lw = -INFINITY;  // beyond this chunk: zero weight
      if (j < j1) {
        X = A.ref4[j];
        lw = A.reflw[j];
      }
      if (expd) {
        // |d_j| capped so that 2 d_i d_j stays finite (weight 0 either way)
        float d = X.w - beta;
        if (fabsf(d) > 1e18f) d = copysignf(1e18f, d);
        s_bl[t] = make_float2(d, __builtin_fmaf(-d, d, lw));
      } else {
        s_bl[t] = make_float2(X.w, lw);
      }
      const __bf16 xh = (__bf16)X.x, yh = (__bf16)X.y, zh = (__bf16)X.z;
      s_vt[0][t] = (__bf16)1.0f;
      s_vt[1][t] = xh;
      s_vt[2][t] = yh;
      s_vt[3][t] = zh;
      s_vt[4][t] = (__bf16)(X.x - (float)xh);
      s_vt[5][t] = (__bf16)(X.y - (float)yh);
      s_vt[6][t] = (__bf16)(X.z - (float)zh);
      s_vt[7][t] = (__bf16)0.0f;
    }
    __syncthreads();
    f32x4 C[MX_RB];
#pragma unroll
    for (int rb = 0; rb < MX_RB; ++rb) C[rb] = f32x4{0.f, 0.f, 0.f, 0.f};
    if (expd) {
#pragma unroll 2
      for (int kb = 0; kb < MX_TJ; kb += 32) {
        const int jb = kb + kq;
        float2 bl[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) bl[e] = s_bl[jb + e];
        const bf16x8 bfrag = *reinterpret_cast<const bf16x8*>(&s_vt[col][jb]);
#pragma unroll
        for (int rb = 0; rb < MX_RB; ++rb) {
          bf16x8 afrag;
#pragma unroll
          for (int e = 0; e < 8; ++e)
            afrag[e] = (__bf16)__builtin_amdgcn_exp2f(__builtin_fmaf(al[rb], bl[e].x, bl[e].y));
          C[rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afrag, bfrag, C[rb], 0, 0, 0);
        }
      }
    } else {
#pragma unroll 2
      for (int kb = 0; kb < MX_TJ; kb += 32) {
        const int jb = kb + kq;
        float2 bl[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) bl[e] = s_bl[jb + e];
        const bf16x8 bfrag = *reinterpret_cast<const bf16x8*>(&s_vt[col][jb]);
#pragma unroll
        for (int rb = 0; rb < MX_RB; ++rb) {
          bf16x8 afrag;
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            const float db = bi[rb] - bl[e].x;
            afrag[e] = (__bf16)__builtin_amdgcn_exp2f(__builtin_fmaf(-db, db, bl[e].y));
          }
          C[rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afrag, bfrag, C[rb], 0, 0, 0);
        }
      }
    }
#pragma unroll
    for (int rb = 0; rb < MX_RB; ++rb)
      for (int e = 0; e < 4; ++e) T[rb][e] += (double)C[rb][e];
  }

  // Gather each template row's 8 column sums (they are spread over lanes).
  if (col < 8) {
#pragma unroll
    for (int rb = 0; rb < MX_RB; ++rb)
      for (int e = 0; e < 4; ++e) s_T[w][rb * 16 + 4 * (l >> 4) + e][col] = T[rb][e];
  }
  __syncthreads();

  // pose: y - xbar = sR (y0 - ybar0) + (sR ybar0 + t - xbar)
  double sR[9], cv[3];
  {
    const double s = A.pose[0];
#pragma unroll
    for (int e = 0; e < 9; ++e) sR[e] = s * A.pose[1 + e];
#pragma unroll
    for (int r = 0; r < 3; ++r)
      cv[r] = sR[3 * r] * D.ybar0[0] + sR[3 * r + 1] * D.ybar0[1] + sR[3 * r + 2] * D.ybar0[2] + A.pose[10 + r] -
              D.xbar[r];
  }
  const double G = A.G > 0 ? A.G : 0.1 * D.G1 + 0.9 * D.G1 / (1.0 + exp(-(((double)A.t - 1.0) - 0.5 * D.E)));
  const double coef = -(G / D.Z) * D.coefL;
  double wv[13];
#pragma unroll
  for (int e = 0; e < 13; ++e) wv[e] = 0.0;
  const int ip = i_wave + l;  // row l of this wave's 64: rb = l / 16, row = l % 16
  if (ip < A.M) {
    const double* S = s_T[w][l];
    float x0, y0, z0;
    double ai, mi;
    if (packed) {
      const float4 P4 = A.tm4[ip];
      const float2 PX = A.tmx[ip];
      x0 = P4.x;
      y0 = P4.y;
      z0 = P4.z;
      ai = (double)PX.x;
      mi = (double)PX.y;
    } else {
      x0 = A.y0x[ip];
      y0 = A.y0y[ip];
      z0 = A.y0z[ip];
      ai = (double)A.aY[ip];
      mi = A.mY ? (double)A.mY[ip] : 1.0;
    }
    const double ex = (double)x0 - D.ybar0[0], ey = (double)y0 - D.ybar0[1], ez = (double)z0 - D.ybar0[2];
    const double cx = sR[0] * ex + sR[1] * ey + sR[2] * ez;
    const double cy = sR[3] * ex + sR[4] * ey + sR[5] * ez;
    const double cz = sR[6] * ex + sR[7] * ey + sR[8] * ez;
    // the float32 point the FP32 path would use
    const double yx = (float)(cx + cv[0]), yy = (float)(cy + cv[1]), yz = (float)(cz + cv[2]);
    const double gi = (D.g_mode == 1.0) ? ai / D.abar : 1.0;
    double sc = 1.0;
    if (expd) {
      const double dl = (double)(b_at(ip) - beta);
      sc = exp2(-dl * dl);
    }
    const double k0 = coef * gi * sc;
    const double fx = k0 * (yx * S[0] - (S[1] + S[4]));
    const double fy = k0 * (yy * S[0] - (S[2] + S[5]));
    const double fz = k0 * (yz * S[0] - (S[3] + S[6]));
    wv[WR_F + 0] = mi * fx;
    wv[WR_F + 1] = mi * fy;
    wv[WR_F + 2] = mi * fz;
    wv[WR_K + 0] = fx * cx;
    wv[WR_K + 1] = fx * cy;
    wv[WR_K + 2] = fx * cz;
    wv[WR_K + 3] = fy * cx;
    wv[WR_K + 4] = fy * cy;
    wv[WR_K + 5] = fy * cz;
    wv[WR_K + 6] = fz * cx;
    wv[WR_K + 7] = fz * cy;
    wv[WR_K + 8] = fz * cz;
    if constexpr (WF) {
      double* fp = A.fpart + ((int64_t)chunk * A.M + ip) * 3;  // visiting order
      fp[0] = fx;
      fp[1] = fy;
      fp[2] = fz;
    }
  }
  block_sum<13, MX_BT>(wv, s_red);
  if (threadIdx.x == 0) {
    double* o = A.wpart + (int64_t)blockIdx.x * WR_STRIDE;
#pragma unroll
    for (int e = 0; e < 13; ++e) o[e] = wv[e];
  }
}

int mixed_points_per_block() { return MX_PTS; }

hipError_t launch_force_mixed(const ForceArgs& A, bool want_f, hipStream_t st) {
  const int n_iblk = (A.M + MX_PTS - 1) / MX_PTS;
  const dim3 grid(n_iblk * A.n_chunks);
  if (want_f)
    hipLaunchKernelGGL(force_mixed_kernel<true>, grid, dim3(MX_BT), 0, st, A);
  else
    hipLaunchKernelGGL(force_mixed_kernel<false>, grid, dim3(MX_BT), 0, st, A);
  return hipGetLastError();
}

}  // namespace sgr
