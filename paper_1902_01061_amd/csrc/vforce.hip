// Force with vector shape descriptors: eq. (3) with |a_i - a_j|^2 summed over
// D dimensions, p = 1 (h = 1), g = s, as a dense contraction on the matrix
// cores.
//
// With centred descriptors c = a - abar (abar the reference mean) and
// kappa = log2(e) / sigma^2, the exponent of a pair,
//   t_ij = lw_j - kappa |c_i - c_j|^2,
// is one dot product of augmented rows
//   At_i = [2 kappa c_i, -kappa |c_i|^2, 1, 0...],
//   Bt_j = [c_j, 1, lw_j - kappa |c_j|^2, 0...],
// (written below with the standardised c / sigma, so that every entry is of
// order one), and c_ij = exp2(At_i . Bt_j) for a 16 x 16 block of pairs
// comes from the matrix cores in one of two forms:
//  - split f16 (default): every entry is split into an f16 head and an f16
//    tail (x = h + l + O(2^-22 |x|)), and h.h + h.l + l.h gives the dot
//    product to about 2^-22 of the size of its terms.  The three products
//    are one contraction of length 3E (E = D + 2 entries per row): template
//    rows [h, h, l], reference rows [h, l, h], zero-padded to 32 NB halves,
//    NB = ceil(3E / 32) 16x16x32 f16 instructions with FP32 accumulation,
//    the last block (all tails) first: 2 instructions for D = 16;
//  - FP32: K/4 FP32 16x16x4 instructions, K = 4 ceil((D + 2) / 4); used when
//    an entry would leave the f16 range (a descriptor more than about 140
//    spreads from the mean) or when the caller asks for it.
// 16 exp2 then turn the block into pair weights.  The p = 1 moment form then
// needs, per template point, sum_j c, sum_j c x_j (and sum_j c |x_j|^2 for
// the energy) over the reference, accumulated in FP32 by the vector ALU.
//
// Far rows: the products lose accuracy as |c| grows (each entry carries a
// rounding of about 2^-24 of log2(e) |c|^2 in FP32, 2^-22 in split f16, and
// the exponent of a pair is their difference), so a template row whose
// standardised descriptor lies more than VF_FAR spreads from the mean is
// left out of the contraction (its exponent is set to the padding value)
// and evaluated after it instead, in FP64 from the standardised descriptors
// (vfar_pairs_kernel), with FP64 sums, the same epilogue and a wrench slot
// of its own (a far row beyond the reach of every reference descriptor has
// no weight above 2^-150 and is left at zero force: far_reachable).
//
// Work decomposition: a block of 256 threads (4 waves) owns 256 template
// points; wave w holds 4 row tiles of 16 points, their At rows resident in
// registers for the whole chunk.  Reference chunks of at most 2048 points
// (multiples of 64) stream through LDS 64 points at a time; each 16-column
// tile gives every lane 4 pairs per row tile (rows 4 (lane / 16) + v, column
// lane % 16).  A lane therefore sums at most 128 terms per quantity in FP32;
// the 16 lanes of a row are then added by shuffles and everything after that
// is FP64, as in the scalar kernel: per-point forces, the block's wrench
// partial in wpart[slot] (same layout, consumed by the same update kernel).
#include <algorithm>
#include <atomic>

#include "common.h"
#include "launch.h"

namespace sgr {

namespace {

constexpr int VF_BT = 256;   // threads
#ifndef SGR_VF_TI
#define SGR_VF_TI 4
#endif
#ifndef SGR_VF_WAVES
#define SGR_VF_WAVES 0
#endif
constexpr int VF_TI = SGR_VF_TI;  // 16-row tiles per wave
constexpr int VF_ROWS = 64 * VF_TI;  // template points per block
static_assert(VF_TI == 1 || VF_TI == 2 || VF_TI == 4, "row tiles per wave");
constexpr int VF_TJ = 64;    // reference points per LDS stage
constexpr double LOG2E = 1.4426950408889634;
constexpr double VF_FAR2 = 64.0;  // |c|^2 beyond which a template row is a far row (8 spreads)

// |c_r|^2 = |a_r - abar|^2 / sigma^2 of descriptor row r, in FP64 (the same
// expression decides far rows in vfar_list_kernel and vpack_kernel).
__device__ inline double std_norm2(const float* __restrict__ a, int64_t r, int D, const double* __restrict__ vd) {
  const double isig = 1.0 / vd[32];
  double n2 = 0.0;
  for (int c = 0; c < D; ++c) {
    const double e = ((double)a[r * D + c] - vd[c]) * isig;
    n2 += e * e;
  }
  return n2;
}

typedef float v4f __attribute__((ext_vector_type(4)));

// LDS row stride of the staged Bt: K words when K/4 is odd, else K + 4, so
// that the 64 lanes of one read (16 columns x 4 k) hit 64 distinct banks.
__host__ __device__ constexpr int bt_stride(int K) { return ((K / 4) & 1) ? K : K + 4; }

// abar, sigma and kappa of the vector descriptors; writes sigma into the
// Derived of the registration (its other fields come from the scalar
// set-up, called without curvatures).
__global__ __launch_bounds__(1024) void vprep_kernel(const float* __restrict__ aX, int64_t N,
                                                     const float* __restrict__ aY, int64_t M, int D, double sigma_in,
                                                     Derived* __restrict__ dv, double* __restrict__ vd) {
  __shared__ double lds[16 * 32];
  __shared__ double mean[32];
  __shared__ double sig_s;
  double s[32];
  for (int c = 0; c < 32; ++c) s[c] = 0.0;
  for (int64_t j = threadIdx.x; j < N; j += 1024) {
#pragma unroll
    for (int c = 0; c < 32; ++c)
      if (c < D) s[c] += (double)aX[j * D + c];
  }
  block_sum<32, 1024>(s, lds);
  if (threadIdx.x == 0)
    for (int c = 0; c < 32; ++c) mean[c] = c < D ? s[c] / (double)N : 0.0;
  __syncthreads();
  double v[1] = {0.0};
  for (int64_t j = threadIdx.x; j < N; j += 1024)
    for (int c = 0; c < D; ++c) {
      const double d = (double)aX[j * D + c] - mean[c];
      v[0] += d * d;
    }
  block_sum<1, 1024>(v, lds);
  if (threadIdx.x == 0) sig_s = sigma_in > 0 ? sigma_in : sqrt(v[0] / (double)N);
  __syncthreads();
  const double sigma = sig_s;
  // largest |a - abar|^2 / sigma^2 (NaN-propagating) over the reference
  // (mr), and over the reference and the template rows that enter the
  // contraction (mx: far rows do not): the host picks the f16 form only if
  // every augmented entry fits its range
  double mx = 0.0, mr = 0.0;
  for (int64_t r = threadIdx.x; r < N + M; r += 1024) {
    const float* a = r < N ? aX + r * D : aY + (r - N) * D;
    double n2 = 0.0;
    for (int c = 0; c < D; ++c) {
      const double e = ((double)a[c] - mean[c]) / sigma;
      n2 += e * e;
    }
    if (r < N) mr = (n2 > mr || n2 != n2) ? n2 : mr;
    if (r < N || !(n2 > VF_FAR2)) mx = (n2 > mx || n2 != n2) ? n2 : mx;
  }
  for (int off = 32; off > 0; off >>= 1) {
    const double o = __shfl_xor(mx, off, 64);
    mx = (o > mx || o != o) ? o : mx;
    const double q = __shfl_xor(mr, off, 64);
    mr = (q > mr || q != q) ? q : mr;
  }
  if ((threadIdx.x & 63) == 0) {
    lds[threadIdx.x >> 6] = mx;
    lds[16 + (threadIdx.x >> 6)] = mr;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  for (int w = 1; w < 16; ++w) {
    mx = (lds[w] > mx || lds[w] != lds[w]) ? lds[w] : mx;
    mr = (lds[16 + w] > mr || lds[16 + w] != lds[16 + w]) ? lds[16 + w] : mr;
  }
  for (int c = 0; c < 32; ++c) vd[c] = mean[c];
  vd[32] = sigma;
  vd[33] = LOG2E / (sigma * sigma);
  vd[34] = mx;
  vd[35] = mr;
  dv->sigma = sigma;
  if (!(sigma > 0) || !isfinite(vd[33])) dv->status |= ST_DEGENERATE;
}

// Augmented rows from the standardised descriptors c = (a - abar) / sigma:
//   At_i = [2 log2(e) c_i, -log2(e) |c_i|^2, 1, 0...],
//   Bt_j = [c_j, 1, lw_j - log2(e) |c_j|^2, 0...],
// FP64 arithmetic, then either rounded once to FP32 (K entries per row) or
// split into f16 head h and tail l and laid out as one contraction of length
// 3E (K = 32 ceil(3E / 32) halves per row, E = D + 2): template [h, h, l],
// reference [h, l, h].  Rows j >= N of the reference are zero-weight padding
// (exponent -30000: exp2 gives 0, and the value is an f16 head with zero
// tail); rows i >= M of the template are harmless padding (their sums are
// dropped).
__device__ inline void put_entry(void* row, int c, double x, bool half, int E, bool tmpl) {
  if (half) {
    _Float16* h = reinterpret_cast<_Float16*>(row);
    const _Float16 hi = (_Float16)x;
    const _Float16 lo = (_Float16)(x - (double)hi);
    h[c] = hi;
    h[E + c] = tmpl ? hi : lo;
    h[2 * E + c] = tmpl ? lo : hi;
  } else {
    reinterpret_cast<float*>(row)[c] = (float)x;
  }
}

__global__ __launch_bounds__(256) void vpack_kernel(const float* __restrict__ X, const float* __restrict__ Y,
                                                    const float* __restrict__ Zc, const float* __restrict__ aX,
                                                    const float* __restrict__ wX, int N, int Npad,
                                                    const float* __restrict__ aY, int M, int Mpad, int D, int K,
                                                    bool half, const Derived* __restrict__ dv,
                                                    const double* __restrict__ vd, void* __restrict__ Bt,
                                                    float4* __restrict__ ref4, void* __restrict__ At) {
  const int r = blockIdx.x * 256 + threadIdx.x;
  const double isig = 1.0 / vd[32];
  const int E = D + 2;  // entries per augmented row
  // exponent of zero-weight rows: exp2 of it is 0, and it is an f16 value
  // (the f16 form is only chosen when every other entry stays below 30000)
  const double pad_exp = half ? -30000.0 : -1e30;
  // K halves (split f16) or K floats per row
  const size_t rb = half ? (size_t)K * sizeof(_Float16) : (size_t)K * sizeof(float);
  if (r < Npad) {
    void* b = reinterpret_cast<char*>(Bt) + (size_t)r * rb;
    for (size_t w = 0; w < rb / 4; ++w) reinterpret_cast<uint32_t*>(b)[w] = 0u;
    if (r < N) {
      double n2 = 0.0;
      for (int c = 0; c < D; ++c) {
        const double e = ((double)aX[(int64_t)r * D + c] - vd[c]) * isig;
        put_entry(b, c, e, half, E, false);
        n2 += e * e;
      }
      const double lw = wX ? log2((double)wX[r]) : 0.0;
      put_entry(b, D, 1.0, half, E, false);
      put_entry(b, D + 1, fmax(lw - LOG2E * n2, pad_exp), half, E, false);
      const Derived& Dd = *dv;
      const float x = (float)((double)X[r] - Dd.xbar[0]), y = (float)((double)Y[r] - Dd.xbar[1]),
                  z = (float)((double)Zc[r] - Dd.xbar[2]);
      ref4[r] = make_float4(x, y, z, (float)((double)x * x + (double)y * y + (double)z * z));
    } else {
      put_entry(b, D, 1.0, half, E, false);
      put_entry(b, D + 1, pad_exp, half, E, false);
      ref4[r] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
  }
  if (r < Mpad) {
    void* a = reinterpret_cast<char*>(At) + (size_t)r * rb;
    for (size_t w = 0; w < rb / 4; ++w) reinterpret_cast<uint32_t*>(a)[w] = 0u;
    if (r < M && std_norm2(aY, r, D, vd) > VF_FAR2) {
      // far row (vfar_kernel): every pair exponent is the padding value
      put_entry(a, D, pad_exp, half, E, true);
      put_entry(a, D + 1, 0.0, half, E, true);
    } else {
      if (r < M) {
        double n2 = 0.0;
        for (int c = 0; c < D; ++c) {
          const double e = ((double)aY[(int64_t)r * D + c] - vd[c]) * isig;
          put_entry(a, c, 2.0 * LOG2E * e, half, E, true);
          n2 += e * e;
        }
        put_entry(a, D, -LOG2E * n2, half, E, true);
      }
      put_entry(a, D + 1, 1.0, half, E, true);
    }
  }
}

__device__ inline double G_of(const Derived& D, int t) {
  return 0.1 * D.G1 + 0.9 * D.G1 / (1.0 + exp(-(((double)t - 1.0) - 0.5 * D.E)));
}

typedef _Float16 v8h __attribute__((ext_vector_type(8)));

// H = false: FP32 rows of K = 4 VK entries, K/4 16x16x4 FP32 instructions.
// H = true: split-f16 rows of K = 32 VK halves, VK 16x16x32 f16
// instructions.  Lane layouts (checked on the device): 16x16x4 f32 takes
// A[i = lane % 16][k = lane / 16] and B[k = lane / 16][j = lane % 16];
// 16x16x32 f16 takes A[i = lane % 16][k = 8 (lane / 16) + e] and
// B[k = 8 (lane / 16) + e][j = lane % 16], e = 0..7; both return
// D[i = 4 (lane / 16) + v][j = lane % 16], v = 0..3.
template <int VK, bool H, bool WU, bool WF>
__global__ __launch_bounds__(VF_BT)
#if SGR_VF_WAVES > 0
__attribute__((amdgpu_waves_per_eu(SGR_VF_WAVES, SGR_VF_WAVES)))
#endif
void vforce_kernel(VForceArgs A) {
  constexpr int K = H ? 32 * VK : 4 * VK;  // halves (H) or floats per row
  constexpr int RW = H ? 16 * VK : K;       // 4-byte words per row
  // LDS words per staged reference row: FP32 rows use bt_stride(K); f16 rows
  // (16 VK words) get 4 more, so that the 16-byte reads of one instruction
  // (16 rows x 4 quarter-blocks) start on 64 distinct banks
  constexpr int KS = H ? RW + 4 : bt_stride(K);
  constexpr int NQ = WU ? 5 : 4;
  constexpr int LDS_B = VF_TJ * KS > NQ * VF_ROWS ? VF_TJ * KS : NQ * VF_ROWS;  // tile, then the row sums
  __shared__ __attribute__((aligned(16))) float s_B[LDS_B];
  __shared__ float4 s_X[VF_TJ];
  __shared__ double s_red[(VF_BT / 64) * 13];
  const int n_iblk = (A.M + VF_ROWS - 1) / VF_ROWS;
  const int iblk = blockIdx.x % n_iblk, chunk = blockIdx.x / n_iblk;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int col = lane & 15, kq = lane >> 4;
  const int row0 = iblk * VF_ROWS + w * 16 * VF_TI;
  // chunk bounds in units of VF_TJ
  const int n_t = (A.N + VF_TJ - 1) / VF_TJ;
  const int j0 = (int)((int64_t)chunk * n_t / A.n_chunks) * VF_TJ;
  const int j1 = (int)((int64_t)(chunk + 1) * n_t / A.n_chunks) * VF_TJ;

  float areg[VF_TI][H ? 1 : VK];
  v8h ah[H ? VF_TI : 1][H ? VK : 1];
  if constexpr (H) {
    const _Float16* At = reinterpret_cast<const _Float16*>(A.At);
#pragma unroll
    for (int r = 0; r < VF_TI; ++r) {
      const _Float16* row = At + (int64_t)(row0 + 16 * r + col) * K;
#pragma unroll
      for (int k = 0; k < VK; ++k) ah[r][k] = *reinterpret_cast<const v8h*>(row + 32 * k + 8 * kq);
    }
  } else {
    const float* At = reinterpret_cast<const float*>(A.At);
#pragma unroll
    for (int r = 0; r < VF_TI; ++r)
#pragma unroll
      for (int s = 0; s < VK; ++s) areg[r][s] = At[(int64_t)(row0 + 16 * r + col) * K + 4 * s + kq];
  }
  float S[VF_TI][4][NQ];
#pragma unroll
  for (int r = 0; r < VF_TI; ++r)
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int q = 0; q < NQ; ++q) S[r][v][q] = 0.f;

  for (int base = j0; base < j1; base += VF_TJ) {
    __syncthreads();
    {
      const float* Bt = reinterpret_cast<const float*>(A.Bt);
      for (int e = threadIdx.x; e < VF_TJ * (RW / 4); e += VF_BT) {
        const int jj = e / (RW / 4), s = e % (RW / 4);
        const float4 b4 = *reinterpret_cast<const float4*>(Bt + (int64_t)(base + jj) * RW + 4 * s);
        *reinterpret_cast<float4*>(&s_B[jj * KS + 4 * s]) = b4;
      }
    }
    if (threadIdx.x < VF_TJ) s_X[threadIdx.x] = A.ref4[base + threadIdx.x];
    __syncthreads();
#pragma unroll 1
    for (int c = 0; c < VF_TJ / 16; ++c) {
      const int jl = 16 * c + col;
      float breg[H ? 1 : VK];
      v8h bh[H ? VK : 1];
      if constexpr (H) {
#pragma unroll
        for (int k = 0; k < VK; ++k) bh[k] = *reinterpret_cast<const v8h*>(&s_B[jl * KS + 16 * k + 4 * kq]);
      } else {
#pragma unroll
        for (int s = 0; s < VK; ++s) breg[s] = s_B[jl * KS + 4 * s + kq];
      }
      const float4 X = s_X[jl];
#pragma unroll
      for (int r = 0; r < VF_TI; ++r) {
        v4f acc = {0.f, 0.f, 0.f, 0.f};
        if constexpr (H) {
          // the last block first: it holds only tail products, the first
          // holds the head products, so small terms are added before large
#pragma unroll
          for (int k = VK - 1; k >= 0; --k) acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[r][k], bh[k], acc, 0, 0, 0);
        } else {
#pragma unroll
          for (int s = 0; s < VK; ++s)
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(areg[r][s], breg[s], acc, 0, 0, 0);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const float cc = __builtin_amdgcn_exp2f(acc[v]);
          S[r][v][0] += cc;
          S[r][v][1] = __builtin_fmaf(cc, X.x, S[r][v][1]);
          S[r][v][2] = __builtin_fmaf(cc, X.y, S[r][v][2]);
          S[r][v][3] = __builtin_fmaf(cc, X.z, S[r][v][3]);
          if constexpr (WU) S[r][v][4] = __builtin_fmaf(cc, X.w, S[r][v][4]);
        }
      }
    }
  }
  // sums over the 16 columns (lanes of equal lane / 16); lane col < 4 then
  // parks row 4 kq + col of each row tile in LDS, where thread t picks up
  // row t of the block, so that the FP64 epilogue holds one row's sums
#pragma unroll
  for (int r = 0; r < VF_TI; ++r)
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        float x = S[r][v][q];
#pragma unroll
        for (int off = 1; off < 16; off <<= 1) x += __shfl_xor(x, off, 64);
        S[r][v][q] = x;
      }
  __syncthreads();  // every wave is done with s_B: reuse it for the sums
  float* s_S = s_B;
  if (col < 4) {
#pragma unroll
    for (int r = 0; r < VF_TI; ++r)
#pragma unroll
      for (int q = 0; q < NQ; ++q)
        s_S[q * VF_ROWS + w * 16 * VF_TI + 16 * r + 4 * kq + col] =
            col == 0 ? S[r][0][q] : col == 1 ? S[r][1][q] : col == 2 ? S[r][2][q] : S[r][3][q];
  }
  __syncthreads();

  const Derived& D = *A.dv;
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
  const double G = A.G > 0 ? A.G : G_of(D, A.t);
  const double coef = -(G / D.Z);
  const double ucoef = 0.5 * (G / D.Z);
  double wr[13];
#pragma unroll
  for (int e = 0; e < 13; ++e) wr[e] = 0.0;
  // thread t < VF_ROWS finishes template point iblk * VF_ROWS + t
  {
    const int ip = iblk * VF_ROWS + threadIdx.x;
    if (threadIdx.x >= VF_ROWS || ip >= A.M) goto done;
    double t[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) t[q] = (double)s_S[q * VF_ROWS + threadIdx.x];
    if constexpr (WU) {
      if (A.spart) {
        // the sums themselves (pose-independent for p = 1): sum_j c, sum_j c x_j
        // (3), sum_j c |x_j|^2 of this chunk
        double* o = A.spart + ((int64_t)chunk * A.M + ip) * 5;
#pragma unroll
        for (int q = 0; q < 5; ++q) o[q] = t[q];
        goto done;
      }
    }
    const double ex = (double)A.y0x[ip] - D.ybar0[0], ey = (double)A.y0y[ip] - D.ybar0[1],
                 ez = (double)A.y0z[ip] - D.ybar0[2];
    const float pxf = (float)(sR[0] * ex + sR[1] * ey + sR[2] * ez + cv[0]);
    const float pyf = (float)(sR[3] * ex + sR[4] * ey + sR[5] * ez + cv[1]);
    const float pzf = (float)(sR[6] * ex + sR[7] * ey + sR[8] * ez + cv[2]);
    const double px = pxf, py = pyf, pz = pzf;
    const double tx = px * t[0] - t[1], ty = py * t[0] - t[2], tz = pz * t[0] - t[3];
    const double mi = A.mY ? (double)A.mY[ip] : 1.0;
    const double fx = coef * tx, fy = coef * ty, fz = coef * tz;
    const double cx = px - cv[0], cy = py - cv[1], cz = pz - cv[2];
    wr[WR_F + 0] += mi * fx;
    wr[WR_F + 1] += mi * fy;
    wr[WR_F + 2] += mi * fz;
    wr[WR_K + 0] += fx * cx;
    wr[WR_K + 1] += fx * cy;
    wr[WR_K + 2] += fx * cz;
    wr[WR_K + 3] += fy * cx;
    wr[WR_K + 4] += fy * cy;
    wr[WR_K + 5] += fy * cz;
    wr[WR_K + 6] += fz * cx;
    wr[WR_K + 7] += fz * cy;
    wr[WR_K + 8] += fz * cz;
    if constexpr (WU)
      wr[WR_U] += ucoef * ((px * px + py * py + pz * pz + D.eps2) * t[0] - 2.0 * (px * t[1] + py * t[2] + pz * t[3]) +
                           t[4]);
    if constexpr (WF) {
      double* fp = A.fpart + ((int64_t)chunk * A.M + ip) * 3;
      fp[0] = fx;
      fp[1] = fy;
      fp[2] = fz;
    }
  }
done:
  block_sum<13, VF_BT>(wr, s_red);
  if (threadIdx.x == 0) {
    double* o = A.wpart + (int64_t)blockIdx.x * WR_STRIDE;
#pragma unroll
    for (int e = 0; e < 13; ++e) o[e] = wr[e];
  }
}

// A far row whose standardised distance from every reference descriptor is
// at least |c_i| - max_j |c_j| (triangle inequality) has no pair weight above
// 2^(lw_max - log2(e) (|c_i| - max_j |c_j|)^2); when that is below 2^-150 its
// force is zero in FP32 and far below any other row's, and it needs no
// evaluation (the contraction already gives it zero weight).
__device__ inline bool far_reachable(double n2, const double* __restrict__ vd, const Derived* __restrict__ dv) {
  const double gap = sqrt(n2) - sqrt(vd[35]);
  return !(gap > 0.0 && gap * gap * LOG2E > dv->lw_max + 150.0);
}

// The far rows that can carry a force, in increasing order: far_idx[0..n)
// and n in far_idx[M].  One block; thread t scans a contiguous range of rows,
// so that an exclusive scan of the per-thread counts places every index
// deterministically.
__global__ __launch_bounds__(1024) void vfar_list_kernel(const float* __restrict__ aY, int M, int D,
                                                         const double* __restrict__ vd,
                                                         const Derived* __restrict__ dv, int* __restrict__ far_idx) {
  __shared__ int cnt[1024];
  const int per = (M + 1023) / 1024;
  const int r0 = min(M, (int)threadIdx.x * per), r1 = min(M, r0 + per);
  auto is_far = [&](int r) {
    const double n2 = std_norm2(aY, r, D, vd);
    return n2 > VF_FAR2 && far_reachable(n2, vd, dv);
  };
  int c = 0;
  for (int r = r0; r < r1; ++r) c += is_far(r);
  cnt[threadIdx.x] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    int acc = 0;
    for (int t = 0; t < 1024; ++t) {
      const int v = cnt[t];
      cnt[t] = acc;
      acc += v;
    }
    far_idx[M] = acc;
  }
  __syncthreads();
  int o = cnt[threadIdx.x];
  for (int r = r0; r < r1; ++r)
    if (is_far(r)) far_idx[o++] = r;
}

// Far-row evaluation.  The pair exponent t_ij = lw_j - log2(e) |c_i - c_j|^2
// is formed in FP64 from the standardised descriptors themselves,
//   t_ij = b_j - n_i + w_i . c_j,  b_j = lw_j - log2(e) |c_j|^2,
//   w_i = 2 log2(e) c_i,  n_i = log2(e) |c_i|^2,
// whose terms carry a rounding of 2^-53 of their size (the contraction's
// 2^-22 or 2^-24 is what made these rows far); the pair weight is then
// exp2 of t rounded to FP32, as in the contraction, and the moment sums are
// FP64.  Work: a block takes a tile of 64 far rows and a segment of the
// reference, staged through LDS VFAR_CH records at a time; a lane holds the
// w_i of RPL rows in registers and meets one reference record per step
// (RPL pairs), the Q = RPL lanes of a row group taking consecutive records.

constexpr int VFAR_CH = 256;      // reference records staged per chunk
constexpr int VFAR_BLOCKS = 2048;  // pair blocks aimed at (tiles x segments)

// Reference record of the far-row evaluation, vfar_stride(D) doubles: c_j
// zero-padded to vfar_db(D) entries, b_j, x, y, z, |x|^2 of ref4, and a
// zero (an even stride whose LDS copies of 4 consecutive records start in
// distinct bank groups); vfar_pad_refs(N) records, those past N of zero
// weight.
__global__ __launch_bounds__(256) void vfar_ref_kernel(const float* __restrict__ aX, const float* __restrict__ wX,
                                                       int N, int D, const double* __restrict__ vd,
                                                       const float4* __restrict__ ref4, double* __restrict__ refd) {
  const int j = blockIdx.x * 256 + threadIdx.x;  // < vfar_pad_refs(N)
  const int DB = vfar_db(D), RS = vfar_stride(D);
  double* r = refd + (int64_t)j * RS;
  if (j >= N) {  // padding: zero weight (exp2 of -1e300 in FP32 is 0)
    for (int c = 0; c < RS; ++c) r[c] = c == DB ? -1e300 : 0.0;
    return;
  }
  const double isig = 1.0 / vd[32];
  double n2 = 0.0;
  for (int c = 0; c < DB; ++c) {
    const double e = c < D ? ((double)aX[(int64_t)j * D + c] - vd[c]) * isig : 0.0;
    r[c] = e;
    n2 += e * e;
  }
  r[DB] = (wX ? log2((double)wX[j]) : 0.0) - LOG2E * n2;
  const float4 X = ref4[j];
  r[DB + 1] = X.x;
  r[DB + 2] = X.y;
  r[DB + 3] = X.z;
  r[DB + 4] = X.w;
  r[DB + 5] = 0.0;
}

// Segments of the reference: one round of pair blocks (bpc resident blocks
// per compute unit, from the kernel's register and LDS budget), whole
// chunks each, so that a block's start-up latency is paid once and its
// chunks stream through the LDS; at most max(VFAR_BLOCKS, row tiles)
// blocks, so part holds at most that many x 320 doubles.
struct VfarGrid {
  int n_rt, n_seg, cps;  // row tiles, segments, chunks per segment
};
inline VfarGrid vfar_grid(int n_far, int N, int slots) {
  VfarGrid g;
  g.n_rt = (n_far + 63) / 64;
  const int n_ch = std::max(1, (N + VFAR_CH - 1) / VFAR_CH);
  slots = std::max(1, std::min(VFAR_BLOCKS, slots));
  const int s = std::max(1, std::min(n_ch, slots / g.n_rt));
  g.cps = (n_ch + s - 1) / s;
  g.n_seg = (n_ch + g.cps - 1) / g.cps;
  return g;
}

// One staged chunk: NG granules of 16 bytes per thread of a block of 256
// (a clang vector type, which stays in registers).
typedef double v2d __attribute__((ext_vector_type(2)));
template <int NG>
__device__ __forceinline__ void vfar_fetch(v2d (&buf)[NG], const double* __restrict__ refd, int ch) {
  const v2d* src = reinterpret_cast<const v2d*>(refd + (int64_t)ch * VFAR_CH * (2 * NG));
#pragma unroll
  for (int i = 0; i < NG; ++i) buf[i] = src[threadIdx.x + 256 * i];
}
template <int NG>
__device__ __forceinline__ void vfar_store(const v2d (&buf)[NG], double* lds) {
#pragma unroll
  for (int i = 0; i < NG; ++i) reinterpret_cast<v2d*>(lds)[threadIdx.x + 256 * i] = buf[i];
}

// Block (row tile rt, segment sg): 64 far rows 64 rt + g + G rr (row group
// g = lane % G, rr < RPL) against the chunks [cps sg, cps (sg + 1)); wave w
// takes records [w CH/4, (w + 1) CH/4) of a staged chunk, lane q = lane / G
// of a row group every Q-th of them.  Sums: over the records of a lane, over
// q (a butterfly), then over the 4 waves in order, into
// part[(sg * 5 + e) * 64 n_rt + row].
template <int DB, bool WU, bool PF>
__global__ __launch_bounds__(256) void vfar_pairs_kernel(const double* __restrict__ refd, int N, int cps,
                                                         const float* __restrict__ aY, int D,
                                                         const double* __restrict__ vd,
                                                         const int* __restrict__ far_idx, int n_far,
                                                         double* __restrict__ part) {
  constexpr int RS = DB + 6, RPL = DB <= 16 ? 4 : 2, G = 64 / RPL, Q = RPL, CW = VFAR_CH / 4;
  constexpr int NS = WU ? 5 : 4;  // sums: c, c x, c y, c z (and c |x|^2 for the energy)
  static_assert(VFAR_CH == 256, "one staged record per thread");
  static_assert(VFAR_CH * RS >= 4 * 64 * 5, "LDS also holds the wave sums");
  constexpr int NG = RS / 2;  // 16-byte granules of a chunk per thread
  // PF: two LDS buffers; chunk ch + 1 is requested before chunk ch is used
  // and lands in registers meanwhile (otherwise it is requested after)
  __shared__ __align__(16) double lds[(PF ? 2 : 1) * VFAR_CH * RS];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane % G, q = lane / G;
  const int64_t nfp = (int64_t)gridDim.x * 64;
  const int n_ch = (N + VFAR_CH - 1) / VFAR_CH;
  const int c0 = (int)blockIdx.y * cps, c1 = min(n_ch, c0 + cps);
  // the far-row indices, then the first chunk, then the rows' descriptors
  // are requested, so that the staging overlaps the row set-up
  int ip[RPL];
#pragma unroll
  for (int rr = 0; rr < RPL; ++rr) {
    const int k = (int)blockIdx.x * 64 + g + G * rr;
    ip[rr] = far_idx[k < n_far ? k : n_far - 1];
  }
  v2d b0[NG];
  if (c0 < c1) vfar_fetch(b0, refd, c0);
  const double isig = 1.0 / vd[32];
  double wi[RPL][DB], ni[RPL];
#pragma unroll
  for (int rr = 0; rr < RPL; ++rr) {
    double n2 = 0.0;
#pragma unroll
    for (int c = 0; c < DB; ++c) {
      const double e = c < D ? ((double)aY[(int64_t)ip[rr] * D + c] - vd[c]) * isig : 0.0;
      wi[rr][c] = 2.0 * LOG2E * e;
      n2 += e * e;
    }
    ni[rr] = LOG2E * n2;
  }
  if (c0 < c1) vfar_store(b0, lds);
  double s[RPL][5];
#pragma unroll
  for (int rr = 0; rr < RPL; ++rr)
#pragma unroll
    for (int e = 0; e < 5; ++e) s[rr][e] = 0.0;
  for (int ch = c0; ch < c1; ++ch) {
    double* cur = lds + (PF ? ((ch - c0) & 1) * VFAR_CH * RS : 0);
    v2d b[NG];
    if constexpr (PF) {
      __syncthreads();  // chunk ch is staged, the buffer of ch + 1 is free
      if (ch + 1 < c1) vfar_fetch(b, refd, ch + 1);
    } else {
      if (ch > c0) {
        vfar_fetch(b, refd, ch);
        __syncthreads();  // the previous chunk is consumed
        vfar_store(b, cur);
      }
      __syncthreads();
    }
#pragma unroll 2
    for (int st = 0; st < CW / Q; ++st) {
      const v2d* r = reinterpret_cast<const v2d*>(cur + (wave * CW + st * Q + q) * RS);
      double v[DB + 6];
#pragma unroll
      for (int c = 0; c < (DB + 6) / 2; ++c) {
        const v2d x = r[c];
        v[2 * c] = x.x;
        v[2 * c + 1] = x.y;
      }
#pragma unroll
      for (int rr = 0; rr < RPL; ++rr) {
        double t = v[DB] - ni[rr];
#pragma unroll
        for (int c = 0; c < DB; ++c) t = fma(wi[rr][c], v[c], t);
        const double cw = (double)__builtin_amdgcn_exp2f((float)t);
        s[rr][0] += cw;
#pragma unroll
        for (int e = 1; e < NS; ++e) s[rr][e] = fma(cw, v[DB + e], s[rr][e]);
      }
    }
    if constexpr (PF) {
      if (ch + 1 < c1) vfar_store(b, lds + ((ch + 1 - c0) & 1) * VFAR_CH * RS);
    }
  }
#pragma unroll
  for (int rr = 0; rr < RPL; ++rr)
#pragma unroll
    for (int e = 0; e < 5; ++e)
#pragma unroll
      for (int off = G; off < 64; off <<= 1) s[rr][e] += __shfl_xor(s[rr][e], off, 64);
  __syncthreads();  // LDS now holds the wave sums [wave][row][e]
  if (q == 0) {
#pragma unroll
    for (int rr = 0; rr < RPL; ++rr)
#pragma unroll
      for (int e = 0; e < 5; ++e) lds[(wave * 64 + g + G * rr) * 5 + e] = s[rr][e];
  }
  __syncthreads();
  if (threadIdx.x < 64) {
    const int k = (int)blockIdx.x * 64 + threadIdx.x;
    if (k < n_far) {
      const int t = threadIdx.x;
#pragma unroll
      for (int e = 0; e < 5; ++e)
        part[((int64_t)blockIdx.y * 5 + e) * nfp + k] =
            ((lds[t * 5 + e] + lds[(64 + t) * 5 + e]) + lds[(128 + t) * 5 + e]) + lds[(192 + t) * 5 + e];
    }
  }
}

// One block per tile of 64 far rows: wave w adds the segments w, w + 4, ...
// of a row in order, the 4 waves' sums are added in order, then lane l of
// wave 0 runs the epilogue of vforce_kernel for far row k = 64 tile + l
// (template point far_idx[k]); the wrench partial goes to slot slot0 + k,
// the per-point force (WF) and the pair sums (WU with spart) to chunk 0
// (vforce_kernel wrote zeros for this row in every chunk).
template <bool WU, bool WF>
__global__ __launch_bounds__(256) void vfar_epi_kernel(VForceArgs A, const int* __restrict__ far_idx, int n_far,
                                                       int n_seg, const double* __restrict__ part, int slot0) {
  __shared__ double red[4][5][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int k = (int)blockIdx.x * 64 + lane;
  const int64_t nfp = (int64_t)gridDim.x * 64;
  double sums[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (k < n_far) {
#pragma unroll 4
    for (int sg = wave; sg < n_seg; sg += 4) {
#pragma unroll
      for (int q = 0; q < 5; ++q) sums[q] += part[((int64_t)sg * 5 + q) * nfp + k];
    }
  }
#pragma unroll
  for (int q = 0; q < 5; ++q) red[wave][q][lane] = sums[q];
  __syncthreads();
  if (wave != 0 || k >= n_far) return;
#pragma unroll
  for (int q = 0; q < 5; ++q) sums[q] = ((red[0][q][lane] + red[1][q][lane]) + red[2][q][lane]) + red[3][q][lane];
  const int ip = far_idx[k];
  double wr[13];
#pragma unroll
  for (int e = 0; e < 13; ++e) wr[e] = 0.0;
  const Derived& D_ = *A.dv;
  bool sums_only = false;
  if constexpr (WU) {
    if (A.spart) {
      double* o = A.spart + (int64_t)ip * 5;  // chunk 0
#pragma unroll
      for (int q = 0; q < 5; ++q) o[q] = sums[q];
      sums_only = true;
    }
  }
  if (!sums_only) {
    double sR[9], cv[3];
    const double s = A.pose[0];
#pragma unroll
    for (int e = 0; e < 9; ++e) sR[e] = s * A.pose[1 + e];
#pragma unroll
    for (int r = 0; r < 3; ++r)
      cv[r] = sR[3 * r] * D_.ybar0[0] + sR[3 * r + 1] * D_.ybar0[1] + sR[3 * r + 2] * D_.ybar0[2] + A.pose[10 + r] -
              D_.xbar[r];
    const double G = A.G > 0 ? A.G : G_of(D_, A.t);
    const double coef = -(G / D_.Z);
    const double ucoef = 0.5 * (G / D_.Z);
    const double ex = (double)A.y0x[ip] - D_.ybar0[0], ey = (double)A.y0y[ip] - D_.ybar0[1],
                 ez = (double)A.y0z[ip] - D_.ybar0[2];
    const double px = (float)(sR[0] * ex + sR[1] * ey + sR[2] * ez + cv[0]);
    const double py = (float)(sR[3] * ex + sR[4] * ey + sR[5] * ez + cv[1]);
    const double pz = (float)(sR[6] * ex + sR[7] * ey + sR[8] * ez + cv[2]);
    const double tx = px * sums[0] - sums[1], ty = py * sums[0] - sums[2], tz = pz * sums[0] - sums[3];
    const double mi = A.mY ? (double)A.mY[ip] : 1.0;
    const double fx = coef * tx, fy = coef * ty, fz = coef * tz;
    const double cx = px - cv[0], cy = py - cv[1], cz = pz - cv[2];
    wr[WR_F + 0] = mi * fx;
    wr[WR_F + 1] = mi * fy;
    wr[WR_F + 2] = mi * fz;
    wr[WR_K + 0] = fx * cx;
    wr[WR_K + 1] = fx * cy;
    wr[WR_K + 2] = fx * cz;
    wr[WR_K + 3] = fy * cx;
    wr[WR_K + 4] = fy * cy;
    wr[WR_K + 5] = fy * cz;
    wr[WR_K + 6] = fz * cx;
    wr[WR_K + 7] = fz * cy;
    wr[WR_K + 8] = fz * cz;
    if constexpr (WU)
      wr[WR_U] = ucoef * ((px * px + py * py + pz * pz + D_.eps2) * sums[0] -
                          2.0 * (px * sums[1] + py * sums[2] + pz * sums[3]) + sums[4]);
    if constexpr (WF) {
      double* fp = A.fpart + (int64_t)ip * 3;  // chunk 0
      fp[0] = fx;
      fp[1] = fy;
      fp[2] = fz;
    }
  }
  double* o = A.wpart + (int64_t)(slot0 + k) * WR_STRIDE;
#pragma unroll
  for (int e = 0; e < 13; ++e) o[e] = wr[e];
}

template <int VK, bool H>
hipError_t launch_vk(const VForceArgs& A, bool wu, bool wf, hipStream_t st) {
  const int n_iblk = (A.M + VF_ROWS - 1) / VF_ROWS;
  const dim3 grid((unsigned)(n_iblk * A.n_chunks)), block(VF_BT);
  if (wu && wf)
    hipLaunchKernelGGL((vforce_kernel<VK, H, true, true>), grid, block, 0, st, A);
  else if (wu)
    hipLaunchKernelGGL((vforce_kernel<VK, H, true, false>), grid, block, 0, st, A);
  else if (wf)
    hipLaunchKernelGGL((vforce_kernel<VK, H, false, true>), grid, block, 0, st, A);
  else
    hipLaunchKernelGGL((vforce_kernel<VK, H, false, false>), grid, block, 0, st, A);
  return hipGetLastError();
}

}  // namespace

int vforce_K(int D) { return 4 * ((D + 2 + 3) / 4); }
int vforce_half_K(int D) { return 32 * ((3 * (D + 2) + 31) / 32); }
int vforce_pad_rows(int M) { return (M + VF_ROWS - 1) / VF_ROWS * VF_ROWS; }
int vforce_pad_refs(int N) { return (N + VF_TJ - 1) / VF_TJ * VF_TJ; }
int vforce_n_iblk(int M) { return (M + VF_ROWS - 1) / VF_ROWS; }

// Chunks: at most 2048 reference points each (so that a lane sums at most 128
// terms in FP32), and enough blocks for about two per compute unit.
int vforce_chunks(int M, int N, int n_cu) {
  const int n_t = (N + VF_TJ - 1) / VF_TJ;
  const int nib = vforce_n_iblk(M);
  int nc = std::max((n_t + 31) / 32, (2 * n_cu + nib - 1) / nib);
  return std::max(1, std::min(nc, n_t));
}

hipError_t launch_vprep(const float* aX, int64_t N, const float* aY, int64_t M, int D, double sigma, Derived* dv,
                        double* vd, hipStream_t st) {
  hipLaunchKernelGGL(vprep_kernel, dim3(1), dim3(1024), 0, st, aX, N, aY, M, D, sigma, dv, vd);
  return hipGetLastError();
}

hipError_t launch_vpack(const float* X, const float* Y, const float* Z, const float* aX, const float* wX, int N,
                        const float* aY, int M, int D, bool half, const Derived* dv, const double* vd, void* Bt,
                        float4* ref4, void* At, hipStream_t st) {
  const int Npad = vforce_pad_refs(N), Mpad = vforce_pad_rows(M), K = half ? vforce_half_K(D) : vforce_K(D);
  const int rows = std::max(Npad, Mpad);
  hipLaunchKernelGGL(vpack_kernel, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, st, X, Y, Z, aX, wX, N, Npad,
                     aY, M, Mpad, D, K, half, dv, vd, Bt, ref4, At);
  return hipGetLastError();
}

hipError_t launch_vforce(const VForceArgs& A, bool wu, bool wf, hipStream_t st) {
  if (A.half) {
    switch (A.K / 32) {
      case 1: return launch_vk<1, true>(A, wu, wf, st);
      case 2: return launch_vk<2, true>(A, wu, wf, st);
      case 3: return launch_vk<3, true>(A, wu, wf, st);
      default: return hipErrorInvalidValue;
    }
  }
  switch (A.K / 4) {
    case 1: return launch_vk<1, false>(A, wu, wf, st);
    case 2: return launch_vk<2, false>(A, wu, wf, st);
    case 3: return launch_vk<3, false>(A, wu, wf, st);
    case 4: return launch_vk<4, false>(A, wu, wf, st);
    case 5: return launch_vk<5, false>(A, wu, wf, st);
    case 6: return launch_vk<6, false>(A, wu, wf, st);
    case 7: return launch_vk<7, false>(A, wu, wf, st);
    case 8: return launch_vk<8, false>(A, wu, wf, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_vfar_list(const float* aY, int M, int D, const double* vd, const Derived* dv, int* far_idx,
                            hipStream_t st) {
  hipLaunchKernelGGL(vfar_list_kernel, dim3(1), dim3(1024), 0, st, aY, M, D, vd, dv, far_idx);
  return hipGetLastError();
}

size_t vfar_part_doubles(int M) { return (size_t)std::max(VFAR_BLOCKS, (M + 63) / 64) * 64 * 5; }
int vfar_pad_refs(int N) { return (N + VFAR_CH - 1) / VFAR_CH * VFAR_CH; }

hipError_t launch_vfar_ref(const float* aX, const float* wX, int N, int D, const double* vd, const float4* ref4,
                           double* refd, hipStream_t st) {
  const int n = vfar_pad_refs(N);
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(vfar_ref_kernel, dim3((unsigned)(n / 256)), dim3(256), 0, st, aX, wX, N, D, vd, ref4, refd);
  return hipGetLastError();
}

// Resident blocks per compute unit of a pair kernel (from its register and
// LDS budget), queried once; vfar_prepare runs the queries outside any
// stream capture.
template <int DB, bool WU>
int vfar_bpc() {
  constexpr bool PF = DB <= 8;  // register prefetch of the next chunk where the registers allow it
  static std::atomic<int> bpc{0};
  int b = bpc.load(std::memory_order_relaxed);
  if (b == 0) {
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, vfar_pairs_kernel<DB, WU, PF>, 256, 0) != hipSuccess)
      b = 0;
    b = std::max(1, b);
    bpc.store(b, std::memory_order_relaxed);
  }
  return b;
}

template <int DB, bool WU>
hipError_t launch_pairs(int n_far, int N, int n_cu, const double* refd, const float* aY, int D, const double* vd,
                        const int* far_idx, double* part, hipStream_t st, VfarGrid& vg) {
  constexpr bool PF = DB <= 8;
  vg = vfar_grid(n_far, N, vfar_bpc<DB, WU>() * n_cu);
  const dim3 grid((unsigned)vg.n_rt, (unsigned)vg.n_seg);
  hipLaunchKernelGGL((vfar_pairs_kernel<DB, WU, PF>), grid, dim3(256), 0, st, refd, N, vg.cps, aY, D, vd, far_idx,
                     n_far, part);
  return hipGetLastError();
}

void vfar_prepare(int D) {
  switch (vfar_db(D)) {
    case 4: vfar_bpc<4, false>(); vfar_bpc<4, true>(); break;
    case 8: vfar_bpc<8, false>(); vfar_bpc<8, true>(); break;
    case 12: vfar_bpc<12, false>(); vfar_bpc<12, true>(); break;
    case 16: vfar_bpc<16, false>(); vfar_bpc<16, true>(); break;
    case 20: vfar_bpc<20, false>(); vfar_bpc<20, true>(); break;
    case 24: vfar_bpc<24, false>(); vfar_bpc<24, true>(); break;
    case 28: vfar_bpc<28, false>(); vfar_bpc<28, true>(); break;
    case 32: vfar_bpc<32, false>(); vfar_bpc<32, true>(); break;
    default: break;
  }
}

hipError_t launch_vfar(const VForceArgs& A, const float* aY, int D, const double* vd, const double* refd,
                       const int* far_idx, int n_far, double* part, int slot0, bool wu, bool wf, int n_cu,
                       hipStream_t st) {
  if (n_far <= 0) return hipSuccess;
  const int N = A.N;
  VfarGrid vg;
  hipError_t e = hipSuccess;
  switch (vfar_db(D) * 2 + (wu ? 1 : 0)) {
    case 8: e = launch_pairs<4, false>(n_far, N, n_cu, refd, aY, D, vd, far_idx, part, st, vg); break;
    case 9: e = launch_pairs<4, true>(n_far, N, n_cu, refd, aY, D, vd, far_idx, part, st, vg); break;
    case 16: e = launch_pairs<8, false>(n_far, N, n_cu, refd, aY, D, vd, far_idx, part, st, vg); break;
    case 17: e = launch_pairs<8, true>(n_far, N, n_cu, refd, aY, D, vd, far_idx, part, st, vg); break;
    case 24: e = launch_pairs<12, false>(n_far, N, n_cu, refd, aY, D, vd, far_idx, part, st, vg); break;
    case 25: e = launch_pairs<12, true>(n_far, N, n_cu, refd, aY, D, vd, far_idx, part, st, vg); break;
    case 32: e = launch_pairs<16, false>(n_far, N, n_cu, refd, aY, D, vd, far_idx, part, st, vg); break;
    case 33: e = launch_pairs<16, true>(n_far, N, n_cu, refd, aY, D, vd, far_idx, part, st, vg); break;
    case 40: e = launch_pairs<20, false>(n_far, N, n_cu, refd, aY, D, vd, far_idx, part, st, vg); break;
    case 41: e = launch_pairs<20, true>(n_far, N, n_cu, refd, aY, D, vd, far_idx, part, st, vg); break;
    case 48: e = launch_pairs<24, false>(n_far, N, n_cu, refd, aY, D, vd, far_idx, part, st, vg); break;
    case 49: e = launch_pairs<24, true>(n_far, N, n_cu, refd, aY, D, vd, far_idx, part, st, vg); break;
    case 56: e = launch_pairs<28, false>(n_far, N, n_cu, refd, aY, D, vd, far_idx, part, st, vg); break;
    case 57: e = launch_pairs<28, true>(n_far, N, n_cu, refd, aY, D, vd, far_idx, part, st, vg); break;
    case 64: e = launch_pairs<32, false>(n_far, N, n_cu, refd, aY, D, vd, far_idx, part, st, vg); break;
    case 65: e = launch_pairs<32, true>(n_far, N, n_cu, refd, aY, D, vd, far_idx, part, st, vg); break;
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  const dim3 block(256);
  const dim3 eg((unsigned)vg.n_rt);
  if (wu && wf)
    hipLaunchKernelGGL((vfar_epi_kernel<true, true>), eg, block, 0, st, A, far_idx, n_far, vg.n_seg, part, slot0);
  else if (wu)
    hipLaunchKernelGGL((vfar_epi_kernel<true, false>), eg, block, 0, st, A, far_idx, n_far, vg.n_seg, part, slot0);
  else if (wf)
    hipLaunchKernelGGL((vfar_epi_kernel<false, true>), eg, block, 0, st, A, far_idx, n_far, vg.n_seg, part, slot0);
  else
    hipLaunchKernelGGL((vfar_epi_kernel<false, false>), eg, block, 0, st, A, far_idx, n_far, vg.n_seg, part, slot0);
  return hipGetLastError();
}

// f16 form possible: every augmented entry below 30000 in magnitude (the
// largest is log2(e) |c|^2 + |lw|; masses within 2^+-100 keep |lw| small).
bool vforce_half_ok(double cmax) { return cmax == cmax && LOG2E * cmax <= 29000.0; }

}  // namespace sgr
